// runtime.hip -- host runtime behind the C ABI in include/dsmc.h: parameter
// checks, the per-instance device arena, work lists and launch shapes of a
// group, step enqueueing and HIP-graph replay, estimator read-back, state
// export and import, and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "dsmc.h"
#include "kernels.hpp"

using namespace dsmc;

namespace {

thread_local std::string g_last_error;

int fail(std::string* sink, int code, const std::string& msg) {
    if (sink) *sink = msg;
    g_last_error = msg;
    return code;
}

#define HIP_TRY(sink, expr)                                                           \
    do {                                                                              \
        const hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess)                                                         \
            return fail(sink, DSMC_ERR_DEVICE,                                        \
                        std::string(#expr ": ") + hipGetErrorString(e_));             \
    } while (0)

constexpr uint64_t kAlign = 256;
// four LDS tables of this many cells fill 160 KiB of LDS
constexpr int64_t kMaxCollisionCells = 10240;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Derived sizes and constants of one instance (the same for footprint and
// creation).  Constants are evaluated once each, in double, in the order
// written, so they equal the reference recipe's.
struct Plan {
    int mode = 0;
    size_t rb = 8;  // bytes per real
    int32_t N = 0, C = 0, Cc = 0, ns = 1, ppc = 0;
    int32_t ncap = 0;     // particle slots (N unless open)
    int open = 0;         // 1: a patch with an open boundary at L
    int32_t tile_items = 256, tiles = 1, nseg = 1;
    double H = 1.0, L = 1.0, lam = 0, dt = 0, g = 0, kntc = 0, crmax0 = 0, sqrt_tw = 1, inv_dy = 0;
    // arena offsets
    uint64_t off_buf[2][4], off_cell, off_counts, off_tkeys, off_segsum, off_kcount, off_koffset, off_count,
        off_offset, off_crmax,
        off_rem, off_acc, off_ncoll, off_est, off_sc, off_os, off_desc, total;
};

// Slots of a particle tile the scatter can lay out in LDS before writing: the
// tile the move-scatter holds in registers (256 x 6 in FP32, 256 x 4 in FP64).
int stage_slots(size_t rb) { return kParticleThreads * (rb == 4 ? kScatterRegs32 : kScatterRegs64); }

int base_items_per_thread(int32_t N, int32_t Cc, size_t rb) {
    // Tiles of 256 * k slots with at least 4 slots per collision cell keep
    // the per-tile histogram traffic near one byte per particle.  A small
    // instance is cut into at least ~128 tiles, so the workgroups an XCD has
    // in flight belong to one or two instances whose scatter destinations
    // fit in its L2, where the partial cache lines of a random scatter merge
    // before they reach HBM.
    int k = (int)std::ceil(4.0 * (double)Cc / (double)kParticleThreads);
    k = std::max(1, std::min(64, k));
    const int k_small = (int)std::ceil((double)N / (128.0 * kParticleThreads));
    if (k_small < k) {
        // and such tiles are small enough for the scatter to stage in LDS
        k = std::max(1, std::min(k_small, stage_slots(rb) / kParticleThreads));
    }
    const int64_t need = (int64_t)((N + kParticleThreads - 1) / kParticleThreads);
    if (need < k) k = (int)std::max<int64_t>(1, need);
    return k;
}

// Instances whose fast-mode steps sort by buckets of cells (the collide
// kernel finishes the sort): fewer than kCoopMin particles per collision cell.
bool bucket_eligible(const dsmc_params* p) {
    return p->precision != DSMC_FP64_DETERMINISTIC &&
           (double)p->particles_per_cell / (double)p->n_sub < (double)kCoopMin;
}

// A small bucket-sorted instance gets 256-slot base tiles, so that a lane
// of a few such instances can cut them fine enough to give the particle
// kernels tens of workgroups; a lane with enough tiles groups them back into
// full register tiles (kScatterRegs per thread).  Tiles never change results.
constexpr int32_t kSmallInstance = 16384;
constexpr int64_t kLaneTilesEnough = 2048;  // 256-slot tiles a lane needs to keep full tiles

int check_params(const dsmc_params* p, std::string* err) {
    if (!p) return fail(err, DSMC_ERR_INVALID_ARG, "params is NULL");
    if (p->struct_size != sizeof(dsmc_params))
        return fail(err, DSMC_ERR_INVALID_ARG, "params.struct_size != sizeof(dsmc_params)");
    if (p->precision != DSMC_FP64_DETERMINISTIC && p->precision != DSMC_FP32_FAST &&
        p->precision != DSMC_FP64_FAST)
        return fail(err, DSMC_ERR_INVALID_ARG, "unknown precision");
    if (!(std::isfinite(p->kn) && p->kn > 0.0)) return fail(err, DSMC_ERR_INVALID_ARG, "kn must be finite and > 0");
    if (!std::isfinite(p->body_force)) return fail(err, DSMC_ERR_INVALID_ARG, "body_force must be finite");
    if (!(std::isfinite(p->wall_temperature) && p->wall_temperature > 0.0))
        return fail(err, DSMC_ERR_INVALID_ARG, "wall_temperature must be finite and > 0");
    if (!std::isfinite(p->dt)) return fail(err, DSMC_ERR_INVALID_ARG, "dt must be finite");
    if (p->n_cells < 1 || p->particles_per_cell < 1 || p->n_sub < 1)
        return fail(err, DSMC_ERR_INVALID_ARG, "n_cells, particles_per_cell and n_sub must be >= 1");
    if ((int64_t)p->n_cells * p->particles_per_cell > (int64_t)INT32_MAX / 2)
        return fail(err, DSMC_ERR_INVALID_ARG, "too many particles for int32 slots");
    if ((int64_t)p->n_cells * p->n_sub > kMaxCollisionCells)
        return fail(err, DSMC_ERR_INVALID_ARG, "n_cells * n_sub exceeds the collision-cell limit");
    if (p->n_transient < 0) return fail(err, DSMC_ERR_INVALID_ARG, "n_transient must be >= 0");
    if (p->debug_phase_mask > DSMC_PHASE_ALL) return fail(err, DSMC_ERR_INVALID_ARG, "bad phase mask");
    if (!(std::isfinite(p->domain_length) && p->domain_length >= 0.0 && p->domain_length <= 1.0))
        return fail(err, DSMC_ERR_INVALID_ARG, "domain_length must be in [0, 1]");
    if (p->domain_length > 0.0 && p->debug_phase_mask != 0)
        return fail(err, DSMC_ERR_INVALID_ARG, "an open domain runs whole steps only");
    return DSMC_OK;
}

constexpr double kPi = 0x1.921fb54442d18p+1;  // pi, correctly rounded

}  // namespace

struct dsmc_handle;
namespace {
void inflow_constants(const dsmc_handle* h, double u, double dudy, double T, double n, double out[6]);
}  // namespace

namespace {

Plan make_plan(const dsmc_params* p) {
    Plan q;
    q.mode = p->precision;
    q.rb = p->precision == DSMC_FP32_FAST ? 4 : 8;
    q.C = p->n_cells;
    q.ns = p->n_sub;
    q.Cc = p->n_cells * p->n_sub;
    q.ppc = p->particles_per_cell;
    q.N = p->n_cells * p->particles_per_cell;
    q.open = p->domain_length > 0.0;
    q.ncap = q.N;
    if (q.open) {
        // the count of an open patch fluctuates about N: room for 25% more,
        // and at least 8 standard deviations plus 64
        const int64_t m1 = (int64_t)q.N / 4, m2 = (int64_t)(8.0 * std::sqrt((double)q.N)) + 64;
        q.ncap = (int32_t)std::min<int64_t>((int64_t)q.N + std::max(m1, m2), (int64_t)INT32_MAX / 2);
    }
    q.H = 1.0;
    q.lam = p->kn * q.H;
    if (p->dt > 0.0) {
        q.dt = p->dt;
    } else {
        const double lref = q.lam < q.H ? q.lam : q.H;
        q.dt = (0.2 * lref) / std::sqrt(2.0);
    }
    q.g = 2.0 * p->body_force;
    q.kntc = (q.dt * (double)p->n_sub) / ((std::sqrt(2.0) * q.lam) * (double)p->particles_per_cell);
    q.crmax0 = 5.0 * std::sqrt(2.0 * p->wall_temperature);
    q.sqrt_tw = std::sqrt(p->wall_temperature);
    q.L = q.open ? p->domain_length : q.H;
    q.inv_dy = (double)q.Cc / q.L;
    int k = base_items_per_thread(q.N, q.Cc, q.rb);
    if (bucket_eligible(p)) {
        // few sort keys: tiles as large as the move-scatter holds in registers
        const int regs = q.rb == 4 ? kScatterRegs32 : kScatterRegs64;
        k = std::max(1, std::min(regs, (q.N + kParticleThreads - 1) / kParticleThreads));
        if (q.N <= kSmallInstance) k = 1;
    }
    q.tile_items = k * kParticleThreads;
    q.tiles = (q.ncap + q.tile_items - 1) / q.tile_items;
    q.nseg = (q.tiles + kSegTiles - 1) / kSegTiles;

    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    // an open instance's sort has one key more (the particles that left)
    const uint64_t keys = (uint64_t)q.Cc + (uint64_t)q.open;
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 4; ++a) q.off_buf[b][a] = take((uint64_t)q.ncap * q.rb);
    q.off_cell = take((uint64_t)q.ncap * 4);
    q.off_counts = take((uint64_t)q.tiles * keys * 4);
    q.off_tkeys = take((uint64_t)q.tiles * 2 * 4);
    q.off_segsum = take((uint64_t)q.nseg * keys * 4);
    q.off_kcount = take(keys * 4);
    q.off_koffset = take(keys * 4);
    q.off_count = take(keys * 4);
    q.off_offset = take(keys * 4);
    q.off_crmax = take((uint64_t)q.Cc * 8);
    q.off_rem = take((uint64_t)q.Cc * 8);
    q.off_acc = take((uint64_t)q.Cc * kMoments * 8);
    q.off_ncoll = take((uint64_t)q.Cc * 4);
    q.off_est = take(((uint64_t)kEstPerCell * q.C + 3) * 8);
    q.off_sc = take(sizeof(DevScalars));
    q.off_os = take(sizeof(OpenState));
    q.off_desc = take(sizeof(InstDesc));
    q.total = o + kAlign;  // slack to align an unaligned arena
    return q;
}

int device_max_lds() {
    static int cached = -1;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (cached < 0) {
        // Largest dynamic LDS a workgroup may use: the device's per-block limit
        // less room for the kernels' static shared variables, if the kernels
        // accept it, else 64 KiB.  Errors of the probing calls are cleared so
        // they do not surface at a later launch.
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        (void)hipGetLastError();
        cached = 65536;
        hipError_t e1 = hipSuccess, e2 = hipSuccess;
        if (v - 1024 > 65536) {
            e1 = dsmc::configure_kernels((size_t)(v - 1024));
            if (e1 == hipSuccess) cached = v - 1024;
            (void)hipGetLastError();
        }
        if (cached == 65536) {
            e2 = dsmc::configure_kernels((size_t)cached);
            (void)hipGetLastError();
        }
        if (std::getenv("DSMC_VERBOSE"))
            std::fprintf(stderr, "dsmc: device max LDS per block %d, using %d (%s / %s)\n", v, cached,
                         hipGetErrorString(e1), hipGetErrorString(e2));
    }
    return cached;
}

// Largest dynamic LDS of the resident kernel: the device's per-block limit
// less room for its static shared variables, else 64 KiB.
int resident_max_lds() {
    static int cached = -1;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (cached < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        (void)hipGetLastError();
        cached = 65536;
        if (v - 1024 > 65536 && dsmc::configure_resident((size_t)(v - 1024)) == hipSuccess)
            cached = v - 1024;
        else
            (void)dsmc::configure_resident((size_t)cached);
        (void)hipGetLastError();
        if (std::getenv("DSMC_VERBOSE"))
            std::fprintf(stderr, "dsmc: resident kernel LDS limit %d\n", cached);
    }
    return cached;
}

// LDS of one CU (160 KiB on MI355X), shared by the workgroups resident on it.
int cu_lds_bytes() {
    static int cached = -1;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    if (cached < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            v <= 0)
            v = 160 * 1024;
        (void)hipGetLastError();
        cached = v;
    }
    return cached;
}

}  // namespace

struct dsmc_group;

struct dsmc_handle {
    dsmc_params p{};
    Plan plan;
    InstDesc desc{};          // host copy; desc.buf etc. point into the arena
    InstDesc* d_desc = nullptr;  // device copy of desc (init, sample, reset)
    void* mem = nullptr;
    bool owns_mem = false;
    hipStream_t stream = nullptr;
    dsmc_group* group = nullptr;  // user group
    dsmc_group* solo = nullptr;   // private group behind dsmc_step
    // true once a sort has run since the last dsmc_set_state: the device cell
    // array then holds pre-sort cells and the current slot order's cells
    // follow from the counts and offsets
    bool sorted = false;
    int32_t* bucket_count = nullptr;   // per-bucket count / offset (bucket-sorted launch shapes)
    int32_t* bucket_offset = nullptr;
    double inflow[kOpenInflowDoubles] = {0, 0, 0, 0, 0, 0};  // source of the inflow copies
    std::string err;
};

namespace {
// Inflow constants of an open instance (the OpenState fields the host sets),
// each evaluated once in double in the order written: mean x velocity in
// sqrt(kT_ref/m) units, sqrt(T), sqrt(2T), the Chapman-Enskog shear weight
// a = (4 Kn/sqrt(pi)) du/dy / (n sqrt(T)) of the factor 1 - a C_x C_y, its
// acceptance bound 1 + 16 |a|, and the particles expected to enter per step,
// n (N / L) sqrt(T / (2 pi)) dt (the Maxwellian inward flux; the shear term
// carries no net number flux).
void inflow_constants(const dsmc_handle* h, double u, double dudy, double T, double n, double out[6]) {
    const Plan& q = h->plan;
    out[0] = u * std::sqrt(2.0);
    out[1] = std::sqrt(T);
    out[2] = std::sqrt(2.0 * T);
    out[3] = (((4.0 * h->p.kn) / std::sqrt(kPi)) * dudy) / (n * out[1]);
    out[4] = 1.0 + 16.0 * std::fabs(out[3]);
    out[5] = ((n * ((double)q.N / q.L)) * std::sqrt(T / (2.0 * kPi))) * q.dt;
}
}  // namespace

// A lane of a group: a subset of its members with their own work lists, step
// graph and stream.  The lanes of a group run concurrently; each step forks
// from the group's stream and joins back to it.
struct Lane {
    std::vector<dsmc_handle*> members;
    void* d_mem = nullptr;   // device-side work lists
    size_t d_bytes = 0;
    Work work{};
    // graphs of 8, 4, 2 and 1 whole steps (kGraphSizes), so that any number
    // of steps is replayed from graphs
    hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
    hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
    hipStream_t cap_stream = nullptr;
    hipStream_t stream = nullptr;    // own stream when the group has several lanes
    hipEvent_t done = nullptr;
    int32_t* d_status = nullptr;  // in d_mem: the members' status words (dsmc_group_sync)
};

struct dsmc_group {
    hipStream_t stream = nullptr;
    int mode = -1;
    bool solo = false;
    std::vector<dsmc_handle*> members;
    bool dirty = true;
    int tile_mult = 0;   // 0 = automatic
    int ppb = 0;         // target particles per fast-collide workgroup, 0 = automatic
    int waves_per_cu = 0;  // occupancy cap of the particle and collide kernels, 0 = automatic
    bool resident = true;  // lanes of small instances step them in one workgroup each
    unsigned phase = DSMC_PHASE_ALL;
    int n_lanes = 1;     // lanes in use (lanes.size() may be larger)
    int resident_lane = -1;  // the lane of the small members of a mixed group, or -1
    std::vector<int> lane_order;  // enqueue order of the lanes: resident ones first
    std::vector<Lane> lanes;
    hipEvent_t fork = nullptr;
    // dsmc_group_sample: the members' descriptors and staging-block offsets
    // in member order, the device staging buffer and its pinned host mirror,
    // rebuilt when the membership changes
    uint64_t version = 0;            // bumped by every add / remove
    uint64_t sample_version = ~0ull;
    InstDesc* d_sdesc = nullptr;
    int64_t* d_soff = nullptr;
    double* d_stage = nullptr;
    double* h_stage = nullptr;
    size_t sdesc_cap = 0, stage_cap = 0;   // members / doubles allocated
    size_t stage_doubles = 0;
    std::vector<int64_t> soff;
    std::string err;
};

namespace {

constexpr int kGraphSteps = 8;
constexpr int kGraphSizes[4] = {8, 4, 2, 1};  // steps of a lane's graphs
constexpr int64_t kResidentChunk = 4096;  // steps per launch of a resident lane

hipStream_t stream_of(const dsmc_handle* h) {
    return h->group ? h->group->stream : h->stream;
}

void drop_graph(Lane& l) {
    for (int i = 0; i < 4; ++i) {
        if (l.gexec[i]) (void)hipGraphExecDestroy(l.gexec[i]);
        if (l.graph[i]) (void)hipGraphDestroy(l.graph[i]);
        l.gexec[i] = nullptr;
        l.graph[i] = nullptr;
    }
}

void drop_graphs(dsmc_group* g) {
    for (Lane& l : g->lanes) drop_graph(l);
}

// Groups of at least this many particles (and two or more members) run in
// two lanes: the kernels are latency-bound, so a second lane fills the gaps
// and tails of the first (about 10% on the 256-instance mix).
constexpr int64_t kLaneMinParticles = 2000000;
constexpr int kMaxLanes = 2;

// The stream the lane's steps go to.
hipStream_t lane_stream(const dsmc_group* g, const Lane& l) {
    return g->n_lanes > 1 ? l.stream : g->stream;
}

int auto_cpb(const dsmc_handle* h, int target_particles) {
    // Cells per workgroup of the staged collide: one by default; a tuning
    // target packs cells up to that many particles.
    const double per_cell = (double)h->plan.N / (double)h->plan.Cc;
    if (target_particles <= 0) return 1;
    const int c = (int)std::floor((double)target_particles / std::max(per_cell, 1.0));
    return std::max(1, std::min(c, 64));
}

// Lanes per cell of the small-cell collide: about one per eight particles,
// a power of two from 4 to 32.
int group_width(double per_cell) {
    int G = 4;
    while (G < 32 && G * 16 <= per_cell) G *= 2;
    return G;
}

// Particles per sort bucket of a small-cell instance, unless tuned.
int usual_bucket(int mode) { return mode == kFp32Fast ? 2048 : 1024; }

// log2 of the cells per sort bucket of a small-cell instance: the largest
// power of two of cells holding at most about `target` particles.
int bucket_shift(double per_cell, int target) {
    int sh = 0;
    while ((1 << (sh + 1)) <= kMaxCellsPerKey && (double)(1 << (sh + 1)) * per_cell <= (double)target)
        ++sh;
    return sh;
}

// Order a work list for the XCDs: workgroups are dealt to the 8 XCDs in
// turn (workgroup p runs on XCD p mod 8), so the list, taken in its natural
// instance-major order, is cut into 8 contiguous stripes and stripe x is
// dealt to positions x, x+8, ...  All tiles of a small instance, and
// neighbouring tiles of a large one, then share one XCD's L2, where the
// scatter's partial cache lines to the same cell regions merge.
template <class T>
std::vector<T> xcd_stripes(const std::vector<T>& in) {
    constexpr int kX = 8;
    const size_t n = in.size();
    if (n <= (size_t)kX) return in;
    std::vector<size_t> beg(kX + 1);
    for (int x = 0; x <= kX; ++x) beg[x] = n * (size_t)x / kX;
    std::vector<size_t> next(beg.begin(), beg.end() - 1);
    std::vector<T> out;
    out.reserve(n);
    for (size_t p = 0; out.size() < n; ++p) {
        int x = (int)(p % kX);
        if (next[x] >= beg[x + 1]) {
            // this stripe is used up (the stripes differ by at most one):
            // take from the stripe with the most left
            int best = -1;
            size_t left = 0;
            for (int y = 0; y < kX; ++y)
                if (beg[y + 1] - next[y] > left) {
                    left = beg[y + 1] - next[y];
                    best = y;
                }
            x = best;
        }
        out.push_back(in[next[x]++]);
    }
    return out;
}

// (Re)build the device work lists and launch shapes of a group.
// Work lists and launch shapes of one lane.
int build_lane(dsmc_group* g, Lane& lane) {
    const int n = (int)lane.members.size();
    std::vector<InstDesc> descs(n);
    std::vector<int2> tiles, wide_tiles;  // tiles the move-scatter holds in registers; larger ones
    std::vector<int4> cols, cblocks, gblocks;
    int max_cc = 1;
    int cap = 64, group_cap = 64;
    int has_open = 0;
    // the lane is resident if every member is small (fast mode, bucket
    // collide shape, few keys, slots within one workgroup's registers)
    std::vector<int2> resident;
    bool all_small = g->resident && g->mode != kFp64Det && g->phase == DSMC_PHASE_ALL && n > 0;
    int resident_cap = 64;
    // a lane with few 256-slot tiles keeps its small instances' tiles fine
    int64_t lane_tiles = 0;
    for (const dsmc_handle* h : lane.members) lane_tiles += (h->plan.ncap + kParticleThreads - 1) / kParticleThreads;
    const bool fine_tiles = lane_tiles < kLaneTilesEnough;
    for (int i = 0; i < n; ++i) {
        dsmc_handle* h = lane.members[i];
        InstDesc d = h->desc;
        if (!g->solo) d.phase_mask = DSMC_PHASE_ALL;
        const double per_cell = (double)d.N / (double)d.Cc;
        // small cells in a fast mode are sorted by buckets of cells (the
        // collide kernel finishes the sort); debug phase masks keep the
        // plain sort by cell
        const bool bucketed = g->mode != kFp64Det && per_cell < kCoopMin &&
                              d.phase_mask == (uint32_t)DSMC_PHASE_ALL;
        int64_t base_items = h->plan.tile_items;
        if (bucketed) {
            // buckets of about `target` particles; a lane starved of
            // workgroups takes a quarter of the usual size
            const int usual = usual_bucket(g->mode);
            const int target = g->ppb > 0 ? g->ppb : (fine_tiles ? usual / 4 : usual);
            d.key_shift = bucket_shift(per_cell, target);
            d.nkeys = ((d.Cc + (1 << d.key_shift) - 1) >> d.key_shift) + d.open;
            d.kcount = h->bucket_count;
            d.koffset = h->bucket_offset;
        } else {
            d.key_shift = 0;
            d.nkeys = d.Cc + d.open;
            d.kcount = d.count;
            d.koffset = d.offset;
        }
        has_open |= d.open;
        // launch shape: tiles may only grow (the histogram matrix is sized
        // for the base tile and all cells)
        int mult = g->tile_mult > 0 ? g->tile_mult : 1;
        if (g->tile_mult <= 0 && !fine_tiles && bucket_eligible(&h->p) && h->plan.N <= kSmallInstance)
            mult = g->mode == kFp32Fast ? kScatterRegs32 : kScatterRegs64;
        const int64_t items = std::min<int64_t>(base_items * mult,
                                                (int64_t)std::max(h->plan.ncap, 1) + kParticleThreads);
        d.tile_items = (int32_t)((items + kParticleThreads - 1) / kParticleThreads * kParticleThreads);
        d.tiles = (d.ncap + d.tile_items - 1) / d.tile_items;
        d.nseg = (d.tiles + kSegTiles - 1) / kSegTiles;
        descs[i] = d;
        const size_t rbm = g->mode == kFp32Fast ? 4 : 8;
        std::vector<int2>& tl = d.tile_items > stage_slots(rbm) ? wide_tiles : tiles;
        for (int t = 0; t < d.tiles; ++t) tl.push_back(make_int2(i, t));
        for (int ch = 0; ch < (d.nkeys + kColThreads - 1) / kColThreads; ++ch)
            for (int sgi = 0; sgi < d.nseg; ++sgi) cols.push_back(make_int4(i, ch, sgi, 0));
        max_cc = std::max(max_cc, d.nkeys);
        if (g->mode == kFp64Det) {
            // one lane per cell, 64 cells per wavefront
            for (int c = 0; c < d.Cc; c += 64) gblocks.push_back(make_int4(i, c, std::min(c + 64, d.Cc), 64));
        } else if (bucketed) {
            // one workgroup per bucket; groups of G lanes per cell.  G is the
            // instance's own (the lanes per cell that fill a workgroup with a
            // bucket of the usual size), never the launch shape's: the lanes
            // that add up a cell's moments set the rounding of its sums, which
            // therefore do not depend on the bucket size, the tuning or the lane
            const int cpk = 1 << d.key_shift;
            // (an instance with fewer cells than a usual bucket fills the
            // workgroup with its cells alone)
            int cpk_usual = 1 << bucket_shift(per_cell, usual_bucket(g->mode));
            while (cpk_usual > 1 && cpk_usual / 2 >= d.Cc) cpk_usual /= 2;
            const int G = std::min(64, std::max(group_width(per_cell), kFastWaves * 64 / cpk_usual));
            for (int b = 0; b < d.nkeys - d.open; ++b) gblocks.push_back(make_int4(i, b, G, 0));
            const double per_block = per_cell * cpk;
            group_cap = std::max(group_cap, (int)std::ceil(per_block + 4.0 * std::sqrt(per_block) + 32.0));
            if (d.Cc + d.open <= kResidentKeys && d.ncap <= resident_slots((Mode)g->mode)) {
                resident.push_back(make_int2(i, G));
                resident_cap = std::max(resident_cap, (d.ncap + 63) / 64 * 64);
            } else {
                all_small = false;
            }
        } else {
            all_small = false;
            const int cpb = auto_cpb(h, g->ppb);
            for (int c = 0; c < d.Cc; c += cpb) cblocks.push_back(make_int4(i, c, std::min(c + cpb, d.Cc), 0));
            // staging room for a block's particles: mean + 4 Poisson sigma
            // (a fuller block works on global memory instead)
            const double per_block = per_cell * cpb;
            const int want = (int)std::ceil(per_block + 4.0 * std::sqrt(per_block) + 32.0);
            cap = std::max(cap, want);
        }
    }
    // the two kinds of tile are launched separately, each list striped
    // over the XCDs on its own
    tiles = xcd_stripes(tiles);
    const int n_narrow = (int)tiles.size();
    wide_tiles = xcd_stripes(wide_tiles);
    tiles.insert(tiles.end(), wide_tiles.begin(), wide_tiles.end());
    cblocks = xcd_stripes(cblocks);
    gblocks = xcd_stripes(gblocks);
    // fit the fast-collide staging area into the device's LDS
    const size_t rb = g->mode == kFp32Fast ? 4 : 8;
    const int max_lds = device_max_lds();
    const size_t fixed = (size_t)kCoopWaves * kCoopTablePerWave * 4 + 1024;  // claim table + static shared
    const int cap_max = (int)(((size_t)max_lds - fixed) / (3 * rb));
    cap = std::min(cap, cap_max);
    // a block that leaves no room for a second workgroup on its CU gets the
    // larger workgroup, if its larger claim table still fits
    int coop_waves = kCoopWaves;
    if (2 * (fast_collide_lds_bytes((Mode)g->mode, cap, kCoopWaves) + 1024) > (size_t)cu_lds_bytes() &&
        fast_collide_lds_bytes((Mode)g->mode, cap, kCoopWavesAlone) + 1024 <= (size_t)max_lds)
        coop_waves = kCoopWavesAlone;
    const size_t gfixed = bucket_collide_lds_bytes((Mode)g->mode, 0) + 256;  // + static shared
    group_cap = std::min(group_cap, (int)(((size_t)max_lds - gfixed) / (3 * rb)));
    if ((size_t)max_cc * 4 * kScatterWaves > (size_t)max_lds)
        return fail(&g->err, DSMC_ERR_INVALID_ARG, "sort keys exceed the LDS tables of the scatter");
    // staged scatter for members whose tiles fit, if the LDS can hold it
    int stage_max = stage_slots(rb);
    bool any_staged = false;
    for (const InstDesc& d : descs) any_staged |= d.tile_items <= stage_max;
    if (!any_staged || scatter_lds_bytes((Mode)g->mode, max_cc, stage_max) > (size_t)max_lds)
        stage_max = 0;
    // the move-scatter's LDS: per-wavefront tables (and staging) for tiles it
    // holds in registers, the chunk layout for larger tiles
    const size_t scatter_lds = scatter_lds_bytes((Mode)g->mode, max_cc, stage_max);
    const size_t wide_lds = wide_scatter_lds_bytes((Mode)g->mode, max_cc);
    if (!wide_tiles.empty() && wide_lds > (size_t)max_lds)
        return fail(&g->err, DSMC_ERR_INVALID_ARG, "sort keys exceed the LDS tables of the scatter");
    if (!all_small || resident_lds_bytes((Mode)g->mode, resident_cap) > (size_t)resident_max_lds())
        resident.clear();
    // the column scans in one workgroup per instance when every count matrix is small
    int scan_small_entries = 0;
    bool small_counts = resident.empty() && n > 0 &&
                        (g->phase & (DSMC_PHASE_MOVE | DSMC_PHASE_SORT)) == (DSMC_PHASE_MOVE | DSMC_PHASE_SORT);
    for (const InstDesc& d : descs) {
        const int64_t e = (int64_t)d.tiles * d.nkeys;
        small_counts &= d.nkeys <= kScanThreads && e <= kCountScanEntries;
        scan_small_entries = std::max<int>(scan_small_entries, (int)std::min<int64_t>(e, INT32_MAX));
    }
    const int scan_small_lds = small_counts ? std::max(scan_small_entries, 1) * (int)sizeof(int) : 0;
    // else in one workgroup per instance with the segment sums in LDS, when
    // they fit for every instance and the lane has instances enough to fill
    // the device with such workgroups (one instance's column kernels spread
    // its segments over many workgroups, and were faster alone: 46 against
    // 52 us per step of the Kn 0.1 instance)
    int scan_seg_entries = 0;
    bool seg_counts = !small_counts && resident.empty() && n >= kSegScanMinInstances &&
                      (g->phase & (DSMC_PHASE_MOVE | DSMC_PHASE_SORT)) == (DSMC_PHASE_MOVE | DSMC_PHASE_SORT);
    for (const InstDesc& d : descs) {
        const int64_t e = ((int64_t)d.nseg + 1) * d.nkeys;
        seg_counts &= e <= kSegScanEntries;
        scan_seg_entries = std::max<int>(scan_seg_entries, (int)std::min<int64_t>(e, INT32_MAX));
    }
    const int scan_seg_lds = seg_counts ? std::max(scan_seg_entries, 1) * (int)sizeof(int) : 0;

    auto bytes_of = [](size_t k, size_t sz) { return align_up(sz * std::max<size_t>(k, 1)); };
    const size_t need = bytes_of(n, sizeof(InstDesc)) + bytes_of(tiles.size(), sizeof(int2)) +
                        bytes_of(cols.size(), sizeof(int4)) + bytes_of(cblocks.size(), sizeof(int4)) +
                        bytes_of(gblocks.size(), sizeof(int4)) + bytes_of(resident.size(), sizeof(int2)) +
                        bytes_of(n, sizeof(int32_t));
    if (need > lane.d_bytes) {
        if (lane.d_mem) (void)hipFree(lane.d_mem);
        lane.d_mem = nullptr;
        lane.d_bytes = 0;
        HIP_TRY(&g->err, hipMalloc(&lane.d_mem, need));
        lane.d_bytes = need;
    }
    char* base = (char*)lane.d_mem;
    size_t o = 0;
    InstDesc* d_desc = (InstDesc*)(base + o);
    o += bytes_of(n, sizeof(InstDesc));
    int2* d_tiles = (int2*)(base + o);
    o += bytes_of(tiles.size(), sizeof(int2));
    int4* d_cols = (int4*)(base + o);
    o += bytes_of(cols.size(), sizeof(int4));
    int4* d_cb = (int4*)(base + o);
    o += bytes_of(cblocks.size(), sizeof(int4));
    int4* d_lb = (int4*)(base + o);
    o += bytes_of(gblocks.size(), sizeof(int4));
    int2* d_res = (int2*)(base + o);
    o += bytes_of(resident.size(), sizeof(int2));
    lane.d_status = (int32_t*)(base + o);
    if (n) HIP_TRY(&g->err, hipMemcpy(d_desc, descs.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice));
    if (!tiles.empty()) HIP_TRY(&g->err, hipMemcpy(d_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice));
    if (!cols.empty()) HIP_TRY(&g->err, hipMemcpy(d_cols, cols.data(), sizeof(int4) * cols.size(), hipMemcpyHostToDevice));
    if (!cblocks.empty()) HIP_TRY(&g->err, hipMemcpy(d_cb, cblocks.data(), sizeof(int4) * cblocks.size(), hipMemcpyHostToDevice));
    if (!gblocks.empty()) HIP_TRY(&g->err, hipMemcpy(d_lb, gblocks.data(), sizeof(int4) * gblocks.size(), hipMemcpyHostToDevice));
    if (!resident.empty()) HIP_TRY(&g->err, hipMemcpy(d_res, resident.data(), sizeof(int2) * resident.size(), hipMemcpyHostToDevice));
    Work& w = lane.work;
    w.desc = d_desc;
    w.n_inst = n;
    w.tiles = d_tiles;
    w.n_tiles = (int)tiles.size();
    w.n_narrow = n_narrow;
    w.cols = d_cols;
    w.n_cols = (int)cols.size();
    w.cblocks = d_cb;
    w.n_cblocks = (int)cblocks.size();
    w.gblocks = d_lb;
    w.n_gblocks = (int)gblocks.size();
    w.group_cap = group_cap;
    w.max_cc = max_cc;
    w.stage_max = stage_max;
    w.scatter_lds = scatter_lds;
    w.wide_lds = wide_lds;
    w.fast_cap = cap;
    w.coop_waves = coop_waves;
    w.has_open = has_open;
    w.resident = d_res;
    w.n_resident = (int)resident.size();
    w.resident_cap = resident_cap;
    w.scan_small_lds = scan_small_lds;
    w.scan_seg_lds = scan_seg_lds;
    // occupancy cap: the count, move-scatter and collide workgroups are 4
    // wavefronts; asking each for 1/k of the CU's LDS (less a margin for
    // static shared variables and allocation granularity) lets at most k
    // share a CU
    w.lds_floor = 0;
    w.lds_floor_coop = 0;
    if (g->waves_per_cu > 0) {
        auto floor_of = [&](int waves_per_group) {
            const int per_cu = std::max(1, g->waves_per_cu / waves_per_group);
            const int floor_bytes = cu_lds_bytes() / per_cu - 2048;
            return (size_t)std::max(0, std::min(floor_bytes, max_lds));
        };
        w.lds_floor = floor_of(4);
        w.lds_floor_coop = floor_of(coop_waves);
    }
    return DSMC_OK;
}

// Capture the lane's graphs of 8, 4, 2 and 1 whole steps when the lane is
// built.  Capture only records the launches (no kernel runs), so the first
// steps that replay them pay no capture or instantiation, and a call's
// steps are all replayed (whole chunks of 8, then at most one graph of each
// smaller size), never launched one kernel at a time.  Resident lanes and
// debug phase masks launch directly and have no graph.
int capture_lane(dsmc_group* g, Lane& l) {
    if (l.members.empty() || l.work.n_resident || g->phase != DSMC_PHASE_ALL) return DSMC_OK;
    if (!l.cap_stream) HIP_TRY(&g->err, hipStreamCreateWithFlags(&l.cap_stream, hipStreamNonBlocking));
    for (int i = 0; i < 4; ++i) {
        HIP_TRY(&g->err, hipStreamBeginCapture(l.cap_stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < kGraphSizes[i]; ++k) launch_step(l.work, (Mode)g->mode, g->phase, l.cap_stream);
        const hipError_t launched = hipGetLastError();
        hipGraph_t graph = nullptr;
        const hipError_t ended = hipStreamEndCapture(l.cap_stream, &graph);
        if (launched != hipSuccess || ended != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(&g->err, DSMC_ERR_DEVICE,
                        std::string("step graph capture: ") +
                            hipGetErrorString(launched != hipSuccess ? launched : ended));
        }
        l.graph[i] = graph;
        HIP_TRY(&g->err, hipGraphInstantiate(&l.gexec[i], graph, nullptr, nullptr, 0));
    }
    return DSMC_OK;
}

// (Re)build the lanes of a group: members are dealt to the lanes largest
// first, each to the lane with the fewest particles so far.
// A member small enough for a resident lane (the conditions build_lane
// checks for a lane to run resident).
bool resident_eligible(const dsmc_group* g, const dsmc_handle* h) {
    if (!g->resident || g->mode == kFp64Det || g->phase != DSMC_PHASE_ALL) return false;
    if (!((double)h->plan.N / (double)h->plan.Cc < (double)kCoopMin)) return false;
    if (h->plan.Cc + h->plan.open > kResidentKeys) return false;
    if (h->plan.ncap > resident_slots((Mode)g->mode)) return false;
    return resident_lds_bytes((Mode)g->mode, (h->plan.ncap + 63) / 64 * 64) <= (size_t)resident_max_lds();
}

// (Re)build the lanes of a group.  Members are dealt to the lanes largest
// first, each to the lane with the fewest particles so far.  A group that
// mixes members small enough to run resident with larger ones gives the
// small ones a lane of their own, which steps them resident beside the
// multi-kernel lanes of the others.
int rebuild(dsmc_group* g) {
    // the streams may still be running the previous graphs and lists: wait
    // for them before either is released
    HIP_TRY(&g->err, hipStreamSynchronize(g->stream));
    for (Lane& l : g->lanes)
        if (l.stream) HIP_TRY(&g->err, hipStreamSynchronize(l.stream));
    drop_graphs(g);
    g->phase = (g->solo && g->members.size() == 1 && g->members[0]->p.debug_phase_mask)
                   ? g->members[0]->p.debug_phase_mask
                   : (unsigned)DSMC_PHASE_ALL;
    std::vector<dsmc_handle*> small, large;
    for (dsmc_handle* h : g->members) (resident_eligible(g, h) ? small : large).push_back(h);
    const bool split = !g->solo && !small.empty() && !large.empty();
    const std::vector<dsmc_handle*>& multi = split ? large : g->members;
    int64_t total = 0;
    for (const dsmc_handle* h : multi) total += h->plan.N;
    const int nm = (!g->solo && multi.size() >= 2 && total >= kLaneMinParticles) ? kMaxLanes : 1;
    const int nl = nm + (split ? 1 : 0);
    if ((int)g->lanes.size() < nl) g->lanes.resize(nl);
    g->n_lanes = nl;
    g->resident_lane = split ? nm : -1;
    if (nl > 1 && !g->fork) HIP_TRY(&g->err, hipEventCreateWithFlags(&g->fork, hipEventDisableTiming));
    for (int k = 0; k < nl; ++k) {
        Lane& l = g->lanes[k];
        l.members.clear();
        if (nl > 1) {
            if (!l.stream) HIP_TRY(&g->err, hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking));
            if (!l.done) HIP_TRY(&g->err, hipEventCreateWithFlags(&l.done, hipEventDisableTiming));
        }
    }
    std::vector<dsmc_handle*> order(multi);
    std::stable_sort(order.begin(), order.end(),
                     [](const dsmc_handle* a, const dsmc_handle* b) { return a->plan.N > b->plan.N; });
    std::vector<int64_t> load(nm, 0);
    for (dsmc_handle* h : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        g->lanes[k].members.push_back(h);
        load[k] += h->plan.N;
    }
    if (split) g->lanes[nm].members = small;
    for (int k = 0; k < nl; ++k) {
        int r = build_lane(g, g->lanes[k]);
        if (r) return r;
        r = capture_lane(g, g->lanes[k]);
        if (r) return r;
    }
    // resident lanes are enqueued first (kept here, so that stepping
    // allocates nothing on the host)
    g->lane_order.clear();
    for (int k = 0; k < nl; ++k)
        if (g->lanes[k].work.n_resident) g->lane_order.push_back(k);
    for (int k = 0; k < nl; ++k)
        if (!g->lanes[k].work.n_resident) g->lane_order.push_back(k);
    g->dirty = false;
    return DSMC_OK;
}

int enqueue_steps(dsmc_group* g, int64_t n_steps) {
    if (n_steps < 0) return fail(&g->err, DSMC_ERR_INVALID_ARG, "n_steps < 0");
    if (g->members.empty() || n_steps == 0) return DSMC_OK;
    if (g->dirty) {
        const int r = rebuild(g);
        if (r) return r;
    }
    const Mode mode = (Mode)g->mode;
    const int nl = g->n_lanes;
    if (nl > 1) HIP_TRY(&g->err, hipEventRecord(g->fork, g->stream));
    // resident lanes are enqueued first: each of their workgroups needs most
    // of a CU's LDS, which a CU has free before the multi-kernel lanes fill
    // it; enqueued after them, they could only start in the gaps between
    // those lanes' kernels and finished after them
    for (int li : g->lane_order) {
        Lane& l = g->lanes[li];
        const hipStream_t st = lane_stream(g, l);
        if (nl > 1) HIP_TRY(&g->err, hipStreamWaitEvent(st, g->fork, 0));
        int64_t left = n_steps;
        if (l.work.n_resident) {
            // whole steps in one launch per chunk
            for (int64_t k = 0; k < n_steps; k += kResidentChunk) {
                launch_resident(l.work, mode, std::min<int64_t>(kResidentChunk, n_steps - k), st);
                HIP_TRY(&g->err, hipGetLastError());
            }
            left = 0;
        }
        // the graphs were captured when the lane was built
        if (l.gexec[0]) {
            while (left >= kGraphSteps) {
                HIP_TRY(&g->err, hipGraphLaunch(l.gexec[0], st));
                left -= kGraphSteps;
            }
            for (int i = 1; i < 4; ++i)
                if (left >= kGraphSizes[i]) {
                    HIP_TRY(&g->err, hipGraphLaunch(l.gexec[i], st));
                    left -= kGraphSizes[i];
                }
        }
        for (int64_t k = 0; k < left; ++k) {
            launch_step(l.work, mode, g->phase, st);
            HIP_TRY(&g->err, hipGetLastError());
        }
        if (nl > 1) {
            HIP_TRY(&g->err, hipEventRecord(l.done, st));
            HIP_TRY(&g->err, hipStreamWaitEvent(g->stream, l.done, 0));
        }
    }
    HIP_TRY(&g->err, hipGetLastError());
    return DSMC_OK;
}

int sync_check(dsmc_handle* h) {
    HIP_TRY(&h->err, hipStreamSynchronize(stream_of(h)));
    DevScalars sc;
    HIP_TRY(&h->err, hipMemcpy(&sc, h->desc.sc, sizeof sc, hipMemcpyDeviceToHost));
    if (sc.status & 1) return fail(&h->err, DSMC_ERR_NUMERIC, "non-finite particle velocity");
    if (sc.status & 2) return fail(&h->err, DSMC_ERR_NUMERIC, "cell counts do not add up to N");
    if (sc.status & 4) return fail(&h->err, DSMC_ERR_NUMERIC, "sorted slot out of range");
    if (sc.status & 8) return fail(&h->err, DSMC_ERR_NUMERIC, "open boundary: particle slots exhausted");
    return DSMC_OK;
}

// Particles in the handle's slots after the last sort (the nominal count
// unless the instance is open).  Synchronises.
int live_count(dsmc_handle* h, int32_t* n) {
    *n = h->plan.N;
    if (!h->plan.open) return DSMC_OK;
    HIP_TRY(&h->err, hipStreamSynchronize(stream_of(h)));
    OpenState os;
    HIP_TRY(&h->err, hipMemcpy(&os, h->desc.os, sizeof os, hipMemcpyDeviceToHost));
    *n = os.n_live;
    return DSMC_OK;
}

int group_init(dsmc_group* g, hipStream_t stream, bool solo) {
    g->stream = stream;
    g->solo = solo;
    return DSMC_OK;
}

void group_free(dsmc_group* g) {
    if (!g) return;
    if (g->stream || !g->members.empty()) (void)hipStreamSynchronize(g->stream);
    for (Lane& l : g->lanes) {
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        drop_graph(l);
        if (l.cap_stream) (void)hipStreamDestroy(l.cap_stream);
        if (l.stream) (void)hipStreamDestroy(l.stream);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.d_mem) (void)hipFree(l.d_mem);
    }
    if (g->fork) (void)hipEventDestroy(g->fork);
    if (g->d_sdesc) (void)hipFree(g->d_sdesc);
    if (g->d_soff) (void)hipFree(g->d_soff);
    if (g->d_stage) (void)hipFree(g->d_stage);
    if (g->h_stage) (void)hipHostFree(g->h_stage);
    delete g;
}

// Staging of dsmc_group_sample for the current members: member i's block of
// kEstPerCell * C + 4 doubles (estimators, mass flow, sampled steps,
// collisions, status) starts at soff[i], rounded up to 32 doubles.
int prepare_group_sample(dsmc_group* g) {
    if (g->sample_version == g->version) return DSMC_OK;
    const size_t n = g->members.size();
    g->soff.assign(n, 0);
    size_t tot = 0;
    for (size_t i = 0; i < n; ++i) {
        g->soff[i] = (int64_t)tot;
        tot += ((size_t)kEstPerCell * g->members[i]->plan.C + 4 + 31) & ~(size_t)31;
    }
    if (n > g->sdesc_cap) {
        if (g->d_sdesc) (void)hipFree(g->d_sdesc);
        if (g->d_soff) (void)hipFree(g->d_soff);
        g->d_sdesc = nullptr;
        g->d_soff = nullptr;
        g->sdesc_cap = 0;
        if (hipMalloc((void**)&g->d_sdesc, n * sizeof(InstDesc)) != hipSuccess ||
            hipMalloc((void**)&g->d_soff, n * sizeof(int64_t)) != hipSuccess)
            return fail(&g->err, DSMC_ERR_OUT_OF_MEMORY, "group sample descriptors");
        g->sdesc_cap = n;
    }
    if (tot > g->stage_cap) {
        if (g->d_stage) (void)hipFree(g->d_stage);
        if (g->h_stage) (void)hipHostFree(g->h_stage);
        g->d_stage = nullptr;
        g->h_stage = nullptr;
        g->stage_cap = 0;
        if (hipMalloc((void**)&g->d_stage, tot * sizeof(double)) != hipSuccess ||
            hipHostMalloc((void**)&g->h_stage, tot * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return fail(&g->err, DSMC_ERR_OUT_OF_MEMORY, "group sample staging");
        g->stage_cap = tot;
    }
    std::vector<InstDesc> hd(n);
    for (size_t i = 0; i < n; ++i) hd[i] = g->members[i]->desc;
    HIP_TRY(&g->err, hipMemcpy(g->d_sdesc, hd.data(), n * sizeof(InstDesc), hipMemcpyHostToDevice));
    HIP_TRY(&g->err, hipMemcpy(g->d_soff, g->soff.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
    g->stage_doubles = tot;
    g->sample_version = g->version;
    return DSMC_OK;
}

// Member i's estimators from its block of a group sample's host staging
// (at soff[i]: kEstPerCell * C estimator values, mass flow, sampled steps,
// collisions, status) into outs[i].
int unpack_group_sample(dsmc_group* g, dsmc_moments* outs, const double* stage, const int64_t* soff) {
    const int n = (int)g->members.size();
    int rc = DSMC_OK;
    for (int i = 0; i < n; ++i) {
        const int C = g->members[i]->plan.C;
        const double* e = stage + soff[i];
        dsmc_moments* out = &outs[i];
        const int status = (int)e[(size_t)kEstPerCell * C + 3];
        if (status) {
            out->n_sampled_steps = -1;
            if (rc == DSMC_OK) {
                const char* why = (status & 1)   ? "non-finite particle velocity"
                                  : (status & 2) ? "cell counts do not add up to N"
                                  : (status & 4) ? "sorted slot out of range"
                                                 : "open boundary: particle slots exhausted";
                rc = fail(&g->err, DSMC_ERR_NUMERIC, "member " + std::to_string(i) + ": " + why);
            }
            continue;
        }
        double* dst[kEstPerCell] = {out->n,  out->ux, out->uy, out->uz,     out->T,
                                    out->pxy, out->qx, out->qy, out->pxy_mid};
        for (int m = 0; m < kEstPerCell; ++m)
            if (dst[m]) std::memcpy(dst[m], e + (size_t)m * C, sizeof(double) * C);
        const double K = e[(size_t)kEstPerCell * C + 1];
        out->n_sampled_steps = (int64_t)K;
        out->mass_flow = K > 0 ? e[(size_t)kEstPerCell * C] : NAN;
        out->n_collisions = (int64_t)e[(size_t)kEstPerCell * C + 2];
    }
    return rc;
}

// ------------------------------------------------- allocation-free sampling
// dsmc_group_sample_noalloc keeps its tables and staging in a fixed device
// array instead of buffers allocated per group: a table of pointers to the
// members' device descriptors, each member's offset in the staging area, and
// the staging area itself.  Each device holds its own copy of the array (at
// its own address, looked up once per device) until the process ends.
constexpr int kScratchMaxMembers = 1024;
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr size_t kScratchTableBytes = (size_t)kScratchMaxMembers * (sizeof(void*) + sizeof(int64_t));
constexpr size_t kScratchStageDoubles = (kScratchBytes - kScratchTableBytes) / sizeof(double);
constexpr int kScratchDevices = 64;
static_assert(kScratchTableBytes % 256 == 0, "the staging area starts 256-byte aligned");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices] = {};   // scratch's address on each device
// host side of the staging area: one copy brings every member's block back
double g_scratch_host[kScratchStageDoubles];

// The current device's address of the scratch array (looked up on the first
// call on that device).  Call with g_scratch_mu held.
int scratch_address(std::string* err, char** out) {
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(err, DSMC_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kScratchDevices)
        return fail(err, DSMC_ERR_DEVICE, "device index beyond the scratch table");
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t r = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (r != hipSuccess || !ptr)
            return fail(err, DSMC_ERR_DEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(r));
        g_scratch_dev[dev] = ptr;
    }
    *out = (char*)g_scratch_dev[dev];
    return DSMC_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char* dsmc_status_string(int status) {
    switch (status) {
        case DSMC_OK: return "ok";
        case DSMC_ERR_INVALID_ARG: return "invalid argument";
        case DSMC_ERR_OUT_OF_MEMORY: return "out of memory";
        case DSMC_ERR_DEVICE: return "device error";
        case DSMC_ERR_STATE: return "invalid state";
        case DSMC_ERR_NUMERIC: return "numeric error";
        default: return "unknown status";
    }
}

const char* dsmc_last_error(const dsmc_handle* h) {
    return h ? h->err.c_str() : g_last_error.c_str();
}

int dsmc_params_init(dsmc_params* p) {
    if (!p) return fail(nullptr, DSMC_ERR_INVALID_ARG, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof(dsmc_params);
    p->precision = DSMC_FP64_DETERMINISTIC;
    p->kn = 1.0;
    p->body_force = 0.0;
    p->wall_temperature = 1.0;
    p->dt = 0.0;
    p->n_cells = 100;
    p->particles_per_cell = 50;
    p->n_sub = 1;
    p->n_transient = 1000;
    p->seed = 0;
    return DSMC_OK;
}

int dsmc_footprint_bytes(const dsmc_params* p, uint64_t* bytes) {
    const int r = check_params(p, nullptr);
    if (r) return r;
    if (!bytes) return fail(nullptr, DSMC_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = make_plan(p).total;
    return DSMC_OK;
}

int dsmc_create(const dsmc_params* p, void* stream, void* arena, uint64_t arena_bytes,
                dsmc_handle** out) {
    if (out) *out = nullptr;
    if (!out) return fail(nullptr, DSMC_ERR_INVALID_ARG, "out is NULL");
    int r = check_params(p, nullptr);
    if (r) return r;
    const Plan q = make_plan(p);
    if (arena && arena_bytes < q.total) return fail(nullptr, DSMC_ERR_OUT_OF_MEMORY, "arena smaller than dsmc_footprint_bytes");
    dsmc_handle* h = new (std::nothrow) dsmc_handle();
    if (!h) return fail(nullptr, DSMC_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->p = *p;
    h->plan = q;
    h->stream = (hipStream_t)stream;
    if (arena) {
        h->mem = arena;
    } else {
        const hipError_t e = hipMalloc(&h->mem, q.total);
        if (e != hipSuccess) {
            delete h;
            return fail(nullptr, e == hipErrorOutOfMemory ? DSMC_ERR_OUT_OF_MEMORY : DSMC_ERR_DEVICE,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        h->owns_mem = true;
    }
    char* base = (char*)(((uintptr_t)h->mem + kAlign - 1) / kAlign * kAlign);
    InstDesc& d = h->desc;
    d.N = q.N;
    d.C = q.C;
    d.Cc = q.Cc;
    d.n_sub = q.ns;
    d.tiles = q.tiles;
    d.tile_items = q.tile_items;
    d.nseg = q.nseg;
    d.ppc = q.ppc;
    d.H = q.L;  // top of the domain: the far plate, or the patch's open boundary
    d.open = q.open;
    d.ncap = q.ncap;
    d.os = q.open ? (OpenState*)(base + q.off_os) : nullptr;
    d.dt = q.dt;
    d.g = q.g;
    d.kntc = q.kntc;
    d.crmax0 = q.crmax0;
    d.sqrt_tw = q.sqrt_tw;
    d.inv_dy = q.inv_dy;
    d.n_transient = p->n_transient;
    d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFull);
    d.key1 = (uint32_t)(p->seed >> 32);
    d.phase_mask = p->debug_phase_mask ? p->debug_phase_mask : (uint32_t)DSMC_PHASE_ALL;
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 4; ++a) d.buf[b][a] = base + q.off_buf[b][a];
    d.cell = (int32_t*)(base + q.off_cell);
    d.counts = (int32_t*)(base + q.off_counts);
    d.tkeys = (int32_t*)(base + q.off_tkeys);
    d.segsum = (int32_t*)(base + q.off_segsum);
    d.count = (int32_t*)(base + q.off_count);
    d.offset = (int32_t*)(base + q.off_offset);
    // sorted by cell unless a group's launch shape sorts it by buckets (an
    // open instance has one key more, past every cell, for the particles
    // that left)
    d.nkeys = q.Cc + q.open;
    d.key_shift = 0;
    d.kcount = d.count;
    d.koffset = d.offset;
    h->bucket_count = (int32_t*)(base + q.off_kcount);
    h->bucket_offset = (int32_t*)(base + q.off_koffset);
    d.crmax = (double*)(base + q.off_crmax);
    d.rem = (double*)(base + q.off_rem);
    d.acc = (double*)(base + q.off_acc);
    d.ncoll = (uint32_t*)(base + q.off_ncoll);
    d.est = (double*)(base + q.off_est);
    d.sc = (DevScalars*)(base + q.off_sc);
    h->d_desc = (InstDesc*)(base + q.off_desc);
    device_max_lds();
    const char* where = "copy of the instance descriptor";
    hipError_t e = hipMemcpyAsync(h->d_desc, &h->desc, sizeof(InstDesc), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && q.open) {
        where = "copy of the inflow";
        inflow_constants(h, 0.0, 0.0, p->wall_temperature, 1.0, h->inflow);
        e = hipMemcpyAsync(d.os, h->inflow, sizeof(h->inflow), hipMemcpyHostToDevice, h->stream);
    }
    if (e == hipSuccess) {
        where = "init kernel launch";
        launch_init(h->desc, h->d_desc, (Mode)q.mode, h->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        where = "init synchronise";
        e = hipStreamSynchronize(h->stream);
    }
    if (e != hipSuccess) {
        if (h->owns_mem) (void)hipFree(h->mem);
        delete h;
        return fail(nullptr, DSMC_ERR_DEVICE, std::string("create: ") + where + ": " + hipGetErrorString(e));
    }
    *out = h;
    return DSMC_OK;
}

int dsmc_step(dsmc_handle* h, int64_t n_steps) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    if (h->group) return fail(&h->err, DSMC_ERR_STATE, "handle belongs to a group; use dsmc_group_step");
    if (n_steps < 0) return fail(&h->err, DSMC_ERR_INVALID_ARG, "n_steps < 0");
    if (!h->solo) {
        h->solo = new (std::nothrow) dsmc_group();
        if (!h->solo) return fail(&h->err, DSMC_ERR_OUT_OF_MEMORY, "host allocation failed");
        group_init(h->solo, h->stream, true);
        h->solo->mode = h->plan.mode;
        h->solo->members.push_back(h);
    }
    const int r = enqueue_steps(h->solo, n_steps);
    if (r) h->err = h->solo->err;
    else if (n_steps > 0 && (h->solo->phase & DSMC_PHASE_SORT)) h->sorted = true;
    return r;
}

int dsmc_sync(dsmc_handle* h) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    return sync_check(h);
}

int dsmc_sample(dsmc_handle* h, dsmc_moments* out, int reset_window) {
    if (!h || !out) return fail(h ? &h->err : nullptr, DSMC_ERR_INVALID_ARG, "NULL argument");
    if (out->n_cells < h->plan.C) return fail(&h->err, DSMC_ERR_INVALID_ARG, "moments.n_cells smaller than the handle's cells");
    hipStream_t s = stream_of(h);
    launch_finalize(h->d_desc, 1, s);
    HIP_TRY(&h->err, hipGetLastError());
    const int C = h->plan.C;
    std::vector<double> est((size_t)kEstPerCell * C + 3);
    HIP_TRY(&h->err, hipMemcpyAsync(est.data(), h->desc.est, est.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<double> raw;
    if (out->raw_sums) {
        raw.resize((size_t)h->plan.Cc * kMoments);
        HIP_TRY(&h->err, hipMemcpyAsync(raw.data(), h->desc.acc, raw.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    DevScalars sc;
    HIP_TRY(&h->err, hipMemcpyAsync(&sc, h->desc.sc, sizeof sc, hipMemcpyDeviceToHost, s));
    int r = sync_check(h);
    if (r) return r;
    double* dst[kEstPerCell] = {out->n,  out->ux, out->uy, out->uz,     out->T,
                                out->pxy, out->qx, out->qy, out->pxy_mid};
    for (int m = 0; m < kEstPerCell; ++m)
        if (dst[m]) std::memcpy(dst[m], est.data() + (size_t)m * C, sizeof(double) * C);
    if (out->raw_sums) {
        // device layout is moment-major; the ABI's is 13 sums per collision cell
        const size_t cc = (size_t)h->plan.Cc;
        for (size_t c = 0; c < cc; ++c)
            for (int k = 0; k < kMoments; ++k) out->raw_sums[c * kMoments + k] = raw[(size_t)k * cc + c];
    }
    out->mass_flow = sc.n_sampled ? est[(size_t)kEstPerCell * C] : NAN;
    out->n_sampled_steps = sc.n_sampled;
    out->n_collisions = (int64_t)est[(size_t)kEstPerCell * C + 2];
    if (reset_window) {
        launch_reset_window(h->d_desc, 1, s);
        HIP_TRY(&h->err, hipGetLastError());
    }
    return DSMC_OK;
}

int dsmc_get_state(dsmc_handle* h, void* y, void* vx, void* vy, void* vz, int32_t* cell,
                   uint64_t* step) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    int r = sync_check(h);
    if (r) return r;
    DevScalars sc;
    HIP_TRY(&h->err, hipMemcpy(&sc, h->desc.sc, sizeof sc, hipMemcpyDeviceToHost));
    int32_t n_live = 0;
    r = live_count(h, &n_live);
    if (r) return r;
    const int b = (int)(sc.step_done & 1);
    const size_t bytes = (size_t)n_live * h->plan.rb;
    void* outs[4] = {y, vx, vy, vz};
    for (int a = 0; a < 4; ++a)
        if (outs[a]) HIP_TRY(&h->err, hipMemcpy(outs[a], h->desc.buf[b][a], bytes, hipMemcpyDeviceToHost));
    if (cell) {
        if (h->sorted) {
            const size_t c = (size_t)h->plan.Cc;
            std::vector<int32_t> count(c), offset(c);
            HIP_TRY(&h->err, hipMemcpy(count.data(), h->desc.count, c * 4, hipMemcpyDeviceToHost));
            HIP_TRY(&h->err, hipMemcpy(offset.data(), h->desc.offset, c * 4, hipMemcpyDeviceToHost));
            for (size_t k = 0; k < c; ++k)
                for (int32_t i = 0; i < count[k]; ++i) cell[offset[k] + i] = (int32_t)k;
        } else {
            HIP_TRY(&h->err, hipMemcpy(cell, h->desc.cell, (size_t)n_live * 4, hipMemcpyDeviceToHost));
        }
    }
    if (step) *step = (uint64_t)sc.step_done;
    return DSMC_OK;
}

int dsmc_set_state(dsmc_handle* h, const void* y, const void* vx, const void* vy, const void* vz,
                   const int32_t* cell, uint64_t step) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    int r = sync_check(h);
    if (r) return r;
    DevScalars sc;
    HIP_TRY(&h->err, hipMemcpy(&sc, h->desc.sc, sizeof sc, hipMemcpyDeviceToHost));
    const int b_old = (int)(sc.step_done & 1);
    sc.step_done = (int64_t)step;
    const int b = (int)(step & 1);
    int32_t n_live = 0;
    r = live_count(h, &n_live);
    if (r) return r;
    const size_t bytes = (size_t)n_live * h->plan.rb;
    const void* ins[4] = {y, vx, vy, vz};
    for (int a = 0; a < 4; ++a) {
        if (ins[a]) {
            HIP_TRY(&h->err, hipMemcpy(h->desc.buf[b][a], ins[a], bytes, hipMemcpyHostToDevice));
        } else if (b != b_old) {
            // arrays not given keep their current values, in the new buffer
            HIP_TRY(&h->err, hipMemcpy(h->desc.buf[b][a], h->desc.buf[b_old][a], bytes, hipMemcpyDeviceToDevice));
        }
    }
    if (cell) HIP_TRY(&h->err, hipMemcpy(h->desc.cell, cell, (size_t)n_live * 4, hipMemcpyHostToDevice));
    HIP_TRY(&h->err, hipMemcpy(h->desc.sc, &sc, sizeof sc, hipMemcpyHostToDevice));
    h->sorted = false;
    return DSMC_OK;
}

int dsmc_set_inflow(dsmc_handle* h, double u, double dudy, double temperature, double density) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    if (!h->plan.open) return fail(&h->err, DSMC_ERR_INVALID_ARG, "the instance has no open boundary");
    if (!(std::isfinite(u) && std::isfinite(dudy) && std::isfinite(temperature) && temperature > 0.0 &&
          std::isfinite(density) && density >= 0.0))
        return fail(&h->err, DSMC_ERR_INVALID_ARG, "inflow must be finite, T > 0, n >= 0");
    double c[kOpenInflowDoubles];
    inflow_constants(h, u, dudy, temperature, density, c);
    // |a| <= 1 keeps the acceptance rate of the inflow draws above 1/17 (and
    // the expansion within its range: |P_xy| <= P/2); the expected entrants
    // of a step must fit the slots
    if (density > 0.0 && !(std::fabs(c[3]) <= 1.0))
        return fail(&h->err, DSMC_ERR_INVALID_ARG,
                    "velocity gradient too large for the Chapman-Enskog inflow (|a| > 1)");
    if (!(c[5] <= (double)h->plan.ncap))
        return fail(&h->err, DSMC_ERR_INVALID_ARG, "inflow density too large for the particle slots");
    // the copy is ordered on the instance's stream: steps enqueued before it
    // use the previous inflow; its source stays with the handle
    HIP_TRY(&h->err, hipStreamSynchronize(stream_of(h)));
    std::memcpy(h->inflow, c, sizeof c);
    HIP_TRY(&h->err, hipMemcpyAsync(h->desc.os, h->inflow, sizeof(h->inflow), hipMemcpyHostToDevice,
                                    stream_of(h)));
    return DSMC_OK;
}

int dsmc_set_open_state(dsmc_handle* h, int32_t n_live, int64_t n_injected, int64_t n_removed,
                        double inj_remainder) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    if (!h->plan.open) return fail(&h->err, DSMC_ERR_INVALID_ARG, "the instance has no open boundary");
    if (n_live < 0 || n_live > h->plan.ncap || n_injected < 0 || n_removed < 0 ||
        !(std::isfinite(inj_remainder) && inj_remainder >= 0.0 && inj_remainder < 1.0))
        return fail(&h->err, DSMC_ERR_INVALID_ARG, "open state out of range");
    const int r = sync_check(h);
    if (r) return r;
    OpenState os;
    HIP_TRY(&h->err, hipMemcpy(&os, h->desc.os, sizeof os, hipMemcpyDeviceToHost));
    os.n_live = n_live;
    os.n_used = n_live;
    os.n_injected = n_injected;
    os.n_deleted = n_removed;
    os.inj_rem = inj_remainder;
    HIP_TRY(&h->err, hipMemcpy(h->desc.os, &os, sizeof os, hipMemcpyHostToDevice));
    return DSMC_OK;
}

int dsmc_open_state(dsmc_handle* h, int32_t* n_live, int64_t* n_injected, int64_t* n_removed,
                    double* inj_remainder) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    if (!h->plan.open) return fail(&h->err, DSMC_ERR_INVALID_ARG, "the instance has no open boundary");
    const int r = sync_check(h);
    if (r) return r;
    OpenState os;
    HIP_TRY(&h->err, hipMemcpy(&os, h->desc.os, sizeof os, hipMemcpyDeviceToHost));
    if (n_live) *n_live = os.n_live;
    if (n_injected) *n_injected = os.n_injected;
    if (n_removed) *n_removed = os.n_deleted;
    if (inj_remainder) *inj_remainder = os.inj_rem;
    return DSMC_OK;
}

int dsmc_get_cells(dsmc_handle* h, double* crmax, double* rem, int32_t* count, int32_t* offset) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    int r = sync_check(h);
    if (r) return r;
    const size_t c = (size_t)h->plan.Cc;
    if (crmax) HIP_TRY(&h->err, hipMemcpy(crmax, h->desc.crmax, c * 8, hipMemcpyDeviceToHost));
    if (rem) HIP_TRY(&h->err, hipMemcpy(rem, h->desc.rem, c * 8, hipMemcpyDeviceToHost));
    if (count) HIP_TRY(&h->err, hipMemcpy(count, h->desc.count, c * 4, hipMemcpyDeviceToHost));
    if (offset) HIP_TRY(&h->err, hipMemcpy(offset, h->desc.offset, c * 4, hipMemcpyDeviceToHost));
    return DSMC_OK;
}

int dsmc_set_cells(dsmc_handle* h, const double* crmax, const double* rem, const int32_t* count,
                   const int32_t* offset) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    int r = sync_check(h);
    if (r) return r;
    const size_t c = (size_t)h->plan.Cc;
    if (count && offset) {
        int64_t tot = 0;
        for (size_t i = 0; i < c; ++i) {
            if (count[i] < 0 || offset[i] != tot) return fail(&h->err, DSMC_ERR_INVALID_ARG, "offsets must be the exclusive scan of counts");
            tot += count[i];
        }
        int32_t n_live = 0;
        r = live_count(h, &n_live);
        if (r) return r;
        if (tot != n_live)
            return fail(&h->err, DSMC_ERR_INVALID_ARG, "counts must add up to the particles held");
    } else if (count || offset) {
        return fail(&h->err, DSMC_ERR_INVALID_ARG, "count and offset must be given together");
    }
    if (crmax) HIP_TRY(&h->err, hipMemcpy(h->desc.crmax, crmax, c * 8, hipMemcpyHostToDevice));
    if (rem) HIP_TRY(&h->err, hipMemcpy(h->desc.rem, rem, c * 8, hipMemcpyHostToDevice));
    if (count) HIP_TRY(&h->err, hipMemcpy(h->desc.count, count, c * 4, hipMemcpyHostToDevice));
    if (offset) HIP_TRY(&h->err, hipMemcpy(h->desc.offset, offset, c * 4, hipMemcpyHostToDevice));
    return DSMC_OK;
}

int dsmc_info(const dsmc_handle* h, int32_t* n_particles, int32_t* n_coll_cells, double* c6) {
    if (!h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "handle is NULL");
    if (n_particles) *n_particles = h->plan.N;
    if (n_coll_cells) *n_coll_cells = h->plan.Cc;
    if (c6) {
        c6[0] = h->plan.dt;
        c6[1] = h->plan.g;
        c6[2] = h->plan.kntc;
        c6[3] = h->plan.crmax0;
        c6[4] = h->plan.inv_dy;
        c6[5] = h->plan.lam;
    }
    return DSMC_OK;
}

int dsmc_destroy(dsmc_handle* h) {
    if (!h) return DSMC_OK;
    if (h->group) dsmc_group_remove(h->group, h);
    (void)hipStreamSynchronize(h->stream);
    if (h->solo) group_free(h->solo);
    if (h->owns_mem && h->mem) (void)hipFree(h->mem);
    delete h;
    return DSMC_OK;
}

int dsmc_profile_step(dsmc_handle* h, int64_t n_steps, double* phase_ms) {
    if (!h || !phase_ms || n_steps < 1) return fail(h ? &h->err : nullptr, DSMC_ERR_INVALID_ARG, "bad argument");
    dsmc_group* g = h->group;
    if (!g) {
        // make sure the private group exists and is current
        int r = dsmc_step(h, 0);
        if (r) return r;
        if (!h->solo) {
            h->solo = new (std::nothrow) dsmc_group();
            if (!h->solo) return fail(&h->err, DSMC_ERR_OUT_OF_MEMORY, "host allocation failed");
            group_init(h->solo, h->stream, true);
            h->solo->mode = h->plan.mode;
            h->solo->members.push_back(h);
        }
        g = h->solo;
    }
    if (g->dirty) {
        const int r = rebuild(g);
        if (r) return r;
    }
    // all steps are enqueued before any wait, so the device runs them back to
    // back and the events bracket kernel execution, not host launch gaps
    // the lanes of a group are timed one after another on the group's
    // stream, so each kernel's time is its own (summed over the lanes)
    const int nl = g->n_lanes;
    const size_t nblk = (size_t)n_steps * nl;
    std::vector<hipEvent_t> ev(nblk * 7, nullptr);
    int rc = DSMC_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(&h->err, DSMC_ERR_DEVICE, "hipEventCreate failed");
    double acc[6] = {0, 0, 0, 0, 0, 0};
    double acc_resident = 0.0;
    if (rc == DSMC_OK && nl > 1) (void)hipStreamSynchronize(g->stream);
    const auto t0 = std::chrono::steady_clock::now();
    if (rc == DSMC_OK) {
        for (int64_t k = 0; k < n_steps; ++k)
            for (int li = 0; li < nl; ++li)
                launch_step_timed(g->lanes[li].work, (Mode)g->mode, g->phase, g->stream,
                                  ev.data() + 7 * ((size_t)k * nl + li));
        if (hipEventSynchronize(ev.back()) != hipSuccess)
            rc = fail(&h->err, DSMC_ERR_DEVICE, "event synchronise failed");
    }
    const auto t1 = std::chrono::steady_clock::now();
    if (rc == DSMC_OK) {
        for (size_t b = 0; b < nblk; ++b) {
            // a resident lane records only the events around its one kernel,
            // a lane with the single-kernel scan none around the column sums
            // and prefixes
            const Work& w = g->lanes[b % nl].work;
            for (int i = 0; i < 6; ++i) {
                if ((w.n_resident && i < 5) || ((w.scan_small_lds || w.scan_seg_lds) && (i == 1 || i == 3)))
                    continue;
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[7 * b + i], ev[7 * b + i + 1]) == hipSuccess) {
                    acc[i] += ms;
                    if (w.n_resident) acc_resident += ms;
                }
            }
        }
        (void)hipGetLastError();
    }
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    if (g->phase & DSMC_PHASE_SORT) {
        if (g->solo) h->sorted = true;
        else for (dsmc_handle* m : g->members) m->sorted = true;
    }
    for (int i = 0; i < 6; ++i) phase_ms[i] = acc[i];
    phase_ms[6] = acc[0] + acc[1] + acc[2] + acc[3] + acc[4] + acc[5];
    phase_ms[7] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    phase_ms[8] = acc_resident;
    return sync_check(h);
}

// ---------------------------------------------------------------- groups
int dsmc_group_create(void* stream, dsmc_group** out) {
    if (out) *out = nullptr;
    if (!out) return fail(nullptr, DSMC_ERR_INVALID_ARG, "out is NULL");
    dsmc_group* g = new (std::nothrow) dsmc_group();
    if (!g) return fail(nullptr, DSMC_ERR_OUT_OF_MEMORY, "host allocation failed");
    group_init(g, (hipStream_t)stream, false);
    *out = g;
    return DSMC_OK;
}

int dsmc_group_add(dsmc_group* g, dsmc_handle* h) {
    if (!g || !h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "NULL argument");
    if (h->group) return fail(&g->err, DSMC_ERR_INVALID_ARG, "handle already belongs to a group");
    if (g->mode >= 0 && !g->members.empty() && g->mode != h->plan.mode)
        return fail(&g->err, DSMC_ERR_INVALID_ARG, "precision differs from the group's");
    HIP_TRY(&g->err, hipStreamSynchronize(h->stream));
    g->mode = h->plan.mode;
    g->members.push_back(h);
    h->group = g;
    g->dirty = true;
    ++g->version;
    return DSMC_OK;
}

int dsmc_group_remove(dsmc_group* g, dsmc_handle* h) {
    if (!g || !h) return fail(nullptr, DSMC_ERR_INVALID_ARG, "NULL argument");
    auto it = std::find(g->members.begin(), g->members.end(), h);
    if (it == g->members.end()) return fail(&g->err, DSMC_ERR_INVALID_ARG, "handle is not in this group");
    HIP_TRY(&g->err, hipStreamSynchronize(g->stream));
    g->members.erase(it);
    h->group = nullptr;
    g->dirty = true;
    ++g->version;
    return DSMC_OK;
}

int dsmc_group_step(dsmc_group* g, int64_t n_steps) {
    if (!g) return fail(nullptr, DSMC_ERR_INVALID_ARG, "group is NULL");
    const int r = enqueue_steps(g, n_steps);
    if (r == DSMC_OK && n_steps > 0)
        for (dsmc_handle* h : g->members) h->sorted = true;
    return r;
}

int dsmc_group_sync(dsmc_group* g) {
    if (!g) return fail(nullptr, DSMC_ERR_INVALID_ARG, "group is NULL");
    if (g->dirty || g->members.empty()) {
        // lanes not built for the current members: check them one by one
        HIP_TRY(&g->err, hipStreamSynchronize(g->stream));
        for (dsmc_handle* h : g->members) {
            const int r = sync_check(h);
            if (r) return r;
        }
        return DSMC_OK;
    }
    // every member's status word gathered per lane, one copy each, then one
    // synchronisation of the group's stream (which every lane joins)
    std::vector<std::vector<int32_t>> st(g->n_lanes);
    for (int li = 0; li < g->n_lanes; ++li) {
        Lane& l = g->lanes[li];
        st[li].assign(l.members.size(), 0);
        if (l.members.empty()) continue;
        launch_gather_status(l.work.desc, (int)l.members.size(), l.d_status, g->stream);
        HIP_TRY(&g->err, hipGetLastError());
        HIP_TRY(&g->err, hipMemcpyAsync(st[li].data(), l.d_status, l.members.size() * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, g->stream));
    }
    HIP_TRY(&g->err, hipStreamSynchronize(g->stream));
    for (int li = 0; li < g->n_lanes; ++li)
        for (size_t i = 0; i < st[li].size(); ++i)
            if (st[li][i]) {
                // the member's own check names the error
                const int r = sync_check(g->lanes[li].members[i]);
                if (r) return fail(&g->err, r, g->lanes[li].members[i]->err);
            }
    return DSMC_OK;
}

int dsmc_group_sample(dsmc_group* g, dsmc_moments* outs, int32_t n_outs, int reset_window) {
    if (!g || (!outs && n_outs)) return fail(g ? &g->err : nullptr, DSMC_ERR_INVALID_ARG, "NULL argument");
    const int n = (int)g->members.size();
    if (n_outs != n) return fail(&g->err, DSMC_ERR_INVALID_ARG, "n_outs differs from the group's member count");
    if (n == 0) return DSMC_OK;
    for (int i = 0; i < n; ++i) {
        if (outs[i].n_cells < g->members[i]->plan.C)
            return fail(&g->err, DSMC_ERR_INVALID_ARG, "moments.n_cells smaller than a member's cells");
        if (outs[i].raw_sums)
            return fail(&g->err, DSMC_ERR_INVALID_ARG, "raw sums are returned by dsmc_sample only");
    }
    int r = prepare_group_sample(g);
    if (r) return r;
    hipStream_t s = g->stream;
    launch_finalize_staged(g->d_sdesc, g->d_soff, g->d_stage, n, s);
    HIP_TRY(&g->err, hipGetLastError());
    HIP_TRY(&g->err, hipMemcpyAsync(g->h_stage, g->d_stage, g->stage_doubles * sizeof(double),
                                    hipMemcpyDeviceToHost, s));
    if (reset_window) {
        launch_reset_window(g->d_sdesc, n, s);
        HIP_TRY(&g->err, hipGetLastError());
    }
    HIP_TRY(&g->err, hipStreamSynchronize(s));
    return unpack_group_sample(g, outs, g->h_stage, g->soff.data());
}

int dsmc_group_sample_noalloc(dsmc_group* g, dsmc_moments* outs, int32_t n_outs, int reset_window) {
    if (!g || (!outs && n_outs)) return fail(g ? &g->err : nullptr, DSMC_ERR_INVALID_ARG, "NULL argument");
    const int n = (int)g->members.size();
    if (n_outs != n) return fail(&g->err, DSMC_ERR_INVALID_ARG, "n_outs differs from the group's member count");
    if (n == 0) return DSMC_OK;
    if (n > kScratchMaxMembers)
        return fail(&g->err, DSMC_ERR_INVALID_ARG,
                    "dsmc_group_sample_noalloc: more than 1024 members (use dsmc_group_sample)");
    for (int i = 0; i < n; ++i) {
        if (outs[i].n_cells < g->members[i]->plan.C)
            return fail(&g->err, DSMC_ERR_INVALID_ARG, "moments.n_cells smaller than a member's cells");
        if (outs[i].raw_sums)
            return fail(&g->err, DSMC_ERR_INVALID_ARG, "raw sums are returned by dsmc_sample only");
    }
    // the descriptor table and the staging offsets, on the host stack
    const InstDesc* ptrs[kScratchMaxMembers];
    int64_t offs[kScratchMaxMembers];
    size_t tot = 0;
    for (int i = 0; i < n; ++i) {
        ptrs[i] = g->members[i]->d_desc;
        offs[i] = (int64_t)tot;
        tot += ((size_t)kEstPerCell * g->members[i]->plan.C + 4 + 31) & ~(size_t)31;
    }
    if (tot > kScratchStageDoubles)
        return fail(&g->err, DSMC_ERR_INVALID_ARG,
                    "dsmc_group_sample_noalloc: the members' estimators exceed the 32 MiB "
                    "scratch (use dsmc_group_sample)");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    char* base = nullptr;
    int r = scratch_address(&g->err, &base);
    if (r) return r;
    const InstDesc** d_ptrs = (const InstDesc**)base;
    int64_t* d_offs = (int64_t*)(base + (size_t)kScratchMaxMembers * sizeof(void*));
    double* d_stage = (double*)(base + kScratchTableBytes);
    hipStream_t s = g->stream;
    HIP_TRY(&g->err, hipMemcpyAsync(d_ptrs, ptrs, sizeof(void*) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(&g->err, hipMemcpyAsync(d_offs, offs, sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    launch_finalize_gather(d_ptrs, d_offs, d_stage, n, s);
    HIP_TRY(&g->err, hipGetLastError());
    HIP_TRY(&g->err, hipMemcpyAsync(g_scratch_host, d_stage, tot * sizeof(double), hipMemcpyDeviceToHost, s));
    if (reset_window) {
        launch_reset_window_gather(d_ptrs, n, s);
        HIP_TRY(&g->err, hipGetLastError());
    }
    // the stack tables above must outlive the copies that read them
    HIP_TRY(&g->err, hipStreamSynchronize(s));
    return unpack_group_sample(g, outs, g_scratch_host, offs);
}

int dsmc_group_size(const dsmc_group* g, int32_t* n) {
    if (!g || !n) return fail(nullptr, DSMC_ERR_INVALID_ARG, "NULL argument");
    *n = (int32_t)g->members.size();
    return DSMC_OK;
}

int dsmc_group_lanes(const dsmc_group* g, int32_t* n) {
    if (!g || !n) return fail(nullptr, DSMC_ERR_INVALID_ARG, "NULL argument");
    *n = (int32_t)g->n_lanes;
    return DSMC_OK;
}

int dsmc_group_lane_info(const dsmc_group* g, int32_t* n_lanes, int32_t* resident_lanes,
                         int64_t* resident_particles, int64_t* resident_cells) {
    if (!g) return fail(nullptr, DSMC_ERR_INVALID_ARG, "group is NULL");
    int32_t rl = 0;
    int64_t rp = 0, rc = 0;
    for (int k = 0; k < g->n_lanes && k < (int)g->lanes.size(); ++k)
        if (g->lanes[k].work.n_resident) {
            ++rl;
            for (const dsmc_handle* h : g->lanes[k].members) {
                rp += h->plan.N;
                rc += h->plan.Cc;
            }
        }
    if (n_lanes) *n_lanes = g->n_lanes;
    if (resident_lanes) *resident_lanes = rl;
    if (resident_particles) *resident_particles = rp;
    if (resident_cells) *resident_cells = rc;
    return DSMC_OK;
}

int dsmc_group_destroy(dsmc_group* g) {
    if (!g) return DSMC_OK;
    if (g->stream || !g->members.empty()) (void)hipStreamSynchronize(g->stream);
    for (dsmc_handle* h : g->members) h->group = nullptr;
    g->members.clear();
    group_free(g);
    return DSMC_OK;
}

int dsmc_group_set_tuning(dsmc_group* g, int32_t tile_mult, int32_t particles_per_block,
                          int32_t waves_per_cu) {
    if (!g) return fail(nullptr, DSMC_ERR_INVALID_ARG, "group is NULL");
    if (tile_mult < 0 || tile_mult > 16 || particles_per_block < 0 || particles_per_block > (1 << 20) ||
        waves_per_cu < 0 || waves_per_cu > 32 || (waves_per_cu > 0 && waves_per_cu < 4))
        return fail(&g->err, DSMC_ERR_INVALID_ARG, "tuning out of range");
    g->tile_mult = tile_mult;
    g->ppb = particles_per_block;
    g->waves_per_cu = waves_per_cu;
    g->dirty = true;
    return DSMC_OK;
}

int dsmc_group_set_resident(dsmc_group* g, int32_t enable) {
    if (!g) return fail(nullptr, DSMC_ERR_INVALID_ARG, "group is NULL");
    if (enable != 0 && enable != 1) return fail(&g->err, DSMC_ERR_INVALID_ARG, "enable must be 0 or 1");
    g->resident = enable != 0;
    g->dirty = true;
    return DSMC_OK;
}

}  // extern "C"

namespace {

struct Tuning {
    int tile_mult, ppb, waves_per_cu;
};

std::mutex g_tune_mu;
std::vector<std::pair<std::string, Tuning>> g_tune_cache;

// Signature of a group's launch problem: precision and the (N, Cc) of every
// member, so groups of the same shape reuse a tuning.
std::string group_signature(const dsmc_group* g) {
    std::vector<std::pair<int, int>> v;
    for (const dsmc_handle* h : g->members) v.emplace_back(h->plan.N, h->plan.Cc);
    std::sort(v.begin(), v.end());
    std::string s = std::to_string(g->mode);
    uint64_t hsh = 1469598103934665603ull;
    for (auto& e : v) {
        hsh = (hsh ^ (uint64_t)e.first) * 1099511628211ull;
        hsh = (hsh ^ (uint64_t)e.second) * 1099511628211ull;
    }
    return s + ":" + std::to_string(v.size()) + ":" + std::to_string(hsh);
}

bool tune_lookup(const std::string& sig, Tuning* t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& e : g_tune_cache)
        if (e.first == sig) {
            *t = e.second;
            return true;
        }
    const char* path = std::getenv("DSMC_AUTOTUNE_CACHE");
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char key[256];
    int a, b, c;
    bool found = false;
    while (std::fscanf(f, "%255s %d %d %d", key, &a, &b, &c) == 4)
        if (sig == key) {
            *t = Tuning{a, b, c};
            found = true;
        }
    std::fclose(f);
    if (found) g_tune_cache.push_back({sig, *t});
    return found;
}

void tune_store(const std::string& sig, const Tuning& t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.push_back({sig, t});
    const char* path = std::getenv("DSMC_AUTOTUNE_CACHE");
    if (!path) return;
    if (FILE* f = std::fopen(path, "a")) {
        std::fprintf(f, "%s %d %d %d\n", sig.c_str(), t.tile_mult, t.ppb, t.waves_per_cu);
        std::fclose(f);
    }
}

// Device milliseconds of kTuneSteps steps of the group at one launch shape,
// after one untimed step (which rebuilds the lanes and captures their graphs).
constexpr int kTuneSteps = 3;
int time_shape(dsmc_group* g, const Tuning& t, hipEvent_t e0, hipEvent_t e1, float* ms) {
    g->tile_mult = t.tile_mult;
    g->ppb = t.ppb;
    g->waves_per_cu = t.waves_per_cu;
    g->dirty = true;
    int rc = enqueue_steps(g, 1);
    if (rc) return rc;
    HIP_TRY(&g->err, hipEventRecord(e0, g->stream));
    rc = enqueue_steps(g, kTuneSteps);
    if (rc) return rc;
    HIP_TRY(&g->err, hipEventRecord(e1, g->stream));
    HIP_TRY(&g->err, hipEventSynchronize(e1));
    HIP_TRY(&g->err, hipEventElapsedTime(ms, e0, e1));
    return DSMC_OK;
}

}  // namespace

extern "C" {

// Coordinate search on the group's own steps: every pair of tile multiplier
// and particles per collide workgroup (which sets the cells per block) at the
// automatic occupancy, then the waves-per-CU caps at the best pair.  These
// are ordinary steps of the members (results do not depend on the launch
// shape).
int dsmc_group_autotune(dsmc_group* g, int32_t* tile_mult_out, int32_t* ppb_out,
                        int32_t* waves_per_cu_out) {
    if (!g) return fail(nullptr, DSMC_ERR_INVALID_ARG, "group is NULL");
    if (g->members.empty()) return fail(&g->err, DSMC_ERR_STATE, "group has no members");
    const std::string sig = group_signature(g);
    Tuning best{1, 0, 0};
    if (!tune_lookup(sig, &best)) {
        static const int tms[] = {1, 2, 4};
        static const int ppbs[] = {0, 1024, 4096};
        static const int wpcs[] = {8, 12, 16};
        hipEvent_t e0, e1;
        HIP_TRY(&g->err, hipEventCreate(&e0));
        HIP_TRY(&g->err, hipEventCreate(&e1));
        float best_ms = 1e30f;
        int rc = DSMC_OK;
        for (int tm : tms) {
            for (int pb : ppbs) {
                float ms = 0.f;
                const Tuning t{tm, pb, 0};
                rc = time_shape(g, t, e0, e1, &ms);
                if (rc) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
            if (rc) break;
        }
        if (!rc) {
            const Tuning pair = best;
            for (int w : wpcs) {
                float ms = 0.f;
                const Tuning t{pair.tile_mult, pair.ppb, w};
                rc = time_shape(g, t, e0, e1, &ms);
                if (rc) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (dsmc_handle* h : g->members) h->sorted = true;
        if (rc) return rc;
        tune_store(sig, best);
    }
    g->tile_mult = best.tile_mult;
    g->ppb = best.ppb;
    g->waves_per_cu = best.waves_per_cu;
    g->dirty = true;
    if (tile_mult_out) *tile_mult_out = best.tile_mult;
    if (ppb_out) *ppb_out = best.ppb;
    if (waves_per_cu_out) *waves_per_cu_out = best.waves_per_cu;
    return DSMC_OK;
}

}  // extern "C"

// kernels.hip -- DSMC hot path for gfx950 (MI355X).
//
// One step of force-driven parallel-plate DSMC (the micro model of arXiv
// 2311.14140, Sec. 2.1: gas between isothermal plates under a body force
// parallel to them) is these launches, each over every instance of a group
// (of one lane of it):
//   k_count         position-only flight of every slot (an open instance's
//                   injections drawn first), per-tile LDS histogram of sort keys
//   k_colsum        per-segment column sums of the tile histograms
//   k_scan          per-instance exclusive scan: key counts and offsets,
//                   segment bases; step counter and open-boundary bookkeeping
//   k_colprefix     per-tile scatter bases (column prefix within a segment)
//                   (k_scan_small does these three in one workgroup per
//                   instance when every count matrix is small)
//   k_move_scatter  the full move (force, diffuse walls, open boundary) and
//                   the stable scatter of the SoA records into key order
//   k_collide_*     NTC hard-sphere collisions per collision cell (the bucket
//                   variant first finishes the sort by cell in LDS), fused
//                   with the FP64 moment sums of the sampling steps
// A lane of small instances runs k_resident instead: one workgroup per
// instance performs whole steps with its particles held in LDS.  Debug phase
// masks use k_move_hist, k_scatter and k_copy, which separate the move from
// the sort.
// Everything is streaming over structure-of-arrays particle records; there
// is no dense contraction anywhere, so no MFMA.
#include <hip/hip_runtime.h>
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

#pragma clang fp contract(off)

namespace dsmc {

namespace {

constexpr unsigned kPhaseMove = 1, kPhaseSort = 2, kPhaseCollide = 4, kPhaseSample = 8;

// Device arrays reached through the descriptor are generic pointers; typed
// into the global address space, their accesses become global_* rather than
// flat_* instructions (flat accesses also wait on the LDS counter and cannot
// use scalar base addresses).
template <class T> struct GlobalSpace {
    typedef __attribute__((address_space(1))) T type;
};
template <class T> using gptr = typename GlobalSpace<T>::type*;
template <class T> __device__ __forceinline__ gptr<T> gmem(void* p) { return (gptr<T>)p; }
template <class T> __device__ __forceinline__ gptr<T> gmem(T* p) { return (gptr<T>)p; }

template <class R> struct P4 {
    gptr<R> y;
    gptr<R> vx;
    gptr<R> vy;
    gptr<R> vz;
};

template <class R> __device__ __forceinline__ P4<R> particles(const InstDesc& d, int b) {
    return P4<R>{gmem<R>(d.buf[b][0]), gmem<R>(d.buf[b][1]), gmem<R>(d.buf[b][2]),
                 gmem<R>(d.buf[b][3])};
}

__device__ __forceinline__ unsigned long long lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ------------------------------------------------------------------ init
// Initial state (the paper's gas at rest between the plates, Sec. 2.1):
// particle p sits in sampling cell p / ppc, uniform inside it, with a
// Maxwellian velocity at T_w.  Drawn in FP64 for every precision, then
// stored in the instance's precision.
template <class R>
__global__ void k_init(const InstDesc* __restrict__ descs) {
    const InstDesc& d = descs[0];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < d.N) {
        const int c = p / d.ppc;
        const double dy = d.H / (double)d.C;
        Stream st(d.key0, d.key1, 0u, (uint32_t)p, 0u, kTagInit);
        double ua, ub;
        Num<double>::uni2(st.next(), ua, ub);
        const double y = ((double)c + (1.0 - ua)) * dy;
        double vx, vy, vz, unused;
        normal_pair<double>(st, d.sqrt_tw, vx, vy);
        normal_pair<double>(st, d.sqrt_tw, vz, unused);
        P4<R> b = particles<R>(d, 0);
        b.y[p] = (R)y;
        b.vx[p] = (R)vx;
        b.vy[p] = (R)vy;
        b.vz[p] = (R)vz;
        d.cell[p] = 0;
    }
    if (p < d.Cc) {
        d.crmax[p] = d.crmax0;
        d.rem[p] = 0.0;
        d.count[p] = 0;
        d.offset[p] = 0;
        d.ncoll[p] = 0u;
        for (int m = 0; m < kMoments; ++m) d.acc[(size_t)m * d.Cc + p] = 0.0;
    }
    if (p == 0) {
        d.sc->step_done = 0;
        d.sc->n_sampled = 0;
        d.sc->status = 0;
        if (d.open) {
            d.os->inj_rem = 0.0;
            d.os->n_injected = 0;
            d.os->n_deleted = 0;
            d.os->n_live = d.N;
            d.os->n_used = d.N;
        }
    }
}

// ------------------------------------------------------------- injection
// Particles entering an open instance through its top at the start of a step
// (the hybrid's inflow: the Chapman-Enskog distribution of pure shear at the
// macro state imposed there, Sec. 2): floor(expected + carried remainder) of
// them, limited to the free slots, take the slots after the live ones of the
// step's source buffer.  The count pass draws them there (no launch of their
// own) and k_scan, once per instance, books their number and the remainder
// carried on.  Injection k of step s draws from tag kTagInject, entity k.
// Per attempt one call gives the acceptance uniform and the flux-weighted
// inward speed sqrt(-2 T ln U), a polar pair from the following calls the
// thermal x and z velocities, and the attempt is kept with probability
// (1 - a C_x C_y) / A, C = c / sqrt(2T); a last call gives the fraction of
// the step spent inside.  The particle starts where a
// straight flight of the whole step brings it across the boundary at that
// moment, with the force's x velocity gain of the outside part taken off, so
// the ordinary move delivers it with the drawn velocity at the boundary.

// Injections of the coming step of an open instance holding `live`
// particles with `rem` carried from the earlier steps, the remainder carried
// past it, and whether the slots ran out.
__device__ __forceinline__ int injections(const InstDesc& d, int live, double rem,
                                          double& rem_next, bool& clipped) {
    const double m = d.os->inj_expected + rem;
    const double f = floor(m);
    rem_next = m - f;
    int64_t n = (int64_t)f;
    clipped = (int64_t)live + n > (int64_t)d.ncap;
    if (clipped) n = (int64_t)d.ncap - (int64_t)live;
    return (int)n;
}

// State of injection k of step s: drawn in FP64 for every precision, then
// rounded to the storage precision.
template <class R>
__device__ __forceinline__ void inject_state(const InstDesc& d, uint32_t s, int k, R& y, R& vx,
                                             R& vy, R& vz) {
    const OpenState* os = d.os;
    const double sqrt_tin = os->sqrt_tin, vt = os->vt_in, a = os->ce_a, A = os->ce_A;
    Stream st(d.key0, d.key1, s, (uint32_t)k, 0u, kTagInject);
    double sp, tx, tz;
    for (;;) {
        double ua, ub;
        Num<double>::uni2(st.next(), ua, ub);
        sp = __builtin_sqrt(-2.0 * series_log(ub)) * sqrt_tin;
        normal_pair<double>(st, sqrt_tin, tx, tz);
        const double cx = tx / vt;
        const double cy = -sp / vt;
        const double gam = 1.0 - a * (cx * cy);
        if (ua * A < gam) break;
    }
    double ut, unused;
    Num<double>::uni2(st.next(), ut, unused);
    const double outside = d.dt - ut * d.dt;
    y = (R)(d.H + sp * outside);
    vx = (R)((os->u_in + tx) - d.g * outside);
    vy = (R)(-sp);
    vz = (R)tz;
}

// ------------------------------------------------------------------ move
// Free flight for dt under the acceleration g along x, followed exactly per
// segment; whenever the particle reaches a plate before its time runs out it
// is re-emitted from the wall Maxwellian at T_w (normal speed
// sqrt(-2 T_w ln U), tangential components a polar normal pair), which may
// happen several times in one step.  flight_start and flight_from_wall split
// the flight at the first plate contact, so that a kernel can run the rare
// re-emissions apart from the straight flights; move_one is the same flight
// as one loop, in the same arithmetic (both forms are checked bit for bit
// against the sequential reference by the FP64 tests).

// Time until the particle reaches the plate it moves towards (infinite when
// it moves parallel to the plates).
template <class R> __device__ __forceinline__ R time_to_wall(const InstDesc& d, R y, R vy) {
    const R H = (R)d.H;
    if (vy > R(0)) return Num<R>::div(H - y, vy);
    if (vy < R(0)) return Num<R>::div(R(0) - y, vy);
    return (R)INFINITY;
}

// The first segment: when no plate is reached within dt the particle flies
// straight (returns true); otherwise the state is left as it is and the
// plate (top or not) and the time left when it is reached are returned.  In
// an open instance the top is the open boundary: a particle reaching it
// leaves the domain (returns true with gone set; its state is then void).
template <class R, bool kOpen>
__device__ __forceinline__ bool flight_start(const InstDesc& d, R& y, R& vx, R vy, R& t_left,
                                             bool& top, bool& gone) {
    const R H = (R)d.H, g = (R)d.g, t = (R)d.dt;
    const R tw = time_to_wall<R>(d, y, vy);
    if (tw >= t) {
        y = y + vy * t;
        vx = vx + g * t;
        if (y < R(0)) y = R(0);
        if (y > H) y = H;
        return true;
    }
    top = vy > R(0);
    if (kOpen && top && d.open) {
        gone = true;
        return true;
    }
    t_left = t - tw;
    return false;
}

// The rest of a flight from the moment the particle reaches a plate with time
// t left: re-emission, further flight and any later hits (draw h of the
// particle's wall stream at its h-th hit).  The incoming y, vx, vy, vz are
// not read.  Returns the number of hits.
template <class R, bool kOpen>
__device__ __forceinline__ int flight_from_wall(const InstDesc& d, uint32_t step, uint32_t slot,
                                                bool top, R t, R& y, R& vx, R& vy, R& vz,
                                                bool& gone) {
    const R H = (R)d.H, g = (R)d.g, sd = (R)d.sqrt_tw;
    int h = 0;
    for (;;) {
        y = top ? H : R(0);
        Stream st(d.key0, d.key1, step, slot, (uint32_t)h, kTagWall);
        R vn;
        wall_draws<R>(st, sd, vn, vx, vz);
        vy = top ? -vn : vn;
        ++h;
        const R tw = time_to_wall<R>(d, y, vy);
        if (tw >= t) {
            y = y + vy * t;
            vx = vx + g * t;
            break;
        }
        top = vy > R(0);
        if (kOpen && top && d.open) {
            gone = true;
            break;
        }
        t = t - tw;
    }
    if (y < R(0)) y = R(0);
    if (y > H) y = H;
    return h;
}

// The whole flight of one step as one loop (the same arithmetic as
// flight_start followed by flight_from_wall).  Returns the number of hits.
// With kVel false only y and vy are followed (vx and vz are left as they
// are): a re-emission then draws its normal speed alone.
template <class R, bool kOpen, bool kVel = true>
__device__ __forceinline__ int move_one(const InstDesc& d, uint32_t step, uint32_t slot, R& y,
                                        R& vx, R& vy, R& vz, bool& gone) {
    const R H = (R)d.H, g = (R)d.g, sd = (R)d.sqrt_tw;
    R t = (R)d.dt;
    int h = 0;
    for (;;) {
        const R tw = time_to_wall<R>(d, y, vy);
        if (tw >= t) {
            y = y + vy * t;
            vx = vx + g * t;
            break;
        }
        const bool top = vy > R(0);
        if (kOpen && top && d.open) {
            gone = true;
            break;
        }
        y = top ? H : R(0);
        t = t - tw;
        Stream st(d.key0, d.key1, step, slot, (uint32_t)h, kTagWall);
        R vn;
        if (kVel)
            wall_draws<R>(st, sd, vn, vx, vz);
        else
            vn = wall_normal_speed<R>(st, sd);
        vy = top ? -vn : vn;
        ++h;
    }
    if (y < R(0)) y = R(0);
    if (y > H) y = H;
    return h;
}

template <class R> __device__ __forceinline__ int cell_of(const InstDesc& d, R y) {
    int c = (int)(y * (R)d.inv_dy);
    if (c >= d.Cc) c = d.Cc - 1;
    if (!(c >= 0)) c = 0;  // only reachable from a non-finite position
    return c;
}

// Sort key after a flight: the particle's cell's key, or, for a particle that
// left through an open boundary, the instance's last key (past every cell).
// The open-boundary branches of the particle kernels are compiled in only
// for launches over lanes that hold an open instance (kOpen).
template <class R, bool kOpen> __device__ __forceinline__ int key_of(const InstDesc& d, R y, bool gone) {
    return (kOpen && gone) ? d.nkeys - 1 : (cell_of<R>(d, y) >> d.key_shift);
}

// Slots of the current step: [0, live) hold the particles carried over,
// [live, used) the injections.  The count pass, before k_scan has booked the
// step, derives them from the open state; the move-scatter pass reads
// k_scan's record of the slots in use.
struct Slots {
    int live, used;
};
template <bool kOpen> __device__ __forceinline__ Slots slots_before_scan(const InstDesc& d) {
    if (!(kOpen && d.open)) return Slots{d.N, d.N};
    const int live = d.os->n_live;
    double rem;
    bool clipped;
    return Slots{live, live + injections(d, live, d.os->inj_rem, rem, clipped)};
}
template <bool kOpen> __device__ __forceinline__ int slots_after_scan(const InstDesc& d) {
    return (kOpen && d.open) ? d.os->n_used : d.N;
}

template <class R, bool kMove>
__global__ __launch_bounds__(kParticleThreads) void k_move_hist(const InstDesc* __restrict__ descs,
                                                               const int2* __restrict__ work) {
    extern __shared__ int hist[];
    __shared__ int blk_bad;
    const int2 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int nk = d.nkeys;
    for (int c = threadIdx.x; c < nk; c += blockDim.x) hist[c] = 0;
    if (threadIdx.x == 0) blk_bad = 0;
    __syncthreads();
    const int64_t s = d.sc->step_done + 1;
    const P4<R> b = particles<R>(d, (int)((s - 1) & 1));
    const int start = w.y * d.tile_items;
    const int end = min(start + d.tile_items, d.N);
    const gptr<int32_t> cellp = gmem(d.cell);
    int bad = 0;
    for (int p = start + (int)threadIdx.x; p < end; p += blockDim.x) {
        int c;
        if (kMove) {
            R y = b.y[p], vx = b.vx[p], vy = b.vy[p], vz = b.vz[p];
            bool gone = false;  // debug paths run closed instances only
            const int h = move_one<R, false>(d, (uint32_t)s, (uint32_t)p, y, vx, vy, vz, gone);
            b.y[p] = y;
            b.vx[p] = vx;
            if (h) {
                b.vy[p] = vy;
                b.vz[p] = vz;
            }
            bad |= !(isfinite(vx) && isfinite(vy) && isfinite(vz));
            c = cell_of<R>(d, y) >> d.key_shift;
            cellp[p] = c;
        } else {
            c = cellp[p];
        }
        atomicAdd(&hist[c], 1);
    }
    if (kMove && bad) atomicOr(&blk_bad, 1);
    __syncthreads();
    const gptr<int32_t> row = gmem(d.counts) + (size_t)w.y * nk;
    for (int c = threadIdx.x; c < nk; c += blockDim.x) row[c] = hist[c];
    // error path only: a non-finite velocity was seen in this tile
    if (kMove && threadIdx.x == 0 && blk_bad) atomicOr(&d.sc->status, 1);
}

// ------------------------------------------------------- column scans
// The tile histograms form a (tiles x nkeys) matrix stored tile-major.  The
// scatter base of (tile t, key c) is koffset[c] + sum_{t' < t} count[t'][c];
// it is built column-wise in segments of kSegTiles tiles so that every access
// is coalesced across consecutive keys.
__global__ __launch_bounds__(kColThreads) void k_colsum(const InstDesc* __restrict__ descs,
                                                      const int4* __restrict__ work) {
    const int4 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int c = w.y * kColThreads + (int)threadIdx.x;
    const int nk = d.nkeys;
    if (c >= nk) return;
    const int t0 = w.z * kSegTiles, t1 = min(t0 + kSegTiles, d.tiles);
    const gptr<int32_t> cnt = gmem(d.counts);
    // every load of the segment issued before the first is used
    int v[kSegTiles];
#pragma unroll
    for (int u = 0; u < kSegTiles; ++u) v[u] = t0 + u < t1 ? cnt[(size_t)(t0 + u) * nk + c] : 0;
    int sum = 0;
#pragma unroll
    for (int u = 0; u < kSegTiles; ++u) sum += v[u];
    d.segsum[(size_t)w.z * nk + c] = sum;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Per instance: for each sort key, the segment sums become their exclusive
// prefix over segments and kcount[c] the column total; koffset = exclusive
// scan of kcount in key order.  Also advances the instance's step counter
// (and the sampled-step count).  The segment loads of a cell are independent,
// so they are issued together.
// Thread 0's bookkeeping of the step's injections at the scan of an open
// instance (they were drawn by the count pass), before its live count is
// replaced: their number and the remainder carried on.  Returns the slots in
// use during the step (N when closed).
__device__ __forceinline__ int book_injections(const InstDesc& d) {
    if (!d.open) return d.N;
    OpenState* os = d.os;
    const int live = os->n_live;
    double rem;
    bool clipped;
    const int n = injections(d, live, os->inj_rem, rem, clipped);
    if (clipped) atomicOr(&d.sc->status, 8);
    os->inj_rem = rem;
    os->n_injected += n;
    os->n_used = live + n;
    return live + n;
}

// Thread 0: the instance's step counter (and the sampled-step count).
__device__ __forceinline__ void advance_step(const InstDesc& d) {
    const int64_t s = d.sc->step_done + 1;
    d.sc->step_done = s;
    if ((d.phase_mask & kPhaseSample) && s > d.n_transient) d.sc->n_sampled += 1;
}

__global__ __launch_bounds__(kScanThreads) void k_scan(const InstDesc* __restrict__ descs,
                                                     int do_scan) {
    const InstDesc& d = descs[blockIdx.x];
    __shared__ int wsum[kScanThreads / 64];
    __shared__ int sh_used;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (do_scan) {
        if (tid == 0) sh_used = book_injections(d);
        const int Cc = d.nkeys, nseg = d.nseg;
        const gptr<int32_t> seg = gmem(d.segsum);
        // column sums of the segments -> exclusive prefix over segments, key
        // c = tid + j * kScanThreads (a wavefront's loads are 64 adjacent
        // keys), 32 segments' loads in flight at a time
        constexpr int B = 32;
        for (int c = tid; c < Cc; c += kScanThreads) {
            int tot = 0;
            for (int g = 0; g < nseg; g += B) {
                int v[B];
#pragma unroll
                for (int u = 0; u < B; ++u) v[u] = g + u < nseg ? seg[(size_t)(g + u) * Cc + c] : 0;
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    if (g + u < nseg) seg[(size_t)(g + u) * Cc + c] = tot;
                    tot += v[u];
                }
            }
            d.kcount[c] = tot;
        }
        // the key totals are read back by other threads below
        __threadfence_block();
        __syncthreads();
        const int per = (Cc + kScanThreads - 1) / kScanThreads;
        const int c0 = min(tid * per, Cc), c1 = min(c0 + per, Cc);
        int local = 0;
        for (int c = c0; c < c1; ++c) local += d.kcount[c];
        const int incl = wave_incl_scan(local, lane);
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        if (wv == 0) {
            int v = lane < kScanThreads / 64 ? wsum[lane] : 0;
            v = wave_incl_scan(v, lane);
            if (lane < kScanThreads / 64) wsum[lane] = v;
        }
        __syncthreads();
        int run = incl - local + (wv ? wsum[wv - 1] : 0);
        for (int c = c0; c < c1; ++c) {
            d.koffset[c] = run;
            // an open instance's last key holds the particles that left: the
            // live ones are those before it
            if (d.open && c == Cc - 1) {
                d.os->n_live = run;
                d.os->n_deleted += d.kcount[c];
            }
            run += d.kcount[c];
        }
        if (tid == kScanThreads - 1 && wsum[kScanThreads / 64 - 1] != sh_used)
            atomicOr(&d.sc->status, 2);
    }
    __syncthreads();
    if (tid == 0) advance_step(d);
}

// Per-tile scatter bases of a segment: koffset[c] + the prefix of the earlier
// segments + the counts of the earlier tiles of this segment.
__global__ __launch_bounds__(kColThreads) void k_colprefix(const InstDesc* __restrict__ descs,
                                                         const int4* __restrict__ work) {
    const int4 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int c = w.y * kColThreads + (int)threadIdx.x;
    const int nk = d.nkeys;
    if (c >= nk) return;
    int run = d.koffset[c] + gmem(d.segsum)[(size_t)w.z * nk + c];
    const int t0 = w.z * kSegTiles, t1 = min(t0 + kSegTiles, d.tiles);
    const gptr<int32_t> cnt = gmem(d.counts);
    // the segment's counts are all loaded before the first base is stored
    // (a load after a store to the same array waited for it)
    int v[kSegTiles];
#pragma unroll
    for (int u = 0; u < kSegTiles; ++u) v[u] = t0 + u < t1 ? cnt[(size_t)(t0 + u) * nk + c] : 0;
#pragma unroll
    for (int u = 0; u < kSegTiles; ++u) {
        if (t0 + u < t1) cnt[(size_t)(t0 + u) * nk + c] = run;
        run += v[u];
    }
}

// --------------------------------------------------------------- scatter
// Stable scatter of one tile by a workgroup of four wavefronts, each owning a
// contiguous quarter of the tile.  A first pass counts each quarter's cells
// into that wavefront's LDS table; the base of (quarter q, cell c) is then
// the tile's base for c plus the counts of c in quarters before q.  In the
// second pass every wavefront walks its quarter in rounds of 64 slots in slot
// order.  Lanes holding the same cell are found with bit-sliced ballots (one
// ballot per bit of the cell index, so the cost does not depend on how many
// distinct cells a round holds); a lane's rank is the number of lower lanes
// with its cell, and only the owning wavefront advances its table, so a
// round needs no barrier.  The destination of every slot is base + (number
// of earlier slots of the tile with the same cell): exactly a stable
// counting sort.  "Cell" here means the instance's sort key: the collision
// cell, or a bucket of cells whose sort the collide kernel finishes.
//
// Tiles of at most stage_max slots are first laid out in LDS in destination
// order (the tile's cells in order, each cell's slots in slot order) and then
// written out by consecutive threads, so each cell's run from the tile
// leaves as one contiguous write instead of one partial cache line per slot;
// this matters at high Kn, where the slots of a tile spread over many cells.
template <class R>
__global__ __launch_bounds__(kParticleThreads) void k_scatter(const InstDesc* __restrict__ descs,
                                                             const int2* __restrict__ work,
                                                             int stage_max) {
    extern __shared__ int tables[];  // kScatterWaves x Cc, then Cc, then the staging area
    const int2 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int Cc = d.nkeys;  // the sort keys play the part of cells here
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t s = d.sc->step_done;
    const P4<R> src = particles<R>(d, (int)((s - 1) & 1));
    const P4<R> dst = particles<R>(d, (int)(s & 1));
    const int start = w.y * d.tile_items;
    const int end = min(start + d.tile_items, d.N);
    const bool staged = d.tile_items <= stage_max;
    int* delta = tables + kScatterWaves * Cc;           // tile base minus local base, per cell
    int* stage_pos = delta + Cc;                         // staged: destination of each local slot
    // staged: 4 x stage_max record words, 16-byte aligned
    R* stage_rec = (R*)(tables + (((kScatterWaves + 1) * Cc + stage_max + 3) & ~3));
    for (int k = threadIdx.x; k < kScatterWaves * Cc; k += blockDim.x) tables[k] = 0;
    const int quarter = (((end - start) + kScatterWaves - 1) / kScatterWaves + 63) / 64 * 64;
    const int q0 = min(start + wv * quarter, end), q1 = min(q0 + quarter, end);
    int* mine = tables + wv * Cc;
    const gptr<int32_t> cellp = gmem(d.cell);
    __syncthreads();
    for (int i = q0 + lane; i < q1; i += 64) atomicAdd(&mine[cellp[i]], 1);
    __syncthreads();
    const gptr<int32_t> brow = gmem(d.counts) + (size_t)w.y * Cc;
    // per-wavefront bases; when staged, the tile's count of each cell goes
    // to delta[] (which exists only then)
    for (int c = threadIdx.x; c < Cc; c += blockDim.x) {
        const int b = brow[c];
        int run = b;
        for (int q = 0; q < kScatterWaves; ++q) {
            const int v = tables[q * Cc + c];
            tables[q * Cc + c] = run;
            run += v;
        }
        if (staged) delta[c] = run - b;
    }
    if (staged) {
        // exclusive scan of the tile's cell counts over cells: the local base
        // of each cell; delta = tile base - local base
        __shared__ int wsum[kParticleThreads / 64];
        __syncthreads();
        const int per = (Cc + (int)blockDim.x - 1) / (int)blockDim.x;
        const int a0 = min((int)threadIdx.x * per, Cc), a1 = min(a0 + per, Cc);
        int local = 0;
        for (int c = a0; c < a1; ++c) local += delta[c];
        int incl = local;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int run = incl - local;
        for (int q = 0; q < wv; ++q) run += wsum[q];
        for (int c = a0; c < a1; ++c) {
            const int cnt = delta[c];
            delta[c] = brow[c] - run;
            run += cnt;
        }
    }
    __syncthreads();
    const unsigned long long lt = lanes_below(lane);
    const int nbits = Cc > 1 ? 32 - __builtin_clz((unsigned)(Cc - 1)) : 0;
    for (int base = q0; base < q1; base += 64) {
        const int i = base + lane;
        const bool valid = i < q1;
        int c = 0;
        R ry = R(0), rvx = R(0), rvy = R(0), rvz = R(0);
        if (valid) {
            c = cellp[i];
            ry = src.y[i];
            rvx = src.vx[i];
            rvy = src.vy[i];
            rvz = src.vz[i];
        }
        unsigned long long m = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (c >> b) & 1;
            const unsigned long long bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        if (valid) {
            const int pos = mine[c] + __popcll(m & lt);
            // every lane of the group reads the base before its leader
            // (lowest lane) advances it: same wavefront, program order
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if ((m & lt) == 0ull) mine[c] = pos + __popcll(m);
            if (staged) {
                const int l = pos - delta[c];
                stage_pos[l] = pos;
                stage_rec[l] = ry;
                stage_rec[stage_max + l] = rvx;
                stage_rec[2 * stage_max + l] = rvy;
                stage_rec[3 * stage_max + l] = rvz;
            } else {
                dst.y[pos] = ry;
                dst.vx[pos] = rvx;
                dst.vy[pos] = rvy;
                dst.vz[pos] = rvz;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (staged) {
        __syncthreads();
        const int n = end - start;
        for (int l = threadIdx.x; l < n; l += blockDim.x) {
            const int pos = stage_pos[l];
            dst.y[pos] = stage_rec[l];
            dst.vx[pos] = stage_rec[stage_max + l];
            dst.vy[pos] = stage_rec[2 * stage_max + l];
            dst.vz[pos] = stage_rec[3 * stage_max + l];
        }
    }
}

// ------------------------------------------------- count + move-scatter
// The default step splits the move differently: a particle's new position,
// and so its cell and sort key, depends only on y, vy and the normal speeds
// drawn at wall hits (never on vx or vz), so a first pass can histogram the
// keys of a tile from y and vy alone, without writing anything.  After the
// scans, k_move_scatter reads each record once, repeats the same move in
// full (the same arithmetic and draws, so the same key) and writes the moved
// record straight to its sorted slot.

// Flight of the position alone: the sort key of the y that move_one would
// produce.
template <class R, bool kOpen>
__device__ __forceinline__ int flight_key(const InstDesc& d, uint32_t step, uint32_t slot, R y, R vy) {
    R vx = R(0), vz = R(0);
    bool gone = false;
    move_one<R, kOpen, false>(d, step, slot, y, vx, vy, vz, gone);
    return key_of<R, kOpen>(d, y, gone);
}

template <class R, bool kOpen>
__global__ __launch_bounds__(kParticleThreads) void k_count(const InstDesc* __restrict__ descs,
                                                           const int2* __restrict__ work) {
    extern __shared__ int hist[];
    const int2 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int nk = d.nkeys;
    for (int c = threadIdx.x; c < nk; c += blockDim.x) hist[c] = 0;
    __syncthreads();
    const int64_t s = d.sc->step_done + 1;
    const P4<R> b = particles<R>(d, (int)((s - 1) & 1));
    const int start = w.y * d.tile_items;
    const Slots sl = slots_before_scan<kOpen>(d);
    const int end_all = min(start + d.tile_items, sl.used);
    const int end = min(end_all, sl.live);
    constexpr int U = 4;
    for (int p0 = start + (int)threadIdx.x; p0 < end; p0 += U * kParticleThreads) {
        R y[U], vy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u * kParticleThreads;
            y[u] = vy[u] = R(0);
            if (p < end) {
                y[u] = b.y[p];
                vy[u] = b.vy[p];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u * kParticleThreads;
            if (p < end) atomicAdd(&hist[flight_key<R, kOpen>(d, (uint32_t)s, (uint32_t)p, y[u], vy[u])], 1);
        }
    }
    // an open instance's injections in this tile: drawn, stored for the
    // move-scatter pass and counted like the others
    if (kOpen)
        for (int p = max(start, sl.live) + (int)threadIdx.x; p < end_all; p += kParticleThreads) {
            R y, vx, vy, vz;
            inject_state<R>(d, (uint32_t)s, p - sl.live, y, vx, vy, vz);
            b.y[p] = y;
            b.vx[p] = vx;
            b.vy[p] = vy;
            b.vz[p] = vz;
            atomicAdd(&hist[flight_key<R, kOpen>(d, (uint32_t)s, (uint32_t)p, y, vy)], 1);
        }
    __syncthreads();
    const gptr<int32_t> row = gmem(d.counts) + (size_t)w.y * nk;
    constexpr int held = kScatterWaves * 64 * (sizeof(R) == 4 ? kScatterRegs32 : kScatterRegs64);
    if (d.tile_items <= held) {
        for (int c = threadIdx.x; c < nk; c += blockDim.x) row[c] = hist[c];
        return;
    }
    // a tile larger than the move-scatter's registers also records its
    // smallest and largest key, for the wide-tile scatter's tables (an empty
    // tile records an empty range)
    int kmn = INT32_MAX, kmx = -1;
    for (int c = threadIdx.x; c < nk; c += blockDim.x) {
        const int v = hist[c];
        row[c] = v;
        if (v) {
            kmn = min(kmn, c);
            kmx = max(kmx, c);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        kmn = min(kmn, __shfl_xor(kmn, o, 64));
        kmx = max(kmx, __shfl_xor(kmx, o, 64));
    }
    __shared__ int kr[2];
    if (threadIdx.x == 0) {
        kr[0] = INT32_MAX;
        kr[1] = -1;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&kr[0], kmn);
        atomicMax(&kr[1], kmx);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        d.tkeys[2 * w.y] = kr[0];
        d.tkeys[2 * w.y + 1] = kr[1];
    }
}

// The column scans in one workgroup per instance, for lanes whose instances
// have small count matrices (tiles x keys within the LDS of one workgroup,
// at most kScanThreads keys): the tile histograms of k_count are read into
// LDS and scanned there, which gives the per-tile scatter bases, key counts
// and offsets and the bookkeeping of k_colsum, k_scan and k_colprefix: one
// launch instead of three.
__global__ __launch_bounds__(kScanThreads) void k_scan_small(const InstDesc* __restrict__ descs) {
    extern __shared__ int hist[];  // tiles x keys: counts, then prefixes over the tiles
    __shared__ int wsum[kScanThreads / 64];
    __shared__ int sh_used;
    const InstDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nk = d.nkeys, T = d.tiles;
    const gptr<int32_t> cnt = gmem(d.counts);
    for (int i = tid; i < T * nk; i += blockDim.x) hist[i] = cnt[i];
    if (tid == 0) sh_used = book_injections(d);
    __syncthreads();
    // key c = tid: exclusive prefix over the tiles and the key's total
    const int c = tid;
    int tot = 0;
    if (c < nk)
        for (int t = 0; t < T; ++t) {
            const int v = hist[t * nk + c];
            hist[t * nk + c] = tot;
            tot += v;
        }
    const int incl = wave_incl_scan(tot, lane);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        int v = lane < kScanThreads / 64 ? wsum[lane] : 0;
        v = wave_incl_scan(v, lane);
        if (lane < kScanThreads / 64) wsum[lane] = v;
    }
    __syncthreads();
    if (c < nk) {
        const int off = incl - tot + (wv ? wsum[wv - 1] : 0);
        d.kcount[c] = tot;
        d.koffset[c] = off;
        // an open instance's last key holds the particles that left: the
        // live ones are those before it
        if (d.open && c == nk - 1) {
            d.os->n_live = off;
            d.os->n_deleted += tot;
        }
        for (int t = 0; t < T; ++t) cnt[(size_t)t * nk + c] = off + hist[t * nk + c];
    }
    if (tid == kScanThreads - 1 && wsum[kScanThreads / 64 - 1] != sh_used) atomicOr(&d.sc->status, 2);
    __syncthreads();
    if (tid == 0) advance_step(d);
}

// The column scans in one workgroup per instance for count matrices too
// large for LDS whose segment sums fit it (lanes where every instance has at
// most kSegScanEntries (segments + 1) x keys): the work of k_colsum,
// k_scan and k_colprefix in one launch.  Items are (64 adjacent keys, one
// segment of kSegTiles tiles), spread over the wavefronts; each issues its
// segment's loads before using them.  First the segment sums go to LDS, then
// each key's exclusive prefix over the segments, its total and offset, and
// last each tile's scatter bases, written over its counts.
__global__ __launch_bounds__(kScanThreads) void k_scan_seg(const InstDesc* __restrict__ descs) {
    extern __shared__ int seg[];  // nseg x keys: segment sums, then their prefixes; then keys: offsets
    __shared__ int wsum[kScanThreads / 64];
    __shared__ int sh_used;
    const InstDesc& d = descs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int nw = kScanThreads / 64;
    const int nk = d.nkeys, T = d.tiles, NS = d.nseg;
    const int KC = (nk + 63) >> 6, items = KC * NS;
    int* koff = seg + (size_t)NS * nk;
    const gptr<int32_t> cnt = gmem(d.counts);
    if (tid == 0) sh_used = book_injections(d);
    for (int it = wv; it < items; it += nw) {
        const int c = (it % KC) * 64 + lane, sg = it / KC;
        const int t0 = sg * kSegTiles, t1 = min(t0 + kSegTiles, T);
        int v[kSegTiles];
#pragma unroll
        for (int u = 0; u < kSegTiles; ++u) v[u] = (c < nk && t0 + u < t1) ? cnt[(size_t)(t0 + u) * nk + c] : 0;
        int sum = 0;
#pragma unroll
        for (int u = 0; u < kSegTiles; ++u) sum += v[u];
        if (c < nk) seg[sg * nk + c] = sum;
    }
    __syncthreads();
    // per key: exclusive prefix over the segments and the total
    for (int c = tid; c < nk; c += kScanThreads) {
        int tot = 0;
        for (int sg = 0; sg < NS; ++sg) {
            const int x = seg[sg * nk + c];
            seg[sg * nk + c] = tot;
            tot += x;
        }
        koff[c] = tot;  // the key's total until the scan below
        d.kcount[c] = tot;
    }
    __syncthreads();
    // exclusive scan of the totals in key order
    const int per = (nk + kScanThreads - 1) / kScanThreads;
    const int c0 = min(tid * per, nk), c1 = min(c0 + per, nk);
    int local = 0;
    for (int c = c0; c < c1; ++c) local += koff[c];
    const int incl = wave_incl_scan(local, lane);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        int x = lane < nw ? wsum[lane] : 0;
        x = wave_incl_scan(x, lane);
        if (lane < nw) wsum[lane] = x;
    }
    __syncthreads();
    int run = incl - local + (wv ? wsum[wv - 1] : 0);
    for (int c = c0; c < c1; ++c) {
        const int tot = koff[c];
        koff[c] = run;
        d.koffset[c] = run;
        // an open instance's last key holds the particles that left: the
        // live ones are those before it
        if (d.open && c == nk - 1) {
            d.os->n_live = run;
            d.os->n_deleted += tot;
        }
        run += tot;
    }
    if (tid == kScanThreads - 1 && wsum[nw - 1] != sh_used) atomicOr(&d.sc->status, 2);
    __syncthreads();
    // per-tile scatter bases
    for (int it = wv; it < items; it += nw) {
        const int c = (it % KC) * 64 + lane, sg = it / KC;
        const int t0 = sg * kSegTiles, t1 = min(t0 + kSegTiles, T);
        int v[kSegTiles];
#pragma unroll
        for (int u = 0; u < kSegTiles; ++u) v[u] = (c < nk && t0 + u < t1) ? cnt[(size_t)(t0 + u) * nk + c] : 0;
        if (c < nk) {
            int r = koff[c] + seg[sg * nk + c];
#pragma unroll
            for (int u = 0; u < kSegTiles; ++u) {
                if (t0 + u < t1) cnt[(size_t)(t0 + u) * nk + c] = r;
                r += v[u];
            }
        }
    }
    __syncthreads();
    if (tid == 0) advance_step(d);
}

// Records per lane k_move_scatter holds in registers (tiles up to
// 256 * this many slots take the one-read path).
template <class R> struct ScatterRegs {
    static constexpr int value = sizeof(R) == 4 ? kScatterRegs32 : kScatterRegs64;
};

template <class R> struct WideRecs {
    static constexpr int value = sizeof(R) == 4 ? kWideRecs32 : kWideRecs64;
};

// Ints of the wide-tile LDS layout before its staged records (kept a
// multiple of four, so the records are 16-byte aligned).
__host__ __device__ constexpr int wide_ints(int nk, int J) {
    return (nk + 2 * J * kScatterWaves * kWideKeys + 2 * kWideKeys + 4 + J * kParticleThreads + 3) & ~3;
}

// Move and stable scatter of a tile larger than k_move_scatter holds in
// registers (a separate kernel, so that its registers do not cost the other
// one occupancy; the runtime lists its tiles after the others).  The
// workgroup walks the tile in chunks of 256 * J slots.  A chunk is read and
// moved in registers and ranked by key over the whole workgroup in slot
// order (round j, wavefront, lane): within each (round, wavefront) group the
// lanes of equal key are found by one ballot per key bit, the group's count
// of each key goes to an LDS table, and one wavefront scans that table key
// by key, 64 keys per pass (a chunk whose keys span more takes more passes).
// The chunk is laid out in LDS in destination order and written from there,
// so each key's run in the chunk is stored to consecutive addresses rather
// than a few records per round.  The next destination of each key lives in
// one LDS table for the whole tile, started from the tile's scatter bases
// (for the keys from the tile's smallest on, as k_count recorded it), so the
// tile needs no histogram of its own here.  Count entries carry the number
// of the pass that wrote them, which spares clearing the table between
// passes.
template <class R, bool kOpen>
__global__ __launch_bounds__(kParticleThreads) void k_move_scatter_wide(const InstDesc* __restrict__ descs,
                                                                       const int2* __restrict__ work) {
    extern __shared__ int lds[];
    const int2 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int tile = w.y;
    const int64_t s = d.sc->step_done;
    const P4<R> src = particles<R>(d, (int)((s - 1) & 1));
    const P4<R> dst = particles<R>(d, (int)(s & 1));
    const int start = tile * d.tile_items;
    const int end = min(start + d.tile_items, slots_after_scan<kOpen>(d));
    constexpr int J = WideRecs<R>::value;
    constexpr int C = J * kParticleThreads;
    constexpr int G = J * kScatterWaves;
    const int nk = d.nkeys;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // next destination of keys tk0 .. tk0 + nrun - 1 of the tile; keys past
    // them (a tile spanning more than kWideRunKeys) keep theirs in the
    // tile's row of the count matrix, updated with atomics
    const int tk0 = d.tkeys[2 * tile], tk1 = d.tkeys[2 * tile + 1];
    const int nrun = min(max(tk1 - tk0 + 1, 0), kWideRunKeys);
    const int nrt = min(nk, kWideRunKeys);  // the table's size in the launch's LDS layout
    int* run = lds;
    int* cnt = run + nrt;              // G x 64: (pass << 8) | count per group and key
    int* pre = cnt + G * kWideKeys;    // G x 64: records of the key in earlier groups of the chunk
    int* koff = pre + G * kWideKeys;   // 64: the key's first staging index
    int* dlt = koff + kWideKeys;       // 64: destination minus staging index
    int* red = dlt + kWideKeys;        // chunk key range, two chunks alternating
    int* spos = red + 4;               // C: destination of each staged record
    R* srec = (R*)(lds + wide_ints(nrt, J));  // 4 x C: y, vx, vy, vz in destination order
    const gptr<int32_t> brow = gmem(d.counts) + (size_t)tile * nk;
    for (int c = tid; c < nrun; c += kParticleThreads) run[c] = brow[tk0 + c];
    for (int e = tid; e < G * kWideKeys; e += kParticleThreads) cnt[e] = 0;
    if (tid < 4) red[tid] = (tid & 1) ? -1 : INT32_MAX;
    __syncthreads();
    const unsigned long long lt = lanes_below(lane);
    int bad = 0, pass = 0, nbase = 0;
    // the next chunk's records are loaded while this one is ranked and
    // written (the barriers wait for LDS operations only)
    R ny[J], nx[J], nv[J], nz[J];
    auto load_chunk = [&](int cb) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = cb + j * kParticleThreads + tid;
            ny[j] = nx[j] = nv[j] = nz[j] = R(0);
            if (i < end) {
                ny[j] = src.y[i];
                nx[j] = src.vx[i];
                nv[j] = src.vy[i];
                nz[j] = src.vz[i];
            }
        }
    };
    if (start < end) load_chunk(start);
    for (int cb = start, ci = 0; cb < end; cb += C, ++ci) {
        const int par = 2 * (ci & 1);
        R ry[J], rx[J], rv[J], rz[J];
        int key[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            ry[j] = ny[j];
            rx[j] = nx[j];
            rv[j] = nv[j];
            rz[j] = nz[j];
        }
        if (cb + C < end) load_chunk(cb + C);
        int kmn = INT32_MAX, kmx = -1;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int i = cb + j * kParticleThreads + tid;
            key[j] = -1;
            if (i < end) {
                bool gone = false;
                move_one<R, kOpen>(d, (uint32_t)s, (uint32_t)i, ry[j], rx[j], rv[j], rz[j], gone);
                bad |= !(isfinite(rx[j]) && isfinite(rv[j]) && isfinite(rz[j]));
                key[j] = key_of<R, kOpen>(d, ry[j], gone);
                kmn = min(kmn, key[j]);
                kmx = max(kmx, key[j]);
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            kmn = min(kmn, __shfl_xor(kmn, o, 64));
            kmx = max(kmx, __shfl_xor(kmx, o, 64));
        }
        if (lane == 0 && kmx >= 0) {
            atomicMin(&red[par], kmn);
            atomicMax(&red[par + 1], kmx);
        }
        __syncthreads();
        const int kmin = red[par], kmax = red[par + 1];
        // the other chunk's range was read before the last barrier
        if (tid == 0) {
            red[2 - par] = INT32_MAX;
            red[3 - par] = -1;
        }
        const int nrec = min(C, end - cb);
        nbase = 0;
        for (int w0 = kmin; w0 <= kmax; w0 += kWideKeys) {
            ++pass;
            int rank[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int kl = key[j] - w0;
                const bool in = key[j] >= 0 && kl >= 0 && kl < kWideKeys;
                unsigned long long m = __ballot(in);
#pragma unroll
                for (int b = 0; b < 6; ++b) {
                    const bool bit = (kl >> b) & 1;
                    const unsigned long long bal = __ballot(bit);
                    m &= bit ? bal : ~bal;
                }
                rank[j] = __popcll(m & lt);
                if (in && rank[j] == 0) cnt[(j * kScatterWaves + wv) * kWideKeys + kl] = (pass << 8) | __popcll(m);
            }
            __syncthreads();
            if (wv == 0) {
                int tot = 0;
                for (int g = 0; g < G; ++g) {
                    const int v = cnt[g * kWideKeys + lane];
                    pre[g * kWideKeys + lane] = tot;
                    tot += (v >> 8) == pass ? (v & 255) : 0;
                }
                const int incl = wave_incl_scan(tot, lane);
                const int ko = nbase + incl - tot;
                koff[lane] = ko;
                if (tot > 0) {  // some record has key w0 + lane, so it is < nk
                    const unsigned kr = (unsigned)(w0 + lane - tk0);
                    int r;
                    if (kr < (unsigned)nrun) {
                        r = run[kr];
                        run[kr] = r + tot;
                    } else {
                        r = atomicAdd((int*)(brow + (w0 + lane)), tot);
                    }
                    dlt[lane] = r - ko;
                }
                nbase += __shfl(incl, 63, 64);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int kl = key[j] - w0;
                if (key[j] >= 0 && kl >= 0 && kl < kWideKeys) {
                    int l = koff[kl] + pre[(j * kScatterWaves + wv) * kWideKeys + kl] + rank[j];
                    const int pos = l + dlt[kl];
                    if (l < 0 || l >= nrec) {
                        bad |= 2;
                        l = l < 0 ? 0 : nrec - 1;
                    }
                    spos[l] = pos;
                    srec[l] = ry[j];
                    srec[C + l] = rx[j];
                    srec[2 * C + l] = rv[j];
                    srec[3 * C + l] = rz[j];
                }
            }
        }
        __syncthreads();
        for (int l = tid; l < nrec; l += kParticleThreads) {
            int pos = spos[l];
            if (pos < 0 || pos >= d.ncap) {
                bad |= 2;
                pos = pos < 0 ? 0 : d.ncap - 1;
            }
            dst.y[pos] = srec[l];
            dst.vx[pos] = srec[C + l];
            dst.vy[pos] = srec[2 * C + l];
            dst.vz[pos] = srec[3 * C + l];
        }
    }
    // error path only: bit 0 a non-finite velocity, bit 2 a slot out of range
    if (bad) atomicOr(&d.sc->status, (bad & 1) | ((bad & 2) << 1));
}

// Move and stable scatter of one tile: the same quarter-per-wavefront
// ranking as k_scatter, with the keys coming from the move.  A tile of at
// most 256 * ScatterRegs slots is read once into registers, moved (wall
// re-emissions queued and run together), counted and placed round by round;
// larger tiles are k_move_scatter_wide's.  A sorted position outside [0, N)
// (only possible if the counts and this pass disagreed) is clamped and
// flagged.
template <class R, bool kOpen>
__global__ __launch_bounds__(kParticleThreads) void k_move_scatter(const InstDesc* __restrict__ descs,
                                                                  const int2* __restrict__ work,
                                                                  int stage_max) {
    constexpr int K = ScatterRegs<R>::value;
    extern __shared__ int tables[];  // kScatterWaves x nkeys, then nkeys, then the staging area
    __shared__ int blk_bad;
    const int2 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int nk = d.nkeys;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t s = d.sc->step_done;
    const P4<R> src = particles<R>(d, (int)((s - 1) & 1));
    const P4<R> dst = particles<R>(d, (int)(s & 1));
    const int start = w.y * d.tile_items;
    const int end = min(start + d.tile_items, slots_after_scan<kOpen>(d));
    const bool staged = d.tile_items <= stage_max;
    int* delta = tables + kScatterWaves * nk;
    int* stage_pos = delta + nk;
    R* stage_rec = (R*)(tables + (((kScatterWaves + 1) * nk + stage_max + 3) & ~3));
    for (int k = threadIdx.x; k < kScatterWaves * nk; k += blockDim.x) tables[k] = 0;
    if (threadIdx.x == 0) blk_bad = 0;
    const int quarter = (((end - start) + kScatterWaves - 1) / kScatterWaves + 63) / 64 * 64;
    const int q0 = min(start + wv * quarter, end), q1 = min(q0 + quarter, end);
    int* mine = tables + wv * nk;
    // the tile's scatter bases, read now so that their latency hides behind
    // the move (thread c holds key c's base when there are at most 256 keys)
    const gptr<int32_t> brow = gmem(d.counts) + (size_t)w.y * nk;
    const int my_base = (int)threadIdx.x < nk ? (int)brow[threadIdx.x] : 0;
    auto base_of = [&](int c) { return c == (int)threadIdx.x ? my_base : (int)brow[c]; };
    __syncthreads();
    R ry[K], rx[K], rv[K], rz[K];
    int key[K];
    int bad = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = q0 + 64 * k + lane;
        ry[k] = rx[k] = rv[k] = rz[k] = R(0);
        if (i < q1) {
            ry[k] = src.y[i];
            rx[k] = src.vx[i];
            rv[k] = src.vy[i];
            rz[k] = src.vz[i];
        }
    }
    // Straight flights at once; records that reach a plate are queued
    // in this wavefront's share of the (not yet used) staging area and
    // re-emitted together, 64 at a time, instead of once per round in
    // which any lane hits.  Queue overflow is handled in place.
    const int qcap = staged ? stage_max / 5 : 0;
    int* qslot = stage_pos + wv * (stage_max / 4);
    R* qt = stage_rec + wv * stage_max;
    R* qy = qt + qcap;
    R* qx = qy + qcap;
    R* qv = qx + qcap;
    R* qz = qv + qcap;
    int nq = 0, jq[K];
    unsigned hitm = 0, gonem = 0;  // queued records; records that left the domain
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = q0 + 64 * k + lane;
        bool hit = false, top = false, gone = false;
        R tl = R(0);
        jq[k] = 0;
        if (i < q1) hit = !flight_start<R, kOpen>(d, ry[k], rx[k], rv[k], tl, top, gone);
        if (gone) gonem |= 1u << k;
        const unsigned long long hm = __ballot(hit);
        if (hit) {
            const int j = nq + __popcll(hm & lanes_below(lane));
            if (j < qcap) {
                qslot[j] = i;
                qt[j] = top ? tl : -tl;  // the time left is > 0; its sign keeps the plate
                jq[k] = j;
                hitm |= 1u << k;
            } else {
                bool gone2 = false;
                flight_from_wall<R, kOpen>(d, (uint32_t)s, (uint32_t)i, top, tl, ry[k], rx[k], rv[k],
                                           rz[k], gone2);
                if (gone2) gonem |= 1u << k;
            }
        }
        nq += __popcll(hm);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int nproc = min(nq, qcap);
    for (int b0 = 0; b0 < nproc; b0 += 64) {
        const int j = b0 + lane;
        if (j < nproc) {
            const R tt = qt[j];
            R y = R(0), vx = R(0), vy = R(0), vz = R(0);
            bool gone3 = false;
            flight_from_wall<R, kOpen>(d, (uint32_t)s, (uint32_t)qslot[j], tt > R(0),
                                       tt > R(0) ? tt : -tt, y, vx, vy, vz, gone3);
            qy[j] = gone3 ? R(-1) : y;  // a flight ends at y >= 0: -1 marks one that left
            qx[j] = vx;
            qv[j] = vy;
            qz[j] = vz;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = q0 + 64 * k + lane;
        key[k] = 0;
        if ((hitm >> k) & 1u) {
            const int j = jq[k];
            ry[k] = qy[j];
            rx[k] = qx[j];
            rv[k] = qv[j];
            rz[k] = qz[j];
            if (kOpen && ry[k] < R(0)) gonem |= 1u << k;
        }
        if (i < q1) {
            bad |= !(isfinite(rx[k]) && isfinite(rv[k]) && isfinite(rz[k]));
            key[k] = key_of<R, kOpen>(d, ry[k], (gonem >> k) & 1u);
            atomicAdd(&mine[key[k]], 1);
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nk; c += blockDim.x) {
        const int b = base_of(c);
        int run = b;
        for (int q = 0; q < kScatterWaves; ++q) {
            const int v = tables[q * nk + c];
            tables[q * nk + c] = run;
            run += v;
        }
        if (staged) delta[c] = run - b;
    }
    if (staged) {
        __shared__ int wsum[kParticleThreads / 64];
        __syncthreads();
        const int per = (nk + (int)blockDim.x - 1) / (int)blockDim.x;
        const int a0 = min((int)threadIdx.x * per, nk), a1 = min(a0 + per, nk);
        int local = 0;
        for (int c = a0; c < a1; ++c) local += delta[c];
        const int incl = wave_incl_scan(local, lane);
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int run = incl - local;
        for (int q = 0; q < wv; ++q) run += wsum[q];
        for (int c = a0; c < a1; ++c) {
            const int cnt = delta[c];
            delta[c] = base_of(c) - run;
            run += cnt;
        }
    }
    __syncthreads();
    const unsigned long long lt = lanes_below(lane);
    const int nbits = nk > 1 ? 32 - __builtin_clz((unsigned)(nk - 1)) : 0;
    const int n_tile = end - start;
    // rank one round of 64 slots and place the records
    auto place = [&](bool valid, int kk, R y, R vx, R vy, R vz) {
        unsigned long long m = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (kk >> b) & 1;
            const unsigned long long bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        if (valid) {
            int pos = mine[kk] + __popcll(m & lt);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if ((m & lt) == 0ull) mine[kk] = pos + __popcll(m);
            if (staged) {
                int l = pos - delta[kk];
                if (l < 0 || l >= n_tile) {
                    bad |= 2;
                    l = l < 0 ? 0 : n_tile - 1;
                }
                stage_pos[l] = pos;
                stage_rec[l] = y;
                stage_rec[stage_max + l] = vx;
                stage_rec[2 * stage_max + l] = vy;
                stage_rec[3 * stage_max + l] = vz;
            } else {
                if (pos < 0 || pos >= d.ncap) {
                    bad |= 2;
                    pos = pos < 0 ? 0 : d.ncap - 1;
                }
                dst.y[pos] = y;
                dst.vx[pos] = vx;
                dst.vy[pos] = vy;
                dst.vz[pos] = vz;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (q0 + 64 * k < q1) place(q0 + 64 * k + lane < q1, key[k], ry[k], rx[k], rv[k], rz[k]);
    if (bad) atomicOr(&blk_bad, bad);
    __syncthreads();
    if (staged) {
        for (int l = threadIdx.x; l < n_tile; l += blockDim.x) {
            int pos = stage_pos[l];
            if (pos < 0 || pos >= d.ncap) pos = pos < 0 ? 0 : d.ncap - 1;  // flagged above
            dst.y[pos] = stage_rec[l];
            dst.vx[pos] = stage_rec[stage_max + l];
            dst.vy[pos] = stage_rec[2 * stage_max + l];
            dst.vz[pos] = stage_rec[3 * stage_max + l];
        }
    }
    // error path only: bit 0 a non-finite velocity, bit 2 a slot out of range
    if (threadIdx.x == 0 && blk_bad) atomicOr(&d.sc->status, (blk_bad & 1) | ((blk_bad & 2) << 1));
}

// Debug path without sorting: the next buffer is a copy of the current one.
template <class R>
__global__ __launch_bounds__(kParticleThreads) void k_copy(const InstDesc* __restrict__ descs,
                                                          const int2* __restrict__ work) {
    const int2 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int64_t s = d.sc->step_done;
    const P4<R> src = particles<R>(d, (int)((s - 1) & 1));
    const P4<R> dst = particles<R>(d, (int)(s & 1));
    const int start = w.y * d.tile_items;
    const int end = min(start + d.tile_items, d.N);
    for (int p = start + (int)threadIdx.x; p < end; p += blockDim.x) {
        dst.y[p] = src.y[p];
        dst.vx[p] = src.vx[p];
        dst.vy[p] = src.vy[p];
        dst.vz[p] = src.vz[p];
    }
}

// ----------------------------------------------------- sampling helpers
struct Mom {
    double s[kMoments];
};

__device__ __forceinline__ void mom_zero(Mom& m) {
#pragma unroll
    for (int k = 0; k < kMoments; ++k) m.s[k] = 0.0;
}

// The deterministic mode's sums: separate products and additions, each
// rounded, as the sequential reference adds them.
__device__ __forceinline__ void mom_add(Mom& m, double x, double y, double z) {
    const double v2 = (x * x + y * y) + z * z;
    m.s[0] += 1.0;
    m.s[1] += x;
    m.s[2] += y;
    m.s[3] += z;
    m.s[4] += x * x;
    m.s[5] += y * y;
    m.s[6] += z * z;
    m.s[7] += x * y;
    m.s[8] += x * z;
    m.s[9] += y * z;
    m.s[10] += v2 * x;
    m.s[11] += v2 * y;
}

// The fast modes' sums: each product added with one fused multiply-add (one
// rounding instead of two, and half the FP64 instructions of the sampling).
// The stress sum before the collisions is fused the same way, so that with no
// collision it equals the vxvy sum after them to the last bit.
__device__ __forceinline__ void mom_add_fused(Mom& m, double x, double y, double z) {
    const double v2 = __builtin_fma(x, x, __builtin_fma(y, y, z * z));
    m.s[0] += 1.0;
    m.s[1] += x;
    m.s[2] += y;
    m.s[3] += z;
    m.s[4] = __builtin_fma(x, x, m.s[4]);
    m.s[5] = __builtin_fma(y, y, m.s[5]);
    m.s[6] = __builtin_fma(z, z, m.s[6]);
    m.s[7] = __builtin_fma(x, y, m.s[7]);
    m.s[8] = __builtin_fma(x, z, m.s[8]);
    m.s[9] = __builtin_fma(y, z, m.s[9]);
    m.s[10] = __builtin_fma(v2, x, m.s[10]);
    m.s[11] = __builtin_fma(v2, y, m.s[11]);
}

// ------------------------------------------------ collide (deterministic)
// NTC (Bird) per collision cell, one lane per cell and 64 cells per
// wavefront: M_real = N(N-1)/2 crmax K + rem candidates; each candidate draws
// a distinct uniform pair, raises crmax to its relative speed if larger, is
// accepted with probability c_r / crmax (hard spheres) and then scatters
// isotropically about the centre of mass.  Candidates run in order, so the
// result is the reference recipe's to the last bit.  The sampling step's
// FP64 sums of the cell follow in slot order: vxvy before the collisions, the
// twelve moments after them.
__global__ __launch_bounds__(64) void k_collide_det(const InstDesc* __restrict__ descs,
                                                   const int4* __restrict__ work, int do_collide) {
    const int4 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int c = w.y + (int)threadIdx.x;
    const int64_t s = d.sc->step_done;
    const bool sample = (d.phase_mask & kPhaseSample) && s > d.n_transient;
    uint32_t ncoll = 0;
    if (c < w.z) {
        const P4<double> b = particles<double>(d, (int)(s & 1));
        const int n = d.count[c], o = d.offset[c];
        const gptr<double> vx = b.vx + o;
        const gptr<double> vy = b.vy + o;
        const gptr<double> vz = b.vz + o;
        // the stress sum before the collisions, in slot order
        double pre = 0.0;
        if (sample)
            for (int q = 0; q < n; ++q) pre += vx[q] * vy[q];
        if (do_collide && n >= 2) {
            double crm = d.crmax[c];
            const double mreal = (((0.5 * (double)n) * (double)(n - 1)) * crm) * d.kntc + d.rem[c];
            const double mf = floor(mreal);
            d.rem[c] = mreal - mf;
            const int64_t M = (int64_t)mf;
            for (int64_t k = 0; k < M; ++k) {
                Stream st(d.key0, d.key1, (uint32_t)s, (uint32_t)c, (uint32_t)k, kTagColl);
                double ua, ub;
                Num<double>::uni2(st.next(), ua, ub);
                int i = (int)(ua * (double)n);
                if (i > n - 1) i = n - 1;
                int j = (int)(ub * (double)(n - 1));
                if (j > n - 2) j = n - 2;
                if (j >= i) ++j;
                const double crx = vx[i] - vx[j];
                const double cry = vy[i] - vy[j];
                const double crz = vz[i] - vz[j];
                const double cr = __builtin_sqrt((crx * crx + cry * cry) + crz * crz);
                if (cr > crm) crm = cr;
                double ua2, ub2;
                Num<double>::uni2(st.next(), ua2, ub2);
                if (ua2 * crm < cr) {
                    double dx, dy, dz;
                    sphere_point<double>(st, dx, dy, dz);
                    const double cmx = 0.5 * (vx[i] + vx[j]);
                    const double cmy = 0.5 * (vy[i] + vy[j]);
                    const double cmz = 0.5 * (vz[i] + vz[j]);
                    const double hh = 0.5 * cr;
                    vx[i] = cmx + hh * dx;
                    vy[i] = cmy + hh * dy;
                    vz[i] = cmz + hh * dz;
                    vx[j] = cmx - hh * dx;
                    vy[j] = cmy - hh * dy;
                    vz[j] = cmz - hh * dz;
                    ++ncoll;
                }
            }
            d.crmax[c] = crm;
            if (ncoll) d.ncoll[c] += ncoll;
        }
        if (sample) {
            Mom m;
            mom_zero(m);
            for (int q = 0; q < n; ++q) mom_add(m, vx[q], vy[q], vz[q]);
            m.s[kMomPreXY] = pre;
            double* a = d.acc + c;  // moment k of cell c at k * Cc + c
#pragma unroll
            for (int k = 0; k < kMoments; ++k) a[(size_t)k * d.Cc] += m.s[k];
        }
    }
}

// ------------------------------------------------------- collide (fast)
// The fast modes draw the same kind of NTC candidates as the sequential
// scheme (pair and acceptance uniform per candidate from the cell's
// counter-based stream) and run them either
//   - in groups of G lanes per cell (k_collide_bucket, G = 4..64) for
//     instances whose collision cells hold fewer than kCoopMin particles on
//     average, or
//   - with a whole workgroup per cell (k_collide_fast), in parallel rounds of
//     blockDim candidates,
// on velocities staged in LDS.  Candidates are numbered in draw order; one
// that shares a particle with a lower-numbered pending candidate waits for a
// later round (claims by atomicMin in an LDS table), so the candidates that
// touch a particle run in number order, as in the sequential scheme: NTC in
// distribution.  The acceptance test uses max(crmax at cell start, its own
// c_r); crmax is raised at the end of the cell.  Which path a cell takes, G
// and the round a candidate runs in do not change any particle's result, so
// states depend only on the instance's data and streams, not on the group,
// the launch shape or the workgroup a cell lands in.
// One pending candidate of a lane: its number, pair, acceptance uniform and
// (FP32) the post-collision direction drawn with it.
template <class R> struct Pend {
    int64_t k;
    int i, j;
    R acc;
    R dirz, dirp;  // FP32: cos(theta) in (-1, 1] and phi / 2pi in [0, 1)
};

template <class R> struct Cand;
template <> struct Cand<float> {
    // One call per candidate: words 0-2 give the pair and the acceptance
    // uniform (top 24 bits each), word 3 gives cos(theta) and the three low
    // bytes of words 0-2 give the azimuth.
    __device__ __forceinline__ static void draw(Stream& st, float& a, float& b, Pend<float>& p) {
        const uint4 x = st.next();
        a = u24(x.x);
        b = u24(x.y);
        p.acc = u24(x.z);
        p.dirz = 2.0f * u24(x.w) - 1.0f;
        p.dirp = (float)((x.x & 0xFFu) | ((x.y & 0xFFu) << 8) | ((x.z & 0xFFu) << 16)) * 0x1p-24f;
    }
    // Uniform direction on the sphere (Archimedes): z uniform, phi uniform;
    // v_sin_f32 / v_cos_f32 take the angle in turns.
    __device__ __forceinline__ static void direction(Stream&, const Pend<float>& p, float& dx,
                                                     float& dy, float& dz) {
        const float z = p.dirz;
        const float omz = 1.0f - z * z;
        const float r = Num<float>::sqrt(omz > 0.0f ? omz : 0.0f);
        dx = r * __builtin_amdgcn_cosf(p.dirp);
        dy = r * __builtin_amdgcn_sinf(p.dirp);
        dz = z;
    }
};
template <> struct Cand<double> {
    __device__ __forceinline__ static void draw(Stream& st, double& a, double& b, Pend<double>& p) {
        const uint4 x = st.next();
        a = u53(x.x, x.y);
        b = u53(x.z, x.w);
        const uint4 y = st.next();
        p.acc = u53(y.x, y.y);
    }
    __device__ __forceinline__ static void direction(Stream& st, const Pend<double>&, double& dx,
                                                     double& dy, double& dz) {
        sphere_point<double>(st, dx, dy, dz);
    }
};

__device__ __forceinline__ double wave_sum_fixed(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <class R>
__device__ __forceinline__ void draw_candidate(const InstDesc& d, uint32_t s, int c, int nc,
                                               int64_t k, Pend<R>& p, Stream& st) {
    st = Stream(d.key0, d.key1, s, (uint32_t)c, (uint32_t)k, kTagColl);
    R ua, ub;
    Cand<R>::draw(st, ua, ub, p);
    p.k = k;
    p.i = min((int)(ua * (R)nc), nc - 1);
    p.j = min((int)(ub * (R)(nc - 1)), nc - 2);
    if (p.j >= p.i) ++p.j;
}

// Execute a candidate that owns both of its particles.
template <class R, class V>
__device__ __forceinline__ void run_candidate(Pend<R>& p, Stream& st, R crmr, V vx, V vy, V vz,
                                              int o, R& lane_max, uint32_t& lane_coll) {
    const int i = o + p.i, j = o + p.j;
    const R xi = vx[i], yi = vy[i], zi = vz[i];
    const R xj = vx[j], yj = vy[j], zj = vz[j];
    const R crx = xi - xj, cry = yi - yj, crz = zi - zj;
    const R cr = Num<R>::sqrt((crx * crx + cry * cry) + crz * crz);
    lane_max = cr > lane_max ? cr : lane_max;
    const R cm = cr > crmr ? cr : crmr;
    if (p.acc * cm < cr) {
        R dx, dy, dz;
        Cand<R>::direction(st, p, dx, dy, dz);
        const R cmx = R(0.5) * (xi + xj), cmy = R(0.5) * (yi + yj), cmz = R(0.5) * (zi + zj);
        const R hh = R(0.5) * cr;
        vx[i] = cmx + hh * dx;
        vy[i] = cmy + hh * dy;
        vz[i] = cmz + hh * dz;
        vx[j] = cmx - hh * dx;
        vy[j] = cmy - hh * dy;
        vz[j] = cmz - hh * dz;
        ++lane_coll;
    }
    p.k = -1;
}

struct CoopShared {
    int idle[kCoopWavesAlone];
    double mx[kCoopWavesAlone];
    uint32_t coll[kCoopWavesAlone];
    double mom[kCoopWavesAlone][kMoments];
};

// NTC of one cell by the whole workgroup (rounds of blockDim candidates).
// Every thread of the workgroup must call it.  A claim is the candidate's
// number with the round's stamp above it (255 minus the round number mod
// 256, in the top byte), so a claim left from an earlier round is larger
// than any of this round's and the table needs no clearing between rounds;
// it is cleared when the stamps wrap (rnd counts the workgroup's rounds over
// all its cells).  A cell with 2^24 candidates or more claims with plain
// numbers and clears its claims after every round.
template <class R, class V>
__device__ void coop_ntc(const InstDesc& d, uint32_t s, int c, int nc, int o, V vx, V vy, V vz,
                         uint32_t* tab, int tab_mask, CoopShared& sh, int& rnd) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const unsigned long long lt = lanes_below(lane);
    const double crm0 = d.crmax[c];
    const double mreal = (((0.5 * (double)nc) * (double)(nc - 1)) * crm0) * d.kntc + d.rem[c];
    const double mf = floor(mreal);
    const int64_t M = (int64_t)mf;
    const R crmr = (R)crm0;
    R lane_max = R(0);
    uint32_t lane_coll = 0;
    int64_t next = 0;
    Pend<R> p;
    p.k = -1;
    p.i = p.j = 0;
    p.acc = R(0);
    Stream st(d.key0, d.key1, s, (uint32_t)c, 0u, kTagColl);
    const bool stamped = M < (int64_t)(1 << 24);
    if (!stamped) {
        // claims of stamped cells before this one may remain
        for (int i = threadIdx.x; i <= tab_mask; i += blockDim.x) tab[i] = 0xFFFFFFFFu;
        __syncthreads();
    }
    for (;;) {
        const bool idle = p.k < 0;
        const unsigned long long im = __ballot(idle);
        if (lane == 0) sh.idle[wv] = __popcll(im);
        __syncthreads();
        int off = 0, tot = 0;
        for (int q = 0; q < nw; ++q) {
            const int v = sh.idle[q];
            off += q < wv ? v : 0;
            tot += v;
        }
        // nothing pending and nothing left to draw: done (the same decision
        // in every thread, from the counts every thread has read)
        const int64_t fresh = M - next < (int64_t)tot ? M - next : (int64_t)tot;
        if ((int)blockDim.x == tot && fresh <= 0) break;
        if (idle) {
            const int64_t k = next + off + __popcll(im & lt);
            if (k < M) draw_candidate<R>(d, s, c, nc, k, p, st);
        }
        next += tot;
        if (stamped && (rnd & 255) == 0 && rnd > 0) {
            // the stamps wrap: every check of the last round is done (the
            // barrier above), so the table can be cleared before this
            // round's claims
            for (int i = threadIdx.x; i <= tab_mask; i += blockDim.x) tab[i] = 0xFFFFFFFFu;
            __syncthreads();
        }
        const bool active = p.k >= 0;
        const int hi = p.i & tab_mask, hj = p.j & tab_mask;
        const uint32_t claim = stamped ? ((255u - (uint32_t)(rnd & 255)) << 24) | (uint32_t)p.k : (uint32_t)p.k;
        if (active) {
            atomicMin(&tab[hi], claim);
            atomicMin(&tab[hj], claim);
        }
        __syncthreads();
        const bool win = active && tab[hi] == claim && tab[hj] == claim;
        if (!stamped) {
            __syncthreads();
            if (active) {
                tab[hi] = 0xFFFFFFFFu;
                tab[hj] = 0xFFFFFFFFu;
            }
        }
        ++rnd;
        if (win) run_candidate<R, V>(p, st, crmr, vx, vy, vz, o, lane_max, lane_coll);
    }
    if (!stamped) rnd = 0;  // the table is clear again
    double mx = (double)lane_max;
    uint32_t cc = lane_coll;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double other = __shfl_xor(mx, off, 64);
        mx = other > mx ? other : mx;
        cc += __shfl_xor(cc, off, 64);
    }
    if (lane == 0) {
        sh.mx[wv] = mx;
        sh.coll[wv] = cc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh.mx[0];
        uint32_t t = sh.coll[0];
        for (int q = 1; q < nw; ++q) {
            m = sh.mx[q] > m ? sh.mx[q] : m;
            t += sh.coll[q];
        }
        d.rem[c] = mreal - mf;
        if (m > crm0) d.crmax[c] = m;
        d.ncoll[c] += t;
    }
    __syncthreads();
}

// Sampling sums of one cell: per lane over a strided share of the cell, then
// a fixed butterfly over the wavefront (and, in workgroup mode, the wavefront
// partials added in wavefront order).  With store set, each velocity read is
// also written to the same index of wx, wy, wz (the staged block's copy back
// to global memory, done in the same pass).
template <class R, class V, int U = 1>
__device__ __forceinline__ void cell_moments(V vx, V vy, V vz, int o, int nc, int first,
                                             int stride, double pre, double tot[kMoments],
                                             bool store, gptr<R> wx, gptr<R> wy, gptr<R> wz) {
    Mom m;
    mom_zero(m);
    // unrolled U times (when registers allow) so that the next records'
    // loads overlap this one's sums; the order of the additions is unchanged
#pragma unroll U
    for (int q = first; q < nc; q += stride) {
        const R x = vx[o + q], y = vy[o + q], z = vz[o + q];
        if (store) {
            wx[o + q] = x;
            wy[o + q] = y;
            wz[o + q] = z;
        }
        mom_add_fused(m, (double)x, (double)y, (double)z);
    }
    m.s[kMomPreXY] = pre;
#pragma unroll
    for (int k = 0; k < kMoments; ++k) tot[k] = wave_sum_fixed(m.s[k]);
}

// The cells [c0, c1) of a staged block, one at a time with the whole
// workgroup.  Inlined once for velocities in LDS and once for velocities in
// global memory, so each copy addresses its memory directly (LDS accesses
// become ds_* instructions rather than flat ones).  With wb set (a staged
// block whose cells are sampled) each cell's velocities are copied back to
// wx, wy, wz (global, indexed like vx, vy, vz) once its collisions are done:
// by the sampling threads as they read them, or, in a workgroup wider than
// those, by the other wavefronts meanwhile.
template <class R, class V, int U>
__device__ __forceinline__ void collide_cells(const InstDesc& d, uint32_t s, int c0, int c1,
                                              int s0, V vx, V vy, V vz, uint32_t* claims,
                                              int tab_mask, CoopShared& sh, bool do_collide,
                                              bool sample, bool wb, gptr<R> wx, gptr<R> wy,
                                              gptr<R> wz) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // the sampling sums are added by the first kCoopWaves wavefronts in the
    // same order whatever the workgroup's width, so that the width (chosen
    // per launch from the LDS a block needs) changes no sum
    constexpr int nt = 64 * kCoopWaves;
    const bool adds = (int)threadIdx.x < nt;
    const bool wide = (int)blockDim.x > nt;
    int rnd = 0;  // NTC rounds since the claim table was last clear
    for (int c = c0; c < c1; ++c) {
        const int nc = d.count[c];
        const int o = d.offset[c] - s0;
        // this thread's share of the stress sum before the collisions; the
        // barrier keeps every read ahead of the first collision's writes
        double pre = 0.0;
        if (sample) {
            if (adds) {
#pragma unroll U
                for (int q = (int)threadIdx.x; q < nc; q += nt) pre = __builtin_fma((double)vx[o + q], (double)vy[o + q], pre);
            }
            __syncthreads();
        }
        if (do_collide && nc >= 2) coop_ntc<R, V>(d, s, c, nc, o, vx, vy, vz, claims, tab_mask, sh, rnd);
        if (sample) {
            if (adds) {
                double tot[kMoments];
                cell_moments<R, V, U>(vx, vy, vz, o, nc, (int)threadIdx.x, nt, pre, tot, wb && !wide,
                                      wx, wy, wz);
                if (lane == 0)
                    for (int k = 0; k < kMoments; ++k) sh.mom[wv][k] = tot[k];
            } else if (wb) {
                for (int q = (int)threadIdx.x - nt; q < nc; q += (int)blockDim.x - nt) {
                    wx[o + q] = vx[o + q];
                    wy[o + q] = vy[o + q];
                    wz[o + q] = vz[o + q];
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double* a = d.acc + c;
                for (int k = 0; k < kMoments; ++k) {
                    double t = sh.mom[0][k];
                    for (int q = 1; q < kCoopWaves; ++q) t += sh.mom[q][k];
                    unsafeAtomicAdd(&a[(size_t)k * d.Cc], t);  // one writer per cell: no read needed
                }
            }
            __syncthreads();
        }
    }
}

// Copy n values from global memory to LDS with loads that write LDS
// directly (global_load_lds_dword: each lane of a wavefront moves one dword to
// the wavefront's LDS base, taken from the LDS pointer, plus four times its
// lane number).  The caller waits for vmcnt(0) before the data is read.
template <class R>
__device__ __forceinline__ void stage_to_lds(gptr<R> src, R* dst, int n) {
    const int nd = n * (int)(sizeof(R) / 4);
    const int lane = threadIdx.x & 63;
    const gptr<uint32_t> s = (gptr<uint32_t>)src;
    uint32_t* d = (uint32_t*)dst;
    for (int i = threadIdx.x; i < nd; i += blockDim.x)
        __builtin_amdgcn_global_load_lds((const void*)(s + i),
                                         (__attribute__((address_space(3))) void*)(d + (i - lane)), 4, 0, 0);
}

template <class R, int W>
__global__ __launch_bounds__(64 * W) void k_collide_fast(const InstDesc* __restrict__ descs,
                                                                 const int4* __restrict__ work,
                                                                 int cap, int do_collide) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ CoopShared sh;
    uint32_t* claims = (uint32_t*)smem;
    constexpr int kTable = W * kCoopTablePerWave;
    R* lds_v = (R*)(claims + kTable);
    const int4 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int c0 = w.y, c1 = w.z;
    const int64_t s = d.sc->step_done;
    const bool sample = (d.phase_mask & kPhaseSample) && s > d.n_transient;
    const P4<R> g = particles<R>(d, (int)(s & 1));
    const int s0 = d.offset[c0];
    const int n = d.offset[c1 - 1] + d.count[c1 - 1] - s0;
    for (int i = threadIdx.x; i < kTable; i += blockDim.x) claims[i] = 0xFFFFFFFFu;
    if (n <= cap) {
        R* vx = lds_v;
        R* vy = lds_v + cap;
        R* vz = lds_v + 2 * cap;
        // staged with loads that write LDS directly: every load of the
        // block is in flight at once, with no registers held (with one large
        // cell per CU there are few other wavefronts to hide the latency)
        stage_to_lds(g.vx + s0, vx, n);
        stage_to_lds(g.vy + s0, vy, n);
        stage_to_lds(g.vz + s0, vz, n);
        __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0): the staged data is in LDS
        __syncthreads();
        // a workgroup alone on its CU has registers to spare for unrolling
        // the sampling loops; four-wavefront ones keep more workgroups
        const bool wb = do_collide && sample;
        collide_cells<R, R*, W == kCoopWavesAlone ? 4 : 1>(d, (uint32_t)s, c0, c1, s0, vx, vy, vz, claims,
                                                           kTable - 1, sh, do_collide, sample, wb,
                                                           g.vx + s0, g.vy + s0, g.vz + s0);
        __syncthreads();
        if (do_collide && !wb) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                g.vx[s0 + i] = vx[i];
                g.vy[s0 + i] = vy[i];
                g.vz[s0 + i] = vz[i];
            }
        }
    } else {
        // a block fuller than the staging room works on global memory
        __syncthreads();
        collide_cells<R, gptr<R>, 1>(d, (uint32_t)s, c0, c1, s0, g.vx + s0, g.vy + s0, g.vz + s0,
                                  claims, kTable - 1, sh, do_collide, sample, false, g.vx, g.vy,
                                  g.vz);
    }
}

// Group sums by recursive halving.  A group of G lanes holds per-lane
// partials of the sampling sums, padded to kHalvingMoments.  At each exchange
// distance off (G/2, G/4, ...) a lane keeps the half of its moments selected
// by its lane bit, adds its partner's copy of that half and passes the other
// half on; first tracks which moments the lane keeps.  The pairs added are
// the pairs of a full xor butterfly, so every total is the same to the bit,
// but a lane exchanges 8 + 4 + 2 + 1 moments rather than all of them at every
// distance, and the totals end on different lanes, which issue their
// atomics in parallel.
constexpr int kHalvingMoments = 16;
static_assert(kMoments <= kHalvingMoments, "the halving covers every moment");

template <int H>
__device__ __forceinline__ void halve(double* r, int off, bool upper, int& first) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double lo = r[k], hi = r[k + H];
        const double pass = upper ? lo : hi;
        const double keep = upper ? hi : lo;
        r[k] = keep + __shfl_xor(pass, off, 64);
    }
    if (upper) first += H;
}

// NTC of small cells by groups of G lanes (G = 4..64, a power of two fixed
// per instance and launch shape): each group of a wavefront owns one cell at
// a time and runs that cell's candidates in rounds of G, with a claim table
// of its own in LDS; the group then reduces the cell's sampling sums.  The
// groups of a wavefront run in lockstep, so a round needs no barrier.  Cell
// c of [c0, c1) holds lcnt[c - c0] particles from index loff[c - c0] of the
// velocity arrays; lcrm / lrem hold copies of its crmax and remainder, read
// before the sort so that their latency hides behind it; the new values go
// to orem[c - c0] and ocrm[c - c0].  Each cell has one writer, so its
// counters and accumulators are updated with atomics that return nothing
// (the same sums as a read-modify-write, without the wait).
template <class R, class V>
__device__ __forceinline__ void group_cells(const InstDesc& d, uint32_t s, int c0, int c1,
                                            const int* lcnt, const int* loff, const double* lcrm,
                                            const double* lrem, V vx, V vy, V vz,
                                            uint32_t* wtab, int G, bool do_collide, bool sample,
                                            double* orem, double* ocrm) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int ngw = 64 / G;
    const int grp = lane / G;
    const unsigned long long gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (grp * G);
    const unsigned long long lt = lanes_below(lane) & gmask;
    const int tsize = kGroupTableFactor * G;
    uint32_t* tab = wtab + grp * tsize;
    const int stride = nw * ngw;
    for (int base = c0; base < c1; base += stride) {
        const int c = base + wv * ngw + grp;
        const bool has = c < c1;
        int nc = 0, o = 0;
        int64_t M = 0;
        double crm0 = 0.0, mreal = 0.0, mf = 0.0;
        if (has) {
            nc = lcnt[c - c0];
            o = loff[c - c0];
            if (do_collide && nc >= 2) {
                crm0 = lcrm[c - c0];
                mreal = (((0.5 * (double)nc) * (double)(nc - 1)) * crm0) * d.kntc + lrem[c - c0];
                mf = floor(mreal);
                M = (int64_t)mf;
            }
        }
        // this lane's share of the cell's stress sum before the collisions
        // (the group's lanes run in lockstep and each loaded value is added
        // before the first candidate runs, so no collision write precedes it)
        double pre = 0.0;
        if (has && sample)
            for (int q = lane - grp * G; q < nc; q += G) pre = __builtin_fma((double)vx[o + q], (double)vy[o + q], pre);
        const R crmr = (R)crm0;
        R lane_max = R(0);
        uint32_t lane_coll = 0;
        int64_t next = 0;
        Pend<R> p;
        p.k = -1;
        p.i = p.j = 0;
        p.acc = R(0);
        Stream st(d.key0, d.key1, s, (uint32_t)c, 0u, kTagColl);
        for (;;) {
            const bool idle = p.k < 0;
            const unsigned long long im = __ballot(idle) & gmask;
            if (idle && has) {
                const int64_t k = next + __popcll(im & lt);
                if (k < M) draw_candidate<R>(d, s, c, nc, k, p, st);
            }
            next += __popcll(im);
            const bool active = p.k >= 0;
            if (__ballot(active) == 0ull) break;
            const int hi = p.i & (tsize - 1), hj = p.j & (tsize - 1);
            if (active) {
                atomicMin(&tab[hi], (uint32_t)p.k);
                atomicMin(&tab[hj], (uint32_t)p.k);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const bool win = active && tab[hi] == (uint32_t)p.k && tab[hj] == (uint32_t)p.k;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (active) {
                tab[hi] = 0xFFFFFFFFu;
                tab[hj] = 0xFFFFFFFFu;
            }
            if (win) run_candidate<R, V>(p, st, crmr, vx, vy, vz, o, lane_max, lane_coll);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // group reductions (butterflies inside the group)
        double mx = (double)lane_max;
        uint32_t cc = lane_coll;
        Mom m;
        mom_zero(m);
        if (has && sample)
            for (int q = lane - grp * G; q < nc; q += G)
                mom_add_fused(m, (double)vx[o + q], (double)vy[o + q], (double)vz[o + q]);
        m.s[kMomPreXY] = pre;
        for (int off = G >> 1; off >= 1; off >>= 1) {
            const double other = __shfl_xor(mx, off, 64);
            mx = other > mx ? other : mx;
            cc += __shfl_xor(cc, off, 64);
        }
        const int gl = lane & (G - 1);
        if (has && gl == 0 && do_collide && nc >= 2) {
            orem[c - c0] = mreal - mf;
            if (mx > crm0) ocrm[c - c0] = mx;
            if (cc) atomicAdd(&d.ncoll[c], cc);
        }
        if (sample) {
            // the moment sums by recursive halving: lane gl ends with the
            // group's totals of moments first .. first + held - 1
            double r[kHalvingMoments];
#pragma unroll
            for (int k = 0; k < kHalvingMoments; ++k) r[k] = k < kMoments ? m.s[k] : 0.0;
            int first = 0, off = G >> 1;
            if (off >= 1) { halve<8>(r, off, (gl & off) != 0, first); off >>= 1; }
            if (off >= 1) { halve<4>(r, off, (gl & off) != 0, first); off >>= 1; }
            if (off >= 1) { halve<2>(r, off, (gl & off) != 0, first); off >>= 1; }
            if (off >= 1) { halve<1>(r, off, (gl & off) != 0, first); off >>= 1; }
            // groups wider than kHalvingMoments finish with full exchanges,
            // after which lanes differing only in the low bits hold the same
            // totals: the one with those bits clear adds them
            const int dup = G > kHalvingMoments ? G / kHalvingMoments - 1 : 0;
            for (; off >= 1; off >>= 1) r[0] += __shfl_xor(r[0], off, 64);
            if (has && (gl & dup) == 0) {
                const int held = G >= kHalvingMoments ? 1 : kHalvingMoments / G;
                double* a = d.acc + c;
#pragma unroll
                for (int k = 0; k < kHalvingMoments / 2; ++k)
                    if (k < held && first + k < kMoments)
                        unsafeAtomicAdd(&a[(size_t)(first + k) * d.Cc], r[k]);
            }
        }
    }
}

// Sort of one bucket of cells [c0, c1) by cell, stable: the bucket's n
// particles sit at slots s0 .. s0 + n - 1 of g in their previous order, and
// are written to sy, sx, sv, sz (indices 0 .. n - 1) sorted by cell.  Four
// wavefronts each own a contiguous quarter: a first pass counts each
// quarter's cells in the wavefront's table wt (kMaxCellsPerKey entries per
// wavefront); lcnt / loff receive the bucket's per-cell counts and local
// offsets; the second pass ranks equal cells of a round of 64 slots with
// bit-sliced ballots, as the global scatter does.  Every thread must call it.
template <class R, class V>
__device__ __forceinline__ void bucket_sort(const InstDesc& d, const P4<R>& g, int s0, int n,
                                            int c0, int ncell, int* wt, int* lcnt, int* loff,
                                            V sy, V sx, V sv, V sz) {
    __shared__ int wsum[kFastWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int quarter = ((n + kFastWaves - 1) / kFastWaves + 63) / 64 * 64;
    const int q0 = min(wv * quarter, n), q1 = min(q0 + quarter, n);
    int* mine = wt + wv * kMaxCellsPerKey;
    for (int i = q0 + lane; i < q1; i += 64) atomicAdd(&mine[cell_of<R>(d, g.y[s0 + i]) - c0], 1);
    __syncthreads();
    // one thread per cell of the bucket (ncell <= kMaxCellsPerKey <= blockDim)
    const int c = threadIdx.x;
    int tot = 0;
    if (c < ncell)
        for (int q = 0; q < kFastWaves; ++q) tot += wt[q * kMaxCellsPerKey + c];
    const int incl = wave_incl_scan(tot, lane);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = incl - tot;
    for (int q = 0; q < wv; ++q) run += wsum[q];
    if (c < ncell) {
        lcnt[c] = tot;
        loff[c] = run;
        for (int q = 0; q < kFastWaves; ++q) {
            const int v = wt[q * kMaxCellsPerKey + c];
            wt[q * kMaxCellsPerKey + c] = run;
            run += v;
        }
    }
    __syncthreads();
    const unsigned long long lt = lanes_below(lane);
    const int nbits = ncell > 1 ? 32 - __builtin_clz((unsigned)(ncell - 1)) : 0;
    for (int base = q0; base < q1; base += 64) {
        const int i = base + lane;
        const bool valid = i < q1;
        int lc = 0;
        R ry = R(0), rx = R(0), rv = R(0), rz = R(0);
        if (valid) {
            ry = g.y[s0 + i];
            rx = g.vx[s0 + i];
            rv = g.vy[s0 + i];
            rz = g.vz[s0 + i];
            lc = cell_of<R>(d, ry) - c0;
        }
        unsigned long long m = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (lc >> b) & 1;
            const unsigned long long bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        if (valid) {
            const int pos = mine[lc] + __popcll(m & lt);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if ((m & lt) == 0ull) mine[lc] = pos + __popcll(m);
            sy[pos] = ry;
            sx[pos] = rx;
            sv[pos] = rv;
            sz[pos] = rz;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
}

// Records per lane a bucket-collide workgroup holds in registers while it
// sorts a bucket (so that all of the bucket's loads are in flight at once).
template <class R> struct BucketRegs { static constexpr int value = sizeof(R) == 4 ? 12 : 6; };

// The same stable sort with the bucket held in registers (n <= 256 *
// BucketRegs): every load is issued before the first barrier, velocities go
// to LDS in cell order and positions straight to their final slots of g (the
// whole bucket is in registers by then).  Round k of wavefront w covers
// slots q0 + 64 k + lane of its quarter, the order of bucket_sort.
template <class R>
__device__ __forceinline__ void bucket_sort_regs(const InstDesc& d, const P4<R>& g, int s0, int n,
                                                 int c0, int ncell, int* wt, int* lcnt, int* loff,
                                                 R* sx, R* sv, R* sz) {
    constexpr int K = BucketRegs<R>::value;
    __shared__ int wsum[kFastWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int quarter = ((n + kFastWaves - 1) / kFastWaves + 63) / 64 * 64;
    const int q0 = min(wv * quarter, n), q1 = min(q0 + quarter, n);
    int* mine = wt + wv * kMaxCellsPerKey;
    R ry[K], rx[K], rv[K], rz[K];
    int lc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = q0 + 64 * k + lane;
        ry[k] = rx[k] = rv[k] = rz[k] = R(0);
        if (i < q1) {
            ry[k] = g.y[s0 + i];
            rx[k] = g.vx[s0 + i];
            rv[k] = g.vy[s0 + i];
            rz[k] = g.vz[s0 + i];
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        lc[k] = 0;
        if (q0 + 64 * k + lane < q1) {
            lc[k] = cell_of<R>(d, ry[k]) - c0;
            atomicAdd(&mine[lc[k]], 1);
        }
    }
    __syncthreads();
    const int c = threadIdx.x;
    int tot = 0;
    if (c < ncell)
        for (int q = 0; q < kFastWaves; ++q) tot += wt[q * kMaxCellsPerKey + c];
    const int incl = wave_incl_scan(tot, lane);
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = incl - tot;
    for (int q = 0; q < wv; ++q) run += wsum[q];
    if (c < ncell) {
        lcnt[c] = tot;
        loff[c] = run;
        for (int q = 0; q < kFastWaves; ++q) {
            const int v = wt[q * kMaxCellsPerKey + c];
            wt[q * kMaxCellsPerKey + c] = run;
            run += v;
        }
    }
    __syncthreads();
    const unsigned long long lt = lanes_below(lane);
    const int nbits = ncell > 1 ? 32 - __builtin_clz((unsigned)(ncell - 1)) : 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (q0 + 64 * k < q1) {  // uniform over the wavefront
            const bool valid = q0 + 64 * k + lane < q1;
            unsigned long long m = __ballot(valid);
            for (int b = 0; b < nbits; ++b) {
                const bool bit = (lc[k] >> b) & 1;
                const unsigned long long bal = __ballot(bit);
                m &= bit ? bal : ~bal;
            }
            if (valid) {
                const int pos = mine[lc[k]] + __popcll(m & lt);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if ((m & lt) == 0ull) mine[lc[k]] = pos + __popcll(m);
                g.y[s0 + pos] = ry[k];
                sx[pos] = rx[k];
                sv[pos] = rv[k];
                sz[pos] = rz[k];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
}

// Collide kernel of bucket-sorted instances: one workgroup per bucket (work
// item: instance, bucket, G).  The bucket is sorted by cell (velocities into
// LDS, positions to their final slots), its cells are collided and sampled
// there, and the velocities are written back to the bucket's slots together
// with each cell's count and offset.  A bucket fuller than the staging room
// is sorted into the same slots of the other particle buffer, which is free
// during this phase, collided there and copied back.  The sort's wavefront
// tables share LDS with the claim tables, which are set up after the sort.
template <class R>
__global__ __launch_bounds__(64 * kFastWaves) void k_collide_bucket(const InstDesc* __restrict__ descs,
                                                                   const int4* __restrict__ work,
                                                                   int cap, int do_collide) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kClaims = kFastWaves * 64 * kGroupTableFactor;
    static_assert(kFastWaves * kMaxCellsPerKey <= kClaims, "sort tables fit in the claim tables");
    uint32_t* claims = (uint32_t*)smem;
    int* wt = (int*)smem;
    double* lcrm = (double*)(claims + kClaims);
    double* lrem = lcrm + kMaxCellsPerKey;
    int* lcnt = (int*)(lrem + kMaxCellsPerKey);
    int* loff = lcnt + kMaxCellsPerKey;
    R* lds = (R*)(loff + kMaxCellsPerKey);
    const int4 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int b = w.y, G = w.z;
    const int c0 = b << d.key_shift, c1 = min(c0 + (1 << d.key_shift), d.Cc);
    const int64_t s = d.sc->step_done;
    const bool sample = (d.phase_mask & kPhaseSample) && s > d.n_transient;
    const P4<R> g = particles<R>(d, (int)(s & 1));
    const int s0 = d.koffset[b], n = d.kcount[b];
    for (int i = threadIdx.x; i < kFastWaves * kMaxCellsPerKey; i += blockDim.x) wt[i] = 0;
    if (do_collide)
        for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) {
            lcrm[c - c0] = d.crmax[c];
            lrem[c - c0] = d.rem[c];
        }
    __syncthreads();
    uint32_t* wtab = claims + (threadIdx.x >> 6) * 64 * kGroupTableFactor;
    if (n <= cap && n <= kFastWaves * 64 * BucketRegs<R>::value) {
        R* sx = lds;
        R* sv = lds + cap;
        R* sz = lds + 2 * cap;
        bucket_sort_regs<R>(d, g, s0, n, c0, c1 - c0, wt, lcnt, loff, sx, sv, sz);
        for (int i = threadIdx.x; i < kClaims; i += blockDim.x) claims[i] = 0xFFFFFFFFu;
        __syncthreads();
        group_cells<R, R*>(d, (uint32_t)s, c0, c1, lcnt, loff, lcrm, lrem, sx, sv, sz, wtab, G,
                           do_collide, sample, d.rem + c0, d.crmax + c0);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            g.vx[s0 + i] = sx[i];
            g.vy[s0 + i] = sv[i];
            g.vz[s0 + i] = sz[i];
        }
    } else {
        const P4<R> o = particles<R>(d, (int)((s - 1) & 1));
        const gptr<R> sy = o.y + s0, sx = o.vx + s0, sv = o.vy + s0, sz = o.vz + s0;
        bucket_sort<R, gptr<R>>(d, g, s0, n, c0, c1 - c0, wt, lcnt, loff, sy, sx, sv, sz);
        for (int i = threadIdx.x; i < kClaims; i += blockDim.x) claims[i] = 0xFFFFFFFFu;
        __syncthreads();
        group_cells<R, gptr<R>>(d, (uint32_t)s, c0, c1, lcnt, loff, lcrm, lrem, sx, sv, sz, wtab, G,
                                do_collide, sample, d.rem + c0, d.crmax + c0);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            g.y[s0 + i] = sy[i];
            g.vx[s0 + i] = sx[i];
            g.vy[s0 + i] = sv[i];
            g.vz[s0 + i] = sz[i];
        }
    }
    for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) {
        d.count[c] = lcnt[c - c0];
        d.offset[c] = s0 + loff[c - c0];
    }
}

// ----------------------------------------------------------- estimators
// Per sampling cell (its collision cells summed in order) with K sampled
// steps and N particles: density nu = S0 C/(K N); u = S1/S0;
// M_ab = S2_ab/S0 - u_a u_b; T = trace(M)/3; P_xy = nu M_xy; the
// time-centred P_xy from the mean of the vxvy sums before and after the
// collisions; <|c|^2 c_a> from the raw moments; q_a = nu <|c|^2 c_a>/2; mass flow
// Q = sum S1_x/(K N).  Velocities, heat fluxes and Q are divided by
// v0 = sqrt(2) and stresses are over n kT: the dimensionless variables of
// Eq. 6.  The sum of Q runs in cell order: all threads stage the cells'
// x-momentum sums in LDS and one thread adds them in order.
constexpr int kFinalizeChunk = 2048;  // sampling cells whose x-momentum sums are staged at a time

// The estimators of one instance into est (kEstPerCell * C + 3 doubles), by
// the whole 256-thread workgroup; col and coll_part are its LDS.
__device__ void finalize_into(const InstDesc& d, double* est, double* col,
                              unsigned long long* coll_part) {
    constexpr int kChunk = kFinalizeChunk;
    const int C = d.C, ns = d.n_sub;
    const double K = (double)d.sc->n_sampled, N = (double)d.N;
    const double v0 = __builtin_sqrt(2.0);
    double q = 0.0;  // only thread 0's copy is used: the sum in cell order
    for (int cs = 0; cs < C; cs += kChunk) {
        const int ce = min(cs + kChunk, C);
        for (int c = cs + (int)threadIdx.x; c < ce; c += blockDim.x) {
            double s[kMoments];
            for (int m = 0; m < kMoments; ++m) s[m] = 0.0;
            for (int k = 0; k < ns; ++k) {
                const double* a = d.acc + ((size_t)c * ns + k);
                for (int m = 0; m < kMoments; ++m) s[m] += a[(size_t)m * d.Cc];
            }
            col[c - cs] = s[1];
            const double n_c = (s[0] * (double)C) / (K * N);
            const double u = s[1] / s[0], v = s[2] / s[0], ww = s[3] / s[0];
            const double mxx = s[4] / s[0] - u * u;
            const double myy = s[5] / s[0] - v * v;
            const double mzz = s[6] / s[0] - ww * ww;
            const double mxy = s[7] / s[0] - u * v;
            const double trace2 = (s[4] + s[5]) + s[6];
            const double usq = (u * u + v * v) + ww * ww;
            const double cx = ((s[10] / s[0] - u * (trace2 / s[0])) -
                               2.0 * (((u * s[4] + v * s[7]) + ww * s[8]) / s[0])) + 2.0 * u * usq;
            const double cy = ((s[11] / s[0] - v * (trace2 / s[0])) -
                               2.0 * (((u * s[7] + v * s[5]) + ww * s[9]) / s[0])) + 2.0 * v * usq;
            double* e = est;
            e[0 * C + c] = n_c;
            e[1 * C + c] = u / v0;
            e[2 * C + c] = v / v0;
            e[3 * C + c] = ww / v0;
            e[4 * C + c] = ((mxx + myy) + mzz) / 3.0;
            e[5 * C + c] = n_c * mxy;
            e[6 * C + c] = (0.5 * n_c * cx) / v0;
            e[7 * C + c] = (0.5 * n_c * cy) / v0;
            e[8 * C + c] = n_c * ((0.5 * (s[7] + s[kMomPreXY])) / s[0] - u * v);
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int c = 0; c < ce - cs; ++c) q += col[c];
        __syncthreads();
    }
    unsigned long long cs = 0;
    for (int c = threadIdx.x; c < d.Cc; c += blockDim.x) cs += d.ncoll[c];
    coll_part[threadIdx.x] = cs;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int t = 0; t < (int)blockDim.x; ++t) tot += coll_part[t];
        est[kEstPerCell * C] = (q / (K * N)) / v0;
        est[kEstPerCell * C + 1] = K;
        est[kEstPerCell * C + 2] = (double)tot;
    }
}

// ----------------------------------------------- resident small instances
// A small instance can run whole steps in one workgroup with its particles
// held in LDS: no global sort, no launch per phase, and as many steps per
// launch as asked.  Small means a fast mode, small cells (the bucket
// collide's shape), at most kResidentKeys sort keys (its cells, and for an
// open instance the key of the particles that left) and at most 6144 slots
// in FP32 (3072 in FP64), ResidentRegs per lane.  Each step is the
// multi-kernel step's arithmetic
// in the same order: the injections of an open instance are drawn into the
// slots after the live ones, slot i is flown with its wall stream (step, i)
// and ranked in slot order by cell (the particles that left after every
// cell), and the cells are collided and sampled by group_cells with the
// multi-kernel launch's lanes per cell G.  Both paths
// therefore leave the same state bit for bit.  At the end of the launch the
// particles, cell tables, step counters and boundary state go back to global
// memory as the multi-kernel step leaves them.
template <class R> struct ResidentRegs {
    static constexpr int value = (sizeof(R) == 4 ? 6144 : 3072) / (64 * kResidentWaves);
};
static_assert(kResidentKeys <= 64 * kResidentWaves, "one key per thread of the resident workgroup");

template <class R, bool kOpen>
__global__ __launch_bounds__(64 * kResidentWaves) void k_resident(const InstDesc* __restrict__ descs,
                                                                 const int2* __restrict__ work,
                                                                 int64_t n_steps, int slot_cap) {
    constexpr int W = kResidentWaves;
    constexpr int K = ResidentRegs<R>::value;
    constexpr int kClaims = W * 64 * kGroupTableFactor;
    constexpr int kKeys = kResidentKeys;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* claims = (uint32_t*)smem;            // claim tables of the cell groups
    int* wt = (int*)(claims + kClaims);            // per wavefront: keys counted, then ranks
    int* lcnt = wt + W * kKeys;                    // particles per key
    int* loff = lcnt + kKeys;                      // first slot of each key
    double* lcrm = (double*)(loff + kKeys);        // crmax per cell
    double* lrem = lcrm + kKeys;                   // NTC remainder per cell
    R* ly = (R*)(lrem + kKeys);                    // the particles, slot order
    R* lx = ly + slot_cap;
    R* lv = lx + slot_cap;
    R* lz = lv + slot_cap;
    __shared__ int sh_live, sh_bad, wsum[W];
    __shared__ double sh_rem;
    __shared__ long long sh_inj, sh_del;
    const int2 w = work[blockIdx.x];
    const InstDesc& d = descs[w.x];
    const int G = w.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int Cc = d.Cc;
    const bool open = kOpen && d.open;
    const int nk = Cc + (open ? 1 : 0);
    int64_t s = d.sc->step_done;
    {
        const int live0 = open ? d.os->n_live : d.N;
        const P4<R> src = particles<R>(d, (int)(s & 1));
        for (int i = tid; i < live0; i += blockDim.x) {
            ly[i] = src.y[i];
            lx[i] = src.vx[i];
            lv[i] = src.vy[i];
            lz[i] = src.vz[i];
        }
        for (int c = tid; c < Cc; c += blockDim.x) {
            lcrm[c] = d.crmax[c];
            lrem[c] = d.rem[c];
        }
        for (int i = tid; i < kClaims; i += blockDim.x) claims[i] = 0xFFFFFFFFu;
        if (tid == 0) {
            sh_live = live0;
            sh_bad = 0;
            if (open) {
                sh_rem = d.os->inj_rem;
                sh_inj = d.os->n_injected;
                sh_del = d.os->n_deleted;
            }
        }
    }
    __syncthreads();
    const int nbits = nk > 1 ? 32 - __builtin_clz((unsigned)(nk - 1)) : 0;
    const unsigned long long lt = lanes_below(lane);
    int* mine = wt + wv * kKeys;
    uint32_t* wtab = claims + wv * 64 * kGroupTableFactor;
    int64_t sampled = 0;
    int used = sh_live;
    for (int64_t t = 0; t < n_steps; ++t) {
        ++s;
        const int live = sh_live;
        used = live;
        double rem_next = 0.0;
        bool clipped = false;
        if (open) {
            used = live + injections(d, live, sh_rem, rem_next, clipped);
            for (int i = live + tid; i < used; i += blockDim.x)
                inject_state<R>(d, (uint32_t)s, i - live, ly[i], lx[i], lv[i], lz[i]);
        }
        for (int k = tid; k < W * kKeys; k += blockDim.x) wt[k] = 0;
        __syncthreads();
        if (tid == 0 && open) {
            sh_rem = rem_next;
            sh_inj += used - live;
            if (clipped) atomicOr(&sh_bad, 8);
        }
        // move: each wavefront takes a contiguous share of the slots and
        // counts its keys
        const int quarter = ((used + W - 1) / W + 63) / 64 * 64;
        const int q0 = min(wv * quarter, used), q1 = min(q0 + quarter, used);
        R ry[K], rx[K], rv[K], rz[K];
        int key[K];
        int bad = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = q0 + 64 * k + lane;
            ry[k] = rx[k] = rv[k] = rz[k] = R(0);
            key[k] = 0;
            if (i < q1) {
                ry[k] = ly[i];
                rx[k] = lx[i];
                rv[k] = lv[i];
                rz[k] = lz[i];
                bool gone = false;
                move_one<R, kOpen>(d, (uint32_t)s, (uint32_t)i, ry[k], rx[k], rv[k], rz[k], gone);
                bad |= !(isfinite(rx[k]) && isfinite(rv[k]) && isfinite(rz[k]));
                key[k] = (kOpen && gone) ? Cc : cell_of<R>(d, ry[k]);
                atomicAdd(&mine[key[k]], 1);
            }
        }
        if (bad) atomicOr(&sh_bad, 1);
        __syncthreads();
        // keys' totals and first slots, and each wavefront's first slot per key
        {
            const int c = tid;
            int tot = 0;
            if (c < nk)
                for (int q = 0; q < W; ++q) tot += wt[q * kKeys + c];
            const int incl = wave_incl_scan(tot, lane);
            if (lane == 63) wsum[wv] = incl;
            __syncthreads();
            int run = incl - tot;
            for (int q = 0; q < wv; ++q) run += wsum[q];
            if (c < nk) {
                lcnt[c] = tot;
                loff[c] = run;
                for (int q = 0; q < W; ++q) {
                    const int v = wt[q * kKeys + c];
                    wt[q * kKeys + c] = run;
                    run += v;
                }
                if (c == nk - 1 && run != used) atomicOr(&sh_bad, 2);
            }
        }
        __syncthreads();
        // stable rank in slot order, written back in place (every slot of the
        // step is in registers)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (q0 + 64 * k < q1) {  // uniform over the wavefront
                const bool valid = q0 + 64 * k + lane < q1;
                unsigned long long m = __ballot(valid);
                for (int b = 0; b < nbits; ++b) {
                    const bool bit = (key[k] >> b) & 1;
                    const unsigned long long bal = __ballot(bit);
                    m &= bit ? bal : ~bal;
                }
                if (valid) {
                    int pos = mine[key[k]] + __popcll(m & lt);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    if ((m & lt) == 0ull) mine[key[k]] = pos + __popcll(m);
                    if (pos < 0 || pos >= used) {
                        atomicOr(&sh_bad, 4);
                        pos = pos < 0 ? 0 : used - 1;
                    }
                    ly[pos] = ry[k];
                    lx[pos] = rx[k];
                    lv[pos] = rv[k];
                    lz[pos] = rz[k];
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        if (tid == 0 && open) {
            sh_live = loff[Cc];
            sh_del += lcnt[Cc];
        }
        // collisions and sampling of all cells at once, with the bucket
        // collide's G (a cell's arithmetic does not depend on which group
        // of which wavefront takes it)
        const bool sample = s > d.n_transient;
        group_cells<R, R*>(d, (uint32_t)s, 0, Cc, lcnt, loff, lcrm, lrem, lx, lv, lz, wtab, G, true,
                           sample, lrem, lcrm);
        if (sample) ++sampled;
        __syncthreads();
    }
    const int live = sh_live;
    const P4<R> dst = particles<R>(d, (int)(s & 1));
    for (int i = tid; i < live; i += blockDim.x) {
        dst.y[i] = ly[i];
        dst.vx[i] = lx[i];
        dst.vy[i] = lv[i];
        dst.vz[i] = lz[i];
    }
    for (int c = tid; c < Cc; c += blockDim.x) {
        d.crmax[c] = lcrm[c];
        d.rem[c] = lrem[c];
        d.count[c] = lcnt[c];
        d.offset[c] = loff[c];
    }
    if (tid == 0) {
        d.sc->step_done = s;
        d.sc->n_sampled += sampled;
        if (sh_bad) atomicOr(&d.sc->status, sh_bad);
        if (open) {
            d.os->n_live = live;
            d.os->n_used = used;
            d.os->inj_rem = sh_rem;
            d.os->n_injected = sh_inj;
            d.os->n_deleted = sh_del;
        }
    }
}

__global__ __launch_bounds__(256) void k_finalize(const InstDesc* __restrict__ descs) {
    __shared__ double col[kFinalizeChunk];
    __shared__ unsigned long long coll_part[256];
    const InstDesc& d = descs[blockIdx.x];
    finalize_into(d, d.est, col, coll_part);
}

// The estimators of many instances into one staging buffer: instance b's
// block at stage + off[b] holds its kEstPerCell * C + 3 estimator values,
// then its status word, so one copy brings a whole group's windows back.
__global__ __launch_bounds__(256) void k_finalize_staged(const InstDesc* __restrict__ descs,
                                                        const int64_t* __restrict__ off,
                                                        double* __restrict__ stage) {
    __shared__ double col[kFinalizeChunk];
    __shared__ unsigned long long coll_part[256];
    const InstDesc& d = descs[blockIdx.x];
    double* est = stage + off[blockIdx.x];
    finalize_into(d, est, col, coll_part);
    if (threadIdx.x == 0) est[kEstPerCell * d.C + 3] = (double)d.sc->status;
}

// The same from a table of pointers to the instances' own device
// descriptors, so that no descriptor array has to be built for the call.
__global__ __launch_bounds__(256) void k_finalize_gather(const InstDesc* const* __restrict__ descs,
                                                        const int64_t* __restrict__ off,
                                                        double* __restrict__ stage) {
    __shared__ double col[kFinalizeChunk];
    __shared__ unsigned long long coll_part[256];
    const InstDesc& d = *descs[blockIdx.x];
    double* est = stage + off[blockIdx.x];
    finalize_into(d, est, col, coll_part);
    if (threadIdx.x == 0) est[kEstPerCell * d.C + 3] = (double)d.sc->status;
}

// The status words of n instances into out (one synchronisation and one
// copy check a whole group).
__global__ __launch_bounds__(256) void k_gather_status(const InstDesc* __restrict__ descs, int n,
                                                      int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = descs[i].sc->status;
}

__device__ __forceinline__ void reset_window_of(const InstDesc& d) {
    const size_t n = (size_t)d.Cc * kMoments;
    for (size_t i = threadIdx.x; i < n; i += blockDim.x) d.acc[i] = 0.0;
    for (int c = threadIdx.x; c < d.Cc; c += blockDim.x) d.ncoll[c] = 0u;
    if (threadIdx.x == 0) d.sc->n_sampled = 0;
}

__global__ __launch_bounds__(256) void k_reset_window(const InstDesc* __restrict__ descs) {
    reset_window_of(descs[blockIdx.x]);
}

__global__ __launch_bounds__(256) void k_reset_window_gather(const InstDesc* const* __restrict__ descs) {
    reset_window_of(*descs[blockIdx.x]);
}

// The kernels of one step under a debug phase mask (a move without the sort,
// a sort without a move, or neither): the move writes the cell index array in
// place, and the sort (if any) is a separate stable scatter from that array.
template <class R, class Mark>
void step_kernels_debug(const Work& w, Mode mode, unsigned phase, hipStream_t st, Mark mark) {
    const size_t hist_lds = (size_t)w.max_cc * sizeof(int);
    if (phase & (kPhaseMove | kPhaseSort)) {
        if (phase & kPhaseMove)
            hipLaunchKernelGGL((k_move_hist<R, true>), dim3(w.n_tiles), dim3(kParticleThreads),
                               hist_lds, st, w.desc, w.tiles);
        else
            hipLaunchKernelGGL((k_move_hist<R, false>), dim3(w.n_tiles), dim3(kParticleThreads),
                               hist_lds, st, w.desc, w.tiles);
    }
    mark(1);
    if (phase & kPhaseSort) {
        hipLaunchKernelGGL(k_colsum, dim3(w.n_cols), dim3(kColThreads), 0, st, w.desc, w.cols);
        mark(2);
        hipLaunchKernelGGL(k_scan, dim3(w.n_inst), dim3(kScanThreads), 0, st, w.desc, 1);
        mark(3);
        hipLaunchKernelGGL(k_colprefix, dim3(w.n_cols), dim3(kColThreads), 0, st, w.desc, w.cols);
        mark(4);
        hipLaunchKernelGGL((k_scatter<R>), dim3(w.n_tiles), dim3(kParticleThreads),
                           scatter_lds_bytes(mode, w.max_cc, w.stage_max), st, w.desc, w.tiles,
                           w.stage_max);
    } else {
        mark(2);
        hipLaunchKernelGGL(k_scan, dim3(w.n_inst), dim3(kScanThreads), 0, st, w.desc, 0);
        mark(3);
        mark(4);
        hipLaunchKernelGGL((k_copy<R>), dim3(w.n_tiles), dim3(kParticleThreads), 0, st, w.desc,
                           w.tiles);
    }
}

template <class R>
void resident_kernel(const Work& w, Mode mode, int64_t n_steps, hipStream_t st) {
    const size_t lds = resident_lds_bytes(mode, w.resident_cap);
    if (w.has_open)
        hipLaunchKernelGGL((k_resident<R, true>), dim3(w.n_resident), dim3(64 * kResidentWaves), lds, st,
                           w.desc, w.resident, n_steps, w.resident_cap);
    else
        hipLaunchKernelGGL((k_resident<R, false>), dim3(w.n_resident), dim3(64 * kResidentWaves), lds, st,
                           w.desc, w.resident, n_steps, w.resident_cap);
}

template <class R>
void step_kernels(const Work& w, Mode mode, unsigned phase, hipStream_t st, hipEvent_t* ev = nullptr) {
    // a tuning may raise the dynamic LDS of the particle and collide kernels
    // above what they use, to cap the workgroups that share a CU
    auto lds = [&](size_t need) { return need > w.lds_floor ? need : w.lds_floor; };
    auto coop_lds = [&](size_t need) { return need > w.lds_floor_coop ? need : w.lds_floor_coop; };
    const size_t hist_lds = lds((size_t)w.max_cc * sizeof(int));
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], st);
    };
    if (w.n_resident) {
        // a resident lane's step is one kernel: it is timed in the collide
        // slot, and the other slots' events are not recorded
        mark(5);
        resident_kernel<R>(w, mode, 1, st);
        mark(6);
        return;
    }
    mark(0);
    if ((phase & kPhaseMove) && (phase & kPhaseSort)) {
        if (w.has_open)
            hipLaunchKernelGGL((k_count<R, true>), dim3(w.n_tiles), dim3(kParticleThreads), hist_lds,
                               st, w.desc, w.tiles);
        else
            hipLaunchKernelGGL((k_count<R, false>), dim3(w.n_tiles), dim3(kParticleThreads), hist_lds,
                               st, w.desc, w.tiles);
        mark(1);
        if (w.scan_small_lds) {
            // the three column scans in one launch, in the scan slot
            mark(2);
            hipLaunchKernelGGL(k_scan_small, dim3(w.n_inst), dim3(kScanThreads),
                               (size_t)w.scan_small_lds, st, w.desc);
            mark(3);
        } else if (w.scan_seg_lds) {
            mark(2);
            hipLaunchKernelGGL(k_scan_seg, dim3(w.n_inst), dim3(kScanThreads), (size_t)w.scan_seg_lds, st,
                               w.desc);
            mark(3);
        } else {
            hipLaunchKernelGGL(k_colsum, dim3(w.n_cols), dim3(kColThreads), 0, st, w.desc, w.cols);
            mark(2);
            hipLaunchKernelGGL(k_scan, dim3(w.n_inst), dim3(kScanThreads), 0, st, w.desc, 1);
            mark(3);
            hipLaunchKernelGGL(k_colprefix, dim3(w.n_cols), dim3(kColThreads), 0, st, w.desc, w.cols);
        }
        mark(4);
        // tiles the registers hold first, then the larger ones
        const int n_wide = w.n_tiles - w.n_narrow;
        if (w.n_narrow) {
            if (w.has_open)
                hipLaunchKernelGGL((k_move_scatter<R, true>), dim3(w.n_narrow), dim3(kParticleThreads),
                                   lds(w.scatter_lds), st, w.desc, w.tiles, w.stage_max);
            else
                hipLaunchKernelGGL((k_move_scatter<R, false>), dim3(w.n_narrow), dim3(kParticleThreads),
                                   lds(w.scatter_lds), st, w.desc, w.tiles, w.stage_max);
        }
        if (n_wide) {
            if (w.has_open)
                hipLaunchKernelGGL((k_move_scatter_wide<R, true>), dim3(n_wide), dim3(kParticleThreads),
                                   lds(w.wide_lds), st, w.desc, w.tiles + w.n_narrow);
            else
                hipLaunchKernelGGL((k_move_scatter_wide<R, false>), dim3(n_wide), dim3(kParticleThreads),
                                   lds(w.wide_lds), st, w.desc, w.tiles + w.n_narrow);
        }
    } else {
        step_kernels_debug<R>(w, mode, phase, st, mark);
    }
    mark(5);
    if (phase & (kPhaseCollide | kPhaseSample)) {
        const int do_collide = (phase & kPhaseCollide) ? 1 : 0;
        if (mode == kFp64Det) {
            hipLaunchKernelGGL(k_collide_det, dim3(w.n_gblocks), dim3(64), 0, st, w.desc, w.gblocks,
                               do_collide);
        } else {
            if (w.n_cblocks) {
                const size_t clds = coop_lds(fast_collide_lds_bytes(mode, w.fast_cap, w.coop_waves));
                if (w.coop_waves == kCoopWavesAlone)
                    hipLaunchKernelGGL((k_collide_fast<R, kCoopWavesAlone>), dim3(w.n_cblocks),
                                       dim3(64 * kCoopWavesAlone), clds, st, w.desc, w.cblocks, w.fast_cap,
                                       do_collide);
                else
                    hipLaunchKernelGGL((k_collide_fast<R, kCoopWaves>), dim3(w.n_cblocks), dim3(64 * kCoopWaves),
                                       clds, st, w.desc, w.cblocks, w.fast_cap, do_collide);
            }
            if (w.n_gblocks)
                hipLaunchKernelGGL((k_collide_bucket<R>), dim3(w.n_gblocks), dim3(64 * kFastWaves),
                                   lds(bucket_collide_lds_bytes(mode, w.group_cap)), st, w.desc,
                                   w.gblocks, w.group_cap, do_collide);
        }
    }
    mark(6);
}

}  // namespace

int resident_slots(Mode mode) {
    return 64 * kResidentWaves * (mode == kFp32Fast ? ResidentRegs<float>::value : ResidentRegs<double>::value);
}

size_t resident_lds_bytes(Mode mode, int slot_cap) {
    const size_t rb = mode == kFp32Fast ? sizeof(float) : sizeof(double);
    return (size_t)kResidentWaves * 64 * kGroupTableFactor * sizeof(uint32_t) +
           (size_t)(kResidentWaves + 2) * kResidentKeys * sizeof(int) +
           (size_t)2 * kResidentKeys * sizeof(double) + (size_t)4 * slot_cap * rb;
}

void launch_resident(const Work& w, Mode mode, int64_t n_steps, hipStream_t s) {
    if (mode == kFp32Fast)
        resident_kernel<float>(w, mode, n_steps, s);
    else
        resident_kernel<double>(w, mode, n_steps, s);
}

size_t scatter_lds_bytes(Mode mode, int max_cc, int stage_max) {
    const size_t rb = mode == kFp32Fast ? sizeof(float) : sizeof(double);
    if (stage_max <= 0) return (size_t)kScatterWaves * max_cc * sizeof(int);
    return (size_t)(kScatterWaves + 1) * max_cc * sizeof(int) +
           (size_t)stage_max * (sizeof(int) + 4 * rb) + 16;
}

size_t wide_scatter_lds_bytes(Mode mode, int max_cc) {
    const int J = mode == kFp32Fast ? kWideRecs32 : kWideRecs64;
    const size_t rb = mode == kFp32Fast ? sizeof(float) : sizeof(double);
    const int nrt = max_cc < kWideRunKeys ? max_cc : kWideRunKeys;
    return (size_t)wide_ints(nrt, J) * sizeof(int) + (size_t)4 * J * kParticleThreads * rb;
}

size_t bucket_collide_lds_bytes(Mode mode, int cap) {
    const size_t rb = mode == kFp32Fast ? sizeof(float) : sizeof(double);
    return (size_t)kFastWaves * 64 * kGroupTableFactor * sizeof(uint32_t) +
           (size_t)2 * kMaxCellsPerKey * (sizeof(double) + sizeof(int)) + 3 * (size_t)cap * rb;
}

size_t fast_collide_lds_bytes(Mode mode, int cap, int waves) {
    const size_t rb = mode == kFp32Fast ? sizeof(float) : sizeof(double);
    return (size_t)waves * kCoopTablePerWave * sizeof(uint32_t) + 3 * (size_t)cap * rb;
}

void launch_init(const InstDesc& d, const InstDesc* d_desc, Mode mode, hipStream_t s) {
    const int n = d.N > d.Cc ? d.N : d.Cc;
    const dim3 grid((n + 255) / 256);
    if (mode == kFp32Fast)
        hipLaunchKernelGGL(k_init<float>, grid, dim3(256), 0, s, d_desc);
    else
        hipLaunchKernelGGL(k_init<double>, grid, dim3(256), 0, s, d_desc);
}

void launch_step(const Work& w, Mode mode, unsigned phase, hipStream_t s) {
    if (mode == kFp32Fast)
        step_kernels<float>(w, mode, phase, s);
    else
        step_kernels<double>(w, mode, phase, s);
}

hipError_t configure_kernels(size_t max_dynamic_lds) {
    const int bytes = (int)max_dynamic_lds;
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (r != hipSuccess) e = r;
    };
    set((const void*)k_collide_fast<float, kCoopWaves>);
    set((const void*)k_collide_fast<double, kCoopWaves>);
    set((const void*)k_collide_fast<float, kCoopWavesAlone>);
    set((const void*)k_collide_fast<double, kCoopWavesAlone>);
    set((const void*)k_collide_bucket<float>);
    set((const void*)k_collide_bucket<double>);
    set((const void*)k_move_hist<float, true>);
    set((const void*)k_move_hist<float, false>);
    set((const void*)k_move_hist<double, true>);
    set((const void*)k_move_hist<double, false>);
    set((const void*)k_scatter<float>);
    set((const void*)k_scatter<double>);
    set((const void*)k_count<float, false>);
    set((const void*)k_count<double, false>);
    set((const void*)k_count<float, true>);
    set((const void*)k_count<double, true>);
    set((const void*)k_move_scatter<float, false>);
    set((const void*)k_move_scatter<double, false>);
    set((const void*)k_move_scatter<float, true>);
    set((const void*)k_move_scatter<double, true>);
    set((const void*)k_move_scatter_wide<float, false>);
    set((const void*)k_move_scatter_wide<double, false>);
    set((const void*)k_move_scatter_wide<float, true>);
    set((const void*)k_move_scatter_wide<double, true>);
    set((const void*)k_scan_small);
    set((const void*)k_scan_seg);
    return e;
}

hipError_t configure_resident(size_t max_dynamic_lds) {
    const int bytes = (int)max_dynamic_lds;
    hipError_t e = hipSuccess;
    for (const void* f : {(const void*)k_resident<float, false>, (const void*)k_resident<float, true>,
                          (const void*)k_resident<double, false>, (const void*)k_resident<double, true>}) {
        const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (r != hipSuccess) e = r;
    }
    return e;
}

void launch_step_timed(const Work& w, Mode mode, unsigned phase, hipStream_t s, hipEvent_t* ev) {
    if (mode == kFp32Fast)
        step_kernels<float>(w, mode, phase, s, ev);
    else
        step_kernels<double>(w, mode, phase, s, ev);
}

void launch_finalize(const InstDesc* d_desc, int n_inst, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(n_inst), dim3(256), 0, s, d_desc);
}

void launch_finalize_staged(const InstDesc* d_desc, const int64_t* d_off, double* d_stage,
                            int n_inst, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_staged, dim3(n_inst), dim3(256), 0, s, d_desc, d_off, d_stage);
}

void launch_reset_window(const InstDesc* d_desc, int n_inst, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_window, dim3(n_inst), dim3(256), 0, s, d_desc);
}

void launch_gather_status(const InstDesc* d_desc, int n_inst, int32_t* d_out, hipStream_t s) {
    if (n_inst > 0)
        hipLaunchKernelGGL(k_gather_status, dim3((n_inst + 255) / 256), dim3(256), 0, s, d_desc, n_inst,
                           d_out);
}

void launch_finalize_gather(const InstDesc* const* d_descs, const int64_t* d_off, double* d_stage,
                            int n_inst, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_gather, dim3(n_inst), dim3(256), 0, s, d_descs, d_off, d_stage);
}

void launch_reset_window_gather(const InstDesc* const* d_descs, int n_inst, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_window_gather, dim3(n_inst), dim3(256), 0, s, d_descs);
}

}  // namespace dsmc

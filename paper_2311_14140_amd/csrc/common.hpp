// common.hpp -- device-resident descriptors shared by the kernels and the
// host runtime of the DSMC library.
#pragma once
#include <stdint.h>

namespace dsmc {

// Per-cell sums of a step: 1, vx, vy, vz, vx2, vy2, vz2, vxvy, vxvz, vyvz,
// v2vx, v2vy after the collisions, and vxvy before them (the only one of the
// stress's sums that the collisions change).
constexpr int kMoments = 13;
constexpr int kMomPreXY = 12;      // index of the pre-collision vxvy sum
constexpr int kEstPerCell = 9;     // n, ux, uy, uz, T, pxy, qx, qy, pxy_mid
constexpr int kParticleThreads = 256;  // threads per particle tile (move, scatter)
constexpr int kScatterWaves = kParticleThreads / 64;  // wavefronts of a scatter tile
constexpr int kColThreads = 256;       // cells per workgroup of the column-scan kernels
constexpr int kScanThreads = 1024;     // threads of the per-instance scan kernel
constexpr int kSegTiles = 32;          // tiles per column-scan segment
constexpr int kCountScanEntries = 8192;  // largest count matrix (tiles x keys) scanned in LDS
// largest (segments + 1) x keys of an instance whose three column scans run
// in one workgroup with its segment sums in LDS
constexpr int kSegScanEntries = 16384;
constexpr int kSegScanMinInstances = 4;  // instances a lane needs for that scan
constexpr int kFastWaves = 4;          // wavefronts per bucket-collide workgroup
constexpr int kCoopMin = 256;          // cells this full are collided by a whole workgroup
constexpr int kGroupTableFactor = 8;   // claim-table entries per lane of a small-cell group
// wavefronts of a workgroup-collide workgroup: 4, or 8 when its staged
// block takes more than half of a CU's LDS (then no second workgroup fits
// beside it, and the extra wavefronts hide latency instead); its claim table
// has 1024 entries per wavefront
constexpr int kCoopWaves = 4, kCoopWavesAlone = 8;
constexpr int kCoopTablePerWave = 1024;
constexpr int kMaxCellsPerKey = 128;   // cells of one sort bucket (a power of two up to this)
constexpr int kResidentKeys = 256;     // sort keys of an instance stepped by one workgroup
constexpr int kResidentWaves = 16;     // wavefronts of that workgroup
// records per lane the move-scatter holds in registers (FP32, FP64): tiles of
// bucket-sorted instances are 256 times this many slots
constexpr int kScatterRegs32 = 5, kScatterRegs64 = 4;
// records per thread of one chunk of a larger tile (FP32, FP64): the
// move-scatter walks such a tile in chunks of 256 times this many slots
constexpr int kWideRecs32 = 4, kWideRecs64 = 2;
constexpr int kWideKeys = 64;  // sort keys ranked per pass over a chunk (one wavefront's lanes)
// keys of a wide tile whose next destinations are kept in LDS (from the
// tile's smallest key on; any beyond use the tile's row in global memory)
constexpr int kWideRunKeys = 1024;

// Scalars an instance keeps on the device so that a step is the same launch
// sequence every time (and can be replayed from a graph).
struct DevScalars {
    int64_t step_done;            // steps completed
    int64_t n_sampled;            // sampled steps in the window
    int32_t status;               // bit 0: non-finite velocity, bit 1: particle count lost,
                                  // bit 2: a sorted slot out of range, bit 3: an
                                  // injection needed more slots than allocated
    int32_t pad_[3];
};

// State of an open boundary (a patch with a wall at y = 0 and an open
// boundary at its top, y = H of the descriptor).  The first six fields are
// the inflow the host sets (dsmc_set_inflow); the rest the kernels keep.
struct OpenState {
    double u_in;          // mean x velocity of the inflow (sqrt(kT_ref/m) units)
    double sqrt_tin;      // sqrt(T) of the inflow
    double vt_in;         // its thermal speed sqrt(2 T)
    double ce_a;          // Chapman-Enskog shear weight a of 1 - a C_x C_y
    double ce_A;          // bound of the weight used by the acceptance test
    double inj_expected;  // particles expected to enter per step
    double inj_rem;       // carried fractional part of the injections
    int64_t n_injected;   // particles injected since creation
    int64_t n_deleted;    // particles removed through the boundary since creation
    int32_t n_live;       // particles after the last sort (slots 0 .. n_live - 1)
    int32_t n_used;       // slots holding particles during the current step
};
constexpr int kOpenInflowDoubles = 6;   // leading doubles of OpenState set by the host

// Counters are kept per collision cell and written only by the wavefront
// that owns the cell: a single device-wide counter updated by every
// workgroup at the end of a kernel serialises hundreds of same-address
// atomics and costs far more than the kernel's own work.
//
// Everything a kernel needs to know about one instance.  Particle arrays are
// structure-of-arrays: buf[b][0..3] = y, vx, vy, vz of buffer b.  After step
// s the state lives in buffer (s & 1): the move of step s works in place on
// buffer ((s - 1) & 1) and the stable scatter writes buffer (s & 1).
//
// The global sort is by key = cell >> key_shift.  With key_shift = 0 the key
// is the collision cell and the scatter leaves the state sorted by cell
// (kcount / koffset are count / offset).  With key_shift > 0 a key is a
// bucket of 2^key_shift consecutive cells: the scatter leaves each bucket's
// particles contiguous, in their previous order, and the collide kernel
// finishes the sort by cell inside each bucket (writing count / offset).
// Both orders end as the stable sort of the particles by cell.
struct InstDesc {
    int32_t N, C, Cc, n_sub;           // nominal particles (C * ppc), sampling cells,
                                       // collision cells, Cc / C
    int32_t tiles, tile_items, nseg, ppc;  // particle tiles, items per tile, scan segments
    double H, dt, g, kntc, crmax0, sqrt_tw, inv_dy, pad0_;  // H: top of the domain
    int64_t n_transient;
    uint32_t key0, key1;
    uint32_t phase_mask;
    int32_t open;                      // 1: the top (y = H) is an open boundary
    int32_t nkeys, key_shift;          // sort keys, log2 of cells per key; an open
                                       // instance's last key gathers the particles
                                       // that left, past every cell
    int32_t ncap, pad2_;               // particle slots allocated (N when closed)
    OpenState* os;                     // open instances: the boundary's state
    void* buf[2][4];
    int32_t* cell;     // N: sort key of each slot (pre-sort order)
    int32_t* counts;   // tiles * nkeys: per-tile histogram, then per-tile scatter bases
    int32_t* tkeys;    // tiles * 2: smallest and largest sort key in each tile after the move
    int32_t* segsum;   // nseg * nkeys: per-segment column sums, then segment bases
    int32_t* kcount;   // nkeys: particles per key
    int32_t* koffset;  // nkeys: first slot of each key
    int32_t* count;    // Cc
    int32_t* offset;   // Cc
    double* crmax;     // Cc
    double* rem;       // Cc
    double* acc;       // kMoments * Cc, moment-major: moment k of cell c at k * Cc + c
    uint32_t* ncoll;   // Cc: accepted collisions in the window, per collision cell
    double* est;       // kEstPerCell * C + 3 (mass flow, sampled steps, collisions)
    DevScalars* sc;
};

}  // namespace dsmc

// kernels.hpp -- host-side launchers of the DSMC kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "common.hpp"

namespace dsmc {

enum Mode : int { kFp64Det = 0, kFp32Fast = 1, kFp64Fast = 2 };

// Work lists built by the runtime for a group of instances.
struct Work {
    const InstDesc* desc;   // device array, one per instance
    int n_inst;
    const int2* tiles;      // (instance, tile) for the particle kernels
    int n_tiles;
    int n_narrow;           // the first n_narrow tiles are held in registers by the
                            // move-scatter; the rest take its wide-tile kernel
    const int4* cols;       // (instance, cell chunk, segment) for the column scans
    int n_cols;
    const int4* cblocks;    // (instance, first cell, end cell) workgroup-staged collide blocks
    int n_cblocks;
    // FP64-det: (instance, first cell, end cell, 64) lane-per-cell collide blocks;
    // fast modes: (instance, bucket, G, 0) bucket collide blocks
    const int4* gblocks;
    int n_gblocks;
    int group_cap;          // particles a bucket collide workgroup stages in LDS
    int max_cc;             // largest sort-key count (LDS of histograms)
    int stage_max;          // tiles of at most this many slots are staged in LDS by the scatter
    size_t scatter_lds;     // dynamic LDS of the move-scatter
    size_t wide_lds;        // and of its wide-tile kernel
    int fast_cap;           // particles a fast-collide workgroup stages in LDS
    int coop_waves;         // wavefronts of a fast-collide workgroup
    int has_open;           // some instance has an open boundary (open-boundary kernel variants)
    // resident lanes (every member small): (instance, G) per workgroup of
    // k_resident, which then runs whole steps instead of the lists above
    const int2* resident;
    int n_resident;
    int resident_cap;       // particle slots each resident workgroup holds in LDS
    // > 0: every instance's count matrix fits one workgroup's LDS, and k_scan_small
    // (this many bytes of it) replaces the three column-scan kernels
    int scan_small_lds;
    // > 0 (and scan_small_lds 0): every instance's segment sums fit LDS, and
    // k_scan_seg (this many bytes of it) replaces the three column-scan kernels
    int scan_seg_lds;
    // dynamic LDS of the count, move-scatter and collide launches is at
    // least this many bytes (0: what they use): it caps how many of their
    // workgroups share a CU, the occupancy knob of the launch-shape tuning
    size_t lds_floor;
    size_t lds_floor_coop;  // the same cap for the workgroup collide's larger workgroups
};

void launch_init(const InstDesc& d, const InstDesc* d_desc, Mode mode, hipStream_t s);
// One step of every instance in the group; phase is a DSMC_PHASE_* mask.
void launch_step(const Work& w, Mode mode, unsigned phase, hipStream_t s);
// The same step with an event recorded before each of its kernels and one
// after the last (ev must hold 7 events); the kernel order is the one of
// dsmc_profile_step.
void launch_step_timed(const Work& w, Mode mode, unsigned phase, hipStream_t s, hipEvent_t* ev);
// n_steps whole steps of a resident lane in one launch.
void launch_resident(const Work& w, Mode mode, int64_t n_steps, hipStream_t s);
// Particle slots an instance may hold to be stepped by one workgroup.
int resident_slots(Mode mode);
size_t resident_lds_bytes(Mode mode, int slot_cap);
void launch_finalize(const InstDesc* d_desc, int n_inst, hipStream_t s);
// Estimators of n_inst instances into stage: instance b at d_off[b], its
// kEstPerCell * C + 3 values followed by its status word.
void launch_finalize_staged(const InstDesc* d_desc, const int64_t* d_off, double* d_stage,
                            int n_inst, hipStream_t s);
void launch_reset_window(const InstDesc* d_desc, int n_inst, hipStream_t s);
// Status word of each of n_inst instances into d_out.
void launch_gather_status(const InstDesc* d_desc, int n_inst, int32_t* d_out, hipStream_t s);
// The same two from a device table of pointers to each instance's descriptor.
void launch_finalize_gather(const InstDesc* const* d_descs, const int64_t* d_off, double* d_stage,
                            int n_inst, hipStream_t s);
void launch_reset_window_gather(const InstDesc* const* d_descs, int n_inst, hipStream_t s);
size_t fast_collide_lds_bytes(Mode mode, int cap, int waves);
size_t bucket_collide_lds_bytes(Mode mode, int cap);
size_t scatter_lds_bytes(Mode mode, int max_cc, int stage_max);
// LDS of the move-scatter's kernel for tiles larger than its registers hold.
size_t wide_scatter_lds_bytes(Mode mode, int max_cc);
// Allow dynamic LDS up to max_dynamic_lds bytes for the kernels that use it.
hipError_t configure_kernels(size_t max_dynamic_lds);
// The same for the resident kernel, which may take most of a CU's LDS.
hipError_t configure_resident(size_t max_dynamic_lds);

}  // namespace dsmc

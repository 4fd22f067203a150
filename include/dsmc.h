/*
 * dsmc.h -- C ABI of the MI355X DSMC micro-solver for force-driven, low-speed
 * rarefied flow between parallel plates (arXiv 2311.14140).
 *
 * The solver is the micro model of the paper's micro-macro-surrogate method:
 * DSMC (Sec. 1 and 2, Bird's method) for a monatomic gas between two plates
 * held at a fixed temperature and driven by a small acceleration parallel to
 * them (Sec. 2.1).  Its outputs are the fields the surrogates are trained on:
 * velocity and shear-stress profiles averaged over windows of time steps
 * (Sec. 2.2, Eqs. 11-13; Sec. 3: 100-step averages), plus density,
 * temperature, heat flux and the mass flow rate.
 *
 * Units follow the paper's statement of the problem: Kn is the hard-sphere
 * mean free path over the plate gap H (Sec. 1 defines Kn = lambda / L), the
 * body force is the dimensionless F = F' H / v0^2 of Eq. 6, the wall
 * temperature is relative to the reference temperature, and time is in
 * H / sqrt(k T_ref / m).  Returned velocities, heat fluxes and the mass flow
 * are over v0 = sqrt(2 k T_ref / m) and stresses over P0 = n k T_ref, the
 * normalisation of Eq. 6.
 *
 * Conventions for every call:
 *   - Status codes: DSMC_OK (0) or a negative DSMC_ERR_*; nothing aborts or
 *     throws across the ABI.
 *   - Out-parameters are written only on success (*out handles are set to
 *     NULL on failure).
 *   - Pointers documented as "host" are ordinary host memory owned by the
 *     caller; pointers documented as "device" are device memory on the
 *     current HIP device, borrowed by the library.
 *   - A handle is used by one host thread at a time; distinct handles are
 *     independent.  dsmc_step and dsmc_group_step only enqueue work; errors
 *     raised on the device surface at the next synchronising call
 *     (dsmc_sample, dsmc_get_state, dsmc_get_cells, dsmc_sync).
 */
#ifndef DSMC_H_
#define DSMC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DSMC_OK = 0,
    DSMC_ERR_INVALID_ARG = -1,  /* bad parameter or pointer; nothing was done */
    DSMC_ERR_OUT_OF_MEMORY = -2,/* device allocation failed or arena too small */
    DSMC_ERR_DEVICE = -3,       /* a HIP call failed */
    DSMC_ERR_STATE = -4,        /* call not allowed in the handle's state */
    DSMC_ERR_NUMERIC = -5       /* non-finite velocity or lost particle seen on device */
};

/* Precision and collision scheme. */
enum {
    /* FP64 state and arithmetic, collisions sequential per cell in candidate
     * order, every operation in a fixed IEEE order with no FMA contraction:
     * reproduces the reference recipe bit for bit. */
    DSMC_FP64_DETERMINISTIC = 0,
    /* FP32 positions and velocities, FP64 accumulators; the candidates of a
     * cell run in parallel rounds (a group of 4..64 lanes per cell for cells
     * of fewer than 256 particles, a 256-thread workgroup for fuller ones),
     * NTC in distribution: each candidate pair is drawn and accepted exactly
     * as in the sequential scheme, and a candidate runs only after every
     * lower-numbered candidate that shares a particle with it.  Deterministic
     * run to run and independent of batching and launch shape. */
    DSMC_FP32_FAST = 1,
    /* The DSMC_FP32_FAST scheme with FP64 state. */
    DSMC_FP64_FAST = 2
};

/* Phase mask for tests (dsmc_params.debug_phase_mask); 0 means all. */
enum {
    DSMC_PHASE_MOVE = 1,
    DSMC_PHASE_SORT = 2,
    DSMC_PHASE_COLLIDE = 4,
    DSMC_PHASE_SAMPLE = 8,
    DSMC_PHASE_ALL = 15
};

typedef struct dsmc_params {
    uint32_t struct_size;       /* = sizeof(dsmc_params); ABI guard */
    int32_t precision;          /* DSMC_FP64_DETERMINISTIC | DSMC_FP32_FAST | DSMC_FP64_FAST */
    double kn;                  /* hard-sphere lambda / H, finite, > 0 */
    double body_force;          /* F of Eq. 6 along x, finite */
    double wall_temperature;    /* T_w / T_ref, finite, > 0 */
    double dt;                  /* time step; <= 0 selects 0.2 min(lambda, H) / sqrt(2) */
    int32_t n_cells;            /* sampling cells across the gap, >= 1 */
    int32_t particles_per_cell; /* initial particles per sampling cell, >= 1 */
    int32_t n_sub;              /* collision cells per sampling cell, >= 1 (1 = plain);
                                   n_cells * n_sub <= 10240 */
    uint32_t debug_phase_mask;  /* DSMC_PHASE_* subset for tests; 0 = all */
    int64_t n_transient;        /* steps before sampling starts, >= 0 */
    uint64_t seed;              /* key of every random stream */
    double domain_length;       /* 0: the closed gap [0, H] between the two plates.
                                   L in (0, H]: a patch of the hybrid (Sec. 2, Sec. 3.2):
                                   the plate at y = 0 and an open boundary at y = L, the
                                   n_cells cells spanning [0, L]; particles crossing L
                                   outward are removed and particles enter through it from
                                   the inflow set by dsmc_set_inflow (Chapman-Enskog,
                                   default: at rest at T_w).  The particle count then
                                   varies around n_cells * particles_per_cell; slots are
                                   allocated for 25% more (at least 8 standard deviations
                                   + 64).  Requires debug_phase_mask = 0. */
} dsmc_params;

/* Estimators over the current window (all arrays host, caller-owned, length
 * n_cells; any array pointer may be NULL to skip it). */
typedef struct dsmc_moments {
    int32_t n_cells;            /* in: capacity of the arrays (>= the handle's cells) */
    int32_t pad_;
    int64_t n_sampled_steps;    /* out: sampled steps K in the window */
    double *n;                  /* density over the mean density */
    double *ux, *uy, *uz;       /* mean velocity over v0 */
    double *T;                  /* temperature over T_ref */
    double *pxy;                /* shear stress P_xy over P0, sampled after the collisions */
    double *qx, *qy;            /* heat flux over P0 v0 */
    double *raw_sums;           /* optional: n_cells*n_sub*13 FP64 sums per collision cell:
                                   1, vx, vy, vz, vx2, vy2, vz2, vxvy, vxvz, vyvz, v2vx, v2vy
                                   after the collisions, then vxvy before them */
    double mass_flow;           /* out: integral of n u_x dy over (n_mean H v0); NaN if K = 0 */
    int64_t n_collisions;       /* out: accepted collisions in the window */
    double *pxy_mid;            /* time-centred shear stress over P0: the mean of the
                                   kinetic estimates before and after the collisions.
                                   Collisions relax the stress by about dt / tau_p per step,
                                   so the post-collision value sits that fraction below the
                                   momentum flux of the free flights; the mean of the two
                                   is the flux to second order in dt and satisfies the
                                   momentum balance dP/dy = 2F (Eqs. 1 and 6).  This is
                                   the P^DSMC of the constitutive surrogates (Eq. 13). */
} dsmc_moments;

typedef struct dsmc_handle dsmc_handle;
typedef struct dsmc_group dsmc_group;

/* Fill *p with the library defaults (Kn 1, F 0, T_w 1, 100 cells x 50,
 * default dt, FP64 deterministic). */
int dsmc_params_init(dsmc_params *p);

/* Device bytes an instance with these parameters needs from an arena. */
int dsmc_footprint_bytes(const dsmc_params *p, uint64_t *bytes);

/* Create one solver instance and enqueue its initial state: every sampling
 * cell gets exactly particles_per_cell particles, uniform inside it, with
 * Maxwellian velocities at the wall temperature.
 *   stream: a hipStream_t borrowed for all of the instance's work, or NULL
 *           for the legacy default stream; must outlive the handle.
 *   arena:  device memory of at least dsmc_footprint_bytes bytes, borrowed
 *           (must outlive the handle), or NULL for the library to allocate.
 * Errors: INVALID_ARG for bad parameters, OUT_OF_MEMORY, DEVICE. */
int dsmc_create(const dsmc_params *p, void *stream, void *arena, uint64_t arena_bytes,
                dsmc_handle **out);

/* Enqueue n_steps >= 0 DSMC steps (move with body force and diffuse walls;
 * stable sort by collision cell; NTC hard-sphere collisions; sampling after
 * the transient).  Asynchronous.  STATE if the handle belongs to a group. */
int dsmc_step(dsmc_handle *h, int64_t n_steps);

/* Synchronise, then fill *out with the estimators of the current window;
 * if reset_window != 0 start a new window afterwards.  Calling it with reset
 * every 100 steps gives the paper's training samples (Sec. 3).
 * NUMERIC if the device flagged a non-finite velocity or a lost particle. */
int dsmc_sample(dsmc_handle *h, dsmc_moments *out, int reset_window);

/* Wait for the handle's enqueued work; surfaces device errors. */
int dsmc_sync(dsmc_handle *h);

/* Release the handle (NULL-safe).  Removes it from its group if any. */
int dsmc_destroy(dsmc_handle *h);

/* Copy the particle state in slot order to host arrays of N elements (double
 * for the FP64 modes, float for FP32; N = n_cells * particles_per_cell, or
 * the n_live of dsmc_open_state for an open instance) and the steps
 * completed.  Any pointer may be NULL.  Synchronises. */
int dsmc_get_state(dsmc_handle *h, void *y, void *vx, void *vy, void *vz, int32_t *cell,
                   uint64_t *step);

/* Replace the particle state (same layout as dsmc_get_state; NULL leaves an
 * array unchanged) and the step counter.  With dsmc_set_cells it restores a
 * checkpoint exactly. */
int dsmc_set_state(dsmc_handle *h, const void *y, const void *vx, const void *vy,
                   const void *vz, const int32_t *cell, uint64_t step);

/* Inflow of an open instance (domain_length > 0) at its open boundary
 * (Sec. 2: the hybrid imposes the Chapman-Enskog distribution at the local
 * macro state there): mean x velocity u and its gradient du/dy in the units
 * of Eq. 6, temperature over T_ref and density over the nominal density.
 * Entering particles follow the flux-weighted distribution of pure shear,
 * f_Maxwell (1 - a C_x C_y) with C = (c - u)/sqrt(2 k T/m) and
 * a = (4 Kn/sqrt(pi)) du/dy / (n sqrt(T)) (Newton's law for hard spheres);
 * floor(expected + carried remainder) enter per step, the expected number
 * being the Maxwellian inward flux n sqrt(kT/(2 pi m)) dt times the nominal
 * line density.  Applies to the steps enqueued after the call (it waits for
 * the earlier ones).  INVALID_ARG if the instance is closed, any value is
 * non-finite, T <= 0, n < 0, |a| > 1 (a stress beyond half the pressure,
 * outside the expansion's range) or more particles would be expected per
 * step than there are slots. */
int dsmc_set_inflow(dsmc_handle *h, double u, double dudy, double temperature, double density);

/* Open instance: particles in the domain after the last step, and particles
 * injected and removed through the boundary since creation, and the carried
 * fraction of the injections (any pointer may be NULL).  Synchronises.
 * dsmc_get_state / dsmc_set_state of an open instance move n_live particles.
 * INVALID_ARG if the instance is closed; NUMERIC if the slots ran out
 * (an injection found no room; the allocation holds 25% over the nominal
 * count). */
int dsmc_open_state(dsmc_handle *h, int32_t *n_live, int64_t *n_injected, int64_t *n_removed,
                    double *inj_remainder);

/* Restore what dsmc_open_state returned (a checkpoint of an open instance:
 * this first, so that dsmc_set_state takes n_live particles, then
 * dsmc_set_state and dsmc_set_cells; the inflow is set again with
 * dsmc_set_inflow).  INVALID_ARG if the instance is closed, n_live exceeds
 * the slots, a count is negative or the remainder is outside [0, 1). */
int dsmc_set_open_state(dsmc_handle *h, int32_t n_live, int64_t n_injected, int64_t n_removed,
                        double inj_remainder);

/* Per collision cell (n_cells*n_sub each, host): crmax, the NTC remainder,
 * particle count and slot offset after the last sort.  NULL skips. */
int dsmc_get_cells(dsmc_handle *h, double *crmax, double *rem, int32_t *count,
                   int32_t *offset);
int dsmc_set_cells(dsmc_handle *h, const double *crmax, const double *rem,
                   const int32_t *count, const int32_t *offset);

/* Particles, collision cells and derived constants of a handle:
 * out[0..5] = dt, g (= 2F), K_ntc, crmax0, cells per unit length, lambda. */
int dsmc_info(const dsmc_handle *h, int32_t *n_particles, int32_t *n_coll_cells,
              double *constants6);

/* Per-phase timing: run n_steps >= 1 steps of the handle (real steps, launched
 * one kernel at a time on its stream) with HIP events around every kernel and
 * write the summed device milliseconds of each kernel to phase_ms[9] (host):
 * move+histogram, column sums, scan, column prefix, scatter, collide+sample,
 * and [6] = all kernels, [7] = wall time of the whole run, [8] = the part of
 * the collide slot spent in resident lanes (whose whole step is one kernel,
 * counted in the collide slot).  Synchronises. */
int dsmc_profile_step(dsmc_handle *h, int64_t n_steps, double *phase_ms);

const char *dsmc_status_string(int status);
/* Last error message of a handle (or of the library when h is NULL). */
const char *dsmc_last_error(const dsmc_handle *h);

/* ---------------------------------------------------------------- batching
 * A group runs many independent instances of one precision together: each
 * phase of a step is one launch over all members, and chunks of steps are
 * replayed from a captured HIP graph; a group of small instances instead runs
 * each in one workgroup for whole steps (dsmc_group_set_resident).
 * Per-instance arithmetic and ordering are the same as alone, so results do
 * not depend on the group's make-up. */
int dsmc_group_create(void *stream, dsmc_group **out);
/* Add an instance (INVALID_ARG if it already belongs to a group or its
 * precision differs from the group's). */
int dsmc_group_add(dsmc_group *g, dsmc_handle *h);
int dsmc_group_remove(dsmc_group *g, dsmc_handle *h);
/* Enqueue n_steps for every member. */
int dsmc_group_step(dsmc_group *g, int64_t n_steps);
int dsmc_group_sync(dsmc_group *g);
int dsmc_group_size(const dsmc_group *g, int32_t *n_members);
/* The windows of every member at once: the estimators of dsmc_sample for
 * member i (in the order the members were added, removals closing the gaps)
 * into outs[i], n_outs = the member count, and with reset_window != 0 a new
 * window for all of them.  One launch computes every member's estimators
 * into a device staging buffer, one copy brings it to pinned host memory and
 * one synchronisation of the group's stream ends the call, instead of a
 * launch, copies and a synchronisation per member: the way to take the
 * 100-step training samples of Sec. 3 from many instances.  Raw sums are
 * not returned (raw_sums must be NULL; dsmc_sample gives them).  The staging
 * buffers are allocated on the first call after the membership changes and
 * kept with the group.  NUMERIC if a member flagged a non-finite velocity or
 * a lost particle: that member's n_sampled_steps is set to -1, its arrays are
 * left untouched, the others are filled, and the error message names the
 * first such member.  INVALID_ARG for a wrong n_outs, a too-small n_cells or
 * non-NULL raw_sums. */
int dsmc_group_sample(dsmc_group *g, dsmc_moments *outs, int32_t n_outs, int reset_window);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): dsmc_group_sample with
 * the same arguments, results and errors, which calls no hipMalloc, hipFree
 * or other allocating routine.  Its descriptor table, offsets and device
 * staging live in one fixed 32 MiB device array of the library (each GPU
 * holds its own copy until the process ends), and the host side of the
 * staging in a fixed host array; nothing is kept with the group.  Limits:
 * at most 1024 members, and the members' estimators (9 n_cells + 4 doubles
 * each, rounded up to 32) within 32 MiB less 16 KiB; beyond them INVALID_ARG
 * and nothing is done.  The current HIP device must be the group's.  Calls
 * in one process are serialised by a lock and each synchronises the group's
 * stream before it returns, so the array keeps the last call's contents;
 * every value read back is written by the call itself.  Calls that overlap
 * on one GPU from outside that lock would race on the array. */
int dsmc_group_sample_noalloc(dsmc_group *g, dsmc_moments *outs, int32_t n_outs,
                              int reset_window);
/* Lanes the members were split into at the last step: a group of at least
 * 2e6 particles and two or more members runs in two lanes (each with its own
 * stream, work lists and step graph, forked from and joined back to the
 * group's stream), so each of a step's kernels is launched once per lane.
 * Results do not depend on it. */
int dsmc_group_lanes(const dsmc_group *g, int32_t *n_lanes);
/* The lanes of the last step in more detail: all lanes, those stepped
 * resident, and the nominal particles and collision cells of the members in
 * resident lanes (any pointer may be NULL).  A group that mixes members small enough to run
 * resident (see dsmc_group_set_resident) with larger ones steps the small
 * ones in a lane of their own, beside the multi-kernel lanes of the others,
 * so a step launches the multi-kernel phases once per multi-kernel lane. */
int dsmc_group_lane_info(const dsmc_group *g, int32_t *n_lanes, int32_t *resident_lanes,
                         int64_t *resident_particles, int64_t *resident_cells);
int dsmc_group_destroy(dsmc_group *g);

/* Launch-shape tuning of a group: tile_mult multiplies each member's base
 * particle tile (the slots one move or scatter workgroup walks; 1..16) and
 * particles_per_block sets how many particles' worth of collision cells one
 * collide workgroup takes.  For instances with fewer than 256 particles per
 * collision cell in the fast modes this is the size of a sort bucket (a
 * power of two of cells, default about 2048 particles in FP32 and 1024 in
 * FP64): the global sort orders particles by bucket and the collide
 * workgroup of the bucket sorts it by cell in LDS.  For fuller cells it packs
 * cells into one LDS-staged collide workgroup (default one cell each).
 * waves_per_cu (0, or 4..32) caps the wavefronts of the count, move-scatter
 * and collide kernels that share a CU: each 4-wavefront workgroup then asks
 * for 1/(waves_per_cu/4) of the CU's LDS, so at most that many fit.  0 keeps
 * the automatic choice (for waves_per_cu: what registers and the LDS the
 * kernels use allow).  Results (particle states and window sums) do not
 * depend on any of them: the lanes per cell that add up a cell's moments
 * are the instance's own, whatever the bucket size.  INVALID_ARG out of
 * range. */
int dsmc_group_set_tuning(dsmc_group *g, int32_t tile_mult, int32_t particles_per_block,
                          int32_t waves_per_cu);
/* Resident stepping of small instances (on by default).  When every member
 * of a lane is small -- a fast mode, fewer than 256 particles per collision
 * cell, at most 256 collision cells (255 for an open instance) and at most
 * 6144 particle slots in FP32 or 3072 in FP64_FAST -- the lane runs each
 * member in one workgroup that holds its particles in LDS and performs whole
 * steps (move, stable sort by cell, collisions, sampling) back to back, as
 * many per launch as dsmc_step / dsmc_group_step enqueue (in launches of up
 * to 4096 steps), instead of a launch per phase.  Results are identical
 * bit for bit either way; enable = 0 keeps the multi-kernel step.  Under
 * dsmc_profile_step a resident lane's step appears as one kernel in the
 * collide slot, and its other slots read 0.  INVALID_ARG unless enable is 0
 * or 1. */
int dsmc_group_set_resident(dsmc_group *g, int32_t enable);
/* Choose the group's launch shape on its own steps: every pair of tile_mult
 * in {1, 2, 4} and particles_per_block in {0, 1024, 4096} at the automatic
 * occupancy, then waves_per_cu in {8, 12, 16} at the fastest pair (4 steps
 * per shape, 3 of them timed with HIP events on the group's stream; they
 * are real steps of the members), keeping the fastest of all.  The choice is
 * cached per group shape (precision and the particles and collision cells of
 * every member), in the process and, if DSMC_AUTOTUNE_CACHE names a file,
 * across processes.  Writes the choice to the three out-parameters (any may
 * be NULL).  STATE if the group is empty. */
int dsmc_group_autotune(dsmc_group *g, int32_t *tile_mult, int32_t *particles_per_block,
                        int32_t *waves_per_cu);

#ifdef __cplusplus
}
#endif

#endif /* DSMC_H_ */

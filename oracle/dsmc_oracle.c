/*
 * dsmc_oracle.c -- plain, sequential, FP64 DSMC for force-driven flow between
 * parallel plates (arXiv 2311.14140, Sec. 2.1: a monatomic gas between two
 * isothermal plates driven by a small acceleration parallel to them; the DSMC
 * micro model of Sec. 1-2 and Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU path is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header, table or constant generator with
 * the GPU library; the two are written independently from the same recipe.
 *
 * The paper does not spell out its DSMC algorithm.  What is written here is
 * textbook DSMC (Bird's method, the paper's reference for DSMC in Sec. 1 and
 * Sec. 2): hard-sphere molecules, no-time-counter (NTC) collision selection
 * within cells, fully diffuse isothermal walls, and a uniform body force.
 * Every choice the paper leaves open is taken as follows (the "readings"):
 *   - Kn is the hard-sphere mean free path over the plate gap H (Sec. 1 defines
 *     Kn = lambda / L).
 *   - Units: m = k_B = T_ref = H = 1; velocities in sqrt(kT_ref/m), so the
 *     paper's most probable speed v0 = sqrt(2); the paper's dimensionless force
 *     F (Eq. 6) becomes the code acceleration g = 2 F.
 *   - dt defaults to 0.2 min(lambda, H) / sqrt(2).
 *   - Initial state: exactly ppc particles per cell, uniform in the cell,
 *     Maxwellian at the wall temperature.
 *   - Force integration is exact per free-flight segment; walls are fully
 *     diffuse at T_w, multiple wall hits per step are followed.
 *   - Collision selection is NTC with the N(N-1) pair count and a carried
 *     fractional remainder; crmax starts at 5 sqrt(2 T_w) and is raised in
 *     candidate order before the acceptance test.  Optional collision
 *     sub-cells (n_sub per sampling cell) narrow the collision cells only.
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed
 *     by the seed and counted by (step, entity, sub-index, tag and call);
 *     uniforms in (0,1] with 53 random bits; logarithm by the atanh series;
 *     normal pairs by the Marsaglia-Bray polar method; isotropic directions by
 *     Marsaglia's (1972) sphere-point method.  No trigonometric function.
 *   - Sampling accumulates twelve FP64 sums per cell every step after the
 *     transient, after the collide phase, and the sum of vx vy before it;
 *     estimators give density, velocity, temperature, shear stress, heat flux
 *     and the mass flow rate.  The shear stress P^DSMC of Eq. 13 is taken as
 *     the time-centred estimate, the mean of the kinetic stresses before and
 *     after the collisions: collisions relax the stress by about dt / tau_p per
 *     step, so the value after them is that fraction below the momentum flux
 *     carried by the free flights, while the mean is that flux to second order
 *     in dt (it satisfies the momentum balance of Eqs. 1 and 6).  The
 *     post-collision stress is reported as well.
 *
 * Build: cc -O2 -ffp-contract=off -fPIC -shared (no fast-math).  Every
 * floating-point expression below is written in the order it is evaluated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TAG_INIT 1u
#define TAG_WALL 2u
#define TAG_COLL 3u
#define TAG_INJECT 5u

static const double PI = 0x1.921fb54442d18p+1; /* pi, correctly rounded */

#define PHASE_MOVE 1u
#define PHASE_SORT 2u
#define PHASE_COLLIDE 4u
#define PHASE_SAMPLE 8u
#define PHASE_ALL 15u

#define NMOM 13 /* 1, vx, vy, vz, vx2, vy2, vz2, vxvy, vxvz, vyvz, v2vx, v2vy after the
                   collisions; vxvy before them */

typedef struct or_params {
    double kn;
    double body_force;
    double wall_temperature;
    double dt;
    int32_t n_cells;
    int32_t particles_per_cell;
    int32_t n_sub;
    int32_t pad_;
    int64_t n_transient;
    uint64_t seed;
    double domain_length; /* 0: the closed gap [0, H]; L in (0, H]: a wall at 0 and
                             an open boundary at L (a DSMC patch of the hybrid) */
} or_params;

typedef struct or_state {
    or_params p;
    int32_t C;    /* sampling cells */
    int32_t Cc;   /* collision cells = C * n_sub */
    int32_t N;    /* particles in the domain (after the last sort) */
    int32_t Nnom; /* nominal particles: C * ppc, the initial count */
    int32_t Ncap; /* slots allocated (open domains hold a margin above Nnom) */
    int32_t Nused;/* slots holding particles during a step: N plus those injected */
    int open;     /* 1 if the top of the domain is an open boundary */
    double H, L, lam, dt, g, kntc, crmax0, sqrt_tw, inv_dy;
    /* inflow at the open boundary: mean x velocity (code units), sqrt(T),
     * thermal speed sqrt(2T), the Chapman-Enskog shear weight a and its
     * bound A, particles expected to enter per step and the carried remainder */
    double u_in, sqrt_tin, vt_in, ce_a, ce_A, inj_expected, inj_rem;
    int64_t n_injected, n_deleted;
    int32_t status;     /* bit 0: an injection needed more slots than allocated */
    uint32_t key[2];
    double *y, *vx, *vy, *vz;
    int32_t *cell;
    double *crmax, *rem;
    int32_t *count, *offset;
    double *acc;
    int64_t step;       /* steps completed */
    int64_t n_sampled;  /* sampled steps in the current window */
    int64_t n_coll;     /* accepted collisions in the current window */
    int64_t n_hits;     /* wall hits since creation */
    double wall_dpx;    /* x momentum given to the walls since creation */
    double wall_de;     /* kinetic energy given to the walls since creation */
    /* sort scratch */
    double *ty, *tvx, *tvy, *tvz;
    int32_t *tcell;
} or_state;

/* ---------------------------------------------------------------- Philox */
/* Philox4x32-10, SC'11 (Salmon et al.), Sec. 4: each round multiplies two
 * counter words by fixed odd constants, mixes the high halves with the other
 * two words and the key, and the key is advanced by the Weyl constants. */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* A random stream: fixed (key, step, entity, sub, tag); successive calls
 * advance the low 24 bits of the last counter word. */
typedef struct stream {
    uint32_t key[2];
    uint32_t step, entity, sub, tag;
    uint32_t call;
} stream;

static stream make_stream(const uint32_t key[2], int64_t step, int64_t entity,
                          int64_t sub, uint32_t tag)
{
    stream s;
    s.key[0] = key[0];
    s.key[1] = key[1];
    s.step = (uint32_t)step;
    s.entity = (uint32_t)entity;
    s.sub = (uint32_t)sub;
    s.tag = tag;
    s.call = 0;
    return s;
}

static void stream_next(stream *s, uint32_t x[4])
{
    uint32_t ctr[4];
    ctr[0] = s->step;
    ctr[1] = s->entity;
    ctr[2] = s->sub;
    ctr[3] = (s->tag << 24) | (s->call & 0xFFFFFFu);
    or_philox(ctr, s->key, x);
    s->call += 1;
}

/* A uniform in (0,1]: 53 random bits k taken as 27 high bits of one word and
 * 26 of the next, mapped to (k + 1) 2^-53.  Exact, never zero. */
static double u53(uint32_t a, uint32_t b)
{
    uint64_t k = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return (double)(k + 1u) * 0x1p-53;
}

/* Two uniforms from one call (words 0,1 and words 2,3). */
static void stream_uniform2(stream *s, double *ua, double *ub)
{
    uint32_t x[4];
    stream_next(s, x);
    *ua = u53(x[0], x[1]);
    *ub = u53(x[2], x[3]);
}

/* Natural logarithm of u in (0,1] by the atanh series:
 * u = 2^e m with m in [1/sqrt2, sqrt2], ln m = 2 atanh(s), s = (m-1)/(m+1),
 * 2 atanh(s) = 2 s (1 + z/3 + z^2/5 + ...), z = s^2, summed by Horner from
 * the z^11 term down; then ln u = e ln2 + 2 s P. */
double or_log(double u)
{
    static const double LN2 = 0x1.62e42fefa39efp-1;
    uint64_t bits;
    memcpy(&bits, &u, sizeof bits);
    int e = (int)((bits >> 52) & 0x7FFu) - 1023;
    uint64_t mb = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &mb, sizeof m);
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    double f = m - 1.0;
    double s = f / (m + 1.0);
    double z = s * s;
    double P = 1.0 / 23.0;
    for (int i = 10; i >= 0; --i) {
        double ci = 1.0 / (double)(2 * i + 1);
        P = P * z + ci;
    }
    return (double)e * LN2 + (s * P) * 2.0;
}

/* Marsaglia-Bray polar method: a normal pair with variance var_sqrt^2. */
static void stream_normal2(stream *s, double sqrt_var, double *n0, double *n1)
{
    for (;;) {
        double ua, ub;
        stream_uniform2(s, &ua, &ub);
        double a = 2.0 * ua - 1.0;
        double b = 2.0 * ub - 1.0;
        double q = a * a + b * b;
        if (q > 0.0 && q < 1.0) {
            double f = sqrt((-2.0 * or_log(q)) / q);
            *n0 = (a * f) * sqrt_var;
            *n1 = (b * f) * sqrt_var;
            return;
        }
    }
}

/* Marsaglia (1972): a point uniform on the unit sphere. */
static void stream_sphere(stream *s, double d[3])
{
    for (;;) {
        double ua, ub;
        stream_uniform2(s, &ua, &ub);
        double a = 2.0 * ua - 1.0;
        double b = 2.0 * ub - 1.0;
        double q = a * a + b * b;
        if (q < 1.0) {
            double r = 2.0 * sqrt(1.0 - q);
            d[0] = a * r;
            d[1] = b * r;
            d[2] = 1.0 - 2.0 * q;
            return;
        }
    }
}

/* Exposed primitives for the tests. */
void or_uniform2(const uint32_t key[2], int64_t step, int64_t entity, int64_t sub,
                 uint32_t tag, uint32_t call, double out[2])
{
    stream s = make_stream(key, step, entity, sub, tag);
    s.call = call;
    stream_uniform2(&s, &out[0], &out[1]);
}

void or_normal2(const uint32_t key[2], int64_t step, int64_t entity, int64_t sub,
                uint32_t tag, uint32_t call, double sqrt_var, double out[2])
{
    stream s = make_stream(key, step, entity, sub, tag);
    s.call = call;
    stream_normal2(&s, sqrt_var, &out[0], &out[1]);
}

void or_sphere(const uint32_t key[2], int64_t step, int64_t entity, int64_t sub,
               uint32_t tag, uint32_t call, double out[3])
{
    stream s = make_stream(key, step, entity, sub, tag);
    s.call = call;
    stream_sphere(&s, out);
}

/* --------------------------------------------------------------- state */
static int params_valid(const or_params *p)
{
    if (!(isfinite(p->kn) && p->kn > 0.0)) return 0;
    if (!isfinite(p->body_force)) return 0;
    if (!(isfinite(p->wall_temperature) && p->wall_temperature > 0.0)) return 0;
    if (!isfinite(p->dt)) return 0;
    if (p->n_cells < 1 || p->particles_per_cell < 1 || p->n_sub < 1) return 0;
    if ((int64_t)p->n_cells * (int64_t)p->particles_per_cell > 2147483647) return 0;
    if ((int64_t)p->n_cells * (int64_t)p->n_sub > 2147483647) return 0;
    if (p->n_transient < 0) return 0;
    if (!(isfinite(p->domain_length) && p->domain_length >= 0.0 && p->domain_length <= 1.0))
        return 0;
    return 1;
}

void or_destroy(or_state *S)
{
    if (!S) return;
    free(S->y); free(S->vx); free(S->vy); free(S->vz); free(S->cell);
    free(S->crmax); free(S->rem); free(S->count); free(S->offset); free(S->acc);
    free(S->ty); free(S->tvx); free(S->tvy); free(S->tvz); free(S->tcell);
    free(S);
}

/* Initial state: particle p sits in cell p / ppc, uniform inside it, with a
 * Maxwellian velocity at T_w (uses tag INIT, step field 0, entity p). */
static void init_particles(or_state *S)
{
    const int32_t ppc = S->p.particles_per_cell;
    const double dy = S->L / (double)S->C;
    for (int32_t p = 0; p < S->N; ++p) {
        int32_t c = p / ppc;
        stream s = make_stream(S->key, 0, p, 0, TAG_INIT);
        double ua, ub, dummy;
        stream_uniform2(&s, &ua, &ub);
        S->y[p] = ((double)c + (1.0 - ua)) * dy;
        stream_normal2(&s, S->sqrt_tw, &S->vx[p], &S->vy[p]);
        stream_normal2(&s, S->sqrt_tw, &S->vz[p], &dummy);
        S->cell[p] = 0;
    }
    for (int32_t c = 0; c < S->Cc; ++c) {
        S->crmax[c] = S->crmax0;
        S->rem[c] = 0.0;
        S->count[c] = 0;
        S->offset[c] = 0;
    }
}

void or_set_inflow(or_state *S, double u, double dudy, double T, double n);

or_state *or_create(const or_params *p)
{
    if (!p || !params_valid(p)) return NULL;
    or_state *S = (or_state *)calloc(1, sizeof *S);
    if (!S) return NULL;
    S->p = *p;
    S->C = p->n_cells;
    S->Cc = p->n_cells * p->n_sub;
    S->N = p->n_cells * p->particles_per_cell;
    S->Nnom = S->N;
    S->open = p->domain_length > 0.0;
    /* an open domain's count fluctuates about Nnom: room for 25% more, and at
     * least 8 standard deviations plus 64 */
    S->Ncap = S->N;
    if (S->open) {
        int64_t m1 = (int64_t)S->N / 4, m2 = (int64_t)(8.0 * sqrt((double)S->N)) + 64;
        int64_t cap = (int64_t)S->N + (m1 > m2 ? m1 : m2);
        if (cap > 2147483647) return NULL;
        S->Ncap = (int32_t)cap;
    }
    S->Nused = S->N;
    /* Constants, each evaluated once in double, left to right. */
    S->H = 1.0;
    S->L = S->open ? p->domain_length : S->H;
    S->lam = p->kn * S->H;
    if (p->dt > 0.0) {
        S->dt = p->dt;
    } else {
        double lref = S->lam < S->H ? S->lam : S->H;
        S->dt = (0.2 * lref) / sqrt(2.0);
    }
    S->g = 2.0 * p->body_force;
    S->kntc = (S->dt * (double)p->n_sub) / ((sqrt(2.0) * S->lam) * (double)p->particles_per_cell);
    S->crmax0 = 5.0 * sqrt(2.0 * p->wall_temperature);
    S->sqrt_tw = sqrt(p->wall_temperature);
    S->inv_dy = (double)S->Cc / S->L;
    S->key[0] = (uint32_t)(p->seed & 0xFFFFFFFFu);
    S->key[1] = (uint32_t)(p->seed >> 32);

    size_t n = (size_t)S->Ncap, cc = (size_t)S->Cc;
    S->y = malloc(n * sizeof(double));
    S->vx = malloc(n * sizeof(double));
    S->vy = malloc(n * sizeof(double));
    S->vz = malloc(n * sizeof(double));
    S->cell = malloc(n * sizeof(int32_t));
    S->ty = malloc(n * sizeof(double));
    S->tvx = malloc(n * sizeof(double));
    S->tvy = malloc(n * sizeof(double));
    S->tvz = malloc(n * sizeof(double));
    S->tcell = malloc(n * sizeof(int32_t));
    S->crmax = malloc(cc * sizeof(double));
    S->rem = malloc(cc * sizeof(double));
    S->count = malloc((cc + 1) * sizeof(int32_t));
    S->offset = malloc((cc + 1) * sizeof(int32_t));
    S->acc = calloc(cc * NMOM, sizeof(double));
    if (!S->y || !S->vx || !S->vy || !S->vz || !S->cell || !S->ty || !S->tvx ||
        !S->tvy || !S->tvz || !S->tcell || !S->crmax || !S->rem || !S->count ||
        !S->offset || !S->acc) {
        or_destroy(S);
        return NULL;
    }
    init_particles(S);
    or_set_inflow(S, 0.0, 0.0, p->wall_temperature, 1.0);
    return S;
}

/* ---------------------------------------------------------------- move */
/* Free flight for dt under the constant acceleration g along x, with diffuse
 * re-emission from a wall at T_w whenever the particle reaches y = 0 or y = H
 * before the time left runs out (Sec. 2.1: isothermal plates, acceleration
 * parallel to them).  The wall draw for the h-th hit of slot p in step s uses
 * tag WALL, entity p, sub-index h: call 0 gives the normal speed (Rayleigh,
 * sqrt(-2 T_w ln U)), later calls a polar normal pair for (vx, vz). */
static int move_one(or_state *S, int64_t step, int64_t slot, double *py, double *pvx,
                    double *pvy, double *pvz)
{
    double y = *py, vx = *pvx, vy = *pvy, vz = *pvz;
    double t = S->dt;
    int64_t h = 0;
    int gone = 0;
    for (;;) {
        double tw;
        if (vy > 0.0)
            tw = (S->L - y) / vy;
        else if (vy < 0.0)
            tw = (0.0 - y) / vy;
        else
            tw = INFINITY;
        if (tw >= t) {
            y = y + vy * t;
            vx = vx + S->g * t;
            break;
        }
        int top = vy > 0.0;
        if (top && S->open) {
            /* leaves through the open boundary */
            y = S->L;
            vx = vx + S->g * tw;
            gone = 1;
            break;
        }
        double vx_hit = vx + S->g * tw;
        double e_hit = (vx_hit * vx_hit + vy * vy) + vz * vz;
        y = top ? S->H : 0.0;
        t = t - tw;
        stream s = make_stream(S->key, step, slot, h, TAG_WALL);
        double ua, ub;
        stream_uniform2(&s, &ua, &ub);
        double vn = sqrt(-2.0 * or_log(ua)) * S->sqrt_tw;
        stream_normal2(&s, S->sqrt_tw, &vx, &vz);
        vy = top ? -vn : vn;
        double e_new = (vx * vx + vy * vy) + vz * vz;
        S->n_hits += 1;
        S->wall_dpx += vx_hit - vx;
        S->wall_de += 0.5 * (e_hit - e_new);
        h += 1;
    }
    if (y < 0.0) y = 0.0;
    if (y > S->L) y = S->L;
    *py = y;
    *pvx = vx;
    *pvy = vy;
    *pvz = vz;
    return gone;
}

static int32_t cell_of(const or_state *S, double y)
{
    int32_t c = (int32_t)(y * S->inv_dy);
    if (c >= S->Cc) c = S->Cc - 1;
    return c;
}

/* --------------------------------------------------------------- inflow */
/* Inflow state at the open boundary (the paper's hybrid imposes the
 * Chapman-Enskog distribution at the local macro state there, Sec. 2 and
 * Sec. 3.2): u and du/dy in the units of Eq. 6, T over T_ref, n over the
 * nominal density.  For pure shear the Chapman-Enskog factor is
 * 1 - a C_x C_y with C = (c - u)/sqrt(2T) and a = -2 P_xy / (n T), where
 * Newton's law gives P_xy = -(2 Kn/sqrt(pi)) sqrt(T) du/dy for hard spheres
 * (viscosity ~ sqrt(T)); so a = (4 Kn/sqrt(pi)) du/dy / (n sqrt(T)).  The
 * inward number flux is the Maxwellian one, n sqrt(T/(2 pi)) per unit area
 * and time in these units (the shear term carries no net number flux). */
void or_set_inflow(or_state *S, double u, double dudy, double T, double n)
{
    S->u_in = u * sqrt(2.0);
    S->sqrt_tin = sqrt(T);
    S->vt_in = sqrt(2.0 * T);
    S->ce_a = (((4.0 * S->p.kn) / sqrt(PI)) * dudy) / (n * S->sqrt_tin);
    S->ce_A = 1.0 + 16.0 * fabs(S->ce_a);
    S->inj_expected = ((n * ((double)S->Nnom / S->L)) * sqrt(T / (2.0 * PI))) * S->dt;
}

/* Particles entering through the open boundary at the start of a step:
 * floor(expected + carried remainder) of them, appended after the N live
 * slots.  Particle k of step s draws from tag INJECT, entity k: per attempt
 * one call gives the acceptance uniform and the flux-weighted inward speed
 * sqrt(-2 T ln U), a polar pair from the following calls gives the thermal
 * x and z velocities, and the attempt is kept with probability
 * (1 - a C_x C_y) / A; a last call gives the time fraction U of the step it
 * spends inside.  It is placed where a straight flight of the whole step
 * brings it across the boundary at that time, beyond the boundary, with the
 * force's x velocity gain of the outside part taken off, so that the
 * ordinary move delivers it with the drawn velocity at the boundary.
 * Returns the number injected. */
void or_inject_one(const or_state *S, int64_t step, int64_t k, double st[4])
{
    stream s = make_stream(S->key, step, k, 0, TAG_INJECT);
    double sp, tx, tz;
    for (;;) {
        double ua, ub;
        stream_uniform2(&s, &ua, &ub);
        sp = sqrt(-2.0 * or_log(ub)) * S->sqrt_tin;
        stream_normal2(&s, S->sqrt_tin, &tx, &tz);
        double cx = tx / S->vt_in;
        double cy = -sp / S->vt_in;
        double gam = 1.0 - S->ce_a * (cx * cy);
        if (ua * S->ce_A < gam) break;
    }
    double ut, unused;
    stream_uniform2(&s, &ut, &unused);
    double outside = S->dt - ut * S->dt;
    st[0] = S->L + sp * outside;
    st[1] = (S->u_in + tx) - S->g * outside;
    st[2] = -sp;
    st[3] = tz;
}

static int32_t inject(or_state *S, int64_t step)
{
    double m = S->inj_expected + S->inj_rem;
    double f = floor(m);
    S->inj_rem = m - f;
    int64_t n = (int64_t)f;
    if ((int64_t)S->N + n > (int64_t)S->Ncap) {
        S->status |= 1;
        n = (int64_t)S->Ncap - (int64_t)S->N;
    }
    for (int64_t k = 0; k < n; ++k) {
        double st[4];
        or_inject_one(S, step, k, st);
        int32_t q = S->N + (int32_t)k;
        S->y[q] = st[0];
        S->vx[q] = st[1];
        S->vy[q] = st[2];
        S->vz[q] = st[3];
        S->cell[q] = 0;
    }
    S->n_injected += n;
    return (int32_t)n;
}

/* Move every slot; a particle that leaves through the open boundary gets the
 * key Cc, after every cell, so that the sort gathers the removed particles
 * past the live ones. */
static void phase_move(or_state *S, int64_t step)
{
    int32_t n = S->N;
    if (S->open) n += inject(S, step);
    S->Nused = n;
    for (int32_t p = 0; p < n; ++p) {
        int gone = move_one(S, step, p, &S->y[p], &S->vx[p], &S->vy[p], &S->vz[p]);
        S->cell[p] = gone ? S->Cc : cell_of(S, S->y[p]);
        S->n_deleted += gone;
    }
}

/* ---------------------------------------------------------------- sort */
/* Stable sort of the slots by collision cell: counting sort, counts, exclusive
 * offsets, then a forward pass placing each slot after the earlier slots of
 * its cell. */
void or_stable_sort_perm(int32_t n, const int32_t *key, int32_t nkeys, int32_t *count,
                         int32_t *offset, int32_t *perm)
{
    for (int32_t c = 0; c < nkeys; ++c) count[c] = 0;
    for (int32_t i = 0; i < n; ++i) count[key[i]] += 1;
    int32_t run = 0;
    for (int32_t c = 0; c < nkeys; ++c) {
        offset[c] = run;
        run += count[c];
    }
    int32_t *next = (int32_t *)malloc((size_t)(nkeys > 0 ? nkeys : 1) * sizeof(int32_t));
    for (int32_t c = 0; c < nkeys; ++c) next[c] = offset[c];
    for (int32_t i = 0; i < n; ++i) perm[next[key[i]]++] = i;
    free(next);
}

static void phase_sort(or_state *S)
{
    const int32_t n = S->Nused;
    int32_t *perm = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    or_stable_sort_perm(n, S->cell, S->Cc + S->open, S->count, S->offset, perm);
    for (int32_t d = 0; d < n; ++d) {
        int32_t s = perm[d];
        S->ty[d] = S->y[s];
        S->tvx[d] = S->vx[s];
        S->tvy[d] = S->vy[s];
        S->tvz[d] = S->vz[s];
        S->tcell[d] = S->cell[s];
    }
    double *t;
    t = S->y; S->y = S->ty; S->ty = t;
    t = S->vx; S->vx = S->tvx; S->tvx = t;
    t = S->vy; S->vy = S->tvy; S->tvy = t;
    t = S->vz; S->vz = S->tvz; S->tvz = t;
    int32_t *tc = S->cell; S->cell = S->tcell; S->tcell = tc;
    free(perm);
    /* the removed particles sit past the live ones */
    if (S->open) S->N = S->offset[S->Cc];
    S->Nused = S->N;
}

/* ------------------------------------------------------------- collide */
/* NTC within each collision cell: M_real = N(N-1)/2 crmax K + rem candidates,
 * each a uniformly drawn distinct pair, accepted with probability c_r/crmax
 * (hard spheres), scattered isotropically in the centre-of-mass frame. */
static void collide_cell(or_state *S, int64_t step, int32_t c)
{
    int32_t n = S->count[c];
    if (n < 2) return;
    double *vx = S->vx + S->offset[c];
    double *vy = S->vy + S->offset[c];
    double *vz = S->vz + S->offset[c];
    double m_real = (((0.5 * (double)n) * (double)(n - 1)) * S->crmax[c]) * S->kntc + S->rem[c];
    double m_floor = floor(m_real);
    S->rem[c] = m_real - m_floor;
    int64_t M = (int64_t)m_floor;
    for (int64_t k = 0; k < M; ++k) {
        stream s = make_stream(S->key, step, c, k, TAG_COLL);
        double ua, ub;
        stream_uniform2(&s, &ua, &ub);
        int32_t i = (int32_t)(ua * (double)n);
        if (i > n - 1) i = n - 1;
        int32_t j = (int32_t)(ub * (double)(n - 1));
        if (j > n - 2) j = n - 2;
        if (j >= i) j = j + 1;
        double crx = vx[i] - vx[j];
        double cry = vy[i] - vy[j];
        double crz = vz[i] - vz[j];
        double cr = sqrt((crx * crx + cry * cry) + crz * crz);
        if (cr > S->crmax[c]) S->crmax[c] = cr;
        double ua2, ub2;
        stream_uniform2(&s, &ua2, &ub2);
        if (ua2 * S->crmax[c] < cr) {
            double d[3];
            stream_sphere(&s, d);
            double cmx = 0.5 * (vx[i] + vx[j]);
            double cmy = 0.5 * (vy[i] + vy[j]);
            double cmz = 0.5 * (vz[i] + vz[j]);
            double hh = 0.5 * cr;
            vx[i] = cmx + hh * d[0];
            vy[i] = cmy + hh * d[1];
            vz[i] = cmz + hh * d[2];
            vx[j] = cmx - hh * d[0];
            vy[j] = cmy - hh * d[1];
            vz[j] = cmz - hh * d[2];
            S->n_coll += 1;
        }
    }
}

static void phase_collide(or_state *S, int64_t step)
{
    for (int32_t c = 0; c < S->Cc; ++c) collide_cell(S, step, c);
}

/* -------------------------------------------------------------- sample */
/* Per collision cell, the step's twelve sums over its slots in slot order
 * after the collide phase, then added to the window's accumulators. */
static void phase_sample(or_state *S)
{
    for (int32_t c = 0; c < S->Cc; ++c) {
        double s[NMOM];
        for (int m = 0; m < NMOM; ++m) s[m] = 0.0;
        int32_t o = S->offset[c], n = S->count[c];
        for (int32_t q = o; q < o + n; ++q) {
            double x = S->vx[q], y = S->vy[q], z = S->vz[q];
            double v2 = (x * x + y * y) + z * z;
            s[0] += 1.0;
            s[1] += x;
            s[2] += y;
            s[3] += z;
            s[4] += x * x;
            s[5] += y * y;
            s[6] += z * z;
            s[7] += x * y;
            s[8] += x * z;
            s[9] += y * z;
            s[10] += v2 * x;
            s[11] += v2 * y;
        }
        double *a = S->acc + (size_t)c * NMOM;
        for (int m = 0; m < NMOM; ++m) a[m] += s[m];
    }
}

/* Per collision cell, the sum of vx vy over its slots in slot order before the
 * collide phase: the stress a sampling step sees before the collisions relax
 * it, for the time-centred stress estimate. */
static void phase_sample_pre(or_state *S)
{
    for (int32_t c = 0; c < S->Cc; ++c) {
        double s = 0.0;
        int32_t o = S->offset[c], n = S->count[c];
        for (int32_t q = o; q < o + n; ++q) s += S->vx[q] * S->vy[q];
        S->acc[(size_t)c * NMOM + 12] += s;
    }
}

/* ----------------------------------------------------------------- step */
void or_step(or_state *S, int64_t n_steps, uint32_t phase_mask)
{
    if (phase_mask == 0) phase_mask = PHASE_ALL;
    for (int64_t k = 0; k < n_steps; ++k) {
        int64_t step = S->step + 1;
        if (phase_mask & PHASE_MOVE) phase_move(S, step);
        if (phase_mask & PHASE_SORT) phase_sort(S);
        const int sampling = (phase_mask & PHASE_SAMPLE) && step > S->p.n_transient;
        if (sampling) phase_sample_pre(S);
        if (phase_mask & PHASE_COLLIDE) phase_collide(S, step);
        if (sampling) {
            phase_sample(S);
            S->n_sampled += 1;
        }
        S->step = step;
    }
}

void or_reset_window(or_state *S)
{
    memset(S->acc, 0, (size_t)S->Cc * NMOM * sizeof(double));
    S->n_sampled = 0;
    S->n_coll = 0;
}

/* ----------------------------------------------------------- estimators */
/* Per sampling cell (its n_sub collision cells summed in order), with K the
 * sampled steps in the window and N the particles:
 *   nu = S0 C / (K N)                     density over the nominal density
 *                                         (N = C ppc, the initial count)
 *   u_a = S1_a / S0, M_ab = S2_ab/S0 - u_a u_b, T = trace(M)/3
 *   P_xy = nu M_xy                        shear stress over n kT_ref
 *   P_xy,mid = nu ((S_xy + S_xy,pre)/2 / S0 - u_x u_y)
 *                                         the time-centred stress: the mean of
 *                                         the kinetic estimates before and
 *                                         after the collide phase
 *   <|c|^2 c_a> from the raw moments, q_a = nu <|c|^2 c_a> / 2
 *   Q = sum_c S1_x / (K N)                mass flow over n H
 * Velocities, heat flux and mass flow are returned over v0 = sqrt(2) and the
 * stress over P0, the normalisation of Eq. 6.  Outputs are NaN when K = 0 or
 * a cell saw no particle. */
void or_estimators(const or_state *S, double *nu, double *ux, double *uy, double *uz,
                   double *T, double *pxy, double *qx, double *qy, double *Q, double *pxy_mid)
{
    const double v0 = sqrt(2.0);
    const int32_t C = S->C, ns = S->p.n_sub;
    const double K = (double)S->n_sampled, N = (double)S->Nnom;
    double qsum = 0.0;
    for (int32_t c = 0; c < C; ++c) {
        double s[NMOM];
        for (int m = 0; m < NMOM; ++m) s[m] = 0.0;
        for (int32_t k = 0; k < ns; ++k) {
            const double *a = S->acc + ((size_t)c * ns + k) * NMOM;
            for (int m = 0; m < NMOM; ++m) s[m] += a[m];
        }
        qsum += s[1];
        double n_c = (s[0] * (double)C) / (K * N);
        double u = s[1] / s[0], v = s[2] / s[0], w = s[3] / s[0];
        double mxx = s[4] / s[0] - u * u;
        double myy = s[5] / s[0] - v * v;
        double mzz = s[6] / s[0] - w * w;
        double mxy = s[7] / s[0] - u * v;
        double trace2 = (s[4] + s[5]) + s[6];
        double usq = (u * u + v * v) + w * w;
        double cx = ((s[10] / s[0] - u * (trace2 / s[0])) -
                     2.0 * (((u * s[4] + v * s[7]) + w * s[8]) / s[0])) + 2.0 * u * usq;
        double cy = ((s[11] / s[0] - v * (trace2 / s[0])) -
                     2.0 * (((u * s[7] + v * s[5]) + w * s[9]) / s[0])) + 2.0 * v * usq;
        if (nu) nu[c] = n_c;
        if (ux) ux[c] = u / v0;
        if (uy) uy[c] = v / v0;
        if (uz) uz[c] = w / v0;
        if (T) T[c] = ((mxx + myy) + mzz) / 3.0;
        if (pxy) pxy[c] = n_c * mxy;
        if (pxy_mid) pxy_mid[c] = n_c * ((0.5 * (s[7] + s[12])) / s[0] - u * v);
        if (qx) qx[c] = (0.5 * n_c * cx) / v0;
        if (qy) qy[c] = (0.5 * n_c * cy) / v0;
    }
    if (Q) *Q = (qsum / (K * N)) / v0;
}

/* --------------------------------------------------------------- access */
int32_t or_n_particles(const or_state *S) { return S->N; }
int32_t or_capacity(const or_state *S) { return S->Ncap; }

/* open-boundary diagnostics: live particles, particles injected and removed
 * since creation, status bits, the injection remainder */
void or_open_diagnostics(const or_state *S, double out[5])
{
    out[0] = (double)S->N;
    out[1] = (double)S->n_injected;
    out[2] = (double)S->n_deleted;
    out[3] = (double)S->status;
    out[4] = S->inj_rem;
}
int32_t or_n_coll_cells(const or_state *S) { return S->Cc; }
int64_t or_step_index(const or_state *S) { return S->step; }
int64_t or_n_sampled(const or_state *S) { return S->n_sampled; }

void or_get_particles(const or_state *S, double *y, double *vx, double *vy, double *vz,
                      int32_t *cell)
{
    size_t n = (size_t)S->N;
    if (y) memcpy(y, S->y, n * sizeof(double));
    if (vx) memcpy(vx, S->vx, n * sizeof(double));
    if (vy) memcpy(vy, S->vy, n * sizeof(double));
    if (vz) memcpy(vz, S->vz, n * sizeof(double));
    if (cell) memcpy(cell, S->cell, n * sizeof(int32_t));
}

void or_set_particles(or_state *S, const double *y, const double *vx, const double *vy,
                      const double *vz, const int32_t *cell)
{
    size_t n = (size_t)S->N;
    if (y) memcpy(S->y, y, n * sizeof(double));
    if (vx) memcpy(S->vx, vx, n * sizeof(double));
    if (vy) memcpy(S->vy, vy, n * sizeof(double));
    if (vz) memcpy(S->vz, vz, n * sizeof(double));
    if (cell) memcpy(S->cell, cell, n * sizeof(int32_t));
}

void or_get_cells(const or_state *S, double *crmax, double *rem, int32_t *count,
                  int32_t *offset)
{
    size_t c = (size_t)S->Cc;
    if (crmax) memcpy(crmax, S->crmax, c * sizeof(double));
    if (rem) memcpy(rem, S->rem, c * sizeof(double));
    if (count) memcpy(count, S->count, c * sizeof(int32_t));
    if (offset) memcpy(offset, S->offset, c * sizeof(int32_t));
}

void or_get_acc(const or_state *S, double *acc)
{
    memcpy(acc, S->acc, (size_t)S->Cc * NMOM * sizeof(double));
}

/* constants: dt, g, kntc, crmax0, inv_dy, lambda */
void or_constants(const or_state *S, double out[6])
{
    out[0] = S->dt;
    out[1] = S->g;
    out[2] = S->kntc;
    out[3] = S->crmax0;
    out[4] = S->inv_dy;
    out[5] = S->lam;
}

/* diagnostics: accepted collisions in window, wall hits, wall x momentum,
 * wall energy (both since creation) */
void or_diagnostics(const or_state *S, double out[4])
{
    out[0] = (double)S->n_coll;
    out[1] = (double)S->n_hits;
    out[2] = S->wall_dpx;
    out[3] = S->wall_de;
}

/* One particle's move, for hand-built kinematics checks; it does not touch
 * the state's particles but does count wall diagnostics. */
void or_move_one(or_state *S, int64_t step, int64_t slot, double st[4])
{
    move_one(S, step, slot, &st[0], &st[1], &st[2], &st[3]);
}

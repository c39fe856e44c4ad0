/*
 * apr.h -- C ABI of libapr.so, an MI355X (gfx950) implementation of the
 * data-parallel hot path of adaptive particle refinement (APR) for
 * compressible SPH (Nealon & Price 2024): neighbour search, the
 * variable-smoothing-length density sum with its h-rho Newton iteration, the
 * pressure-gradient + artificial-viscosity + du/dt force sum over particles of
 * mixed mass, the split/merge pass at refinement-zone boundaries, leapfrog
 * integration, and the adjoint of the density and force sums.
 *
 * Conventions
 *  - Every call returns an int status (APR_OK = 0 or an APR_ERR_* code) and
 *    never throws.  apr_last_error() gives a message for the last failure.
 *  - Particle arrays are caller-owned DEVICE pointers (one GPU), structure of
 *    arrays, n valid entries out of `capacity` allocated ones (capacity at
 *    most 2^31 - 1: cell starts and particle slots are 32-bit; larger states
 *    are rejected with APR_ERR_INVALID).  The library
 *    owns only its workspace (sort buffers, cells, tree, per-particle
 *    derived values), which lives in the context and grows as needed.
 *  - Calls enqueue work on the context's HIP stream and return without
 *    waiting, except where a call says it synchronises.
 *  - Mass is never passed: a particle of level l has mass m0 / 2^l (paper
 *    Sec. 2.1, rules 4 and 5).
 *  - "void *" arrays are float * when params.precision == APR_FP32 and
 *    double * when it is APR_FP64.
 *  - Kernel (params.kernel): the M4 cubic spline (paper appendix A, kernel
 *    table, h_fact = 1.2 there) or the Wendland C2 kernel that the paper's
 *    example applications use (Sec. 3: kernel radius 2h, h_fact = 1.3).  Both
 *    have support 2h and are written W(r, h) = f(r/h)/(pi h^3):
 *      M4   f = 1 - 3/2 q^2 + 3/4 q^3 (q < 1),  1/4 (2 - q)^3 (1 <= q < 2)
 *      WC2  f = 21/16 (1 - q/2)^4 (1 + 2 q)      (q < 2)
 *    h_fact is params.hfact whichever the kernel; set 1.3 with Wendland C2.
 */
#ifndef APR_H
#define APR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    APR_OK = 0,
    APR_ERR_INVALID = 1,    /* bad argument, size or parameter */
    APR_ERR_CAPACITY = 2,   /* splits need more than state->capacity */
    APR_ERR_NOCONVERGE = 3, /* some h-rho Newton solves did not converge */
    APR_ERR_HIP = 4,        /* a HIP runtime call failed */
    APR_ERR_OVERFLOW = 5,   /* reserved (no internal list has a fixed capacity) */
    APR_ERR_RANGE = 6       /* a smoothing length reached a periodic box's limit */
};

enum { APR_FP64 = 0, APR_FP32 = 1 };
enum { APR_EOS_ISOTHERMAL = 0, APR_EOS_LOCALLY_ISOTHERMAL = 1, APR_EOS_ADIABATIC = 2 };
enum { APR_SPLIT_TANGENTIAL = 0, APR_SPLIT_RANDOM = 1 };
enum { APR_KERNEL_M4 = 0, APR_KERNEL_WC2 = 1 };

typedef struct apr_ctx apr_ctx;

/* Particle state, structure of arrays of device pointers.  ax..dudt hold the
 * total acceleration (hydro + sink gravity) and du/dt that the leapfrog needs
 * between steps; they may be NULL for calls that do not integrate. */
typedef struct {
    int64_t n;        /* particles in use */
    int64_t capacity; /* particles every array has room for */
    int64_t next_id;  /* id given to the next particle a split creates (host value);
                         must exceed every id in the state, so that ids stay unique */
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *u;        /* specific thermal energy (adiabatic EOS) */
    double *h;        /* smoothing length */
    double *ax, *ay, *az, *dudt;
    int8_t *level;    /* refinement level l, mass m0 / 2^l */
    int64_t *id;      /* persistent particle id */
} apr_state;

/* A refinement zone (paper Sec. 2.1, rule 1): nested spheres about one
 * centre, radii r[0] > r[1] > ... (outer to inner) with levels ell[k].  The
 * level at a point is that of the innermost sphere with |x - c|^2 < r^2
 * (strict), or the background level outside them.  Several zones combine by
 * max (refinement) or by min (params.derefine != 0; paper Sec. 2.1, rule 3).
 * shape = APR_ZONE_CYLINDER makes them cylinders along z through c: the
 * distance leaves out z, and the tangential split axis uses the offset from
 * the axis (the circular region of the paper's sound-wave test in a thin box,
 * appendix A). */
enum { APR_ZONE_SPHERE = 0, APR_ZONE_CYLINDER = 1 };
typedef struct {
    double c[3];
    int32_t n;       /* number of spheres, 1..8 */
    int32_t ell[8];
    int32_t shape;   /* APR_ZONE_SPHERE or APR_ZONE_CYLINDER */
    double r[8];
} apr_zone;

/* A point mass (sink) acting on the gas with gravity G m / (r^2 + eps^2). */
typedef struct {
    double x[3];
    double m;
    double eps;
} apr_sink;

typedef struct {
    int32_t precision;  /* APR_FP64 or APR_FP32 (pair arithmetic and derived outputs) */
    int32_t eos;        /* APR_EOS_* */
    double hfact;       /* h = hfact (m / rho)^(1/3); 1.2 for M4, 1.3 for Wendland C2 */
    double tol_h;       /* Newton stops when |dh| < tol_h h */
    int32_t max_iter;   /* Newton iterations per particle, 1 .. 1000 */
    int32_t kernel;     /* APR_KERNEL_M4 or APR_KERNEL_WC2 (support 2h either way) */
    double cs0;         /* sound speed (isothermal) or its value at R = r_ref */
    double q_cs;        /* locally isothermal: cs = cs0 (R / r_ref)^-q_cs, R cylindrical */
    double r_ref;
    double gamma;       /* adiabatic index */
    double av_alpha;    /* artificial viscosity: vsig = alpha c + beta |v_ab . rhat| */
    double av_beta;
    int32_t periodic;   /* 1: periodic box [box_lo, box_hi) */
    double box_lo[3];   /* domain box; also the frame of the Morton keys and of the */
    double box_hi[3];   /* merge tree's quantised coordinates (particles are clamped) */
    double m0;          /* mass of a level-0 particle */
    double r_sep_factor;/* split offset r_sep = r_sep_factor h (0.2 in the paper) */
    double nn_cap;      /* cap r_sep at nn_cap * nearest-neighbour distance; <= 0: off */
    int32_t split_mode; /* APR_SPLIT_TANGENTIAL (paper) or APR_SPLIT_RANDOM */
    int32_t ell_background;
    int32_t derefine;   /* zones combine by min instead of max */
    uint64_t seed;      /* split-axis random stream */
    double G;           /* gravitational constant for sinks */
} apr_params;

/* Fills *p with defaults: FP32, M4 kernel, adiabatic, hfact 1.2, tol 1e-6, 50 iterations,
 * alpha 1, beta 2, gamma 5/3, r_sep 0.2, nn_cap 0.35, tangential, G = 1. */
void apr_default_params(apr_params *p);

/* Creates a context on the current HIP device.  stream is a hipStream_t (NULL:
 * the null stream).  Returns APR_ERR_INVALID for bad parameters. */
int apr_ctx_create(apr_ctx **ctx, const apr_params *p, void *stream);
int apr_ctx_destroy(apr_ctx *ctx);
int apr_ctx_set_stream(apr_ctx *ctx, void *stream);

/* Launch grid (workgroups, one target cell each) of the per-cell kernels from
 * the next apr_build_cells on; 0 restores the default, the last cell count
 * read back plus 1/8 and 64.  An implementation setting with no counterpart
 * in the paper: results do not depend on it (cells beyond the grid are taken
 * by a second, normally empty launch), so it serves tuning and tests.
 * Returns APR_ERR_INVALID for grid < 0. */
int apr_set_cell_grid(apr_ctx *ctx, int64_t grid);
const char *apr_last_error(const apr_ctx *ctx);

/* Sorts the particles into Morton order IN PLACE (all non-NULL state arrays
 * are permuted) and builds the cell lists and the cell tree the other calls
 * search.  perm (device, optional) receives, for every new slot, the slot the
 * particle came from.  Replaces the k-d tree neighbour search of the paper's
 * host code (Sec. 2.3) with Morton-ordered leaf cells of at most 64
 * particles.  Periodic boxes need 2 max(h) < box / 4 (the minimum image of a cell
 * pair then holds for all its particle pairs); apr_density flags a converged
 * h beyond that (APR_ERR_RANGE from apr_sync_status). */
int apr_build_cells(apr_ctx *ctx, apr_state *s, int64_t *perm);

/* Density and smoothing length (paper Sec. 2.2, which defers to Phantom's
 * iterative h-rho solve): for every particle a, solves
 *   rho_a = sum_b m_b W(|x_a - x_b|, h_a)  (b = a included),
 *   h_a = hfact (m_a / rho_a)^(1/3)
 * by Newton steps with Halley's second-derivative correction from the
 * current h (until |dh| < tol_h h, or a Halley step below sqrt(tol_h) h,
 * whose h + dh is written with rho and Omega carried to it by their Taylor
 * series); writes the converged h into s->h and
 *   Omega_a = 1 + h_a / (3 rho_a) sum_b m_b dW_ab/dh_a.
 * rho, omega: [n] (float or double); nneigh (optional) counts b with
 * r_ab < 2 h_a at the h written, self included; iters (optional) Newton
 * passes per particle.  Membership is that of the FP64 predicate of
 * apr_neighbours (mode 0) in both precisions: the pair-precision test is
 * decided again in FP64 on absolute positions inside a guard band about the
 * support's edge.
 * Needs apr_build_cells on the same positions.  Asynchronous: failures to
 * converge are counted on the device; apr_sync_status reports them. */
int apr_density(apr_ctx *ctx, apr_state *s, void *rho, void *omega, int32_t *nneigh,
                int32_t *iters);

/* Hydrodynamic acceleration and du/dt.  The paper runs Phantom's
 * compressible SPH and states no force formula (Sec. 2.2 defers the SPH
 * machinery to it; Sec. 3.1 and 3.2 give the locally isothermal EOS of the
 * disc applications, appendix A the adiabatic one of its tests); the form
 * here is the standard grad-h one, consistent with the density of
 * apr_density, with a per-particle artificial viscosity:
 *   a_a = -sum_b m_b [(P_a + q^a)/(Omega_a rho_a^2) F_ab(h_a)
 *                   + (P_b + q^b)/(Omega_b rho_b^2) F_ab(h_b)] rhat_ab,
 *   du_a/dt = sum_b m_b (P_a + q^a)/(Omega_a rho_a^2) (v_ab . rhat) F_ab(h_a),
 * F_ab(h) = W'(r)/... for r < 2h, q^a = -rho_a vsig_a (v_ab . rhat)/2 for
 * approaching pairs; pairs with r < 2 max(h_a, h_b).  P and c come from the
 * EOS.  vsig (optional) = max over pairs of alpha c_a + beta max(0, -v_ab.rhat).
 * npair (optional, int32 [n]) counts each target's pairs: b != a with
 * r_ab < 2 max(h_a, h_b).  Membership is that of the FP64 predicate of
 * apr_neighbours (mode 1) in both precisions: the pair-precision test is
 * decided again in FP64 on absolute positions inside a guard band about
 * either support's edge.  rho, omega from apr_density on the same state.
 * Outputs [n]. */
int apr_forces(apr_ctx *ctx, const apr_state *s, const void *rho, const void *omega, void *ax,
               void *ay, void *az, void *dudt, void *vsig, int32_t *npair);

/* Vector-Jacobian product of the density and force sums (the adjoint; the
 * paper has none, it serves to tune split offsets against the density error
 * of Sec. 2.2 and 3.3).  One entry point covers both products: with the
 * force cotangents ax_bar .. dudt_bar all NULL it is the density VJP alone
 * (an apr_density_vjp), and with them it is the VJP of density and forces
 * together (an apr_forces_vjp that also chains through rho, h and Omega).
 * Forward: rho, Omega at the h that solves
 * rho_sum(h) = m (hfact/h)^3 (apr_density, whose h s->h holds), then
 * apr_forces' a and du/dt.  Given cotangents rho_bar [n], h_bar [n],
 * ax_bar, ay_bar, az_bar, dudt_bar [n] (each may be NULL: zero), writes
 *   xbar, ybar, zbar [n] = dL/dx, dL/dy, dL/dz,   mbar [n] = dL/dm_a,
 * L = sum_a rho_bar rho + h_bar h + abar . a + dudt_bar du/dt, with h
 * implicit in (x, m) (implicit-function theorem on the h-rho relation: the
 * density tangent is (d rho_sum at fixed h)/Omega) and m_a = m0 2^-level_a
 * taken as a free per-particle variable.  Velocities, u and sink terms are
 * held fixed.  Neighbours are searched again, not stored.  rho, omega,
 * cotangents and outputs are of the context precision; the cells must be
 * those of the forward (apr_build_cells, then apr_density).  Asynchronous. */
int apr_vjp(apr_ctx *ctx, const apr_state *s, const void *rho, const void *omega,
            const void *rho_bar, const void *h_bar, const void *ax_bar, const void *ay_bar,
            const void *az_bar, const void *dudt_bar, void *xbar, void *ybar, void *zbar,
            void *mbar);

/* Individual timesteps (paper Sec. 2.5).  bin [capacity] (device, int8,
 * caller-owned) holds each particle's timestep bin k: its step is dt_max 2^-k.
 * apr_bins_init takes density, forces and sink gravity for every particle
 * (like apr_accel), keeps each particle's rho, Omega, vsig and nearest
 * distance in the context, and sets every bin from the Courant limit: the
 * smallest k in 0..max_bin with dt_max 2^-k <= c_cfl h / vsig.
 * apr_step_bins advances the state by dt_max in 2^K substeps of dt_max 2^-K
 * (K the largest bin).  In substep s a particle whose step starts (s a
 * multiple of 2^(K-k)) takes its opening half kick with its own dt; all
 * particles drift; those whose step ends ((s+1) a multiple of 2^(K-k)) are
 * active: the split/merge pass examines only them (random key step*4096 + s),
 * density, forces and sink gravity are taken for them and for what the pass
 * made (the others keep h, rho, Omega and a from their last turn, which their
 * neighbours use), and they take their closing half kick; an active
 * particle's bin then follows the Courant limit, clamped to K within the step
 * and to max_bin at its end, and lengthens only where the longer step starts
 * at this boundary; particles a split made or a merge kept take bin K.  The
 * state and bin are reordered together (cell order); *n_substeps gets 2^K.
 * The state needs ax, ay, az, dudt and u, and room for the splits of all
 * substeps (APR_ERR_CAPACITY leaves the step half done).  Any other call that
 * reorders the state (apr_build_cells, apr_step, apr_split_merge, apr_relax)
 * voids the stored values: apr_step_bins then returns APR_ERR_INVALID until
 * apr_bins_init runs again.  Synchronises once per substep with zones.
 * Errors (APR_ERR_INVALID, nothing changed): an empty state, a missing bin
 * array, dt_max or c_cfl not > 0, max_bin outside 0..20, a negative bin or
 * one above max_bin in bin. */
int apr_bins_init(apr_ctx *ctx, apr_state *s, int8_t *bin, const apr_sink *sinks,
                  int32_t nsinks, double dt_max, double c_cfl, int32_t max_bin);
int apr_step_bins(apr_ctx *ctx, apr_state *s, int8_t *bin, const apr_zone *zones,
                  int32_t nzones, const apr_sink *sinks, int32_t nsinks, double dt_max,
                  double c_cfl, int32_t max_bin, int64_t step, int32_t *n_substeps);

/* Relaxing (paper Sec. 2.4) of the particles a split/merge pass introduced:
 * those of s whose id is not below ref->next_id, or whose level differs from
 * the level ref gives the same id.  Each shuffle computes the hydro
 * accelerations a_new of s (cells, apr_density, apr_forces on ctx), the
 * reference accelerations interpolated at the same points by the reference
 * set's own SPH interpolant
 *   a_ref(x) = sum_b (m_b / rho_b) a_b W(|x - x_b|, h_b)   (r < 2 h_b),
 * and moves each introduced particle by dx = 0.5 dt^2 (a_new - a_ref), dt =
 * 0.3 h / c_s of the particle, with |dx| capped at h (periodic wrap).
 * KE = sum |dx| / dt^2 over the moved particles; the shuffles stop once KE <=
 * ke_frac * KE of the first shuffle (the paper: 0.005) or after max_shuffles
 * (the paper: 50, at most 1000).  The interpolation and the shift are FP64.
 *   ref_ctx   a context with the same precision, kernel, box and m0 whose
 *             cells were built on ref (apr_build_cells), then apr_density
 *             and apr_forces on ref: ref_rho, ref_ax, ref_ay, ref_az [ref->n]
 *             are their outputs (context precision) in ref's order;
 *   ref       the reference set (the state before the pass; ids below
 *             ref->next_id, at most 2^31 - 1);
 *   s         the new set; its positions and h change, its cells are rebuilt
 *             (it is reordered like apr_build_cells) and are stale on return.
 * *n_shuffles, *ke_first, *ke_last (each may be NULL) receive the number of
 * shuffles and the first and last KE.  Synchronises once per shuffle.
 * Returns APR_ERR_INVALID for mismatched contexts, ref cells not built on
 * ref, or bad limits. */
int apr_relax(apr_ctx *ctx, apr_state *s, apr_ctx *ref_ctx, const apr_state *ref,
              const void *ref_rho, const void *ref_ax, const void *ref_ay, const void *ref_az,
              int32_t max_shuffles, double ke_frac, int32_t *n_shuffles, double *ke_first,
              double *ke_last);

/* Neighbour lists for a given h (device, [n]), with the FP64 predicate
 * r_ab^2 < (2 h_a)^2 (mode 0) or r_ab^2 < (2 max(h_a, h_b))^2 (mode 1), b != a,
 * evaluated on absolute positions with the minimum-image convention and no
 * fused multiply-add.  Call once with list == NULL: counts [n] and offsets
 * [n + 1] (prefix) are written and the total returned in *total (this
 * synchronises).  Call again with list of room `cap` to get the neighbour
 * slots of particle a in list[offsets[a] .. offsets[a+1]).  Test export. */
int apr_neighbours(apr_ctx *ctx, const apr_state *s, const double *h, int32_t mode,
                   int64_t *counts, int64_t *offsets, int64_t *list, int64_t cap,
                   int64_t *total);

/* One split/merge pass (paper Sec. 2.2, 2.3 and 2.5): split from the lowest
 * level up, then merge from the highest level down; a particle changes level
 * at most once per pass.
 * Split: a particle whose level is below its zone level becomes two
 * children of level + 1, h (1/2)^(1/3), same v and u, at x +- r_sep w with w
 * tangential to the zone (rotated about x - c by a random angle) or random;
 * r_sep = r_sep_factor h, capped at nn_cap * (nearest-neighbour distance from
 * the last apr_density) when nn_cap > 0.  The parent slot keeps the + child;
 * the - children are appended in ascending parent slot and numbered next_id,
 * next_id + 1, ... in ascending parent id (so the ids, and every later pass,
 * do not depend on the order of the arrays).
 * Random stream: s = F(seed ^ F(id ^ F(step))), F(v) the first SplitMix64
 * output from state v; rotation angle 2 pi U1 (tangential) or axis from
 * (U1, U2) (random), Uk = (k-th SplitMix64 output from s >> 11) 2^-53.
 * Merge, for l = max level .. 1: the level-l particles not changed in this
 * pass, in ascending id, the highest id left out if their number is odd, are
 * paired by a k-d tree on 2^21-step quantised coordinates over the box (cut
 * on the widest axis at the floor of the mean, an even count forced on each
 * side, leaves of two); a leaf whose centre of mass lies in a zone of level
 * < l merges: the lower id stays at the centre of mass with the mean velocity
 * and mean u, level l - 1, h 2^(1/3); the other is removed.  In a periodic
 * box the centre of mass takes the other particle at its minimum image about
 * the kept one and is wrapped back into the box (a pair across the boundary
 * merges beside it).  Survivors keep their order.
 * Synchronises.  Updates s->n and s->next_id.  flags: bit 0 split, bit 1
 * merge (0 means both).  If the splits need more than s->capacity the state is
 * left unchanged, *n_split receives the capacity needed and APR_ERR_CAPACITY
 * is returned.  After a pass the cells must be rebuilt. */
int apr_split_merge(apr_ctx *ctx, apr_state *s, const apr_zone *zones, int32_t nzones,
                    int64_t step, int32_t flags, int64_t *n_split, int64_t *n_merged,
                    int64_t *n_spare);

/* Kick-drift-kick leapfrog step of size dt on the state (the paper's host
 * code integrates; the scheme here is the standard KDK):
 *   v += dt/2 a, u += dt/2 du/dt;  x += dt v (wrapped if periodic), and the
 *   Newton guess h *= exp(dt D / 3), D the velocity divergence of the last
 *   force pass, extrapolated with the one before it when both are at hand
 *   (D + dt/(2 dt_last) (D - D_prev)), the factor clamped to [0.8, 1.25];
 *   split/merge if nzones > 0 (Sec. 2.6: refinement opens the step; the
 *   nearest-neighbour cap uses the last density pass);
 *   rebuild cells, density;  hydro forces + sink gravity -> a, du/dt;
 *   v += dt/2 a, u += dt/2 du/dt.
 * s->ax..dudt must hold the acceleration of the current positions on entry
 * (apr_accel computes it).  sinks are at their positions for the end of the
 * step.  Synchronises only if nzones > 0 or on error checks. */
int apr_step(apr_ctx *ctx, apr_state *s, const apr_zone *zones, int32_t nzones,
             const apr_sink *sinks, int32_t nsinks, double dt, int64_t step);

/* Rebuilds cells, solves density and writes the total acceleration (hydro +
 * sinks) and du/dt into s->ax..dudt.  Asynchronous. */
int apr_accel(apr_ctx *ctx, apr_state *s, const apr_sink *sinks, int32_t nsinks);

/* Courant timestep C min_a h_a / vsig_a from the last apr_accel/apr_step
 * (0.3 by analogy with the paper's relaxation step, Sec. 2.4).  Synchronises. */
int apr_timestep(apr_ctx *ctx, const apr_state *s, double C, double *dt);

/* For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  apr_timestep without any
 * allocation and without host synchronisation: enqueues on the context's
 * stream the reduction C min_a h_a / vsig_a over the state's last
 * apr_accel / apr_step and writes it to dt_dev (one double in device memory,
 * caller-owned).  The reduction's partial minima live in a fixed library
 * array of 1024 doubles per GPU (8 KB, held until the process ends), set up
 * by apr_ctx_create on that GPU; every n fits it (the reduction strides), so
 * no size is refused for it.  All calls on one GPU share that array and keep
 * the last call's contents: calls that overlap on one GPU (several streams
 * or host threads) race and must be ordered by the caller.  Errors
 * (APR_ERR_INVALID, nothing enqueued): an empty state, a NULL dt_dev, no
 * force evaluation of this state in the context. */
int apr_timestep_noalloc(apr_ctx *ctx, const apr_state *s, double C, double *dt_dev);

/* Waits for the stream and returns APR_ERR_NOCONVERGE / APR_ERR_RANGE if
 * a kernel since the last call flagged one; *count receives the number of
 * particles that failed to converge (may be NULL).  Clears the flags. */
int apr_sync_status(apr_ctx *ctx, int64_t *count);

/* Kernel timing (diagnostics).  While enabled, HIP events on the context's
 * stream bracket every launch of the timed kernels: index APR_PROF_DENSITY
 * (h-rho Newton kernel), APR_PROF_FORCES (force kernel), APR_PROF_CELLS
 * (whole cell build), APR_PROF_SPLITMERGE (whole split/merge pass),
 * APR_PROF_VJP (the three kernels of apr_vjp), APR_PROF_CAND (the candidate-cell
 * walks ahead of the density, force and adjoint kernels).
 * apr_profile_read synchronises, writes the summed milliseconds and launch
 * counts per index (arrays of APR_PROF_N) and, if reset, clears them. */
enum { APR_PROF_DENSITY = 0, APR_PROF_FORCES = 1, APR_PROF_CELLS = 2, APR_PROF_SPLITMERGE = 3,
       APR_PROF_VJP = 4, APR_PROF_CAND = 5, APR_PROF_N = 6 };
int apr_profile_enable(apr_ctx *ctx, int on);
/* Restricts the timing to the indices whose bit (1 << index) is set in mask
 * (every index by default; 0 records no event even while enabled).  Each
 * timed launch adds two event records to the stream, and each record waits
 * for the work before it, so a caller that times a whole step brackets only
 * the kernel it needs.  Takes effect at the next launch; no GPU work. */
int apr_profile_select(apr_ctx *ctx, uint32_t mask);
/* Work counters since the last reset (diagnostics), written to
 * c[0 .. APR_COUNTERS_N-1]:
 * [0] h-rho solves that hit max_iter, [1] smoothing lengths at the periodic limit,
 * [2] density cells whose candidates did not fit in one LDS window (staged
 * window by window instead), [3] the same for forces, [4] sub-block lists
 * that did not fit, [5] density searches repeated with a larger radius,
 * [6] density Newton passes summed over cells, [7] windows staged by the
 * density kernel summed over cells and passes, [8] density targets so far
 * from their cell's centre (|x - c|_1 >= 252 h) that the staging slack no
 * longer covers the guard band of the support test (none expected; exact
 * membership is then not assured), [9] pair tests decided in FP64 inside
 * the guard band (density and forces).  Synchronises. */
enum { APR_COUNTERS_N = 10 };
int apr_counters(apr_ctx *ctx, int64_t *c, int reset);
int apr_profile_read(apr_ctx *ctx, double *ms, int64_t *launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* APR_H */

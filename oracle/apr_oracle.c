/*
 * apr_oracle.c -- plain FP64 CPU oracle for the adaptive-particle-refinement
 * (APR) compressible SPH hot path of Nealon & Price, "Adaptive particle
 * refinement for compressible smoothed particle hydrodynamics" (2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * It is slow on purpose: every neighbour search is brute force over all
 * particles, every particle is handled on its own, and every step follows the
 * order in which the paper (or, where the paper defers to Phantom, the
 * standard grad-h SPH definition) states it.  All arithmetic is IEEE FP64.
 * Build with -ffp-contract=off so that every product and sum is rounded on its
 * own; the exact predicates below (neighbour membership, zone membership,
 * quantised coordinates, merge centres of mass) rely on that.
 *
 * Readings of points the paper leaves open are stated next to the code that
 * takes them.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* threads the OpenMP loops below use */
int32_t orc_num_threads(void) { return (int32_t)omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* M4 cubic spline (Monaghan & Lattanzio 1985), 3D, compact support 2h.      */
/* The paper compares it with the Wendland kernels in its appendix on kernel */
/* choice and pairs it with h_fact = 1.2 in the kernel table there.          */
/*   W(r,h) = f(q)/(pi h^3),  q = r/h                                        */
/*   f(q)   = 1 - 3/2 q^2 + 3/4 q^3      0 <= q < 1                          */
/*          = 1/4 (2 - q)^3              1 <= q < 2                          */
/*          = 0                          q >= 2                              */
/* ------------------------------------------------------------------------ */
double orc_m4_f(double q)
{
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) { double t = 2.0 - q; return 0.25 * t * t * t; }
    return 0.0;
}

/* df/dq */
double orc_m4_df(double q)
{
    if (q < 1.0) return -3.0 * q + 2.25 * q * q;
    if (q < 2.0) { double t = 2.0 - q; return -0.75 * t * t; }
    return 0.0;
}

/* d2f/dq2 (used only by the pins) */
double orc_m4_d2f(double q)
{
    if (q < 1.0) return -3.0 + 4.5 * q;
    if (q < 2.0) return 1.5 * (2.0 - q);
    return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Wendland C2 (Wendland 1995), 3D, compact support 2h: the kernel of the    */
/* paper's example applications (Sec. 3, with h_fact = 1.3 and kernel       */
/* radius 2h).  Written in the same form W = f(q)/(pi h^3):                 */
/*   f(q) = 21/16 (1 - q/2)^4 (1 + 2 q)   0 <= q < 2,   0 for q >= 2         */
/* The factor 21/16 normalises it: 4 int_0^2 q^2 (1 - q/2)^4 (1 + 2 q) dq    */
/* = 16/21 (two Beta integrals after q = 2 s).                              */
/* ------------------------------------------------------------------------ */
double orc_wc2_f(double q)
{
    if (q >= 2.0) return 0.0;
    double u = 1.0 - 0.5 * q;
    return (21.0 / 16.0) * u * u * u * u * (1.0 + 2.0 * q);
}

/* df/dq = -105/16 q (1 - q/2)^3 */
double orc_wc2_df(double q)
{
    if (q >= 2.0) return 0.0;
    double u = 1.0 - 0.5 * q;
    return -(105.0 / 16.0) * q * u * u * u;
}

/* d2f/dq2 = -105/16 (1 - q/2)^2 (1 - 2 q) */
double orc_wc2_d2f(double q)
{
    if (q >= 2.0) return 0.0;
    double u = 1.0 - 0.5 * q;
    return -(105.0 / 16.0) * u * u * (1.0 - 2.0 * q);
}

/* Kernel choice: 0 = M4 cubic spline, 1 = Wendland C2 (both support 2h). */
double orc_kf(int32_t kernel, double q) { return kernel == 1 ? orc_wc2_f(q) : orc_m4_f(q); }
double orc_kdf(int32_t kernel, double q) { return kernel == 1 ? orc_wc2_df(q) : orc_m4_df(q); }
double orc_kd2f(int32_t kernel, double q)
{
    return kernel == 1 ? orc_wc2_d2f(q) : orc_m4_d2f(q);
}

/* W(r, h) */
double orc_wk(int32_t kernel, double r, double h)
{
    return orc_kf(kernel, r / h) / (ORC_PI * h * h * h);
}

/* dW/dh at fixed r:  -(3 f + q f') / (pi h^4) */
double orc_dwdhk(int32_t kernel, double r, double h)
{
    double q = r / h;
    return -(3.0 * orc_kf(kernel, q) + q * orc_kdf(kernel, q)) / (ORC_PI * h * h * h * h);
}

/* the M4 forms of the two above */
double orc_w(double r, double h) { return orc_wk(0, r, h); }
double orc_dwdh(double r, double h) { return orc_dwdhk(0, r, h); }

/* Particle mass from the refinement level: m(l) = m(0) / 2^l
 * (paper, Sec. 2.1, rules 4 and 5 and the equation under them). */
static double pmass(double m0, int level) { return ldexp(m0, -level); }

/* One component of x_a - x_b, with the minimum-image convention in a
 * periodic box of side L. */
static double sep(double xa, double xb, int periodic, double L)
{
    double d = xa - xb;
    if (periodic) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

/* ------------------------------------------------------------------------ */
/* Density and the h-rho relation.                                          */
/*                                                                          */
/* The paper says Phantom solves density and smoothing length iteratively   */
/* (Sec. 2.1, citing the Phantom paper's Sec. 2.1.4).  Written out:         */
/*   rho_a   = sum_b m_b W(|x_a - x_b|, h_a)        (b = a included)        */
/*   h_a     = h_fact (m_a / rho_a)^(1/3)                                    */
/* Both hold at once: solve F(h) = rho_sum(h) - m_a (h_fact/h)^3 = 0 by      */
/* Newton with F'(h) = sum_b m_b dW/dh + 3 m_a h_fact^3 / h^4.              */
/*   Omega_a = 1 + h_a / (3 rho_a) sum_b m_b dW_ab/dh_a                      */
/* Readings:                                                                */
/*  - neighbours of a are the b with r_ab^2 < (2 h_a)^2, strict;            */
/*  - Newton stops when |h_new - h| < tol h; the h reported is the one the  */
/*    last sums were taken at, so rho, Omega and h are consistent;          */
/*  - if F' <= 0 the step is the fixed-point one h_fact (m/rho_sum)^(1/3);  */
/*    every step is clamped to [h/2, 2h];                                   */
/*  - dnn is the distance to the nearest other particle inside 2h (or      */
/*    +inf), used to cap the split offset.                                 */
/* Returns the number of targets that did not converge in max_iter steps.  */
/* ------------------------------------------------------------------------ */
int64_t orc_density(int64_t n, const double *x, const double *y, const double *z,
                    const int8_t *level, double m0, double hfact, double tol,
                    int32_t max_iter, int32_t periodic, const double *lo, const double *hi,
                    int64_t nt, const int64_t *targets, const double *h_in,
                    double *h_out, double *rho, double *omega, int32_t *nneigh,
                    double *dnn, int32_t *iters, int32_t kernel)
{
    double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    int64_t failures = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : failures)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = targets ? targets[t] : t;
        double ma = pmass(m0, level[a]);
        double h = h_in[t];
        double hs = h; /* the h the last sums were taken at */
        int converged = 0;
        int it;
        double rs = 0.0, drs = 0.0, dmin = INFINITY;
        int32_t nn = 0;
        for (it = 0; it < max_iter; ++it) {
            hs = h;
            double R2 = (2.0 * h) * (2.0 * h);
            rs = 0.0; drs = 0.0; nn = 0; dmin = INFINITY;
            for (int64_t b = 0; b < n; ++b) {
                double dx = sep(x[a], x[b], periodic, L[0]);
                double dy = sep(y[a], y[b], periodic, L[1]);
                double dz = sep(z[a], z[b], periodic, L[2]);
                double r2 = dx * dx + dy * dy + dz * dz;
                if (!(r2 < R2)) continue;
                double r = sqrt(r2);
                double mb = pmass(m0, level[b]);
                rs += mb * orc_wk(kernel, r, h);
                drs += mb * orc_dwdhk(kernel, r, h);
                nn += 1;
                if (b != a && r < dmin) dmin = r;
            }
            double rhoh = ma * (hfact / h) * (hfact / h) * (hfact / h);
            double F = rs - rhoh;
            double dF = drs + 3.0 * rhoh / h;
            double hn;
            if (dF > 0.0) hn = h - F / dF;
            else hn = hfact * cbrt(ma / rs);
            if (hn < 0.5 * h) hn = 0.5 * h;
            if (hn > 2.0 * h) hn = 2.0 * h;
            if (fabs(hn - h) < tol * h) { converged = 1; break; }
            h = hn;
        }
        if (!converged) failures += 1;
        h_out[t] = hs;
        rho[t] = rs;
        omega[t] = 1.0 + hs * drs / (3.0 * rs);
        if (nneigh) nneigh[t] = nn;
        if (dnn) dnn[t] = dmin;
        if (iters) iters[t] = converged ? it + 1 : max_iter;
    }
    return failures;
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists for a given h (brute force).                              */
/*  mode 0 ("gather"):    b != a with r_ab^2 < (2 h_a)^2                     */
/*  mode 1 ("symmetric"): b != a with r_ab^2 < (2 h_a)^2 or < (2 h_b)^2      */
/* Lists are in ascending b order.  With list == NULL only counts are        */
/* written; otherwise offsets[t] (prefix of counts) says where t's list      */
/* starts.                                                                   */
/* ------------------------------------------------------------------------ */
void orc_neighbours(int64_t n, const double *x, const double *y, const double *z,
                    const double *h, int32_t mode, int32_t periodic, const double *lo,
                    const double *hi, int64_t nt, const int64_t *targets, int64_t *counts,
                    const int64_t *offsets, int64_t *list)
{
    double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = targets ? targets[t] : t;
        double Ra2 = (2.0 * h[a]) * (2.0 * h[a]);
        int64_t c = 0;
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double dx = sep(x[a], x[b], periodic, L[0]);
            double dy = sep(y[a], y[b], periodic, L[1]);
            double dz = sep(z[a], z[b], periodic, L[2]);
            double r2 = dx * dx + dy * dy + dz * dz;
            int in = r2 < Ra2;
            if (mode == 1 && !in) {
                double Rb2 = (2.0 * h[b]) * (2.0 * h[b]);
                in = r2 < Rb2;
            }
            if (!in) continue;
            if (list) list[offsets[t] + c] = b;
            c += 1;
        }
        counts[t] = c;
    }
}

/* ------------------------------------------------------------------------ */
/* Equation of state.  The paper's discs are vertically (locally)           */
/* isothermal and its box tests adiabatic (Sec. 3 introduction, appendix A; */
/* c_s proportional to R^-q in the planet-disc set-up, Sec. 3.2).           */
/*  eos 0  isothermal          P = cs0^2 rho,             c = cs0           */
/*  eos 1  locally isothermal  c = cs0 (R / r_ref)^-q,    P = c^2 rho       */
/*         R the cylindrical radius about the z axis                         */
/*  eos 2  adiabatic           P = (gamma - 1) rho u,     c = sqrt(gamma P/rho)
 * ------------------------------------------------------------------------ */
void orc_eos_one(int32_t eos, double cs0, double q_cs, double r_ref, double gamma,
                 double x, double y, double rho, double u, double *P, double *c)
{
    if (eos == 0) {
        *c = cs0;
        *P = cs0 * cs0 * rho;
    } else if (eos == 1) {
        double R = sqrt(x * x + y * y);
        double cs = cs0 * pow(R / r_ref, -q_cs);
        *c = cs;
        *P = cs * cs * rho;
    } else {
        double p = (gamma - 1.0) * rho * u;
        *P = p;
        *c = sqrt(gamma * p / rho);
    }
}

void orc_eos(int64_t n, int32_t eos, double cs0, double q_cs, double r_ref, double gamma,
             const double *x, const double *y, const double *rho, const double *u,
             double *P, double *c)
{
    for (int64_t i = 0; i < n; ++i)
        orc_eos_one(eos, cs0, q_cs, r_ref, gamma, x[i], y[i], rho[i], u ? u[i] : 0.0,
                    &P[i], &c[i]);
}

/* ------------------------------------------------------------------------ */
/* Hydrodynamic force, artificial viscosity and du/dt.                       */
/* The paper is silent on these (it runs Phantom's compressible SPH); the    */
/* reading is the grad-h form with a per-particle artificial viscosity:     */
/*   a_a = - sum_b m_b [ (P_a + q^a_ab)/(Omega_a rho_a^2) F_ab(h_a)          */
/*                     + (P_b + q^b_ab)/(Omega_b rho_b^2) F_ab(h_b) ] rhat   */
/*   F_ab(h) = f'(r/h)/(pi h^4) for r < 2h, else 0;  rhat = (x_a - x_b)/r    */
/*   q^a_ab = -1/2 rho_a vsig_a (v_ab . rhat)  if v_ab . rhat < 0, else 0     */
/*   vsig_a = alpha c_a + beta |v_ab . rhat|                                 */
/*   du_a/dt = sum_b m_b (P_a + q^a_ab)/(Omega_a rho_a^2) (v_ab . rhat) F_ab(h_a)
 * Pairs: b != a with r < 2 max(h_a, h_b); a pair at r = 0 adds nothing.     */
/* Also returned per target: vsig = max over pairs of                        */
/* alpha c_a + beta max(0, -v_ab . rhat) (at least alpha c_a), and the L1    */
/* sums anorm = sum_b |pair acceleration|, unorm = sum_b |pair du/dt| that   */
/* bound the rounding error of the sums.                                     */
/* ------------------------------------------------------------------------ */
void orc_forces(int64_t n, const double *x, const double *y, const double *z,
                const double *vx, const double *vy, const double *vz, const double *u,
                const int8_t *level, const double *h, const double *rho, const double *omega,
                double m0, int32_t eos, double cs0, double q_cs, double r_ref, double gamma,
                double alpha, double beta, int32_t periodic, const double *lo,
                const double *hi, int64_t nt, const int64_t *targets, double *ax, double *ay,
                double *az, double *dudt, double *vsig, double *anorm, double *unorm,
                int32_t kernel)
{
    double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = targets ? targets[t] : t;
        double Pa, ca;
        orc_eos_one(eos, cs0, q_cs, r_ref, gamma, x[a], y[a], rho[a], u ? u[a] : 0.0, &Pa,
                    &ca);
        double ha = h[a];
        double Ra2 = (2.0 * ha) * (2.0 * ha);
        double sax = 0.0, say = 0.0, saz = 0.0, sdu = 0.0, vs = alpha * ca;
        double an = 0.0, un = 0.0;
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double dx = sep(x[a], x[b], periodic, L[0]);
            double dy = sep(y[a], y[b], periodic, L[1]);
            double dz = sep(z[a], z[b], periodic, L[2]);
            double r2 = dx * dx + dy * dy + dz * dz;
            double hb = h[b];
            double Rb2 = (2.0 * hb) * (2.0 * hb);
            int ina = r2 < Ra2, inb = r2 < Rb2;
            if (!ina && !inb) continue;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double rx = dx / r, ry = dy / r, rz = dz / r;
            double Fa = ina ? orc_kdf(kernel, r / ha) / (ORC_PI * ha * ha * ha * ha) : 0.0;
            double Fb = inb ? orc_kdf(kernel, r / hb) / (ORC_PI * hb * hb * hb * hb) : 0.0;
            double Pb, cb;
            orc_eos_one(eos, cs0, q_cs, r_ref, gamma, x[b], y[b], rho[b], u ? u[b] : 0.0,
                        &Pb, &cb);
            double vdr = (vx[a] - vx[b]) * rx + (vy[a] - vy[b]) * ry + (vz[a] - vz[b]) * rz;
            double qa = 0.0, qb = 0.0;
            if (vdr < 0.0) {
                double vsa = alpha * ca + beta * fabs(vdr);
                double vsb = alpha * cb + beta * fabs(vdr);
                qa = -0.5 * rho[a] * vsa * vdr;
                qb = -0.5 * rho[b] * vsb * vdr;
                if (vsa > vs) vs = vsa;
            }
            double mb = pmass(m0, level[b]);
            double Aa = (Pa + qa) / (omega[a] * rho[a] * rho[a]);
            double Bb = (Pb + qb) / (omega[b] * rho[b] * rho[b]);
            double term = mb * (Aa * Fa + Bb * Fb);
            sax -= term * rx;
            say -= term * ry;
            saz -= term * rz;
            double du = mb * Aa * vdr * Fa;
            sdu += du;
            an += fabs(term);
            un += fabs(du);
        }
        ax[t] = sax; ay[t] = say; az[t] = saz; dudt[t] = sdu;
        if (vsig) vsig[t] = vs;
        if (anorm) anorm[t] = an;
        if (unorm) unorm[t] = un;
    }
}

/* ------------------------------------------------------------------------ */
/* Interpolation of a field carried by a reference particle set, for the   */
/* relaxing of Sec. 2.4 (the reference accelerations at the positions of    */
/* the new particles).  Reading: the reference set's own SPH interpolant,   */
/*   A(x) = sum_b (m_b / rho_b) A_b W(|x - x_b|, h_b),                      */
/* over the b with |x - x_b|^2 < (2 h_b)^2 (strict), periodic minimum image. */
/* The caller passes q_b = (m_b / rho_b) A_b per component.                 */
/* ------------------------------------------------------------------------ */
void orc_interp(int64_t nt, const double *tx, const double *ty, const double *tz,
                int64_t nr, const double *rx, const double *ry, const double *rz,
                const double *rh, const double *q0, const double *q1, const double *q2,
                int32_t kernel, int32_t periodic, const double *lo, const double *hi,
                double *o0, double *o1, double *o2)
{
    double L[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int64_t b = 0; b < nr; ++b) {
            double dx = sep(tx[i], rx[b], periodic, L[0]);
            double dy = sep(ty[i], ry[b], periodic, L[1]);
            double dz = sep(tz[i], rz[b], periodic, L[2]);
            double r2 = dx * dx + dy * dy + dz * dz;
            double R = 2.0 * rh[b];
            if (!(r2 < R * R)) continue;
            double w = orc_wk(kernel, sqrt(r2), rh[b]);
            s0 += q0[b] * w;
            s1 += q1[b] * w;
            s2 += q2[b] * w;
        }
        o0[i] = s0;
        o1[i] = s1;
        o2[i] = s2;
    }
}

/* ------------------------------------------------------------------------ */
/* Time integration (not described by the paper; the standard kick-drift-   */
/* kick leapfrog) and the point-mass gravity of sink particles.             */
/* ------------------------------------------------------------------------ */
void orc_kick(int64_t n, double *vx, double *vy, double *vz, double *u, const double *ax,
              const double *ay, const double *az, const double *dudt, double dt)
{
    for (int64_t i = 0; i < n; ++i) {
        vx[i] += dt * ax[i];
        vy[i] += dt * ay[i];
        vz[i] += dt * az[i];
        if (u && dudt) u[i] += dt * dudt[i];
    }
}

void orc_drift(int64_t n, double *x, double *y, double *z, const double *vx,
               const double *vy, const double *vz, double dt, int32_t periodic,
               const double *lo, const double *hi)
{
    double *p[3] = {x, y, z};
    const double *v[3] = {vx, vy, vz};
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) {
            double xn = p[k][i] + dt * v[k][i];
            if (periodic) {
                double L = hi[k] - lo[k];
                if (xn >= hi[k]) xn -= L;
                else if (xn < lo[k]) xn += L;
            }
            p[k][i] = xn;
        }
    }
}

/* a += -G M_s (x - x_s) / (|x - x_s|^2 + eps_s^2)^(3/2), summed over sinks */
void orc_sink_gravity(int64_t n, const double *x, const double *y, const double *z,
                      int32_t ns, const double *sx, const double *sm, const double *seps,
                      double G, double *ax, double *ay, double *az)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int s = 0; s < ns; ++s) {
            double dx = x[i] - sx[3 * s + 0];
            double dy = y[i] - sx[3 * s + 1];
            double dz = z[i] - sx[3 * s + 2];
            double d2 = dx * dx + dy * dy + dz * dz + seps[s] * seps[s];
            double inv3 = 1.0 / (d2 * sqrt(d2));
            ax[i] -= G * sm[s] * dx * inv3;
            ay[i] -= G * sm[s] * dy * inv3;
            az[i] -= G * sm[s] * dz * inv3;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood 2014): state += gamma, then the mix13    */
/* finaliser.  Used for the random rotation of the split axis.              */
/* Per-particle stream: s = mix(seed ^ mix(id ^ mix(step))), where          */
/* mix(v) is the SplitMix64 output for state v; draw k (k = 1, 2) is the    */
/* k-th SplitMix64 output starting from state s.                            */
/* ------------------------------------------------------------------------ */
#define SM64_GAMMA 0x9e3779b97f4a7c15ULL

static uint64_t sm64_fin(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* k-th output (k >= 1) of SplitMix64 started from state s */
uint64_t orc_splitmix64(uint64_t s, uint64_t k) { return sm64_fin(s + k * SM64_GAMMA); }

static uint64_t stream_state(uint64_t seed, int64_t step, int64_t id)
{
    uint64_t a = orc_splitmix64((uint64_t)step, 1);
    uint64_t b = orc_splitmix64((uint64_t)id ^ a, 1);
    return orc_splitmix64(seed ^ b, 1);
}

/* uniform in [0, 1) from the top 53 bits */
static double u53(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------------ */
/* Refinement zones (paper Sec. 2.1, rule 1: the level is set only by       */
/* position).  A zone is a set of nested spheres about one centre, listed   */
/* outer to inner, with their levels.  A point's level in one zone is the   */
/* level of the innermost sphere with |x - c|^2 < r^2 (strict), or the       */
/* background level outside all of them.  Several zones combine by max      */
/* (refinement, background level 0) or by min (derefinement, background     */
/* l_max) (paper Sec. 2.1, rule 3).  *which is the first zone that gives    */
/* the combined level from one of its spheres, or -1.                       */
/* A zone of shape 1 is made of cylinders about the z axis through c        */
/* instead of spheres: the distance drops its z component.  The paper's     */
/* sound-wave test refines a circle in the x-y plane of a thin box (its     */
/* appendix A), which is such a cylinder.                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nz;
    const double *c;     /* nz x 3 */
    const int32_t *nsh;  /* nz */
    const double *r;     /* nz x 8, outer -> inner */
    const int32_t *ell;  /* nz x 8 */
    const int32_t *shape; /* nz: 0 spheres, 1 cylinders along z */
    int32_t background;
    int32_t derefine;
} orc_zones;

/* z offset from zone k's centre as its shape counts it */
static double zone_dz(const orc_zones *Z, int k, double z)
{
    return Z->shape[k] == 1 ? 0.0 : z - Z->c[3 * k + 2];
}

static int zone_level(const orc_zones *Z, double x, double y, double z, int *which)
{
    int best = Z->background;
    int w = -1;
    for (int k = 0; k < Z->nz; ++k) {
        double dx = x - Z->c[3 * k + 0];
        double dy = y - Z->c[3 * k + 1];
        double dz = zone_dz(Z, k, z);
        double d2 = dx * dx + dy * dy + dz * dz;
        int lev = -1;
        for (int s = 0; s < Z->nsh[k]; ++s) {
            double rr = Z->r[8 * k + s];
            if (d2 < rr * rr) lev = Z->ell[8 * k + s];
        }
        if (lev < 0) continue;
        if (Z->derefine ? (lev < best) : (lev > best)) { best = lev; w = k; }
        else if (lev == best && w < 0) w = k;
    }
    if (which) *which = w;
    return best;
}

int32_t orc_zone_level(double x, double y, double z, int32_t nz, const double *zc,
                       const int32_t *znsh, const double *zr, const int32_t *zell,
                       const int32_t *zshape, int32_t background, int32_t derefine)
{
    orc_zones Z = {nz, zc, znsh, zr, zell, zshape, background, derefine};
    return zone_level(&Z, x, y, z, NULL);
}

/* ------------------------------------------------------------------------ */
/* Split (paper Sec. 2.2).  A particle whose level is below its zone level  */
/* is split: the parent slot becomes one child and a new child is appended; */
/* both take the parent's velocity and u, level + 1 and h (1/2)^(1/3); they  */
/* sit on opposite sides of the parent at distance r_sep along an axis w.   */
/*  - r_sep = r_sep_factor h (0.2 h in the paper), capped at nn_cap times    */
/*    the nearest-neighbour distance when nn_cap > 0 (paper Sec. 2.2, after  */
/*    Franchini et al.);                                                    */
/*  - tangential mode: v = x - zone centre (z part dropped for a cylinder    */
/*    zone); w0 = unit(v x e_k), k the axis                                  */
/*    of smallest |v_k| (ties to the lowest k); w = w0 cos t + (vhat x w0)   */
/*    sin t with t = 2 pi U, a random rotation about v (paper Sec. 2.2);    */
/*  - random mode (or no zone centre, or v = 0): w uniform on the sphere    */
/*    from two draws (cos theta = 2U1 - 1, phi = 2 pi U2).                  */
/* Each coordinate of the two children is built so that x+ + x- = 2x        */
/* exactly whenever the offset is no larger than |x|: the child on the far  */
/* side from zero is rounded first, the exact shift d' = x_far - x taken,    */
/* and the near child set to x - d' (exact).                                */
/* Reading: the paper loops over levels from the lowest up; since a child    */
/* made in this pass is not examined again, the set of splits is the same   */
/* in any order, and new children are appended in ascending parent index.   */
/* ------------------------------------------------------------------------ */
#define ORC_CBRT_HALF 0.79370052598409973737585281963615 /* 2^(-1/3) */
#define ORC_CBRT_TWO 1.2599210498948731647672106072782   /* 2^(1/3)  */

static void split_pair_coord(double x, double d, double *xp, double *xm)
{
    if (x != 0.0 && fabs(d) <= fabs(x)) {
        double sgn = x > 0.0 ? 1.0 : -1.0;
        double far = x + sgn * fabs(d);
        double dd = far - x;
        double near = x - dd;
        int plus_is_far = (d * sgn) >= 0.0;
        *xp = plus_is_far ? far : near;
        *xm = plus_is_far ? near : far;
    } else {
        *xp = x + d;
        *xm = x - d;
    }
}

static void split_axis(const orc_zones *Z, int zone, int mode, uint64_t s, double x,
                       double y, double z, double w[3])
{
    double U1 = u53(orc_splitmix64(s, 1));
    double U2 = u53(orc_splitmix64(s, 2));
    if (mode == 0 && zone >= 0) {
        double v[3] = {x - Z->c[3 * zone + 0], y - Z->c[3 * zone + 1], zone_dz(Z, zone, z)};
        double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (vn > 0.0) {
            int k = 0;
            if (fabs(v[1]) < fabs(v[k])) k = 1;
            if (fabs(v[2]) < fabs(v[k])) k = 2;
            double e[3] = {0.0, 0.0, 0.0};
            e[k] = 1.0;
            double w0[3] = {v[1] * e[2] - v[2] * e[1], v[2] * e[0] - v[0] * e[2],
                            v[0] * e[1] - v[1] * e[0]};
            double wn = sqrt(w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2]);
            w0[0] /= wn; w0[1] /= wn; w0[2] /= wn;
            double vh[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
            double b[3] = {vh[1] * w0[2] - vh[2] * w0[1], vh[2] * w0[0] - vh[0] * w0[2],
                           vh[0] * w0[1] - vh[1] * w0[0]};
            double t = 2.0 * ORC_PI * U1;
            double ct = cos(t), st = sin(t);
            for (int i = 0; i < 3; ++i) w[i] = w0[i] * ct + b[i] * st;
            return;
        }
    }
    double cth = 2.0 * U1 - 1.0;
    double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
    double ph = 2.0 * ORC_PI * U2;
    w[0] = sth * cos(ph);
    w[1] = sth * sin(ph);
    w[2] = cth;
}

static double wrap(double v, int periodic, double lo, double hi)
{
    if (!periodic) return v;
    if (v >= hi) return v - (hi - lo);
    if (v < lo) return v + (hi - lo);
    return v;
}

/* Centre of mass of a merging pair along one axis (Sec. 2.3: the merged
 * particle sits at the pair's centre of mass; equal masses).  In a periodic
 * box the removed particle's coordinate o is taken at its minimum image about
 * the kept one's, k, before averaging, and the mean is wrapped back into the
 * box, so that a pair across the boundary merges next to the boundary and
 * not at mid-box.  Pairs closer than half the box average as they are. */
static double merge_mid(double k, double o, int periodic, double lo, double hi)
{
    if (periodic) {
        double L = hi - lo, d = o - k;
        if (d > 0.5 * L) o -= L;
        else if (d < -0.5 * L) o += L;
    }
    return wrap((k + o) * 0.5, periodic, lo, hi);
}

/* ------------------------------------------------------------------------ */
/* The pairing tree used for merging (paper Sec. 2.3): a k-d tree cut       */
/* through the centre of mass, with an even count forced on each side, so   */
/* that every leaf holds exactly two particles.                             */
/* Readings: coordinates are quantised to 2^21 steps per axis over the box; */
/* each node is cut on the axis of largest quantised extent (ties x<y<z) at */
/* c = floor(mean quantised coordinate), left meaning coord < c.  If no     */
/* coordinate lies below c the cut moves up one step (coord <= c); if then  */
/* every coordinate is equal (all particles at one quantised point) the left */
/* side is the first 2 floor(n/4) in id order.  With k the resulting left   */
/* count, an odd k is made even by moving one particle across the cut      */
/* towards balance: k + 1 (the smallest of the right side in (coordinate,  */
/* id) order joins the left) if the left side is the smaller, else k - 1     */
/* (the largest of the left side joins the right).  So the left side is    */
/* always the k' smallest in (coordinate, id) order, and both sides keep    */
/* ascending id order.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    const int64_t *qc[3]; /* quantised coordinates */
    const int64_t *id;
} tree_ctx;

/* qsort is not re-entrant; the pairing runs on one thread */
static const tree_ctx *g_tree;
static int g_axis;

static int cmp_coord_id(const void *pa, const void *pb)
{
    int64_t p = *(const int64_t *)pa, q = *(const int64_t *)pb;
    int64_t cp = g_tree->qc[g_axis][p], cq = g_tree->qc[g_axis][q];
    if (cp != cq) return (cp > cq) - (cp < cq);
    return (g_tree->id[p] > g_tree->id[q]) - (g_tree->id[p] < g_tree->id[q]);
}

static int cmp_id(const void *pa, const void *pb)
{
    int64_t p = *(const int64_t *)pa, q = *(const int64_t *)pb;
    return (g_tree->id[p] > g_tree->id[q]) - (g_tree->id[p] < g_tree->id[q]);
}

static int cmp_i64(const void *pa, const void *pb)
{
    int64_t p = *(const int64_t *)pa, q = *(const int64_t *)pb;
    return (p > q) - (p < q);
}

/* idx[0..n) in ascending id order; appends the leaf pairs to pairs */
static void pair_tree(const tree_ctx *T, int64_t *idx, int64_t n, int64_t *pairs,
                      int64_t *npairs)
{
    if (n < 2) return;
    if (n == 2) {
        pairs[2 * *npairs + 0] = idx[0];
        pairs[2 * *npairs + 1] = idx[1];
        *npairs += 1;
        return;
    }
    int64_t mn[3], mx[3];
    for (int k = 0; k < 3; ++k) { mn[k] = INT64_MAX; mx[k] = INT64_MIN; }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            int64_t v = T->qc[k][idx[i]];
            if (v < mn[k]) mn[k] = v;
            if (v > mx[k]) mx[k] = v;
        }
    int ax = 0;
    for (int k = 1; k < 3; ++k)
        if (mx[k] - mn[k] > mx[ax] - mn[ax]) ax = k;
    int64_t sum = 0;
    for (int64_t i = 0; i < n; ++i) sum += T->qc[ax][idx[i]];
    int64_t c = sum / n;
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (T->qc[ax][idx[i]] < c) k += 1;
    if (k == 0) {
        /* no coordinate below the cut: move it up one quantisation step */
        c += 1;
        for (int64_t i = 0; i < n; ++i)
            if (T->qc[ax][idx[i]] < c) k += 1;
    }
    int64_t kp;
    if (k == n) kp = 2 * (n / 4); /* all at one point: split by id */
    else if (k % 2 == 0) kp = k;
    else if (k < n - k) kp = k + 1;
    else kp = k - 1;
    /* the left side is the kp smallest in (coordinate, id) order */
    g_tree = T;
    g_axis = ax;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_coord_id);
    /* each side back to ascending id order */
    qsort(idx, (size_t)kp, sizeof(int64_t), cmp_id);
    qsort(idx + kp, (size_t)(n - kp), sizeof(int64_t), cmp_id);
    pair_tree(T, idx, kp, pairs, npairs);
    pair_tree(T, idx + kp, n - kp, pairs, npairs);
}

/* Quantised coordinate: floor((x - lo) * 2^21 / (hi - lo)), clamped. */
static int64_t quantise(double v, double lo, double hi)
{
    double s = 2097152.0 / (hi - lo);
    double f = floor((v - lo) * s);
    if (f < 0.0) f = 0.0;
    if (f > 2097151.0) f = 2097151.0;
    return (int64_t)f;
}

/* Pairing of an explicit set (exported for the pins): cand[0..nc) are
 * particle indices; writes floor(nc/2) pairs.  The set is first put in
 * ascending id order and, if odd, its highest id is left out. */
int64_t orc_pair_tree(int64_t nc, const int64_t *cand, const double *x, const double *y,
                      const double *z, const int64_t *id, const double *lo, const double *hi,
                      int64_t n, int64_t *pairs)
{
    int64_t *qc[3];
    for (int k = 0; k < 3; ++k) qc[k] = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < nc; ++i) {
        int64_t p = cand[i];
        qc[0][p] = quantise(x[p], lo[0], hi[0]);
        qc[1][p] = quantise(y[p], lo[1], hi[1]);
        qc[2][p] = quantise(z[p], lo[2], hi[2]);
    }
    int64_t *idx = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    memcpy(idx, cand, (size_t)nc * sizeof(int64_t));
    tree_ctx T = {{qc[0], qc[1], qc[2]}, id};
    g_tree = &T;
    qsort(idx, (size_t)nc, sizeof(int64_t), cmp_id);
    int64_t m = nc - (nc % 2);
    int64_t np = 0;
    pair_tree(&T, idx, m, pairs, &np);
    free(idx);
    for (int k = 0; k < 3; ++k) free(qc[k]);
    return np;
}

/* ------------------------------------------------------------------------ */
/* One split/merge pass over all particles (paper Sec. 2.5 and Fig. 2:      */
/* split from the lowest level up, then merge from the highest level down;  */
/* a particle changes level at most once per pass).                         */
/* Split: each child is appended after the survivors; the children are     */
/* numbered next_id, next_id + 1, ... in ascending order of their parents'  */
/* ids, so the numbering does not depend on the order of the arrays.       */
/* Merge (paper Sec. 2.3), for l = l_max .. 1: the candidates are the level- */
/* l particles not changed earlier in this pass, in ascending id order; if  */
/* their number is odd the highest id is left out until the next pass (the  */
/* paper leaves out "the last listed").  They are paired by the tree above. */
/* A leaf merges when the zone level at its centre of mass (x1 + x2)/2 is    */
/* below l: the lower id is kept at the centre of mass with the mean        */
/* velocity and mean u (mass is equal), level l - 1 and h 2^(1/3); the other */
/* is removed.  Survivors keep their order.                                 */
/* With individual timesteps (paper Sec. 2.5) only the particles with      */
/* active[a] != 0 are examined for splitting or paired for merging (active */
/* NULL: all).  origin (room for cap, may be NULL) receives, per slot after */
/* the pass, the slot the particle held before it (an appended child: its  */
/* parent's); changed_out (room for cap, may be NULL) flags the particles  */
/* a split made or a merge kept.                                           */
/* Arrays must have room for `cap` particles.  Returns 0, or 2 if the        */
/* splits need more than cap (then nothing is changed and *n_split holds the */
/* number of particles needed).                                             */
/* ------------------------------------------------------------------------ */
int32_t orc_split_merge(int64_t n, int64_t cap, double *x, double *y, double *z, double *vx,
                        double *vy, double *vz, double *u, double *h, int8_t *level,
                        int64_t *id, int64_t *next_id, const double *dnn, int32_t nz,
                        const double *zc, const int32_t *znsh, const double *zr,
                        const int32_t *zell, const int32_t *zshape, int32_t background,
                        int32_t derefine, double r_sep_factor, double nn_cap, int32_t split_mode, uint64_t seed,
                        int64_t step, int32_t periodic, const double *lo, const double *hi,
                        int32_t do_split, int32_t do_merge, int64_t *n_out, int64_t *n_split,
                        int64_t *n_merged, int64_t *n_spare, const unsigned char *active,
                        int64_t *origin, unsigned char *changed_out)
{
    orc_zones Z = {nz, zc, znsh, zr, zell, zshape, background, derefine};
    int64_t ns = 0;
    *n_split = 0; *n_merged = 0; *n_spare = 0; *n_out = n;

    unsigned char *changed = (unsigned char *)calloc((size_t)(cap > 0 ? cap : 1), 1);
    int *zone_of = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    unsigned char *do_sp = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    const int64_t n0 = n;
    if (origin)
        for (int64_t a = 0; a < n; ++a) origin[a] = a;

    if (do_split) {
        for (int64_t a = 0; a < n; ++a) {
            int w;
            int lz = zone_level(&Z, x[a], y[a], z[a], &w);
            zone_of[a] = w;
            if (level[a] < lz && (!active || active[a])) { do_sp[a] = 1; ns += 1; }
        }
        if (n + ns > cap) {
            *n_split = n + ns;
            free(changed); free(zone_of); free(do_sp);
            return 2;
        }
        /* the children are numbered in the order of their parents' ids */
        int64_t *pid = (int64_t *)malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int64_t));
        int64_t np = 0;
        for (int64_t a = 0; a < n; ++a)
            if (do_sp[a]) pid[np++] = id[a];
        qsort(pid, (size_t)np, sizeof(int64_t), cmp_i64);
        int64_t slot = n;
        for (int64_t a = 0; a < n; ++a) {
            if (!do_sp[a]) continue;
            const int64_t *at = (const int64_t *)bsearch(&id[a], pid, (size_t)np, sizeof(int64_t),
                                                         cmp_i64);
            uint64_t s = stream_state(seed, step, id[a]);
            double w[3];
            split_axis(&Z, zone_of[a], split_mode, s, x[a], y[a], z[a], w);
            double r = r_sep_factor * h[a];
            if (nn_cap > 0.0 && dnn && isfinite(dnn[a]) && nn_cap * dnn[a] < r)
                r = nn_cap * dnn[a];
            double p[3] = {x[a], y[a], z[a]};
            double xp[3], xm[3];
            for (int k = 0; k < 3; ++k) split_pair_coord(p[k], r * w[k], &xp[k], &xm[k]);
            x[slot] = wrap(xm[0], periodic, lo[0], hi[0]);
            y[slot] = wrap(xm[1], periodic, lo[1], hi[1]);
            z[slot] = wrap(xm[2], periodic, lo[2], hi[2]);
            x[a] = wrap(xp[0], periodic, lo[0], hi[0]);
            y[a] = wrap(xp[1], periodic, lo[1], hi[1]);
            z[a] = wrap(xp[2], periodic, lo[2], hi[2]);
            vx[slot] = vx[a]; vy[slot] = vy[a]; vz[slot] = vz[a];
            u[slot] = u[a];
            double hc = h[a] * ORC_CBRT_HALF;
            h[a] = hc; h[slot] = hc;
            level[a] = (int8_t)(level[a] + 1);
            level[slot] = level[a];
            id[slot] = *next_id + (at - pid);
            changed[a] = 1; changed[slot] = 1;
            if (origin) origin[slot] = a;
            slot += 1;
        }
        free(pid);
        *next_id += ns;
        n = n + ns;
        *n_split = ns;
    }

    if (do_merge) {
        int lmax = 0;
        for (int64_t a = 0; a < n; ++a)
            if (level[a] > lmax) lmax = level[a];
        unsigned char *removed = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
        int64_t *cand = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int64_t *pairs = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        for (int l = lmax; l >= 1; --l) {
            int64_t nc = 0;
            for (int64_t a = 0; a < n; ++a)
                if (level[a] == l && !changed[a] && !removed[a] &&
                    (a >= n0 || !active || active[a]))
                    cand[nc++] = a;
            if (nc % 2) *n_spare += 1;
            int64_t np = orc_pair_tree(nc, cand, x, y, z, id, lo, hi, n, pairs);
            for (int64_t k = 0; k < np; ++k) {
                int64_t p = pairs[2 * k], q = pairs[2 * k + 1];
                int64_t keep = id[p] < id[q] ? p : q;
                int64_t gone = keep == p ? q : p;
                double cx = merge_mid(x[keep], x[gone], periodic, lo[0], hi[0]);
                double cy = merge_mid(y[keep], y[gone], periodic, lo[1], hi[1]);
                double cz = merge_mid(z[keep], z[gone], periodic, lo[2], hi[2]);
                if (!(zone_level(&Z, cx, cy, cz, NULL) < l)) continue;
                x[keep] = cx; y[keep] = cy; z[keep] = cz;
                vx[keep] = (vx[p] + vx[q]) * 0.5;
                vy[keep] = (vy[p] + vy[q]) * 0.5;
                vz[keep] = (vz[p] + vz[q]) * 0.5;
                u[keep] = (u[p] + u[q]) * 0.5;
                h[keep] = h[keep] * ORC_CBRT_TWO;
                level[keep] = (int8_t)(l - 1);
                changed[keep] = 1;
                removed[gone] = 1;
                *n_merged += 1;
            }
        }
        int64_t w = 0;
        for (int64_t a = 0; a < n; ++a) {
            if (removed[a]) continue;
            if (w != a) {
                x[w] = x[a]; y[w] = y[a]; z[w] = z[a];
                vx[w] = vx[a]; vy[w] = vy[a]; vz[w] = vz[a];
                u[w] = u[a]; h[w] = h[a]; level[w] = level[a]; id[w] = id[a];
                changed[w] = changed[a];
                if (origin) origin[w] = origin[a];
            }
            w += 1;
        }
        n = w;
        free(removed); free(cand); free(pairs);
    }
    *n_out = n;
    if (changed_out)
        for (int64_t a = 0; a < n; ++a) changed_out[a] = changed[a];
    free(changed); free(zone_of); free(do_sp);
    return 0;
}

/*
 * sscn_sym_oracle.c -- plain FP64 CPU oracle for split-step Crank-Nicolson
 * propagation of the Gross-Pitaevskii equation in the symmetric traps of the
 * paper's program summary ("Nature of problem": circular symmetry in 2D,
 * radial (spherical) and axial symmetry in 3D; "Summary of revisions": the
 * imagcir/realcir, imagsph/realsph and imagaxi/realaxi programs).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path loads this file:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header, table or helper with the GPU library.
 *
 * The paper prints no discretisation, so the following is stated here (the
 * readings are listed with the others in the design notes):
 *
 *   GP equation   i dpsi/dt = [ -1/2 Lap + V + g |psi|^2 ] psi
 *   circular      psi(r), 2D:  Lap = (1/r) d/dr (r d/dr),   V = w^2 r^2 / 2
 *   spherical     psi(r), 3D:  Lap = (1/r^2) d/dr (r^2 d/dr), V = w^2 r^2 / 2
 *   axial         psi(rho, z): Lap = (1/rho) d/drho (rho d/drho) + d2/dz2,
 *                 V = (w_rho^2 rho^2 + w_z^2 z^2) / 2
 *
 * Radial grid: n cells [i dr, (i+1) dr], values at the centres
 * r_i = (i + 1/2) dr.  The radial Laplacian is the finite-volume (flux)
 * form with face weights F_i = (i dr)^k at r = i dr and cell weights
 * W_i = (1/dr) * integral of r^k over cell i (k = 1: W_i = r_i; k = 2:
 * W_i = r_i^2 + dr^2 / 12):
 *
 *   (Lap psi)_i = [F_{i+1} (psi_{i+1} - psi_i) - F_i (psi_i - psi_{i-1})] / (W_i dr^2).
 *
 * F_0 = 0: no flux through the origin, so no value at r = 0 is needed (the
 * regularity condition).  psi = 0 on the ghost cell past the outer edge.
 * z (axial) is a Cartesian axis as in the anisotropic oracle: n_z points at
 * z_j = (j - (n_z - 1)/2) dz, psi = 0 on the ghosts at both ends.
 *
 * Inner product and norm: <a, b> = c dr (dz) sum W_i conj(a) b with c = 2 pi
 * (circular, axial) or 4 pi (spherical); the discrete Laplacian is
 * self-adjoint in it, so the real-time Crank-Nicolson substeps conserve the
 * norm exactly.
 *
 * One step of length dt (Lie splitting, the same order as the anisotropic
 * oracle): the pointwise substep, then the Crank-Nicolson substep along r,
 * then (axial) along z; in imaginary time then renormalise to unit norm.
 * The r substep solves (1 + tau H_r) v = (1 - tau H_r) u on every radial
 * line, H_r = -Lap_r / 2, tau = dt/2 (imaginary) or i dt/2 (real), with a
 * general tridiagonal Thomas elimination (no pivoting: the matrix is
 * strictly diagonally dominant).
 *
 * Observables (the energy functional of the discrete Hamiltonian):
 *   N = <psi, psi>,  K = Re <psi, H_kin psi>,  P = <psi, V psi>,
 *   where K is evaluated in its gradient form (summation by parts, an exact
 *   identity): K = c dr (dz) [ 1/2 sum_j sum_faces F_f |psi_f - psi_{f-1}|^2 / dr^2
 *   + 1/2 sum_i W_i sum_z-edges |psi_{j+1} - psi_j|^2 / dz^2 ], ghosts zero
 *   (the operator form loses about eps * d_i / |H psi| to cancellation on
 *   fine grids),
 *   I = c dr (dz) sum W |psi|^4,
 *   E = (K + P + g I / 2) / N,  mu = (K + P + g I) / N,
 *   moments <r>, <r^2> (radial), <z>, <z^2> (axial), divided by N.
 *
 * Layout: axial states are (n_z, n_r) arrays, r fastest; circular and
 * spherical states are one line of n_r values.  Complex values interleaved.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORS_PI 3.14159265358979323846

#define ORS_IMAG 0
#define ORS_REAL 1
#define ORS_CIR 1
#define ORS_SPH 2
#define ORS_AXI 3

typedef struct {
    int geom;          /* ORS_CIR, ORS_SPH or ORS_AXI */
    int n[2];          /* n[0] radial cells, n[1] z points (axial; 1 otherwise) */
    double dx[2];      /* dr, dz */
    double omega[2];   /* omega_r (omega_rho), omega_z (axial) */
    double g;
    double dt;
    int mode;          /* ORS_IMAG or ORS_REAL */
    int renorm_every;  /* imaginary time: renormalise every this many steps */
} ors_problem;

static int ors_check(const ors_problem *pb)
{
    if (pb->geom != ORS_CIR && pb->geom != ORS_SPH && pb->geom != ORS_AXI) return -1;
    if (pb->n[0] < 1 || pb->n[1] < 1) return -1;
    if (pb->geom != ORS_AXI && pb->n[1] != 1) return -1;
    if (!(pb->dx[0] > 0.0)) return -1;
    if (pb->geom == ORS_AXI && !(pb->dx[1] > 0.0)) return -1;
    if (!(pb->dt > 0.0)) return -1;
    if (pb->mode != ORS_IMAG && pb->mode != ORS_REAL) return -1;
    return 0;
}

static int ors_k(const ors_problem *pb) { return pb->geom == ORS_SPH ? 2 : 1; }

static double ors_c(const ors_problem *pb) { return pb->geom == ORS_SPH ? 4.0 * ORS_PI : 2.0 * ORS_PI; }

static double ors_r(const ors_problem *pb, int i) { return (i + 0.5) * pb->dx[0]; }

static double ors_z(const ors_problem *pb, int j)
{
    return pb->geom == ORS_AXI ? (j - 0.5 * (pb->n[1] - 1)) * pb->dx[1] : 0.0;
}

/* face weight at r = i dr */
static double ors_face(const ors_problem *pb, int i)
{
    double r = i * pb->dx[0];
    return ors_k(pb) == 1 ? r : r * r;
}

/* cell weight: (1/dr) * integral of r^k over cell i */
static double ors_cell(const ors_problem *pb, int i)
{
    double r = ors_r(pb, i), h = pb->dx[0];
    return ors_k(pb) == 1 ? r : r * r + h * h / 12.0;
}

/* H_r = -Lap_r / 2 on cell i: d_i psi_i - l_i psi_{i-1} - u_i psi_{i+1} */
static void ors_radial_coefs(const ors_problem *pb, int i, double *l, double *d, double *u)
{
    double h2 = pb->dx[0] * pb->dx[0], w = ors_cell(pb, i);
    *l = ors_face(pb, i) / (2.0 * h2 * w);
    *u = ors_face(pb, i + 1) / (2.0 * h2 * w);
    *d = *l + *u;
}

static double ors_potential(const ors_problem *pb, int i, int j)
{
    double r = ors_r(pb, i), z = ors_z(pb, j);
    double v = 0.5 * pb->omega[0] * pb->omega[0] * r * r;
    if (pb->geom == ORS_AXI) v += 0.5 * pb->omega[1] * pb->omega[1] * z * z;
    return v;
}

/* volume element of the inner product apart from W_i */
static double ors_dvol(const ors_problem *pb)
{
    double dv = ors_c(pb) * pb->dx[0];
    if (pb->geom == ORS_AXI) dv *= pb->dx[1];
    return dv;
}

/* Textbook Thomas elimination for a x_{i-1} + b x_i + c x_{i+1} = r,
 * a[0] and c[n-1] unused; cp, dp scratch of length n. */
static void ors_thomas(int n, const double complex *a, const double complex *b,
                       const double complex *c, const double complex *r,
                       double complex *x, double complex *cp, double complex *dp)
{
    cp[0] = c[0] / b[0];
    dp[0] = r[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double complex den = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / den;
        dp[i] = (r[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

static double complex ors_tau(const ors_problem *pb)
{
    return pb->mode == ORS_REAL ? I * 0.5 * pb->dt : 0.5 * pb->dt;
}

/* Crank-Nicolson substep along r on one radial line u[0..n-1] (in place);
 * w is scratch of 7 n. */
static void ors_radial_line(const ors_problem *pb, double complex *u, double complex *w)
{
    const int n = pb->n[0];
    double complex *a = w, *b = w + n, *c = w + 2 * n, *rhs = w + 3 * n;
    double complex *x = w + 4 * n, *cp = w + 5 * n, *dp = w + 6 * n;
    const double complex tau = ors_tau(pb);
    for (int i = 0; i < n; ++i) {
        double l, d, up;
        ors_radial_coefs(pb, i, &l, &d, &up);
        double complex left = (i > 0) ? u[i - 1] : 0.0;
        double complex right = (i + 1 < n) ? u[i + 1] : 0.0;
        double complex hu = d * u[i] - l * left - up * right;
        rhs[i] = u[i] - tau * hu;
        a[i] = -tau * l;
        b[i] = 1.0 + tau * d;
        c[i] = -tau * up;
    }
    ors_thomas(n, a, b, c, rhs, x, cp, dp);
    for (int i = 0; i < n; ++i) u[i] = x[i];
}

/* Crank-Nicolson substep along z (axial) on one z line with stride n_r;
 * H_z = -d2/dz2 / 2 with the 3-point Laplacian and zero ghosts. */
static void ors_z_line(const ors_problem *pb, double complex *psi, int i, double complex *w)
{
    const int m = pb->n[1], nr = pb->n[0];
    double complex *a = w, *b = w + m, *c = w + 2 * m, *rhs = w + 3 * m;
    double complex *x = w + 4 * m, *cp = w + 5 * m, *dp = w + 6 * m;
    const double complex tau = ors_tau(pb);
    const double k = 1.0 / (2.0 * pb->dx[1] * pb->dx[1]);
    for (int j = 0; j < m; ++j) {
        double complex v = psi[i + (long)nr * j];
        double complex lo = (j > 0) ? psi[i + (long)nr * (j - 1)] : 0.0;
        double complex hi = (j + 1 < m) ? psi[i + (long)nr * (j + 1)] : 0.0;
        double complex hu = k * (2.0 * v - lo - hi);
        rhs[j] = v - tau * hu;
        a[j] = -tau * k;
        b[j] = 1.0 + tau * 2.0 * k;
        c[j] = -tau * k;
    }
    ors_thomas(m, a, b, c, rhs, x, cp, dp);
    for (int j = 0; j < m; ++j) psi[i + (long)nr * j] = x[j];
}

static long ors_points(const ors_problem *pb) { return (long)pb->n[0] * pb->n[1]; }

static void ors_pointwise(const ors_problem *pb, double complex *psi)
{
    for (int j = 0; j < pb->n[1]; ++j)
        for (int i = 0; i < pb->n[0]; ++i) {
            long p = i + (long)pb->n[0] * j;
            double q = creal(psi[p]) * creal(psi[p]) + cimag(psi[p]) * cimag(psi[p]);
            double phi = pb->dt * (ors_potential(pb, i, j) + pb->g * q);
            if (pb->mode == ORS_IMAG)
                psi[p] = exp(-phi) * psi[p];
            else
                psi[p] = (cos(phi) - I * sin(phi)) * psi[p];
        }
}

static int ors_sweep(const ors_problem *pb, double complex *psi, int axis)
{
    int m = (axis == 0) ? pb->n[0] : pb->n[1];
    double complex *w = malloc(sizeof(double complex) * 7 * (size_t)m);
    if (!w) return -2;
    if (axis == 0)
        for (int j = 0; j < pb->n[1]; ++j) ors_radial_line(pb, psi + (long)pb->n[0] * j, w);
    else
        for (int i = 0; i < pb->n[0]; ++i) ors_z_line(pb, psi, i, w);
    free(w);
    return 0;
}

static double ors_norm_c(const ors_problem *pb, const double complex *psi)
{
    double acc = 0.0;
    for (int j = 0; j < pb->n[1]; ++j)
        for (int i = 0; i < pb->n[0]; ++i) {
            double complex v = psi[i + (long)pb->n[0] * j];
            acc += ors_cell(pb, i) * (creal(v) * creal(v) + cimag(v) * cimag(v));
        }
    return ors_dvol(pb) * acc;
}

static int ors_step(const ors_problem *pb, double complex *psi, long step_index)
{
    ors_pointwise(pb, psi);
    if (ors_sweep(pb, psi, 0)) return -2;
    if (pb->geom == ORS_AXI && ors_sweep(pb, psi, 1)) return -2;
    if (pb->mode == ORS_IMAG && pb->renorm_every > 0 && step_index % pb->renorm_every == 0) {
        double scale = 1.0 / sqrt(ors_norm_c(pb, psi));
        long np = ors_points(pb);
        for (long p = 0; p < np; ++p) psi[p] *= scale;
    }
    return 0;
}

/* out[0..11] = N, mu, E, K, P, I, <r>, <z>, 0, <r^2>, <z^2>, 0 */
static void ors_observe_c(const ors_problem *pb, const double complex *psi, double *out)
{
    const int nr = pb->n[0], nz = pb->n[1];
    const double dr2 = pb->dx[0] * pb->dx[0];
    const double dz2 = (pb->geom == ORS_AXI) ? pb->dx[1] * pb->dx[1] : 1.0;
    double s2 = 0, sk = 0, sp = 0, s4 = 0, mr = 0, mz = 0, mr2 = 0, mz2 = 0;
    for (int j = 0; j < nz; ++j)
        for (int i = 0; i < nr; ++i) {
            long p = i + (long)nr * j;
            double complex v = psi[p];
            double w = ors_cell(pb, i);
            double q = creal(v) * creal(v) + cimag(v) * cimag(v);
            /* the radial face above cell i (the ghost cell past the edge is 0) */
            double complex up = (i + 1 < nr) ? psi[p + 1] : 0.0;
            double complex dd = up - v;
            sk += 0.5 * ors_face(pb, i + 1) * (creal(dd) * creal(dd) + cimag(dd) * cimag(dd)) / dr2;
            if (pb->geom == ORS_AXI) {
                /* the z edge above point j, and below the first point */
                double complex hi = (j + 1 < nz) ? psi[p + nr] : 0.0;
                double complex dz = hi - v;
                double e = creal(dz) * creal(dz) + cimag(dz) * cimag(dz);
                if (j == 0) e += q;
                sk += 0.5 * w * e / dz2;
            }
            double r = ors_r(pb, i), z = ors_z(pb, j);
            s2 += w * q;
            sp += w * ors_potential(pb, i, j) * q;
            s4 += w * q * q;
            mr += w * r * q;
            mr2 += w * r * r * q;
            mz += w * z * q;
            mz2 += w * z * z * q;
        }
    double dv = ors_dvol(pb);
    double N = dv * s2, K = dv * sk, P = dv * sp, In = dv * s4;
    out[0] = N;
    out[1] = (K + P + pb->g * In) / N;
    out[2] = (K + P + 0.5 * pb->g * In) / N;
    out[3] = K;
    out[4] = P;
    out[5] = In;
    out[6] = dv * mr / N;
    out[7] = dv * mz / N;
    out[8] = 0.0;
    out[9] = dv * mr2 / N;
    out[10] = dv * mz2 / N;
    out[11] = 0.0;
}

/* ------------------------------------------------------------------ */
/* Exported entry points (interleaved complex psi)                     */
/* ------------------------------------------------------------------ */

static double complex *ors_load(const ors_problem *pb, const double *psi)
{
    long np = ors_points(pb);
    double complex *c = malloc(sizeof(double complex) * (size_t)np);
    if (!c) return NULL;
    for (long p = 0; p < np; ++p) c[p] = psi[2 * p] + I * psi[2 * p + 1];
    return c;
}

static void ors_store(const ors_problem *pb, const double complex *c, double *psi)
{
    long np = ors_points(pb);
    for (long p = 0; p < np; ++p) {
        psi[2 * p] = creal(c[p]);
        psi[2 * p + 1] = cimag(c[p]);
    }
}

/* The coefficients of H_r on every radial cell and the cell weights (for
 * the line-solver pin and the quadrature pins). */
int ors_coefs(const ors_problem *pb, double *l, double *d, double *u, double *w)
{
    if (ors_check(pb)) return -1;
    for (int i = 0; i < pb->n[0]; ++i) {
        ors_radial_coefs(pb, i, &l[i], &d[i], &u[i]);
        w[i] = ors_cell(pb, i);
    }
    return 0;
}

int ors_observe(const ors_problem *pb, const double *psi, double *out)
{
    if (ors_check(pb)) return -1;
    double complex *c = ors_load(pb, psi);
    if (!c) return -2;
    ors_observe_c(pb, c, out);
    free(c);
    return 0;
}

/* which = -1 pointwise substep, 0 the r substep, 1 the z substep (axial) */
int ors_substep(const ors_problem *pb, double *psi, int which)
{
    if (ors_check(pb)) return -1;
    if (which < -1 || which > 1 || (which == 1 && pb->geom != ORS_AXI)) return -1;
    double complex *c = ors_load(pb, psi);
    if (!c) return -2;
    int rc = 0;
    if (which < 0) ors_pointwise(pb, c);
    else rc = ors_sweep(pb, c, which);
    ors_store(pb, c, psi);
    free(c);
    return rc;
}

/* As orc_run of the anisotropic oracle: nsteps steps from first_step, a row
 * {step, N, mu, E, K, P, I, <r>, <z>, 0, <r^2>, <z^2>, 0} every
 * observe_every steps and after the last, and the mu_tol stop rule between
 * consecutive observations.  Returns 0, 1 (mu_tol > 0 and not converged) or
 * negative on bad input. */
int ors_run(const ors_problem *pb, double *psi, long nsteps, long first_step, int observe_every,
            double mu_tol, double *trace, long trace_cap, long *trace_rows, long *steps_done)
{
    if (ors_check(pb) || nsteps < 0 || observe_every < 0) return -1;
    double complex *c = ors_load(pb, psi);
    if (!c) return -2;
    long rows = 0, done = 0;
    int have_prev = 0, converged = 0;
    double prev_mu = 0.0, obs[12];
    for (long t = 0; t < nsteps; ++t) {
        long step = first_step + t;
        if (ors_step(pb, c, step)) {
            free(c);
            return -2;
        }
        done = t + 1;
        int observe_now = (observe_every > 0 && step % observe_every == 0) || (t == nsteps - 1);
        if (!observe_now) continue;
        ors_observe_c(pb, c, obs);
        if (trace && rows < trace_cap) {
            double *row = trace + 13 * rows;
            row[0] = (double)step;
            for (int q = 0; q < 12; ++q) row[1 + q] = obs[q];
            ++rows;
        }
        if (mu_tol > 0.0 && observe_every > 0 && step % observe_every == 0) {
            if (have_prev && fabs(obs[1] - prev_mu) < mu_tol) {
                converged = 1;
                break;
            }
            prev_mu = obs[1];
            have_prev = 1;
        }
    }
    ors_store(pb, c, psi);
    free(c);
    if (trace_rows) *trace_rows = rows;
    if (steps_done) *steps_done = done;
    if (mu_tol > 0.0 && !converged) return 1;
    return 0;
}

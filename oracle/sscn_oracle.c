/*
 * sscn_oracle.c -- plain FP64 CPU oracle for split-step Crank-Nicolson (SSCN)
 * propagation of the Gross-Pitaevskii (GP) equation in a 1D/2D/3D
 * anisotropic harmonic trap.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path loads this file:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header, table or helper with the GPU library; the
 * two meet only through seeded input arrays built by a separate module.
 *
 * What is computed.  The paper ("Nature of problem" and "Solution method" of
 * the program summary) solves the time-dependent GP equation for a condensate
 * with contact interaction in a harmonic trap by the split-step Crank-Nicolson
 * method, discretised in space and time, propagated over small steps in
 * imaginary time (stationary states) or real time (dynamics).  It prints no
 * formula for the scheme, so this file states the standard dimensionless form
 *
 *     i dpsi/dt = [ -1/2 Lap + V + g |psi|^2 ] psi,
 *     V = (w_x^2 x^2 + w_y^2 y^2 + w_z^2 z^2) / 2,
 *
 * and one SSCN step of length dt in the following order (Lie splitting):
 *
 *   1. pointwise substep (potential + nonlinearity, explicit |psi|^2):
 *        imaginary time:  psi <- exp(-dt (V + g|psi|^2)) psi
 *        real time:       psi <- exp(-i dt (V + g|psi|^2)) psi
 *   2. for each axis a = x, y, z (axes below dim only), for every line along
 *      a, one Crank-Nicolson kinetic substep with the 3-point Laplacian and
 *      psi = 0 on the virtual points just outside the grid:
 *        (1 + s T) v = (1 - s T) u,   T = tridiag(-1, 2, -1),
 *        s = dt / (4 dx_a^2)          in imaginary time,
 *        s = i dt / (4 dx_a^2)        in real time,
 *      solved by the Thomas algorithm without pivoting (the matrix is
 *      strictly diagonally dominant for both kinds of s).
 *   3. imaginary time only: renormalise psi to unit norm dV * sum |psi|^2.
 *
 * Grid: n_a stored unknowns per axis at x_a(i) = (i - (n_a - 1)/2) dx_a.
 * Layout: x fastest, p = i + n_x (j + n_y k); psi is stored as interleaved
 * (re, im) doubles in both modes (imaginary-time states carry im = 0).
 *
 * Observables: with forward differences that include the two edges to the
 * zero ghost points of every line,
 *   K = 1/2 dV sum_a sum_edges |psi_{p+e_a} - psi_p|^2 / dx_a^2,
 *   P = dV sum V |psi|^2,  I = dV sum |psi|^4,  N = dV sum |psi|^2,
 *   E = (K + P + g I / 2) / N,   mu = (K + P + g I) / N.
 * K equals <psi, -1/2 Lap_h psi> exactly (summation by parts), so these are
 * the energy functional and chemical potential of the discrete Hamiltonian
 * that the propagator uses.
 *
 * The outer loops over lines are OpenMP-parallel only so that the CPU
 * baseline uses the host's cores; each line is a serial, textbook solve.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_IMAG 0
#define ORC_REAL 1

/* Problem description, private to the oracle (mirrored by its ctypes
 * binding).  Unused axes have n = 1. */
typedef struct {
    int dim;
    int n[3];
    double dx[3];
    double omega[3];
    double g;
    double dt;
    int mode;          /* ORC_IMAG or ORC_REAL */
    int renorm_every;  /* imaginary time: renormalise every this many steps */
} orc_problem;

static long orc_points(const orc_problem *pb)
{
    return (long)pb->n[0] * pb->n[1] * pb->n[2];
}

static double orc_dvol(const orc_problem *pb)
{
    double dv = 1.0;
    for (int a = 0; a < pb->dim; ++a) dv *= pb->dx[a];
    return dv;
}

/* Coordinate of grid index i on axis a (grid centred on the trap). */
static double orc_coord(const orc_problem *pb, int a, int i)
{
    return (i - 0.5 * (pb->n[a] - 1)) * pb->dx[a];
}

/* Trap potential at grid point (i, j, k); axes at or above dim contribute
 * nothing. */
static double orc_potential_at(const orc_problem *pb, int i, int j, int k)
{
    int idx[3] = {i, j, k};
    double v = 0.0;
    for (int a = 0; a < pb->dim; ++a) {
        double x = orc_coord(pb, a, idx[a]);
        v += 0.5 * pb->omega[a] * pb->omega[a] * x * x;
    }
    return v;
}

/* ------------------------------------------------------------------ */
/* Tridiagonal pieces                                                  */
/* ------------------------------------------------------------------ */

/* Thomas algorithm for tridiag(-s, 1 + 2s, -s) x = r on n unknowns.
 * cp and dp are caller scratch of length n. */
static void orc_thomas_c(int n, double complex s, const double complex *r,
                         double complex *x, double complex *cp,
                         double complex *dp)
{
    const double complex lo = -s, di = 1.0 + 2.0 * s, up = -s;
    cp[0] = up / di;
    dp[0] = r[0] / di;
    for (int i = 1; i < n; ++i) {
        double complex den = di - lo * cp[i - 1];
        cp[i] = up / den;
        dp[i] = (r[i] - lo * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
}

/* One Crank-Nicolson kinetic substep on a single line u[0..n-1]:
 * r = (1 - sT) u with zero ghosts, then (1 + sT) v = r.  v may alias u.
 * w is scratch of length 4n. */
static void orc_cn_line_c(int n, double complex s, const double complex *u,
                          double complex *v, double complex *w)
{
    double complex *r = w, *cp = w + n, *dp = w + 2 * n, *x = w + 3 * n;
    for (int i = 0; i < n; ++i) {
        double complex left = (i > 0) ? u[i - 1] : 0.0;
        double complex right = (i < n - 1) ? u[i + 1] : 0.0;
        r[i] = (1.0 - 2.0 * s) * u[i] + s * (left + right);
    }
    orc_thomas_c(n, s, r, x, cp, dp);
    for (int i = 0; i < n; ++i) v[i] = x[i];
}

/* Exported for the Thomas and line-sweep pins: interleaved complex arrays. */
int orc_thomas(int n, double s_re, double s_im, const double *rhs, double *x)
{
    if (n < 1) return -1;
    double complex s = s_re + I * s_im;
    double complex *w = malloc(sizeof(double complex) * 4 * (size_t)n);
    if (!w) return -2;
    double complex *r = w, *cp = w + n, *dp = w + 2 * n, *xx = w + 3 * n;
    for (int i = 0; i < n; ++i) r[i] = rhs[2 * i] + I * rhs[2 * i + 1];
    orc_thomas_c(n, s, r, xx, cp, dp);
    for (int i = 0; i < n; ++i) {
        x[2 * i] = creal(xx[i]);
        x[2 * i + 1] = cimag(xx[i]);
    }
    free(w);
    return 0;
}

int orc_cn_line(int n, double s_re, double s_im, const double *u, double *v)
{
    if (n < 1) return -1;
    double complex s = s_re + I * s_im;
    double complex *buf = malloc(sizeof(double complex) * 5 * (size_t)n);
    if (!buf) return -2;
    double complex *uu = buf + 4 * n;
    for (int i = 0; i < n; ++i) uu[i] = u[2 * i] + I * u[2 * i + 1];
    orc_cn_line_c(n, s, uu, uu, buf);
    for (int i = 0; i < n; ++i) {
        v[2 * i] = creal(uu[i]);
        v[2 * i + 1] = cimag(uu[i]);
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------ */
/* The SSCN step                                                       */
/* ------------------------------------------------------------------ */

static int orc_check(const orc_problem *pb)
{
    if (pb->dim < 1 || pb->dim > 3) return -1;
    for (int a = 0; a < 3; ++a) {
        if (pb->n[a] < 1) return -1;
        if (a >= pb->dim && pb->n[a] != 1) return -1;
        if (a < pb->dim && !(pb->dx[a] > 0.0)) return -1;
    }
    if (!(pb->dt > 0.0)) return -1;
    if (pb->mode != ORC_IMAG && pb->mode != ORC_REAL) return -1;
    return 0;
}

/* Step 1: the pointwise potential + nonlinear substep. */
static void orc_pointwise(const orc_problem *pb, double complex *psi)
{
    const int nx = pb->n[0], ny = pb->n[1], nz = pb->n[2];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = i + (long)nx * (j + (long)ny * k);
                double q = creal(psi[p]) * creal(psi[p]) +
                           cimag(psi[p]) * cimag(psi[p]);
                double phi = pb->dt * (orc_potential_at(pb, i, j, k) + pb->g * q);
                if (pb->mode == ORC_IMAG)
                    psi[p] = exp(-phi) * psi[p];
                else
                    psi[p] = (cos(phi) - I * sin(phi)) * psi[p];
            }
}

/* Step 2: one CN substep on every line along axis a. */
static void orc_sweep(const orc_problem *pb, double complex *psi, int a)
{
    const int n[3] = {pb->n[0], pb->n[1], pb->n[2]};
    const long stride[3] = {1, n[0], (long)n[0] * n[1]};
    const int m = n[a];
    double complex s = pb->dt / (4.0 * pb->dx[a] * pb->dx[a]);
    if (pb->mode == ORC_REAL) s = I * s;
    /* the two axes other than a enumerate the lines */
    const int b = (a == 0) ? 1 : 0;
    const int c = (a == 2) ? 1 : 2;
    const long nlines = (long)n[b] * n[c];
#pragma omp parallel
    {
        double complex *line = malloc(sizeof(double complex) * 5 * (size_t)m);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; ++l) {
            long ib = l % n[b], ic = l / n[b];
            long base = ib * stride[b] + ic * stride[c];
            double complex *u = line + 4 * m;
            for (int i = 0; i < m; ++i) u[i] = psi[base + i * stride[a]];
            orc_cn_line_c(m, s, u, u, line);
            for (int i = 0; i < m; ++i) psi[base + i * stride[a]] = u[i];
        }
        free(line);
    }
}

/* dV * sum |psi|^2 */
static double orc_norm_c(const orc_problem *pb, const double complex *psi)
{
    long np = orc_points(pb);
    double acc = 0.0;
    for (long p = 0; p < np; ++p)
        acc += creal(psi[p]) * creal(psi[p]) + cimag(psi[p]) * cimag(psi[p]);
    return acc * orc_dvol(pb);
}

/* One full SSCN step; step_index counts from 1 and selects renormalisation. */
static void orc_step_c(const orc_problem *pb, double complex *psi, long step_index)
{
    orc_pointwise(pb, psi);
    for (int a = 0; a < pb->dim; ++a) orc_sweep(pb, psi, a);
    if (pb->mode == ORC_IMAG && pb->renorm_every > 0 &&
        step_index % pb->renorm_every == 0) {
        double nrm = orc_norm_c(pb, psi);
        double scale = 1.0 / sqrt(nrm);
        long np = orc_points(pb);
        for (long p = 0; p < np; ++p) psi[p] *= scale;
    }
}

/* ------------------------------------------------------------------ */
/* Observables                                                         */
/* ------------------------------------------------------------------ */

/* out[0..11] = norm, mu, energy, K, P, I, <x>, <y>, <z>, <x^2>, <y^2>, <z^2>
 * (K, P, I are the raw integrals; the moments are divided by the norm). */
static void orc_observe_c(const orc_problem *pb, const double complex *psi,
                          double *out)
{
    const int nx = pb->n[0], ny = pb->n[1], nz = pb->n[2];
    const int n[3] = {nx, ny, nz};
    const long stride[3] = {1, nx, (long)nx * ny};
    double sum2 = 0, sumk = 0, sump = 0, sum4 = 0;
    double m1[3] = {0, 0, 0}, m2[3] = {0, 0, 0};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int idx[3] = {i, j, k};
                long p = i + (long)nx * (j + (long)ny * k);
                double complex v = psi[p];
                double q = creal(v) * creal(v) + cimag(v) * cimag(v);
                sum2 += q;
                sum4 += q * q;
                sump += orc_potential_at(pb, i, j, k) * q;
                for (int a = 0; a < pb->dim; ++a) {
                    double xa = orc_coord(pb, a, idx[a]);
                    m1[a] += xa * q;
                    m2[a] += xa * xa * q;
                    /* forward edge p -> p + e_a (ghost zero past the end) */
                    double complex nb = (idx[a] + 1 < n[a]) ? psi[p + stride[a]] : 0.0;
                    double complex d = nb - v;
                    double e = (creal(d) * creal(d) + cimag(d) * cimag(d)) /
                               (pb->dx[a] * pb->dx[a]);
                    /* the edge from the ghost below the first point */
                    if (idx[a] == 0) e += q / (pb->dx[a] * pb->dx[a]);
                    sumk += e;
                }
            }
    double dv = orc_dvol(pb);
    double N = dv * sum2, K = 0.5 * dv * sumk, P = dv * sump, In = dv * sum4;
    out[0] = N;
    out[1] = (K + P + pb->g * In) / N;
    out[2] = (K + P + 0.5 * pb->g * In) / N;
    out[3] = K;
    out[4] = P;
    out[5] = In;
    for (int a = 0; a < 3; ++a) {
        out[6 + a] = dv * m1[a] / N;
        out[9 + a] = dv * m2[a] / N;
    }
}

/* ------------------------------------------------------------------ */
/* Exported entry points (interleaved complex psi, length 2 * points)  */
/* ------------------------------------------------------------------ */

static double complex *orc_load(const orc_problem *pb, const double *psi)
{
    long np = orc_points(pb);
    double complex *c = malloc(sizeof(double complex) * (size_t)np);
    if (!c) return NULL;
    for (long p = 0; p < np; ++p) c[p] = psi[2 * p] + I * psi[2 * p + 1];
    return c;
}

static void orc_store(const orc_problem *pb, const double complex *c, double *psi)
{
    long np = orc_points(pb);
    for (long p = 0; p < np; ++p) {
        psi[2 * p] = creal(c[p]);
        psi[2 * p + 1] = cimag(c[p]);
    }
}

int orc_observe(const orc_problem *pb, const double *psi, double *out)
{
    if (orc_check(pb)) return -1;
    double complex *c = orc_load(pb, psi);
    if (!c) return -2;
    orc_observe_c(pb, c, out);
    free(c);
    return 0;
}

/* Fill V on the grid (length = points), for tests. */
int orc_potential(const orc_problem *pb, double *v)
{
    if (orc_check(pb)) return -1;
    for (int k = 0; k < pb->n[2]; ++k)
        for (int j = 0; j < pb->n[1]; ++j)
            for (int i = 0; i < pb->n[0]; ++i)
                v[i + (long)pb->n[0] * (j + (long)pb->n[1] * k)] =
                    orc_potential_at(pb, i, j, k);
    return 0;
}

/* Only the pointwise substep, or only the sweep along one axis (for pins). */
int orc_substep(const orc_problem *pb, double *psi, int which)
{
    if (orc_check(pb)) return -1;
    if (which < -1 || which >= pb->dim) return -1;
    double complex *c = orc_load(pb, psi);
    if (!c) return -2;
    if (which < 0) orc_pointwise(pb, c);
    else orc_sweep(pb, c, which);
    orc_store(pb, c, psi);
    free(c);
    return 0;
}

/*
 * Run nsteps SSCN steps from psi (updated in place).  Step numbering starts
 * at first_step (so a run can be continued).  Every observe_every steps, and
 * after the last step, a row {step, norm, mu, E, K, P, I, <x>, <y>, <z>,
 * <x^2>, <y^2>, <z^2>} (13 doubles) is appended to trace while room is left.
 *
 * If mu_tol > 0 the run stops at the first observation step s at which
 * |mu(s) - mu(s - observe_every)| < mu_tol (a chemical-potential convergence
 * test between consecutive observations); *steps_done reports the step count.
 * Returns 0 when stopped by convergence or when mu_tol <= 0, 1 when mu_tol > 0
 * and nsteps ran out first, negative on bad input.
 */
int orc_run(const orc_problem *pb, double *psi, long nsteps, long first_step,
            int observe_every, double mu_tol, double *trace, long trace_cap,
            long *trace_rows, long *steps_done)
{
    if (orc_check(pb) || nsteps < 0 || observe_every < 0) return -1;
    double complex *c = orc_load(pb, psi);
    if (!c) return -2;
    long rows = 0, done = 0;
    int have_prev = 0, converged = 0;
    double prev_mu = 0.0;
    double obs[12];
    for (long t = 0; t < nsteps; ++t) {
        long step = first_step + t;
        orc_step_c(pb, c, step);
        done = t + 1;
        int observe_now = (observe_every > 0 && step % observe_every == 0) ||
                          (t == nsteps - 1);
        if (!observe_now) continue;
        orc_observe_c(pb, c, obs);
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
    orc_store(pb, c, psi);
    free(c);
    if (trace_rows) *trace_rows = rows;
    if (steps_done) *steps_done = done;
    if (mu_tol > 0.0 && !converged) return 1;
    return 0;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel regions (the CPU baseline times one core
 * and all cores); n < 1 is rejected. */
int orc_set_threads(int n)
{
    if (n < 1) return -1;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return 0;
}

/* Integrated densities (the paper's n_1D and n_2D outputs): integrate
 * |psi|^2 dV over every axis except `keep` (out has n[keep] entries), or over
 * the single axis `drop` (out has the points of the remaining two axes in
 * layout order). */
int orc_density_1d(const orc_problem *pb, const double *psi, int keep, double *out)
{
    if (orc_check(pb) || keep < 0 || keep >= pb->dim) return -1;
    const int n[3] = {pb->n[0], pb->n[1], pb->n[2]};
    double w = orc_dvol(pb) / pb->dx[keep];
    for (int i = 0; i < n[keep]; ++i) out[i] = 0.0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int idx[3] = {i, j, k};
                long p = i + (long)n[0] * (j + (long)n[1] * k);
                double q = psi[2 * p] * psi[2 * p] + psi[2 * p + 1] * psi[2 * p + 1];
                out[idx[keep]] += w * q;
            }
    return 0;
}

int orc_density_2d(const orc_problem *pb, const double *psi, int drop, double *out)
{
    if (orc_check(pb) || pb->dim != 3 || drop < 0 || drop > 2) return -1;
    const int n[3] = {pb->n[0], pb->n[1], pb->n[2]};
    const int u = (drop == 0) ? 1 : 0, v = (drop == 2) ? 1 : 2;
    double w = pb->dx[drop];
    for (long q = 0; q < (long)n[u] * n[v]; ++q) out[q] = 0.0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int idx[3] = {i, j, k};
                long p = i + (long)n[0] * (j + (long)n[1] * k);
                double q = psi[2 * p] * psi[2 * p] + psi[2 * p + 1] * psi[2 * p + 1];
                out[idx[u] + (long)n[u] * idx[v]] += w * q;
            }
    return 0;
}

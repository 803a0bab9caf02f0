// sscn_kernels.hip -- gfx950 kernels of one SSCN step and its reductions.
//
// Per step (the paper's split-step Crank-Nicolson propagation; equations in
// sscn.h):
//   k_row   x lines: pending renormalisation scale + pointwise potential and
//           nonlinear substep fused into the load, then the CN x solve
//           (ROW geometry, see sscn_dev.hpp).  One read and one write of psi.
//   k_col   y and z lines (COL geometry); the last sweep of the step also
//           emits one FP64 partial of sum |psi|^2 per block.
//   k_norm_final  fixed-order sum of those partials -> renormalisation
//           factor kept on the device and applied by the next k_row load.
//           With few partials (small grids) the next step's k_row forms the
//           factor itself, bitwise alike, and k_norm_final only ends a run
//           of steps: one launch less per step.
// Fallbacks for lines too long to keep in registers: k_pointwise (separate
// pointwise substep), k_stream (one thread per line, exact Thomas with the
// forward intermediates stored in place) and k_norm_partials.
#include <hip/hip_ext.h>

#include "sscn_lines.hpp"

namespace sscn {

// ===========================================================================
// ROW: x lines, G = 64 * wpl threads per line, C points per thread.
// Single-wave lines (MW = false) stage the lane-major table (C * G entries)
// in LDS; multi-wave lines (MW = true, long 1D lines) read it from global
// memory and exchange 4 values per wave through LDS.  SEG < 64: lines of at
// most SEG * C points, G = SEG lanes each, 64/SEG lines per wave.
// ===========================================================================
template <class T, bool CPLX, int C, bool LAST, bool MW, int SEG = 64>
__global__ void __launch_bounds__(MW ? 1024 : 256) k_row(RowArgs a)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    extern __shared__ unsigned char lds_raw[];
    __shared__ double red[16];

    const int G = MW ? 64 * a.wpl : SEG;
    const int tid = threadIdx.x;
    const int lb = tid / G;
    const int t = tid - lb * G;
    const int lane = tid & 63;
    const int wl = t >> 6;
    LTab<T, CPLX> *tl = reinterpret_cast<LTab<T, CPLX> *>(lds_raw);
    V *xs = reinterpret_cast<V *>(lds_raw) + lb * a.wpl * 4;
    const V sig = A::coef(a.sig_re, a.sig_im);
    // the pending renormalisation factor: from memory, or (short lines of
    // small grids) formed from the previous step's norm partials once this
    // wave's first line is loaded (their loads overlap the line's)
    T scale = T(1);
    double fp[kFoldWaves];
    bool need = false;
    if constexpr (!CPLX) {
        if (SEG < 64 && a.fold) {
#pragma unroll
            for (int w = 0; w < kFoldWaves; ++w)
                fp[w] = (w * 64 + lane < a.fold_np) ? a.fold[w * 64 + lane] : 0.0;
            need = true;
        } else {
            scale = T(*a.scale);
        }
    }
    const T dt = T(a.pp.dt), g = T(a.pp.g);
    V *psi = reinterpret_cast<V *>(a.psi);
    double nacc = 0.0;

    // single-wave lines move their values through a per-wave LDS buffer
    // after the table (row_load_tr), so every global access is coalesced,
    // when table and buffers fit 64 KB (the host sizes the LDS alike)
    constexpr bool TR = SEG == 64 && sizeof(V) >= 16 &&
                        (size_t)C * 64 * sizeof(LTab<T, CPLX>) + 4 * ((size_t)C * 64 + 64) * sizeof(V) <= 65536;
    V *buf = reinterpret_cast<V *>(tl + C * G) + lb * (C * 64 + 64);
    // 4- and 8-byte values move as 16-byte groups where the line length and
    // the state's alignment allow (a.v16)
    constexpr bool V16 = sizeof(V) <= 8 && C % (16 / sizeof(V)) == 0;
    const long long gstep = (long long)gridDim.x * a.lpb;
    if constexpr (MW) {
        for (long long gb = (long long)blockIdx.x * a.lpb; gb < a.nlines; gb += gstep) {
            const long long line = gb + lb;
            if (need) {
                scale = T(fold_scale(fp, a.fold_np, a.fold_dvol));
                need = false;
            }
            nacc += row_line<T, CPLX, C, true>(psi, line, line < a.nlines, a.lt.n, a.lt.tab, G, t, lane, wl, a.wpl,
                                               xs, sig, scale, dt, g, a.pp, a.lt.depth, LAST);
        }
    } else {
        auto load = [&](long long line, bool active, V (&u)[C]) {
            if constexpr (V16) {
                if (a.v16) row_load_v16<T, CPLX, C>(psi, line, active, a.lt.n, t, u);
                else row_load<T, CPLX, C>(psi, line, active, a.lt.n, t, u);
            } else if constexpr (TR) {
                row_load_tr<T, CPLX, C>(psi, line, active, a.lt.n, lane, buf, u);
            } else {
                row_load<T, CPLX, C>(psi, line, active, a.lt.n, t, u);
            }
        };
        // short lines (small grids: a block has one line group): the first
        // line's values are loaded before the table is staged, so that the
        // two memory latencies overlap.  Longer lines keep a plain loop (the
        // early load measured slower there)
        const long long gb0 = (long long)blockIdx.x * a.lpb;
        V u[C];
        bool loaded = false;
        if constexpr (SEG < 64) {
            if (gb0 < a.nlines) {
                load(gb0 + lb, gb0 + lb < a.nlines, u);
                loaded = true;
            }
        }
        stage_table<T, CPLX>(a.lt, tl, C * G, G, C);
        __syncthreads();
        for (long long gb = gb0; gb < a.nlines; gb += gstep) {
            const long long line = gb + lb;
            const bool active = line < a.nlines;
            if constexpr (SEG < 64) {
                if (!loaded) load(line, active, u);
                loaded = false;
            } else {
                load(line, active, u);
            }
            if (need) {
                scale = T(fold_scale(fp, a.fold_np, a.fold_dvol));
                need = false;
            }
            const LTab<T, CPLX> *tc = tl;
            if constexpr (V16) {
                nacc += row_solve<T, CPLX, C, false, true, SEG>(psi, line, active, a.lt.n, tc, G, t, lane, wl, 1, xs, sig,
                                                     scale, dt, g, a.pp, a.lt.depth, LAST, u, true);
                if (a.v16) row_store_v16<T, CPLX, C>(psi, line, active, a.lt.n, t, u);
                else row_store<T, CPLX, C>(psi, line, active, a.lt.n, t, u);
            } else if constexpr (TR) {
                nacc += row_solve<T, CPLX, C, false, true, SEG>(psi, line, active, a.lt.n, tc, G, t, lane, wl, 1, xs, sig,
                                                     scale, dt, g, a.pp, a.lt.depth, LAST, u, true);
                row_store_tr<T, CPLX, C>(psi, line, active, a.lt.n, lane, buf, u);
            } else {
                nacc += row_solve<T, CPLX, C, false, true, SEG>(psi, line, active, a.lt.n, tc, G, t, lane, wl, 1, xs, sig,
                                                     scale, dt, g, a.pp, a.lt.depth, LAST, u);
            }
        }
    }
    if constexpr (LAST) {
        const double s = block_sum(nacc, red);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
    }
}

// ===========================================================================
// COL: 64/L lines per block, W*L chunks of C points per line.  LDS: the
// table (W*L*C entries), then two chunk x line exchange arrays.
// ===========================================================================
template <class T, bool CPLX, int C, bool LAST>
__global__ void __launch_bounds__(1024) k_col(ColArgs a)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    extern __shared__ unsigned char lds_raw[];
    __shared__ double red[16];
    const int L = a.L;
    const int LPB = 64 / L;
    const int nch = a.W * L;
    LTab<T, CPLX> *tb = reinterpret_cast<LTab<T, CPLX> *>(lds_raw);
    V *xs0 = reinterpret_cast<V *>(tb + nch * C);
    V *xs1 = xs0 + nch * LPB;

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int sub = lane / LPB;
    const int li = lane - sub * LPB;
    const int ch = w * L + sub;
    const long long line = (long long)blockIdx.x * LPB + li;
    const bool active = line < a.nlines;
    long long base = 0;
    if (active) base = (line % a.m1) * a.s1 + (line / a.m1) * a.s2;
    // the values are loaded before the table is staged, so that the two
    // memory latencies overlap; col_solve synchronises the block before it
    // reads the table
    V u[C];
    col_load<T, CPLX, C>(reinterpret_cast<V *>(a.psi), active, base, a.lt.n, a.stride, ch, u);
    stage_table<T, CPLX>(a.lt, tb, nch * C, 0, C);
    double nacc = col_solve<T, CPLX, C>(reinterpret_cast<V *>(a.psi), active, base, a.lt.n, a.stride, nch, ch, LPB,
                                        li, tb, xs0, xs1, A::coef(a.sig_re, a.sig_im), a.lt.depth, LAST, u);
    if (a.unit_scale && blockIdx.x == 0 && threadIdx.x == 0) *a.unit_scale = 1.0;
    if constexpr (LAST) {
        // the axial trap weighs each z line by its radial cell weight
        if (a.wline && active) nacc *= a.wline[line % a.m1];
        const double s = block_sum(nacc, red);
        if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
    }
}

// ===========================================================================
// Fallbacks
// ===========================================================================
template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_stream(ColArgs a)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= a.nlines) return;
    const long long base = (line % a.m1) * a.s1 + (line / a.m1) * a.s2;
    V *p = reinterpret_cast<V *>(a.psi) + base;
    const long long st = a.stride;
    const int n = a.lt.n;
    const V sig = A::coef(a.sig_re, a.sig_im);
    // forward: d_i stored in place of psi_i; the original u_{i-1}, u_i kept
    V um = A::zero(), u0 = p[0];
    V d = A::zero();
    for (int i = 0; i < n; ++i) {
        const V up = (i + 1 < n) ? p[(long long)(i + 1) * st] : A::zero();
        const V r = cn_rhs<T, CPLX>(um, u0, up, sig);
        const LTab<T, CPLX> e = tab_at<T, CPLX>(a.lt.tab, i);
        d = e.afma(d, e.mmul(r));
        p[(long long)i * st] = d;
        um = u0;
        u0 = up;
    }
    V v = A::zero();
    for (int i = n - 1; i >= 0; --i) {
        v = tab_at<T, CPLX>(a.lt.tab, i).afma(v, p[(long long)i * st]);
        p[(long long)i * st] = v;
    }
}

template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_pointwise(PointArgs a)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    V *psi = reinterpret_cast<V *>(a.psi);
    const T scale = CPLX ? T(1) : T(*a.scale);
    const T dt = T(a.pp.dt), g = T(a.pp.g);
    const long long nx = a.pp.n[0], ny = a.pp.n[1];
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < a.npts;
         p += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(p % nx);
        const int j = (int)((p / nx) % ny);
        const int k = (int)(p / (nx * ny));
        const T x = coord<T>(i, a.pp.cen[0], a.pp.dx[0]);
        const T y = coord<T>(j, a.pp.cen[1], a.pp.dx[1]);
        const T z = coord<T>(k, a.pp.cen[2], a.pp.dx[2]);
        // the potential rounded as in the x sweep (row_solve)
        const T vp = fmaT(T(a.pp.w2h[0]) * x, x, fmaT(T(a.pp.w2h[2]) * z, z, T(a.pp.w2h[1]) * y * y));
        psi[p] = apply_point<T, CPLX>(psi[p], scale, vp, dt, g);
    }
}

template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_norm_partials(const void *psi_, long long npts, double *partial)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    __shared__ double red[16];
    const V *psi = reinterpret_cast<const V *>(psi_);
    double acc = 0.0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
         p += (long long)gridDim.x * blockDim.x)
        acc += A::norm2(psi[p]);
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// scalars[0] = pending scale, scalars[1] = last norm
__global__ void __launch_bounds__(1024) k_norm_final(const double *partial, int np, double dvol,
                                                     int do_renorm, double *scalars)
{
    __shared__ double red[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) {
        if (do_renorm) {
            const double N = dvol * s;
            scalars[1] = N;
            scalars[0] = 1.0 / sqrt(N);
        } else {
            scalars[0] = 1.0;
        }
    }
}

template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_scale_state(void *psi_, long long npts, const double *scalars)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    V *psi = reinterpret_cast<V *>(psi_);
    const T s = T(scalars[0]);
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
         p += (long long)gridDim.x * blockDim.x)
        psi[p] = A::scal(s, psi[p]);
}

__global__ void k_set_unit_scale(double *scalars)
{
    if (threadIdx.x == 0) scalars[0] = 1.0;
}

// ===========================================================================
// Observables
// ===========================================================================
#define SSCN_NOBS 12

template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_obs_partials(ObsArgs a)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    __shared__ double red[SSCN_NOBS][4];
    const V *psi = reinterpret_cast<const V *>(a.psi);
    const long long nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const long long sx[3] = {1, nx, nx * ny};
    double acc[SSCN_NOBS];
#pragma unroll
    for (int q = 0; q < SSCN_NOBS; ++q) acc[q] = 0.0;
    double inv2[3];                       // 1 / dx_a^2
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) inv2[ax] = ax < a.dim ? 1.0 / (a.dx[ax] * a.dx[ax]) : 0.0;
    // acc: 0 sum q, 1 sum kinetic edges, 2 sum V q, 3 sum q^2, 4..6 x_a q, 7..9 x_a^2 q
    // The grid indices of this thread's first point come from two
    // divisions; after that each grid-stride step adds the stride's own
    // decomposition with carries (no division per point).
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int idx[3] = {(int)(p % nx), (int)((p / nx) % ny), (int)(p / (nx * ny))};
    // a state whose renormalisation is still pending: every value is taken
    // times the factor, as the pass that applies it would store it
    const bool scaled = !CPLX && a.scale != nullptr;
    const T sc = scaled ? T(*a.scale) : T(1);
    const int di = (int)(stride % nx), dj = (int)((stride / nx) % ny), dk = (int)(stride / (nx * ny));
    (void)nz;
    // U grid-stride points per pass: all their loads (the point and its
    // three forward neighbours) are issued before any is used, so a pass
    // waits for memory once; the sums take the points in the same order as
    // one point per pass
    constexpr int U = 4;
    for (; p < a.npts; p += U * stride) {
        V v[U], nb[U][3];
        int id[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) id[u][ax] = idx[ax];
            int c = 0;
            idx[0] += di;
            if (idx[0] >= a.n[0]) {
                idx[0] -= a.n[0];
                c = 1;
            }
            idx[1] += dj + c;
            c = 0;
            if (idx[1] >= a.n[1]) {
                idx[1] -= a.n[1];
                c = 1;
            }
            idx[2] += dk + c;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long pu = p + (long long)u * stride;
            const bool in = pu < a.npts;
            v[u] = in ? psi[pu] : A::zero();
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                nb[u][ax] = (in && ax < a.dim && id[u][ax] + 1 < a.n[ax]) ? psi[pu + sx[ax]] : A::zero();
            if (scaled) {
                v[u] = A::scal(sc, v[u]);
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) nb[u][ax] = A::scal(sc, nb[u][ax]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + (long long)u * stride >= a.npts) break;
            const double q = A::norm2(v[u]);
            double vp = 0.0, kin = 0.0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                if (ax >= a.dim) break;
                const double x = (double(id[u][ax]) - a.cen[ax]) * a.dx[ax];
                vp = fmaT(a.w2h[ax] * x, x, vp);
                acc[4 + ax] = fmaT(x, q, acc[4 + ax]);
                acc[7 + ax] = fmaT(x * x, q, acc[7 + ax]);
                double e = A::norm2(A::sub(nb[u][ax], v[u]));
                if (id[u][ax] == 0) e += q;
                kin = fmaT(e, inv2[ax], kin);
            }
            acc[0] += q;
            acc[1] += kin;
            acc[2] = fmaT(vp, q, acc[2]);
            acc[3] = fmaT(q, q, acc[3]);
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < SSCN_NOBS - 2; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < SSCN_NOBS - 2) {
        const int q = threadIdx.x;
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[q][w];
        a.partial[(size_t)blockIdx.x * SSCN_NOBS + q] = s;
    }
}

__global__ void __launch_bounds__(256) k_obs_final(const double *partial, int np, double dvol,
                                                   double g, double *out)
{
    constexpr int NQ = SSCN_NOBS - 2;
    __shared__ double red[16][NQ];
    // every quantity in one pass over the partial rows, then one barrier;
    // the order of each sum is that of a block_sum per quantity
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const double *row = partial + (size_t)i * SSCN_NOBS;
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += row[q];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[wid][q] = v;
    }
    __syncthreads();
    double tot[NQ];
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int q = 0; q < NQ; ++q) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[w][q];
            tot[q] = s;
        }
    }
    if (threadIdx.x == 0) {
        const double N = dvol * tot[0];
        const double K = 0.5 * dvol * tot[1];
        const double P = dvol * tot[2];
        const double I = dvol * tot[3];
        out[0] = N;
        out[1] = fmaT(g, I, K + P) / N;
        out[2] = fmaT(0.5 * g, I, K + P) / N;
        out[3] = K;
        out[4] = P;
        out[5] = I;
        for (int ax = 0; ax < 3; ++ax) {
            out[6 + ax] = dvol * tot[4 + ax] / N;
            out[9 + ax] = dvol * tot[7 + ax] / N;
        }
        out[12] = (__builtin_isfinite(out[0]) && __builtin_isfinite(out[1])) ? 1.0 : 0.0;
    }
}

// ===========================================================================
// Integrated densities
// ===========================================================================
template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_density_1d(const void *psi_, int nx, int ny, int nz,
                                                    int keep, double w, double *out)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    __shared__ double red[16];
    const V *psi = reinterpret_cast<const V *>(psi_);
    const int c = blockIdx.x;  // index along `keep`
    const long long n3[3] = {nx, ny, nz};
    const long long sx[3] = {1, nx, (long long)nx * ny};
    const int u = (keep == 0) ? 1 : 0, v = (keep == 2) ? 1 : 2;
    const long long cnt = n3[u] * n3[v];
    double acc = 0.0;
    for (long long q = threadIdx.x; q < cnt; q += blockDim.x) {
        const long long iu = q % n3[u], iv = q / n3[u];
        acc += A::norm2(psi[c * sx[keep] + iu * sx[u] + iv * sx[v]]);
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[c] = w * s;
}

// n_1D keeping x, pass 1: block b sums |psi|^2 over its contiguous range of
// rows (x lines) for each x, threads along x (coalesced), into
// part[b * nx + x]
template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_density_x_rows(const void *psi_, int nx, long long rows, double *part)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const V *psi = reinterpret_cast<const V *>(psi_);
    const long long r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        double acc = 0.0;
#pragma unroll 8
        for (long long r = r0; r < r1; ++r) acc += A::norm2(psi[r * nx + x]);
        part[(long long)blockIdx.x * nx + x] = acc;
    }
}

// Sums of |psi|^2 along x lines, one wave per line: out[r] = w * sum_x.
// These are n_2D without x (layout order of (y, z) is the line index) and
// the first pass of n_1D keeping y or z.
template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_density_rows(const void *psi_, int nx, long long rows, double w, double *out)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const long long r = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;  // a whole wave
    const V *row = reinterpret_cast<const V *>(psi_) + r * nx;
    double acc = 0.0;
#pragma unroll 4
    for (int x = lane; x < nx; x += 64) acc += A::norm2(row[x]);
    acc = wave_sum(acc);
    if (lane == 0) out[r] = w * acc;
}

// n_1D keeping y (keep = 1) or z (keep = 2) from the x-line sums rs
// (index j + ny k): one wave per output, lanes over the other axis.
__global__ void __launch_bounds__(256) k_density_rows_fin(const double *rs, int ny, int nz, int keep, double w,
                                                          double *out)
{
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nc = keep == 1 ? ny : nz, no = keep == 1 ? nz : ny;
    if (c >= nc) return;  // a whole wave
    double acc = 0.0;
    for (int o = lane; o < no; o += 64) acc += keep == 1 ? rs[c + (long long)ny * o] : rs[o + (long long)ny * c];
    acc = wave_sum(acc);
    if (lane == 0) out[c] = w * acc;
}

// pass 2: out[x] = w * sum_b part[b * nx + x].  A block covers 64 x; its 16
// waves take consecutive ranges of b and are added in wave order.
__global__ void __launch_bounds__(1024) k_density_x_fin(const double *part, int nx, int nb, double w, double *out)
{
    __shared__ double red[16][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (x < nx) {
        const int b0 = (int)((long long)nb * wv / 16), b1 = (int)((long long)nb * (wv + 1) / 16);
#pragma unroll 8
        for (int b = b0; b < b1; ++b) acc += part[(long long)b * nx + x];
    }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && x < nx) {
        double s = 0.0;
        for (int q = 0; q < 16; ++q) s += red[q][lane];
        out[x] = w * s;
    }
}

template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_density_2d(const void *psi_, int nx, int ny, int nz,
                                                    int drop, double w, double *out)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const V *psi = reinterpret_cast<const V *>(psi_);
    const long long n3[3] = {nx, ny, nz};
    const long long sx[3] = {1, nx, (long long)nx * ny};
    const int u = (drop == 0) ? 1 : 0, v = (drop == 2) ? 1 : 2;
    const long long cnt = n3[u] * n3[v];
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cnt) return;
    const long long iu = q % n3[u], iv = q / n3[u];
    // threads along x read coalesced rows; the unrolled loop keeps several
    // independent loads of the dropped axis in flight (sum order unchanged)
    const V *p0 = psi + iu * sx[u] + iv * sx[v];
    const long long sd = sx[drop];
    double acc = 0.0;
#pragma unroll 8
    for (long long k = 0; k < n3[drop]; ++k) acc += A::norm2(p0[k * sd]);
    out[q] = w * acc;
}

// ===========================================================================
// launchers
// ===========================================================================
#define SSCN_ELEM_DISPATCH(elem, MACRO)           \
    switch (elem) {                               \
    case 0: MACRO(double, false); break;          \
    case 1: MACRO(float, false); break;           \
    case 2: MACRO(double, true); break;           \
    case 3: MACRO(float, true); break;            \
    default: return hipErrorInvalidValue;         \
    }

// The sweep launches go through hipExtLaunchKernelGGL: with a start/stop
// event pair (timing runs) the events take the kernel's own begin and end
// times; with null events it is a plain launch.
template <class T, bool CPLX, int C>
static void row_launch_c(bool last, const RowArgs &a, int grid, int block, size_t lds, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1)
{
    const bool mw = a.wpl > 1;
    if constexpr (C == 4) {
        // lines of at most 64 points: 16 lanes each, four per wave
        if (a.seg == 16 && !mw) {
            if (last)
                hipExtLaunchKernelGGL((k_row<T, CPLX, C, true, false, 16>), dim3(grid), dim3(block), lds, st, e0, e1, 0,
                                      a);
            else
                hipExtLaunchKernelGGL((k_row<T, CPLX, C, false, false, 16>), dim3(grid), dim3(block), lds, st, e0, e1,
                                      0, a);
            return;
        }
    }
    if (last && mw)
        hipExtLaunchKernelGGL((k_row<T, CPLX, C, true, true>), dim3(grid), dim3(block), lds, st, e0, e1, 0, a);
    else if (last)
        hipExtLaunchKernelGGL((k_row<T, CPLX, C, true, false>), dim3(grid), dim3(block), lds, st, e0, e1, 0, a);
    else if (mw)
        hipExtLaunchKernelGGL((k_row<T, CPLX, C, false, true>), dim3(grid), dim3(block), lds, st, e0, e1, 0, a);
    else
        hipExtLaunchKernelGGL((k_row<T, CPLX, C, false, false>), dim3(grid), dim3(block), lds, st, e0, e1, 0, a);
}

template <class T, bool CPLX>
static hipError_t row_launch(int C, bool last, const RowArgs &a, int grid, int block, size_t lds,
                             hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    switch (C) {
    case 1: row_launch_c<T, CPLX, 1>(last, a, grid, block, lds, st, e0, e1); break;
    case 2: row_launch_c<T, CPLX, 2>(last, a, grid, block, lds, st, e0, e1); break;
    case 4: row_launch_c<T, CPLX, 4>(last, a, grid, block, lds, st, e0, e1); break;
    case 8: row_launch_c<T, CPLX, 8>(last, a, grid, block, lds, st, e0, e1); break;
    case 16:
        if constexpr (sizeof(typename Alg<T, CPLX>::V) <= 8) {
            row_launch_c<T, CPLX, 16>(last, a, grid, block, lds, st, e0, e1);
            break;
        }
        return hipErrorInvalidValue;
    case 32:
        if constexpr (sizeof(typename Alg<T, CPLX>::V) <= 4) {
            row_launch_c<T, CPLX, 32>(last, a, grid, block, lds, st, e0, e1);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_row(int elem, int C, bool last, const RowArgs &a, int grid, int block, size_t lds,
                      hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
#define ROW_CASE(T, CP) return row_launch<T, CP>(C, last, a, grid, block, lds, st, e0, e1)
    SSCN_ELEM_DISPATCH(elem, ROW_CASE)
#undef ROW_CASE
}

template <class T, bool CPLX, int C>
static void col_launch_c(bool last, const ColArgs &a, int grid, int block, size_t lds, hipStream_t st,
                         hipEvent_t e0, hipEvent_t e1)
{
    if (last) hipExtLaunchKernelGGL((k_col<T, CPLX, C, true>), dim3(grid), dim3(block), lds, st, e0, e1, 0, a);
    else hipExtLaunchKernelGGL((k_col<T, CPLX, C, false>), dim3(grid), dim3(block), lds, st, e0, e1, 0, a);
}

template <class T, bool CPLX>
static hipError_t col_launch(int C, bool last, const ColArgs &a, int grid, int block, size_t lds,
                             hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    switch (C) {
    case 1: col_launch_c<T, CPLX, 1>(last, a, grid, block, lds, st, e0, e1); break;
    case 2: col_launch_c<T, CPLX, 2>(last, a, grid, block, lds, st, e0, e1); break;
    case 4: col_launch_c<T, CPLX, 4>(last, a, grid, block, lds, st, e0, e1); break;
    case 8: col_launch_c<T, CPLX, 8>(last, a, grid, block, lds, st, e0, e1); break;
    case 16: col_launch_c<T, CPLX, 16>(last, a, grid, block, lds, st, e0, e1); break;
    case 32:
        if constexpr (sizeof(typename Alg<T, CPLX>::V) <= 8) {
            col_launch_c<T, CPLX, 32>(last, a, grid, block, lds, st, e0, e1);
            break;
        }
        return hipErrorInvalidValue;
    case 64:
        if constexpr (sizeof(typename Alg<T, CPLX>::V) <= 4) {
            col_launch_c<T, CPLX, 64>(last, a, grid, block, lds, st, e0, e1);
            break;
        }
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_col(int elem, int C, bool last, const ColArgs &a, int grid, int block, size_t lds,
                      hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
#define COL_CASE(T, CP) return col_launch<T, CP>(C, last, a, grid, block, lds, st, e0, e1)
    SSCN_ELEM_DISPATCH(elem, COL_CASE)
#undef COL_CASE
}

hipError_t launch_stream(int elem, const ColArgs &a, int grid, int block, hipStream_t st)
{
#define ST_CASE(T, CP) hipLaunchKernelGGL((k_stream<T, CP>), dim3(grid), dim3(block), 0, st, a)
    SSCN_ELEM_DISPATCH(elem, ST_CASE)
#undef ST_CASE
    return hipGetLastError();
}

hipError_t launch_pointwise(int elem, const PointArgs &a, int grid, int block, hipStream_t st)
{
#define PW_CASE(T, CP) hipLaunchKernelGGL((k_pointwise<T, CP>), dim3(grid), dim3(block), 0, st, a)
    SSCN_ELEM_DISPATCH(elem, PW_CASE)
#undef PW_CASE
    return hipGetLastError();
}

hipError_t launch_norm_partials(int elem, const void *psi, int64_t npts, double *partial, int grid,
                                int block, hipStream_t st)
{
#define NP_CASE(T, CP) \
    hipLaunchKernelGGL((k_norm_partials<T, CP>), dim3(grid), dim3(block), 0, st, psi, (long long)npts, partial)
    SSCN_ELEM_DISPATCH(elem, NP_CASE)
#undef NP_CASE
    return hipGetLastError();
}

hipError_t launch_norm_final(const double *partial, int np, double dvol, int do_renorm, double *scalars,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(1024), 0, st, partial, np, dvol, do_renorm, scalars);
    return hipGetLastError();
}

hipError_t launch_scale_state(int elem, void *psi, int64_t npts, const double *scalars, int grid,
                              int block, hipStream_t st)
{
#define SC_CASE(T, CP) \
    hipLaunchKernelGGL((k_scale_state<T, CP>), dim3(grid), dim3(block), 0, st, psi, (long long)npts, scalars)
    SSCN_ELEM_DISPATCH(elem, SC_CASE)
#undef SC_CASE
    return hipGetLastError();
}

hipError_t launch_set_unit_scale(double *scalars, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_unit_scale, dim3(1), dim3(64), 0, st, scalars);
    return hipGetLastError();
}

hipError_t launch_obs_partials(int elem, const ObsArgs &a, int grid, int block, hipStream_t st)
{
#define OB_CASE(T, CP) hipLaunchKernelGGL((k_obs_partials<T, CP>), dim3(grid), dim3(block), 0, st, a)
    SSCN_ELEM_DISPATCH(elem, OB_CASE)
#undef OB_CASE
    return hipGetLastError();
}

hipError_t launch_obs_final(const double *partial, int np, double dvol, double g, double *out,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, st, partial, np, dvol, g, out);
    return hipGetLastError();
}

hipError_t launch_density_1d(int elem, const void *psi, const int32_t *n, int keep, double w, double *out,
                             double *scratch, int dens_blocks, hipStream_t st)
{
    if (keep == 0) {
        // x is the contiguous axis: partial sums over row blocks, then a
        // fixed-order sum over the blocks
        const long long rows = (long long)n[1] * n[2];
#define DX_CASE(T, CP)                                                                                         \
    hipLaunchKernelGGL((k_density_x_rows<T, CP>), dim3(dens_blocks), dim3(256), 0, st, psi, n[0], rows, scratch)
        SSCN_ELEM_DISPATCH(elem, DX_CASE)
#undef DX_CASE
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_density_x_fin, dim3((n[0] + 63) / 64), dim3(1024), 0, st, scratch, n[0], dens_blocks,
                           w, out);
        return hipGetLastError();
    }
    const long long rows = (long long)n[1] * n[2];
    if (rows <= 262144) {
        // x-line sums into the scratch, then a sum over the other axis
#define DR_CASE(T, CP)                                                                                        \
    hipLaunchKernelGGL((k_density_rows<T, CP>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, psi, n[0], \
                       rows, 1.0, scratch)
        SSCN_ELEM_DISPATCH(elem, DR_CASE)
#undef DR_CASE
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_density_rows_fin, dim3((n[keep] + 3) / 4), dim3(256), 0, st, scratch, n[1], n[2], keep,
                           w, out);
        return hipGetLastError();
    }
#define D1_CASE(T, CP) \
    hipLaunchKernelGGL((k_density_1d<T, CP>), dim3(n[keep]), dim3(256), 0, st, psi, n[0], n[1], n[2], keep, w, out)
    SSCN_ELEM_DISPATCH(elem, D1_CASE)
#undef D1_CASE
    return hipGetLastError();
}

hipError_t launch_density_2d(int elem, const void *psi, const int32_t *n, int drop, double w, double *out,
                             hipStream_t st)
{
    const int u = (drop == 0) ? 1 : 0, v = (drop == 2) ? 1 : 2;
    const long long cnt = (long long)n[u] * n[v];
    if (drop == 0) {
        // the x-line sums themselves, in (y, z) layout order
#define DR_CASE(T, CP)                                                                                          \
    hipLaunchKernelGGL((k_density_rows<T, CP>), dim3((unsigned)((cnt + 3) / 4)), dim3(256), 0, st, psi, n[0], cnt, \
                       w, out)
        SSCN_ELEM_DISPATCH(elem, DR_CASE)
#undef DR_CASE
        return hipGetLastError();
    }
    const int grid = (int)((cnt + 255) / 256);
#define D2_CASE(T, CP) \
    hipLaunchKernelGGL((k_density_2d<T, CP>), dim3(grid), dim3(256), 0, st, psi, n[0], n[1], n[2], drop, w, out)
    SSCN_ELEM_DISPATCH(elem, D2_CASE)
#undef D2_CASE
    return hipGetLastError();
}

}  // namespace sscn

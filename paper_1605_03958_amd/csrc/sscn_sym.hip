// sscn_sym.hip -- gfx950 kernels of the symmetric traps (circular,
// spherical and axial; the equations are in sscn.h).
//
//   k_rad  one radial line per block: pending renormalisation scale and the
//          pointwise substep fused into the load, then the Crank-Nicolson
//          substep along r, whose tridiagonal system has a coefficient set
//          per cell (the finite-volume radial Laplacian).  Thomas
//          elimination with the FP64 tables computed on the host turns the
//          line into two first-order recurrences,
//              forward   d_i = alpha_i d_{i-1} + m_i r_i    (alpha_0 = 0)
//              backward  v_i = beta_i v_{i+1} + d_i         (v_n = 0)
//          Each thread holds C consecutive cells in registers and composes
//          its chunk into an affine map; an exact block-wide scan of those
//          maps (shuffles within a wave, wave totals through LDS) gives
//          every chunk its incoming value, and the chunk recurrences are
//          re-run with it.  The last sweep of an imaginary-time step also
//          emits the block's FP64 sum of W_i |psi_i|^2.
//   k_sym_obs_partials  per-block FP64 sums of the observables in the
//          weighted inner product, in the row layout k_obs_final reads.
#include <hip/hip_ext.h>

#include "sscn_lines.hpp"
#include "sscn_sym.hpp"

namespace sscn {

// u - i X (real time) or u - X (imaginary time)
template <class T, bool CPLX>
__device__ __forceinline__ typename Alg<T, CPLX>::V rhs_sub(typename Alg<T, CPLX>::V u,
                                                            typename Alg<T, CPLX>::V x)
{
    if constexpr (CPLX) return typename Alg<T, CPLX>::V{u.re + x.im, u.im - x.re};
    else return u - x;
}

// Incoming value of this thread's chunk from an exclusive scan over the
// block of the affine maps x -> a x + b: in increasing thread order (FWD,
// the first chunk receives 0) or decreasing (backward, the last chunk
// receives 0).  ta, tb: one slot per wave.
template <class T, bool CPLX, bool FWD>
__device__ __forceinline__ typename Alg<T, CPLX>::V chunk_incoming(typename Alg<T, CPLX>::V a,
                                                                   typename Alg<T, CPLX>::V b,
                                                                   typename Alg<T, CPLX>::V *ta,
                                                                   typename Alg<T, CPLX>::V *tb)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // inclusive scan within the wave: compose with the maps of lanes before
    // (FWD) or after (backward) this one
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        V pa, pb;
        bool take;
        if constexpr (FWD) {
            pa = A::shfl_up(a, o);
            pb = A::shfl_up(b, o);
            take = lane >= o;
        } else {
            pa = A::shfl_down(a, o);
            pb = A::shfl_down(b, o);
            take = lane + o < 64;
        }
        if (take) {
            b = A::fma(a, pb, b);
            a = A::mul(a, pa);
        }
    }
    V ea, eb;
    if constexpr (FWD) {
        ea = A::shfl_up(a, 1);
        eb = A::shfl_up(b, 1);
        if (lane == 0) {
            ea = A::one();
            eb = A::zero();
        }
    } else {
        ea = A::shfl_down(a, 1);
        eb = A::shfl_down(b, 1);
        if (lane == 63) {
            ea = A::one();
            eb = A::zero();
        }
    }
    __syncthreads();   // the slots are free
    if (lane == (FWD ? 63 : 0)) {
        ta[w] = a;
        tb[w] = b;
    }
    __syncthreads();
    // the value entering this wave: the totals of the waves before (after) it
    // applied in order to 0
    V x = A::zero();
    if constexpr (FWD) {
        for (int q = 0; q < w; ++q) x = A::fma(ta[q], x, tb[q]);
    } else {
        for (int q = nw - 1; q > w; --q) x = A::fma(ta[q], x, tb[q]);
    }
    return A::fma(ea, x, eb);
}

// The table entries of a thread's C cells: with PRE (short chunks) all of
// them are loaded into registers at the start of the kernel, so their
// latency overlaps the state's load instead of adding a round trip to each
// phase; otherwise each phase loads what it needs.
template <int C, bool PRE>
struct RadTab {
    const double *tab;
    int Q, G, t;
    double v[PRE ? RQ_N : 1][PRE ? C : 1];
    __device__ __forceinline__ void init(const double *tb, int q, int g, int th)
    {
        tab = tb;
        Q = q;
        G = g;
        t = th;
        if constexpr (PRE) {
#pragma unroll
            for (int qq = 0; qq < RQ_N; ++qq)
#pragma unroll
                for (int k = 0; k < C; ++k) v[qq][k] = tab[qq * Q + k * G + t];
        }
    }
    __device__ __forceinline__ double at(int q, int k) const
    {
        if constexpr (PRE) return v[q][k];
        else return tab[q * Q + k * G + t];
    }
};

template <class T, bool CPLX, class TB>
__device__ __forceinline__ typename Alg<T, CPLX>::V rad_coef(const TB &tb, int qre, int qim, int k)
{
    return Alg<T, CPLX>::coef(tb.at(qre, k), CPLX ? tb.at(qim, k) : 0.0);
}

template <class T, bool CPLX, int C, bool LAST>
__global__ void __launch_bounds__(1024) k_rad(RadArgs a)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    __shared__ V first_v[16], last_v[16];
    __shared__ V ta[16], tb[16];
    __shared__ double red[16];
    const int G = blockDim.x;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = G >> 6;
    const int Q = G * C;
    const int n = a.n;
    RadTab<C, (C <= 4)> rt;
    rt.init(a.tab, Q, G, t);
    V *psi = reinterpret_cast<V *>(a.psi) + (long long)blockIdx.x * n;
    const T scale = CPLX ? T(1) : T(*a.scale);
    const T dt = T(a.dt), g = T(a.g);
    const double z = (double(blockIdx.x) - a.cen_z) * a.dz;
    const double vz = a.w2h_z * z * z;

    // load, pending scale and pointwise substep
    V u[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = t * C + k;
        u[k] = A::zero();
        if (i < n) {
            const double r = (i + 0.5) * a.dr;
            u[k] = apply_point<T, CPLX>(psi[i], scale, T(fmaT(a.w2h_r * r, r, vz)), dt, g);
        }
    }

    // right-hand side (1 - tau H_r) u: neighbours across chunk boundaries
    V left = A::shfl_up(u[C - 1], 1), right = A::shfl_down(u[0], 1);
    if (lane == 0) first_v[w] = u[0];
    if (lane == 63) last_v[w] = u[C - 1];
    __syncthreads();
    if (lane == 0) left = (w > 0) ? last_v[w - 1] : A::zero();
    if (lane == 63) right = (w + 1 < nw) ? first_v[w + 1] : A::zero();
    {
        V prev = left;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const T L = T(rt.at(RQ_L, k)), D = T(rt.at(RQ_D, k)), U = T(rt.at(RQ_U, k));
            const V next = (k + 1 < C) ? u[k + 1] : right;
            const V x = A::sub(A::scal(D, u[k]), A::add(A::scal(L, prev), A::scal(U, next)));
            prev = u[k];
            u[k] = rhs_sub<T, CPLX>(u[k], x);
        }
    }

    // forward recurrence: chunk map, scan, re-run
    {
        V fa = A::one(), fb = A::zero();
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const V m = rad_coef<T, CPLX>(rt, RQ_MR, RQ_MI, k);
            const V al = rad_coef<T, CPLX>(rt, RQ_AR, RQ_AI, k);
            fb = A::fma(al, fb, A::mul(m, u[k]));
            fa = A::mul(al, fa);
        }
        V d = chunk_incoming<T, CPLX, true>(fa, fb, ta, tb);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const V m = rad_coef<T, CPLX>(rt, RQ_MR, RQ_MI, k);
            const V al = rad_coef<T, CPLX>(rt, RQ_AR, RQ_AI, k);
            d = A::fma(al, d, A::mul(m, u[k]));
            u[k] = d;
        }
    }
    // backward recurrence
    {
        V ba = A::one(), bb = A::zero();
#pragma unroll
        for (int k = C - 1; k >= 0; --k) {
            const V be = rad_coef<T, CPLX>(rt, RQ_BR, RQ_BI, k);
            bb = A::fma(be, bb, u[k]);
            ba = A::mul(be, ba);
        }
        V v = chunk_incoming<T, CPLX, false>(ba, bb, ta, tb);
#pragma unroll
        for (int k = C - 1; k >= 0; --k) {
            const V be = rad_coef<T, CPLX>(rt, RQ_BR, RQ_BI, k);
            v = A::fma(be, v, u[k]);
            u[k] = v;
        }
    }

    double nacc = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = t * C + k;
        if (i < n) {
            psi[i] = u[k];
            if constexpr (LAST) nacc = fmaT(rt.at(RQ_W, k), A::norm2(u[k]), nacc);
        }
    }
    if constexpr (LAST) {
        const double s = block_sum(nacc, red);
        if (threadIdx.x == 0) {
            a.partial[blockIdx.x] = s;
            if (a.scalars) {
                // every thread read the old factor before block_sum's barriers
                const double N = a.dvol * s;
                a.scalars[1] = N;
                a.scalars[0] = 1.0 / sqrt(N);
            }
        }
    }
}

template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_sym_obs_partials(SymObsArgs a)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    constexpr int NQ = 10;
    __shared__ double red[NQ][4];
    const V *psi = reinterpret_cast<const V *>(a.psi);
    const long long nr = a.nr, nz = a.nz;
    const double dr = a.dr, dr2 = dr * dr, dz2 = a.dz * a.dz;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    // acc: 0 sum W q, 1 sum kinetic faces and edges, 2 sum W V q, 3 sum W q^2,
    // 4 sum W r q, 5 sum W z q, 7 sum W r^2 q, 8 sum W z^2 q (6, 9 unused)
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < a.npts;
         p += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(p % nr);
        const int j = (int)(p / nr);
        const V v = psi[p];
        const double q = A::norm2(v);
        const double r = (i + 0.5) * dr;
        const double W = (a.k == 1) ? r : fmaT(r, r, dr2 / 12.0);
        const double f = (i + 1) * dr;
        const double F = (a.k == 1) ? f : f * f;
        const V nb = (i + 1 < nr) ? psi[p + 1] : A::zero();
        double kin = F * A::norm2(A::sub(nb, v)) / dr2;
        const double z = (double(j) - a.cen_z) * a.dz;
        if (a.axial) {
            const V nz_ = (j + 1 < nz) ? psi[p + nr] : A::zero();
            double e = A::norm2(A::sub(nz_, v));
            if (j == 0) e += q;
            kin = fmaT(W, e / dz2, kin);
        }
        const double vp = fmaT(a.w2h_r * r, r, a.w2h_z * z * z);
        const double wq = W * q;
        acc[0] += wq;
        acc[1] += kin;
        acc[2] = fmaT(vp, wq, acc[2]);
        acc[3] = fmaT(wq, q, acc[3]);
        acc[4] = fmaT(r, wq, acc[4]);
        acc[5] = fmaT(z, wq, acc[5]);
        acc[7] = fmaT(r * r, wq, acc[7]);
        acc[8] = fmaT(z * z, wq, acc[8]);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        const int q = threadIdx.x;
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[q][w];
        a.partial[(size_t)blockIdx.x * 12 + q] = s;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define SYM_ELEM_DISPATCH(elem, MACRO)        \
    switch (elem) {                           \
    case 0: MACRO(double, false); break;      \
    case 1: MACRO(float, false); break;       \
    case 2: MACRO(double, true); break;       \
    case 3: MACRO(float, true); break;        \
    default: return hipErrorInvalidValue;     \
    }

template <class T, bool CPLX, int C>
static void rad_launch_c(bool last, const RadArgs &a, int grid, int block, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1)
{
    if (last) hipExtLaunchKernelGGL((k_rad<T, CPLX, C, true>), dim3(grid), dim3(block), 0, st, e0, e1, 0, a);
    else hipExtLaunchKernelGGL((k_rad<T, CPLX, C, false>), dim3(grid), dim3(block), 0, st, e0, e1, 0, a);
}

template <class T, bool CPLX>
static hipError_t rad_launch(int C, bool last, const RadArgs &a, int grid, int block, hipStream_t st,
                             hipEvent_t e0, hipEvent_t e1)
{
    switch (C) {
    case 4: rad_launch_c<T, CPLX, 4>(last, a, grid, block, st, e0, e1); break;
    case 8: rad_launch_c<T, CPLX, 8>(last, a, grid, block, st, e0, e1); break;
    case 16: rad_launch_c<T, CPLX, 16>(last, a, grid, block, st, e0, e1); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rad(int elem, int C, bool last, const RadArgs &a, int grid, int block, hipStream_t st,
                      hipEvent_t e0, hipEvent_t e1)
{
    if (block < 64 || block > 1024 || block % 64 != 0) return hipErrorInvalidValue;
#define RAD_CASE(T, CP) return rad_launch<T, CP>(C, last, a, grid, block, st, e0, e1)
    SYM_ELEM_DISPATCH(elem, RAD_CASE)
#undef RAD_CASE
}

hipError_t launch_sym_obs_partials(int elem, const SymObsArgs &a, int grid, int block, hipStream_t st)
{
#define SO_CASE(T, CP) hipLaunchKernelGGL((k_sym_obs_partials<T, CP>), dim3(grid), dim3(block), 0, st, a)
    SYM_ELEM_DISPATCH(elem, SO_CASE)
#undef SO_CASE
    return hipGetLastError();
}

}  // namespace sscn

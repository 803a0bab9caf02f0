// sscn_dev.hpp -- device-side building blocks of the gfx950 SSCN propagator.
//
// One SSCN step (the paper's split-step Crank-Nicolson scheme, see sscn.h for
// the equations) is, per axis, a family of independent constant-coefficient
// tridiagonal systems
//     -s v_{i-1} + (1 + 2s) v_i - s v_{i+1} = r_i,   r = (1 - sT) u,
// one per grid line.  Thomas elimination with the FP64 tables computed on the
// host,
//     m_0 = 1/(1+2s),  m_i = 1/(1 + 2s - s^2 m_{i-1}),  alpha_i = s m_i,
// turns each line into two first-order linear recurrences that share alpha:
//     forward   d_i = alpha_i d_{i-1} + m_i r_i         (d_{-1} = 0)
//     backward  v_i = alpha_i v_{i+1} + d_i             (v_n = 0)
// A line is split into contiguous chunks held in registers by a group of
// threads.  Each thread composes its chunk into an affine map x -> A x + B
// (A = product of alpha over the chunk), an exclusive scan of those maps
// across the group gives every chunk its exact incoming value, and the chunk
// recurrences are re-run with it.  Nothing is truncated: the result is the
// Thomas solution up to the order of rounding.
//
// Two geometries use the same chunk algebra:
//   ROW  (x lines, stride 1): the G = 64*WPL threads of a line group hold
//        consecutive chunks of one line; the scan runs over lanes with
//        cross-lane shuffles and, for WPL > 1, across waves through LDS.
//   COL  (y and z lines): the 64 lanes of a wave hold 64 different lines
//        (adjacent line indices, so every load and store of a wave is
//        contiguous); the W waves of a block hold consecutive chunks; the
//        scan runs across waves through LDS and the table entries are
//        wave-uniform.
// Padding beyond the line end uses zero tables and zero data, which makes
// every padded value exactly zero and leaves the real points untouched.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sscn {

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// lane moves: the value of lane i - d (up) or i + d (down) of the wave.  A
// shift by one lane is one register move per 32 bits (the data-parallel-
// primitive whole-wave shift); shifts of up to 4 lanes repeat it, longer
// ones go through the LDS crossbar (ds_bpermute).  Lanes with no source
// lane receive unspecified values: callers mask them.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <class T>
__device__ __forceinline__ T lane_up(T v, int d)
{
    if (d <= 4) {
        for (int j = 0; j < d; ++j) v = dpp_mov<0x138>(v);   // wave_shr:1
        return v;
    }
    return __shfl_up(v, d, 64);
}
template <class T>
__device__ __forceinline__ T lane_down(T v, int d)
{
    if (d <= 4) {
        for (int j = 0; j < d; ++j) v = dpp_mov<0x130>(v);   // wave_shl:1
        return v;
    }
    return __shfl_down(v, d, 64);
}

// ---------------------------------------------------------------------------
// value algebra: real (imaginary time) or complex (real time)
// ---------------------------------------------------------------------------
template <class T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <class T, bool CPLX>
struct Alg;

template <class T>
struct Alg<T, false> {
    using V = T;
    __device__ __forceinline__ static V zero() { return T(0); }
    __device__ __forceinline__ static V one() { return T(1); }
    __device__ __forceinline__ static V mul(V a, V b) { return a * b; }
    __device__ __forceinline__ static V fma(V a, V b, V c) { return fmaT(a, b, c); }
    __device__ __forceinline__ static V add(V a, V b) { return a + b; }
    __device__ __forceinline__ static V sub(V a, V b) { return a - b; }
    __device__ __forceinline__ static V scal(T s, V a) { return s * a; }
    __device__ __forceinline__ static double norm2(V a) { return double(a) * double(a); }
    __device__ __forceinline__ static T norm2t(V a) { return a * a; }
    // coefficient from an FP64 (re, im) table entry
    __device__ __forceinline__ static V coef(double re, double) { return T(re); }
    __device__ __forceinline__ static V shfl_up(V a, int d) { return lane_up(a, d); }
    __device__ __forceinline__ static V shfl_down(V a, int d) { return lane_down(a, d); }
    // through the LDS crossbar at any distance
    __device__ __forceinline__ static V xshfl_up(V a, int d) { return __shfl_up(a, d, 64); }
    __device__ __forceinline__ static V xshfl_down(V a, int d) { return __shfl_down(a, d, 64); }
    __device__ __forceinline__ static bool finite(V a) { return __builtin_isfinite(a); }
};

template <class T>
struct Alg<T, true> {
    using V = cpx<T>;
    __device__ __forceinline__ static V zero() { return V{T(0), T(0)}; }
    __device__ __forceinline__ static V one() { return V{T(1), T(0)}; }
    __device__ __forceinline__ static V mul(V a, V b) {
        return V{fmaT(a.re, b.re, -a.im * b.im), fmaT(a.re, b.im, a.im * b.re)};
    }
    __device__ __forceinline__ static V fma(V a, V b, V c) {
        return V{fmaT(a.re, b.re, fmaT(-a.im, b.im, c.re)),
                 fmaT(a.re, b.im, fmaT(a.im, b.re, c.im))};
    }
    __device__ __forceinline__ static V add(V a, V b) { return V{a.re + b.re, a.im + b.im}; }
    __device__ __forceinline__ static V sub(V a, V b) { return V{a.re - b.re, a.im - b.im}; }
    __device__ __forceinline__ static V scal(T s, V a) { return V{s * a.re, s * a.im}; }
    // explicit FMAs: a contractible a*b + c*d could be fused either way, and
    // differently in different kernels; every path must round alike
    __device__ __forceinline__ static double norm2(V a) {
        return fmaT(double(a.re), double(a.re), double(a.im) * double(a.im));
    }
    __device__ __forceinline__ static T norm2t(V a) { return fmaT(a.re, a.re, a.im * a.im); }
    __device__ __forceinline__ static V coef(double re, double im) { return V{T(re), T(im)}; }
    __device__ __forceinline__ static V shfl_up(V a, int d) { return V{lane_up(a.re, d), lane_up(a.im, d)}; }
    __device__ __forceinline__ static V shfl_down(V a, int d) { return V{lane_down(a.re, d), lane_down(a.im, d)}; }
    __device__ __forceinline__ static V xshfl_up(V a, int d) {
        return V{__shfl_up(a.re, d, 64), __shfl_up(a.im, d, 64)};
    }
    __device__ __forceinline__ static V xshfl_down(V a, int d) {
        return V{__shfl_down(a.re, d, 64), __shfl_down(a.im, d, 64)};
    }
    __device__ __forceinline__ static bool finite(V a) {
        return __builtin_isfinite(a.re) && __builtin_isfinite(a.im);
    }
};

// ---------------------------------------------------------------------------
// tables and parameters
// ---------------------------------------------------------------------------

// One Thomas table entry (FP64 always): alpha_i = s m_i and m_i, as (re, im).
struct TabEntry {
    double ar, ai, mr, mi;
};

// Pointwise-substep parameters for the x sweep (the first sweep of a step).
struct PointParams {
    double dt, g;
    double dx[3];
    double cen[3];   // (n_a - 1) / 2
    double w2h[3];   // omega_a^2 / 2 (0 on unused axes)
    int32_t n[3];
};

// r = (1 - sT) u at one point given its two neighbours (zero past the ends).
template <class T, bool CPLX>
__device__ __forceinline__ typename Alg<T, CPLX>::V
cn_rhs(typename Alg<T, CPLX>::V um, typename Alg<T, CPLX>::V u0, typename Alg<T, CPLX>::V up,
       typename Alg<T, CPLX>::V sig)
{
    using A = Alg<T, CPLX>;
    // u + s (u_{i-1} + u_{i+1} - 2 u_i)
    typename A::V lap = A::sub(A::add(um, up), A::add(u0, u0));
    return A::fma(sig, lap, u0);
}

// ---------------------------------------------------------------------------
// block reductions (FP64, fixed order)
// ---------------------------------------------------------------------------
// v taken from another lane by the data-parallel-primitive controls: each
// 32-bit half moves with the same control; lanes of rows outside ROWS get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the wave's 64 lanes in a fixed order, returned to every lane.
// The wave must be whole (all lanes active).  Quads first (swap neighbours,
// then pairs), then 8- and 16-lane groups by mirroring within each row of 16;
// then lane 15 of rows 0 and 2 is added into rows 1 and 3, and lane 31 into
// rows 2 and 3, which leaves the total in lane 63.  Register moves only: no
// LDS round trips as with shuffles.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_take<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_take<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_take<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_take<0x140, 0xF>(v);   // row_mirror
    v += dpp_take<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
    v += dpp_take<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Sum of v over the block, returned to thread 0; red needs blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += red[w];
    }
    return s;
}

// The renormalisation factor 1/sqrt(dvol * sum) over np <= 64 * kFoldWaves
// partials, formed by one whole wave in k_norm_final's order (partial i on
// thread i of its 1024-thread block, the 64-lane wave sums added in wave
// order, zero sums left out: adding +0 changes nothing), so every wave of
// another kernel obtains bitwise the factor k_norm_final would write.
// p[w] holds partial w*64 + lane, zero past np.
constexpr int kFoldWaves = 4;
__device__ __forceinline__ double fold_scale(const double (&p)[kFoldWaves], int np, double dvol)
{
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kFoldWaves; ++w)
        if (w * 64 < np) s += wave_sum(p[w]);
    return 1.0 / sqrt(dvol * s);
}

}  // namespace sscn

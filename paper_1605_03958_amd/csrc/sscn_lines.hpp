// sscn_lines.hpp -- line solves of one SSCN step, shared by the
// single-problem kernels (sscn_kernels.hip) and the batched persistent
// kernel (sscn_batch.hip), so both run the same arithmetic.
//
// ROW (x lines): a line group of G = 64 * wpl threads holds consecutive
// chunks of C points of one line; the pointwise substep and the pending
// renormalisation are applied to the loaded values; the chunk maps are
// scanned across lanes (and across waves through LDS when wpl > 1).
// COL (y, z lines): 64/L adjacent lines per tile, chunk ch = w*L + l/(64/L)
// of line l%(64/L) on lane l of wave w; chunk maps folded through LDS.
#pragma once

#include "sscn_launch.hpp"

namespace sscn {

// FP32: the hardware base-2 exponential of x log2(e) (within about 2 ulp
// for the arguments of the pointwise substep); the library form spends a
// dozen instructions per point on range reduction and rounding below the
// FP32 state's own rounding.
template <class T>
__device__ __forceinline__ T dev_exp(T x)
{
    if constexpr (sizeof(T) == 8) return exp(x); else return __expf(x);
}

template <class T>
__device__ __forceinline__ void dev_sincos(T x, T *s, T *c)
{
    if constexpr (sizeof(T) == 8) sincos(x, s, c); else sincosf(x, s, c);
}

// sin and cos for |x| <= pi/4 from their Maclaurin series, through x^17 and
// x^18 in FP64 (remainders below 1e-19 there) and through x^9 and x^10 in
// FP32 (below 3e-9).  Horner form in x^2.
template <class T>
__device__ __forceinline__ void sincos_small(T x, T *s, T *c)
{
    const T x2 = x * x;
    if constexpr (sizeof(T) == 8) {
        T p = T(1.0 / 355687428096000.0);           //  1/17!
        p = fmaT(p, -x2, T(1.0 / 1307674368000.0));  //  1/15!
        p = fmaT(p, -x2, T(1.0 / 6227020800.0));     //  1/13!
        p = fmaT(p, -x2, T(1.0 / 39916800.0));       //  1/11!
        p = fmaT(p, -x2, T(1.0 / 362880.0));         //  1/9!
        p = fmaT(p, -x2, T(1.0 / 5040.0));           //  1/7!
        p = fmaT(p, -x2, T(1.0 / 120.0));            //  1/5!
        p = fmaT(p, -x2, T(1.0 / 6.0));              //  1/3!
        p = fmaT(p, -x2, T(1.0));
        *s = x * p;
        T q = T(1.0 / 6402373705728000.0);          //  1/18!
        q = fmaT(q, -x2, T(1.0 / 20922789888000.0)); //  1/16!
        q = fmaT(q, -x2, T(1.0 / 87178291200.0));    //  1/14!
        q = fmaT(q, -x2, T(1.0 / 479001600.0));      //  1/12!
        q = fmaT(q, -x2, T(1.0 / 3628800.0));        //  1/10!
        q = fmaT(q, -x2, T(1.0 / 40320.0));          //  1/8!
        q = fmaT(q, -x2, T(1.0 / 720.0));            //  1/6!
        q = fmaT(q, -x2, T(1.0 / 24.0));             //  1/4!
        q = fmaT(q, -x2, T(1.0 / 2.0));              //  1/2!
        q = fmaT(q, -x2, T(1.0));
        *c = q;
    } else {
        T p = T(1.0 / 362880.0);
        p = fmaT(p, -x2, T(1.0 / 5040.0));
        p = fmaT(p, -x2, T(1.0 / 120.0));
        p = fmaT(p, -x2, T(1.0 / 6.0));
        p = fmaT(p, -x2, T(1.0));
        *s = x * p;
        T q = T(1.0 / 3628800.0);
        q = fmaT(q, -x2, T(1.0 / 40320.0));
        q = fmaT(q, -x2, T(1.0 / 720.0));
        q = fmaT(q, -x2, T(1.0 / 24.0));
        q = fmaT(q, -x2, T(1.0 / 2.0));
        q = fmaT(q, -x2, T(1.0));
        *c = q;
    }
}

// Library sin/cos for phases outside [-pi/4, pi/4], kept out of line so the
// common small-phase path does not carry its registers.
// FP64 sin and cos for |x| <= 1/8: the same series through x^9 and x^10
// (remainders below 3e-18 and 3e-20 there), four and five fewer FMAs.
__device__ __forceinline__ void sincos_tiny(double x, double *s, double *c)
{
    const double x2 = x * x;
    double p = 1.0 / 362880.0;                       //  1/9!
    p = fmaT(p, -x2, 1.0 / 5040.0);                  //  1/7!
    p = fmaT(p, -x2, 1.0 / 120.0);                   //  1/5!
    p = fmaT(p, -x2, 1.0 / 6.0);                     //  1/3!
    p = fmaT(p, -x2, 1.0);
    *s = x * p;
    double q = 1.0 / 3628800.0;                      //  1/10!
    q = fmaT(q, -x2, 1.0 / 40320.0);                 //  1/8!
    q = fmaT(q, -x2, 1.0 / 720.0);                   //  1/6!
    q = fmaT(q, -x2, 1.0 / 24.0);                    //  1/4!
    q = fmaT(q, -x2, 1.0 / 2.0);                     //  1/2!
    q = fmaT(q, -x2, 1.0);
    *c = q;
}

template <class T>
__device__ __attribute__((noinline)) cpx<T> phase_slow(T x)
{
    T sn, cs;
    dev_sincos<T>(x, &sn, &cs);
    return cpx<T>{cs, sn};
}

// Pointwise substep on one value (imaginary time: scale first; real time: phase).
template <class T, bool CPLX>
__device__ __forceinline__ typename Alg<T, CPLX>::V
apply_point(typename Alg<T, CPLX>::V u, T scale, T vpot, T dt, T g)
{
    using A = Alg<T, CPLX>;
    if constexpr (!CPLX) {
        u = A::scal(scale, u);
        T phi = dt * fmaT(g, A::norm2t(u), vpot);
        return dev_exp<T>(-phi) * u;
    } else {
        (void)scale;
        T phi = dt * fmaT(g, A::norm2t(u), vpot);
        T sn, cs;
        const T aphi = __builtin_fabs(phi);
        if (sizeof(T) == 8 && aphi <= T(0.125)) {
            if constexpr (sizeof(T) == 8) sincos_tiny(phi, &sn, &cs);
        } else if (aphi <= T(0.78539816339744830962)) {
            sincos_small<T>(phi, &sn, &cs);
        } else {
            const cpx<T> e = phase_slow<T>(phi);
            cs = e.re;
            sn = e.im;
        }
        return typename A::V{fmaT(cs, u.re, sn * u.im), fmaT(cs, u.im, -sn * u.re)};
    }
}

// Grid coordinate (i - cen) dx: FP64 for FP64 states; FP32 for FP32 ones
// (i - cen is a multiple of 1/2 below 2^23, exact in FP32, so only dx and
// the product round).
template <class T>
__device__ __forceinline__ T coord(int i, double cen, double dx)
{
    if constexpr (sizeof(T) == 4) return (T(i) - T(cen)) * T(dx);
    else return T((double(i) - cen) * dx);
}

// A Thomas table entry as the sweeps use it.  FP64: (alpha, m).  FP32: each
// FP64 coefficient c is kept as the unevaluated pair hi + lo with hi = fl32(c)
// and lo = fl32(c - hi), and every product c x is formed as hi x + lo x in
// FP32.  The coefficients then carry ~48 bits, so the FP32 operator stays
// the FP64 one up to the rounding of the data arithmetic: rounding the
// coefficients once would perturb every line of every step identically and
// the real-time norm would drift coherently (about 1e-4 over 1000 steps).
template <class T, bool CPLX>
struct LTab;

template <bool CPLX>
struct LTab<double, CPLX> {
    using A = Alg<double, CPLX>;
    using V = typename A::V;
    V al, m;
    __device__ __forceinline__ static LTab make(const TabEntry &e)
    {
        return LTab{A::coef(e.ar, e.ai), A::coef(e.mr, e.mi)};
    }
    __device__ __forceinline__ V afma(V x, V y) const { return A::fma(al, x, y); }   // alpha x + y
    __device__ __forceinline__ V mmul(V r) const { return A::mul(m, r); }            // m r
    __device__ __forceinline__ V alpha() const { return al; }
};

template <bool CPLX>
struct LTab<float, CPLX> {
    using A = Alg<float, CPLX>;
    using V = typename A::V;
    V al, al_lo, m, m_lo;
    __device__ __forceinline__ static V lo_of(double re, double im, V hi)
    {
        if constexpr (CPLX) return V{float(re - double(hi.re)), float(im - double(hi.im))};
        else return float(re - double(hi));
    }
    __device__ __forceinline__ static LTab make(const TabEntry &e)
    {
        LTab t;
        t.al = A::coef(e.ar, e.ai);
        t.m = A::coef(e.mr, e.mi);
        t.al_lo = lo_of(e.ar, e.ai, t.al);
        t.m_lo = lo_of(e.mr, e.mi, t.m);
        return t;
    }
    __device__ __forceinline__ V afma(V x, V y) const { return A::fma(al, x, A::fma(al_lo, x, y)); }
    __device__ __forceinline__ V mmul(V r) const { return A::fma(m, r, A::mul(m_lo, r)); }
    __device__ __forceinline__ V alpha() const { return al; }
};

// Fill a kernel's table slice in LDS (cnt entries) in the working
// representation; the caller synchronises before reading it.  Slot q holds
// line point i = pos(q) (ROW: lane-major, i = (q % G) * C + q / G with G =
// group threads; COL: i = q).  Only the head of the table below lt.i_conv
// is read from memory; the constant tail is written from lt's constant
// entry and points past the line end get zeros.
// Element access to the state through a generic pointer or a global one
// (address space 1).  A complex value in global memory moves as a native
// two-element vector: class types cannot be copied through such pointers.
template <class V>
__device__ __forceinline__ V ld_elem(const V *p, long long i)
{
    return p[i];
}
template <class V>
__device__ __forceinline__ void st_elem(V *p, long long i, V v)
{
    p[i] = v;
}
template <class T>
__device__ __forceinline__ T ld_elem(const __attribute__((address_space(1))) T *p, long long i)
{
    return p[i];
}
template <class T>
__device__ __forceinline__ void st_elem(__attribute__((address_space(1))) T *p, long long i, T v)
{
    p[i] = v;
}
template <class T>
__device__ __forceinline__ cpx<T> ld_elem(const __attribute__((address_space(1))) cpx<T> *p, long long i)
{
    typedef T W __attribute__((ext_vector_type(2)));
    const W w = reinterpret_cast<const __attribute__((address_space(1))) W *>(p)[i];
    return cpx<T>{w.x, w.y};
}
template <class T>
__device__ __forceinline__ void st_elem(__attribute__((address_space(1))) cpx<T> *p, long long i, cpx<T> v)
{
    typedef T W __attribute__((ext_vector_type(2)));
    W w;
    w.x = v.re;
    w.y = v.im;
    reinterpret_cast<__attribute__((address_space(1))) W *>(p)[i] = w;
}

// One FP64 table entry through a generic or a global pointer (field by
// field: a struct cannot be copied through an address-space pointer).
__device__ __forceinline__ TabEntry ld_tab(const TabEntry *p, int q) { return p[q]; }
__device__ __forceinline__ TabEntry ld_tab(const __attribute__((address_space(1))) TabEntry *p, int q)
{
    const __attribute__((address_space(1))) double *d = reinterpret_cast<const __attribute__((address_space(1))) double *>(p + q);
    return TabEntry{d[0], d[1], d[2], d[3]};
}

// As stage_table, reading the table through tab (a pointer of any address
// space to lt's table).
template <class T, bool CPLX, class TP>
__device__ __forceinline__ void stage_table_from(const LineTab &lt, TP tab, LTab<T, CPLX> *dst, int cnt, int G, int C)
{
    const LTab<T, CPLX> tail = LTab<T, CPLX>::make(TabEntry{lt.ac_re, lt.ac_im, lt.mc_re, lt.mc_im});
    const LTab<T, CPLX> zero = LTab<T, CPLX>::make(TabEntry{0.0, 0.0, 0.0, 0.0});
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
        const int i = (G > 0) ? (q % G) * C + q / G : q;
        LTab<T, CPLX> e = tail;
        if (i >= lt.n) e = zero;
        else if (i < lt.i_conv) e = LTab<T, CPLX>::make(ld_tab(tab, q));
        dst[q] = e;
    }
}

template <class T, bool CPLX>
__device__ __forceinline__ void stage_table(const LineTab &lt, LTab<T, CPLX> *dst, int cnt, int G, int C)
{
    stage_table_from<T, CPLX>(lt, lt.tab, dst, cnt, G, C);
}

// Table entry q from LDS (staged) or from the FP64 table in global memory.
template <class T, bool CPLX>
__device__ __forceinline__ LTab<T, CPLX> tab_at(const LTab<T, CPLX> *tb, int q)
{
    return tb[q];
}

template <class T, bool CPLX>
__device__ __forceinline__ LTab<T, CPLX> tab_at(const TabEntry *tb, int q)
{
    return LTab<T, CPLX>::make(tb[q]);
}

template <class T, bool CPLX>
__device__ __forceinline__ LTab<T, CPLX> tab_at(const __attribute__((address_space(1))) TabEntry *tb, int q)
{
    return LTab<T, CPLX>::make(ld_tab(tb, q));
}

// Entry k of thread t's chunk in a ROW line group of G threads: slot k*G + t
// of a lane-major table (staged or in memory).  Other table forms add their
// own overload (found by argument-dependent lookup).
template <class T, bool CPLX, class TB>
__device__ __forceinline__ LTab<T, CPLX> row_tab(const TB *tb, int k, int G, int t)
{
    return tab_at<T, CPLX>(tb, k * G + t);
}

// ---------------------------------------------------------------------------
// ROW: one x line per line group.  xs: 4 values per wave of the group (LDS,
// used when MW).  Returns the thread's sum |v|^2 when `last`.  The load of
// the lane's values (row_load) is apart from the solve (row_solve), so a
// caller can issue the next line's loads before solving the current one;
// row_line does both.  With `keep` the solution replaces u instead of being
// stored (a caller that holds its line in registers across steps).
// SEG < 64: a wave holds 64/SEG lines of SEG lanes each (t = lane % SEG,
// G = SEG); the scans stop at the segment's ends, so short lines take fewer
// scan steps and fewer lanes' worth of per-line work.
// ---------------------------------------------------------------------------
template <class T, bool CPLX, int C, bool MW, bool UNR = true, int SEG = 64, class TB, class PV>
__device__ __forceinline__ double row_solve(PV __restrict__ psi, long long line,
                                            bool active, int n, const TB *tb, int G, int t, int lane, int wl,
                                            int wpl, typename Alg<T, CPLX>::V *xs, typename Alg<T, CPLX>::V sig,
                                            T scale, T dt, T g, const PointParams &pp, int ks, bool last,
                                            typename Alg<T, CPLX>::V (&u)[C], bool keep = false)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    static_assert(SEG == 64 || (!MW && SEG >= 1 && SEG < 64 && (SEG & (SEG - 1)) == 0), "segment of a wave");
    constexpr int LOGS = SEG >= 64 ? 6 : SEG >= 32 ? 5 : SEG >= 16 ? 4 : SEG >= 8 ? 3 : SEG >= 4 ? 2 : SEG >= 2 ? 1 : 0;
    const int sl = lane & (SEG - 1);   // lane within the line's segment
    const int i0 = t * C;
    const long long base = line * (long long)n;

    // ---- pointwise substep ----
    T vyz = T(0);
    if (active) {
        const int j = (int)(line % pp.n[1]);
        const int k = (int)(line / pp.n[1]);
        const T y = coord<T>(j, pp.cen[1], pp.dx[1]);
        const T z = coord<T>(k, pp.cen[2], pp.dx[2]);
        vyz = fmaT(T(pp.w2h[2]) * z, z, T(pp.w2h[1]) * y * y);
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = i0 + k;
        const T x = coord<T>(i, pp.cen[0], pp.dx[0]);
        u[k] = apply_point<T, CPLX>(u[k], scale, fmaT(T(pp.w2h[0]) * x, x, vyz), dt, g);
    }

    // ---- neighbours across chunk boundaries ----
    // (UNR: register moves between lanes and unrolled scans; otherwise
    // LDS-crossbar shuffles in a loop over the scan depth, which keeps fewer
    // registers live -- the batched kernels, which are register-bound)
    V left = UNR ? A::shfl_up(u[C - 1], 1) : A::xshfl_up(u[C - 1], 1);
    V right = UNR ? A::shfl_down(u[0], 1) : A::xshfl_down(u[0], 1);
    if (sl == 0) left = A::zero();
    if (sl == SEG - 1) right = A::zero();
    if constexpr (MW) {
        if (lane == 0) xs[wl * 4 + 0] = u[0];
        if (lane == 63) xs[wl * 4 + 1] = u[C - 1];
        __syncthreads();
        if (lane == 0 && wl > 0) left = xs[(wl - 1) * 4 + 1];
        if (lane == 63 && wl < wpl - 1) right = xs[(wl + 1) * 4 + 0];
        __syncthreads();
    }

    // ---- m_i (1 - sT)u, and the chunk's forward map d -> Ac d + d_loc ----
    V be[C];
    V Ac = A::one(), d = A::zero();
    {
        V prev = left;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const V nxt = (k + 1 < C) ? u[k + 1] : right;
            const V r = cn_rhs<T, CPLX>(prev, u[k], nxt, sig);
            prev = u[k];
            const LTab<T, CPLX> e = row_tab<T, CPLX>(tb, k, G, t);
            be[k] = e.mmul(r);
            d = e.afma(d, be[k]);
            Ac = A::mul(e.alpha(), Ac);
        }
    }

    // ---- forward: scan of chunk maps over the preceding chunks ----
    V din;
    {
        V PA = Ac, PB = d;
        if constexpr (UNR) {
            // unrolled: each step's lane distance is a constant
#pragma unroll
            for (int s = 0; s < LOGS; ++s) {
                if (s >= ks) break;
                const int o = 1 << s;
                const V a2 = A::shfl_up(PA, o), b2 = A::shfl_up(PB, o);
                if (sl >= o) {
                    PB = A::fma(PA, b2, PB);
                    PA = A::mul(PA, a2);
                }
            }
        } else {
            for (int s = 0; s < ks; ++s) {
                const int o = 1 << s;
                const V a2 = A::xshfl_up(PA, o), b2 = A::xshfl_up(PB, o);
                if (sl >= o) {
                    PB = A::fma(PA, b2, PB);
                    PA = A::mul(PA, a2);
                }
            }
        }
        V EA = UNR ? A::shfl_up(PA, 1) : A::xshfl_up(PA, 1), EB = UNR ? A::shfl_up(PB, 1) : A::xshfl_up(PB, 1);
        if (sl == 0) {
            EA = A::one();
            EB = A::zero();
        }
        if constexpr (MW) {
            if (lane == 63) {
                xs[wl * 4 + 2] = PA;
                xs[wl * 4 + 3] = PB;
            }
            __syncthreads();
            // a truncated scan (ks < 6) reaches back fewer than 64 chunks, so
            // only the previous wave feeds this one: the earlier waves' terms
            // carry more chunk factors than the truncation keeps
            V Dw = A::zero();
            for (int q = ks < 6 ? max(0, wl - 1) : 0; q < wl; ++q) Dw = A::fma(xs[q * 4 + 2], Dw, xs[q * 4 + 3]);
            __syncthreads();
            din = A::fma(EA, Dw, EB);
        } else {
            din = EB;
        }
    }
    d = din;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        d = row_tab<T, CPLX>(tb, k, G, t).afma(d, be[k]);
        be[k] = d;
    }

    // ---- backward ----
    V v = A::zero();
#pragma unroll
    for (int k = C - 1; k >= 0; --k) v = row_tab<T, CPLX>(tb, k, G, t).afma(v, be[k]);
    V vin;
    {
        V PA = Ac, PB = v;
        if constexpr (UNR) {
#pragma unroll
            for (int s = 0; s < LOGS; ++s) {
                if (s >= ks) break;
                const int o = 1 << s;
                const V a2 = A::shfl_down(PA, o), b2 = A::shfl_down(PB, o);
                if (sl + o < SEG) {
                    PB = A::fma(PA, b2, PB);
                    PA = A::mul(PA, a2);
                }
            }
        } else {
            for (int s = 0; s < ks; ++s) {
                const int o = 1 << s;
                const V a2 = A::xshfl_down(PA, o), b2 = A::xshfl_down(PB, o);
                if (sl + o < SEG) {
                    PB = A::fma(PA, b2, PB);
                    PA = A::mul(PA, a2);
                }
            }
        }
        V EA = UNR ? A::shfl_down(PA, 1) : A::xshfl_down(PA, 1),
          EB = UNR ? A::shfl_down(PB, 1) : A::xshfl_down(PB, 1);
        if (sl == SEG - 1) {
            EA = A::one();
            EB = A::zero();
        }
        if constexpr (MW) {
            if (lane == 0) {
                xs[wl * 4 + 2] = PA;
                xs[wl * 4 + 3] = PB;
            }
            __syncthreads();
            V Vw = A::zero();
            for (int q = ks < 6 ? min(wpl - 1, wl + 1) : wpl - 1; q > wl; --q)
                Vw = A::fma(xs[q * 4 + 2], Vw, xs[q * 4 + 3]);
            __syncthreads();
            vin = A::fma(EA, Vw, EB);
        } else {
            vin = EB;
        }
    }
    v = vin;
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
        v = row_tab<T, CPLX>(tb, k, G, t).afma(v, be[k]);
        be[k] = v;
    }

    // ---- store ----
    double nacc = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = i0 + k;
        if (keep) u[k] = be[k];
        if (active && i < n) {
            if (!keep) st_elem(psi, base + i, be[k]);
            if (last) nacc += A::norm2(be[k]);
        }
    }
    return nacc;
}

// The C values of this lane's chunk of one line (zero past the end).
template <class T, bool CPLX, int C, class PV>
__device__ __forceinline__ void row_load(PV __restrict__ psi, long long line,
                                         bool active, int n, int t, typename Alg<T, CPLX>::V (&u)[C])
{
    using A = Alg<T, CPLX>;
    const int i0 = t * C;
    const long long base = line * (long long)n;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = i0 + k;
        u[k] = (active && i < n) ? ld_elem(psi, base + i) : A::zero();
    }
}

// A lane's chunk moved as 16-byte groups of 16/S values (S = 4 or 8 bytes;
// C a multiple of the group, the line length too, and an aligned state, so
// every group lies inside the line or wholly past its end): 16/S times fewer
// memory instructions than element-wise accesses strided by the chunk.
template <class T, bool CPLX, int C>
__device__ __forceinline__ void row_load_v16(const typename Alg<T, CPLX>::V *__restrict__ psi, long long line,
                                             bool active, int n, int t, typename Alg<T, CPLX>::V (&u)[C])
{
    using V = typename Alg<T, CPLX>::V;
    constexpr int PV = 16 / sizeof(V);
    static_assert(sizeof(V) <= 8 && C % PV == 0, "whole 16-byte groups");
    const int i0 = t * C;
    const float4 *q = reinterpret_cast<const float4 *>(psi + line * (long long)n + i0);
#pragma unroll
    for (int j = 0; j < C / PV; ++j) {
        float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
        if (active && i0 + PV * j < n) w = q[j];
        __builtin_memcpy(&u[PV * j], &w, 16);
    }
}

template <class T, bool CPLX, int C>
__device__ __forceinline__ void row_store_v16(typename Alg<T, CPLX>::V *__restrict__ psi, long long line,
                                              bool active, int n, int t, const typename Alg<T, CPLX>::V (&v)[C])
{
    using V = typename Alg<T, CPLX>::V;
    constexpr int PV = 16 / sizeof(V);
    const int i0 = t * C;
    float4 *q = reinterpret_cast<float4 *>(psi + line * (long long)n + i0);
#pragma unroll
    for (int j = 0; j < C / PV; ++j) {
        if (active && i0 + PV * j < n) {
            float4 w;
            __builtin_memcpy(&w, &v[PV * j], 16);
            q[j] = w;
        }
    }
}

// Coalesced ROW load and store for single-wave lines (G = 64) through a
// per-wave LDS buffer: lane l moves points k*64 + l (each wave access is one
// contiguous run), and the buffer regroups them into the lane's chunk of C
// consecutive points.  Point i sits at buf[i + i / C]: one pad slot per
// chunk, so the chunk reads of the 64 lanes spread over the banks.  The
// buffer holds C*64 + 64 values; only this wave touches it, and a wave's LDS
// accesses complete in order.
template <class T, bool CPLX, int C, class PV>
__device__ __forceinline__ void row_load_tr(PV __restrict__ psi, long long line, bool active, int n, int lane,
                                            typename Alg<T, CPLX>::V *buf, typename Alg<T, CPLX>::V (&u)[C])
{
    using A = Alg<T, CPLX>;
    const long long base = line * (long long)n;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int e = k * 64 + lane;
        buf[e + e / C] = (active && e < n) ? ld_elem(psi, base + e) : A::zero();
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < C; ++k) u[k] = buf[lane * (C + 1) + k];
}

template <class T, bool CPLX, int C, class PV>
__device__ __forceinline__ void row_store_tr(PV __restrict__ psi, long long line, bool active, int n, int lane,
                                             typename Alg<T, CPLX>::V *buf, const typename Alg<T, CPLX>::V (&v)[C])
{
    const long long base = line * (long long)n;
#pragma unroll
    for (int k = 0; k < C; ++k) buf[lane * (C + 1) + k] = v[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int e = k * 64 + lane;
        if (active && e < n) st_elem(psi, base + e, buf[e + e / C]);
    }
}

// The C values of this lane's chunk back to the line (the store of row_solve).
template <class T, bool CPLX, int C, class PV>
__device__ __forceinline__ void row_store(PV __restrict__ psi, long long line, bool active, int n, int t,
                                          const typename Alg<T, CPLX>::V (&v)[C])
{
    const int i0 = t * C;
    const long long base = line * (long long)n;
#pragma unroll
    for (int k = 0; k < C; ++k)
        if (active && i0 + k < n) st_elem(psi, base + i0 + k, v[k]);
}

template <class T, bool CPLX, int C, bool MW, bool UNR = true, class TB, class PV>
__device__ __forceinline__ double row_line(PV __restrict__ psi, long long line,
                                           bool active, int n, const TB *tb, int G, int t, int lane, int wl,
                                           int wpl, typename Alg<T, CPLX>::V *xs, typename Alg<T, CPLX>::V sig,
                                           T scale, T dt, T g, const PointParams &pp, int ks, bool last)
{
    typename Alg<T, CPLX>::V u[C];
    row_load<T, CPLX, C>(psi, line, active, n, t, u);
    return row_solve<T, CPLX, C, MW, UNR, 64, TB, PV>(psi, line, active, n, tb, G, t, lane, wl, wpl, xs, sig, scale, dt,
                                                  g, pp, ks, last, u);
}

// ---------------------------------------------------------------------------
// COL: one tile of LPB = 64/L lines, nch = W*L chunks per line.  `line` and
// `base` are this lane's line and its first point; tb is the staged table;
// xs0/xs1 hold nch x LPB values each.  Returns sum |v|^2 when `last`.
// col_load / col_solve split it like row_load / row_solve.
// ---------------------------------------------------------------------------
template <class T, bool CPLX, int C, class PV>
__device__ __forceinline__ double col_solve(PV __restrict__ psi, bool active,
                                            long long base, int n, long long st, int nch, int ch, int LPB, int li,
                                            const LTab<T, CPLX> *tb, typename Alg<T, CPLX>::V *xs0,
                                            typename Alg<T, CPLX>::V *xs1, typename Alg<T, CPLX>::V sig, int depth,
                                            bool last, typename Alg<T, CPLX>::V (&u)[C])
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const int i0 = ch * C;
    const int qlo = max(0, ch - depth);
    const int qhi = min(nch - 1, ch + depth);

    // neighbours from the adjacent chunks
    xs0[ch * LPB + li] = u[0];
    xs1[ch * LPB + li] = u[C - 1];
    __syncthreads();
    const V left = (ch > 0) ? xs1[(ch - 1) * LPB + li] : A::zero();
    const V right = (ch + 1 < nch) ? xs0[(ch + 1) * LPB + li] : A::zero();
    __syncthreads();

    V be[C];
    V Ac = A::one(), d = A::zero();
    {
        V prev = left;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const V nxt = (k + 1 < C) ? u[k + 1] : right;
            const V r = cn_rhs<T, CPLX>(prev, u[k], nxt, sig);
            prev = u[k];
            const LTab<T, CPLX> e = tab_at<T, CPLX>(tb, i0 + k);
            be[k] = e.mmul(r);
            d = e.afma(d, be[k]);
            Ac = A::mul(e.alpha(), Ac);
        }
    }
    xs0[ch * LPB + li] = Ac;
    xs1[ch * LPB + li] = d;
    __syncthreads();
    V din = A::zero();
    for (int q = qlo; q < ch; ++q) din = A::fma(xs0[q * LPB + li], din, xs1[q * LPB + li]);
    __syncthreads();
    d = din;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        d = tab_at<T, CPLX>(tb, i0 + k).afma(d, be[k]);
        be[k] = d;
    }

    // backward
    V v = A::zero();
#pragma unroll
    for (int k = C - 1; k >= 0; --k) v = tab_at<T, CPLX>(tb, i0 + k).afma(v, be[k]);
    xs1[ch * LPB + li] = v;
    __syncthreads();
    V vin = A::zero();
    for (int q = qhi; q > ch; --q) vin = A::fma(xs0[q * LPB + li], vin, xs1[q * LPB + li]);
    v = vin;
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
        v = tab_at<T, CPLX>(tb, i0 + k).afma(v, be[k]);
        be[k] = v;
    }
    double nacc = 0.0;
    if (active && i0 + C <= n) {
        // a whole chunk: one address, stepped by the stride
        PV p = psi + (base + (long long)i0 * st);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            st_elem(p, 0, be[k]);
            if (last) nacc += A::norm2(be[k]);
            p += st;
        }
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int i = i0 + k;
            if (active && i < n) {
                st_elem(psi, base + (long long)i * st, be[k]);
                if (last) nacc += A::norm2(be[k]);
            }
        }
    }
    return nacc;
}

// The C values of chunk ch of this lane's line (zero past the end).
template <class T, bool CPLX, int C, class PV>
__device__ __forceinline__ void col_load(PV __restrict__ psi, bool active,
                                         long long base, int n, long long st, int ch,
                                         typename Alg<T, CPLX>::V (&u)[C])
{
    using A = Alg<T, CPLX>;
    const int i0 = ch * C;
    if (active && i0 + C <= n) {
        // a whole chunk: one address, stepped by the stride
        PV p = psi + (base + (long long)i0 * st);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            u[k] = ld_elem(p, 0);
            p += st;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int i = i0 + k;
        u[k] = (active && i < n) ? ld_elem(psi, base + (long long)i * st) : A::zero();
    }
}

template <class T, bool CPLX, int C, class PV>
__device__ __forceinline__ double col_tile(PV __restrict__ psi, bool active,
                                           long long base, int n, long long st, int nch, int ch, int LPB, int li,
                                           const LTab<T, CPLX> *tb, typename Alg<T, CPLX>::V *xs0,
                                           typename Alg<T, CPLX>::V *xs1, typename Alg<T, CPLX>::V sig, int depth,
                                           bool last)
{
    typename Alg<T, CPLX>::V u[C];
    col_load<T, CPLX, C>(psi, active, base, n, st, ch, u);
    return col_solve<T, CPLX, C>(psi, active, base, n, st, nch, ch, LPB, li, tb, xs0, xs1, sig, depth, last, u);
}

}  // namespace sscn

// sscn_batch.hip -- batched persistent SSCN step on gfx950 (FP32 forms).
//
// One launch advances every running instance of the batch by one step (the
// ordering and waiting scheme is described in sscn_batch.hpp).  Work items:
//   x tile    ROW line solve (pointwise substep + pending scale fused)
//   y/z tile  COL line solve; the last sweep writes one FP64 norm partial
//   obs tile  FP64 sums of the observables over a block of points, on
//             observation steps only
//   fin       fixed-order sums -> renormalisation factor, mu, E, the
//             convergence test and the instance's step count
// The line solves are those of the single-problem kernels (sscn_lines.hpp).
#include "sscn_batch.hpp"
#include "sscn_lines.hpp"

namespace sscn {

// Pointers the kernel reads from the instance table are generic, and a
// generic access is a flat instruction, which counts against the LDS
// counter as well: every LDS wait of the line solve would then also wait for
// the state loads in flight.  They all point to device memory, so they are
// used as global pointers (the compiler then emits global loads and stores).
template <class P>
using GP = __attribute__((address_space(1))) P *;
// The instance table and the work list are written by the host only (at
// admission and when the list is rebuilt) and read-only during a launch, so
// they are read through the constant address space: with a wave-uniform
// index the compiler loads the sweep's descriptors with scalar loads into
// scalar registers, which leaves the vector registers to the line solve.
#if defined(__HIP_DEVICE_COMPILE__)
template <class P>
using KP = const __attribute__((address_space(4))) P *;
#else
// the host pass only parses device code; it has no constant address space
template <class P>
using KP = const P *;
#endif

// ---------------------------------------------------------------------------
// items
// ---------------------------------------------------------------------------
template <class T, bool CPLX, int C, bool MW>
__device__ __forceinline__ void batch_row(KP<BInst> Ik, const BState &S, int tile, unsigned char *lds,
                                          double *red, bool last)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const BAxis X = Ik->ax[0];
    const GP<const TabEntry> tab = (GP<const TabEntry>)X.lt.tab;
    const PointParams pp = Ik->pp;
    const int G = MW ? 64 * X.wpl : 64;
    const int tid = threadIdx.x;
    const int lb = tid / G;
    const int t = tid - lb * G;
    const int lane = tid & 63;
    const int wl = t >> 6;
    LTab<T, CPLX> *tl = reinterpret_cast<LTab<T, CPLX> *>(lds);
    V *xs = reinterpret_cast<V *>(lds) + lb * X.wpl * 4;
    if constexpr (!MW) {
        stage_table_from<T, CPLX>(X.lt, tab, tl, C * 64, 64, C);
        __syncthreads();
    }
    const V sig = A::coef(X.sig_re, X.sig_im);
    const T scale = CPLX ? T(1) : T(S.scale);
    const GP<V> psi = (GP<V>)Ik->psi;
    const GP<double> norm_part = (GP<double>)Ik->norm_part;
    double nacc = 0.0;
    const long long line0 = (long long)tile * X.rep * X.lpi + lb;
    if constexpr (MW) {
        for (int r = 0; r < X.rep; ++r) {
            const long long line = line0 + (long long)r * X.lpi;
            nacc += row_line<T, CPLX, C, true, false>(psi, line, line < X.nlines, X.lt.n, tab, G, t, lane, wl, X.wpl,
                                               xs, sig, scale, T(pp.dt), T(pp.g), pp, X.lt.depth, last);
        }
    } else {
        // one block runs an item, so the loads of the next line group are
        // issued before the current one is solved (when the extra
        // registers are few): memory latency overlaps the solve
        constexpr bool PF = C * sizeof(V) <= 32;
        V u[C];
        row_load<T, CPLX, C>(psi, line0, line0 < X.nlines, X.lt.n, t, u);
        for (int r = 0; r < X.rep; ++r) {
            const long long line = line0 + (long long)r * X.lpi;
            V nx[C];
            if constexpr (PF) {
                if (r + 1 < X.rep) row_load<T, CPLX, C>(psi, line + X.lpi, line + X.lpi < X.nlines, X.lt.n, t, nx);
            } else if (r > 0) {
                row_load<T, CPLX, C>(psi, line, line < X.nlines, X.lt.n, t, u);
            }
            nacc += row_solve<T, CPLX, C, false, false>(psi, line, line < X.nlines, X.lt.n,
                                                 static_cast<const LTab<T, CPLX> *>(tl), G, t, lane, wl, 1, xs, sig,
                                                 scale, T(pp.dt), T(pp.g), pp, X.lt.depth, last, u);
            if constexpr (PF) {
#pragma unroll
                for (int k = 0; k < C; ++k) u[k] = nx[k];
            }
        }
    }
    if (last) {
        const double s = block_sum(nacc, red);
        if (tid == 0) norm_part[tile] = s;
    }
}

template <class T, bool CPLX, int C>
__device__ __forceinline__ void batch_col(KP<BInst> Ik, int axis, int tile, unsigned char *lds, double *red,
                                          bool last)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const BAxis X = Ik->ax[axis];
    const GP<const TabEntry> tab = (GP<const TabEntry>)X.lt.tab;
    const GP<double> norm_part = (GP<double>)Ik->norm_part;
    const int L = X.L, W = X.W;
    const int LPB = 64 / L;
    const int nch = W * L;
    const int wave = threadIdx.x >> 6;
    const int st_i = wave / W;          // sub-tile of this wave
    const int w = wave - st_i * W;
    const int lane = threadIdx.x & 63;
    const int sub = lane / LPB;
    const int li = lane - sub * LPB;
    const int ch = w * L + sub;
    LTab<T, CPLX> *tb = reinterpret_cast<LTab<T, CPLX> *>(lds);
    V *xs0 = reinterpret_cast<V *>(tb + nch * C) + st_i * (2 * nch * LPB);
    V *xs1 = xs0 + nch * LPB;
    stage_table_from<T, CPLX>(X.lt, tab, tb, nch * C, 0, C);
    const GP<V> psi = (GP<V>)Ik->psi;
    // this lane's line in set r, and its first point
    auto line_of = [&](int r) { return (((long long)tile * X.rep + r) * X.tpi + st_i) * LPB + li; };
    auto base_of = [&](long long line) {
        return line < X.nlines ? (line % X.m1) * X.s1 + (line / X.m1) * X.s2 : 0LL;
    };
    // loads of the next set are issued before the current set is solved
    // when the extra registers are few (see batch_row)
    constexpr bool PF = C * sizeof(V) <= 32;
    double nacc = 0.0;
    V u[C];
    {
        const long long l0 = line_of(0);
        col_load<T, CPLX, C>(psi, l0 < X.nlines, base_of(l0), X.lt.n, X.stride, ch, u);
    }
    for (int r = 0; r < X.rep; ++r) {
        const long long line = line_of(r);
        const bool active = line < X.nlines;
        const long long base = base_of(line);
        V nx[C];
        if constexpr (PF) {
            if (r + 1 < X.rep) {
                const long long ln = line_of(r + 1);
                col_load<T, CPLX, C>(psi, ln < X.nlines, base_of(ln), X.lt.n, X.stride, ch, nx);
            }
        } else if (r > 0) {
            col_load<T, CPLX, C>(psi, active, base, X.lt.n, X.stride, ch, u);
        }
        // the previous set's last LDS reads finish before the next set's writes
        if (r > 0) __syncthreads();
        nacc += col_solve<T, CPLX, C>(psi, active, base, X.lt.n, X.stride, nch, ch, LPB, li, tb, xs0, xs1,
                                      A::coef(X.sig_re, X.sig_im), X.lt.depth, last, u);
        if constexpr (PF) {
#pragma unroll
            for (int k = 0; k < C; ++k) u[k] = nx[k];
        }
    }
    if (last) {
        const double s = block_sum(nacc, red);
        if (threadIdx.x == 0) norm_part[tile] = s;
    }
}

__device__ __forceinline__ bool batch_observes(const BInst &I, const BState &S)
{
    const int64_t s = S.step + 1;
    return (s % I.observe_every) == 0 || s >= I.max_steps;
}

// FP64 sums over one tile of points: q, kinetic edges, V q, q^2, x_a q, x_a^2 q.
template <class T, bool CPLX>
__device__ __forceinline__ void batch_obs(const BInst &I, const BState &S, int tile, double (*redq)[16])
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    if (!batch_observes(I, S)) return;
    const GP<const V> psi = (GP<const V>)I.psi;
    const PointParams pp = I.pp;
    const int dim = I.dim;
    const long long npts = I.npts;
    const GP<double> obs_part = (GP<double>)I.obs_part;
    const long long nx = pp.n[0], ny = pp.n[1];
    const int n3[3] = {pp.n[0], pp.n[1], pp.n[2]};
    const long long sx[3] = {1, nx, nx * ny};
    double acc[BATCH_NOBS];
#pragma unroll
    for (int q = 0; q < BATCH_NOBS; ++q) acc[q] = 0.0;
    double inv2[3];                       // 1 / dx_a^2
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) inv2[ax] = ax < dim ? 1.0 / (pp.dx[ax] * pp.dx[ax]) : 0.0;
    // grid indices of a point: two divisions, in 32 bits when the point
    // count allows (64-bit divisions are long instruction sequences)
    const bool narrow = npts < (1LL << 31);
    const long long p0 = (long long)tile * I.obs_pts;
    const long long p1 = min(npts, p0 + (long long)I.obs_pts);
    for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        int idx[3];
        if (dim == 1) {
            idx[0] = (int)p;
            idx[1] = idx[2] = 0;
        } else if (narrow) {
            const unsigned up = (unsigned)p, r = up / (unsigned)nx, r2 = r / (unsigned)ny;
            idx[0] = (int)(up - r * (unsigned)nx);
            idx[1] = (int)(r - r2 * (unsigned)ny);
            idx[2] = (int)r2;
        } else {
            const long long r = p / nx, r2 = r / ny;
            idx[0] = (int)(p - r * nx);
            idx[1] = (int)(r - r2 * ny);
            idx[2] = (int)r2;
        }
        const V v = ld_elem(psi, p);
        const double q = A::norm2(v);
        double vp = 0.0, kin = 0.0;
        // unrolled over the three axes so that every index is static (the
        // arrays stay in registers); explicit FMAs fix the rounding
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (ax >= dim) break;
            const double x = (double(idx[ax]) - pp.cen[ax]) * pp.dx[ax];
            vp = fmaT(pp.w2h[ax] * x, x, vp);
            acc[4 + ax] = fmaT(x, q, acc[4 + ax]);
            acc[7 + ax] = fmaT(x * x, q, acc[7 + ax]);
            const V nb = (idx[ax] + 1 < n3[ax]) ? ld_elem(psi, p + sx[ax]) : A::zero();
            double e = A::norm2(A::sub(nb, v));
            if (idx[ax] == 0) e += q;
            kin = fmaT(e, inv2[ax], kin);
        }
        acc[0] += q;
        acc[1] += kin;
        acc[2] = fmaT(vp, q, acc[2]);
        acc[3] = fmaT(q, q, acc[3]);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < BATCH_NOBS; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) redq[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < BATCH_NOBS) {
        const int q = threadIdx.x;
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += redq[q][w];
        obs_part[(size_t)tile * BATCH_NOBS + q] = s;
    }
}

// The finalisation arithmetic of one step, given the step's raw norm sum
// and, on observation steps, the observation sums (thread 0 only).  S may be
// the instance state in memory or a copy of it in LDS.
__device__ __forceinline__ void fin_core(const BInst &I, BState &S, double nraw, const double *tot, bool obs_now)
{
    const double dv = I.dvol;
    const double N = dv * nraw;
    const double s = I.imag ? 1.0 / sqrt(N) : 1.0;   // renormalisation every step in imaginary time
    int32_t status = S.status;
    if (!__builtin_isfinite(N) || !(N > 0.0)) status = BS_NONFINITE;
    if (obs_now && status == BS_RUNNING) {
        // observables of the step's state, renormalised in imaginary time:
        // K and P scale with s^2, I with s^4, the norm with s^2
        const double s2 = s * s;
        const double Nq = dv * tot[0] * s2;
        const double K = 0.5 * dv * tot[1] * s2;
        const double P = dv * tot[2] * s2;
        const double In = dv * tot[3] * s2 * s2;
        const double g = I.pp.g;
        const double mu = fmaT(g, In, K + P) / Nq;
        S.obs[0] = Nq;
        S.obs[1] = mu;
        S.obs[2] = fmaT(0.5 * g, In, K + P) / Nq;
        S.obs[3] = K;
        S.obs[4] = P;
        S.obs[5] = In;
        for (int ax = 0; ax < 3; ++ax) {
            S.obs[6 + ax] = dv * tot[4 + ax] * s2 / Nq;
            S.obs[9 + ax] = dv * tot[7 + ax] * s2 / Nq;
        }
        S.obs_step = S.step + 1;
        if (!__builtin_isfinite(mu)) {
            status = BS_NONFINITE;
        } else if (I.mu_tol > 0.0 && ((S.step + 1) % I.observe_every) == 0) {
            if (S.have_prev && fabs(mu - S.mu_prev) < I.mu_tol) status = BS_CONVERGED;
            S.mu_prev = mu;
            S.have_prev = 1;
        }
    }
    S.norm = N;
    S.scale = s;
    S.step += 1;
    if (status == BS_RUNNING && S.step >= I.max_steps) status = BS_DONE;
    S.status = status;
}

// Finalisation of one instance's step (one block).
__device__ __forceinline__ void batch_fin(const BInst &I, BState &S, double *red)
{
    const int nt = I.ax[I.last_pass].ntiles;
    const bool obs_now = batch_observes(I, S);
    const GP<const double> norm_part = (GP<const double>)I.norm_part;
    const GP<const double> obs_part = (GP<const double>)I.obs_part;
    double nraw = 0.0;
    double tot[BATCH_NOBS];
    for (int q = 0; q < BATCH_NOBS; ++q) tot[q] = 0.0;
    // one partial: thread 0 takes it as it is (the block sum would add
    // exact zeros to it); several: fixed-order block sums
    if (nt == 1) {
        if (threadIdx.x == 0) nraw = norm_part[0];
    } else {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nt; i += blockDim.x) acc += norm_part[i];
        nraw = block_sum(acc, red);
    }
    if (obs_now) {
        if (I.obs_tiles == 1) {
            if (threadIdx.x == 0)
                for (int q = 0; q < BATCH_NOBS; ++q) tot[q] = obs_part[q];
        } else {
            for (int q = 0; q < BATCH_NOBS; ++q) {
                double a = 0.0;
                for (int i = threadIdx.x; i < I.obs_tiles; i += blockDim.x)
                    a += obs_part[(size_t)i * BATCH_NOBS + q];
                tot[q] = block_sum(a, red);
            }
        }
    }
    if (threadIdx.x == 0) fin_core(I, S, nraw, tot, obs_now);
}

// ---------------------------------------------------------------------------
// solo instances: whole steps of one 1D line inside one block
// ---------------------------------------------------------------------------
// The ROW table of a solo line (a row_tab overload): a head (i < i_conv), a
// constant tail entry and zeros past the line end.  The waves that hold head
// entries or the line end read their entries from an LDS copy in the
// lane-major order (p = the lane's first slot, entry k at p[k*64]); every
// other wave uses one entry for all its points (the tail, or zero past the
// line end), chosen per wave, so it reads no memory for its table.
template <class T, bool CPLX>
struct EdgeTab {
    const LTab<T, CPLX> *p;
    int uniform;                 // the same for all lanes of the wave
    LTab<T, CPLX> e;             // the entry of a uniform wave
};

template <class T, bool CPLX>
__device__ __forceinline__ LTab<T, CPLX> row_tab(const EdgeTab<T, CPLX> *tb, int k, int, int)
{
    if (tb->uniform) return tb->e;
    return tb->p[k * 64];
}

// A solo instance's steps with its line in registers for the whole call:
// the state is read once and written once (and on observation steps), the
// table is an EdgeTab (LDS entries for the first wave and the line-end wave,
// one entry for each other wave), the norm and the finalisation pass through
// LDS between block barriers, and thread 0 keeps the instance state in LDS
// (sS), writing it back at the end.  Each
// step is the split items' line solve, observation sums and finalisation,
// so the results are theirs bit for bit.  Runs `steps` steps, fewer if the
// instance stops or (target >= 0) once the persistent launches that run
// beside it have all finished (BCtl::reg_epoch reaches target).
// block_sum without its leading barrier.  In the solo step loop the last
// reads of red (thread 0, in the previous step) come before that step's
// closing barrier, which every wave passes before it writes red again.
__device__ __forceinline__ double block_sum_after_barrier(double v, double *red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += red[w];
    }
    return s;
}

template <class T, bool CPLX, int C, bool MW>
__device__ void solo_run(const BInst &I, BState &S, BState &sS, int steps, int target, BCtl *ctl,
                         unsigned char *lds, double *red, double (*redq)[16], int *s_go)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    const BAxis X = I.ax[0];
    const PointParams pp = I.pp;
    const GP<const TabEntry> tab = (GP<const TabEntry>)X.lt.tab;
    const GP<V> psi = (GP<V>)I.psi;
    const int G = MW ? 64 * X.wpl : 64;
    const int tid = threadIdx.x;
    const int lb = tid / G;
    const int t = tid - lb * G;
    const int lane = tid & 63;
    const int wl = t >> 6;
    const bool active = lb == 0;          // the line is line 0 of group 0
    const int n = X.lt.n;
    // table entries: wave 0 (the head, i < i_conv <= 64*C) and the wave that
    // holds the line end read an LDS copy of their entries (slots 0 and 1,
    // lane-major); the waves between read the tail entry, those past the end
    // a zero entry, without memory accesses
    const int W = MW ? X.wpl : 1;
    const int span = 64 * C;                   // points per wave
    const int wb = n / span;                   // the wave holding the line end (== W: none)
    const int nslot = (W > 1 && wb < W) ? 2 : 1;
    const LTab<T, CPLX> tail = LTab<T, CPLX>::make(TabEntry{X.lt.ac_re, X.lt.ac_im, X.lt.mc_re, X.lt.mc_im});
    const LTab<T, CPLX> zero = LTab<T, CPLX>::make(TabEntry{0.0, 0.0, 0.0, 0.0});
    LTab<T, CPLX> *etab = reinterpret_cast<LTab<T, CPLX> *>(lds);
    V *xs = reinterpret_cast<V *>(etab + nslot * span) + lb * X.wpl * 4;
    for (int q = tid; q < nslot * span; q += blockDim.x) {
        const int slot = q / span, r = q - slot * span;
        const int i = ((slot == 0 ? 0 : wb) * 64 + (r & 63)) * C + (r >> 6);
        LTab<T, CPLX> e = tail;
        if (i >= n) e = zero;
        else if (i < X.lt.i_conv) e = LTab<T, CPLX>::make(ld_tab(tab, (i % C) * G + i / C));  // lane-major: k*G + t
        etab[q] = e;
    }
    EdgeTab<T, CPLX> ht;
    {
        int slot = -1;
        if (active && wl == 0) slot = 0;
        else if (active && wl == wb) slot = 1;
        ht.uniform = __builtin_amdgcn_readfirstlane(slot < 0 ? 1 : 0);
        ht.p = etab + (slot < 0 ? 0 : slot) * span + lane;
        ht.e = (!active || wl > wb) ? zero : tail;
    }
    const V sig = A::coef(X.sig_re, X.sig_im);
    const GP<const double> obs_part = (GP<const double>)I.obs_part;
    auto store_line = [&](const V (&v)[C]) {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int i = t * C + k;
            if (active && i < n) st_elem(psi, (long long)i, v[k]);
        }
    };
    V u[C];
    row_load<T, CPLX, C>(psi, 0, active, n, t, u);
    if (tid == 0) sS = S;
    __syncthreads();
    for (int k = 1;; ++k) {
        // the launch count is read early: its latency overlaps the step
        int re = 0;
        if (target >= 0 && tid == 0) re = __hip_atomic_load(&ctl->reg_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const T scale = CPLX ? T(1) : T(sS.scale);
        const bool obs_now = batch_observes(I, sS);
        // a single-wave line reads its staged table directly (slot 0 is the
        // whole lane-major table), as the persistent kernel's x item does:
        // through the per-wave form the compiler rounded some lines of few
        // points per thread differently (last-bit differences, measured)
        double nacc;
        if constexpr (MW)
            nacc = row_solve<T, CPLX, C, MW, true>(psi, 0, active, n, &ht, G, t, lane, wl, X.wpl, xs, sig, scale, T(pp.dt),
                                             T(pp.g), pp, X.lt.depth, true, u, true);
        else
            nacc = row_solve<T, CPLX, C, MW, true>(psi, 0, active, n, static_cast<const LTab<T, CPLX> *>(etab), G, t, lane,
                                             wl, X.wpl, xs, sig, scale, T(pp.dt), T(pp.g), pp, X.lt.depth, true, u,
                                             true);
        const double nraw = block_sum_after_barrier(nacc, red);
        if (obs_now) {
            // the observation item's own sums over the stored line, so the
            // observables are those of the split items bit for bit
            store_line(u);
            __syncthreads();
            batch_obs<T, CPLX>(I, sS, 0, redq);
            __syncthreads();
        }
        if (tid == 0) {
            double tot[BATCH_NOBS];
            for (int q = 0; q < BATCH_NOBS; ++q) tot[q] = obs_now ? obs_part[q] : 0.0;
            fin_core(I, sS, nraw, tot, obs_now);
            *s_go = sS.status == BS_RUNNING && k < steps && (target < 0 || (int)((unsigned)re - (unsigned)target) < 0);
        }
        __syncthreads();
        if (!*s_go) break;
    }
    store_line(u);
    if (tid == 0) S = sS;
}

// The register-resident solo steps of an instance; false (nothing done) if
// its geometry has none.
template <bool BIG>
__device__ __forceinline__ bool solo_fast(const BInst &I, BState &S, BState &sS, int steps, int target, BCtl *ctl,
                                         unsigned char *lds, double *red, double (*redq)[16], int *s_go)
{
    const BAxis &X = I.ax[0];
    if (min(X.lt.i_conv, X.lt.n) > BATCH_SOLO_HEAD || X.lt.i_conv > 64 * X.C) return false;
#define SOLO(CPLX, C, MW) solo_run<float, CPLX, C, MW>(I, S, sS, steps, target, ctl, lds, red, redq, s_go)
    if (I.elem == 1) {
        if (X.wpl > 1) {
            switch (X.C) {
            case 8: SOLO(false, 8, true); return true;
            case 12:
                if constexpr (BIG) { SOLO(false, 12, true); return true; }
                return false;
            case 16:
                if constexpr (BIG) { SOLO(false, 16, true); return true; }
                return false;
            default: return false;
            }
        }
        switch (X.C) {
        case 1: SOLO(false, 1, false); return true;
        case 2: SOLO(false, 2, false); return true;
        case 3: SOLO(false, 3, false); return true;
        case 4: SOLO(false, 4, false); return true;
        case 6: SOLO(false, 6, false); return true;
        case 8: SOLO(false, 8, false); return true;
        case 12: SOLO(false, 12, false); return true;
        case 16: SOLO(false, 16, false); return true;
        default: return false;
        }
    }
    if (X.wpl > 1) {
        // complex lines of 16 points per thread need more registers than a
        // 1024-thread block has (they spill): those run the persistent
        // kernel's solo cycle
        if (X.C == 8) {
            SOLO(true, 8, true);
            return true;
        }
        return false;
    }
    switch (X.C) {
    case 1: SOLO(true, 1, false); return true;
    case 2: SOLO(true, 2, false); return true;
    case 3: SOLO(true, 3, false); return true;
    case 4: SOLO(true, 4, false); return true;
    case 6: SOLO(true, 6, false); return true;
    case 8: SOLO(true, 8, false); return true;
    default: return false;
    }
#undef SOLO
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
// FULL: every x-line form; otherwise only those of 2D and 3D instances (at
// most 4 points per thread: one wave, or 4 per thread over several waves),
// which leaves the kernel far fewer registers to spill.  Returns false when
// the item's form is not in this kernel.
template <class T, bool CPLX, bool BIG, bool FULL>
__device__ __forceinline__ bool batch_sweep(KP<BInst> I, const BState &S, int pass, int tile, unsigned char *lds,
                                            double *red)
{
    const bool last = pass == I->last_pass;
    const BAxis X = I->ax[pass];
    bool done = true;
    if (pass == BP_X) {
        if (X.wpl > 1) {
            switch (X.C) {
            case 4: batch_row<T, CPLX, 4, true>(I, S, tile, lds, red, last); break;
            case 8:
                if constexpr (FULL) batch_row<T, CPLX, 8, true>(I, S, tile, lds, red, last);
                else done = false;
                break;
            case 12:
                if constexpr (FULL && BIG && !CPLX) batch_row<T, CPLX, 12, true>(I, S, tile, lds, red, last);
                else done = false;
                break;
            case 16:
                if constexpr (FULL && BIG) batch_row<T, CPLX, 16, true>(I, S, tile, lds, red, last);
                else done = false;
                break;
            default: done = false; break;
            }
        } else {
            switch (X.C) {
            case 1: batch_row<T, CPLX, 1, false>(I, S, tile, lds, red, last); break;
            case 2: batch_row<T, CPLX, 2, false>(I, S, tile, lds, red, last); break;
            case 3: batch_row<T, CPLX, 3, false>(I, S, tile, lds, red, last); break;
            case 4: batch_row<T, CPLX, 4, false>(I, S, tile, lds, red, last); break;
            case 6:
                if constexpr (FULL) batch_row<T, CPLX, 6, false>(I, S, tile, lds, red, last);
                else done = false;
                break;
            case 8:
                if constexpr (FULL) batch_row<T, CPLX, 8, false>(I, S, tile, lds, red, last);
                else done = false;
                break;
            case 12:
                if constexpr (FULL && !CPLX) batch_row<T, CPLX, 12, false>(I, S, tile, lds, red, last);
                else done = false;
                break;
            case 16:
                if constexpr (FULL && !CPLX) batch_row<T, CPLX, 16, false>(I, S, tile, lds, red, last);
                else done = false;
                break;
            default: done = false; break;
            }
        }
    } else {
        switch (X.C) {
        case 2: batch_col<T, CPLX, 2>(I, pass, tile, lds, red, last); break;
        case 3: batch_col<T, CPLX, 3>(I, pass, tile, lds, red, last); break;
        case 4: batch_col<T, CPLX, 4>(I, pass, tile, lds, red, last); break;
        case 5: batch_col<T, CPLX, 5>(I, pass, tile, lds, red, last); break;
        case 6: batch_col<T, CPLX, 6>(I, pass, tile, lds, red, last); break;
        case 8: batch_col<T, CPLX, 8>(I, pass, tile, lds, red, last); break;
        case 10:
            if constexpr (!CPLX) batch_col<T, CPLX, 10>(I, pass, tile, lds, red, last);
            break;
        case 12:
            if constexpr (!CPLX) batch_col<T, CPLX, 12>(I, pass, tile, lds, red, last);
            break;
        case 16:
            if constexpr (BIG && !CPLX) batch_col<T, CPLX, 16>(I, pass, tile, lds, red, last);
            else done = false;
            break;
        default: done = false; break;
        }
    }
    return done;
}

// BIG adds the variants for 1D lines longer than 8192 points (12 or 16
// points per thread over the whole block) and y/z chunks of 16, whose
// registers the other paths do not need.  FULL adds the x-line forms of 1D
// instances (and the solo cycle); the host launches the other form when the
// list holds only 2D and 3D items with at most 4 points per thread on x
// (an item outside the form sets error bit 2 instead of running).
template <bool BIG, bool FULL>
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch_step(BatchArgs a)
{
    extern __shared__ unsigned char lds_raw[];
    __shared__ double red[16];
    __shared__ double redq[BATCH_NOBS][16];
    __shared__ int s_item;
    __shared__ int s_go;
    const int total = a.ctl->total_items;
    const int solo_min = a.ctl->solo_min;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(&a.ctl->ticket, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= total) break;
        const BItem w = ((KP<BItem>)a.items)[it];
        const BInst &I = a.inst[w.slot];
        BState &S = a.state[w.slot];
        if (S.status != BS_RUNNING) continue;
        const bool solo = w.pass == BP_SOLO;
        if (!FULL && solo) {
            if (threadIdx.x == 0) atomicOr(&a.ctl->error, 4);
            continue;
        }

        // wait until the instance's previous pass has completed (bounded)
        const int dep = solo ? -1 : I.dep[w.pass];
        if (dep >= 0) {
            if (threadIdx.x == 0) {
                int32_t *cnt = a.done + (size_t)w.slot * 4 + dep;
                const int32_t need = I.need[w.pass];
                int spins = 0;
                // bounded: after spin_limit polls (or once any wait of the
                // launch has given up) the item proceeds and the error flag
                // marks the launch's results invalid.  The polls are relaxed
                // (an acquire load would invalidate the caches on every
                // poll, under the feet of the other blocks); one acquire
                // fence after the count is reached orders the item's reads
                // after the producers' releases.
                while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    ++spins;
                    if (spins > a.spin_limit ||
                        ((spins & 1023) == 0 &&
                         __hip_atomic_load(&a.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                        atomicOr(&a.ctl->error, 1);
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            // thread 0's acquire invalidated this CU's caches; the barrier
            // orders the other waves' reads after it
            __syncthreads();
        }

        // A solo item cycles x solve -> observation -> finalisation of its
        // single tile, whole steps in a row, with block barriers in place of
        // the counters (the block's waves share one CU, so a barrier orders
        // their global stores and loads).  It repeats while the instance
        // runs, up to BATCH_SOLO_MAX steps, and past solo_min steps only
        // while items of the launch are still unclaimed.
        int pass = solo ? BP_X : w.pass;
        for (int k = 1;;) {
            if (pass <= BP_Z) {
                KP<BInst> Ik = (KP<BInst>)a.inst + w.slot;
                const bool ok = I.elem == 1 ? batch_sweep<float, false, BIG, FULL>(Ik, S, pass, w.tile, lds_raw, red)
                                            : batch_sweep<float, true, BIG, FULL>(Ik, S, pass, w.tile, lds_raw, red);
                if (!ok && threadIdx.x == 0) atomicOr(&a.ctl->error, 4);
            } else if (pass == BP_OBS) {
                if (I.elem == 1) batch_obs<float, false>(I, S, w.tile, redq);
                else batch_obs<float, true>(I, S, w.tile, redq);
            } else {
                batch_fin(I, S, red);
            }
            if (!solo) break;
            __syncthreads();
            if (pass == BP_FIN) {
                if (threadIdx.x == 0) {
                    bool go = S.status == BS_RUNNING && k < BATCH_SOLO_MAX;
                    if (go && k >= solo_min)
                        go = __hip_atomic_load(&a.ctl->ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < total;
                    s_go = go ? 1 : 0;
                }
                __syncthreads();
                if (!s_go) break;
                ++k;
            }
            pass = pass == BP_X ? BP_OBS : pass == BP_OBS ? BP_FIN : BP_X;
        }

        if (w.pass < BP_FIN) {
            // the barrier makes every wave's stores visible to thread 0, whose
            // agent-scope release (one L2 write-back per item) publishes them
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(a.done + (size_t)w.slot * 4 + w.pass, 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // the last block out resets the counters for the next launch and sets
    // solo_min from whether any instance other than a solo one still runs
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int prev = atomicAdd(&a.ctl->exited, 1);
        s_go = prev == (int)gridDim.x - 1;
        if (s_go) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!s_go) return;
    const int ns = a.ctl->max_slots;
    int regular = 0;
    for (int q = threadIdx.x; q < ns; q += blockDim.x) {
        a.done[4 * q + 0] = 0;
        a.done[4 * q + 1] = 0;
        a.done[4 * q + 2] = 0;
        a.done[4 * q + 3] = 0;
        if (a.state[q].status == BS_RUNNING && !a.inst[q].solo) regular = 1;
    }
    regular = __syncthreads_or(regular);
    if (threadIdx.x == 0) {
        a.ctl->solo_min = regular ? 1 : BATCH_SOLO_ONLY;
        a.ctl->ticket = 0;
        a.ctl->exited = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        atomicAdd(&a.ctl->reg_epoch, 1);
    }
}

// Solo launches: block b runs the solo instance of work item b (the solo
// items lead the work list) for up to `steps` steps with its line in
// registers; with target >= 0 (beside persistent launches on another
// stream) only until reg_epoch reaches target, and at least one step.  The
// blocks share nothing.
template <bool BIG>
__global__ void __launch_bounds__(BATCH_BLOCK) k_batch_solo(BatchArgs a, int steps, int target)
{
    extern __shared__ unsigned char lds_raw[];
    __shared__ double red[16];
    __shared__ double redq[BATCH_NOBS][16];
    __shared__ int s_go;
    __shared__ BState sS;
    const BItem w = a.items[blockIdx.x];
    const BInst &I = a.inst[w.slot];
    BState &S = a.state[w.slot];
    if (w.pass == BP_SOLO && S.status == BS_RUNNING &&
        !solo_fast<BIG>(I, S, sS, steps, target, a.ctl, lds_raw, red, redq, &s_go) && threadIdx.x == 0)
        atomicOr(&a.ctl->error, 2);
}

// Apply the pending renormalisation factor of a finished instance and clear it.
template <class T, bool CPLX>
__global__ void __launch_bounds__(256) k_batch_scale(void *psi_, long long npts, const double *scale)
{
    using A = Alg<T, CPLX>;
    using V = typename A::V;
    V *psi = reinterpret_cast<V *>(psi_);
    const T s = T(*scale);
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
         p += (long long)gridDim.x * blockDim.x)
        psi[p] = A::scal(s, psi[p]);
}

__global__ void k_batch_unit(double *scale)
{
    if (threadIdx.x == 0) *scale = 1.0;
}

hipError_t launch_batch_step(const BatchArgs &a, bool big, bool full, int grid, size_t lds, hipStream_t st)
{
    if (big && full) hipLaunchKernelGGL((k_batch_step<true, true>), dim3(grid), dim3(BATCH_BLOCK), lds, st, a);
    else if (big) hipLaunchKernelGGL((k_batch_step<true, false>), dim3(grid), dim3(BATCH_BLOCK), lds, st, a);
    else if (full) hipLaunchKernelGGL((k_batch_step<false, true>), dim3(grid), dim3(BATCH_BLOCK), lds, st, a);
    else hipLaunchKernelGGL((k_batch_step<false, false>), dim3(grid), dim3(BATCH_BLOCK), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_solo(const BatchArgs &a, bool big, int grid, size_t lds, hipStream_t st, int steps,
                             int target)
{
    if (big) hipLaunchKernelGGL(k_batch_solo<true>, dim3(grid), dim3(BATCH_BLOCK), lds, st, a, steps, target);
    else hipLaunchKernelGGL(k_batch_solo<false>, dim3(grid), dim3(BATCH_BLOCK), lds, st, a, steps, target);
    return hipGetLastError();
}

hipError_t batch_step_occupancy(bool big, size_t lds, int *blocks_per_cu)
{
    // (the forms with every x-line variant: the others take no more
    // registers or LDS)
    if (big)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_step<true, true>, BATCH_BLOCK, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_step<false, true>, BATCH_BLOCK, lds);
}

hipError_t launch_batch_scale(int elem, void *psi, int64_t npts, double *scale, hipStream_t st)
{
    const int grid = (int)std::min<int64_t>((npts + 255) / 256, 4096);
    if (elem == 1) hipLaunchKernelGGL((k_batch_scale<float, false>), dim3(grid), dim3(256), 0, st, psi, (long long)npts, scale);
    else if (elem == 3) hipLaunchKernelGGL((k_batch_scale<float, true>), dim3(grid), dim3(256), 0, st, psi, (long long)npts, scale);
    else return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_unit, dim3(1), dim3(64), 0, st, scale);
    return hipGetLastError();
}

}  // namespace sscn

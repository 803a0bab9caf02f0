// sscn_api.cpp -- host runtime behind include/sscn.h.
//
// Validation, FP64 Thomas-table precompute, workspace layout, kernel
// planning and launch of the SSCN step on a caller-owned HIP stream.  The
// library allocates no device memory: the state and the workspace belong to
// the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "sscn.h"
#include "sscn_launch.hpp"
#include "sscn_plan.hpp"
#include "sscn_sym.hpp"

using namespace sscn;

namespace sscn {

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int pow2ceil(int64_t v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int elem_of(const sscn_problem &pb)
{
    return (pb.mode == SSCN_REAL ? 2 : 0) + (pb.prec == SSCN_F32 ? 1 : 0);
}

size_t elem_bytes(int elem)
{
    static const size_t b[4] = {8, 4, 16, 8};
    return b[elem];
}

int validate(const sscn_problem *pb)
{
    if (!pb) return SSCN_E_INVALID;
    if (pb->dim < 1 || pb->dim > 3) return SSCN_E_INVALID;
    double pts = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (pb->n[a] < 1) return SSCN_E_INVALID;
        if (a >= pb->dim && pb->n[a] != 1) return SSCN_E_INVALID;
        if (a < pb->dim && !(std::isfinite(pb->dx[a]) && pb->dx[a] > 0.0)) return SSCN_E_INVALID;
        if (!(std::isfinite(pb->omega[a]) && pb->omega[a] >= 0.0)) return SSCN_E_INVALID;
        pts *= pb->n[a];
    }
    if (!std::isfinite(pb->g)) return SSCN_E_INVALID;
    if (!(std::isfinite(pb->dt) && pb->dt > 0.0)) return SSCN_E_INVALID;
    if (pb->mode != SSCN_IMAG && pb->mode != SSCN_REAL) return SSCN_E_INVALID;
    if (pb->prec != SSCN_F64 && pb->prec != SSCN_F32) return SSCN_E_INVALID;
    if (pb->mode == SSCN_IMAG && pb->renorm_every < 1) return SSCN_E_INVALID;
    if (pb->mode == SSCN_REAL && pb->renorm_every != 0) return SSCN_E_INVALID;
    if (pb->observe_every < 0) return SSCN_E_INVALID;
    if (pb->geom < SSCN_GEOM_CART || pb->geom > SSCN_GEOM_AXI || pb->pad_ != 0) return SSCN_E_INVALID;
    if ((pb->geom == SSCN_GEOM_CIR || pb->geom == SSCN_GEOM_SPH) && pb->dim != 1) return SSCN_E_INVALID;
    if (pb->geom == SSCN_GEOM_AXI && pb->dim != 2) return SSCN_E_INVALID;
    if (pts > 1099511627776.0) return SSCN_E_UNSUPPORTED;
    if (pb->geom != SSCN_GEOM_CART && pb->n[0] > SSCN_RADIAL_MAX) return SSCN_E_UNSUPPORTED;
    return SSCN_OK;
}

double inner_dvol(const sscn_problem &pb)
{
    double dv = 1.0;
    for (int a = 0; a < pb.dim; ++a) dv *= pb.dx[a];
    constexpr double kPi = 3.14159265358979323846;
    if (pb.geom == SSCN_GEOM_SPH) dv *= 4.0 * kPi;
    else if (pb.geom != SSCN_GEOM_CART) dv *= 2.0 * kPi;
    return dv;
}

// Radial cell weights W_i = (1/dr) * integral of r^k over cell i.
void rad_weights(const sscn_problem &pb, std::vector<double> &w)
{
    const int n = pb.n[0];
    const double h = pb.dx[0];
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        const double r = (i + 0.5) * h;
        w[i] = (pb.geom == SSCN_GEOM_SPH) ? r * r + h * h / 12.0 : r;
    }
}

// Radial table (layout in sscn_sym.hpp): the finite-volume operator
// H_r psi_i = d_i psi_i - l_i psi_{i-1} - u_i psi_{i+1} with
// l_i = F_i / (2 dr^2 W_i), u_i = F_{i+1} / (2 dr^2 W_i), d_i = l_i + u_i,
// F_i = (i dr)^k, and the Thomas elimination of (1 + tau H_r) v = rhs in FP64:
// m_i = 1 / (1 + tau d_i - tau l_i * tau u_{i-1} m_{i-1}), alpha_i = tau l_i m_i,
// beta_i = tau u_i m_i.
void build_rad_table(const sscn_problem &pb, const Plan &P, std::vector<double> &out)
{
    const AxisPlan &X = P.ax[0];
    const int n = X.n, G = X.block, C = X.C, Q = G * C;
    const double h = pb.dx[0], theta = 0.5 * pb.dt;
    const std::complex<double> tau = (pb.mode == SSCN_REAL) ? std::complex<double>(0.0, theta)
                                                             : std::complex<double>(theta, 0.0);
    const int k = (pb.geom == SSCN_GEOM_SPH) ? 2 : 1;
    auto face = [&](int i) { const double f = i * h; return k == 1 ? f : f * f; };
    std::vector<double> w;
    rad_weights(pb, w);
    out.assign((size_t)RQ_N * Q, 0.0);
    std::complex<double> m_prev = 0.0, tu_prev = 0.0;
    for (int i = 0; i < n; ++i) {
        const double l = face(i) / (2.0 * h * h * w[i]);
        const double u = face(i + 1) / (2.0 * h * h * w[i]);
        const double d = l + u;
        const std::complex<double> tl = tau * l, tu = tau * u;
        const std::complex<double> den = 1.0 + tau * d - (i > 0 ? tl * tu_prev * m_prev : 0.0);
        const std::complex<double> m = 1.0 / den;
        const std::complex<double> al = tl * m, be = tu * m;
        const int t = i / C, kk = i - t * C;
        const size_t s = (size_t)kk * G + t;
        out[RQ_MR * (size_t)Q + s] = m.real();
        out[RQ_MI * (size_t)Q + s] = m.imag();
        out[RQ_AR * (size_t)Q + s] = al.real();
        out[RQ_AI * (size_t)Q + s] = al.imag();
        out[RQ_BR * (size_t)Q + s] = be.real();
        out[RQ_BI * (size_t)Q + s] = be.imag();
        out[RQ_L * (size_t)Q + s] = theta * l;
        out[RQ_D * (size_t)Q + s] = theta * d;
        out[RQ_U * (size_t)Q + s] = theta * u;
        out[RQ_W * (size_t)Q + s] = w[i];
        m_prev = m;
        tu_prev = tu;
    }
}

void thomas_coefs(double s_re, double s_im, int n, std::vector<double> &m_re, std::vector<double> &m_im,
                  std::vector<double> &a_re, std::vector<double> &a_im)
{
    const std::complex<double> s(s_re, s_im);
    const std::complex<double> b = 1.0 + 2.0 * s;
    m_re.resize(n);
    m_im.resize(n);
    a_re.resize(n);
    a_im.resize(n);
    std::complex<double> m = 1.0 / b;
    for (int i = 0; i < n; ++i) {
        if (i > 0) m = 1.0 / (b - s * s * m);
        const std::complex<double> al = s * m;
        m_re[i] = m.real();
        m_im[i] = m.imag();
        a_re[i] = al.real();
        a_im[i] = al.imag();
    }
}

// Table metadata of axis a for its chunk geometry (C points per chunk).
void table_meta(AxisPlan &X, bool fp32)
{
    std::vector<double> mr, mi, ar, ai;
    thomas_coefs(X.sig_re, X.sig_im, X.n, mr, mi, ar, ai);
    const int n = X.n;
    // constant tail: first index from which every entry equals the last one
    int ic = n - 1;
    while (ic > 0 && mr[ic - 1] == mr[n - 1] && mi[ic - 1] == mi[n - 1] && ar[ic - 1] == ar[n - 1] &&
           ai[ic - 1] == ai[n - 1])
        --ic;
    X.i_conv = ic;
    X.ac_re = ar[n - 1];
    X.ac_im = ai[n - 1];
    X.mc_re = mr[n - 1];
    X.mc_im = mi[n - 1];
    // largest product of |alpha| over a full chunk, and the number of
    // preceding chunks whose contribution can exceed the threshold
    double amax = 0.0;
    const int C = std::max(1, X.C);
    for (int c0 = 0; c0 + C <= n; c0 += C) {
        double p = 1.0;
        for (int i = c0; i < c0 + C; ++i) p *= std::hypot(ar[i], ai[i]);
        amax = std::max(amax, p);
    }
    const double lthr = fp32 ? -35.0 * std::log(2.0) : -64.0 * std::log(2.0);
    int d = 1;
    if (amax > 0.0) {
        const double q = lthr / std::log(amax);  // a^q = thr
        d = (q > 1e6) ? 1000000 : std::max(1, (int)std::ceil(q));
    }
    if (X.kind == K_ROW) {
        // Kogge-Stone steps, at most log2 of the lanes per line
        const int lmax = (X.seg > 0 && X.seg < 64) ? __builtin_ctz((unsigned)X.seg) : 6;
        int ks = 0;
        while ((1 << ks) < d && ks < lmax) ++ks;
        X.depth = ks;
    } else {
        X.depth = std::min(d, std::max(1, X.W * std::max(1, X.L)));
    }
}

// Bytes of one staged table entry: (alpha, m) in FP64, hi/lo pairs in FP32.
static size_t ltab_bytes(const Plan &P) { return (P.elem == 1 || P.elem == 3) ? 4 * P.S : 2 * P.S; }

// Dynamic LDS of one COL block at most (the table and the two exchange
// arrays; a gfx950 workgroup may take up to 160 KB).
constexpr size_t kColLdsMax = 160 * 1024 - 1024;

// Largest chunk length per thread kept in registers, by element size.
static int cmax_row(size_t S) { return S >= 16 ? 8 : (S >= 8 ? 16 : 32); }
static int cmax_col(size_t S) { return S >= 16 ? 16 : (S >= 8 ? 32 : 64); }

int make_plan(const sscn_problem &pb, const TileOverride *ov, Plan &P)
{
    std::memset(&P, 0, sizeof(P));
    P.elem = elem_of(pb);
    P.S = elem_bytes(P.elem);
    P.npts = (int64_t)pb.n[0] * pb.n[1] * pb.n[2];
    const bool imag = pb.mode == SSCN_IMAG;
    const int64_t nx = pb.n[0], ny = pb.n[1];
    for (int a = 0; a < pb.dim; ++a) {
        AxisPlan &X = P.ax[a];
        const int64_t n = pb.n[a];
        X.n = (int)n;
        X.nlines = P.npts / n;
        double s = pb.dt / (4.0 * pb.dx[a] * pb.dx[a]);
        X.sig_re = imag ? s : 0.0;
        X.sig_im = imag ? 0.0 : s;
        X.kind = K_STREAM;
        if (a == 0 && pb.geom != SSCN_GEOM_CART) {
            // radial axis: one line per block, C cells per thread, up to 16
            // waves (k_rad); the table is RQ_N doubles per padded cell
            X.kind = K_RAD;
            X.C = n <= 4096 ? 4 : (n <= 8192 ? 8 : 16);
            X.wpl = (int)ceil_div(n, 64 * (int64_t)X.C);
            X.block = 64 * X.wpl;
            X.grid = (int)X.nlines;
            X.lds = 0;
            X.m1 = (int)ny;
            X.s1 = nx;
            X.s2 = nx * ny;
            X.stride = 1;
            X.tab_entries = ceil_div((int64_t)RQ_N * X.block * X.C * (int64_t)sizeof(double),
                                     (int64_t)sizeof(TabEntry));
            X.i_conv = X.n;
            X.depth = 0;
            continue;
        }
        if (a == 0) {
            X.m1 = (int)ny;
            X.s1 = nx;
            X.s2 = nx * ny;
            X.stride = 1;
            int c = pow2ceil(ceil_div(n, 64));
            int wpl = 1;
            if (ov && ov->row_c > 0) {
                c = ov->row_c;
                wpl = pow2ceil(ceil_div(n, 64 * (int64_t)c));
            } else if (c > cmax_row(P.S)) {
                c = cmax_row(P.S);
                wpl = pow2ceil(ceil_div(n, 64 * (int64_t)c));
            } else if (n <= 64) {
                c = 4;
            }
            // lines of at most 64 points in chunks of 4: 16 lanes per line
            // and four lines per wave (fewer scan steps and a quarter of the
            // per-line instructions of one line over 64 lanes)
            const int seg = (c == 4 && n <= 64) ? 16 : 64;
            if (wpl <= 16 && c <= cmax_row(P.S) && (int64_t)c * seg * wpl >= n) {
                X.kind = K_ROW;
                X.C = c;
                X.wpl = wpl;
                X.seg = seg;
                X.lpb = std::max(1, 4 / wpl) * (64 / seg);
                X.block = 64 * wpl * std::max(1, 4 / wpl);
                X.grid = (int)std::min<int64_t>(ceil_div(X.nlines, X.lpb), 4096);
                // single-wave lines stage their table in LDS and move their
                // values through a per-wave buffer of c*64 + 64 values when
                // both fit 64 KB (k_row decides alike; not for short lines);
                // multi-wave lines exchange 4 values per wave
                if (wpl == 1) {
                    const size_t tab = (size_t)c * seg * ltab_bytes(P), tr = (size_t)X.lpb * (c * 64 + 64) * P.S;
                    X.lds = (seg == 64 && P.S >= 16 && tab + tr <= 65536) ? tab + tr : tab;
                } else {
                    X.lds = (size_t)X.lpb * wpl * 4 * P.S;
                }
                X.tab_entries = (size_t)c * seg * wpl;
            }
        } else {
            X.m1 = (int)nx;
            X.s1 = 1;
            X.s2 = (a == 1) ? nx * ny : nx;
            X.stride = (a == 1) ? nx : nx * ny;
            // 4 points per thread (registers for two 1024-thread blocks per
            // CU), more only when 16 waves x Lmax lanes cannot cover the
            // line; Lmax keeps a wave's row segment (64/L lines x S bytes)
            // at 128 bytes or more.  A sweep of fewer than 256 blocks (one
            // per CU) takes more lanes per line, up to Lmax: fewer lines
            // and waves per block, more blocks (small grids)
            const int lmax = std::max(1, std::min(8, (int)(P.S / 2)));
            int c = 4;
            while (c < 64 && ceil_div(n, c) > 16 * lmax) c *= 2;
            c = std::min<int64_t>(c, pow2ceil(ceil_div(n, 16)));
            // a line longer than 16 waves x Lmax lanes x the longest chunk
            // takes the longest chunk and up to 8 lanes (row segments down
            // to 64 bytes) rather than the one-thread-per-line form
            if (c > cmax_col(P.S)) c = cmax_col(P.S);
            if (ov && ov->col_c[a] > 0) c = ov->col_c[a];
            const int64_t K = ceil_div(n, c);           // chunks per line
            int L = pow2ceil(ceil_div(K, 16));          // lanes per line
            while (L < lmax && L < K && ceil_div(X.nlines, 64 / L) < 256) L *= 2;
            const int64_t W = ceil_div(K, L);
            const size_t lds = (size_t)W * L * c * ltab_bytes(P) + (size_t)2 * W * 64 * P.S;
            if (c <= cmax_col(P.S) && L <= 8 && lds <= kColLdsMax) {
                X.kind = K_COL;
                X.C = c;
                X.W = (int)W;
                X.L = L;
                X.block = 64 * (int)W;
                X.grid = (int)ceil_div(X.nlines, 64 / L);
                X.lds = lds;
                X.tab_entries = (size_t)W * L * c;
            }
        }
        if (X.kind == K_STREAM) {
            X.block = 256;
            X.grid = (int)ceil_div(X.nlines, 256);
            X.tab_entries = (size_t)n;
        }
        table_meta(X, pb.prec == SSCN_F32);
        if (X.kind == K_STREAM) X.i_conv = X.n;
        if (X.grid > 2147483647 / 2) return SSCN_E_UNSUPPORTED;
    }
    const AxisPlan &L = P.ax[pb.dim - 1];
    // the axial trap's z sweep weighs its norm terms in the last sweep's
    // kernel, which only the COL kernel does
    if (pb.geom == SSCN_GEOM_AXI && L.kind != K_COL) return SSCN_E_UNSUPPORTED;
    P.sep_pointwise = P.ax[0].kind == K_STREAM;
    // a one-line radial sweep finalises the norm in its own (single) block
    P.fused_norm = imag && pb.dim == 1 && L.kind == K_RAD && L.grid == 1;
    P.sep_norm = imag && L.kind == K_STREAM;
    P.pw_grid = (int)std::min<int64_t>(ceil_div(P.npts, 256), 4096);
    P.np_norm = P.sep_norm ? P.pw_grid : L.grid;
    // few partials: the next step's x sweep sums them itself (every wave of
    // it reads them all), which saves the final sum's launch on the small
    // grids that launches bound; short x lines (the k_row form that takes
    // four lines per wave carries the code), and x not the last sweep (its
    // blocks would read partials that others overwrite)
    P.fold_norm = imag && pb.dim >= 2 && P.ax[0].kind == K_ROW && P.ax[0].seg < 64 && L.kind == K_COL &&
                  P.np_norm <= 64 * kFoldWaves;
    P.obs_grid = (int)std::min<int64_t>(ceil_div(P.npts, 256), 1024);

    size_t off = 0;
    P.off_scal = off;
    off += 256;
    P.off_obs = off;
    off += 256;
    for (int a = 0; a < pb.dim; ++a) {
        P.ax[a].tab_off = off;
        off = align256(off + P.ax[a].tab_entries * sizeof(TabEntry));
    }
    P.off_wline = 0;
    if (pb.geom == SSCN_GEOM_AXI) {
        P.off_wline = off;
        off = align256(off + (size_t)pb.n[0] * sizeof(double));
    }
    P.off_part = off;
    off = align256(off + (size_t)P.np_norm * sizeof(double));
    P.off_obspart = off;
    off = align256(off + (size_t)P.obs_grid * 12 * sizeof(double));
    // n_1D keeping x: partial sums over blocks of rows, one per (block, x);
    // up to 256 blocks (1024 made the final sum 9.6 us of 53 at 256^3,
    // 256 blocks 43 us in all) and 256K doubles
    {
        const int64_t rows = P.npts / pb.n[0];
        P.dens_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(rows, 256),
                                                                    (int64_t)262144 / pb.n[0]));
    }
    // and the x-line sums of n_1D keeping y or z, when there are at most
    // 256K x lines
    P.off_dens = off;
    {
        const int64_t rows = P.npts / pb.n[0];
        const int64_t dn = std::max<int64_t>((int64_t)P.dens_blocks * pb.n[0], rows <= 262144 ? rows : 0);
        off = align256(off + (size_t)dn * sizeof(double));
    }
    P.ws_bytes = off;
    return SSCN_OK;
}

// FP64 Thomas tables of axis a in the layout its kernel reads.
void build_table(const sscn_problem &pb, const Plan &P, int a, std::vector<TabEntry> &out)
{
    const AxisPlan &X = P.ax[a];
    const int n = X.n;
    std::vector<double> mr, mi, ar, ai;
    thomas_coefs(X.sig_re, X.sig_im, n, mr, mi, ar, ai);
    out.assign(X.tab_entries, TabEntry{0, 0, 0, 0});
    auto put = [&](size_t slot, int i) { out[slot] = TabEntry{ar[i], ai[i], mr[i], mi[i]}; };
    if (X.kind == K_ROW) {
        const int G = (X.seg > 0 && X.seg < 64) ? X.seg : 64 * X.wpl;
        for (int t = 0; t < G; ++t)
            for (int k = 0; k < X.C; ++k) {
                const int i = t * X.C + k;
                if (i < n) put((size_t)k * G + t, i);
            }
    } else {
        for (int i = 0; i < n; ++i) put((size_t)i, i);
    }
    (void)pb;
}

struct HintEntry {
    int32_t dim, n[3], mode, prec;
    TileOverride ov;
};
static std::mutex g_hint_mu;
static std::vector<HintEntry> g_hints;

static bool hint_match(const HintEntry &h, const sscn_problem &pb)
{
    return pb.geom == SSCN_GEOM_CART && h.dim == pb.dim && h.n[0] == pb.n[0] && h.n[1] == pb.n[1] && h.n[2] == pb.n[2] &&
           h.mode == pb.mode && h.prec == pb.prec;
}

bool tile_hint_copy(const sscn_problem &pb, TileOverride &out)
{
    std::lock_guard<std::mutex> lk(g_hint_mu);
    for (const HintEntry &h : g_hints)
        if (hint_match(h, pb)) {
            out = h.ov;
            return true;
        }
    return false;
}

}  // namespace sscn

struct sscn_solver {
    sscn_problem pb;
    Plan P;
    void *psi;
    char *ws;
    hipStream_t st;
    int64_t step;
    double g;
    double host_obs[16];
    // captured runs of 2^lg steps (lg <= kGraphLog), keyed by lg and by
    // which of their steps renormalise; their kernel arguments hold g
    std::map<int64_t, hipGraphExec_t> graphs;
    bool graphs_off;          // capture failed once on this stream: launch directly
    bool pending;             // inside sscn_run: the last renormalisation factor is not yet applied to psi
    int static_dev;           // sscn_create_noalloc: the device whose static workspace it holds, else -1
};

static void drop_graphs(sscn_solver *s)
{
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
}

static double *scal_ptr(sscn_solver *s) { return reinterpret_cast<double *>(s->ws + s->P.off_scal); }

static PointParams point_params(const sscn_solver *s)
{
    PointParams pp;
    std::memset(&pp, 0, sizeof(pp));
    pp.dt = s->pb.dt;
    pp.g = s->g;
    for (int a = 0; a < 3; ++a) {
        pp.n[a] = s->pb.n[a];
        pp.dx[a] = (a < s->pb.dim) ? s->pb.dx[a] : 0.0;
        pp.cen[a] = 0.5 * (s->pb.n[a] - 1);
        pp.w2h[a] = (a < s->pb.dim) ? 0.5 * s->pb.omega[a] * s->pb.omega[a] : 0.0;
    }
    return pp;
}

static LineTab line_tab(sscn_solver *s, int a)
{
    const AxisPlan &X = s->P.ax[a];
    LineTab t;
    t.tab = reinterpret_cast<const TabEntry *>(s->ws + X.tab_off);
    t.n = X.n;
    t.i_conv = X.i_conv;
    t.ac_re = X.ac_re;
    t.ac_im = X.ac_im;
    t.mc_re = X.mc_re;
    t.mc_im = X.mc_im;
    t.depth = X.depth;
    return t;
}

static ColArgs col_args(sscn_solver *s, int a, bool last)
{
    const AxisPlan &X = s->P.ax[a];
    ColArgs c;
    c.psi = s->psi;
    c.lt = line_tab(s, a);
    c.nlines = (int32_t)X.nlines;
    c.stride = X.stride;
    c.m1 = X.m1;
    c.s1 = X.s1;
    c.s2 = X.s2;
    c.W = X.W;
    c.L = X.L;
    c.sig_re = X.sig_re;
    c.sig_im = X.sig_im;
    c.partial = last ? reinterpret_cast<double *>(s->ws + s->P.off_part) : nullptr;
    c.wline = (last && s->P.off_wline) ? reinterpret_cast<const double *>(s->ws + s->P.off_wline) : nullptr;
    c.unit_scale = nullptr;
    return c;
}

// Kernel classes for timing: 0 x (+pointwise), 1 y, 2 z, 3 norm final, 4 scale.
// Each timed launch takes a start/stop event pair: the sweep kernels pass it
// to the launch (the events take the kernel's own begin and end times);
// other kernels are bracketed by event records on the stream.
struct Timer {
    std::vector<hipEvent_t> ev;
    std::vector<int> cls;
    size_t used = 0;
    hipStream_t st;
    // next pair for class c, or nulls when the pool is used up
    void pair(int c, hipEvent_t &a, hipEvent_t &b)
    {
        a = b = nullptr;
        if (used + 2 > ev.size()) return;
        cls[used] = c;
        a = ev[used];
        b = ev[used + 1];
        used += 2;
    }
};

// fold_in: the previous step renormalised and left its norm partials for
// this step's x sweep (fold_norm plans, within a run of steps).  final_sum:
// a renormalising step launches the norm's final sum (always, unless the
// plan folds it into the next step and this step is not a run's last).
static hipError_t enqueue_step(sscn_solver *s, bool do_renorm, bool fold_in, bool final_sum, Timer *tm)
{
    const Plan &P = s->P;
    const sscn_problem &pb = s->pb;
    const bool imag = pb.mode == SSCN_IMAG;
    const int dim = pb.dim;
    double *scal = scal_ptr(s);
    double *part = reinterpret_cast<double *>(s->ws + P.off_part);
    hipError_t e;
#define CHK(x)                          \
    do {                                \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // x sweep with the pointwise substep
    {
        if (tm) tm->pair(0, e0, e1);
        const AxisPlan &X = P.ax[0];
        const bool last = imag && do_renorm && dim == 1 && X.kind == K_ROW;
        if (X.kind == K_ROW) {
            RowArgs r;
            r.psi = s->psi;
            r.lt = line_tab(s, 0);
            r.nlines = (int32_t)X.nlines;
            r.wpl = X.wpl;
            r.seg = X.seg;
            r.lpb = X.lpb;
            r.v16 = P.S <= 8 && (X.n % (int)(16 / P.S) == 0) && (reinterpret_cast<uintptr_t>(s->psi) % 16 == 0);
            r.sig_re = X.sig_re;
            r.sig_im = X.sig_im;
            r.pp = point_params(s);
            r.scale = scal;
            r.partial = last ? part : nullptr;
            r.fold = fold_in ? part : nullptr;
            r.fold_np = P.np_norm;
            r.fold_dvol = inner_dvol(pb);
            CHK(launch_row(P.elem, X.C, last, r, X.grid, X.block, X.lds, s->st, e0, e1));
        } else if (X.kind == K_RAD) {
            const bool rlast = imag && do_renorm && dim == 1;
            RadArgs r;
            r.psi = s->psi;
            r.tab = reinterpret_cast<const double *>(s->ws + X.tab_off);
            r.n = X.n;
            r.dt = pb.dt;
            r.g = s->g;
            r.dr = pb.dx[0];
            r.w2h_r = 0.5 * pb.omega[0] * pb.omega[0];
            const bool axial = pb.geom == SSCN_GEOM_AXI;
            r.dz = axial ? pb.dx[1] : 0.0;
            r.cen_z = axial ? 0.5 * (pb.n[1] - 1) : 0.0;
            r.w2h_z = axial ? 0.5 * pb.omega[1] * pb.omega[1] : 0.0;
            r.scale = scal;
            r.partial = rlast ? part : nullptr;
            r.scalars = (rlast && P.fused_norm) ? scal : nullptr;
            r.dvol = inner_dvol(pb);
            CHK(launch_rad(P.elem, X.C, rlast, r, X.grid, X.block, s->st, e0, e1));
        } else {
            PointArgs pa;
            pa.psi = s->psi;
            pa.npts = P.npts;
            pa.pp = point_params(s);
            pa.scale = scal;
            if (e0) CHK(hipEventRecord(e0, s->st));
            CHK(launch_pointwise(P.elem, pa, P.pw_grid, 256, s->st));
            CHK(launch_stream(P.elem, col_args(s, 0, false), X.grid, X.block, s->st));
            if (e1) CHK(hipEventRecord(e1, s->st));
        }
    }
    for (int a = 1; a < dim; ++a) {
        const AxisPlan &X = P.ax[a];
        const bool last = imag && do_renorm && a == dim - 1 && X.kind == K_COL;
        if (tm) tm->pair(a, e0, e1);
        if (X.kind == K_COL) {
            ColArgs c = col_args(s, a, last);
            // a step that does not renormalise resets the pending scale in its
            // last sweep (the x sweep has applied it) instead of a launch
            if (imag && !do_renorm && a == dim - 1) c.unit_scale = scal;
            CHK(launch_col(P.elem, X.C, last, c, X.grid, X.block, X.lds, s->st, e0, e1));
        } else {
            if (e0) CHK(hipEventRecord(e0, s->st));
            CHK(launch_stream(P.elem, col_args(s, a, false), X.grid, X.block, s->st));
            if (e1) CHK(hipEventRecord(e1, s->st));
        }
    }
    // the norm's final sum (renormalising steps), or the scale's reset in a
    // step that does not renormalise, unless its last sweep is a COL kernel,
    // which resets the scale itself
    const bool col_reset = dim > 1 && P.ax[dim - 1].kind == K_COL;
    if (imag && (do_renorm ? !P.fused_norm && final_sum : !col_reset)) {
        if (tm) tm->pair(3, e0, e1);
        if (e0) CHK(hipEventRecord(e0, s->st));
        if (do_renorm && P.sep_norm)
            CHK(launch_norm_partials(P.elem, s->psi, P.npts, part, P.pw_grid, 256, s->st));
        CHK(launch_norm_final(part, P.np_norm, inner_dvol(pb), do_renorm ? 1 : 0, scal, s->st));
        if (e1) CHK(hipEventRecord(e1, s->st));
    }
#undef CHK
    return hipSuccess;
}

// Captured graphs.  Small problems are bound by launch overhead (four
// kernels of a few microseconds per step); a graph replay issues a run of
// steps with one call.  A call of n steps replays the graphs of its binary
// decomposition into runs of 32, 16, ..., 1 steps, so every length is
// replayed, not only multiples of 32.  The replayed kernels and arguments are
// those the direct path would launch, except that a plan that folds the
// norm's final sum into the next step ends every run with it (the folded
// factor is bitwise the one the final sum writes), so results are the same.
constexpr int kGraphLog = 5;                 // longest run: 32 steps
constexpr size_t kMaxGraphs = 192;           // renormalisation patterns x lengths

// A run's graph is fixed by its length and by which of its steps
// renormalise: bit k-1 of the mask is set when step after+k does.
static int64_t graph_key(const sscn_solver *s, int64_t after_step, int lg)
{
    int64_t mask = 0;
    if (s->pb.mode == SSCN_IMAG)
        for (int64_t k = 1; k <= (int64_t(1) << lg); ++k)
            if ((after_step + k) % s->pb.renorm_every == 0) mask |= int64_t(1) << (k - 1);
    return mask * 8 + lg;
}

// Length exponent of the next graph run for `left` steps.
static int run_log(int64_t left)
{
    int lg = 0;
    while (lg < kGraphLog && (int64_t(2) << lg) <= left) ++lg;
    return lg;
}

static hipError_t capture_run(sscn_solver *s, int64_t after_step, int lg, hipGraphExec_t *out)
{
    const bool imag = s->pb.mode == SSCN_IMAG;
    hipError_t e = hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    const int64_t len = int64_t(1) << lg;
    bool prev_renorm = false;
    for (int64_t k = 1; k <= len && le == hipSuccess; ++k) {
        const int64_t step = after_step + k;
        const bool renorm = imag && (step % s->pb.renorm_every == 0);
        le = enqueue_step(s, renorm, s->P.fold_norm && prev_renorm, !s->P.fold_norm || k == len, nullptr);
        prev_renorm = renorm;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s->st, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le != hipSuccess ? le : e;
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

// The graph for a run of 2^lg steps after step `after_step`, captured on
// first use; nullptr when graphs are off for this solver.
static hipGraphExec_t graph_for(sscn_solver *s, int64_t after_step, int lg)
{
    if (s->st == nullptr || s->graphs_off) return nullptr;   // the legacy default stream cannot be captured
    const int64_t key = graph_key(s, after_step, lg);
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) return it->second;
    if (s->graphs.size() >= kMaxGraphs) drop_graphs(s);
    hipGraphExec_t ex = nullptr;
    if (capture_run(s, after_step, lg, &ex) != hipSuccess) {
        (void)hipGetLastError();
        s->graphs_off = true;
        return nullptr;
    }
    try {
        s->graphs.emplace(key, ex);
    } catch (...) {
        (void)hipGraphExecDestroy(ex);
        return nullptr;
    }
    return ex;
}

// Capture, without launching anything, every graph a later call of nsteps
// steps from the current step will replay, and upload each to the device
// (a graph's first launch otherwise pays for the upload).
static hipError_t prepare_graphs(sscn_solver *s, int64_t nsteps)
{
    int64_t step = s->step;
    while (nsteps > 0) {
        const int lg = run_log(nsteps);
        hipGraphExec_t ex = graph_for(s, step, lg);
        if (!ex) return hipSuccess;             // graphs off: sscn_step launches directly
        hipError_t e = hipGraphUpload(ex, s->st);
        if (e != hipSuccess) return e;
        step += int64_t(1) << lg;
        nsteps -= int64_t(1) << lg;
    }
    return hipSuccess;
}

// A pending renormalisation factor applied to psi (and the factor reset).
static hipError_t finalize_state(sscn_solver *s, Timer *tm)
{
    if (!s->pending) return hipSuccess;
    s->pending = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) tm->pair(4, e0, e1);
    hipError_t e = hipSuccess;
    if (e0 && (e = hipEventRecord(e0, s->st)) != hipSuccess) return e;
    if ((e = launch_scale_state(s->P.elem, s->psi, s->P.npts, scal_ptr(s), s->P.pw_grid, 256, s->st)) != hipSuccess)
        return e;
    if ((e = launch_set_unit_scale(scal_ptr(s), s->st)) != hipSuccess) return e;
    if (e1 && (e = hipEventRecord(e1, s->st)) != hipSuccess) return e;
    return hipSuccess;
}

// finalize: apply a pending renormalisation factor to psi at the end (every
// public call that returns a state); sscn_run's observations take it in
// their loads instead and the run applies it once at its end.
static hipError_t enqueue_steps(sscn_solver *s, int64_t nsteps, Timer *tm, bool finalize = true)
{
    if (nsteps <= 0) return hipSuccess;
    const bool imag = s->pb.mode == SSCN_IMAG;
    bool last_renorm = false;
    // graph runs (not when timing: the timed path launches each kernel with
    // its own events)
    while (!tm && nsteps > 0) {
        const int lg = run_log(nsteps);
        hipGraphExec_t ex = graph_for(s, s->step, lg);
        if (!ex) break;
        hipError_t e = hipGraphLaunch(ex, s->st);
        if (e != hipSuccess) return e;
        s->step += int64_t(1) << lg;
        nsteps -= int64_t(1) << lg;
        last_renorm = imag && (s->step % s->pb.renorm_every == 0);
    }
    // direct launches: the rest of the call is one run
    bool prev_renorm = false;
    for (int64_t t = 0; t < nsteps; ++t) {
        const int64_t step = s->step + 1;
        const bool do_renorm = imag && (step % s->pb.renorm_every == 0);
        hipError_t e = enqueue_step(s, do_renorm, s->P.fold_norm && prev_renorm,
                                    !s->P.fold_norm || t == nsteps - 1, tm);
        if (e != hipSuccess) return e;
        s->step = step;
        last_renorm = do_renorm;
        prev_renorm = do_renorm;
    }
    // the steps consumed any earlier factor (in the first x sweep's load);
    // the last one leaves a new one when it renormalised
    s->pending = imag && last_renorm;
    return finalize ? finalize_state(s, tm) : hipSuccess;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int sscn_abi_version(void) { return SSCN_ABI_VERSION; }

const char *sscn_status_string(int status)
{
    switch (status) {
    case SSCN_OK: return "ok";
    case SSCN_NOT_CONVERGED: return "not converged (step cap reached)";
    case SSCN_E_INVALID: return "invalid argument";
    case SSCN_E_HIP: return "HIP runtime error";
    case SSCN_E_NONFINITE: return "non-finite norm or chemical potential";
    case SSCN_E_NOSPACE: return "no space (slot busy or buffer too small)";
    case SSCN_E_UNSUPPORTED: return "unsupported problem size";
    default: return "unknown status";
    }
}

int sscn_validate(const sscn_problem *pb) { return validate(pb); }

int sscn_units_to_g(const sscn_units *u, double *g, double *length_m, double *time_s)
{
    if (!u || !g || u->dim < 1 || u->dim > 3 || u->pad_ != 0) return SSCN_E_INVALID;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(u->atoms) || !pos(u->mass) || !pos(u->omega) || !std::isfinite(u->scattering_length))
        return SSCN_E_INVALID;
    if (u->dim <= 2 && !pos(u->tight[0])) return SSCN_E_INVALID;
    if (u->dim == 1 && !pos(u->tight[1])) return SSCN_E_INVALID;
    // CODATA 2018: reduced Planck constant, unified atomic mass unit, Bohr radius
    constexpr double kHbar = 1.054571817e-34, kAmu = 1.66053906660e-27, kBohr = 5.29177210903e-11;
    constexpr double kPi = 3.14159265358979323846;
    const double l = std::sqrt(kHbar / (u->mass * kAmu * u->omega));
    double gv = 4.0 * kPi * u->atoms * u->scattering_length * kBohr / l;
    if (u->dim == 2) gv *= std::sqrt(u->tight[0] / (2.0 * kPi));
    if (u->dim == 1) gv *= std::sqrt(u->tight[0] * u->tight[1]) / (2.0 * kPi);
    *g = gv;
    if (length_m) *length_m = l;
    if (time_s) *time_s = 1.0 / u->omega;
    return SSCN_OK;
}

int sscn_set_tile_hint(const sscn_problem *pb, const int32_t chunk[3])
{
    int v = validate(pb);
    if (v != SSCN_OK) return v;
    if (pb->geom != SSCN_GEOM_CART) return SSCN_E_UNSUPPORTED;
    if (!chunk) return SSCN_E_INVALID;
    for (int a = 0; a < 3; ++a) {
        const int c = chunk[a];
        if (c < 0 || c > 64 || (c & (c - 1)) != 0) return SSCN_E_INVALID;
    }
    HintEntry h;
    std::memset(&h, 0, sizeof(h));
    h.dim = pb->dim;
    for (int a = 0; a < 3; ++a) h.n[a] = pb->n[a];
    h.mode = pb->mode;
    h.prec = pb->prec;
    h.ov.row_c = chunk[0];
    h.ov.col_c[0] = 0;
    h.ov.col_c[1] = chunk[1];
    h.ov.col_c[2] = chunk[2];
    Plan P;
    v = make_plan(*pb, &h.ov, P);
    if (v != SSCN_OK) return v;
    for (int a = 0; a < pb->dim; ++a)
        if (chunk[a] != 0 && P.ax[a].kind == K_STREAM) return SSCN_E_UNSUPPORTED;
    try {
        std::lock_guard<std::mutex> lk(g_hint_mu);
        for (HintEntry &e : g_hints)
            if (hint_match(e, *pb)) {
                e = h;
                return SSCN_OK;
            }
        g_hints.push_back(h);
    } catch (...) {
        return SSCN_E_INVALID;
    }
    return SSCN_OK;
}

int sscn_clear_tile_hints(void)
{
    std::lock_guard<std::mutex> lk(g_hint_mu);
    g_hints.clear();
    return SSCN_OK;
}

int sscn_plan_info(const sscn_problem *pb, int32_t *info, int32_t cap)
{
    int v = validate(pb);
    if (v != SSCN_OK) return v;
    if (!info || cap < 24) return SSCN_E_INVALID;
    Plan P;
    TileOverride ov;
    v = make_plan(*pb, tile_hint_copy(*pb, ov) ? &ov : nullptr, P);
    if (v != SSCN_OK) return v;
    for (int a = 0; a < 3; ++a) {
        const AxisPlan &X = P.ax[a];
        const bool used = a < pb->dim;
        int32_t *o = info + 8 * a;
        o[0] = used ? X.kind : -1;
        o[1] = used ? X.C : 0;
        o[2] = used ? ((X.kind == K_ROW || X.kind == K_RAD) ? X.wpl : X.W) : 0;
        o[3] = used ? (X.kind == K_COL ? X.L : (X.kind == K_ROW ? X.seg : 1)) : 0;
        o[4] = used ? X.grid : 0;
        o[5] = used ? X.block : 0;
        o[6] = used ? X.i_conv : 0;
        o[7] = used ? X.depth : 0;
    }
    return SSCN_OK;
}

int sscn_state_bytes(const sscn_problem *pb, size_t *bytes)
{
    int v = validate(pb);
    if (v != SSCN_OK) return v;
    if (!bytes) return SSCN_E_INVALID;
    *bytes = (size_t)pb->n[0] * pb->n[1] * pb->n[2] * elem_bytes(elem_of(*pb));
    return SSCN_OK;
}

int sscn_workspace_bytes(const sscn_problem *pb, size_t *bytes)
{
    int v = validate(pb);
    if (v != SSCN_OK) return v;
    if (!bytes) return SSCN_E_INVALID;
    Plan P;
    TileOverride ov;
    v = make_plan(*pb, tile_hint_copy(*pb, ov) ? &ov : nullptr, P);
    if (v != SSCN_OK) return v;
    *bytes = P.ws_bytes;
    return SSCN_OK;
}

}  // extern "C"

// A solver over caller memory.  whole_ws: upload an image of the whole
// workspace (zeros past the tables) instead of its head only, for a
// workspace whose earlier contents are unknown.
static int create_solver(const sscn_problem *pb, void *d_psi, void *d_ws, void *hip_stream, bool whole_ws,
                         int static_dev, sscn_solver **out)
{
    sscn_solver *s = new (std::nothrow) sscn_solver();   // value-initialised: members zero, map empty
    if (!s) return SSCN_E_INVALID;
    s->pb = *pb;
    s->psi = d_psi;
    s->ws = static_cast<char *>(d_ws);
    s->st = static_cast<hipStream_t>(hip_stream);
    s->g = pb->g;
    s->static_dev = static_dev;
    TileOverride ov;
    int v = make_plan(*pb, tile_hint_copy(*pb, ov) ? &ov : nullptr, s->P);
    if (v != SSCN_OK) {
        delete s;
        return v;
    }
    // host image of the workspace head and tables, uploaded in one pass
    try {
        std::vector<char> img(whole_ws ? s->P.ws_bytes : s->P.off_part, 0);
        double *scal = reinterpret_cast<double *>(img.data() + s->P.off_scal);
        scal[0] = 1.0;
        scal[1] = 1.0;
        std::vector<TabEntry> tab;
        for (int a = 0; a < pb->dim; ++a) {
            if (s->P.ax[a].kind == K_RAD) {
                std::vector<double> rt;
                build_rad_table(*pb, s->P, rt);
                std::memcpy(img.data() + s->P.ax[a].tab_off, rt.data(), rt.size() * sizeof(double));
                continue;
            }
            build_table(*pb, s->P, a, tab);
            std::memcpy(img.data() + s->P.ax[a].tab_off, tab.data(), tab.size() * sizeof(TabEntry));
        }
        if (s->P.off_wline) {
            std::vector<double> w;
            rad_weights(*pb, w);
            std::memcpy(img.data() + s->P.off_wline, w.data(), w.size() * sizeof(double));
        }
        if (hipMemcpyAsync(s->ws, img.data(), img.size(), hipMemcpyHostToDevice, s->st) != hipSuccess ||
            hipStreamSynchronize(s->st) != hipSuccess) {
            delete s;
            return SSCN_E_HIP;
        }
    } catch (...) {
        delete s;
        return SSCN_E_INVALID;
    }
    *out = s;
    return SSCN_OK;
}

// ---------------------------------------------------------------------------
// Static workspace of sscn_create_noalloc: one array per device, which every
// GPU the library runs on holds until the process ends.  In host code the
// array's name is only a stand-in: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is used.
// ---------------------------------------------------------------------------
constexpr size_t kStaticWsBytes = SSCN_STATIC_WS_BYTES;
static __device__ __align__(256) char scratch[kStaticWsBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static void *g_static_ptr[kMaxDevices];                  // device address of `scratch`, per device
static const sscn_solver *g_static_owner[kMaxDevices];   // the live solver holding it, per device

extern "C" {

int sscn_create(const sscn_problem *pb, void *d_psi, void *d_ws, void *hip_stream, sscn_solver **out)
{
    int v = validate(pb);
    if (v != SSCN_OK) return v;
    if (!d_psi || !d_ws || !out) return SSCN_E_INVALID;
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return SSCN_E_INVALID;
    if (reinterpret_cast<uintptr_t>(d_psi) % 16 != 0) return SSCN_E_INVALID;
    return create_solver(pb, d_psi, d_ws, hip_stream, false, -1, out);
}

int sscn_create_noalloc(const sscn_problem *pb, void *d_psi, void *hip_stream, sscn_solver **out)
{
    int v = validate(pb);
    if (v != SSCN_OK) return v;
    if (!d_psi || !out) return SSCN_E_INVALID;
    if (reinterpret_cast<uintptr_t>(d_psi) % 16 != 0) return SSCN_E_INVALID;
    Plan P;
    TileOverride ov;
    v = make_plan(*pb, tile_hint_copy(*pb, ov) ? &ov : nullptr, P);
    if (v != SSCN_OK) return v;
    if (P.ws_bytes > kStaticWsBytes) return SSCN_E_UNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SSCN_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return SSCN_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return SSCN_E_HIP;
        }
        g_static_ptr[dev] = ptr;
    }
    if (g_static_owner[dev]) return SSCN_E_NOSPACE;
    sscn_solver *s = nullptr;
    v = create_solver(pb, d_psi, g_static_ptr[dev], hip_stream, true, dev, &s);
    if (v != SSCN_OK) return v;
    g_static_owner[dev] = s;
    *out = s;
    return SSCN_OK;
}

int sscn_step(sscn_solver *s, int64_t nsteps)
{
    if (!s || nsteps < 0) return SSCN_E_INVALID;
    return enqueue_steps(s, nsteps, nullptr) == hipSuccess ? SSCN_OK : SSCN_E_HIP;
}

int sscn_prepare(sscn_solver *s, int64_t nsteps)
{
    if (!s || nsteps < 0) return SSCN_E_INVALID;
    return prepare_graphs(s, nsteps) == hipSuccess ? SSCN_OK : SSCN_E_HIP;
}

int sscn_step_timed(sscn_solver *s, int64_t nsteps, double *ms)
{
    if (!s || nsteps < 0 || !ms) return SSCN_E_INVALID;
    Timer tm;
    tm.st = s->st;
    const size_t need = (size_t)nsteps * 8 + 4;   // a pair per kernel class and step
    try {
        tm.ev.resize(need);
        tm.cls.resize(need, -1);
    } catch (...) {
        return SSCN_E_INVALID;
    }
    size_t made = 0;
    for (; made < need; ++made)
        if (hipEventCreate(&tm.ev[made]) != hipSuccess) break;
    int rc = SSCN_OK;
    if (made < need) rc = SSCN_E_HIP;
    if (rc == SSCN_OK && enqueue_steps(s, nsteps, &tm) != hipSuccess) rc = SSCN_E_HIP;
    if (rc == SSCN_OK && hipStreamSynchronize(s->st) != hipSuccess) rc = SSCN_E_HIP;
    double tot[SSCN_NKERNELS] = {0};
    int cnt[SSCN_NKERNELS] = {0};
    if (rc == SSCN_OK) {
        for (size_t i = 0; i + 1 < tm.used; i += 2) {
            const int c = tm.cls[i];
            if (c < 0 || c >= SSCN_NKERNELS) continue;
            float f = 0.f;
            if (hipEventElapsedTime(&f, tm.ev[i], tm.ev[i + 1]) != hipSuccess) {
                rc = SSCN_E_HIP;
                break;
            }
            tot[c] += f;
            cnt[c] += 1;
        }
    }
    for (int c = 0; c < SSCN_NKERNELS; ++c) ms[c] = cnt[c] ? tot[c] / cnt[c] : 0.0;
    for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(tm.ev[i]);
    return rc;
}

// Enqueue the observation kernels; the 13 results land at *dobs (device).
// The observation kernels of the current state; the 13 results go to `dest`
// (device-accessible; null: the workspace's slot), whose address is
// returned in *dobs_out.
static hipError_t obs_enqueue(sscn_solver *s, double **dobs_out, double *dest = nullptr)
{
    const Plan &P = s->P;
    double *dobs = dest ? dest : reinterpret_cast<double *>(s->ws + P.off_obs);
    *dobs_out = dobs;
    if (s->pb.geom != SSCN_GEOM_CART) {
        const sscn_problem &pb = s->pb;
        const bool axial = pb.geom == SSCN_GEOM_AXI;
        SymObsArgs so;
        std::memset(&so, 0, sizeof(so));
        so.psi = s->psi;
        so.nr = pb.n[0];
        so.nz = axial ? pb.n[1] : 1;
        so.k = (pb.geom == SSCN_GEOM_SPH) ? 2 : 1;
        so.axial = axial ? 1 : 0;
        so.dr = pb.dx[0];
        so.dz = axial ? pb.dx[1] : 0.0;
        so.cen_z = axial ? 0.5 * (pb.n[1] - 1) : 0.0;
        so.w2h_r = 0.5 * pb.omega[0] * pb.omega[0];
        so.w2h_z = axial ? 0.5 * pb.omega[1] * pb.omega[1] : 0.0;
        so.npts = P.npts;
        so.partial = reinterpret_cast<double *>(s->ws + P.off_obspart);
        hipError_t e = launch_sym_obs_partials(P.elem, so, P.obs_grid, 256, s->st);
        if (e == hipSuccess) e = launch_obs_final(so.partial, P.obs_grid, inner_dvol(pb), s->g, dobs, s->st);
        return e;
    }
    ObsArgs oa;
    std::memset(&oa, 0, sizeof(oa));
    oa.psi = s->psi;
    oa.dim = s->pb.dim;
    double dv = 1.0;
    for (int a = 0; a < 3; ++a) {
        oa.n[a] = s->pb.n[a];
        oa.dx[a] = (a < s->pb.dim) ? s->pb.dx[a] : 0.0;
        oa.cen[a] = 0.5 * (s->pb.n[a] - 1);
        oa.w2h[a] = (a < s->pb.dim) ? 0.5 * s->pb.omega[a] * s->pb.omega[a] : 0.0;
        if (a < s->pb.dim) dv *= s->pb.dx[a];
    }
    oa.npts = P.npts;
    oa.partial = reinterpret_cast<double *>(s->ws + P.off_obspart);
    oa.scale = s->pending ? scal_ptr(s) : nullptr;
    hipError_t e = launch_obs_partials(P.elem, oa, P.obs_grid, 256, s->st);
    if (e == hipSuccess) e = launch_obs_final(oa.partial, P.obs_grid, dv, s->g, dobs, s->st);
    return e;
}

// An observation row from its 13 results (h) at global step `step`.
static int obs_from_host(const double *h, int64_t step, sscn_obs *out)
{
    out->step = step;
    out->norm = h[0];
    out->mu = h[1];
    out->energy = h[2];
    out->ekin = h[3];
    out->epot = h[4];
    out->eint = h[5];
    for (int a = 0; a < 3; ++a) {
        out->mean[a] = h[6 + a];
        out->msq[a] = h[9 + a];
    }
    out->status = (h[12] != 0.0) ? SSCN_OK : SSCN_E_NONFINITE;
    out->pad_ = 0;
    return out->status;
}

int sscn_observe(sscn_solver *s, sscn_obs *out)
{
    if (!s || !out) return SSCN_E_INVALID;
    double *dobs = nullptr;
    if (obs_enqueue(s, &dobs) != hipSuccess) return SSCN_E_HIP;
    if (hipMemcpyAsync(s->host_obs, dobs, 13 * sizeof(double), hipMemcpyDeviceToHost, s->st) != hipSuccess)
        return SSCN_E_HIP;
    if (hipStreamSynchronize(s->st) != hipSuccess) return SSCN_E_HIP;
    return obs_from_host(s->host_obs, s->step, out);
}

// sscn_run without a convergence test: observations are queued behind the
// steps, their results copied into pinned host rows without waits, and read
// back once per group of kRunGroup observations.
constexpr int64_t kRunGroup = 4096;

static int run_queued(sscn_solver *s, int64_t max_steps, sscn_obs *trace, int64_t trace_cap, int64_t *rows)
{
    const int64_t every = s->pb.observe_every;
    std::vector<int64_t> at;
    try {
        at.resize((size_t)kRunGroup);
    } catch (...) {
        return SSCN_E_INVALID;
    }
    // the observation rows are written by the final-sum kernel straight
    // into mapped pinned host memory (one copy command per observation
    // otherwise: it tripled the time of an observed step at 128^3)
    double *stage = nullptr, *dstage = nullptr;
    if (hipHostMalloc(reinterpret_cast<void **>(&stage), (size_t)kRunGroup * 13 * sizeof(double),
                      hipHostMallocMapped) != hipSuccess)
        return SSCN_E_HIP;
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&dstage), stage, 0) != hipSuccess) {
        (void)hipHostFree(stage);
        return SSCN_E_HIP;
    }
    int64_t nrow = 0, done = 0;
    int rc = SSCN_NOT_CONVERGED;
    bool stop = false;
    while (done < max_steps && !stop) {
        int64_t nq = 0;
        while (done < max_steps && nq < kRunGroup) {
            int64_t k = every - (s->step % every);
            if (k > max_steps - done) k = max_steps - done;
            double *dobs = nullptr;
            if (enqueue_steps(s, k, nullptr, s->pb.geom != SSCN_GEOM_CART) != hipSuccess ||
                obs_enqueue(s, &dobs, dstage + 13 * nq) != hipSuccess) {
                (void)hipStreamSynchronize(s->st);
                (void)hipHostFree(stage);
                return SSCN_E_HIP;
            }
            done += k;
            at[(size_t)nq++] = s->step;
        }
        if (hipStreamSynchronize(s->st) != hipSuccess) {
            (void)hipHostFree(stage);
            return SSCN_E_HIP;
        }
        for (int64_t q = 0; q < nq; ++q) {
            sscn_obs o;
            const int r = obs_from_host(stage + 13 * q, at[(size_t)q], &o);
            if (trace && nrow < trace_cap) trace[nrow] = o;
            ++nrow;
            if (r != SSCN_OK) {
                rc = r;
                stop = true;
                break;
            }
        }
    }
    (void)hipHostFree(stage);
    if (finalize_state(s, nullptr) != hipSuccess) return SSCN_E_HIP;
    if (rows) *rows = std::min(nrow, trace_cap);
    return rc;
}

int sscn_run(sscn_solver *s, int64_t max_steps, double mu_tol, sscn_obs *trace, int64_t trace_cap,
             int64_t *rows)
{
    if (!s || max_steps < 0 || !(mu_tol >= 0.0) || s->pb.observe_every < 1) return SSCN_E_INVALID;
    if (trace_cap < 0 || (trace_cap > 0 && !trace)) return SSCN_E_INVALID;
    if (mu_tol == 0.0) return run_queued(s, max_steps, trace, trace_cap, rows);
    const int64_t every = s->pb.observe_every;
    const bool fin_each = s->pb.geom != SSCN_GEOM_CART;   // symmetric traps: finalize every interval
    int64_t nrow = 0, done = 0;
    bool have_prev = false;
    double prev = 0.0;
    int rc = SSCN_NOT_CONVERGED;
    while (done < max_steps) {
        // advance to the next observation step (global step multiple of `every`)
        int64_t k = every - (s->step % every);
        if (k > max_steps - done) k = max_steps - done;
        // (Cartesian problems leave the renormalisation pending between
        // observations: the observation kernel applies it to its loads)
        if (enqueue_steps(s, k, nullptr, fin_each) != hipSuccess) return SSCN_E_HIP;
        done += k;
        sscn_obs o;
        int r = sscn_observe(s, &o);
        if (r == SSCN_E_HIP) return r;
        if (trace && nrow < trace_cap) trace[nrow] = o;
        ++nrow;
        if (r == SSCN_E_NONFINITE) {
            rc = r;
            break;
        }
        if (s->step % every != 0) break;  // cap reached between observations
        if (have_prev && std::fabs(o.mu - prev) < mu_tol) {
            rc = SSCN_OK;
            break;
        }
        prev = o.mu;
        have_prev = true;
    }
    if (finalize_state(s, nullptr) != hipSuccess) return SSCN_E_HIP;
    if (rows) *rows = std::min(nrow, trace_cap);
    return rc;
}

int sscn_set_g(sscn_solver *s, double g)
{
    if (!s || !std::isfinite(g)) return SSCN_E_INVALID;
    s->g = g;
    drop_graphs(s);           // captured arguments hold the old g
    return SSCN_OK;
}

int sscn_destroy(sscn_solver *s)
{
    if (!s) return SSCN_E_INVALID;
    (void)hipStreamSynchronize(s->st);
    drop_graphs(s);
    if (s->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[s->static_dev] == s) g_static_owner[s->static_dev] = nullptr;
    }
    delete s;
    return SSCN_OK;
}

int sscn_density_1d(sscn_solver *s, int keep, void *d_out)
{
    if (!s || !d_out || keep < 0 || keep >= s->pb.dim) return SSCN_E_INVALID;
    if (s->pb.geom != SSCN_GEOM_CART) return SSCN_E_UNSUPPORTED;
    double w = 1.0;
    for (int a = 0; a < s->pb.dim; ++a)
        if (a != keep) w *= s->pb.dx[a];
    double *dens_scratch = reinterpret_cast<double *>(s->ws + s->P.off_dens);
    return launch_density_1d(s->P.elem, s->psi, s->pb.n, keep, w, static_cast<double *>(d_out), dens_scratch,
                             s->P.dens_blocks, s->st) ==
                   hipSuccess
               ? SSCN_OK
               : SSCN_E_HIP;
}

int sscn_density_2d(sscn_solver *s, int drop, void *d_out)
{
    if (!s || !d_out || s->pb.dim != 3 || drop < 0 || drop > 2) return SSCN_E_INVALID;
    if (s->pb.geom != SSCN_GEOM_CART) return SSCN_E_UNSUPPORTED;
    return launch_density_2d(s->P.elem, s->psi, s->pb.n, drop, s->pb.dx[drop], static_cast<double *>(d_out),
                             s->st) == hipSuccess
               ? SSCN_OK
               : SSCN_E_HIP;
}

}  // extern "C"

// sscn_batch_api.cpp -- host runtime of the batched persistent SSCN step.
//
// A batch is a caller-owned device region (the control block: counters,
// instance table, per-instance state and the work list) plus up to
// max_slots admitted instances, each with its own caller-owned state and
// workspace.  sscn_batch_step enqueues one launch of k_batch_step per step;
// on a non-null stream the launches are captured once per step count into a
// hipGraph and replayed.  The kernel reads the instance table and the work
// list through pointers, so admissions and evictions only rewrite device
// memory and never invalidate a captured graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "sscn.h"
#include "sscn_batch.hpp"
#include "sscn_plan.hpp"

using namespace sscn;

namespace {

constexpr size_t kBatchLds = BATCH_LDS;  // dynamic LDS of every persistent block
constexpr int kSpinLimit = 1 << 24;      // bounded waits: ~1 s of polling before giving up

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
int p2ceil(int64_t v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

struct CtlLayout {
    size_t done, inst, state, items, total;
};

CtlLayout ctl_layout(int max_slots, int64_t max_items)
{
    CtlLayout L;
    size_t off = a256(sizeof(BCtl));
    L.done = off;
    off = a256(off + sizeof(int32_t) * 4 * (size_t)max_slots);
    L.inst = off;
    off = a256(off + sizeof(BInst) * (size_t)max_slots);
    L.state = off;
    off = a256(off + sizeof(BState) * (size_t)max_slots);
    L.items = off;
    off = a256(off + sizeof(BItem) * (size_t)max_items);
    L.total = off;
    return L;
}

// Geometry of one instance in the persistent kernel's 1024-thread blocks.
struct BPlan {
    AxisPlan ax[3];
    BAxis bax[3];
    bool big;
    size_t lds;
    size_t off_tab[3], off_norm, off_obs, ws_bytes;
    int obs_tiles;
    int64_t obs_pts;
    int64_t units[3];      // line groups (x) or sub-tile sets (y, z) per pass
};

size_t ltab_size(bool cplx) { return cplx ? 32 : 16; }  // (alpha, m) hi/lo pairs of float / complex<float>

// Points per thread the persistent kernel is compiled for (sscn_batch.hip).
const int kRowChunks[] = {1, 2, 3, 4, 6, 8, 12, 16};   // 12, 16: float only
const int kColChunks[] = {2, 3, 4, 5, 6, 8, 10, 12, 16};  // 10, 12: float only; 16: float, BIG kernel

bool row_chunk_ok(int c, bool cplx)
{
    for (int v : kRowChunks)
        if (v == c) return cplx ? c <= 8 : true;
    return false;
}
bool col_chunk_ok(int c, bool cplx)
{
    for (int v : kColChunks)
        if (v == c) return cplx ? c <= 8 : true;
    return false;
}

// COL geometry for lines of n points with c points per thread: W waves of
// L lanes per line (W*L*c >= n), 16/W sub-tiles of 64/L lines per block.
// The time of one sub-tile set grows like c plus a fixed part (barriers,
// the LDS folds), and a set covers (64/L)*(16/W) lines, so the cost per
// point goes like (c + 6) * L * W; lanes per line beyond 4 also split the
// 128-byte segments of a row of lines, which costs extra.
bool col_geometry(int64_t n, int c, int &L, int &W, double &cost)
{
    const int64_t K = cdiv(n, c);                  // chunks per line
    bool found = false;
    for (int l = 1; l <= 8; l *= 2)
        for (int w = 1; w <= 16; w *= 2) {
            if ((int64_t)w * l < K) continue;
            double q = (double)(c + 6) * l * w * (l == 8 ? 1.25 : 1.0);
            if (!found || q < cost) {
                found = true;
                cost = q;
                L = l;
                W = w;
            }
        }
    return found;
}

// Batch tile hints: shape-keyed chunk choices (0: keep the model's choice),
// set by the tuner.  An instance's geometry still depends only on its shape.
struct BHint {
    int32_t dim, n[3], mode;
    int32_t chunk[3];
};
std::mutex g_bhint_mu;
std::vector<BHint> g_bhints;

bool bhint_find(const sscn_problem &pb, int32_t chunk[3])
{
    std::lock_guard<std::mutex> lk(g_bhint_mu);
    for (const BHint &h : g_bhints)
        if (h.dim == pb.dim && h.n[0] == pb.n[0] && h.n[1] == pb.n[1] && h.n[2] == pb.n[2] && h.mode == pb.mode) {
            for (int a = 0; a < 3; ++a) chunk[a] = h.chunk[a];
            return true;
        }
    return false;
}

// Grid points per work item of an instance: about 1/parts of the instance
// per pass, at least 32K and at most 256K.  Each item pays a claim, a wait
// and a release (an L2 write-back): fewer, larger items cost less per point
// when the batch fills the device; more, smaller ones spread a few running
// instances over more blocks (latency).  parts is a setting of the batch
// (sscn_batch_set_split), fixed while it holds instances, so an instance's
// geometry depends only on its shape and that setting.
constexpr int kDefaultSplit = 32;

int64_t item_points(int64_t npts, int parts)
{
    return std::min<int64_t>(262144, std::max<int64_t>(32768, npts / parts));
}

int batch_plan(const sscn_problem &pb, BPlan &B, int parts = kDefaultSplit)
{
    int32_t hint[3] = {0, 0, 0};
    bhint_find(pb, hint);
    std::memset(&B, 0, sizeof(B));
    const bool cplx = pb.mode == SSCN_REAL;
    const size_t S = cplx ? 8 : 4;
    const int64_t npts = (int64_t)pb.n[0] * pb.n[1] * pb.n[2];
    const int64_t nx = pb.n[0], ny = pb.n[1];
    size_t lds = 0;
    for (int a = 0; a < pb.dim; ++a) {
        AxisPlan &X = B.ax[a];
        BAxis &Y = B.bax[a];
        const int64_t n = pb.n[a];
        X.n = (int)n;
        X.nlines = npts / n;
        const double s = pb.dt / (4.0 * pb.dx[a] * pb.dx[a]);
        X.sig_re = cplx ? 0.0 : s;
        X.sig_im = cplx ? s : 0.0;
        if (a == 0) {
            X.kind = K_ROW;
            X.m1 = (int)ny;
            X.s1 = nx;
            X.s2 = nx * ny;
            X.stride = 1;
            // single-wave lines: up to 16 points per thread (8 complex) for
            // a 1D line, which runs whole steps in one block (the solo
            // kernel); up to 4 for the x lines of 2D and 3D instances, whose
            // longer single-wave forms spill in the persistent kernel
            // (752 B per lane at 8 points): those lines take 4 points per
            // thread over several waves instead
            const int cmax1 = pb.dim == 1 ? (cplx ? 8 : 16) : 4;
            int c = cmax1 + 1;
            for (int v : kRowChunks)            // fewest points per thread that cover the line
                if (v <= cmax1 && row_chunk_ok(v, cplx) && (int64_t)v * 64 >= n) {
                    c = v;
                    break;
                }
            if (hint[a] > 0 && hint[a] <= cmax1 && row_chunk_ok(hint[a], cplx) && (int64_t)hint[a] * 64 >= n)
                c = hint[a];
            int wpl = 1;
            if (c > cmax1) {
                c = pb.dim == 1 ? 8 : 4;        // multi-wave lines, 8 (1D) or 4 points per thread
                wpl = p2ceil(cdiv(n, 64 * c));
                if (wpl > 16 && c == 4) {
                    c = 8;
                    wpl = p2ceil(cdiv(n, 64 * 8));
                }
                if (wpl > 16) {
                    // ... or, long 1D lines, 12 (real, when 16 waves of 12
                    // cover the line: fewer points per thread and fewer
                    // waves past the line end than 16) or 16
                    c = (!cplx && n <= (int64_t)16 * 64 * 12) ? 12 : 16;
                    wpl = p2ceil(cdiv(n, 64 * c));
                    B.big = true;
                }
                if (wpl > 16) return SSCN_E_UNSUPPORTED;
            }
            X.C = c;
            X.wpl = wpl;
            X.lpb = 16 / wpl;
            X.tab_entries = (size_t)c * 64 * wpl;
            Y.lpi = X.lpb;
            // several line groups per item (item_points)
            const int64_t units = cdiv(X.nlines, X.lpb);
            Y.rep = (int)std::max<int64_t>(1, std::min<int64_t>(64, item_points(npts, parts) / std::max<int64_t>(1, (int64_t)X.lpb * n)));
            B.units[a] = units;
            Y.rep = (int)std::min<int64_t>(Y.rep, units);
            Y.ntiles = (int)cdiv(units, Y.rep);
            lds = std::max(lds, wpl == 1 ? (size_t)c * 64 * ltab_size(cplx) : (size_t)16 * 4 * S);
        } else {
            X.kind = K_COL;
            X.m1 = (int)nx;
            X.s1 = 1;
            X.s2 = (a == 1) ? nx * ny : nx;
            X.stride = (a == 1) ? nx : nx * ny;
            // the cheapest chunk by the cost model (16 only for lines that
            // need it: it takes the BIG kernel), or the hinted one
            int c = 0, L = 0, W = 0;
            double best = 0.0;
            for (int v : kColChunks) {
                if (!col_chunk_ok(v, cplx) || (v == 16 && c != 0)) continue;
                int l, w;
                double q;
                if (!col_geometry(n, v, l, w, q)) continue;
                if (c == 0 || q < best) {
                    c = v;
                    L = l;
                    W = w;
                    best = q;
                }
            }
            if (hint[a] > 0 && col_chunk_ok(hint[a], cplx)) {
                int l, w;
                double q;
                if (col_geometry(n, hint[a], l, w, q)) {
                    c = hint[a];
                    L = l;
                    W = w;
                }
            }
            if (c == 0) return SSCN_E_UNSUPPORTED;
            if (c == 16) B.big = true;
            X.C = c;
            X.W = W;
            X.L = L;
            X.tab_entries = (size_t)W * L * c;
            Y.tpi = 16 / W;
            const int64_t lines_per_set = (int64_t)Y.tpi * (64 / L);
            const int64_t units = cdiv(X.nlines, lines_per_set);
            Y.rep = (int)std::max<int64_t>(1, std::min<int64_t>(64, item_points(npts, parts) / std::max<int64_t>(1, lines_per_set * n)));
            B.units[a] = units;
            Y.rep = (int)std::min<int64_t>(Y.rep, units);
            Y.ntiles = (int)cdiv(units, Y.rep);
            lds = std::max(lds, (size_t)W * L * c * ltab_size(cplx) + (size_t)Y.tpi * 2 * W * 64 * S);
        }
        table_meta(X, true);
        Y.kind = X.kind;
        Y.C = X.C;
        Y.wpl = X.wpl;
        Y.W = X.W;
        Y.L = X.L;
        Y.nlines = X.nlines;
        Y.stride = X.stride;
        Y.s1 = X.s1;
        Y.s2 = X.s2;
        Y.m1 = X.m1;
        Y.sig_re = X.sig_re;
        Y.sig_im = X.sig_im;
        Y.lt.n = X.n;
        Y.lt.i_conv = X.i_conv;
        Y.lt.ac_re = X.ac_re;
        Y.lt.ac_im = X.ac_im;
        Y.lt.mc_re = X.mc_re;
        Y.lt.mc_im = X.mc_im;
        Y.lt.depth = X.depth;
    }
    if (lds > kBatchLds) return SSCN_E_UNSUPPORTED;
    B.lds = lds;
    B.obs_pts = std::max<int64_t>(BATCH_OBS_PTS, item_points(npts, parts));
    B.obs_tiles = (int)cdiv(npts, B.obs_pts);
    // the partials are sized for the finest split (one line group or set
    // per item, BATCH_OBS_PTS per observation tile), so the workspace of a
    // shape does not depend on the batch's setting
    size_t off = 0;
    for (int a = 0; a < pb.dim; ++a) {
        B.off_tab[a] = off;
        off = a256(off + B.ax[a].tab_entries * sizeof(TabEntry));
    }
    B.off_norm = off;
    off = a256(off + sizeof(double) * (size_t)B.units[pb.dim - 1]);
    B.off_obs = off;
    off = a256(off + sizeof(double) * BATCH_NOBS * (size_t)cdiv(npts, BATCH_OBS_PTS));
    B.ws_bytes = off;
    return SSCN_OK;
}

int batch_validate(const sscn_problem *pb)
{
    int v = validate(pb);
    if (v != SSCN_OK) return v;
    if (pb->prec != SSCN_F32) return SSCN_E_UNSUPPORTED;  // the batch runs the FP32 forms
    if (pb->geom != SSCN_GEOM_CART) return SSCN_E_UNSUPPORTED;  // and the Cartesian traps
    if (pb->mode == SSCN_IMAG && pb->renorm_every != 1) return SSCN_E_INVALID;
    if (pb->observe_every < 1) return SSCN_E_INVALID;
    return SSCN_OK;
}

}  // namespace

struct sscn_batch {
    int max_slots;
    int parts;                      // item split (item_points), fixed while instances are admitted
    int64_t max_items;
    char *ctl;
    CtlLayout lay;
    hipStream_t st;
    int grid_small, grid_big;
    std::vector<BPlan> plan;
    std::vector<char> used;
    std::vector<int64_t> work;      // work estimate per slot (ordering of the list)
    BInst *h_inst;                  // pinned staging
    BState *h_state;                // pinned mirror of the device state
    BState *h_state_init;           // pinned staging of state resets
    BItem *h_items;                 // pinned work list
    int32_t *h_total;
    bool dirty;
    int mode;                       // MODE_* of the current work list
    int32_t n_fast;                 // solo items at the head of the list that the solo kernel runs
    bool full;                      // the persistent kernel's list needs its form with every x-line variant
    bool big_step, big_solo;        // its items (and the fast solo items) need the BIG forms
    hipStream_t st2;                // second stream of MODE_SPLIT (null without a caller stream)
    hipEvent_t ev_fork, ev_join;
    int32_t total;
    std::map<std::pair<int, int64_t>, hipGraphExec_t> graphs;
    int64_t reg_launched;           // persistent launches enqueued since the list was uploaded
    hipEvent_t ev;
    bool ev_valid;
};

// How a step is launched:
//   UNION      one persistent launch runs everything (solo items cycle in it)
//   SOLO_ONLY  every instance is a fast solo one: k_batch_solo alone
//   SPLIT      k_batch_solo for the fast solo instances on the second stream
//              beside the persistent launch of the rest (caller stream only)
enum { MODE_UNION = 0, MODE_SOLO_ONLY = 1, MODE_SPLIT = 2 };

static BCtl *ctl_of(sscn_batch *b) { return reinterpret_cast<BCtl *>(b->ctl); }

// A solo instance the solo kernel has a register-resident form for: a table
// head within the first wave's points, and not a complex line of 16 points
// per thread.
static bool solo_fast_ok(const BInst &I)
{
    return I.solo && std::min(I.ax[0].lt.i_conv, I.ax[0].lt.n) <= BATCH_SOLO_HEAD && I.ax[0].lt.i_conv <= 64 * I.ax[0].C &&
           !(I.elem == 3 && I.ax[0].C == 16);
}
static BInst *dinst(sscn_batch *b) { return reinterpret_cast<BInst *>(b->ctl + b->lay.inst); }
static BState *dstate(sscn_batch *b) { return reinterpret_cast<BState *>(b->ctl + b->lay.state); }

// Work list in dependency order: every pass of every slot before the next pass.
static int64_t count_items(const sscn_batch *b)
{
    int64_t t = 0;
    for (int i = 0; i < b->max_slots; ++i) {
        if (!b->used[i]) continue;
        const BInst &I = b->h_inst[i];
        if (I.solo) {
            t += 1;
            continue;
        }
        for (int a = 0; a < I.dim; ++a) t += I.ax[a].ntiles;
        t += I.obs_tiles + 1;
    }
    return t;
}

static void build_items(sscn_batch *b)
{
    std::vector<int> order;
    for (int i = 0; i < b->max_slots; ++i)
        if (b->used[i]) order.push_back(i);
    // larger instances first inside each pass (longest-processing-time order)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->work[x] > b->work[y]; });
    int32_t t = 0;
    // solo instances first (those the solo kernel runs at the very head):
    // their items never wait and overlap the rest
    for (int i : order)
        if (solo_fast_ok(b->h_inst[i])) b->h_items[t++] = BItem{(uint16_t)i, (uint8_t)BP_SOLO, 0, 0};
    b->n_fast = t;
    for (int i : order)
        if (b->h_inst[i].solo && !solo_fast_ok(b->h_inst[i])) b->h_items[t++] = BItem{(uint16_t)i, (uint8_t)BP_SOLO, 0, 0};
    for (int pass = BP_X; pass <= BP_FIN; ++pass)
        for (int i : order) {
            const BInst &I = b->h_inst[i];
            if (I.solo) continue;
            int nt = 0;
            if (pass <= BP_Z) nt = (pass < I.dim) ? I.ax[pass].ntiles : 0;
            else if (pass == BP_OBS) nt = I.obs_tiles;
            else nt = 1;
            for (int k = 0; k < nt; ++k) b->h_items[t++] = BItem{(uint16_t)i, (uint8_t)pass, 0, k};
        }
    b->total = t;
}

static hipError_t upload_items(sscn_batch *b)
{
    hipError_t e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) return e;
    build_items(b);
    bool regular = false;
    for (int i = 0; i < b->max_slots; ++i)
        if (b->used[i] && !b->h_inst[i].solo) regular = true;
    b->h_total[2] = regular ? 1 : BATCH_SOLO_ONLY;
    if (b->total > 0 && b->n_fast == b->total) b->mode = MODE_SOLO_ONLY;
    else if (b->n_fast > 0 && b->st2 && b->n_fast <= b->grid_small / 2) b->mode = MODE_SPLIT;
    else b->mode = MODE_UNION;
    // the persistent kernel's list: without the fast solo items in SPLIT
    *b->h_total = b->mode == MODE_SPLIT ? b->total - b->n_fast : b->total;
    // its kernel form: every x-line variant when the list holds a 1D or solo
    // item or an x line of more than 4 points per thread, else the form
    // without them (fewer spilled registers)
    b->full = false;
    for (int k = b->mode == MODE_SPLIT ? b->n_fast : 0; k < b->total && !b->full; ++k) {
        const BInst &I = b->h_inst[b->h_items[k].slot];
        if (I.solo || I.dim == 1 || I.ax[0].C > 4) b->full = true;
    }
    // the BIG forms, for each kernel only where its own items need them
    b->big_step = b->big_solo = false;
    for (int k = 0; k < b->total; ++k) {
        if (!b->plan[b->h_items[k].slot].big) continue;
        if (k < b->n_fast) b->big_solo = true;
        if (b->mode != MODE_SPLIT || k >= b->n_fast) b->big_step = true;
    }
    b->h_total[3] = 0;                                     // the launch count restarts with the list
    b->reg_launched = 0;
    if (b->total > 0) {
        e = hipMemcpyAsync(b->ctl + b->lay.items, b->h_items, sizeof(BItem) * (size_t)b->total,
                           hipMemcpyHostToDevice, b->st);
        if (e != hipSuccess) return e;
    }
    e = hipMemcpyAsync(&ctl_of(b)->total_items, b->h_total, sizeof(int32_t), hipMemcpyHostToDevice, b->st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&ctl_of(b)->solo_min, b->h_total + 2, sizeof(int32_t), hipMemcpyHostToDevice, b->st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&ctl_of(b)->reg_epoch, b->h_total + 3, sizeof(int32_t), hipMemcpyHostToDevice, b->st);
    if (e != hipSuccess) return e;
    b->dirty = false;
    return hipStreamSynchronize(b->st);
}

static BatchArgs batch_args(sscn_batch *b)
{
    BatchArgs a;
    a.ctl = ctl_of(b);
    a.done = reinterpret_cast<int32_t *>(b->ctl + b->lay.done);
    a.inst = dinst(b);
    a.state = dstate(b);
    a.items = reinterpret_cast<const BItem *>(b->ctl + b->lay.items);
    a.spin_limit = kSpinLimit;
    return a;
}

extern "C" {

int sscn_batch_ctl_bytes(int32_t max_slots, int64_t max_items, size_t *bytes)
{
    if (max_slots < 1 || max_slots > 65535 || max_items < 1 || max_items > (1LL << 30) || !bytes)
        return SSCN_E_INVALID;
    *bytes = ctl_layout(max_slots, max_items).total;
    return SSCN_OK;
}

int sscn_batch_workspace_bytes(const sscn_problem *pb, size_t *bytes)
{
    int v = batch_validate(pb);
    if (v != SSCN_OK) return v;
    if (!bytes) return SSCN_E_INVALID;
    BPlan B;
    v = batch_plan(*pb, B);
    if (v != SSCN_OK) return v;
    *bytes = B.ws_bytes;
    return SSCN_OK;
}

int sscn_batch_set_tile_hint(const sscn_problem *pb, const int32_t chunk[3])
{
    if (!chunk || validate(pb) != SSCN_OK) return SSCN_E_INVALID;
    const bool cplx = pb->mode == SSCN_REAL;
    for (int a = 0; a < 3; ++a) {
        if (chunk[a] == 0) continue;
        if (a >= pb->dim) return SSCN_E_INVALID;
        if (a == 0 ? !row_chunk_ok(chunk[a], cplx) : !col_chunk_ok(chunk[a], cplx)) return SSCN_E_INVALID;
    }
    BHint h;
    std::memset(&h, 0, sizeof(h));
    h.dim = pb->dim;
    h.mode = pb->mode;
    for (int a = 0; a < 3; ++a) {
        h.n[a] = pb->n[a];
        h.chunk[a] = chunk[a];
    }
    try {
        std::lock_guard<std::mutex> lk(g_bhint_mu);
        for (BHint &e : g_bhints)
            if (e.dim == h.dim && e.n[0] == h.n[0] && e.n[1] == h.n[1] && e.n[2] == h.n[2] && e.mode == h.mode) {
                e = h;
                return SSCN_OK;
            }
        g_bhints.push_back(h);
    } catch (...) {
        return SSCN_E_INVALID;
    }
    return SSCN_OK;
}

int sscn_batch_clear_tile_hints(void)
{
    std::lock_guard<std::mutex> lk(g_bhint_mu);
    g_bhints.clear();
    return SSCN_OK;
}

int sscn_batch_plan_info(const sscn_problem *pb, int32_t *info, int32_t cap)
{
    int v = batch_validate(pb);
    if (v != SSCN_OK) return v;
    if (!info || cap < 24) return SSCN_E_INVALID;
    BPlan B;
    v = batch_plan(*pb, B);
    if (v != SSCN_OK) return v;
    for (int a = 0; a < 3; ++a) {
        int32_t *o = info + 8 * a;
        if (a >= pb->dim) {
            for (int q = 0; q < 8; ++q) o[q] = -1;
            continue;
        }
        const BAxis &X = B.bax[a];
        o[0] = X.kind == K_ROW ? 0 : 1;
        o[1] = X.C;
        o[2] = X.kind == K_ROW ? X.wpl : X.W;
        o[3] = X.kind == K_ROW ? 1 : X.L;
        o[4] = X.ntiles;
        o[5] = X.rep;
        o[6] = X.lt.depth;
        o[7] = B.big ? 1 : 0;
    }
    return SSCN_OK;
}

int sscn_batch_create(int32_t max_slots, int64_t max_items, void *d_ctl, size_t ctl_bytes, void *hip_stream,
                      sscn_batch **out)
{
    size_t need = 0;
    int v = sscn_batch_ctl_bytes(max_slots, max_items, &need);
    if (v != SSCN_OK) return v;
    if (!d_ctl || !out || ctl_bytes < need || reinterpret_cast<uintptr_t>(d_ctl) % 256) return SSCN_E_INVALID;
    sscn_batch *b = new (std::nothrow) sscn_batch;
    if (!b) return SSCN_E_INVALID;
    b->max_slots = max_slots;
    b->parts = kDefaultSplit;
    b->max_items = max_items;
    b->ctl = static_cast<char *>(d_ctl);
    b->lay = ctl_layout(max_slots, max_items);
    b->st = static_cast<hipStream_t>(hip_stream);
    b->dirty = true;
    b->mode = MODE_UNION;
    b->n_fast = 0;
    b->full = true;
    b->big_step = b->big_solo = false;
    b->reg_launched = 0;
    b->st2 = nullptr;
    b->ev_fork = b->ev_join = nullptr;
    b->total = 0;
    b->ev_valid = false;
    b->h_inst = nullptr;
    b->h_state = nullptr;
    b->h_state_init = nullptr;
    b->h_items = nullptr;
    b->h_total = nullptr;
    auto fail = [&](int code) {
        if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
        if (b->ev_join) (void)hipEventDestroy(b->ev_join);
        if (b->st2) (void)hipStreamDestroy(b->st2);
        if (b->h_inst) (void)hipHostFree(b->h_inst);
        if (b->h_state) (void)hipHostFree(b->h_state);
        if (b->h_state_init) (void)hipHostFree(b->h_state_init);
        if (b->h_items) (void)hipHostFree(b->h_items);
        if (b->h_total) (void)hipHostFree(b->h_total);
        delete b;
        return code;
    };
    try {
        b->plan.resize(max_slots);
        b->used.assign(max_slots, 0);
        b->work.assign(max_slots, 0);
    } catch (...) {
        return fail(SSCN_E_INVALID);
    }
    if (hipHostMalloc((void **)&b->h_inst, sizeof(BInst) * max_slots) != hipSuccess ||
        hipHostMalloc((void **)&b->h_state, sizeof(BState) * max_slots) != hipSuccess ||
        hipHostMalloc((void **)&b->h_state_init, sizeof(BState) * max_slots) != hipSuccess ||
        hipHostMalloc((void **)&b->h_items, std::max(sizeof(BItem) * (size_t)max_items, sizeof(BCtl))) != hipSuccess ||
        hipHostMalloc((void **)&b->h_total, sizeof(int32_t) * 64) != hipSuccess)
        return fail(SSCN_E_HIP);
    std::memset(b->h_inst, 0, sizeof(BInst) * max_slots);
    std::memset(b->h_state, 0, sizeof(BState) * max_slots);
    std::memset(b->h_state_init, 0, sizeof(BState) * max_slots);
    // persistent grid: as many 1024-thread blocks as the device keeps resident
    int dev = 0, cus = 0, per_small = 0, per_big = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        batch_step_occupancy(false, kBatchLds, &per_small) != hipSuccess ||
        batch_step_occupancy(true, kBatchLds, &per_big) != hipSuccess)
        return fail(SSCN_E_HIP);
    b->grid_small = std::max(1, cus * std::max(1, per_small));
    b->grid_big = std::max(1, cus * std::max(1, per_big));
    // the second stream of MODE_SPLIT (default priority, like the caller's)
    if (b->st && (hipStreamCreateWithFlags(&b->st2, hipStreamNonBlocking) != hipSuccess ||
                  hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
                  hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess))
        return fail(SSCN_E_HIP);
    // clear the control block (not captured: plain memset)
    BCtl *hc = reinterpret_cast<BCtl *>(b->h_items);  // scratch use of the pinned buffer (sized for it)
    if (hipMemsetAsync(b->ctl, 0, need, b->st) != hipSuccess) return fail(SSCN_E_HIP);
    BCtl c0;
    std::memset(&c0, 0, sizeof(c0));
    c0.max_slots = max_slots;
    std::memcpy(hc, &c0, sizeof(c0));
    if (hipMemcpyAsync(b->ctl, hc, sizeof(BCtl), hipMemcpyHostToDevice, b->st) != hipSuccess ||
        hipStreamSynchronize(b->st) != hipSuccess || hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess)
        return fail(SSCN_E_HIP);
    *out = b;
    return SSCN_OK;
}

int sscn_batch_set_split(sscn_batch *b, int32_t parts)
{
    if (!b || parts < 1 || parts > 4096) return SSCN_E_INVALID;
    for (int i = 0; i < b->max_slots; ++i)
        if (b->used[i]) return SSCN_E_INVALID;
    b->parts = parts;
    return SSCN_OK;
}

int sscn_batch_admit(sscn_batch *b, int32_t slot, const sscn_problem *pb, void *d_psi, void *d_ws, double mu_tol,
                     int64_t max_steps)
{
    if (!b || slot < 0 || slot >= b->max_slots) return SSCN_E_INVALID;
    if (b->used[slot]) return SSCN_E_NOSPACE;
    int v = batch_validate(pb);
    if (v != SSCN_OK) return v;
    if (!d_psi || !d_ws || reinterpret_cast<uintptr_t>(d_ws) % 256 || reinterpret_cast<uintptr_t>(d_psi) % 16)
        return SSCN_E_INVALID;
    if (!(mu_tol >= 0.0) || !std::isfinite(mu_tol) || max_steps < 1) return SSCN_E_INVALID;
    BPlan B;
    v = batch_plan(*pb, B, b->parts);
    if (v != SSCN_OK) return v;

    BInst I;
    std::memset(&I, 0, sizeof(I));
    I.psi = d_psi;
    I.elem = pb->mode == SSCN_REAL ? 3 : 1;
    I.dim = pb->dim;
    I.npts = (int64_t)pb->n[0] * pb->n[1] * pb->n[2];
    I.pp.dt = pb->dt;
    I.pp.g = pb->g;
    I.dvol = 1.0;
    for (int a = 0; a < 3; ++a) {
        I.pp.n[a] = pb->n[a];
        I.pp.dx[a] = (a < pb->dim) ? pb->dx[a] : 0.0;
        I.pp.cen[a] = 0.5 * (pb->n[a] - 1);
        I.pp.w2h[a] = (a < pb->dim) ? 0.5 * pb->omega[a] * pb->omega[a] : 0.0;
        if (a < pb->dim) I.dvol *= pb->dx[a];
    }
    char *ws = static_cast<char *>(d_ws);
    for (int a = 0; a < pb->dim; ++a) {
        I.ax[a] = B.bax[a];
        I.ax[a].lt.tab = reinterpret_cast<const TabEntry *>(ws + B.off_tab[a]);
    }
    I.norm_part = reinterpret_cast<double *>(ws + B.off_norm);
    I.obs_part = reinterpret_cast<double *>(ws + B.off_obs);
    I.obs_tiles = B.obs_tiles;
    I.obs_pts = B.obs_pts;
    I.observe_every = pb->observe_every;
    I.mu_tol = mu_tol;
    I.max_steps = max_steps;
    I.imag = pb->mode == SSCN_IMAG;
    I.last_pass = pb->dim - 1;
    for (int p = 0; p < BP_NPASS; ++p) {
        I.dep[p] = -1;
        I.need[p] = 0;
    }
    for (int p = 1; p < pb->dim; ++p) {
        I.dep[p] = p - 1;
        I.need[p] = B.bax[p - 1].ntiles;
    }
    I.dep[BP_OBS] = I.last_pass;
    I.need[BP_OBS] = B.bax[I.last_pass].ntiles;
    I.dep[BP_FIN] = BP_OBS;
    I.need[BP_FIN] = B.obs_tiles;
    I.solo = pb->dim == 1 && B.bax[0].ntiles == 1 && B.obs_tiles == 1;

    // the work list must fit
    const int was = b->used[slot];
    b->used[slot] = 1;
    b->h_inst[slot] = I;
    const int64_t tot = count_items(b);
    if (tot > b->max_items) {
        b->used[slot] = (char)was;
        return SSCN_E_NOSPACE;
    }

    // FP64 tables into the instance workspace
    try {
        std::vector<char> img(B.off_norm, 0);
        sscn_problem p2 = *pb;
        Plan P;
        std::memset(&P, 0, sizeof(P));
        std::vector<TabEntry> tab;
        for (int a = 0; a < pb->dim; ++a) {
            P.ax[a] = B.ax[a];
            build_table(p2, P, a, tab);
            std::memcpy(img.data() + B.off_tab[a], tab.data(), tab.size() * sizeof(TabEntry));
        }
        if (hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, b->st) != hipSuccess ||
            hipStreamSynchronize(b->st) != hipSuccess) {
            b->used[slot] = (char)was;
            return SSCN_E_HIP;
        }
    } catch (...) {
        b->used[slot] = (char)was;
        return SSCN_E_INVALID;
    }
    BState S0;
    std::memset(&S0, 0, sizeof(S0));
    S0.status = BS_RUNNING;
    S0.scale = 1.0;
    b->h_state_init[slot] = S0;
    if (hipMemcpyAsync(dinst(b) + slot, b->h_inst + slot, sizeof(BInst), hipMemcpyHostToDevice, b->st) !=
            hipSuccess ||
        hipMemcpyAsync(dstate(b) + slot, b->h_state_init + slot, sizeof(BState), hipMemcpyHostToDevice, b->st) !=
            hipSuccess ||
        hipStreamSynchronize(b->st) != hipSuccess) {
        b->used[slot] = (char)was;
        return SSCN_E_HIP;
    }
    b->plan[slot] = B;
    b->work[slot] = I.npts * pb->dim;
    b->dirty = true;
    return SSCN_OK;
}

int sscn_batch_evict(sscn_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->used[slot]) return SSCN_E_INVALID;
    const BInst &I = b->h_inst[slot];
    if (I.imag && launch_batch_scale(I.elem, I.psi, I.npts, &dstate(b)[slot].scale, b->st) != hipSuccess)
        return SSCN_E_HIP;
    BState S0;
    std::memset(&S0, 0, sizeof(S0));
    S0.status = BS_EMPTY;
    b->h_state_init[slot] = S0;
    if (hipMemcpyAsync(&dstate(b)[slot].status, &b->h_state_init[slot].status, sizeof(int32_t),
                       hipMemcpyHostToDevice, b->st) != hipSuccess ||
        hipStreamSynchronize(b->st) != hipSuccess)
        return SSCN_E_HIP;
    b->used[slot] = 0;
    b->dirty = true;
    return SSCN_OK;
}

int sscn_batch_step(sscn_batch *b, int32_t nsteps)
{
    if (!b || nsteps < 0) return SSCN_E_INVALID;
    if (b->dirty && upload_items(b) != hipSuccess) return SSCN_E_HIP;
    if (nsteps > 0 && b->total > 0) {
        const bool solo = b->mode == MODE_SOLO_ONLY;
        const bool split = b->mode == MODE_SPLIT;
        const bool big = solo ? b->big_solo : b->big_step;   // the form this call's graph launches
        // the launches on the caller's stream: the persistent kernel over the
        // list (in SPLIT, the part after the fast solo items, with a grid that
        // leaves the solo blocks' CUs free), or the solo kernel alone.  No
        // more blocks than items: a block that finds no item still costs a
        // dispatch and two atomics on the shared counters.
        BatchArgs a = batch_args(b);
        const BatchArgs a_solo = a;
        int items = (int)b->total, cap = big ? b->grid_big : b->grid_small;
        if (split) {
            a.items += b->n_fast;
            items -= b->n_fast;
            cap -= b->n_fast;
        }
        const int grid = solo ? items : std::max(1, std::min(cap, items));
        auto launch = [&]() {
            return solo ? launch_batch_solo(a, big, grid, kBatchLds, b->st, BATCH_SOLO_ONLY, -1)
                        : launch_batch_step(a, big, b->full, grid, kBatchLds, b->st);
        };
        if (split) {
            // the solo kernel on the second stream, once for the whole call:
            // its blocks step until the persistent kernel has counted this
            // call's launches (and at most a bounded number of steps, so they
            // end even if those launches were held back)
            b->reg_launched += nsteps;
            const int steps = (int)std::min<int64_t>(1 << 30, (int64_t)nsteps * BATCH_SOLO_MAX);
            if (hipEventRecord(b->ev_fork, b->st) != hipSuccess || hipStreamWaitEvent(b->st2, b->ev_fork, 0) != hipSuccess ||
                launch_batch_solo(a_solo, b->big_solo, b->n_fast, kBatchLds, b->st2, steps, (int32_t)b->reg_launched) !=
                    hipSuccess ||
                hipEventRecord(b->ev_join, b->st2) != hipSuccess)
                return SSCN_E_HIP;
        }
        if (b->st == nullptr) {
            for (int k = 0; k < nsteps; ++k)
                if (launch() != hipSuccess) return SSCN_E_HIP;
        } else {
            // replayed from a graph per (steps, launch shape, list offset)
            const auto key = std::make_pair(nsteps, (int64_t)(8 * grid + (b->full ? 4 : 0) + (big ? 2 : 0) + (solo ? 1 : 0)) *
                                                            65536 +
                                                        (split ? b->n_fast : 0));
            auto it = b->graphs.find(key);
            if (it == b->graphs.end() && b->graphs.size() >= 16) {
                for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
                b->graphs.clear();
            }
            if (it == b->graphs.end()) {
                hipGraph_t g = nullptr;
                hipGraphExec_t ex = nullptr;
                if (hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SSCN_E_HIP;
                hipError_t le = hipSuccess;
                for (int k = 0; k < nsteps && le == hipSuccess; ++k) le = launch();
                if (hipStreamEndCapture(b->st, &g) != hipSuccess || le != hipSuccess) return SSCN_E_HIP;
                const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) return SSCN_E_HIP;
                it = b->graphs.emplace(key, ex).first;
            }
            if (hipGraphLaunch(it->second, b->st) != hipSuccess) return SSCN_E_HIP;
        }
        if (split && hipStreamWaitEvent(b->st, b->ev_join, 0) != hipSuccess) return SSCN_E_HIP;
    }
    if (hipMemcpyAsync(b->h_state, dstate(b), sizeof(BState) * b->max_slots, hipMemcpyDeviceToHost, b->st) !=
            hipSuccess ||
        hipEventRecord(b->ev, b->st) != hipSuccess)
        return SSCN_E_HIP;
    b->ev_valid = true;
    return SSCN_OK;
}

int sscn_batch_poll(sscn_batch *b, sscn_batch_slot *out, int32_t nslots, int32_t wait)
{
    if (!b || (nslots > 0 && !out) || nslots < 0) return SSCN_E_INVALID;
    if (b->ev_valid) {
        if (wait) {
            if (hipEventSynchronize(b->ev) != hipSuccess) return SSCN_E_HIP;
        } else {
            const hipError_t q = hipEventQuery(b->ev);
            if (q == hipErrorNotReady) return SSCN_BUSY;
            if (q != hipSuccess) return SSCN_E_HIP;
        }
    }
    const int n = std::min(nslots, b->max_slots);
    for (int i = 0; i < n; ++i) {
        sscn_batch_slot &o = out[i];
        std::memset(&o, 0, sizeof(o));
        const BState &S = b->h_state[i];
        o.state = b->used[i] ? S.status : SSCN_SLOT_EMPTY;
        o.steps = S.step;
        o.last_norm = S.norm;
        o.obs.step = S.obs_step;
        o.obs.norm = S.obs[0];
        o.obs.mu = S.obs[1];
        o.obs.energy = S.obs[2];
        o.obs.ekin = S.obs[3];
        o.obs.epot = S.obs[4];
        o.obs.eint = S.obs[5];
        for (int a = 0; a < 3; ++a) {
            o.obs.mean[a] = S.obs[6 + a];
            o.obs.msq[a] = S.obs[9 + a];
        }
        o.obs.status = (S.status == BS_NONFINITE) ? SSCN_E_NONFINITE : SSCN_OK;
    }
    return SSCN_OK;
}

int sscn_batch_error(sscn_batch *b, int32_t *flag)
{
    if (!b || !flag) return SSCN_E_INVALID;
    if (hipMemcpyAsync(b->h_total + 1, &ctl_of(b)->error, sizeof(int32_t), hipMemcpyDeviceToHost, b->st) !=
            hipSuccess ||
        hipStreamSynchronize(b->st) != hipSuccess)
        return SSCN_E_HIP;
    *flag = b->h_total[1];
    return SSCN_OK;
}

int sscn_batch_destroy(sscn_batch *b)
{
    if (!b) return SSCN_E_INVALID;
    (void)hipStreamSynchronize(b->st);
    if (b->st2) (void)hipStreamSynchronize(b->st2);
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    (void)hipEventDestroy(b->ev);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->st2) (void)hipStreamDestroy(b->st2);
    (void)hipHostFree(b->h_inst);
    (void)hipHostFree(b->h_state);
    (void)hipHostFree(b->h_state_init);
    (void)hipHostFree(b->h_items);
    (void)hipHostFree(b->h_total);
    delete b;
    return SSCN_OK;
}

}  // extern "C"

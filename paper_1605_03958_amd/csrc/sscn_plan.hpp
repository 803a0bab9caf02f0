// sscn_plan.hpp -- kernel plan of one problem: geometry per axis and the
// workspace layout.  Deterministic in the problem (and any tile hint for its
// shape), so the workspace size reported before create matches the plan
// used by create.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "sscn.h"
#include "sscn_dev.hpp"

namespace sscn {

enum { K_ROW = 0, K_COL = 1, K_STREAM = 2, K_RAD = 3 };

struct AxisPlan {
    int kind;
    int n;
    int C;        // points per thread
    int wpl;      // ROW: waves per line
    int seg;      // ROW: lanes per line within a wave (64, or 16: four short lines per wave)
    int lpb;      // ROW: lines per block
    int W;        // COL: waves per block
    int L;        // COL: lanes per line (chunks per line = W * L)
    int grid, block;
    size_t lds;
    size_t tab_off, tab_entries;
    int64_t nlines;
    int m1;
    int64_t s1, s2, stride;
    double sig_re, sig_im;
    // table metadata (see LineTab): first index of the constant tail, the
    // constant entry, and the scan / fold depth of the chunk geometry
    int i_conv;
    double ac_re, ac_im, mc_re, mc_im;
    int depth;
};

struct Plan {
    int elem;
    size_t S;
    int64_t npts;
    AxisPlan ax[3];
    bool sep_pointwise, sep_norm;
    bool fused_norm;       // the last sweep's single block also finalises the norm
    bool fold_norm;        // the next step's x sweep forms the factor from the partials
    int pw_grid, np_norm, obs_grid;
    int dens_blocks;       // row blocks of the n_1D-along-x partial sums
    size_t off_scal, off_obs, off_part, off_obspart, off_dens, ws_bytes;
    size_t off_wline;      // axial trap: radial cell weights of the z lines (n_0 doubles)
};

// Chunk lengths chosen by the tuner for one shape (0 = default choice).
struct TileOverride {
    int row_c;
    int col_c[3];
};

int elem_of(const sscn_problem &pb);
size_t elem_bytes(int elem);
int validate(const sscn_problem *pb);
int make_plan(const sscn_problem &pb, const TileOverride *ov, Plan &P);
void build_table(const sscn_problem &pb, const Plan &P, int a, std::vector<TabEntry> &out);
// Radial axis of a symmetric trap: its table in the layout k_rad reads
// (sscn_sym.hpp) and the cell weights W_i.
void build_rad_table(const sscn_problem &pb, const Plan &P, std::vector<double> &out);
void rad_weights(const sscn_problem &pb, std::vector<double> &w);
// The inner product's volume factor: prod dx (Cartesian), times 2 pi
// (circular, axial) or 4 pi (spherical).
double inner_dvol(const sscn_problem &pb);
// Constant-tail index, constant entry and scan depth of an axis whose kind,
// n, C, W, L and sigma are set.
void table_meta(AxisPlan &X, bool fp32);
// FP64 Thomas coefficients m_i and alpha_i = s m_i of tridiag(-s, 1+2s, -s).
void thomas_coefs(double s_re, double s_im, int n, std::vector<double> &m_re, std::vector<double> &m_im,
                  std::vector<double> &a_re, std::vector<double> &a_im);

// Tile hints registered through the ABI, keyed by (dim, n, mode, prec):
// copies the hint for pb's shape into out and returns true if there is one.
bool tile_hint_copy(const sscn_problem &pb, TileOverride &out);

}  // namespace sscn

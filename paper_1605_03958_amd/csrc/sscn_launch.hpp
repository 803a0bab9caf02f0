// sscn_launch.hpp -- host-side launch interface between the runtime
// (sscn_api.cpp) and the kernels (sscn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sscn_dev.hpp"

namespace sscn {

// Thomas coefficients of one axis as the line kernels read them.  Entries
// at i >= i_conv are all equal to (alpha_inf, m_inf) (the FP64 recurrence
// has reached its fixed point) and are not loaded; entries past the line end
// are zero.  `depth` bounds how many preceding chunks feed a chunk's
// incoming value: the neglected terms carry a product of at least that many
// chunk factors |prod alpha| and are below 2^-64 (FP64) / 2^-35 (FP32) of
// the largest term, i.e. below the rounding of the exact sum.
struct LineTab {
    const TabEntry *tab;
    int32_t n;
    int32_t i_conv;
    double ac_re, ac_im, mc_re, mc_im;
    int32_t depth;         // ROW: Kogge-Stone steps (0..6); COL: chunks folded
};

// x sweep with the pointwise substep fused into its load (ROW geometry).
struct RowArgs {
    void *psi;
    LineTab lt;            // tab lane-major: entry (k, t) at [k * 64 * wpl + t]
    int32_t nlines;        // n_y * n_z
    int32_t wpl;           // waves per line (power of two, <= 16)
    int32_t seg;           // lanes per line within a wave: 64, or 16 (lines of <= 64 points, C = 4)
    int32_t lpb;           // lines per block
    int32_t v16;           // 1: 16-byte groups of 4- or 8-byte values (line length a multiple, psi aligned)
    double sig_re, sig_im; // CN coefficient s
    PointParams pp;
    const double *scale;   // pending renormalisation factor (imaginary time)
    double *partial;       // norm partial per block when this is the last sweep
    // non-null: the factor is not in *scale but formed from the previous
    // step's fold_np (<= 64 * kFoldWaves) norm partials, as k_norm_final would
    const double *fold;
    int32_t fold_np;
    double fold_dvol;
};

// y or z sweep (COL geometry) and the one-thread-per-line fallback.
// Line l starts at (l % m1) * s1 + (l / m1) * s2; its points are `stride`
// apart.
struct ColArgs {
    void *psi;
    LineTab lt;            // tab: entry i at [i]
    int32_t nlines;
    int64_t stride;
    int32_t m1;
    int64_t s1, s2;
    int32_t W;             // COL: waves per block
    int32_t L;             // COL: lanes per line (chunks per line = W * L)
    double sig_re, sig_im;
    double *partial;
    const double *wline;   // last sweep: weight of line l's norm terms at [l % m1] (axial trap), or null
    double *unit_scale;    // non-null: set to 1 (a step that does not renormalise; the x sweep has read it)
};

struct PointArgs {
    void *psi;
    int64_t npts;
    PointParams pp;
    const double *scale;
};

// Kernel launchers.  elem: 0 double, 1 float, 2 complex<double>, 3 complex<float>.
// e0/e1: optional start/stop events that take the kernel's own begin and
// end times (null: a plain launch).
hipError_t launch_row(int elem, int C, bool last, const RowArgs &a, int grid, int block,
                      size_t lds, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_col(int elem, int C, bool last, const ColArgs &a, int grid, int block,
                      size_t lds, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_stream(int elem, const ColArgs &a, int grid, int block, hipStream_t st);
hipError_t launch_pointwise(int elem, const PointArgs &a, int grid, int block, hipStream_t st);
hipError_t launch_norm_partials(int elem, const void *psi, int64_t npts, double *partial,
                                int grid, int block, hipStream_t st);
hipError_t launch_norm_final(const double *partial, int np, double dvol, int do_renorm,
                             double *scalars, hipStream_t st);
hipError_t launch_scale_state(int elem, void *psi, int64_t npts, const double *scalars,
                              int grid, int block, hipStream_t st);
hipError_t launch_set_unit_scale(double *scalars, hipStream_t st);

struct ObsArgs {
    const void *psi;
    int32_t dim;
    int32_t n[3];
    double dx[3], cen[3], w2h[3];
    int64_t npts;
    double *partial;       // 12 doubles per block
    const double *scale;   // non-null: a pending renormalisation factor applied to every loaded value
};
hipError_t launch_obs_partials(int elem, const ObsArgs &a, int grid, int block, hipStream_t st);
// out[0..15]: norm, mu, E, K, P, I, <x>, <y>, <z>, <x^2>, <y^2>, <z^2>, finite flag
hipError_t launch_obs_final(const double *partial, int np, double dvol, double g, double *out,
                            hipStream_t st);

hipError_t launch_density_1d(int elem, const void *psi, const int32_t *n, int keep, double w,
                             double *out, double *scratch, int dens_blocks, hipStream_t st);
hipError_t launch_density_2d(int elem, const void *psi, const int32_t *n, int drop, double w,
                             double *out, hipStream_t st);

}  // namespace sscn

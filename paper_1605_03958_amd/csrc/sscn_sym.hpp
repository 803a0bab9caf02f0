// sscn_sym.hpp -- launch interface of the symmetric-trap kernels
// (sscn_sym.hip) for the runtime (sscn_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sscn {

// Radial table: FP64, structure of arrays, lane-major.  Quantity q of chunk
// point k (cell t * C + k) of thread t is at [q * G * C + k * G + t], with G
// threads per line and C cells per thread; cells past the line end are 0.
//   m, alpha, beta: Thomas elimination of (1 + tau H_r) v = rhs, complex
//     (re, im; im = 0 in imaginary time);
//   L, D, U: theta l_i, theta d_i, theta u_i with H_r psi_i =
//     d_i psi_i - l_i psi_{i-1} - u_i psi_{i+1} and tau = theta (imaginary)
//     or i theta (real), theta = dt / 2;
//   W: the cell weight of the inner product.
enum { RQ_MR, RQ_MI, RQ_AR, RQ_AI, RQ_BR, RQ_BI, RQ_L, RQ_D, RQ_U, RQ_W, RQ_N };

struct RadArgs {
    void *psi;             // line l at psi + l * n (r fastest)
    const double *tab;     // RQ_N * G * C doubles
    int32_t n;             // cells per radial line
    double dt, g;
    double dr, w2h_r;      // omega_r^2 / 2
    double dz, cen_z, w2h_z;   // axial: line l at z = (l - cen_z) dz; 0 otherwise
    const double *scale;   // pending renormalisation factor (imaginary time)
    double *partial;       // last sweep: sum W |psi|^2 per block
    // one-block sweeps that renormalise every step: also finalise here,
    // as the norm's final sum would (scalars[1] = dvol * sum, scalars[0] =
    // its inverse square root); null otherwise
    double *scalars;
    double dvol;
};

struct SymObsArgs {
    const void *psi;
    int32_t nr, nz;
    int32_t k;             // 1 (circular, axial) or 2 (spherical)
    int32_t axial;
    double dr, dz, cen_z, w2h_r, w2h_z;
    int64_t npts;
    double *partial;       // 12 doubles per block, the rows k_obs_final reads
};

// elem: 0 double, 1 float, 2 complex<double>, 3 complex<float>; C in {4, 8, 16}
hipError_t launch_rad(int elem, int C, bool last, const RadArgs &a, int grid, int block, hipStream_t st,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_sym_obs_partials(int elem, const SymObsArgs &a, int grid, int block, hipStream_t st);

}  // namespace sscn

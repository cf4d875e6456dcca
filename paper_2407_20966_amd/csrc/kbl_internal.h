// Internal declarations shared by the HIP translation units of libkbl.
// Not part of the public interface (include/kbl.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kbl.h"

namespace kbl {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Arguments of the bounds kernels, passed by value.
struct BoundsArgs {
    const double* states;
    const int32_t* rowptr;
    const int32_t* cols;
    double* bounds;
    uint32_t* status;
    int64_t n_elem;
    int64_t n_src;      // source units the stencil columns index (elements, or nodes)
    int64_t n_nodes;    // columns of `states` = n_src * n_s
    int64_t nnz;
    int32_t n_s;        // nodes per source unit (1 for node-level stencils)
    int32_t grid_mode;
    int32_t energy_perstate;
    int32_t nx, ny, nz;  // velocity nodes per direction (1 past the dimension)
    double lo0, lo1, lo2, hi0, hi1, hi2, k;
    double gm1;         // gamma - 1
    double half_delta;  // delta / 2, delta = 2/(gamma-1) - d
    double r_fac;
    double rho_floor;
    int64_t grid_blocks;  // host launch shape: 0 = one workgroup per element,
                          // > 0 = persistent grid of that many workgroups,
                          // < 0 = -grid_blocks elements per workgroup
};

// Workgroups to launch for n_elem elements under a BoundsArgs::grid_blocks choice.
inline unsigned bounds_grid(const BoundsArgs& a) {
    int64_t g = a.n_elem;
    if (a.grid_blocks > 0 && a.grid_blocks < a.n_elem) g = a.grid_blocks;
    if (a.grid_blocks < 0 && a.n_elem > 0) {
        // -grid_blocks consecutive elements per workgroup (at most n_elem):
        // a multiple of 8 workgroups, ceil(ceil(n_elem / 8) / k) per XCD, so
        // that every XCD's chunks cover its range (see xcd_range)
        const int64_t k = a.grid_blocks < -a.n_elem ? a.n_elem : -a.grid_blocks;
        g = 8 * (((a.n_elem + 7) / 8 + k - 1) / k);
    }
    if (g > (int64_t)INT32_MAX) g = INT32_MAX;
    return (unsigned)g;
}

// Arguments of the limiter kernel.
constexpr int kMaxLimitNodes = 64;
struct LimitArgs {
    const double* solution;
    const double* bounds;
    double* limited;
    double* alpha;
    uint32_t* status;
    int64_t n_elem;
    int64_t n_nodes;
    int32_t n_s;
    double gm1;
    double p_floor;
    double eps;
    double inv_csum;                 // 1 / sum_j c_j
    int32_t independent;             // per-component alpha instead of the coupled minimum
    double c[kMaxLimitNodes];        // element mean weights (>= 0, positive sum)
};

// Arguments of the Riemann-averaged state kernel.
struct RiemannArgs {
    const double* states;
    int64_t n_nodes;
    const int32_t* ni;
    const int32_t* nj;
    const double* normals;    // [d][n_pairs]
    const double* lam;        // [n_pairs] or null (wavespeed estimate)
    const double* bounds;     // [2(d+2)][n_elem] or null
    const int32_t* elem;      // [n_pairs] or null
    int64_t n_elem;
    double* bar;              // [d+2][n_pairs]
    uint32_t* status;         // [n_pairs] or null
    int64_t n_pairs;
    double gamma;
    double gm1;
};

// Host-side launchers (one per translation unit).  They return hipSuccess or
// the launch error; argument checking happened before.
// tile < 0 selects the default 2D tile for the grid size.
hipError_t launch_bounds_fp64(const BoundsArgs& a, int dim, hipStream_t stream, int tile);
// Energy bounds from the per-state integrand (KBL_FLAG_ENERGY_PERSTATE).
hipError_t launch_bounds_fp64_energy(const BoundsArgs& a, int dim, hipStream_t stream);
// d = 3: FP64 bounds over a 3D velocity grid (tile < 0: default for the grid).
hipError_t launch_bounds_fp64_3d(const BoundsArgs& a, hipStream_t stream, int tile);
int bounds_tile_count_3d();
bool bounds_tile_fits_3d(int tile, int nx, int ny, int nz);
int bounds_default_tile_3d(int nx, int ny, int nz);
int bounds_tile_count_2d();
bool bounds_tile_fits_2d(int tile, int nx, int ny);
int mixed_tile_count();
int bounds_default_tile_2d(int nx, int ny);
int mixed_default_tile_2d(int nx, int ny, int precision);
bool mixed_tile_fits_2d(int tile, int nx, int ny);
// tile < 0 (or a tile that does not fit) selects the default for the grid size.
hipError_t launch_bounds_mixed(const BoundsArgs& a, int precision, hipStream_t stream, int tile);
hipError_t launch_limit_fp64(const LimitArgs& a, int dim, hipStream_t stream);
hipError_t launch_riemann_fp64(const RiemannArgs& a, int dim, hipStream_t stream);
// The elements whose bounds' adjoint is nonzero (a bound binds the limiter):
// the limiter's adjoint appends them to `list` (order unspecified: nothing
// computed from the list depends on it) and sets flag[e] for every element.
struct ActiveSet {
    uint32_t* count;   // [1] number listed (the limiter's adjoint clears it first)
    int32_t* list;     // [n_elem]
    uint8_t* flag;     // [n_elem] 1 if listed, else 0
};
// Bounds backward over the listed elements, gather and status.  mixed:
// winners from the FP32 envelopes of the mixed-precision forward (2D only);
// everything else stays FP64.
hipError_t launch_bounds_bwd_fp64(const BoundsArgs& f, const uint32_t* fstatus, const double* gbnd,
                                  const ActiveSet& act, double* slot, double* grad_states,
                                  uint32_t* status, int dim, bool mixed, hipStream_t stream);
// Per-bit counts of n status words into counts[32] (cleared first).
hipError_t launch_status_summary(const uint32_t* st, int64_t n, uint64_t* counts,
                                 hipStream_t stream);
hipError_t launch_limit_bwd_fp64(const LimitArgs& a, int dim, const double* grad, double* gsol,
                                 double* gbnd, const ActiveSet& act, hipStream_t stream);

}  // namespace kbl

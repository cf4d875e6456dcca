// C-ABI entry points of libkbl: host-side argument checks, then launches on
// the caller's stream.  See include/kbl.h for the contract.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "kbl_internal.h"

namespace {

constexpr int kMax2DNodesPerDim = 64;
constexpr int kMax1DNodes = 4096;
constexpr int kMax1DBackwardNodes = 2048;

// delta = 2/(gamma-1) - d (Sec. 3.6); tiny negative round-off is clamped to 0.
bool internal_dof(int dim, double gamma, double* half_delta) {
    const double delta = (2.0 - dim * (gamma - 1.0)) / (gamma - 1.0);
    if (delta < -1e-12) return false;
    *half_delta = delta > 0.0 ? 0.5 * delta : 0.0;
    return true;
}

kbl_status check_params(const kbl_params* p, int32_t dim, double* half_delta) {
    if (!p || (dim != 1 && dim != 2) || p->reserved != 0) return KBL_ERR_ARG;
    if (!(p->gamma > 1.0) || !isfinite(p->gamma)) return KBL_ERR_GAMMA;
    if (!internal_dof(dim, p->gamma, half_delta)) return KBL_ERR_GAMMA;
    if (!(p->r_fac >= 0.0 && p->r_fac < 1.0)) return KBL_ERR_ARG;
    if (!(p->rho_floor >= 0.0) || !isfinite(p->rho_floor)) return KBL_ERR_ARG;
    if (!isfinite(p->p_floor) || !(p->eps_alpha >= 0.0) || !isfinite(p->eps_alpha))
        return KBL_ERR_ARG;
    return KBL_OK;
}

// Shared checks of the bounds geometry; fills the kernel arguments.
kbl_status make_bounds_args(const kbl_params* params, int32_t dim, int64_t n_elem, int32_t n_s,
                            int64_t nnz, const double* states, const int32_t* rowptr,
                            const int32_t* cols, const kbl_vgrid* vgrid, int max1d,
                            kbl::BoundsArgs* a) {
    double half_delta = 0.0;
    kbl_status rc = check_params(params, dim, &half_delta);
    if (rc != KBL_OK) return rc;
    if (n_elem < 0 || n_s < 1 || nnz < 0 || !vgrid) return KBL_ERR_ARG;
    if (n_elem > 0 && (!states || !rowptr)) return KBL_ERR_ARG;
    if (nnz > 0 && !cols) return KBL_ERR_ARG;
    if (n_elem > INT64_MAX / n_s || nnz > INT64_MAX / (n_s * 8)) return KBL_ERR_ARG;
    const kbl_vgrid g = *vgrid;
    if (g.mode != KBL_GRID_GLOBAL && g.mode != KBL_GRID_STENCIL) return KBL_ERR_GRID;
    for (int j = 0; j < dim; ++j) {
        if (g.n[j] < 2) return KBL_ERR_GRID;
        if (g.n[j] > (dim == 2 ? kMax2DNodesPerDim : max1d)) return KBL_ERR_GRID;
        if (g.mode == KBL_GRID_GLOBAL &&
            !(isfinite(g.lo[j]) && isfinite(g.hi[j]) && g.hi[j] > g.lo[j]))
            return KBL_ERR_GRID;
    }
    if (g.mode == KBL_GRID_STENCIL && !(g.k > 0.0 && isfinite(g.k))) return KBL_ERR_GRID;
    memset(a, 0, sizeof(*a));
    a->states = states;
    a->rowptr = rowptr;
    a->cols = cols;
    a->n_elem = n_elem;
    a->n_nodes = n_elem * n_s;
    a->nnz = nnz;
    a->n_s = n_s;
    a->grid_mode = g.mode;
    a->nx = g.n[0];
    a->ny = dim == 2 ? g.n[1] : 1;
    a->lo0 = g.lo[0];
    a->hi0 = g.hi[0];
    a->lo1 = dim == 2 ? g.lo[1] : 0.0;
    a->hi1 = dim == 2 ? g.hi[1] : 0.0;
    a->k = g.k;
    a->gm1 = params->gamma - 1.0;
    a->half_delta = half_delta;
    a->r_fac = params->r_fac;
    a->rho_floor = params->rho_floor;
    return KBL_OK;
}

kbl_status make_limit_args(const kbl_params* params, int32_t dim, int64_t n_elem, int32_t n_s,
                           const double* node_weights, kbl::LimitArgs* a) {
    double half_delta = 0.0;
    kbl_status rc = check_params(params, dim, &half_delta);
    if (rc != KBL_OK) return rc;
    if (n_elem < 0 || n_s < 1 || n_s > kbl::kMaxLimitNodes || !node_weights) return KBL_ERR_ARG;
    if (n_elem > INT64_MAX / n_s) return KBL_ERR_ARG;
    memset(a, 0, sizeof(*a));
    double csum = 0.0;
    for (int j = 0; j < n_s; ++j) {
        const double c = node_weights[j];
        if (!(c > 0.0) || !isfinite(c)) return KBL_ERR_ARG;
        a->c[j] = c;
        csum += c;
    }
    a->n_elem = n_elem;
    a->n_nodes = n_elem * n_s;
    a->n_s = n_s;
    a->gm1 = params->gamma - 1.0;
    a->p_floor = params->p_floor;
    a->eps = params->eps_alpha;
    a->inv_csum = 1.0 / csum;
    return KBL_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

void kbl_default_params(kbl_params* p, double gamma) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->gamma = gamma;
    p->r_fac = 1e-3;      // Sec. 3.5
    p->rho_floor = 1e-12; // Sec. 3.8
    p->p_floor = 1e-12;   // Sec. 3.8
    p->eps_alpha = 1e-13; // Sec. 3.4
    p->precision = KBL_PREC_FP64;
}

int32_t kbl_version(void) { return 100; }

const char* kbl_status_string(kbl_status s) {
    switch (s) {
        case KBL_OK: return "ok";
        case KBL_ERR_ARG: return "invalid argument";
        case KBL_ERR_GAMMA: return "gamma <= 1 or negative internal degrees of freedom (delta < 0)";
        case KBL_ERR_GRID: return "invalid velocity grid (n < 2, hi <= lo, k <= 0, or too many nodes)";
        case KBL_ERR_UNSUPPORTED: return "unsupported configuration";
        case KBL_ERR_HIP: return "HIP runtime or launch failure";
        case KBL_ERR_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

kbl_status kbl_compute_bounds(const kbl_params* params, int32_t dim, int64_t n_elem,
                              int32_t n_s, int64_t nnz, const double* states,
                              const int32_t* rowptr, const int32_t* cols,
                              const kbl_vgrid* vgrid, double* bounds,
                              uint32_t* elem_status, void* stream) {
    kbl::BoundsArgs a;
    kbl_status rc = make_bounds_args(params, dim, n_elem, n_s, nnz, states, rowptr, cols, vgrid,
                                     kMax1DNodes, &a);
    if (rc != KBL_OK) return rc;
    if (n_elem > 0 && !bounds) return KBL_ERR_ARG;
    const int prec = params->precision;
    if (prec != KBL_PREC_FP64 && prec != KBL_PREC_MIXED_BF16 && prec != KBL_PREC_MIXED_FP16 &&
        prec != KBL_PREC_MIXED_FP32)
        return KBL_ERR_UNSUPPORTED;
    if (prec != KBL_PREC_FP64 && dim != 2) return KBL_ERR_UNSUPPORTED;
    a.bounds = bounds;
    a.status = elem_status;
    // KBL_BOUNDS_TILE / KBL_MIXED_TILE (tuning knobs) force a tile configuration
    int tile = -1;
    if (const char* env = getenv(prec == KBL_PREC_FP64 ? "KBL_BOUNDS_TILE" : "KBL_MIXED_TILE")) {
        tile = atoi(env);
        if (prec == KBL_PREC_FP64 && dim == 2 && !kbl::bounds_tile_fits_2d(tile, a.nx, a.ny))
            tile = -1;
    }
    hipError_t err = prec == KBL_PREC_FP64
                         ? kbl::launch_bounds_fp64(a, dim, (hipStream_t)stream, tile)
                         : kbl::launch_bounds_mixed(a, prec, (hipStream_t)stream, tile);
    return err == hipSuccess ? KBL_OK : KBL_ERR_HIP;
}

kbl_status kbl_limit(const kbl_params* params, int32_t dim, int64_t n_elem, int32_t n_s,
                     const double* solution, const double* bounds,
                     const double* node_weights, double* limited, double* alpha,
                     uint32_t* elem_status, void* stream) {
    kbl::LimitArgs a;
    kbl_status rc = make_limit_args(params, dim, n_elem, n_s, node_weights, &a);
    if (rc != KBL_OK) return rc;
    if (n_elem > 0 && (!solution || !bounds || !limited)) return KBL_ERR_ARG;
    a.solution = solution;
    a.bounds = bounds;
    a.limited = limited;
    a.alpha = alpha;
    a.status = elem_status;
    hipError_t err = kbl::launch_limit_fp64(a, dim, (hipStream_t)stream);
    return err == hipSuccess ? KBL_OK : KBL_ERR_HIP;
}

size_t kbl_backward_workspace_bytes(int32_t dim, int64_t n_elem, int32_t n_s, int64_t nnz) {
    if ((dim != 1 && dim != 2) || n_elem < 0 || n_s < 1 || nnz < 0) return 0;
    const size_t nv = (size_t)dim + 2;
    return align256(2 * nv * (size_t)n_elem * 8) + align256((size_t)n_elem * 4) +
           align256(2 * nv * (size_t)n_elem * 8) + align256(nv * (size_t)nnz * (size_t)n_s * 8);
}

kbl_status kbl_bounds_limit_backward(const kbl_params* params, int32_t dim, int64_t n_elem,
                                     int32_t n_s, int64_t nnz, const double* states,
                                     const int32_t* rowptr, const int32_t* cols,
                                     const kbl_vgrid* vgrid, const double* solution,
                                     const double* node_weights, const double* grad_limited,
                                     double* grad_states, double* grad_solution,
                                     double* grad_bounds, uint32_t* elem_status,
                                     void* workspace, size_t workspace_bytes, void* stream) {
    kbl::BoundsArgs fa;
    kbl_status rc = make_bounds_args(params, dim, n_elem, n_s, nnz, states, rowptr, cols, vgrid,
                                     kMax1DBackwardNodes, &fa);
    if (rc != KBL_OK) return rc;
    kbl::LimitArgs la;
    rc = make_limit_args(params, dim, n_elem, n_s, node_weights, &la);
    if (rc != KBL_OK) return rc;
    if (params->precision != KBL_PREC_FP64) return KBL_ERR_UNSUPPORTED;
    if (n_elem == 0) return KBL_OK;
    if (!solution || !grad_limited || !grad_states || !grad_solution) return KBL_ERR_ARG;
    const size_t need = kbl_backward_workspace_bytes(dim, n_elem, n_s, nnz);
    if (!workspace || workspace_bytes < need) return KBL_ERR_WORKSPACE;
    const size_t nv = (size_t)dim + 2;
    char* ws = (char*)workspace;
    double* wb = (double*)ws;                          ws += align256(2 * nv * (size_t)n_elem * 8);
    uint32_t* wst = (uint32_t*)ws;                     ws += align256((size_t)n_elem * 4);
    double* wgb = (double*)ws;                         ws += align256(2 * nv * (size_t)n_elem * 8);
    double* wslot = (double*)ws;
    double* gbnd = grad_bounds ? grad_bounds : wgb;
    hipStream_t st = (hipStream_t)stream;
    fa.bounds = wb;
    fa.status = wst;
    hipError_t err = kbl::launch_bounds_fp64(fa, dim, st, -1);
    if (err != hipSuccess) return KBL_ERR_HIP;
    la.solution = solution;
    la.bounds = wb;
    err = kbl::launch_limit_bwd_fp64(la, dim, grad_limited, grad_solution, gbnd, st);
    if (err != hipSuccess) return KBL_ERR_HIP;
    err = kbl::launch_bounds_bwd_fp64(fa, wst, gbnd, wslot, grad_states, elem_status, dim, st);
    return err == hipSuccess ? KBL_OK : KBL_ERR_HIP;
}

}  // extern "C"

// Riemann-averaged states of Thm. 4.3 (Sec. 4) and their check against the
// element bounds, gfx950, FP64.
//
// For a pair of node states (i, j) across a face with unit normal n (from i
// to j) the averaged state is
//   wbar = (w_i + w_j)/2 - (F(w_j) - F(w_i)).n / (2 lambda)
// with the Euler flux F (Sec. 2.1) and lambda given per pair or taken as the
// wavespeed estimate max(|U.n| + sqrt(gamma theta)) of the two states (the
// remark after the theorem).  This is what a flux-corrected / convex-limiting
// scheme consumes next to the bounds.  One lane per pair; the node gathers
// dominate (HBM / latency bound), the arithmetic is a few dozen FP64 ops.
#include <math.h>

#include "kbl_internal.h"

namespace kbl {
namespace {

template <int D>
__device__ __forceinline__ bool load_state(const RiemannArgs& a, int64_t node, double* w,
                                           double* U, double* P) {
    if (node < 0 || node >= a.n_nodes) return false;
    bool ok = true;
#pragma unroll
    for (int v = 0; v < D + 2; ++v) {
        w[v] = a.states[(int64_t)v * a.n_nodes + node];
        ok = ok && isfinite(w[v]);
    }
    double mm = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        U[j] = w[1 + j] / w[0];
        mm += w[1 + j] * w[1 + j];
    }
    *P = a.gm1 * (w[D + 1] - 0.5 * mm / w[0]);
    return ok && w[0] > 0.0 && *P > 0.0 && isfinite(*P / w[0]);
}

template <int D>
__device__ __forceinline__ void flux_n(const double* w, const double* U, double P,
                                       const double* n, double* f) {
    double un = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) un += U[j] * n[j];
    f[0] = w[0] * un;
#pragma unroll
    for (int j = 0; j < D; ++j) f[1 + j] = w[1 + j] * un + P * n[j];
    f[D + 1] = (w[D + 1] + P) * un;
}

template <int D>
__global__ __launch_bounds__(256) void riemann_fp64(RiemannArgs a) {
    constexpr int NV = D + 2;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < a.n_pairs;
         q += (int64_t)gridDim.x * 256) {
        double wi[NV], wj[NV], Ui[3] = {0, 0, 0}, Uj[3] = {0, 0, 0}, Pi, Pj;
        const bool ok_i = load_state<D>(a, a.ni[q], wi, Ui, &Pi);
        const bool ok_j = load_state<D>(a, a.nj[q], wj, Uj, &Pj);
        const bool ok = ok_i && ok_j;
        if (!ok) {
#pragma unroll
            for (int v = 0; v < NV; ++v) a.bar[(int64_t)v * a.n_pairs + q] = __longlong_as_double(0x7ff8000000000000LL);
            if (a.status) a.status[q] = KBL_RS_BAD_INPUT;
            continue;
        }
        double n[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < D; ++j) n[j] = a.normals[(int64_t)j * a.n_pairs + q];
        double lam;
        if (a.lam) {
            lam = a.lam[q];
        } else {
            double ui = 0.0, uj = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) { ui += Ui[j] * n[j]; uj += Uj[j] * n[j]; }
            const double si = fabs(ui) + sqrt(a.gamma * (Pi / wi[0]));
            const double sj = fabs(uj) + sqrt(a.gamma * (Pj / wj[0]));
            lam = si > sj ? si : sj;
        }
        double fi[NV], fj[NV];
        flux_n<D>(wi, Ui, Pi, n, fi);
        flux_n<D>(wj, Uj, Pj, n, fj);
        uint32_t st = 0;
        const int64_t e = a.elem ? a.elem[q] : -1;
        const bool check = a.bounds && e >= 0 && e < a.n_elem;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double w = 0.5 * (wi[v] + wj[v]) - (fj[v] - fi[v]) / (2.0 * lam);
            a.bar[(int64_t)v * a.n_pairs + q] = w;
            if (check) {
                if (w < a.bounds[(int64_t)v * a.n_elem + e]) st |= KBL_RS_BELOW(v);
                if (w > a.bounds[(int64_t)(NV + v) * a.n_elem + e]) st |= KBL_RS_ABOVE(v);
            }
        }
        if (a.status) a.status[q] = st;
    }
}

}  // namespace

hipError_t launch_riemann_fp64(const RiemannArgs& a, int dim, hipStream_t stream) {
    if (a.n_pairs == 0) return hipSuccess;
    const int64_t blocks = (a.n_pairs + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65535 * 16 ? blocks : 65535 * 16);
    if (dim == 3) hipLaunchKernelGGL(riemann_fp64<3>, dim3(g), dim3(256), 0, stream, a);
    else if (dim == 2) hipLaunchKernelGGL(riemann_fp64<2>, dim3(g), dim3(256), 0, stream, a);
    else hipLaunchKernelGGL(riemann_fp64<1>, dim3(g), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace kbl

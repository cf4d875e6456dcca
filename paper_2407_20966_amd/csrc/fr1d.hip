// One-dimensional flux reconstruction Euler solver with the kinetic bounds
// and squeeze limiter after every SSP-RK3 stage (the setup of Sec. 5), gfx950.
//
// Kernels (one thread per element; 1D problems of the paper have at most a
// few thousand elements, so the step is launch- and latency-bound and each
// kernel touches an element's p + 3 nodes once):
//  - fr1d_rhs<P>: point fluxes, end values of the element and of its two
//    neighbours (Lagrange interpolation to x = -1, +1), HLLC common fluxes
//    at both ends, and the corrected flux divergence at the solution points.
//    The common flux of a face is computed by both adjacent elements from
//    bitwise identical inputs with the same operation sequence, so the
//    scheme stays exactly conservative.
//  - fr1d_stage<P>: the Shu-Osher stage combination, then the end values of
//    the new solution and the ghost elements.
//  - fr1d_csr: the node stencils of the bounds (constant per mesh).
//  - fr1d_max_speed: max |u| + c over the solution points.
// The bounds and the limiter are the library's own entry points
// (kbl_compute_bounds_nodes, kbl_limit) on the node layout of kbl_fr1d.h.
// Every stage follows the overview of Sec. 3.9: bounds from the stage's
// input state, the update, then the limiting of the updated state into
// those bounds.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "../../include/kbl_fr1d.h"
#include "kbl_internal.h"

namespace kbl {
namespace {

constexpr int kMaxNs = KBL_FR_MAX_DEGREE + 1;
constexpr int kThreadsFr = 256;

// Element operators on the reference element [-1, 1].
struct FrOps {
    double at_m1[kMaxNs];            // l_j(-1)
    double at_p1[kMaxNs];            // l_j(+1)
    double D[kMaxNs * kMaxNs];       // D[j*NS + k] = l_k'(x_j)
    double dgL[kMaxNs];              // g_L'(x_j)
    double dgR[kMaxNs];              // g_R'(x_j)
};

struct FrArgs {
    double* U;          // [3][cols]
    double* U0;         // [3][cols] stage-start copy
    double* R;          // [3][n_elem * NS]
    int64_t n_elem, n_tot, cols;
    int32_t n_v, bc;
    int32_t save_u0;
    double inv_jac;     // 2 / h
    double gm1;
    double gamma;
    double left[3], right[3];
    double a, b, dt;    // U <- a U0 + b (U + dt R)
    const double* tdt;  // device (t, dt): dt read from tdt[1] when not null
    FrOps ops;
};

// Lagrange interpolation of NS nodal values to one end (explicit fma chain,
// the same sequence wherever it is used).
template <int NS>
__device__ __forceinline__ double interp(const double* at, const double* u) {
    double s = at[0] * u[0];
#pragma unroll
    for (int j = 1; j < NS; ++j) s = fma(at[j], u[j], s);
    return s;
}

__device__ __forceinline__ void euler_flux(double gm1, const double w[3], double f[3]) {
#pragma clang fp contract(off)
    const double u = w[1] / w[0];
    const double P = gm1 * (w[2] - 0.5 * w[1] * u);
    f[0] = w[1];
    f[1] = w[1] * u + P;
    f[2] = (w[2] + P) * u;
}

// HLLC flux (Toro, Spruce and Speares) with the speeds
// S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).
__device__ __forceinline__ void hllc(double gamma, double gm1, const double L[3], const double Rr[3],
                                     double F[3]) {
#pragma clang fp contract(off)
    const double ul = L[1] / L[0], ur = Rr[1] / Rr[0];
    const double pl = gm1 * (L[2] - 0.5 * L[1] * ul);
    const double pr = gm1 * (Rr[2] - 0.5 * Rr[1] * ur);
    const double cl = sqrt(gamma * pl / L[0]), cr = sqrt(gamma * pr / Rr[0]);
    const double SL = fmin(ul - cl, ur - cr);
    const double SR = fmax(ul + cl, ur + cr);
    const double dl = L[0] * (SL - ul), dr = Rr[0] * (SR - ur);
    const double Ss = (pr - pl + ul * dl - ur * dr) / (dl - dr);
    double fl[3], fr[3];
    euler_flux(gm1, L, fl);
    euler_flux(gm1, Rr, fr);
    if (0.0 <= SL) {
        F[0] = fl[0]; F[1] = fl[1]; F[2] = fl[2];
    } else if (0.0 <= Ss) {
        const double k = dl / (SL - Ss);
        const double e = k * (L[2] / L[0] + (Ss - ul) * (Ss + pl / dl));
        F[0] = fl[0] + SL * (k - L[0]);
        F[1] = fl[1] + SL * (k * Ss - L[1]);
        F[2] = fl[2] + SL * (e - L[2]);
    } else if (0.0 <= SR) {
        const double k = dr / (SR - Ss);
        const double e = k * (Rr[2] / Rr[0] + (Ss - ur) * (Ss + pr / dr));
        F[0] = fr[0] + SR * (k - Rr[0]);
        F[1] = fr[1] + SR * (k * Ss - Rr[1]);
        F[2] = fr[2] + SR * (e - Rr[2]);
    } else {
        F[0] = fr[0]; F[1] = fr[1]; F[2] = fr[2];
    }
}

template <int NS>
__device__ __forceinline__ void load_elem(const FrArgs& a, int64_t e, double u[3][NS]) {
    const int64_t c0 = e * a.n_v;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int j = 0; j < NS; ++j) u[v][j] = a.U[v * a.cols + c0 + j];
}

template <int P>
__global__ __launch_bounds__(kThreadsFr) void fr1d_rhs(FrArgs a) {
    constexpr int NS = P + 1;
    const int64_t e = (int64_t)blockIdx.x * kThreadsFr + threadIdx.x;
    if (e >= a.n_elem) return;
    const FrOps& o = a.ops;
    double u[3][NS];
    load_elem<NS>(a, e, u);
    double uL[3], uR[3], nl[3], nr[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        uL[v] = interp<NS>(o.at_m1, u[v]);
        uR[v] = interp<NS>(o.at_p1, u[v]);
    }
    // neighbours' end values on the shared faces
    const bool periodic = a.bc == KBL_FR_PERIODIC;
    if (periodic || e > 0) {
        double t[3][NS];
        load_elem<NS>(a, e > 0 ? e - 1 : a.n_elem - 1, t);
#pragma unroll
        for (int v = 0; v < 3; ++v) nl[v] = interp<NS>(o.at_p1, t[v]);
    } else {
#pragma unroll
        for (int v = 0; v < 3; ++v) nl[v] = a.left[v];
    }
    if (periodic || e < a.n_elem - 1) {
        double t[3][NS];
        load_elem<NS>(a, e < a.n_elem - 1 ? e + 1 : 0, t);
#pragma unroll
        for (int v = 0; v < 3; ++v) nr[v] = interp<NS>(o.at_m1, t[v]);
    } else {
#pragma unroll
        for (int v = 0; v < 3; ++v) nr[v] = a.right[v];
    }
    double Fs_l[3], Fs_r[3];
    hllc(a.gamma, a.gm1, nl, uL, Fs_l);
    hllc(a.gamma, a.gm1, uR, nr, Fs_r);
    // point fluxes and their interpolants at the ends
    double F[3][NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const double w[3] = {u[0][j], u[1][j], u[2][j]};
        double f[3];
        euler_flux(a.gm1, w, f);
        F[0][j] = f[0]; F[1][j] = f[1]; F[2][j] = f[2];
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const double jl = Fs_l[v] - interp<NS>(o.at_m1, F[v]);
        const double jr = Fs_r[v] - interp<NS>(o.at_p1, F[v]);
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < NS; ++k) d = fma(o.D[j * NS + k], F[v][k], d);
            d = fma(jl, o.dgL[j], d);
            d = fma(jr, o.dgR[j], d);
            a.R[v * (a.n_elem * NS) + e * NS + j] = -a.inv_jac * d;
        }
    }
}

template <int P>
__global__ __launch_bounds__(kThreadsFr) void fr1d_stage(FrArgs a) {
    constexpr int NS = P + 1;
    const int64_t e = (int64_t)blockIdx.x * kThreadsFr + threadIdx.x;
    if (e >= a.n_tot) return;
    const int64_t c0 = e * a.n_v;
    if (e >= a.n_elem) {      // constant ghost element
        const double* g = (e == a.n_elem) ? a.left : a.right;
        for (int j = 0; j < a.n_v; ++j)
#pragma unroll
            for (int v = 0; v < 3; ++v) a.U[v * a.cols + c0 + j] = g[v];
        return;
    }
    const double dt = a.tdt ? a.tdt[1] : a.dt;
    double u[3][NS];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int64_t c = v * a.cols + c0 + j;
            const double x = a.U[c];
            double nu = x;
            if (a.b != 0.0) {
                const double u0 = a.save_u0 ? x : a.U0[c];
                if (a.save_u0) a.U0[c] = x;
                nu = a.a * u0 + a.b * (x + dt * a.R[v * (a.n_elem * NS) + e * NS + j]);
            }
            u[v][j] = nu;
            a.U[c] = nu;
        }
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        a.U[v * a.cols + c0 + NS] = interp<NS>(a.ops.at_m1, u[v]);
        a.U[v * a.cols + c0 + NS + 1] = interp<NS>(a.ops.at_p1, u[v]);
    }
}

// Node stencils.  Stage stencil (Sec. 5): row e < n_elem lists the
// element's n_v nodes and the neighbours' end values on the shared faces.
// Initial stencil: the solution points of the element and of its two face
// neighbours.  Ghost rows list their own nodes.
__global__ __launch_bounds__(kThreadsFr) void fr1d_csr(int64_t n_elem, int64_t n_tot, int32_t n_v,
                                                       int32_t bc, int32_t initial, int32_t* rowptr,
                                                       int32_t* cols) {
    const int64_t r = (int64_t)blockIdx.x * kThreadsFr + threadIdx.x;
    if (r >= n_tot) return;
    const int32_t ns = n_v - 2;
    const int64_t row_len = initial ? 3 * ns : n_v + 2;
    const int64_t start = r < n_elem ? r * row_len : n_elem * row_len + (r - n_elem) * n_v;
    int64_t len = n_v;
    if (r < n_elem) {
        int64_t lnb, rnb;
        if (bc == KBL_FR_PERIODIC) {
            lnb = r > 0 ? r - 1 : n_elem - 1;
            rnb = r < n_elem - 1 ? r + 1 : 0;
        } else {
            lnb = r > 0 ? r - 1 : n_elem;
            rnb = r < n_elem - 1 ? r + 1 : n_elem + 1;
        }
        if (initial) {
            const int64_t q[3] = {r, lnb, rnb};
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < ns; ++j) cols[start + i * ns + j] = (int32_t)(q[i] * n_v + j);
        } else {
            for (int j = 0; j < n_v; ++j) cols[start + j] = (int32_t)(r * n_v + j);
            cols[start + n_v] = (int32_t)(lnb * n_v + ns + 1);      // left neighbour's right end
            cols[start + n_v + 1] = (int32_t)(rnb * n_v + ns);      // right neighbour's left end
        }
        len = row_len;
    } else {
        for (int j = 0; j < n_v; ++j) cols[start + j] = (int32_t)(r * n_v + j);
    }
    rowptr[r] = (int32_t)start;
    if (r == n_tot - 1) rowptr[n_tot] = (int32_t)(start + len);
}

// Initial limiting: elements whose n_v node values are all admissible keep
// their data (NaN bounds: the limiter passes them through unchanged).
__global__ __launch_bounds__(kThreadsFr) void fr1d_keep_admissible(const double* U, int64_t n_tot,
                                                                   int64_t cols, int32_t n_v,
                                                                   double gm1, double* bounds) {
    const int64_t e = (int64_t)blockIdx.x * kThreadsFr + threadIdx.x;
    if (e >= n_tot) return;
    bool good = true;
    for (int j = 0; j < n_v; ++j) {
        const int64_t c = e * n_v + j;
        const double r = U[c], m = U[cols + c], E = U[2 * cols + c];
        const double P = gm1 * (E - 0.5 * m * m / r);
        good = good && r > 0.0 && P > 0.0 && isfinite(r) && isfinite(P);
    }
    if (good) {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);
        for (int v = 0; v < 6; ++v) bounds[v * n_tot + e] = nan;
    }
}

// max |u| + c over the solution points; NaN when a point is not admissible.
// With tdt (device (t, dt)): instead writes the CFL time step
// dt = min(cfl_h / s, t_end - t) and advances t (NaN for both when a point
// is not admissible).
__global__ __launch_bounds__(1024) void fr1d_max_speed(const double* U, int64_t n_elem, int64_t cols,
                                                       int32_t n_v, int32_t ns, double gamma,
                                                       double* out, double* tdt, double cfl_h,
                                                       double t_end) {
    __shared__ double red[1024];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    double m = 0.0;
    int b = 0;
    for (int64_t i = threadIdx.x; i < n_elem * ns; i += 1024) {
        const int64_t c = (i / ns) * n_v + i % ns;
        const double r = U[c], mo = U[cols + c], E = U[2 * cols + c];
        const double u = mo / r;
        const double P = (gamma - 1.0) * (E - 0.5 * mo * u);
        const double s = fabs(u) + sqrt(gamma * P / r);
        if (!(r > 0.0) || !(P >= 0.0) || !isfinite(s)) b = 1;
        else m = fmax(m, s);
    }
    if (b) atomicOr(&bad, 1);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    if (!tdt) {
        *out = bad ? nan : red[0];
        return;
    }
    const double t = tdt[0];
    double dt = cfl_h / red[0];
    const double rem = t_end - t;
    double tn;
    if (!(rem > 0.0)) { dt = 0.0; tn = t; }
    else if (dt >= rem) { dt = rem; tn = t_end; }
    else tn = t + dt;
    if (bad || !(red[0] > 0.0)) { dt = nan; tn = nan; }
    tdt[0] = tn;
    tdt[1] = dt;
}

// ------------------------------------------------------------ host side

// Legendre polynomial P_n and its derivative at x (three-term recurrence).
void legendre(int n, double x, double* P, double* dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    *P = p1;
    // (1 - x^2) P_n' = n (P_{n-1} - x P_n), used at interior points only
    *dP = n * (p0 - x * p1) / (1.0 - x * x);
}

// Gauss-Legendre nodes and weights (Newton on P_n from the Chebyshev-like guess).
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, z, &P, &dP);
            const double dz = P / dP;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double P, dP;
        legendre(n, z, &P, &dP);
        x[n - 1 - i] = z;   // ascending
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dP * dP);
    }
}

void make_ops(int p, FrOps* o, double* w) {
    const int ns = p + 1;
    double x[kMaxNs];
    gauss_legendre(ns, x, w);
    memset(o, 0, sizeof(*o));
    // barycentric weights lambda_k = 1 / prod_{m != k} (x_k - x_m)
    double lam[kMaxNs];
    for (int k = 0; k < ns; ++k) {
        double q = 1.0;
        for (int m = 0; m < ns; ++m)
            if (m != k) q *= x[k] - x[m];
        lam[k] = 1.0 / q;
    }
    for (int end = 0; end < 2; ++end) {
        const double t = end ? 1.0 : -1.0;
        double den = 0.0;
        for (int k = 0; k < ns; ++k) den += lam[k] / (t - x[k]);
        for (int k = 0; k < ns; ++k) (end ? o->at_p1 : o->at_m1)[k] = lam[k] / (t - x[k]) / den;
    }
    for (int j = 0; j < ns; ++j) {
        double diag = 0.0;
        for (int k = 0; k < ns; ++k) {
            if (k == j) continue;
            const double d = (lam[k] / lam[j]) / (x[j] - x[k]);
            o->D[j * ns + k] = d;
            diag -= d;
        }
        o->D[j * ns + j] = diag;
    }
    // g_L = (-1)^p / 2 (P_p - P_{p+1}),  g_R = (P_p + P_{p+1}) / 2
    const double sgn = (p % 2) ? -1.0 : 1.0;
    for (int j = 0; j < ns; ++j) {
        double Pp, dPp, Pq, dPq;
        legendre(p, x[j], &Pp, &dPp);
        legendre(p + 1, x[j], &Pq, &dPq);
        o->dgL[j] = 0.5 * sgn * (dPp - dPq);
        o->dgR[j] = 0.5 * (dPp + dPq);
    }
}

bool admissible(const double w[3], double gamma) {
    if (!(isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2])) || !(w[0] > 0.0)) return false;
    const double P = (gamma - 1.0) * (w[2] - 0.5 * w[1] * w[1] / w[0]);
    return P > 0.0;
}

bool valid_cfg(const kbl_fr1d* c) {
    return c && c->p >= 1 && c->p <= KBL_FR_MAX_DEGREE &&
           (c->bc == KBL_FR_PERIODIC || c->bc == KBL_FR_DIRICHLET) && c->n_elem >= 2 &&
           isfinite(c->x0) && isfinite(c->x1) && c->x1 > c->x0 && (c->limit == 0 || c->limit == 1) &&
           c->reserved == 0 && c->n_elem < (int64_t)1 << 26;
}

int64_t n_total(const kbl_fr1d* c) { return c->n_elem + (c->bc == KBL_FR_DIRICHLET ? 2 : 0); }

int64_t stencil_nnz(const kbl_fr1d* c, bool initial) {
    const int64_t nv = c->p + 3;
    const int64_t row = initial ? 3 * (c->p + 1) : nv + 2;
    return c->n_elem * row + (n_total(c) - c->n_elem) * nv;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Ws {
    double* U0;
    double* R;
    double* bounds;
    uint32_t* bstat;
    int32_t* rowptr;
    int32_t* cols;
};

size_t ws_layout(const kbl_fr1d* c, char* base, Ws* w) {
    const int64_t nt = n_total(c), cols = nt * (c->p + 3);
    size_t off = 0;
    auto take = [&](size_t bytes) { char* p = base ? base + off : nullptr; off += al256(bytes); return p; };
    Ws t;
    t.U0 = (double*)take(3 * (size_t)cols * 8);
    t.R = (double*)take(3 * (size_t)c->n_elem * (c->p + 1) * 8);
    t.bounds = (double*)take(6 * (size_t)nt * 8);
    t.bstat = (uint32_t*)take((size_t)nt * 4);
    t.rowptr = (int32_t*)take((size_t)(nt + 1) * 4);
    const int64_t nnz = std::max(stencil_nnz(c, false), stencil_nnz(c, true));
    t.cols = (int32_t*)take((size_t)nnz * 4);
    if (w) *w = t;
    return off;
}

kbl_status make_args(const kbl_fr1d* c, double gamma, double* U, FrArgs* a, double* w) {
    if (!valid_cfg(c) || !(gamma > 1.0) || !isfinite(gamma)) return KBL_ERR_ARG;
    if (c->bc == KBL_FR_DIRICHLET && (!admissible(c->left, gamma) || !admissible(c->right, gamma)))
        return KBL_ERR_ARG;
    memset(a, 0, sizeof(*a));
    a->U = U;
    a->n_elem = c->n_elem;
    a->n_tot = n_total(c);
    a->n_v = c->p + 3;
    a->cols = a->n_tot * a->n_v;
    a->bc = c->bc;
    a->inv_jac = 2.0 / ((c->x1 - c->x0) / (double)c->n_elem);
    a->gamma = gamma;
    a->gm1 = gamma - 1.0;
    for (int v = 0; v < 3; ++v) {
        a->left[v] = c->bc == KBL_FR_DIRICHLET ? c->left[v] : 0.0;
        a->right[v] = c->bc == KBL_FR_DIRICHLET ? c->right[v] : 0.0;
    }
    make_ops(c->p, &a->ops, w);
    return KBL_OK;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreadsFr - 1) / kThreadsFr); }

hipError_t launch_rhs(const FrArgs& a, int p, hipStream_t st) {
    const dim3 g(blocks_for(a.n_elem)), b(kThreadsFr);
    switch (p) {
        case 1: hipLaunchKernelGGL(fr1d_rhs<1>, g, b, 0, st, a); break;
        case 2: hipLaunchKernelGGL(fr1d_rhs<2>, g, b, 0, st, a); break;
        case 3: hipLaunchKernelGGL(fr1d_rhs<3>, g, b, 0, st, a); break;
        case 4: hipLaunchKernelGGL(fr1d_rhs<4>, g, b, 0, st, a); break;
        case 5: hipLaunchKernelGGL(fr1d_rhs<5>, g, b, 0, st, a); break;
        case 6: hipLaunchKernelGGL(fr1d_rhs<6>, g, b, 0, st, a); break;
        case 7: hipLaunchKernelGGL(fr1d_rhs<7>, g, b, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stage(const FrArgs& a, int p, hipStream_t st) {
    const dim3 g(blocks_for(a.n_tot)), b(kThreadsFr);
    switch (p) {
        case 1: hipLaunchKernelGGL(fr1d_stage<1>, g, b, 0, st, a); break;
        case 2: hipLaunchKernelGGL(fr1d_stage<2>, g, b, 0, st, a); break;
        case 3: hipLaunchKernelGGL(fr1d_stage<3>, g, b, 0, st, a); break;
        case 4: hipLaunchKernelGGL(fr1d_stage<4>, g, b, 0, st, a); break;
        case 5: hipLaunchKernelGGL(fr1d_stage<5>, g, b, 0, st, a); break;
        case 6: hipLaunchKernelGGL(fr1d_stage<6>, g, b, 0, st, a); break;
        case 7: hipLaunchKernelGGL(fr1d_stage<7>, g, b, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Bounds of the node stencils of the current state (steps 1-3 of Sec. 3.9).
kbl_status stencil_bounds(const kbl_fr1d* c, const kbl_params* params, const kbl_vgrid* vgrid,
                          const FrArgs& a, const Ws& ws, bool initial, hipStream_t st) {
    return kbl_compute_bounds_nodes(params, 1, a.n_tot, a.cols, stencil_nnz(c, initial), a.U,
                                    ws.rowptr, ws.cols, vgrid, ws.bounds, ws.bstat, st);
}

// Squeeze limiter and pressure step of the current state over V into the
// bounds in the workspace (steps 5-7 of Sec. 3.9; end values weight 0).
kbl_status limit_into(const kbl_fr1d* c, const kbl_params* params, const FrArgs& a, const Ws& ws,
                      const double* w, uint32_t* elem_status, hipStream_t st) {
    double cw[kMaxNs + 2];
    for (int j = 0; j < c->p + 1; ++j) cw[j] = w[j];
    cw[c->p + 1] = 0.0;
    cw[c->p + 2] = 0.0;
    return kbl_limit(params, 1, a.n_tot, a.n_v, a.U, ws.bounds, cw, a.U, nullptr, elem_status, st);
}

hipError_t launch_csr(const FrArgs& a, const Ws& ws, bool initial, hipStream_t st) {
    hipLaunchKernelGGL(fr1d_csr, dim3(blocks_for(a.n_tot)), dim3(kThreadsFr), 0, st, a.n_elem,
                       a.n_tot, a.n_v, a.bc, initial ? 1 : 0, ws.rowptr, ws.cols);
    return hipGetLastError();
}

// Checks shared by the limiting entry points (before any launch).
kbl_status check_limit_args(const kbl_fr1d* c, const kbl_params* params, const kbl_vgrid* vgrid,
                            double* U, void* workspace, size_t workspace_bytes) {
    if (!valid_cfg(c) || !params || !vgrid || !U) return KBL_ERR_ARG;
    if (params->precision != KBL_PREC_FP64 || params->flags & KBL_FLAG_ENERGY_PERSTATE)
        return KBL_ERR_UNSUPPORTED;
    if (!workspace || workspace_bytes < ws_layout(c, nullptr, nullptr)) return KBL_ERR_WORKSPACE;
    // params and the velocity grid, checked by the bounds entry point itself
    // on an empty problem (which launches nothing)
    return kbl_compute_bounds_nodes(params, 1, 0, 0, 0, nullptr, nullptr, nullptr, vgrid, nullptr,
                                    nullptr, nullptr);
}

}  // namespace
}  // namespace kbl

extern "C" {

int64_t kbl_fr1d_columns(const kbl_fr1d* cfg) {
    if (!kbl::valid_cfg(cfg)) return 0;
    return kbl::n_total(cfg) * (cfg->p + 3);
}

size_t kbl_fr1d_workspace_bytes(const kbl_fr1d* cfg) {
    if (!kbl::valid_cfg(cfg)) return 0;
    return kbl::ws_layout(cfg, nullptr, nullptr);
}

kbl_status kbl_fr1d_rhs(const kbl_fr1d* cfg, double gamma, const double* U, double* R,
                        void* stream) {
    kbl::FrArgs a;
    double w[kbl::kMaxNs];
    if (!U || !R) return KBL_ERR_ARG;
    kbl_status rc = kbl::make_args(cfg, gamma, const_cast<double*>(U), &a, w);
    if (rc != KBL_OK) return rc;
    a.R = R;
    return kbl::launch_rhs(a, cfg->p, (hipStream_t)stream) == hipSuccess ? KBL_OK : KBL_ERR_HIP;
}

kbl_status kbl_fr1d_limit(const kbl_fr1d* cfg, const kbl_params* params, const kbl_vgrid* vgrid,
                          double* U, void* workspace, size_t workspace_bytes,
                          uint32_t* elem_status, void* stream) {
    kbl_status rc = kbl::check_limit_args(cfg, params, vgrid, U, workspace, workspace_bytes);
    if (rc != KBL_OK) return rc;
    kbl::FrArgs a;
    double w[kbl::kMaxNs];
    rc = kbl::make_args(cfg, params->gamma, U, &a, w);
    if (rc != KBL_OK) return rc;
    kbl::Ws ws;
    kbl::ws_layout(cfg, (char*)workspace, &ws);
    hipStream_t st = (hipStream_t)stream;
    a.a = 1.0;
    a.b = 0.0;   // end values and ghosts only
    if (kbl::launch_stage(a, cfg->p, st) != hipSuccess) return KBL_ERR_HIP;
    if (!cfg->limit) return KBL_OK;
    if (kbl::launch_csr(a, ws, true, st) != hipSuccess) return KBL_ERR_HIP;
    rc = kbl::stencil_bounds(cfg, params, vgrid, a, ws, true, st);
    if (rc != KBL_OK) return rc;
    hipLaunchKernelGGL(kbl::fr1d_keep_admissible, dim3(kbl::blocks_for(a.n_tot)),
                       dim3(kbl::kThreadsFr), 0, st, a.U, a.n_tot, a.cols, a.n_v, a.gm1, ws.bounds);
    if (hipGetLastError() != hipSuccess) return KBL_ERR_HIP;
    return kbl::limit_into(cfg, params, a, ws, w, elem_status, st);
}

}  // extern "C"

namespace kbl {
namespace {

// One SSP-RK3 step; dt from the argument, or from tdt[1] in device memory.
kbl_status step_impl(const kbl_fr1d* cfg, const kbl_params* params, const kbl_vgrid* vgrid,
                     double dt, const double* tdt, double* U, void* workspace,
                     size_t workspace_bytes, uint32_t* elem_status, void* stream) {
    kbl_status rc = kbl::check_limit_args(cfg, params, vgrid, U, workspace, workspace_bytes);
    if (rc != KBL_OK) return rc;
    if (!tdt && (!(dt > 0.0) || !isfinite(dt))) return KBL_ERR_ARG;
    kbl::FrArgs a;
    double w[kbl::kMaxNs];
    rc = kbl::make_args(cfg, params->gamma, U, &a, w);
    if (rc != KBL_OK) return rc;
    kbl::Ws ws;
    kbl::ws_layout(cfg, (char*)workspace, &ws);
    hipStream_t st = (hipStream_t)stream;
    a.U0 = ws.U0;
    a.R = ws.R;
    a.dt = dt;
    a.tdt = tdt;
    if (cfg->limit) {
        if (kbl::launch_csr(a, ws, false, st) != hipSuccess) return KBL_ERR_HIP;
        // end values and ghosts of the input state (its bounds need them)
        a.a = 1.0;
        a.b = 0.0;
        if (kbl::launch_stage(a, cfg->p, st) != hipSuccess) return KBL_ERR_HIP;
    }
    // Shu-Osher SSP-RK3: u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
    // u^{n+1} = 1/3 u + 2/3 (u2 + dt L(u2)).  Each stage: bounds of its input
    // state, update, limiting of the updated state into those bounds.
    const double ca[3] = {0.0, 0.75, 1.0 / 3.0};
    const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int s = 0; s < 3; ++s) {
        if (cfg->limit) {
            rc = kbl::stencil_bounds(cfg, params, vgrid, a, ws, false, st);
            if (rc != KBL_OK) return rc;
        }
        if (kbl::launch_rhs(a, cfg->p, st) != hipSuccess) return KBL_ERR_HIP;
        a.a = ca[s];
        a.b = cb[s];
        a.save_u0 = s == 0;
        if (kbl::launch_stage(a, cfg->p, st) != hipSuccess) return KBL_ERR_HIP;
        if (cfg->limit) {
            rc = kbl::limit_into(cfg, params, a, ws, w, s == 2 ? elem_status : nullptr, st);
            if (rc != KBL_OK) return rc;
        }
    }
    return KBL_OK;
}

}  // namespace
}  // namespace kbl

extern "C" {

kbl_status kbl_fr1d_step(const kbl_fr1d* cfg, const kbl_params* params, const kbl_vgrid* vgrid,
                         double dt, double* U, void* workspace, size_t workspace_bytes,
                         uint32_t* elem_status, void* stream) {
    return kbl::step_impl(cfg, params, vgrid, dt, nullptr, U, workspace, workspace_bytes,
                          elem_status, stream);
}

kbl_status kbl_fr1d_step_dev(const kbl_fr1d* cfg, const kbl_params* params,
                             const kbl_vgrid* vgrid, const double* tdt, double* U,
                             void* workspace, size_t workspace_bytes, uint32_t* elem_status,
                             void* stream) {
    if (!tdt) return KBL_ERR_ARG;
    return kbl::step_impl(cfg, params, vgrid, 0.0, tdt, U, workspace, workspace_bytes,
                          elem_status, stream);
}

kbl_status kbl_fr1d_max_speed(const kbl_fr1d* cfg, double gamma, const double* U, double* out,
                              void* stream) {
    if (!kbl::valid_cfg(cfg) || !U || !out || !(gamma > 1.0)) return KBL_ERR_ARG;
    const int64_t nt = kbl::n_total(cfg);
    hipLaunchKernelGGL(kbl::fr1d_max_speed, dim3(1), dim3(1024), 0, (hipStream_t)stream, U,
                       cfg->n_elem, nt * (cfg->p + 3), cfg->p + 3, cfg->p + 1, gamma, out,
                       nullptr, 0.0, 0.0);
    return hipGetLastError() == hipSuccess ? KBL_OK : KBL_ERR_HIP;
}

kbl_status kbl_fr1d_cfl_dt(const kbl_fr1d* cfg, double gamma, const double* U, double cfl,
                           double t_end, double* tdt, void* stream) {
    if (!kbl::valid_cfg(cfg) || !U || !tdt || !(gamma > 1.0) || !(cfl > 0.0) || !isfinite(cfl) ||
        !isfinite(t_end))
        return KBL_ERR_ARG;
    const int64_t nt = kbl::n_total(cfg);
    const double h = (cfg->x1 - cfg->x0) / (double)cfg->n_elem;
    hipLaunchKernelGGL(kbl::fr1d_max_speed, dim3(1), dim3(1024), 0, (hipStream_t)stream, U,
                       cfg->n_elem, nt * (cfg->p + 3), cfg->p + 3, cfg->p + 1, gamma, nullptr, tdt,
                       cfl * h / (2.0 * cfg->p + 1.0), t_end);
    return hipGetLastError() == hipSuccess ? KBL_OK : KBL_ERR_HIP;
}

}  // extern "C"

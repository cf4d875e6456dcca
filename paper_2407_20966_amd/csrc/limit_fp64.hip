// FP64 coupled squeeze limiter and pressure step (steps 5-7 of the overview
// in Sec. 3.9), gfx950.
//
// HBM-bound: each node is read once and written once.  One lane owns one node
// (all d+2 variables); the G = next power of two >= n_s lanes of an element
// form an aligned lane group inside a wave64, so the element reductions (the
// weighted mean, the nodal max/min per variable and the minimum pressure) are
// exchanges within the group: on the DPP network inside a row of 16 lanes,
// by shuffles across rows.  Consecutive lanes read consecutive nodes of
// the SoA rows, so loads and stores are coalesced.  A workgroup limits two
// groups of elements and issues the loads of both before the arithmetic of
// the first, which doubles the bytes in flight per wave (tri2m 243 -> 234
// us, hex32 29.5 -> 25.8 us; four groups ran slower at fewer waves).
//  - mean with positive weights c_j (Assumption (iii)(a) of Sec. 4);
//  - alpha_i per component (eq. alpha) with the epsilon rule, coupled by the
//    minimum (eq. limiter), or each component with its own alpha_i (the
//    independent option of the same section);
//  - P_min over the limited nodes (eq. pmin) and, below the floor, the second
//    blend with alpha_P (eq. doublelimit).  An undefined pressure counts as
//    below the floor.  P(mean) <= floor gives alpha_P = 0 (flattened element).
#include <math.h>

#include "kbl_internal.h"

namespace kbl {
namespace {

constexpr int kThreads = 256;
constexpr double kInf = __builtin_inf();

// Group exchanges.  Stage k pairs each lane with a partner in the other
// half of its aligned block of 2^(k+1) lanes: inside a row of 16 on the DPP
// network (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror), across rows (groups of 32 or 64 lanes) by shuffles.  After
// the last stage every lane of the group holds the same combination.
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)b);
    const int hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// The partner of stage `o` (block half-size o = 1, 2, 4, ... G/2).
template <int O>
__device__ __forceinline__ double grp_partner(double v) {
    if (O == 1) return dpp_f64<kDppQuadXor1>(v);
    if (O == 2) return dpp_f64<kDppQuadXor2>(v);
    if (O == 4) return dpp_f64<kDppRowHalfMirror>(v);
    if (O == 8) return dpp_f64<kDppRowMirror>(v);
    return __shfl_xor(v, O, 64);
}
template <int O>
__device__ __forceinline__ int grp_partner_i32(int v) {
    if (O == 1) return dpp_i32<kDppQuadXor1>(v);
    if (O == 2) return dpp_i32<kDppQuadXor2>(v);
    if (O == 4) return dpp_i32<kDppRowHalfMirror>(v);
    if (O == 8) return dpp_i32<kDppRowMirror>(v);
    return __shfl_xor(v, O, 64);
}
template <int G, class F>
__device__ __forceinline__ double grp_reduce(double v, F f) {
    if (G >= 2) v = f(v, grp_partner<1>(v));
    if (G >= 4) v = f(v, grp_partner<2>(v));
    if (G >= 8) v = f(v, grp_partner<4>(v));
    if (G >= 16) v = f(v, grp_partner<8>(v));
    if (G >= 32) v = f(v, grp_partner<16>(v));
    if (G >= 64) v = f(v, grp_partner<32>(v));
    return v;
}
template <int G>
__device__ __forceinline__ double grp_sum(double v) {
    return grp_reduce<G>(v, [](double a, double b) { return a + b; });
}
template <int G>
__device__ __forceinline__ double grp_min(double v) {
    return grp_reduce<G>(v, [](double a, double b) { return fmin(a, b); });
}
template <int G>
__device__ __forceinline__ double grp_max(double v) {
    return grp_reduce<G>(v, [](double a, double b) { return fmax(a, b); });
}

// Compensated sums for the backward, whose results can be small differences
// of large terms: a value is carried as hi + lo, Knuth's TwoSum keeps the
// rounding error of every addition and fma that of every product.
struct Acc {
    double hi = 0.0, lo = 0.0;
    __device__ __forceinline__ void add(double x) {
        const double s = hi + x, bb = s - hi;
        lo += (hi - (s - bb)) + (x - bb);
        hi = s;
    }
    __device__ __forceinline__ void add_prod(double a, double b) {
        const double pr = a * b;
        lo += fma(a, b, -pr);
        add(pr);
    }
    __device__ __forceinline__ double value() const { return hi + lo; }
};
template <int O>
__device__ __forceinline__ void acc_stage(Acc& a) {
    const double h = grp_partner<O>(a.hi), l = grp_partner<O>(a.lo);
    a.add(h);
    a.lo += l;
}
template <int G>
__device__ __forceinline__ double grp_sum_c(Acc a) {
    if (G >= 2) acc_stage<1>(a);
    if (G >= 4) acc_stage<2>(a);
    if (G >= 8) acc_stage<4>(a);
    if (G >= 16) acc_stage<8>(a);
    if (G >= 32) acc_stage<16>(a);
    if (G >= 64) acc_stage<32>(a);
    return a.value();
}

template <int D>
__device__ __forceinline__ double pressure(double gm1, const double* w) {
    double mm = w[1] * w[1];
#pragma unroll
    for (int j = 2; j <= D; ++j) mm += w[j] * w[j];
    return gm1 * (w[D + 1] - 0.5 * mm / w[0]);
}

template <int D, int G>
__global__ __launch_bounds__(kThreads) void limit_fp64(LimitArgs p) {
    constexpr int NV = D + 2;
    constexpr int EPB = kThreads / G;   // elements per workgroup and group
    constexpr int H = 2;                // element groups per workgroup
    const int tid = threadIdx.x;
    const int j = tid % G;
    const int64_t e0 = (int64_t)blockIdx.x * (H * EPB) + tid / G;
    // Lanes past the last element or past n_s take part in the shuffles with
    // neutral values and never touch memory.  The nodes are read once and the
    // limited nodes written once: both streams go through the caches with the
    // non-temporal hint, which measured about 5% faster on 1 GB calls (the
    // bounds, read by every lane of the group, keep the default policy).
    double W[H][NV], Bv[H][2 * NV];
    bool BAD[H];
    const double c = j < p.n_s ? p.c[j] : 0.0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int64_t e = e0 + h * EPB;
        const bool live = (e < p.n_elem) && (j < p.n_s);
        const int64_t node = live ? e * p.n_s + j : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v)
            W[h][v] = live ? __builtin_nontemporal_load(&p.solution[(int64_t)v * p.n_nodes + node]) : 0.0;
        BAD[h] = false;
#pragma unroll
        for (int v = 0; v < 2 * NV; ++v) {
            Bv[h][v] = (e < p.n_elem) ? p.bounds[(int64_t)v * p.n_elem + e] : 0.0;
            BAD[h] |= !isfinite(Bv[h][v]);
        }
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int64_t e = e0 + h * EPB;
        const bool live = (e < p.n_elem) && (j < p.n_s);
        const int64_t node = live ? e * p.n_s + j : 0;
        double w[NV], b[2 * NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = W[h][v];
#pragma unroll
        for (int v = 0; v < 2 * NV; ++v) b[v] = Bv[h][v];
        const bool bad_b = BAD[h];
        // alpha_v = min(1, |b_max - wbar| / |w_max - wbar|, |b_min - wbar| /
        // |w_min - wbar|) (eq. alpha).  The ratios are ordered by cross products
        // of their (non-negative) numerators and denominators, which are bounded
        // below by eps, and only the smallest is divided: one division per
        // element for the coupled minimum, one per component when independent.
        uint32_t st = 0;
        double wbar[NV], rn[NV], rd[NV];
        bool eps0 = false;
    #pragma unroll
        for (int v = 0; v < NV; ++v) {
            wbar[v] = grp_sum<G>(c * w[v]) * p.inv_csum;
            const double wmax = grp_max<G>(live ? w[v] : -kInf);
            const double wmin = grp_min<G>(live ? w[v] : kInf);
            if (wbar[v] < b[v] || wbar[v] > b[NV + v]) st |= KBL_ST_MEAN_OUTSIDE;
            const double du = fabs(wmax - wbar[v]), dl = fabs(wmin - wbar[v]);
            const double nu = fabs(b[NV + v] - wbar[v]), nl = fabs(b[v] - wbar[v]);
            const bool lo = nl * du < nu * dl;          // the lower side binds first
            const bool ev = dl < p.eps || du < p.eps;
            eps0 |= ev;
            rn[v] = ev ? 0.0 : (lo ? nl : nu);          // ratio 0 under the eps rule
            rd[v] = ev ? 1.0 : (lo ? dl : du);
        }
        if (eps0) st |= KBL_ST_EPS_RULE;
        double acomp[NV];
        double amin;
        if (!p.independent) {
            double Nm = 1.0, Dm = 1.0;                  // smallest ratio, as Nm / Dm
    #pragma unroll
            for (int v = 0; v < NV; ++v)
                if (rn[v] * Dm < Nm * rd[v]) { Nm = rn[v]; Dm = rd[v]; }
            amin = Nm < Dm ? Nm / Dm : 1.0;
    #pragma unroll
            for (int v = 0; v < NV; ++v) acomp[v] = amin;
        } else {
            amin = 1.0;
    #pragma unroll
            for (int v = 0; v < NV; ++v) {
                acomp[v] = rn[v] < rd[v] ? rn[v] / rd[v] : 1.0;
                amin = fmin(amin, acomp[v]);
            }
        }
        if (amin < 1.0) st |= KBL_ST_LIMITED;

        // coupled (eq. limiter) or independent per-component blend
        double wt[NV];
    #pragma unroll
        for (int v = 0; v < NV; ++v) wt[v] = wbar[v] + acomp[v] * (w[v] - wbar[v]);

        double P = live ? pressure<D>(p.gm1, wt) : kInf;
        if (isnan(P)) P = -kInf;
        const double pmin = grp_min<G>(P);
        double aP = 1.0;
        if (pmin < p.p_floor) {
            st |= KBL_ST_PSTEP;
            const double pbar = pressure<D>(p.gm1, wbar);
            if (pbar > p.p_floor) aP = fabs((p.p_floor - pbar) / (pmin - pbar));
            else { aP = 0.0; st |= KBL_ST_PMEAN_FLOOR; }
    #pragma unroll
            for (int v = 0; v < NV; ++v) wt[v] = wbar[v] + aP * (wt[v] - wbar[v]);
        }

        if (bad_b) {
            st = KBL_ST_BAD_BOUNDS;
            amin = 1.0;
            aP = 1.0;
    #pragma unroll
            for (int v = 0; v < NV; ++v) wt[v] = w[v];
        }
        if (live) {
    #pragma unroll
            for (int v = 0; v < NV; ++v)
                __builtin_nontemporal_store(wt[v], &p.limited[(int64_t)v * p.n_nodes + node]);
            if (j == 0) {
                if (p.alpha) {
                    p.alpha[e] = amin;
                    p.alpha[p.n_elem + e] = aP;
                }
                if (p.status) p.status[e] = st;
            }
        }
    }
}

template <int D>
__device__ __forceinline__ void pressure_grad(double gm1, const double* w, double* g) {
    double mm = w[1] * w[1];
#pragma unroll
    for (int j = 2; j <= D; ++j) mm += w[j] * w[j];
    g[0] = gm1 * 0.5 * mm / (w[0] * w[0]);
#pragma unroll
    for (int j = 1; j <= D; ++j) g[j] = -gm1 * w[j] / w[0];
    g[D + 1] = gm1;
}

// Value and first lane (within the group) of the group maximum / minimum.
template <int G>
__device__ __forceinline__ int grp_first(bool hit, int j) {
    int idx = hit ? j : 1 << 30;
    if (G >= 2) idx = min(idx, grp_partner_i32<1>(idx));
    if (G >= 4) idx = min(idx, grp_partner_i32<2>(idx));
    if (G >= 8) idx = min(idx, grp_partner_i32<4>(idx));
    if (G >= 16) idx = min(idx, grp_partner_i32<8>(idx));
    if (G >= 32) idx = min(idx, grp_partner_i32<16>(idx));
    if (G >= 64) idx = min(idx, grp_partner_i32<32>(idx));
    return idx;
}

// Backward of the limiter: replays the forward decisions (same arithmetic as
// limit_fp64) and applies the chain rule through the element mean, the
// binding alpha term, the pressure step and the blends.  Ties pick the first
// node / variable.  Writes dJ/dsolution per node and dJ/dbounds per element.
template <int D, int G>
__global__ __launch_bounds__(kThreads) void limit_bwd_fp64(LimitArgs p, const double* grad,
                                                           double* gsol, double* gbnd,
                                                           ActiveSet act) {
    constexpr int NV = D + 2;
    constexpr int EPB = kThreads / G;
    const int tid = threadIdx.x;
    const int j = tid % G;
    const int64_t e = (int64_t)blockIdx.x * EPB + tid / G;
    const bool live = (e < p.n_elem) && (j < p.n_s);
    const int64_t node = live ? e * p.n_s + j : 0;

    double w[NV], Gw[NV];
    const double c = live ? p.c[j] : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        w[v] = live ? p.solution[(int64_t)v * p.n_nodes + node] : 0.0;
        Gw[v] = live ? grad[(int64_t)v * p.n_nodes + node] : 0.0;
    }
    double b[2 * NV];
    bool bad_b = false;
#pragma unroll
    for (int v = 0; v < 2 * NV; ++v) {
        b[v] = (e < p.n_elem) ? p.bounds[(int64_t)v * p.n_elem + e] : 0.0;
        bad_b |= !isfinite(b[v]);
    }

    double wbar[NV];
    double amin = 1.0, dstar = 0.0;
    int vstar = -1, upper = 0, jstar = -1;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        wbar[v] = grp_sum<G>(c * w[v]) * p.inv_csum;
        const double wmax = grp_max<G>(live ? w[v] : -kInf);
        const double wmin = grp_min<G>(live ? w[v] : kInf);
        const int jmax = grp_first<G>(live && w[v] == wmax, j);
        const int jmin = grp_first<G>(live && w[v] == wmin, j);
        const double dp = wmax - wbar[v], dm = wmin - wbar[v];
        double av;
        int vv = -1, up = 0, jj = -1;
        double dd = 0.0;
        if (fabs(dm) < p.eps || fabs(dp) < p.eps) {
            av = 0.0;
        } else {
            av = 1.0;
            const double ru = fabs((b[NV + v] - wbar[v]) / dp);
            const double rl = fabs((b[v] - wbar[v]) / dm);
            if (ru < av) { av = ru; vv = v; up = 1; jj = jmax; dd = dp; }
            if (rl < av) { av = rl; vv = v; up = 0; jj = jmin; dd = dm; }
        }
        if (av < amin) { amin = av; vstar = vv; upper = up; jstar = jj; dstar = dd; }
    }
    double wt[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) wt[v] = wbar[v] + amin * (w[v] - wbar[v]);
    double P = live ? pressure<D>(p.gm1, wt) : kInf;
    if (isnan(P)) P = -kInf;
    const double pmin = grp_min<G>(P);
    const int jp = grp_first<G>(live && P == pmin, j);

    // Element sums (the adjoint of the mean, the alpha_P and alpha terms)
    // are compensated: they can be small differences of large terms.
    double gwt[NV];
    Acc gwbar[NV];
    if (pmin < p.p_floor) {
        const double pbar = pressure<D>(p.gm1, wbar);
        if (pbar > p.p_floor) {
            const double N = p.p_floor - pbar, Dn = pmin - pbar;
            const double aP = fabs(N / Dn);
            const double sg = (N / Dn) >= 0.0 ? 1.0 : -1.0;
            Acc gaP_l;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                gwt[v] = aP * Gw[v];
                // w~ - wbar = alpha (w - wbar) (eq. limiter): formed from
                // w - wbar, not by the cancelling difference w~ - wbar
                gaP_l.add_prod(Gw[v], amin * (w[v] - wbar[v]));
                Acc t;
                t.add_prod(1.0 - aP, Gw[v]);
                gwbar[v].add(grp_sum_c<G>(t));
            }
            const double gaP = grp_sum_c<G>(gaP_l);
            const double gPbar = gaP * sg * (-1.0 / Dn + N / (Dn * Dn));
            const double gPmin = gaP * sg * (-N / (Dn * Dn));
            double gp[NV];
            pressure_grad<D>(p.gm1, wbar, gp);
#pragma unroll
            for (int v = 0; v < NV; ++v) gwbar[v].add_prod(gPbar, gp[v]);
            if (j == jp) {
                pressure_grad<D>(p.gm1, wt, gp);
#pragma unroll
                for (int v = 0; v < NV; ++v) gwt[v] += gPmin * gp[v];
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                gwt[v] = 0.0;
                Acc t;
                t.add(Gw[v]);
                gwbar[v].add(grp_sum_c<G>(t));
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) gwt[v] = Gw[v];
    }
    double gw[NV];
    Acc ga_l;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        gw[v] = amin * gwt[v];
        Acc t;
        t.add_prod(1.0 - amin, gwt[v]);
        gwbar[v].add(grp_sum_c<G>(t));
        ga_l.add_prod(gwt[v], w[v] - wbar[v]);
    }
    const double galpha = grp_sum_c<G>(ga_l);
    double gb_term = 0.0;
    if (vstar >= 0) {
        double bnd = 0.0, wb = 0.0;          // register-array selects (no dynamic indexing)
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v == vstar) { bnd = upper ? b[NV + v] : b[v]; wb = wbar[v]; }
        const double r = (bnd - wb) / dstar;
        const double g = galpha * (r >= 0.0 ? 1.0 : -1.0);
        gb_term = g / dstar;
        const double gdd = -g * (bnd - wb) / (dstar * dstar);
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v == vstar) { gwbar[v].add(-gb_term); gwbar[v].add(-gdd); }
        if (j == jstar) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v == vstar) gw[v] += gdd;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) gw[v] += gwbar[v].value() * c * p.inv_csum;

    if (bad_b) {
#pragma unroll
        for (int v = 0; v < NV; ++v) gw[v] = Gw[v];
    }
    if (live) {
#pragma unroll
        for (int v = 0; v < NV; ++v) gsol[(int64_t)v * p.n_nodes + node] = gw[v];
        if (j == 0) {
#pragma unroll
            for (int v = 0; v < 2 * NV; ++v) {
                const bool hit = !bad_b && vstar >= 0 && v == (upper ? NV + vstar : vstar);
                gbnd[(int64_t)v * p.n_elem + e] = hit ? gb_term : 0.0;
            }
        }
    }
    // Elements with a nonzero bounds' adjoint (bit test: +-0 stays out, a NaN
    // is listed) go on the active list: one atomic per workgroup, each listed
    // element at the workgroup's base plus the listed lanes of the waves
    // before it plus its rank among its wave's listed lanes.
    const bool head = j == 0 && e < p.n_elem;
    const bool listed = head && !bad_b && vstar >= 0 &&
                        ((uint64_t)__double_as_longlong(gb_term) << 1) != 0;
    if (head) act.flag[e] = listed ? 1 : 0;
    constexpr int NW = kThreads / 64;
    __shared__ uint32_t wcount[NW + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t m = __ballot(listed);
    if (lane == 0) wcount[wid] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += wcount[w];
        wcount[NW] = t ? atomicAdd(act.count, t) : 0u;
    }
    __syncthreads();
    if (listed) {
        uint32_t base = wcount[NW];
        for (int w = 0; w < wid; ++w) base += wcount[w];
        act.list[base + __popcll(m & ((1ull << lane) - 1))] = (int32_t)e;
    }
}

__global__ void clear_count(uint32_t* count) {
    if (threadIdx.x == 0) *count = 0;
}

template <int D, int G>
hipError_t launch_bwd_g(const LimitArgs& a, const double* grad, double* gsol, double* gbnd,
                        const ActiveSet& act, hipStream_t stream) {
    constexpr int EPB = kThreads / G;
    const int64_t blocks = (a.n_elem + EPB - 1) / EPB;
    if (blocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((limit_bwd_fp64<D, G>), dim3((unsigned)blocks), dim3(kThreads), 0, stream,
                       a, grad, gsol, gbnd, act);
    return hipGetLastError();
}

template <int D>
hipError_t launch_bwd_d(const LimitArgs& a, const double* grad, double* gsol, double* gbnd,
                        const ActiveSet& act, hipStream_t stream) {
    if (a.n_s <= 1) return launch_bwd_g<D, 1>(a, grad, gsol, gbnd, act, stream);
    if (a.n_s <= 2) return launch_bwd_g<D, 2>(a, grad, gsol, gbnd, act, stream);
    if (a.n_s <= 4) return launch_bwd_g<D, 4>(a, grad, gsol, gbnd, act, stream);
    if (a.n_s <= 8) return launch_bwd_g<D, 8>(a, grad, gsol, gbnd, act, stream);
    if (a.n_s <= 16) return launch_bwd_g<D, 16>(a, grad, gsol, gbnd, act, stream);
    if (a.n_s <= 32) return launch_bwd_g<D, 32>(a, grad, gsol, gbnd, act, stream);
    return launch_bwd_g<D, 64>(a, grad, gsol, gbnd, act, stream);
}

template <int D, int G>
hipError_t launch_g(const LimitArgs& a, hipStream_t stream) {
    constexpr int EPB = 2 * kThreads / G;
    const int64_t blocks = (a.n_elem + EPB - 1) / EPB;
    if (blocks > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((limit_fp64<D, G>), dim3((unsigned)blocks), dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

template <int D>
hipError_t launch_d(const LimitArgs& a, hipStream_t stream) {
    if (a.n_s <= 1) return launch_g<D, 1>(a, stream);
    if (a.n_s <= 2) return launch_g<D, 2>(a, stream);
    if (a.n_s <= 4) return launch_g<D, 4>(a, stream);
    if (a.n_s <= 8) return launch_g<D, 8>(a, stream);
    if (a.n_s <= 16) return launch_g<D, 16>(a, stream);
    if (a.n_s <= 32) return launch_g<D, 32>(a, stream);
    return launch_g<D, 64>(a, stream);
}

}  // namespace

hipError_t launch_limit_fp64(const LimitArgs& a, int dim, hipStream_t stream) {
    if (a.n_elem == 0) return hipSuccess;
    if (dim == 3) return launch_d<3>(a, stream);
    return dim == 2 ? launch_d<2>(a, stream) : launch_d<1>(a, stream);
}

hipError_t launch_limit_bwd_fp64(const LimitArgs& a, int dim, const double* grad, double* gsol,
                                 double* gbnd, const ActiveSet& act, hipStream_t stream) {
    // the count is cleared by a kernel (capturable; no memset node)
    hipLaunchKernelGGL(clear_count, dim3(1), dim3(64), 0, stream, act.count);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || a.n_elem == 0) return err;
    return dim == 2 ? launch_bwd_d<2>(a, grad, gsol, gbnd, act, stream)
                    : launch_bwd_d<1>(a, grad, gsol, gbnd, act, stream);
}

}  // namespace kbl

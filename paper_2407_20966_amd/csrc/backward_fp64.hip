// FP64 backward of the kinetic bounds (the differentiable form), gfx950.
//
// Given dJ/db per element (from the limiter backward), this computes dJ/d(state)
// for every stencil state of every element, then gathers them per node.  The
// adjoint is linear in dJ/db, which is zero wherever no bound binds the
// limiter (alpha = 1 or set by the epsilon rule, eq. alpha): only the
// elements the limiter's adjoint listed are visited, and the gather skips
// the others.
//
// Per listed element (one workgroup, the FP64 forward's tiling):
//  1. Prologue as in the forward (coefficients in LDS, velocity box); in
//     per-stencil box mode the states that set each box end are located
//     (first in stencil order on ties).
//  2. The log-Maxwellian envelopes are recomputed together with their winning
//     state per velocity node.  Nothing from the forward is stored.  In FP64
//     each log value is shifted below -1 (by the element's log-peak plus one,
//     folded into the per-state constant) and its lowest 8 mantissa bits are
//     replaced by the state's index; one running min/max of these keys then
//     yields the envelope's winner as well (a key differs from the log value
//     by less than 2^-44 of it, so only states within that of each other can
//     swap).  All keys being negative, among equal keys the maximum takes
//     the first state in stencil order and the minimum the last.  The
//     winner's log value is then recomputed exactly.  The mixed form tracks
//     its FP32 winners with explicit comparisons (first state wins ties).
//  3. Per node and envelope, the adjoint weight Phi of the moment rows
//     (eq. rhobounds, Ebounds, mmbounds, mpbounds with the relaxation of
//     eq. relaxed, the internal part of Sec. 3.6 and the trapezoid weights of
//     Sec. 3.7) times the envelope value gives that node's share of J; its
//     derivative w.r.t. the winner's (rho, U, theta) is
//       d ln g / d rho = 1/rho,  d/dU = (u - U)/theta,
//       d/dtheta = -d/(2 theta) + |u - U|^2/(2 theta^2) (+ 1/theta for g_I).
//     These are summed per winning state in a fixed order: each wave walks
//     the winners among its own nodes in increasing state order (DPP wave
//     sums, no barriers), and the per-wave sums are added in wave order, so
//     the result is bitwise deterministic.
//  4. In per-stencil box mode the node positions and trapezoid weights move
//     with the box ends; their adjoint is accumulated per node and passed to
//     the extreme states (lo = U - k sqrt(theta), hi = U + k sqrt(theta)).
//  5. (rho, U, theta) adjoints are mapped to conserved variables and written
//     to this element's stencil slots.
// A gather kernel then sums, for each node, the slots of listed elements that
// refer to it, walking the (symmetric) stencil in CSR order.
#include <type_traits>

#include "bounds_common.h"

namespace kbl {
namespace {

struct BwdArgs {
    BoundsArgs f;              // forward geometry and parameters
    const uint32_t* fstatus;   // forward status per element
    const double* gbnd;        // [2nv][n_elem] dJ/dbounds
    const uint32_t* act_count; // number of listed elements
    const int32_t* act_list;   // elements whose bounds' adjoint is nonzero
    double* slot;              // [nv][nnz * n_s] per-slot state gradients (out; listed
                               // elements' slots only)
};

template <int D, int NT>
__device__ __forceinline__ void write_slots_zero(const BwdArgs& a, int64_t row0, int64_t S) {
    const int64_t nslot = a.f.nnz * a.f.n_s;
    for (int64_t s = threadIdx.x; s < S; s += NT)
#pragma unroll
        for (int v = 0; v < D + 2; ++v) a.slot[(int64_t)v * nslot + row0 * a.f.n_s + s] = 0.0;
}

constexpr int kNoKey = 0x7fffffff;   // retired winner slot

// Envelope keys: a negative log value with its lowest 8 mantissa bits
// replaced by the state index s < 256.  One byte permute on the low dword:
// bytes 3..1 from the value, byte 0 from s (selector bytes 4..7 pick the
// first operand's bytes, 0..3 the second's).
__device__ __forceinline__ double keyed(double v, int s) {
    const uint32_t lo = __builtin_amdgcn_perm((uint32_t)__double2loint(v), (uint32_t)s, 0x07060500u);
    return __hiloint2double(__double2hiint(v), (int)lo);
}
__device__ __forceinline__ int key_index(double k) { return __double2loint(k) & 0xff; }

// Minimum waves per SIMD the register allocator targets.
#ifndef KBL_BWD_WAVES
#define KBL_BWD_WAVES 2
#endif

template <int D, int BX, int BY, int TX, int TY, bool F32>
__global__ __launch_bounds__(BX * BY) __attribute__((amdgpu_waves_per_eu(KBL_BWD_WAVES))) void bounds_bwd_fp64(BwdArgs a) {
    constexpr int NT = BX * BY;
    constexpr int NW = NT / 64;
    static_assert(NT % 64 == 0 && NT <= kThreads, "workgroup must be 1-4 waves");
    static_assert(!F32 || D == 2, "the mixed-precision form is 2D");
    __shared__ Coef sC[kMaxStates];
    __shared__ CoefF sF[F32 ? kMaxStates : 1];
    __shared__ double sZw[NW][kMaxStates][5];     // per-wave sums per winning state
    __shared__ int sExt[4];
    __shared__ Red red;

    const BoundsArgs& p = a.f;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int tx = tid % BX, ty = tid / BX;
    const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;
    const int64_t nslot = p.nnz * p.n_s;

    // only the listed elements: every other element's bounds' adjoint is
    // zero, and so is its contribution (the gather skips its slots)
    const uint32_t n_act = *a.act_count;
    for (uint32_t ia = blockIdx.x; ia < n_act; ia += gridDim.x) {
        const int64_t e = a.act_list[ia];
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) continue;  // no addressable slots
        const int64_t S = (row1 - row0) * p.n_s;
        const uint32_t fst = a.fstatus[e];
        if (S > kMaxStates || (fst & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE))) {
            write_slots_zero<D, NT>(a, row0, S);
            continue;
        }
        double gb[2 * (D + 2)];
#pragma unroll
        for (int v = 0; v < 2 * (D + 2); ++v) gb[v] = a.gbnd[(int64_t)v * p.n_elem + e];
        if (fst & KBL_ST_RHO_FLOOR) gb[0] = 0.0;   // the floored rho_min is constant
        // Every term below is linear in dJ/dbounds; a listed element whose
        // only nonzero entry was the floored rho_min contributes zero.
        // Bit test: +-0 only (a NaN or infinite adjoint is propagated).
        bool active = false;
#pragma unroll
        for (int v = 0; v < 2 * (D + 2); ++v)
            active |= ((uint64_t)__double_as_longlong(gb[v]) << 1) != 0;
        if (!active) {
            write_slots_zero<D, NT>(a, row0, S);
            continue;
        }
        constexpr int NV = D + 2;

        double box[4], ref[2];
        __syncthreads();
        stencil_prologue<D, NT>(p, row0, S, red, sC, box, ref);
        const double cx = box[0] + 0.5 * (box[1] - box[0]);
        const double cy = D == 2 ? box[2] + 0.5 * (box[3] - box[2]) : 0.0;
        if (F32) {
            // the mixed forward's FP32 coefficients (shifted, centred)
            const bool has_i = p.half_delta > 0.0;
            for (int s = tid; s < (int)S; s += NT) {
                const Coef c = sC[s];
                CoefF f;
                f.a = (float)(c.a - ref[0]);
                f.al = has_i ? (float)(c.al - ref[1]) : -kInfF;
                f.ux = (float)(c.ux - cx);
                f.uy = (float)(c.uy - cy);
                f.nk = (float)c.nk;
                sF[F32 ? s : 0] = f;
            }
        }
        // states setting the box ends (first in stencil order); per-wave sums zeroed
        if (tid < 4) sExt[tid] = 1 << 30;
        for (int i = tid; i < NW * (int)S * 5; i += NT) {
            const int w = i / (5 * (int)S), r = i - w * 5 * (int)S;
            sZw[w][r / 5][r % 5] = 0.0;
        }
        __syncthreads();
        if (p.grid_mode == KBL_GRID_STENCIL) {
            for (int s = tid; s < (int)S; s += NT) {
                const Prim st = load_prim<D>(p, state_node(p, row0, s));
                const double sd = sqrt(st.th);
                if (box_lo(st.ux, p.k, sd) == box[0]) atomicMin(&sExt[0], s);
                if (box_hi(st.ux, p.k, sd) == box[1]) atomicMin(&sExt[1], s);
                if (D == 2) {
                    if (box_lo(st.uy, p.k, sd) == box[2]) atomicMin(&sExt[2], s);
                    if (box_hi(st.uy, p.k, sd) == box[3]) atomicMin(&sExt[3], s);
                }
            }
        }
        const double hx = (box[1] - box[0]) / (double)(p.nx - 1);
        const double hy = D == 2 ? (box[3] - box[2]) / (double)(p.ny - 1) : 0.0;
        // compact tiles: thread (tx, ty) owns nodes (TX tx + i, TY ty + j), so
        // the winners a wave sees are few (winner regions are contiguous)
        double ux[TX], uy[TY];
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            const int x = TX * tx + i;
            ux[i] = node_pos(box[0], x < p.nx ? x : p.nx - 1, hx);
        }
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int y = TY * ty + j;
            uy[j] = D == 2 ? node_pos(box[2], y < p.ny ? y : p.ny - 1, hy) : 0.0;
        }
        // envelopes and their winners: Tmin, Tmax, Imin, Imax
        double q[4][TX][TY];
        int wn[4][TX][TY];
#pragma unroll
        for (int i = 0; i < TX; ++i)
#pragma unroll
            for (int j = 0; j < TY; ++j) wn[0][i][j] = wn[1][i][j] = wn[2][i][j] = wn[3][i][j] = 0;
        // Envelopes whose adjoint weight is identically zero are not formed:
        // env 0/1 (min/max of g) carry the rho, m and E bounds, env 2/3 (min/max
        // of g_I) the E bounds only (eq. Ebounds).  The limiter's adjoint gives
        // one binding bound, so mostly one or two envelopes are needed.
        auto nz = [](double v) { return ((uint64_t)__double_as_longlong(v) << 1) != 0; };
        bool gm = false;
#pragma unroll
        for (int k = 0; k < D; ++k) gm = gm || nz(gb[1 + k]) || nz(gb[NV + 1 + k]);
        const int need = ((nz(gb[0]) || nz(gb[D + 1]) || gm) ? 1 : 0) |
                         ((nz(gb[NV]) || nz(gb[NV + D + 1]) || gm) ? 2 : 0) |
                         (nz(gb[D + 1]) ? 4 : 0) | (nz(gb[NV + D + 1]) ? 8 : 0);
        // the loop variant: the smallest of {1, 2, 3, 5, 10, 15} covering `need`
        const int mask = need == 1 ? 1 : need == 2 ? 2 : (need & ~3) == 0 ? 3
                       : (need & ~5) == 0 ? 5 : (need & ~10) == 0 ? 10 : 15;
        if (!F32) {
#pragma unroll
            for (int i = 0; i < TX; ++i)
#pragma unroll
                for (int j = 0; j < TY; ++j) {
                    q[0][i][j] = kInf; q[1][i][j] = -kInf; q[2][i][j] = kInf; q[3][i][j] = -kInf;
                }
            // shifts that put every log value at or below -1 (a <= log-peak);
            // without internal degrees of freedom the internal envelopes get
            // a finite stand-in far below any other value
            const bool has_i = p.half_delta > 0.0;
            const double kt = ref[0] + 1.0;
            const double ki = has_i ? ref[1] + 1.0 : 0.0;
            auto envelopes = [&](auto mc) {
                constexpr int M = decltype(mc)::value;
                for (int s = 0; s < (int)S; ++s) {
                    const Coef c = sC[s];
                    const double at = c.a - kt;
                    const double ai = has_i ? c.al - ki : -1e300;
                    double A[TX], AI[TX], B[TY];
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        const double d = ux[i] - c.ux;
                        const double t = c.nk * d;
                        if (M & 3) A[i] = fma(t, d, at);
                        if (M & 12) AI[i] = fma(t, d, ai);
                    }
#pragma unroll
                    for (int j = 0; j < TY; ++j) {
                        const double d = uy[j] - c.uy;
                        B[j] = D == 2 ? (c.nk * d) * d : 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < TX; ++i)
#pragma unroll
                        for (int j = 0; j < TY; ++j) {
                            if (M & 3) {
                                const double qt = keyed(A[i] + B[j], s);
                                if (M & 1) q[0][i][j] = fmin(q[0][i][j], qt);
                                if (M & 2) q[1][i][j] = fmax(q[1][i][j], qt);
                            }
                            if (M & 12) {
                                const double qi = keyed(AI[i] + B[j], s);
                                if (M & 4) q[2][i][j] = fmin(q[2][i][j], qi);
                                if (M & 8) q[3][i][j] = fmax(q[3][i][j], qi);
                            }
                        }
                }
            };
            switch (mask) {
                case 1: envelopes(std::integral_constant<int, 1>{}); break;
                case 2: envelopes(std::integral_constant<int, 2>{}); break;
                case 3: envelopes(std::integral_constant<int, 3>{}); break;
                case 5: envelopes(std::integral_constant<int, 5>{}); break;
                case 10: envelopes(std::integral_constant<int, 10>{}); break;
                default: envelopes(std::integral_constant<int, 15>{}); break;
            }
#pragma unroll
            for (int env = 0; env < 4; ++env)
#pragma unroll
                for (int i = 0; i < TX; ++i)
#pragma unroll
                    for (int j = 0; j < TY; ++j)
                        wn[env][i][j] = ((mask >> env) & 1) ? key_index(q[env][i][j]) : kNoKey;
        } else {
            // winners from the FP32 envelopes; their FP64 log values are then
            // recomputed from the FP64 coefficients of the winning states
            float uxf[TX], uyf[TY], qf[4][TX][TY];
#pragma unroll
            for (int i = 0; i < TX; ++i) uxf[i] = (float)(ux[i] - cx);
#pragma unroll
            for (int j = 0; j < TY; ++j) uyf[j] = (float)(uy[j] - cy);
#pragma unroll
            for (int i = 0; i < TX; ++i)
#pragma unroll
                for (int j = 0; j < TY; ++j) {
                    qf[0][i][j] = kInfF; qf[1][i][j] = -kInfF; qf[2][i][j] = kInfF; qf[3][i][j] = -kInfF;
                }
            for (int s = 0; s < (int)S; ++s) {
                const CoefF c = sF[F32 ? s : 0];
                float A[TX], AI[TX], B[TY];
#pragma unroll
                for (int i = 0; i < TX; ++i) {
                    const float d = uxf[i] - c.ux;
                    const float t = c.nk * d;
                    A[i] = fmaf(t, d, c.a);
                    AI[i] = fmaf(t, d, c.al);
                }
#pragma unroll
                for (int j = 0; j < TY; ++j) {
                    const float d = uyf[j] - c.uy;
                    B[j] = (c.nk * d) * d;
                }
#pragma unroll
                for (int i = 0; i < TX; ++i)
#pragma unroll
                    for (int j = 0; j < TY; ++j) {
                        const float qt = A[i] + B[j], qi = AI[i] + B[j];
                        wn[0][i][j] = qt < qf[0][i][j] ? s : wn[0][i][j];
                        wn[1][i][j] = qt > qf[1][i][j] ? s : wn[1][i][j];
                        wn[2][i][j] = qi < qf[2][i][j] ? s : wn[2][i][j];
                        wn[3][i][j] = qi > qf[3][i][j] ? s : wn[3][i][j];
                        qf[0][i][j] = fminf(qf[0][i][j], qt);
                        qf[1][i][j] = fmaxf(qf[1][i][j], qt);
                        qf[2][i][j] = fminf(qf[2][i][j], qi);
                        qf[3][i][j] = fmaxf(qf[3][i][j], qi);
                    }
            }
            // (the FP64 log values of the winners are recomputed per node below)
        }
        // the winners, one byte per envelope (S <= 256 states)
        uint32_t pk[TX][TY];
#pragma unroll
        for (int i = 0; i < TX; ++i)
#pragma unroll
            for (int j = 0; j < TY; ++j)
                pk[i][j] = (uint32_t)(wn[0][i][j] & 0xff) | ((uint32_t)(wn[1][i][j] & 0xff) << 8) |
                           ((uint32_t)(wn[2][i][j] & 0xff) << 16) |
                           ((uint32_t)(wn[3][i][j] & 0xff) << 24);
        // Envelope by envelope (only those with a nonzero adjoint weight): per
        // node the adjoint weight Phi of the moment rows, the share M Phi f of
        // the winner and the box-end adjoint; then, per wave and winner in
        // increasing state order, the shares and their moments about the
        // winner's mean velocity, added to the wave's sums in envelope order
        // (no barriers inside; deterministic).
        double gl[2] = {0.0, 0.0}, gh[2] = {0.0, 0.0};
        const double inv_n1[2] = {1.0 / (double)(p.nx - 1), D == 2 ? 1.0 / (double)(p.ny - 1) : 0.0};
        const double inv_w[2] = {1.0 / (hx * (p.nx - 1)), D == 2 ? 1.0 / (hy * (p.ny - 1)) : 0.0};
#pragma unroll
        for (int env = 0; env < 4; ++env) {
            if (!((mask >> env) & 1)) continue;                  // zero adjoint weight
            const bool upper = env & 1, internal = env >= 2;
            const double r = upper ? rp : rm;
            const int b0 = upper ? NV : 0;                         // rho row of this side
            int w[TX][TY];
            double wv[TX][TY];
            int lk = kNoKey;                                       // smallest winner left
#pragma unroll
            for (int i = 0; i < TX; ++i)
#pragma unroll
                for (int j = 0; j < TY; ++j) {
                    const int x = TX * tx + i, y = TY * ty + j;
                    const bool valid = x < p.nx && (D == 1 || y < p.ny);
                    const double u[2] = {ux[i], uy[j]};
                    double M = hx * ((x == 0 || x == p.nx - 1) ? 0.5 : 1.0);
                    if (D == 2) M *= hy * ((y == 0 || y == p.ny - 1) ? 0.5 : 1.0);
                    if (!valid) M = 0.0;
                    // Phi: density + energy rows, and the momentum rows split
                    // by the sign of u (the lower bound takes the upper
                    // envelope where u < 0); g_I only enters the energy
                    double phi, dphi[2] = {0.0, 0.0};
                    if (!internal) {
                        double hu2 = 0.5 * u[0] * u[0];
                        if (D == 2) hu2 += 0.5 * u[1] * u[1];
                        phi = r * (gb[b0] + gb[b0 + D + 1] * hu2);
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const double gmin = gb[1 + k], gmax = gb[NV + 1 + k];
                            const double gk = (u[k] < 0.0) == upper ? gmin : gmax;
                            phi += r * gk * u[k];
                            dphi[k] = r * gk;
                            dphi[k] += r * gb[b0 + D + 1] * u[k];
                        }
                    } else {
                        phi = r * gb[b0 + D + 1];
                    }
                    // the winner's log value in FP64, as the forward forms it
                    const int sw = (int)((pk[i][j] >> (8 * env)) & 0xff);
                    const Coef& c = sC[sw];
                    const double dx = u[0] - c.ux;
                    double qv = fma(c.nk * dx, dx, internal ? c.al : c.a);
                    if (D == 2) {
                        const double dy = u[1] - c.uy;
                        qv += (c.nk * dy) * dy;
                    }
                    const double f = exp(qv);
                    const double wf = M * phi * f;
                    if (p.grid_mode == KBL_GRID_STENCIL && valid) {
                        const int t[2] = {x, y};
                        const double cu[2] = {c.ux, c.uy};
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const double dJdu = M * dphi[k] * f + wf * 2.0 * c.nk * (u[k] - cu[k]);
                            const double fr = (double)t[k] * inv_n1[k];
                            const double jw = wf * inv_w[k];
                            gl[k] += dJdu * (1.0 - fr) - jw;
                            gh[k] += dJdu * fr + jw;
                        }
                    }
                    wv[i][j] = wf;
                    w[i][j] = valid ? sw : kNoKey;
                    lk = min(lk, w[i][j]);
                }
            for (;;) {
                const int s = wave_min_i32(lk);
                if (s == kNoKey) break;
                const Coef c = sC[s];
                double z[4] = {0.0, 0.0, 0.0, 0.0};
                int nlk = kNoKey;
#pragma unroll
                for (int i = 0; i < TX; ++i)
#pragma unroll
                    for (int j = 0; j < TY; ++j) {
                        // the node's share if s won it, selected by a 0/1
                        // factor (shares are finite: M = 0 outside the grid)
                        const bool m = w[i][j] == s;
                        const double wf = (m ? 1.0 : 0.0) * wv[i][j];
                        w[i][j] = m ? kNoKey : w[i][j];
                        nlk = min(nlk, w[i][j]);
                        const double dx = ux[i] - c.ux, dy = D == 2 ? uy[j] - c.uy : 0.0;
                        const double d2 = dx * dx + dy * dy;
                        z[0] += wf;
                        z[1] = fma(wf, dx, z[1]);
                        if (D == 2) z[2] = fma(wf, dy, z[2]);
                        z[3] = fma(wf, d2, z[3]);
                    }
                lk = nlk;
                double zz[8] = {z[0], z[1], z[2], z[3], internal ? z[0] : 0.0, 0.0, 0.0, 0.0};
                const double zs = wave_transpose8<OpSum>(zz);   // lane l: sum k = l / 8
                if ((lane & 7) == 0 && (lane >> 3) < 5) sZw[wid][s][lane >> 3] += zs;
            }
        }
        double ext[4] = {gl[0], gh[0], gl[1], gh[1]};
        block_sum_t<NT, 4>(ext, red);    // valid in thread 0; contains the barriers
        if (tid == 0)
#pragma unroll
            for (int k = 0; k < 4; ++k) red.v[0][8 + k] = ext[k];
        __syncthreads();
        const double gext[4] = {red.v[0][8], red.v[0][9], red.v[0][10], red.v[0][11]};
        // (rho, U, theta) adjoints -> conserved variables, one thread per state;
        // the per-wave sums are combined in wave order
        for (int s = tid; s < (int)S; s += NT) {
            double z[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                z[k] = sZw[0][s][k];
#pragma unroll
                for (int w = 1; w < NW; ++w) z[k] += sZw[w][s][k];
            }
            const int64_t node = state_node(p, row0, s);
            const Prim st = load_prim<D>(p, node);
            const double th = st.th;
            double g_rho = z[0] / st.rho;
            double gU[2] = {z[1] / th, z[2] / th};
            double g_th = -0.5 * D / th * z[0] + 0.5 * z[3] / (th * th) + z[4] / th;
            if (p.grid_mode == KBL_GRID_STENCIL) {
                const double half_k_sd = 0.5 * p.k / sqrt(th);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    if (s == sExt[2 * k]) { gU[k] += gext[2 * k]; g_th -= gext[2 * k] * half_k_sd; }
                    if (s == sExt[2 * k + 1]) { gU[k] += gext[2 * k + 1]; g_th += gext[2 * k + 1] * half_k_sd; }
                }
            }
            const double U[2] = {st.ux, st.uy};
            double U2 = st.ux * st.ux;
            if (D == 2) U2 += st.uy * st.uy;
            double out_rho = g_rho + g_th * (p.gm1 * 0.5 * U2 - th) / st.rho;
            const int64_t at = row0 * p.n_s + s;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                out_rho -= gU[k] * U[k] / st.rho;
                a.slot[(int64_t)(1 + k) * nslot + at] = gU[k] / st.rho - g_th * p.gm1 * U[k] / st.rho;
            }
            a.slot[at] = out_rho;
            a.slot[(int64_t)(D + 1) * nslot + at] = g_th * p.gm1 / st.rho;
        }
    }
}

// dJ/dstates[v][node] = sum over the distinct elements e of the stencil row of
// the node's element J (stencils are symmetric: J's row lists every element
// whose stencil holds J) of the slots of every entry of J in row e.  An
// element listed twice in J's row (e.g. the left and right neighbour of a
// periodic mesh two elements wide) is counted once; when row e lists J
// twice, the tied copies of J's states share its envelopes between their two
// slots, so both are summed.  Fixed CSR order: deterministic.
template <int D>
__global__ __launch_bounds__(256) void gather_slots(BoundsArgs p, const double* slot,
                                                    const uint8_t* act_flag, double* gst) {
    constexpr int NV = D + 2;
    const int64_t nslot = p.nnz * p.n_s;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < p.n_nodes;
         n += (int64_t)gridDim.x * 256) {
        const int64_t J = n / p.n_s, jn = n % p.n_s;
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
        const int64_t r0 = p.rowptr[J], r1 = p.rowptr[J + 1];
        if (r0 >= 0 && r1 > r0 && r1 <= p.nnz) {
            for (int64_t r = r0; r < r1; ++r) {
                const int32_t e = p.cols[r];
                if (e < 0 || e >= p.n_elem || !act_flag[e]) continue;   // unlisted: zero
                bool seen = false;
                for (int64_t q = r0; q < r && !seen; ++q) seen = p.cols[q] == e;
                if (seen) continue;
                const int64_t q0 = p.rowptr[e], q1 = p.rowptr[e + 1];
                if (q0 < 0 || q1 <= q0 || q1 > p.nnz) continue;
                for (int64_t k = q0; k < q1; ++k) {
                    if (p.cols[k] == (int32_t)J) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[v] += slot[(int64_t)v * nslot + k * p.n_s + jn];
                    }
                }
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) gst[(int64_t)v * p.n_nodes + n] = acc[v];
    }
}

// Backward status per element: the forward's status, KBL_ST_BAD_STENCIL alone
// for a row outside the stencil arrays, KBL_ST_TOO_LARGE beyond kMaxStates
// states (zero gradient), and KBL_ST_ASYMMETRIC when the stencil lists an
// element J whose own row does not list it back (the gather would miss
// that slot).
__global__ __launch_bounds__(256) void bwd_status(BoundsArgs p, const uint32_t* fstatus,
                                                  uint32_t* status) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < p.n_elem;
         e += (int64_t)gridDim.x * 256) {
        const int64_t r0 = p.rowptr[e], r1 = p.rowptr[e + 1];
        if (r0 < 0 || r1 <= r0 || r1 > p.nnz) {
            status[e] = KBL_ST_BAD_STENCIL;
            continue;
        }
        uint32_t st = fstatus[e];
        if ((r1 - r0) * p.n_s > kMaxStates) st |= KBL_ST_TOO_LARGE;
        bool ok = true;
        for (int64_t r = r0; r < r1 && ok; ++r) {
            const int32_t J = p.cols[r];
            if (J < 0 || J >= p.n_elem) continue;
            const int64_t q0 = p.rowptr[J], q1 = p.rowptr[J + 1];
            bool found = false;
            if (q0 >= 0 && q1 > q0 && q1 <= p.nnz)
                for (int64_t k = q0; k < q1; ++k)
                    if (p.cols[k] == (int32_t)e) { found = true; break; }
            ok = found;
        }
        status[e] = ok ? st : (st | KBL_ST_ASYMMETRIC);
    }
}

// A grid of up to 4096 workgroups walks the active list (its length is on
// the device): a few per CU at a time, each taking every 4096th entry.
template <int D, int BX, int BY, int TX, int TY, bool F32 = false>
hipError_t launch_bwd(const BwdArgs& a, hipStream_t stream) {
    const int64_t g = a.f.n_elem < 4096 ? a.f.n_elem : 4096;
    hipLaunchKernelGGL((bounds_bwd_fp64<D, BX, BY, TX, TY, F32>), dim3((unsigned)g),
                       dim3(BX * BY), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bounds_bwd_fp64(const BoundsArgs& f, const uint32_t* fstatus, const double* gbnd,
                                  const ActiveSet& act, double* slot, double* grad_states,
                                  uint32_t* status, int dim, bool mixed, hipStream_t stream) {
    if (f.n_elem == 0) return hipSuccess;
    BwdArgs a;
    a.f = f;
    a.fstatus = fstatus;
    a.gbnd = gbnd;
    a.act_count = act.count;
    a.act_list = act.list;
    a.slot = slot;
    hipError_t err;
    if (dim == 2 && mixed) {
        const int n = f.nx > f.ny ? f.nx : f.ny;
        if (n <= 16) err = launch_bwd<2, 16, 16, 1, 1, true>(a, stream);
        else if (n <= 32) err = launch_bwd<2, 16, 16, 2, 2, true>(a, stream);
        else if (n <= 48) err = launch_bwd<2, 16, 16, 3, 3, true>(a, stream);
        else if (n <= 64) err = launch_bwd<2, 16, 16, 4, 4, true>(a, stream);
        else return hipErrorInvalidValue;
    } else if (mixed) {
        return hipErrorInvalidValue;
    } else if (dim == 2) {
        const int n = f.nx > f.ny ? f.nx : f.ny;
        if (n <= 16) err = launch_bwd<2, 16, 16, 1, 1>(a, stream);
        else if (n <= 32) err = launch_bwd<2, 16, 16, 2, 2>(a, stream);
        else if (n <= 48) err = launch_bwd<2, 16, 16, 3, 3>(a, stream);
        else if (n <= 64) err = launch_bwd<2, 16, 16, 4, 4>(a, stream);
        else return hipErrorInvalidValue;
    } else {
        if (f.nx <= 256) err = launch_bwd<1, 256, 1, 1, 1>(a, stream);
        else if (f.nx <= 512) err = launch_bwd<1, 256, 1, 2, 1>(a, stream);
        else if (f.nx <= 1024) err = launch_bwd<1, 256, 1, 4, 1>(a, stream);
        else if (f.nx <= 2048) err = launch_bwd<1, 256, 1, 8, 1>(a, stream);
        else return hipErrorInvalidValue;
    }
    if (err != hipSuccess) return err;
    const int64_t blocks = (f.n_nodes + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65535 * 16 ? blocks : 65535 * 16);
    if (dim == 2)
        hipLaunchKernelGGL(gather_slots<2>, dim3(g), dim3(256), 0, stream, f, slot, act.flag,
                           grad_states);
    else
        hipLaunchKernelGGL(gather_slots<1>, dim3(g), dim3(256), 0, stream, f, slot, act.flag,
                           grad_states);
    err = hipGetLastError();
    if (err != hipSuccess || !status) return err;
    const int64_t eb = (f.n_elem + 255) / 256;
    hipLaunchKernelGGL(bwd_status, dim3((unsigned)(eb < 65535 * 16 ? eb : 65535 * 16)),
                       dim3(256), 0, stream, f, fstatus, status);
    return hipGetLastError();
}

}  // namespace kbl

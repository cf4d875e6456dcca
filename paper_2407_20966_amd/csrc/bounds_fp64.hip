// FP64 kinetic bounds (steps 1-3 of the overview in Sec. 3.9), gfx950.
//
// One workgroup (1-4 wave64) owns one element at a time.
//  1. Prologue: every stencil state (every node of every element of the CSR
//     row) is read once, checked for admissibility (Assumption (i) of Sec. 4)
//     and turned into the coefficients of its log-Maxwellian
//       q_i(u) = ln rho_i - (d/2) ln(2 pi theta_i) - |u - U_i|^2 / (2 theta_i),
//     which are staged in LDS; in STENCIL mode the velocity box of
//     eq. truncdomain is reduced on the way.
//  2. Hot loop over the states: q_i is separable on the Cartesian velocity
//     grid, q_i = A_i[jx] + B_i[jy].  Each thread evaluates A (and
//     A + ln(theta delta / 2)) for its x nodes and B for its y nodes, then
//     spends two adds and four min/max per (state, node) pair.  Because exp is
//     monotone, min_i g_i = exp(min_i q_i) (eq. fminmax), and likewise for the
//     internal part g_I = (theta delta / 2) g (Sec. 3.6): four running extrema
//     per node stay in registers and only four exp per node are taken at the
//     end.  (Tile variants read B, or A and B, from LDS tables instead.)
//  3. Relaxation (eq. relaxed), trapezoid weights (Sec. 3.7) and the moment
//     contraction (eq. rhobounds, Ebounds, mmbounds, mpbounds) are done per
//     node, then reduced across the workgroup in a fixed order (bitwise
//     deterministic), floored (Sec. 3.8) and stored.
// Each thread owns a TX x TY tile of velocity nodes, strided by 16 so that
// the LDS table reads of a wave are contiguous or broadcast.  Tile modes:
// BTAB = 0 computes A and B per state in registers; 1 reads B from a table
// built per chunk of states; 2 reads A, A + ln(theta delta / 2) and B from
// such tables (per state: a few LDS reads instead of 4 TX + 3 TY VALU ops).
// Inputs are validated before the hot loop, which therefore never sees a NaN
// (only finite values and -inf when delta = 0).
#include "bounds_common.h"

namespace kbl {
namespace {

// ---------------------------------------------------------------- 2D kernel
// BX x BY threads; thread (tx, ty) owns velocity nodes (tx + BX i, ty + BY j),
// i < TX, j < TY.  BTAB = 1 reads B (and BTAB = 2 also A, A + l) from LDS
// tables built per sub-chunk of kTabStates states (fewer VALU ops, more LDS
// traffic and barriers).
template <int BX, int BY, int TX, int TY, int BTAB>
__global__ __launch_bounds__(BX * BY)
__attribute__((amdgpu_waves_per_eu(BTAB == 2 ? (TX * TY <= 9 ? 3 : 2) : 1))) void bounds_fp64_2d(BoundsArgs p) {
    constexpr int NT = BX * BY;
    constexpr int NXM = BX * TX;
    constexpr int NYM = BY * TY;
    constexpr int kTabStates = 32;
    static_assert(NT % 64 == 0 && NT <= kThreads, "workgroup must be 1-4 waves");
    static_assert(BTAB == 0 || (NXM == NYM && NYM <= NT), "table tiles are square");
    __shared__ Coef sC[kMaxStates];
    __shared__ double sB[BTAB ? kTabStates : 1][BTAB ? NYM : 1];
    // BTAB = 2: A and A + l tables too (row 2s: A, row 2s+1: A + l)
    __shared__ double sA[BTAB == 2 ? 2 * kTabStates : 1][BTAB == 2 ? NXM : 1];
    __shared__ ExpPair sExp[256];
    __shared__ Red red;

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;
    stage_exp_table<NT>(sExp);   // published by the prologue's barriers

    for (ElemRange er = xcd_range(p.n_elem, p.grid_blocks); er.e < er.end; er.e += er.step) {
        const int64_t e = er.e;
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<2>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        double box[4];
        const uint32_t flags = stencil_prologue<2, NT>(p, row0, S, red, sC, box);
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<2>(p, e, flags);
            continue;
        }
        const double lox = box[0], loy = box[2];
        const double hx = (box[1] - box[0]) / (double)(p.nx - 1);
        const double hy = (box[3] - box[2]) / (double)(p.ny - 1);

        // node coordinates (clamped into the grid for the ragged tail)
        double ux[TX], uy[TY];
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            const int j = tx + BX * i;
            ux[i] = node_pos(lox, j < p.nx ? j : p.nx - 1, hx);
        }
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int jj = ty + BY * j;
            uy[j] = node_pos(loy, jj < p.ny ? jj : p.ny - 1, hy);
        }

        // No +-inf starting values (two moves per accumulator): the
        // stencil's first state writes the envelopes in the peeled first
        // step of the hot loop; the empty asm gives the registers a defined
        // value until then.
        double qtn[TX][TY], qtx[TX][TY], qin[TX][TY], qix[TX][TY];
#pragma unroll
        for (int i = 0; i < TX; ++i)
#pragma unroll
            for (int j = 0; j < TY; ++j)
                asm volatile("" : "=v"(qtn[i][j]), "=v"(qtx[i][j]), "=v"(qin[i][j]), "=v"(qix[i][j]));

        for (int64_t c0 = 0; c0 < S; c0 += kMaxStates) {
            const int cn = (int)((S - c0) < kMaxStates ? (S - c0) : kMaxStates);
            if (c0 > 0) stage_chunk<2, NT>(p, row0, c0, cn, sC);
            for (int t0 = 0; t0 < cn; t0 += (BTAB ? kTabStates : kMaxStates)) {
                const int tn = BTAB ? ((cn - t0) < kTabStates ? (cn - t0) : kTabStates) : cn;
                if (BTAB) {
                    // Table columns: thread t fills node t % NYM of states
                    // t / NYM, t / NYM + NT / NYM, ... (one node coordinate
                    // per thread, no index arithmetic per entry).  The thread
                    // index goes through an empty asm statement so that the
                    // column and its coordinate are formed here, not kept
                    // live across the hot loop.
                    int ot = tid;
                    asm volatile("" : "+v"(ot));
                    const int j = ot % NYM, sj = ot / NYM;
                    const double yj = node_pos(loy, j < p.ny ? j : p.ny - 1, hy);
                    const double xj = node_pos(lox, j < p.nx ? j : p.nx - 1, hx);
                    __syncthreads();
                    if (sj < NT / NYM) {
                        // fully unrolled (LDS offsets become immediates)
                        constexpr int kPass = NT / NYM;
#pragma unroll
                        for (int k = 0; k < (kTabStates + kPass - 1) / kPass; ++k) {
                            const int s = sj + kPass * k;
                            if (s >= tn) break;
                            const Coef c = sC[t0 + s];
                            const double d = yj - c.uy;
                            sB[s][j] = (c.nk * d) * d;
                            if (BTAB == 2) {
                                const double dx = xj - c.ux;
                                const double t = c.nk * dx;
                                sA[2 * s][j] = fma(t, dx, c.a);
                                sA[2 * s + 1][j] = fma(t, dx, c.al);
                            }
                        }
                    }
                    __syncthreads();
                }
                if constexpr (BTAB == 2 && TX * TY > 9) {
                    // Software-pipelined: the table values of state s + 1 are
                    // read before the pair work of state s, so the LDS latency
                    // is covered by that work within the wave (tiles at two
                    // waves per SIMD: tri2m 159.4 -> 155.5 ms; the three-wave
                    // tiles hide it across waves and measured slower with
                    // it).  The last iteration re-reads its own state (in
                    // range, unused).
                    double ca[TX], cai[TX], cb[TY];
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        ca[i] = sA[0][tx + BX * i];
                        cai[i] = sA[1][tx + BX * i];
                    }
#pragma unroll
                    for (int j = 0; j < TY; ++j) cb[j] = sB[0][ty + BY * j];
                    // The stencil's first state sets the envelopes (q is its
                    // own min and max) instead of comparing with +-inf:
                    // tri2m 152.0 -> 150.6 ms, bounds bitwise the same (v_min
                    // and v_max return the number where the other operand
                    // is NaN, so only a stencil whose every state gave NaN
                    // at a node could differ).
                    int s0 = 0;
                    if (c0 == 0 && t0 == 0) {
                        const int sn = tn > 1 ? 1 : 0;
                        double na[TX], nai[TX], nb[TY];
#pragma unroll
                        for (int i = 0; i < TX; ++i) {
                            na[i] = sA[2 * sn][tx + BX * i];
                            nai[i] = sA[2 * sn + 1][tx + BX * i];
                        }
#pragma unroll
                        for (int j = 0; j < TY; ++j) nb[j] = sB[sn][ty + BY * j];
#pragma unroll
                        for (int i = 0; i < TX; ++i)
#pragma unroll
                            for (int j = 0; j < TY; ++j) {
                                const double q = ca[i] + cb[j];
                                const double qi = cai[i] + cb[j];
                                qtn[i][j] = q;
                                qtx[i][j] = q;
                                qin[i][j] = qi;
                                qix[i][j] = qi;
                            }
#pragma unroll
                        for (int i = 0; i < TX; ++i) { ca[i] = na[i]; cai[i] = nai[i]; }
#pragma unroll
                        for (int j = 0; j < TY; ++j) cb[j] = nb[j];
                        s0 = 1;
                    }
#pragma unroll 2
                    for (int s = s0; s < tn; ++s) {
                        const int sn = s + 1 < tn ? s + 1 : s;
                        double na[TX], nai[TX], nb[TY];
#pragma unroll
                        for (int i = 0; i < TX; ++i) {
                            na[i] = sA[2 * sn][tx + BX * i];
                            nai[i] = sA[2 * sn + 1][tx + BX * i];
                        }
#pragma unroll
                        for (int j = 0; j < TY; ++j) nb[j] = sB[sn][ty + BY * j];
#pragma unroll
                        for (int i = 0; i < TX; ++i)
#pragma unroll
                            for (int j = 0; j < TY; ++j) {
                                const double q = ca[i] + cb[j];
                                const double qi = cai[i] + cb[j];
                                qtn[i][j] = fmin(qtn[i][j], q);
                                qtx[i][j] = fmax(qtx[i][j], q);
                                qin[i][j] = fmin(qin[i][j], qi);
                                qix[i][j] = fmax(qix[i][j], qi);
                            }
#pragma unroll
                        for (int i = 0; i < TX; ++i) { ca[i] = na[i]; cai[i] = nai[i]; }
#pragma unroll
                        for (int j = 0; j < TY; ++j) cb[j] = nb[j];
                    }
                    continue;
                }
                // the x terms a, a + l and the y terms b of state s at this
                // thread's nodes, from the tables or from the coefficients
                auto terms = [&](int s, double* a, double* ai, double* b) {
                    if (BTAB == 2) {
#pragma unroll
                        for (int i = 0; i < TX; ++i) {
                            a[i] = sA[2 * s][tx + BX * i];
                            ai[i] = sA[2 * s + 1][tx + BX * i];
                        }
                    } else {
                        const Coef c = sC[t0 + s];
#pragma unroll
                        for (int i = 0; i < TX; ++i) {
                            const double d = ux[i] - c.ux;
                            const double t = c.nk * d;
                            a[i] = fma(t, d, c.a);
                            ai[i] = fma(t, d, c.al);
                        }
                    }
                    if (BTAB) {
#pragma unroll
                        for (int j = 0; j < TY; ++j) b[j] = sB[s][ty + BY * j];
                    } else {
                        const Coef c = sC[t0 + s];
#pragma unroll
                        for (int j = 0; j < TY; ++j) {
                            const double d = uy[j] - c.uy;
                            b[j] = (c.nk * d) * d;
                        }
                    }
                };
                int s0 = 0;
                if (c0 == 0 && t0 == 0) {
                    // the stencil's first state sets the envelopes
                    double a[TX], ai[TX], b[TY];
                    terms(0, a, ai, b);
#pragma unroll
                    for (int i = 0; i < TX; ++i)
#pragma unroll
                        for (int j = 0; j < TY; ++j) {
                            const double q = a[i] + b[j];
                            const double qi = ai[i] + b[j];
                            qtn[i][j] = q;
                            qtx[i][j] = q;
                            qin[i][j] = qi;
                            qix[i][j] = qi;
                        }
                    s0 = 1;
                }
#pragma unroll 2
                for (int s = s0; s < tn; ++s) {
                    double a[TX], ai[TX], b[TY];
                    terms(s, a, ai, b);
#pragma unroll
                    for (int i = 0; i < TX; ++i)
#pragma unroll
                        for (int j = 0; j < TY; ++j) {
                            const double q = a[i] + b[j];
                            const double qi = ai[i] + b[j];
                            qtn[i][j] = fmin(qtn[i][j], q);
                            qtx[i][j] = fmax(qtx[i][j], q);
                            qin[i][j] = fmin(qin[i][j], qi);
                            qix[i][j] = fmax(qix[i][j], qi);
                        }
                }
            }
        }

        // exp, relaxation, trapezoid weights and the moment contraction.  The
        // node coordinates and weights are formed here from box values passed
        // through an empty asm statement: otherwise the compiler computes
        // them (and other element-invariant parts of this contraction) before
        // the hot loop and keeps them live across it (register pressure).
        // The sums run over the unrelaxed envelopes g = exp(q); the factors
        // (1 -+ r) of eq. relaxed are applied once per thread afterwards.
        // Momentum (eq. mmbounds, mpbounds): the lower bound takes the upper
        // envelope where u < 0 and the lower one where u >= 0 (the upper
        // bound the reverse), so M u is split by sign into min(M u, 0) and
        // max(M u, 0), which feed separate sums without selects.
        double cx = lox, cy = loy, dx = hx, dy = hy;
        int otx = tx, oty = ty;
        asm volatile("" : "+v"(cx), "+v"(cy), "+v"(dx), "+v"(dy), "+v"(otx), "+v"(oty));
        // The weights and moment polynomials are separable, M = wx wy,
        // |u|^2 / 2 = vx^2 / 2 + vy^2 / 2 and the sign of M u_k depends on
        // u_k alone, so each node only feeds per-row sums over y (R: lower
        // and upper envelope, internal parts) and per-column sums over x (C:
        // lower and upper envelope), six fma per node; the moments are then
        // formed once per row and once per column.
        double sr[2] = {0, 0}, se[2] = {0, 0};    // rho, E: (lower, upper) envelope sums
        double mn[2][2] = {{0, 0}, {0, 0}};       // [dir][0]: sum u<0 of M u g_max, [1]: u>=0, M u g_min
        double mx[2][2] = {{0, 0}, {0, 0}};       // [dir][0]: sum u<0 of M u g_min, [1]: u>=0, M u g_max
        double ctn[TY], ctx[TY];                  // per column: sum over x of wx g_min, wx g_max
#pragma unroll
        for (int j = 0; j < TY; ++j) { ctn[j] = 0.0; ctx[j] = 0.0; }
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            const int jx = otx + BX * i;
            if (jx >= p.nx) continue;
            const double vx = node_pos(cx, jx, dx);
            const double wx = dx * ((jx == 0 || jx == p.nx - 1) ? 0.5 : 1.0);
            double rtn = 0.0, rtx = 0.0, rin = 0.0, rix = 0.0;   // per row: sum over y of wy g
            if constexpr (TX * TY == 16 && TY % 2 == 0) {
                // two nodes at a time, in three phases: the eight indices and
                // polynomials, the eight table reads together, the products
                // (otherwise each exp waits for its own table read right
                // after issuing it: tri2m 155.4 -> 153.1 ms)
#pragma unroll
                for (int j = 0; j < TY; j += 2) {
                    double xs[8];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        xs[4 * h + 0] = qtn[i][j + h]; xs[4 * h + 1] = qtx[i][j + h];
                        xs[4 * h + 2] = qin[i][j + h]; xs[4 * h + 3] = qix[i][j + h];
                    }
                    ExpPrep pr[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) pr[k] = exp_prep(xs[k]);
                    __builtin_amdgcn_sched_barrier(0);
                    ExpPair T[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) T[k] = sExp[pr[k].ni & 255];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int jy = oty + BY * (j + h);
                        // nodes past the grid (finite values) add zero
                        const double wy = jy < p.ny ? dy * ((jy == 0 || jy == p.ny - 1) ? 0.5 : 1.0) : 0.0;
                        const double gtn = exp_fin(pr[4 * h + 0], T[4 * h + 0]);
                        const double gtx = exp_fin(pr[4 * h + 1], T[4 * h + 1]);
                        const double gin = exp_fin(pr[4 * h + 2], T[4 * h + 2]);
                        const double gix = exp_fin(pr[4 * h + 3], T[4 * h + 3]);
                        rtn = fma(wy, gtn, rtn);
                        rtx = fma(wy, gtx, rtx);
                        rin = fma(wy, gin, rin);
                        rix = fma(wy, gix, rix);
                        ctn[j + h] = fma(wx, gtn, ctn[j + h]);
                        ctx[j + h] = fma(wx, gtx, ctx[j + h]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int jy = oty + BY * j;
                if (jy >= p.ny) continue;
                const double wy = dy * ((jy == 0 || jy == p.ny - 1) ? 0.5 : 1.0);
                const double gtn = exp_tab(qtn[i][j], sExp);
                const double gtx = exp_tab(qtx[i][j], sExp);
                const double gin = exp_tab(qin[i][j], sExp);
                const double gix = exp_tab(qix[i][j], sExp);
                rtn = fma(wy, gtn, rtn);
                rtx = fma(wy, gtx, rtx);
                rin = fma(wy, gin, rin);
                rix = fma(wy, gix, rix);
                ctn[j] = fma(wx, gtn, ctn[j]);
                ctx[j] = fma(wx, gtx, ctx[j]);
                // two nodes at a time: the exps of a pair interleave (their
                // LDS table reads overlap), while the temporaries of more
                // nodes would not fit the registers
                if (j & 1) __builtin_amdgcn_sched_barrier(0);
            }
            }
            const double hx2 = 0.5 * vx * vx;
            sr[0] = fma(wx, rtn, sr[0]);
            sr[1] = fma(wx, rtx, sr[1]);
            se[0] = fma(wx, fma(hx2, rtn, rin), se[0]);
            se[1] = fma(wx, fma(hx2, rtx, rix), se[1]);
            const double mu = wx * vx;
            const double neg = fmin(mu, 0.0), pos = fmax(mu, 0.0);
            mn[0][0] = fma(neg, rtx, mn[0][0]);
            mn[0][1] = fma(pos, rtn, mn[0][1]);
            mx[0][0] = fma(neg, rtn, mx[0][0]);
            mx[0][1] = fma(pos, rtx, mx[0][1]);
        }
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int jy = oty + BY * j;
            if (jy >= p.ny) continue;
            const double vy = node_pos(cy, jy, dy);
            const double wy = dy * ((jy == 0 || jy == p.ny - 1) ? 0.5 : 1.0);
            const double wy2 = wy * (0.5 * vy * vy);
            se[0] = fma(wy2, ctn[j], se[0]);
            se[1] = fma(wy2, ctx[j], se[1]);
            const double mu = wy * vy;
            const double neg = fmin(mu, 0.0), pos = fmax(mu, 0.0);
            mn[1][0] = fma(neg, ctx[j], mn[1][0]);
            mn[1][1] = fma(pos, ctn[j], mn[1][1]);
            mx[1][0] = fma(neg, ctn[j], mx[1][0]);
            mx[1][1] = fma(pos, ctx[j], mx[1][1]);
        }
        double part[8] = {rm * sr[0], rp * sr[1], rm * se[0], rp * se[1],
                          rp * mn[0][0] + rm * mn[0][1], rm * mx[0][0] + rp * mx[0][1],
                          rp * mn[1][0] + rm * mn[1][1], rm * mx[1][0] + rp * mx[1][1]};
        const double sum = block_sum8<NT>(part, red);
        if (tid < 8) store_bound_value<2>(p, e, tid, sum, flags);
    }
}

// ------------------------------------------- energy from per-state integrand
// Reading of Sec. 3.6 where the energy integrand is taken per state,
// E_min/max = sum_u M min/max_i g_i(u) (|u|^2/2 + theta_i delta/2), relaxed by
// (1 -+ r) like the distributions (eq. relaxed); rho and m as before.  The
// product g_i (h + c_i) has no log-domain shortcut, so the envelopes are kept
// in value space.  In 2D g_i is still separable in value space,
// g_i = exp(A_i[x]) exp(B_i[y]): both factors come from LDS tables built per
// chunk of states, and a pair costs one multiply for g, an add and a multiply
// for the integrand and four min/max.
// The 4 x 4 tile asks for two waves per SIMD of the register allocator (292
// VGPRs at one wave): it then keeps a few values in scratch, but the second
// wave hides the table reads (tri2m 270.7 -> 175.9 ms).
template <int BX, int BY, int TX, int TY>
__global__ __launch_bounds__(BX * BY)
__attribute__((amdgpu_waves_per_eu(TX * TY == 16 ? 2 : 1))) void bounds_fp64_2d_energy(BoundsArgs p) {
    constexpr int NT = BX * BY;
    constexpr int NXM = BX * TX;
    constexpr int NYM = BY * TY;
    constexpr int kTabStates = 32;
    static_assert(NT % 64 == 0 && NT <= kThreads, "workgroup must be 1-4 waves");
    __shared__ Coef sC[kMaxStates];
    __shared__ double sEA[kTabStates][NXM];
    __shared__ double sEB[kTabStates][NYM];
    __shared__ double sCs[kTabStates];        // theta delta / 2 per state
    __shared__ ExpPair sExp[256];
    __shared__ Red red;
    static_assert(NXM == NYM && NXM <= NT, "tables built by columns");

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;
    stage_exp_table<NT>(sExp);   // published by the prologue's barriers

    for (ElemRange er = xcd_range(p.n_elem, p.grid_blocks); er.e < er.end; er.e += er.step) {
        const int64_t e = er.e;
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<2>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        double box[4];
        const uint32_t flags = stencil_prologue<2, NT>(p, row0, S, red, sC, box);
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<2>(p, e, flags);
            continue;
        }
        const double lox = box[0], loy = box[2];
        const double hx = (box[1] - box[0]) / (double)(p.nx - 1);
        const double hy = (box[3] - box[2]) / (double)(p.ny - 1);
        double ux[TX], uy[TY], hux[TX], huy[TY];
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            const int j = tx + BX * i;
            ux[i] = node_pos(lox, j < p.nx ? j : p.nx - 1, hx);
            hux[i] = 0.5 * ux[i] * ux[i];
        }
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int jj = ty + BY * j;
            uy[j] = node_pos(loy, jj < p.ny ? jj : p.ny - 1, hy);
            huy[j] = 0.5 * uy[j] * uy[j];
        }
        // no +-inf starting values: the stencil's first state sets the
        // envelopes (the empty asm gives the registers a defined value)
        double gn[TX][TY], gx[TX][TY], en[TX][TY], ex[TX][TY];
#pragma unroll
        for (int i = 0; i < TX; ++i)
#pragma unroll
            for (int j = 0; j < TY; ++j)
                asm volatile("" : "=v"(gn[i][j]), "=v"(gx[i][j]), "=v"(en[i][j]), "=v"(ex[i][j]));

        for (int64_t c0 = 0; c0 < S; c0 += kMaxStates) {
            const int cn = (int)((S - c0) < kMaxStates ? (S - c0) : kMaxStates);
            if (c0 > 0) stage_chunk<2, NT>(p, row0, c0, cn, sC);
            for (int t0 = 0; t0 < cn; t0 += kTabStates) {
                const int tn = (cn - t0) < kTabStates ? (cn - t0) : kTabStates;
                __syncthreads();
                {
                    // by columns: thread t fills node t % NXM of states
                    // t / NXM, t / NXM + NT / NXM, ...
                    constexpr int kPass = NT / NXM;
                    const int j = tid % NXM, sj = tid / NXM;
                    const double xj = node_pos(lox, j < p.nx ? j : p.nx - 1, hx);
                    const double yj = node_pos(loy, j < p.ny ? j : p.ny - 1, hy);
                    if (sj < kPass) {
                        for (int s = sj; s < tn; s += kPass) {
                            const Coef& c = sC[t0 + s];
                            const double dx = xj - c.ux;
                            sEA[s][j] = exp_tab(fma(c.nk * dx, dx, c.a), sExp);
                            const double dy = yj - c.uy;
                            sEB[s][j] = exp_tab((c.nk * dy) * dy, sExp);
                        }
                    }
                }
                for (int s = tid; s < tn; s += NT) sCs[s] = p.half_delta * (-0.5 / sC[t0 + s].nk);
                __syncthreads();
                int s0 = 0;
                if (c0 == 0 && t0 == 0) {
                    const double cs = sCs[0];
                    double ea[TX], hc[TX], eb[TY];
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        ea[i] = sEA[0][tx + BX * i];
                        hc[i] = hux[i] + cs;
                    }
#pragma unroll
                    for (int j = 0; j < TY; ++j) eb[j] = sEB[0][ty + BY * j];
#pragma unroll
                    for (int i = 0; i < TX; ++i)
#pragma unroll
                        for (int j = 0; j < TY; ++j) {
                            const double g = ea[i] * eb[j];
                            const double eg = g * (hc[i] + huy[j]);
                            gn[i][j] = g;
                            gx[i][j] = g;
                            en[i][j] = eg;
                            ex[i][j] = eg;
                        }
                    s0 = 1;
                }
#pragma unroll 2
                for (int s = s0; s < tn; ++s) {
                    const double cs = sCs[s];
                    double ea[TX], hc[TX], eb[TY];
#pragma unroll
                    for (int i = 0; i < TX; ++i) {
                        ea[i] = sEA[s][tx + BX * i];
                        hc[i] = hux[i] + cs;
                    }
#pragma unroll
                    for (int j = 0; j < TY; ++j) eb[j] = sEB[s][ty + BY * j];
#pragma unroll
                    for (int i = 0; i < TX; ++i)
#pragma unroll
                        for (int j = 0; j < TY; ++j) {
                            const double g = ea[i] * eb[j];
                            const double eg = g * (hc[i] + huy[j]);
                            gn[i][j] = fmin(gn[i][j], g);
                            gx[i][j] = fmax(gx[i][j], g);
                            en[i][j] = fmin(en[i][j], eg);
                            ex[i][j] = fmax(ex[i][j], eg);
                        }
                }
            }
        }

        // separable contraction (M = wx wy; the sign of M u_k is the sign of
        // u_k): each node feeds per-row sums over y and per-column sums over
        // x, the moments are formed once per row and column, and (1 -+ r) is
        // applied to the sums
        double sr[2] = {0, 0}, se[2] = {0, 0}, mxs[2][2] = {{0, 0}, {0, 0}}, mys[2][2] = {{0, 0}, {0, 0}};
        double cn[TY], cx[TY];   // per column: sum over x of wx g_min, wx g_max
#pragma unroll
        for (int j = 0; j < TY; ++j) { cn[j] = 0.0; cx[j] = 0.0; }
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            const int jx = tx + BX * i;
            if (jx >= p.nx) continue;
            const double wx = hx * ((jx == 0 || jx == p.nx - 1) ? 0.5 : 1.0);
            double rn = 0.0, rx = 0.0, ren = 0.0, rex = 0.0;   // per row: sum over y of wy g, wy e
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int jy = ty + BY * j;
                if (jy >= p.ny) continue;
                const double wy = hy * ((jy == 0 || jy == p.ny - 1) ? 0.5 : 1.0);
                rn = fma(wy, gn[i][j], rn);
                rx = fma(wy, gx[i][j], rx);
                ren = fma(wy, en[i][j], ren);
                rex = fma(wy, ex[i][j], rex);
                cn[j] = fma(wx, gn[i][j], cn[j]);
                cx[j] = fma(wx, gx[i][j], cx[j]);
            }
            sr[0] = fma(wx, rn, sr[0]);
            sr[1] = fma(wx, rx, sr[1]);
            se[0] = fma(wx, ren, se[0]);
            se[1] = fma(wx, rex, se[1]);
            const double mu = wx * ux[i];
            const double neg = fmin(mu, 0.0), pos = fmax(mu, 0.0);
            mxs[0][0] = fma(neg, rx, mxs[0][0]);   // lower bound: u < 0 takes g_max
            mxs[0][1] = fma(pos, rn, mxs[0][1]);   //              u >= 0 takes g_min
            mxs[1][0] = fma(neg, rn, mxs[1][0]);   // upper bound: u < 0 takes g_min
            mxs[1][1] = fma(pos, rx, mxs[1][1]);   //              u >= 0 takes g_max
        }
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int jy = ty + BY * j;
            if (jy >= p.ny) continue;
            const double wy = hy * ((jy == 0 || jy == p.ny - 1) ? 0.5 : 1.0);
            const double mu = wy * uy[j];
            const double neg = fmin(mu, 0.0), pos = fmax(mu, 0.0);
            mys[0][0] = fma(neg, cx[j], mys[0][0]);
            mys[0][1] = fma(pos, cn[j], mys[0][1]);
            mys[1][0] = fma(neg, cn[j], mys[1][0]);
            mys[1][1] = fma(pos, cx[j], mys[1][1]);
        }
        double part[8] = {rm * sr[0], rp * sr[1], rm * se[0], rp * se[1],
                          rp * mxs[0][0] + rm * mxs[0][1], rm * mxs[1][0] + rp * mxs[1][1],
                          rp * mys[0][0] + rm * mys[0][1], rm * mys[1][0] + rp * mys[1][1]};
        block_sum_t<NT, 8>(part, red);
        if (tid == 0) store_bounds<2>(p, e, part, flags);
    }
}

// 1D: no separability; one exp per (state, node) pair.
template <int NT, int T>
__global__ __launch_bounds__(NT) void bounds_fp64_1d_energy(BoundsArgs p) {
    __shared__ Coef sC[kMaxStates];
    __shared__ ExpPair sExp[256];
    __shared__ Red red;
    const int tid = threadIdx.x;
    const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;
    stage_exp_table<NT>(sExp);   // published by the prologue's barriers
    for (ElemRange er = xcd_range(p.n_elem, p.grid_blocks); er.e < er.end; er.e += er.step) {
        const int64_t e = er.e;
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<1>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        double box[4];
        const uint32_t flags = stencil_prologue<1, NT>(p, row0, S, red, sC, box);
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<1>(p, e, flags);
            continue;
        }
        const double lo = box[0];
        const double h = (box[1] - box[0]) / (double)(p.nx - 1);
        double u[T], hu[T], gn[T], gx[T], en[T], ex[T];
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = tid + NT * i;
            u[i] = node_pos(lo, j < p.nx ? j : p.nx - 1, h);
            hu[i] = 0.5 * u[i] * u[i];
            gn[i] = kInf; gx[i] = -kInf; en[i] = kInf; ex[i] = -kInf;
        }
        for (int64_t c0 = 0; c0 < S; c0 += kMaxStates) {
            const int cn = (int)((S - c0) < kMaxStates ? (S - c0) : kMaxStates);
            if (c0 > 0) stage_chunk<1, NT>(p, row0, c0, cn, sC);
            for (int s = 0; s < cn; ++s) {
                const Coef c = sC[s];
                const double cs = p.half_delta * (-0.5 / c.nk);
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const double d = u[i] - c.ux;
                    const double g = exp_tab(fma(c.nk * d, d, c.a), sExp);
                    const double eg = g * (hu[i] + cs);
                    gn[i] = fmin(gn[i], g);
                    gx[i] = fmax(gx[i], g);
                    en[i] = fmin(en[i], eg);
                    ex[i] = fmax(ex[i], eg);
                }
            }
        }
        double part[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = tid + NT * i;
            if (j >= p.nx) continue;
            const double M = h * ((j == 0 || j == p.nx - 1) ? 0.5 : 1.0);
            const double ftn = rm * gn[i], ftx = rp * gx[i];
            part[0] += M * ftn;
            part[1] += M * ftx;
            part[2] += M * (rm * en[i]);
            part[3] += M * (rp * ex[i]);
            if (u[i] < 0.0) { part[4] += M * u[i] * ftx; part[5] += M * u[i] * ftn; }
            else            { part[4] += M * u[i] * ftn; part[5] += M * u[i] * ftx; }
        }
        block_sum_t<NT, 6>(part, red);
        if (tid == 0) store_bounds<1>(p, e, part, flags);
    }
}

// ---------------------------------------------------------------- 1D kernel
// No separability to exploit: each pair costs sub, mul and two fma before the
// four min/max.  Coefficients are broadcast from LDS.
// Up to 8 nodes per thread, three waves per SIMD are required of the register
// allocation (168 VGPRs): at T = 8 the compiler then keeps a few
// element-invariant values in scratch, reloaded outside the state loop, and
// small launches (one-dimensional meshes of a few thousand elements) run
// 7% faster than at two waves per SIMD; four waves would spill too much.
template <int NT, int T>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(T <= 8 ? 3 : 1)))
void bounds_fp64_1d(BoundsArgs p) {
    __shared__ Coef sC[kMaxStates];
    __shared__ ExpPair sExp[256];
    __shared__ Red red;
    const int tid = threadIdx.x;
    const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;
    stage_exp_table<NT>(sExp);   // published by the prologue's barriers
    for (ElemRange er = xcd_range(p.n_elem, p.grid_blocks); er.e < er.end; er.e += er.step) {
        const int64_t e = er.e;
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<1>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        double box[4];
        const uint32_t flags = stencil_prologue<1, NT>(p, row0, S, red, sC, box);
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<1>(p, e, flags);
            continue;
        }
        const double lo = box[0];
        const double h = (box[1] - box[0]) / (double)(p.nx - 1);
        // no +-inf starting values: the stencil's first state sets the
        // envelopes (the empty asm gives the registers a defined value)
        double u[T], qtn[T], qtx[T], qin[T], qix[T];
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = tid + NT * i;
            u[i] = node_pos(lo, j < p.nx ? j : p.nx - 1, h);
            asm volatile("" : "=v"(qtn[i]), "=v"(qtx[i]), "=v"(qin[i]), "=v"(qix[i]));
        }
        for (int64_t c0 = 0; c0 < S; c0 += kMaxStates) {
            const int cn = (int)((S - c0) < kMaxStates ? (S - c0) : kMaxStates);
            if (c0 > 0) stage_chunk<1, NT>(p, row0, c0, cn, sC);
            int s0 = 0;
            if (c0 == 0) {
                const Coef c = sC[0];
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const double d = u[i] - c.ux;
                    const double t = c.nk * d;
                    const double q = fma(t, d, c.a);
                    const double qi = fma(t, d, c.al);
                    qtn[i] = q;
                    qtx[i] = q;
                    qin[i] = qi;
                    qix[i] = qi;
                }
                s0 = 1;
            }
            for (int s = s0; s < cn; ++s) {
                const Coef c = sC[s];
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const double d = u[i] - c.ux;
                    const double t = c.nk * d;
                    const double q = fma(t, d, c.a);
                    const double qi = fma(t, d, c.al);
                    qtn[i] = fmin(qtn[i], q);
                    qtx[i] = fmax(qtx[i], q);
                    qin[i] = fmin(qin[i], qi);
                    qix[i] = fmax(qix[i], qi);
                }
            }
        }
        // unrelaxed envelope sums, relaxed once per thread afterwards; the
        // momentum sums split M u by sign (as in the 2D kernel)
        double sr[2] = {0, 0}, se[2] = {0, 0}, mn[2] = {0, 0}, mx[2] = {0, 0};
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = tid + NT * i;
            if (j >= p.nx) continue;
            const double M = h * ((j == 0 || j == p.nx - 1) ? 0.5 : 1.0);
            const double gtn = exp_tab(qtn[i], sExp);
            const double gtx = exp_tab(qtx[i], sExp);
            const double gin = exp_tab(qin[i], sExp);
            const double gix = exp_tab(qix[i], sExp);
            const double hu2 = 0.5 * u[i] * u[i];
            sr[0] += M * gtn;
            sr[1] += M * gtx;
            se[0] += M * (hu2 * gtn + gin);
            se[1] += M * (hu2 * gtx + gix);
            const double mu = M * u[i];
            const double neg = fmin(mu, 0.0), pos = fmax(mu, 0.0);
            mn[0] += neg * gtx;
            mn[1] += pos * gtn;
            mx[0] += neg * gtn;
            mx[1] += pos * gtx;
            __builtin_amdgcn_sched_barrier(0);
        }
        double part[8] = {rm * sr[0], rp * sr[1], rm * se[0], rp * se[1],
                          rp * mn[0] + rm * mn[1], rm * mx[0] + rp * mx[1], 0.0, 0.0};
        const double sum = block_sum8<NT>(part, red);
        if (tid < 6) store_bound_value<1>(p, e, tid, sum, flags);
    }
}

template <typename K>
hipError_t launch(K kernel, int threads, const BoundsArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(kernel, dim3(bounds_grid(a)), dim3(threads), 0, stream, a);
    return hipGetLastError();
}

// 2D tile configurations: (BX, BY, TX, TY, BTAB) covers nx <= BX*TX, ny <= BY*TY.
struct Tile2D {
    int bx, by, tx, ty, btab;
    hipError_t (*fn)(const BoundsArgs&, hipStream_t);
};

template <int BX, int BY, int TX, int TY, int BTAB>
hipError_t launch_2d(const BoundsArgs& a, hipStream_t stream) {
    return launch(bounds_fp64_2d<BX, BY, TX, TY, BTAB>, BX * BY, a, stream);
}

#define KBL_TILE(BX, BY, TX, TY, M) {BX, BY, TX, TY, M, launch_2d<BX, BY, TX, TY, M>}
constexpr Tile2D kTiles2D[] = {
    KBL_TILE(16, 16, 1, 1, 0),   // 0: n <= 16
    KBL_TILE(16, 16, 2, 2, 0),   // 1: n <= 32
    KBL_TILE(16, 16, 3, 3, 0),   // 2: n <= 48
    KBL_TILE(16, 16, 3, 3, 1),   // 3: n <= 48, B from LDS
    KBL_TILE(16, 8, 3, 6, 0),    // 4: n <= 48, two waves
    KBL_TILE(16, 16, 4, 4, 0),   // 5: n <= 64
    KBL_TILE(16, 16, 4, 4, 1),   // 6: n <= 64, B from LDS
    KBL_TILE(32, 8, 2, 8, 1),    // 7: n <= 64, B from LDS
    KBL_TILE(16, 16, 2, 4, 0),   // 8: nx <= 32, ny <= 64
    KBL_TILE(16, 16, 4, 2, 0),   // 9: nx <= 64, ny <= 32
    KBL_TILE(16, 16, 2, 2, 2),   // 10: n <= 32, A and B from LDS
    KBL_TILE(16, 16, 3, 3, 2),   // 11: n <= 48, A and B from LDS
    KBL_TILE(16, 16, 4, 4, 2),   // 12: n <= 64, A and B from LDS
    KBL_TILE(16, 8, 3, 6, 2),    // 13: n <= 48, two waves, A and B from LDS
};
#undef KBL_TILE
constexpr int kNumTiles2D = sizeof(kTiles2D) / sizeof(kTiles2D[0]);

// Defaults from a measured sweep: with A, A + l and B read from LDS tables
// the inner loop is the pair work alone (tiles 11 and 12); kbl_autotune_bounds
// may still pick another tile or a persistent grid for a given shape.
int default_tile_2d(int nx, int ny) {
    const int n = nx > ny ? nx : ny;
    if (n <= 16) return 0;
    if (n <= 32) return 1;
    if (n <= 48) return 11;
    return 12;
}

}  // namespace

int bounds_tile_count_2d() { return kNumTiles2D; }
int bounds_default_tile_2d(int nx, int ny) { return default_tile_2d(nx, ny); }

bool bounds_tile_fits_2d(int tile, int nx, int ny) {
    if (tile < 0 || tile >= kNumTiles2D) return false;
    const Tile2D& t = kTiles2D[tile];
    return nx <= t.bx * t.tx && ny <= t.by * t.ty;
}

hipError_t launch_bounds_fp64_energy(const BoundsArgs& a, int dim, hipStream_t stream) {
    if (a.n_elem == 0) return hipSuccess;
    if (dim == 2) {
        const int n = a.nx > a.ny ? a.nx : a.ny;
        if (n <= 16) return launch(bounds_fp64_2d_energy<16, 16, 1, 1>, 256, a, stream);
        if (n <= 32) return launch(bounds_fp64_2d_energy<16, 16, 2, 2>, 256, a, stream);
        if (n <= 48) return launch(bounds_fp64_2d_energy<16, 16, 3, 3>, 256, a, stream);
        if (n <= 64) return launch(bounds_fp64_2d_energy<16, 16, 4, 4>, 256, a, stream);
        return hipErrorInvalidValue;
    }
    if (a.nx <= 64) return launch(bounds_fp64_1d_energy<64, 1>, 64, a, stream);
    if (a.nx <= 256) return launch(bounds_fp64_1d_energy<256, 1>, kThreads, a, stream);
    if (a.nx <= 512) return launch(bounds_fp64_1d_energy<256, 2>, kThreads, a, stream);
    if (a.nx <= 1024) return launch(bounds_fp64_1d_energy<256, 4>, kThreads, a, stream);
    if (a.nx <= 2048) return launch(bounds_fp64_1d_energy<256, 8>, kThreads, a, stream);
    if (a.nx <= 4096) return launch(bounds_fp64_1d_energy<256, 16>, kThreads, a, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_bounds_fp64(const BoundsArgs& a, int dim, hipStream_t stream, int tile) {
    if (a.n_elem == 0) return hipSuccess;
    if (dim == 2) {
        if (tile < 0) tile = default_tile_2d(a.nx, a.ny);
        if (!bounds_tile_fits_2d(tile, a.nx, a.ny)) return hipErrorInvalidValue;
        return kTiles2D[tile].fn(a, stream);
    }
    if (a.nx <= 64) return launch(bounds_fp64_1d<64, 1>, 64, a, stream);
    if (a.nx <= 256) return launch(bounds_fp64_1d<256, 1>, kThreads, a, stream);
    if (a.nx <= 512) return launch(bounds_fp64_1d<256, 2>, kThreads, a, stream);
    if (a.nx <= 1024) return launch(bounds_fp64_1d<256, 4>, kThreads, a, stream);
    if (a.nx <= 2048) return launch(bounds_fp64_1d<256, 8>, kThreads, a, stream);
    if (a.nx <= 4096) return launch(bounds_fp64_1d<256, 16>, kThreads, a, stream);
    return hipErrorInvalidValue;
}

}  // namespace kbl

// Mixed-precision kinetic bounds (steps 1-3 of the overview in Sec. 3.9), gfx950.
//
// Same method as the FP64 kernels; what changes is the arithmetic of the
// hot loop and of the moment contraction:
//  - FP64: stencil prologue (admissibility, velocity box of eq. truncdomain,
//    log-Maxwellian coefficients), the per-element log-peak references, the
//    relaxation factors of eq. relaxed, the final scaling and the density
//    floor of Sec. 3.8.
//  - FP32: the envelopes.  Coefficients are shifted by the element's log-peak
//    reference and velocities are centred on the box, then q = A[x] + B[y]
//    and the four running extrema are kept in FP32; two states are folded
//    per step with three-input min/max.  On the MFMA paths each envelope is
//    then exponentiated relative to a power of two at its maximum over the
//    wave's nodes.
//  - Contraction of the moments (eq. rhobounds, Ebounds, mmbounds, mpbounds)
//    with the trapezoid weights (Sec. 3.7).  The weights and moment
//    polynomials are separable, M psi(u) = X(ux) Y(uy), so the contraction
//    is done in two stages: over y with four factors
//    Y = Wy {1, uy<0 ? uy : 0, uy>=0 ? uy : 0, uy^2}, then over x with
//    X = Wx {1, ux<0 ? ux : 0, ux>=0 ? ux : 0, ux^2}.  The y stage runs on
//    MFMA (v_mfma_f32_16x16x16, FP16 operands split hi/lo, or BF16 operands
//    split in three, FP32 accumulation) or on the FP32 VALU; the x stage and
//    everything after it is FP64.
//
// Workgroup = NW waves; the x nodes come in tiles of 16 and a wave owns TXW
// of them.  Lane l owns x node 16t + l%16 of each of its tiles t and the y
// nodes 16k + 4(l/16) + i (i < 4, k < KS): per tile, exactly the A-operand
// layout of the 16x16x16 MFMA with M = x, K = y, so the envelope values feed
// the matrix core straight from registers.  The B operand (lane l: factor
// l%16 at the same y nodes) is built per element in registers; the C result
// (lane l: factor l%16 at x rows 16t + 4(l/16) + i) is contracted with X in
// FP64.  The per-state y terms (B at each y node) come from an LDS table
// built per chunk of states, one node column per thread, and one B-table
// read serves the TXW x nodes of a lane; the four-wave tiles take the x
// terms (A and A + l at each x node) from a second table built alongside.
#include "bounds_common.h"

namespace kbl {
namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

typedef float float2_t __attribute__((ext_vector_type(2)));

// Minimum waves per SIMD the register allocator targets (1 = no constraint).
#ifndef KBL_MIXED_WAVES
#define KBL_MIXED_WAVES 1
#endif
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kF16Scale = 16384.0f;            // 2^14, exact
constexpr float kF16Log2Scale = 14.0f;

// FP32 -> BF16 (and FP16) by gfx950's conversion instructions, round to
// nearest even; BF16 -> FP32 is exact.
typedef __bf16 bf16v4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float bf_up(__bf16 b) { return (float)b; }

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Maximum over the wave, uniform: rows on DPP, then the four row results by
// readlane.
__device__ __forceinline__ float wave_max_f32(float v) {
    v = fmaxf(v, dpp_f32<kDppXor1>(v));
    v = fmaxf(v, dpp_f32<kDppXor2>(v));
    v = fmaxf(v, dpp_f32<kDppHalfMirror>(v));
    v = fmaxf(v, dpp_f32<kDppMirror>(v));
    const int b = __float_as_int(v);
    return fmaxf(fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 0)), __int_as_float(__builtin_amdgcn_readlane(b, 16))),
                 fmaxf(__int_as_float(__builtin_amdgcn_readlane(b, 32)), __int_as_float(__builtin_amdgcn_readlane(b, 48))));
}

// The y factors (B operand) split once per element: FP16 hi/lo of the
// factor scaled by 2^14, or BF16 in three parts.
template <int KS, int CT>
struct YSplit {
    half4_t h[KS], l[KS];          // FP16
    bf16x4_t b1[KS], b2[KS], b3[KS];   // BF16
};
template <int KS, int CT>
__device__ __forceinline__ void split_y(const float* yb, YSplit<KS, CT>& y) {
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        if (CT == KBL_PREC_MIXED_FP16) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float bv = yb[4 * k + i] * kF16Scale;
                y.h[k][i] = (_Float16)bv;
                y.l[k][i] = (_Float16)(bv - (float)y.h[k][i]);
            }
        } else {
            bf16v4_t t1, t2, t3;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float bv = yb[4 * k + i];
                t1[i] = (__bf16)bv; bv -= bf_up(t1[i]);
                t2[i] = (__bf16)bv; bv -= bf_up(t2[i]);
                t3[i] = (__bf16)bv;
            }
            y.b1[k] = __builtin_bit_cast(bf16x4_t, t1);
            y.b2[k] = __builtin_bit_cast(bf16x4_t, t2);
            y.b3[k] = __builtin_bit_cast(bf16x4_t, t3);
        }
    }
}

// y-stage contraction of one envelope (one x tile) on MFMA: returns C
// (lane l: factor l%16 at x rows 4(l/16) + i of the tile).
template <int KS, int CT>
__device__ __forceinline__ float4_t mfma_ystage(const float* f, const YSplit<KS, CT>& y) {
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        if (CT == KBL_PREC_MIXED_FP16) {
            // both operands are scaled by 2^14 (envelopes <= 1, factors < 2)
            // so that the low halves stay clear of FP16 subnormals; the
            // envelope values arrive scaled (the shift is in their exp2)
            half4_t ah, al;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float av = f[4 * k + i];
                ah[i] = (_Float16)av;
                al[i] = (_Float16)(av - (float)ah[i]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, y.h[k], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(al, y.h[k], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, y.l[k], acc, 0, 0, 0);
        } else {
            bf16v4_t t1, t2, t3;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float av = f[4 * k + i];
                t1[i] = (__bf16)av; av -= bf_up(t1[i]);
                t2[i] = (__bf16)av; av -= bf_up(t2[i]);
                t3[i] = (__bf16)av;
            }
            const bf16x4_t a1 = __builtin_bit_cast(bf16x4_t, t1);
            const bf16x4_t a2 = __builtin_bit_cast(bf16x4_t, t2);
            const bf16x4_t a3 = __builtin_bit_cast(bf16x4_t, t3);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, y.b1[k], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, y.b2[k], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, y.b1[k], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, y.b3[k], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, y.b2[k], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, y.b1[k], acc, 0, 0, 0);
        }
    }
    return acc;
}

// Trapezoid weight (Sec. 3.7) times the x factors X = Wx {1, ux<0, ux>=0, ux^2}.
struct XF {
    double w, m, p, q;
};
// Nodes past the grid (the ragged tail of the last tile) get zero factors;
// selects rather than a branch, since the lanes of a wave differ.
__device__ __forceinline__ XF x_factors(const BoundsArgs& p, const double* box, double hx, int x) {
    const bool in = x < p.nx;
    const double u = node_pos(box[0], in ? x : p.nx - 1, hx);
    XF f;
    f.w = in ? hx * ((x == 0 || x == p.nx - 1) ? 0.5 : 1.0) : 0.0;
    f.m = u < 0.0 ? f.w * u : 0.0;
    f.p = u < 0.0 ? 0.0 : f.w * u;
    f.q = f.w * u * u;
    return f;
}

// Partial sums, in this order: T_min: S0, SXm, SXp, SYm, SYp, S2; T_max: the
// same six; I_min: S0; I_max: S0.
constexpr int kNP = 14;

// NW waves; wave w owns the x tiles w + NW i (i < TXW) of 16 nodes each; lane
// l owns x node 16 t + l%16 of each of its tiles and the y nodes
// 16 k + 4 (l/16) + i (i < 4, k < KS).
template <int TXW, int KS, int NW, int CT>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(KBL_MIXED_WAVES))) void bounds_mixed_2d(BoundsArgs p) {
    constexpr int NT = NW * 64;
    constexpr int NY = 16 * KS;     // y nodes covered
    constexpr int TY = 4 * KS;      // y nodes per lane
    constexpr int NX = 16 * TXW * NW;   // x nodes covered
    static_assert(NX == NY, "the tables are built by columns of a square tile");
    constexpr int kTab = 64;            // states per table chunk
    // The four-wave tiles (two workgroups per CU) also take the per-state x
    // terms from LDS: measured faster there; the smaller tiles run three or
    // more workgroups per CU, whose LDS share the table would exceed, and
    // form them in registers.
    constexpr bool ATAB = NW == 4;
    // the FP64 coefficients are only needed until the FP32 copies exist; the
    // tables reuse their space: B = nk (uy - Uy)^2 per (state, y node), and
    // per (state, x node) the pair A = a + nk (ux - Ux)^2, A + l
    union Stage {
        Coef c[kMaxStates];
        struct {
            float b[kTab][NY];
            float2_t ai[ATAB ? kTab : 1][ATAB ? NX : 1];
        } t;
    };
    __shared__ __align__(16) Stage stage;
    __shared__ CoefF sF[kMaxStates];
    __shared__ Red red;
    // the y factors Wy {1, uy<0 ? uy : 0, uy>=0 ? uy : 0, uy^2} of the
    // element's y nodes, zero past the grid (FP32, rounded from FP64)
    __shared__ __align__(16) float yfac[4][NY];

    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63, xr = l & 15, g = l >> 4;

    for (ElemRange er = xcd_range(p.n_elem, p.grid_blocks); er.e < er.end; er.e += er.step) {
        const int64_t e = er.e;
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<2>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        if (S > kMaxStates) {
            // the mixed path keeps every stencil state in LDS
            if (tid == 0) store_nan<2>(p, e, KBL_ST_TOO_LARGE);
            continue;
        }
        double box[4], ref[2];
        __syncthreads();   // the previous element's B table is no longer read
        const uint32_t flags = stencil_prologue<2, NT>(p, row0, S, red, stage.c, box, ref);
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<2>(p, e, flags);
            continue;
        }
        const bool has_i = p.half_delta > 0.0;
        const double hx = (box[1] - box[0]) / (double)(p.nx - 1);
        const double hy = (box[3] - box[2]) / (double)(p.ny - 1);
        const double cx = box[0] + 0.5 * (box[1] - box[0]);
        const double cy = box[2] + 0.5 * (box[3] - box[2]);
        const int ns = (int)S;
        // shifted, centred FP32 coefficients of every state
        for (int s = tid; s < ns; s += NT) {
            const Coef c = stage.c[s];
            CoefF f;
            f.a = (float)(c.a - ref[0]);
            f.al = has_i ? (float)(c.al - ref[1]) : -kInfF;
            f.ux = (float)(c.ux - cx);
            f.uy = (float)(c.uy - cy);
            f.nk = (float)c.nk;
            sF[s] = f;
        }
        for (int t = tid; t < 4 * NY; t += NT) {
            const int fc = t / NY, ty = t % NY;
            float v = 0.f;
            if (ty < p.ny) {
                const double u = node_pos(box[2], ty, hy);
                const double wy = hy * ((ty == 0 || ty == p.ny - 1) ? 0.5 : 1.0);
                v = (float)(fc == 0 ? wy
                          : fc == 1 ? (u < 0.0 ? wy * u : 0.0)
                          : fc == 2 ? (u < 0.0 ? 0.0 : wy * u)
                                    : wy * u * u);
            }
            yfac[fc][ty] = v;
        }

        // centred x coordinates of this lane's nodes (clamped for the ragged
        // tail), for the tiles that form the x terms in registers
        float uxc[TXW];
#pragma unroll
        for (int i = 0; i < TXW; ++i) {
            const int x = 16 * (w + NW * i) + xr;
            uxc[i] = ATAB ? 0.f : (float)(node_pos(box[0], x < p.nx ? x : p.nx - 1, hx) - cx);
        }
        float tn[TXW][TY], tX[TXW][TY], in_[TXW][TY], iX[TXW][TY];
#pragma unroll
        for (int i = 0; i < TXW; ++i)
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                tn[i][j] = kInfF; tX[i][j] = -kInfF; in_[i][j] = kInfF; iX[i][j] = -kInfF;
            }

        for (int c0 = 0; c0 < ns; c0 += kTab) {
            const int cn = (ns - c0) < kTab ? (ns - c0) : kTab;
            __syncthreads();
            {
                // by columns: thread t fills node t % NY of states t / NY,
                // t / NY + NT / NY, ... (one node coordinate per thread, no
                // index division per entry); the same values as per entry
                static_assert(NY <= NT, "one column per thread at least");
                constexpr int kPass = NT / NY;
                const int j = tid % NY, sj = tid / NY;
                if (sj < kPass) {
                    const float uyc = (float)(node_pos(box[2], j < p.ny ? j : p.ny - 1, hy) - cy);
                    const float uxc = ATAB ? (float)(node_pos(box[0], j < p.nx ? j : p.nx - 1, hx) - cx) : 0.f;
                    for (int s = sj; s < cn; s += kPass) {
                        const CoefF c = sF[c0 + s];
                        const float d = uyc - c.uy;
                        stage.t.b[s][j] = (c.nk * d) * d;
                        if constexpr (ATAB) {
                            const float dx = uxc - c.ux, t = c.nk * dx;
                            float2_t v;
                            v[0] = fmaf(t, dx, c.a);
                            v[1] = fmaf(t, dx, c.al);
                            stage.t.ai[s][j] = v;
                        }
                    }
                }
            }
            __syncthreads();
            int s = 0;
            for (; s + 1 < cn; s += 2) {
                float A1[TXW], I1[TXW], A2[TXW], I2[TXW];
#pragma unroll
                for (int i = 0; i < TXW; ++i) {
                    if constexpr (ATAB) {
                        const float2_t v1 = stage.t.ai[s][16 * (w + NW * i) + xr];
                        const float2_t v2 = stage.t.ai[s + 1][16 * (w + NW * i) + xr];
                        A1[i] = v1[0]; I1[i] = v1[1];
                        A2[i] = v2[0]; I2[i] = v2[1];
                    } else {
                        const CoefF c1 = sF[c0 + s], c2 = sF[c0 + s + 1];
                        const float d1 = uxc[i] - c1.ux, t1 = c1.nk * d1;
                        const float d2 = uxc[i] - c2.ux, t2 = c2.nk * d2;
                        A1[i] = fmaf(t1, d1, c1.a); I1[i] = fmaf(t1, d1, c1.al);
                        A2[i] = fmaf(t2, d2, c2.a); I2[i] = fmaf(t2, d2, c2.al);
                    }
                }
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const float4_t b1 = *reinterpret_cast<const float4_t*>(&stage.t.b[s][16 * k + 4 * g]);
                    const float4_t b2 = *reinterpret_cast<const float4_t*>(&stage.t.b[s + 1][16 * k + 4 * g]);
#pragma unroll
                    for (int i = 0; i < TXW; ++i)
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const int j = 4 * k + m;
                            const float q1 = A1[i] + b1[m], q2 = A2[i] + b2[m];
                            const float r1 = I1[i] + b1[m], r2 = I2[i] + b2[m];
                            tn[i][j] = fminf(tn[i][j], fminf(q1, q2));
                            tX[i][j] = fmaxf(tX[i][j], fmaxf(q1, q2));
                            in_[i][j] = fminf(in_[i][j], fminf(r1, r2));
                            iX[i][j] = fmaxf(iX[i][j], fmaxf(r1, r2));
                        }
                }
            }
            if (s < cn) {
#pragma unroll
                for (int i = 0; i < TXW; ++i) {
                    float A1, I1;
                    if constexpr (ATAB) {
                        const float2_t v1 = stage.t.ai[s][16 * (w + NW * i) + xr];
                        A1 = v1[0]; I1 = v1[1];
                    } else {
                        const CoefF c1 = sF[c0 + s];
                        const float d1 = uxc[i] - c1.ux, t1 = c1.nk * d1;
                        A1 = fmaf(t1, d1, c1.a); I1 = fmaf(t1, d1, c1.al);
                    }
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        const float4_t b1 = *reinterpret_cast<const float4_t*>(&stage.t.b[s][16 * k + 4 * g]);
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const int j = 4 * k + m;
                            tn[i][j] = fminf(tn[i][j], A1 + b1[m]);
                            tX[i][j] = fmaxf(tX[i][j], A1 + b1[m]);
                            in_[i][j] = fminf(in_[i][j], I1 + b1[m]);
                            iX[i][j] = fmaxf(iX[i][j], I1 + b1[m]);
                        }
                    }
                }
            }
        }

        // The contraction starts from copies of the box, its spacing and the
        // lane indices passed through an empty asm statement: otherwise the
        // compiler forms the element-invariant node coordinates, weights and
        // factors before the hot loop and keeps them live across it, which
        // leaves one wave per SIMD.
        double ebox[4] = {box[0], box[1], box[2], box[3]};
        double ehx = hx, ehy = hy;
        int ew = w, eg = g, exr = xr;
        asm volatile("" : "+v"(ebox[0]), "+v"(ebox[1]), "+v"(ebox[2]), "+v"(ebox[3]), "+v"(ehx),
                     "+v"(ehy), "+v"(ew), "+v"(eg), "+v"(exr));

        // MFMA paths: each envelope is exponentiated relative to its largest
        // value over the wave's nodes, rounded up to a power of two:
        // f = 2^(q log2 e - n) with n = ceil(max q log2 e), so the wave's
        // largest value lies in (1/2, 1] however far the stencil's log-peaks
        // spread.  The FP16/BF16 splits of the y stage resolve values down to
        // ~2^-38 of the largest; without the shift, states at theta ~ 1
        // beside a nearly cold one (~1e-12 below the cold log-peak) would be
        // lost.  The wave's FP64 partials are scaled back by 2^n exactly
        // before the workgroup sum.  An envelope that is -inf everywhere (no
        // internal energy term) keeps n = 0 and exponentiates to 0; n is
        // clamped at -2000, where both sides of the scaling underflow to 0.
        // The FP32 VALU path needs no shift: its exp reaches e^-87.
        float nsh[4] = {0.f, 0.f, 0.f, 0.f};   // n, uniform over the wave
        if (CT != KBL_PREC_MIXED_FP32) {
            float em[4] = {-kInfF, -kInfF, -kInfF, -kInfF};
#pragma unroll
            for (int i = 0; i < TXW; ++i)
#pragma unroll
                for (int j = 0; j < TY; ++j) {
                    em[0] = fmaxf(em[0], tn[i][j]);
                    em[1] = fmaxf(em[1], tX[i][j]);
                    em[2] = fmaxf(em[2], in_[i][j]);
                    em[3] = fmaxf(em[3], iX[i][j]);
                }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float m = wave_max_f32(em[k]);
                nsh[k] = m > -kInfF ? fmaxf(ceilf(m * kLog2e), -2000.f) : 0.f;
            }
        }

        double part[kNP];
#pragma unroll
        for (int i = 0; i < kNP; ++i) part[i] = 0.0;

        if (CT == KBL_PREC_MIXED_FP32) {
#pragma unroll
            for (int i = 0; i < TXW; ++i) {
                // y stage on the VALU (FP32), then the x stage in FP64
                float H[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, HI[2] = {0, 0};
                float4_t Y[4];
#pragma unroll
                for (int j = 0; j < TY; ++j) {
                    if (j % 4 == 0) {
#pragma unroll
                        for (int fc = 0; fc < 4; ++fc)
                            Y[fc] = *reinterpret_cast<const float4_t*>(&yfac[fc][16 * (j / 4) + 4 * eg]);
                    }
                    const float y0 = Y[0][j % 4], y1 = Y[1][j % 4], y2 = Y[2][j % 4], y3 = Y[3][j % 4];
                    const float fa = __builtin_amdgcn_exp2f(tn[i][j] * kLog2e);
                    const float fb = __builtin_amdgcn_exp2f(tX[i][j] * kLog2e);
                    H[0][0] = fmaf(fa, y0, H[0][0]); H[0][1] = fmaf(fa, y1, H[0][1]);
                    H[0][2] = fmaf(fa, y2, H[0][2]); H[0][3] = fmaf(fa, y3, H[0][3]);
                    H[1][0] = fmaf(fb, y0, H[1][0]); H[1][1] = fmaf(fb, y1, H[1][1]);
                    H[1][2] = fmaf(fb, y2, H[1][2]); H[1][3] = fmaf(fb, y3, H[1][3]);
                    HI[0] = fmaf(__builtin_amdgcn_exp2f(in_[i][j] * kLog2e), y0, HI[0]);
                    HI[1] = fmaf(__builtin_amdgcn_exp2f(iX[i][j] * kLog2e), y0, HI[1]);
                    __builtin_amdgcn_sched_barrier(0);
                }
                const XF X = x_factors(p, ebox, ehx, 16 * (ew + NW * i) + exr);
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    part[6 * v + 0] += X.w * H[v][0];
                    part[6 * v + 1] += X.m * H[v][0];
                    part[6 * v + 2] += X.p * H[v][0];
                    part[6 * v + 3] += X.w * H[v][1];
                    part[6 * v + 4] += X.w * H[v][2];
                    part[6 * v + 5] += 0.5 * (X.q * H[v][0] + X.w * H[v][3]);
                }
                part[12] += X.w * HI[0];
                part[13] += X.w * HI[1];
            }
        } else {
            // B operand: factor n = l%16 (0..3 used) at this lane's y nodes,
            // scaled by a power of two into [1, 2)
            const double umax = fmax(fabs(ebox[2]), fabs(ebox[3]));
            const double bound = exr == 0 ? ehy : (exr == 3 ? ehy * umax * umax : ehy * umax);
            const double yscale = (exr < 4 && bound > 0.0) ? ldexp(1.0, -ilogb(bound)) : 1.0;
            const double unscale =
                (CT == KBL_PREC_MIXED_FP16 ? 1.0 / ((double)kF16Scale * kF16Scale) : 1.0) / yscale;
            // this lane's factor (zero in the unused columns), times the
            // column's power of two
            const float ysf = exr < 4 ? (float)yscale : 0.f;
            float yb[TY];
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const float4_t y4 = *reinterpret_cast<const float4_t*>(&yfac[exr & 3][16 * k + 4 * eg]);
#pragma unroll
                for (int i = 0; i < 4; ++i) yb[4 * k + i] = y4[i] * ysf;
            }
            YSplit<KS, CT> ysp;
            split_y<KS, CT>(yb, ysp);
            // x stage without branches on the lane's column: every lane sums
            // X.{w, m, p, q} times its C entries of each T envelope and X.w
            // times those of each I envelope; which partials these are
            // depends only on the column (exr) and is settled after the
            // tiles.  The sums are the products of the per-entry form in
            // the same order, and the column's unscale (a power of two) is
            // exact at either place.
            const float fsh = CT == KBL_PREC_MIXED_FP16 ? kF16Log2Scale : 0.f;
            double sT[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}}, sI[2] = {0.0, 0.0};
#pragma unroll
            for (int i = 0; i < TXW; ++i) {
                // x rows of the C result held by this lane
                XF X[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) X[r] = x_factors(p, ebox, ehx, 16 * (ew + NW * i) + 4 * eg + r);
#pragma unroll
                for (int env = 0; env < 4; ++env) {
                    float f[TY];
                    const float sh = fsh - nsh[env];
#pragma unroll
                    for (int j = 0; j < TY; ++j) {
                        const float q = env == 0 ? tn[i][j] : env == 1 ? tX[i][j] : env == 2 ? in_[i][j] : iX[i][j];
                        f[j] = __builtin_amdgcn_exp2f(fmaf(q, kLog2e, sh));
                    }
                    const float4_t c = mfma_ystage<KS, CT>(f, ysp);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double h = c[r];
                        if (env < 2) {
                            sT[env][0] += X[r].w * h; sT[env][1] += X[r].m * h;
                            sT[env][2] += X[r].p * h; sT[env][3] += X[r].q * h;
                        } else {
                            sI[env - 2] += X[r].w * h;
                        }
                    }
                }
            }
            const double u0 = exr == 0 ? unscale : 0.0, u1 = exr == 1 ? unscale : 0.0;
            const double u2 = exr == 2 ? unscale : 0.0, u3 = exr == 3 ? unscale : 0.0;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                part[6 * v + 0] = u0 * sT[v][0];
                part[6 * v + 1] = u0 * sT[v][1];
                part[6 * v + 2] = u0 * sT[v][2];
                part[6 * v + 3] = u1 * sT[v][0];
                part[6 * v + 4] = u2 * sT[v][0];
                part[6 * v + 5] = 0.5 * (u0 * sT[v][3] + u3 * sT[v][0]);
            }
            part[12] = u0 * sI[0];
            part[13] = u0 * sI[1];
        }
        if (CT != KBL_PREC_MIXED_FP32) {
            // back to the element's log-peak scale (exact powers of two)
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                part[i] = ldexp(part[i], (int)nsh[0]);
                part[6 + i] = ldexp(part[6 + i], (int)nsh[1]);
            }
            part[12] = ldexp(part[12], (int)nsh[2]);
            part[13] = ldexp(part[13], (int)nsh[3]);
        }
        block_sum_t<NT, kNP>(part, red);
        if (tid == 0) {
            const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;
            const double eT = exp(ref[0]);
            const double eI = has_i ? exp(ref[1]) : 0.0;
            double sums[8];
            sums[0] = rm * eT * part[0];                         // rho_min
            sums[1] = rp * eT * part[6];                         // rho_max
            sums[2] = rm * (eT * part[5] + eI * part[12]);       // E_min
            sums[3] = rp * (eT * part[11] + eI * part[13]);      // E_max
            sums[4] = eT * (rp * part[7] + rm * part[2]);        // m_x,min
            sums[5] = eT * (rm * part[1] + rp * part[8]);        // m_x,max
            sums[6] = eT * (rp * part[9] + rm * part[4]);        // m_y,min
            sums[7] = eT * (rm * part[3] + rp * part[10]);       // m_y,max
            store_bounds<2>(p, e, sums, flags);
        }
    }
}

template <int TXW, int KS, int NW, int CT>
hipError_t launch_mixed(const BoundsArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL((bounds_mixed_2d<TXW, KS, NW, CT>), dim3(bounds_grid(a)), dim3(NW * 64), 0,
                       stream, a);
    return hipGetLastError();
}

// Tile configurations (TXW, KS, NW): x tiles of 16 nodes per wave, y steps
// of 16, waves per workgroup.  Covers nx <= 16 TXW NW, ny <= 16 KS.
struct MixedTile {
    int txw, ks, nw;
    hipError_t (*fn[3])(const BoundsArgs&, hipStream_t);
};
#define KBL_MTILE(T, K, W) \
    {T, K, W, {launch_mixed<T, K, W, KBL_PREC_MIXED_BF16>, launch_mixed<T, K, W, KBL_PREC_MIXED_FP16>, \
               launch_mixed<T, K, W, KBL_PREC_MIXED_FP32>}}
constexpr MixedTile kMixedTiles[] = {
    KBL_MTILE(1, 1, 1),   // 0: n <= 16
    KBL_MTILE(2, 2, 1),   // 1: n <= 32
    KBL_MTILE(1, 2, 2),   // 2: n <= 32, two waves
    KBL_MTILE(3, 3, 1),   // 3: n <= 48, one wave
    KBL_MTILE(1, 3, 3),   // 4: n <= 48, three waves
    KBL_MTILE(2, 4, 2),   // 5: n <= 64, two waves
    KBL_MTILE(1, 4, 4),   // 6: n <= 64, four waves
};
#undef KBL_MTILE
constexpr int kNumMixedTiles = sizeof(kMixedTiles) / sizeof(kMixedTiles[0]);

bool mixed_tile_fits(int t, int nx, int ny) {
    if (t < 0 || t >= kNumMixedTiles) return false;
    const MixedTile& m = kMixedTiles[t];
    return nx <= 16 * m.txw * m.nw && ny <= 16 * m.ks;
}

// Defaults from a measured sweep (48x48: three single-tile waves for every
// contraction; 64x64: the FP16 MFMA contraction two waves of two tiles, the
// FP32 VALU and BF16 MFMA contractions four single-tile waves).
int default_mixed_tile(int nx, int ny, int precision) {
    const int n = nx > ny ? nx : ny;
    if (n <= 16) return 0;
    if (n <= 32) return 1;
    if (n <= 48) return 4;
    return precision == KBL_PREC_MIXED_FP16 ? 5 : 6;
}

}  // namespace

int mixed_tile_count() { return kNumMixedTiles; }
bool mixed_tile_fits_2d(int tile, int nx, int ny) { return mixed_tile_fits(tile, nx, ny); }
int mixed_default_tile_2d(int nx, int ny, int precision) { return default_mixed_tile(nx, ny, precision); }

hipError_t launch_bounds_mixed(const BoundsArgs& a, int precision, hipStream_t stream, int tile) {
    if (a.n_elem == 0) return hipSuccess;
    if (tile < 0 || !mixed_tile_fits(tile, a.nx, a.ny)) tile = default_mixed_tile(a.nx, a.ny, precision);
    if (!mixed_tile_fits(tile, a.nx, a.ny)) return hipErrorInvalidValue;
    const int slot = precision == KBL_PREC_MIXED_BF16 ? 0 : precision == KBL_PREC_MIXED_FP16 ? 1
                   : precision == KBL_PREC_MIXED_FP32 ? 2 : -1;
    if (slot < 0) return hipErrorInvalidValue;
    return kMixedTiles[tile].fn[slot](a, stream);
}

}  // namespace kbl

// Mixed-precision kinetic bounds (steps 1-3 of the overview in Sec. 3.9), gfx950.
//
// Same method as the FP64 kernels; what changes is the arithmetic of the
// hot loop and of the moment contraction:
//  - FP64: stencil prologue (admissibility, velocity box of eq. truncdomain,
//    log-Maxwellian coefficients), the per-element log-peak references, the
//    relaxation factors of eq. relaxed, the final scaling and the density
//    floor of Sec. 3.8.
//  - FP32: the envelopes.  Coefficients are shifted by the element's log-peak
//    reference (so exp lands in (0, 1]) and velocities are centred on the
//    box, then q = A[x] + B[y] and the four running extrema are kept in FP32;
//    two states are folded per step with three-input min/max.
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
// Workgroup = NW waves; wave w owns x nodes 16w..16w+15.  Lane l of a wave
// owns x node 16w + l%16 and the y nodes 16k + 4(l/16) + i (i < 4, k < KS):
// exactly the A-operand layout of the 16x16x16 MFMA with M = x, K = y, so the
// envelope values feed the matrix core straight from registers.  The B
// operand (lane l: factor l%16 at the same y nodes) is built per element in
// registers; the C result (lane l: factor l%16 at x rows 16w + 4(l/16) + i)
// is contracted with X in FP64.
#include "bounds_common.h"

namespace kbl {
namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kTab = 64;            // states per FP32 coefficient / B-table chunk
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kF16Scale = 16384.0f;            // 2^14, exact

struct CoefF {
    float a;    // a - ref_T
    float al;   // a + l - ref_I   (-inf without internal degrees of freedom)
    float ux;   // U_x - box centre
    float uy;   // U_y - box centre
    float nk;   // -1 / (2 theta)
};

__device__ __forceinline__ short f2bf(float x) {   // round to nearest even
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf2f(short b) {
    return __uint_as_float(((uint32_t)(uint16_t)b) << 16);
}

// y-stage contraction of one envelope on MFMA: returns C (lane l: factor
// l%16 at x rows 4(l/16) + i of the wave's 16 rows).
template <int KS, int CT>
__device__ __forceinline__ float4_t mfma_ystage(const float* f, const float* yb) {
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        if (CT == KBL_PREC_MIXED_FP16) {
            // both operands are scaled by 2^14 (envelopes <= 1, factors < 2)
            // so that the low halves stay clear of FP16 subnormals
            half4_t ah, al, bh, bl;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float av = f[4 * k + i] * kF16Scale, bv = yb[4 * k + i] * kF16Scale;
                ah[i] = (_Float16)av;
                al[i] = (_Float16)(av - (float)ah[i]);
                bh[i] = (_Float16)bv;
                bl[i] = (_Float16)(bv - (float)bh[i]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, bl, acc, 0, 0, 0);
        } else {
            bf16x4_t a1, a2, a3, b1, b2, b3;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float av = f[4 * k + i], bv = yb[4 * k + i];
                a1[i] = f2bf(av); av -= bf2f(a1[i]);
                a2[i] = f2bf(av); av -= bf2f(a2[i]);
                a3[i] = f2bf(av);
                b1[i] = f2bf(bv); bv -= bf2f(b1[i]);
                b2[i] = f2bf(bv); bv -= bf2f(b2[i]);
                b3[i] = f2bf(bv);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b2, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, b1, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b3, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, b2, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, b1, acc, 0, 0, 0);
        }
    }
    return acc;
}

// Partial sums per envelope, in this order: T_min: S0, SXm, SXp, SYm, SYp, S2;
// T_max: the same six; I_min: S0; I_max: S0.
constexpr int kNP = 14;

template <int NW, int KS, int CT>
__global__ __launch_bounds__(NW * 64) void bounds_mixed_2d(BoundsArgs p) {
    constexpr int NT = NW * 64;
    constexpr int NY = 16 * KS;     // y nodes covered
    constexpr int TY = 4 * KS;      // y nodes per lane
    __shared__ Coef sC[kMaxStates];
    __shared__ CoefF sF[kTab];
    __shared__ __align__(16) float sB[kTab][NY];
    __shared__ Red red;

    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63, xr = l & 15, g = l >> 4;
    const int tx = 16 * w + xr;

    for (int64_t e = blockIdx.x; e < p.n_elem; e += gridDim.x) {
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<2>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        double box[4], ref[2];
        const uint32_t flags = stencil_prologue<2, NT>(p, row0, S, red, sC, box, ref);
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<2>(p, e, flags);
            continue;
        }
        const bool has_i = p.half_delta > 0.0;
        const double hx = (box[1] - box[0]) / (double)(p.nx - 1);
        const double hy = (box[3] - box[2]) / (double)(p.ny - 1);
        const double cx = box[0] + 0.5 * (box[1] - box[0]);
        const double cy = box[2] + 0.5 * (box[3] - box[2]);

        // centred node coordinates of this lane (clamped for the ragged tail)
        const float uxc = (float)((box[0] + (tx < p.nx ? tx : p.nx - 1) * hx) - cx);
        float tn[TY], tX[TY], in_[TY], iX[TY];
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            tn[j] = kInfF; tX[j] = -kInfF; in_[j] = kInfF; iX[j] = -kInfF;
        }

        for (int64_t c0 = 0; c0 < S; c0 += kTab) {
            const int cn = (int)((S - c0) < kTab ? (S - c0) : kTab);
            __syncthreads();
            for (int s = tid; s < cn; s += NT) {
                const int64_t gs = c0 + s;
                const Coef c = gs < kMaxStates ? sC[gs]
                                               : make_coef<2>(p, load_prim<2>(p, state_node(p, row0, gs)));
                CoefF f;
                f.a = (float)(c.a - ref[0]);
                f.al = has_i ? (float)(c.al - ref[1]) : -kInfF;
                f.ux = (float)(c.ux - cx);
                f.uy = (float)(c.uy - cy);
                f.nk = (float)c.nk;
                sF[s] = f;
            }
            __syncthreads();
            for (int idx = tid; idx < cn * NY; idx += NT) {
                const int s = idx / NY, j = idx - s * NY;
                const float uyc = (float)((box[2] + (j < p.ny ? j : p.ny - 1) * hy) - cy);
                const float d = uyc - sF[s].uy;
                sB[s][j] = (sF[s].nk * d) * d;
            }
            __syncthreads();
            int s = 0;
            for (; s + 1 < cn; s += 2) {
                const CoefF c1 = sF[s], c2 = sF[s + 1];
                const float d1 = uxc - c1.ux, t1 = c1.nk * d1;
                const float d2 = uxc - c2.ux, t2 = c2.nk * d2;
                const float A1 = fmaf(t1, d1, c1.a), I1 = fmaf(t1, d1, c1.al);
                const float A2 = fmaf(t2, d2, c2.a), I2 = fmaf(t2, d2, c2.al);
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const float4_t b1 = *reinterpret_cast<const float4_t*>(&sB[s][16 * k + 4 * g]);
                    const float4_t b2 = *reinterpret_cast<const float4_t*>(&sB[s + 1][16 * k + 4 * g]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int j = 4 * k + i;
                        const float q1 = A1 + b1[i], q2 = A2 + b2[i];
                        const float r1 = I1 + b1[i], r2 = I2 + b2[i];
                        tn[j] = fminf(tn[j], fminf(q1, q2));
                        tX[j] = fmaxf(tX[j], fmaxf(q1, q2));
                        in_[j] = fminf(in_[j], fminf(r1, r2));
                        iX[j] = fmaxf(iX[j], fmaxf(r1, r2));
                    }
                }
            }
            if (s < cn) {
                const CoefF c1 = sF[s];
                const float d1 = uxc - c1.ux, t1 = c1.nk * d1;
                const float A1 = fmaf(t1, d1, c1.a), I1 = fmaf(t1, d1, c1.al);
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const float4_t b1 = *reinterpret_cast<const float4_t*>(&sB[s][16 * k + 4 * g]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int j = 4 * k + i;
                        const float q1 = A1 + b1[i], r1 = I1 + b1[i];
                        tn[j] = fminf(tn[j], q1);
                        tX[j] = fmaxf(tX[j], q1);
                        in_[j] = fminf(in_[j], r1);
                        iX[j] = fmaxf(iX[j], r1);
                    }
                }
            }
        }

        // envelope values exp(q - ref) in (0, 1]
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            tn[j] = __builtin_amdgcn_exp2f(tn[j] * kLog2e);
            tX[j] = __builtin_amdgcn_exp2f(tX[j] * kLog2e);
            in_[j] = __builtin_amdgcn_exp2f(in_[j] * kLog2e);
            iX[j] = __builtin_amdgcn_exp2f(iX[j] * kLog2e);
        }

        double part[kNP];
#pragma unroll
        for (int i = 0; i < kNP; ++i) part[i] = 0.0;

        if (CT == KBL_PREC_MIXED_FP32) {
            // y stage on the VALU (FP32) for this lane's single x node
            float H[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, HI[2] = {0, 0};
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int ty = 16 * (j / 4) + 4 * g + (j % 4);
                if (ty >= p.ny) continue;
                const double uyd = box[2] + ty * hy;
                const double wy = hy * ((ty == 0 || ty == p.ny - 1) ? 0.5 : 1.0);
                const float y0 = (float)wy;
                const float y1 = (float)(uyd < 0.0 ? wy * uyd : 0.0);
                const float y2 = (float)(uyd < 0.0 ? 0.0 : wy * uyd);
                const float y3 = (float)(wy * uyd * uyd);
                H[0][0] = fmaf(tn[j], y0, H[0][0]); H[0][1] = fmaf(tn[j], y1, H[0][1]);
                H[0][2] = fmaf(tn[j], y2, H[0][2]); H[0][3] = fmaf(tn[j], y3, H[0][3]);
                H[1][0] = fmaf(tX[j], y0, H[1][0]); H[1][1] = fmaf(tX[j], y1, H[1][1]);
                H[1][2] = fmaf(tX[j], y2, H[1][2]); H[1][3] = fmaf(tX[j], y3, H[1][3]);
                HI[0] = fmaf(in_[j], y0, HI[0]);
                HI[1] = fmaf(iX[j], y0, HI[1]);
            }
            if (tx < p.nx) {
                const double uxd = box[0] + tx * hx;
                const double wx = hx * ((tx == 0 || tx == p.nx - 1) ? 0.5 : 1.0);
                const double x1 = uxd < 0.0 ? wx * uxd : 0.0, x2 = uxd < 0.0 ? 0.0 : wx * uxd;
                const double x3 = wx * uxd * uxd;
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    part[6 * v + 0] = wx * H[v][0];
                    part[6 * v + 1] = x1 * H[v][0];
                    part[6 * v + 2] = x2 * H[v][0];
                    part[6 * v + 3] = wx * H[v][1];
                    part[6 * v + 4] = wx * H[v][2];
                    part[6 * v + 5] = 0.5 * (x3 * H[v][0] + wx * H[v][3]);
                }
                part[12] = wx * HI[0];
                part[13] = wx * HI[1];
            }
        } else {
            // B operand: factor n = l%16 (0..3 used) at this lane's y nodes,
            // scaled by a power of two so that it stays well inside the
            // FP16/BF16 range
            const double umax = fmax(fabs(box[2]), fabs(box[3]));
            const double bound = xr == 0 ? hy : (xr == 3 ? hy * umax * umax : hy * umax);
            const double yscale = (xr < 4 && bound > 0.0) ? ldexp(1.0, -ilogb(bound)) : 1.0;
            float yb[TY];
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int ty = 16 * (j / 4) + 4 * g + (j % 4);
                double v = 0.0;
                if (ty < p.ny && xr < 4) {
                    const double uyd = box[2] + ty * hy;
                    const double wy = hy * ((ty == 0 || ty == p.ny - 1) ? 0.5 : 1.0);
                    v = xr == 0 ? wy
                      : xr == 1 ? (uyd < 0.0 ? wy * uyd : 0.0)
                      : xr == 2 ? (uyd < 0.0 ? 0.0 : wy * uyd)
                                : wy * uyd * uyd;
                }
                yb[j] = (float)(v * yscale);
            }
            const float4_t c_tn = mfma_ystage<KS, CT>(tn, yb);
            const float4_t c_tx = mfma_ystage<KS, CT>(tX, yb);
            const float4_t c_in = mfma_ystage<KS, CT>(in_, yb);
            const float4_t c_ix = mfma_ystage<KS, CT>(iX, yb);
            const double unscale =
                (CT == KBL_PREC_MIXED_FP16 ? 1.0 / ((double)kF16Scale * kF16Scale) : 1.0) / yscale;
            // x stage: lane holds factor xr at x rows 16w + 4g + i
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = 16 * w + 4 * g + i;
                if (x >= p.nx || xr >= 4) continue;
                const double uxd = box[0] + x * hx;
                const double wx = hx * ((x == 0 || x == p.nx - 1) ? 0.5 : 1.0);
                const double x1 = uxd < 0.0 ? wx * uxd : 0.0, x2 = uxd < 0.0 ? 0.0 : wx * uxd;
                const double x3 = wx * uxd * uxd;
                const double htn = c_tn[i] * unscale, htx = c_tx[i] * unscale;
                if (xr == 0) {
                    part[0] += wx * htn; part[1] += x1 * htn; part[2] += x2 * htn; part[5] += 0.5 * x3 * htn;
                    part[6] += wx * htx; part[7] += x1 * htx; part[8] += x2 * htx; part[11] += 0.5 * x3 * htx;
                    part[12] += wx * (c_in[i] * unscale);
                    part[13] += wx * (c_ix[i] * unscale);
                } else if (xr == 1) {
                    part[3] += wx * htn; part[9] += wx * htx;
                } else if (xr == 2) {
                    part[4] += wx * htn; part[10] += wx * htx;
                } else {
                    part[5] += 0.5 * wx * htn; part[11] += 0.5 * wx * htx;
                }
            }
        }
        block_sum<NT, kNP>(part, red);
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

template <int NW, int KS, int CT>
hipError_t launch_mixed(const BoundsArgs& a, hipStream_t stream) {
    const int64_t grid = a.n_elem < (int64_t)INT32_MAX ? a.n_elem : (int64_t)INT32_MAX;
    hipLaunchKernelGGL((bounds_mixed_2d<NW, KS, CT>), dim3((unsigned)grid), dim3(NW * 64), 0,
                       stream, a);
    return hipGetLastError();
}

template <int CT>
hipError_t launch_ct(const BoundsArgs& a, hipStream_t stream) {
    const int mx = (a.nx + 15) / 16, my = (a.ny + 15) / 16;
    const int m = mx > my ? mx : my;
    if (m <= 1) return launch_mixed<1, 1, CT>(a, stream);
    if (m <= 2) return launch_mixed<2, 2, CT>(a, stream);
    if (m <= 3) return launch_mixed<3, 3, CT>(a, stream);
    if (m <= 4) return launch_mixed<4, 4, CT>(a, stream);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_bounds_mixed(const BoundsArgs& a, int precision, hipStream_t stream) {
    if (a.n_elem == 0) return hipSuccess;
    switch (precision) {
        case KBL_PREC_MIXED_FP32: return launch_ct<KBL_PREC_MIXED_FP32>(a, stream);
        case KBL_PREC_MIXED_FP16: return launch_ct<KBL_PREC_MIXED_FP16>(a, stream);
        case KBL_PREC_MIXED_BF16: return launch_ct<KBL_PREC_MIXED_BF16>(a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace kbl

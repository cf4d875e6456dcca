// FP64 kinetic bounds (steps 1-3 of the overview in Sec. 3.9), gfx950.
//
// One workgroup of 256 threads (four wave64) owns one element at a time.
//  1. The stencil states (every node of every element of the CSR row) are
//     read once to check admissibility (Assumption (i) of Sec. 4) and, in
//     STENCIL mode, to reduce the velocity box of eq. truncdomain.
//  2. The states are then streamed through LDS in chunks.  For each state i
//     the log-Maxwellian  q_i(u) = ln rho_i - (d/2) ln(2 pi theta_i)
//     - |u - U_i|^2 / (2 theta_i)  is separable on the Cartesian velocity
//     grid: q_i = A_i[jx] + B_i[jy].  The chunk's A, A + ln(theta delta/2)
//     and B tables are built once in LDS, so the hot loop costs two adds and
//     four min/max per (state, velocity node) pair.  Because exp is monotone,
//     min_i g_i = exp(min_i q_i) (eq. fminmax), and likewise for the internal
//     part g_I = (theta delta / 2) g (Sec. 3.6): four running extrema per node
//     stay in registers and only four exp per node are taken at the end.
//  3. Relaxation (eq. relaxed), trapezoid weights (Sec. 3.7) and the moment
//     contraction (eq. rhobounds, Ebounds, mmbounds, mpbounds) are done per
//     node, then reduced across the workgroup in a fixed order (bitwise
//     deterministic), floored (Sec. 3.8) and stored.
// Each thread owns a TX x TY tile of velocity nodes, strided by 16 so that
// the LDS table reads of a wave are contiguous or broadcast.
// Inputs are validated before the hot loop, which therefore never sees a NaN
// (only finite values and -inf when delta = 0).
#include <math.h>

#include "kbl_internal.h"

namespace kbl {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kChunk = 16;          // stencil states per LDS chunk
constexpr double kInf = __builtin_inf();

struct Prim {
    double rho, ux, uy, th;
    bool ok;
};

// This translation unit is compiled with -fno-honor-nans so that the running
// min/max of the hot loop need no NaN canonicalisation; finiteness is
// therefore tested on the bit pattern, which that flag cannot fold away.
__device__ __forceinline__ bool finite_bits(double x) {
    return (__double_as_longlong(x) & 0x7ff0000000000000LL) != 0x7ff0000000000000LL;
}

template <int D>
__device__ __forceinline__ Prim load_prim(const BoundsArgs& p, int64_t node) {
    Prim s;
    const double rho = p.states[node];
    const double mx = p.states[p.n_nodes + node];
    const double my = (D == 2) ? p.states[2 * p.n_nodes + node] : 0.0;
    const double E = p.states[(D + 1) * p.n_nodes + node];
    const double mm = (D == 2) ? mx * mx + my * my : mx * mx;
    const double P = p.gm1 * (E - 0.5 * mm / rho);
    s.rho = rho;
    s.ux = mx / rho;
    s.uy = (D == 2) ? my / rho : 0.0;
    s.th = P / rho;
    s.ok = finite_bits(rho) && finite_bits(mx) && finite_bits(my) && finite_bits(E) &&
           finite_bits(P) && finite_bits(s.th) && rho > 0.0 && P > 0.0;
    return s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Shared scratch for the per-element prologue and epilogue.
struct Red {
    double v[kWaves][8];
    uint32_t flags;
};

// Prologue: admissibility + velocity box.  Returns status bits (uniform).
template <int D>
__device__ uint32_t stencil_prologue(const BoundsArgs& p, int64_t e, int64_t row0, int64_t S,
                                     Red& red, double box[4]) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    uint32_t bad = 0;
    double lx = kInf, hx = -kInf, ly = kInf, hy = -kInf;
    for (int64_t s = tid; s < S; s += kThreads) {
        const int64_t r = row0 + s / p.n_s;
        const int32_t col = p.cols[r];
        if (col < 0 || col >= p.n_elem) { bad |= KBL_ST_BAD_STENCIL; continue; }
        const Prim st = load_prim<D>(p, (int64_t)col * p.n_s + s % p.n_s);
        if (!st.ok) { bad |= KBL_ST_INADMISSIBLE; continue; }
        if (p.grid_mode == KBL_GRID_STENCIL) {
            const double sd = sqrt(st.th);
            lx = fmin(lx, st.ux - p.k * sd);
            hx = fmax(hx, st.ux + p.k * sd);
            if (D == 2) {
                ly = fmin(ly, st.uy - p.k * sd);
                hy = fmax(hy, st.uy + p.k * sd);
            }
        }
    }
    if (tid == 0) red.flags = 0;
    lx = wave_min(lx); hx = wave_max(hx); ly = wave_min(ly); hy = wave_max(hy);
    __syncthreads();
    if (bad) atomicOr(&red.flags, bad);
    if (lane == 0) {
        red.v[wid][0] = lx; red.v[wid][1] = hx; red.v[wid][2] = ly; red.v[wid][3] = hy;
    }
    __syncthreads();
    if (p.grid_mode == KBL_GRID_STENCIL) {
        box[0] = red.v[0][0]; box[1] = red.v[0][1]; box[2] = red.v[0][2]; box[3] = red.v[0][3];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            box[0] = fmin(box[0], red.v[w][0]); box[1] = fmax(box[1], red.v[w][1]);
            box[2] = fmin(box[2], red.v[w][2]); box[3] = fmax(box[3], red.v[w][3]);
        }
    } else {
        box[0] = p.lo0; box[1] = p.hi0; box[2] = p.lo1; box[3] = p.hi1;
    }
    const uint32_t flags = red.flags;
    __syncthreads();   // red is reused by the caller
    return flags;
}

// Per-state coefficients of the log-Maxwellian (Sec. 2.2, Sec. 3.6).
struct Coef {
    double a;    // ln rho - (d/2) ln(2 pi theta)
    double l;    // ln(theta delta / 2)  (-inf when delta == 0)
    double ux, uy;
    double kap;  // 1 / (2 theta)
};

template <int D>
__device__ __forceinline__ Coef make_coef(const BoundsArgs& p, const Prim& s) {
    Coef c;
    c.a = log(s.rho) - (0.5 * D) * log(2.0 * kPi * s.th);
    c.l = (p.half_delta > 0.0) ? log(s.th * p.half_delta) : -kInf;
    c.ux = s.ux;
    c.uy = s.uy;
    c.kap = 0.5 / s.th;
    return c;
}

template <int D>
__device__ __forceinline__ void store_bounds(const BoundsArgs& p, int64_t e, const double* sums,
                                             uint32_t flags) {
    // sums: rho_min, rho_max, E_min, E_max, then (m_min, m_max) per direction
    const int nv = D + 2;
    double rmin = sums[0];
    if (rmin < p.rho_floor) { rmin = p.rho_floor; flags |= KBL_ST_RHO_FLOOR; }
    p.bounds[0 * p.n_elem + e] = rmin;
    p.bounds[(int64_t)nv * p.n_elem + e] = sums[1];
    p.bounds[(int64_t)(D + 1) * p.n_elem + e] = sums[2];
    p.bounds[(int64_t)(nv + D + 1) * p.n_elem + e] = sums[3];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        p.bounds[(int64_t)(1 + j) * p.n_elem + e] = sums[4 + 2 * j];
        p.bounds[(int64_t)(nv + 1 + j) * p.n_elem + e] = sums[5 + 2 * j];
    }
    if (p.status) p.status[e] = flags;
}

template <int D>
__device__ __forceinline__ void store_nan(const BoundsArgs& p, int64_t e, uint32_t flags) {
    const double nan = __builtin_nan("");
    for (int v = 0; v < 2 * (D + 2); ++v) p.bounds[(int64_t)v * p.n_elem + e] = nan;
    if (p.status) p.status[e] = flags;
}

// Fixed-order workgroup sum of NV partials; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double* part, Red& red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) part[i] = wave_sum(part[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red.v[wid][i] = part[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = red.v[0][i];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) s += red.v[w][i];
            part[i] = s;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- 2D kernel
template <int TX, int TY>
__global__ __launch_bounds__(kThreads) void bounds_fp64_2d(BoundsArgs p) {
    constexpr int NXM = 16 * TX, NYM = 16 * TY;
    __shared__ double sA[kChunk][NXM];
    __shared__ double sAI[kChunk][NXM];
    __shared__ double sB[kChunk][NYM];
    __shared__ Coef sC[kChunk];
    __shared__ Red red;

    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;

    for (int64_t e = blockIdx.x; e < p.n_elem; e += gridDim.x) {
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<2>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        double box[4];
        const uint32_t flags = stencil_prologue<2>(p, e, row0, S, red, box);
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<2>(p, e, flags);
            continue;
        }
        const double lox = box[0], loy = box[2];
        const double hx = (box[1] - box[0]) / (double)(p.nx - 1);
        const double hy = (box[3] - box[2]) / (double)(p.ny - 1);

        double qtn[TX][TY], qtx[TX][TY], qin[TX][TY], qix[TX][TY];
#pragma unroll
        for (int i = 0; i < TX; ++i)
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                qtn[i][j] = kInf; qtx[i][j] = -kInf; qin[i][j] = kInf; qix[i][j] = -kInf;
            }

        for (int64_t c0 = 0; c0 < S; c0 += kChunk) {
            const int cn = (int)((S - c0) < kChunk ? (S - c0) : kChunk);
            __syncthreads();
            if (tid < cn) {
                const int64_t s = c0 + tid;
                const int32_t col = p.cols[row0 + s / p.n_s];
                sC[tid] = make_coef<2>(p, load_prim<2>(p, (int64_t)col * p.n_s + s % p.n_s));
            }
            __syncthreads();
            for (int idx = tid; idx < cn * NXM; idx += kThreads) {
                const int s = idx / NXM, j = idx - s * NXM;
                const int jc = j < p.nx ? j : p.nx - 1;
                const double d = (lox + jc * hx) - sC[s].ux;
                const double A = fma(-sC[s].kap * d, d, sC[s].a);
                sA[s][j] = A;
                sAI[s][j] = A + sC[s].l;
            }
            for (int idx = tid; idx < cn * NYM; idx += kThreads) {
                const int s = idx / NYM, j = idx - s * NYM;
                const int jc = j < p.ny ? j : p.ny - 1;
                const double d = (loy + jc * hy) - sC[s].uy;
                sB[s][j] = -sC[s].kap * d * d;
            }
            __syncthreads();
            for (int s = 0; s < cn; ++s) {
                double a[TX], ai[TX], b[TY];
#pragma unroll
                for (int i = 0; i < TX; ++i) { a[i] = sA[s][tx + 16 * i]; ai[i] = sAI[s][tx + 16 * i]; }
#pragma unroll
                for (int j = 0; j < TY; ++j) b[j] = sB[s][ty + 16 * j];
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

        // exp, relaxation, trapezoid weights and the moment contraction
        double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < TX; ++i) {
            const int jx = tx + 16 * i;
            if (jx >= p.nx) continue;
            const double ux = lox + jx * hx;
            const double wx = hx * ((jx == 0 || jx == p.nx - 1) ? 0.5 : 1.0);
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int jy = ty + 16 * j;
                if (jy >= p.ny) continue;
                const double uy = loy + jy * hy;
                const double M = wx * (hy * ((jy == 0 || jy == p.ny - 1) ? 0.5 : 1.0));
                const double ftn = rm * exp(qtn[i][j]);
                const double ftx = rp * exp(qtx[i][j]);
                const double fin = rm * exp(qin[i][j]);
                const double fix = rp * exp(qix[i][j]);
                const double hu2 = 0.5 * ux * ux + 0.5 * uy * uy;
                part[0] += M * ftn;
                part[1] += M * ftx;
                part[2] += M * (hu2 * ftn + fin);
                part[3] += M * (hu2 * ftx + fix);
                if (ux < 0.0) { part[4] += M * ux * ftx; part[5] += M * ux * ftn; }
                else          { part[4] += M * ux * ftn; part[5] += M * ux * ftx; }
                if (uy < 0.0) { part[6] += M * uy * ftx; part[7] += M * uy * ftn; }
                else          { part[6] += M * uy * ftn; part[7] += M * uy * ftx; }
            }
        }
        block_sum<8>(part, red);
        if (tid == 0) store_bounds<2>(p, e, part, flags);
    }
}

// ---------------------------------------------------------------- 1D kernel
// No separability to exploit: each pair costs sub, mul, fma (+ add for the
// internal part) before the four min/max.  Coefficients are broadcast from LDS.
template <int NT, int T>
__global__ __launch_bounds__(NT) void bounds_fp64_1d(BoundsArgs p) {
    __shared__ Coef sC[kChunk];
    __shared__ Red red;
    const int tid = threadIdx.x;
    const double rm = 1.0 - p.r_fac, rp = 1.0 + p.r_fac;
    for (int64_t e = blockIdx.x; e < p.n_elem; e += gridDim.x) {
        const int64_t row0 = p.rowptr[e], row1 = p.rowptr[e + 1];
        if (row0 < 0 || row1 <= row0 || row1 > p.nnz) {
            if (tid == 0) store_nan<1>(p, e, KBL_ST_BAD_STENCIL);
            continue;
        }
        const int64_t S = (row1 - row0) * p.n_s;
        double box[4];
        uint32_t flags;
        if constexpr (NT == kThreads) {
            flags = stencil_prologue<1>(p, e, row0, S, red, box);
        } else {
            // small workgroups: one wave does the prologue serially-strided
            __shared__ double sbox[2];
            __shared__ uint32_t sflags;
            if (tid < 64) {
                uint32_t bad = 0;
                double lx = kInf, hx = -kInf;
                for (int64_t s = tid; s < S; s += 64) {
                    const int32_t col = p.cols[row0 + s / p.n_s];
                    if (col < 0 || col >= p.n_elem) { bad |= KBL_ST_BAD_STENCIL; continue; }
                    const Prim st = load_prim<1>(p, (int64_t)col * p.n_s + s % p.n_s);
                    if (!st.ok) { bad |= KBL_ST_INADMISSIBLE; continue; }
                    const double sd = sqrt(st.th);
                    lx = fmin(lx, st.ux - p.k * sd);
                    hx = fmax(hx, st.ux + p.k * sd);
                }
                lx = wave_min(lx); hx = wave_max(hx);
                for (int o = 32; o > 0; o >>= 1) bad |= (uint32_t)__shfl_xor((int)bad, o, 64);
                if (tid == 0) { sbox[0] = lx; sbox[1] = hx; sflags = bad; }
            }
            __syncthreads();
            if (p.grid_mode == KBL_GRID_STENCIL) { box[0] = sbox[0]; box[1] = sbox[1]; }
            else { box[0] = p.lo0; box[1] = p.hi0; }
            flags = sflags;
            __syncthreads();
        }
        if (flags & (KBL_ST_BAD_STENCIL | KBL_ST_INADMISSIBLE)) {
            if (tid == 0) store_nan<1>(p, e, flags);
            continue;
        }
        const double lo = box[0];
        const double h = (box[1] - box[0]) / (double)(p.nx - 1);
        double u[T], qtn[T], qtx[T], qin[T], qix[T];
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = tid + NT * i;
            u[i] = lo + (j < p.nx ? j : p.nx - 1) * h;
            qtn[i] = kInf; qtx[i] = -kInf; qin[i] = kInf; qix[i] = -kInf;
        }
        for (int64_t c0 = 0; c0 < S; c0 += kChunk) {
            const int cn = (int)((S - c0) < kChunk ? (S - c0) : kChunk);
            __syncthreads();
            if (tid < cn) {
                const int64_t s = c0 + tid;
                const int32_t col = p.cols[row0 + s / p.n_s];
                sC[tid] = make_coef<1>(p, load_prim<1>(p, (int64_t)col * p.n_s + s % p.n_s));
            }
            __syncthreads();
            for (int s = 0; s < cn; ++s) {
                const Coef c = sC[s];
                const double aI = c.a + c.l;
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const double d = u[i] - c.ux;
                    const double t = -c.kap * d;
                    const double q = fma(t, d, c.a);
                    const double qi = fma(t, d, aI);
                    qtn[i] = fmin(qtn[i], q);
                    qtx[i] = fmax(qtx[i], q);
                    qin[i] = fmin(qin[i], qi);
                    qix[i] = fmax(qix[i], qi);
                }
            }
        }
        double part[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const int j = tid + NT * i;
            if (j >= p.nx) continue;
            const double M = h * ((j == 0 || j == p.nx - 1) ? 0.5 : 1.0);
            const double ftn = rm * exp(qtn[i]);
            const double ftx = rp * exp(qtx[i]);
            const double fin = rm * exp(qin[i]);
            const double fix = rp * exp(qix[i]);
            const double hu2 = 0.5 * u[i] * u[i];
            part[0] += M * ftn;
            part[1] += M * ftx;
            part[2] += M * (hu2 * ftn + fin);
            part[3] += M * (hu2 * ftx + fix);
            if (u[i] < 0.0) { part[4] += M * u[i] * ftx; part[5] += M * u[i] * ftn; }
            else            { part[4] += M * u[i] * ftn; part[5] += M * u[i] * ftx; }
        }
        if constexpr (NT == kThreads) {
            block_sum<6>(part, red);
        } else {
            const int lane = tid & 63, wid = tid >> 6;
#pragma unroll
            for (int i = 0; i < 6; ++i) part[i] = wave_sum(part[i]);
            if (lane == 0)
                for (int i = 0; i < 6; ++i) red.v[wid][i] = part[i];
            __syncthreads();
            if (tid == 0)
                for (int i = 0; i < 6; ++i) {
                    double s = red.v[0][i];
                    for (int w = 1; w < NT / 64; ++w) s += red.v[w][i];
                    part[i] = s;
                }
            __syncthreads();
        }
        if (tid == 0) store_bounds<1>(p, e, part, flags);
    }
}

template <typename K>
hipError_t launch(K kernel, int threads, const BoundsArgs& a, hipStream_t stream) {
    const int64_t grid = a.n_elem < (int64_t)INT32_MAX ? a.n_elem : (int64_t)INT32_MAX;
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(threads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bounds_fp64(const BoundsArgs& a, int dim, hipStream_t stream) {
    if (a.n_elem == 0) return hipSuccess;
    if (dim == 2) {
        const int nmax = a.nx > a.ny ? a.nx : a.ny;
        if (nmax <= 16) return launch(bounds_fp64_2d<1, 1>, kThreads, a, stream);
        if (nmax <= 32) return launch(bounds_fp64_2d<2, 2>, kThreads, a, stream);
        if (nmax <= 48) return launch(bounds_fp64_2d<3, 3>, kThreads, a, stream);
        if (nmax <= 64) return launch(bounds_fp64_2d<4, 4>, kThreads, a, stream);
        return hipErrorInvalidValue;
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

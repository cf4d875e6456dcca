// Device helpers shared by the FP64 and mixed-precision bounds kernels:
// state loading and admissibility, log-Maxwellian coefficients, the stencil
// prologue (Sec. 3.9 step 1, eq. truncdomain), reductions and stores.
// Included by translation units compiled with -fno-honor-nans: finiteness is
// tested on bit patterns.
#pragma once

#include <math.h>

#include "kbl_internal.h"
#include "exp2_table.h"

namespace kbl {
namespace {


constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxStates = 256;     // stencil states staged in LDS at once
constexpr double kInf = __builtin_inf();
constexpr float kInfF = __builtin_inff();

struct Prim {
    double rho, ux, uy, uz, th;
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
    static_assert(D >= 1 && D <= 3, "d = 1, 2 or 3");
    Prim s;
    const double rho = p.states[node];
    const double mx = p.states[p.n_nodes + node];
    const double my = (D >= 2) ? p.states[2 * p.n_nodes + node] : 0.0;
    const double mz = (D == 3) ? p.states[3 * p.n_nodes + node] : 0.0;
    const double E = p.states[(D + 1) * p.n_nodes + node];
    double mm, P;
    {
#pragma clang fp contract(off)
        mm = mx * mx;
        if (D >= 2) mm = mm + my * my;
        if (D == 3) mm = mm + mz * mz;
        P = p.gm1 * (E - 0.5 * mm / rho);
    }
    s.rho = rho;
    s.ux = mx / rho;
    s.uy = (D >= 2) ? my / rho : 0.0;
    s.uz = (D == 3) ? mz / rho : 0.0;
    s.th = P / rho;
    s.ok = finite_bits(rho) && finite_bits(mx) && finite_bits(my) && finite_bits(mz) &&
           finite_bits(E) && finite_bits(P) && finite_bits(s.th) && rho > 0.0 && P > 0.0;
    return s;
}

// Wave64 reductions on the lane networks (no LDS round trips): DPP inside
// rows of 16 lanes (neighbour and pair swaps by quad_perm, half-row and row
// mirrors, row rotation by 8) and gfx950's permlane swaps across rows and
// half-waves.  Each step combines the same two operands in every lane that
// keeps the result, so results are bit-identical across those lanes and
// deterministic.  All 64 lanes must be active.
constexpr int kDppXor1 = 0xB1;          // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;          // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;   // row_half_mirror
constexpr int kDppMirror = 0x140;       // row_mirror
constexpr int kDppRor8 = 0x128;         // row_ror:8 (lane i <-> lane i ^ 8 in a row)

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

struct OpSum { __device__ static double f(double a, double b) { return a + b; } };
struct OpMin { __device__ static double f(double a, double b) { return fmin(a, b); } };

// Lane swaps of gfx950 on doubles, one 32-bit half at a time.  ROW16 false
// (v_permlane32_swap): lanes 32-63 of a <-> lanes 0-31 of b.  ROW16 true
// (v_permlane16_swap): odd rows of a <-> even rows of b (rows of 16 lanes).
template <bool ROW16>
__device__ __forceinline__ void lane_swap(double& a, double& b) {
    const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
    const unsigned alo = (unsigned)ia, ahi = (unsigned)(ia >> 32);
    const unsigned blo = (unsigned)ib, bhi = (unsigned)(ib >> 32);
    const auto lo = ROW16 ? __builtin_amdgcn_permlane16_swap(alo, blo, false, false)
                          : __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto hi = ROW16 ? __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false)
                          : __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    a = __longlong_as_double(((long long)hi[0] << 32) | (long long)lo[0]);
    b = __longlong_as_double(((long long)hi[1] << 32) | (long long)lo[1]);
}

// Eight wave reductions at once, by transposition: each exchange stage
// halves the number of values a lane carries, so a wave spends about 35 VALU
// ops where eight separate reductions spend about 190.
//  1. v[k] and v[k + 4] exchange half-waves: lanes 0-31 then carry values
//     0-3 combined over lanes l and l + 32, lanes 32-63 values 4-7.
//  2. v[0] and v[2], v[1] and v[3] exchange rows: row r of v[0] carries
//     value 2r, of v[1] value 2r + 1.
//  3. Within a row, lanes 0-7 keep v[0] and lanes 8-15 v[1] (exchange over
//     lane bit 3), then bits 0-2 go over the DPP network.
// Returns in lane l the reduction of value l / 8 over the wave (identical
// across lanes l / 8 * 8 ... + 7).  The order of the combinations is fixed,
// so sums are deterministic.  All 64 lanes must be active.
template <class Op>
__device__ __forceinline__ double wave_transpose8(double* v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lane_swap<false>(v[k], v[k + 4]);
        v[k] = Op::f(v[k], v[k + 4]);
    }
    lane_swap<true>(v[0], v[2]);
    v[0] = Op::f(v[0], v[2]);
    lane_swap<true>(v[1], v[3]);
    v[1] = Op::f(v[1], v[3]);
    const bool upper = (lane & 8) != 0;
    double y = upper ? v[1] : v[0];
    const double give = upper ? v[0] : v[1];
    y = Op::f(y, dpp_f64<kDppRor8>(give));
    y = Op::f(y, dpp_f64<kDppXor1>(y));
    y = Op::f(y, dpp_f64<kDppXor2>(y));
    y = Op::f(y, dpp_f64<kDppHalfMirror>(y));
    return y;
}

// Integer minimum over the wave, uniform: rows on DPP, then the four row
// results by readlane in a fixed order.
__device__ __forceinline__ int wave_min_i32(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppXor1, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppXor2, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppHalfMirror, 0xF, 0xF, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppMirror, 0xF, 0xF, false));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Shared scratch for the per-element prologue and epilogue (up to 4 waves).
struct Red {
    double v[kWaves][16];
    uint32_t flags;
};

// XCD-aware element order.  Workgroups are dispatched round-robin over the
// XCDs (8 on MI355X, each with its own L2), so workgroup b runs on XCD b % 8.
// Each XCD is given a contiguous range of elements, walked by its workgroups
// in a grid stride: stencil neighbours (nearby element ids on structured and
// locally numbered meshes) are then read through the same L2.  With
// grid_blocks = -k (k elements per workgroup) workgroup j of an XCD takes
// the k consecutive elements from j k on instead, so that the elements in
// flight on an XCD stay one contiguous band (a grid stride would put its
// two or four passes half or a quarter of the range apart); the host sizes
// that grid so that the chunks cover every XCD's range, else the grid
// stride is kept.  Every element is visited exactly once for any grid size
// >= 1.
constexpr int kXcds = 8;
struct ElemRange {
    int64_t e, end, step;
};
__device__ __forceinline__ ElemRange xcd_range(int64_t n, int64_t grid_blocks) {
    static_assert(kXcds == 8, "shifts below assume 8 XCDs");
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (G >= kXcds) {
        // the usual case, in shifts and masks: all scalar work (a 64-bit
        // division of uniform values would be expanded on the VALU, about a
        // hundred instructions per workgroup)
        const int64_t x = b & (kXcds - 1), j = b >> 3;
        const int64_t gx = (G >> 3) + (x < (G & (kXcds - 1)) ? 1 : 0);
        const int64_t q = n >> 3, r = n & (kXcds - 1);
        const int64_t start = x * q + (x < r ? x : r);
        const int64_t cnt = q + (x < r ? 1 : 0);
        if (grid_blocks < 0) {
            const int64_t k = grid_blocks < -n ? n : -grid_blocks;
            if (gx * k >= cnt) {
                const int64_t e0 = start + j * k;
                return ElemRange{e0, e0 + k < start + cnt ? e0 + k : start + cnt, 1};
            }
        }
        return ElemRange{start + j, start + cnt, gx};
    }
    // fewer workgroups than XCDs: one group per workgroup
    const int64_t q = n / G, r = n % G;
    const int64_t start = b * q + (b < r ? b : r);
    const int64_t cnt = q + (b < r ? 1 : 0);
    return ElemRange{start, start + cnt, 1};
}

// Ends of one state's velocity interval U -+ k sqrt(theta) (eq. truncdomain).
// Written with an explicit fma so that every kernel rounds them identically
// (the backward locates the extreme states by equality).
// Rounded like the plain definition (no fused multiply-add), as are the
// node positions and the primitive variables below: values deep in the
// Maxwellian tails are very sensitive to the node positions (d q / d u =
// -(u - U)/theta), so the box ends and nodes are kept bit-identical to the
// straightforward evaluation.
__device__ __forceinline__ double box_lo(double u, double k, double sd) {
#pragma clang fp contract(off)
    return u - k * sd;
}
__device__ __forceinline__ double box_hi(double u, double k, double sd) {
#pragma clang fp contract(off)
    return u + k * sd;
}
// exp for the moment contraction, by Tang's table-driven method (ACM TOMS
// 15(2), 1989): x = (256 m + j) ln(2)/256 + r with |r| <= ln(2)/512, so that
// exp(x) = 2^m 2^(j/256) exp(r).  n = 256 m + j is rounded by adding
// 1.5 2^52, which leaves n in the low word of the sum; r is reduced with
// ln(2)/256 in two parts.  exp(r) - 1 is its degree-4 Taylor polynomial
// (remainder below 4e-17), evaluated as r (24 + r (12 + r (4 + r))) / 24 with
// the 1/24 taken from the table (T/24 next to T), so that the polynomial's
// constants are inline or one scalar operand each.  Error about 1 ulp.  The
// argument is clamped below at -1100 (-inf gives 0); the callers' arguments
// are bounded above by the log-peaks of admissible states (far below the
// 5.8e6 at which n would leave 32 bits).  14 VALU ops and one LDS read,
// against 22 VALU ops of the general-purpose exp.  tab: the table staged in LDS by stage_exp_table (a global table read
// per lane waits on memory latency).
__device__ __forceinline__ double exp_tab(double x, const ExpPair* tab) {
    constexpr double kInvStep = 0x1.71547652b82fep+8;   // 256 / ln 2
    // the empty asm keeps the clamp at the use; otherwise the compiler
    // clamps every accumulator of the caller at once (register pressure)
    asm volatile("" : "+v"(x));
    x = fmax(x, -1100.0);
    const double t = fma(x, kInvStep, 0x1.8p52);
    const double n = t - 0x1.8p52;
    const int ni = __double2loint(t);
    double r = fma(-n, kLn2By256Hi, x);
    r = fma(-n, kLn2By256Lo, r);
    double q = r + 4.0;
    q = fma(r, q, 12.0);
    q = fma(r, q, 24.0);
    q = r * q;
    const ExpPair T = tab[ni & 255];
    return ldexp(fma(T.t24, q, T.t), ni >> 8);
}

// exp_tab in two parts, the same operations in the same order: the index
// and the polynomial of the reduced argument, then the table product.  A
// caller can issue the table reads of several values together between the
// two parts.
struct ExpPrep {
    double q;
    int ni;
};
__device__ __forceinline__ ExpPrep exp_prep(double x) {
    constexpr double kInvStep = 0x1.71547652b82fep+8;   // 256 / ln 2
    x = fmax(x, -1100.0);
    const double t = fma(x, kInvStep, 0x1.8p52);
    const double n = t - 0x1.8p52;
    ExpPrep e;
    e.ni = __double2loint(t);
    double r = fma(-n, kLn2By256Hi, x);
    r = fma(-n, kLn2By256Lo, r);
    double q = r + 4.0;
    q = fma(r, q, 12.0);
    q = fma(r, q, 24.0);
    e.q = r * q;
    return e;
}
__device__ __forceinline__ double exp_fin(const ExpPrep& e, const ExpPair& T) {
    return ldexp(fma(T.t24, e.q, T.t), e.ni >> 8);
}

// Copies the exp table into LDS; the caller's next barrier publishes it.
template <int NT>
__device__ __forceinline__ void stage_exp_table(ExpPair* tab) {
    for (int i = threadIdx.x; i < 256; i += NT) tab[i] = kExp2Tab[i];
}

// Velocity node j of a trapezoid grid starting at lo with spacing h.
__device__ __forceinline__ double node_pos(double lo, int j, double h) {
#pragma clang fp contract(off)
    return lo + (double)j * h;
}

// Per-state coefficients of the log-Maxwellian (Sec. 2.2, Sec. 3.6).
struct Coef {
    double a;    // ln rho - (d/2) ln(2 pi theta)
    double al;   // a + ln(theta delta / 2)   (-inf when delta == 0)
    double ux, uy;
    double nk;   // -1 / (2 theta)
};
// The same for d = 3 (kept apart so that the LDS staging of the d <= 2
// kernels does not grow).
struct Coef3 {
    double a, al;
    double ux, uy, uz;
    double nk;
};

// FP32 coefficients of the mixed-precision forms: shifted by the element's
// log-peak references and centred on the velocity box.
struct CoefF {
    float a;    // a - ref_T
    float al;   // a + l - ref_I   (-inf without internal degrees of freedom)
    float ux;   // U_x - box centre
    float uy;   // U_y - box centre
    float nk;   // -1 / (2 theta)
};

template <int D, class CT = Coef>
__device__ __forceinline__ CT make_coef(const BoundsArgs& p, const Prim& s) {
    CT c;
    c.a = log(s.rho) - (0.5 * D) * log(2.0 * kPi * s.th);
    c.al = (p.half_delta > 0.0) ? c.a + log(s.th * p.half_delta) : -kInf;
    c.ux = s.ux;
    c.uy = s.uy;
    if constexpr (D == 3) c.uz = s.uz;
    c.nk = -0.5 / s.th;
    return c;
}

// Stencil state s of the row starting at row0 (the caller validated the row).
__device__ __forceinline__ int64_t state_node(const BoundsArgs& p, int64_t row0, int64_t s) {
    const int32_t col = p.cols[row0 + s / p.n_s];
    return (int64_t)col * p.n_s + s % p.n_s;
}

// Prologue: admissibility, velocity box, and (if sC is given) the
// coefficients of the first kMaxStates states staged in sC.  Returns status
// bits (uniform).  box: (lo, hi) per direction, box[2j] and box[2j+1] for
// j < D.
// ref (optional): max over the stencil of a and of a + l, the log-peak
// references the mixed-precision kernels shift by.
template <int D, int NT, class CT>
__device__ uint32_t stencil_prologue(const BoundsArgs& p, int64_t row0, int64_t S, Red& red,
                                     CT* sC, double box[2 * D], double* ref = nullptr) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    uint32_t bad = 0;
    double lx = kInf, hx = -kInf, ly = kInf, hy = -kInf, lz = kInf, hz = -kInf;
    double ra = -kInf, rl = -kInf;
    for (int64_t s = tid; s < S; s += NT) {
        const int32_t col = p.cols[row0 + s / p.n_s];
        if (col < 0 || col >= p.n_src) { bad |= KBL_ST_BAD_STENCIL; continue; }
        const Prim st = load_prim<D>(p, (int64_t)col * p.n_s + s % p.n_s);
        if (!st.ok) { bad |= KBL_ST_INADMISSIBLE; continue; }
        const CT c = make_coef<D, CT>(p, st);
        if (sC && s < kMaxStates) sC[s] = c;
        ra = fmax(ra, c.a);
        rl = fmax(rl, c.al);
        if (p.grid_mode == KBL_GRID_STENCIL) {
            const double sd = sqrt(st.th);
            lx = fmin(lx, box_lo(st.ux, p.k, sd));
            hx = fmax(hx, box_hi(st.ux, p.k, sd));
            if (D >= 2) {
                ly = fmin(ly, box_lo(st.uy, p.k, sd));
                hy = fmax(hy, box_hi(st.uy, p.k, sd));
            }
            if (D == 3) {
                lz = fmin(lz, box_lo(st.uz, p.k, sd));
                hz = fmax(hz, box_hi(st.uz, p.k, sd));
            }
        }
    }
    if (tid == 0) red.flags = 0;
    // one transposed minimum over the wave for the box ends and log-peaks,
    // maxima taken as minima of the negated values (exact)
    double ext[8] = {lx, -hx, ly, -hy, lz, -hz, -ra, -rl};
    const double m = wave_transpose8<OpMin>(ext);
    __syncthreads();
    if (bad) atomicOr(&red.flags, bad);
    if ((lane & 7) == 0) red.v[wid][lane >> 3] = m;
    __syncthreads();
    // wave w's extremum j sits in red.v[w][j]; the maxima are negated
    auto ext_min = [&](int j) {
        double r = red.v[0][j];
#pragma unroll
        for (int w = 1; w < NW; ++w) r = fmin(r, red.v[w][j]);
        return r;
    };
    if (ref) {
        ref[0] = -ext_min(6);
        ref[1] = -ext_min(7);
    }
    if (p.grid_mode == KBL_GRID_STENCIL) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            box[2 * j] = ext_min(2 * j);
            box[2 * j + 1] = -ext_min(2 * j + 1);
        }
    } else {
        const double glo[3] = {p.lo0, p.lo1, p.lo2}, ghi[3] = {p.hi0, p.hi1, p.hi2};
#pragma unroll
        for (int j = 0; j < D; ++j) { box[2 * j] = glo[j]; box[2 * j + 1] = ghi[j]; }
    }
    uint32_t flags = red.flags;
    // a bad row is reported alone (its other states are not a stencil)
    if (flags & KBL_ST_BAD_STENCIL) flags = KBL_ST_BAD_STENCIL;
    __syncthreads();   // red is reused by the caller
    return flags;
}

// Stage the coefficients of states [c0, c0 + cn) into sC (chunks after the
// first, for stencils larger than kMaxStates).  Bracketed by barriers.
template <int D, int NT, class CT>
__device__ __forceinline__ void stage_chunk(const BoundsArgs& p, int64_t row0, int64_t c0, int cn,
                                            CT* sC) {
    __syncthreads();
    for (int s = threadIdx.x; s < cn; s += NT)
        sC[s] = make_coef<D, CT>(p, load_prim<D>(p, state_node(p, row0, c0 + s)));
    __syncthreads();
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

// One of the 2 (D + 2) sums, in the order of store_bounds, stored by its
// own thread; thread t == 0 (rho_min) applies the floor and writes the status.
template <int D>
__device__ __forceinline__ void store_bound_value(const BoundsArgs& p, int64_t e, int t, double v,
                                                  uint32_t flags) {
    const int nv = D + 2;
    int row;
    if (t < 4) row = (t & 1) * nv + (t >> 1) * (D + 1);
    else row = ((t - 4) & 1) * nv + 1 + ((t - 4) >> 1);
    if (t == 0) {
        if (v < p.rho_floor) { v = p.rho_floor; flags |= KBL_ST_RHO_FLOOR; }
        if (p.status) p.status[e] = flags;
    }
    p.bounds[(int64_t)row * p.n_elem + e] = v;
}

template <int D>
__device__ __forceinline__ void store_nan(const BoundsArgs& p, int64_t e, uint32_t flags) {
    // quiet NaN by its bit pattern (these translation units assume no NaN
    // arithmetic, but a stored pattern is just data)
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    for (int v = 0; v < 2 * (D + 2); ++v) p.bounds[(int64_t)v * p.n_elem + e] = nan;
    if (p.status) p.status[e] = flags;
}

// Fixed-order workgroup sum of 8 partials: wave_transpose8, then lanes 0,
// 8, ..., 56 publish their wave's sums and thread t < 8 adds the waves' sums
// of value t in wave order.  Returns value t in thread t < 8 (0 elsewhere).
// All lanes active; contains the barriers.
template <int NT>
__device__ __forceinline__ double block_sum8(double* v, Red& red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double y = wave_transpose8<OpSum>(v);
    if ((lane & 7) == 0) red.v[wid][lane >> 3] = y;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < 8) {
        r = red.v[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < NW; ++w) r += red.v[w][threadIdx.x];
    }
    __syncthreads();   // red is reused by the caller
    return r;
}

// Fixed-order workgroup sum of NV <= 16 partials by wave_transpose8 on
// groups of eight (zero-padded); the sums are valid in thread 0 (part[0 ..
// NV-1]).  All lanes active; contains the barriers.
template <int NT, int NV>
__device__ __forceinline__ void block_sum_t(double* part, Red& red) {
    static_assert(NV >= 1 && NV <= 16, "up to 16 partials");
    constexpr int NW = NT / 64;
    constexpr int NG = (NV + 7) / 8;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (8 * g + k < NV) ? part[8 * g + k] : 0.0;
        const double y = wave_transpose8<OpSum>(v);
        if ((lane & 7) == 0) red.v[wid][8 * g + (lane >> 3)] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double t = red.v[0][i];
#pragma unroll
            for (int w = 1; w < NW; ++w) t += red.v[w][i];
            part[i] = t;
        }
    }
    __syncthreads();
}


}  // namespace
}  // namespace kbl

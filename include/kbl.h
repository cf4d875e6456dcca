/*
 * kbl.h - kinetic maximum-principle bounds and squeeze limiting for the Euler
 * equations on AMD Instinct MI355X (gfx950).
 *
 * Method: Dzanic & Martinelli, "High-order limiting methods using maximum
 * principle bounds derived from the Boltzmann equation I: Euler equations".
 * For every element, the Maxwellian of each state in the element's stencil is
 * evaluated on a discrete velocity grid (Sec. 2.2, eq. maxwell), the pointwise
 * min/max distribution is taken (Sec. 3.2-3.3, eq. fminmax; relaxed per
 * Sec. 3.5), its moments give bounds on density, momentum and total energy
 * (eq. rhobounds, Ebounds, mmbounds, mpbounds; internal energy per Sec. 3.6;
 * trapezoid quadrature per Sec. 3.7), and the coupled squeeze limiter pulls
 * the element's nodal solution into those bounds (Sec. 3.4, eq. alpha,
 * eq. limiter) followed by the pressure step of Sec. 3.8.
 *
 * Conventions for every entry point
 *  - Array pointers are DEVICE pointers owned by the caller unless stated
 *    otherwise.  The library allocates nothing and keeps no device memory
 *    between calls.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it and the call returns without synchronising.
 *  - Argument errors are detected on the host before any launch and returned
 *    synchronously (nothing is enqueued).  A launch failure returns
 *    KBL_ERR_HIP.  Data-dependent conditions never fail a call: they are
 *    reported per element in `elem_status` bits (see KBL_ST_*).
 *  - Conserved states are stored SoA: row v of a [d+2][n_elem*n_s] array
 *    holds variable v (rho, m_1..m_d, E) of every node; the nodes of element e
 *    are e*n_s .. e*n_s+n_s-1.
 *  - Spatial dimension d is 1, 2 or 3.  gamma > 1 and delta = 2/(gamma-1) - d
 *    must be >= 0 (Sec. 3.6).  d = 3 (the extension the paper's conclusion
 *    names as costly, Sec. 7) is built for the FP64 bounds with the default
 *    energy model, the limiter and the Riemann-averaged states; the mixed
 *    precisions, KBL_FLAG_ENERGY_PERSTATE and the backward return
 *    KBL_ERR_UNSUPPORTED for it.
 *  - No exception crosses this interface.
 */
#ifndef KBL_H
#define KBL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KBL_OK = 0,
    KBL_ERR_ARG = 1,          /* bad dimension, size, pointer or parameter */
    KBL_ERR_GAMMA = 2,        /* gamma <= 1 or delta = 2/(gamma-1) - d < 0 */
    KBL_ERR_GRID = 3,         /* velocity grid: n < 2, hi <= lo, k <= 0 or too many nodes */
    KBL_ERR_UNSUPPORTED = 4,  /* combination not built (see kbl_status_string) */
    KBL_ERR_HIP = 5,          /* a HIP runtime call or launch failed */
    KBL_ERR_WORKSPACE = 6     /* workspace missing or too small */
} kbl_status;

/* Velocity-grid modes (Sec. 3.7). */
#define KBL_GRID_GLOBAL  0    /* one box [lo, hi] for every element */
#define KBL_GRID_STENCIL 1    /* per element: [min_S(U - k sqrt(theta)), max_S(U + k sqrt(theta))] */

/* Arithmetic of the bounds pass. */
#define KBL_PREC_FP64        0   /* every step in FP64 */
#define KBL_PREC_MIXED_BF16  1   /* FP32 envelopes/exp, BF16 MFMA contraction (hi/lo split) */
#define KBL_PREC_MIXED_FP16  2   /* FP32 envelopes/exp, FP16 MFMA contraction (hi/lo split) */
#define KBL_PREC_MIXED_FP32  3   /* FP32 envelopes/exp, FP32 VALU contraction */

/* Per-element status bits.  kbl_compute_bounds writes bits 0x1-0x2 and 0x100-0x200;
 * kbl_limit writes bits 0x4-0x80. */
#define KBL_ST_INADMISSIBLE  0x1u    /* a stencil state has rho<=0, P<=0 or a non-finite value: bounds are NaN */
#define KBL_ST_RHO_FLOOR     0x2u    /* rho_min was raised to rho_floor (Sec. 3.8) */
#define KBL_ST_EPS_RULE      0x4u    /* some alpha_i was set to 0 by the epsilon rule (Sec. 3.4) */
#define KBL_ST_LIMITED       0x8u    /* alpha_min < 1 */
#define KBL_ST_PSTEP         0x10u   /* the pressure step fired (Sec. 3.8) */
#define KBL_ST_PMEAN_FLOOR   0x20u   /* P(mean) <= p_floor: alpha_P = 0 (element flattened) */
#define KBL_ST_MEAN_OUTSIDE  0x40u   /* element mean lies outside its bounds */
#define KBL_ST_BAD_BOUNDS    0x80u   /* bounds not finite: element passed through unchanged */
#define KBL_ST_BAD_STENCIL   0x100u  /* stencil row out of range (rowptr or cols): bounds are NaN; set alone */
#define KBL_ST_TOO_LARGE     0x200u  /* mixed precision and backward: more than 256 stencil states (NaN bounds / zero gradient) */
#define KBL_ST_ASYMMETRIC    0x400u  /* backward: a stencil neighbour does not list this element back */

typedef struct {
    int32_t mode;       /* KBL_GRID_GLOBAL or KBL_GRID_STENCIL */
    int32_t n[3];       /* nodes per direction, endpoints included (entries >= d ignored);
                           at most 4096 (d = 1; 2048 for the backward) or 64 per direction (d = 2, 3) */
    double  lo[3];      /* GLOBAL: lower box corner */
    double  hi[3];      /* GLOBAL: upper box corner */
    double  k;          /* STENCIL: extent in thermal units (the paper uses 4 in 2D, 8 in 1D) */
} kbl_vgrid;

typedef struct {
    double  gamma;      /* ratio of specific heats */
    double  r_fac;      /* relaxation factor, 0 <= r_fac < 1 (Sec. 3.5; the paper uses 1e-3) */
    double  rho_floor;  /* density floor on rho_min (Sec. 3.8; 1e-12) */
    double  p_floor;    /* pressure floor of the pressure step (Sec. 3.8; 1e-12) */
    double  eps_alpha;  /* epsilon of the limiter's degenerate-range rule (Sec. 3.4; 1e-13) */
    int32_t precision;  /* KBL_PREC_* (kbl_compute_bounds only) */
    int32_t flags;      /* KBL_FLAG_* bits, 0 for the paper's default method */
} kbl_params;

/* kbl_params.flags */
/* kbl_limit: limit each component with its own alpha_i instead of the coupled
 * minimum (the independent option of Sec. 3.4).  alpha[0] still reports
 * min_i alpha_i. */
#define KBL_FLAG_INDEPENDENT_ALPHA 0x1
/* kbl_compute_bounds(_nodes), FP64 only: energy bounds from the envelope of
 * the per-state energy integrand g_i (|u|^2/2 + theta_i delta/2) instead of
 * separate envelopes of g_T and g_I = (theta delta/2) g_T (Sec. 3.6). */
#define KBL_FLAG_ENERGY_PERSTATE 0x2

/* Fills `p` with the paper's defaults for the given gamma (r_fac 1e-3, floors
 * 1e-12, epsilon 1e-13, FP64). */
void kbl_default_params(kbl_params* p, double gamma);

/*
 * kbl_compute_bounds - kinetic local-maximum-principle bounds per element.
 * Follows steps 1-3 of the overview in Sec. 3.9: collect the stencil states,
 * evaluate f_min/f_max (eq. fminmax, eq. relaxed) on the velocity grid of
 * Sec. 3.7 with the internal-energy model of Sec. 3.6, integrate the moments
 * (eq. rhobounds, Ebounds, mmbounds, mpbounds) and floor rho_min (Sec. 3.8).
 *
 *   states       [d+2][n_elem*n_s] FP64 conserved states of every node.
 *   rowptr, cols element stencil in CSR form: row e lists element ids
 *                (self included by the caller); every node of every listed
 *                element is a stencil state.  rowptr has n_elem+1 entries,
 *                cols has nnz entries.  Rows that leave [0, nnz] or name an
 *                element outside [0, n_elem) get KBL_ST_BAD_STENCIL and NaN
 *                bounds; nothing outside the two arrays is read.
 *   vgrid        host pointer, copied during the call.
 *   bounds       out [2(d+2)][n_elem] FP64: rows (rho, m_1..m_d, E)_min then
 *                (rho, m_1..m_d, E)_max.
 *   elem_status  out [n_elem] or NULL.
 * Precision KBL_PREC_MIXED_* (d = 2 only) computes the envelopes in FP32
 * (shifted by the element's log-peak so exp stays in (0, 1]) and contracts
 * the moments on MFMA (BF16 split in three or FP16 split hi/lo, FP32
 * accumulation) or on the FP32 VALU; the admissibility checks, velocity box,
 * exp scaling, relaxation and floors stay FP64.  Results agree with the FP64
 * path to about 1e-6 relative (momentum relative to the stencil's momentum
 * scale).  With KBL_FLAG_ENERGY_PERSTATE (FP64 only) the energy rows come
 * from the per-state energy integrand instead.
 */
kbl_status kbl_compute_bounds(const kbl_params* params, int32_t dim, int64_t n_elem,
                              int32_t n_s, int64_t nnz, const double* states,
                              const int32_t* rowptr, const int32_t* cols,
                              const kbl_vgrid* vgrid, double* bounds,
                              uint32_t* elem_status, void* stream);

/*
 * kbl_compute_bounds_nodes - the same bounds for node-level stencils: row e
 * lists node ids, and each listed node is one stencil state.  This is the
 * stencil of Sec. 5 (the element's solution points, its own flux points and
 * the neighbours' flux points on the shared faces), or any other set of
 * nodes, e.g. per-node neighbourhoods.
 *
 *   states       [d+2][n_nodes] FP64 conserved states of every node that a
 *                stencil may list (solution and flux points alike).
 *   rowptr, cols node stencil in CSR form; ids outside [0, n_nodes) give
 *                KBL_ST_BAD_STENCIL and NaN bounds.
 *   the rest     as in kbl_compute_bounds (launch choices as for n_s = 1).
 */
kbl_status kbl_compute_bounds_nodes(const kbl_params* params, int32_t dim, int64_t n_elem,
                                    int64_t n_nodes, int64_t nnz, const double* states,
                                    const int32_t* rowptr, const int32_t* cols,
                                    const kbl_vgrid* vgrid, double* bounds,
                                    uint32_t* elem_status, void* stream);

/*
 * Tuning knobs read from the environment at each kbl_compute_bounds call
 * (meant for measurements and tests; they override kbl_autotune_bounds):
 *   KBL_BOUNDS_TILE=<t>        FP64 tile configuration index of the 2D or 3D
 *                              kernel (ignored if it does not cover the
 *                              velocity grid)
 *   KBL_MIXED_TILE=<t>         mixed-precision tile configuration index
 *   KBL_PERSISTENT_BLOCKS=<g>  grid of g workgroups walking the elements
 *                              (0 = one workgroup per element, -k = k
 *                              elements per workgroup)
 * Without either, a 2D launch has each workgroup compute two elements (half
 * as many workgroups as elements), a 1D or 3D launch one workgroup per
 * element.
 */
/*
 * kbl_autotune_bounds - picks the launch configuration of kbl_compute_bounds
 * for this problem shape by timing every candidate on the caller's inputs:
 * each tile configuration that fits the velocity grid, launched with one,
 * two or four elements per workgroup or as a persistent grid of 1, 2, 4 or 8
 * workgroups per compute unit (each workgroup then walks elements in a grid
 * stride).  Timing uses the first `sample_elems` elements (all when <= 0);
 * each candidate keeps the better of two trials, and the default launch is
 * kept unless another candidate is more than 3% faster.
 * The choice is kept (per process) for later kbl_compute_bounds calls with
 * the same dimension, precision, grid size, nodes per element and grid mode.
 * Synchronises `stream`; leaves the full bounds of all elements in `bounds`
 * (and the status in `elem_status` when non-null).  Returns 8 * tile + shape
 * for the chosen candidate (tile: index of the tile configuration, 0 in 1D;
 * shape: 0 = one workgroup per element, 1..4 = 1, 2, 4, 8 workgroups per
 * compute unit, 5 = two and 6 = four elements per workgroup), or -1 on bad
 * arguments or a HIP failure.
 */
int32_t kbl_autotune_bounds(const kbl_params* params, int32_t dim, int64_t n_elem, int32_t n_s,
                            int64_t nnz, const double* states, const int32_t* rowptr,
                            const int32_t* cols, const kbl_vgrid* vgrid, double* bounds,
                            uint32_t* elem_status, int64_t sample_elems, void* stream);

/* Forgets every choice made by kbl_autotune_bounds. */
void kbl_autotune_clear(void);

/*
 * kbl_limit - coupled squeeze limiter (Sec. 3.4, eq. alpha and eq. limiter,
 * with the epsilon rule) and pressure step (Sec. 3.8, eq. pmin and
 * eq. doublelimit), all in FP64.  Steps 5-7 of the overview in Sec. 3.9.
 *
 *   solution     [d+2][n_elem*n_s] nodal solution to limit.
 *   bounds       [2(d+2)][n_elem] as written by kbl_compute_bounds.
 *   node_weights HOST pointer, n_s weights c_j of the element mean
 *                (Assumption (iii)(a) of Sec. 4), copied during the call:
 *                non-negative with a positive sum; nodes of V that are not
 *                quadrature nodes of the mean (flux points) take weight 0.
 *   limited      out [d+2][n_elem*n_s]; may alias `solution`.
 *   alpha        out [2][n_elem] (alpha_min, alpha_P; alpha_P = 1 when the
 *                pressure step does not fire) or NULL.
 *   elem_status  out [n_elem] or NULL.
 * n_s (nodes of V per element) must be at most 64.  When P(mean) <= p_floor
 * the pressure step uses alpha_P = 0.  Non-finite bounds leave the element
 * unchanged.  KBL_FLAG_INDEPENDENT_ALPHA blends each component with its own
 * alpha_i instead of the coupled minimum.
 */
kbl_status kbl_limit(const kbl_params* params, int32_t dim, int64_t n_elem, int32_t n_s,
                     const double* solution, const double* bounds,
                     const double* node_weights, double* limited, double* alpha,
                     uint32_t* elem_status, void* stream);

/* Status bits of kbl_riemann_states, per pair. */
#define KBL_RS_BELOW(v)   (1u << (v))        /* wbar_v < w_min,v of the pair's element */
#define KBL_RS_ABOVE(v)   (1u << (8 + (v)))  /* wbar_v > w_max,v */
#define KBL_RS_BAD_INPUT  (1u << 16)         /* node id out of range or state not admissible */

/*
 * kbl_riemann_states - Riemann-averaged states of Thm. 4.3 (Sec. 4) for pairs
 * of node states across faces, and their position relative to the bounds:
 *   wbar = (w_i + w_j)/2 - (F(w_j) - F(w_i)).n / (2 lambda)
 * with the Euler flux F (Sec. 2.1).  The theorem places wbar in the bounds
 * of any stencil holding both states when lambda bounds the particle speeds
 * of the velocity domain; the remark after it uses the macroscopic wavespeed
 * estimate instead.  FP64.
 *
 *   states       [d+2][n_nodes] conserved node states.
 *   node_i, node_j [n_pairs] node ids (i on the element side, j across).
 *   normals      [d][n_pairs] unit normals pointing from i to j.
 *   lambda       [n_pairs] wavespeed bounds, or NULL for
 *                max(|U_i.n| + sqrt(gamma theta_i), |U_j.n| + sqrt(gamma theta_j)).
 *   bounds, elem [2(d+2)][n_elem] bounds and [n_pairs] element of each pair
 *                (both NULL to skip the check).
 *   bar          out [d+2][n_pairs]; NaN for KBL_RS_BAD_INPUT pairs.
 *   pair_status  out [n_pairs] KBL_RS_* bits, or NULL.
 * All arrays are device memory; only params->gamma is used.
 */
kbl_status kbl_riemann_states(const kbl_params* params, int32_t dim, int64_t n_pairs,
                              int64_t n_nodes, const double* states, const int32_t* node_i,
                              const int32_t* node_j, const double* normals,
                              const double* lambda, const double* bounds, const int32_t* elem,
                              int64_t n_elem, double* bar, uint32_t* pair_status, void* stream);

/*
 * kbl_backward_workspace_bytes - device workspace kbl_bounds_limit_backward
 * needs: the recomputed forward bounds and status, dJ/dbounds, and one
 * gradient slot per (stencil entry, node, variable): 8 (d+2) nnz n_s bytes
 * plus O(n_elem).
 */
size_t kbl_backward_workspace_bytes(int32_t dim, int64_t n_elem, int32_t n_s, int64_t nnz);

/*
 * kbl_bounds_limit_backward - gradient of J(limited) where
 *   limited = kbl_limit(solution, kbl_compute_bounds(states)),
 * given G = dJ/dlimited: the derivatives of eq. fminmax, relaxed, rhobounds,
 * Ebounds, mmbounds, mpbounds, truncdomain (Sec. 3.3-3.7), the density floor
 * and eq. alpha, limiter, pmin, doublelimit (Sec. 3.4, 3.8).  The min/max
 * distributions are recomputed, never stored; at a tie the max envelopes
 * take their subgradient at the first winning state in stencil order and
 * the min envelopes at the last, the limiter at its active term (first node
 * and variable on ties); alpha capped at 1, alpha set to 0 by the epsilon
 * rule, alpha_P = 0 and a floored rho_min are constants.  In
 * KBL_GRID_STENCIL mode the velocity box moves with its extreme states and
 * that dependence is differentiated too.  The bounds' adjoint is linear in
 * dJ/dbounds, which is zero for every element whose limiter binds no bound:
 * such elements contribute exactly zero and their distributions are not
 * recomputed, so the cost grows with the number of limited elements.
 *
 * params->precision selects the forward being differentiated:
 *   KBL_PREC_FP64   everything in FP64;
 *   KBL_PREC_MIXED_* (d = 2) the mixed-precision forward: the limiter
 *                backward runs on its bounds, and the envelope winners come
 *                from FP32 envelopes of the same shifted, box-centred
 *                coefficients; shares, moments and all chain-rule terms stay
 *                FP64.
 *
 *   states, rowptr, cols, vgrid, solution, node_weights: as in the forward
 *                calls.  The stencil relation must be symmetric (e lists J
 *                iff J lists e), which face- and vertex-neighbour stencils
 *                are; elements that violate it get KBL_ST_ASYMMETRIC.
 *   fwd_bounds   [2(d+2)][n_elem] the bounds kbl_compute_bounds returned for
 *                these inputs and params, or NULL to recompute them in the
 *                workspace.
 *   fwd_status   the status that call returned (required with fwd_bounds).
 *   grad_limited [d+2][n_elem*n_s] dJ/dlimited.
 *   grad_states  out [d+2][n_elem*n_s] dJ/dstates (through the bounds).
 *   grad_solution out [d+2][n_elem*n_s] dJ/dsolution (through the limiter).
 *   grad_bounds  out [2(d+2)][n_elem] dJ/dbounds, or NULL.
 *   elem_status  out [n_elem] forward bounds status plus KBL_ST_ASYMMETRIC /
 *                KBL_ST_TOO_LARGE, or NULL.
 *   workspace    device memory of at least kbl_backward_workspace_bytes().
 * Element-level stencils and params->flags == 0 only (KBL_ERR_UNSUPPORTED
 * otherwise).  Stencils of more than 256 states contribute no state gradient
 * (KBL_ST_TOO_LARGE).  Grids: up to 64 x 64 (d = 2), 2048 nodes (d = 1);
 * d = 3 is not built.  The result is bitwise deterministic.
 */
kbl_status kbl_bounds_limit_backward(const kbl_params* params, int32_t dim, int64_t n_elem,
                                     int32_t n_s, int64_t nnz, const double* states,
                                     const int32_t* rowptr, const int32_t* cols,
                                     const kbl_vgrid* vgrid, const double* fwd_bounds,
                                     const uint32_t* fwd_status, const double* solution,
                                     const double* node_weights, const double* grad_limited,
                                     double* grad_states, double* grad_solution,
                                     double* grad_bounds, uint32_t* elem_status,
                                     void* workspace, size_t workspace_bytes, void* stream);

/* Size of the device array that kbl_bounds_limit_backward_noalloc uses as its
 * workspace: 256 MiB per GPU. */
#define KBL_NOALLOC_WORKSPACE_BYTES (256ull * 1024ull * 1024ull)

/*
 * kbl_bounds_limit_backward_noalloc - kbl_bounds_limit_backward for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and errors as kbl_bounds_limit_backward, without the workspace: it uses a
 * file-scope device array of KBL_NOALLOC_WORKSPACE_BYTES instead, one per
 * GPU (its device address is looked up on the first call on each device;
 * the array is held until the process ends).  Nothing is allocated: no
 * hipMalloc, hipFree or allocating library call.
 *   Returns KBL_ERR_WORKSPACE, before touching the device, when
 *   kbl_backward_workspace_bytes() for these sizes exceeds
 *   KBL_NOALLOC_WORKSPACE_BYTES (the quad mesh of 256 x 256 elements with
 *   16 nodes and 5-element stencils needs about 172 MB).
 * Every call on a GPU shares that GPU's array and leaves its contents there;
 * every part of it that a call reads is written earlier in the same call, so
 * nothing needs clearing.  Calls that overlap on one GPU (different streams
 * or host threads) race on the array: serialise them.
 */
kbl_status kbl_bounds_limit_backward_noalloc(const kbl_params* params, int32_t dim,
                                             int64_t n_elem, int32_t n_s, int64_t nnz,
                                             const double* states, const int32_t* rowptr,
                                             const int32_t* cols, const kbl_vgrid* vgrid,
                                             const double* fwd_bounds,
                                             const uint32_t* fwd_status,
                                             const double* solution,
                                             const double* node_weights,
                                             const double* grad_limited, double* grad_states,
                                             double* grad_solution, double* grad_bounds,
                                             uint32_t* elem_status, void* stream);

/*
 * kbl_status_summary - how many entries of a status array carry each bit:
 * counts[b] = number of i < n with bit b of elem_status[i] set, for b = 0..31.
 * Works on any array of KBL_ST_* words (kbl_compute_bounds, kbl_limit, the
 * backward) or of the KBL_RS_* pair bits of kbl_riemann_states; it is the
 * on-demand reduction of the per-element conditions of Sec. 3.4 and 3.8
 * (epsilon rule, pressure step, alpha_P = 0, ...) that the calls themselves
 * only flag, without a host synchronisation.
 *   elem_status  [n] device status words (may be NULL when n == 0).
 *   counts       out [32] device uint64, overwritten (zeros when n == 0).
 * Enqueues two small launches on `stream` (clear, then count) and returns;
 * allocates nothing.  KBL_ERR_ARG for n < 0, counts == NULL, or
 * elem_status == NULL with n > 0.  The counts are exact and independent of
 * scheduling.
 */
kbl_status kbl_status_summary(const uint32_t* elem_status, int64_t n, uint64_t* counts,
                              void* stream);

/* Human-readable text for a status code (static storage). */
const char* kbl_status_string(kbl_status s);

/* Library version as 10000*major + 100*minor + patch. */
int32_t kbl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KBL_H */

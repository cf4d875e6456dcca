/*
 * kbl_fr1d.h - one-dimensional flux reconstruction (FR) Euler solver with the
 * kinetic bounds and squeeze limiter applied after every Runge-Kutta stage:
 * the numerical setup of Sec. 5 in one dimension, on AMD Instinct MI355X
 * (gfx950).
 *
 * Scheme (Sec. 5):
 *  - p + 1 Gauss-Legendre solution points per element; the two element ends
 *    are the flux points (an open node set).
 *  - Huynh's flux reconstruction with the DG correction functions (the left
 *    and right Radau polynomials): the discontinuous flux is the Lagrange
 *    interpolant of the point fluxes, corrected at each end to the common
 *    interface flux.
 *  - Common interface flux: HLLC (Toro, Spruce and Speares), wave speeds
 *    S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).
 *  - Three-stage third-order SSP Runge-Kutta (Shu-Osher form).  Every stage
 *    follows the overview of Sec. 3.9: the bounds of
 *    kbl_compute_bounds_nodes are taken from the stage's input state over the
 *    node stencil S (the element's solution points and end values plus the
 *    neighbours' end values on the shared faces); after the update,
 *    kbl_limit limits the element into those bounds over V (its solution
 *    points and end values, the end values with zero mean weight).
 *
 * State layout.  A state array is FP64 [3][n_tot * (p + 3)]: row v holds
 * variable v (rho, m, E).  Element e owns columns e*(p+3) .. e*(p+3)+p+2:
 * its p + 1 solution points, then its left and right end values.  With
 * periodic boundaries n_tot = n_elem; with Dirichlet boundaries two constant
 * ghost elements follow (n_tot = n_elem + 2; element n_elem holds the left
 * state, n_elem + 1 the right one).  Callers write the solution points of
 * the n_elem real elements; the library writes the end values and ghosts.
 *
 * Conventions as in kbl.h: device pointers owned by the caller, work
 * enqueued on `stream`, argument errors returned before any launch.  The
 * workspace is scratch: its contents do not carry over between calls.
 */
#ifndef KBL_FR1D_H
#define KBL_FR1D_H

#include "kbl.h"

#ifdef __cplusplus
extern "C" {
#endif

#define KBL_FR_PERIODIC   0
#define KBL_FR_DIRICHLET  1
#define KBL_FR_MAX_DEGREE 7

typedef struct {
    int32_t p;          /* polynomial degree, 1..KBL_FR_MAX_DEGREE */
    int32_t bc;         /* KBL_FR_PERIODIC or KBL_FR_DIRICHLET */
    int64_t n_elem;     /* uniform elements of [x0, x1], >= 2 */
    double  x0, x1;     /* domain, x1 > x0 */
    double  left[3];    /* Dirichlet: conserved ghost state on the left (rho, m, E) */
    double  right[3];   /* Dirichlet: conserved ghost state on the right */
    int32_t limit;      /* 1: bounds + squeeze limiter after every stage; 0: none */
    int32_t reserved;   /* 0 */
} kbl_fr1d;

/* Columns of a state array: n_tot * (p + 3); 0 for an invalid cfg. */
int64_t kbl_fr1d_columns(const kbl_fr1d* cfg);

/* Workspace bytes of kbl_fr1d_step / kbl_fr1d_limit; 0 for an invalid cfg. */
size_t kbl_fr1d_workspace_bytes(const kbl_fr1d* cfg);

/*
 * kbl_fr1d_rhs - the FR residual du/dt at the solution points.
 *   U   [3][columns] state (solution points read; end values and ghosts not).
 *   R   out [3][n_elem*(p+1)], element-major solution points.
 * A non-admissible end value (rho <= 0 or P < 0) gives NaN residuals in the
 * elements that use it.
 */
kbl_status kbl_fr1d_rhs(const kbl_fr1d* cfg, double gamma, const double* U, double* R,
                        void* stream);

/*
 * kbl_fr1d_limit - repair of initial data: writes the end values and ghosts
 * of U from its solution points; an element whose polynomial has a
 * non-admissible node value (rho <= 0 or P <= 0 at a solution point or end
 * value, as the end values of discontinuous data can) is limited in place
 * into the bounds of the solution points of the element and its two face
 * neighbours.  Every other element is left unchanged (its status reads
 * KBL_ST_BAD_BOUNDS).  params and vgrid as for kbl_compute_bounds (d = 1;
 * the paper uses k = 8 and 2048 velocity nodes in 1D).  elem_status: out
 * [n_tot] limiter status or NULL.  Does nothing but the end values and
 * ghosts when cfg->limit is 0.
 */
kbl_status kbl_fr1d_limit(const kbl_fr1d* cfg, const kbl_params* params, const kbl_vgrid* vgrid,
                          double* U, void* workspace, size_t workspace_bytes,
                          uint32_t* elem_status, void* stream);

/*
 * kbl_fr1d_step - one SSP-RK3 step of size dt with the stage limiting above
 * (when cfg->limit is 1).  U is updated in place; its end values need not
 * be current on entry and are on return.  elem_status: the last stage's
 * limiter status, or NULL.
 */
kbl_status kbl_fr1d_step(const kbl_fr1d* cfg, const kbl_params* params, const kbl_vgrid* vgrid,
                         double dt, double* U, void* workspace, size_t workspace_bytes,
                         uint32_t* elem_status, void* stream);

/*
 * kbl_fr1d_max_speed - max over the solution points of |u| + c, written to
 * one device double `out` (NaN if any solution point is not admissible);
 * the time step of a CFL condition follows from it.
 */
kbl_status kbl_fr1d_max_speed(const kbl_fr1d* cfg, double gamma, const double* U, double* out,
                              void* stream);

/*
 * kbl_fr1d_cfl_dt - the CFL time step in device memory, for runs with no
 * host synchronisation per step (e.g. batches of steps captured in a HIP
 * graph).  tdt: device (t, dt).  Reads t = tdt[0]; writes
 * dt = min(cfl h / ((2p + 1) max(|u| + c)), t_end - t) (0 once t >= t_end)
 * to tdt[1] and the time after the step to tdt[0] (exactly t_end on the
 * last step).  Both become NaN when a solution point is not admissible.
 */
kbl_status kbl_fr1d_cfl_dt(const kbl_fr1d* cfg, double gamma, const double* U, double cfl,
                           double t_end, double* tdt, void* stream);

/*
 * kbl_fr1d_step_dev - kbl_fr1d_step with dt read from device memory (tdt[1],
 * as written by kbl_fr1d_cfl_dt) when the kernels run.  Enqueues the same
 * work; allocates nothing and does not synchronise, so it can be captured.
 */
kbl_status kbl_fr1d_step_dev(const kbl_fr1d* cfg, const kbl_params* params,
                             const kbl_vgrid* vgrid, const double* tdt, double* U,
                             void* workspace, size_t workspace_bytes, uint32_t* elem_status,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KBL_FR1D_H */

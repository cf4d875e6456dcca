/*
 * Plain FP64 CPU oracle for kinetic maximum-principle bounds and the squeeze
 * limiter (Dzanic & Martinelli, "High-order limiting methods using maximum
 * principle bounds derived from the Boltzmann equation I: Euler equations").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test suite, the smoke check and the CPU-baseline leg of the bench
 * load.  The product library never links or calls it, and it shares no code,
 * header or constant with the HIP path.
 *
 * Everything is written the slow, literal way on purpose:
 *   - each stencil state's Maxwellian is evaluated in its direct form
 *     rho (2 pi theta)^(-d/2) exp(-|u-U|^2 / (2 theta))  (Sec. 2.2, eq. maxwell)
 *     at every velocity node, one exp per (state, node) pair;
 *   - the envelopes are min/max of those *values* (Sec. 3.3, eq. fminmax),
 *     relaxed by (1 -+ r) (Sec. 3.5, eq. relaxed);
 *   - the internal-energy part follows the reduced-distribution model of
 *     Sec. 3.6: g_I = (theta delta / 2) g_T with delta = 2/(gamma-1) - d, and
 *     f_I gets its own min/max envelope (the transported-scalar reading);
 *   - moments use a uniform trapezoid rule on a Cartesian velocity grid
 *     (Sec. 3.7) over a global box or the per-stencil box of eq. truncdomain
 *     (upper end read as max(U + k sqrt(theta)), i.e. k standard deviations
 *     on both sides);
 *   - sums are Neumaier-compensated;
 *   - the limiter is the coupled squeeze limiter of Sec. 3.4 (eq. alpha,
 *     eq. limiter, epsilon rule), followed by the pressure step of Sec. 3.8
 *     (eq. pmin, eq. doublelimit).
 * OpenMP parallelises over elements only; every element is computed by one
 * thread from start to end.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_ST_INADMISSIBLE 0x1u   /* a stencil state has rho<=0, P<=0 or is not finite */
#define OR_ST_RHO_FLOOR    0x2u   /* rho_min was raised to the density floor */
#define OR_ST_EPS_RULE     0x4u   /* some alpha_i was set to 0 by the epsilon rule */
#define OR_ST_LIMITED      0x8u   /* alpha_min < 1 */
#define OR_ST_PSTEP        0x10u  /* the pressure step fired */
#define OR_ST_PMEAN_FLOOR  0x20u  /* P(mean) <= pressure floor, alpha_P set to 0 */
#define OR_ST_MEAN_OUTSIDE 0x40u  /* element mean lies outside the bounds */
#define OR_ST_BAD_BOUNDS   0x80u  /* bounds not finite: element passed through */
#define OR_ST_BAD_STENCIL  0x100u /* stencil row empty or out of range: bounds are NaN */

#define OR_MAXV 4                 /* d+2 for d<=2 */

/* ---------------------------------------------------------------- helpers */

typedef struct { double s, c; } nsum;   /* Neumaier running sum */

static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_val(const nsum* a) { return a->s + a->c; }

/* Ideal-gas pressure from conserved variables (Sec. 2.1). */
static double pressure(int d, double gamma, const double* w) {
    double mm = 0.0;
    for (int j = 0; j < d; ++j) mm += w[1 + j] * w[1 + j];
    return (gamma - 1.0) * (w[d + 1] - 0.5 * mm / w[0]);
}

/* Internal degrees of freedom delta = 2/(gamma-1) - d (Sec. 3.6). */
double oracle_delta(int d, double gamma) {
    return (2.0 - d * (gamma - 1.0)) / (gamma - 1.0);
}

/* Primitive state of one node: rho, U, theta = P/rho (Sec. 2.1, 2.2). */
typedef struct { double rho, U[2], theta; int ok; } prim_t;

static prim_t node_prim(int d, double gamma, const double* states, int64_t n_nodes, int64_t node) {
    prim_t p;
    double w[OR_MAXV];
    for (int v = 0; v < d + 2; ++v) w[v] = states[(int64_t)v * n_nodes + node];
    p.rho = w[0];
    p.U[0] = p.U[1] = 0.0;
    for (int j = 0; j < d; ++j) p.U[j] = w[1 + j] / w[0];
    double P = pressure(d, gamma, w);
    p.theta = P / w[0];
    p.ok = 1;
    for (int v = 0; v < d + 2; ++v) if (!isfinite(w[v])) p.ok = 0;
    if (!(w[0] > 0.0) || !(P > 0.0) || !isfinite(p.theta)) p.ok = 0;
    return p;
}

/* Maxwellian value of one state at one velocity node (Sec. 2.2, eq. maxwell). */
static double maxwellian(int d, const prim_t* s, const double* u) {
    double c2 = 0.0;
    for (int j = 0; j < d; ++j) { double c = u[j] - s->U[j]; c2 += c * c; }
    return s->rho * pow(2.0 * M_PI * s->theta, -0.5 * d) * exp(-c2 / (2.0 * s->theta));
}

/* ------------------------------------------------------------ bounds core */

/*
 * Bounds of one element.  out[0..d+1] = (rho, m_1..m_d, E)_min,
 * out[d+2..2d+3] = (rho, m, E)_max.  Returns status bits.
 * grid_mode 0: box [lo, hi] given; 1: box from the stencil with factor k.
 */
static unsigned element_bounds(int d, double gamma, double r_fac, double rho_floor,
                               int grid_mode, const int* n, const double* lo_in,
                               const double* hi_in, double k, int n_s,
                               const double* states, int64_t n_elem, int64_t nnz,
                               const int* rowptr, const int* cols, int64_t e,
                               double* out) {
    const int nv = d + 2;
    const int64_t n_nodes = n_elem * n_s;
    const int row0 = rowptr[e], row1 = rowptr[e + 1];
    /* a row must be non-empty, inside [0, nnz] and name existing elements */
    int bad_row = (row0 < 0 || row1 <= row0 || row1 > nnz);
    for (int r = row0; !bad_row && r < row1; ++r)
        if (cols[r] < 0 || cols[r] >= n_elem) bad_row = 1;
    if (bad_row) {
        for (int v = 0; v < 2 * nv; ++v) out[v] = NAN;
        return OR_ST_BAD_STENCIL;
    }
    const int S = (row1 - row0) * n_s;
    prim_t* st = (prim_t*)malloc(sizeof(prim_t) * (size_t)S);
    unsigned status = 0;

    /* Step 1 of Sec. 3.9: collect the stencil states (CSR order, node order). */
    int s = 0;
    for (int r = row0; r < row1; ++r)
        for (int j = 0; j < n_s; ++j) {
            st[s] = node_prim(d, gamma, states, n_nodes, (int64_t)cols[r] * n_s + j);
            if (!st[s].ok) status |= OR_ST_INADMISSIBLE;
            ++s;
        }
    if (status & OR_ST_INADMISSIBLE) {
        for (int v = 0; v < 2 * nv; ++v) out[v] = NAN;
        free(st);
        return status;
    }

    const double delta = oracle_delta(d, gamma);

    /* Velocity box (Sec. 3.7, eq. truncdomain) and trapezoid spacing. */
    double lo[2] = {0, 0}, hi[2] = {0, 0}, h[2] = {0, 0};
    for (int j = 0; j < d; ++j) {
        if (grid_mode == 0) { lo[j] = lo_in[j]; hi[j] = hi_in[j]; }
        else {
            lo[j] = INFINITY; hi[j] = -INFINITY;
            for (int i = 0; i < S; ++i) {
                double sd = sqrt(st[i].theta);
                double a = st[i].U[j] - k * sd, b = st[i].U[j] + k * sd;
                if (a < lo[j]) lo[j] = a;
                if (b > hi[j]) hi[j] = b;
            }
        }
        h[j] = (hi[j] - lo[j]) / (double)(n[j] - 1);
    }

    nsum rmin = {0, 0}, rmax = {0, 0}, emin = {0, 0}, emax = {0, 0};
    nsum mmin[2] = {{0, 0}, {0, 0}}, mmax[2] = {{0, 0}, {0, 0}};
    const int n1 = (d == 2) ? n[1] : 1;

    for (int ty = 0; ty < n1; ++ty)
        for (int tx = 0; tx < n[0]; ++tx) {
            int t[2] = {tx, ty};
            double u[2] = {0, 0}, M = 1.0;
            for (int j = 0; j < d; ++j) {
                u[j] = lo[j] + t[j] * h[j];
                double wt = (t[j] == 0 || t[j] == n[j] - 1) ? 0.5 : 1.0;
                M *= h[j] * wt;
            }
            /* Step 2 of Sec. 3.9: min/max distribution over the stencil
             * (eq. fminmax) for the translational part g and the internal
             * part g_I = (theta delta/2) g (Sec. 3.6). */
            double fTmin = INFINITY, fTmax = -INFINITY, fImin = INFINITY, fImax = -INFINITY;
            for (int i = 0; i < S; ++i) {
                double g = maxwellian(d, &st[i], u);
                double gI = 0.5 * st[i].theta * delta * g;
                if (g < fTmin) fTmin = g;
                if (g > fTmax) fTmax = g;
                if (gI < fImin) fImin = gI;
                if (gI > fImax) fImax = gI;
            }
            /* Relaxation of the envelopes (eq. relaxed). */
            fTmin *= (1.0 - r_fac); fImin *= (1.0 - r_fac);
            fTmax *= (1.0 + r_fac); fImax *= (1.0 + r_fac);

            double half_u2 = 0.0;
            for (int j = 0; j < d; ++j) half_u2 += 0.5 * u[j] * u[j];
            /* Density and energy: non-negative invariants (eq. rhobounds, Ebounds),
             * energy invariant extended by the internal part (Sec. 3.6). */
            nsum_add(&rmin, M * fTmin);
            nsum_add(&rmax, M * fTmax);
            nsum_add(&emin, M * (half_u2 * fTmin + fImin));
            nsum_add(&emax, M * (half_u2 * fTmax + fImax));
            /* Momentum: split by the sign of u_j (eq. mmbounds, mpbounds). */
            for (int j = 0; j < d; ++j) {
                if (u[j] < 0.0) {
                    nsum_add(&mmin[j], M * u[j] * fTmax);
                    nsum_add(&mmax[j], M * u[j] * fTmin);
                } else {
                    nsum_add(&mmin[j], M * u[j] * fTmin);
                    nsum_add(&mmax[j], M * u[j] * fTmax);
                }
            }
        }

    out[0] = nsum_val(&rmin);
    out[nv] = nsum_val(&rmax);
    for (int j = 0; j < d; ++j) { out[1 + j] = nsum_val(&mmin[j]); out[nv + 1 + j] = nsum_val(&mmax[j]); }
    out[d + 1] = nsum_val(&emin);
    out[nv + d + 1] = nsum_val(&emax);
    /* Step 3 of Sec. 3.9: density floor (Sec. 3.8). */
    if (out[0] < rho_floor) { out[0] = rho_floor; status |= OR_ST_RHO_FLOOR; }
    free(st);
    return status;
}

/*
 * Bounds for a selection of elements.
 *   states  [d+2][n_elem*n_s] conserved variables, SoA, element-major nodes
 *   rowptr  [n_elem+1], cols[nnz]: element stencils (element ids); bad rows
 *           are flagged OR_ST_BAD_STENCIL with NaN bounds
 *   elems   [n_sel] element ids to evaluate (NULL: all, n_sel = n_elem)
 *   bounds  out [2(d+2)][n_sel]: rows (rho, m.., E)_min then (rho, m.., E)_max
 *   status  out [n_sel] or NULL
 * Returns 0, or -1 on bad arguments.
 */
int oracle_bounds(int d, double gamma, double r_fac, double rho_floor,
                  int grid_mode, const int* n, const double* lo, const double* hi, double k,
                  int64_t n_elem, int n_s, int64_t nnz, const double* states,
                  const int* rowptr, const int* cols,
                  const int64_t* elems, int64_t n_sel,
                  double* bounds, unsigned* status) {
    if (d < 1 || d > 2 || n_s < 1 || !(gamma > 1.0)) return -1;
    for (int j = 0; j < d; ++j) if (n[j] < 2) return -1;
    if (oracle_delta(d, gamma) < 0.0) return -1;
    const int nv = d + 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_sel; ++q) {
        int64_t e = elems ? elems[q] : q;
        double out[2 * OR_MAXV];
        unsigned st = element_bounds(d, gamma, r_fac, rho_floor, grid_mode, n, lo, hi, k,
                                     n_s, states, n_elem, nnz, rowptr, cols, e, out);
        for (int v = 0; v < 2 * nv; ++v) bounds[(int64_t)v * n_sel + q] = out[v];
        if (status) status[q] = st;
    }
    return 0;
}

/* ------------------------------------------------------------------ limiter */

/*
 * Coupled squeeze limiter (Sec. 3.4) and pressure step (Sec. 3.8) of one
 * element.  w[v*n_s + j]: the element's nodal solution; b: its bounds;
 * out: limited nodal solution; alpha[0] = alpha_min, alpha[1] = alpha_P.
 */
static unsigned element_limit(int d, double gamma, double p_floor, double eps, int n_s,
                              const double* w, const double* b, const double* c,
                              double* out, double* alpha) {
    const int nv = d + 2;
    unsigned status = 0;
    for (int v = 0; v < 2 * nv; ++v)
        if (!isfinite(b[v])) status |= OR_ST_BAD_BOUNDS;
    if (status) {
        memcpy(out, w, sizeof(double) * (size_t)(nv * n_s));
        alpha[0] = 1.0; alpha[1] = 1.0;
        return status;
    }

    /* Element mean with positive weights (Assumption (iii)(a) of Sec. 4). */
    double wbar[OR_MAXV];
    nsum csum = {0, 0};
    for (int j = 0; j < n_s; ++j) nsum_add(&csum, c[j]);
    for (int v = 0; v < nv; ++v) {
        nsum acc = {0, 0};
        for (int j = 0; j < n_s; ++j) nsum_add(&acc, c[j] * w[v * n_s + j]);
        wbar[v] = nsum_val(&acc) / nsum_val(&csum);
    }
    for (int v = 0; v < nv; ++v)
        if (wbar[v] < b[v] || wbar[v] > b[nv + v]) status |= OR_ST_MEAN_OUTSIDE;

    /* Limiting factor per component (eq. alpha) with the epsilon rule. */
    double amin = 1.0;
    for (int v = 0; v < nv; ++v) {
        double wmax = -INFINITY, wmin = INFINITY;
        for (int j = 0; j < n_s; ++j) {
            if (w[v * n_s + j] > wmax) wmax = w[v * n_s + j];
            if (w[v * n_s + j] < wmin) wmin = w[v * n_s + j];
        }
        double dp = wmax - wbar[v], dm = wmin - wbar[v];
        double av;
        if (fabs(dm) < eps || fabs(dp) < eps) { av = 0.0; status |= OR_ST_EPS_RULE; }
        else {
            av = 1.0;
            double ru = fabs((b[nv + v] - wbar[v]) / dp);
            double rl = fabs((b[v] - wbar[v]) / dm);
            if (ru < av) av = ru;
            if (rl < av) av = rl;
        }
        if (av < amin) amin = av;
    }
    if (amin < 1.0) status |= OR_ST_LIMITED;

    /* Coupled blend towards the mean (eq. limiter). */
    for (int v = 0; v < nv; ++v)
        for (int j = 0; j < n_s; ++j)
            out[v * n_s + j] = wbar[v] + amin * (w[v * n_s + j] - wbar[v]);

    /* Pressure step (eq. pmin, eq. doublelimit). */
    double pmin = INFINITY;
    for (int j = 0; j < n_s; ++j) {
        double wn[OR_MAXV];
        for (int v = 0; v < nv; ++v) wn[v] = out[v * n_s + j];
        double P = pressure(d, gamma, wn);
        if (isnan(P)) P = -INFINITY;      /* an undefined pressure counts as below the floor */
        if (P < pmin) pmin = P;
    }
    double aP = 1.0;
    if (pmin < p_floor) {
        double pbar = pressure(d, gamma, wbar);
        status |= OR_ST_PSTEP;
        if (pbar > p_floor) aP = fabs((p_floor - pbar) / (pmin - pbar));
        else { aP = 0.0; status |= OR_ST_PMEAN_FLOOR; }
        for (int v = 0; v < nv; ++v)
            for (int j = 0; j < n_s; ++j)
                out[v * n_s + j] = wbar[v] + aP * (out[v * n_s + j] - wbar[v]);
    }
    alpha[0] = amin;
    alpha[1] = aP;
    return status;
}

/*
 * Limit a selection of elements.
 *   solution [d+2][n_elem*n_s]; bounds [2(d+2)][n_sel] (one column per
 *   selected element); c [n_s] positive weights;
 *   limited out [d+2][n_sel*n_s]; alpha out [2][n_sel]; status out [n_sel].
 */
int oracle_limit(int d, double gamma, double p_floor, double eps,
                 int64_t n_elem, int n_s, const double* solution,
                 const double* bounds, const double* c,
                 const int64_t* elems, int64_t n_sel,
                 double* limited, double* alpha, unsigned* status) {
    if (d < 1 || d > 2 || n_s < 1 || n_s > 4096 || !(gamma > 1.0)) return -1;
    for (int j = 0; j < n_s; ++j) if (!(c[j] > 0.0)) return -1;
    const int nv = d + 2;
    const int64_t n_nodes = n_elem * n_s;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n_sel; ++q) {
        int64_t e = elems ? elems[q] : q;
        double* w = (double*)malloc(sizeof(double) * (size_t)(nv * n_s));
        double* o = (double*)malloc(sizeof(double) * (size_t)(nv * n_s));
        double b[2 * OR_MAXV], al[2];
        for (int v = 0; v < nv; ++v)
            for (int j = 0; j < n_s; ++j) w[v * n_s + j] = solution[(int64_t)v * n_nodes + e * n_s + j];
        for (int v = 0; v < 2 * nv; ++v) b[v] = bounds[(int64_t)v * n_sel + q];
        unsigned st = element_limit(d, gamma, p_floor, eps, n_s, w, b, c, o, al);
        for (int v = 0; v < nv; ++v)
            for (int j = 0; j < n_s; ++j) limited[(int64_t)v * n_sel * n_s + q * n_s + j] = o[v * n_s + j];
        alpha[q] = al[0];
        alpha[n_sel + q] = al[1];
        if (status) status[q] = st;
        free(w); free(o);
    }
    return 0;
}

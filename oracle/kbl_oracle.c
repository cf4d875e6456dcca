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
 * Dimensions d = 1, 2, 3 (the backward: d <= 2).
 * Everything is written the slow, literal way on purpose:
 *   - each stencil state's Maxwellian is evaluated in its direct form
 *     rho (2 pi theta)^(-d/2) exp(-|u-U|^2 / (2 theta))  (Sec. 2.2, eq. maxwell)
 *     at every velocity node, one exp per (state, node) pair;
 *   - the envelopes are min/max of those *values* (Sec. 3.3, eq. fminmax),
 *     relaxed by (1 -+ r) (Sec. 3.5, eq. relaxed);
 *   - the internal-energy part follows the reduced-distribution model of
 *     Sec. 3.6: g_I = (theta delta / 2) g_T with delta = 2/(gamma-1) - d, and
 *     f_I gets its own min/max envelope (the transported-scalar reading);
 *     optionally (energy_mode 1) the energy integrand is taken per state
 *     instead, min/max over i of g_i (|u|^2/2 + theta_i delta/2);
 *   - moments use a uniform trapezoid rule on a Cartesian velocity grid
 *     (Sec. 3.7) over a global box or the per-stencil box of eq. truncdomain
 *     (upper end read as max(U + k sqrt(theta)), i.e. k standard deviations
 *     on both sides);
 *   - sums are Neumaier-compensated;
 *   - the limiter is the coupled squeeze limiter of Sec. 3.4 (eq. alpha,
 *     eq. limiter, epsilon rule), or its independent per-component form
 *     described there, followed by the pressure step of Sec. 3.8 (eq. pmin,
 *     eq. doublelimit);
 *   - a stencil lists source units: elements (n_s nodes each) or single
 *     nodes (n_s = 1), so node-level stencils such as the solution and
 *     flux points of Sec. 5 use the same code;
 *   - the Riemann-averaged state of two states across a face (Thm. 4.3 of
 *     Sec. 4) from the Euler fluxes, checked against an element's bounds.
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

#define OR_MAXV 5                 /* d+2 for d<=3 */

/* ---------------------------------------------------------------- helpers */

typedef struct { double s, c; } nsum;   /* Neumaier running sum */

static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_val(const nsum* a) { return a->s + a->c; }
/* adds the product a b, including its rounding error (by fma) */
static void nsum_add_prod(nsum* acc, double a, double b) {
    const double p = a * b;
    nsum_add(acc, p);
    acc->c += fma(a, b, -p);
}

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
typedef struct { double rho, U[3], theta; int ok; } prim_t;

static prim_t node_prim(int d, double gamma, const double* states, int64_t n_nodes, int64_t node) {
    prim_t p;
    double w[OR_MAXV];
    for (int v = 0; v < d + 2; ++v) w[v] = states[(int64_t)v * n_nodes + node];
    p.rho = w[0];
    p.U[0] = p.U[1] = p.U[2] = 0.0;
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
                               const double* states, int64_t n_src, int64_t nnz,
                               const int* rowptr, const int* cols, int64_t e,
                               int energy_mode, double* out) {
    const int nv = d + 2;
    const int64_t n_nodes = n_src * n_s;
    const int row0 = rowptr[e], row1 = rowptr[e + 1];
    /* a row must be non-empty, inside [0, nnz] and name existing source units */
    int bad_row = (row0 < 0 || row1 <= row0 || row1 > nnz);
    for (int r = row0; !bad_row && r < row1; ++r)
        if (cols[r] < 0 || cols[r] >= n_src) bad_row = 1;
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
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, h[3] = {0, 0, 0};
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
    nsum mmin[3] = {{0, 0}, {0, 0}, {0, 0}}, mmax[3] = {{0, 0}, {0, 0}, {0, 0}};
    const int n1 = (d >= 2) ? n[1] : 1;
    const int n2 = (d >= 3) ? n[2] : 1;

    for (int tz = 0; tz < n2; ++tz)
    for (int ty = 0; ty < n1; ++ty)
        for (int tx = 0; tx < n[0]; ++tx) {
            int t[3] = {tx, ty, tz};
            double u[3] = {0, 0, 0}, M = 1.0;
            for (int j = 0; j < d; ++j) {
                u[j] = lo[j] + t[j] * h[j];
                double wt = (t[j] == 0 || t[j] == n[j] - 1) ? 0.5 : 1.0;
                M *= h[j] * wt;
            }
            /* Step 2 of Sec. 3.9: min/max distribution over the stencil
             * (eq. fminmax) for the translational part g and the internal
             * part g_I = (theta delta/2) g (Sec. 3.6). */
            double half_u2 = 0.0;
            for (int j = 0; j < d; ++j) half_u2 += 0.5 * u[j] * u[j];
            double fTmin = INFINITY, fTmax = -INFINITY, fImin = INFINITY, fImax = -INFINITY;
            double eAmin = INFINITY, eAmax = -INFINITY;   /* per-state energy integrand */
            for (int i = 0; i < S; ++i) {
                double g = maxwellian(d, &st[i], u);
                double gI = 0.5 * st[i].theta * delta * g;
                double eA = g * (half_u2 + 0.5 * st[i].theta * delta);
                if (g < fTmin) fTmin = g;
                if (g > fTmax) fTmax = g;
                if (gI < fImin) fImin = gI;
                if (gI > fImax) fImax = gI;
                if (eA < eAmin) eAmin = eA;
                if (eA > eAmax) eAmax = eA;
            }
            /* Relaxation of the envelopes (eq. relaxed). */
            fTmin *= (1.0 - r_fac); fImin *= (1.0 - r_fac); eAmin *= (1.0 - r_fac);
            fTmax *= (1.0 + r_fac); fImax *= (1.0 + r_fac); eAmax *= (1.0 + r_fac);

            /* Density and energy: non-negative invariants (eq. rhobounds, Ebounds),
             * energy invariant extended by the internal part (Sec. 3.6): either
             * separate envelopes of g_T and g_I, or the envelope of the
             * per-state energy integrand. */
            nsum_add(&rmin, M * fTmin);
            nsum_add(&rmax, M * fTmax);
            if (energy_mode == 1) {
                nsum_add(&emin, M * eAmin);
                nsum_add(&emax, M * eAmax);
            } else {
                nsum_add(&emin, M * (half_u2 * fTmin + fImin));
                nsum_add(&emax, M * (half_u2 * fTmax + fImax));
            }
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
 *   states  [d+2][n_src*n_s] conserved variables, SoA, unit-major nodes
 *   rowptr  [n_elem+1], cols[nnz]: stencils listing source units (elements of
 *           n_s nodes, or single nodes with n_s = 1); bad rows are flagged
 *           OR_ST_BAD_STENCIL with NaN bounds
 *   elems   [n_sel] element ids to evaluate (NULL: all, n_sel = n_elem)
 *   energy_mode 0: separate g_T / g_I envelopes; 1: per-state integrand
 *   bounds  out [2(d+2)][n_sel]: rows (rho, m.., E)_min then (rho, m.., E)_max
 *   status  out [n_sel] or NULL
 * Returns 0, or -1 on bad arguments.
 */
int oracle_bounds(int d, double gamma, double r_fac, double rho_floor,
                  int grid_mode, const int* n, const double* lo, const double* hi, double k,
                  int64_t n_elem, int64_t n_src, int n_s, int64_t nnz, const double* states,
                  const int* rowptr, const int* cols,
                  const int64_t* elems, int64_t n_sel, int energy_mode,
                  double* bounds, unsigned* status) {
    if (d < 1 || d > 3 || n_s < 1 || !(gamma > 1.0)) return -1;
    if (energy_mode != 0 && energy_mode != 1) return -1;
    for (int j = 0; j < d; ++j) if (n[j] < 2) return -1;
    if (oracle_delta(d, gamma) < 0.0) return -1;
    const int nv = d + 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_sel; ++q) {
        int64_t e = elems ? elems[q] : q;
        double out[2 * OR_MAXV];
        unsigned st = element_bounds(d, gamma, r_fac, rho_floor, grid_mode, n, lo, hi, k,
                                     n_s, states, n_src, nnz, rowptr, cols, e, energy_mode, out);
        for (int v = 0; v < 2 * nv; ++v) bounds[(int64_t)v * n_sel + q] = out[v];
        if (status) status[q] = st;
    }
    return 0;
}

/* ------------------------------------------------------------------ limiter */

/*
 * Squeeze limiter (Sec. 3.4) and pressure step (Sec. 3.8) of one element.
 * w[v*n_s + j]: the element's nodal values (V); b: its bounds; c: mean
 * weights (zero for nodes that do not enter the mean, e.g. flux points);
 * out: limited nodal values; alpha[0] = alpha_min, alpha[1] = alpha_P.
 * independent = 0: every component blended with alpha_min (eq. limiter);
 * 1: each component blended with its own alpha_i.
 */
static unsigned element_limit(int d, double gamma, double p_floor, double eps, int n_s,
                              const double* w, const double* b, const double* c,
                              int independent, double* out, double* alpha) {
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
    double amin = 1.0, acomp[OR_MAXV];
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
        acomp[v] = av;
        if (av < amin) amin = av;
    }
    if (amin < 1.0) status |= OR_ST_LIMITED;

    /* Blend towards the mean: coupled (eq. limiter) or per component. */
    for (int v = 0; v < nv; ++v) {
        const double a = independent ? acomp[v] : amin;
        for (int j = 0; j < n_s; ++j)
            out[v * n_s + j] = wbar[v] + a * (w[v * n_s + j] - wbar[v]);
    }

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
 *   selected element); c [n_s] non-negative weights with a positive sum;
 *   independent: per-component blending instead of the coupled minimum;
 *   limited out [d+2][n_sel*n_s]; alpha out [2][n_sel]; status out [n_sel].
 */
int oracle_limit(int d, double gamma, double p_floor, double eps,
                 int64_t n_elem, int n_s, const double* solution,
                 const double* bounds, const double* c, int independent,
                 const int64_t* elems, int64_t n_sel,
                 double* limited, double* alpha, unsigned* status) {
    if (d < 1 || d > 3 || n_s < 1 || n_s > 4096 || !(gamma > 1.0)) return -1;
    double csum = 0.0;
    for (int j = 0; j < n_s; ++j) {
        if (!(c[j] >= 0.0) || !isfinite(c[j])) return -1;
        csum += c[j];
    }
    if (!(csum > 0.0)) return -1;
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
        unsigned st = element_limit(d, gamma, p_floor, eps, n_s, w, b, c, independent, o, al);
        for (int v = 0; v < nv; ++v)
            for (int j = 0; j < n_s; ++j) limited[(int64_t)v * n_sel * n_s + q * n_s + j] = o[v * n_s + j];
        alpha[q] = al[0];
        alpha[n_sel + q] = al[1];
        if (status) status[q] = st;
        free(w); free(o);
    }
    return 0;
}

/* --------------------------------------------------------------- backward */

/*
 * Analytic subgradient of J through the limiter and the bounds, written out
 * from the chain rule (a plain reference, not an efficient one).
 *
 * Forward chain per element e (Sec. 3.3-3.8): bounds b_e(states of S_e) and
 * limited nodes w~_e(solution_e, b_e).  Given G = dJ/dw~ for every node, this
 * returns dJ/dsolution (through the limiter) and dJ/dstates (through the
 * bounds of every element whose stencil holds the state).
 *
 * Conventions: ties of the envelopes go to the first state in stencil order
 * for a maximum and to the last for a minimum; other min/max ties pick the
 * first candidate (stencil order for the box ends, node order for extreme
 * nodes, variable order for alpha_min);
 * alpha capped at 1 or set to 0 by the epsilon rule is locally constant; a
 * floored rho_min is constant; the indicator u_j < 0 of the momentum split
 * contributes nothing because its integrand vanishes at u_j = 0.  In
 * per-stencil (STENCIL) grid mode the box ends follow the extreme states of
 * eq. truncdomain, so node positions and trapezoid weights carry gradient.
 */

/* Pressure gradient dP/dw for the ideal gas (Sec. 2.1). */
static void pressure_grad(int d, double gamma, const double* w, double* g) {
    double mm = 0.0;
    for (int j = 0; j < d; ++j) mm += w[1 + j] * w[1 + j];
    g[0] = (gamma - 1.0) * 0.5 * mm / (w[0] * w[0]);
    for (int j = 0; j < d; ++j) g[1 + j] = -(gamma - 1.0) * w[1 + j] / w[0];
    g[d + 1] = gamma - 1.0;
}

/*
 * Limiter backward of one element.  w, out as in element_limit; G = dJ/dout;
 * gw = dJ/dw (out), gb = dJ/db (out, 2nv).
 */
static void element_limit_backward(int d, double gamma, double p_floor, double eps, int n_s,
                                   const double* w, const double* b, const double* c,
                                   const double* G, double* gw, double* gb) {
    const int nv = d + 2;
    for (int i = 0; i < nv * n_s; ++i) gw[i] = 0.0;
    for (int i = 0; i < 2 * nv; ++i) gb[i] = 0.0;
    for (int v = 0; v < 2 * nv; ++v)
        if (!isfinite(b[v])) {           /* passed through unchanged */
            for (int i = 0; i < nv * n_s; ++i) gw[i] = G[i];
            return;
        }
    double csum = 0.0;
    for (int j = 0; j < n_s; ++j) csum += c[j];
    double wbar[OR_MAXV];
    for (int v = 0; v < nv; ++v) {
        double acc = 0.0;
        for (int j = 0; j < n_s; ++j) acc += c[j] * w[v * n_s + j];
        wbar[v] = acc / csum;
    }
    /* recompute alpha and which term set it */
    double amin = 1.0;
    int vstar = -1, upper = 0, jstar = -1;
    double dstar = 0.0;
    for (int v = 0; v < nv; ++v) {
        int jmax = 0, jmin = 0;
        for (int j = 1; j < n_s; ++j) {
            if (w[v * n_s + j] > w[v * n_s + jmax]) jmax = j;
            if (w[v * n_s + j] < w[v * n_s + jmin]) jmin = j;
        }
        double dp = w[v * n_s + jmax] - wbar[v], dm = w[v * n_s + jmin] - wbar[v];
        double av;
        int vv = -1, up = 0, jj = -1;
        double dd = 0.0;
        if (fabs(dm) < eps || fabs(dp) < eps) av = 0.0;      /* constant */
        else {
            av = 1.0;
            double ru = fabs((b[nv + v] - wbar[v]) / dp);
            double rl = fabs((b[v] - wbar[v]) / dm);
            if (ru < av) { av = ru; vv = v; up = 1; jj = jmax; dd = dp; }
            if (rl < av) { av = rl; vv = v; up = 0; jj = jmin; dd = dm; }
        }
        if (av < amin) { amin = av; vstar = vv; upper = up; jstar = jj; dstar = dd; }
    }
    double wt[OR_MAXV * 64];
    for (int v = 0; v < nv; ++v)
        for (int j = 0; j < n_s; ++j) wt[v * n_s + j] = wbar[v] + amin * (w[v * n_s + j] - wbar[v]);
    /* pressure step */
    double pmin = INFINITY;
    int jp = 0;
    for (int j = 0; j < n_s; ++j) {
        double wn[OR_MAXV];
        for (int v = 0; v < nv; ++v) wn[v] = wt[v * n_s + j];
        double P = pressure(d, gamma, wn);
        if (isnan(P)) P = -INFINITY;
        if (P < pmin) { pmin = P; jp = j; }
    }
    /* the element sums below (adjoints of the mean, of alpha_P and of alpha)
       can be small differences of large terms: they are compensated */
    double gwt[OR_MAXV * 64];      /* dJ/dw~ */
    nsum gwbar[OR_MAXV];
    for (int v = 0; v < OR_MAXV; ++v) gwbar[v].s = gwbar[v].c = 0.0;
    if (pmin < p_floor) {
        double pbar = pressure(d, gamma, wbar);
        if (pbar > p_floor) {
            double N = p_floor - pbar, D = pmin - pbar;
            double aP = fabs(N / D);
            double s = (N / D) >= 0 ? 1.0 : -1.0;
            nsum gaPs = {0.0, 0.0};
            for (int v = 0; v < nv; ++v)
                for (int j = 0; j < n_s; ++j) {
                    gwt[v * n_s + j] = aP * G[v * n_s + j];
                    /* w~ - wbar = alpha (w - wbar) by eq. limiter */
                    nsum_add_prod(&gaPs, G[v * n_s + j], amin * (w[v * n_s + j] - wbar[v]));
                    nsum_add_prod(&gwbar[v], 1.0 - aP, G[v * n_s + j]);
                }
            const double gaP = nsum_val(&gaPs);
            /* aP = s N / D: d aP = s (dN / D - N dD / D^2), dN = -dPbar, dD = dPmin - dPbar */
            double gPbar = gaP * s * (-1.0 / D + N / (D * D));
            double gPmin = gaP * s * (-N / (D * D));
            double gp[OR_MAXV];
            pressure_grad(d, gamma, wbar, gp);
            for (int v = 0; v < nv; ++v) nsum_add_prod(&gwbar[v], gPbar, gp[v]);
            double wn[OR_MAXV];
            for (int v = 0; v < nv; ++v) wn[v] = wt[v * n_s + jp];
            pressure_grad(d, gamma, wn, gp);
            for (int v = 0; v < nv; ++v) gwt[v * n_s + jp] += gPmin * gp[v];
        } else {
            /* alpha_P = 0: every node equals the mean */
            for (int v = 0; v < nv; ++v) {
                for (int j = 0; j < n_s; ++j) { gwt[v * n_s + j] = 0.0; nsum_add(&gwbar[v], G[v * n_s + j]); }
            }
        }
    } else {
        for (int i = 0; i < nv * n_s; ++i) gwt[i] = G[i];
    }
    /* w~ = wbar + alpha (w - wbar) */
    nsum galphas = {0.0, 0.0};
    for (int v = 0; v < nv; ++v)
        for (int j = 0; j < n_s; ++j) {
            gw[v * n_s + j] += amin * gwt[v * n_s + j];
            nsum_add_prod(&gwbar[v], 1.0 - amin, gwt[v * n_s + j]);
            nsum_add_prod(&galphas, gwt[v * n_s + j], w[v * n_s + j] - wbar[v]);
        }
    const double galpha = nsum_val(&galphas);
    if (vstar >= 0) {
        /* alpha = |(bnd - wbar) / dd|, dd = w[jstar] - wbar */
        const int v = vstar;
        double bnd = upper ? b[nv + v] : b[v];
        double r = (bnd - wbar[v]) / dstar;
        double s = r >= 0 ? 1.0 : -1.0;
        double g = galpha * s;
        double gbnd = g / dstar;
        double gdd = -g * (bnd - wbar[v]) / (dstar * dstar);
        if (upper) gb[nv + v] += gbnd; else gb[v] += gbnd;
        nsum_add(&gwbar[v], -gbnd);      /* from bnd - wbar */
        gw[v * n_s + jstar] += gdd;      /* dd = w[jstar] - wbar */
        nsum_add(&gwbar[v], -gdd);
    }
    /* wbar = sum c w / sum c */
    for (int v = 0; v < nv; ++v)
        for (int j = 0; j < n_s; ++j) gw[v * n_s + j] += nsum_val(&gwbar[v]) * c[j] / csum;
}

/*
 * Bounds backward of one element: given gb = dJ/db (2nv), accumulate dJ/dstates
 * into gstates (full [nv][n_nodes] array).
 */
static void element_bounds_backward(int d, double gamma, double r_fac, double rho_floor,
                                    int grid_mode, const int* n, const double* lo_in,
                                    const double* hi_in, double k, int n_s,
                                    const double* states, int64_t n_elem,
                                    const int* rowptr, const int* cols, int64_t e,
                                    const double* gb_in, double* gstates) {
    const int nv = d + 2;
    const int64_t n_nodes = n_elem * n_s;
    const int row0 = rowptr[e], row1 = rowptr[e + 1];
    const int S = (row1 - row0) * n_s;
    prim_t* st = (prim_t*)malloc(sizeof(prim_t) * (size_t)S);
    int64_t* node = (int64_t*)malloc(sizeof(int64_t) * (size_t)S);
    int s = 0;
    for (int r = row0; r < row1; ++r)
        for (int j = 0; j < n_s; ++j) {
            node[s] = (int64_t)cols[r] * n_s + j;
            st[s] = node_prim(d, gamma, states, n_nodes, node[s]);
            ++s;
        }
    double gb[2 * OR_MAXV];
    for (int i = 0; i < 2 * nv; ++i) gb[i] = gb_in[i];
    /* recompute rho_min to know whether the floor was active */
    double out[2 * OR_MAXV];
    element_bounds(d, gamma, r_fac, rho_floor, grid_mode, n, lo_in, hi_in, k, n_s, states,
                   n_elem, rowptr[n_elem], rowptr, cols, e, 0, out);
    if (out[0] == rho_floor) gb[0] = 0.0;
    const double delta = oracle_delta(d, gamma);

    double lo[2] = {0, 0}, hi[2] = {0, 0}, h[2] = {0, 0};
    int ilo[2] = {-1, -1}, ihi[2] = {-1, -1};
    for (int j = 0; j < d; ++j) {
        if (grid_mode == 0) { lo[j] = lo_in[j]; hi[j] = hi_in[j]; }
        else {
            lo[j] = INFINITY; hi[j] = -INFINITY;
            for (int i = 0; i < S; ++i) {
                double sd = sqrt(st[i].theta);
                double a = st[i].U[j] - k * sd, bb = st[i].U[j] + k * sd;
                if (a < lo[j]) { lo[j] = a; ilo[j] = i; }
                if (bb > hi[j]) { hi[j] = bb; ihi[j] = i; }
            }
        }
        h[j] = (hi[j] - lo[j]) / (double)(n[j] - 1);
    }
    /* per-state adjoints of (rho, U_1..U_d, theta) */
    double* gp = (double*)calloc((size_t)S * (size_t)nv, sizeof(double));
    double glo[2] = {0, 0}, ghi[2] = {0, 0};
    const double rm = 1.0 - r_fac, rp = 1.0 + r_fac;
    const int n1 = (d == 2) ? n[1] : 1;
    for (int ty = 0; ty < n1; ++ty)
        for (int tx = 0; tx < n[0]; ++tx) {
            int t[2] = {tx, ty};
            double u[2] = {0, 0}, M = 1.0;
            for (int j = 0; j < d; ++j) {
                u[j] = lo[j] + t[j] * h[j];
                M *= h[j] * ((t[j] == 0 || t[j] == n[j] - 1) ? 0.5 : 1.0);
            }
            /* the subgradient of a min/max of tied states may take any of
               them: a maximum goes to the first tied state in stencil order,
               a minimum to the last */
            int win[4] = {0, 0, 0, 0};     /* Tmin, Tmax, Imin, Imax */
            double fv[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
            for (int i = 0; i < S; ++i) {
                double g = maxwellian(d, &st[i], u);
                double gI = 0.5 * st[i].theta * delta * g;
                if (g <= fv[0]) { fv[0] = g; win[0] = i; }
                if (g > fv[1]) { fv[1] = g; win[1] = i; }
                if (gI <= fv[2]) { fv[2] = gI; win[2] = i; }
                if (gI > fv[3]) { fv[3] = gI; win[3] = i; }
            }
            double hu2 = 0.0;
            for (int j = 0; j < d; ++j) hu2 += 0.5 * u[j] * u[j];
            /* adjoint weight Phi of each envelope (J = sum M Phi f) and dPhi/du_j */
            double phi[4], dphi[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
            phi[0] = rm * (gb[0] + gb[d + 1] * hu2);
            phi[1] = rp * (gb[nv] + gb[nv + d + 1] * hu2);
            phi[2] = rm * gb[d + 1];
            phi[3] = rp * gb[nv + d + 1];
            for (int j = 0; j < d; ++j) {
                /* m_min = sum_{u<0} u f_max + sum_{u>=0} u f_min ; m_max swapped */
                double gmin = gb[1 + j], gmax = gb[nv + 1 + j];
                if (u[j] < 0.0) { phi[1] += rp * gmin * u[j]; phi[0] += rm * gmax * u[j];
                                  dphi[1][j] += rp * gmin; dphi[0][j] += rm * gmax; }
                else            { phi[0] += rm * gmin * u[j]; phi[1] += rp * gmax * u[j];
                                  dphi[0][j] += rm * gmin; dphi[1][j] += rp * gmax; }
                dphi[0][j] += rm * gb[d + 1] * u[j];
                dphi[1][j] += rp * gb[nv + d + 1] * u[j];
            }
            double Jt = 0.0, dJdu[2] = {0, 0};
            for (int env = 0; env < 4; ++env) {
                const prim_t* w = &st[win[env]];
                double f = fv[env];
                double wf = M * phi[env] * f;
                Jt += wf;
                double c2 = 0.0;
                for (int j = 0; j < d; ++j) { double cc = u[j] - w->U[j]; c2 += cc * cc; }
                /* d ln g / d(rho, U_j, theta) */
                double* a = gp + (size_t)win[env] * nv;
                a[0] += wf / w->rho;
                for (int j = 0; j < d; ++j) a[1 + j] += wf * (u[j] - w->U[j]) / w->theta;
                double dth = -0.5 * d / w->theta + 0.5 * c2 / (w->theta * w->theta);
                if (env >= 2) dth += 1.0 / w->theta;   /* g_I carries theta delta / 2 */
                a[d + 1] += wf * dth;
                for (int j = 0; j < d; ++j)
                    dJdu[j] += M * (dphi[env][j] * f - phi[env] * f * (u[j] - w->U[j]) / w->theta);
            }
            if (grid_mode == 1) {
                for (int j = 0; j < d; ++j) {
                    double fr = (double)t[j] / (double)(n[j] - 1);
                    /* u = lo + t h, h = (hi - lo)/(n-1), M proportional to h_j */
                    glo[j] += dJdu[j] * (1.0 - fr) - Jt / (h[j] * (n[j] - 1));
                    ghi[j] += dJdu[j] * fr + Jt / (h[j] * (n[j] - 1));
                }
            }
        }
    if (grid_mode == 1)
        for (int j = 0; j < d; ++j) {
            /* lo = U - k sqrt(theta), hi = U + k sqrt(theta) of the extreme states */
            double* a = gp + (size_t)ilo[j] * nv;
            a[1 + j] += glo[j];
            a[d + 1] += glo[j] * (-0.5 * k / sqrt(st[ilo[j]].theta));
            a = gp + (size_t)ihi[j] * nv;
            a[1 + j] += ghi[j];
            a[d + 1] += ghi[j] * (0.5 * k / sqrt(st[ihi[j]].theta));
        }
    /* (rho, U, theta) -> (rho, m, E) */
    for (int i = 0; i < S; ++i) {
        const prim_t* w = &st[i];
        const double* a = gp + (size_t)i * nv;
        double U2 = 0.0;
        for (int j = 0; j < d; ++j) U2 += w->U[j] * w->U[j];
        double g_rho = a[0] + a[d + 1] * ((gamma - 1.0) * 0.5 * U2 - w->theta) / w->rho;
        for (int j = 0; j < d; ++j) g_rho += a[1 + j] * (-w->U[j] / w->rho);
        gstates[node[i]] += g_rho;
        for (int j = 0; j < d; ++j)
            gstates[(int64_t)(1 + j) * n_nodes + node[i]] +=
                a[1 + j] / w->rho - a[d + 1] * (gamma - 1.0) * w->U[j] / w->rho;
        gstates[(int64_t)(d + 1) * n_nodes + node[i]] += a[d + 1] * (gamma - 1.0) / w->rho;
    }
    free(gp); free(st); free(node);
}

/*
 * Full backward: bounds from `states`, limiting of `solution`, G = dJ/dlimited.
 * Outputs (all elements): gsol = dJ/dsolution [nv][n_nodes], gstates =
 * dJ/dstates [nv][n_nodes], gbounds = dJ/dbounds [2nv][n_elem].
 * Elements with non-finite bounds pass G through and contribute nothing to
 * gstates.  Serial on purpose (gstates is accumulated across elements).
 */
int oracle_backward(int d, double gamma, double r_fac, double rho_floor, double p_floor,
                    double eps, int grid_mode, const int* n, const double* lo, const double* hi,
                    double k, int64_t n_elem, int n_s, const double* states, const int* rowptr,
                    const int* cols, const double* solution, const double* c, const double* G,
                    double* gsol, double* gstates, double* gbounds) {
    if (d < 1 || d > 2 || n_s < 1 || n_s > 64) return -1;
    const int nv = d + 2;
    const int64_t n_nodes = n_elem * n_s;
    for (int64_t i = 0; i < (int64_t)nv * n_nodes; ++i) gstates[i] = 0.0;
    double* bnd = (double*)malloc(sizeof(double) * 2 * nv * (size_t)(n_elem > 0 ? n_elem : 1));
    unsigned* st = (unsigned*)malloc(sizeof(unsigned) * (size_t)(n_elem > 0 ? n_elem : 1));
    oracle_bounds(d, gamma, r_fac, rho_floor, grid_mode, n, lo, hi, k, n_elem, n_elem, n_s,
                  rowptr[n_elem], states, rowptr, cols, NULL, n_elem, 0, bnd, st);
    double w[OR_MAXV * 64], g[OR_MAXV * 64], gw[OR_MAXV * 64], b[2 * OR_MAXV], gb[2 * OR_MAXV];
    for (int64_t e = 0; e < n_elem; ++e) {
        for (int v = 0; v < nv; ++v)
            for (int j = 0; j < n_s; ++j) {
                w[v * n_s + j] = solution[(int64_t)v * n_nodes + e * n_s + j];
                g[v * n_s + j] = G[(int64_t)v * n_nodes + e * n_s + j];
            }
        for (int v = 0; v < 2 * nv; ++v) b[v] = bnd[(int64_t)v * n_elem + e];
        element_limit_backward(d, gamma, p_floor, eps, n_s, w, b, c, g, gw, gb);
        for (int v = 0; v < nv; ++v)
            for (int j = 0; j < n_s; ++j) gsol[(int64_t)v * n_nodes + e * n_s + j] = gw[v * n_s + j];
        for (int v = 0; v < 2 * nv; ++v) gbounds[(int64_t)v * n_elem + e] = gb[v];
        if (st[e] & (OR_ST_INADMISSIBLE | OR_ST_BAD_STENCIL)) continue;
        element_bounds_backward(d, gamma, r_fac, rho_floor, grid_mode, n, lo, hi, k, n_s, states,
                                n_elem, rowptr, cols, e, gb, gstates);
    }
    free(bnd); free(st);
    return 0;
}

/* ------------------------------------------------ Riemann-averaged states */

/* Euler flux projected on the unit normal n (Sec. 2.1). */
static void euler_flux_n(int d, double gamma, const double* w, const double* n, double* f) {
    const double rho = w[0];
    const double P = pressure(d, gamma, w);
    double un = 0.0;
    for (int j = 0; j < d; ++j) un += (w[1 + j] / rho) * n[j];
    f[0] = rho * un;
    for (int j = 0; j < d; ++j) f[1 + j] = w[1 + j] * un + P * n[j];
    f[d + 1] = (w[d + 1] + P) * un;
}

/*
 * Riemann-averaged states of Thm. 4.3 for pairs of node states (i, j) with
 * unit normal n_ij pointing from i to j:
 *   wbar = (w_i + w_j)/2 - (F(w_j) - F(w_i)).n / (2 lambda),
 * lambda given per pair, or (lam == NULL) the wavespeed estimate of the
 * remark after the theorem, max over the two states of |U.n| + sqrt(gamma theta).
 *   states  [d+2][n_nodes]; ni, nj [n_pairs] node ids; normals [d][n_pairs]
 *   bounds  [2(d+2)][n_elem] and elem [n_pairs] (or NULL): bounds to test
 *   bar     out [d+2][n_pairs]; status out [n_pairs] (or NULL): bit v if
 *           wbar_v < w_min,v, bit 8+v if wbar_v > w_max,v, bit 16 if a node
 *           id is out of range or an input state is not admissible (wbar is
 *           then NaN)
 * Returns 0, or -1 on bad arguments.
 */
int oracle_riemann(int d, double gamma, int64_t n_pairs, int64_t n_nodes, const double* states,
                   const int* ni, const int* nj, const double* normals, const double* lam,
                   const double* bounds, const int* elem, int64_t n_elem,
                   double* bar, unsigned* status) {
    if (d < 1 || d > 3 || !(gamma > 1.0)) return -1;
    const int nv = d + 2;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n_pairs; ++q) {
        double wi[OR_MAXV], wj[OR_MAXV], fi[OR_MAXV], fj[OR_MAXV], n[3] = {0, 0, 0};
        unsigned st = 0;
        const int64_t a = ni[q], b = nj[q];
        int ok = a >= 0 && a < n_nodes && b >= 0 && b < n_nodes;
        prim_t pa, pb;
        if (ok) {
            for (int v = 0; v < nv; ++v) {
                wi[v] = states[(int64_t)v * n_nodes + a];
                wj[v] = states[(int64_t)v * n_nodes + b];
            }
            pa = node_prim(d, gamma, states, n_nodes, a);
            pb = node_prim(d, gamma, states, n_nodes, b);
            ok = pa.ok && pb.ok;
        }
        if (!ok) {
            for (int v = 0; v < nv; ++v) bar[(int64_t)v * n_pairs + q] = NAN;
            if (status) status[q] = 1u << 16;
            continue;
        }
        for (int j = 0; j < d; ++j) n[j] = normals[(int64_t)j * n_pairs + q];
        double l;
        if (lam) l = lam[q];
        else {
            double ua = 0.0, ub = 0.0;
            for (int j = 0; j < d; ++j) { ua += pa.U[j] * n[j]; ub += pb.U[j] * n[j]; }
            double sa = fabs(ua) + sqrt(gamma * pa.theta), sb = fabs(ub) + sqrt(gamma * pb.theta);
            l = sa > sb ? sa : sb;
        }
        euler_flux_n(d, gamma, wi, n, fi);
        euler_flux_n(d, gamma, wj, n, fj);
        for (int v = 0; v < nv; ++v) {
            const double w = 0.5 * (wi[v] + wj[v]) - (fj[v] - fi[v]) / (2.0 * l);
            bar[(int64_t)v * n_pairs + q] = w;
            if (bounds && elem) {
                const int64_t e = elem[q];
                if (e >= 0 && e < n_elem) {
                    if (w < bounds[(int64_t)v * n_elem + e]) st |= 1u << v;
                    if (w > bounds[(int64_t)(nv + v) * n_elem + e]) st |= 1u << (8 + v);
                }
            }
        }
        if (status) status[q] = st;
    }
    return 0;
}

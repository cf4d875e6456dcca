/*
 * Test driver for the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (built and run by tests/test_oracle_sanitizers.py; host code
 * only).  It calls every entry point of kbl_oracle.c on small seeded meshes,
 * including the degenerate inputs the oracle must reject or flag: rows that
 * leave the stencil arrays, element ids out of range, non-finite and
 * inadmissible states, empty inputs.  Exit status 0 and no sanitizer report
 * means every access stayed in bounds and no undefined behaviour occurred.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_bounds(int d, double gamma, double r_fac, double rho_floor, int grid_mode,
                  const int* n, const double* lo, const double* hi, double k, int64_t n_elem,
                  int64_t n_src, int n_s, int64_t nnz, const double* states, const int* rowptr,
                  const int* cols, const int64_t* elems, int64_t n_sel, int energy_mode,
                  double* bounds, unsigned* status);
int oracle_limit(int d, double gamma, double p_floor, double eps, int64_t n_elem, int n_s,
                 const double* solution, const double* bounds, const double* c, int independent,
                 const int64_t* elems, int64_t n_sel, double* limited, double* alpha,
                 unsigned* status);
int oracle_backward(int d, double gamma, double r_fac, double rho_floor, double p_floor,
                    double eps, int grid_mode, const int* n, const double* lo, const double* hi,
                    double k, int64_t n_elem, int n_s, const double* states, const int* rowptr,
                    const int* cols, const double* solution, const double* c, const double* G,
                    double* gsol, double* gstates, double* gbounds);
int oracle_riemann(int d, double gamma, int64_t n_pairs, int64_t n_nodes, const double* states,
                   const int* ni, const int* nj, const double* normals, const double* lam,
                   const double* bounds, const int* elem, int64_t n_elem, double* bar,
                   unsigned* status);
double oracle_delta(int d, double gamma);

static uint64_t rng_state = 240720966u;
static double urand(void) {   /* 53-bit uniform in [0, 1) from a 64-bit LCG */
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

/* conserved states of n_nodes nodes, d dimensions, SoA [d+2][n_nodes] */
static double* make_states(int d, int64_t n_nodes, double gamma) {
    double* w = (double*)malloc(sizeof(double) * (size_t)(d + 2) * (size_t)n_nodes);
    for (int64_t i = 0; i < n_nodes; ++i) {
        const double rho = 0.2 + 2.0 * urand(), p = 0.1 + 5.0 * urand();
        double ke = 0.0;
        w[i] = rho;
        for (int j = 0; j < d; ++j) {
            const double u = 2.0 * urand() - 1.0;
            w[(int64_t)(1 + j) * n_nodes + i] = rho * u;
            ke += 0.5 * rho * u * u;
        }
        w[(int64_t)(d + 1) * n_nodes + i] = p / (gamma - 1.0) + ke;
    }
    return w;
}

/* periodic Cartesian mesh of N^d elements, self + 2d face neighbours */
static void make_stencil(int d, int N, int** rowptr, int** cols, int64_t* n_elem) {
    int64_t ne = 1;
    for (int j = 0; j < d; ++j) ne *= N;
    const int per = 1 + 2 * d;
    *rowptr = (int*)malloc(sizeof(int) * (size_t)(ne + 1));
    *cols = (int*)malloc(sizeof(int) * (size_t)(ne * per));
    for (int64_t e = 0; e < ne; ++e) {
        (*rowptr)[e] = (int)(e * per);
        int64_t c[3] = {0, 0, 0}, r = e;
        for (int j = 0; j < d; ++j) { c[j] = r % N; r /= N; }
        (*cols)[e * per] = (int)e;
        for (int j = 0; j < d; ++j)
            for (int s = 0; s < 2; ++s) {
                int64_t cc[3] = {c[0], c[1], c[2]};
                cc[j] = (cc[j] + (s ? 1 : N - 1)) % N;
                int64_t id = 0;
                for (int q = d - 1; q >= 0; --q) id = id * N + cc[q];
                (*cols)[e * per + 1 + 2 * j + s] = (int)id;
            }
    }
    (*rowptr)[ne] = (int)(ne * per);
    *n_elem = ne;
}

static void run_dim(int d, int N, int n_s, const int* grid_n) {
    const double gamma = 1.4;
    int *rowptr, *cols;
    int64_t n_elem;
    make_stencil(d, N, &rowptr, &cols, &n_elem);
    const int64_t n_nodes = n_elem * n_s, nnz = rowptr[n_elem];
    const int nv = d + 2;
    double* st = make_states(d, n_nodes, gamma);
    double* sol = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)n_nodes);
    for (int64_t i = 0; i < (int64_t)nv * n_nodes; ++i) sol[i] = st[i] * (1.0 + 0.05 * (urand() - 0.5));
    double* c = (double*)malloc(sizeof(double) * (size_t)n_s);
    for (int j = 0; j < n_s; ++j) c[j] = 0.5 + urand();
    double* b = (double*)malloc(sizeof(double) * 2 * (size_t)nv * (size_t)n_elem);
    unsigned* bs = (unsigned*)malloc(sizeof(unsigned) * (size_t)n_elem);
    const double lo[3] = {-4, -4, -4}, hi[3] = {4, 4, 4};
    for (int mode = 0; mode < 2; ++mode)
        for (int em = 0; em < 2; ++em) {
            CHECK(oracle_bounds(d, gamma, 1e-3, 1e-12, mode, grid_n, lo, hi, 4.0, n_elem, n_elem,
                                n_s, nnz, st, rowptr, cols, NULL, n_elem, em, b, bs) == 0);
            for (int64_t e = 0; e < n_elem; ++e) {
                CHECK(bs[e] == 0 || bs[e] == 0x2u);
                CHECK(b[e] > 0.0 && b[(int64_t)nv * n_elem + e] >= b[e]);
            }
        }
    /* a selection of elements, ids given in any order */
    int64_t sel[3] = {n_elem - 1, 0, n_elem / 2};
    double bsel[2 * 5 * 3];
    unsigned ssel[3];
    CHECK(oracle_bounds(d, gamma, 0.0, 1e-12, 1, grid_n, lo, hi, 4.0, n_elem, n_elem, n_s, nnz, st,
                        rowptr, cols, sel, 3, 0, bsel, ssel) == 0);
    /* limiter: coupled and independent, all elements and a selection */
    double* lim = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)n_nodes);
    double* al = (double*)malloc(sizeof(double) * 2 * (size_t)n_elem);
    unsigned* ls = (unsigned*)malloc(sizeof(unsigned) * (size_t)n_elem);
    CHECK(oracle_bounds(d, gamma, 1e-3, 1e-12, 1, grid_n, lo, hi, 4.0, n_elem, n_elem, n_s, nnz,
                        st, rowptr, cols, NULL, n_elem, 0, b, bs) == 0);
    for (int ind = 0; ind < 2; ++ind) {
        CHECK(oracle_limit(d, gamma, 1e-12, 1e-13, n_elem, n_s, sol, b, c, ind, NULL, n_elem, lim,
                           al, ls) == 0);
        for (int64_t e = 0; e < n_elem; ++e) CHECK(al[e] >= 0.0 && al[e] <= 1.0);
    }
    double lsel[5 * 64 * 3], asel[6];
    CHECK(oracle_limit(d, gamma, 1e-12, 1e-13, n_elem, n_s, sol, bsel, c, 0, sel, 3, lsel, asel,
                       ssel) == 0);
    /* non-finite bounds: passed through */
    b[0] = NAN;
    CHECK(oracle_limit(d, gamma, 1e-12, 1e-13, n_elem, n_s, sol, b, c, 0, NULL, n_elem, lim, al,
                       ls) == 0);
    CHECK(ls[0] & 0x80u);
    /* backward (d <= 2) */
    if (d <= 2) {
        double* G = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)n_nodes);
        double* gsol = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)n_nodes);
        double* gst = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)n_nodes);
        double* gb = (double*)malloc(sizeof(double) * 2 * (size_t)nv * (size_t)n_elem);
        for (int64_t i = 0; i < (int64_t)nv * n_nodes; ++i) G[i] = urand() - 0.5;
        for (int mode = 0; mode < 2; ++mode)
            CHECK(oracle_backward(d, gamma, 1e-3, 1e-12, 1e-12, 1e-13, mode, grid_n, lo, hi, 4.0,
                                  n_elem, n_s, st, rowptr, cols, sol, c, G, gsol, gst, gb) == 0);
        free(G); free(gsol); free(gst); free(gb);
    }
    /* Riemann-averaged states of node pairs, with and without bounds */
    const int64_t np = 17;
    int ni[17], nj[17], pe[17];
    double* nrm = (double*)malloc(sizeof(double) * (size_t)d * (size_t)np);
    double bar[5 * 17], lam[17];
    unsigned rs[17];
    for (int64_t q = 0; q < np; ++q) {
        ni[q] = (int)(urand() * (double)n_nodes);
        nj[q] = (int)(urand() * (double)n_nodes);
        pe[q] = ni[q] / n_s;
        lam[q] = 10.0;
        double s = 0.0;
        for (int j = 0; j < d; ++j) { nrm[j * np + q] = urand() - 0.5; s += nrm[j * np + q] * nrm[j * np + q]; }
        for (int j = 0; j < d; ++j) nrm[j * np + q] /= sqrt(s);
    }
    ni[3] = -1;          /* out of range: flagged, NaN */
    nj[5] = (int)n_nodes;
    CHECK(oracle_riemann(d, gamma, np, n_nodes, st, ni, nj, nrm, NULL, b, pe, n_elem, bar, rs) == 0);
    CHECK(rs[3] & (1u << 16));
    CHECK(rs[5] & (1u << 16));
    CHECK(oracle_riemann(d, gamma, np, n_nodes, st, ni, nj, nrm, lam, NULL, NULL, 0, bar, NULL) == 0);
    /* degenerate stencils: row past nnz, bad column, non-finite and inadmissible states */
    int* rp2 = (int*)malloc(sizeof(int) * (size_t)(n_elem + 1));
    int* cl2 = (int*)malloc(sizeof(int) * (size_t)nnz);
    memcpy(rp2, rowptr, sizeof(int) * (size_t)(n_elem + 1));
    memcpy(cl2, cols, sizeof(int) * (size_t)nnz);
    cl2[1] = (int)n_elem + 7;
    cl2[rp2[1] + 1] = -3;
    st[n_s] = NAN;                                  /* node 0 of element 1 */
    st[(int64_t)(d + 1) * n_nodes + 2 * n_s] = -1.0; /* negative energy in element 2 */
    rp2[n_elem] = (int)nnz + 5;                     /* last row runs past nnz */
    CHECK(oracle_bounds(d, gamma, 1e-3, 1e-12, 1, grid_n, lo, hi, 4.0, n_elem, n_elem, n_s, nnz,
                        st, rp2, cl2, NULL, n_elem, 0, b, bs) == 0);
    CHECK(bs[0] & 0x100u);
    CHECK(bs[n_elem - 1] & 0x100u);
    CHECK(isnan(b[0]));
    /* empty input */
    CHECK(oracle_bounds(d, gamma, 1e-3, 1e-12, 1, grid_n, lo, hi, 4.0, 0, 0, n_s, 0, st, rowptr,
                        cols, NULL, 0, 0, b, bs) == 0);
    CHECK(oracle_limit(d, gamma, 1e-12, 1e-13, 0, n_s, sol, b, c, 0, NULL, 0, lim, al, ls) == 0);
    /* argument errors */
    CHECK(oracle_bounds(d, 1.0, 1e-3, 1e-12, 1, grid_n, lo, hi, 4.0, n_elem, n_elem, n_s, nnz, st,
                        rowptr, cols, NULL, n_elem, 0, b, bs) == -1);
    CHECK(oracle_limit(d, gamma, 1e-12, 1e-13, n_elem, 0, sol, b, c, 0, NULL, n_elem, lim, al,
                       ls) == -1);
    free(rp2); free(cl2); free(nrm); free(lim); free(al); free(ls);
    free(st); free(sol); free(c); free(b); free(bs); free(rowptr); free(cols);
}

int main(void) {
    const int g1[3] = {97, 2, 2}, g2[3] = {13, 17, 2}, g3[3] = {7, 6, 5};
    CHECK(fabs(oracle_delta(2, 1.4) - 3.0) < 1e-12);
    run_dim(1, 6, 4, g1);
    run_dim(2, 3, 9, g2);
    run_dim(3, 2, 8, g3);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: ok\n");
    return 0;
}

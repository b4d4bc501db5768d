/*
 * oracle_check.c -- drives every entry point of oracle/oracle.c on small,
 * ragged and degenerate grids for a host AddressSanitizer / UndefinedBehavior
 * Sanitizer build (tests/test_sanitizers.py compiles and runs it). Besides
 * the sanitizers' own checks it asserts properties fixed by the operator's
 * definition, so a run that only "completes" without them still fails:
 *   - A applied to the ones vector gives 6 minus the number of in-grid
 *     neighbours, i.e. the number of the point's boundary faces;
 *   - the variable-coefficient operator with k = c everywhere is c A;
 *   - the compressed-row form of A gives the matrix-free product up to the
 *     summation order;
 *   - the two PCG forms and the compressed-row PCG converge, their solutions'
 *     FP64 residuals meet the tolerance, and thread counts do not change bits;
 *   - a stored matrix with a non-positive diagonal is refused.
 * Exit status 0 on success; the first failed check prints and exits 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_threads(void);
void oracle_set_threads(int n);
void oracle_stencil(int nx, int ny, int nz, const double *x, double *y);
void oracle_vstencil(int nx, int ny, int nz, const double *kc, const double *u, double *y);
void oracle_vdiag(int nx, int ny, int nz, const double *kc, double *d);
void oracle_axpy(int64_t n, double a, const double *x, const double *y, double *z);
double oracle_dot(int64_t n, const double *x, const double *y);
void oracle_csr_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val,
                     const double *x, double *y);
int oracle_pcg(int nx, int ny, int nz, const double *kc, const double *b, double *x, double rtol,
               int maxit, double *hist, int *iters, double *relres);
int oracle_csr_pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, const double *b,
                   double *x, double rtol, int maxit, double *hist, int *iters, double *relres);
int oracle_pcg_sr(int nx, int ny, int nz, const double *kc, const double *b, double *x, double rtol,
                  int maxit, double *hist, int *iters, double *relres);
void oracle_residual(int nx, int ny, int nz, const double *kc, const double *b, const double *x,
                     double *r, double *norm, double *amax); /* norm = ||b - A x||_2 */

#define CHECK(cond, ...)                                                    \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "oracle_check: %s:%d: ", __FILE__, __LINE__);   \
            fprintf(stderr, __VA_ARGS__);                                   \
            fputc('\n', stderr);                                            \
            exit(1);                                                        \
        }                                                                   \
    } while (0)

/* splitmix64 (Steele, Lea and Flood, OOPSLA 2014): a value in [-1, 1). */
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform(void)
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

/* Exactly-sized heap arrays (at least one element, so that empty grids still
 * hand the oracle valid pointers), so that ASan sees any access past the end. */
static double *vec(int64_t n) { return calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static int boundary_faces(int nx, int ny, int nz, int i, int j, int k)
{
    return (i == 0) + (i == nx - 1) + (j == 0) + (j == ny - 1) + (k == 0) + (k == nz - 1);
}

/* The seven-point matrix in compressed-row form, columns in increasing order. */
static void build_csr(int nx, int ny, int nz, int64_t **rowptr, int32_t **col, double **val)
{
    int64_t n = (int64_t)nx * ny * nz;
    *rowptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    *col = malloc(sizeof(int32_t) * (size_t)(7 * (n > 0 ? n : 1)));
    *val = malloc(sizeof(double) * (size_t)(7 * (n > 0 ? n : 1)));
    int64_t e = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t p = ((int64_t)k * ny + j) * nx + i;
                (*rowptr)[p] = e;
                const int64_t nb[7] = {k > 0 ? p - (int64_t)nx * ny : -1, j > 0 ? p - nx : -1, i > 0 ? p - 1 : -1, p,
                                       i < nx - 1 ? p + 1 : -1, j < ny - 1 ? p + nx : -1,
                                       k < nz - 1 ? p + (int64_t)nx * ny : -1};
                for (int t = 0; t < 7; ++t)
                    if (nb[t] >= 0) {
                        (*col)[e] = (int32_t)nb[t];
                        (*val)[e] = nb[t] == p ? 6.0 : -1.0;
                        ++e;
                    }
            }
    (*rowptr)[n] = e;
}

static void check_operators(int nx, int ny, int nz)
{
    int64_t n = (int64_t)nx * ny * nz;
    double *one = vec(n), *y = vec(n), *u = vec(n), *kc = vec(n), *y2 = vec(n), *d = vec(n), *z = vec(n);
    for (int64_t p = 0; p < n; ++p) {
        one[p] = 1.0;
        u[p] = uniform();
        kc[p] = 2.5;
    }
    oracle_stencil(nx, ny, nz, one, y);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int64_t p = ((int64_t)k * ny + j) * nx + i;
                CHECK(y[p] == boundary_faces(nx, ny, nz, i, j, k), "A 1 at (%d,%d,%d) of %dx%dx%d", i, j, k, nx, ny,
                      nz);
            }
    oracle_stencil(nx, ny, nz, u, y);
    oracle_vstencil(nx, ny, nz, kc, u, y2);
    oracle_vdiag(nx, ny, nz, kc, d);
    for (int64_t p = 0; p < n; ++p) {
        CHECK(fabs(y2[p] - 2.5 * y[p]) <= 1e-12 * (1.0 + fabs(y[p])), "A_k with k = 2.5 at %lld", (long long)p);
        CHECK(d[p] == 15.0, "diagonal of A_k with k = 2.5 at %lld", (long long)p);
    }
    int64_t *rowptr;
    int32_t *col;
    double *val;
    build_csr(nx, ny, nz, &rowptr, &col, &val);
    oracle_csr_spmv(n, rowptr, col, val, u, y2);
    /* equal up to the summation order: within 8 ulps of sum |a_pq u_q| (<= 12) */
    for (int64_t p = 0; p < n; ++p)
        CHECK(fabs(y2[p] - y[p]) <= 8 * 0x1.0p-52 * 12.0, "compressed-row product at %lld", (long long)p);
    oracle_axpy(n, -0.5, u, one, z);
    double s = oracle_dot(n, z, one), ref = 0.0;
    for (int64_t p = 0; p < n; ++p) ref += 1.0 - 0.5 * u[p];
    CHECK(fabs(s - ref) <= 1e-12 * (1.0 + fabs(ref)), "dot of the axpy: %g vs %g", s, ref);
    free(rowptr); free(col); free(val);
    free(one); free(y); free(u); free(kc); free(y2); free(d); free(z);
}

static void check_solvers(int nx, int ny, int nz, int variable)
{
    int64_t n = (int64_t)nx * ny * nz;
    const int maxit = 2000;
    const double rtol = 1e-10;
    double *b = vec(n), *x = vec(n), *x2 = vec(n), *kc = variable ? vec(n) : NULL, *r = vec(n);
    double *hist = vec(maxit + 1);
    for (int64_t p = 0; p < n; ++p) {
        b[p] = uniform();
        if (kc) kc[p] = exp(2.0 * uniform());
    }
    for (int form = 0; form < 2; ++form) {
        int iters = -1, iters2 = -1;
        double rel = -1.0, rel2 = -1.0, nr, amax, nb2 = oracle_dot(n, b, b);
        memset(x, 0, sizeof(double) * (size_t)n);
        memset(x2, 0, sizeof(double) * (size_t)n);
        oracle_set_threads(1);
        int st = form ? oracle_pcg_sr(nx, ny, nz, kc, b, x, rtol, maxit, hist, &iters, &rel)
                      : oracle_pcg(nx, ny, nz, kc, b, x, rtol, maxit, hist, &iters, &rel);
        oracle_set_threads(3);
        int st2 = form ? oracle_pcg_sr(nx, ny, nz, kc, b, x2, rtol, maxit, NULL, &iters2, &rel2)
                       : oracle_pcg(nx, ny, nz, kc, b, x2, rtol, maxit, NULL, &iters2, &rel2);
        CHECK(st == 0 && st2 == 0, "PCG form %d on %dx%dx%d: status %d / %d", form, nx, ny, nz, st, st2);
        CHECK(iters == iters2 && rel == rel2 && memcmp(x, x2, sizeof(double) * (size_t)n) == 0,
              "PCG form %d: thread count changed the result", form);
        oracle_residual(nx, ny, nz, kc, b, x, r, &nr, &amax);
        CHECK(nr <= 10 * rtol * sqrt(nb2), "PCG form %d: true residual %g", form, nr / sqrt(nb2));
    }
    if (!variable) {
        int64_t *rowptr;
        int32_t *col;
        double *val;
        int iters = -1;
        double rel = -1.0;
        build_csr(nx, ny, nz, &rowptr, &col, &val);
        memset(x2, 0, sizeof(double) * (size_t)n);
        int st = oracle_csr_pcg(n, rowptr, col, val, b, x2, rtol, maxit, hist, &iters, &rel);
        CHECK(st == 0, "compressed-row PCG status %d", st);
        double nr, amax, nb2 = oracle_dot(n, b, b);
        oracle_residual(nx, ny, nz, NULL, b, x2, r, &nr, &amax);
        CHECK(nr <= 10 * rtol * sqrt(nb2), "compressed-row PCG: true residual %g", nr / sqrt(nb2));
        /* a non-positive diagonal is refused before any iteration */
        for (int64_t e = rowptr[0]; e < rowptr[1]; ++e)
            if (col[e] == 0) val[e] = -1.0;
        st = oracle_csr_pcg(n, rowptr, col, val, b, x2, rtol, maxit, hist, &iters, &rel);
        CHECK(st == 4, "non-positive diagonal: status %d, expected breakdown", st);
        free(rowptr); free(col); free(val);
    }
    free(b); free(x); free(x2); free(kc); free(r); free(hist);
}

int main(void)
{
    CHECK(oracle_threads() >= 1, "thread count");
    static const int shapes[][3] = {{1, 1, 1}, {2, 1, 1}, {1, 3, 1}, {5, 3, 7}, {17, 9, 4}, {8, 8, 8}, {33, 2, 3}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        check_operators(shapes[s][0], shapes[s][1], shapes[s][2]);
    /* empty grids and vectors */
    check_operators(0, 4, 4);
    CHECK(oracle_dot(0, NULL, NULL) == 0.0, "empty dot");
    /* a dot over more than one reduction chunk */
    {
        int64_t n = 3 * 65536 + 17;
        double *a = vec(n), *c = vec(n);
        for (int64_t i = 0; i < n; ++i) { a[i] = (double)(i % 7); c[i] = 1.0; }
        double ref = 0.0;
        for (int64_t i = 0; i < n; ++i) ref += (double)(i % 7);
        CHECK(oracle_dot(n, a, c) == ref, "chunked dot");
        free(a); free(c);
    }
    check_solvers(1, 1, 1, 0);
    check_solvers(6, 5, 4, 0);
    check_solvers(6, 5, 4, 1);
    check_solvers(13, 7, 3, 1);
    /* b = 0: x = 0 at once */
    {
        double b[8] = {0}, x[8] = {1, 2, 3, 4, 5, 6, 7, 8}, hist[4];
        int iters = -1;
        double rel = -1.0;
        CHECK(oracle_pcg(2, 2, 2, NULL, b, x, 1e-8, 3, hist, &iters, &rel) == 0 && iters == 0 && x[7] == 0.0,
              "zero right-hand side");
    }
    puts("oracle_check: ok");
    return 0;
}

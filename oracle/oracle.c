/*
 * oracle.c -- plain FP64 CPU reference for the Jacobi-PCG hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it. It shares no code with the HIP library.
 *
 * What it computes (the paper's Sec. VII: PCG for a 3D seven-point
 * finite-difference operator with zero Dirichlet boundaries, applied
 * matrix-free, with a Jacobi preconditioner):
 *   - the constant-coefficient operator (Ax)_p = 6 x_p - sum of the six
 *     face neighbours, neighbours outside the grid read as 0 (Sec. VI and
 *     Sec. VII; weights 6/-1 with no h^2 scaling);
 *   - the variable-coefficient operator (A_k u)_p = sum_f k_f (u_p - u_nb),
 *     k_f the harmonic mean of the two cell values, k_f = k_p on a boundary
 *     face, u = 0 outside, and its diagonal D_p = sum_f k_f;
 *   - axpy, dot (Sec. IV, Sec. V: element-wise update and global sum);
 *   - SpMV of a general sparse matrix in compressed-row form (Sec. VII-A's
 *     GPU comparison system builds CG from norm, dot, axpy and SpMV);
 *   - Jacobi-preconditioned CG in the Hestenes-Stiefel form (Saad,
 *     Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 9.1),
 *     stopping on the recursive residual relative to ||b||, and the same
 *     method with one global reduction per iteration (Chronopoulos-Gear).
 *
 * Arrays are C-order [nz][ny][nx], x contiguous. All arithmetic is FP64.
 * Reductions use a fixed order (contiguous chunks summed left to right, chunk
 * sums added in index order), so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_NOCONV 3
#define ORACLE_BREAKDOWN 4
#define ORACLE_NOMEM 5

#define CHUNK 65536

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Use n threads in the parallel loops from now on (n >= 1); the reductions
 * keep their fixed order, so results do not depend on it. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static inline double nb_val(const double *x, int nx, int ny, int nz, int i, int j, int k)
{
    if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz)
        return 0.0;
    return x[((int64_t)k * ny + j) * nx + i];
}

/* y = A x, constant coefficients: diagonal 6, six face neighbours -1. */
void oracle_stencil(int nx, int ny, int nz, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double s = 6.0 * x[((int64_t)k * ny + j) * nx + i];
                s -= nb_val(x, nx, ny, nz, i - 1, j, k);
                s -= nb_val(x, nx, ny, nz, i + 1, j, k);
                s -= nb_val(x, nx, ny, nz, i, j - 1, k);
                s -= nb_val(x, nx, ny, nz, i, j + 1, k);
                s -= nb_val(x, nx, ny, nz, i, j, k - 1);
                s -= nb_val(x, nx, ny, nz, i, j, k + 1);
                y[((int64_t)k * ny + j) * nx + i] = s;
            }
}

static const int FACE[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

/* Face coefficient between cell p (value kp) and the cell across face f;
 * returns kp on a boundary face and sets *inside accordingly. */
static inline double face_k(const double *kc, int nx, int ny, int nz, int i, int j, int k, int f,
                            int *inside)
{
    double kp = kc[((int64_t)k * ny + j) * nx + i];
    int a = i + FACE[f][0], b = j + FACE[f][1], c = k + FACE[f][2];
    if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz) {
        *inside = 0;
        return kp;
    }
    *inside = 1;
    double kq = kc[((int64_t)c * ny + b) * nx + a];
    return 2.0 * kp * kq / (kp + kq);
}

/* y = A_k u, variable coefficients (harmonic-mean faces, k_f = k_p on the boundary). */
void oracle_vstencil(int nx, int ny, int nz, const double *kc, const double *u, double *y)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double up = u[((int64_t)k * ny + j) * nx + i];
                double s = 0.0;
                for (int f = 0; f < 6; ++f) {
                    int inside;
                    double kf = face_k(kc, nx, ny, nz, i, j, k, f, &inside);
                    double un = inside ? nb_val(u, nx, ny, nz, i + FACE[f][0], j + FACE[f][1],
                                                k + FACE[f][2])
                                       : 0.0;
                    s += kf * (up - un);
                }
                y[((int64_t)k * ny + j) * nx + i] = s;
            }
}

/* d = diag(A_k): the sum of the six face coefficients. */
void oracle_vdiag(int nx, int ny, int nz, const double *kc, double *d)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int f = 0; f < 6; ++f) {
                    int inside;
                    s += face_k(kc, nx, ny, nz, i, j, k, f, &inside);
                }
                d[((int64_t)k * ny + j) * nx + i] = s;
            }
}

/* z = a x + y */
void oracle_axpy(int64_t n, double a, const double *x, const double *y, double *z)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        z[i] = a * x[i] + y[i];
}

/* sum_i x_i y_i in a fixed order. */
double oracle_dot(int64_t n, const double *x, const double *y)
{
    int64_t nc = (n + CHUNK - 1) / CHUNK;
    if (nc == 0)
        return 0.0;
    double *part = (double *)malloc(sizeof(double) * (size_t)nc);
    if (!part)
        return NAN;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t lo = c * CHUNK, hi = lo + CHUNK < n ? lo + CHUNK : n;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i)
            s += x[i] * y[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nc; ++c)
        s += part[c];
    free(part);
    return s;
}

/*
 * y = A x for a general sparse matrix in compressed-row form: row i holds the
 * entries val[k] at columns col[k] for rowptr[i] <= k < rowptr[i+1], and
 * y_i is their sum of val[k] * x[col[k]], taken in storage order. This is the
 * SpMV of the GPU comparison system in Sec. VII-A (which stores the operator
 * in a sliced-ELLPACK format); compressed rows are the plain definition.
 */
void oracle_csr_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *col, const double *val,
                     const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

static void apply_op(int nx, int ny, int nz, const double *kc, const double *x, double *y)
{
    if (kc)
        oracle_vstencil(nx, ny, nz, kc, x, y);
    else
        oracle_stencil(nx, ny, nz, x, y);
}

/*
 * Jacobi-PCG (Saad Alg. 9.1 with M = D):
 *   r = b - A x0; if ||b|| = 0 then x = 0 and stop;
 *   z = D^-1 r; p = z; rho = r.z
 *   for k = 1..maxit:
 *     q = A p; sigma = p.q; breakdown if sigma <= 0 or not finite
 *     alpha = rho / sigma; x += alpha p; r -= alpha q
 *     stop when ||r|| <= rtol ||b||   (recursive residual, tested before z)
 *     z = D^-1 r; rho' = r.z; beta = rho'/rho; rho = rho'; p = z + beta p
 *
 * kc: cell coefficients (NULL for the constant operator, D = 6 I).
 * x: in = x0, out = final iterate. hist (optional, maxit+1 entries) receives
 * ||r_k|| / ||b|| for k = 0..iters. *iters = number of A p products.
 * Returns ORACLE_OK, ORACLE_NOCONV (maxit reached, last iterate kept) or
 * ORACLE_BREAKDOWN.
 */
/* The operator of a solve: the grid operators (kc NULL or cell coefficients)
 * or a compressed-row matrix. */
typedef struct {
    int nx, ny, nz;
    const double *kc;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
} op_t;

static void op_apply(const op_t *op, int64_t n, const double *x, double *y)
{
    if (op->rowptr)
        oracle_csr_spmv(n, op->rowptr, op->col, op->val, x, y);
    else
        apply_op(op->nx, op->ny, op->nz, op->kc, x, y);
}

/* Jacobi-PCG as above for an operator with inverse diagonal dinv. */
static int pcg_core(const op_t *op, int64_t n, const double *dinv, const double *b, double *x, double rtol,
                    int maxit, double *hist, int *iters, double *relres)
{
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    if (!r || !z || !p || !q) {
        free(r); free(z); free(p); free(q);
        return ORACLE_NOMEM;
    }
    int status = ORACLE_OK;
    *iters = 0;
    double nb = sqrt(oracle_dot(n, b, b));
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * n);
        *relres = 0.0;
        if (hist)
            hist[0] = 0.0;
        goto done;
    }
    op_apply(op, n, x, q);
    for (int64_t i = 0; i < n; ++i)
        r[i] = b[i] - q[i];
    double rn = sqrt(oracle_dot(n, r, r));
    if (hist)
        hist[0] = rn / nb;
    *relres = rn / nb;
    if (rn <= rtol * nb)
        goto done;
    for (int64_t i = 0; i < n; ++i)
        z[i] = dinv[i] * r[i];
    memcpy(p, z, sizeof(double) * n);
    double rho = oracle_dot(n, r, z);
    status = ORACLE_NOCONV;
    for (int k = 1; k <= maxit; ++k) {
        op_apply(op, n, p, q);
        double sigma = oracle_dot(n, p, q);
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            status = ORACLE_BREAKDOWN;
            break;
        }
        double alpha = rho / sigma;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        *iters = k;
        rn = sqrt(oracle_dot(n, r, r));
        *relres = rn / nb;
        if (hist)
            hist[k] = rn / nb;
        if (!isfinite(rn)) {
            status = ORACLE_BREAKDOWN;
            break;
        }
        if (rn <= rtol * nb) {
            status = ORACLE_OK;
            break;
        }
        for (int64_t i = 0; i < n; ++i)
            z[i] = dinv[i] * r[i];
        double rho_new = oracle_dot(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
    }
done:
    free(r); free(z); free(p); free(q);
    return status;
}

int oracle_pcg(int nx, int ny, int nz, const double *kc, const double *b, double *x, double rtol,
               int maxit, double *hist, int *iters, double *relres)
{
    int64_t n = (int64_t)nx * ny * nz;
    double *dinv = malloc(sizeof(double) * n);
    if (!dinv)
        return ORACLE_NOMEM;
    if (kc) {
        oracle_vdiag(nx, ny, nz, kc, dinv);
        for (int64_t i = 0; i < n; ++i)
            dinv[i] = 1.0 / dinv[i];
    } else {
        for (int64_t i = 0; i < n; ++i)
            dinv[i] = 1.0 / 6.0;
    }
    op_t op = {nx, ny, nz, kc, NULL, NULL, NULL};
    int status = pcg_core(&op, n, dinv, b, x, rtol, maxit, hist, iters, relres);
    free(dinv);
    return status;
}

/*
 * Jacobi-PCG as oracle_pcg for a square compressed-row matrix (the CG of the
 * GPU comparison system in Sec. VII-A runs on a stored sparse matrix). The
 * diagonal D_i is the sum of row i's entries in column i; a row whose D_i is
 * not positive gives ORACLE_BREAKDOWN before any iteration.
 */
int oracle_csr_pcg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, const double *b,
                   double *x, double rtol, int maxit, double *hist, int *iters, double *relres)
{
    double *dinv = malloc(sizeof(double) * (n > 0 ? n : 1));
    if (!dinv)
        return ORACLE_NOMEM;
    *iters = 0;
    *relres = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i)
                d += val[k];
        if (!(d > 0.0)) {
            free(dinv);
            return ORACLE_BREAKDOWN;
        }
        dinv[i] = 1.0 / d;
    }
    op_t op = {0, 0, 0, NULL, rowptr, col, val};
    int status = pcg_core(&op, n, dinv, b, x, rtol, maxit, hist, iters, relres);
    free(dinv);
    return status;
}

/*
 * Jacobi-preconditioned CG with one global reduction per iteration, in the
 * form of Chronopoulos and Gear (J. Comput. Appl. Math. 25 (1989), the s = 1
 * case of their s-step CG): the search direction's product s = A p is
 * carried by a recurrence, so the two inner products of an iteration are
 * taken together on the new residual. In exact arithmetic its iterates are
 * those of oracle_pcg. With M = D^-1:
 *
 *   r0 = b - A x0, u0 = M r0, w0 = A u0,
 *   gamma0 = r0.u0, delta0 = w0.u0, alpha0 = gamma0 / delta0, beta0 = 0;
 *   iteration i = 0, 1, ...:
 *     p_i = u_i + beta_i p_{i-1};   s_i = w_i + beta_i s_{i-1}   (p, s = 0 before)
 *     x_{i+1} = x_i + alpha_i p_i;  r_{i+1} = r_i - alpha_i s_i
 *     stop when ||r_{i+1}|| <= rtol ||b||
 *     u_{i+1} = M r_{i+1};  w_{i+1} = A u_{i+1}
 *     gamma_{i+1} = r_{i+1}.u_{i+1};  delta_{i+1} = w_{i+1}.u_{i+1}
 *     beta_{i+1} = gamma_{i+1} / gamma_i
 *     alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1} / alpha_i)
 *
 * Arguments and results as oracle_pcg (*iters = updates of x); a
 * non-positive or non-finite alpha denominator is a breakdown.
 */
int oracle_pcg_sr(int nx, int ny, int nz, const double *kc, const double *b, double *x, double rtol,
                  int maxit, double *hist, int *iters, double *relres)
{
    int64_t n = (int64_t)nx * ny * nz;
    double *r = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * n);
    double *w = malloc(sizeof(double) * n), *p = calloc(n, sizeof(double));
    double *sv = calloc(n, sizeof(double)), *dinv = malloc(sizeof(double) * n);
    if (!r || !u || !w || !p || !sv || !dinv) {
        free(r); free(u); free(w); free(p); free(sv); free(dinv);
        return ORACLE_NOMEM;
    }
    if (kc) {
        oracle_vdiag(nx, ny, nz, kc, dinv);
        for (int64_t i = 0; i < n; ++i)
            dinv[i] = 1.0 / dinv[i];
    } else {
        for (int64_t i = 0; i < n; ++i)
            dinv[i] = 1.0 / 6.0;
    }
    int status = ORACLE_OK;
    *iters = 0;
    double nb = sqrt(oracle_dot(n, b, b));
    if (nb == 0.0) {
        memset(x, 0, sizeof(double) * n);
        *relres = 0.0;
        if (hist)
            hist[0] = 0.0;
        goto done;
    }
    apply_op(nx, ny, nz, kc, x, w);
    for (int64_t i = 0; i < n; ++i)
        r[i] = b[i] - w[i];
    double rn = sqrt(oracle_dot(n, r, r));
    if (hist)
        hist[0] = rn / nb;
    *relres = rn / nb;
    if (rn <= rtol * nb)
        goto done;
    for (int64_t i = 0; i < n; ++i)
        u[i] = dinv[i] * r[i];
    apply_op(nx, ny, nz, kc, u, w);
    double gamma = oracle_dot(n, r, u), delta = oracle_dot(n, w, u);
    if (!(delta > 0.0) || !isfinite(delta) || !isfinite(gamma)) {
        status = ORACLE_BREAKDOWN;
        goto done;
    }
    double alpha = gamma / delta, beta = 0.0;
    status = ORACLE_NOCONV;
    for (int k = 1; k <= maxit; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            p[i] = u[i] + beta * p[i];
            sv[i] = w[i] + beta * sv[i];
            x[i] += alpha * p[i];
            r[i] -= alpha * sv[i];
        }
        *iters = k;
        rn = sqrt(oracle_dot(n, r, r));
        *relres = rn / nb;
        if (hist)
            hist[k] = rn / nb;
        if (!isfinite(rn)) {
            status = ORACLE_BREAKDOWN;
            break;
        }
        if (rn <= rtol * nb) {
            status = ORACLE_OK;
            break;
        }
        for (int64_t i = 0; i < n; ++i)
            u[i] = dinv[i] * r[i];
        apply_op(nx, ny, nz, kc, u, w);
        double gamma_new = oracle_dot(n, r, u);
        delta = oracle_dot(n, w, u);
        beta = gamma_new / gamma;
        double denom = delta - beta * gamma_new / alpha;
        if (!(denom > 0.0) || !isfinite(denom)) {
            status = ORACLE_BREAKDOWN;
            break;
        }
        alpha = gamma_new / denom;
        gamma = gamma_new;
    }
done:
    free(r); free(u); free(w); free(p); free(sv); free(dinv);
    return status;
}

/* r = b - A x (FP64) together with ||r||_2 and max_i |r_i|. */
void oracle_residual(int nx, int ny, int nz, const double *kc, const double *b, const double *x,
                     double *r, double *norm2, double *amax)
{
    int64_t n = (int64_t)nx * ny * nz;
    apply_op(nx, ny, nz, kc, x, r);
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - r[i];
        double a = fabs(r[i]);
        if (a > m)
            m = a;
    }
    *norm2 = sqrt(oracle_dot(n, r, r));
    *amax = m;
}

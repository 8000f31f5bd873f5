/*
 * FP64 CPU oracle for the semi-implicit PHS-RBF meshless solver of
 * Shahane & Vanka, "A Semi-Implicit Meshless Method for Incompressible Flows
 * in Complex Geometries" (arXiv 2106.07616).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path never
 * does. It shares no code, header, table or helper with the HIP library.
 *
 * Everything here is plain, sequential-order FP64 arithmetic, compiled with
 * -ffp-contract=off (no fused multiply-add). Loops over independent points
 * may run under OpenMP; every sum runs sequentially in index order.
 *
 * Readings of places where the paper is silent (the same readings the HIP
 * library follows; see the design notes):
 *   - cloud = the q nearest points including the point itself, ordered by
 *     (squared distance, index); squared distance is
 *     ((dx*dx + dy*dy) + dz*dz) with dx = x_j - x_i, no FMA;
 *   - local coordinates xi = (x_j - x_i) / s, s = distance to the q-th
 *     neighbour; weights are unscaled by s^order afterwards;
 *   - monomials in graded order, within a degree descending x power, then
 *     descending y power;
 *   - "direct linear solver" = LU with partial pivoting (largest |a|, ties to
 *     the lowest original row); singular when |pivot| <= 1e-13 max|A|;
 *   - only the centre point's row of B1 is kept;
 *   - "preconditioned BiCGSTAB" = BiCGSTAB with a right Jacobi preconditioner.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_OOM (-2)
#define ORC_E_SINGULAR (-3)
#define ORC_E_NOCONV (-4)

/* ---------------------------------------------------------------------- */
/* monomial basis (Sec. 2, the polynomial block P)                         */
/* ---------------------------------------------------------------------- */

int orc_num_monomials(int dim, int k)
{
    /* binomial(k + dim, dim) */
    long num = 1, den = 1;
    for (int i = 1; i <= dim; ++i) {
        num *= (k + i);
        den *= i;
    }
    return (int)(num / den);
}

/* Exponents (ex, ey, ez) of each monomial, graded by total degree; within a
 * degree, descending power of x, then descending power of y. */
int orc_monomial_exponents(int dim, int k, int *ex)
{
    int m = 0;
    for (int t = 0; t <= k; ++t) {
        if (dim == 2) {
            for (int a = t; a >= 0; --a) {
                ex[3 * m + 0] = a;
                ex[3 * m + 1] = t - a;
                ex[3 * m + 2] = 0;
                ++m;
            }
        } else {
            for (int a = t; a >= 0; --a)
                for (int b = t - a; b >= 0; --b) {
                    ex[3 * m + 0] = a;
                    ex[3 * m + 1] = b;
                    ex[3 * m + 2] = t - a - b;
                    ++m;
                }
        }
    }
    return m;
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r = r * x;
    return r;
}

/* ---------------------------------------------------------------------- */
/* cloud selection: brute-force k nearest neighbours (Sec. 2 and 3.1)      */
/* ---------------------------------------------------------------------- */

static double sqdist(int dim, const double *a, const double *b)
{
    double dx = b[0] - a[0];
    double dy = b[1] - a[1];
    double d2 = dx * dx + dy * dy;
    if (dim == 3) {
        double dz = b[2] - a[2];
        d2 = d2 + dz * dz;
    }
    return d2;
}

/* For each query point (all points when qidx == NULL) list its q nearest
 * points by the total order (squared distance, index). Returns ORC_E_ARG on a
 * duplicated point or q > n. */
int orc_knn(int dim, int64_t n, const double *xyz, int q, int64_t nq, const int64_t *qidx,
            int32_t *nbr)
{
    if (q < 1 || q > n || (dim != 2 && dim != 3)) return ORC_E_ARG;
    int status = ORC_OK;
#pragma omp parallel
    {
        double *bd = (double *)malloc(sizeof(double) * q);
        int64_t *bi = (int64_t *)malloc(sizeof(int64_t) * q);
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < nq; ++t) {
            int64_t i = qidx ? qidx[t] : t;
            const double *xi = xyz + i * dim;
            int cnt = 0;
            for (int64_t j = 0; j < n; ++j) {
                double d2 = sqdist(dim, xi, xyz + j * dim);
                if (j != i && d2 == 0.0) {
#pragma omp atomic write
                    status = ORC_E_ARG;
                }
                /* keys arrive with increasing j, so an equal distance never beats
                 * an entry already held */
                if (cnt == q && !(d2 < bd[q - 1])) continue;
                int pos = (cnt < q) ? cnt : q - 1;
                while (pos > 0 && d2 < bd[pos - 1]) {
                    bd[pos] = bd[pos - 1];
                    bi[pos] = bi[pos - 1];
                    --pos;
                }
                bd[pos] = d2;
                bi[pos] = j;
                if (cnt < q) ++cnt;
            }
            for (int a = 0; a < q; ++a) nbr[t * q + a] = (int32_t)bi[a];
        }
        free(bd);
        free(bi);
    }
    return status;
}

/* ---------------------------------------------------------------------- */
/* local PHS + polynomial collocation (Sec. 2, Eqs. RBF_interp ... B1)     */
/* ---------------------------------------------------------------------- */

static double phs(double r, int p)
{
    return ipow(r, p);
}

/* Build the scaled saddle system of point i:
 *   A = [Phi P; P^T 0] (ns x ns, row-major), B (ns x R, row-major) holding one
 *   right-hand side per operator: d/dx, d/dy, (d/dz), Laplacian at the centre.
 * Returns the scale s. */
static double build_system(int dim, const double *xyz, int q, const int32_t *cl, int k, int p,
                           double *A, double *B, double *xi /* q*dim */, const int *ex, int m)
{
    const int ns = q + m;
    const int R = dim + 1;
    const double *c = xyz + (int64_t)cl[0] * dim;
    double s = sqrt(sqdist(dim, c, xyz + (int64_t)cl[q - 1] * dim));
    for (int a = 0; a < q; ++a)
        for (int e = 0; e < dim; ++e) xi[a * dim + e] = (xyz[(int64_t)cl[a] * dim + e] - c[e]) / s;
    memset(A, 0, sizeof(double) * ns * ns);
    memset(B, 0, sizeof(double) * ns * R);
    for (int a = 0; a < q; ++a) {
        for (int b = 0; b < q; ++b) {
            double d2 = sqdist(dim, xi + a * dim, xi + b * dim);
            A[a * ns + b] = phs(sqrt(d2), p);
        }
        for (int al = 0; al < m; ++al) {
            double v = 1.0;
            for (int e = 0; e < dim; ++e) v = v * ipow(xi[a * dim + e], ex[3 * al + e]);
            A[a * ns + q + al] = v;
            A[(q + al) * ns + a] = v;
        }
        /* L phi(||x - x_a||) at x = centre (xi = 0): d/dx_e gives
         * -p r^(p-2) xi_e, the Laplacian p (p + dim - 2) r^(p-2) */
        double rr = 0.0;
        for (int e = 0; e < dim; ++e) rr = rr + xi[a * dim + e] * xi[a * dim + e];
        double r = sqrt(rr);
        double rp2 = ipow(r, p - 2);
        for (int e = 0; e < dim; ++e) B[a * R + e] = -(double)p * rp2 * xi[a * dim + e];
        B[a * R + dim] = (double)(p * (p + dim - 2)) * rp2;
    }
    /* L P_alpha at the centre */
    for (int al = 0; al < m; ++al) {
        int tot = ex[3 * al] + ex[3 * al + 1] + ex[3 * al + 2];
        if (tot == 1)
            for (int e = 0; e < dim; ++e)
                if (ex[3 * al + e] == 1) B[(q + al) * R + e] = 1.0;
        if (tot == 2)
            for (int e = 0; e < dim; ++e)
                if (ex[3 * al + e] == 2) B[(q + al) * R + dim] = 2.0;
    }
    (void)k;
    return s;
}

/* LU with partial pivoting (pivot: largest |a| among rows not yet used, ties
 * to the lowest original row), applied to all right-hand sides, then back
 * substitution. A and B are overwritten. X is ns x nrhs. */
static int lu_solve(int ns, int nrhs, double *A, double *B, double *X, int *step_row,
                    unsigned char *used)
{
    double amax = 0.0;
    for (int i = 0; i < ns * ns; ++i)
        if (fabs(A[i]) > amax) amax = fabs(A[i]);
    memset(used, 0, ns);
    for (int k = 0; k < ns; ++k) {
        int prow = -1;
        double best = -1.0;
        for (int i = 0; i < ns; ++i) {
            if (used[i]) continue;
            double v = fabs(A[i * ns + k]);
            if (v > best) {
                best = v;
                prow = i;
            }
        }
        if (!(best > 1e-13 * amax)) return ORC_E_SINGULAR;
        used[prow] = 1;
        step_row[k] = prow;
        const double piv = A[prow * ns + k];
        for (int i = 0; i < ns; ++i) {
            if (used[i]) continue;
            double l = A[i * ns + k] / piv;
            for (int j = k + 1; j < ns; ++j) A[i * ns + j] = A[i * ns + j] - l * A[prow * ns + j];
            for (int r = 0; r < nrhs; ++r) B[i * nrhs + r] = B[i * nrhs + r] - l * B[prow * nrhs + r];
        }
    }
    for (int k = ns - 1; k >= 0; --k) {
        int prow = step_row[k];
        for (int r = 0; r < nrhs; ++r) {
            double sacc = B[prow * nrhs + r];
            for (int j = k + 1; j < ns; ++j) sacc = sacc - A[prow * ns + j] * X[j * nrhs + r];
            X[k * nrhs + r] = sacc / A[prow * ns + k];
        }
    }
    return ORC_OK;
}

/* Expose the scaled system of one point (for tests): A[ns*ns], B[ns*R]. */
int orc_saddle_system(int dim, int64_t n, const double *xyz, int q, const int32_t *nbr, int k,
                      int p, int64_t i, double *A, double *B, double *scale)
{
    if (i < 0 || i >= n) return ORC_E_ARG;
    int ex[3 * 128];
    int m = orc_monomial_exponents(dim, k, ex);
    double xi[3 * 256];
    if (q > 256 || m > 128) return ORC_E_ARG;
    *scale = build_system(dim, xyz, q, nbr + i * q, k, p, A, B, xi, ex, m);
    return ORC_OK;
}

/* Differentiation weights of the centre row of B1 for each query point.
 * w is [R][nq*q] (R = dim+1 operators: d/dx, d/dy, (d/dz), Laplacian), in the
 * order of the point's cloud. *bad receives the lowest singular point index. */
int orc_weights(int dim, int64_t n, const double *xyz, int q, const int32_t *nbr, int k, int p,
                int64_t nq, const int64_t *qidx, double *w, int64_t *bad)
{
    if ((dim != 2 && dim != 3) || k < 0 || (p != 3 && p != 5) || q < 1 || q > n) return ORC_E_ARG;
    int ex[3 * 128];
    if (orc_num_monomials(dim, k) > 128) return ORC_E_ARG;
    int m = orc_monomial_exponents(dim, k, ex);
    if (q <= m) return ORC_E_ARG;
    const int ns = q + m, R = dim + 1;
    int64_t first_bad = -1;
#pragma omp parallel
    {
        double *A = (double *)malloc(sizeof(double) * ns * ns);
        double *B = (double *)malloc(sizeof(double) * ns * R);
        double *X = (double *)malloc(sizeof(double) * ns * R);
        double *xi = (double *)malloc(sizeof(double) * q * dim);
        int *step_row = (int *)malloc(sizeof(int) * ns);
        unsigned char *used = (unsigned char *)malloc(ns);
#pragma omp for schedule(dynamic, 32)
        for (int64_t t = 0; t < nq; ++t) {
            int64_t i = qidx ? qidx[t] : t;
            double s = build_system(dim, xyz, q, nbr + i * q, k, p, A, B, xi, ex, m);
            int st = lu_solve(ns, R, A, B, X, step_row, used);
            if (st != ORC_OK) {
#pragma omp critical
                if (first_bad < 0 || i < first_bad) first_bad = i;
            }
            for (int r = 0; r < R; ++r) {
                double sc = (r < dim) ? s : s * s;
                for (int a = 0; a < q; ++a) w[(int64_t)r * nq * q + t * q + a] = X[a * R + r] / sc;
            }
        }
        free(A); free(B); free(X); free(xi); free(step_row); free(used);
    }
    if (bad) *bad = first_bad;
    return first_bad >= 0 ? ORC_E_SINGULAR : ORC_OK;
}

/* Interpolation weights at an arbitrary point xs from the q cloud points
 * cl[0..q-1] (Eq. RBF_interp evaluated off the nodes): local coordinates
 * centred at xs, scaled by the largest distance from xs to the cloud. */
int orc_interp_weights(int dim, const double *xyz, int q, const int32_t *cl, const double *xs,
                       int k, int p, double *w)
{
    int ex[3 * 128];
    if (orc_num_monomials(dim, k) > 128) return ORC_E_ARG;
    int m = orc_monomial_exponents(dim, k, ex);
    if (q <= m) return ORC_E_ARG;
    const int ns = q + m;
    double *A = (double *)calloc((size_t)ns * ns, sizeof(double));
    double *B = (double *)calloc((size_t)ns, sizeof(double));
    double *X = (double *)calloc((size_t)ns, sizeof(double));
    double *xi = (double *)calloc((size_t)q * dim, sizeof(double));
    int *step_row = (int *)malloc(sizeof(int) * ns);
    unsigned char *used = (unsigned char *)malloc(ns);
    double s2 = 0.0;
    for (int a = 0; a < q; ++a) {
        double d2 = sqdist(dim, xs, xyz + (int64_t)cl[a] * dim);
        if (d2 > s2) s2 = d2;
    }
    double s = sqrt(s2);
    for (int a = 0; a < q; ++a)
        for (int e = 0; e < dim; ++e) xi[a * dim + e] = (xyz[(int64_t)cl[a] * dim + e] - xs[e]) / s;
    for (int a = 0; a < q; ++a) {
        for (int b = 0; b < q; ++b) A[a * ns + b] = phs(sqrt(sqdist(dim, xi + a * dim, xi + b * dim)), p);
        for (int al = 0; al < m; ++al) {
            double v = 1.0;
            for (int e = 0; e < dim; ++e) v = v * ipow(xi[a * dim + e], ex[3 * al + e]);
            A[a * ns + q + al] = v;
            A[(q + al) * ns + a] = v;
        }
        double rr = 0.0;
        for (int e = 0; e < dim; ++e) rr = rr + xi[a * dim + e] * xi[a * dim + e];
        B[a] = phs(sqrt(rr), p);
    }
    B[q] = 1.0; /* the constant monomial at the evaluation point; all others vanish at xi = 0 */
    int st = lu_solve(ns, 1, A, B, X, step_row, used);
    for (int a = 0; a < q; ++a) w[a] = X[a];
    free(A); free(B); free(X); free(xi); free(step_row); free(used);
    return st;
}

/* ---------------------------------------------------------------------- */
/* sparse operators (B1 stored for the whole run)                          */
/* ---------------------------------------------------------------------- */

/* CSR with q entries per row (row_ptr[i] = i*q): each row's columns sorted
 * ascending, the R weight arrays permuted alongside. */
int orc_csr(int64_t n, int q, const int32_t *nbr, int R, const double *w, int32_t *col, double *val)
{
#pragma omp parallel
    {
        int *perm = (int *)malloc(sizeof(int) * q);
#pragma omp for
        for (int64_t i = 0; i < n; ++i) {
            const int32_t *c = nbr + i * q;
            for (int a = 0; a < q; ++a) perm[a] = a;
            for (int a = 1; a < q; ++a) { /* insertion sort by column */
                int v = perm[a], b = a;
                while (b > 0 && c[perm[b - 1]] > c[v]) {
                    perm[b] = perm[b - 1];
                    --b;
                }
                perm[b] = v;
            }
            for (int a = 0; a < q; ++a) {
                col[i * q + a] = c[perm[a]];
                for (int r = 0; r < R; ++r) val[(int64_t)r * n * q + i * q + a] = w[(int64_t)r * n * q + i * q + perm[a]];
            }
        }
        free(perm);
    }
    return ORC_OK;
}

/* y = A x for a CSR matrix with q entries per row; each row summed in column order. */
void orc_spmv(int64_t n, int q, const int32_t *col, const double *val, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int a = 0; a < q; ++a) s = s + val[i * q + a] * x[col[i * q + a]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

/* Diagonal entry of row i: the sum of the row's entries whose column is i
 * (a row may repeat a column with explicit zeros). */
static double diag_value(int q, const int32_t *col, const double *val, int64_t i)
{
    double d = 0.0;
    for (int a = 0; a < q; ++a)
        if (col[i * q + a] == i) d = d + val[i * q + a];
    return d;
}

/* ---------------------------------------------------------------------- */
/* BiCGSTAB with right Jacobi preconditioning (Sec. 3: "preconditioned    */
/* BiCGSTAB"), van der Vorst's iteration, on any linear operator.          */
/* ---------------------------------------------------------------------- */

typedef void (*orc_apply_fn)(const void *ctx, const double *x, double *y);

static int bicgstab_run(int64_t n, orc_apply_fn apply, const void *actx, const double *dinv,
                        const double *b, double *x, double tol, int maxit, int *iters_out,
                        double *relres_out)
{
    double *r = (double *)malloc(sizeof(double) * n);
    double *rh = (double *)malloc(sizeof(double) * n);
    double *pv = (double *)calloc(n, sizeof(double));
    double *ph = (double *)malloc(sizeof(double) * n);
    double *v = (double *)calloc(n, sizeof(double));
    double *s = (double *)malloc(sizeof(double) * n);
    double *sh = (double *)malloc(sizeof(double) * n);
    double *t = (double *)malloc(sizeof(double) * n);
    int status = ORC_E_NOCONV, it = 0;
    const double bn = sqrt(dot(n, b, b));
    double relres = 0.0;
    double rho_old = 1.0, alpha = 1.0, omega = 1.0, rn;
    if (bn == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = ORC_OK;
        goto done;
    }
    apply(actx, x, r);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - r[i];
        rh[i] = r[i];
    }
    rn = sqrt(dot(n, r, r));
    relres = rn / bn;
    if (rn <= tol * bn) {
        status = ORC_OK;
        goto done;
    }
    for (it = 1; it <= maxit; ++it) {
        double rho = dot(n, rh, r);
        if (it == 1 || fabs(rho) < 1e-300 || fabs(rho) < 1e-30 * rn * rn) {
            if (it > 1) { /* breakdown of the shadow residual: restart with r-hat = r */
                for (int64_t i = 0; i < n; ++i) rh[i] = r[i];
                rho = dot(n, rh, r);
            }
            for (int64_t i = 0; i < n; ++i) pv[i] = r[i];
        } else {
            double beta = (rho / rho_old) * (alpha / omega);
            for (int64_t i = 0; i < n; ++i) pv[i] = r[i] + beta * (pv[i] - omega * v[i]);
        }
        for (int64_t i = 0; i < n; ++i) ph[i] = dinv[i] * pv[i];
        apply(actx, ph, v);
        alpha = rho / dot(n, rh, v);
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double sn = sqrt(dot(n, s, s));
        if (sn <= tol * bn) {
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * ph[i];
            relres = sn / bn;
            status = ORC_OK;
            break;
        }
        for (int64_t i = 0; i < n; ++i) sh[i] = dinv[i] * s[i];
        apply(actx, sh, t);
        double tt = dot(n, t, t);
        omega = (tt > 0.0) ? dot(n, t, s) / tt : 0.0;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * ph[i] + omega * sh[i];
            r[i] = s[i] - omega * t[i];
        }
        rho_old = rho;
        rn = sqrt(dot(n, r, r));
        relres = rn / bn;
        if (rn <= tol * bn) {
            status = ORC_OK;
            break;
        }
        if (omega == 0.0) break;
    }
    if (it > maxit) it = maxit;
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = relres;
    free(r); free(rh); free(pv); free(ph); free(v); free(s); free(sh); free(t);
    return status;
}

/* BiCGSTAB with up to two restarts from the true residual: when the recursive
 * residual has met the tolerance but ||b - A x|| exceeds 10 tol ||b||, the
 * iteration starts again from the current x. A true residual still above
 * 10 tol ||b|| after the restarts is reported as non-convergence. */
static int bicgstab_op(int64_t n, orc_apply_fn apply, const void *actx, const double *dinv,
                       const double *b, double *x, double tol, int maxit, int *iters_out,
                       double *relres_out)
{
    double *r = (double *)malloc(sizeof(double) * n);
    const double bn = sqrt(dot(n, b, b));
    int total = 0, st = ORC_OK;
    double rel = 0.0;
    for (int attempt = 0; attempt < 3; ++attempt) {
        int its = 0;
        st = bicgstab_run(n, apply, actx, dinv, b, x, tol, maxit - total, &its, &rel);
        total += its;
        if (st != ORC_OK || bn == 0.0) break;
        apply(actx, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        rel = sqrt(dot(n, r, r)) / bn;
        if (rel <= 10.0 * tol || total >= maxit) break;
    }
    /* the recursion met the tolerance but the true residual still misses it
     * by more than 10x after the restarts: the solve has not converged */
    if (st == ORC_OK && bn != 0.0 && !(rel <= 10.0 * tol)) st = ORC_E_NOCONV;
    free(r);
    if (iters_out) *iters_out = total;
    if (relres_out) *relres_out = rel;
    return st;
}

typedef struct {
    int64_t n;
    int q;
    const int32_t *col;
    const double *val;
} csr_op;

static void csr_apply(const void *ctx, const double *x, double *y)
{
    const csr_op *c = (const csr_op *)ctx;
    orc_spmv(c->n, c->q, c->col, c->val, x, y);
}

/* BiCGSTAB on a CSR matrix with q entries per row; Jacobi scaling by the
 * diagonal (the sum of a row's entries in its own column). */
int orc_bicgstab(int64_t n, int q, const int32_t *col, const double *val, const double *b,
                 double *x, double tol, int maxit, int *iters_out, double *relres_out)
{
    double *dinv = (double *)malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) {
        double d = diag_value(q, col, val, i);
        dinv[i] = (d != 0.0) ? 1.0 / d : 1.0;
    }
    csr_op op = {n, q, col, val};
    int st = bicgstab_op(n, csr_apply, &op, dinv, b, x, tol, maxit, iters_out, relres_out);
    free(dinv);
    return st;
}

/* ---------------------------------------------------------------------- */
/* pressure-correction matrix (Eq. pressure poisson, Sec. 3.1)             */
/* ---------------------------------------------------------------------- */
/* Rows: the PHS Laplacian at interior points, the outward normal derivative
 * (homogeneous Neumann, N . grad p' = 0) at velocity-Dirichlet boundary points
 * (kind 1), p' = 0 at prescribed-pressure boundary points (kind 2) and at
 * outlets (kind 3: prescribed pressure, zero normal velocity gradient), and p' = 0
 * at the pinned interior point (pin >= 0), which removes the constant null
 * space when every boundary is of kind 1. Same sparsity as the operators. */
int orc_poisson_values(int dim, int64_t n, int q, const uint8_t *kind, const double *normal,
                       int64_t pin, const int32_t *col, const double *val, const int64_t *rows, double *pval)
{
    const int64_t nnz = n * q;
    for (int64_t i = 0; i < n; ++i) {
        /* the point row i stands for: itself, or rows[i] for a subset of rows */
        const int64_t g = rows ? rows[i] : i;
        for (int a = 0; a < q; ++a) {
            int64_t e = i * q + a;
            double v;
            if (g == pin || kind[i] == 2 || kind[i] == 3) {
                /* pinned point, or prescribed-pressure boundary: p' = 0 */
                v = (col[e] == g) ? 1.0 : 0.0;
            } else if (kind[i] == 0) {
                v = val[(int64_t)dim * nnz + e];
            } else {
                v = normal[i * dim + 0] * val[e] + normal[i * dim + 1] * val[nnz + e];
                if (dim == 3) v = v + normal[i * dim + 2] * val[2 * nnz + e];
            }
            pval[e] = v;
        }
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* one BDF2 time step with outer iterations (Sec. 3 and its step list)    */
/* ---------------------------------------------------------------------- */

typedef struct {
    int dim;
    int q;
    int64_t n;
    const uint8_t *kind;
    const double *normal;
    int64_t pin;
    const int32_t *col;   /* sorted CSR columns, q per row */
    const double *val;    /* [R][n*q]: d/dx, d/dy, (d/dz), Laplacian */
    const double *pval;   /* [n*q] pressure-correction matrix */
    double rho, mu, dt;
    double alpha[3];
    double tol_outer, tol_krylov;
    int max_outer, max_krylov;
    double force[3];      /* constant body force per unit volume (mean pressure gradient) */
} orc_step_cfg;

typedef struct {
    int outer_iters;
    int krylov_mom;
    int krylov_p;
    int krylov_b;
    int status;
    double delta;
    double eps_steady;
    double div_l1;            /* mean over interior points of |sum_e D_e u_e^{n+1}| */
    double final_relres_p;    /* true relative residual of the last p' solve */
    double krylov_relres_max; /* largest true relative residual of the step's solves */
} orc_step_stats;

/* u, u_prev: [dim][n] velocity at t^n and t^{n-1}, replaced by t^{n+1} and t^n.
 * p: pressure at t^n, replaced by t^{n+1}. u_bc: [dim][n] Dirichlet velocity at
 * t^{n+1} (read on boundary rows only). p_bc: [n] pressure at t^{n+1} on
 * prescribed-pressure (kind 2) points, may be NULL when there are none. */
int orc_simple_step(const orc_step_cfg *c, double *u, double *u_prev, double *p, const double *u_bc,
                    const double *p_bc, orc_step_stats *st)
{
    const int dim = c->dim, q = c->q;
    const int64_t n = c->n, nnz = n * q;
    const double rho = c->rho, mu = c->mu, dt = c->dt;
    const double a1 = c->alpha[0], a2 = c->alpha[1], a3 = c->alpha[2];
    double *ur = (double *)malloc(sizeof(double) * dim * n);   /* u^r */
    double *ut = (double *)malloc(sizeof(double) * dim * n);   /* u-tilde */
    double *un = (double *)malloc(sizeof(double) * dim * n);   /* u^{r+1} */
    double *pr = (double *)malloc(sizeof(double) * n);         /* p^r */
    double *pa = (double *)malloc(sizeof(double) * n);         /* interior-corrected p */
    double *pc = (double *)malloc(sizeof(double) * n);         /* p' */
    double *f = (double *)malloc(sizeof(double) * n);
    double *bm = (double *)malloc(sizeof(double) * dim * n);
    double *mval = (double *)malloc(sizeof(double) * nnz);
    /* velocity-Dirichlet (kind 1) and symmetry (kind 4) points: homogeneous
     * Neumann p' and the pressure from the normal momentum equation */
    int64_t nb = 0;
    for (int64_t i = 0; i < n; ++i) nb += (c->kind[i] == 1 || c->kind[i] == 4);
    int64_t *bidx = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
    int64_t *bpos = (int64_t *)malloc(sizeof(int64_t) * n);
    int32_t *gcol = (int32_t *)malloc(sizeof(int32_t) * (nb * q + 1));
    double *gval = (double *)malloc(sizeof(double) * (nb * q + 1));
    double *bb = (double *)malloc(sizeof(double) * (nb + 1));
    double *pb = (double *)malloc(sizeof(double) * (nb + 1));
    for (int64_t i = 0, b = 0; i < n; ++i) {
        bpos[i] = (c->kind[i] == 1 || c->kind[i] == 4) ? b : -1;
        if (c->kind[i] == 1 || c->kind[i] == 4) bidx[b++] = i;
    }
    /* block of the normal-derivative rows over kind-1 points: columns of the
     * other points are moved to the right-hand side (zero value, own column) */
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t i = bidx[b];
        for (int a = 0; a < q; ++a) {
            int64_t k = i * q + a, j = c->col[k];
            const int in_block = (c->kind[j] == 1 || c->kind[j] == 4);
            gcol[b * q + a] = in_block ? (int32_t)bpos[j] : (int32_t)b;
            gval[b * q + a] = in_block ? c->pval[k] : 0.0;
        }
    }

    int status = ORC_OK, kit_m = 0, kit_p = 0, kit_b = 0, outer = 0;
    double delta = 0.0, relres_p = 0.0, relres_max = 0.0;
    /* step 1: the iterate starts from the old time level, with the Dirichlet
     * values of the new time level on velocity-prescribed points (kinds 1, 2) */
    for (int e = 0; e < dim; ++e)
        for (int64_t i = 0; i < n; ++i)
            ur[e * n + i] = (c->kind[i] == 1 || c->kind[i] == 2) ? u_bc[e * n + i] : u[e * n + i];
    memcpy(pr, p, sizeof(double) * n);

    for (outer = 1; outer <= c->max_outer; ++outer) {
        /* step 2: momentum matrix and right-hand sides (Eqs. u:tilde, v:tilde) */
        for (int64_t i = 0; i < n; ++i) {
            if (c->kind[i] == 3 || c->kind[i] == 4) {
                /* outlet and symmetry (Sec. 3.1): N . grad u_e = 0; on a
                 * symmetry point the normal component is set to u = 0 below,
                 * component by component */
                for (int a = 0; a < q; ++a) {
                    double v = 0.0;
                    for (int d = 0; d < dim; ++d) v = v + c->normal[i * dim + d] * c->val[d * nnz + i * q + a];
                    mval[i * q + a] = v;
                }
                for (int e = 0; e < dim; ++e) bm[e * n + i] = 0.0;
                continue;
            }
            if (c->kind[i] != 0) {
                for (int a = 0; a < q; ++a) mval[i * q + a] = (c->col[i * q + a] == i) ? 1.0 : 0.0;
                for (int e = 0; e < dim; ++e) bm[e * n + i] = u_bc[e * n + i];
                continue;
            }
            for (int a = 0; a < q; ++a) {
                int64_t k = i * q + a;
                double conv = 0.0;
                for (int e = 0; e < dim; ++e) conv = conv + ur[e * n + i] * c->val[e * nnz + k];
                double v = rho * conv - mu * c->val[dim * nnz + k];
                if (c->col[k] == i) v = v + rho * a1 / dt;
                mval[k] = v;
            }
            for (int e = 0; e < dim; ++e) {
                double g = 0.0;
                for (int a = 0; a < q; ++a) g = g + c->val[e * nnz + i * q + a] * pr[c->col[i * q + a]];
                bm[e * n + i] = -rho * (a2 * u[e * n + i] + a3 * u_prev[e * n + i]) / dt - g + c->force[e];
            }
        }
        /* momentum solves, one per velocity component, started from u^r */
        for (int e = 0; e < dim; ++e) {
            int its = 0;
            /* symmetry points (Sec. 3.1: no flow through the plane, no normal
             * derivative of the tangential velocity). With the plane's unit
             * normal n, component s (largest |n_s|, lowest index on ties)
             * takes u . n = 0 as n_s u_s = -sum_{d != s} n_d u_d; every other
             * component a takes the tangent t_a = e_a - n_a n, i.e.
             * (1 - n_a^2) N.grad u_a = sum_{d != a} n_a n_d N.grad u_d. The
             * other components enter at the outer iterate u^r, so both hold
             * once the outer iteration has converged. A normal along an axis
             * gives u_s = 0 and N.grad u_a = 0, right-hand sides 0. */
            for (int64_t i = 0; i < n; ++i) {
                if (c->kind[i] != 4) continue;
                const double *nv = c->normal + i * dim;
                int sc = 0;
                for (int d = 1; d < dim; ++d)
                    if (fabs(nv[d]) > fabs(nv[sc])) sc = d;
                const int axis = fabs(nv[sc]) == 1.0;
                const double scale = (e == sc) ? (axis ? 1.0 : nv[sc]) : (axis ? 1.0 : 1.0 - nv[e] * nv[e]);
                for (int a = 0; a < q; ++a) {
                    double v = 0.0;
                    if (e == sc) {
                        v = (c->col[i * q + a] == i) ? scale : 0.0;
                    } else {
                        for (int d = 0; d < dim; ++d) v = v + nv[d] * c->val[d * nnz + i * q + a];
                        v = scale * v;
                    }
                    mval[i * q + a] = v;
                }
                double r = 0.0;
                if (!axis && e == sc) {
                    for (int d = 0; d < dim; ++d)
                        if (d != sc) r = r - nv[d] * ur[d * n + i];
                } else if (!axis) {
                    for (int d = 0; d < dim; ++d) {
                        if (d == e) continue;
                        double g = 0.0;   /* (N . grad u_d)(x_i) at the iterate */
                        for (int a = 0; a < q; ++a) {
                            double w = 0.0;
                            for (int cc = 0; cc < dim; ++cc) w = w + nv[cc] * c->val[cc * nnz + i * q + a];
                            g = g + w * ur[d * n + c->col[i * q + a]];
                        }
                        r = r + nv[e] * nv[d] * g;
                    }
                }
                bm[e * n + i] = r;
            }
            memcpy(ut + e * n, ur + e * n, sizeof(double) * n);
            double rel = 0.0;
            int s = orc_bicgstab(n, q, c->col, mval, bm + e * n, ut + e * n, c->tol_krylov, c->max_krylov, &its, &rel);
            kit_m += its;
            if (rel > relres_max) relres_max = rel;
            if (s != ORC_OK) status = s;
        }
        /* step 3: pressure-correction right-hand side (Eq. pressure poisson) */
        for (int64_t i = 0; i < n; ++i) {
            if (c->kind[i] != 0 || i == c->pin) {
                f[i] = 0.0;
                continue;
            }
            double dv = 0.0;
            for (int e = 0; e < dim; ++e) {
                double g = 0.0;
                for (int a = 0; a < q; ++a) g = g + c->val[e * nnz + i * q + a] * ut[e * n + c->col[i * q + a]];
                dv = dv + g;
            }
            f[i] = rho * a1 / dt * dv;
        }
        /* pressure-correction solve from p' = 0 */
        {
            int its = 0;
            memset(pc, 0, sizeof(double) * n);
            double rel = 0.0;
            int s = orc_bicgstab(n, q, c->col, c->pval, f, pc, c->tol_krylov, c->max_krylov, &its, &rel);
            kit_p += its;
            relres_p = rel;
            if (rel > relres_max) relres_max = rel;
            if (s != ORC_OK) status = s;
        }
        /* step 4: interior pressure correction (Eq. p:correction); prescribed
         * pressure on kind-2 and outlet (kind-3) points */
        for (int64_t i = 0; i < n; ++i)
            pa[i] = (c->kind[i] == 0) ? pr[i] + pc[i] : ((c->kind[i] == 2 || c->kind[i] == 3) ? p_bc[i] : pr[i]);
        /* step 5: boundary pressure from the normal momentum equation (Eq. normal
         * momentum), evaluated with u-tilde (the newest velocity at this step)
         * and solved for the whole boundary block with the corrected interior
         * pressures held fixed:  G_BB p_B = R_B - G_BI p_I,  G = N . grad. */
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t i = bidx[b];
            double rhs = 0.0;
            for (int e = 0; e < dim; ++e) {
                double dudt = rho * (a1 * ut[e * n + i] + a2 * u[e * n + i] + a3 * u_prev[e * n + i]) / dt;
                double adv = 0.0;
                for (int g = 0; g < dim; ++g) {
                    double d = 0.0;
                    for (int a = 0; a < q; ++a) d = d + c->val[g * nnz + i * q + a] * ut[e * n + c->col[i * q + a]];
                    adv = adv + ut[g * n + i] * d;
                }
                double lap = 0.0;
                for (int a = 0; a < q; ++a) lap = lap + c->val[dim * nnz + i * q + a] * ut[e * n + c->col[i * q + a]];
                double comp = -dudt - rho * adv + mu * lap + c->force[e];
                rhs = rhs + c->normal[i * dim + e] * comp;
            }
            for (int a = 0; a < q; ++a) {
                int64_t k = i * q + a, j = c->col[k];
                if (c->kind[j] == 1 || c->kind[j] == 4) continue;
                rhs = rhs - c->pval[k] * pa[j];
            }
            bb[b] = rhs;
            pb[b] = pr[i]; /* start from the previous boundary pressures */
        }
        if (nb > 0) {
            int its = 0;
            double rel = 0.0;
            int s = orc_bicgstab(nb, q, gcol, gval, bb, pb, c->tol_krylov, c->max_krylov, &its, &rel);
            kit_b += its;
            if (rel > relres_max) relres_max = rel;
            if (s != ORC_OK) status = s;
        }
        for (int64_t i = 0; i < n; ++i) pr[i] = (c->kind[i] == 1 || c->kind[i] == 4) ? pb[bpos[i]] : pa[i];
        /* step 6: velocity correction (Eqs. u:correction, v:correction) */
        const double coef = dt / (rho * a1);
        for (int e = 0; e < dim; ++e)
            for (int64_t i = 0; i < n; ++i) {
                if (c->kind[i] != 0) {
                    un[e * n + i] = ut[e * n + i];
                    continue;
                }
                double g = 0.0;
                for (int a = 0; a < q; ++a) g = g + c->val[e * nnz + i * q + a] * pc[c->col[i * q + a]];
                un[e * n + i] = ut[e * n + i] - coef * g;
            }
        /* step 7: change over the iteration, sum over components of the mean |.| */
        delta = 0.0;
        for (int e = 0; e < dim; ++e) {
            double sacc = 0.0;
            for (int64_t i = 0; i < n; ++i) sacc = sacc + fabs(un[e * n + i] - ur[e * n + i]);
            delta = delta + sacc / (double)n;
        }
        memcpy(ur, un, sizeof(double) * dim * n);
        /* step 8 */
        if (delta < c->tol_outer) break;
    }
    if (outer > c->max_outer) {
        outer = c->max_outer;
        /* tol_outer <= 0 asks for exactly max_outer iterations: not a failure */
        if (status == ORC_OK && c->tol_outer > 0.0) status = ORC_E_NOCONV;
    }
    /* steady-state rate: max over components of mean |u^{n+1} - u^n| / dt */
    double eps = 0.0;
    for (int e = 0; e < dim; ++e) {
        double sacc = 0.0;
        for (int64_t i = 0; i < n; ++i) sacc = sacc + fabs(ur[e * n + i] - u[e * n + i]);
        sacc = sacc / (double)n / dt;
        if (sacc > eps) eps = sacc;
    }
    /* the discrete continuity equation (Eq. continuity:n+1) at the interior
     * points, applied to the new velocity: mean of |sum_e D_e u_e| */
    double div_sum = 0.0;
    int64_t n_int = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (c->kind[i] != 0) continue;
        double dv = 0.0;
        for (int e = 0; e < dim; ++e) {
            double g = 0.0;
            for (int a = 0; a < q; ++a) g = g + c->val[e * nnz + i * q + a] * ur[e * n + c->col[i * q + a]];
            dv = dv + g;
        }
        div_sum = div_sum + fabs(dv);
        n_int++;
    }
    memcpy(u_prev, u, sizeof(double) * dim * n);
    memcpy(u, ur, sizeof(double) * dim * n);
    memcpy(p, pr, sizeof(double) * n);
    if (st) {
        st->div_l1 = n_int > 0 ? div_sum / (double)n_int : 0.0;
        st->final_relres_p = relres_p;
        st->krylov_relres_max = relres_max;
        st->outer_iters = outer;
        st->krylov_mom = kit_m;
        st->krylov_p = kit_p;
        st->krylov_b = kit_b;
        st->status = status;
        st->delta = delta;
        st->eps_steady = eps;
    }
    free(ur); free(ut); free(un); free(pr); free(pa); free(pc); free(f); free(bm); free(mval);
    free(bidx); free(bpos); free(gcol); free(gval); free(bb); free(pb);
    return status;
}

/* ---------------------------------------------------------------------- */
/* time step from a Courant number (Sec. 3: Co = |lambda|max dt / 2)       */
/* ---------------------------------------------------------------------- */

/* Largest eigenvalue magnitude of the discrete convection-diffusion operator
 * -rho (u0 . grad) + mu Laplacian on interior rows (boundary rows zero), by
 * 'iters' normalised power iterations from the start vector
 * x_i = 1 + (i mod 7)/7. Returns |lambda|max. */
double orc_convdiff_lambda(int dim, int64_t n, int q, const uint8_t *kind, const int32_t *col,
                           const double *val, const double *u0, double rho, double mu, int iters)
{
    const int64_t nnz = n * q;
    double *cv = (double *)malloc(sizeof(double) * nnz);
    double *x = (double *)malloc(sizeof(double) * n);
    double *y = (double *)malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < q; ++a) {
            int64_t k = i * q + a;
            if (kind[i] != 0) {
                cv[k] = 0.0;
                continue;
            }
            double conv = 0.0;
            for (int e = 0; e < dim; ++e) conv = conv + u0[e * n + i] * val[e * nnz + k];
            cv[k] = -rho * conv + mu * val[dim * nnz + k];
        }
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0 + (double)(i % 7) / 7.0;
    double xn = sqrt(dot(n, x, x));
    for (int64_t i = 0; i < n; ++i) x[i] = x[i] / xn;
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        orc_spmv(n, q, col, cv, x, y);
        double yn = sqrt(dot(n, y, y));
        lam = yn; /* x has unit norm */
        if (yn == 0.0) break;
        for (int64_t i = 0; i < n; ++i) x[i] = y[i] / yn;
    }
    free(cv); free(x); free(y);
    return lam;
}

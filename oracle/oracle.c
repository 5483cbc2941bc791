/*
 * Plain FP64 CPU oracle for the multigrid Poisson solve, the projection
 * time step and the implicit advection-diffusion multigrid of "Neural
 * Physics" (Chen, Heaney, Pain, arXiv 2402.17913).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; it shares no source with the HIP path.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Every routine is a direct, unfused loop over cells, written to be checked
 * against the paper by eye.  Floating point is FP64 throughout.
 *
 * The OpenMP pragmas on the cell loops of the multigrid solve only matter in
 * the separate host-timing build (compiled with -fopenmp); the build the
 * tests load is compiled without it, so they are ignored there and every
 * loop, reductions included, runs in the order written.
 *
 * Grid convention.  A d-dimensional grid (d = 2 or 3) of n cells per axis,
 * cell index (i, j, k) with i fastest: idx = (k*n + j)*n + i.  Cell i has its
 * centre at (i + 1/2) h.  Two boundary treatments, both realised as padding
 * (ghost values) as in Section 2.1 ("additional ghost cells or halo nodes"):
 *   OR_BC_DIRICHLET0: ghost = -(adjacent interior value), i.e. the padding
 *                     that makes the solution vanish on the cell faces that
 *                     bound the domain (reading of the paper's zero padding
 *                     for a cell-centred grid);
 *   OR_BC_PERIODIC:   ghost = value on the opposite side (wrap);
 *   OR_BC_NEUMANN:    ghost = the adjacent interior value (the copy padding
 *                     of Section 2.4 for a zero normal derivative; used by
 *                     the explicit step only).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BC_DIRICHLET0 0
#define OR_BC_PERIODIC 1
#define OR_BC_NEUMANN 2

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOCONV (-2)

typedef int64_t i64;

static i64 ncells(int d, i64 n) { return d == 2 ? n * n : n * n * n; }

/* Value of grid function x at integer cell position (i, j, k), where each
 * coordinate may lie one cell (or, for prolongation corners, one cell in
 * several axes) outside [0, n).  Out-of-range axes are resolved one at a
 * time by the boundary rule, so a corner ghost under DIRICHLET0 carries the
 * product of the per-axis sign flips. */
static double ghost_at(const double *x, int d, i64 n, int bc, i64 i, i64 j, i64 k)
{
    double sign = 1.0;
    i64 c[3] = {i, j, k};
    for (int a = 0; a < d; ++a) {
        if (c[a] < 0) {
            if (bc == OR_BC_PERIODIC) c[a] += n;
            else { c[a] = -1 - c[a]; if (bc == OR_BC_DIRICHLET0) sign = -sign; }
        } else if (c[a] >= n) {
            if (bc == OR_BC_PERIODIC) c[a] -= n;
            else { c[a] = 2 * n - 1 - c[a]; if (bc == OR_BC_DIRICHLET0) sign = -sign; }
        }
    }
    if (d == 2) c[2] = 0;
    return sign * x[(c[2] * n + c[1]) * n + c[0]];
}

/* ---------------------------------------------------------------------- */
/* Operator.  A x = (2d x_c - sum of the 2d face neighbours)/h^2: the
 * central second-difference diffusion filter of Section 2.1 (the 5-point
 * 3x3 filter with centre 4) and its 3D 7-point form of Appendix A (centre 6),
 * with unit diffusivity and without the factor dt.  A is the negative
 * discrete Laplacian, i.e. the paper's positive filter. */
void or_apply_A(int d, i64 n, double h, int bc, const double *x, double *y)
{
    const double inv_h2 = 1.0 / (h * h);
    const i64 nz = d == 3 ? n : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                double s = ghost_at(x, d, n, bc, i - 1, j, k) + ghost_at(x, d, n, bc, i + 1, j, k)
                         + ghost_at(x, d, n, bc, i, j - 1, k) + ghost_at(x, d, n, bc, i, j + 1, k);
                if (d == 3)
                    s += ghost_at(x, d, n, bc, i, j, k - 1) + ghost_at(x, d, n, bc, i, j, k + 1);
                const double xc = x[(k * n + j) * n + i];
                y[(k * n + j) * n + i] = (2.0 * d * xc - s) * inv_h2;
            }
}

/* Residual r = f - A x (Appendix B, the residual of A*T = b). */
void or_residual(int d, i64 n, double h, int bc, const double *f, const double *x, double *r)
{
    const i64 m = ncells(d, n);
    or_apply_A(d, n, h, bc, x, r);
#pragma omp parallel for schedule(static)
    for (i64 c = 0; c < m; ++c) r[c] = f[c] - r[c];
}

static double dot(i64 m, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (i64 c = 0; c < m; ++c) s += a[c] * b[c];
    return s;
}

/* Relative residual ||f - A x||_2 / ||f||_2, the convergence gauge that
 * replaces the paper's successive-difference L1 norm (Section 3.2).  This is
 * the judge of every result, whatever produced x. */
double or_rel_res(int d, i64 n, double h, int bc, const double *f, const double *x)
{
    const i64 m = ncells(d, n);
    double *r = malloc(sizeof(double) * m);
    or_residual(d, n, h, bc, f, x, r);
    const double nr = sqrt(dot(m, r, r)), nf = sqrt(dot(m, f, f));
    free(r);
    return nf > 0.0 ? nr / nf : nr;
}

/* One weighted-Jacobi sweep: every cell is updated from the old iterate,
 * x_new = x + omega (f - A x) / A_00, with A_00 = 2d/h^2 the centre weight of
 * the filter (Section 2.2, relaxed Jacobi dividing by the filter centre;
 * Appendix B, division of the residual by A_0,0 / A_0,0,0).  Writes x_out,
 * which must not alias x_in. */
void or_jacobi(int d, i64 n, double h, int bc, double omega, const double *f, const double *x_in,
               double *x_out)
{
    const i64 m = ncells(d, n);
    const double a00 = 2.0 * d / (h * h);
    or_apply_A(d, n, h, bc, x_in, x_out);
#pragma omp parallel for schedule(static)
    for (i64 c = 0; c < m; ++c) x_out[c] = x_in[c] + omega * (f[c] - x_out[c]) / a00;
}

/* Restriction (Section 2.2 and Appendix B): the coarse value is the average
 * of the 2^d fine cells it covers, i.e. a 2x2 (2x2x2) filter of 1/4 (1/8)
 * applied with stride 2.  n is the fine size. */
void or_restrict(int d, i64 n, const double *r, double *fc)
{
    const i64 nc = n / 2, nzc = d == 3 ? nc : 1;
    const double w = d == 3 ? 0.125 : 0.25;
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 K = 0; K < nzc; ++K)
        for (i64 J = 0; J < nc; ++J)
            for (i64 I = 0; I < nc; ++I) {
                double s = 0.0;
                for (int c = 0; c < (d == 3 ? 2 : 1); ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const i64 k = d == 3 ? 2 * K + c : 0;
                            s += r[(k * n + 2 * J + b) * n + 2 * I + a];
                        }
                fc[(K * nc + J) * nc + I] = w * s;
            }
}

/* Prolongation and correction x += P e.  The paper's prolongation copies a
 * coarse value to its 2^d fine cells (Section 2.2); the configured transfer
 * here is its cell-centred linear refinement: along each axis a fine cell
 * takes 3/4 of its own coarse cell and 1/4 of the coarse neighbour on its
 * side, and the d-dimensional weights are the products (9/16, 3/16, 3/16,
 * 1/16 in 2D).  Coarse ghosts follow the boundary rule.  nc is the coarse
 * size. */
void or_prolong_add(int d, i64 nc, int bc, const double *e, double *x)
{
    const i64 n = 2 * nc, nz = d == 3 ? n : 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 own[3] = {i / 2, j / 2, k / 2};
                const i64 nb[3] = {(i % 2) ? i / 2 + 1 : i / 2 - 1, (j % 2) ? j / 2 + 1 : j / 2 - 1,
                                   (k % 2) ? k / 2 + 1 : k / 2 - 1};
                double s = 0.0;
                for (int c = 0; c < (d == 3 ? 2 : 1); ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) *
                                             (d == 3 ? (c ? 0.25 : 0.75) : 1.0);
                            s += w * ghost_at(e, d, nc, bc, a ? nb[0] : own[0], b ? nb[1] : own[1],
                                              d == 3 ? (c ? nb[2] : own[2]) : 0);
                        }
                x[(k * n + j) * n + i] += s;
            }
}

/* Dense Cholesky factorisation A = L L^T in place (lower triangle), m x m. */
static int cholesky(i64 m, double *a)
{
    for (i64 j = 0; j < m; ++j) {
        double s = a[j * m + j];
        for (i64 p = 0; p < j; ++p) s -= a[j * m + p] * a[j * m + p];
        if (!(s > 0.0)) return OR_EINVAL;
        const double ljj = sqrt(s);
        a[j * m + j] = ljj;
        for (i64 i = j + 1; i < m; ++i) {
            double t = a[i * m + j];
            for (i64 p = 0; p < j; ++p) t -= a[i * m + p] * a[j * m + p];
            a[i * m + j] = t / ljj;
        }
    }
    return OR_OK;
}

/* Exact coarsest-grid solve (Section 2.2, "solve the system exactly"): the
 * matrix of A on the coarsest grid is assembled column by column from the
 * operator itself, factorised by Cholesky and applied to the residual, so
 * x <- x + A^{-1} (f - A x).  For a periodic grid A is singular with the
 * constants as null space; the matrix A + 1 1^T / m is solved instead, which
 * for a mean-free right-hand side yields the mean-free solution of A x = f. */
int or_coarse_solve(int d, i64 n, double h, int bc, const double *f, double *x)
{
    const i64 m = ncells(d, n);
    double *a = malloc(sizeof(double) * m * m), *e = calloc(m, sizeof(double));
    double *col = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    for (i64 j = 0; j < m; ++j) {
        e[j] = 1.0;
        or_apply_A(d, n, h, bc, e, col);
        e[j] = 0.0;
        for (i64 i = 0; i < m; ++i) a[i * m + j] = col[i] + (bc == OR_BC_PERIODIC ? 1.0 / m : 0.0);
    }
    int st = cholesky(m, a);
    if (st == OR_OK) {
        or_residual(d, n, h, bc, f, x, r);
        for (i64 i = 0; i < m; ++i) { /* forward: L y = r */
            double t = r[i];
            for (i64 p = 0; p < i; ++p) t -= a[i * m + p] * r[p];
            r[i] = t / a[i * m + i];
        }
        for (i64 i = m - 1; i >= 0; --i) { /* backward: L^T z = y */
            double t = r[i];
            for (i64 p = i + 1; p < m; ++p) t -= a[p * m + i] * r[p];
            r[i] = t / a[i * m + i];
        }
        for (i64 i = 0; i < m; ++i) x[i] += r[i];
    }
    free(a); free(e); free(col); free(r);
    return st;
}

/* One V(nu1, nu2) cycle on the level with n cells per axis and spacing h
 * (Section 2.2, the multigrid cycle steps (1)-(8)): nu1 Jacobi sweeps,
 * residual, restriction, recursive cycle for the coarse error from a zero
 * guess, prolongation and correction, nu2 Jacobi sweeps.  Each coarser level
 * re-discretises the operator with its own spacing 2h (Appendix B: the
 * filters change between layers because the grid spacing changes). */
int or_vcycle(int d, i64 n, double h, int bc, int nu1, int nu2, double omega, i64 n_coarsest,
              const double *f, double *x)
{
    if (n <= n_coarsest) return or_coarse_solve(d, n, h, bc, f, x);
    const i64 m = ncells(d, n), nc = n / 2, mc = ncells(d, nc);
    double *t = malloc(sizeof(double) * m);
    double *fc = malloc(sizeof(double) * mc), *ec = calloc(mc, sizeof(double));
    for (int s = 0; s < nu1; ++s) {
        or_jacobi(d, n, h, bc, omega, f, x, t);
        memcpy(x, t, sizeof(double) * m);
    }
    or_residual(d, n, h, bc, f, x, t);
    or_restrict(d, n, t, fc);
    int st = or_vcycle(d, nc, 2.0 * h, bc, nu1, nu2, omega, n_coarsest, fc, ec);
    or_prolong_add(d, nc, bc, ec, x);
    for (int s = 0; s < nu2; ++s) {
        or_jacobi(d, n, h, bc, omega, f, x, t);
        memcpy(x, t, sizeof(double) * m);
    }
    free(t); free(fc); free(ec);
    return st;
}

static int is_pow2(i64 n) { return n > 0 && (n & (n - 1)) == 0; }

/* Solve driver.  The paper starts from a zero estimate (Section 2.2, the
 * initial estimate of the solution is zero) and chains cycles; here cycles
 * run until ||f - A x||_2 / ||f||_2 <= tol, tested before every cycle, or
 * exactly fixed_cycles cycles when fixed_cycles > 0.  For a periodic grid the
 * right-hand side is first made mean-free (compatibility of the singular
 * problem) and the returned solution is the mean-free one.
 * hist (may be NULL) receives the relative residual before each cycle and
 * after the last one, at most hist_len entries. */
int or_mg_solve(int d, i64 n, double h, int bc, const double *f_in, double *x, double tol, int nu1,
                int nu2, double omega, int max_cycles, int fixed_cycles, int warm_start,
                i64 n_coarsest, int *cycles_out, double *rel_res_out, double *hist, int hist_len)
{
    if ((d != 2 && d != 3) || !is_pow2(n) || n < 4 || !is_pow2(n_coarsest) || n_coarsest < 2 ||
        !(h > 0.0) || !(tol > 0.0) || nu1 < 0 || nu2 < 0)
        return OR_EINVAL;
    const i64 m = ncells(d, n);
    double *f = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    memcpy(f, f_in, sizeof(double) * m);
    if (bc == OR_BC_PERIODIC) {
        double mean = 0.0;
        for (i64 c = 0; c < m; ++c) mean += f[c];
        mean /= (double)m;
        for (i64 c = 0; c < m; ++c) f[c] -= mean;
    }
    const double nf = sqrt(dot(m, f, f));
    int st = OR_OK, k = 0;
    double rr = 0.0;
    if (nf == 0.0) {
        memset(x, 0, sizeof(double) * m);
    } else {
        if (!warm_start) memset(x, 0, sizeof(double) * m);
        for (;;) {
            or_residual(d, n, h, bc, f, x, r);
            rr = sqrt(dot(m, r, r)) / nf;
            if (hist && k < hist_len) hist[k] = rr;
            if (fixed_cycles > 0) {
                if (k >= fixed_cycles) break;
            } else {
                if (rr <= tol) break;
                if (k >= max_cycles) { st = OR_ENOCONV; break; }
            }
            int s = or_vcycle(d, n, h, bc, nu1, nu2, omega, n_coarsest, f, x);
            if (s != OR_OK) { st = s; break; }
            ++k;
        }
        if (bc == OR_BC_PERIODIC) {
            double mean = 0.0;
            for (i64 c = 0; c < m; ++c) mean += x[c];
            mean /= (double)m;
            for (i64 c = 0; c < m; ++c) x[c] -= mean;
        }
    }
    if (cycles_out) *cycles_out = k;
    if (rel_res_out) *rel_res_out = rr;
    free(f); free(r);
    return st;
}

/* ---------------------------------------------------------------------- */
/* The paper's own cycle (Section 2.2, the sawtooth cycle; Appendix B, the
 * multigrid written as a U-Net).  Not the default cycle of the solver; kept
 * to measure it against V(2,2). */

/* The paper's prolongation (Section 2.2): every fine cell receives the value
 * of the coarse cell that contains it (a 2x2 / 2x2x2 filter of ones with
 * stride 2), added to x.  nc is the coarse size. */
void or_prolong_const_add(int d, i64 nc, const double *e, double *x)
{
    const i64 n = 2 * nc, nz = d == 3 ? n : 1;
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i)
                x[(k * n + j) * n + i] += e[((k / 2) * nc + j / 2) * nc + i / 2];
}

/* One sawtooth cycle, Appendix B: the residual of the finest grid,
 * r_0 = f - A x; its restrictions r_{l+1} = R r_l down to the coarsest grid
 * (no smoothing on the way down); then from the coarsest grid up, on every
 * level the correction starts as r_l / A_00 (the Jacobi step from zero, the
 * division of the residual by the filter centre) plus the prolongated
 * correction of the coarser level (none on the coarsest), and is smoothed by
 * nu relaxed-Jacobi steps e <- e + alpha (r_l - A e) / A_00 on that level's
 * residual equation; finally x <- x + e_0.  The paper uses alpha = 1, nu = 1
 * and the copying prolongation (prolong_const = 1).  Coarser levels
 * re-discretise A with spacing 2^l h. */
int or_sawtooth(int d, i64 n, double h, int bc, double alpha, int nu, int prolong_const, i64 n_coarsest,
                const double *f, double *x)
{
    int L = 0;
    while ((n >> L) > n_coarsest) ++L;
    double **r = calloc(L + 1, sizeof(double *)), **e = calloc(L + 1, sizeof(double *));
    for (int l = 0; l <= L; ++l) {
        r[l] = malloc(sizeof(double) * ncells(d, n >> l));
        e[l] = calloc(ncells(d, n >> l), sizeof(double));
    }
    double *t = malloc(sizeof(double) * ncells(d, n));
    or_residual(d, n, h, bc, f, x, r[0]);
    for (int l = 0; l < L; ++l) or_restrict(d, n >> l, r[l], r[l + 1]);
    for (int l = L; l >= 0; --l) {
        const i64 nl = n >> l, ml = ncells(d, nl);
        const double hl = h * (double)((i64)1 << l), a00 = 2.0 * d / (hl * hl);
        for (i64 c = 0; c < ml; ++c) e[l][c] = r[l][c] / a00;
        if (l < L) {
            if (prolong_const) or_prolong_const_add(d, nl / 2, e[l + 1], e[l]);
            else or_prolong_add(d, nl / 2, bc, e[l + 1], e[l]);
        }
        for (int s = 0; s < nu; ++s) {
            or_jacobi(d, nl, hl, bc, alpha, r[l], e[l], t);
            memcpy(e[l], t, sizeof(double) * ml);
        }
    }
    const i64 m = ncells(d, n);
    for (i64 c = 0; c < m; ++c) x[c] += e[0][c];
    for (int l = 0; l <= L; ++l) { free(r[l]); free(e[l]); }
    free(r); free(e); free(t);
    return OR_OK;
}

/* Tolerance driver of the sawtooth cycle, with the same stopping rule,
 * periodic treatment and outputs as or_mg_solve. */
int or_saw_solve(int d, i64 n, double h, int bc, const double *f_in, double *x, double tol, double alpha,
                 int nu, int prolong_const, int max_cycles, int fixed_cycles, i64 n_coarsest, int *cycles_out,
                 double *rel_res_out, double *hist, int hist_len)
{
    if ((d != 2 && d != 3) || !is_pow2(n) || n < 4 || !is_pow2(n_coarsest) || n_coarsest < 2 ||
        !(h > 0.0) || !(tol > 0.0) || nu < 0)
        return OR_EINVAL;
    const i64 m = ncells(d, n);
    double *f = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    memcpy(f, f_in, sizeof(double) * m);
    if (bc == OR_BC_PERIODIC) {
        double mean = 0.0;
        for (i64 c = 0; c < m; ++c) mean += f[c];
        mean /= (double)m;
        for (i64 c = 0; c < m; ++c) f[c] -= mean;
    }
    const double nf = sqrt(dot(m, f, f));
    int st = OR_OK, k = 0;
    double rr = 0.0;
    memset(x, 0, sizeof(double) * m);
    if (nf > 0.0) {
        for (;;) {
            or_residual(d, n, h, bc, f, x, r);
            rr = sqrt(dot(m, r, r)) / nf;
            if (hist && k < hist_len) hist[k] = rr;
            if (fixed_cycles > 0) {
                if (k >= fixed_cycles) break;
            } else {
                if (rr <= tol) break;
                if (k >= max_cycles || !(rr < 1e300)) { st = OR_ENOCONV; break; }
            }
            or_sawtooth(d, n, h, bc, alpha, nu, prolong_const, n_coarsest, f, x);
            ++k;
        }
        if (bc == OR_BC_PERIODIC) {
            double mean = 0.0;
            for (i64 c = 0; c < m; ++c) mean += x[c];
            mean /= (double)m;
            for (i64 c = 0; c < m; ++c) x[c] -= mean;
        }
    }
    if (cycles_out) *cycles_out = k;
    if (rel_res_out) *rel_res_out = rr;
    free(f); free(r);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Implicit advection-diffusion: the backward-Euler step of Section 2.2 (the
 * implicit advection-diffusion equation and its filter), solved by multigrid
 * in Section 3.2.  The operator is
 *   A T = T + dt * sum_e a_e D_e T + nu * dt * (2d T_c - sum of the 2d face
 *         neighbours) / h^2,
 * with D_e the derivative along axis e: upwind (scheme 0: the backward
 * difference (T_c - T_-e)/h for a_e >= 0, the forward one for a_e < 0) or
 * central (scheme 1: (T_+e - T_-e)/(2h)).  Constant coefficients; ghosts by
 * the boundary rule.  On coarser levels the same dt, nu and a with the
 * level's spacing. */
typedef struct {
    int d, bc, scheme;
    double dt, nu, a[3];
} or_adop;

/* The operator's centre weight c0 and its weights on the -e and +e neighbours. */
static void adop_weights(const or_adop *op, double h, double *c0, double *cm, double *cp)
{
    const double dif = op->nu * op->dt / (h * h);
    *c0 = 1.0 + 2.0 * op->d * dif;
    for (int e = 0; e < op->d; ++e) {
        const double ad = op->a[e] * op->dt / h;
        cm[e] = -dif;
        cp[e] = -dif;
        if (op->scheme == 0) {
            if (op->a[e] >= 0.0) { *c0 += ad; cm[e] -= ad; }
            else { *c0 -= ad; cp[e] += ad; }
        } else {
            cm[e] -= 0.5 * ad;
            cp[e] += 0.5 * ad;
        }
    }
}

/* y = A x on a grid of n cells per axis and spacing h. */
void or_ad_apply(const or_adop *op, i64 n, double h, const double *x, double *y)
{
    const int d = op->d;
    double c0, cm[3], cp[3];
    adop_weights(op, h, &c0, cm, cp);
    const i64 nz = d == 3 ? n : 1;
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 c = (k * n + j) * n + i;
                double s = c0 * x[c];
                s += cm[0] * ghost_at(x, d, n, op->bc, i - 1, j, k) + cp[0] * ghost_at(x, d, n, op->bc, i + 1, j, k);
                s += cm[1] * ghost_at(x, d, n, op->bc, i, j - 1, k) + cp[1] * ghost_at(x, d, n, op->bc, i, j + 1, k);
                if (d == 3)
                    s += cm[2] * ghost_at(x, d, n, op->bc, i, j, k - 1) + cp[2] * ghost_at(x, d, n, op->bc, i, j, k + 1);
                y[c] = s;
            }
}

static void ad_residual(const or_adop *op, i64 n, double h, const double *f, const double *x, double *r)
{
    or_ad_apply(op, n, h, x, r);
    const i64 m = ncells(op->d, n);
    for (i64 c = 0; c < m; ++c) r[c] = f[c] - r[c];
}

/* Weighted Jacobi on the operator: x_out = x + omega (f - A x) / c0. */
void or_ad_jacobi(const or_adop *op, i64 n, double h, double omega, const double *f, const double *x_in,
                  double *x_out)
{
    double c0, cm[3], cp[3];
    adop_weights(op, h, &c0, cm, cp);
    or_ad_apply(op, n, h, x_in, x_out);
    const i64 m = ncells(op->d, n);
    for (i64 c = 0; c < m; ++c) x_out[c] = x_in[c] + omega * (f[c] - x_out[c]) / c0;
}

/* Exact solve on the coarsest grid: the matrix assembled column by column
 * from the operator, Gaussian elimination with partial pivoting (A is not
 * symmetric); x <- x + A^{-1} (f - A x). */
int or_ad_coarse_solve(const or_adop *op, i64 n, double h, const double *f, double *x)
{
    const i64 m = ncells(op->d, n);
    double *a = malloc(sizeof(double) * m * m), *e = calloc(m, sizeof(double));
    double *col = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    for (i64 j = 0; j < m; ++j) {
        e[j] = 1.0;
        or_ad_apply(op, n, h, e, col);
        e[j] = 0.0;
        for (i64 i = 0; i < m; ++i) a[i * m + j] = col[i];
    }
    ad_residual(op, n, h, f, x, r);
    int st = OR_OK;
    for (i64 p = 0; p < m && st == OR_OK; ++p) {
        i64 piv = p;
        for (i64 i = p + 1; i < m; ++i)
            if (fabs(a[i * m + p]) > fabs(a[piv * m + p])) piv = i;
        if (!(fabs(a[piv * m + p]) > 0.0)) { st = OR_EINVAL; break; }
        if (piv != p) {
            for (i64 q = 0; q < m; ++q) { const double t = a[p * m + q]; a[p * m + q] = a[piv * m + q]; a[piv * m + q] = t; }
            const double t = r[p]; r[p] = r[piv]; r[piv] = t;
        }
        for (i64 i = p + 1; i < m; ++i) {
            const double l = a[i * m + p] / a[p * m + p];
            for (i64 q = p; q < m; ++q) a[i * m + q] -= l * a[p * m + q];
            r[i] -= l * r[p];
        }
    }
    if (st == OR_OK) {
        for (i64 i = m - 1; i >= 0; --i) {
            double t = r[i];
            for (i64 q = i + 1; q < m; ++q) t -= a[i * m + q] * r[q];
            r[i] = t / a[i * m + i];
        }
        for (i64 i = 0; i < m; ++i) x[i] += r[i];
    }
    free(a); free(e); free(col); free(r);
    return st;
}

/* One V(nu1, nu2) cycle of the operator (the steps of or_vcycle with this
 * operator, its Jacobi and its exact coarsest solve). */
int or_ad_vcycle(const or_adop *op, i64 n, double h, int nu1, int nu2, double omega, i64 n_coarsest,
                 const double *f, double *x)
{
    const int d = op->d;
    if (n <= n_coarsest) return or_ad_coarse_solve(op, n, h, f, x);
    const i64 m = ncells(d, n), nc = n / 2, mc = ncells(d, nc);
    double *t = malloc(sizeof(double) * m);
    double *fc = malloc(sizeof(double) * mc), *ec = calloc(mc, sizeof(double));
    for (int s = 0; s < nu1; ++s) {
        or_ad_jacobi(op, n, h, omega, f, x, t);
        memcpy(x, t, sizeof(double) * m);
    }
    ad_residual(op, n, h, f, x, t);
    or_restrict(d, n, t, fc);
    int st = or_ad_vcycle(op, nc, 2.0 * h, nu1, nu2, omega, n_coarsest, fc, ec);
    or_prolong_add(d, nc, op->bc, ec, x);
    for (int s = 0; s < nu2; ++s) {
        or_ad_jacobi(op, n, h, omega, f, x, t);
        memcpy(x, t, sizeof(double) * m);
    }
    free(t); free(fc); free(ec);
    return st;
}

/* One sawtooth cycle of the operator (the steps of or_sawtooth with this
 * operator; its centre weight c0 plays the role of A_00). */
int or_ad_sawtooth(const or_adop *op, i64 n, double h, double alpha, int nu, int prolong_const, i64 n_coarsest,
                   const double *f, double *x)
{
    const int d = op->d;
    int L = 0;
    while ((n >> L) > n_coarsest) ++L;
    double **r = calloc(L + 1, sizeof(double *)), **e = calloc(L + 1, sizeof(double *));
    for (int l = 0; l <= L; ++l) {
        r[l] = malloc(sizeof(double) * ncells(d, n >> l));
        e[l] = calloc(ncells(d, n >> l), sizeof(double));
    }
    double *t = malloc(sizeof(double) * ncells(d, n));
    ad_residual(op, n, h, f, x, r[0]);
    for (int l = 0; l < L; ++l) or_restrict(d, n >> l, r[l], r[l + 1]);
    for (int l = L; l >= 0; --l) {
        const i64 nl = n >> l, ml = ncells(d, nl);
        const double hl = h * (double)((i64)1 << l);
        double c0, cm[3], cp[3];
        adop_weights(op, hl, &c0, cm, cp);
        for (i64 c = 0; c < ml; ++c) e[l][c] = r[l][c] / c0;
        if (l < L) {
            if (prolong_const) or_prolong_const_add(d, nl / 2, e[l + 1], e[l]);
            else or_prolong_add(d, nl / 2, op->bc, e[l + 1], e[l]);
        }
        for (int s = 0; s < nu; ++s) {
            or_ad_jacobi(op, nl, hl, alpha, r[l], e[l], t);
            memcpy(e[l], t, sizeof(double) * ml);
        }
    }
    const i64 m = ncells(d, n);
    for (i64 c = 0; c < m; ++c) x[c] += e[0][c];
    for (int l = 0; l <= L; ++l) { free(r[l]); free(e[l]); }
    free(r); free(e); free(t);
    return OR_OK;
}

/* Tolerance driver: from x = 0, cycles (cycle 0: V(nu1, nu2) with omega;
 * cycle 1: sawtooth with alpha = omega, nu2 steps, prolong_const) until
 * ||f - A x||_2 / ||f||_2 <= tol, tested before every cycle, or exactly
 * fixed_cycles cycles.  The operator is nonsingular for both boundary rules
 * (identity term), so no mean is removed.  hist as in or_mg_solve; l1diff
 * (may be NULL) receives the L1 norm of x_k - x_{k-1} after each cycle, the
 * paper's convergence gauge of Section 3.2. */
int or_ad_solve(const or_adop *op, i64 n, double h, const double *f, double *x, double tol, int cycle, int nu1,
                int nu2, double omega, int prolong_const, int max_cycles, int fixed_cycles, i64 n_coarsest,
                int *cycles_out, double *rel_res_out, double *hist, double *l1diff, int hist_len)
{
    const int d = op->d;
    if ((d != 2 && d != 3) || !is_pow2(n) || n < 4 || !is_pow2(n_coarsest) || n_coarsest < 1 || !(h > 0.0) ||
        !(tol > 0.0) || nu1 < 0 || nu2 < 0 || (cycle != 0 && cycle != 1))
        return OR_EINVAL;
    const i64 m = ncells(d, n);
    double *r = malloc(sizeof(double) * m), *xo = malloc(sizeof(double) * m);
    const double nf = sqrt(dot(m, f, f));
    int st = OR_OK, k = 0;
    double rr = 0.0;
    memset(x, 0, sizeof(double) * m);
    if (nf > 0.0) {
        for (;;) {
            ad_residual(op, n, h, f, x, r);
            rr = sqrt(dot(m, r, r)) / nf;
            if (hist && k < hist_len) hist[k] = rr;
            if (fixed_cycles > 0) {
                if (k >= fixed_cycles) break;
            } else {
                if (rr <= tol) break;
                if (k >= max_cycles || !(rr < 1e300)) { st = OR_ENOCONV; break; }
            }
            memcpy(xo, x, sizeof(double) * m);
            int s = cycle == 0 ? or_ad_vcycle(op, n, h, nu1, nu2, omega, n_coarsest, f, x)
                               : or_ad_sawtooth(op, n, h, omega, nu2, prolong_const, n_coarsest, f, x);
            if (s != OR_OK) { st = s; break; }
            if (l1diff && k < hist_len) {
                double l1 = 0.0;
                for (i64 c = 0; c < m; ++c) l1 += fabs(x[c] - xo[c]);
                l1diff[k] = l1;
            }
            ++k;
        }
    }
    if (cycles_out) *cycles_out = k;
    if (rel_res_out) *rel_res_out = rr;
    free(r); free(xo);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Scalar advection-diffusion step (Section 2.1, predictor-corrector of the
 * advection-diffusion filter).  With R(T) = sum_e a_e (T[+e] - T[-e])/(2h)
 * - nu (discrete Laplacian of T), the predictor is T~ = T^n - dt R(T^n) and
 * the corrector T^{n+1} = T^n - dt R((T~ + T^n)/2).  a holds d velocity
 * arrays at the cells (collocated; NULL for no advection).  The central
 * differences are the paper's first-derivative filters; the Laplacian is
 * the negative of the diffusion filter's action. */
static void ad_rate(int d, i64 n, double h, int bc, double nu, const double *const *a,
                    const double *T, double *R)
{
    const i64 nz = d == 3 ? n : 1;
    or_apply_A(d, n, h, bc, T, R); /* R = -Lap T */
    for (i64 c = 0; c < ncells(d, n); ++c) R[c] *= nu;
    if (!a) return;
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 c = (k * n + j) * n + i;
                double adv = a[0][c] * (ghost_at(T, d, n, bc, i + 1, j, k) - ghost_at(T, d, n, bc, i - 1, j, k))
                           + a[1][c] * (ghost_at(T, d, n, bc, i, j + 1, k) - ghost_at(T, d, n, bc, i, j - 1, k));
                if (d == 3)
                    adv += a[2][c] * (ghost_at(T, d, n, bc, i, j, k + 1) - ghost_at(T, d, n, bc, i, j, k - 1));
                R[c] += adv / (2.0 * h);
            }
}

int or_ad_scalar_step(int d, i64 n, double h, int bc, double *T, const double *const *a, double dt,
                      double nu)
{
    if ((d != 2 && d != 3) || n < 3 || !(h > 0.0)) return OR_EINVAL;
    const i64 m = ncells(d, n);
    double *R = malloc(sizeof(double) * m), *Tp = malloc(sizeof(double) * m);
    ad_rate(d, n, h, bc, nu, a, T, R);
    for (i64 c = 0; c < m; ++c) Tp[c] = T[c] - dt * R[c];            /* predictor */
    for (i64 c = 0; c < m; ++c) Tp[c] = 0.5 * (Tp[c] + T[c]);        /* T^{n+1/2} */
    ad_rate(d, n, h, bc, nu, a, Tp, R);
    for (i64 c = 0; c < m; ++c) T[c] = T[c] - dt * R[c];              /* corrector */
    free(R); free(Tp);
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Explicit advection-diffusion step with the filter families of Section 2.1
 * and Appendix A, the same predictor-corrector as or_ad_scalar_step:
 *   scheme 0: central first differences, 5-/7-point diffusion (Section 2.1);
 *   scheme 1: first-order upwind advection (Section 2.1's upwind filter, read
 *             with the value taken from upstream: backward difference for a
 *             positive velocity component, forward for a negative one), the
 *             same diffusion;
 *   scheme 2: the finite-element filters of Appendix A: 2D 9-point
 *             (bilinear) advection and diffusion, 3D 27-point (trilinear).
 * Tables below are the printed filters.  In 2D the row is the x offset and
 * the column the y offset (the paper's [T] matrix has rows l-1..l+1 and
 * columns m-1..m+1).  In 3D the first index is the slice: read as z+1, z,
 * z-1, which makes the printed z-advection filter +w dT/dz (the symmetric
 * filters do not depend on it).  Each table multiplies its prefactor:
 * diffusion nu/(4 h^2) (2D) and nu/(26 h^2) (3D), advection a_e/(12 h) (2D)
 * and a_e/(72 h) (3D); the rate is R = sum_e a_e (D_e T) + nu (diffusion
 * filter * T), every filter applied with the ghost rule of bc. */
static const double FE2_DIFF[3][3] = {{-1, -2, -1}, {-2, 12, -2}, {-1, -2, -1}};
static const double FE2_ADV[2][3][3] = {
    {{-1, -4, -1}, {0, 0, 0}, {1, 4, 1}},  /* x */
    {{-1, 0, 1}, {-4, 0, 4}, {-1, 0, 1}},  /* y */
};
static const double FE3_DIFF[3][3][3] = {
    {{-2, -3, -2}, {-3, -6, -3}, {-2, -3, -2}},
    {{-3, -6, -3}, {-6, 88, -6}, {-3, -6, -3}},
    {{-2, -3, -2}, {-3, -6, -3}, {-2, -3, -2}},
};
static const double FE3_ADV[3][3][3][3] = {
    { /* x */
        {{-1, -4, -1}, {0, 0, 0}, {1, 4, 1}},
        {{-4, -16, -4}, {0, 0, 0}, {4, 16, 4}},
        {{-1, -4, -1}, {0, 0, 0}, {1, 4, 1}},
    },
    { /* y */
        {{-1, 0, 1}, {-4, 0, 4}, {-1, 0, 1}},
        {{-4, 0, 4}, {-16, 0, 16}, {-4, 0, 4}},
        {{-1, 0, 1}, {-4, 0, 4}, {-1, 0, 1}},
    },
    { /* z */
        {{1, 4, 1}, {4, 16, 4}, {1, 4, 1}},
        {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}},
        {{-1, -4, -1}, {-4, -16, -4}, {-1, -4, -1}},
    },
};

/* Weight of a table at offset (dx, dy, dz). */
static double fe_w2(const double t[3][3], int dx, int dy) { return t[dx + 1][dy + 1]; }
static double fe_w3(const double t[3][3][3], int dx, int dy, int dz) { return t[1 - dz][dx + 1][dy + 1]; }

static void adx_rate(int d, i64 n, double h, int bc, int scheme, double nu, const double *const *a,
                     const double *T, double *R)
{
    const i64 nz = d == 3 ? n : 1;
    const int kz = d == 3 ? 1 : 0;
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 c = (k * n + j) * n + i;
                const double tc = T[c];
                double dif = 0.0, adv = 0.0;
                if (scheme == 2) {
                    for (int dz = -kz; dz <= kz; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                const double v = ghost_at(T, d, n, bc, i + dx, j + dy, k + dz);
                                if (d == 2) {
                                    dif += fe_w2(FE2_DIFF, dx, dy) * v;
                                    if (a)
                                        for (int e = 0; e < 2; ++e) adv += a[e][c] * fe_w2(FE2_ADV[e], dx, dy) * v;
                                } else {
                                    dif += fe_w3(FE3_DIFF, dx, dy, dz) * v;
                                    if (a)
                                        for (int e = 0; e < 3; ++e) adv += a[e][c] * fe_w3(FE3_ADV[e], dx, dy, dz) * v;
                                }
                            }
                    dif /= (d == 2 ? 4.0 : 26.0) * h * h;
                    adv /= (d == 2 ? 12.0 : 72.0) * h;
                } else {
                    for (int e = 0; e < d; ++e) {
                        const i64 o[3][2] = {{i - (e == 0), i + (e == 0)}, {j - (e == 1), j + (e == 1)},
                                             {k - (e == 2), k + (e == 2)}};
                        const double tm = ghost_at(T, d, n, bc, o[0][0], o[1][0], o[2][0]);
                        const double tp = ghost_at(T, d, n, bc, o[0][1], o[1][1], o[2][1]);
                        dif += 2.0 * tc - tm - tp;
                        if (!a) continue;
                        const double ae = a[e][c];
                        if (scheme == 0) adv += ae * (tp - tm) / (2.0 * h);
                        else adv += ae >= 0.0 ? ae * (tc - tm) / h : ae * (tp - tc) / h;
                    }
                    dif /= h * h;
                }
                R[c] = adv + nu * dif;
            }
}

int or_ad_explicit_step(int d, i64 n, double h, int bc, int scheme, double *T, const double *const *a,
                        double dt, double nu)
{
    if ((d != 2 && d != 3) || n < 3 || !(h > 0.0) || bc < 0 || bc > 2 || scheme < 0 || scheme > 2)
        return OR_EINVAL;
    const i64 m = ncells(d, n);
    double *R = malloc(sizeof(double) * m), *Tp = malloc(sizeof(double) * m);
    adx_rate(d, n, h, bc, scheme, nu, a, T, R);
    for (i64 c = 0; c < m; ++c) Tp[c] = T[c] - dt * R[c];            /* predictor */
    for (i64 c = 0; c < m; ++c) Tp[c] = 0.5 * (Tp[c] + T[c]);        /* T^{n+1/2} */
    adx_rate(d, n, h, bc, scheme, nu, a, Tp, R);
    for (i64 c = 0; c < m; ++c) T[c] = T[c] - dt * R[c];              /* corrector */
    free(R); free(Tp);
    return OR_OK;
}

/* The rate R(T) of or_ad_explicit_step alone (for the pins). */
int or_ad_explicit_rate(int d, i64 n, double h, int bc, int scheme, const double *T, const double *const *a,
                        double nu, double *R)
{
    if ((d != 2 && d != 3) || n < 3 || !(h > 0.0) || bc < 0 || bc > 2 || scheme < 0 || scheme > 2)
        return OR_EINVAL;
    adx_rate(d, n, h, bc, scheme, nu, a, T, R);
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Projection time step on a periodic staggered (MAC) grid (Section 2.4,
 * the projection algorithm).  Pressure p sits at cell centres; velocity
 * component q_c sits on the faces normal to axis c: q_c[idx] lives at
 * idx + e_c/2.  Periodic boundaries only. */

static i64 wrap_idx(int d, i64 n, i64 i, i64 j, i64 k)
{
    i = (i + n) % n; j = (j + n) % n; k = d == 3 ? (k + n) % n : 0;
    return (k * n + j) * n + i;
}

/* Divergence at cell centres: (D q)[idx] = sum_c (q_c[idx] - q_c[idx - e_c]) / h. */
void or_divergence(int d, i64 n, double h, const double *const *q, double *div)
{
    const i64 nz = d == 3 ? n : 1;
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 c = (k * n + j) * n + i;
                double s = (q[0][c] - q[0][wrap_idx(d, n, i - 1, j, k)])
                         + (q[1][c] - q[1][wrap_idx(d, n, i, j - 1, k)]);
                if (d == 3) s += q[2][c] - q[2][wrap_idx(d, n, i, j, k - 1)];
                div[c] = s / h;
            }
}

/* Gradient on faces: (G p)_c[idx] = (p[idx + e_c] - p[idx]) / h. */
void or_gradient(int d, i64 n, double h, const double *p, double *const *g)
{
    const i64 nz = d == 3 ? n : 1;
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 c = (k * n + j) * n + i;
                g[0][c] = (p[wrap_idx(d, n, i + 1, j, k)] - p[c]) / h;
                g[1][c] = (p[wrap_idx(d, n, i, j + 1, k)] - p[c]) / h;
                if (d == 3) g[2][c] = (p[wrap_idx(d, n, i, j, k + 1)] - p[c]) / h;
            }
}

/* Advecting velocity component e evaluated on the faces of component c.
 * e == c: the value on the face itself.  e != c: the average of the four
 * e-faces that surround the c-face, at idx, idx + e_c, idx - e_e and
 * idx + e_c - e_e. */
static double adv_vel(int d, i64 n, const double *const *a, int c, int e, i64 i, i64 j, i64 k)
{
    if (e == c) return a[e][wrap_idx(d, n, i, j, k)];
    i64 oc[3] = {0, 0, 0}, oe[3] = {0, 0, 0};
    oc[c] = 1; oe[e] = 1;
    return 0.25 * (a[e][wrap_idx(d, n, i, j, k)] + a[e][wrap_idx(d, n, i + oc[0], j + oc[1], k + oc[2])]
                 + a[e][wrap_idx(d, n, i - oe[0], j - oe[1], k - oe[2])]
                 + a[e][wrap_idx(d, n, i + oc[0] - oe[0], j + oc[1] - oe[1], k + oc[2] - oe[2])]);
}

/* Momentum rate for component c (Section 2.3 momentum form and the
 * discretised momentum equation of the projection algorithm, sigma = 0):
 *   F_c(q) = sum_e a_e (q_c[+e] - q_c[-e])/(2h) - nu Lap(q_c) + (G p)_c
 * with a = the lagged velocity u^n interpolated to the c-faces. */
static void mom_rate(int d, i64 n, double h, double nu, const double *const *a, const double *p,
                     int c, const double *qc, double *F)
{
    const i64 nz = d == 3 ? n : 1;
    const double inv_h2 = 1.0 / (h * h);
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 ix = (k * n + j) * n + i;
                double adv = 0.0, lap = -2.0 * d * qc[ix];
                for (int e = 0; e < d; ++e) {
                    i64 o[3] = {0, 0, 0};
                    o[e] = 1;
                    const double qp = qc[wrap_idx(d, n, i + o[0], j + o[1], k + o[2])];
                    const double qm = qc[wrap_idx(d, n, i - o[0], j - o[1], k - o[2])];
                    adv += adv_vel(d, n, a, c, e, i, j, k) * (qp - qm) / (2.0 * h);
                    lap += qp + qm;
                }
                i64 o[3] = {0, 0, 0};
                o[c] = 1;
                const double gp = (p[wrap_idx(d, n, i + o[0], j + o[1], k + o[2])] - p[ix]) / h;
                F[ix] = adv - nu * lap * inv_h2 + gp;
            }
}

/* Explicit momentum stages of the projection step: predictor
 * q~ = q^n - dt F(q^n), corrector q* = q^n - dt F((q~ + q^n)/2), advecting
 * velocity lagged at u^n (second-order predictor-corrector of Section 2.1
 * applied to each component, Section 2.3).  q is overwritten with q*. */
void or_ns_momentum(int d, i64 n, double h, double dt, double nu, double *const *q, const double *p)
{
    const i64 m = ncells(d, n);
    double *a[3] = {0, 0, 0}, *F = malloc(sizeof(double) * m), *half[3] = {0, 0, 0};
    for (int c = 0; c < d; ++c) {
        a[c] = malloc(sizeof(double) * m);
        memcpy(a[c], q[c], sizeof(double) * m);
        half[c] = malloc(sizeof(double) * m);
    }
    for (int c = 0; c < d; ++c) {
        mom_rate(d, n, h, nu, (const double *const *)a, p, c, a[c], F);
        for (i64 x = 0; x < m; ++x) half[c][x] = 0.5 * ((a[c][x] - dt * F[x]) + a[c][x]);
    }
    for (int c = 0; c < d; ++c) {
        mom_rate(d, n, h, nu, (const double *const *)a, p, c, half[c], F);
        for (i64 x = 0; x < m; ++x) q[c][x] = a[c][x] - dt * F[x];
    }
    for (int c = 0; c < d; ++c) { free(a[c]); free(half[c]); }
    free(F);
}

/* Full projection step (the projection algorithm of Section 2.4):
 *  1. momentum predictor-corrector to q* with the old pressure gradient;
 *  2. pressure correction: A dp = -(1/dt) D q*, A = -Lap (the paper's
 *     positive filter), solved by the multigrid driver from a zero guess;
 *  3. velocity correction dq = -dt G dp (explicit gradient);
 *  4. p <- p + dp;  5. q <- q* + dq.
 * Periodic boundaries.  Solver settings as for or_mg_solve. */
int or_ns_step(int d, i64 n, double h, double *u, double *v, double *w, double *p, double dt,
               double nu, double tol, int nu1, int nu2, double omega, int max_cycles,
               int fixed_cycles, i64 n_coarsest, int *cycles_out, double *rel_res_out)
{
    if ((d != 2 && d != 3) || (d == 3 && !w) || !(dt > 0.0) || nu < 0.0) return OR_EINVAL;
    const i64 m = ncells(d, n);
    double *q[3] = {u, v, w};
    or_ns_momentum(d, n, h, dt, nu, q, p);
    double *rhs = malloc(sizeof(double) * m), *dp = calloc(m, sizeof(double));
    or_divergence(d, n, h, (const double *const *)q, rhs);
    for (i64 c = 0; c < m; ++c) rhs[c] *= -1.0 / dt;
    int st = or_mg_solve(d, n, h, OR_BC_PERIODIC, rhs, dp, tol, nu1, nu2, omega, max_cycles,
                         fixed_cycles, 0, n_coarsest, cycles_out, rel_res_out, NULL, 0);
    double *g[3] = {0, 0, 0};
    for (int c = 0; c < d; ++c) g[c] = malloc(sizeof(double) * m);
    or_gradient(d, n, h, dp, g);
    for (int c = 0; c < d; ++c)
        for (i64 x = 0; x < m; ++x) q[c][x] -= dt * g[c][x];
    for (i64 x = 0; x < m; ++x) p[x] += dp[x];
    for (int c = 0; c < d; ++c) free(g[c]);
    free(rhs); free(dp);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Projection step on a collocated grid with the paper's own discretisation
 * choices (Section 2.4: velocity and pressure at the same nodes, the
 * finite-element filters of Appendix A for the advection and diffusion
 * terms, the projection algorithm), periodic boundaries.  scheme as in
 * or_ad_explicit_step (0 central, 1 upwind advection, 2 finite element).
 * The first derivative D_e of the scheme (the finite-element filter for
 * scheme 2, the central difference otherwise) gives the pressure gradient
 * and the divergence; the pressure equation uses the multigrid operator
 * A = -Lap_h, so D.D differs from -A and the projection is approximate. */

/* g = D_e f (periodic). */
void or_nsc_derivative(int d, i64 n, double h, int scheme, int e, const double *f, double *g)
{
    const i64 nz = d == 3 ? n : 1;
    const int kz = d == 3 ? 1 : 0;
    for (i64 k = 0; k < nz; ++k)
        for (i64 j = 0; j < n; ++j)
            for (i64 i = 0; i < n; ++i) {
                const i64 c = (k * n + j) * n + i;
                double s = 0.0;
                if (scheme == 2) {
                    for (int dz = -kz; dz <= kz; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                const double v = ghost_at(f, d, n, OR_BC_PERIODIC, i + dx, j + dy, k + dz);
                                s += (d == 2 ? fe_w2(FE2_ADV[e], dx, dy) : fe_w3(FE3_ADV[e], dx, dy, dz)) * v;
                            }
                    s /= (d == 2 ? 12.0 : 72.0) * h;
                } else {
                    const i64 o[3] = {e == 0, e == 1, e == 2};
                    s = (ghost_at(f, d, n, OR_BC_PERIODIC, i + o[0], j + o[1], k + o[2]) -
                         ghost_at(f, d, n, OR_BC_PERIODIC, i - o[0], j - o[1], k - o[2])) / (2.0 * h);
                }
                g[c] = s;
            }
}

/* Momentum predictor-corrector (the projection algorithm's first step,
 * sigma = 0) on collocated components q_c, advected by the lagged u^n = q^n:
 *   R_c(w) = sum_e u^n_e D_e w + nu (diffusion filter * w) + D_c p^n,
 *   q~_c = q^n_c - dt R_c(q^n_c),  q*_c = q^n_c - dt R_c((q~_c + q^n_c)/2),
 * the advection and diffusion filters those of or_ad_explicit_step. */
void or_nsc_momentum(int d, i64 n, double h, int scheme, double dt, double nu, double *const *q, const double *p)
{
    const i64 m = ncells(d, n);
    double *qn[3] = {0, 0, 0}, *R = malloc(sizeof(double) * m), *g = malloc(sizeof(double) * m);
    double *half = malloc(sizeof(double) * m);
    for (int c = 0; c < d; ++c) {
        qn[c] = malloc(sizeof(double) * m);
        memcpy(qn[c], q[c], sizeof(double) * m);
    }
    for (int c = 0; c < d; ++c) {
        or_nsc_derivative(d, n, h, scheme, c, p, g);
        adx_rate(d, n, h, OR_BC_PERIODIC, scheme, nu, (const double *const *)qn, qn[c], R);
        for (i64 x = 0; x < m; ++x) half[x] = 0.5 * ((qn[c][x] - dt * (R[x] + g[x])) + qn[c][x]);
        adx_rate(d, n, h, OR_BC_PERIODIC, scheme, nu, (const double *const *)qn, half, R);
        for (i64 x = 0; x < m; ++x) q[c][x] = qn[c][x] - dt * (R[x] + g[x]);
    }
    for (int c = 0; c < d; ++c) free(qn[c]);
    free(R); free(g); free(half);
}

/* The pressure-correction and velocity-correction steps: A dp = -(1/dt)
 * sum_e D_e q*_e (multigrid, periodic, mean-free), q = q* - dt D dp, p += dp.
 * dp_out (may be NULL) receives dp. */
int or_nsc_project(int d, i64 n, double h, int scheme, double dt, double *const *q, double *p, double tol,
                   int fixed_cycles, int *cycles_out, double *dp_out)
{
    const i64 m = ncells(d, n);
    double *rhs = calloc(m, sizeof(double)), *g = malloc(sizeof(double) * m), *dp = calloc(m, sizeof(double));
    for (int e = 0; e < d; ++e) {
        or_nsc_derivative(d, n, h, scheme, e, q[e], g);
        for (i64 x = 0; x < m; ++x) rhs[x] += g[x];
    }
    for (i64 x = 0; x < m; ++x) rhs[x] *= -1.0 / dt;
    double rr;
    int st = or_mg_solve(d, n, h, OR_BC_PERIODIC, rhs, dp, tol, 2, 2, 2.0 / 3.0, 200, fixed_cycles, 0, 4,
                         cycles_out, &rr, NULL, 0);
    for (int e = 0; e < d; ++e) {
        or_nsc_derivative(d, n, h, scheme, e, dp, g);
        for (i64 x = 0; x < m; ++x) q[e][x] -= dt * g[x];
    }
    for (i64 x = 0; x < m; ++x) p[x] += dp[x];
    if (dp_out) memcpy(dp_out, dp, sizeof(double) * m);
    free(rhs); free(g); free(dp);
    return st;
}

/* One collocated projection step: momentum, then the projection. */
int or_nsc_step(int d, i64 n, double h, int scheme, double dt, double nu, double *const *q, double *p, double tol,
                int fixed_cycles, int *cycles_out)
{
    if ((d != 2 && d != 3) || !is_pow2(n) || n < 4 || !(dt > 0.0) || nu < 0.0 || scheme < 0 || scheme > 2)
        return OR_EINVAL;
    or_nsc_momentum(d, n, h, scheme, dt, nu, q, p);
    return or_nsc_project(d, n, h, scheme, dt, q, p, tol, fixed_cycles, cycles_out, NULL);
}

/* ---------------------------------------------------------------------- */
/* Thread count of the OpenMP loops in the host-timing build (nthreads > 0
 * sets it); returns the count in effect: 1 in the test build. */
#ifdef _OPENMP
#include <omp.h>
#endif
int or_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

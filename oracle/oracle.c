/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, single-threaded CPU implementation (IEEE double, round to
 * nearest) of what the GPU library computes, used only by the tests, by the
 * package's smoke check and by the benchmark's CPU-baseline leg.  It shares no
 * code, header or constant with the HIP library and imports nothing from it.
 *
 * What it follows (arXiv 2212.11675, "Gaia AVU-GSR parallel solver ..."):
 *   - Section 3 (coefficient matrix structure) and Algorithm 1 / Algorithm 2
 *     (OpenMP columns) for the compressed row format and the two products
 *     aprod 1 (y += A x) and aprod 2 (x += A^T y);
 *   - Section 2 (related work, the PC-LSQR paragraph) for the column-norm
 *     preconditioner: divide each column by its norm, keep the factors in p,
 *     multiply the solution by p at the end;
 *   - Section 3 (the flowchart paragraph) for the initial aprod 2 call and the
 *     LSQR loop, and Paige & Saunders (1982, ACM TOMS 8(1), Section 4,
 *     "Algorithm LSQR") for the bidiagonalization / Givens recurrences, which
 *     the paper cites but does not print.
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - the per-row map holds the star number and the attitude start t relative
 *     to the attitude section; axis a of the attitude block starts at
 *     5*n_stars + a*n_dfa + t (Algorithm 1, attitude loop);
 *   - instrumental column j of row i is 5*n_stars + 3*n_dfa + instr[6i+j];
 *     the global column is 5*n_stars + 3*n_dfa + n_instr;
 *   - "norm of the column" is the Euclidean norm and p holds its reciprocal;
 *     an all-zero column gets p = 0;
 *   - the stopping rule is Paige & Saunders' tests (atol/btol, the condition
 *     estimate against conlim, and the same three at machine precision), or a
 *     fixed iteration count; an exact breakdown (alpha or beta = 0) always stops;
 *   - the variances the paper updates every iteration (Section 3, flowchart
 *     paragraph) are Paige & Saunders' estimate of diag((A^T A)^-1): the sum over
 *     the iterations of (w_i / rho_i)^2 in the preconditioned unknowns, multiplied
 *     by p^2 at the end like the solution is multiplied by p;
 *   - the constraint equations (Section 3: extra equations that make the
 *     solution unique; Algorithms 1 and 2 end with a "constraints
 *     computation" region after the observation rows) are sparse rows C,
 *     given by the caller, appended below the observation rows: the system
 *     becomes [A; C] x ~ [b; c].  aprod 1 writes their entries after the n_rows
 *     observation entries of y, aprod 2 adds C^T y_c after the observation part,
 *     and the column norms of the preconditioner include them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n_rows;
    int64_t n_stars;
    int32_t n_dfa;
    int32_t n_instr;
    int32_t n_glob;
} or_dims;

typedef struct {
    int32_t itn;     /* iterations performed                                  */
    int32_t istop;   /* 0 limit, 1 test1 (compatible), 2 test2 (LS), 3 exact
                        breakdown, 4 zero right-hand side, 5 acond > conlim,
                        6/7/8 test1/test2/1/acond at machine precision         */
    double rnorm;    /* ||b - B z|| estimate  (phibar)                        */
    double arnorm;   /* ||B^T (b - B z)|| estimate (phibar * alpha * |c|)     */
    double anorm;    /* Frobenius estimate of ||B||                           */
    double znorm;    /* ||z|| (exact)                                         */
    double bnorm;    /* ||b||                                                 */
    double acond;    /* estimate of cond(B) = ||B||_F ||B^+||_F: anorm times
                        sqrt(sum ||w_i / rho_i||^2)                           */
} or_info;

/* Constraint equations: n_con sparse rows in compressed row form; row k holds
 * val[ptr[k] .. ptr[k+1]-1] at the absolute columns col[...] (repeated columns
 * add up).  A NULL or_con means no constraint rows. */
typedef struct {
    int64_t n_con;
    const int64_t *ptr;
    const int64_t *col;
    const double *val;
} or_con;

static int64_t con_rows(const or_con *con) { return con ? con->n_con : 0; }

/* Number of unknowns: astrometric, attitude, instrumental and global sections. */
int64_t or_n_cols(const or_dims *d)
{
    return 5 * d->n_stars + 3 * (int64_t)d->n_dfa + d->n_instr + d->n_glob;
}

/* Column of coefficient k (0..23) of row i, following the slot order of the
 * compressed row (Section 3: 5 astrometric, 12 attitude, 6 instrumental, 1
 * global) and the index expressions of Algorithm 1. */
static int64_t col_of(const or_dims *d, const int32_t *star, const int32_t *att,
                      const int32_t *instr, int64_t i, int k)
{
    const int64_t att0 = 5 * d->n_stars;
    const int64_t ins0 = att0 + 3 * (int64_t)d->n_dfa;
    const int64_t glb0 = ins0 + d->n_instr;
    if (k < 5)
        return 5 * (int64_t)star[i] + k;
    if (k < 17) {
        const int axis = (k - 5) / 4, j = (k - 5) % 4;
        return att0 + (int64_t)axis * d->n_dfa + att[i] + j;
    }
    if (k < 23)
        return ins0 + instr[6 * i + (k - 17)];
    return glb0;
}

/* aprod 1 (Algorithm 1): y[i] += sum_k A_d[i,k] x[col(i,k)], rows in order,
 * coefficients in slot order; then the constraint rows ("constraints
 * computation"): y[n_rows + k] += sum_e val[e] x[col[e]]. */
void or_aprod1(const or_dims *d, const double *vals, const int32_t *star, const int32_t *att,
               const int32_t *instr, const or_con *con, const double *x, double *y)
{
    for (int64_t i = 0; i < d->n_rows; ++i) {
        double sum = 0.0;
        for (int k = 0; k < 24; ++k)
            sum += vals[24 * i + k] * x[col_of(d, star, att, instr, i, k)];
        y[i] += sum;
    }
    for (int64_t k = 0; k < con_rows(con); ++k) {
        double sum = 0.0;
        for (int64_t e = con->ptr[k]; e < con->ptr[k + 1]; ++e)
            sum += con->val[e] * x[con->col[e]];
        y[d->n_rows + k] += sum;
    }
}

/* aprod 2 (Algorithm 2): x[col(i,k)] += A_d[i,k] * y[i], rows in order; then the
 * constraint rows: x[col[e]] += val[e] * y[n_rows + k]. */
void or_aprod2(const or_dims *d, const double *vals, const int32_t *star, const int32_t *att,
               const int32_t *instr, const or_con *con, const double *y, double *x)
{
    for (int64_t i = 0; i < d->n_rows; ++i)
        for (int k = 0; k < 24; ++k)
            x[col_of(d, star, att, instr, i, k)] += vals[24 * i + k] * y[i];
    for (int64_t k = 0; k < con_rows(con); ++k)
        for (int64_t e = con->ptr[k]; e < con->ptr[k + 1]; ++e)
            x[con->col[e]] += con->val[e] * y[d->n_rows + k];
}

/* Column-norm preconditioner (Section 2, PC-LSQR paragraph):
 * p[j] = 1 / ||[A; C] e_j||_2, or 0 for an all-zero column. */
void or_colnorm(const or_dims *d, const double *vals, const int32_t *star, const int32_t *att,
                const int32_t *instr, const or_con *con, double *p)
{
    const int64_t n = or_n_cols(d);
    double *ss = calloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < d->n_rows; ++i)
        for (int k = 0; k < 24; ++k) {
            const double a = vals[24 * i + k];
            ss[col_of(d, star, att, instr, i, k)] += a * a;
        }
    for (int64_t k = 0; k < con_rows(con); ++k)
        for (int64_t e = con->ptr[k]; e < con->ptr[k + 1]; ++e)
            ss[con->col[e]] += con->val[e] * con->val[e];
    for (int64_t j = 0; j < n; ++j)
        p[j] = ss[j] > 0.0 ? 1.0 / sqrt(ss[j]) : 0.0;
    free(ss);
}

/* ----------------------------------------------------------------------------------------
 * The operator LSQR works on.  B = A D with D = diag(p) (p == NULL: D = I), or its
 * transpose B = D A^T when `transpose` is set (used by the adjoint solve).
 * mv:  y += B x      rmv: x += B^T y
 */
typedef struct {
    const or_dims *d;
    const double *vals;
    const int32_t *star, *att, *instr;
    const or_con *con; /* constraint rows below A (NULL: none) */
    const double *p;
    int transpose;
    double *tmp; /* n_cols scratch */
} or_op;

static int64_t all_rows(const or_op *op) { return op->d->n_rows + con_rows(op->con); }
static int64_t op_rows(const or_op *op) { return op->transpose ? or_n_cols(op->d) : all_rows(op); }
static int64_t op_cols(const or_op *op) { return op->transpose ? all_rows(op) : or_n_cols(op->d); }

/* y += A (p o x) */
static void apply_AD(const or_op *op, const double *x, double *y)
{
    const int64_t n = or_n_cols(op->d);
    for (int64_t j = 0; j < n; ++j)
        op->tmp[j] = op->p ? op->p[j] * x[j] : x[j];
    or_aprod1(op->d, op->vals, op->star, op->att, op->instr, op->con, op->tmp, y);
}

/* x += p o (A^T y) */
static void apply_DAt(const or_op *op, const double *y, double *x)
{
    const int64_t n = or_n_cols(op->d);
    memset(op->tmp, 0, (size_t)n * sizeof(double));
    or_aprod2(op->d, op->vals, op->star, op->att, op->instr, op->con, y, op->tmp);
    for (int64_t j = 0; j < n; ++j)
        x[j] += op->p ? op->p[j] * op->tmp[j] : op->tmp[j];
}

static void op_mv(const or_op *op, const double *x, double *y)
{
    if (op->transpose)
        apply_DAt(op, x, y);
    else
        apply_AD(op, x, y);
}

static void op_rmv(const or_op *op, const double *y, double *x)
{
    if (op->transpose)
        apply_AD(op, y, x);
    else
        apply_DAt(op, y, x);
}

static double nrm2(const double *v, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += v[i] * v[i];
    return sqrt(s);
}

static void scal(double *v, int64_t n, double a)
{
    for (int64_t i = 0; i < n; ++i)
        v[i] *= a;
}

/*
 * LSQR (Paige & Saunders 1982, Section 4) on the operator `op`, right-hand side b,
 * starting from z = 0.  Writes the iterate z (in the operator's own unknowns).
 *
 *   beta_1 u_1 = b,  alpha_1 v_1 = B^T u_1,  w_1 = v_1,  phibar_1 = beta_1,  rhobar_1 = alpha_1
 *   for i = 1, 2, ...
 *     beta_{i+1} u_{i+1}  = B v_i - alpha_i u_i
 *     alpha_{i+1} v_{i+1} = B^T u_{i+1} - beta_{i+1} v_i
 *     rho_i = sqrt(rhobar_i^2 + beta_{i+1}^2), c_i = rhobar_i / rho_i, s_i = beta_{i+1} / rho_i
 *     theta_{i+1} = s_i alpha_{i+1}, rhobar_{i+1} = -c_i alpha_{i+1}
 *     phi_i = c_i phibar_i, phibar_{i+1} = s_i phibar_i
 *     z_i = z_{i-1} + (phi_i / rho_i) w_i,  w_{i+1} = v_{i+1} - (theta_{i+1} / rho_i) w_i
 *
 * Stopping (unless `fixed`): test1 ||r|| <= btol ||b|| + atol ||B|| ||z||,
 * test2 ||B^T r|| <= atol ||B|| ||r||, with ||r|| = phibar_{i+1},
 * ||B^T r|| = phibar_{i+1} alpha_{i+1} |c_i| and ||B||^2 estimated by
 * sum (alpha_i^2 + beta_{i+1}^2).  alpha or beta exactly zero ends the iteration.
 * Then, in this order: test3 = 1 / acond <= 1 / conlim (conlim > 0), and, at machine
 * precision (1 + t <= 1), t1 = test1 / (1 + ||B|| ||z|| / ||b||), test2 = ||B^T r|| /
 * (||B|| ||r||), test3; acond = ||B|| (sum_i ||w_i / rho_i||^2)^(1/2) (Paige & Saunders,
 * Section 5.1).
 * If `hist_rnorm` is not NULL it receives phibar_{i+1} for i = 1..itn.
 */
static int lsqr_core(const or_op *op, const double *b, int32_t itnlim, int32_t fixed, double atol,
                     double btol, double conlim, double *z, or_info *info, double *hist_rnorm,
                     double *var)
{
    const int64_t m = op_rows(op), n = op_cols(op);
    double *u = malloc((size_t)m * sizeof(double));
    double *v = calloc((size_t)n, sizeof(double));
    double *w = malloc((size_t)n * sizeof(double));
    memcpy(u, b, (size_t)m * sizeof(double));
    memset(z, 0, (size_t)n * sizeof(double));
    if (var)
        memset(var, 0, (size_t)n * sizeof(double));
    memset(info, 0, sizeof *info);

    double beta = nrm2(u, m);
    info->bnorm = beta;
    double alpha = 0.0;
    if (beta > 0.0) {
        scal(u, m, 1.0 / beta);
        op_rmv(op, u, v); /* the "initial" aprod 2 */
        alpha = nrm2(v, n);
    }
    if (alpha > 0.0)
        scal(v, n, 1.0 / alpha);
    memcpy(w, v, (size_t)n * sizeof(double));

    double rhobar = alpha, phibar = beta, anorm2 = 0.0, ddnorm = 0.0;
    const double ctol = conlim > 0.0 ? 1.0 / conlim : 0.0;
    info->rnorm = beta;
    info->arnorm = alpha * beta;
    if (beta == 0.0) {
        info->istop = 4;
        goto done;
    }
    if (alpha == 0.0) {
        info->istop = 3;
        goto done;
    }

    for (int32_t itn = 1; itn <= itnlim; ++itn) {
        /* beta u = B v - alpha u */
        scal(u, m, -alpha);
        op_mv(op, v, u);
        beta = nrm2(u, m);
        anorm2 += alpha * alpha + beta * beta;
        if (beta > 0.0) {
            scal(u, m, 1.0 / beta);
            /* alpha v = B^T u - beta v */
            scal(v, n, -beta);
            op_rmv(op, u, v);
            alpha = nrm2(v, n);
            if (alpha > 0.0)
                scal(v, n, 1.0 / alpha);
        }

        const double rho = sqrt(rhobar * rhobar + beta * beta);
        const double c = rhobar / rho, s = beta / rho;
        const double theta = s * alpha;
        rhobar = -c * alpha;
        const double phi = c * phibar;
        phibar = s * phibar;
        const double t1 = phi / rho, t2 = theta / rho;
        for (int64_t j = 0; j < n; ++j) {
            /* d = w / rho (w before its update): var += d^2, ddnorm += ||d||^2 */
            const double dj = w[j] / rho;
            if (var)
                var[j] += dj * dj;
            ddnorm += dj * dj;
            z[j] += t1 * w[j];
            w[j] = v[j] - t2 * w[j];
        }

        info->itn = itn;
        info->rnorm = phibar;
        info->arnorm = phibar * alpha * fabs(c);
        info->anorm = sqrt(anorm2);
        info->znorm = nrm2(z, n);
        info->acond = info->anorm * sqrt(ddnorm);
        if (hist_rnorm)
            hist_rnorm[itn - 1] = phibar;

        if (beta == 0.0 || alpha == 0.0) {
            info->istop = 3;
            break;
        }
        if (!fixed) {
            if (info->rnorm <= btol * info->bnorm + atol * info->anorm * info->znorm) {
                info->istop = 1;
                break;
            }
            if (info->arnorm <= atol * info->anorm * info->rnorm) {
                info->istop = 2;
                break;
            }
            /* the remaining tests of Paige & Saunders (Section 6): the condition estimate
             * against conlim, then the three tests with the tolerances at machine precision */
            const double test2 = info->arnorm / (info->anorm * info->rnorm);
            const double test3 = 1.0 / info->acond;
            const double t1 = (info->rnorm / info->bnorm) /
                              (1.0 + info->anorm * info->znorm / info->bnorm);
            if (test3 <= ctol) {
                info->istop = 5;
                break;
            }
            if (1.0 + t1 <= 1.0) {
                info->istop = 6;
                break;
            }
            if (1.0 + test2 <= 1.0) {
                info->istop = 7;
                break;
            }
            if (1.0 + test3 <= 1.0) {
                info->istop = 8;
                break;
            }
        }
    }
done:
    info->znorm = nrm2(z, n);
    free(u);
    free(v);
    free(w);
    return info->istop;
}

/*
 * PC-LSQR: solve min ||A x - b|| with the column-norm preconditioner.  LSQR runs on
 * A D (D = diag(p), p from or_colnorm; p == NULL runs plain LSQR on A) and the
 * solution is re-multiplied by p at the end (Section 3, flowchart paragraph).
 */
int or_pclsqr(const or_dims *d, const double *vals, const int32_t *star, const int32_t *att,
              const int32_t *instr, const or_con *con, const double *p, const double *b,
              int32_t itnlim,
              int32_t fixed, double atol, double btol, double conlim, double *x,
              or_info *info, double *hist_rnorm)
{
    const int64_t n = or_n_cols(d);
    or_op op = {d, vals, star, att, instr, con, p, 0, malloc((size_t)n * sizeof(double))};
    const int rc =
        lsqr_core(&op, b, itnlim, fixed, atol, btol, conlim, x, info, hist_rnorm, NULL);
    if (p)
        for (int64_t j = 0; j < n; ++j)
            x[j] *= p[j];
    free(op.tmp);
    return rc;
}

/*
 * PC-LSQR with the variance estimate: var[j] estimates diag((A^T A)^-1)_j (the
 * preconditioned sum of (w_i / rho_i)^2 times p_j^2).  The standard error of x_j
 * under independent residuals is sqrt(var[j]) * ||r|| / sqrt(n_rows - n_cols).
 */
int or_pclsqr_var(const or_dims *d, const double *vals, const int32_t *star,
                  const int32_t *att, const int32_t *instr, const or_con *con, const double *p,
                  const double *b,
                  int32_t itnlim, int32_t fixed, double atol, double btol, double conlim,
                  double *x, double *var, or_info *info)
{
    const int64_t n = or_n_cols(d);
    or_op op = {d, vals, star, att, instr, con, p, 0, malloc((size_t)n * sizeof(double))};
    const int rc = lsqr_core(&op, b, itnlim, fixed, atol, btol, conlim, x, info, NULL, var);
    if (p)
        for (int64_t j = 0; j < n; ++j) {
            x[j] *= p[j];
            var[j] *= p[j] * p[j];
        }
    free(op.tmp);
    return rc;
}

/*
 * Minimum-norm solution mu (length n_rows + n_con) of A^T mu = g (A with its constraint
 * rows): LSQR from zero on the transposed, row-scaled system D A^T mu = D g (same solution
 * set when p has no zeros).  Used by the adjoint of the least-squares solve.
 */
int or_lsqr_transposed(const or_dims *d, const double *vals, const int32_t *star,
                       const int32_t *att, const int32_t *instr, const or_con *con,
                       const double *p, const double *g,
                       int32_t itnlim, int32_t fixed, double atol, double btol, double conlim,
                       double *mu, or_info *info)
{
    const int64_t n = or_n_cols(d);
    double *rhs = malloc((size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j)
        rhs[j] = p ? p[j] * g[j] : g[j];
    or_op op = {d, vals, star, att, instr, con, p, 1, malloc((size_t)n * sizeof(double))};
    const int rc = lsqr_core(&op, rhs, itnlim, fixed, atol, btol, conlim, mu, info, NULL, NULL);
    free(op.tmp);
    free(rhs);
    return rc;
}

/* r = b - A x (over the observation and the constraint rows) */
void or_residual(const or_dims *d, const double *vals, const int32_t *star, const int32_t *att,
                 const int32_t *instr, const or_con *con, const double *b, const double *x,
                 double *r)
{
    const int64_t m = d->n_rows + con_rows(con);
    for (int64_t i = 0; i < m; ++i)
        r[i] = 0.0;
    or_aprod1(d, vals, star, att, instr, con, x, r);
    for (int64_t i = 0; i < m; ++i)
        r[i] = b[i] - r[i];
}

/*
 * Mixed-precision form: vals_lo holds the same coefficients rounded to binary32 and
 * widened back (exactly) to double (constraint rows, if any, stay binary64 on both
 * sides).  Residual correction:
 *   x_0 = 0, r_0 = b;  for k = 0, 1, ...:  d_k = PC-LSQR(A_lo, r_k) with p_lo from A_lo,
 *   x_{k+1} = x_k + d_k; stop when ||d_k|| <= refine_tol ||x_{k+1}||;
 *   otherwise r_{k+1} = b - A x_{k+1} with the double-precision coefficients.
 * The first inner solve takes at most inner_itnlim iterations, the later ones (which only
 * correct an error at the binary32 level) at most later_itnlim (0: inner_itnlim).  With
 * first_tol > 0 the first inner solve stops on the Paige & Saunders tests at
 * atol = btol = first_tol, the later ones at inner_atol, inner_btol.
 * Returns the number of outer steps; inner iteration counts go to inner_itn[k].
 */
int32_t or_refine(const or_dims *d, const double *vals, const double *vals_lo,
                  const int32_t *star, const int32_t *att, const int32_t *instr,
                  const or_con *con, const double *b, int32_t max_outer, double refine_tol,
                  int32_t inner_itnlim, int32_t later_itnlim, int32_t inner_fixed, double inner_atol,
                  double inner_btol, double first_tol, double *x, int32_t *inner_itn)
{
    const int64_t m = d->n_rows + con_rows(con), n = or_n_cols(d);
    double *p_lo = malloc((size_t)n * sizeof(double));
    double *r = malloc((size_t)m * sizeof(double));
    double *dx = malloc((size_t)n * sizeof(double));
    or_colnorm(d, vals_lo, star, att, instr, con, p_lo);
    memcpy(r, b, (size_t)m * sizeof(double));
    memset(x, 0, (size_t)n * sizeof(double));
    int32_t k = 0;
    while (k < max_outer) {
        or_info info;
        /* the correction solves after the first may take a shorter iteration limit */
        const int32_t itnlim = (k > 0 && later_itnlim > 0) ? later_itnlim : inner_itnlim;
        /* ... and the first one its own (looser) tolerance: its result cannot be closer to
         * the binary64 solution than the binary32 rounding of the coefficients allows */
        const double ta = (k == 0 && first_tol > 0.0) ? first_tol : inner_atol;
        const double tb = (k == 0 && first_tol > 0.0) ? first_tol : inner_btol;
        or_pclsqr(d, vals_lo, star, att, instr, con, p_lo, r, itnlim, inner_fixed, ta, tb, 0.0,
                  dx, &info, NULL);
        if (inner_itn)
            inner_itn[k] = info.itn;
        for (int64_t j = 0; j < n; ++j)
            x[j] += dx[j];
        ++k;
        if (nrm2(dx, n) <= refine_tol * nrm2(x, n))
            break;
        or_residual(d, vals, star, att, instr, con, b, x, r);
    }
    free(p_lo);
    free(r);
    free(dx);
    return k;
}

/*
 * Gradient of a loss L(x*) with respect to the stored coefficients, given
 * r = b - A x*, lam = (A^T A)^{-1} dL/dx* and mu = A lam (= dL/db):
 *   dL/dA[i, col] = r_i lam_col - mu_i x*_col   on the stored pattern.
 * (Differentiate the normal equations A^T A x = A^T b.)
 */
void or_grad_vals(const or_dims *d, const int32_t *star, const int32_t *att, const int32_t *instr,
                  const double *r, const double *mu, const double *x, const double *lam,
                  double *dvals)
{
    for (int64_t i = 0; i < d->n_rows; ++i)
        for (int k = 0; k < 24; ++k) {
            const int64_t c = col_of(d, star, att, instr, i, k);
            dvals[24 * i + k] = r[i] * lam[c] - mu[i] * x[c];
        }
}

/*
 * gsr.h -- C ABI of the MI355X (gfx950) PC-LSQR hot path of the Gaia AVU-GSR solver
 * (arXiv 2212.11675).
 *
 * The library solves  min || A x - b ||_2  for the astrometric observation matrix A of
 * Section 3 of the paper, stored in its compressed row form ("A_d", 24 coefficients per
 * row) with the per-row index map ("M_i": star number and attitude start; "I_c": six
 * instrumental indices).  Column order of the unknowns x (Section 3):
 *
 *     [ astrometric 5*n_stars | attitude 3*n_dfa | instrumental n_instr | global 1 ]
 *
 * Row i, slot k of `vals` (k = 0..23) multiplies
 *     k = 0..4    : x[5*star[i] + k]
 *     k = 5..16   : x[5*n_stars + a*n_dfa + att[i] + j],  a = (k-5)/4, j = (k-5)%4
 *     k = 17..22  : x[5*n_stars + 3*n_dfa + instr[6*i + (k-17)]]
 *     k = 23      : x[5*n_stars + 3*n_dfa + n_instr]
 * (index expressions of Algorithm 1; att and instr are stored relative to their section).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors) unless the
 *     comment says "host".  The caller owns them.  Buffers passed to gsr_lsqr_setup /
 *     gsr_batch_setup are referenced, not copied, and must stay valid and unchanged until
 *     the matching destroy call.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are stream-ordered and
 *     asynchronous except where the comment says the call synchronizes.
 *   - Errors are returned as gsr_status; nothing aborts or exits.  Arguments are checked on
 *     the host before any device work; gsr_last_error() gives a message for the last
 *     failing call on the calling thread.
 *   - A handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef GSR_H
#define GSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_ABI_VERSION 4

typedef enum gsr_status {
    GSR_OK = 0,
    GSR_E_INVAL = -1,       /* bad argument: null pointer, negative or inconsistent size   */
    GSR_E_LAYOUT = -2,      /* matrix data violates the layout (index out of range, stars
                               not sorted, all-zero column when not allowed)              */
    GSR_E_NOMEM = -3,       /* device allocation failed                                    */
    GSR_E_HIP = -4,         /* a HIP runtime call failed                                   */
    GSR_E_BREAKDOWN = -5,   /* non-finite value met inside the iteration                   */
    GSR_E_UNSUPPORTED = -6, /* valid request the library does not support                  */
    GSR_E_NODEVICE = -7     /* no usable gfx950 device                                     */
} gsr_status;

/* Sizes of one system (Section 3).  n_glob must be 1 (the PPN gamma column), n_dfa >= 4
 * (one 4-wide B-spline block per attitude axis), n_instr >= 6 (six distinct instrumental
 * columns per row).  n_cols = 5*n_stars + 3*n_dfa + n_instr + n_glob. */
typedef struct gsr_dims {
    int64_t n_rows;
    int64_t n_stars;
    int32_t n_dfa;
    int32_t n_instr;
    int32_t n_glob;
} gsr_dims;

typedef enum gsr_precision {
    GSR_F64 = 0, /* coefficients read as stored (binary64)                              */
    GSR_F32V = 1 /* coefficients read from a binary32 copy, binary64 accumulation, with
                    binary64 residual correction around the inner solves                */
} gsr_precision;

typedef struct gsr_setup_opts {
    int32_t build_f32;        /* 1: also build the library-owned binary32 coefficient copy
                                 (needed by the GSR_F32V entry points)                   */
    int32_t validate;         /* 1: check index ranges and star order on the device      */
    int32_t allow_empty_cols; /* 1: accept all-zero columns (their unknown is set to 0);
                                 0: such a column makes setup fail with GSR_E_LAYOUT      */
    int32_t reserved;
} gsr_setup_opts;

typedef struct gsr_solve_opts {
    int32_t itnlim;      /* maximum LSQR iterations (per inner solve in the F32V form)    */
    int32_t fixed_iters; /* 1: run exactly itnlim iterations; only an exact breakdown
                            (alpha or beta = 0) ends the iteration earlier               */
    double atol, btol;   /* Paige-Saunders tests, used when fixed_iters = 0:
                            ||r|| <= btol ||b|| + atol ||A D|| ||z||  or
                            ||(A D)^T r|| <= atol ||A D|| ||r||                          */
    int32_t precision;   /* gsr_precision                                                 */
    int32_t max_refine;  /* GSR_F32V: maximum outer residual-correction steps (>= 1)      */
    double refine_tol;   /* GSR_F32V: stop when ||dx|| <= refine_tol ||x||                */
    int32_t check_every; /* iterations between host reads of the stop flag (0 = 16)       */
    int32_t profile;     /* 1: launch the iterations one by one (no graph) with HIP events
                            around every product; averages go to gsr_solve_info           */
    double conlim;       /* used when fixed_iters = 0: stop once the condition estimate
                            acond of A D reaches conlim (0 = no limit).  After the atol /
                            btol and conlim tests, Paige & Saunders' three tests at
                            machine precision also stop the iteration (istop 6, 7, 8)    */
    int32_t refine_itnlim; /* GSR_F32V: iteration limit of the correction solves after the
                            first (0 = itnlim)                                          */
    int32_t reserved;
    double refine_first_tol; /* GSR_F32V, fixed_iters = 0: atol = btol of the first inner
                            solve (0 = atol, btol).  Its result cannot come closer to the
                            binary64 solution than the binary32 rounding of the
                            coefficients allows, so it may stop early; the correction
                            solves use atol, btol                                         */
} gsr_solve_opts;

typedef struct gsr_solve_info {
    int32_t itn;      /* LSQR iterations performed (summed over refinement steps)          */
    int32_t istop;    /* 0 itnlim reached, 1 compatible-system test, 2 least-squares test,
                         3 exact breakdown, 4 zero right-hand side, 5 acond >= conlim,
                         6 / 7 / 8 the compatible, least-squares and condition tests with
                         the tolerances at machine precision (1 + t <= 1)                 */
    int32_t n_refine; /* outer steps taken (GSR_F32V), 1 otherwise                         */
    int32_t nonfinite; /* 1 if a non-finite value stopped the recurrence                    */
    double rnorm;     /* estimate of ||b - A x|| (last inner solve)                        */
    double arnorm;    /* estimate of ||(A D)^T r||                                         */
    double anorm;     /* Frobenius estimate of ||A D||                                      */
    double znorm;     /* ||z||, z = x / p the preconditioned unknowns                      */
    double bnorm;     /* ||b|| (of the last inner right-hand side)                         */
    double ms_pass1;  /* profile = 1: mean duration per iteration of the row-ordered pass
                         (aprod 1, fused with the star-ordered part of aprod 2 when the
                         instrumental columns fit in LDS)                                   */
    double ms_pass2;  /* profile = 1: mean duration per iteration of the rest of aprod 2
                         (block-sum reduction and attitude pass; all of aprod 2 if unfused) */
    int32_t n_pass;   /* number of iterations averaged                                      */
    int32_t fused;    /* 1 if the row-ordered pass was fused                                */
    double acond;     /* estimate of cond(A D) = ||A D||_F ||(A D)^+||_F: anorm times
                         (sum_i ||w_i / rho_i||^2)^(1/2) (Paige & Saunders, Section 5.1);
                         after an exact breakdown it omits the last step's term           */
} gsr_solve_info;

typedef struct gsr_handle gsr_handle;

/* ABI version this library was built with (GSR_ABI_VERSION). */
int32_t gsr_abi_version(void);

/* Text for a status code; static storage. */
const char *gsr_status_string(gsr_status s);

/* Message for the last failing call on this thread ("" if none); thread-local storage. */
const char *gsr_last_error(void);

/*
 * Set up a system for the products and the solver (Section 3 layout, Section 2
 * column-norm preconditioning).
 *   dims   host; sizes as above.
 *   vals   [n_rows*24] binary64, row-major in the slot order above.
 *   star   [n_rows] int32, non-decreasing, in [0, n_stars)  (rows sorted by star).
 *   att    [n_rows] int32 in [0, n_dfa-4]: attitude start relative to the section.
 *   instr  [n_rows*6] int32 in [0, n_instr): instrumental indices relative to the section.
 *   opts   host, may be NULL (defaults: no f32 copy, validate, reject empty columns).
 *   out    host; receives the handle.
 * Computes the preconditioner p_j = 1/||A e_j||_2 (0 for an all-zero column) on the device.
 * Ownership: the four arrays stay the caller's and must stay allocated and unchanged while
 * the handle lives; the library also builds its own copies of them at setup (coefficient and
 * index tiles, a copy of the attitude coefficients grouped by attitude start, binary32
 * copies), so a change made after setup would reach only some of the products.  Set up a
 * new handle instead (or bring new values in with gsr_update_values).
 * Synchronizes `stream`.  Errors: GSR_E_INVAL, GSR_E_LAYOUT, GSR_E_NOMEM, GSR_E_HIP,
 * GSR_E_NODEVICE.
 */
gsr_status gsr_lsqr_setup(const gsr_dims *dims, const double *vals, const int32_t *star,
                          const int32_t *att, const int32_t *instr, const gsr_setup_opts *opts,
                          void *stream, gsr_handle **out);

/* Release the handle and everything it owns.  NULL is accepted. */
gsr_status gsr_destroy(gsr_handle *h);

/* Sizes of the handle's system (host out-pointers, any may be NULL): rows of the operator
 * (n_rows plus the constraint rows of gsr_set_constraints) and unknowns. */
gsr_status gsr_get_size(const gsr_handle *h, int64_t *n_rows, int64_t *n_cols);

/* aprod mode 1 (Section 3; Algorithm 1):  y[i] += sum_k A[i,k] x[col(i,k)].
 *   x [n_cols], y [n_rows], binary64; y is read and written.  Unpreconditioned A.
 *   With constraint rows (gsr_set_constraints) y has n_rows + n_con entries, y_c += C x last. */
gsr_status gsr_aprod1(gsr_handle *h, const double *x, double *y, void *stream);

/* aprod mode 2 (Section 3; Algorithm 2):  x[col(i,k)] += A[i,k] y[i]  (x += A^T y).
 *   y [n_rows], x [n_cols], binary64; x is read and written.  Unpreconditioned A.
 *   With constraint rows y has n_rows + n_con entries and x += C^T y_c as well.
 *   Summation order varies between calls (device atomics): results agree to rounding. */
gsr_status gsr_aprod2(gsr_handle *h, const double *y, double *x, void *stream);

/* The same two products with the binary32 coefficient copy (setup with build_f32 = 1),
 * products and sums in binary64.  GSR_E_UNSUPPORTED if the copy was not built. */
gsr_status gsr_aprod1_f32v(gsr_handle *h, const double *x, double *y, void *stream);
gsr_status gsr_aprod2_f32v(gsr_handle *h, const double *y, double *x, void *stream);

/* Copy the preconditioner p [n_cols] (Section 2: reciprocal column norms) into `p`
 * (device).  `precision` selects the factors of the binary64 or the binary32 coefficients. */
gsr_status gsr_precond(gsr_handle *h, int32_t precision, double *p, void *stream);

/* r = b - A x with the binary64 coefficients.  b, r [n_rows] ([n_rows + n_con] with
 * constraint rows); x [n_cols]. */
gsr_status gsr_residual(gsr_handle *h, const double *b, const double *x, double *r,
                        void *stream);

/*
 * PC-LSQR (Section 3 flowchart; LSQR of Paige & Saunders 1982 on A D, D = diag(p),
 * x = p o z at the end).  b [n_rows] ([n_rows + n_con] with constraint rows, their
 * right-hand side last), x [n_cols] output (the caller's buffer, overwritten).
 * opts host (NULL: 100 iterations, fixed, binary64); info host, may be NULL.
 * GSR_F32V runs  x_0 = 0, r_0 = b;  d_k = PC-LSQR(A_32, r_k);  x_{k+1} = x_k + d_k;
 * r_{k+1} = b - A x_{k+1} (binary64 coefficients) until ||d_k|| <= refine_tol ||x_{k+1}||
 * or max_refine steps.  Synchronizes `stream` (to read the stop flag and fill info).
 */
gsr_status gsr_lsqr_solve(gsr_handle *h, const double *b, double *x, const gsr_solve_opts *opts,
                          gsr_solve_info *info, void *stream);

/*
 * The same binary64 PC-LSQR plus the variances the paper updates every iteration (Section 3,
 * flowchart paragraph): Paige & Saunders' estimate of diag((A^T A)^-1), the running sum of
 * (w_i / rho_i)^2 in the preconditioned unknowns, multiplied by p^2 at the end like the
 * solution is multiplied by p.  var [n_cols] output (device).  The standard error of x_j
 * under independent residuals is sqrt(var_j) * info.rnorm / sqrt(n_rows - n_cols)
 * (n_rows > n_cols).  The estimate is complete only after a full Krylov space (n_cols
 * steps in exact arithmetic); fewer steps give a lower bound.  opts->precision must be
 * GSR_F64 (GSR_E_UNSUPPORTED otherwise).  Synchronizes `stream`.
 */
gsr_status gsr_lsqr_solve_var(gsr_handle *h, const double *b, double *x, double *var,
                              const gsr_solve_opts *opts, gsr_solve_info *info, void *stream);

/*
 * The PC-LSQR of gsr_lsqr_solve (Section 3, flowchart paragraph), stream-ordered: every
 * launch goes to `stream`, in order, with no host synchronization, no allocation and no
 * memset, so the call may be captured into a HIP graph (the graph then repeats the solve on
 * the current contents of b).  All opts->itnlim iterations are enqueued one kernel at a
 * time; once the device-side stop flag is set (fixed_iters = 0, or an exact breakdown) the
 * remaining launches return at once.  GSR_F32V (setup with build_f32 = 1, else
 * GSR_E_UNSUPPORTED): all opts->max_refine correction steps are enqueued, each with its
 * inner solve, the update x += d_k and the test ||d_k|| <= refine_tol ||x|| taken on the
 * device; once a test ends the loop, the launches of the later steps return at once.
 * When the stream reaches the end, x [n_cols] holds the solution and *info_dev (DEVICE
 * memory, one gsr_solve_info) the solve information (itn summed over the inner solves,
 * n_refine the correction steps taken; ms_pass1 = ms_pass2 = 0 and n_pass = 0); a
 * non-finite value sets info_dev->nonfinite instead of returning GSR_E_BREAKDOWN.
 * opts->profile must be 0 (GSR_E_INVAL).  The workspaces it uses belong to the handle and
 * are allocated by gsr_lsqr_setup: calls on one handle must not overlap (nor overlap any
 * other solve on the handle).
 */
gsr_status gsr_lsqr_solve_async(gsr_handle *h, const double *b, double *x,
                                const gsr_solve_opts *opts, gsr_solve_info *info_dev,
                                void *stream);

/*
 * Adjoint of the least-squares solve, for a loss L(x*) with g = dL/dx* [n_cols]:
 *   mu  [n_rows] = minimum-norm solution of A^T mu = g  (LSQR on D A^T, rhs D g) = dL/db
 *       ([n_rows + n_con] with constraint rows: A is then the stacked [A; C]),
 *   lam [n_cols] = argmin || A lam - mu ||               (PC-LSQR)  = (A^T A)^{-1} g.
 * opts as for gsr_lsqr_solve (binary64 only); info (host, may be NULL) receives two entries
 * (info[0] for mu, info[1] for lam).  Synchronizes `stream`.
 */
gsr_status gsr_lsqr_solve_adjoint(gsr_handle *h, const double *g, double *mu, double *lam,
                                  const gsr_solve_opts *opts, gsr_solve_info *info,
                                  void *stream);

/* dL/dvals[i*24+k] = r[i] lam[col(i,k)] - mu[i] x[col(i,k)]  (differentiating the normal
 * equations A^T A x = A^T b), with r = b - A x*.  r, mu [n_rows] (with constraint rows
 * [n_rows + n_con], of which the first n_rows are read); x, lam [n_cols]; dvals [n_rows*24]
 * output: the gradient of the observation coefficients only. */
gsr_status gsr_grad_vals(gsr_handle *h, const double *r, const double *mu, const double *x,
                         const double *lam, double *dvals, void *stream);

/*
 * New coefficient values for the handle's system, same index map (star, att, instr) and
 * sizes: the library's copies of the coefficients (row tiles, the copy grouped by attitude
 * start, the binary32 copies when built) are rebuilt in place and the preconditioner is
 * recomputed (Section 2), without the sort and the allocations of gsr_lsqr_setup.  For
 * callers that change the coefficients between solves (the differentiation form's training
 * loop).
 *   vals  [n_rows*24] binary64 (device), 16-byte aligned; referenced from now on in place of
 *         the array given to gsr_lsqr_setup (or to the previous call), under the same
 *         contract.
 * Must not overlap any other call on the handle.  Synchronizes `stream`.  Errors:
 * GSR_E_INVAL; GSR_E_LAYOUT if a column became all-zero and the handle was set up without
 * allow_empty_cols (the new values are in place all the same, with p = 0 for that column);
 * GSR_E_HIP.
 */
gsr_status gsr_update_values(gsr_handle *h, const double *vals, void *stream);

/*
 * Constraint equations (Section 3: the extra equations a unique solution needs; the
 * "constraints computation" region that closes Algorithms 1 and 2).  Attaches n_con sparse
 * rows C, in compressed row form, below the n_rows observation rows: from this call on every
 * product, residual and solve of the handle acts on the stacked [A; C], which has
 * n_rows + n_con rows (gsr_get_size reports them).  Row-space vectors -- y of the products,
 * b and r of gsr_residual, b of the solves, mu of the adjoint solve -- then hold
 * n_rows + n_con entries, the constraint rows last (their right-hand side c at the end of b).
 * The preconditioner is recomputed over [A; C]; the constraint coefficients stay binary64 in
 * the GSR_F32V form.
 *   n_con   rows of C; 0 removes the handle's constraint rows.
 *   ptr     [n_con + 1] int64 (device), ptr[0] = 0, non-decreasing: row k holds the entries
 *           ptr[k] .. ptr[k+1]-1 (a row may be empty).
 *   col     [ptr[n_con]] int64 (device), absolute columns in [0, n_cols); a column repeated
 *           within a row adds up.
 *   val     [ptr[n_con]] binary64 (device) coefficients.
 * The arrays are referenced, not copied (the library builds its own copy grouped by column):
 * they must stay valid and unchanged until the next gsr_set_constraints or gsr_destroy.  The
 * solve workspaces are reallocated (the row count changes), so the call must not overlap any
 * other call on the handle.  The batched API has no constraint rows.  Synchronizes `stream`.
 * Errors: GSR_E_INVAL, GSR_E_LAYOUT (ptr[0] != 0, ptr decreasing, column out of range),
 * GSR_E_UNSUPPORTED (n_con or ptr[n_con] above 2^31-1), GSR_E_NOMEM, GSR_E_HIP; after an
 * error the handle has no constraint rows.
 */
gsr_status gsr_set_constraints(gsr_handle *h, int64_t n_con, const int64_t *ptr,
                               const int64_t *col, const double *val, void *stream);

/*
 * aprod mode 2 (x += A^T y) straight on the caller's arrays, with no handle and no allocation:
 * for callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation), who therefore cannot call gsr_lsqr_setup either.
 * The arguments are those of gsr_lsqr_setup (dims host; vals [n_rows*24] binary64, star,
 * att [n_rows] int32, instr [n_rows*6] int32, device, same layout and sorting) plus y
 * [n_rows] and x [n_cols] (device; x is read and written), and the stream.  The kernels'
 * block partial sums of the instrumental and global columns live in a fixed device array of
 * the library (32 MiB, one per GPU the library runs on, held until the process ends); the
 * attitude columns take one atomic add per coefficient (no attitude-ordered copy without a
 * setup), so this is slower than gsr_aprod2.  Indices are not validated.  Every call on a GPU
 * shares that array: calls that overlap on one GPU (several streams or threads) race.
 * Errors: GSR_E_INVAL; GSR_E_UNSUPPORTED when n_instr exceeds 10240, the most one block's
 * LDS sums and the fixed array allow; GSR_E_NODEVICE; GSR_E_HIP.
 */
gsr_status gsr_aprod2_noalloc(const gsr_dims *dims, const double *vals, const int32_t *star,
                              const int32_t *att, const int32_t *instr, const double *y,
                              double *x, void *stream);

/* ---- batching: many independent systems, k right-hand sides each ------------------------ */

typedef struct gsr_batch gsr_batch;

/*
 * Set up n_sys independent systems stored back to back.
 *   dims        host [n_sys].
 *   row_offset  host [n_sys+1]: system s owns rows row_offset[s] .. row_offset[s+1]-1 of
 *               the concatenated arrays (row_offset[0] = 0).
 *   vals/star/att/instr  device, concatenated; indices are relative to each system; vals
 *               16-byte and instr 8-byte aligned (GSR_E_INVAL otherwise).
 *   k           right-hand sides per system, 1, 2, 4 or 8 (GSR_E_UNSUPPORTED otherwise).
 * Unknowns of system s occupy columns col_offset[s] .. col_offset[s+1]-1 of the batched
 * unknown vector (gsr_batch_col_offsets), each system in the column order above.
 * Synchronizes `stream`.
 */
gsr_status gsr_batch_setup(int32_t n_sys, const gsr_dims *dims, const int64_t *row_offset,
                           const double *vals, const int32_t *star, const int32_t *att,
                           const int32_t *instr, int32_t k, const gsr_setup_opts *opts,
                           void *stream, gsr_batch **out);
gsr_status gsr_batch_destroy(gsr_batch *b);

/* host out [n_sys+1] */
gsr_status gsr_batch_col_offsets(const gsr_batch *b, int64_t *col_offset);

/* Multi-RHS products over all systems at once (RHS-minor storage, element (row, j) at
 * row*k + j):  Y[i, j] += sum A[i,c] X[c, j]  and  X[c, j] += sum A[i,c] Y[i, j].  X and Y
 * must be 16-byte aligned (GSR_E_INVAL otherwise). */
gsr_status gsr_batch_aprod1(gsr_batch *b, const double *X, double *Y, void *stream);
gsr_status gsr_batch_aprod2(gsr_batch *b, const double *Y, double *X, void *stream);

/* PC-LSQR of every (system, rhs) pair: B [sum rows * k], X [sum cols * k] output, both
 * RHS-minor; each pair has its own scalars and stopping state.  info host [n_sys*k] or
 * NULL (entry s*k + j).  A non-finite value in any pair returns GSR_E_BREAKDOWN; info is
 * filled all the same and info[s*k + j].nonfinite names the pairs that broke down (the
 * others ran on to their own stop).  Synchronizes `stream`. */
gsr_status gsr_batch_solve(gsr_batch *b, const double *B, double *X, const gsr_solve_opts *opts,
                           gsr_solve_info *info, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */

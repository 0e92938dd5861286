/*
 * rsrr.h -- C ABI of the MI355X resolvent-sampling library (RSRR hot path).
 *
 * Method: the resolvent sampling based Rayleigh-Ritz method of Xiao, Zhang,
 * Huang and Sakurai for the nonlinear eigenvalue problem T(lambda) v = 0
 * (Sec. 1, eq. gnep).  The library owns the steps of the RSRR algorithm
 * (Sec. 4.3) that follow the choice of contour, points and probes:
 *
 *   rsrr_sample   Step 2 and eq. hatS: S = [T(z_0)^-1 U, ..., T(z_{N-1})^-1 U]
 *   rsrr_basis    Step 3: normalise the columns of S (Sec. 4.2) and keep the
 *                 left singular vectors with sigma > delta*sigma_1
 *   rsrr_project  Step 4, first half / eq. Ts-NEP: T_Q(z) = Q^H T(z) Q
 *   rsrr_solve    Step 4, second half, and Step 5: SS-FULL (Sec. 3.3) on the
 *                 projected NEP, lift v = Q g, residuals
 *   rsrr_moments  the moment matrix M = S Z of the moment scheme (Sec. 4.1)
 *   rsrr_two_stage        the two-stage strategy of Sec. 5.4 and Sec. 6: stage-1
 *                 eigenvalue estimates become extra sampling points
 *   rsrr_sample_batched   Step 2 for a ragged batch of NEP instances
 *   rsrr_sample_gmres     Step 2 with an iterative solver: flexible GMRES,
 *                 preconditioned by LU factors reused across points
 *   rsrr_server_* a request loop that runs all of the above for many NEPs at
 *                 once (continuous batching of their sampling points)
 *
 * plus rsrr_contour for the ellipse nodes and trapezoid weights of Sec. 5.1
 * (eq. ellip-contour, eq. ellip-contour-xw).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Complex numbers are interleaved pairs of doubles (re, im).  Matrices are
 *   column-major with an explicit leading dimension counted in complex
 *   elements.
 * - "device" pointers are HIP device memory on the context's device; "host"
 *   pointers are ordinary host memory.  Every buffer is owned by the caller;
 *   the library never frees or keeps a caller pointer after a call returns.
 * - Work is enqueued on the context's stream.  Calls that return host
 *   results (point info, k, sigma, eigenvalues) synchronise that stream
 *   before returning; device outputs are complete when the call returns.
 * - Return value: RSRR_OK (0); a negative value -i names the i-th argument
 *   (1-based) as invalid, and nothing was enqueued; a positive value is a
 *   numerical or runtime condition listed below.
 * - One context per host thread.  Calls on one context must not overlap.
 * - Exception: a server (rsrr_server_*) keeps the caller's request buffers
 *   until the request has finished (rsrr_server_wait returned it).
 */
#ifndef RSRR_H
#define RSRR_H

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define RSRR_API __attribute__((visibility("default")))
#else
#define RSRR_API
#endif

typedef int rsrr_status;

enum {
    RSRR_OK = 0,
    RSRR_ESINGULAR = 1,      /* an exact zero pivot: T(z_k) singular in working precision      */
    RSRR_WARN_FALLBACK = 2,  /* refinement stalled at some point; that point was redone in FP64 */
    RSRR_WARN_GAP = 3,       /* SS-FULL: largest singular-value gap below tol_gap (eq. gap)     */
    RSRR_ENOMEM = 4,         /* device allocation of workspace failed                         */
    RSRR_EDEVICE = 5,        /* a HIP runtime call failed                                      */
    RSRR_ENOTCONV = 6,       /* an iterative eigen/singular-value solve did not converge        */
    RSRR_ENAN = 7,           /* a NaN or Inf reached a pivot                                   */
    RSRR_ETIMEOUT = 8,       /* rsrr_server_wait: the request had not finished in time          */
    RSRR_ELIMIT = 9,         /* a size beyond a documented limit of the library (see the call)   */
    RSRR_WARN_MORE = 10      /* rsrr_solve: more eigenpairs than max_eigs; those of lowest
                                elliptic level were returned                                     */
};

/* Kinds of T(z).  SEPARABLE: T(z) = sum_j f_j(z) A_j (the form of every
 * example of Sec. 2.1 except the boundary-element kernels).  HELMHOLTZ: the
 * single-layer Nystrom matrix of a point set on a surface (kernel G of
 * eq. nyes): T_ij = w e^{i z r_ij} / (4 pi r_ij), T_ii = sqrt(w/pi)/2 + i z w/(4 pi).
 * SPARSE: the separable form with every A_j in compressed sparse row storage
 * (rsrr_csr), the storage of the finite-element models that Sec. 4.3 and
 * Sec. 6 solve with sparse direct and iterative solvers.  rsrr_sample forms
 * dense T(z_k) from it; rsrr_sample_gmres applies T(z_k) from the sparse
 * rows (the preconditioner is still a dense factorisation at the reference
 * points); rsrr_project forms A_j Q from the sparse rows; rsrr_solve and
 * rsrr_two_stage accept it; rsrr_sample_batched and the server refuse it. */
enum { RSRR_T_SEPARABLE = 0, RSRR_T_HELMHOLTZ = 1, RSRR_T_SPARSE = 2 };

/* One coefficient matrix of a SPARSE nep (n x n, compressed sparse rows, all
 * arrays on the device and owned by the caller): row i holds the entries
 * rowptr[i] .. rowptr[i+1]-1 (rowptr: n+1 ints, rowptr[0] = 0, rowptr[n] =
 * nnz); entry e lies in column col[e] (0-based) with the value
 * val[2e] + i val[2e+1].  The entries of a row may come in any order and a
 * repeated (row, column) pair is summed.  The device kernels check every row
 * range against [0, nnz] and every column against [0, n): an entry outside
 * is skipped and the call returns -2 (S or AQ then hold partial results). */
typedef struct {
    int nnz;
    int pad;
    const int *rowptr;
    const int *col;
    const double *val;
} rsrr_csr;

/* Arithmetic of the sampling step.  C128: complex FP64 LU and solves.
 * C64_IR: complex FP32 LU on the matrix cores, then iterative refinement
 * against FP64 residuals until FP64 backward error; a point that does not
 * converge is redone with the C128 path (flagged in rsrr_point_info).
 * R32_IR (rsrr_sample only): real sampling for a real NEP (Sec. 4.3 and
 * Sec. 5: real points, e.g. Chebyshev points of an interval): real FP32 LU
 * and solves, refined against the FP64 residual of the complex problem as
 * given; requires a SEPARABLE nep and real points.  A T(z_k) or U that is not
 * real makes the refinement stall, and the point is redone on the C128 path. */
enum { RSRR_PREC_C128 = 0, RSRR_PREC_C64_IR = 1, RSRR_PREC_R32_IR = 2 };

/* One scalar coefficient f(z) = c (z - z0)^p exp(-tau z) / (z - s)^q. */
typedef struct {
    double c_re, c_im;
    int p;
    double z0_re, z0_im;
    double tau;
    double s_re, s_im;
    int q;
} rsrr_term;

/* The NEP T(z).
 * SEPARABLE: n, J, A (device, J matrices n x n, matrix j at A + 2*j*lda*n
 *            doubles), lda >= n, terms (host, J entries).
 * HELMHOLTZ: n, points (device, n x 3 doubles, x y z of point i at
 *            points + 3*i), w (quadrature weight per point).
 * SPARSE:    n, J (1..64), terms (host, J entries), csr (host, J
 *            descriptors; matrix j is csr[j]). */
typedef struct {
    int kind;
    int n;
    int J;
    const double *A;
    int lda;
    const rsrr_term *terms;
    const double *points;
    double w;
    const rsrr_csr *csr;
} rsrr_nep;

/* Per sampling point diagnostics of rsrr_sample. */
typedef struct {
    int info;          /* 0, or i+1 when U(i,i) == 0 exactly (getrf semantics)       */
    int ir_iters;      /* refinement corrections applied (0 for C128)               */
    int fallback;      /* 1 when the point was redone on the C128 path               */
    int pad;
    double resid;      /* max over columns of ||u_c - T(z_k) x_c||_2 / ||u_c||_2, FP64 */
} rsrr_point_info;

/* Diagnostics of rsrr_solve. */
typedef struct {
    int nbar;          /* eigenvalue count from the gap rule (eq. gap)    */
    int warn_gap;      /* 1 when g_max < tol_gap                          */
    double gmax;       /* largest sigma_j / sigma_{j+1} of H              */
    int n_sigma;       /* number of singular values of H computed (leading) */
    int truncated;     /* 1 when nbar > max_eigs and only max_eigs eigenpairs were returned */
} rsrr_solve_info;

typedef struct rsrr_ctx rsrr_ctx;

/* Create a context on HIP device `device` that enqueues on `stream` (a
 * hipStream_t; NULL = the null stream).  Workspace is allocated lazily and
 * owned by the context.  The per-call point buffers of rsrr_sample and
 * rsrr_sample_gmres are sized to half of the free device memory, or to the
 * environment variable RSRR_WS_BUDGET_MB (MiB) when it is set at creation;
 * larger calls run in chunks of points.
 * Errors: -1 ctx NULL, -2 bad device, RSRR_EDEVICE. */
RSRR_API rsrr_status rsrr_create(rsrr_ctx **ctx, int device, void *stream);

/* Versioned options of a context (the knobs the library otherwise fixes).
 * `size` comes first: the library reads only the fields that lie inside the
 * caller's `size` bytes and keeps its defaults for the rest, so a caller built
 * against an older, shorter struct stays valid.  Initialise with
 * rsrr_options_init, change fields, then rsrr_set_options.
 *   ir_max_iters          rsrr_sample (C64_IR, R32_IR): most refinement
 *                         corrections per point (default 10; 0..100; 0 = no
 *                         correction: a point whose first solve is above
 *                         fallback_resid is redone on the C128 path).
 *   ir_max_iters_batched  the same for rsrr_sample_batched and the server's
 *                         sampling launches, whose refinement runs on the
 *                         device (default 3; 0..16).
 *   basis_sketch_max      rsrr_basis: columns of the first range sketch of S
 *                         (default 1024; >= 8); it doubles until it resolves
 *                         the range (see rsrr_basis).
 *   ir_tol                refinement stops when a point's normwise backward
 *                         error max_c ||r_c|| / (||T||_F ||x_c|| + ||u_c||) is at
 *                         most ir_tol * u * sqrt(n), u = 2^-53 (default 4; > 0).
 *   fallback_resid        a refined point whose relative residual
 *                         max_c ||u_c - T x_c||_2 / ||u_c||_2 is above this is
 *                         redone on the C128 path (default 1e-10; (0, 1)).
 *   delta, tol_gap        rank truncation (Sec. 4.3, Step 3) and gap threshold
 *                         (eq. gap) where the library chooses them: server
 *                         requests with delta = 0, and the server's SS-FULL
 *                         (defaults 1e-14 and 1e3).
 * Errors of rsrr_set_options: -1 ctx NULL, -2 opt NULL or size too small to
 * hold `version`, -3 .. -9 the fields in the order above out of range. */
#define RSRR_OPTIONS_VERSION 1
typedef struct {
    unsigned long long size;   /* sizeof(rsrr_options) as the caller compiled it */
    int version;               /* RSRR_OPTIONS_VERSION as the caller compiled it */
    int ir_max_iters;
    int ir_max_iters_batched;
    int basis_sketch_max;
    double ir_tol;
    double fallback_resid;
    double delta;
    double tol_gap;
} rsrr_options;

/* Fill *opt with the defaults, its size and version.  Errors: -1 opt NULL. */
RSRR_API rsrr_status rsrr_options_init(rsrr_options *opt);

/* Apply options to a context (later calls on it use them). */
RSRR_API rsrr_status rsrr_set_options(rsrr_ctx *ctx, const rsrr_options *opt);

/* Read a context's options (opt->size set by the caller, as for rsrr_set_options).
 * Errors: -1 ctx NULL, -2 opt NULL or size too small. */
RSRR_API rsrr_status rsrr_get_options(rsrr_ctx *ctx, rsrr_options *opt);

/* Release the context and its workspace.  Errors: -1 ctx NULL. */
RSRR_API rsrr_status rsrr_destroy(rsrr_ctx *ctx);

/* Ellipse nodes and trapezoid weights (Sec. 5.1, eq. ellip-contour-xw):
 * z_j = gamma + a cos(t_j) + i b sin(t_j), w_j = (-a sin t_j + i b cos t_j)/N,
 * t_j = 2 pi (j + 1/2)/N.  z, w: host, 2N doubles each (w may be NULL).
 * Errors: -3/-4 a, b <= 0; -5 N < 1; -6 z NULL. */
RSRR_API rsrr_status rsrr_contour(double gamma_re, double gamma_im, double a, double b, int N,
                         double *z, double *w);

/* Resolvent sampling (RSRR Step 2, eq. hatS).  For each of the N points z_k
 * (host, 2N doubles): assemble T(z_k), factor it by blocked LU with partial
 * pivoting, and solve for the L probe columns U (device, n x L, ldu >= n).
 * Block k of S (device, n x N*L, lds >= n) receives X_k = T(z_k)^-1 U in
 * columns k*L .. k*L+L-1.  info: host, N entries (may be NULL).
 * prec: RSRR_PREC_C128 or RSRR_PREC_C64_IR.
 * Status: RSRR_ESINGULAR if any point had an exact zero pivot (its block of S
 * is then not meaningful), RSRR_WARN_FALLBACK if any point was redone in FP64.
 * Errors: -2 nep invalid (or not SEPARABLE with R32_IR; or a SPARSE entry out of
 * bounds, found on the device), -3 N < 1, -4 z NULL
 * (or a point off the real axis with R32_IR), -5 U NULL, -6 L < 1, -7 ldu < n,
 * -8 prec, -9 S NULL, -10 lds < n. */
RSRR_API rsrr_status rsrr_sample(rsrr_ctx *ctx, const rsrr_nep *nep, int N, const double *z,
                        const double *U, int L, int ldu, int prec,
                        double *S, int lds, rsrr_point_info *info);

/* Per sampling point diagnostics of rsrr_sample_gmres. */
typedef struct {
    int iters;         /* Arnoldi steps, max over the point's columns              */
    int restarts;      /* restart cycles after the first, max over its columns     */
    int converged;     /* 1 when every column met tol                               */
    int ref;           /* the reference point whose factors preconditioned it      */
    double resid;      /* max over columns of ||u_c - T(z_k) x_c||_2 / ||u_c||_2, FP64 */
    int matrix_free;   /* 1 when the operator generated its entries (HELMHOLTZ)     */
    int pad;
} rsrr_gmres_info;

/* Resolvent sampling with an iterative solver (RSRR Step 2, eq. hatS; Sec. 4.3
 * leaves the solver of T(z_k)^-1 U to the host software and names iterative
 * solvers for large boundary-element and finite-element models, as used in
 * Sec. 6).  Every point k and probe column l is one system T(z_k) x = u_l,
 * solved by restarted flexible GMRES with right preconditioning.  The
 * preconditioner of point k is the complex FP32 LU of T(zref[r]) at one of
 * nref reference points (host, 2*nref doubles): r = ref[k] (host, N ints in
 * [0, nref)), or the nearest reference when ref is NULL; each used reference
 * is factored once.  The operator T(z_k), the Krylov vectors and the
 * residuals are FP64.  For a SPARSE nep the operator walks the sparse rows
 * (no n x n matrix per point; the references are formed densely for their
 * factorisation, which checks every row's bounds first).  For a HELMHOLTZ nep the operator uses the points'
 * assembled FP64 matrices (16 n^2 bytes per point of a chunk), or, with flags
 * RSRR_GMRES_MATRIX_FREE or when they would take more than half of the
 * workspace budget, generates the entries inside every application
 * (matrix-free; flags is otherwise 0).  A column stops when its FP64 relative residual
 * ||u - T(z_k) x||_2 / ||u||_2 is at most tol (0 < tol < 1), measured on the
 * true residual at the end of each restart cycle of at most `restart` steps
 * (1..64), or after max_iters steps.  z, U, S, lds and ldu are as for
 * rsrr_sample (S: device, n x N*L, block k in columns k*L .. k*L+L-1).
 * info: host, N entries (may be NULL).  Phase times (ms) of the last call via
 * rsrr_last_timings: [reference assembly + LU and per-point FP64 operator
 * assembly, operator applications, preconditioner applications, Krylov
 * cycles (all of the iteration), total].
 * Status: RSRR_ENOTCONV if a column missed tol within max_iters (S still holds
 * the last iterate; info says which points), RSRR_ESINGULAR / RSRR_ENAN if a
 * reference matrix had an exact zero / non-finite pivot (nothing solved).
 * Errors: -2 nep invalid (n > 8192; or a SPARSE entry out of bounds), -3 N < 1,
 * -4 z NULL, -5 nref < 1,
 * -6 zref NULL, -7 a ref[k] out of range, -8 U NULL, -9 L < 1, -10 ldu < n,
 * -11 tol, -12 restart, -13 max_iters < 1, -14 flags, -15 S NULL, -16 lds < n. */
enum { RSRR_GMRES_MATRIX_FREE = 1 };
RSRR_API rsrr_status rsrr_sample_gmres(rsrr_ctx *ctx, const rsrr_nep *nep, int N, const double *z,
                                       int nref, const double *zref, const int *ref,
                                       const double *U, int L, int ldu, double tol, int restart,
                                       int max_iters, int flags, double *S, int lds,
                                       rsrr_gmres_info *info);

/* Basis (RSRR Step 3, Sec. 4.2-4.3).  S (device, n x NL, lds) is normalised
 * in place to unit column norms; then the number k of singular values above
 * delta*sigma_1 and the first min(k, kmax) left singular vectors (Q: device,
 * n x kmax, ldq >= n) are computed in FP64.  *k (host) receives k even when
 * k > kmax.  The range of S is found by a seeded Gaussian sketch S Omega of
 * basis_sketch_max columns (rsrr_options, default 1024; S itself when NL is
 * no wider), orthonormalised by block CGS2 with numerically dependent columns
 * dropped; the sketch width doubles (up to min(n, NL)) until the sketch comes
 * out rank deficient or its smallest singular value is at the rounding floor
 * (<= 1e-15 sigma_1).  The SVD of S restricted to that range (one-sided
 * Jacobi) gives r <= min(n, NL) singular values.  sigma (host, min(n, NL)
 * doubles, may be NULL) receives those r values, descending, followed by
 * zeros for the values the sketch did not resolve.  Those lie at the rounding
 * level of S: below 1e-15 sigma_1 when the sketch stopped at that floor, or
 * below the block CGS2 dropping level (4 u sqrt(n) of a sketch column's norm,
 * u = 2^-53) when it came out rank deficient; a count k near delta*sigma_1
 * can therefore differ from a full SVD's by the values within that level.
 * Errors: -2 n < 1, -3 NL < 1, -4 S NULL, -5 lds < n, -6 delta not in (0,1),
 * -7 Q NULL, -8 ldq < n, -9 kmax < 1, -10 k NULL.  RSRR_ENOTCONV if the
 * one-sided Jacobi SVD did not converge. */
RSRR_API rsrr_status rsrr_basis(rsrr_ctx *ctx, int n, int NL, double *S, int lds, double delta,
                       double *Q, int ldq, int kmax, int *k, double *sigma);

/* Projection (RSRR Step 4, eq. Ts-NEP): T_Q(z) = Q^H T(z) Q with Q (device,
 * n x k, ldq).  SEPARABLE: AQ_j = Q^H A_j Q for each j and the same terms
 * (SPARSE: the same, with A_j Q formed from the sparse rows).
 * HELMHOLTZ: T(z) is expanded about gamma (host, 2 doubles) in powers of
 * (z - gamma), with the degree chosen so that the remainder is below 1e-17
 * relative for |z - gamma| <= radius; AQ_p = Q^H T_p Q, term p = (z-gamma)^p.
 * AQ: device, max_terms matrices k x k (matrix j at AQ + 2*j*k*k doubles).
 * J_eff (host) receives the number of matrices written; terms_out (host,
 * max_terms entries) their coefficients.
 * Errors: -2 nep, -3 Q NULL, -4 ldq < n, -5 k < 1, -6 gamma NULL,
 * -7 radius <= 0, -8 AQ NULL, -9 max_terms too small, -10 J_eff NULL,
 * -11 terms_out NULL. */
RSRR_API rsrr_status rsrr_project(rsrr_ctx *ctx, const rsrr_nep *nep, const double *Q, int ldq, int k,
                         const double *gamma, double radius, double *AQ, int max_terms,
                         int *J_eff, rsrr_term *terms_out);

/* Projected NEP solve (RSRR Steps 4-5 via SS-FULL, Sec. 3.3).  T_Q(z) =
 * sum_j f_j(z) AQ_j (device AQ, J_eff matrices k x k; host terms).  SS-FULL
 * on the ellipse (gamma, a, b) with NQ trapezoid nodes and KQ moment blocks:
 * moments of T_Q^-1 in zeta = (z - gamma)/max(a, b), block Hankel H and H^<
 * (eq. HH), SVD of H, count nbar by the largest gap (eq. gap), reduced matrix
 * A = V0^H H^< W0 Sigma0^-1 of order nbar (eq. A, every retained singular
 * triplet), its nbar eigenpairs, lift g = M W0 Sigma0^-1 b and v = Q g.
 * Of the nbar eigenpairs, the min(nbar, max_eigs) of lowest elliptic level
 * |Re(lambda-gamma)/a|^2 + |Im(lambda-gamma)/b|^2 are returned, in increasing
 * level; max_eigs never changes the arithmetic, only how many are copied out.
 * Outputs: count (host) eigenvalues lambda (host, 2*max_eigs doubles),
 * eigenvectors V (device, n x max_eigs, ldv >= n, unit 2-norm; may be NULL),
 * residuals resid (host, max_eigs; ||T(lambda)v||_2 / (||T(lambda)||_1 ||v||_2)
 * in FP64 against the full nep; may be NULL only if V is NULL).  sigma_H
 * (host, KQ*k doubles, may be NULL) receives the singular values of H,
 * descending: all KQ*k of them, or, when H is numerically of low rank and a
 * range sketch of it shows a clear gap (g_max >= 10 tol_gap), the
 * sinfo->n_sigma leading ones followed by zeros.  sinfo (host, may be NULL):
 * nbar, g_max, the gap warning and whether the output was truncated.
 * Status RSRR_WARN_GAP when g_max < tol_gap (results are best effort; takes
 * precedence over RSRR_WARN_MORE), RSRR_WARN_MORE when nbar > max_eigs,
 * RSRR_ELIMIT when nbar > 1024 (the reduced eigenproblem's size limit;
 * nothing is returned, sinfo->nbar tells the count).
 * Errors: -2 nep, -3 k < 1, -4 AQ NULL, -5 J_eff < 1, -6 terms NULL,
 * -7 Q NULL, -8 ldq, -9 gamma NULL, -10 a, -11 b, -12 NQ < 2*KQ+1,
 * -13 KQ < 1, -14 tol_gap, -15 max_eigs < 1, -16 lambda NULL, -17 ldv,
 * -18 count NULL. */
RSRR_API rsrr_status rsrr_solve(rsrr_ctx *ctx, const rsrr_nep *nep, int k, const double *AQ, int J_eff,
                       const rsrr_term *terms, const double *Q, int ldq,
                       const double *gamma, double a, double b, int NQ, int KQ, double tol_gap,
                       int max_eigs, double *lambda, double *V, int ldv, double *resid,
                       int *count, double *sigma_H, rsrr_solve_info *sinfo);

/* Phase timings (milliseconds, device events) of the last rsrr_sample call:
 * t[0] assembly, t[1] LU factorisation, t[2] solves (getrs, all iterations),
 * t[3] FP64 residuals, t[4] total.  t: host, 5 doubles.  Errors: -2 t NULL. */
RSRR_API rsrr_status rsrr_last_timings(rsrr_ctx *ctx, double *t);

/* One NEP instance of a ragged batch: T(z) (nep), N sampling points z (host,
 * 2N doubles), probes U (device, n x L, ldu >= n) and the output S (device,
 * n x N*L, lds >= n; block k = T(z_k)^-1 U). */
typedef struct {
    rsrr_nep nep;
    int N;
    const double *z;
    const double *U;
    int L;
    int ldu;
    double *S;
    int lds;
} rsrr_instance;

/* Flags of rsrr_sample_batched. */
enum {
    RSRR_BATCH_GRAPH = 1,     /* capture the whole call in one hipGraph (every size bucket an
                                 independent branch, spread over the bucket streams) and replay it
                                 with one launch when the same batch (same buffers, sizes and
                                 points) is submitted again                                        */
    RSRR_BATCH_AUTOTUNE = 2   /* time panel widths x update tiles on the first call for each size bucket */
};

/* Resolvent sampling for a ragged batch of instances (RSRR Step 2, eq. hatS,
 * for many NEPs at once).  Instances are grouped by n rounded up to 64; each
 * group runs as one batch of padded matrices diag(T(z_k), I) (the padded
 * solve returns T(z_k)^-1 U exactly).  With C64_IR the refinement runs on the
 * device with at most ir_max_iters_batched corrections (rsrr_options,
 * default 3); points above fallback_resid (default 1e-10) relative residual
 * are redone on the FP64 path.  info: host, sum of N entries in instance
 * order (may be NULL).  The library keeps per-bucket buffers (and the last
 * call's graph) in the context until rsrr_destroy.  With RSRR_BATCH_AUTOTUNE, the first call
 * for a size bucket times one bucket pass for every candidate configuration
 * (LU panel width 32/64/128 x workgroup tile of the complex FP32 trailing
 * update: 3M 128x64, 3M 64x64, 4M 128x128, 4M 64x64, all four waves and two
 * LDS stages; FP64: panel width 32/64) and keeps the fastest per (bucket,
 * precision, device architecture); when the environment variable
 * RSRR_TUNE_FILE names a file the choices are read from and written to it as
 * JSON ({"arch": ..., "entries": [{"P", "prec", "nb", "update_tile",
 * "update_tile_name", "ms"}, ...]}).
 * Status as rsrr_sample.  Errors: -2 count < 1, -3 an instance is invalid,
 * -4 prec. */
RSRR_API rsrr_status rsrr_sample_batched(rsrr_ctx *ctx, int count, const rsrr_instance *inst, int prec, int flags,
                                         rsrr_point_info *info);

/* Moment matrix of the resolvent moment scheme (Sec. 4.1, eq. Malpha,
 * eq. M-pr) from the sampling matrix: M = S Z (eq. MS), i.e.
 * M_alpha = sum_i omega_i zeta_i^alpha X_i for alpha = 0 .. K-1, where X_i is
 * block i of S (columns i L .. i L + L - 1), zeta_i = (z_i - gamma)/rho and
 * omega_i = 1 / prod_{j != i} ((zeta_i - zeta_j)/C) are the barycentric
 * weights (eq. bary-wt) with every factor divided by the capacity C
 * (Sec. 3.3, item 3; for an ellipse of semi-axes a, b and rho = max(a, b):
 * C = (a + b) / (2 rho)).  Block alpha of M is columns alpha L .. alpha L + L - 1.
 * S: device, n x N L, lds; z: host, 2N doubles (the points of S's blocks);
 * gamma: host, 2 doubles; M: device, n x K L, ldm (caller-owned).  The moment
 * variant of SS-RR runs rsrr_basis, rsrr_project and rsrr_solve on M.
 * Errors: -2 n, -3 N, -4 L, -5 S, -6 lds, -7 z NULL or two equal points,
 * -8 gamma, -9 rho, -10 capacity, -11 K not in [1, N], -12 M, -13 ldm. */
RSRR_API rsrr_status rsrr_moments(rsrr_ctx *ctx, int n, int N, int L, const double *S, int lds, const double *z,
                                  const double *gamma, double rho, double capacity, int K, double *M, int ldm);

/* rsrr_moments without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * rsrr_moments; the points and the N x K coefficient table live in a static
 * per-GPU scratch array of 65536 complex entries (1 MiB, held by each GPU the
 * library runs on until the process ends) instead of context workspace.
 * Limit: N + N*K <= 65536, else RSRR_ELIMIT with nothing enqueued.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * contexts or streams at once) race; a call has finished with it when it
 * returns (the call synchronises its stream). */
RSRR_API rsrr_status rsrr_moments_noalloc(rsrr_ctx *ctx, int n, int N, int L, const double *S, int lds,
                                          const double *z, const double *gamma, double rho, double capacity,
                                          int K, double *M, int ldm);

/* Diagnostics of rsrr_two_stage. */
typedef struct {
    int k1, count1, nbar1;   /* stage 1: rank of S, eigenvalues returned, SS-FULL count   */
    int n_new;               /* distinct stage-1 estimates inside C, sampled in stage 2   */
    int k2, nbar2;           /* stage 2: rank of S, SS-FULL count                         */
    double resid1_max;       /* largest stage-1 eigen-residual inside C                   */
} rsrr_two_stage_info;

/* Two-stage sampling (Sec. 5.4, Example 2; Sec. 6, Example 3).  Stage 1: RSRR (Steps
 * 2-5) with N1 points on the ellipse (gamma, a, b).  The distinct stage-1
 * eigenvalue estimates inside the ellipse (elliptic level < 1; estimates within
 * 1e-6 max(1, |lambda|) of an earlier one are dropped; at most max_new) become
 * extra sampling points: their blocks T(z)^-1 U are appended to S after the N1
 * stage-1 blocks, which are reused, and Steps 3-5 run again on all
 * (N1 + n_new) L columns.
 * S: device, n x (N1 + max_new) L, lds >= n (caller-owned; normalised in place).
 * z_new: host, 2 max_new doubles (the points added).  The outputs lambda,
 * V (device, required: the residuals need it), resid and count are those of
 * rsrr_solve for stage 2; tinfo (host, may be NULL) gets both stages' figures.
 * Errors: -2 nep, -3 gamma NULL, -4 a, -5 b, -6 N1, -7 U, -8 L, -9 ldu,
 * -10 prec, -11 S, -12 lds, -13 max_new < 0, -14 delta, -15 NQ/KQ,
 * -17 tol_gap, -18 max_eigs, -19 lambda, -20 V, -21 ldv, -22 resid,
 * -23 count, -24 z_new NULL with max_new > 0. */
RSRR_API rsrr_status rsrr_two_stage(rsrr_ctx *ctx, const rsrr_nep *nep, const double *gamma, double a, double b,
                                    int N1, const double *U, int L, int ldu, int prec, double *S, int lds,
                                    int max_new, double delta, int NQ, int KQ, double tol_gap, int max_eigs,
                                    double *lambda, double *V, int ldv, double *resid, int *count, double *z_new,
                                    rsrr_two_stage_info *tinfo);

/* ---------------------------------------------------------------------------
 * Serving: a request loop for many NEP solves on one device.
 *
 * Each request is the whole method of Sec. 4.3 for one NEP: contour nodes
 * (eq. ellip-contour-xw), resolvent sampling (Step 2), basis (Step 3),
 * projection and SS-FULL (Steps 4-5).
 *
 * Admission by footprint.  A request is admitted when a slot is free and its
 * whole per-request device footprint fits in the server's HBM arena (first
 * come, first served): S (16 n N (L + L_extra) bytes), its LU factors kept on
 * the device (complex FP32 or FP64 factors of every point, P x P with P = n
 * rounded up to 64, plus interchanges and diagonal-block inverses), the basis
 * Q (16 n min(n, N (L + L_extra)) bytes) and the eigenvectors V (16 n max_eigs
 * bytes); rsrr_server_footprint gives the figure.  What is not per request is
 * fixed at creation: the sampling launches' buffers (batch_bytes, trimmed back
 * after a launch that needed more) and each solve thread's budget solve_bytes
 * (projected matrices, the chunked phases of Steps 3-5 and the solves of a
 * re-probe), so device use is bounded by arena_bytes + batch_bytes +
 * solvers * solve_bytes plus the caller's own inputs.
 *
 * Continuous batching.  The sampling points of every admitted request are
 * batched together: each sampling launch takes points from all admitted
 * requests in admission order, up to batch_bytes of LU workspace, grouped by
 * (n rounded up to 64, L), so points that arrive while others are on the GPU
 * join the next launch.  Solve threads, each with its own stream, run basis,
 * projection and SS-FULL of requests whose sampling has finished, overlapping
 * each other and the next sampling launches on the device.
 *
 * Kept factors and re-probes.  A request's factors stay in its arena block
 * from factorisation until it finishes.  When SS-FULL's gap test fails
 * (g_max < tol_gap, eq. gap) or an eigenpair inside the contour has residual
 * above 1e-10, the paper's remedy is more probe columns (Sec. 3.3): the
 * request's L_extra reserve columns of U are then solved with the kept
 * factors (triangular solves and refinement only, no refactorisation),
 * appended to S, and Steps 3-5 run again on all N (L + L_extra) columns.
 *
 * Per-point work (tile shapes, panel width, refinement) depends only on
 * (n, L, precision), never on what else is in the launch, so a request's
 * results do not depend on the mix it ran in.
 * ------------------------------------------------------------------------- */
typedef struct rsrr_server rsrr_server;

typedef struct {
    int device;
    int prec;                 /* RSRR_PREC_C128 or RSRR_PREC_C64_IR                        */
    int max_slots;            /* requests admitted at the same time (>= 1)                 */
    int flags;                /* RSRR_SERVE_*                                               */
    int solvers;              /* solve threads, each with its own stream (0: 2; at most 8)  */
    int pad;
    unsigned long long arena_bytes;  /* HBM for the admitted requests' footprints           */
    unsigned long long batch_bytes;  /* HBM cap of one sampling launch's LU workspace       */
    unsigned long long solve_bytes;  /* HBM budget of each solve thread (0: 4 GiB)          */
    const rsrr_options *options;     /* options of every context of the server (NULL: defaults);
                                        read at creation                                     */
} rsrr_server_config;

enum {
    RSRR_SERVE_NO_BATCH = 1,  /* one request's points per sampling launch (no mixing)      */
    RSRR_SERVE_SERIAL = 2     /* no solve threads: basis/projection/solve run between the
                                 sampling launches, on the sampling stream                */
};

/* One request.  nep device data, U (device, n x (L + L_extra), ldu >= n) and
 * the host output arrays stay owned by the caller and must stay valid until
 * rsrr_server_wait has returned this request.  Outputs: lambda (host,
 * 2*max_eigs doubles), resid (host, max_eigs; ||T(lambda)v|| / (||T(lambda)||_1
 * ||v||)), V (host, n x max_eigs column-major with ld n, unit 2-norm columns;
 * may be NULL).  The first L columns of U are the probes; the L_extra after
 * them are solved only on a re-probe. */
typedef struct {
    rsrr_nep nep;
    double gamma_re, gamma_im;   /* ellipse centre */
    double a, b;                 /* ellipse semi-axes (real, imaginary) */
    int N;                       /* sampling points */
    int L;                       /* probe columns */
    const double *U;
    int ldu;
    int NQ;                      /* SS-FULL quadrature nodes (0: 500)  */
    int KQ;                      /* SS-FULL moment blocks (0: 2)       */
    double delta;                /* rank truncation (0: the options' delta, 1e-14) */
    int max_eigs;
    double *lambda;
    double *resid;
    double *V;
    int L_extra;                 /* reserve probe columns for a re-probe (>= 0) */
    int pad;
} rsrr_request;

/* Result of one request; times are seconds on the server's steady clock
 * (0 = server creation). */
typedef struct {
    int id;
    rsrr_status status;          /* RSRR_OK or the first failing step's status           */
    int count;                   /* eigenpairs written (eigenvalues inside or near C)    */
    int k;                       /* rank of S kept by the basis                          */
    int nbar;                    /* SS-FULL eigenvalue count                             */
    int fallbacks;               /* sampling points redone on the FP64 path              */
    int ir_iters_max;
    int launches;                /* sampling launches that carried this request's points */
    double sample_resid_max;     /* max relative residual of the refined solves          */
    double t_submit, t_admit, t_sampled, t_done;
    int reprobes;                /* re-probes (0 or 1) solved from the kept factors      */
    int L_used;                  /* probe columns in the final S (L or L + L_extra)      */
    unsigned long long footprint;  /* bytes of the request's arena block                  */
} rsrr_result;

/* Per-request device footprint (bytes) that admission charges against the
 * arena for request req on a server configured by cfg (host computation).
 * Errors: -1 cfg NULL, -2 req NULL or invalid, -3 bytes NULL. */
RSRR_API rsrr_status rsrr_server_footprint(const rsrr_server_config *cfg, const rsrr_request *req,
                                           unsigned long long *bytes);

/* Create a server (a sampling thread and cfg->solvers solve threads, each on
 * its own non-blocking stream on cfg->device) and allocate its arena.  Errors:
 * -1 srv NULL, -2 cfg invalid (or its options refused by rsrr_set_options),
 * RSRR_ENOMEM, RSRR_EDEVICE. */
RSRR_API rsrr_status rsrr_server_create(rsrr_server **srv, const rsrr_server_config *cfg);

/* Queue a request (thread safe, does not block on the GPU).  *id receives its
 * id.  Errors: -1 srv, -2 request invalid, -3 id NULL; RSRR_ENOMEM when its
 * footprint alone exceeds the arena. */
RSRR_API rsrr_status rsrr_server_submit(rsrr_server *srv, const rsrr_request *req, int *id);

/* Wait until request id has finished (timeout_s < 0: no limit) and fill out.
 * Each id can be waited for once.  Errors: -1 srv, -2 unknown id, -4 out NULL;
 * RSRR_ETIMEOUT. */
RSRR_API rsrr_status rsrr_server_wait(rsrr_server *srv, int id, double timeout_s, rsrr_result *out);

/* Server counters (host, 12 doubles): requests finished, points factored,
 * sampling launches, arena bytes in use at peak, largest launch (points),
 * seconds the sampling thread was busy, seconds the solve threads were busy,
 * peak device memory in use (bytes, from hipMemGetInfo), current server time,
 * requests waiting for admission, points solved again from kept factors
 * (re-probes), re-probes.  Errors: -1 srv, -2 out NULL. */
RSRR_API rsrr_status rsrr_server_stats(rsrr_server *srv, double *out);

/* Finish every submitted request, stop the threads and free the server.
 * Errors: -1 srv NULL. */
RSRR_API rsrr_status rsrr_server_destroy(rsrr_server *srv);

/* Device-event statistics of the LU trailing-update kernel (A22 -= L21 U12,
 * the matrix-core hot loop of rsrr_sample).  enable = 1 starts recording a
 * pair of events around every trailing-update launch of later rsrr_sample
 * calls, 0 stops; reset = 1 clears the totals.  out (host, 8 doubles, may be
 * NULL): launches timed, summed kernel time in ms, algorithmic flops of the
 * timed launches (8 m n k per complex m x n x k update and matrix), launches
 * not timed (event pool exhausted), algorithmic bytes of the timed launches
 * (the m x n block read and written once, the m x k and k x n operands read
 * once), then of those launches the ones that ran on the look-ahead's
 * CU-masked stream: their summed time (ms) and flops, and the fraction of
 * the device's CUs that stream may use.  Errors: -1 ctx NULL. */
RSRR_API rsrr_status rsrr_update_stats(rsrr_ctx *ctx, int enable, int reset, double *out);

/* Library version string (static storage). */
RSRR_API const char *rsrr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RSRR_H */

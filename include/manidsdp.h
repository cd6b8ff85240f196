/*
 * manidsdp.h -- C ABI of the MI355X (gfx950) ManiDSDP subproblem library.
 *
 * The library evaluates, on one GPU, the quantities inside each ALM
 * subproblem of ManiDSDP (Wang, Hu, Xia, arXiv 2512.04406) for SDPs of the
 * form DSDP (introduction):
 *
 *     inf_y  b^T y   s.t.  S = A*(y) - C  PSD,  diag(S) = 1,
 *
 * whose constraint matrices A_gamma are 0/1 indicators of pairwise disjoint
 * sets of matrix entries ("classes"), as in moment relaxations, so that AA* is
 * diagonal (remarks after Algorithm alg1).  With S = Y Y^T, Y in R^{n x p} with
 * unit rows (oblique manifold, eq. maniY), Z = S + C, and the projectors
 * P = A*(AA*)^{-1}A, Q = I - P (eq. projection-operators):
 *
 *   cost    Psi(Y)   = <D + Xt, Z> + sigma/2 ||Q(Z)||_F^2  (eq. reduced-ALM-subproblem)
 *   G                = Xt + D + sigma Q(Z)                  (Lemma lm:suboptimality)
 *   egrad            = 2 G Y
 *   z                = diag(G S) = rowdot(G Y, Y)
 *   rgrad            = egrad - Diag(rowdot(egrad, Y)) Y = 2 X Y  (Prop. prop, eq. sec4:eq6)
 *   ehess[U]         = 2 G U + 2 sigma Q(Y U^T + U Y^T) Y   (Prop. prop)
 *   rhess[U]         = ehess[U] - Diag(rowdot(ehess[U], Y)) Y - 2 Diag(z) U  (eq. sec4:eq7)
 *
 * where D = A*(AA*)^{-1} b and Xt is the ALM multiplier (dense symmetric).
 *
 * Conventions for every entry point:
 *  - Return value: MDSDP_OK or a negative mdsdp_status; mdsdp_last_error()
 *    gives a message (thread-local).  Nothing is thrown across the ABI.
 *  - "dev" pointers are device (HBM) pointers owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller.  The library never
 *    frees caller memory.  Host inputs are copied before the call returns.
 *  - Matrices Y, U, V, outputs: FP64, row-major n x p, contiguous (ld = p).
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL = the
 *    default stream) and is asynchronous unless stated; device scalar outputs
 *    become valid when the stream reaches them.
 *  - Argument errors are detected synchronously (MDSDP_EINVAL) before any work
 *    is enqueued.  A problem handle must not be used from two streams at once.
 *  - p may be 1..512 for every call that takes a factor width (staged in
 *    widths 16, 32, 64 or a multiple of 64; the product kernels work on
 *    slices of at most 64 columns, MFMA tiles are 16 wide).  p > 512 returns
 *    MDSDP_EUNSUPPORTED.
 */
#ifndef MANIDSDP_H
#define MANIDSDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdsdp_problem_s* mdsdp_problem;

typedef enum {
  MDSDP_OK = 0,
  MDSDP_EINVAL = -1,      /* bad argument (sizes, ids, NULL where required) */
  MDSDP_ENOMEM = -2,      /* device allocation failed */
  MDSDP_EHIP = -3,        /* a HIP runtime call failed */
  MDSDP_ENOTORTH = -4,    /* sparse A supports overlap: AA* not diagonal */
  MDSDP_ENONFINITE = -5,  /* NaN/Inf met in an input or a reduction */
  MDSDP_EUNSUPPORTED = -6,/* e.g. no gfx950 device */
  MDSDP_ENOCONV = -7      /* iteration limit reached before the tolerance */
} mdsdp_status;

/* Tile precision of the HVP pass.  Class sums are accumulated in FP64
 * (structured BQP path) or in 64-bit fixed point (generic class maps); cost,
 * gradient, multiplier update and KKT are always FP64. */
typedef enum { MDSDP_FP64 = 0, MDSDP_FP32 = 1 } mdsdp_prec;

/* Basis order for the BQP builder: paper order (lexicographic products) or the
 * colex order (products by larger index) that groups each class's entries. */
typedef enum { MDSDP_ORDER_LEX = 0, MDSDP_ORDER_COLEX = 1 } mdsdp_order;

const char* mdsdp_last_error(void);
const char* mdsdp_version(void);

/* ---- BQP relaxation builder (host only, no device work) -------------------
 * Order-2 moment relaxation of min x^T Q x + c^T x over x in {-1,1}^q
 * (paragraph "Binary quadratic programs", basis v(x) and eq.
 * bqp-number-moments): n = 1 + q + q(q-1)/2, m = sum_{d<=4} C(q,d).  The class
 * of entry (alpha, beta) is the symmetric difference of the index sets; class
 * ids are ordered by degree, then by colex rank of the sorted index set
 * (id = off[d] + sum_i C(c_i, i), 0-based c_1 < ... < c_d).
 * mdsdp_bqp_sizes: writes n and m.
 * mdsdp_bqp_classmap: writes n(n+1)/2 int32 ids of the packed upper triangle,
 *   row-major (row a holds columns a..n-1), into host buffer cls_out.
 * mdsdp_bqp_b: writes b (length m, host): b_{} = tr Q, b_{i} = c_i,
 *   b_{ij} = Q_ij + Q_ji, 0 for degree 3 and 4.  Q: q*q row-major host. */
mdsdp_status mdsdp_bqp_sizes(int32_t q, int32_t* n_out, int64_t* m_out);
mdsdp_status mdsdp_bqp_classmap(int32_t q, int32_t order, int32_t* cls_out);
mdsdp_status mdsdp_bqp_b(int32_t q, const double* Q_host, const double* c_host, double* b_out);

/* ---- Hermitian UCQP relaxation builder (host only, no device work) ----------
 * Order-2 Hermitian moment relaxation of min z^H Q z over |z_i| = 1, z in C^q
 * (paragraph on unit-modulus complex quadratic programs; this keeps the
 * complex moments), in the real embedding S = [[Re M, -Im M], [Im M, Re M]] of
 * the moment matrix M: basis 1, z_i, z_i z_j (i <= j) lexicographically,
 * n_c = 1 + q + q(q+1)/2, n = 2 n_c.  Entries of M are classed by the exponent
 * difference d = alpha - beta up to sign (representative gamma with its first
 * nonzero component positive, d = s gamma): class re(gamma) holds (a, c) and
 * (n_c + a, n_c + c) with coefficient +1; class im(gamma), gamma != 0, holds
 * (n_c + a, c) with coefficient s and (a, n_c + c) with -s; the imaginary
 * parts of the diagonal class are in no class (coefficient 0).  Class ids:
 * representatives in ascending order as integer vectors, re(gamma) = rank,
 * im(gamma) = m_re + rank - 1, m = 2 m_re - 1.  b: tr Q on class 0,
 * 2 Re Q_ij on re(e_i - e_j), 2 Im Q_ij on im(e_i - e_j) (i < j).
 * mdsdp_ucqp_sizes: n and m.  mdsdp_ucqp_structure: packed upper triangle
 * (row-major, n(n+1)/2 entries) of class ids and coefficients (+1, -1, 0).
 * mdsdp_ucqp_b: b (length m) from Q = Qre + i Qim (q x q row-major).
 * 1 <= q <= 60. */
mdsdp_status mdsdp_ucqp_sizes(int32_t q, int32_t* n_out, int64_t* m_out);
mdsdp_status mdsdp_ucqp_structure(int32_t q, int32_t* cls_out, int8_t* coef_out);
mdsdp_status mdsdp_ucqp_b(int32_t q, const double* Qre_host, const double* Qim_host, double* b_out);

/* ---- problem lifetime ------------------------------------------------------
 * mdsdp_create_classmap: cls_host = packed upper-triangle class ids (row-major,
 * length n(n+1)/2, ids in [0, m), every class non-empty); b_host
 * length m; C_host = dense symmetric n x n row-major or NULL for C = 0.
 * Computes |gamma| (= AA*), D = b/|gamma|, A(C), builds the tile-major device
 * layout and allocates all workspaces.  Xt starts at 0, sigma at 1.
 * Errors: EINVAL for n < 1, m < 1, ids out of range or empty classes;
 * ENOMEM; EUNSUPPORTED if the current device is not gfx950. */
mdsdp_status mdsdp_create_classmap(int32_t n, int64_t m, const int32_t* cls_host,
                                   const double* b_host, const double* C_host,
                                   mdsdp_problem* out);
/* BQP relaxation built in-library from Q (q x q row-major host) and c (q,
 * host), in the given basis order.  With MDSDP_ORDER_COLEX the class sums use
 * structured kernels that read no class map and use no atomics (the class
 * structure of the order-2 BQP relaxation is arithmetic); results agree with
 * the generic class-map path to rounding.  Errors as mdsdp_create_classmap. */
mdsdp_status mdsdp_create_bqp(int32_t q, int32_t order, const double* Q_host, const double* c_host,
                              mdsdp_problem* out);
/* Hermitian UCQP relaxation built in-library from Q = Qre + i Qim (q x q
 * row-major host, Hermitian; EINVAL otherwise, ENONFINITE for NaN/Inf), with
 * the class structure of mdsdp_ucqp_structure (signed coefficients; the
 * generic class-map kernels). */
mdsdp_status mdsdp_create_ucqp(int32_t q, const double* Qre_host, const double* Qim_host,
                               mdsdp_problem* out);
/* Sparse A given as a list of (class, row, col, value) with row <= col: the
 * entry (row, col) and its mirror have coefficient `value` in A_class.  Values
 * must be +1 or -1 (signed unit coefficients, as in the real embedding of a
 * Hermitian moment matrix, whose imaginary parts appear with opposite signs in
 * the two off-diagonal blocks); supports must be pairwise disjoint, so that
 * AA* = Diag(sum of squared coefficients per class) (remarks after Algorithm
 * alg1).  An entry no triplet covers belongs to no class: A*(y) is zero there,
 * so the constraint S = A*(y) - C fixes S_e = -C_e.  Overlaps: ENOTORTH; other
 * values: EUNSUPPORTED; non-finite values: ENONFINITE; a class with no entry:
 * EINVAL.  All checked on the host before any device work. */
mdsdp_status mdsdp_create_sparse_A(int32_t n, int64_t m, int64_t nnz, const int32_t* cls_host,
                                   const int32_t* row_host, const int32_t* col_host,
                                   const double* val_host, const double* b_host,
                                   const double* C_host, mdsdp_problem* out);
mdsdp_status mdsdp_destroy(mdsdp_problem prob);
mdsdp_status mdsdp_problem_info(mdsdp_problem prob, int32_t* n, int64_t* m, int64_t* n_slots,
                                int32_t* n_tiles);

/* ---- multiplier and penalty ------------------------------------------------
 * set: Xt_dev = dense symmetric n x n row-major FP64 device matrix, or NULL for
 * Xt = 0; it clears the non-finite flag (mdsdp_sync_status).  Writing the subproblem residual as Q(S + C) - lambda/sigma, the
 * multiplier lambda is -Xt.  get: writes the same layout. */
mdsdp_status mdsdp_set_multiplier(mdsdp_problem prob, const double* Xt_dev, double sigma,
                                  void* stream);
mdsdp_status mdsdp_get_multiplier(mdsdp_problem prob, double* Xt_dev, void* stream);
mdsdp_status mdsdp_set_sigma(mdsdp_problem prob, double sigma);

/* ---- direct-DSDP subproblem (ablation) --------------------------------------
 * on = 1 switches the problem to the S-subproblem of the two-block ADMM applied
 * directly to DSDP (section "Why solve DSDP' instead of DSDP",
 * eq. direct-ALM-subproblem): cost <D + Xt, Z> + sigma/2 ||Z - P(Z^k)||^2 with
 * the stale class averages y^k, gradient 2 (Xt + D + sigma (Z - P(Z^k))) Y and
 * Hessian sigma I in S (eq. hessian-comparison).  With Y_dev (n x p, FP64) y^k
 * is set to the class averages of Y Y^T + C; otherwise the last computed ones
 * are kept.  mdsdp_update_multiplier refreshes y^k (the ADMM y-update).  on = 0
 * returns to the variable-projected subproblem of DSDP'. */
mdsdp_status mdsdp_set_direct(mdsdp_problem prob, int32_t on, int32_t p, const double* Y_dev, void* stream);

/* ---- device status (non-finite guard) --------------------------------------
 * Kernels raise a sticky flag in device memory when they meet a non-finite
 * value: the multiplier given to mdsdp_set_multiplier, the cost, an HVP
 * output, or ||Q(Z)|| / sum z in the multiplier update.  mdsdp_set_multiplier
 * clears it (a new multiplier starts a new state).  sync_status synchronises
 * `stream` and returns MDSDP_ENONFINITE if the flag is raised, else MDSDP_OK.
 * Host inputs (b, C, Q, c) are checked when a problem is created:
 * MDSDP_ENONFINITE before any device work. */
mdsdp_status mdsdp_sync_status(mdsdp_problem prob, void* stream);

/* ---- subproblem evaluation -------------------------------------------------
 * cost_grad at Y (dev, n x p): f_dev (1 double, nullable), egrad_dev and
 * rgrad_dev (n x p, nullable).  Caches y(S) (class averages), z = diag(G S)
 * and the class coefficients used by the following mdsdp_hvp calls at the
 * same Y.  Section: eq. reduced-ALM-subproblem, Lemma lm:suboptimality,
 * Proposition prop. */
mdsdp_status mdsdp_cost_grad(mdsdp_problem prob, int32_t p, const double* Y_dev, double* f_dev,
                             double* egrad_dev, double* rgrad_dev, void* stream);
/* HVP at the Y of the last mdsdp_cost_grad call (same Y_dev contents; the
 * class averages, diag(G S) and Y^T Y of that point are reused).
 * riemannian = 0: ehess[U]; 1: rhess[U] (U should be tangent).  prec selects
 * the tile precision.  Proposition prop, eq. sec4:eq7. */
mdsdp_status mdsdp_hvp(mdsdp_problem prob, int32_t p, int32_t prec, const double* Y_dev,
                       const double* U_dev, double* HU_dev, int32_t riemannian, void* stream);
/* Class averages y(S) of Z = Y Y^T + C (variable projection, section 3):
 * y_dev length m. */
mdsdp_status mdsdp_class_average(mdsdp_problem prob, int32_t p, const double* Y_dev,
                                 double* y_dev, void* stream);
/* Retraction R_Y(t V) = rows of (Y + t V) normalised; Yout may alias Y. */
mdsdp_status mdsdp_retract(int32_t n, int32_t p, const double* Y_dev, const double* V_dev,
                           double t, double* Yout_dev, void* stream);
/* Tangent projection P_Y(U) = U - Diag(U Y^T) Y (Lemma sec4:lm1); out may alias U. */
mdsdp_status mdsdp_project_tangent(int32_t n, int32_t p, const double* Y_dev,
                                   const double* U_dev, double* out_dev, void* stream);

/* ---- outer-loop steps (Algorithm alg1, steps 5-8) --------------------------
 * update_multiplier: y = class averages of Z, Xt <- Xt + sigma Q(Z),
 * z = diag((Xt + D) S).  Outputs (dev, nullable): y (m), z (n),
 * kkt[4] = { ||Q(Z)||_F, b^T y, sum z, <C, X + Diag z> }.  FP64. */
mdsdp_status mdsdp_update_multiplier(mdsdp_problem prob, int32_t p, const double* Y_dev,
                                     double* y_dev, double* z_dev, double* kkt_dev, void* stream);
/* X v = (Xt + D) v - z o v for k vectors (columns of V, n x k row-major,
 * k <= 512), with z from the last update_multiplier.  FP64. */
mdsdp_status mdsdp_certificate_matvec(mdsdp_problem prob, int32_t k, const double* V_dev,
                                      double* XV_dev, void* stream);
/* The k smallest eigenpairs and the largest eigenvalue of the certificate
 * X = Xt + D - Diag(z) (eq. res; step 9 of Algorithm alg1, where the
 * eigenvectors of negative eigenvalues form the direction of Theorem
 * sec5:thm1), by Lanczos with full reorthogonalisation.  Synchronous.
 * evals_host: k doubles, ascending; lambda_max_host: 1 double; evecs_dev
 * (nullable): n*k doubles, eigenvector i at offset i*n (unit norm).  Stops when
 * the residuals ||X v_i - theta_i v_i|| of all k smallest Ritz pairs are
 * <= tol (1 + |lambda_max|), or after maxit steps: then MDSDP_ENOCONV with the
 * best estimates written.  EINVAL: k < 1, k > n, maxit < k + 2, tol <= 0. */
mdsdp_status mdsdp_min_eigpair(mdsdp_problem prob, int32_t k, double tol, int32_t maxit, uint64_t seed,
                               double* evals_host, double* lambda_max_host, double* evecs_dev,
                               int32_t* iters, void* stream);
/* Allocation-free variant of mdsdp_min_eigpair, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments and results, but the
 * Lanczos basis and coefficients live in a fixed device scratch of 4 Mi
 * doubles (32 MiB) per GPU, held until the process ends, instead of buffers
 * the problem allocates on demand.  Needs n (maxit' + 1) + n + 4 maxit' + 16
 * <= 4194304 doubles with maxit' = min(maxit, n), else MDSDP_EINVAL before any
 * work; the current device must be the problem's.  Every call on a GPU uses
 * that GPU's one scratch: calls that overlap on one GPU (other threads or
 * streams) race and must be serialised by the caller.  Makes no hipMalloc,
 * hipFree or allocating library call. */
mdsdp_status mdsdp_min_eigpair_noalloc(mdsdp_problem prob, int32_t k, double tol, int32_t maxit,
                                       uint64_t seed, double* evals_host, double* lambda_max_host,
                                       double* evecs_dev, int32_t* iters, void* stream);
/* The certificate spectrum estimate the solver uses for eta_d (eq. res):
 * Lanczos from `warm_dev` (n doubles, nullable: a random start) plus a small
 * random component, stopping when the error estimate of theta_min -- its
 * residual, or residual^2 / gap when the gap theta_2 - residual_2 - theta_min
 * is positive -- is <= tol (1 + |theta_max|), or after maxit steps.
 * out_host[4] = {theta_min, theta_max, error estimate, converged (0/1)};
 * evec_dev (nullable, n doubles) receives the Ritz vector of theta_min.  The
 * solver takes max(0, -(theta_min - error)) / (1 + |theta_max|) for eta_d
 * when the run did not converge.  Synchronous; MDSDP_OK either way. */
mdsdp_status mdsdp_certificate_estimate(mdsdp_problem prob, double tol, int32_t maxit, uint64_t seed,
                                        const double* warm_dev, double* out_host, double* evec_dev,
                                        int32_t* iters, void* stream);
/* Adjoint of the optimal value w.r.t. C: dv/dC = X + Diag z = Xt + D
 * (Lagrangian duality, dual problem PSDP).  Writes a dense n x n FP64 device
 * matrix. */
/* Certified lower bound of lambda_min of the certificate X = Xt + D - Diag(z)
 * (z of the last mdsdp_update_multiplier) as a solve ends on it (eq. res,
 * eta_d): Lanczos on the complement of range(Y) (Y_dev: n x p FP64 device,
 * 1 <= p <= min(512, n - 2)) from a random start, run until theta_min has
 * converged to tol (1 + |theta_max|) or maxit steps, combined with the
 * compression to range(Y): lambda_min(X) >= the smaller eigenvalue of
 * [[lambda_min(Q^T X Q), -||B||], [-||B||, lambda_min(C)]] (B the coupling,
 * C the complement block).  out_host[4] = {lower bound, largest Ritz value,
 * Lanczos steps, converged (1/0)}.  Allocates its work buffers. */
mdsdp_status mdsdp_certificate_bound(mdsdp_problem prob, int32_t p, const double* Y_dev, double tol,
                                    int32_t maxit, uint64_t seed, double* out_host, void* stream);
mdsdp_status mdsdp_adjoint_C(mdsdp_problem prob, double* dC_dev, void* stream);

/* ---- full solve (Algorithm alg1 with RTR + truncated CG) ------------------- */
typedef struct {
  double tol;          /* stop when eta_max <= tol (eq. res; the eta_d a solve ends on comes from a
                          verify eigensolve: random start, residual error, no early stop); default 1e-8 */
  int32_t max_outer;   /* default 200 */
  double sigma0, sigma_min, sigma_max, gamma, kappa1, kappa2; /* eq. sec5:eq1 */
  int32_t p_max;       /* largest factor width, 1..512 (default 512) */
  int32_t n_neg;       /* negative-curvature directions added per outer step (Theorem sec5:thm1);
                          default 15, so that one column plus the carried ones fit 16-column tiles */
  double tau_rank;     /* drop singular directions below tau_rank * s_1 (default 1e-7) */
  double gtol0, gtol_min;  /* inner tolerance of subproblem k (see gtol_ratio); default 1e-2, 1e-10 */
  double gtol_decay;   /* in (0, 1]; used only when gtol_ratio <= 0 */
  double gtol_ratio;   /* > 0 (default 0.1): RTR for subproblem k stops at
                          ||grad|| <= max(gtol_min, min(gtol0, gtol_ratio ||R^k|| / (1 + ||b||))), the
                          scaled primal residual that eq. sec5:eq1 weighs against ||grad|| (gtol0 at
                          k = 0); <= 0: max(gtol_min, min(gtol0, 0.1 eta_max, gtol_decay * previous)) */
  double gtol_stall;   /* > 0: when an RTR call starts below its tolerance (takes no step), cap all
                          later tolerances at gtol_stall * ||grad||; default 0 (off) */
  int32_t sigma_hold;  /* 1 (default): eq. sec5:eq1, but its decrease branch is not taken after an RTR
                          call that stopped at its iteration budget (||grad|| then measures the
                          unfinished inner solve, not a dual residual); 0: the rule as printed */
  int32_t rtr_maxiter, tcg_maxinner; /* RTR iterations per subproblem (default 10; see rtr_maxiter_polish)
                          and truncated-CG steps per RTR iteration (default 200) */
  int32_t hvp_prec;    /* mdsdp_prec for tCG HVPs */
  int32_t polish_fp64; /* switch HVPs to FP64 once eta_max < polish_eta (default 1e-4) */
  double polish_eta;
  double eig_tol;
  int32_t eig_maxit;
  double time_limit_s; /* 0 = none */
  int32_t verbose;     /* 0 quiet; 1 one stderr line per outer iteration; 2 also one per RTR step */
  uint64_t seed;
  int32_t resume;      /* 0: start from Xt = 0, sigma = sigma0; 1: continue from the problem's current
                          multiplier Xt with sigma = sigma0 (e.g. the sigma a previous solve returned) */
  int32_t escape_when_solved; /* 1: form the carried direction of Theorem sec5:thm1 and add its zero
                          columns only after an RTR call that reached its tolerance; 0 (default): after
                          every outer step whose certificate has curvature below
                          -max(1e-12, tol) (1 + |lambda_max|) (step 9 of Algorithm alg1) */
  int32_t deflate;     /* 1 (default): the certificate eigensolve runs on the complement of range(Y)
                          and combines it with the compression Q^T X Q to range(Y) (the block bound of
                          mdsdp_certificate_bound); 0: plain Lanczos on X */
  int32_t direct_admm; /* 1: solve DSDP by the two-block ADMM with the direct S-subproblem
                          (mdsdp_set_direct; the ablation of section "Why solve DSDP' instead of
                          DSDP"); 0 (default): ManiDSDP on DSDP' */
  int32_t rtr_warm_radius; /* 1 (default): each RTR call starts from the previous call's final trust
                          radius (capped at Delta_bar / 8); 0: from Delta_bar / 8 */
  int32_t rtr_maxiter_polish; /* RTR iteration budget once eta_max < polish_eta (default 50; the budget
                          before that is rtr_maxiter, default 10) */
  int32_t round_rank_one; /* 1 (default): rank-one compression test of Theorem thm:finite-locking and
                          Remark rem:inexact-near-locking: after an outer step with eta_max < round_eta
                          whose Y has s_2 <= round_gap s_1, eq. res is evaluated at Y1 = sign(Y v_1)
                          (n x 1) with the current multiplier and no multiplier step; the solve stops
                          there (p_final = 1, rank_one_round = 1) when that point meets tol, and the
                          iteration is unchanged otherwise.  0: off */
  double round_eta;    /* default 1e-3 */
  double round_gap;    /* in [0, 1], default 0.1 */
  int32_t tcg_maxinner_polish; /* truncated-CG steps per RTR iteration once eta_max < polish_eta
                          (default 1000; before that tcg_maxinner) */
  int32_t rtr_stall;   /* > 0: an RTR call also ends after this many consecutive iterations that leave
                          ||grad|| above 0.9 times its best value in the call; 0 (default): off */
} mdsdp_options;

typedef struct {
  int32_t status;       /* mdsdp_status of the solve */
  int32_t outer_iters;
  int64_t rtr_iters, hvps, cost_grads, eig_iters;  /* hvps: HVPs whose result the solver used (the one
                                                      speculative HVP a truncated-CG stop discards is
                                                      not counted; its time is) */
  int32_t p_final, p_max_reached;
  double value;         /* b^T y */
  double eta_p, eta_d, eta_g;
  double sigma;
  double seconds;
  double t_eval, t_hvp, t_eig, t_update; /* seconds per phase */
  int32_t rank_one_round; /* 1: the final point is the rank-one compression (see round_rank_one) */
} mdsdp_result;

void mdsdp_default_options(mdsdp_options* opt);
/* Y_dev: device buffer of n * p_max doubles; on entry its first n*p0 values
 * (row-major n x p0) are the start (rows are normalised); on exit it holds
 * the final Y as row-major n x p_final.  history_host (nullable) receives up
 * to history_cap records of 8 doubles per outer iteration:
 * {k, p, sigma, eta_p, eta_d, eta_g, value, hvps}. */
mdsdp_status mdsdp_solve(mdsdp_problem prob, const mdsdp_options* opt, int32_t p0, double* Y_dev,
                         mdsdp_result* res, double* history_host, int32_t history_cap,
                         void* stream);

/* Batch of independent problems (e.g. many small relaxations of uneven size):
 * nworkers host threads, each with its own HIP stream (default priority),
 * take problems from a shared work queue ordered by decreasing n and run
 * mdsdp_solve on them, so the kernels of different problems overlap on the
 * GPU.  probs[i], p0[i], Ybufs[i] (device, n_i * p_max doubles) as for
 * mdsdp_solve; results[i] receives each solve's result (status included);
 * the same options for all.  Returns MDSDP_OK when every problem reached the
 * tolerance, MDSDP_ENOCONV if one did not, or the first error met.  Each
 * problem must be used by no other thread during the call. */
mdsdp_status mdsdp_solve_batch(int32_t nprob, mdsdp_problem* probs, const mdsdp_options* opt,
                               const int32_t* p0, double* const* Ybufs, mdsdp_result* results,
                               int32_t nworkers);

/* ---- diagnostics -----------------------------------------------------------
 * Export internal tile-major arrays back to packed order (host buffers of
 * n(n+1)/2): the class map as seen by the kernels, and Xt. */
mdsdp_status mdsdp_export_classmap(mdsdp_problem prob, int32_t* cls_host);
mdsdp_status mdsdp_export_multiplier_packed(mdsdp_problem prob, double* Xt_host);
/* Per-kernel device timing of the most recent call of each entry point,
 * measured with HIP events on the launch stream (milliseconds). */
mdsdp_status mdsdp_kernel_times(mdsdp_problem prob, double* ms_out, int32_t cap,
                                int32_t* count);
mdsdp_status mdsdp_enable_timing(mdsdp_problem prob, int32_t on);
/* Average duration (microseconds) of the HVP product pass -- the per-entry
 * residual/product kernel of the last mdsdp_hvp call, with that call's
 * precision, factor width and staged inputs -- measured by re-launching it
 * `reps` times back to back on `stream` between two HIP events.  Synchronous.
 * The pass only rewrites its own partial sums, so the state is unchanged.
 * EINVAL if no HVP has been evaluated yet. */
mdsdp_status mdsdp_time_product_pass(mdsdp_problem prob, int32_t reps, double* us_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MANIDSDP_H */

/*
 * igafd.h -- C ABI of the MI355X (gfx950) fast-diagonalisation preconditioned
 * CG solver for the isogeometric Galerkin Poisson problem.
 *
 * Method: Sangalli & Tani, "Isogeometric preconditioners based on fast solvers
 * for the Sylvester equation" (arXiv 1602.01636).
 *
 *   problem     -div(K grad u) = f on Omega = F([0,1]^d), u = 0 on the boundary,
 *               K = kappa(x) I                                   (Sec. 2.1 eq. poisson)
 *   space       tensor B-splines of degree p on open knot vectors, Dirichlet
 *               functions 2..m-1 per direction, n_d = m_d - 2   (Sec. 2.1 eq. Vh)
 *   system      A u = b, A_ij = int grad(B_i)^T Q grad(B_j),
 *               Q = |det J| J^-1 K J^-T (J_ij = dF_i/dxi_j)     (Sec. 2.1 eq. A, eq. Q)
 *   precond.    P = Kronecker sum of the 1D stiffness/mass       (Sec. 3 eq. prec)
 *               applied by fast diagonalisation                  (Sec. 4.1 Alg. 1, Sec. 5.1 Alg. 3)
 *   solver      preconditioned CG                                (Sec. 3)
 *
 * Conventions shared by every call:
 *  - Vectors are caller-owned device buffers of N = prod n_d doubles laid out
 *    as a C array [n3][n2][n1] (2D: [n2][n1]): direction 1 is the fastest
 *    index, as the scalar index of Sec. 2.1.
 *  - Every call is ordered on the stream given to igafd_setup (a hipStream_t,
 *    NULL = the null stream).  Calls returning data to host memory
 *    synchronise that stream before returning; device results are complete
 *    when the stream reaches them.
 *  - Errors are reported by the returned status; nothing throws across the
 *    ABI.  igafd_last_error() gives a thread-local message for the last
 *    non-OK status.  A status > 0 is a warning with results written.
 *  - The context owns every device allocation it makes (matrix band,
 *    eigenvector copies, workspace); igafd_destroy frees them.
 */
#ifndef IGAFD_H
#define IGAFD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct igafd_ctx igafd_ctx;

typedef enum {
  IGAFD_OK = 0,
  IGAFD_NOT_CONVERGED = 1,     /* maxit reached; best iterate written, info filled */
  IGAFD_ERR_ARG = -1,          /* invalid argument (message says which)            */
  IGAFD_ERR_ALLOC = -2,        /* device or host allocation failed                 */
  IGAFD_ERR_HIP = -3,          /* a HIP runtime call failed                        */
  IGAFD_ERR_GEOMETRY = -4,     /* det J <= 0 at a quadrature point                 */
  IGAFD_ERR_NOT_SPD = -5,      /* Cholesky of a 1D mass matrix failed              */
  IGAFD_ERR_BREAKDOWN = -6     /* CG breakdown: p^T A p <= 0 or not finite         */
} igafd_status;

/* precision of the mode products inside the preconditioner apply.
 * IGAFD_BF16X3: split BF16 (Henry, Tang and Heinecke, "Leveraging the bfloat16
 * artificial intelligence datatype for higher-precision computations", 2019):
 * each FP32 operand x is held as hi + lo with hi = bf16(x), lo = bf16(x - hi),
 * and a product a b is taken as lo_a hi_b + hi_a lo_b + hi_a hi_b (three BF16
 * MFMAs, FP32 accumulation): at most about 3 * 2^-16 relative error per product
 * instead of BF16's 2^-8, on the same BF16 matrix cores. */
typedef enum { IGAFD_FP64 = 0, IGAFD_FP32 = 1, IGAFD_BF16 = 2, IGAFD_BF16X3 = 3 } igafd_precision;

/* geometry maps F (analytic, evaluated exactly at the quadrature points) */
enum {
  IGAFD_GEOM_IDENTITY = 0,  /* F(xi) = xi (unit square / cube); no parameters                  */
  IGAFD_GEOM_RING = 1,      /* F = ((1+xi1)cos(pi xi2/2), (1+xi1)sin(pi xi2/2) [, xi3]);
                               2D quarter annulus / 3D thick quarter ring; no parameters       */
  IGAFD_GEOM_WARPED = 2     /* F = xi + a sum_k c_k prod_l sin(pi m_kl xi_l), k = 1..K <= 16;
                               params = [a, K, c_1 (d values), ..., c_K, m_1 (d values), ..., m_K] */
};

/* coefficient kappa(x), K = kappa I, evaluated at x = F(xi) */
enum {
  IGAFD_COEF_ONE = 0,       /* kappa = 1                                                       */
  IGAFD_COEF_SINCOS = 1     /* kappa = 1 + a sin(2 pi f1 x + phi1) cos(2 pi f2 y + phi2);
                               params = [a, f1, f2, phi1, phi2]                                */
};

/* right-hand sides f for igafd_load_vector */
enum {
  IGAFD_RHS_SINPROD = 0,    /* f = d pi^2 prod_i sin(pi x_i)                                   */
  IGAFD_RHS_PAPER_POLY = 1, /* f = 2 sum_i (x_i^2 - x_i)  (the paper's Sec. 7 choice)          */
  IGAFD_RHS_BUBBLE = 2,     /* f = 2 sum_i prod_{l != i} x_l (1 - x_l)                         */
  IGAFD_RHS_ONE = 3         /* f = 1                                                           */
};

typedef struct {
  int dim;                     /* d in {2, 3}                                                  */
  int degree;                  /* p in 1..6, the same in every direction (Sec. 2.1)            */
  int nknots[3];               /* knot-vector lengths m_d + p + 1                              */
  const double* knots[3];      /* host arrays; open on [0,1] (eq. knot-vector), nondecreasing,
                                  interior multiplicity <= p; copied during setup              */
  int geom_kind;               /* IGAFD_GEOM_*                                                 */
  int n_geom_params;
  const double* geom_params;   /* host, see IGAFD_GEOM_*                                       */
  int coef_kind;               /* IGAFD_COEF_*                                                 */
  int n_coef_params;
  const double* coef_params;   /* host, see IGAFD_COEF_*                                       */
  int quad_per_dir;            /* Gauss points per element and direction: 0 or p+1             */
  int want_features;           /* 1: igafd_setup also sums the per-dof inputs of the learned
                                  scaling (igafd_features) from the Gauss-point values it
                                  evaluates for A, and keeps them (8N floats)                  */
} igafd_problem;

/*
 * Setup (host + device): validate the knots, evaluate the B-splines at the
 * Gauss points (Sec. 2.1 eq. cox-deboor), build the 1D M_d, K_d (Sec. 3),
 * their generalised eigendecompositions K U = M U D with U^T M U = I by
 * Cholesky + symmetric eigensolver (Sec. 4.1 computational cost), upload
 * U_d, D_d, and assemble A on the device (eq. A).  `stream` is a hipStream_t
 * or NULL.  On success *out owns all device memory of the problem.
 */
igafd_status igafd_setup(const igafd_problem* prob, void* stream, igafd_ctx** out);

/*
 * Preconditioner-only setup: everything igafd_setup builds for P (the
 * univariate matrices, U_d, D_d, the FD intermediates: 2N doubles), but no A
 * and no CG workspace.  On the unit square / cube with kappa = 1, P = A
 * (Sec. 3), so igafd_apply_precond is then the fast-diagonalisation direct
 * solver of Sec. 4.1 / 5.1 (the paper's Tables square and cube), also at sizes
 * whose A would not fit (10^9 unknowns take 4 vectors of 8.6 GB, not 1.5 TB
 * of band).  apply_precond, set_scaling, set_adi, get_adi, load_vector,
 * spectral_bounds, sizes (band_bytes = 0) and get_eigen work; calls that need
 * A (apply_A, solve, solve_batched, diagonals, features, scaling_targets,
 * set_scaling_diag_ratio, autotune) return IGAFD_ERR_ARG.
 */
igafd_status igafd_setup_precond(const igafd_problem* prob, void* stream, igafd_ctx** out);

/* Sizes of the discrete problem (Sec. 2.1 eq. Vh: n_d = m_d - 2 Dirichlet
 * functions per direction; eq. A: A has at most (2p+1)^d nonzeros per row).
 * Host outputs, any may be NULL: n[3] dofs per direction (n[2] = 1 in 2D),
 * N = prod n, nnz = nonzeros of A counted over the full matrix, band_bytes =
 * device bytes of the stored half band (0 for a preconditioner-only context).
 * IGAFD_ERR_ARG on a NULL context. */
igafd_status igafd_sizes(const igafd_ctx* ctx, int n[3], long long* N, long long* nnz,
                         long long* band_bytes);

/* Load vector of the Galerkin system (Sec. 2.1, the right-hand side of
 * eq. A's system): b_i = int_Omega f B_i dx = sum_t w_t |det J(t)| f(F(t)) B_i(t)
 * with the Gauss rule of A.  f is IGAFD_RHS_<rhs_kind>; rhs_params (host,
 * n_rhs_params values, NULL / 0 for the defaults) scale and tune it:
 *   SINPROD     [amp, k_1, .., k_d]: f = amp prod_i sin(k_i pi x_i)
 *               (default amp = d pi^2, k_i = 1)
 *   PAPER_POLY, BUBBLE, ONE   [amp]: f times amp (default 1)
 * b_dev: N doubles (device), overwritten.  IGAFD_ERR_ARG for an unknown kind
 * or a wrong parameter count. */
igafd_status igafd_load_vector(igafd_ctx* ctx, int rhs_kind, const double* rhs_params, int n_rhs_params,
                               double* b_dev);

/* y = A x (banded FP64 product, Sec. 2.1 eq. A); x_dev, y_dev: N doubles, distinct. */
igafd_status igafd_apply_A(igafd_ctx* ctx, const double* x_dev, double* y_dev);

/* s = P^-1 r by fast diagonalisation (Alg. 1 / Alg. 3), mode products in the
 * given precision (FP64, FP32, BF16 inputs with FP32 accumulation, or split BF16); r and s
 * stay FP64.  With a scaling set (igafd_set_scaling) computes S P^-1 S r.
 * r_dev, s_dev: N doubles; s may not alias r. */
igafd_status igafd_apply_precond(igafd_ctx* ctx, int precision, const double* r_dev, double* s_dev);

/* Diagonal scaling S > 0 (N doubles, device, copied into the context; NULL
 * disables it) for the preconditioner S P^-1 S.  The paper's P ignores the
 * variation of Q over the domain (Sec. 3, Prop. 1 and the remark after it);
 * S, e.g. predicted by the network below, corrects the local magnitude.
 * Allocates N doubles on first use.  IGAFD_ERR_ARG for the L-shaped context. */
igafd_status igafd_set_scaling(igafd_ctx* ctx, const double* S_dev);

typedef struct {
  double rtol;                 /* stop when ||r_k||_2 <= rtol ||b||_2 (recursive residual)     */
  int maxit;                   /* maximum CG iterations (0 -> 2000)                            */
  int precision;               /* igafd_precision of the preconditioner apply                  */
  int flexible;                /* 1: Polak-Ribiere beta (required for all but FP64 applies)    */
  int use_scaling;             /* 1: S P^-1 S with the scaling set by igafd_set_scaling;
                                  2: decided by igafd_scaling_gate (default gain 2): S P^-1 S
                                  when the gate passes and a scaling is set, else plain P     */
  int check_every;             /* iterations enqueued between host checks (0 -> 4)             */
  int use_x0;                  /* 1: u_dev holds the initial guess; 0: x0 = 0                  */
  double* history;             /* optional host array of maxit+1 relative residuals: entry k is
                                  ||r_k||/||b|| after iteration k (k = 0: the start); at most
                                  maxit+1 entries are written, also when a fallback or a
                                  restart runs more iterations (info.history_len says how
                                  many).  maxit > 2000 with a history grows the context's
                                  device history buffer once                               */
  int timers;                  /* 1: time the phases (events between kernels; adds a few us
                                  per iteration) into info.t_spmv_ms / t_fd_ms / t_vec_ms   */
} igafd_solve_opts;

typedef struct {
  int iters;                   /* CG iterations (one A product + one apply each)               */
  int restarts;                /* restarts from the true residual                              */
  double relres;               /* final recursive ||r||/||b||                                  */
  double true_relres;          /* ||b - A u||/||b|| evaluated in FP64 at exit                   */
  int status;                  /* igafd_status of the solve                                    */
  double t_solve_ms;           /* device time of the whole solve (events on the ctx stream)    */
  int fallback;                /* 1: the scaled preconditioner stagnated and plain P finished  */
  int history_len;             /* entries written to opts.history (0 without one)              */
  double t_setup_ms;           /* host wall time of the context's setup (1D setup, uploads,
                                  assembly of A)                                              */
  double t_spmv_ms;            /* with opts.timers: device time in A products and their (p, q)
                                  reductions (the true-residual product included)            */
  double t_fd_ms;              /* with opts.timers: preconditioner applies and (r, z) reductions */
  double t_vec_ms;             /* with opts.timers: vector updates, init, residual and the other
                                  reductions; t_solve - (spmv + fd + vec) is host wait time   */
  int scaled;                  /* 1: the solve started with S P^-1 S                             */
  double kappa_bound;          /* qmax / qmin of Prop. 1 when the gate ran (use_scaling = 2)    */
} igafd_solve_info;

/* PCG for A u = b preconditioned by P (or S P^-1 S).  b_dev, u_dev: N doubles.
 * Returns IGAFD_OK, IGAFD_NOT_CONVERGED (u holds the last iterate) or an error. */
igafd_status igafd_solve(igafd_ctx* ctx, const double* b_dev, double* u_dev,
                         const igafd_solve_opts* opts, igafd_solve_info* info);

/* Independent problems solved together (the batch workload).  When every
 * problem is 3D with the fused FD passes, each step of a CG iteration is one
 * grouped launch over all running problems (device job tables allocated for
 * the call), on one stream that the contexts share for the duration of the
 * call; otherwise the contexts are bound to a pool of streams.  Each chunk of
 * check_every iterations (rounded up to even) is captured into one HIP graph
 * and replayed until every problem has converged (re-captured when problems
 * finish).  Every problem's iterates are bitwise those of its own igafd_solve.
 * b[i], u[i]: device vectors of ctxs[i]; x0 = 0.  infos (count entries) and
 * wall_ms (device time of the CG loops) optional.  Environment (testing):
 * IGAFD_BATCH_GROUPED=0 forces the stream pool. */
igafd_status igafd_solve_batched(igafd_ctx* const* ctxs, int count, const double* const* b, double* const* u,
                                 const igafd_solve_opts* opts, igafd_solve_info* infos, double* wall_ms);

/* Kernel shape of one problem: fd_tiles (16-row tiles per wave in the mode
 * products, 1..8) and spmv_rows (rows per thread of the row-parallel A
 * product: 1, 2, 4; a nonzero value selects that kernel instead of the 3D
 * tiled one).  Zero for both: time the candidates on this problem (row
 * counts, and tile shapes at 256 and 512 threads per block) and keep the
 * fastest (a later candidate must win by 1%, so near-ties resolve the same
 * way each time); may allocate the tile buffer, so call it at setup time,
 * not inside a timed or captured region. */
igafd_status igafd_autotune(igafd_ctx* ctx, int fd_tiles, int spmv_rows);

/* Kernel shape in use (host outputs, any may be NULL): tile_b2, tile_b3 = the
 * lines per tile of the 3D tiled A product (0 when the row-parallel kernel
 * with spmv_rows rows per thread is used) and tile_threads its threads per
 * block (256 or 512); fd_fused = 1 when the 3D FD apply runs as three fused
 * passes, fd_tiles = row tiles per wave of the generic mode products
 * otherwise. */
igafd_status igafd_get_shape(const igafd_ctx* ctx, int* spmv_rows, int* tile_b2, int* tile_b3, int* fd_fused,
                             int* fd_tiles, int* tile_threads);

/* Diagonals of A and P (N doubles each, device; either may be NULL). */
igafd_status igafd_diagonals(igafd_ctx* ctx, double* diagA_dev, double* diagP_dev);

/* A-priori bounds of the preconditioned spectrum (Sec. 3, Prop. 1): every
 * eigenvalue of P^-1 A lies in [qmin, qmax], the smallest and largest
 * eigenvalue of Q = kappa |det J| J^-1 J^-T over the Gauss points of the
 * mesh (A and P are assembled with the same rule, so the bound holds for the
 * discrete matrices); qmax / qmin bounds the condition number that drives
 * the CG iteration count.  qloc = the largest local ratio
 * lambda_max(Q(x)) / lambda_min(Q(x)) over the same points: the anisotropy
 * of Q at a point, which no diagonal scaling of P removes.  Host outputs (any
 * may be NULL).  Computed once per context (synchronises its stream), cached
 * afterwards.  IGAFD_ERR_ARG for the L-shaped context. */
igafd_status igafd_spectral_bounds(igafd_ctx* ctx, double* qmin, double* qmax, double* qloc);

/* Gate of the scaled preconditioner, from the bounds above (Sec. 3, Prop. 1
 * and the remark after it, that the quality of P is decided by how much Q
 * varies): a diagonal scaling S P^-1 S can at best remove the variation of
 * Q's magnitude over the domain, so its Prop. 1-type bound cannot drop below
 * qloc.  *use = 1 when (qmax / qmin) / qloc >= gain, i.e. when the bound
 * could shrink by at least `gain` (> 0; igafd_solve's use_scaling = 2 takes
 * gain 2); *kappa_q = qmax / qmin, *kappa_loc = qloc (host outputs, any may be
 * NULL).  Examples: the thick ring has Q = diag(w, 1/w, w) at every point, so
 * qmax / qmin = qloc = pi^2 and the gate stays closed; a coefficient varying
 * by 3x on a mildly warped cube opens it. */
igafd_status igafd_scaling_gate(igafd_ctx* ctx, double gain, int* use, double* kappa_q, double* kappa_loc);

/* Host copy of U_d (n_d x n_d row-major, U[i][k] = component i of eigenvector k,
 * U^T M U = I) and of the eigenvalues D_d for direction dir (0-based). */
igafd_status igafd_get_eigen(const igafd_ctx* ctx, int dir, double* U_host, double* lam_host);

/* Host-only: 1D matrices and generalised eigendecomposition for one knot
 * vector (Sec. 3, Sec. 4.1).  M, K, U: n x n row-major, lam: n; n = nknots-p-3
 * is written to *n_out.  Needs no GPU. */
igafd_status igafd_univariate(int degree, int nknots, const double* knots, int quad,
                              double* M, double* K, double* U, double* lam, int* n_out);

/* ---------------- three-variable ADI (inexact P^-1) ----------------
 * Sec. 5.2 (eq. ADI3D, Alg. "3D ADI method") and Sec. 4.2 Thm. ADIprec: J
 * steps of the ADI iteration of Douglas for P s = r from s_0 = 0 give
 * s_J = P_J^-1 r with P_J symmetric positive definite and
 * kappa(P_J^-1 A) <= (1 + eps)/(1 - eps) kappa(P^-1 A) when ||T_J|| <= eps.
 * Parameters: geometric between the smallest and largest eigenvalue a, b of
 * the M_d^-1 K_d, omega_j = a (b/a)^((j-1)/(J-1)); J the smallest count with
 * ||T_J|| <= eps (||T_J|| evaluated exactly over the triples of univariate
 * eigenvalues), at most J0 = ceil(1.16 ln(b/a) ln(1/eps)) (eq. ADI3Diter).
 */

/* From now on igafd_apply_precond and igafd_solve apply P_J^-1 (FP64 only,
 * no scaling) instead of the exact fast diagonalisation; eps in (0, 1), or 0
 * to switch back to FD.  3D single-patch contexts.  Allocates the univariate
 * bands and factors and 5 N doubles of workspace.  *J (steps) and *rho
 * (= ||T_J||) are optional host outputs. */
igafd_status igafd_set_adi(igafd_ctx* ctx, double eps, int* J, double* rho);

/* As igafd_set_adi with the greedy parameters of Sec. 5.2 eq. greedy1/2:
 * after k steps the eigenvalue triple of largest |prod_j g_j| (the first in
 * (k3, k2, k1) order on ties) gives omega_{k+1}, the omega >= 0 minimising
 * |g| there (in closed form: the smaller positive root of
 * w^3 - S w^2 + e2 w + e3 when it has one, else the positive root of
 * w^3 - e2 w - 2 e3, with S, e2, e3 the symmetric functions of the triple);
 * omega_1 = sqrt(a b).  Stops at the first J with ||T_J|| <= eps, at most J0.
 * Needs n1 n2 n3 <= 2^28 (one host double per triple during setup). */
igafd_status igafd_set_adi_greedy(igafd_ctx* ctx, double eps, int* J, double* rho);

/* Parameters in use (all outputs optional, host): J = 0 when ADI is off;
 * omegas: capacity >= J values. */
igafd_status igafd_get_adi(const igafd_ctx* ctx, int* J, int* J0, double* rho, double* omegas, int capacity);

/* ---------------- multi-patch: L-shaped domain, additive Schwarz ----------------
 * Sec. 6 (eq. Pias) and the multi-patch experiment of Sec. 7: the L-shaped
 * domain [0,1]^2 without (1/2,1] x (1/2,1], made of three square patches
 * (the corner patch [0,1/2]^2, the patch above it and the patch to its
 * right) with C^0 continuity across the two interfaces and the Dirichlet
 * Poisson problem (K = I) on it.  The overlapping subdomains are the two
 * pairs of patches sharing an interface (Theta_1 = corner + upper patch,
 * Theta_2 = corner + right patch); the preconditioner is
 *     P_IAS^-1 = sum_i R_i^T P_i^-1 R_i,
 * P_i the Kronecker-sum preconditioner of Theta_i in its own parameter domain
 * (one patch along one direction, two joined by a p-fold knot along the
 * other), applied by fast diagonalisation.
 *
 * Layout: vectors of an L-shaped context live on the bounding square's grid,
 * n x n with n = 2h + 1 (h = interior functions per patch and direction,
 * direction 1 fastest); the entries with i1 >= h and i2 >= h are not unknowns
 * of the problem.  Every entry point of such a context writes zeros there
 * and ignores what its inputs hold there.  igafd_apply_A, igafd_apply_precond
 * (P_IAS^-1, any precision), igafd_load_vector (f evaluated at x = xi),
 * igafd_solve and igafd_autotune work as for one patch; the scaled
 * preconditioner, the diagonals, the learned-scaling calls, the spectral
 * bounds and igafd_solve_batched return IGAFD_ERR_ARG.
 */

/* Setup of the L-shaped problem: every patch carries, in both directions, the
 * open knot vector `knots` on [0,1] (host, nknots values, copied), so the
 * patch meshes are conforming.  Assembles A on the device and factors the two
 * subdomains' univariate matrices.  `stream` as in igafd_setup. */
igafd_status igafd_lshape_setup(int degree, int nknots, const double* knots, void* stream, igafd_ctx** out);

/* *hole = h, the first index (in both directions) of the grid entries that are
 * not unknowns, or -1 for a single-patch context; *ndofs = number of unknowns
 * (N - (n - h)^2, or N).  Either output may be NULL. */
igafd_status igafd_lshape_corner(const igafd_ctx* ctx, int* hole, long long* ndofs);

/* ---------------- learned diagonal scaling (S P^-1 S) ----------------
 * The paper notes that P degrades when Q varies strongly over the domain
 * (Sec. 3, remarks after Prop. 1).  A small network predicts a diagonal S from
 * local geometry/coefficient statistics; the solver then uses S P^-1 S, with
 * plain P as the fallback when the scaled solve fails to converge.
 */

/* Per-dof inputs, N x 8 FP32 (device): the B_i-weighted quadrature averages
 * over supp B_i of the entries (11, 22, 33, 12, 13, 23) of |det J| J^-1 J^-T
 * and of kappa, then the degree p.  A context set up with want_features
 * copies the ones it assembled with A; otherwise they are computed now
 * (allocates and frees an accumulator of 8N doubles, synchronises the
 * stream). */
igafd_status igafd_features(igafd_ctx* ctx, float* feat_dev);

/* igafd_features for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same output as igafd_features; allocates nothing, frees nothing and does
 * not synchronise (kernel launches on the context's stream only, the
 * accumulator cleared by a kernel, not a memset).  A context set up with
 * want_features is copied as by igafd_features; otherwise the feature sums
 * go through a static device accumulator of 8 doubles per dof for at most
 * 2^20 = 1,048,576 dofs (64 MiB, held by each GPU the library runs on until
 * the process ends): a larger N returns IGAFD_ERR_ARG.  Every call on one
 * GPU shares that accumulator, which keeps the last call's contents (each
 * call clears what it uses first): calls that overlap on one GPU (other
 * streams, other host threads) race.  The context's device must be current. */
igafd_status igafd_features_noalloc(igafd_ctx* ctx, float* feat_dev);

/* Training targets t_i = 1/2 log(P_ii / A_ii) (N floats, device). */
igafd_status igafd_scaling_targets(igafd_ctx* ctx, float* t_dev);

/* Sets the scaling to the exact diagonal ratio S_i = (P_ii / A_ii)^(1/2)
 * (the quantity the network learns; reference point for its gain). */
igafd_status igafd_set_scaling_diag_ratio(igafd_ctx* ctx);

/* Network 8 -> 64 -> 64 -> 1 (tanh), BF16 weights with FP32 accumulation on
 * MFMA, FP32 master weights, Adam.  Parameters (igafd_mlp_num_params floats)
 * are W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3, followed in the
 * get/set arrays by the input normalisation mean[8], 1/std[8].  Calls are
 * ordered on `stream`; the object owns its device buffers. */
typedef struct igafd_mlp igafd_mlp;
int igafd_mlp_num_params(void);
igafd_status igafd_mlp_create(unsigned long long seed, void* stream, igafd_mlp** out);
void igafd_mlp_destroy(igafd_mlp* mlp);
/* input normalisation from n feature rows (device, n x 8) */
igafd_status igafd_mlp_fit_normalization(igafd_mlp* mlp, const float* feat_dev, long long n);
/* host arrays of igafd_mlp_num_params() + 16 floats */
igafd_status igafd_mlp_get_params(const igafd_mlp* mlp, float* host);
igafd_status igafd_mlp_set_params(igafd_mlp* mlp, const float* host);
/* t = MLP(feat) (n floats, optional) and S = exp(t) (n doubles, optional), device */
igafd_status igafd_mlp_forward(igafd_mlp* mlp, const float* feat_dev, long long n, float* t_dev, double* S_dev);
/* gradient of L = (1/n) sum (t - target)^2 w.r.t. the parameters (host array of
 * igafd_mlp_num_params floats) and L; no update */
igafd_status igafd_mlp_gradient(igafd_mlp* mlp, const float* feat_dev, const float* target_dev, long long n,
                                float* grad_host, float* loss_host);
/* one Adam step on the minibatch (feat n x 8, target n); loss_host optional (syncs) */
igafd_status igafd_mlp_train_step(igafd_mlp* mlp, const float* feat_dev, const float* target_dev, long long n,
                                  float lr, float* loss_host);

void igafd_destroy(igafd_ctx* ctx);
const char* igafd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGAFD_H */

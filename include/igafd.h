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

/* precision of the mode products inside the preconditioner apply */
typedef enum { IGAFD_FP64 = 0, IGAFD_FP32 = 1, IGAFD_BF16 = 2 } igafd_precision;

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

/* Sizes: n[3] dofs per direction (n[2] = 1 in 2D), N = prod n, nnz = stored
 * nonzeros of A counted over the full matrix, band_bytes = device bytes of A. */
igafd_status igafd_sizes(const igafd_ctx* ctx, int n[3], long long* N, long long* nnz,
                         long long* band_bytes);

/* b_i = int_Omega f B_i (same Gauss rule as A); b_dev: N doubles (device). */
igafd_status igafd_load_vector(igafd_ctx* ctx, int rhs_kind, double* b_dev);

/* y = A x (banded FP64 product, Sec. 2.1 eq. A); x_dev, y_dev: N doubles, distinct. */
igafd_status igafd_apply_A(igafd_ctx* ctx, const double* x_dev, double* y_dev);

/* s = P^-1 r by fast diagonalisation (Alg. 1 / Alg. 3), mode products in the
 * given precision (FP64, FP32, or BF16 inputs with FP32 accumulation); r and s
 * stay FP64.  With a scaling set (igafd_set_scaling) computes S P^-1 S r.
 * r_dev, s_dev: N doubles; s may not alias r. */
igafd_status igafd_apply_precond(igafd_ctx* ctx, int precision, const double* r_dev, double* s_dev);

/* Diagonal scaling S > 0 for the preconditioner S P^-1 S (copied; NULL disables). */
igafd_status igafd_set_scaling(igafd_ctx* ctx, const double* S_dev);

typedef struct {
  double rtol;                 /* stop when ||r_k||_2 <= rtol ||b||_2 (recursive residual)     */
  int maxit;                   /* maximum CG iterations (0 -> 2000)                            */
  int precision;               /* igafd_precision of the preconditioner apply                  */
  int flexible;                /* 1: Polak-Ribiere beta (required for FP32/BF16 applies)       */
  int use_scaling;             /* 1: S P^-1 S with the scaling set by igafd_set_scaling        */
  int check_every;             /* iterations enqueued between host checks (0 -> 4)             */
  int use_x0;                  /* 1: u_dev holds the initial guess; 0: x0 = 0                  */
  double* history;             /* optional host array of maxit+1 relative residuals            */
} igafd_solve_opts;

typedef struct {
  int iters;                   /* CG iterations (one A product + one apply each)               */
  int restarts;                /* restarts from the true residual                              */
  double relres;               /* final recursive ||r||/||b||                                  */
  double true_relres;          /* ||b - A u||/||b|| evaluated in FP64 at exit                   */
  int status;                  /* igafd_status of the solve                                    */
  double t_solve_ms;           /* device time of the whole solve (events on the ctx stream)    */
} igafd_solve_info;

/* PCG for A u = b preconditioned by P (or S P^-1 S).  b_dev, u_dev: N doubles.
 * Returns IGAFD_OK, IGAFD_NOT_CONVERGED (u holds the last iterate) or an error. */
igafd_status igafd_solve(igafd_ctx* ctx, const double* b_dev, double* u_dev,
                         const igafd_solve_opts* opts, igafd_solve_info* info);

/* Diagonals of A and P (N doubles each, device; either may be NULL). */
igafd_status igafd_diagonals(igafd_ctx* ctx, double* diagA_dev, double* diagP_dev);

/* Host copy of U_d (n_d x n_d row-major, U[i][k] = component i of eigenvector k,
 * U^T M U = I) and of the eigenvalues D_d for direction dir (0-based). */
igafd_status igafd_get_eigen(const igafd_ctx* ctx, int dir, double* U_host, double* lam_host);

/* Host-only: 1D matrices and generalised eigendecomposition for one knot
 * vector (Sec. 3, Sec. 4.1).  M, K, U: n x n row-major, lam: n; n = nknots-p-3
 * is written to *n_out.  Needs no GPU. */
igafd_status igafd_univariate(int degree, int nknots, const double* knots, int quad,
                              double* M, double* K, double* U, double* lam, int* n_out);

void igafd_destroy(igafd_ctx* ctx);
const char* igafd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGAFD_H */

// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "igafd.h"

struct igafd_ctx;

namespace igafd {

constexpr int kMaxDegree = 6;
constexpr int kMaxModes = 16;
constexpr int kBlock = 256;
constexpr long long kTileLdsDefault = 80 * 1024;  // two tiled-product blocks per CU (160 KB LDS)
// Degrees whose setup considers 512-thread tiles (one block per CU, up to
// kTile512Lds of LDS) beside the 256-thread ones, keeping the better score of
// the shape model (whose grid-tail factor favours the smaller tiles on small
// problems): measured faster at p = 3 (128^3: 6x6 lines 578 us against 6x3 of
// 256 threads, 597 us) and p = 5 (96^3: 964 against 1031 us), slower at p = 4
// (112^3: every 512-thread shape 907 us or more against 834)
constexpr bool kTile512Default[kMaxDegree + 1] = {false, false, false, true, false, true, false};
constexpr long long kTile512Lds = 128 * 1024;

void set_error(const std::string& msg);
// block partials (per sum) a context's reductions may write; sizes its buffer
int partial_capacity(const igafd_ctx* c);

#define IGAFD_HIP_CHECK(expr)                                                        \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::igafd::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
      return IGAFD_ERR_HIP;                                                         \
    }                                                                               \
  } while (0)

// Geometry map and coefficient, passed by value to the device.
struct GeomDesc {
  int dim;
  int kind;
  double amp;
  int nmodes;
  double c[kMaxModes][3];
  double m[kMaxModes][3];
  int coef_kind;
  double camp, f1, f2, phi1, phi2;
};

// Host data of one parameter direction.
struct Dir1D {
  int p = 0, q = 0, m = 0, n = 0, nel = 0;
  std::vector<double> knots;
  std::vector<int> elem_first;   // B-spline index (0-based) of the first function nonzero on element e
  std::vector<double> qx, qw;    // [nel][q] Gauss points and weights
  std::vector<double> val, der;  // [nel][q][p+1] values / derivatives of those functions
  std::vector<double> M, K;      // n x n row-major
  std::vector<double> U, lam;    // n x n row-major (U[i][k] = eigenvector k), n eigenvalues
};

// eig = false: element tables and M, K only (no eigendecomposition)
igafd_status build_direction(int p, int q, int nknots, const double* knots, Dir1D* out, bool eig = true);

// Device copies of one direction.
struct DevDir {
  int n = 1, nel = 1, npad = 32;
  int* elem_first = nullptr;
  double* qx = nullptr;
  double* qw = nullptr;
  double* val = nullptr;
  double* der = nullptr;
  double* lam = nullptr;
  double* W64[2] = {nullptr, nullptr};      // [0] = U^T (forward), [1] = U (backward), npad x npad
  float* W32[2] = {nullptr, nullptr};
  uint16_t* Wbf[2] = {nullptr, nullptr};
  double* diagM = nullptr;
  double* diagK = nullptr;
};

// CG scalars kept on the device so that iterations can be enqueued ahead.
struct SolverState {
  double bb, tol2;
  double rho, pq, rr, rz, rzold, alpha, beta, rrtrue;
  int iters, maxit, flag, flexible;
  int hist_cap;  // entries of the device history the reductions may write (0: none)
};
enum { FLAG_RUNNING = 0, FLAG_CONVERGED = 1, FLAG_BREAKDOWN = 2, FLAG_MAXIT = 3 };

}  // namespace igafd

// Three-variable ADI state (adi.hip): parameters and device bands/factors
struct igafd_adi {
  double eps = 0.0, rho = 1.0;
  std::vector<double> omega;
  int J0 = 0;
  // device: per direction the bands of K_d and M_d ([n][2p+1], entry (i, i+k-p))
  // and the lower band Cholesky factors ([n][p+1], entry (i, i-k)) of M_d
  // (slot 0) and of K_d + omega_j M_d (slot j)
  double* bandK[3] = {nullptr, nullptr, nullptr};
  double* bandM[3] = {nullptr, nullptr, nullptr};
  double* fac[3] = {nullptr, nullptr, nullptr};
  double* bandKw1 = nullptr;  // K_1 - omega_j M_1 for every j: [J][n1][2p+1]
  double* work = nullptr;  // rt, v, u, t1, t2: 5 N doubles
};

struct igafd_ctx {
  int dim = 0, p = 0;
  int n[3] = {1, 1, 1};
  long long N = 0;
  hipStream_t stream = nullptr;
  int device = 0;                          // device current at setup
  igafd::GeomDesc geom{};
  igafd::Dir1D dir[3];
  igafd::DevDir ddir[3];
  // symmetric band of A: plane h (0..H-1) holds the entries of offset
  // center+h of the (2p+1)^d stencil, row-indexed; lower entries are read
  // from the mirrored plane at the column row.  Plane h starts at band + h*Ns;
  // row i is at offset halo + i; the halo rows are zero.
  double* band = nullptr;
  int H = 0;
  long long Ns = 0;
  long long halo = 0;
  long long nnz = 0;
  int spmv_rows = 2;                       // rows per thread of the row-parallel A product
  int tile_b2 = 0, tile_b3 = 0;            // 3D tiled A product: lines per tile (0: row-parallel kernel)
  int tile_tb = 256;                       // its threads per block (256: two blocks per CU; 512: one)
  double* ext = nullptr;                   // per-tile extended accumulators of the tiled product
  long long ext_cap = 0;                   // doubles allocated at ext
  int fd_tiles = 2;                        // 16-row tiles per wave in the mode products
  int fd_fused = 1;                        // 3D: three fused passes instead of six products
  int fd_gemm = -1;                        // 2D: tiled products (1), per-strip products (0), by size (-1)
  // L-shaped multi-patch context: the grid is the bounding square's, the
  // quarter i1 >= hole && i2 >= hole is not part of the domain (held at zero);
  // sub[0], sub[1]: preconditioner-only contexts of the two Schwarz subdomains
  int hole = -1;
  igafd_ctx* sub[2] = {nullptr, nullptr};
  igafd_adi* adi = nullptr;                // set: the preconditioner is P_J (three-variable ADI)
  // workspace
  double *r = nullptr, *z = nullptr, *q = nullptr, *zold = nullptr;
  double* pv_pad = nullptr;                // search direction with the band's zero halo
  double* pv = nullptr;                    // = pv_pad + halo
  double* xpad = nullptr;                  // staging buffer with zero halo for caller vectors
  double* fdbuf[2] = {nullptr, nullptr};   // FD intermediates (double or float)
  double* scaling = nullptr;
  bool scaling_set = false;
  double* partial = nullptr;               // per-block partial sums
  int npartial = 0;
  igafd::SolverState* state = nullptr;     // device
  igafd::SolverState* hstate = nullptr;    // pinned host mirror
  int* dflag = nullptr;                    // device error flag (geometry)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  float* feat = nullptr;                   // per-dof features (N x 8) assembled with A, when asked for
  double* hist = nullptr;                  // device residual history of igafd_solve
  int hist_alloc = 0;                      // doubles allocated at hist
  double t_setup_ms = 0.0;                 // host wall time of the setup
  // Prop. 1 bounds of the geometry, computed once on demand
  bool bounds_valid = false;
  double qmin = 0.0, qmax = 0.0, qloc = 0.0;
  // phase timers of a timed solve: events between kernels, the phase each
  // recorded segment belongs to (-1: none), accumulated milliseconds
  bool timing = false;
  std::vector<hipEvent_t> tev;
  std::vector<int> tphase;
  int tused = 0;
  double tacc[3] = {0.0, 0.0, 0.0};
};

namespace igafd {
// assembly.hip
igafd_status assemble_band(igafd_ctx* c, bool with_features);
igafd_status assemble_load(igafd_ctx* c, int rhs_kind, const double* params, int nparams, double* b);
igafd_status diagonals(igafd_ctx* c, double* dA, double* dP);
igafd_status features(igafd_ctx* c, float* feat);
// on-demand features with a caller-given accumulator of 8N doubles (no
// allocation, no synchronisation)
igafd_status features_into(igafd_ctx* c, double* acc, float* feat);
igafd_status scaling_targets(igafd_ctx* c, float* t);
igafd_status diag_ratio_scaling(igafd_ctx* c, double* S);
igafd_status spectral_bounds(igafd_ctx* c, double* qmin, double* qmax, double* qloc);
// spmv.hip
igafd_status spmv(igafd_ctx* c, const double* xpad, double* y, double* partial, const int* flag);
igafd_status spmv_unpadded(igafd_ctx* c, const double* x, double* y, double* partial, const int* flag);
int spmv_blocks(const igafd_ctx* c);
bool spmv_pick_tile(const igafd_ctx* c, long long lds_limit, int* b2, int* b3, int tb = 256,
                    double* score = nullptr);
igafd_status spmv_set_tile(igafd_ctx* c, int b2, int b3, int tb = 256);
igafd_status mask_hole(igafd_ctx* c, double* y);
// fd.hip
igafd_status fd_apply(igafd_ctx* c, int prec, const double* r, double* s, const double* scaling,
                      double* partial_rz, const int* flag);
int fd_dot_blocks(const igafd_ctx* c, int prec);
int fd_dot_blocks_max(const igafd_ctx* c);
int fd_npad(int n);
bool fd_fused_ok(const igafd_ctx* c);
// gemm.hip: 2D apply by tiled products (prec FP64 or FP32); r and s may be
// sub-blocks of wider grids (row strides ldr, lds; 0 = n1)
igafd_status fd_apply_gemm2d(igafd_ctx* c, int prec, const double* r, double* s, const double* scaling,
                             double* partial_rz, const int* flag, int ldr, int lds);
igafd_status fd_apply_gemm3d(igafd_ctx* c, int prec, const double* r, double* s, const double* scaling,
                             double* partial, const int* flag);
int fd_gemm_blocks(const igafd_ctx* c);  // blocks (= (r, s) partials) of the last product
// adi.hip
constexpr int kAdiGeometric = 0, kAdiGreedy = 1;  // parameter rules of the three-variable ADI
igafd_status adi_setup(igafd_ctx* c, double eps, int rule);
igafd_status adi_apply(igafd_ctx* c, int prec, const double* r, double* s, const double* scaling,
                       double* partial_rz, const int* flag);
void adi_free(igafd_ctx* c);
// two independent 2D applies (no scaling, no partials) whose passes share launches
igafd_status fd_apply_gemm2d_pair(int prec, igafd_ctx* c0, const double* r0, int ldr0, double* s0, int lds0,
                                  igafd_ctx* c1, const double* r1, int ldr1, double* s1, int lds1, const int* flag);

// ---- grouped launches: one launch runs the same step for several problems ----
// Block b of a grouped launch works on job j with start[j] <= b < start[j+1]
// (start ascending, start[0] = 0).
__device__ inline int group_job(const int* __restrict__ start, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Job tables of grouped launches: appended on the host, then copied to the
// device once, before (and outside any capture of) the launches that read
// them.  A step is one enqueued launch that reads its tables at `dev`.
struct GroupArena {
  std::vector<unsigned char> host;
  unsigned char* dev = nullptr;
  size_t cap = 0;
  size_t push(const void* p, size_t bytes);  // offset (a multiple of 64) of the appended bytes
  igafd_status upload(hipStream_t st);        // (re)allocates when too small; waits for the copy
  void release();
  template <class T>
  const T* at(size_t off) const {
    return reinterpret_cast<const T*>(dev + off);
  }
};
using GroupStep = std::function<igafd_status(hipStream_t)>;

// Per problem i of a grouped A product (3D problems): y_i = A_i x_i, x_i in the
// zero-halo layout, block partials of (x_i, y_i) into partial_i (may be null),
// each problem on the kernel and shape it has selected; stop_flags: a problem
// whose CG has stopped is skipped (its stop flag is set).
igafd_status spmv_grouped(GroupArena& a, std::vector<GroupStep>& steps, const std::vector<igafd_ctx*>& cs,
                          const std::vector<const double*>& x, const std::vector<double*>& y,
                          const std::vector<double*>& partial, bool stop_flags = true);
bool spmv_groupable(const igafd_ctx* c);
// Per problem i of a grouped FD apply (3D fused passes): s_i = M_i r_i with
// M_i = P^-1 or S_i P^-1 S_i, block partials of (r_i, s_i) into partial_i.
igafd_status fd_grouped(GroupArena& a, std::vector<GroupStep>& steps, const std::vector<igafd_ctx*>& cs, int prec,
                        const std::vector<const double*>& r, const std::vector<double*>& s,
                        const std::vector<const double*>& S, const std::vector<double*>& partial);
bool fd_groupable(const igafd_ctx* c, int prec);
}  // namespace igafd

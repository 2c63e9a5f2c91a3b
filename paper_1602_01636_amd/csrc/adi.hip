// Three-variable ADI of Douglas as an inexact application of P^-1
// (Sec. 5.2 eq. ADI3D, eq. ADI3D2, Alg. "3D ADI method"; used inside CG as
// the preconditioner P_J of Sec. 4.2 Thm. ADIprec, which keeps it SPD).
//
// Parameters: [a, b] spans the eigenvalues of M_d^-1 K_d over the three
// directions; for a count J the parameters are geometric between a and b,
// omega_j = a (b/a)^((j-1)/(J-1)); J is the smallest count whose error
// operator has ||T_J|| <= eps, at most J0 = ceil(1.16 ln(b/a) ln(1/eps))
// (eq. ADI3Diter).  T_J is diagonal in the eigenvector basis of the three
// pencils with entries prod_j g_j(l1, l2, l3),
//   g_j = 1 - 2 omega_j^2 (l1 + l2 + l3) / ((omega_j + l1)(omega_j + l2)(omega_j + l3)),
// so ||T_J|| is evaluated exactly as the largest |prod_j g_j| over the
// triples of eigenvalues (host, at setup).
//
// Device: every step of the algorithm is a banded product or a banded
// Cholesky solve along one direction of the grid, done by one thread per grid
// line walking the line with a sliding window of 2p+1 (product) or p
// (solve) values in registers.  Lines of directions 2 and 3 are taken by
// consecutive threads at consecutive i1, so their loads are coalesced.
#include <algorithm>
#include <cmath>
#include <memory>
#include <thread>
#include <vector>

#include "internal.h"
#include "reduce.h"

namespace igafd {
namespace {

// Lines of direction DIR: count, start offset and stride in the (n3, n2, n1) grid.
template <int DIR>
__device__ inline bool line_of(long long l, int n1, int n2, int n3, long long* base, long long* stride, int* len) {
  if (DIR == 0) {
    if (l >= (long long)n2 * n3) return false;
    *base = l * n1;
    *stride = 1;
    *len = n1;
  } else if (DIR == 1) {
    if (l >= (long long)n1 * n3) return false;
    const long long i3 = l / n1, i1 = l % n1;
    *base = i3 * n1 * n2 + i1;
    *stride = n1;
    *len = n2;
  } else {
    if (l >= (long long)n1 * n2) return false;
    *base = l;
    *stride = (long long)n1 * n2;
    *len = n3;
  }
  return true;
}

// y = cz z + (ca A + cb B) (x + c2 x2) along direction DIR; A, B bands [n][2P+1].
// z may be y (each thread reads z_i before writing y_i); x, x2 may not be y.
template <int P, int DIR>
__global__ __launch_bounds__(kBlock) void k_line_apply(const double* __restrict__ A, const double* __restrict__ B,
                                                      double ca, double cb, const double* __restrict__ x,
                                                      const double* __restrict__ x2, double c2, const double* z,
                                                      double cz, double* y, int n1, int n2, int n3,
                                                      const int* __restrict__ flag) {
  if (flag && *flag) return;
  long long base, stride;
  int len;
  if (!line_of<DIR>((long long)blockIdx.x * kBlock + threadIdx.x, n1, n2, n3, &base, &stride, &len)) return;
  constexpr int W = 2 * P + 1;
  double win[W];  // win[k] = w_{i + k - P}, w = x + c2 x2, zero outside the line
  auto w_at = [&](int j) -> double {
    if (j < 0 || j >= len) return 0.0;
    const long long o = base + (long long)j * stride;
    return x2 ? x[o] + c2 * x2[o] : x[o];
  };
#pragma unroll
  for (int k = 0; k < W; ++k) win[k] = w_at(k - P);
  for (int i = 0; i < len; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      double a = 0.0;
      if (A) a += ca * A[(long long)i * W + k];
      if (B) a += cb * B[(long long)i * W + k];
      acc = fma(a, win[k], acc);
    }
    const long long o = base + (long long)i * stride;
    y[o] = (z ? cz * z[o] : 0.0) + acc;
#pragma unroll
    for (int k = 0; k + 1 < W; ++k) win[k] = win[k + 1];
    win[W - 1] = w_at(i + P + 1);
  }
}

// y = (L L^T)^-1 (alpha x) along direction DIR; L lower band [n][P+1] with
// L[i][k] = L_{i, i-k}.  In place (x == y) allowed.
template <int P, int DIR>
__global__ __launch_bounds__(kBlock) void k_line_solve(const double* __restrict__ L, double alpha, const double* x,
                                                      double* y, int n1, int n2, int n3,
                                                      const int* __restrict__ flag) {
  if (flag && *flag) return;
  long long base, stride;
  int len;
  if (!line_of<DIR>((long long)blockIdx.x * kBlock + threadIdx.x, n1, n2, n3, &base, &stride, &len)) return;
  constexpr int W = P + 1;
  double win[P > 0 ? P : 1];  // the last P values (most recent last)
#pragma unroll
  for (int k = 0; k < P; ++k) win[k] = 0.0;
  for (int i = 0; i < len; ++i) {  // forward: L t = alpha x
    const long long o = base + (long long)i * stride;
    double t = alpha * x[o];
#pragma unroll
    for (int k = 1; k <= P; ++k) t -= L[(long long)i * W + k] * win[P - k];
    t /= L[(long long)i * W];
    y[o] = t;
#pragma unroll
    for (int k = 0; k + 1 < P; ++k) win[k] = win[k + 1];
    if (P > 0) win[P - 1] = t;
  }
#pragma unroll
  for (int k = 0; k < P; ++k) win[k] = 0.0;
  for (int i = len - 1; i >= 0; --i) {  // backward: L^T z = t
    const long long o = base + (long long)i * stride;
    double zv = y[o];
#pragma unroll
    for (int k = 1; k <= P; ++k)
      if (i + k < len) zv -= L[(long long)(i + k) * W + k] * win[P - k];
    zv /= L[(long long)i * W];
    y[o] = zv;
#pragma unroll
    for (int k = 0; k + 1 < P; ++k) win[k] = win[k + 1];
    if (P > 0) win[P - 1] = zv;
  }
}

__global__ void k_adi_fill0(double* __restrict__ a, double* __restrict__ b, long long N, const int* __restrict__ flag) {
  if (flag && *flag) return;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < N) {
    a[i] = 0.0;
    b[i] = 0.0;
  }
}

// v = v + omega (s2 - s); with partial: block sums of r . s
__global__ __launch_bounds__(kBlock) void k_adi_vupdate(double* __restrict__ v, const double* __restrict__ s2,
                                                       const double* __restrict__ s, double omega, long long N,
                                                       const double* __restrict__ r, double* __restrict__ partial,
                                                       const int* __restrict__ flag) {
  if (flag && *flag) return;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (i < N) {
    v[i] += omega * (s2[i] - s[i]);
    if (partial) dot = r[i] * s[i];
  }
  if (partial) {
    const double sum = block_sum(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
  }
}

// Band of a dense symmetric n x n matrix: [n][2p+1], entry (i, i+k-p).
std::vector<double> band_of(const std::vector<double>& X, int n, int p) {
  const int W = 2 * p + 1;
  std::vector<double> b((size_t)n * W, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < W; ++k) {
      const int j = i + k - p;
      if (j >= 0 && j < n) b[(size_t)i * W + k] = X[(size_t)i * n + j];
    }
  return b;
}

// Lower band Cholesky of K + w M (both [n][2p+1] bands): [n][p+1], entry (i, i-k).
bool band_cholesky(const std::vector<double>& K, const std::vector<double>& M, double cK, double w, int n, int p,
                   double* L) {
  const int W = 2 * p + 1, WL = p + 1;
  auto a = [&](int i, int j) -> double {  // entry (i, j), |i - j| <= p
    const int k = j - i + p;
    return cK * K[(size_t)i * W + k] + w * M[(size_t)i * W + k];
  };
  auto l = [&](int i, int j) -> double& { return L[(size_t)i * WL + (i - j)]; };
  for (int j = 0; j < n; ++j) {
    double s = a(j, j);
    for (int k = std::max(0, j - p); k < j; ++k) s -= l(j, k) * l(j, k);
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    l(j, j) = ljj;
    for (int i = j + 1; i <= std::min(n - 1, j + p); ++i) {
      double v = a(i, j);
      for (int k = std::max(0, i - p); k < j; ++k) v -= l(i, k) * l(j, k);
      l(i, j) = v / ljj;
    }
  }
  return true;
}

// ||T_J|| for the parameters w: the largest |prod_j g_j| over all triples of
// eigenvalues (host threads over the direction-3 eigenvalues).
double error_norm(const std::vector<double>& w, const std::vector<double>& l1, const std::vector<double>& l2,
                  const std::vector<double>& l3) {
  const unsigned hw = std::thread::hardware_concurrency();
  const int T = (int)std::max(1u, std::min(16u, hw));
  std::vector<double> part(T, 0.0);
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t]() {
      double m = 0.0;
      for (size_t c = t; c < l3.size(); c += T)
        for (double b2 : l2)
          for (double a1 : l1) {
            const double s = a1 + b2 + l3[c];
            double g = 1.0;
            for (double om : w) g *= 1.0 - 2.0 * om * om * s / ((om + a1) * (om + b2) * (om + l3[c]));
            m = std::max(m, std::fabs(g));
          }
      part[t] = m;
    });
  for (auto& x : th) x.join();
  return *std::max_element(part.begin(), part.end());
}

template <int P, int DIR>
igafd_status line_apply(igafd_ctx* c, const double* A, const double* B, double ca, double cb, const double* x,
                        const double* x2, double c2, const double* z, double cz, double* y, const int* flag) {
  const long long lines = DIR == 0 ? (long long)c->n[1] * c->n[2] : DIR == 1 ? (long long)c->n[0] * c->n[2]
                                                                            : (long long)c->n[0] * c->n[1];
  hipLaunchKernelGGL((k_line_apply<P, DIR>), dim3((unsigned)((lines + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, A, B, ca, cb, x, x2, c2, z, cz, y, c->n[0], c->n[1], c->n[2], flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

template <int P, int DIR>
igafd_status line_solve(igafd_ctx* c, const double* L, double alpha, const double* x, double* y, const int* flag) {
  const long long lines = DIR == 0 ? (long long)c->n[1] * c->n[2] : DIR == 1 ? (long long)c->n[0] * c->n[2]
                                                                            : (long long)c->n[0] * c->n[1];
  hipLaunchKernelGGL((k_line_solve<P, DIR>), dim3((unsigned)((lines + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, L, alpha, x, y, c->n[0], c->n[1], c->n[2], flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

// s = P_J^-1 r by the steps of Alg. "3D ADI method" (s_0 = v_0 = 0)
template <int P>
igafd_status apply_p(igafd_ctx* c, const double* r, double* s, double* partial, const int* flag) {
  igafd_adi* a = c->adi;
  const long long N = c->N;
  double* rt = a->work;
  double* v = rt + N;
  double* u = v + N;
  double* t1 = u + N;
  double* t2 = t1 + N;
  const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2];
  auto facM = [&](int d) { return a->fac[d]; };
  auto facW = [&](int d, int j) { return a->fac[d] + (size_t)(j + 1) * (d == 0 ? n1 : d == 1 ? n2 : n3) * (P + 1); };
  igafd_status st;
#define IGAFD_T(x)               \
  if ((st = (x)) != IGAFD_OK) \
    return st;
  // r~ = 2 (I x M2 x M3)^-1 r
  IGAFD_T((line_solve<P, 1>(c, facM(1), 2.0, r, t1, flag)));
  IGAFD_T((line_solve<P, 2>(c, facM(2), 1.0, t1, rt, flag)));
  const unsigned vb = (unsigned)((N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adi_fill0, dim3(vb), dim3(kBlock), 0, c->stream, s, v, N, flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  const int J = (int)a->omega.size();
  for (int j = 0; j < J; ++j) {
    const double w = a->omega[j];
    // u_j = (I x M2^-1 K2 x I) s_{j-1}
    IGAFD_T((line_apply<P, 1>(c, a->bandK[1], nullptr, 1.0, 0.0, s, nullptr, 0.0, nullptr, 0.0, t1, flag)));
    IGAFD_T((line_solve<P, 1>(c, facM(1), 1.0, t1, u, flag)));
    // r*_j = r~ - ((K1 - w M1) x I x I) s_{j-1} - (2 M1 x I x I)(u_j + v_j); s*_j
    IGAFD_T((line_apply<P, 0>(c, a->bandK[0], a->bandM[0], -1.0, w, s, nullptr, 0.0, rt, 1.0, t1, flag)));
    IGAFD_T((line_apply<P, 0>(c, nullptr, a->bandM[0], 0.0, -2.0, u, v, 1.0, t1, 1.0, t1, flag)));
    IGAFD_T((line_solve<P, 0>(c, facW(0, j), 1.0, t1, t1, flag)));
    // r**_j = (I x M2 x I)(u_j + w s*_j); s**_j
    IGAFD_T((line_apply<P, 1>(c, nullptr, a->bandM[1], 0.0, 1.0, u, t1, w, nullptr, 0.0, t2, flag)));
    IGAFD_T((line_solve<P, 1>(c, facW(1, j), 1.0, t2, t2, flag)));
    // b_j = v_j + w s**_j; r_j = (I x I x M3) b_j; s_j; v_{j+1} = b_j - w s_j
    IGAFD_T((line_apply<P, 2>(c, nullptr, a->bandM[2], 0.0, 1.0, v, t2, w, nullptr, 0.0, t1, flag)));
    IGAFD_T((line_solve<P, 2>(c, facW(2, j), 1.0, t1, s, flag)));
    hipLaunchKernelGGL(k_adi_vupdate, dim3(vb), dim3(kBlock), 0, c->stream, v, t2, s, w, N, r,
                       j + 1 == J ? partial : nullptr, flag);
    IGAFD_HIP_CHECK(hipGetLastError());
  }
#undef IGAFD_T
  if (J == 0 && partial) {
    set_error("internal: ADI without steps");
    return IGAFD_ERR_ARG;
  }
  (void)n3;
  return IGAFD_OK;
}

}  // namespace

void adi_free(igafd_ctx* c) {
  igafd_adi* a = c->adi;
  if (!a) return;
  for (int d = 0; d < 3; ++d) {
    if (a->bandK[d]) (void)hipFree(a->bandK[d]);
    if (a->bandM[d]) (void)hipFree(a->bandM[d]);
    if (a->fac[d]) (void)hipFree(a->fac[d]);
  }
  if (a->work) (void)hipFree(a->work);
  delete a;
  c->adi = nullptr;
}

igafd_status adi_setup(igafd_ctx* c, double eps) {
  if (c->dim != 3) {
    set_error("the three-variable ADI is for 3D problems");
    return IGAFD_ERR_ARG;
  }
  if (!(eps > 0.0 && eps < 1.0)) {
    set_error("ADI tolerance must lie in (0, 1)");
    return IGAFD_ERR_ARG;
  }
  for (int d = 0; d < 3; ++d)
    if (c->dir[d].lam.empty()) {
      set_error("this context holds no univariate eigenvalues");
      return IGAFD_ERR_ARG;
    }
  const int p = c->p;
  double a = c->dir[0].lam.front(), b = c->dir[0].lam.back();
  for (int d = 0; d < 3; ++d) {
    a = std::min(a, *std::min_element(c->dir[d].lam.begin(), c->dir[d].lam.end()));
    b = std::max(b, *std::max_element(c->dir[d].lam.begin(), c->dir[d].lam.end()));
  }
  const int J0 = std::max(1, (int)std::ceil(1.16 * std::log(b / a) * std::log(1.0 / eps)));
  std::vector<double> w;
  double rho = 1.0;
  for (int J = 1; J <= J0; ++J) {
    w.assign(J, 0.0);
    for (int j = 0; j < J; ++j) w[j] = J == 1 ? std::sqrt(a * b) : a * std::pow(b / a, (double)j / (J - 1));
    rho = error_norm(w, c->dir[0].lam, c->dir[1].lam, c->dir[2].lam);
    if (rho <= eps) break;
  }
  std::unique_ptr<igafd_adi> st(new igafd_adi());
  st->eps = eps;
  st->rho = rho;
  st->omega = w;
  st->J0 = J0;
  const int W = 2 * p + 1, WL = p + 1, J = (int)w.size();
  // device buffers are owned by st until it is installed: free them on failure
  struct Guard {
    igafd_adi* a;
    ~Guard() {
      if (!a) return;
      for (int d = 0; d < 3; ++d) {
        if (a->bandK[d]) (void)hipFree(a->bandK[d]);
        if (a->bandM[d]) (void)hipFree(a->bandM[d]);
        if (a->fac[d]) (void)hipFree(a->fac[d]);
      }
      if (a->work) (void)hipFree(a->work);
    }
  } guard{st.get()};
  for (int d = 0; d < 3; ++d) {
    const int n = c->dir[d].n;
    const std::vector<double> bK = band_of(c->dir[d].K, n, p), bM = band_of(c->dir[d].M, n, p);
    std::vector<double> fac((size_t)(J + 1) * n * WL, 0.0);
    bool ok = band_cholesky(bK, bM, 0.0, 1.0, n, p, fac.data());
    for (int j = 0; j < J && ok; ++j) ok = band_cholesky(bK, bM, 1.0, w[j], n, p, fac.data() + (size_t)(j + 1) * n * WL);
    if (!ok) {
      set_error("band Cholesky of K_d + omega M_d failed");
      return IGAFD_ERR_NOT_SPD;
    }
    IGAFD_HIP_CHECK(hipMalloc((void**)&st->bandK[d], sizeof(double) * bK.size()));
    IGAFD_HIP_CHECK(hipMalloc((void**)&st->bandM[d], sizeof(double) * bM.size()));
    IGAFD_HIP_CHECK(hipMalloc((void**)&st->fac[d], sizeof(double) * fac.size()));
    IGAFD_HIP_CHECK(hipMemcpy(st->bandK[d], bK.data(), sizeof(double) * bK.size(), hipMemcpyHostToDevice));
    IGAFD_HIP_CHECK(hipMemcpy(st->bandM[d], bM.data(), sizeof(double) * bM.size(), hipMemcpyHostToDevice));
    IGAFD_HIP_CHECK(hipMemcpy(st->fac[d], fac.data(), sizeof(double) * fac.size(), hipMemcpyHostToDevice));
  }
  IGAFD_HIP_CHECK(hipMalloc((void**)&st->work, sizeof(double) * 5 * (size_t)c->N));
  (void)W;
  adi_free(c);
  guard.a = nullptr;
  c->adi = st.release();
  return IGAFD_OK;
}

igafd_status adi_apply(igafd_ctx* c, int prec, const double* r, double* s, const double* S, double* partial,
                       const int* flag) {
  if (prec != IGAFD_FP64) {
    set_error("the ADI preconditioner runs in FP64 only");
    return IGAFD_ERR_ARG;
  }
  if (S) {
    set_error("the scaled preconditioner is not defined with ADI");
    return IGAFD_ERR_ARG;
  }
  if (partial && (long long)((c->N + kBlock - 1) / kBlock) > c->npartial) {
    set_error("internal: ADI grid larger than the partial-sum buffer");
    return IGAFD_ERR_ARG;
  }
  switch (c->p) {
#define IGAFD_P(P) \
  case P:          \
    return apply_p<P>(c, r, s, partial, flag);
    IGAFD_P(1) IGAFD_P(2) IGAFD_P(3) IGAFD_P(4) IGAFD_P(5) IGAFD_P(6)
#undef IGAFD_P
    default:
      set_error("unsupported degree");
      return IGAFD_ERR_ARG;
  }
}

}  // namespace igafd

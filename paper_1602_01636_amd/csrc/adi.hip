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
// Device: every step of the algorithm is a banded product along one direction
// of the grid (one thread per grid point) or a banded Cholesky solve along one
// direction (one thread per grid line, walking it in chunks: the next chunk's
// values load while the recurrence runs on the current one in registers with
// a window of p values).  Lines of directions 2 and 3 are taken by
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

constexpr int kLineBlock = 64;  // threads per block of the line solves (few lines: spread over CUs)
constexpr int kChunk = 16;      // line values loaded together in the solves

// y = cz z + ca B (x + c2 x2) along direction DIR, B a band [n][2P+1]: one
// thread per grid point (the neighbours along DIR are other threads' points,
// read through the caches).  z may be y; x and x2 may not.
template <int P, int DIR>
__global__ __launch_bounds__(kBlock) void k_band_apply(const double* __restrict__ Bd, double ca,
                                                      const double* __restrict__ x, const double* __restrict__ x2,
                                                      double c2, const double* z, double cz, double* y, int n1, int n2,
                                                      int n3, const int* __restrict__ flag) {
  if (flag && *flag) return;
  const long long N = (long long)n1 * n2 * n3;
  const long long o = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (o >= N) return;
  int i, len;
  long long stride;
  if (DIR == 0) {
    i = (int)(o % n1);
    len = n1;
    stride = 1;
  } else if (DIR == 1) {
    i = (int)((o / n1) % n2);
    len = n2;
    stride = n1;
  } else {
    i = (int)(o / ((long long)n1 * n2));
    len = n3;
    stride = (long long)n1 * n2;
  }
  constexpr int W = 2 * P + 1;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int j = i + k - P;
    if (j >= 0 && j < len) {
      const long long q = o + (long long)(k - P) * stride;
      const double w = x2 ? x[q] + c2 * x2[q] : x[q];
      acc = fma(Bd[(long long)i * W + k], w, acc);
    }
  }
  y[o] = (z ? cz * z[o] : 0.0) + ca * acc;
}

// y = (L L^T)^-1 (alpha x) along direction DIR; L lower band [len][P+1] with
// L[i][k] = L_{i, i-k} for k >= 1 and L[i][0] = 1 / L_{i,i}.  One thread per
// line.  The factor (the same for every line) is staged in LDS first, so the
// recurrence reads its coefficients from LDS, not memory; the line is read in
// chunks of kChunk values, the next chunk's loads issued before the current
// chunk's recurrence.  len is the (uniform) line length.  In place (x == y)
// allowed: a chunk is loaded before any of its values is written, and writes
// never reach a chunk that is still to be loaded.
template <int P, int DIR>
__global__ __launch_bounds__(kLineBlock) void k_line_solve(const double* __restrict__ L, double alpha, const double* x,
                                                          double* y, int n1, int n2, int n3, int len,
                                                          const int* __restrict__ flag) {
  if (flag && *flag) return;
  extern __shared__ double Ls[];  // [len][P+1]
  constexpr int W = P + 1;
  for (int e = threadIdx.x; e < len * W; e += kLineBlock) Ls[e] = L[e];
  __syncthreads();
  long long base, stride;
  int len_t;
  if (!line_of<DIR>((long long)blockIdx.x * kLineBlock + threadIdx.x, n1, n2, n3, &base, &stride, &len_t)) return;
  const int nch = (len + kChunk - 1) / kChunk;
  auto ld = [&](const double* src, int i0, double (&b)[kChunk]) {
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int i = i0 + c < len ? i0 + c : len - 1;
      b[c] = src[base + (long long)i * stride];
    }
  };
  auto st = [&](int i0, const double (&b)[kChunk]) {
#pragma unroll
    for (int c = 0; c < kChunk; ++c)
      if (i0 + c < len) y[base + (long long)(i0 + c) * stride] = b[c];
  };
  double win[P > 0 ? P : 1];  // the last P values (most recent last)
  double cur[kChunk], nxt[kChunk];
#pragma unroll
  for (int k = 0; k < P; ++k) win[k] = 0.0;
  ld(x, 0, cur);
  for (int q = 0; q < nch; ++q) {  // forward: L t = alpha x
    const int i0 = q * kChunk;
    if (q + 1 < nch) ld(x, i0 + kChunk, nxt);
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int i = i0 + c;
      if (i < len) {
        double t = alpha * cur[c];
#pragma unroll
        for (int k = 1; k <= P; ++k) t -= Ls[i * W + k] * win[P - k];
        t *= Ls[i * W];
        cur[c] = t;
#pragma unroll
        for (int k = 0; k + 1 < P; ++k) win[k] = win[k + 1];
        if (P > 0) win[P - 1] = t;
      }
    }
    st(i0, cur);
#pragma unroll
    for (int c = 0; c < kChunk; ++c) cur[c] = nxt[c];
  }
#pragma unroll
  for (int k = 0; k < P; ++k) win[k] = 0.0;
  ld(y, (nch - 1) * kChunk, cur);
  for (int q = nch - 1; q >= 0; --q) {  // backward: L^T z = t, chunks from the end
    const int i0 = q * kChunk;
    if (q > 0) ld(y, i0 - kChunk, nxt);
#pragma unroll
    for (int c = kChunk - 1; c >= 0; --c) {
      const int i = i0 + c;
      if (i < len) {
        double zv = cur[c];
#pragma unroll
        for (int k = 1; k <= P; ++k)
          if (i + k < len) zv -= Ls[(i + k) * W + k] * win[P - k];
        zv *= Ls[i * W];
        cur[c] = zv;
#pragma unroll
        for (int k = 0; k + 1 < P; ++k) win[k] = win[k + 1];
        if (P > 0) win[P - 1] = zv;
      }
    }
    st(i0, cur);
#pragma unroll
    for (int c = 0; c < kChunk; ++c) cur[c] = nxt[c];
  }
}

// The same solve with the block's 64 lines staged in LDS as a [len][65] tile
// (element i of the block's line t at i * 65 + t; the odd row length keeps
// the cooperative reads of direction 1 off a single bank): one read of the
// lines, both sweeps on the thread's LDS column, one write; lines of up to
// kLdsLineMax points.
constexpr int kLdsLineMax = 256;
constexpr int kTS = kLineBlock + 1;  // row stride of the LDS tile

template <int P, int DIR>
__global__ __launch_bounds__(kLineBlock) void k_line_solve_lds(const double* __restrict__ L, double alpha,
                                                              const double* x, double* y, int n1, int n2, int n3,
                                                              int len, const int* __restrict__ flag) {
  if (flag && *flag) return;
  extern __shared__ double sm[];
  constexpr int W = P + 1;
  double* Ls = sm;                      // [len][P+1]
  double* T = sm + ((len * W + 1) & ~1);  // [len][kTS]
  for (int e = threadIdx.x; e < len * W; e += kLineBlock) Ls[e] = L[e];
  const long long l0 = (long long)blockIdx.x * kLineBlock;
  const long long nlines = DIR == 0 ? (long long)n2 * n3 : DIR == 1 ? (long long)n1 * n3 : (long long)n1 * n2;
  const int nl = (int)(nlines - l0 < kLineBlock ? nlines - l0 : kLineBlock);
  // this thread's line (directions 2 and 3: consecutive threads at consecutive i1)
  long long base = 0, stride = 0;
  int len_t = 0;
  const bool mine = line_of<DIR>(l0 + threadIdx.x, n1, n2, n3, &base, &stride, &len_t);
  if (DIR == 0) {  // the block's lines are contiguous: read them as one run, e = t * len + i
    const long long b0 = l0 * n1;
    int t = (int)threadIdx.x / len, i = (int)threadIdx.x % len;
    for (int e = threadIdx.x; e < nl * len; e += kLineBlock) {
      T[i * kTS + t] = x[b0 + e];
      i += kLineBlock;
      while (i >= len) {
        i -= len;
        ++t;
      }
    }
  } else if (mine) {
    for (int i = 0; i < len; ++i) T[i * kTS + threadIdx.x] = x[base + (long long)i * stride];
  }
  __syncthreads();
  if ((int)threadIdx.x < nl) {
    // sweeps in chunks of kChunk: the chunk's values and coefficients are read
    // from LDS into registers before any of the chunk is written back (the
    // compiler cannot move a read of the shared array above a write to it)
    double* col = T + threadIdx.x;  // element i at col[i * kTS]
    double win[P > 0 ? P : 1];
#pragma unroll
    for (int k = 0; k < P; ++k) win[k] = 0.0;
    for (int i0 = 0; i0 < len; i0 += kChunk) {  // forward: L t = alpha x
      double v[kChunk], cf[kChunk][P + 1];
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        const int i = i0 + c < len ? i0 + c : len - 1;
        v[c] = col[i * kTS];
#pragma unroll
        for (int k = 0; k <= P; ++k) cf[c][k] = Ls[i * W + k];
      }
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        if (i0 + c < len) {
          double t = alpha * v[c];
#pragma unroll
          for (int k = 1; k <= P; ++k) t -= cf[c][k] * win[P - k];
          t *= cf[c][0];
          v[c] = t;
#pragma unroll
          for (int k = 0; k + 1 < P; ++k) win[k] = win[k + 1];
          if (P > 0) win[P - 1] = t;
        }
      }
#pragma unroll
      for (int c = 0; c < kChunk; ++c)
        if (i0 + c < len) col[(i0 + c) * kTS] = v[c];
    }
#pragma unroll
    for (int k = 0; k < P; ++k) win[k] = 0.0;
    const int nch = (len + kChunk - 1) / kChunk;
    for (int q = nch - 1; q >= 0; --q) {  // backward: L^T z = t (entries past the end read as 0)
      const int i0 = q * kChunk;
      double v[kChunk], d0[kChunk], cf[kChunk][P + 1];  // cf[c][k] = L_{i+k, i} = Ls[(i+k)][k]
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        const int i = i0 + c < len ? i0 + c : len - 1;
        v[c] = col[i * kTS];
        d0[c] = Ls[i * W];
#pragma unroll
        for (int k = 1; k <= P; ++k) cf[c][k] = i + k < len ? Ls[(i + k) * W + k] : 0.0;
      }
#pragma unroll
      for (int c = kChunk - 1; c >= 0; --c) {
        if (i0 + c < len) {
          double zv = v[c];
#pragma unroll
          for (int k = 1; k <= P; ++k) zv -= cf[c][k] * win[P - k];
          zv *= d0[c];
          v[c] = zv;
#pragma unroll
          for (int k = 0; k + 1 < P; ++k) win[k] = win[k + 1];
          if (P > 0) win[P - 1] = zv;
        }
      }
#pragma unroll
      for (int c = 0; c < kChunk; ++c)
        if (i0 + c < len) col[(i0 + c) * kTS] = v[c];
    }
  }
  __syncthreads();
  if (DIR == 0) {
    const long long b0 = l0 * n1;
    int t = (int)threadIdx.x / len, i = (int)threadIdx.x % len;
    for (int e = threadIdx.x; e < nl * len; e += kLineBlock) {
      y[b0 + e] = T[i * kTS + t];
      i += kLineBlock;
      while (i >= len) {
        i -= len;
        ++t;
      }
    }
  } else if (mine) {
    for (int i = 0; i < len; ++i) y[base + (long long)i * stride] = T[i * kTS + threadIdx.x];
  }
}

template <int P, int DIR>
size_t lds_solve_bytes(int len) {
  return sizeof(double) * ((size_t)((len * (P + 1) + 1) & ~1) + (size_t)len * kTS);
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

// Lower band Cholesky of cK K + w M (both [n][2p+1] bands): [n][p+1], entry (i, i-k),
// the diagonal stored as its reciprocal.
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
  for (int j = 0; j < n; ++j) l(j, j) = 1.0 / l(j, j);  // the solves multiply by the reciprocal
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
igafd_status band_apply(igafd_ctx* c, const double* Bd, double ca, const double* x, const double* x2, double c2,
                        const double* z, double cz, double* y, const int* flag) {
  hipLaunchKernelGGL((k_band_apply<P, DIR>), dim3((unsigned)((c->N + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream,
                     Bd, ca, x, x2, c2, z, cz, y, c->n[0], c->n[1], c->n[2], flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

template <int P, int DIR>
igafd_status line_solve(igafd_ctx* c, const double* L, double alpha, const double* x, double* y, const int* flag) {
  const long long lines = DIR == 0 ? (long long)c->n[1] * c->n[2] : DIR == 1 ? (long long)c->n[0] * c->n[2]
                                                                            : (long long)c->n[0] * c->n[1];
  const int len = c->n[DIR];
  const dim3 grid((unsigned)((lines + kLineBlock - 1) / kLineBlock));
  if (len <= kLdsLineMax) {  // attribute for > 64 KB set at setup (adi_lds_attr)
    const size_t lds = lds_solve_bytes<P, DIR>(len);
    hipLaunchKernelGGL((k_line_solve_lds<P, DIR>), grid, dim3(kLineBlock), lds, c->stream, L, alpha, x, y, c->n[0],
                       c->n[1], c->n[2], len, flag);
  } else {
    const size_t lds = sizeof(double) * (size_t)len * (P + 1);
    if (lds > 64 * 1024) {
      set_error("ADI line too long for the LDS-staged factor");
      return IGAFD_ERR_ARG;
    }
    hipLaunchKernelGGL((k_line_solve<P, DIR>), grid, dim3(kLineBlock), lds, c->stream, L, alpha, x, y, c->n[0], c->n[1],
                       c->n[2], len, flag);
  }
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

// Dynamic LDS above 64 KB needs the kernel attribute; set once per problem at
// setup (never inside a launch sequence that may be captured).
template <int P>
igafd_status lds_attr(const igafd_ctx* c) {
  const void* fn[3] = {(const void*)&k_line_solve_lds<P, 0>, (const void*)&k_line_solve_lds<P, 1>,
                       (const void*)&k_line_solve_lds<P, 2>};
  const size_t need[3] = {lds_solve_bytes<P, 0>(c->n[0]), lds_solve_bytes<P, 1>(c->n[1]), lds_solve_bytes<P, 2>(c->n[2])};
  for (int d = 0; d < 3; ++d)
    if (c->n[d] <= kLdsLineMax && need[d] > 64 * 1024)
      IGAFD_HIP_CHECK(hipFuncSetAttribute(fn[d], hipFuncAttributeMaxDynamicSharedMemorySize, (int)need[d]));
  return IGAFD_OK;
}

igafd_status adi_lds_attr(const igafd_ctx* c) {
  switch (c->p) {
#define IGAFD_P(P) \
  case P:          \
    return lds_attr<P>(c);
    IGAFD_P(1) IGAFD_P(2) IGAFD_P(3) IGAFD_P(4) IGAFD_P(5) IGAFD_P(6)
#undef IGAFD_P
    default:
      set_error("unsupported degree");
      return IGAFD_ERR_ARG;
  }
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
    IGAFD_T((band_apply<P, 1>(c, a->bandK[1], 1.0, s, nullptr, 0.0, nullptr, 0.0, t1, flag)));
    IGAFD_T((line_solve<P, 1>(c, facM(1), 1.0, t1, u, flag)));
    // r*_j = r~ - ((K1 - w M1) x I x I) s_{j-1} - (2 M1 x I x I)(u_j + v_j); s*_j
    IGAFD_T((band_apply<P, 0>(c, a->bandKw1 + (size_t)j * n1 * (2 * P + 1), -1.0, s, nullptr, 0.0, rt, 1.0, t1, flag)));
    IGAFD_T((band_apply<P, 0>(c, a->bandM[0], -2.0, u, v, 1.0, t1, 1.0, t1, flag)));
    IGAFD_T((line_solve<P, 0>(c, facW(0, j), 1.0, t1, t1, flag)));
    // r**_j = (I x M2 x I)(u_j + w s*_j); s**_j
    IGAFD_T((band_apply<P, 1>(c, a->bandM[1], 1.0, u, t1, w, nullptr, 0.0, t2, flag)));
    IGAFD_T((line_solve<P, 1>(c, facW(1, j), 1.0, t2, t2, flag)));
    // b_j = v_j + w s**_j; r_j = (I x I x M3) b_j; s_j; v_{j+1} = b_j - w s_j
    IGAFD_T((band_apply<P, 2>(c, a->bandM[2], 1.0, v, t2, w, nullptr, 0.0, t1, flag)));
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
  if (a->bandKw1) (void)hipFree(a->bandKw1);
  if (a->work) (void)hipFree(a->work);
  delete a;
  c->adi = nullptr;
}

// eq. greedy2: the omega >= 0 minimising |g(omega; l1, l2, l3)|.  g = 0 at the
// positive roots of f(w) = w^3 - S w^2 + e2 w + e3 (none or two); the smaller
// one is taken.  f(0) = e3 > 0 and f has its local minimum at
// w+ = (S + sqrt(S^2 - 3 e2)) / 3: roots exist iff f(w+) <= 0, and the smaller
// lies between max(0, w-) (the local maximum) and w+.  Without roots g > 0 and
// its minimum is at the one positive root of w^3 - e2 w - 2 e3 (where
// 2 S w^2 / prod(w + l_d) peaks).  Both by bisection to the last bit.
double best_parameter(double l1, double l2, double l3) {
  const double S = l1 + l2 + l3, e2 = l1 * l2 + l1 * l3 + l2 * l3, e3 = l1 * l2 * l3;
  auto bisect = [](auto f, double lo, double hi) {  // f(lo) > 0 >= f(hi) or f(lo) < 0 <= f(hi)
    const bool up = f(lo) < 0.0;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if ((f(mid) < 0.0) == up)
        lo = mid;
      else
        hi = mid;
    }
    return 0.5 * (lo + hi);
  };
  auto f = [&](double w) { return ((w - S) * w + e2) * w + e3; };
  const double disc = std::sqrt(std::max(0.0, S * S - 3.0 * e2));
  const double wp = (S + disc) / 3.0, wm = std::max(0.0, (S - disc) / 3.0);
  if (f(wp) <= 0.0) return bisect(f, wm, wp);
  auto q = [&](double w) { return (w * w - e2) * w - 2.0 * e3; };
  double hi = std::sqrt(e2) + std::cbrt(2.0 * e3) + 1e-300;
  while (q(hi) <= 0.0) hi *= 2.0;
  return bisect(q, 0.0, hi);
}

// Greedy parameters (eq. greedy1/2): after k steps, the triple of largest
// |prod_j g_j| over the eigenvalue triples (the first in (k3, k2, k1) order on
// ties) picks omega_{k+1} = best_parameter(triple); the first parameter is
// sqrt(a b).  Stops once max |prod g_j| <= eps or at J0 steps.  The products
// are kept per triple (n1 n2 n3 doubles on the host, threads over k3).
igafd_status greedy_parameters(const igafd_ctx* c, double a, double b, double eps, int J0, std::vector<double>* w,
                               double* rho) {
  const std::vector<double>&l1 = c->dir[0].lam, &l2 = c->dir[1].lam, &l3 = c->dir[2].lam;
  const size_t n1 = l1.size(), n2 = l2.size(), n3 = l3.size(), total = n1 * n2 * n3;
  if (total > (size_t(1) << 28)) {
    set_error("greedy ADI parameters: too many eigenvalue triples (more than 2^28)");
    return IGAFD_ERR_ARG;
  }
  std::vector<double> G(total, 1.0);
  const unsigned hw = std::thread::hardware_concurrency();
  const int T = (int)std::max(1u, std::min(16u, hw));
  w->assign(1, std::sqrt(a * b));
  for (;;) {
    const double om = w->back();
    std::vector<double> best(T, -1.0);
    std::vector<size_t> at(T, 0);
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
      th.emplace_back([&, t]() {
        for (size_t k3 = t; k3 < n3; k3 += T)
          for (size_t k2 = 0; k2 < n2; ++k2)
            for (size_t k1 = 0; k1 < n1; ++k1) {
              const size_t i = (k3 * n2 + k2) * n1 + k1;
              const double s = l1[k1] + l2[k2] + l3[k3];
              G[i] = G[i] * (1.0 - 2.0 * om * om * s / ((om + l1[k1]) * (om + l2[k2]) * (om + l3[k3])));
              const double v = std::fabs(G[i]);
              if (v > best[t] || (v == best[t] && i < at[t])) {
                best[t] = v;
                at[t] = i;
              }
            }
      });
    for (auto& x : th) x.join();
    int tb = 0;
    for (int t = 1; t < T; ++t)
      if (best[t] > best[tb] || (best[t] == best[tb] && at[t] < at[tb])) tb = t;
    *rho = best[tb];
    if (*rho <= eps || (int)w->size() >= J0) return IGAFD_OK;
    const size_t i = at[tb];
    const size_t k1 = i % n1, k2 = (i / n1) % n2, k3 = i / (n1 * n2);
    w->push_back(best_parameter(l1[k1], l2[k2], l3[k3]));
  }
}

igafd_status adi_setup(igafd_ctx* c, double eps, int rule) {
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
  if (rule == kAdiGreedy) {
    const igafd_status gs = greedy_parameters(c, a, b, eps, J0, &w, &rho);
    if (gs != IGAFD_OK) return gs;
  } else {
    for (int J = 1; J <= J0; ++J) {
      w.assign(J, 0.0);
      for (int j = 0; j < J; ++j) w[j] = J == 1 ? std::sqrt(a * b) : a * std::pow(b / a, (double)j / (J - 1));
      rho = error_norm(w, c->dir[0].lam, c->dir[1].lam, c->dir[2].lam);
      if (rho <= eps) break;
    }
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
      if (a->bandKw1) (void)hipFree(a->bandKw1);
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
  {  // K1 - omega_j M1 per parameter, direction 1
    const int n = c->dir[0].n;
    const std::vector<double> bK = band_of(c->dir[0].K, n, p), bM = band_of(c->dir[0].M, n, p);
    std::vector<double> kw((size_t)J * n * W);
    for (int j = 0; j < J; ++j)
      for (size_t e = 0; e < bK.size(); ++e) kw[(size_t)j * n * W + e] = bK[e] - w[j] * bM[e];
    IGAFD_HIP_CHECK(hipMalloc((void**)&st->bandKw1, sizeof(double) * kw.size()));
    IGAFD_HIP_CHECK(hipMemcpy(st->bandKw1, kw.data(), sizeof(double) * kw.size(), hipMemcpyHostToDevice));
  }
  IGAFD_HIP_CHECK(hipMalloc((void**)&st->work, sizeof(double) * 5 * (size_t)c->N));
  igafd_status sa = adi_lds_attr(c);
  if (sa != IGAFD_OK) return sa;
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

// y = A x for the symmetric banded stiffness matrix (Sec. 2.1 eq. A: at most
// (2p+1)^d nonzeros per row, at the offsets of the tensor stencil).
//
// Storage: only the upper half of the stencil.  Plane h (offset center+h)
// holds A(i, i+o_h) at row i; the lower entry A(i, i-o_h) = A(i-o_h, i) is read
// from the same plane at row i-o_h.  Every plane (and the input vector) has a
// zero halo of M >= max |o| rows on both sides, and the assembly never writes
// an entry whose column leaves the tensor grid.  So every load of the stencil
// is in bounds and entries outside the grid read an exact zero: the kernel is
// branch-free, all loads of a thread share one vector offset with uniform
// bases, and nothing waits between offsets.
//
// Each thread computes R consecutive rows; for every (o2, o3) pair of the
// stencil it loads the window of R + 2p input values once and reuses it for
// the (2p+1) R products of that pair.
//
// Optionally fuses the dot product (x, y) as one partial sum per block (fixed
// reduction tree: deterministic).
#include "internal.h"
#include "reduce.h"

namespace igafd {
namespace {

// KIND 0: every o1 offset of this (o2, o3) pair is in the lower half;
// 1: the center pair (o1 < 0 lower, o1 >= 0 upper); 2: all upper.
template <int D, int P, int R, int KIND>
__device__ __forceinline__ void pair_step(int o32, const double* __restrict__ band, long long Ns,
                                          const double* __restrict__ x, long long i0, long long s2, long long s3,
                                          double* acc) {
  constexpr int W = 2 * P + 1;
  constexpr int S = (D == 3) ? W * W * W : W * W;
  constexpr int C = (S - 1) / 2;
  const int o3 = (D == 3) ? o32 / W - P : 0;
  const int o2 = o32 % W - P;
  const long long base = o2 * s2 + o3 * s3;
  double xw[R + 2 * P];
  const double* xq = x + base - P + i0;
#pragma unroll
  for (int t = 0; t < R + 2 * P; ++t) xw[t] = xq[t];
#pragma unroll
  for (int o1 = -P; o1 <= P; ++o1) {
    const int oidx = o32 * W + o1 + P;
    const bool upper = KIND == 2 || (KIND == 1 && o1 >= 0);
    const double* bp = upper ? band + (long long)(oidx - C) * Ns + i0 : band + (long long)(C - oidx) * Ns + base + o1 + i0;
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = fma(bp[r], xw[r + o1 + P], acc[r]);
  }
}

// band, x point at row 0 of plane 0 / of the vector (halos before and after).
template <int D, int P, int R>
__global__ __launch_bounds__(kBlock) void k_spmv(const double* __restrict__ band, long long Ns,
                                                 const double* __restrict__ x, double* __restrict__ y, int n1, int n2,
                                                 long long N, double* __restrict__ partial,
                                                 const int* __restrict__ flag) {
  if (flag && *flag) return;  // CG already stopped: iteration enqueued ahead is a no-op
  constexpr int W = 2 * P + 1;
  constexpr int NPAIR = (D == 3) ? W * W : W;
  constexpr int MID = (NPAIR - 1) / 2;
  const long long i0 = ((long long)blockIdx.x * kBlock + threadIdx.x) * R;
  double dot = 0.0;
  if (i0 < N) {
    const long long s2 = n1, s3 = (long long)n1 * n2;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int o32 = 0; o32 < MID; ++o32) pair_step<D, P, R, 0>(o32, band, Ns, x, i0, s2, s3, acc);
    pair_step<D, P, R, 1>(MID, band, Ns, x, i0, s2, s3, acc);
    for (int o32 = MID + 1; o32 < NPAIR; ++o32) pair_step<D, P, R, 2>(o32, band, Ns, x, i0, s2, s3, acc);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (i0 + r < N) {
        y[i0 + r] = acc[r];
        dot += x[i0 + r] * acc[r];
      }
  }
  if (partial) {
    const double s = block_sum(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// copy a vector into the interior of a zero-halo buffer
__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, long long N) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < N) dst[i] = src[i];
}

template <int D, int P, int R>
igafd_status launch(igafd_ctx* c, const double* xpad, double* y, double* partial, const int* flag) {
  const long long rows = (c->N + R - 1) / R;
  const unsigned blocks = (unsigned)((rows + kBlock - 1) / kBlock);
  if (partial && (long long)blocks > c->npartial) {
    set_error("internal: A-product grid larger than the partial-sum buffer");
    return IGAFD_ERR_ARG;
  }
  hipLaunchKernelGGL((k_spmv<D, P, R>), dim3(blocks), dim3(kBlock), 0, c->stream, c->band + c->halo, c->Ns, xpad, y,
                     c->n[0], c->n[1], c->N, partial, flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

template <int D, int P>
igafd_status launch_r(igafd_ctx* c, const double* xpad, double* y, double* partial, const int* flag) {
  switch (c->spmv_rows) {
    case 1:
      return launch<D, P, 1>(c, xpad, y, partial, flag);
    case 4:
      return launch<D, P, 4>(c, xpad, y, partial, flag);
    default:
      return launch<D, P, 2>(c, xpad, y, partial, flag);
  }
}

}  // namespace

int spmv_blocks(const igafd_ctx* c) {
  const int R = (c->spmv_rows == 1 || c->spmv_rows == 4) ? c->spmv_rows : 2;
  const long long rows = (c->N + R - 1) / R;
  return (int)((rows + kBlock - 1) / kBlock);
}

// xpad: a vector with the zero halo of the band (row 0 at xpad[0]).
igafd_status spmv(igafd_ctx* c, const double* xpad, double* y, double* partial, const int* flag) {
  switch (c->dim * 10 + c->p) {
#define IGAFD_CASE(D, P) \
  case D * 10 + P:       \
    return launch_r<D, P>(c, xpad, y, partial, flag);
    IGAFD_CASE(2, 1) IGAFD_CASE(2, 2) IGAFD_CASE(2, 3) IGAFD_CASE(2, 4) IGAFD_CASE(2, 5) IGAFD_CASE(2, 6)
    IGAFD_CASE(3, 1) IGAFD_CASE(3, 2) IGAFD_CASE(3, 3) IGAFD_CASE(3, 4) IGAFD_CASE(3, 5) IGAFD_CASE(3, 6)
#undef IGAFD_CASE
    default:
      set_error("unsupported dimension/degree");
      return IGAFD_ERR_ARG;
  }
}

// y = A x for a caller vector without halo: staged through the context's
// zero-halo buffer.
igafd_status spmv_unpadded(igafd_ctx* c, const double* x, double* y, double* partial, const int* flag) {
  const unsigned blocks = (unsigned)((c->N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kBlock), 0, c->stream, x, c->xpad + c->halo, c->N);
  IGAFD_HIP_CHECK(hipGetLastError());
  return spmv(c, c->xpad + c->halo, y, partial, flag);
}

}  // namespace igafd

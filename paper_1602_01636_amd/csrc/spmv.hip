// y = A x for the symmetric banded stiffness matrix (Sec. 2.1 eq. A: at most
// (2p+1)^d nonzeros per row, at the offsets of the tensor stencil).
//
// Storage: only the upper half of the stencil, plane h = offset center+h,
// indexed by the row.  Row i reads its upper entries from plane h at i and its
// lower entries A(i, i-o) = A(i-o, i) from plane h(o) at the column i-o.  No
// column indices are stored: the offsets follow from the tensor structure
// (direction 1 fastest).  Out-of-range neighbours are predicated off, so the
// zero padding of boundary rows is never read.
//
// The kernel is HBM-bound: every stored value is needed once per product; the
// mirrored reads of a plane trail the direct reads by at most p n1 n2 rows and
// are served from the last-level cache when it holds that window.  x is read
// through L1/L2 with (2p+1)^d reuse per element.
//
// Optionally fuses the dot product (x, y) as one partial sum per block (fixed
// reduction tree: deterministic).
#include "internal.h"
#include "reduce.h"

namespace igafd {
namespace {

template <int D, int P>
__global__ __launch_bounds__(kBlock) void k_spmv(const double* __restrict__ band, long long Np,
                                                 const double* __restrict__ x, double* __restrict__ y, int n1,
                                                 int n2, int n3, long long N, double* __restrict__ partial,
                                                 const int* __restrict__ flag) {
  if (flag && *flag) return;  // CG already stopped: iteration enqueued ahead is a no-op
  constexpr int W = 2 * P + 1;
  constexpr int S = (D == 3) ? W * W * W : W * W;
  constexpr int CENTER = (S - 1) / 2;
  constexpr int R3 = (D == 3) ? P : 0;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  double acc = 0.0, xi = 0.0;
  if (i < N) {
    const int i1 = (int)(i % n1);
    const long long t = i / n1;
    const int i2 = (int)(t % n2), i3 = (int)(t / n2);
    const long long s2 = n1, s3 = (long long)n1 * n2;
    xi = x[i];
#pragma unroll
    for (int o3 = -R3; o3 <= R3; ++o3) {
      const bool v3 = (unsigned)(i3 + o3) < (unsigned)n3;
#pragma unroll
      for (int o2 = -P; o2 <= P; ++o2) {
        const bool v2 = v3 && (unsigned)(i2 + o2) < (unsigned)n2;
#pragma unroll
        for (int o1 = -P; o1 <= P; ++o1) {
          const bool v = v2 && (unsigned)(i1 + o1) < (unsigned)n1;
          const int oidx = ((o3 + R3) * W + (o2 + P)) * W + (o1 + P);
          if (v) {
            const long long j = i + o1 + o2 * s2 + o3 * s3;
            const double a = (oidx >= CENTER) ? band[(long long)(oidx - CENTER) * Np + i]
                                              : band[(long long)(CENTER - oidx) * Np + j];
            acc = fma(a, x[j], acc);
          }
        }
      }
    }
    y[i] = acc;
  }
  if (partial) {
    const double s = block_sum(xi * acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

template <int D, int P>
igafd_status launch(igafd_ctx* c, const double* x, double* y, double* partial, const int* flag) {
  const unsigned blocks = (unsigned)((c->N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_spmv<D, P>), dim3(blocks), dim3(kBlock), 0, c->stream, c->band, c->Np, x, y, c->n[0],
                     c->n[1], c->n[2], c->N, partial, flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

}  // namespace

int spmv_blocks(const igafd_ctx* c) { return (int)((c->N + kBlock - 1) / kBlock); }

igafd_status spmv(igafd_ctx* c, const double* x, double* y, double* partial, const int* flag) {
  switch (c->dim * 10 + c->p) {
#define IGAFD_CASE(D, P) \
  case D * 10 + P:       \
    return launch<D, P>(c, x, y, partial, flag);
    IGAFD_CASE(2, 1) IGAFD_CASE(2, 2) IGAFD_CASE(2, 3) IGAFD_CASE(2, 4) IGAFD_CASE(2, 5) IGAFD_CASE(2, 6)
    IGAFD_CASE(3, 1) IGAFD_CASE(3, 2) IGAFD_CASE(3, 3) IGAFD_CASE(3, 4) IGAFD_CASE(3, 5) IGAFD_CASE(3, 6)
#undef IGAFD_CASE
    default:
      set_error("unsupported dimension/degree");
      return IGAFD_ERR_ARG;
  }
}

}  // namespace igafd

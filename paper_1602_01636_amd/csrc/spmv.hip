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
#include <algorithm>
#include <map>
#include <tuple>

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
// Block bx of the rows.
template <int D, int P, int R>
__device__ __forceinline__ void row_body(const double* __restrict__ band, long long Ns, const double* __restrict__ x,
                                         double* __restrict__ y, int n1, int n2, long long N,
                                         double* __restrict__ partial, int hole, int bx) {
  constexpr int W = 2 * P + 1;
  constexpr int NPAIR = (D == 3) ? W * W : W;
  constexpr int MID = (NPAIR - 1) / 2;
  const long long i0 = ((long long)bx * kBlock + threadIdx.x) * R;
  double dot = 0.0;
  if (i0 < N) {
    // rows of the removed quarter of an L-shaped domain (2D, hole >= 0) are
    // not unknowns: written as zero, computed only when the thread also owns
    // a row of the domain
    bool out[R];
    bool all_out = hole >= 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      out[r] = false;
      if (hole >= 0) {
        const long long i = i0 + r;
        out[r] = i % n1 >= hole && i / n1 >= hole;
        all_out = all_out && out[r];
      }
    }
    const long long s2 = n1, s3 = (long long)n1 * n2;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    if (!all_out) {
      for (int o32 = 0; o32 < MID; ++o32) pair_step<D, P, R, 0>(o32, band, Ns, x, i0, s2, s3, acc);
      pair_step<D, P, R, 1>(MID, band, Ns, x, i0, s2, s3, acc);
      for (int o32 = MID + 1; o32 < NPAIR; ++o32) pair_step<D, P, R, 2>(o32, band, Ns, x, i0, s2, s3, acc);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (i0 + r < N) {
        const double v = out[r] ? 0.0 : acc[r];
        y[i0 + r] = v;
        dot += x[i0 + r] * v;
      }
  }
  if (partial) {
    const double s = block_sum(dot);
    if (threadIdx.x == 0) partial[bx] = s;
  }
}

template <int D, int P, int R>
__global__ __launch_bounds__(kBlock) void k_spmv(const double* __restrict__ band, long long Ns,
                                                 const double* __restrict__ x, double* __restrict__ y, int n1, int n2,
                                                 long long N, double* __restrict__ partial,
                                                 const int* __restrict__ flag, int hole) {
  if (flag && *flag) return;  // CG already stopped: iteration enqueued ahead is a no-op
  row_body<D, P, R>(band, Ns, x, y, n1, n2, N, partial, hole, (int)blockIdx.x);
}

// Grouped form (3D problems of one degree and row count per thread)
struct RowJob {
  const double* band;
  long long Ns;
  const double* x;
  double* y;
  int n1, n2;
  long long N;
  double* partial;
  const int* flag;
};

template <int P, int R>
__global__ __launch_bounds__(kBlock) void k_spmv_g(const RowJob* __restrict__ jobs, const int* __restrict__ start,
                                                   int njobs) {
  const int j = group_job(start, njobs, (int)blockIdx.x);
  const RowJob& t = jobs[j];
  if (t.flag && *t.flag) return;
  row_body<3, P, R>(t.band, t.Ns, t.x, t.y, t.n1, t.n2, t.N, t.partial, -1, (int)blockIdx.x - start[j]);
}

// copy a vector into the interior of a zero-halo buffer; entries of the
// removed quarter of an L-shaped domain (hole >= 0) become zero
__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, long long N, int n1, int hole) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < N) dst[i] = (hole >= 0 && i % n1 >= hole && i / n1 >= hole) ? 0.0 : src[i];
}

// zero the removed quarter i1, i2 >= hole of an n1 x n1 grid in place
__global__ void k_zero_hole(double* __restrict__ y, int n1, int hole) {
  const int w = n1 - hole;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < (long long)w * w) y[(long long)(hole + i / w) * n1 + hole + i % w] = 0.0;
}

// ------------------------------------------------------------------------
// Tiled 3D product: every stored value read from HBM once.
//
// A block owns a tile of B2 x B3 grid lines (a line = the n1 rows of one
// (i2, i3)); the B2 lines of one i3 form a run of contiguous rows, and each
// lane takes two consecutive rows of a run (B2 n1 even), so every load moves
// 16 bytes per lane.  For one line offset d = (o2, o3) of the upper stencil,
// the lane at rows i, i+1 of line L computes
//   gather   sum_o1 A(i, i+o) x[i+o]                   for its rows
//   scatter  sum_o1 A(i-o1, i-o1+o) x[i-o1]            for the rows (L+d, t)
// with o = o1 + o2 n1 + o3 n1 n2.  Both read stored upper values of rows of
// the own run (the scatter ones o1 rows away, in the lines the gather just
// fetched); values whose column leaves the grid are stored zeros, so rows
// crossing a line end contribute exactly nothing.  The gather goes to
// registers, the scatter to the LDS accumulator of the tile's extended region
// (target lines i2 in [a0-p, a0+B2+p), i3 in [c0, c0+B3+p)): one add per row
// and offset, each target slot written by one lane per offset, a barrier
// between offsets, so every sum has a fixed order.  The accumulator goes to
// a per-tile buffer; k_spmv_combine adds, for each row, the tiles covering it
// in a fixed order (bitwise reproducible).
// ------------------------------------------------------------------------
constexpr int kTileMaxCh = 8;  // row pairs per thread (chunks of 256 pairs)
// largest chunk count per degree that the compiler keeps in registers
constexpr int kTileMaxChP[kMaxDegree + 1] = {0, 8, 8, 8, 4, 1, 1};

// Tiles of at most this many chunks (per degree) keep the scatter's x window
// of their own rows (the same for every line offset) in registers instead of
// reloading it per offset: 4(p+1) VGPRs per chunk, within the 256 of two waves
// per SIMD.  At p = 3 five chunks spill 36 bytes per lane and still gain
// (fewer address operations); at p = 4 three chunks would spill 244.
constexpr int kXsRegMaxChP[kMaxDegree + 1] = {0, 8, 4, 5, 2, 1, 1};

// chunks of tb row pairs (one per thread of a tb-thread block) of a B2 x B3 tile
inline int tile_chunks(int b2, int b3, int n1, int tb = kBlock) { return ((b2 * b3 * n1 + 1) / 2 + tb - 1) / tb; }

typedef const __attribute__((address_space(1))) char* gbytes;  // global memory, byte addressed
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) d2_t __attribute__((aligned(8))) gd2;

// 16 bytes at a uniform base plus a per-lane byte offset (32 bits: the tiled
// path is used only when every row offset fits) plus a constant
__device__ __forceinline__ d2_t ld2(gbytes base, unsigned off, int k) {
  return *reinterpret_cast<gd2*>(base + off + 8 * k);
}

// a uniform global base the optimiser cannot relate across iterations
__device__ __forceinline__ gbytes opaque(const double* p) {
  unsigned long long v = reinterpret_cast<unsigned long long>(p);
  asm volatile("" : "+s"(v));
  return reinterpret_cast<gbytes>(v);
}

// Values one lane loads for one chunk (rows i, i+1) and one line offset.
template <int P>
struct ChunkVals {
  d2_t bg[2 * P + 1];  // A(i, i+o), A(i+1, i+1+o) per o1
  d2_t bs[2 * P + 1];  // A(i-o1, i-o1+o), A(i+1-o1, i+1-o1+o) per o1
  d2_t xg[P + 1];      // x[i+o2 n1+o3 n1n2 - p .. +1+p]
  d2_t xs[P + 1];      // x[i-p .. i+1+p]
};

__device__ __forceinline__ double el(const d2_t* w, int k) { return (k & 1) ? w[k >> 1].y : w[k >> 1].x; }

// One line offset (o2, o3); CENTER: o2 = o3 = 0 (o1 >= 0 stored; the
// scatter lands on the own rows and stays in registers).  go[m]: byte
// offset of the chunk's first row; tb[m]: its accumulator slot (rows of the
// chunk whose bit in own is clear add to discard slots).  The chunks are
// software pipelined: the loads of chunk m+1 are issued before the
// arithmetic of chunk m.
template <int P, int CH, bool CENTER>
__device__ __forceinline__ void tile_pair(int o2, int o3, const double* __restrict__ band, long long Ns,
                                          const double* __restrict__ x, double* lds, int n1, long long n12, int E2,
                                          int trash, unsigned own, const unsigned (&go)[CH], const int (&tb)[CH],
                                          d2_t (&acc)[CH], const d2_t (&xw)[CH][P + 1]) {
  constexpr bool XREG = CH <= kXsRegMaxChP[P];
  constexpr int W = 2 * P + 1;
  constexpr int CTR = (W * W * W - 1) / 2;
  constexpr int LO = CENTER ? 0 : -P;
  const double* xg = x + (long long)o2 * n1 + (long long)o3 * n12;  // x shifted to the target line
  const int shift = (o3 * E2 + o2) * n1;
  const double* bp0 = band + (long long)(((o3 + P) * W + (o2 + P)) * W + P - CTR) * Ns;  // plane of o1 = 0
  // Uniform bases, opaque to the optimiser: addresses stay "scalar base +
  // lane offset" per line offset instead of per-lane pointer induction
  // variables carried across offsets (one per chunk and o1, too many
  // registers); the scatter's x window, the same for every offset, is
  // reloaded (an L1 hit) unless the tile is small enough to keep it in
  // registers (xw).
  const gbytes xsb = opaque(x), xgb = opaque(xg), bpb = opaque(bp0);
  const long long plane = 8 * Ns;
  auto load = [&](int m, ChunkVals<P>& v) {
    const unsigned g = go[m];
#pragma unroll
    for (int o1 = LO; o1 <= P; ++o1) {
      const gbytes pl = bpb + o1 * plane;
      v.bg[o1 + P] = ld2(pl, g, 0);
      if (!CENTER || o1 > 0) v.bs[o1 + P] = ld2(pl, g, -o1);
    }
#pragma unroll
    for (int k = 0; k <= P; ++k) {
      v.xg[k] = ld2(xgb, g, 2 * k - P);
      if (!XREG) v.xs[k] = ld2(xsb, g, 2 * k - P);
    }
  };
  auto compute = [&](int m, const ChunkVals<P>& v) {
    const d2_t* xs = XREG ? xw[m] : v.xs;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int o1 = LO; o1 <= P; ++o1) {
      acc[m].x = fma(v.bg[o1 + P].x, el(v.xg, o1 + P), acc[m].x);
      acc[m].y = fma(v.bg[o1 + P].y, el(v.xg, o1 + P + 1), acc[m].y);
      if (!CENTER || o1 > 0) {
        s0 = fma(v.bs[o1 + P].x, el(xs, P - o1), s0);
        s1 = fma(v.bs[o1 + P].y, el(xs, P - o1 + 1), s1);
      }
    }
    if (CENTER) {
      acc[m].x += s0;
      acc[m].y += s1;
    } else {
      // no branch around the update (it would serialise the chunks' loads):
      // rows without a slot add to their lane's discard slots
      const int d = trash + 2 * (int)(threadIdx.x & 63);
      const int i0 = (own & (1u << (2 * m))) ? tb[m] + shift : d;
      const int i1 = (own & (2u << (2 * m))) ? tb[m] + shift + 1 : d + 1;
      lds[i0] += s0;
      lds[i1] += s1;
    }
  };
  ChunkVals<P> v0, v1;
  load(0, v0);
#pragma unroll
  for (int m = 0; m < CH; ++m) {
    ChunkVals<P>& cur = (m & 1) ? v1 : v0;
    ChunkVals<P>& nxt = (m & 1) ? v0 : v1;
    if (m + 1 < CH) load(m + 1, nxt);
    __builtin_amdgcn_sched_barrier(0);
    compute(m, cur);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// band, x: row 0 of plane 0 / of the zero-halo vector; ext: T2*T3 tiles of
// E2*E3*n1 values (E2 = B2+2p, E3 = B3+p), line (e3, e2) = target line
// (c0+e3, a0+e2-p).  LDS: the accumulator plus 128 discard slots.  Row pair
// q = threadIdx.x + TB m of the tile: rows 2q, 2q+1 of the concatenated runs.
// Two waves per SIMD (two 256-thread blocks or one 512-thread block per CU):
// the occupancy target lets the scheduler keep a chunk's loads in flight
// together.
// tile_body: the work of tile `tile` (t2 fastest) by TB threads.
template <int P, int CH, int TB>
__device__ __forceinline__ void tile_body(const double* __restrict__ band, long long Ns, const double* __restrict__ x,
                                          double* __restrict__ ext, int n1, int n2, int n3, int B2, int B3, int T2,
                                          int tile) {
  extern __shared__ double lds[];
  const int E2 = B2 + 2 * P, E3 = B3 + P;
  const int elems = E2 * E3 * n1;
  const int t2 = tile % T2, t3 = tile / T2;
  const int a0 = t2 * B2, c0 = t3 * B3;
  for (int k = threadIdx.x; k < elems; k += TB) lds[k] = 0.0;
  const int run = B2 * n1;                                  // rows of one run (even)
  const int valid_run = (n2 - a0 < B2 ? n2 - a0 : B2) * n1;  // rows of a run inside the grid
  const long long n12 = (long long)n1 * n2;
  unsigned go[CH];
  int tb[CH];
  d2_t acc[CH];
  unsigned own = 0;  // bits 2m, 2m+1: rows of chunk m with an accumulator slot
#pragma unroll
  for (int m = 0; m < CH; ++m) {
    const int r = 2 * (threadIdx.x + TB * m);  // first row of the pair in the tile
    const int j = r / run, off = r - j * run;       // run (= b3) and row in the run
    const bool ok0 = j < B3 && c0 + j < n3 && off < valid_run;
    const bool ok1 = ok0 && off + 1 < valid_run;
    go[m] = ok0 ? 8u * (unsigned)((long long)n1 * a0 + n12 * (c0 + j) + off) : 0u;
    tb[m] = ok0 ? (j * E2 + P) * n1 + off : 0;
    acc[m] = d2_t{0.0, 0.0};
    own |= (ok0 ? 1u : 0u) << (2 * m);
    own |= (ok1 ? 2u : 0u) << (2 * m);
  }
  const int trash = elems;
  // the scatter's x window of the own rows (register-held tiles only)
  d2_t xw[CH][P + 1];
  if constexpr (CH <= kXsRegMaxChP[P]) {
    const gbytes xb = opaque(x);
#pragma unroll
    for (int m = 0; m < CH; ++m)
#pragma unroll
      for (int k = 0; k <= P; ++k) xw[m][k] = ld2(xb, go[m], 2 * k - P);
  }
  tile_pair<P, CH, true>(0, 0, band, Ns, x, lds, n1, n12, E2, trash, own, go, tb, acc, xw);
  __syncthreads();  // accumulator zeroed
#pragma unroll 1
  for (int o2 = 1; o2 <= P; ++o2) {
    tile_pair<P, CH, false>(o2, 0, band, Ns, x, lds, n1, n12, E2, trash, own, go, tb, acc, xw);
    __syncthreads();
  }
#pragma unroll 1
  for (int o3 = 1; o3 <= P; ++o3)
#pragma unroll 1
    for (int o2 = -P; o2 <= P; ++o2) {
      tile_pair<P, CH, false>(o2, o3, band, Ns, x, lds, n1, n12, E2, trash, own, go, tb, acc, xw);
      __syncthreads();
    }
  // own rows: no other lane writes them in this phase
#pragma unroll
  for (int m = 0; m < CH; ++m) {
    if (own & (1u << (2 * m))) lds[tb[m]] += acc[m].x;
    if (own & (2u << (2 * m))) lds[tb[m] + 1] += acc[m].y;
  }
  __syncthreads();
  // streaming stores: the tile buffer is read once, by k_spmv_combine (regular
  // stores made the kernel 4-6% slower at p = 3..5)
  double* out = ext + (long long)tile * elems;
  for (int k = threadIdx.x; k < elems; k += TB) __builtin_nontemporal_store(lds[k], out + k);
}

// TB = 256: two blocks per CU (LDS permitting); TB = 512: one larger tile per CU
template <int P, int CH, int TB>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_spmv_tile(
    const double* __restrict__ band, long long Ns, const double* __restrict__ x, double* __restrict__ ext, int n1,
    int n2, int n3, int B2, int B3, int T2, const int* __restrict__ flag) {
  if (flag && *flag) return;
  tile_body<P, CH, TB>(band, Ns, x, ext, n1, n2, n3, B2, B3, T2, (int)blockIdx.x);
}

// Grouped form: the tiles of several problems in one launch (block b works on
// job j with start[j] <= b < start[j + 1]); a job whose CG has stopped exits.
struct TileJob {
  const double* band;
  long long Ns;
  const double* x;
  double* ext;
  int n1, n2, n3, B2, B3, T2;
  const int* flag;
};

template <int P, int CH, int TB>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_spmv_tile_g(
    const TileJob* __restrict__ jobs, const int* __restrict__ start, int njobs) {
  const int j = group_job(start, njobs, (int)blockIdx.x);
  const TileJob& t = jobs[j];
  if (t.flag && *t.flag) return;
  tile_body<P, CH, TB>(t.band, t.Ns, t.x, t.ext, t.n1, t.n2, t.n3, t.B2, t.B3, t.T2, (int)blockIdx.x - start[j]);
}

__device__ inline int ceil_div(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }

// y[i] = sum over the tiles whose extended region holds row i (t3 in [t3lo,
// t3hi], t2 in [t2lo, t2hi]; added in the order t3, then t2 ascending);
// optional per-block partial of (x, y).  Block bx of the rows.  M3, M2 > 0:
// at most M3 x M2 covering tiles (the launch's tile shape guarantees it), all
// of their loads issued before the first add (slots past the row's range read
// a covered tile and are skipped by a select, so the sum and its order are
// those of the loop); 0, 0: the loop.
template <int M3, int M2>
__device__ __forceinline__ void combine_body(const double* __restrict__ ext, const double* __restrict__ x,
                                             double* __restrict__ y, int n1, int n2, int n3, int P, int B2, int B3,
                                             int T2, int T3, long long N, double* __restrict__ partial, int bx) {
  const long long i = (long long)bx * kBlock + threadIdx.x;
  double dot = 0.0;
  if (i < N) {
    // 32-bit index arithmetic: the tiled product needs N < 2^29
    const unsigned iu = (unsigned)i, rest = iu / (unsigned)n1;
    const int i1 = (int)(iu - rest * (unsigned)n1);
    const int i3 = (int)(rest / (unsigned)n2), i2 = (int)(rest - (unsigned)i3 * (unsigned)n2);
    const int E2 = B2 + 2 * P, E3 = B3 + P;
    const long long elems = (long long)E2 * E3 * n1;
    const int t3lo = max(0, ceil_div(i3 - E3 + 1, B3)), t3hi = min(T3 - 1, i3 / B3);
    const int t2lo = max(0, ceil_div(i2 - B2 - P + 1, B2)), t2hi = min(T2 - 1, (i2 + P) / B2);
    auto at = [&](int t3, int t2) {
      const int line = (i3 - t3 * B3) * E2 + (i2 - t2 * B2 + P);
      return ext[((long long)t3 * T2 + t2) * elems + (long long)line * n1 + i1];
    };
    double s = 0.0;
    if constexpr (M3 > 0) {
      double v[M3][M2];
#pragma unroll
      for (int k3 = 0; k3 < M3; ++k3)
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) v[k3][k2] = at(min(t3lo + k3, t3hi), min(t2lo + k2, t2hi));
#pragma unroll
      for (int k3 = 0; k3 < M3; ++k3)
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) s = (t3lo + k3 <= t3hi && t2lo + k2 <= t2hi) ? s + v[k3][k2] : s;
    } else {
      for (int t3 = t3lo; t3 <= t3hi; ++t3)
        for (int t2 = t2lo; t2 <= t2hi; ++t2) s += at(t3, t2);
    }
    y[i] = s;
    dot = x[i] * s;
  }
  if (partial) {
    const double sum = block_sum(dot);
    if (threadIdx.x == 0) partial[bx] = sum;
  }
}

template <int M3, int M2>
__global__ __launch_bounds__(kBlock) void k_spmv_combine(const double* __restrict__ ext,
                                                         const double* __restrict__ x, double* __restrict__ y,
                                                         int n1, int n2, int n3, int P, int B2, int B3, int T2,
                                                         int T3, long long N, double* __restrict__ partial,
                                                         const int* __restrict__ flag) {
  if (flag && *flag) return;
  combine_body<M3, M2>(ext, x, y, n1, n2, n3, P, B2, B3, T2, T3, N, partial, (int)blockIdx.x);
}

struct CombineJob {
  const double* ext;
  const double* x;
  double* y;
  int n1, n2, n3, P, B2, B3, T2, T3;
  long long N;
  double* partial;
  const int* flag;
};

__global__ __launch_bounds__(kBlock) void k_spmv_combine_g(const CombineJob* __restrict__ jobs,
                                                           const int* __restrict__ start, int njobs) {
  const int j = group_job(start, njobs, (int)blockIdx.x);
  const CombineJob& t = jobs[j];
  if (t.flag && *t.flag) return;
  combine_body<0, 0>(t.ext, t.x, t.y, t.n1, t.n2, t.n3, t.P, t.B2, t.B3, t.T2, t.T3, t.N, t.partial,
                     (int)blockIdx.x - start[j]);
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
                     c->n[0], c->n[1], c->N, partial, flag, c->dim == 2 ? c->hole : -1);
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


// Dynamic LDS above 64 KB needs the kernel attribute; set once when a tile
// shape is selected (never inside a launch sequence that may be captured).
template <int P, int TB>
igafd_status tile_lds_attr_tb(int ch, int lds) {
  const void* fn = nullptr;
  switch (ch) {
#define IGAFD_CH(K)                              \
  case K:                                        \
    fn = (const void*)&k_spmv_tile<P, K, TB>;    \
    break;
    IGAFD_CH(1) IGAFD_CH(2) IGAFD_CH(3) IGAFD_CH(4) IGAFD_CH(5) IGAFD_CH(6) IGAFD_CH(7) IGAFD_CH(8)
#undef IGAFD_CH
    default:
      set_error("internal: bad tile chunk count");
      return IGAFD_ERR_ARG;
  }
  IGAFD_HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
  return IGAFD_OK;
}

template <int P>
igafd_status tile_lds_attr(int ch, int lds, int tb) {
  return tb == 512 ? tile_lds_attr_tb<P, 512>(ch, lds) : tile_lds_attr_tb<P, 256>(ch, lds);
}

template <int P, int CH>
igafd_status launch_tile_ch(igafd_ctx* c, const double* xpad, int T2, size_t lds, const int* flag) {
  const int T3 = (c->n[2] + c->tile_b3 - 1) / c->tile_b3;
  if (c->tile_tb == 512)
    hipLaunchKernelGGL((k_spmv_tile<P, CH, 512>), dim3((unsigned)(T2 * T3)), dim3(512), lds, c->stream,
                       c->band + c->halo, c->Ns, xpad, c->ext, c->n[0], c->n[1], c->n[2], c->tile_b2, c->tile_b3, T2,
                       flag);
  else
    hipLaunchKernelGGL((k_spmv_tile<P, CH, 256>), dim3((unsigned)(T2 * T3)), dim3(256), lds, c->stream,
                       c->band + c->halo, c->Ns, xpad, c->ext, c->n[0], c->n[1], c->n[2], c->tile_b2, c->tile_b3, T2,
                       flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

template <int P>
igafd_status launch_tile(igafd_ctx* c, const double* xpad, double* y, double* partial, const int* flag) {
  const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2];
  const int B2 = c->tile_b2, B3 = c->tile_b3;
  const int T2 = (n2 + B2 - 1) / B2, T3 = (n3 + B3 - 1) / B3;
  const int E2 = B2 + 2 * P, E3 = B3 + P;
  const size_t lds = sizeof(double) * ((size_t)E2 * E3 * n1 + 2 * 64);
  const int ch = tile_chunks(B2, B3, n1, c->tile_tb);
  if ((long long)T2 * T3 * E2 * E3 * n1 > c->ext_cap || ch < 1 || ch > kTileMaxCh) {
    set_error("internal: tile shape does not fit the tile buffer");
    return IGAFD_ERR_ARG;
  }
  const unsigned vb = (unsigned)((c->N + kBlock - 1) / kBlock);
  if (partial && (long long)vb > c->npartial) {
    set_error("internal: A-product grid larger than the partial-sum buffer");
    return IGAFD_ERR_ARG;
  }
  igafd_status s = IGAFD_OK;
  switch (ch) {
#define IGAFD_CH(K)                                          \
  case K:                                                    \
    s = launch_tile_ch<P, K>(c, xpad, T2, lds, flag);        \
    break;
    IGAFD_CH(1) IGAFD_CH(2) IGAFD_CH(3) IGAFD_CH(4) IGAFD_CH(5) IGAFD_CH(6) IGAFD_CH(7) IGAFD_CH(8)
#undef IGAFD_CH
  }
  if (s != IGAFD_OK) return s;
  // covering tiles per row: at most (E - 1) / B + 1 per direction
  const int m3 = (B3 + P - 1) / B3 + 1, m2 = (B2 + 2 * P - 1) / B2 + 1;
#define IGAFD_COMB(M3, M2)                                                                                        \
  hipLaunchKernelGGL((k_spmv_combine<M3, M2>), dim3(vb), dim3(kBlock), 0, c->stream, c->ext, xpad, y, n1, n2, n3, P, \
                     B2, B3, T2, T3, c->N, partial, flag)
  if (m3 <= 2 && m2 <= 2)
    IGAFD_COMB(2, 2);
  else if (m3 <= 2 && m2 <= 3)
    IGAFD_COMB(2, 3);
  else if (m3 <= 3 && m2 <= 3)
    IGAFD_COMB(3, 3);
  else if (m3 <= 2 && m2 <= 6)
    IGAFD_COMB(2, 6);
  else
    IGAFD_COMB(0, 0);
#undef IGAFD_COMB
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

}  // namespace

int spmv_blocks(const igafd_ctx* c) {
  if (c->tile_b2 > 0) return (int)((c->N + kBlock - 1) / kBlock);
  const int R = (c->spmv_rows == 1 || c->spmv_rows == 4) ? c->spmv_rows : 2;
  const long long rows = (c->N + R - 1) / R;
  return (int)((rows + kBlock - 1) / kBlock);
}

// Tile shape of the 3D tiled product, among those whose LDS accumulator fits
// `lds_limit` bytes, whose runs hold an even number of rows (row pairs never
// straddle two runs) and whose chunk count the compiler keeps in registers:
// the best product of (owned lines / extended lines: stored values read per
// accumulator value written), (row pairs / lanes of the chunks: lane use) and
// (tiles / resident-block slots of the rounds the grid takes: tail of the
// grid).  Returns false when no shape fits (or the problem is 2D or too large
// for 32-bit row offsets): the row-parallel kernel is used then.  tb: threads
// per block (256: up to two blocks per CU; 512: one).
bool spmv_pick_tile(const igafd_ctx* c, long long lds_limit, int* b2_out, int* b3_out, int tb, double* score_out) {
  if (c->dim != 3 || c->N >= (1LL << 29)) return false;  // byte offsets of rows fit 32 bits
  const int p = c->p, n1 = c->n[0], n2 = c->n[1], n3 = c->n[2];
  int dev = 0, cus = 256, lds_cu = 160 * 1024;
  if (hipGetDevice(&dev) == hipSuccess) {
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  }
  double best = 0.0;
  for (int b3 = 1; b3 <= 16 && b3 <= n3; ++b3)
    for (int b2 = 1; b2 <= 32 && b2 <= n2; ++b2) {
      const int lines = b2 * b3;
      if (lines < 2) continue;
      const int ch = tile_chunks(b2, b3, n1, tb);
      if ((b2 * n1) % 2 != 0 || ch > kTileMaxChP[p]) continue;
      const long long e = (long long)(b2 + 2 * p) * (b3 + p);
      const long long lds = 8 * (e * n1 + 128);
      if (lds > lds_limit) continue;
      const long long tiles = (long long)((n2 + b2 - 1) / b2) * ((n3 + b3 - 1) / b3);
      const long long slots = (long long)cus * (tb == 512 ? 1LL : std::max(1LL, (long long)lds_cu / lds));
      const long long rounds = (tiles + slots - 1) / slots;
      double score = (double)lines / (double)e * ((double)lines * n1 / 2.0 / ((double)ch * tb)) *
                     ((double)tiles / (double)(rounds * slots));
      // shapes that keep the own-row x window in registers issue fewer loads
      // per line offset (p = 4, 112^3: 4 x 2 lines 887 us against 4 x 3, 968 us)
      if (p >= 3 && ch <= kXsRegMaxChP[p]) score *= 1.2;
      if (score > best * (1.0 + 1e-9)) {
        best = score;
        *b2_out = b2;
        *b3_out = b3;
      }
    }
  if (score_out) *score_out = best;
  return best > 0.0;
}

// Select a tile shape (b2 = 0: the row-parallel kernel) and its threads per
// block (256 or 512), and make the tile buffer large enough (setup-time
// allocation only).
igafd_status spmv_set_tile(igafd_ctx* c, int b2, int b3, int tb) {
  if (b2 <= 0) {
    c->tile_b2 = c->tile_b3 = 0;
    c->tile_tb = 256;
    return IGAFD_OK;
  }
  if (c->dim != 3 || b3 <= 0 || b2 > c->n[1] || b3 > c->n[2] || (b2 * c->n[0]) % 2 != 0 || (tb != 256 && tb != 512) ||
      tile_chunks(b2, b3, c->n[0], tb) > kTileMaxChP[c->p] || c->N >= (1LL << 29)) {
    set_error("tile shape not usable for this problem");
    return IGAFD_ERR_ARG;
  }
  const int p = c->p;
  const long long T2 = (c->n[1] + b2 - 1) / b2, T3 = (c->n[2] + b3 - 1) / b3;
  const long long need = T2 * T3 * (b2 + 2 * p) * (b3 + p) * (long long)c->n[0];
  const long long lds = 8LL * ((b2 + 2 * p) * (b3 + p) * (long long)c->n[0] + 128);
  int dev = 0, maxlds = 0;
  IGAFD_HIP_CHECK(hipGetDevice(&dev));
  IGAFD_HIP_CHECK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (lds > maxlds) {
    set_error("tile accumulator larger than the device's LDS per block");
    return IGAFD_ERR_ARG;
  }
  if (lds > 65536) {
    const int ch = tile_chunks(b2, b3, c->n[0], tb);
    igafd_status s = IGAFD_OK;
    switch (p) {
#define IGAFD_TCASE(P)                          \
  case P:                                       \
    s = tile_lds_attr<P>(ch, (int)lds, tb);     \
    break;
      IGAFD_TCASE(1) IGAFD_TCASE(2) IGAFD_TCASE(3) IGAFD_TCASE(4) IGAFD_TCASE(5) IGAFD_TCASE(6)
#undef IGAFD_TCASE
      default:
        set_error("unsupported degree");
        return IGAFD_ERR_ARG;
    }
    if (s != IGAFD_OK) return s;
  }
  if (need > c->ext_cap) {
    if (c->ext) IGAFD_HIP_CHECK(hipFree(c->ext));
    c->ext = nullptr;
    c->ext_cap = 0;
    IGAFD_HIP_CHECK(hipMalloc((void**)&c->ext, sizeof(double) * (size_t)need));
    c->ext_cap = need;
  }
  c->tile_b2 = b2;
  c->tile_b3 = b3;
  c->tile_tb = tb;
  return IGAFD_OK;
}

// xpad: a vector with the zero halo of the band (row 0 at xpad[0]).
igafd_status spmv(igafd_ctx* c, const double* xpad, double* y, double* partial, const int* flag) {
  if (c->tile_b2 > 0 && c->dim == 3) {
    switch (c->p) {
#define IGAFD_TCASE(P) \
  case P:              \
    return launch_tile<P>(c, xpad, y, partial, flag);
      IGAFD_TCASE(1) IGAFD_TCASE(2) IGAFD_TCASE(3) IGAFD_TCASE(4) IGAFD_TCASE(5) IGAFD_TCASE(6)
#undef IGAFD_TCASE
      default:
        break;
    }
  }
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
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kBlock), 0, c->stream, x, c->xpad + c->halo, c->N, c->n[0],
                     c->dim == 2 ? c->hole : -1);
  IGAFD_HIP_CHECK(hipGetLastError());
  return spmv(c, c->xpad + c->halo, y, partial, flag);
}

igafd_status mask_hole(igafd_ctx* c, double* y) {
  if (c->hole < 0 || c->dim != 2) return IGAFD_OK;
  const long long w = c->n[0] - c->hole;
  if (w <= 0) return IGAFD_OK;
  hipLaunchKernelGGL(k_zero_hole, dim3((unsigned)((w * w + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, y,
                     c->n[0], c->hole);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

// ---- grouped A products (batched solves) ----

bool spmv_groupable(const igafd_ctx* c) { return c->dim == 3 && c->p >= 1 && c->p <= kMaxDegree; }

namespace {

template <int P, int CH, int TB>
igafd_status tile_g_launch(const TileJob* jobs, const int* start, int njobs, int blocks, size_t lds,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_spmv_tile_g<P, CH, TB>), dim3((unsigned)blocks), dim3(TB), lds, st, jobs, start, njobs);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

template <int P, int CH, int TB>
igafd_status tile_g_attr(size_t lds) {
  IGAFD_HIP_CHECK(hipFuncSetAttribute((const void*)k_spmv_tile_g<P, CH, TB>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return IGAFD_OK;
}

template <int P, int CH>
igafd_status tile_g_tb(int tb, bool attr, const TileJob* jobs, const int* start, int njobs, int blocks, size_t lds,
                       hipStream_t st) {
  if (tb == 512) return attr ? tile_g_attr<P, CH, 512>(lds) : tile_g_launch<P, CH, 512>(jobs, start, njobs, blocks, lds, st);
  return attr ? tile_g_attr<P, CH, 256>(lds) : tile_g_launch<P, CH, 256>(jobs, start, njobs, blocks, lds, st);
}

// (p, chunk count, threads per block) -> the grouped tile kernel's launch or
// attribute call
template <int P>
igafd_status tile_g_dispatch(int ch, int tb, bool attr, const TileJob* jobs, const int* start, int njobs, int blocks,
                             size_t lds, hipStream_t st) {
  switch (ch) {
#define IGAFD_CH(K) \
  case K:           \
    return tile_g_tb<P, K>(tb, attr, jobs, start, njobs, blocks, lds, st);
    IGAFD_CH(1) IGAFD_CH(2) IGAFD_CH(3) IGAFD_CH(4) IGAFD_CH(5) IGAFD_CH(6) IGAFD_CH(7) IGAFD_CH(8)
#undef IGAFD_CH
    default:
      set_error("internal: bad tile chunk count");
      return IGAFD_ERR_ARG;
  }
}

template <int P>
igafd_status row_g_dispatch(int r, const RowJob* jobs, const int* start, int njobs, int blocks, hipStream_t st) {
  switch (r) {
    case 1:
      hipLaunchKernelGGL((k_spmv_g<P, 1>), dim3((unsigned)blocks), dim3(kBlock), 0, st, jobs, start, njobs);
      break;
    case 4:
      hipLaunchKernelGGL((k_spmv_g<P, 4>), dim3((unsigned)blocks), dim3(kBlock), 0, st, jobs, start, njobs);
      break;
    default:
      hipLaunchKernelGGL((k_spmv_g<P, 2>), dim3((unsigned)blocks), dim3(kBlock), 0, st, jobs, start, njobs);
      break;
  }
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

igafd_status row_g(int p, int r, const RowJob* jobs, const int* start, int njobs, int blocks, hipStream_t st) {
  switch (p) {
#define IGAFD_TCASE(P) \
  case P:              \
    return row_g_dispatch<P>(r, jobs, start, njobs, blocks, st);
    IGAFD_TCASE(1) IGAFD_TCASE(2) IGAFD_TCASE(3) IGAFD_TCASE(4) IGAFD_TCASE(5) IGAFD_TCASE(6)
#undef IGAFD_TCASE
    default:
      set_error("unsupported degree");
      return IGAFD_ERR_ARG;
  }
}

igafd_status tile_g(int p, int ch, int tb, bool attr, const TileJob* jobs, const int* start, int njobs, int blocks,
                    size_t lds, hipStream_t st) {
  switch (p) {
#define IGAFD_TCASE(P) \
  case P:              \
    return tile_g_dispatch<P>(ch, tb, attr, jobs, start, njobs, blocks, lds, st);
    IGAFD_TCASE(1) IGAFD_TCASE(2) IGAFD_TCASE(3) IGAFD_TCASE(4) IGAFD_TCASE(5) IGAFD_TCASE(6)
#undef IGAFD_TCASE
    default:
      set_error("unsupported degree");
      return IGAFD_ERR_ARG;
  }
}

}  // namespace

igafd_status spmv_grouped(GroupArena& a, std::vector<GroupStep>& steps, const std::vector<igafd_ctx*>& cs,
                          const std::vector<const double*>& x, const std::vector<double*>& y,
                          const std::vector<double*>& partial, bool stop_flags) {
  const int n = (int)cs.size();
  if (n == 0) return IGAFD_OK;
  // tiled problems: a launch per (degree, chunk count), the dynamic LDS the
  // largest accumulator of the group, then one combine launch; row-parallel
  // problems: a launch per (degree, rows per thread)
  std::map<std::pair<int, int>, std::vector<int>> rgroups;
  std::map<std::tuple<int, int, int>, std::vector<int>> tgroups;  // (degree, chunks, threads per block)
  std::vector<int> tiled;
  for (int i = 0; i < n; ++i) {
    const igafd_ctx* c = cs[i];
    if (!spmv_groupable(c)) {
      set_error("internal: grouped A product needs 3D problems");
      return IGAFD_ERR_ARG;
    }
    const int p = c->p;
    if (c->tile_b2 > 0) {
      const int ch = tile_chunks(c->tile_b2, c->tile_b3, c->n[0], c->tile_tb);
      const long long T2 = (c->n[1] + c->tile_b2 - 1) / c->tile_b2, T3 = (c->n[2] + c->tile_b3 - 1) / c->tile_b3;
      if (T2 * T3 * (c->tile_b2 + 2 * p) * (c->tile_b3 + p) * (long long)c->n[0] > c->ext_cap || ch < 1 ||
          ch > kTileMaxCh) {
        set_error("internal: tile shape does not fit the tile buffer");
        return IGAFD_ERR_ARG;
      }
      if (partial[i] && (c->N + kBlock - 1) / kBlock > c->npartial) {
        set_error("internal: A-product grid larger than the partial-sum buffer");
        return IGAFD_ERR_ARG;
      }
      tgroups[std::make_tuple(p, ch, c->tile_tb)].push_back(i);
      tiled.push_back(i);
    } else {
      const int R = (c->spmv_rows == 1 || c->spmv_rows == 4) ? c->spmv_rows : 2;
      if (partial[i] && spmv_blocks(c) > c->npartial) {
        set_error("internal: A-product grid larger than the partial-sum buffer");
        return IGAFD_ERR_ARG;
      }
      rgroups[{p, R}].push_back(i);
    }
  }
  for (const auto& g : rgroups) {
    const int p = g.first.first, R = g.first.second;
    std::vector<RowJob> jobs;
    std::vector<int> start(1, 0);
    for (int i : g.second) {
      igafd_ctx* c = cs[i];
      jobs.push_back(RowJob{c->band + c->halo, c->Ns, x[i], y[i], c->n[0], c->n[1], c->N, partial[i],
                            stop_flags ? &c->state->flag : nullptr});
      start.push_back(start.back() + spmv_blocks(c));
    }
    const size_t oj = a.push(jobs.data(), sizeof(RowJob) * jobs.size());
    const size_t os = a.push(start.data(), sizeof(int) * start.size());
    const int nj = (int)jobs.size(), blocks = start.back();
    steps.push_back([&a, p, R, oj, os, nj, blocks](hipStream_t st) {
      return row_g(p, R, a.at<RowJob>(oj), a.at<int>(os), nj, blocks, st);
    });
  }
  for (const auto& g : tgroups) {
    const int p = std::get<0>(g.first), ch = std::get<1>(g.first), tb = std::get<2>(g.first);
    std::vector<TileJob> jobs;
    std::vector<int> start(1, 0);
    size_t lds = 0;
    for (int i : g.second) {
      igafd_ctx* c = cs[i];
      const int B2 = c->tile_b2, B3 = c->tile_b3;
      const int T2 = (c->n[1] + B2 - 1) / B2, T3 = (c->n[2] + B3 - 1) / B3;
      jobs.push_back(TileJob{c->band + c->halo, c->Ns, x[i], c->ext, c->n[0], c->n[1], c->n[2], B2, B3, T2,
                             stop_flags ? &c->state->flag : nullptr});
      start.push_back(start.back() + T2 * T3);
      lds = std::max(lds, sizeof(double) * ((size_t)(B2 + 2 * p) * (B3 + p) * c->n[0] + 2 * 64));
    }
    if (lds > 65536) {
      const igafd_status sa = tile_g(p, ch, tb, true, nullptr, nullptr, 0, 0, lds, nullptr);
      if (sa != IGAFD_OK) return sa;
    }
    const size_t oj = a.push(jobs.data(), sizeof(TileJob) * jobs.size());
    const size_t os = a.push(start.data(), sizeof(int) * start.size());
    const int nj = (int)jobs.size(), blocks = start.back();
    steps.push_back([&a, p, ch, tb, oj, os, nj, blocks, lds](hipStream_t st) {
      return tile_g(p, ch, tb, false, a.at<TileJob>(oj), a.at<int>(os), nj, blocks, lds, st);
    });
  }
  if (tiled.empty()) return IGAFD_OK;
  std::vector<CombineJob> cj;
  std::vector<int> start(1, 0);
  for (int i : tiled) {
    igafd_ctx* c = cs[i];
    const int B2 = c->tile_b2, B3 = c->tile_b3;
    const int T2 = (c->n[1] + B2 - 1) / B2, T3 = (c->n[2] + B3 - 1) / B3;
    cj.push_back(CombineJob{c->ext, x[i], y[i], c->n[0], c->n[1], c->n[2], c->p, B2, B3, T2, T3, c->N, partial[i],
                            stop_flags ? &c->state->flag : nullptr});
    start.push_back(start.back() + (int)((c->N + kBlock - 1) / kBlock));
  }
  const size_t oj = a.push(cj.data(), sizeof(CombineJob) * cj.size());
  const size_t os = a.push(start.data(), sizeof(int) * start.size());
  const int nc = (int)cj.size(), blocks = start.back();
  steps.push_back([&a, oj, os, nc, blocks](hipStream_t st) -> igafd_status {
    hipLaunchKernelGGL(k_spmv_combine_g, dim3((unsigned)blocks), dim3(kBlock), 0, st, a.at<CombineJob>(oj),
                       a.at<int>(os), nc);
    IGAFD_HIP_CHECK(hipGetLastError());
    return IGAFD_OK;
  });
  return IGAFD_OK;
}

}  // namespace igafd

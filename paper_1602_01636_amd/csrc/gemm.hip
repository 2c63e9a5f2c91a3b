// Mode products of long directions (2D grids with n_d in the hundreds or
// thousands) as tiled dense products on the MFMA units.
//
// The 2D fast-diagonalisation apply (Sec. 4.1, Alg. 1) on a row-major
// (n2 x n1) grid is four products
//   T = R U1,  Y = (U2^T T) / (lam2 (+) lam1),  Z = U2 Y,  S = Z U1^T,
// each of the form C (M x N) = A (M x K) B with B = Bm (K x N) or Bm^T
// (Bm stored N x K), all row-major.  A block computes a BM x BN tile of C
// from BK-deep slices of A and B staged in LDS k-major (double-buffered);
// four waves in a 2 x 2 grid, each TM x TN tiles of 16 x 16
// (v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4).  Global loads run two slices
// ahead: slice t+2 is loading while slice t feeds the MFMAs and slice t+1
// goes from registers to LDS; loads use clamped (in-bounds) indices and the
// values outside the matrices are zeroed only when they are stored to LDS,
// so no load is waited for early.  Epilogue: division by lam_row[m] +
// lam_col[n], the diagonal scalings of S P^-1 S, (r, s) block partials.
// Tiles go to the 8 XCDs in contiguous runs (blockIdx % 8 is the XCD), so
// blocks that share an A row panel share an L2.
//
// This file is compiled with the MFMA accumulators in VGPRs (the build's
// per-file flags): with them in AGPRs the compiler copied all accumulators
// between the register files on every slice.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "internal.h"
#include "reduce.h"

namespace igafd {
namespace {

typedef double gd4_t __attribute__((ext_vector_type(4)));
typedef float gf4_t __attribute__((ext_vector_type(4)));
typedef double gd2u_t __attribute__((ext_vector_type(2), aligned(8)));
typedef float gf4u_t __attribute__((ext_vector_type(4), aligned(4)));

// Operand layouts (gfx950): A lane l holds row l%16, B lane l holds column
// l%16, both with contracted index l/16.  Result register r of lane l holds
// column l%16 and row l/16 + 4r (f64) or 4(l/16) + r (f32).
struct G64 {
  using V = double;
  using acc = gd4_t;
  static constexpr bool ROW_STRIDE4 = true;
  static constexpr bool BF16 = false;
  static constexpr bool SPLIT = false;
};
struct G32 {
  using V = float;
  using acc = gf4_t;
  static constexpr bool ROW_STRIDE4 = false;
  static constexpr bool BF16 = false;
  static constexpr bool SPLIT = false;
};
// BF16 operands, FP32 accumulation (v_mfma_f32_16x16x16_bf16): the slices are
// staged in FP32 as for G32; per 16-deep slice each lane rounds four k values
// of an operand to BF16 and one MFMA covers the slice.  The lane group l/16
// takes k = l/16 + 4 j (j = 0..3) on both operands (the sum over k does not
// care which lane holds which k, and LDS rows LA apart hit distinct banks).
struct G16 {
  using V = float;
  using acc = gf4_t;
  static constexpr bool ROW_STRIDE4 = false;
  static constexpr bool BF16 = true;
  static constexpr bool SPLIT = false;
};
// Split BF16 (Henry, Tang and Heinecke, 2019): as G16, but each staged FP32
// value x is split at the LDS store into hi = bf16(x) and lo = bf16(x - hi),
// packed in one word (hi in the lower half), and a product is taken as
// lo_a hi_b + hi_a lo_b + hi_a hi_b (three MFMAs per slice).
struct G16X3 {
  using V = float;
  using acc = gf4_t;
  static constexpr bool ROW_STRIDE4 = false;
  static constexpr bool BF16 = true;
  static constexpr bool SPLIT = true;
};

typedef short gs4_t __attribute__((ext_vector_type(4)));

// round to nearest even
__device__ inline short bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
// the low part x - bf16(x) (exact in FP32), rounded to BF16
__device__ inline short bf16_low(float f, short hi) {
  return bf16_bits(f - __uint_as_float((unsigned)(unsigned short)hi << 16));
}

__device__ inline gd4_t mma(double a, double b, gd4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline gf4_t mma(float a, float b, gf4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kBK = 16;
// LDS row padding (elements): the four lane groups of an MFMA operand read
// four consecutive k-rows; a 16-element shift puts each group on its own banks
constexpr int kPad = 16;

struct GEpi {
  const double* lrow = nullptr;  // with lcol: C[m][n] /= lrow[m] + lcol[n]
  const double* lcol = nullptr;
  const double* lcol2 = nullptr; // 3D: C[m][n] /= lrow[m] + lcol[n % n1] + lcol2[n / n1]
  int n1 = 1;
  const double* Sa = nullptr;    // A[m][k] *= Sa[m * lda + k] (PRE)
  const double* Sc = nullptr;    // C[m][n] *= Sc[m * ldc + n]
  const double* rdot = nullptr;  // with partial: block sums of rdot[m * ldc + n] * C[m][n]
  double* partial = nullptr;
  const int* flag = nullptr;     // CG stop flag: nonzero -> the launch is a no-op
};

// One product C = A op(B); a launch runs one or two of them (the two
// subdomains of the Schwarz apply share each pass: twice the tiles per launch
// evens out the work per CU)
template <typename TA, typename TB, typename TC>
struct GProb {
  const TA* A;
  long long lda;
  const TB* B;
  long long ldb;
  TC* C;
  long long ldc;
  int M, N, K, tiles_n, ntiles;
  // batch of products sharing A: B and C of product b start b * sb, b * sc
  // further (the epilogue arrays index like C)
  int batch, tiles_b;
  long long sb, sc;
  // tile order: false = along N first (blocks of a run share an A row panel),
  // true = along M first (they share a B column panel; for M << N)
  bool mfast;
  GEpi ep;
};

template <int TM, int TN, typename V>
constexpr size_t lds_bytes() {
  return sizeof(V) * 2 * kBK * ((2 * TM * 16 + kPad) + (2 * TN * 16 + kPad));
}

// N consecutive values from p (8- or 4-byte aligned), as V
template <int N, typename T, typename V>
__device__ inline void ldv(const T* p, V* o) {
  if constexpr (sizeof(T) == 8) {
    static_assert(N % 2 == 0, "pairs of doubles");
#pragma unroll
    for (int j = 0; j < N; j += 2) {
      const gd2u_t u = *reinterpret_cast<const gd2u_t*>(p + j);
      o[j] = (V)u.x;
      o[j + 1] = (V)u.y;
    }
  } else {
    static_assert(N % 4 == 0, "quads of floats");
#pragma unroll
    for (int j = 0; j < N; j += 4) {
      const gf4u_t u = *reinterpret_cast<const gf4u_t*>(p + j);
      o[j] = (V)u.x;
      o[j + 1] = (V)u.y;
      o[j + 2] = (V)u.z;
      o[j + 3] = (V)u.w;
    }
  }
}

// PRE: A is scaled by ep.Sa (the input scaling of S P^-1 S)
template <class G, int TM, int TN, bool BT, bool PRE, typename TA, typename TB, typename TC>
__global__ __launch_bounds__(kBlock) void k_gemm(GProb<TA, TB, TC> p0, GProb<TA, TB, TC> p1, int grid0) {
  // blocks [0, grid0) work on p0, the rest on p1 (uniform per block)
  const bool second = (int)blockIdx.x >= grid0;
  const int bid = second ? (int)blockIdx.x - grid0 : (int)blockIdx.x;
  const TA* __restrict__ A = second ? p1.A : p0.A;
  const TB* __restrict__ B = second ? p1.B : p0.B;
  TC* __restrict__ C = second ? p1.C : p0.C;
  const long long lda = second ? p1.lda : p0.lda, ldb = second ? p1.ldb : p0.ldb, ldc = second ? p1.ldc : p0.ldc;
  const int M = second ? p1.M : p0.M, N = second ? p1.N : p0.N, K = second ? p1.K : p0.K;
  const int tiles_n = second ? p1.tiles_n : p0.tiles_n, ntiles = second ? p1.ntiles : p0.ntiles;
  const int tiles_b = second ? p1.tiles_b : p0.tiles_b;
  const bool mfast = second ? p1.mfast : p0.mfast;
  const long long sb = second ? p1.sb : p0.sb, sc = second ? p1.sc : p0.sc;
  const GEpi ep = second ? p1.ep : p0.ep;
  using V = typename G::V;
  using acc_t = typename G::acc;
  constexpr int BM = 2 * TM * 16, BN = 2 * TN * 16, BK = kBK;
  constexpr int LA = BM + kPad, LB = BN + kPad;
  constexpr int EA = BM * BK / kBlock, EB = BN * BK / kBlock;  // values per thread per slice
  constexpr int APR = BK / EA;                                 // threads per row of the A slice
  constexpr int BPR = BT ? BK / EB : BN / EB;                  // threads per row of the stored B slice
  extern __shared__ __align__(16) unsigned char gsm[];
  V* As = reinterpret_cast<V*>(gsm);  // [2][BK][LA]
  V* Bs = As + 2 * BK * LA;           // [2][BK][LB]
  if (ep.flag && *ep.flag) return;
  const int per = (ntiles + 7) / 8;
  const int tile = (bid & 7) * per + (bid >> 3);
  if (tile >= ntiles) {
    if (ep.partial && threadIdx.x == 0) ep.partial[bid] = 0.0;
    return;
  }
  const int bt = tile / tiles_b, tl = tile - bt * tiles_b;
  const int tiles_m = tiles_b / tiles_n;
  const int tm0 = (mfast ? tl % tiles_m : tl / tiles_n) * BM, tn0 = (mfast ? tl / tiles_m : tl % tiles_n) * BN;
  B += bt * sb;
  const long long cb = bt * sc;  // offset of this product's C (and epilogue arrays)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int wm0 = (wave >> 1) * TM * 16, wn0 = (wave & 1) * TN * 16;
  const int ar = tid / APR, ak = (tid % APR) * EA;
  const int br = tid / BPR, bc = (tid % BPR) * EB;
  // this thread's A row and (BT) Bm row, clamped into the matrices
  const int am = tm0 + ar;
  const bool am_ok = am < M;
  const TA* arow = A + (long long)(am_ok ? am : M - 1) * lda;
  const double* srow = PRE ? ep.Sa + (long long)(am_ok ? am : M - 1) * lda : nullptr;
  const int bn = BT ? tn0 + br : tn0 + bc;  // BT: row of Bm; else first column
  const bool bn_ok = bn < N;
  const TB* brow = BT ? B + (long long)(bn_ok ? bn : N - 1) * ldb : nullptr;
  const bool bvec = !BT && bn + EB <= N;    // NN: this thread's EB columns all inside

  struct Stage {
    V a[EA], b[EB];
    double s[PRE ? EA : 1];
  };
  auto load = [&](int k0, Stage& q) {
    if (k0 + BK <= K) {  // full slice: runs of consecutive k (A, BT) or n (NN) as vectors
      ldv<EA>(arow + k0 + ak, q.a);
      if (PRE) ldv<EA>(srow + k0 + ak, q.s);
      if (BT) {
        ldv<EB>(brow + k0 + bc, q.b);
      } else {
        const TB* bp = B + (long long)(k0 + br) * ldb;
        if (bvec) {
          ldv<EB>(bp + bn, q.b);
        } else {
#pragma unroll
          for (int j = 0; j < EB; ++j) q.b[j] = (V)bp[bn + j < N ? bn + j : N - 1];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < EA; ++j) {
        const int k = k0 + ak + j < K ? k0 + ak + j : K - 1;
        q.a[j] = (V)arow[k];
        if (PRE) q.s[j] = srow[k];
      }
      if (BT) {
#pragma unroll
        for (int j = 0; j < EB; ++j) q.b[j] = (V)brow[k0 + bc + j < K ? k0 + bc + j : K - 1];
      } else {
        const TB* bp = B + (long long)(k0 + br < K ? k0 + br : K - 1) * ldb;
#pragma unroll
        for (int j = 0; j < EB; ++j) q.b[j] = (V)bp[bn + j < N ? bn + j : N - 1];
      }
    }
  };
  // G16X3 splits each value once here, not in every wave that reads it: hi in
  // the lower half of the word, lo in the upper half (zero stays zero).  G16
  // rounds as it reads (measured 1.5-2 % faster than rounding here: the store
  // then waits for the conversion, the reads overlap it with the MFMAs).
  auto lds_word = [](V v) -> V {
    if constexpr (G::SPLIT) {
      const short h = bf16_bits(v), l = bf16_low(v, h);
      return __uint_as_float((unsigned)(unsigned short)h | ((unsigned)(unsigned short)l << 16));
    } else {
      return v;
    }
  };
  // zero what lies outside the matrices, then write the slice to LDS
  auto store = [&](int buf, int k0, const Stage& q) {
    V* as = As + buf * BK * LA;
    V* bs = Bs + buf * BK * LB;
#pragma unroll
    for (int j = 0; j < EA; ++j) {
      V v = q.a[j];
      if (PRE) v = (V)((double)v * q.s[j]);
      as[(ak + j) * LA + ar] = (am_ok && k0 + ak + j < K) ? lds_word(v) : V(0);
    }
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      if (BT)
        bs[(bc + j) * LB + br] = (bn_ok && k0 + bc + j < K) ? lds_word(q.b[j]) : V(0);
      else
        bs[br * LB + bc + j] = (k0 + br < K && bn + j < N) ? lds_word(q.b[j]) : V(0);
    }
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  auto compute = [&](int buf) {
    const V* as = As + buf * BK * LA;
    const V* bs = Bs + buf * BK * LB;
    if constexpr (G::SPLIT) {
      gs4_t pa[TM], la[TM], pb[TN], lb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const unsigned w = __float_as_uint(as[(grp + 4 * j) * LA + wm0 + i * 16 + col]);
          pa[i][j] = (short)(w & 0xFFFFu);
          la[i][j] = (short)(w >> 16);
        }
#pragma unroll
      for (int t = 0; t < TN; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const unsigned w = __float_as_uint(bs[(grp + 4 * j) * LB + wn0 + t * 16 + col]);
          pb[t][j] = (short)(w & 0xFFFFu);
          lb[t][j] = (short)(w >> 16);
        }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int t = 0; t < TN; ++t) {
          acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(la[i], pb[t], acc[i][t], 0, 0, 0);
          acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[i], lb[t], acc[i][t], 0, 0, 0);
          acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[i], pb[t], acc[i][t], 0, 0, 0);
        }
      return;
    } else if constexpr (G::BF16) {
      gs4_t pa[TM], pb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) pa[i][j] = bf16_bits(as[(grp + 4 * j) * LA + wm0 + i * 16 + col]);
#pragma unroll
      for (int t = 0; t < TN; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) pb[t][j] = bf16_bits(bs[(grp + 4 * j) * LB + wn0 + t * 16 + col]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int t = 0; t < TN; ++t)
          acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[i], pb[t], acc[i][t], 0, 0, 0);
      return;
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      V a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = as[(ks + grp) * LA + wm0 + i * 16 + col];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = bs[(ks + grp) * LB + wn0 + j * 16 + col];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mma(a[i], b[j], acc[i][j]);
    }
  };
  // slice t is loaded into stage t & 1 and stored to LDS buffer t & 1
  const int nk = (K + BK - 1) / BK;
  Stage q0, q1;
  load(0, q0);
  store(0, 0, q0);
  if (nk > 1) load(BK, q1);
  __syncthreads();
  // step t: load slice t+2 into stage t&1, compute slice t, store slice t+1
  auto step = [&](int t, Stage& ql, const Stage& qs) {
    if (t + 2 < nk) load((t + 2) * BK, ql);
    compute(t & 1);
    if (t + 1 < nk) store((t + 1) & 1, (t + 1) * BK, qs);
    __syncthreads();
  };
  int t = 0;
  for (; t + 1 < nk; t += 2) {
    step(t, q0, q1);
    step(t + 1, q1, q0);
  }
  if (t < nk) step(t, q0, q1);

  double dot = 0.0;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = tm0 + wm0 + i * 16 + (G::ROW_STRIDE4 ? grp + 4 * r : 4 * grp + r);
        const int n = tn0 + wn0 + j * 16 + col;
        if (m < M && n < N) {
          double v = (double)acc[i][j][r];
          const long long c = cb + (long long)m * ldc + n;
          if (ep.lrow) v /= ep.lcol2 ? ep.lrow[m] + ep.lcol[n % ep.n1] + ep.lcol2[n / ep.n1] : ep.lrow[m] + ep.lcol[n];
          if (ep.Sc) v *= ep.Sc[c];
          C[c] = (TC)v;
          if (ep.partial) dot += ep.rdot[c] * v;
        }
      }
  if (ep.partial) {
    const double sum = block_sum(dot);
    if (threadIdx.x == 0) ep.partial[bid] = sum;
  }
}

struct Cfg {
  int tm, tn;
};

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

// Tile shape: the one with the least work on the busiest CU, estimated as
// ceil(tiles / CUs) x tile area (tiles are dealt evenly, all take the same
// time), among the shapes whose LDS fits 64 KB.  Ties go to the larger tile
// (fewer re-reads of A and B) when it still gives every CU a tile, else to the
// smaller one (more waves in flight): measured on 2045^2 products, 128 x 64
// (512 tiles) beats 64 x 64 in FP64, while on 1025^2 products (153 tiles of
// 128 x 64) 64 x 64 is faster in both precisions.  The choice does not depend on the precision,
// so the number of blocks of the last product (which carry the (r, s)
// partials) is known from the shape alone.  IGAFD_GEMM_TILE=<tm>x<tn>
// overrides it (tuning).
Cfg pick(int M, int N, int M1 = 0, int N1 = 0, int batch = 1) {
  if (const char* e = std::getenv("IGAFD_GEMM_TILE")) {
    const int tm = std::atoi(e), tn = std::strchr(e, 'x') ? std::atoi(std::strchr(e, 'x') + 1) : 0;
    if ((tm == 2 || tm == 4) && (tn == 2 || tn == 4)) return {tm, tn};
  }
  const Cfg cand[4] = {{4, 4}, {4, 2}, {2, 4}, {2, 2}};
  const long long cus = device_cus();
  Cfg best{2, 2};
  long long best_cost = -1, best_tiles = 0;
  for (const Cfg& g : cand) {
    const size_t lds = sizeof(double) * 2 * kBK * ((2 * g.tm * 16 + kPad) + (2 * g.tn * 16 + kPad));
    if (lds > 64 * 1024) continue;
    long long tiles = (long long)batch * ((M + 32 * g.tm - 1) / (32 * g.tm)) * ((N + 32 * g.tn - 1) / (32 * g.tn));
    if (M1 > 0) tiles += (long long)((M1 + 32 * g.tm - 1) / (32 * g.tm)) * ((N1 + 32 * g.tn - 1) / (32 * g.tn));
    const long long cost = (tiles + cus - 1) / cus * (32LL * g.tm) * (32LL * g.tn);
    // candidates run from large to small tiles
    if (best_cost < 0 || cost < best_cost || (cost == best_cost && best_tiles < cus)) {
      best_cost = cost;
      best_tiles = tiles;
      best = g;
    }
  }
  return best;
}

// blocks whose LDS exceeds the default 64 KB need the attribute raised once
template <typename K>
hipError_t lds_attr(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

int grid_of(int M, int N, Cfg g, int batch = 1) {
  const long long tiles = (long long)batch * ((M + 32 * g.tm - 1) / (32 * g.tm)) * ((N + 32 * g.tn - 1) / (32 * g.tn));
  return (int)(8 * ((tiles + 7) / 8));
}

// Launch one product, or two sharing a launch (q1 == nullptr: one).
template <class G, bool BT, typename TA, typename TB, typename TC>
igafd_status launch(hipStream_t st, GProb<TA, TB, TC> q0, const GProb<TA, TB, TC>* q1) {
  using V = typename G::V;
  if (q1 && (q0.batch != 1 || q1->batch != 1)) {
    set_error("internal: paired products are not batched");
    return IGAFD_ERR_ARG;
  }
  const Cfg g = q1 ? pick(q0.M, q0.N, q1->M, q1->N) : pick(q0.M, q0.N, 0, 0, q0.batch);
  auto shape = [&](GProb<TA, TB, TC>& q) {
    q.tiles_n = (q.N + 32 * g.tn - 1) / (32 * g.tn);
    q.tiles_b = ((q.M + 32 * g.tm - 1) / (32 * g.tm)) * q.tiles_n;
    q.ntiles = q.tiles_b * q.batch;
  };
  shape(q0);
  GProb<TA, TB, TC> p1 = q1 ? *q1 : q0;
  shape(p1);
  const long long grid_all = (long long)grid_of(q0.M, q0.N, g, q0.batch) + (q1 ? grid_of(p1.M, p1.N, g) : 0);
  if ((long long)q0.tiles_b * q0.batch >= (1LL << 31) || grid_all >= (1LL << 31)) {
    set_error("product too large for one launch");
    return IGAFD_ERR_ARG;
  }
  const int grid0 = grid_of(q0.M, q0.N, g, q0.batch);
  const dim3 grid((unsigned)grid_all);
#define IGAFD_G(TM, TN)                                                                                         \
  if (g.tm == TM && g.tn == TN) {                                                                               \
    constexpr size_t lds = lds_bytes<TM, TN, V>();                                                              \
    if (lds > 64 * 1024) {                                                                                      \
      static const hipError_t e0 = lds_attr(k_gemm<G, TM, TN, BT, false, TA, TB, TC>, lds);                    \
      static const hipError_t e1 = lds_attr(k_gemm<G, TM, TN, BT, true, TA, TB, TC>, lds);                     \
      IGAFD_HIP_CHECK(e0);                                                                                      \
      IGAFD_HIP_CHECK(e1);                                                                                      \
    }                                                                                                           \
    if (q0.ep.Sa || p1.ep.Sa)                                                                                   \
      hipLaunchKernelGGL((k_gemm<G, TM, TN, BT, true, TA, TB, TC>), grid, dim3(kBlock), lds, st, q0, p1, grid0); \
    else                                                                                                        \
      hipLaunchKernelGGL((k_gemm<G, TM, TN, BT, false, TA, TB, TC>), grid, dim3(kBlock), lds, st, q0, p1, grid0); \
    IGAFD_HIP_CHECK(hipGetLastError());                                                                         \
    return IGAFD_OK;                                                                                            \
  }
  IGAFD_G(4, 4) IGAFD_G(4, 2) IGAFD_G(2, 4) IGAFD_G(2, 2)
#undef IGAFD_G
  set_error("internal: bad product tile");
  return IGAFD_ERR_ARG;
}

template <typename TA, typename TB, typename TC>
GProb<TA, TB, TC> prob(const TA* A, long long lda, const TB* B, long long ldb, TC* C, long long ldc, int M, int N,
                       int K, const GEpi& ep) {
  GProb<TA, TB, TC> q{};
  q.A = A;
  q.lda = lda;
  q.B = B;
  q.ldb = ldb;
  q.C = C;
  q.ldc = ldc;
  q.M = M;
  q.N = N;
  q.K = K;
  q.batch = 1;
  q.sb = q.sc = 0;
  q.mfast = false;
  q.ep = ep;
  return q;
}

template <class G>
const typename G::V* wm(const DevDir& d, int which);
template <>
const double* wm<G64>(const DevDir& d, int which) { return d.W64[which]; }
template <>
const float* wm<G32>(const DevDir& d, int which) { return d.W32[which]; }
template <>
const float* wm<G16>(const DevDir& d, int which) { return d.W32[which]; }
template <>
const float* wm<G16X3>(const DevDir& d, int which) { return d.W32[which]; }

// One 2D FD apply (Sec. 4.1 Alg. 1) by four products, or two independent
// ones (contexts c and c1, same precision) whose four passes share launches.
// T: intermediate type (double for FP64, float for FP32).
struct Job {
  igafd_ctx* c;
  const double* r;
  double* s;
  int ldr, lds;
};

template <class G, typename T>
igafd_status apply2d(const Job* jobs, int count, const double* S, double* partial, const int* flag) {
  using V = typename G::V;
  using P1 = GProb<double, V, T>;
  using P2 = GProb<V, T, T>;
  using P4 = GProb<T, V, double>;
  P1 a1[2];
  P2 a2[2], a3[2];
  P4 a4[2];
  for (int j = 0; j < count; ++j) {
    igafd_ctx* c = jobs[j].c;
    const DevDir* d = c->ddir;
    const int n1 = c->n[0], n2 = c->n[1];
    const int ldr = jobs[j].ldr > 0 ? jobs[j].ldr : n1, lds = jobs[j].lds > 0 ? jobs[j].lds : n1;
    T* b0 = reinterpret_cast<T*>(c->fdbuf[0]);
    T* b1 = reinterpret_cast<T*>(c->fdbuf[1]);
    GEpi e1, e2, e3, e4;
    e1.flag = e2.flag = e3.flag = e4.flag = flag;
    e1.Sa = S;
    e2.lrow = d[1].lam;
    e2.lcol = d[0].lam;
    e4.Sc = S;
    if (partial) {
      if (count != 1 || fd_gemm_blocks(c) > c->npartial) {
        set_error("internal: FD grid larger than the partial-sum buffer");
        return IGAFD_ERR_ARG;
      }
      e4.rdot = jobs[j].r;
      e4.partial = partial;
    }
    // T = R U1: C[i2][k1] = sum_i1 R[i2][i1] W1f[k1][i1]
    a1[j] = prob(jobs[j].r, ldr, wm<G>(d[0], 0), d[0].npad, b0, n1, n2, n1, n1, e1);
    // Y = (U2^T T) / (lam2[k2] + lam1[k1])
    a2[j] = prob(wm<G>(d[1], 0), d[1].npad, (const T*)b0, n1, b1, n1, n2, n1, n2, e2);
    // Z = U2 Y
    a3[j] = prob(wm<G>(d[1], 1), d[1].npad, (const T*)b1, n1, b0, n1, n2, n1, n2, e3);
    // S = Z U1^T: C[i2][i1] = sum_k1 Z[i2][k1] W1b[i1][k1]
    a4[j] = prob((const T*)b0, n1, wm<G>(d[0], 1), d[0].npad, jobs[j].s, lds, n2, n1, n1, e4);
  }
  const hipStream_t st = jobs[0].c->stream;
  const bool two = count == 2;
  igafd_status stt;
  if ((stt = launch<G, true>(st, a1[0], two ? &a1[1] : nullptr)) != IGAFD_OK) return stt;
  if ((stt = launch<G, false>(st, a2[0], two ? &a2[1] : nullptr)) != IGAFD_OK) return stt;
  if ((stt = launch<G, false>(st, a3[0], two ? &a3[1] : nullptr)) != IGAFD_OK) return stt;
  return launch<G, true>(st, a4[0], two ? &a4[1] : nullptr);
}

// One 3D FD apply (Sec. 5.1 Alg. 3, transposes as in the 2D algorithm) by six
// products on the (n3, n2, n1) tensor:
//   direction 1: C (n2 n3 x n1) = X (n2 n3 x n1) Wm^T      (the fast axis)
//   direction 2: C_i3 (n2 x n1) = Wm X_i3 (n2 x n1)         (n3 products, one launch)
//   direction 3: C (n3 x n1 n2) = Wm X (n3 x n1 n2)         (tiles along M first)
// with the division by lam1 + lam2 + lam3 in the epilogue of the forward
// direction-3 product, S on the first input and the last output, and the
// (r, s) partials in the last epilogue.
template <class G, typename T>
igafd_status apply3d(igafd_ctx* c, const double* r, double* s, const double* S, double* partial, const int* flag) {
  using V = typename G::V;
  const DevDir* d = c->ddir;
  const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2];
  const long long plane = (long long)n1 * n2;
  if ((long long)n2 * n3 >= (1LL << 31) || plane >= (1LL << 31)) {
    set_error("grid too large for the tiled products");
    return IGAFD_ERR_ARG;
  }
  T* b0 = reinterpret_cast<T*>(c->fdbuf[0]);
  T* b1 = reinterpret_cast<T*>(c->fdbuf[1]);
  GEpi e0, e_in, e_lam, e_out;
  e0.flag = e_in.flag = e_lam.flag = e_out.flag = flag;
  e_in.Sa = S;
  e_lam.lrow = d[2].lam;
  e_lam.lcol = d[0].lam;
  e_lam.lcol2 = d[1].lam;
  e_lam.n1 = n1;
  e_out.Sc = S;
  if (partial) {
    if (fd_gemm_blocks(c) > c->npartial) {
      set_error("internal: FD grid larger than the partial-sum buffer");
      return IGAFD_ERR_ARG;
    }
    e_out.rdot = r;
    e_out.partial = partial;
  }
  auto dir1 = [&](const auto* X, auto* Y, int which, const GEpi& ep) {
    return prob(X, n1, wm<G>(d[0], which), d[0].npad, Y, n1, n2 * n3, n1, n1, ep);
  };
  auto dir2 = [&](const T* X, T* Y, int which) {
    auto q = prob(wm<G>(d[1], which), d[1].npad, X, n1, Y, n1, n2, n1, n2, e0);
    q.batch = n3;
    q.sb = q.sc = plane;
    return q;
  };
  auto dir3 = [&](const T* X, T* Y, int which, const GEpi& ep) {
    auto q = prob(wm<G>(d[2], which), d[2].npad, X, plane, Y, plane, n3, (int)plane, n3, ep);
    q.mfast = true;
    return q;
  };
  const hipStream_t st = c->stream;
  igafd_status stt;
  if ((stt = launch<G, true>(st, dir1(r, b0, 0, e_in), (const GProb<double, V, T>*)nullptr)) != IGAFD_OK) return stt;
  if ((stt = launch<G, false>(st, dir2(b0, b1, 0), (const GProb<V, T, T>*)nullptr)) != IGAFD_OK) return stt;
  if ((stt = launch<G, false>(st, dir3(b1, b0, 0, e_lam), (const GProb<V, T, T>*)nullptr)) != IGAFD_OK) return stt;
  if ((stt = launch<G, false>(st, dir3(b0, b1, 1, e0), (const GProb<V, T, T>*)nullptr)) != IGAFD_OK) return stt;
  if ((stt = launch<G, false>(st, dir2(b1, b0, 1), (const GProb<V, T, T>*)nullptr)) != IGAFD_OK) return stt;
  return launch<G, true>(st, dir1((const T*)b0, s, 1, e_out), (const GProb<T, V, double>*)nullptr);
}

}  // namespace

// blocks of the last product (one partial each): 2D S = Z U1^T has n2 rows,
// 3D the direction-1 product has n2 n3
int fd_gemm_blocks(const igafd_ctx* c) {
  const int rows = (int)(c->N / c->n[0]);
  return grid_of(rows, c->n[0], pick(rows, c->n[0]));
}

igafd_status fd_apply_gemm3d(igafd_ctx* c, int prec, const double* r, double* s, const double* S, double* partial,
                             const int* flag) {
  if (c->dim != 3) {
    set_error("internal: 3D tiled products need a 3D context");
    return IGAFD_ERR_ARG;
  }
  switch (prec) {
    case IGAFD_FP64:
      return apply3d<G64, double>(c, r, s, S, partial, flag);
    case IGAFD_FP32:
      return apply3d<G32, float>(c, r, s, S, partial, flag);
    case IGAFD_BF16:
      return apply3d<G16, float>(c, r, s, S, partial, flag);
    case IGAFD_BF16X3:
      return apply3d<G16X3, float>(c, r, s, S, partial, flag);
    default:
      set_error("internal: unknown precision for the tiled products");
      return IGAFD_ERR_ARG;
  }
}

igafd_status fd_apply_gemm2d(igafd_ctx* c, int prec, const double* r, double* s, const double* S, double* partial,
                             const int* flag, int ldr, int lds) {
  if (c->dim != 2) {
    set_error("internal: tiled products are for 2D grids");
    return IGAFD_ERR_ARG;
  }
  const Job job{c, r, s, ldr, lds};
  switch (prec) {
    case IGAFD_FP64:
      return apply2d<G64, double>(&job, 1, S, partial, flag);
    case IGAFD_FP32:
      return apply2d<G32, float>(&job, 1, S, partial, flag);
    case IGAFD_BF16:
      return apply2d<G16, float>(&job, 1, S, partial, flag);
    case IGAFD_BF16X3:
      return apply2d<G16X3, float>(&job, 1, S, partial, flag);
    default:
      set_error("internal: unknown precision for the tiled products");
      return IGAFD_ERR_ARG;
  }
}

igafd_status fd_apply_gemm2d_pair(int prec, igafd_ctx* c0, const double* r0, int ldr0, double* s0, int lds0,
                                  igafd_ctx* c1, const double* r1, int ldr1, double* s1, int lds1, const int* flag) {
  if (c0->dim != 2 || c1->dim != 2 || c0->stream != c1->stream) {
    set_error("internal: paired tiled products need two 2D contexts on one stream");
    return IGAFD_ERR_ARG;
  }
  const Job jobs[2] = {{c0, r0, s0, ldr0, lds0}, {c1, r1, s1, ldr1, lds1}};
  switch (prec) {
    case IGAFD_FP64:
      return apply2d<G64, double>(jobs, 2, nullptr, nullptr, flag);
    case IGAFD_FP32:
      return apply2d<G32, float>(jobs, 2, nullptr, nullptr, flag);
    case IGAFD_BF16:
      return apply2d<G16, float>(jobs, 2, nullptr, nullptr, flag);
    case IGAFD_BF16X3:
      return apply2d<G16X3, float>(jobs, 2, nullptr, nullptr, flag);
    default:
      set_error("internal: unknown precision for the tiled products");
      return IGAFD_ERR_ARG;
  }
}

}  // namespace igafd

// Fast-diagonalisation apply s = P^-1 r (Sec. 4.1 Alg. 1, Sec. 5.1 Alg. 3).
//
// With K_d U_d = M_d U_d D_d, U_d^T M_d U_d = I (direction 1 the fastest index):
//   r~ = (U_d (x) .. (x) U_1)^T r          forward mode products with U_l^T
//   s~ = r~ / (lam_1[k1] + .. + lam_d[kd])  (fused into the last forward product)
//   s  = (U_d (x) .. (x) U_1) s~           backward mode products with U_l
// (the 3D listing swaps the transposes; the factorisation U^T M U = I and the
// 2D algorithm fix the forward product as the transposed one).
//
// Each mode product is a small-K GEMM on the MFMA units:
//   D[k][c] = sum_i Wm[k][i] X(i, c),   Wm = U^T (forward) or U (backward),
// where c runs over the other two tensor indices.  For directions 2 and 3 the
// contracted index is a slow axis: X(i, c) = X[b][i][c] (contiguous c);
// for direction 1 it is the fast axis: X(i, c) = X[c][i].  One wave computes a
// 16-column strip for MT 16-row tiles (MT*16 >= n rows split over at most a
// few row blocks), looping over the contracted index in MFMA K-steps; the
// matrices Wm (at most npad x npad, zero padded) stay in L1/L2.
//
// Precisions: FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_16x16x4),
// BF16 inputs with FP32 accumulation, and split BF16 (each FP32 operand as
// hi + lo BF16 parts, three BF16 MFMAs per product).  The fused 3D passes use
// gfx950's 32-deep v_mfma_f32_16x16x32_bf16; the generic per-strip products
// (small 2D problems) the 16-deep v_mfma_f32_16x16x16_bf16.  r and s are
// FP64; intermediates are FP64 for FP64 and FP32 otherwise.
//
// Fused epilogues: scaling by the eigenvalue sums, the diagonal S of the
// scaled preconditioner S P^-1 S on input and output, and the partial sums of
// (r, s) for the CG recurrence.
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "reduce.h"

namespace igafd {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef short s8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

__device__ inline short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (short)(u >> 16);
}
__device__ inline float from_bf16(short h) { return __uint_as_float((unsigned)(unsigned short)h << 16); }

// Split BF16 (Henry, Tang and Heinecke, 2019): x = hi + lo + e with
// hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in FP32), |e| <= 2^-16 |x|.
__device__ inline void split4(const float* x, s4_t& hi, s4_t& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    hi[j] = to_bf16(x[j]);
    lo[j] = to_bf16(x[j] - from_bf16(hi[j]));
  }
}
// a b ~ lo_a hi_b + hi_a lo_b + hi_a hi_b (the lo_a lo_b term, <= 2^-16 |a b|,
// is dropped; at most about 3 * 2^-16 |a b| in all); the small terms go first
// into the FP32 accumulator
__device__ inline f4_t mma_bf16x3(const s4_t& ahi, const s4_t& alo, const s4_t& bhi, const s4_t& blo, f4_t c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, c, 0, 0, 0);
}

// gfx950's 32-deep BF16 MFMA: lane group g = l / 16 supplies 8 contracted
// indices of its row (A) or column (B); which 8 does not matter as long as both
// operands use the same ones.  The fused passes give it the two 16-deep groups
// of a pipeline stage: values j = 0..3 of the first group, then of the second.
__device__ inline s8_t cat8(const s4_t& lo, const s4_t& hi) {
  return s8_t{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}
__device__ inline f4_t mma32(const s8_t& a, const s8_t& b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b), c, 0, 0,
                                                 0);
}
// split BF16 with 32-deep operands (see mma_bf16x3)
__device__ inline f4_t mma32_x3(const s8_t& ahi, const s8_t& alo, const s8_t& bhi, const s8_t& blo, f4_t c) {
  c = mma32(alo, bhi, c);
  c = mma32(ahi, blo, c);
  return mma32(ahi, bhi, c);
}

// Operand layouts (checked on gfx950): A lane l holds row l%16, B lane l holds
// column l%16, both with contracted index KPL*(l/16) + j.  Result register r
// of lane l holds column l%16 and row 4*(l/16) + r for the f32 results, but
// row l/16 + 4*r for the f64 result (ROW_STRIDE4).
struct PF64 {
  using W = double;
  using acc = d4_t;
  static constexpr int KS = 4;
  static constexpr int KPL = 1;  // contracted-index values per lane per K-step
  static constexpr bool ROW_STRIDE4 = true;
  static constexpr bool SPLIT = false;
  static constexpr int ID = IGAFD_FP64;
};
struct PF32 {
  using W = float;
  using acc = f4_t;
  static constexpr int KS = 4;
  static constexpr int KPL = 1;
  static constexpr bool ROW_STRIDE4 = false;
  static constexpr bool SPLIT = false;
  static constexpr int ID = IGAFD_FP32;
};
struct PBF16 {
  using W = short;
  using acc = f4_t;
  static constexpr int KS = 16;
  static constexpr int KPL = 4;
  static constexpr bool ROW_STRIDE4 = false;
  static constexpr bool SPLIT = false;
  static constexpr int ID = IGAFD_BF16;
};
// split BF16: the matrices are read in FP32 and split per lane like the data
struct PBF16X3 {
  using W = float;
  using acc = f4_t;
  static constexpr int KS = 16;
  static constexpr int KPL = 4;
  static constexpr bool ROW_STRIDE4 = false;
  static constexpr bool SPLIT = true;
  static constexpr int ID = IGAFD_BF16X3;
};

enum { EPI_LAMBDA = 1, EPI_PRESCALE = 2, EPI_POSTSCALE = 4, EPI_DOT = 8 };

struct Epi {
  int flags;
  int dim;
  int n1;
  const double* lamK;   // eigenvalues of the contracted direction (output row k)
  const double* lam1;   // direction 1
  const double* lam2;   // direction 2 (3D)
  const double* S;      // diagonal scaling (PRESCALE / POSTSCALE)
  const double* rdot;   // r for the (r, s) partial sums
  double* partial;
  const int* flag;      // CG stop flag: nonzero -> the launch is a no-op
};

template <class Pr>
__device__ inline typename Pr::acc mfma(const typename Pr::W* a, const float* bf, const double* bd,
                                        typename Pr::acc c);

template <>
__device__ inline d4_t mfma<PF64>(const double* a, const float*, const double* bd, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], bd[0], c, 0, 0, 0);
}
template <>
__device__ inline f4_t mfma<PF32>(const float* a, const float* bf, const double*, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], bf[0], c, 0, 0, 0);
}
template <>
__device__ inline f4_t mfma<PBF16>(const short* a, const float* bf, const double*, f4_t c) {
  s4_t av = {a[0], a[1], a[2], a[3]};
  s4_t bv = {to_bf16(bf[0]), to_bf16(bf[1]), to_bf16(bf[2]), to_bf16(bf[3])};
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
}
template <>
__device__ inline f4_t mfma<PBF16X3>(const float* a, const float* bf, const double*, f4_t c) {
  s4_t ahi, alo, bhi, blo;
  split4(a, ahi, alo);
  split4(bf, bhi, blo);
  return mma_bf16x3(ahi, alo, bhi, blo, c);
}

// D[k][c] = sum_i Wm[k][i] X(i, c) for k in this block's row range and the
// wave's 16 columns.  TRX: X(i, c) = X[c * ldx + i] and D -> Y[c * ldy + k]
// (ldx = ldy = n for a whole grid; larger for a sub-block of a wider grid);
// otherwise X(i, c) = X[b * bstride + i * C + c] and D -> Y[b * bstride + k * C + c].
//
// Block order: the nblk row blocks of one 64-column group run on the same XCD
// (blocks are dealt to the 8 XCDs round robin), so the input tile they share
// is read into one L2.  Operands of UNR K-steps are loaded before their MFMAs.
template <class Pr, int MT, bool TRX, typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_mode(const Tin* __restrict__ X, Tout* __restrict__ Y,
                                                 const typename Pr::W* __restrict__ Wm, int npad, int n, int C,
                                                 long long bstride, int nblk, int ncolblk, int ngroups, Epi ep,
                                                 int ldx, int ldy) {
  using acc_t = typename Pr::acc;
  constexpr int KS = Pr::KS, KPL = Pr::KPL;
  constexpr int UNR = 4;
  if (ep.flag && *ep.flag) return;
  // work item (batch b, column block cb, row block rb); the row blocks of one
  // (b, cb) group share their input tile and go to the same XCD
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int rb = slot % nblk, group = (slot / nblk) * 8 + xcd;
  if (group >= ngroups) {  // idle block of the XCD-rounded grid
    if ((ep.flags & EPI_DOT) && threadIdx.x == 0) ep.partial[blockIdx.x] = 0.0;
    return;
  }
  const int cb = group % ncolblk;
  const long long bidx = group / ncolblk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int c0 = (cb * (kBlock / 64) + wave) * 16;
  const int k0 = rb * MT * 16;
  const long long boff = bidx * bstride;
  const int c = c0 + col;
  const bool cok = c < C;

  acc_t accv[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) accv[t] = acc_t{0, 0, 0, 0};

  if (c0 < C) {
    const typename Pr::W* wbase = Wm + (long long)(k0 + col) * npad + grp * KPL;
    for (int i0 = 0; i0 < n; i0 += UNR * KS) {
      float bf[UNR][KPL];
      double bd[UNR][KPL];
      typename Pr::W a[UNR][MT][KPL];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
          const int i = i0 + u * KS + grp * KPL + j;
          double v = 0.0;
          if (cok && i < n) {
            const long long addr = TRX ? (long long)c * ldx + i : boff + (long long)i * C + c;
            v = (double)X[addr];
            if (ep.flags & EPI_PRESCALE) v *= ep.S[addr];
          }
          bd[u][j] = v;
          bf[u][j] = (float)v;
        }
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
          for (int j = 0; j < KPL; ++j)
            // rows k0 + t*16 + col < npad and columns < npad: W is zero padded
            a[u][t][j] = (i0 + u * KS < npad) ? wbase[(long long)t * 16 * npad + i0 + u * KS + j] : 0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int t = 0; t < MT; ++t) accv[t] = mfma<Pr>(a[u][t], bf[u], bd[u], accv[t]);
    }
  }

  double dot = 0.0;
#pragma unroll
  for (int t = 0; t < MT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = k0 + t * 16 + (Pr::ROW_STRIDE4 ? grp + 4 * r : grp * 4 + r);
      if (k < n && cok) {
        double v = (double)accv[t][r];
        const long long addr = TRX ? (long long)c * ldy + k : boff + (long long)k * C + c;
        if (ep.flags & EPI_LAMBDA) {
          const double ls = ep.dim == 3 ? ep.lamK[k] + ep.lam2[c / ep.n1] + ep.lam1[c % ep.n1]
                                        : ep.lamK[k] + ep.lam1[c];
          v = v / ls;
        }
        if (ep.flags & EPI_POSTSCALE) v *= ep.S[addr];
        Y[addr] = (Tout)v;
        if (ep.flags & EPI_DOT) dot += ep.rdot[addr] * v;
      }
    }
  }
  if (ep.flags & EPI_DOT) {
    const double s = block_sum(dot);
    if (threadIdx.x == 0) ep.partial[blockIdx.x] = s;
  }
}

struct ModeShape {
  int nblk, mt;
};

// mt_max: row tiles per wave (fewer -> more waves, less reuse of each input tile)
ModeShape mode_shape(int n, int mt_max) {
  const int ntiles = (n + 15) / 16;
  int mt = mt_max < 1 ? 1 : (mt_max > 8 ? 8 : mt_max);
  if (mt > ntiles) mt = ntiles;
  const int nblk = (ntiles + mt - 1) / mt;
  return {nblk, mt};
}

int grid_x(int C, int B, int nblk) {
  const int ngroups = B * ((C + 63) / 64);
  return 8 * nblk * ((ngroups + 7) / 8);
}

template <class Pr, bool TRX, typename Tin, typename Tout>
igafd_status launch_mode(hipStream_t st, int mt_max, const Tin* X, Tout* Y, const typename Pr::W* Wm, int npad, int n,
                         int C, int B, long long bstride, const Epi& ep, int ldx = 0, int ldy = 0) {
  const ModeShape ms = mode_shape(n, mt_max);
  if (ldx <= 0) ldx = n;
  if (ldy <= 0) ldy = n;
  const int ncolblk = (C + 63) / 64;
  const dim3 grid((unsigned)grid_x(C, B, ms.nblk), 1, 1);
  switch (ms.mt) {
#define IGAFD_MT(M)                                                                                    \
  case M:                                                                                              \
    hipLaunchKernelGGL((k_mode<Pr, M, TRX, Tin, Tout>), grid, dim3(kBlock), 0, st, X, Y, Wm, npad, n, C, \
                       bstride, ms.nblk, ncolblk, B * ncolblk, ep, ldx, ldy);                          \
    break;
    IGAFD_MT(1) IGAFD_MT(2) IGAFD_MT(3) IGAFD_MT(4) IGAFD_MT(5) IGAFD_MT(6) IGAFD_MT(7) IGAFD_MT(8)
#undef IGAFD_MT
    default:
      set_error("internal: bad mode tile count");
      return IGAFD_ERR_ARG;
  }
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

// ------------------------------------------------------------------------
// Fused 3D passes.  The mode products of different directions commute, so
// the apply is done in three passes over the tensor instead of six:
//   A  per i3 slice X (n2 x n1):  Y = V2 (X V1^T)       directions 1, 2 forward
//   B  per group of columns c = (i2, i1) of the (n3 x n1 n2) view:
//      Z = W3b ((W3f X) / (lam1 + lam2 + lam3))       direction 3 and the scaling
//   C  as A with the backward matrices                directions 1, 2 backward
// The intermediate of each pass stays in LDS; the small matrices are read
// from L2; every input element is read once per pass and every output written
// once, so a pass moves 2 N values instead of the 4 N of two separate
// products.
// ------------------------------------------------------------------------

// Operands of one 16-wide group of the contracted index for one lane: the
// four consecutive indices k + 4g .. k + 4g + 3 (g = lane / 16), fetched with
// 16- or 32-byte loads.  FP64 and FP32 feed value s of every lane to the s-th
// of four 16x16x4 MFMAs (the same permutation of the contracted index on
// both operands, so the sum is the same); BF16 packs the four values into
// one 16x16x16 operand.
template <class Pr>
struct Grp;
template <>
struct Grp<PF64> {
  using V = double;
  static constexpr int G = 1;  // groups per pipeline stage
};
template <>
struct Grp<PF32> {
  using V = float;
  static constexpr int G = 2;
};
template <>
struct Grp<PBF16> {
  using V = float;
  static constexpr int G = 2;
};
template <>
struct Grp<PBF16X3> {
  using V = float;
  static constexpr int G = 2;
};

typedef double d2u_t __attribute__((ext_vector_type(2), aligned(8)));
typedef float f4u_t __attribute__((ext_vector_type(4), aligned(4)));

// four consecutive values (8-byte / 4-byte aligned), converted to V
template <typename V>
__device__ inline void ld4(const double* p, V (&o)[4]) {
  const d2u_t u = *reinterpret_cast<const d2u_t*>(p), w = *reinterpret_cast<const d2u_t*>(p + 2);
  o[0] = (V)u.x;
  o[1] = (V)u.y;
  o[2] = (V)w.x;
  o[3] = (V)w.y;
}
template <typename V>
__device__ inline void ld4(const float* p, V (&o)[4]) {
  const f4u_t u = *reinterpret_cast<const f4u_t*>(p);
  o[0] = (V)u.x;
  o[1] = (V)u.y;
  o[2] = (V)u.z;
  o[3] = (V)u.w;
}
// the first `valid` of four values, zeros after
template <typename T, typename V>
__device__ inline void ld4_tail(const T* p, int valid, V (&o)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) o[j] = j < valid ? (V)p[j] : V(0);
}

template <class Pr>
__device__ inline void grp_mma(const typename Grp<Pr>::V (&a)[4], const typename Grp<Pr>::V (&b)[4],
                               typename Pr::acc& c);
template <>
__device__ inline void grp_mma<PF64>(const double (&a)[4], const double (&b)[4], d4_t& c) {
#pragma unroll
  for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], c, 0, 0, 0);
}
template <>
__device__ inline void grp_mma<PF32>(const float (&a)[4], const float (&b)[4], f4_t& c) {
#pragma unroll
  for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
}

template <class Pr>
__device__ inline int row_of(int grp, int r) {
  return Pr::ROW_STRIDE4 ? grp + 4 * r : 4 * grp + r;
}

// output columns (k1) per slice block: 16 NT with NT = 2 or 3 column tiles,
// whichever pads the direction-1 tiles least (ties: 3, fewer blocks reload the
// matrices): n = 129 (9 tiles) takes 48, n = 99 (7) and n = 114 (8) take 32
__host__ __device__ constexpr int slice_nt(int n1) {
  const int tiles = (n1 + 15) / 16;
  return ((tiles + 2) / 3) * 3 <= ((tiles + 1) / 2) * 2 ? 3 : 2;
}
constexpr int kDir3Cols = 32;   // columns (i2, i1) per direction-3 block
// waves per block of the fused passes; a direction of up to 160 (10 row
// tiles of 16) gives each wave at most kMaxTilesPerWave tiles
constexpr int kFusedWaves = 4;
constexpr int kFusedThreads = 64 * kFusedWaves;
constexpr int kMaxTilesPerWave = (10 + kFusedWaves - 1) / kFusedWaves;
static_assert(kFusedWaves * kMaxTilesPerWave >= 10, "row-tile slots");

// row length of the transposed LDS tile (a multiple of 16 bytes)
template <typename T>
__host__ __device__ inline int lds_ld(int mtiles) {
  return mtiles * 16 + 16 / (int)sizeof(T);
}

// Two chained contractions D = A2 (A1 B1) over a 48- or 32-column group:
// the generic body of the fused passes.  loadA1(k, tile, v[4]) /
// loadB1(k, t, v[4]) fill the four values at contracted indices k..k+3 (k a
// multiple of 4, k < K1 rounded up to 16; values past K1 must be zero on at
// least one side).  The step-1 tile goes through LDS transposed (column c of
// the block holds its rows contiguously, so step 2 reads 16-byte vectors),
// rescaled on the way by `mid`.  Operand loads are double buffered: while the
// MFMAs of one stage run, the loads of the next are in flight.
template <class Pr, int NT, bool SYNC_MID, typename Tmid, typename A1, typename B1, typename Mid, typename A2>
__device__ inline void two_step(typename Pr::acc (&acc)[kMaxTilesPerWave][NT], int K1, int K2, int mtiles, int wave,
                                int grp, int col, Tmid* sT, int ldt, A1 loadA1, B1 loadB1, Mid mid, A2 loadA2) {
  using acc_t = typename Pr::acc;
  using V = typename Grp<Pr>::V;
  constexpr int G = Grp<Pr>::G, STEP = 16 * G, MT = kMaxTilesPerWave;
  V av[2][G][MT][4], bv[2][G][NT][4];
  auto zero4 = [](V (&v)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = V(0);
  };
  auto load1 = [&](int k0, V (&a)[G][MT][4], V (&b)[G][NT][4]) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int k = k0 + 16 * u + 4 * grp;
      const bool on = k0 + 16 * u < K1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (on)
          loadB1(k, t, b[u][t]);
        else
          zero4(b[u][t]);
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        if (on && wave + kFusedWaves * m < mtiles)
          loadA1(k, wave + kFusedWaves * m, a[u][m]);
        else
          zero4(a[u][m]);
      }
    }
  };
  auto load2 = [&](int k0, V (&a)[G][MT][4], V (&b)[G][NT][4]) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int k = k0 + 16 * u + 4 * grp;
      const bool on = k0 + 16 * u < K2;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (on)
          ld4(sT + (t * 16 + col) * ldt + k, b[u][t]);
        else
          zero4(b[u][t]);
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        if (on && wave + kFusedWaves * m < mtiles)
          loadA2(k, wave + kFusedWaves * m, a[u][m]);
        else
          zero4(a[u][m]);
      }
    }
  };
  auto compute = [&](int k0, int K, V (&a)[G][MT][4], V (&b)[G][NT][4]) {
    if constexpr (Pr::KPL != 1) {
      // BF16 and split BF16: both 16-deep groups of the stage in one 32-deep
      // MFMA (a second group past K was loaded as zeros)
      static_assert(G == 2, "32-deep BF16 products take two 16-deep groups");
      auto bf4 = [](const V (&v)[4]) { return s4_t{to_bf16(v[0]), to_bf16(v[1]), to_bf16(v[2]), to_bf16(v[3])}; };
      if constexpr (Pr::SPLIT) {
        s8_t pa[MT], la[MT], pb[NT], lb[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          s4_t h0, l0, h1, l1;
          split4(a[0][m], h0, l0);
          split4(a[1][m], h1, l1);
          pa[m] = cat8(h0, h1);
          la[m] = cat8(l0, l1);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          s4_t h0, l0, h1, l1;
          split4(b[0][t], h0, l0);
          split4(b[1][t], h1, l1);
          pb[t] = cat8(h0, h1);
          lb[t] = cat8(l0, l1);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m)
          if (wave + kFusedWaves * m < mtiles) {
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mma32_x3(pa[m], la[m], pb[t], lb[t], acc[m][t]);
          }
      } else {
        s8_t pa[MT], pb[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) pa[m] = cat8(bf4(a[0][m]), bf4(a[1][m]));
#pragma unroll
        for (int t = 0; t < NT; ++t) pb[t] = cat8(bf4(b[0][t]), bf4(b[1][t]));
#pragma unroll
        for (int m = 0; m < MT; ++m)
          if (wave + kFusedWaves * m < mtiles) {
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] = mma32(pa[m], pb[t], acc[m][t]);
          }
      }
    } else {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (k0 + 16 * u >= K) break;
#pragma unroll
        for (int m = 0; m < MT; ++m)
          if (wave + kFusedWaves * m < mtiles) {
#pragma unroll
            for (int t = 0; t < NT; ++t) grp_mma<Pr>(a[u][m], b[u][t], acc[m][t]);
          }
      }
    }
  };
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = acc_t{0, 0, 0, 0};
  // step 1
  load1(0, av[0], bv[0]);
  for (int k0 = 0; k0 < K1; k0 += 2 * STEP) {
    if (k0 + STEP < K1) load1(k0 + STEP, av[1], bv[1]);
    compute(k0, K1, av[0], bv[0]);
    if (k0 + 2 * STEP < K1) load1(k0 + 2 * STEP, av[0], bv[0]);
    if (k0 + STEP < K1) compute(k0 + STEP, K1, av[1], bv[1]);
  }
  // intermediate tile to LDS, transposed (rows past the problem hold zeros);
  // SYNC_MID: step 1 read its B operand from the same LDS area
  if (SYNC_MID) __syncthreads();
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int mt = wave + kFusedWaves * m;
    if (mt >= mtiles) break;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mt * 16 + row_of<Pr>(grp, r);
        sT[(t * 16 + col) * ldt + row] = (Tmid)mid(row, t, (double)acc[m][t][r]);
      }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = acc_t{0, 0, 0, 0};
  // step 2: K2 rows of the LDS tile
  load2(0, av[0], bv[0]);
  for (int k0 = 0; k0 < K2; k0 += 2 * STEP) {
    if (k0 + STEP < K2) load2(k0 + STEP, av[1], bv[1]);
    compute(k0, K2, av[0], bv[0]);
    if (k0 + 2 * STEP < K2) load2(k0 + 2 * STEP, av[0], bv[0]);
    if (k0 + STEP < K2) compute(k0 + STEP, K2, av[1], bv[1]);
  }
}

// Pass A / C: Out[i2][k1] = sum_j2 V2[i2][j2] sum_i1 X[j2][i1] V1[k1][i1] for
// slice blockIdx.y and output columns k1 in [blockIdx.x * 16 NT, +16 NT).  X, Out:
// slice-contiguous (n2 x n1); V1, V2 row-major, zero padded to npad1, npad2.
template <class Pr, int NT, typename Tin, typename Tout, typename Tw, typename Tmid>
__device__ __forceinline__ void slice_body(const Tin* __restrict__ X, Tout* __restrict__ Out,
                                           const Tw* __restrict__ V1, const Tw* __restrict__ V2, int n1, int n2,
                                           int npad1, int npad2, const Epi& ep, int bx, int by, int gx) {
  using acc_t = typename Pr::acc;
  using V = typename Grp<Pr>::V;
  constexpr int kSliceCols = 16 * NT;
  extern __shared__ char smem_raw[];
  Tmid* sT = reinterpret_cast<Tmid*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int mtiles = (n2 + 15) / 16;
  const int ldt = lds_ld<Tmid>(mtiles);
  const int cb = bx;
  const long long sbase = (long long)by * n1 * n2;
  const Tin* Xs = X + sbase;
  acc_t acc[kMaxTilesPerWave][NT];
  // step 1: A = X (rows j2, contracted i1), B = V1^T (contracted i1, columns k1)
  auto loadA1 = [&](int i1, int mt, V (&v)[4]) {
    const int j2 = mt * 16 + col;
    if (j2 >= n2) {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = V(0);
      return;
    }
    const long long addr = (long long)j2 * n1 + i1;
    if (i1 + 4 <= n1)
      ld4(Xs + addr, v);
    else
      ld4_tail(Xs + addr, n1 - i1, v);
    if (ep.flags & EPI_PRESCALE) {
      V s[4];
      if (i1 + 4 <= n1)
        ld4(ep.S + sbase + addr, s);
      else
        ld4_tail(ep.S + sbase + addr, n1 - i1, s);
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (V)((double)v[j] * (double)s[j]);
    }
  };
  auto loadB1 = [&](int i1, int t, V (&v)[4]) {
    const int k1 = cb * kSliceCols + t * 16 + col;
    if (k1 < n1) {
      ld4(V1 + (long long)k1 * npad1 + i1, v);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = V(0);
    }
  };
  auto mid = [&](int, int, double v) { return v; };
  // step 2: A = V2 (rows i2, contracted j2), B = the LDS tile
  auto loadA2 = [&](int j2, int mt, V (&v)[4]) { ld4(V2 + (long long)(mt * 16 + col) * npad2 + j2, v); };
  two_step<Pr, NT, false>(acc, n1, n2, mtiles, wave, grp, col, sT, ldt, loadA1, loadB1, mid, loadA2);
  double dot = 0.0;
#pragma unroll
  for (int m = 0; m < kMaxTilesPerWave; ++m) {
    const int mt = wave + kFusedWaves * m;
    if (mt >= mtiles) break;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i2 = mt * 16 + row_of<Pr>(grp, r);
        const int k1 = cb * kSliceCols + t * 16 + col;
        if (i2 < n2 && k1 < n1) {
          const long long addr = sbase + (long long)i2 * n1 + k1;
          double v = (double)acc[m][t][r];
          if (ep.flags & EPI_POSTSCALE) v *= ep.S[addr];
          Out[addr] = (Tout)v;
          if (ep.flags & EPI_DOT) dot += ep.rdot[addr] * v;
        }
      }
  }
  if (ep.flags & EPI_DOT) {
    const double sum = block_sum<kFusedThreads>(dot);
    if (threadIdx.x == 0) ep.partial[bx + (long long)gx * by] = sum;
  }
}

template <class Pr, int NT, typename Tin, typename Tout, typename Tw, typename Tmid>
__global__ __launch_bounds__(kFusedThreads) void k_slice(const Tin* __restrict__ X, Tout* __restrict__ Out,
                                                  const Tw* __restrict__ V1, const Tw* __restrict__ V2, int n1, int n2,
                                                  int npad1, int npad2, Epi ep) {
  if (ep.flag && *ep.flag) return;
  slice_body<Pr, NT, Tin, Tout, Tw, Tmid>(X, Out, V1, V2, n1, n2, npad1, npad2, ep, (int)blockIdx.x, (int)blockIdx.y,
                                          (int)gridDim.x);
}

// Grouped form of a slice pass (several problems in one launch): job j owns
// blocks [start[j], start[j+1]), gx column blocks per slice.
template <typename Tin, typename Tout, typename Tw>
struct SliceJob {
  const Tin* X;
  Tout* Out;
  const Tw* V1;
  const Tw* V2;
  int n1, n2, npad1, npad2, gx;
  Epi ep;
};

template <class Pr, int NT, typename Tin, typename Tout, typename Tw, typename Tmid>
__global__ __launch_bounds__(kFusedThreads) void k_slice_g(const SliceJob<Tin, Tout, Tw>* __restrict__ jobs,
                                                    const int* __restrict__ start, int njobs) {
  const int j = group_job(start, njobs, (int)blockIdx.x);
  const SliceJob<Tin, Tout, Tw>& t = jobs[j];
  if (t.ep.flag && *t.ep.flag) return;
  const int local = (int)blockIdx.x - start[j];
  slice_body<Pr, NT, Tin, Tout, Tw, Tmid>(t.X, t.Out, t.V1, t.V2, t.n1, t.n2, t.npad1, t.npad2, t.ep, local % t.gx,
                                          local / t.gx, t.gx);
}

// Pass B: Out[i3][c] = sum_k3 Wb[i3][k3] (sum_j3 Wf[k3][j3] X[j3][c]) / lamsum(k3, c)
// for the 32 columns c of block blockIdx.x (c = i2 n1 + i1, C = n1 n2).
template <class Pr, typename Tw, typename Tmid>
__device__ __forceinline__ void dir3_body(const Tmid* __restrict__ X, Tmid* __restrict__ Out,
                                          const Tw* __restrict__ Wf, const Tw* __restrict__ Wb, int n3, int C,
                                          int npad3, const Epi& ep, int bx) {
  using acc_t = typename Pr::acc;
  using V = typename Grp<Pr>::V;
  constexpr int NT = kDir3Cols / 16;
  extern __shared__ char smem_raw[];
  Tmid* sT = reinterpret_cast<Tmid*>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int mtiles = (n3 + 15) / 16;
  const int ldt = lds_ld<Tmid>(mtiles);
  const int c0 = bx * kDir3Cols;
  acc_t acc[kMaxTilesPerWave][NT];
  // the block's 32 input columns, staged transposed in LDS (column c holds its
  // n3 values contiguously, zeros up to the padded height) with 16-byte
  // loads along the rows; the step-1 B operand is read from there
  {
    constexpr int VEC = 16 / (int)sizeof(Tmid), PER_ROW = kDir3Cols / VEC;
    const int rows = mtiles * 16;
    for (int idx = threadIdx.x; idx < rows * PER_ROW; idx += kFusedThreads) {
      const int j3 = idx / PER_ROW, cq = (idx - j3 * PER_ROW) * VEC;
      const int c = c0 + cq;
      Tmid v[VEC];
      if (j3 < n3 && c + VEC <= C) {
        const Tmid* src = X + (long long)j3 * C + c;
        if constexpr (VEC == 2) {
          const d2u_t u = *reinterpret_cast<const d2u_t*>(src);
          v[0] = u.x;
          v[1] = u.y;
        } else {
          const f4u_t u = *reinterpret_cast<const f4u_t*>(src);
          v[0] = u.x;
          v[1] = u.y;
          v[2] = u.z;
          v[3] = u.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < VEC; ++j) v[j] = (j3 < n3 && c + j < C) ? X[(long long)j3 * C + c + j] : Tmid(0);
      }
#pragma unroll
      for (int j = 0; j < VEC; ++j) sT[(cq + j) * ldt + j3] = v[j];
    }
    __syncthreads();
  }
  // step 1: A = Wf (rows k3, contracted j3), B = X (contracted j3, columns c)
  auto loadA1 = [&](int j3, int mt, V (&v)[4]) { ld4(Wf + (long long)(mt * 16 + col) * npad3 + j3, v); };
  auto loadB1 = [&](int j3, int t, V (&v)[4]) { ld4(sT + (t * 16 + col) * ldt + j3, v); };
  // scaling by the eigenvalue sums between the two contractions
  auto mid = [&](int k3, int t, double v) -> double {
    const int c = c0 + t * 16 + col;
    return (k3 < n3 && c < C) ? v / (ep.lamK[k3] + ep.lam2[c / ep.n1] + ep.lam1[c % ep.n1]) : 0.0;
  };
  auto loadA2 = [&](int k3, int mt, V (&v)[4]) { ld4(Wb + (long long)(mt * 16 + col) * npad3 + k3, v); };
  two_step<Pr, NT, true>(acc, n3, n3, mtiles, wave, grp, col, sT, ldt, loadA1, loadB1, mid, loadA2);
#pragma unroll
  for (int m = 0; m < kMaxTilesPerWave; ++m) {
    const int mt = wave + kFusedWaves * m;
    if (mt >= mtiles) break;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i3 = mt * 16 + row_of<Pr>(grp, r);
        const int c = c0 + t * 16 + col;
        if (i3 < n3 && c < C) Out[(long long)i3 * C + c] = (Tmid)acc[m][t][r];
      }
  }
}

template <class Pr, typename Tw, typename Tmid>
__global__ __launch_bounds__(kFusedThreads) void k_dir3(const Tmid* __restrict__ X, Tmid* __restrict__ Out,
                                                 const Tw* __restrict__ Wf, const Tw* __restrict__ Wb, int n3, int C,
                                                 int npad3, Epi ep) {
  if (ep.flag && *ep.flag) return;
  dir3_body<Pr, Tw, Tmid>(X, Out, Wf, Wb, n3, C, npad3, ep, (int)blockIdx.x);
}

template <typename Tw, typename Tmid>
struct Dir3Job {
  const Tmid* X;
  Tmid* Out;
  const Tw* Wf;
  const Tw* Wb;
  int n3, C, npad3;
  Epi ep;
};

template <class Pr, typename Tw, typename Tmid>
__global__ __launch_bounds__(kFusedThreads) void k_dir3_g(const Dir3Job<Tw, Tmid>* __restrict__ jobs,
                                                   const int* __restrict__ start, int njobs) {
  const int j = group_job(start, njobs, (int)blockIdx.x);
  const Dir3Job<Tw, Tmid>& t = jobs[j];
  if (t.ep.flag && *t.ep.flag) return;
  dir3_body<Pr, Tw, Tmid>(t.X, t.Out, t.Wf, t.Wb, t.n3, t.C, t.npad3, t.ep, (int)blockIdx.x - start[j]);
}

// the fused path needs each direction's row tiles (at most 10) to fit the
// waves' tile slots and the LDS tile of a slice pass within 64 KB (n2 <= 160
// in FP64)
bool fused_ok(const igafd_ctx* c) {
  return c->dim == 3 && c->n[0] <= 160 && c->n[1] <= 160 && c->n[2] <= 160;
}

int slice_blocks(const igafd_ctx* c) {
  const int cols = 16 * slice_nt(c->n[0]);
  return ((c->n[0] + cols - 1) / cols) * c->n[2];
}

template <class Pr, typename T, typename Tw>
igafd_status apply_fused(igafd_ctx* c, const Tw* const* Wf, const Tw* const* Wb, const double* r, double* s,
                         const double* S, double* partial, const int* flag) {
  const DevDir* d = c->ddir;
  const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2];
  T* b0 = reinterpret_cast<T*>(c->fdbuf[0]);
  T* b1 = reinterpret_cast<T*>(c->fdbuf[1]);
  const hipStream_t st = c->stream;
  Epi e_in{}, e_lam{}, e_out{};
  e_in.flag = e_lam.flag = e_out.flag = flag;
  if (S) {
    e_in.flags |= EPI_PRESCALE;
    e_in.S = S;
    e_out.flags |= EPI_POSTSCALE;
    e_out.S = S;
  }
  if (partial) {
    if (slice_blocks(c) > c->npartial) {
      set_error("internal: FD grid larger than the partial-sum buffer");
      return IGAFD_ERR_ARG;
    }
    e_out.flags |= EPI_DOT;
    e_out.rdot = r;
    e_out.partial = partial;
  }
  e_lam.n1 = n1;
  e_lam.lamK = d[2].lam;
  e_lam.lam1 = d[0].lam;
  e_lam.lam2 = d[1].lam;
  const int nt = slice_nt(n1), cols = 16 * nt;
  const dim3 gs((unsigned)((n1 + cols - 1) / cols), (unsigned)n3);
  const size_t lds_s = sizeof(T) * (size_t)cols * lds_ld<T>((n2 + 15) / 16);
  const size_t lds_3 = sizeof(T) * (size_t)kDir3Cols * lds_ld<T>((n3 + 15) / 16);
  const int C = n1 * n2;
  if (nt == 3)
    hipLaunchKernelGGL((k_slice<Pr, 3, double, T, Tw, T>), gs, dim3(kFusedThreads), lds_s, st, r, b0, Wf[0], Wf[1], n1,
                       n2, d[0].npad, d[1].npad, e_in);
  else
    hipLaunchKernelGGL((k_slice<Pr, 2, double, T, Tw, T>), gs, dim3(kFusedThreads), lds_s, st, r, b0, Wf[0], Wf[1], n1,
                       n2, d[0].npad, d[1].npad, e_in);
  IGAFD_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_dir3<Pr, Tw, T>), dim3((unsigned)((C + kDir3Cols - 1) / kDir3Cols)), dim3(kFusedThreads), lds_3, st,
                     b0, b1, Wf[2], Wb[2], n3, C, d[2].npad, e_lam);
  IGAFD_HIP_CHECK(hipGetLastError());
  if (nt == 3)
    hipLaunchKernelGGL((k_slice<Pr, 3, T, double, Tw, T>), gs, dim3(kFusedThreads), lds_s, st, b1, s, Wb[0], Wb[1], n1,
                       n2, d[0].npad, d[1].npad, e_out);
  else
    hipLaunchKernelGGL((k_slice<Pr, 2, T, double, Tw, T>), gs, dim3(kFusedThreads), lds_s, st, b1, s, Wb[0], Wb[1], n1,
                       n2, d[0].npad, d[1].npad, e_out);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

template <class Pr>
const typename Pr::W* wmat(const DevDir& d, int which);
template <>
const double* wmat<PF64>(const DevDir& d, int which) { return d.W64[which]; }
template <>
const float* wmat<PF32>(const DevDir& d, int which) { return d.W32[which]; }
template <>
const short* wmat<PBF16>(const DevDir& d, int which) { return reinterpret_cast<const short*>(d.Wbf[which]); }
template <>
const float* wmat<PBF16X3>(const DevDir& d, int which) { return d.W32[which]; }

int dot_blocks_for(const igafd_ctx* c) {
  const ModeShape ms = mode_shape(c->n[0], c->fd_tiles);
  const int C = (c->dim == 3) ? c->n[1] * c->n[2] : c->n[1];
  return grid_x(C, 1, ms.nblk);
}

// Applies with long directions use the tiled products of gemm.hip (in every
// precision): 2D grids with n1 + n2 >= 384, 3D tensors with a direction
// longer than the fused passes take.  IGAFD_FD_GEMM=0/1 at setup forces the
// choice.
constexpr int kGemmAutoN = 384;
bool use_gemm(const igafd_ctx* c, int prec) {
  (void)prec;  // the same choice for every precision
  if (c->fd_gemm >= 0) return c->fd_gemm != 0;
  if (c->dim == 3) return !fused_ok(c);
  return c->n[0] + c->n[1] >= kGemmAutoN;
}

// T: intermediate type (double for FP64, float otherwise)
// ldr, lds (2D): row strides of r and s when they are sub-blocks of a wider
// grid (0: n1)
template <class Pr, typename T>
igafd_status apply(igafd_ctx* c, const double* r, double* s, const double* S, double* partial, const int* flag,
                   int ldr = 0, int lds = 0) {
  const DevDir* d = c->ddir;
  const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2];
  T* b0 = reinterpret_cast<T*>(c->fdbuf[0]);
  T* b1 = reinterpret_cast<T*>(c->fdbuf[1]);
  const hipStream_t st = c->stream;
  Epi e0{};
  e0.dim = c->dim;
  e0.n1 = n1;
  e0.lam1 = d[0].lam;
  e0.lam2 = d[1].lam;
  e0.flag = flag;
  Epi e_in = e0, e_lam = e0, e_out = e0;
  if (S) {
    e_in.flags |= EPI_PRESCALE;
    e_in.S = S;
    e_out.flags |= EPI_POSTSCALE;
    e_out.S = S;
  }
  if (partial) {
    if (dot_blocks_for(c) > c->npartial) {
      set_error("internal: FD grid larger than the partial-sum buffer");
      return IGAFD_ERR_ARG;
    }
    e_out.flags |= EPI_DOT;
    e_out.rdot = r;
    e_out.partial = partial;
  }
  e_lam.flags = EPI_LAMBDA;
  igafd_status stt;
#define IGAFD_TRY(x)           \
  if ((stt = (x)) != IGAFD_OK) \
    return stt;
  if (c->dim == 3) {
    {
      const int prec = Pr::ID;
      if (use_gemm(c, prec)) return fd_apply_gemm3d(c, prec, r, s, S, partial, flag);
    }
    // forward: direction 1 (fast axis), 2, 3 (+ eigenvalue scaling)
    IGAFD_TRY((launch_mode<Pr, true, double, T>(st, c->fd_tiles, r, b0, wmat<Pr>(d[0], 0), d[0].npad, n1, n2 * n3, 1, 0, e_in)));
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b0, b1, wmat<Pr>(d[1], 0), d[1].npad, n2, n1, n3,
                                             (long long)n1 * n2, e0)));
    e_lam.lamK = d[2].lam;
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b1, b0, wmat<Pr>(d[2], 0), d[2].npad, n3, n1 * n2, 1, 0, e_lam)));
    // backward: direction 3, 2, 1
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b0, b1, wmat<Pr>(d[2], 1), d[2].npad, n3, n1 * n2, 1, 0, e0)));
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b1, b0, wmat<Pr>(d[1], 1), d[1].npad, n2, n1, n3,
                                             (long long)n1 * n2, e0)));
    IGAFD_TRY((launch_mode<Pr, true, T, double>(st, c->fd_tiles, b0, s, wmat<Pr>(d[0], 1), d[0].npad, n1, n2 * n3, 1, 0, e_out)));
  } else {
    {
      const int prec = Pr::ID;
      if (use_gemm(c, prec)) return fd_apply_gemm2d(c, prec, r, s, S, partial, flag, ldr, lds);
    }
    IGAFD_TRY((launch_mode<Pr, true, double, T>(st, c->fd_tiles, r, b0, wmat<Pr>(d[0], 0), d[0].npad, n1, n2, 1, 0, e_in,
                                                 ldr, n1)));
    e_lam.lamK = d[1].lam;
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b0, b1, wmat<Pr>(d[1], 0), d[1].npad, n2, n1, 1, 0, e_lam)));
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b1, b0, wmat<Pr>(d[1], 1), d[1].npad, n2, n1, 1, 0, e0)));
    IGAFD_TRY((launch_mode<Pr, true, T, double>(st, c->fd_tiles, b0, s, wmat<Pr>(d[0], 1), d[0].npad, n1, n2, 1, 0, e_out,
                                                 n1, lds)));
  }
#undef IGAFD_TRY
  return IGAFD_OK;
}

// ------------------------------------------------------------------------
// Overlapping additive Schwarz on the L-shaped three-patch domain (Sec. 6
// eq. Pias with the local approximations P_i):
//   s = R_1^T P_1^-1 R_1 r + R_2^T P_2^-1 R_2 r.
// Vectors use the bounding square's n x n grid (direction 1 fastest) with the
// removed quarter i1, i2 >= h held at zero.  The subdomains are tensor
// sub-blocks of that grid:
//   Theta_2 = rows i2 < h (all i1): contiguous, an n x h grid;
//   Theta_1 = columns i1 < h of every row: an h x n grid of row stride n.
// P_2^-1 R_2 r is written straight into the first h rows of s, P_1^-1 R_1 r
// into t (h x n, contiguous); the combine pass adds them, zeroes the removed
// quarter and forms the (r, s) block partials.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_schwarz_combine(const double* __restrict__ t, double* __restrict__ s,
                                                            const double* __restrict__ r, int n, int h, long long N,
                                                            double* __restrict__ partial, const int* __restrict__ flag) {
  if (flag && *flag) return;
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  double dot = 0.0;
  if (i < N) {
    const int i1 = (int)(i % n), i2 = (int)(i / n);
    double v = i2 < h ? s[i] : 0.0;
    if (i1 < h) v += t[(long long)i2 * h + i1];
    s[i] = v;
    dot = r[i] * v;
  }
  if (partial) {
    const double sum = block_sum(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
  }
}

int schwarz_blocks(const igafd_ctx* c) { return (int)((c->N + kBlock - 1) / kBlock); }

template <class Pr, typename T>
igafd_status schwarz(igafd_ctx* c, const double* r, double* s, double* partial, const int* flag) {
  igafd_ctx* s1 = c->sub[0];
  igafd_ctx* s2 = c->sub[1];
  const int n = c->n[0], h = c->hole;
  if (!s1 || !s2 || c->dim != 2 || c->n[1] != n || s1->n[0] != h || s1->n[1] != n || s2->n[0] != n ||
      s2->n[1] != h) {
    set_error("internal: Schwarz subdomains do not match the L-shaped grid");
    return IGAFD_ERR_ARG;
  }
  if (partial && schwarz_blocks(c) > c->npartial) {
    set_error("internal: Schwarz grid larger than the partial-sum buffer");
    return IGAFD_ERR_ARG;
  }
  s1->fd_tiles = s2->fd_tiles = c->fd_tiles;
  igafd_status st;
  constexpr int prec = Pr::ID;
  if (use_gemm(s1, prec) && use_gemm(s2, prec)) {
    // both subdomain applies by tiled products, each pass of the two in one launch
    st = fd_apply_gemm2d_pair(prec, s2, r, n, s, n, s1, r, n, c->fdbuf[0], h, flag);
    if (st != IGAFD_OK) return st;
  } else {
    if ((st = apply<Pr, T>(s2, r, s, nullptr, nullptr, flag, n, n)) != IGAFD_OK) return st;
    if ((st = apply<Pr, T>(s1, r, c->fdbuf[0], nullptr, nullptr, flag, n, h)) != IGAFD_OK) return st;
  }
  hipLaunchKernelGGL(k_schwarz_combine, dim3((unsigned)schwarz_blocks(c)), dim3(kBlock), 0, c->stream, c->fdbuf[0], s,
                     r, n, h, c->N, partial, flag);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

igafd_status schwarz_apply(igafd_ctx* c, int prec, const double* r, double* s, const double* S, double* partial,
                           const int* flag) {
  if (S) {
    set_error("the scaled preconditioner is not defined for the L-shaped multi-patch problem");
    return IGAFD_ERR_ARG;
  }
  switch (prec) {
    case IGAFD_FP64:
      return schwarz<PF64, double>(c, r, s, partial, flag);
    case IGAFD_FP32:
      return schwarz<PF32, float>(c, r, s, partial, flag);
    case IGAFD_BF16:
      return schwarz<PBF16, float>(c, r, s, partial, flag);
    case IGAFD_BF16X3:
      return schwarz<PBF16X3, float>(c, r, s, partial, flag);
    default:
      set_error("unknown precision");
      return IGAFD_ERR_ARG;
  }
}

}  // namespace

bool fd_fused_ok(const igafd_ctx* c) { return fused_ok(c) && !use_gemm(c, IGAFD_FP64); }

int fd_dot_blocks(const igafd_ctx* c, int prec) {
  if (c->adi) return (int)((c->N + kBlock - 1) / kBlock);
  if (c->hole >= 0) return schwarz_blocks(c);
  if (use_gemm(c, prec)) return fd_gemm_blocks(c);
  return (c->fd_fused && fused_ok(c)) ? slice_blocks(c) : dot_blocks_for(c);
}

int fd_dot_blocks_max(const igafd_ctx* c) {
  const int C = (c->dim == 3) ? c->n[1] * c->n[2] : c->n[1];
  int m = std::max(slice_blocks(c), schwarz_blocks(c));
  m = std::max(m, fd_gemm_blocks(c));
  for (int t = 1; t <= 8; ++t) {
    const int g = grid_x(C, 1, mode_shape(c->n[0], t).nblk);
    if (g > m) m = g;
  }
  return m;
}

igafd_status fd_apply(igafd_ctx* c, int prec, const double* r, double* s, const double* S, double* partial,
                      const int* flag) {
  if (c->adi) return adi_apply(c, prec, r, s, S, partial, flag);
  if (c->hole >= 0) return schwarz_apply(c, prec, r, s, S, partial, flag);
  if (c->fd_fused && fused_ok(c) && !use_gemm(c, prec)) {
    const DevDir* d = c->ddir;
    switch (prec) {
      case IGAFD_FP64: {
        const double* Wf[3] = {d[0].W64[0], d[1].W64[0], d[2].W64[0]};
        const double* Wb[3] = {d[0].W64[1], d[1].W64[1], d[2].W64[1]};
        return apply_fused<PF64, double, double>(c, Wf, Wb, r, s, S, partial, flag);
      }
      case IGAFD_FP32:
      case IGAFD_BF16:
      case IGAFD_BF16X3: {
        const float* Wf[3] = {d[0].W32[0], d[1].W32[0], d[2].W32[0]};
        const float* Wb[3] = {d[0].W32[1], d[1].W32[1], d[2].W32[1]};
        if (prec == IGAFD_FP32) return apply_fused<PF32, float, float>(c, Wf, Wb, r, s, S, partial, flag);
        if (prec == IGAFD_BF16) return apply_fused<PBF16, float, float>(c, Wf, Wb, r, s, S, partial, flag);
        return apply_fused<PBF16X3, float, float>(c, Wf, Wb, r, s, S, partial, flag);
      }
      default:
        break;
    }
  }
  switch (prec) {
    case IGAFD_FP64:
      return apply<PF64, double>(c, r, s, S, partial, flag);
    case IGAFD_FP32:
      return apply<PF32, float>(c, r, s, S, partial, flag);
    case IGAFD_BF16:
      return apply<PBF16, float>(c, r, s, S, partial, flag);
    case IGAFD_BF16X3:
      return apply<PBF16X3, float>(c, r, s, S, partial, flag);
    default:
      set_error("unknown precision");
      return IGAFD_ERR_ARG;
  }
}

// ---- grouped FD applies (batched solves) ----

namespace {

template <class Pr, int NT, typename Tin, typename Tout, typename Tw, typename Tmid>
igafd_status slice_g_launch(const GroupArena& a, size_t oj, size_t os, int nj, int blocks, size_t lds,
                            hipStream_t st) {
  hipLaunchKernelGGL((k_slice_g<Pr, NT, Tin, Tout, Tw, Tmid>), dim3((unsigned)blocks), dim3(kFusedThreads), lds, st,
                     a.at<SliceJob<Tin, Tout, Tw>>(oj), a.at<int>(os), nj);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

// one slice pass for every problem: a launch per column-block width
template <class Pr, typename Tin, typename Tout, typename Tw, typename Tmid>
void slice_pass_g(GroupArena& a, std::vector<GroupStep>& steps, const std::vector<igafd_ctx*>& cs,
                  const std::vector<SliceJob<Tin, Tout, Tw>>& jobs) {
  for (int nt : {3, 2}) {
    std::vector<SliceJob<Tin, Tout, Tw>> jj;
    std::vector<int> start(1, 0);
    size_t lds = 0;
    for (size_t i = 0; i < cs.size(); ++i) {
      const igafd_ctx* c = cs[i];
      if (slice_nt(c->n[0]) != nt) continue;
      jj.push_back(jobs[i]);
      start.push_back(start.back() + jobs[i].gx * c->n[2]);
      lds = std::max(lds, sizeof(Tmid) * (size_t)(16 * nt) * lds_ld<Tmid>((c->n[1] + 15) / 16));
    }
    if (jj.empty()) continue;
    const size_t oj = a.push(jj.data(), sizeof(jj[0]) * jj.size());
    const size_t os = a.push(start.data(), sizeof(int) * start.size());
    const int nj = (int)jj.size(), blocks = start.back();
    if (nt == 3)
      steps.push_back([&a, oj, os, nj, blocks, lds](hipStream_t st) {
        return slice_g_launch<Pr, 3, Tin, Tout, Tw, Tmid>(a, oj, os, nj, blocks, lds, st);
      });
    else
      steps.push_back([&a, oj, os, nj, blocks, lds](hipStream_t st) {
        return slice_g_launch<Pr, 2, Tin, Tout, Tw, Tmid>(a, oj, os, nj, blocks, lds, st);
      });
  }
}

template <class Pr, typename T, typename Tw>
igafd_status fused_g(GroupArena& a, std::vector<GroupStep>& steps, const std::vector<igafd_ctx*>& cs,
                     const std::vector<const double*>& r, const std::vector<double*>& s,
                     const std::vector<const double*>& S, const std::vector<double*>& partial) {
  const int n = (int)cs.size();
  std::vector<SliceJob<double, T, Tw>> ja(n);
  std::vector<SliceJob<T, double, Tw>> jc(n);
  std::vector<Dir3Job<Tw, T>> jb(n);
  std::vector<int> start3(1, 0);
  size_t lds3 = 0;
  for (int i = 0; i < n; ++i) {
    igafd_ctx* c = cs[i];
    const DevDir* d = c->ddir;
    const Tw* Wf[3];
    const Tw* Wb[3];
    for (int l = 0; l < 3; ++l) {
      if constexpr (std::is_same<Tw, double>::value) {
        Wf[l] = d[l].W64[0];
        Wb[l] = d[l].W64[1];
      } else {
        Wf[l] = d[l].W32[0];
        Wb[l] = d[l].W32[1];
      }
    }
    const int n1 = c->n[0], n2 = c->n[1], n3 = c->n[2];
    T* b0 = reinterpret_cast<T*>(c->fdbuf[0]);
    T* b1 = reinterpret_cast<T*>(c->fdbuf[1]);
    const int* flag = &c->state->flag;
    Epi e_in{}, e_lam{}, e_out{};
    e_in.flag = e_lam.flag = e_out.flag = flag;
    if (S[i]) {
      e_in.flags |= EPI_PRESCALE;
      e_in.S = S[i];
      e_out.flags |= EPI_POSTSCALE;
      e_out.S = S[i];
    }
    if (partial[i]) {
      if (slice_blocks(c) > c->npartial) {
        set_error("internal: FD grid larger than the partial-sum buffer");
        return IGAFD_ERR_ARG;
      }
      e_out.flags |= EPI_DOT;
      e_out.rdot = r[i];
      e_out.partial = partial[i];
    }
    e_lam.n1 = n1;
    e_lam.lamK = d[2].lam;
    e_lam.lam1 = d[0].lam;
    e_lam.lam2 = d[1].lam;
    const int cols = 16 * slice_nt(n1), gx = (n1 + cols - 1) / cols, C = n1 * n2;
    ja[i] = SliceJob<double, T, Tw>{r[i], b0, Wf[0], Wf[1], n1, n2, d[0].npad, d[1].npad, gx, e_in};
    jb[i] = Dir3Job<Tw, T>{b0, b1, Wf[2], Wb[2], n3, C, d[2].npad, e_lam};
    jc[i] = SliceJob<T, double, Tw>{b1, s[i], Wb[0], Wb[1], n1, n2, d[0].npad, d[1].npad, gx, e_out};
    start3.push_back(start3.back() + (C + kDir3Cols - 1) / kDir3Cols);
    lds3 = std::max(lds3, sizeof(T) * (size_t)kDir3Cols * lds_ld<T>((n3 + 15) / 16));
  }
  slice_pass_g<Pr, double, T, Tw, T>(a, steps, cs, ja);
  const size_t ob = a.push(jb.data(), sizeof(jb[0]) * jb.size());
  const size_t os = a.push(start3.data(), sizeof(int) * start3.size());
  const int blocks3 = start3.back();
  steps.push_back([&a, ob, os, n, blocks3, lds3](hipStream_t st) -> igafd_status {
    hipLaunchKernelGGL((k_dir3_g<Pr, Tw, T>), dim3((unsigned)blocks3), dim3(kFusedThreads), lds3, st,
                       a.at<Dir3Job<Tw, T>>(ob), a.at<int>(os), n);
    IGAFD_HIP_CHECK(hipGetLastError());
    return IGAFD_OK;
  });
  slice_pass_g<Pr, T, double, Tw, T>(a, steps, cs, jc);
  return IGAFD_OK;
}

}  // namespace

igafd_status fd_grouped(GroupArena& a, std::vector<GroupStep>& steps, const std::vector<igafd_ctx*>& cs, int prec,
                        const std::vector<const double*>& r, const std::vector<double*>& s,
                        const std::vector<const double*>& S, const std::vector<double*>& partial) {
  for (const igafd_ctx* c : cs)
    if (c->adi || c->hole >= 0 || !(c->fd_fused && fused_ok(c) && !use_gemm(c, prec))) {
      set_error("internal: grouped FD apply needs the fused 3D passes");
      return IGAFD_ERR_ARG;
    }
  switch (prec) {
    case IGAFD_FP64:
      return fused_g<PF64, double, double>(a, steps, cs, r, s, S, partial);
    case IGAFD_FP32:
      return fused_g<PF32, float, float>(a, steps, cs, r, s, S, partial);
    case IGAFD_BF16:
      return fused_g<PBF16, float, float>(a, steps, cs, r, s, S, partial);
    case IGAFD_BF16X3:
      return fused_g<PBF16X3, float, float>(a, steps, cs, r, s, S, partial);
    default:
      set_error("unknown precision");
      return IGAFD_ERR_ARG;
  }
}

bool fd_groupable(const igafd_ctx* c, int prec) {
  return !c->adi && c->hole < 0 && c->fd_fused && fused_ok(c) && !use_gemm(c, prec);
}

// Row padding of the U matrices: every row tile any tile count can address.
int fd_npad(int n) {
  const int ntiles = (n + 15) / 16;
  int rows = 0;
  for (int mt = 1; mt <= 8; ++mt) {
    const int m = mt > ntiles ? ntiles : mt;
    const int r = ((ntiles + m - 1) / m) * m * 16;
    if (r > rows) rows = r;
  }
  if (rows < n) rows = n;
  return (rows + 63) / 64 * 64;
}



}  // namespace igafd

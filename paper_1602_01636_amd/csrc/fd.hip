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
// BF16 inputs with FP32 accumulation (v_mfma_f32_16x16x16_bf16).  r and s are
// FP64; intermediates are FP64 for FP64 and FP32 otherwise.
//
// Fused epilogues: scaling by the eigenvalue sums, the diagonal S of the
// scaled preconditioner S P^-1 S on input and output, and the partial sums of
// (r, s) for the CG recurrence.
#include "internal.h"
#include "reduce.h"

namespace igafd {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (short)(u >> 16);
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
};
struct PF32 {
  using W = float;
  using acc = f4_t;
  static constexpr int KS = 4;
  static constexpr int KPL = 1;
  static constexpr bool ROW_STRIDE4 = false;
};
struct PBF16 {
  using W = short;
  using acc = f4_t;
  static constexpr int KS = 16;
  static constexpr int KPL = 4;
  static constexpr bool ROW_STRIDE4 = false;
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

// D[k][c] = sum_i Wm[k][i] X(i, c) for k in this block's row range and the
// wave's 16 columns.  TRX: X(i, c) = X[c * n + i] and D -> Y[c * n + k];
// otherwise X(i, c) = X[b * bstride + i * C + c] and D -> Y[b * bstride + k * C + c].
//
// Block order: the nblk row blocks of one 64-column group run on the same XCD
// (blocks are dealt to the 8 XCDs round robin), so the input tile they share
// is read into one L2.  Operands of UNR K-steps are loaded before their MFMAs.
template <class Pr, int MT, bool TRX, typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_mode(const Tin* __restrict__ X, Tout* __restrict__ Y,
                                                 const typename Pr::W* __restrict__ Wm, int npad, int n, int C,
                                                 long long bstride, int nblk, int ncolblk, int ngroups, Epi ep) {
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
            const long long addr = TRX ? (long long)c * n + i : boff + (long long)i * C + c;
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
        const long long addr = TRX ? (long long)c * n + k : boff + (long long)k * C + c;
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
                         int C, int B, long long bstride, const Epi& ep) {
  const ModeShape ms = mode_shape(n, mt_max);
  const int ncolblk = (C + 63) / 64;
  const dim3 grid((unsigned)grid_x(C, B, ms.nblk), 1, 1);
  switch (ms.mt) {
#define IGAFD_MT(M)                                                                                    \
  case M:                                                                                              \
    hipLaunchKernelGGL((k_mode<Pr, M, TRX, Tin, Tout>), grid, dim3(kBlock), 0, st, X, Y, Wm, npad, n, C, \
                       bstride, ms.nblk, ncolblk, B * ncolblk, ep);                                    \
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

template <class Pr>
const typename Pr::W* wmat(const DevDir& d, int which);
template <>
const double* wmat<PF64>(const DevDir& d, int which) { return d.W64[which]; }
template <>
const float* wmat<PF32>(const DevDir& d, int which) { return d.W32[which]; }
template <>
const short* wmat<PBF16>(const DevDir& d, int which) { return reinterpret_cast<const short*>(d.Wbf[which]); }

int dot_blocks_for(const igafd_ctx* c) {
  const ModeShape ms = mode_shape(c->n[0], c->fd_tiles);
  const int C = (c->dim == 3) ? c->n[1] * c->n[2] : c->n[1];
  return grid_x(C, 1, ms.nblk);
}

// T: intermediate type (double for FP64, float otherwise)
template <class Pr, typename T>
igafd_status apply(igafd_ctx* c, const double* r, double* s, const double* S, double* partial, const int* flag) {
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
    IGAFD_TRY((launch_mode<Pr, true, double, T>(st, c->fd_tiles, r, b0, wmat<Pr>(d[0], 0), d[0].npad, n1, n2, 1, 0, e_in)));
    e_lam.lamK = d[1].lam;
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b0, b1, wmat<Pr>(d[1], 0), d[1].npad, n2, n1, 1, 0, e_lam)));
    IGAFD_TRY((launch_mode<Pr, false, T, T>(st, c->fd_tiles, b1, b0, wmat<Pr>(d[1], 1), d[1].npad, n2, n1, 1, 0, e0)));
    IGAFD_TRY((launch_mode<Pr, true, T, double>(st, c->fd_tiles, b0, s, wmat<Pr>(d[0], 1), d[0].npad, n1, n2, 1, 0, e_out)));
  }
#undef IGAFD_TRY
  return IGAFD_OK;
}

}  // namespace

int fd_dot_blocks(const igafd_ctx* c) { return dot_blocks_for(c); }

int fd_dot_blocks_max(const igafd_ctx* c) {
  const int C = (c->dim == 3) ? c->n[1] * c->n[2] : c->n[1];
  int m = 0;
  for (int t = 1; t <= 8; ++t) {
    const int g = grid_x(C, 1, mode_shape(c->n[0], t).nblk);
    if (g > m) m = g;
  }
  return m;
}

igafd_status fd_apply(igafd_ctx* c, int prec, const double* r, double* s, const double* S, double* partial,
                      const int* flag) {
  switch (prec) {
    case IGAFD_FP64:
      return apply<PF64, double>(c, r, s, S, partial, flag);
    case IGAFD_FP32:
      return apply<PF32, float>(c, r, s, S, partial, flag);
    case IGAFD_BF16:
      return apply<PBF16, float>(c, r, s, S, partial, flag);
    default:
      set_error("unknown precision");
      return IGAFD_ERR_ARG;
  }
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

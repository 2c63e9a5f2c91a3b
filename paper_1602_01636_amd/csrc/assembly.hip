// Device assembly of the Galerkin stiffness matrix A and of the load vector b.
//
// Paper Sec. 2.1 eq. A / eq. Q: A_ij = int_[0,1]^d grad(B_i)^T Q grad(B_j) with
// Q = |det J| J^-1 K J^-T (J_ij = dF_i/dxi_j), by the tensor (p+1)-point Gauss
// rule on every element.  One workgroup per element:
//   1. geometry at the element's (p+1)^d Gauss points -> C = w Q in LDS
//      (Q = kappa adj(J) adj(J)^T / |det J|, computed without an inverse),
//   2. local matrix by sum factorisation over the tensor Gauss rule: for a
//      fixed pair of direction-3 functions, contract the t3 points, then the t2
//      points, then the t1 points (the same sum, reordered),
//   3. add into the symmetric band.  Elements are processed in (p+1)^d colour
//      classes (element index mod p+1 per direction): two elements of one class
//      share no basis function, so the += needs no atomics and the summation
//      order is fixed (bitwise reproducible).
// Only the upper half of the stencil is stored: plane h holds offset
// center + h of the (2p+1)^d stencil, indexed by the row.
#include "internal.h"

namespace igafd {
namespace {

// right-hand side f of igafd_load_vector: kind, amplitude, SINPROD frequencies
struct RhsDesc {
  int kind;
  double amp;
  double k[3];
};

struct Tables {
  const int* first[3];
  const double* qx[3];
  const double* qw[3];
  const double* val[3];
  const double* der[3];
  int n[3];
};

template <int D>
__device__ inline void map_eval(const GeomDesc& g, const double xi[3], double x[3], double J[3][3]) {
  for (int a = 0; a < 3; ++a) {
    x[a] = xi[a];
    for (int b = 0; b < 3; ++b) J[a][b] = (a == b) ? 1.0 : 0.0;
  }
  if (g.kind == IGAFD_GEOM_RING) {
    const double r = 1.0 + xi[0];
    const double th = 0.5 * M_PI * xi[1];
    double s, c;
    sincos(th, &s, &c);
    x[0] = r * c;
    x[1] = r * s;
    J[0][0] = c;
    J[0][1] = -0.5 * M_PI * r * s;
    J[1][0] = s;
    J[1][1] = 0.5 * M_PI * r * c;
  } else if (g.kind == IGAFD_GEOM_WARPED) {
    for (int k = 0; k < g.nmodes; ++k) {
      double sn[3], dc[3];
      for (int l = 0; l < D; ++l) {
        double s, c;
        sincos(M_PI * g.m[k][l] * xi[l], &s, &c);
        sn[l] = s;
        dc[l] = M_PI * g.m[k][l] * c;
      }
      double prod = 1.0;
      for (int l = 0; l < D; ++l) prod *= sn[l];
      for (int a = 0; a < D; ++a) x[a] += g.amp * g.c[k][a] * prod;
      for (int j = 0; j < D; ++j) {
        double others = dc[j];
        for (int l = 0; l < D; ++l)
          if (l != j) others *= sn[l];
        for (int a = 0; a < D; ++a) J[a][j] += g.amp * g.c[k][a] * others;
      }
    }
  }
}

__device__ inline double kappa_eval(const GeomDesc& g, const double x[3]) {
  if (g.coef_kind == IGAFD_COEF_SINCOS)
    return 1.0 + g.camp * sin(2.0 * M_PI * g.f1 * x[0] + g.phi1) * cos(2.0 * M_PI * g.f2 * x[1] + g.phi2);
  return 1.0;
}

// det J and the cofactor matrix adj(J) (so that J^-1 = adj / det).
template <int D>
__device__ inline double adjugate(const double J[3][3], double A[3][3]) {
  if (D == 2) {
    A[0][0] = J[1][1];
    A[0][1] = -J[0][1];
    A[1][0] = -J[1][0];
    A[1][1] = J[0][0];
    return J[0][0] * J[1][1] - J[0][1] * J[1][0];
  }
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
}

template <int D>
__host__ __device__ constexpr int sym_index(int a, int b) {
  return (a == b) ? a : (D == 2 ? 2 : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5)));
}

// Per-dof statistics of the learned scaling, one element's share: for the
// NCH channels ch0..ch0+NCH-1 and every local function a = (a1, a2, a3) of
// the element, sum_t B_a(t) v(ch, t) over the element's Gauss points t, where
// v(ch, t) = w_t G_ch(t) (ch < 6: the entries 11, 22, 33, 12, 13, 23 of
// G = |det J| J^-1 J^-T), w_t kappa(t) (ch = 6) or w_t (ch = 7), given in
// vals[ch - ch0][t].  The sum is taken one direction at a time (sum
// factorisation: t1, then t2, then t3) and added into acc[8 row + ch] for the
// functions that are dofs; the element's colour class guarantees no other
// block adds to those rows.  F1 (NCH L Q Q3 doubles) and F2 (NCH L L Q3) are
// LDS scratch; vals may share F2's storage (it is last read before F2 is
// written).
template <int D, int P, int NCH>
__device__ void feature_sums(int ch0, const double* vals, const double (*sV)[P + 1][P + 1], const int* first,
                             const Tables& T, double* F1, double* F2, double* __restrict__ acc) {
  constexpr int Q = P + 1, L = P + 1;
  constexpr int Q3 = (D == 3) ? Q : 1;
  constexpr int L3 = (D == 3) ? L : 1;
  constexpr int NQ = Q * Q * Q3;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NCH * L * Q * Q3; idx += kBlock) {  // F1[c][t2 + Q t3][a1]
    const int c = idx / (L * Q * Q3), r = idx % (L * Q * Q3);
    const int a1 = r % L, t23 = r / L;
    double s = 0.0;
#pragma unroll
    for (int t1 = 0; t1 < Q; ++t1) s += sV[0][t1][a1] * vals[c * NQ + t1 + Q * t23];
    F1[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < NCH * L * L * Q3; idx += kBlock) {  // F2[c][t3][a2][a1]
    const int c = idx / (L * L * Q3), r = idx % (L * L * Q3);
    const int a1 = r % L, a2 = (r / L) % L, t3 = r / (L * L);
    double s = 0.0;
#pragma unroll
    for (int t2 = 0; t2 < Q; ++t2) s += sV[1][t2][a2] * F1[c * (L * Q * Q3) + (t2 + Q * t3) * L + a1];
    F2[idx] = s;
  }
  __syncthreads();
  // one thread per local function: its NCH channel sums, then one
  // read-modify-write of the NCH consecutive doubles of its row (a 32- or
  // 64-byte run, instead of NCH scattered 8-byte accesses from as many waves)
  static_assert(NCH % 4 == 0, "channel quadruples");
  typedef double dpair __attribute__((ext_vector_type(2)));
  constexpr int DOFS = L * L * L3, PER = (DOFS + kBlock - 1) / kBlock;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int r = tid + k * kBlock;
    if (r >= DOFS) break;
    const int a1 = r % L, a2 = (r / L) % L, a3 = r / (L * L);
    const int r1 = first[0] + a1 - 1, r2 = first[1] + a2 - 1, r3 = (D == 3) ? first[2] + a3 - 1 : 0;
    if (r1 < 0 || r1 >= T.n[0] || r2 < 0 || r2 >= T.n[1] || r3 < 0 || r3 >= T.n[2]) continue;
    dpair* row = reinterpret_cast<dpair*>(acc + 8 * (r1 + (long long)T.n[0] * (r2 + (long long)T.n[1] * r3)) + ch0);
    // four channels at a time (the registers of eight sums and their old
    // values would cost the p = 4 assembly a wave per SIMD)
#pragma unroll
    for (int h = 0; h < NCH; h += 4) {
      const dpair o0 = row[h / 2], o1 = row[h / 2 + 1];
      double sv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int t3 = 0; t3 < Q3; ++t3) s += sV[2][t3][a3] * F2[(h + c) * (L * L * Q3) + (t3 * L + a2) * L + a1];
        sv[c] = s;
      }
      row[h / 2] = dpair{o0.x + sv[0], o0.y + sv[1]};
      row[h / 2 + 1] = dpair{o1.x + sv[2], o1.y + sv[3]};
    }
  }
  __syncthreads();
}

// FEAT = 1: also the per-dof feature sums of the learned scaling into acc
// (8 doubles per dof), from the same Gauss-point evaluation of the map.
template <int D, int P, int FEAT>
__global__ __launch_bounds__(kBlock, (D == 3 && P <= 4) ? 5 : 1) void k_assemble(Tables T, GeomDesc g, double* __restrict__ band,
                                                     long long Ns, int c1, int c2, int c3, int m1, int m2,
                                                     int* __restrict__ err, double* __restrict__ acc) {
  constexpr int Q = P + 1, L = P + 1;
  constexpr int Q3 = (D == 3) ? Q : 1;
  constexpr int L3 = (D == 3) ? L : 1;
  constexpr int NQ = Q * Q * Q3;
  constexpr int NC = (D == 3) ? 6 : 3;
  constexpr int NAB = D * D;
  constexpr int W = 2 * P + 1;
  constexpr int S = (D == 3) ? W * W * W : W * W;
  constexpr int CENTER = (S - 1) / 2;
  constexpr int R3 = (D == 3) ? P : 0;

  __shared__ double sC[NC][NQ];
  __shared__ double sV[3][Q][L];
  __shared__ double sD[3][Q][L];
  __shared__ double sH[NAB][Q * Q];
  __shared__ double sG[NAB][L * L][Q];
  __shared__ int sFirst[3];
  // features: kappa and the weight per point, F2 of the contraction (F1 lives in sG)
  __shared__ double sKap[FEAT ? NQ : 1], sW[FEAT ? NQ : 1];
  // feature channels per pass: all eight, or four at a time from p = 5 on
  // (eight made the LDS of p = 5 allow three blocks per CU instead of four)
  constexpr int NCH = (P >= 5) ? 4 : 8;
  __shared__ double sF2[FEAT ? NCH * L * L * Q3 : 1];  // the channel values, then F2
  static_assert(!FEAT || NAB * L * L * Q >= NCH * L * Q * Q3, "feature scratch F1 must fit in sG");
  static_assert(!FEAT || L * L * Q3 >= NQ, "channel values must fit in sF2");

  int bid = blockIdx.x;
  const int j1 = bid % m1;
  bid /= m1;
  const int j2 = bid % m2;
  const int j3 = bid / m2;
  const int e[3] = {c1 + j1 * (P + 1), c2 + j2 * (P + 1), (D == 3) ? c3 + j3 * (P + 1) : 0};
  const int tid = threadIdx.x;

  for (int idx = tid; idx < 3 * Q * L; idx += kBlock) {
    const int l = idx / (Q * L), t = (idx / L) % Q, a = idx % L;
    if (l < D) {
      sV[l][t][a] = T.val[l][(e[l] * Q + t) * L + a];
      sD[l][t][a] = T.der[l][(e[l] * Q + t) * L + a];
    } else {
      sV[l][t][a] = (t == 0 && a == 0) ? 1.0 : 0.0;
      sD[l][t][a] = 0.0;
    }
  }
  if (tid < 3) sFirst[tid] = (tid < D) ? T.first[tid][e[tid]] : 1;

  for (int t = tid; t < NQ; t += kBlock) {
    const int t1 = t % Q, t2 = (t / Q) % Q, t3 = t / (Q * Q);
    double xi[3] = {T.qx[0][e[0] * Q + t1], T.qx[1][e[1] * Q + t2], 0.0};
    double w = T.qw[0][e[0] * Q + t1] * T.qw[1][e[1] * Q + t2];
    if (D == 3) {
      xi[2] = T.qx[2][e[2] * Q + t3];
      w *= T.qw[2][e[2] * Q + t3];
    }
    double x[3], J[3][3], A[3][3];
    map_eval<D>(g, xi, x, J);
    const double det = adjugate<D>(J, A);
    if (!(det > 0.0)) *err = 1;
    const double kap = kappa_eval(g, x);
    const double f = w * kap / fabs(det);
    for (int a = 0; a < D; ++a)
      for (int b = a; b < D; ++b) {
        double s = 0.0;
        for (int k = 0; k < D; ++k) s += A[a][k] * A[b][k];
        sC[sym_index<D>(a, b)][t] = f * s;
      }
    if (FEAT) {
      sKap[t] = kap;
      sW[t] = w;
    }
  }
  __syncthreads();
  if (FEAT) {
    // the channel values at the Gauss points, once each per pass: w G_ab =
    // C_ab / kappa; the channel order is (11, 22, 33, 12, 13, 23, kappa, 1)
    for (int ch0 = 0; ch0 < 8; ch0 += NCH) {
      for (int idx = tid; idx < NCH * NQ; idx += kBlock) {
        const int ch = ch0 + idx / NQ, t = idx % NQ;
        constexpr int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
        double v;
        if (ch == 6)
          v = sW[t] * sKap[t];
        else if (ch == 7)
          v = sW[t];
        else if (ia[ch] >= D || ib[ch] >= D)
          v = 0.0;
        else
          v = sC[sym_index<D>(ia[ch], ib[ch])][t] / sKap[t];
        sF2[idx] = v;
      }
      __syncthreads();
      feature_sums<D, P, NCH>(ch0, sF2, sV, sFirst, T, &sG[0][0][0], sF2, acc);
    }
  }

  for (int a3 = 0; a3 < L3; ++a3) {
    for (int b3 = a3; b3 < L3; ++b3) {
      // H[ab][t1 + Q t2] = sum_t3 C_ab(t) phi3(a3) phi3(b3)
      for (int idx = tid; idx < NAB * Q * Q; idx += kBlock) {
        const int ab = idx / (Q * Q), t12 = idx % (Q * Q);
        const int a = ab / D, b = ab % D;
        const int ci = sym_index<D>(a, b);
        double s = 0.0;
#pragma unroll
        for (int t3 = 0; t3 < Q3; ++t3) {
          const double fa = (a == 2) ? sD[2][t3][a3] : sV[2][t3][a3];
          const double fb = (b == 2) ? sD[2][t3][b3] : sV[2][t3][b3];
          s += sC[ci][t12 + Q * Q * t3] * fa * fb;
        }
        sH[ab][t12] = s;
      }
      __syncthreads();
      // G[ab][a2 + L b2][t1] = sum_t2 H[ab][t1 + Q t2] phi2(a2) phi2(b2)
      for (int idx = tid; idx < NAB * L * L * Q; idx += kBlock) {
        const int ab = idx / (L * L * Q), rem = idx % (L * L * Q);
        const int a2b2 = rem / Q, t1 = rem % Q;
        const int a2 = a2b2 % L, b2 = a2b2 / L;
        const int a = ab / D, b = ab % D;
        double s = 0.0;
#pragma unroll
        for (int t2 = 0; t2 < Q; ++t2) {
          const double fa = (a == 1) ? sD[1][t2][a2] : sV[1][t2][a2];
          const double fb = (b == 1) ? sD[1][t2][b2] : sV[1][t2][b2];
          s += sH[ab][t1 + Q * t2] * fa * fb;
        }
        sG[ab][a2b2][t1] = s;
      }
      __syncthreads();
      // local entry (a1 a2 a3 | b1 b2 b3) = sum_ab sum_t1 G phi1(a1) phi1(b1)
      for (int idx = tid; idx < L * L * L * L; idx += kBlock) {
        const int a1 = idx % L, b1 = (idx / L) % L, a2 = (idx / (L * L)) % L, b2 = idx / (L * L * L);
        const int o1 = b1 - a1, o2 = b2 - a2, o3 = b3 - a3;
        if (o3 == 0 && (o2 < 0 || (o2 == 0 && o1 < 0))) continue;  // lower half: not stored
        const int r1 = sFirst[0] + a1 - 1, r2 = sFirst[1] + a2 - 1, r3 = (D == 3) ? sFirst[2] + a3 - 1 : 0;
        const int q1 = r1 + o1, q2 = r2 + o2, q3 = r3 + o3;
        if (r1 < 0 || r1 >= T.n[0] || r2 < 0 || r2 >= T.n[1] || r3 < 0 || r3 >= T.n[2]) continue;
        if (q1 < 0 || q1 >= T.n[0] || q2 < 0 || q2 >= T.n[1] || q3 < 0 || q3 >= T.n[2]) continue;
        double s = 0.0;
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) {
          const int a = ab / D, b = ab % D;
#pragma unroll
          for (int t1 = 0; t1 < Q; ++t1) {
            const double fa = (a == 0) ? sD[0][t1][a1] : sV[0][t1][a1];
            const double fb = (b == 0) ? sD[0][t1][b1] : sV[0][t1][b1];
            s += sG[ab][a2 + L * b2][t1] * fa * fb;
          }
        }
        const int oidx = ((o3 + R3) * W + (o2 + P)) * W + (o1 + P);
        const long long row = r1 + (long long)T.n[0] * (r2 + (long long)T.n[1] * r3);
        band[(long long)(oidx - CENTER) * Ns + row] += s;
      }
      __syncthreads();
    }
  }
}

template <int D>
__device__ inline double rhs_eval(const RhsDesc& f, const double x[3]) {
  switch (f.kind) {
    case IGAFD_RHS_SINPROD: {
      double s = f.amp;
      for (int l = 0; l < D; ++l) s *= sin(f.k[l] * M_PI * x[l]);
      return s;
    }
    case IGAFD_RHS_PAPER_POLY: {
      double s = 0.0;
      for (int l = 0; l < D; ++l) s += 2.0 * (x[l] * x[l] - x[l]);
      return f.amp * s;
    }
    case IGAFD_RHS_BUBBLE: {
      double s = 0.0;
      for (int i = 0; i < D; ++i) {
        double pr = 2.0;
        for (int l = 0; l < D; ++l)
          if (l != i) pr *= x[l] * (1.0 - x[l]);
        s += pr;
      }
      return f.amp * s;
    }
    default:
      return f.amp;
  }
}

// b_i += sum_t w_t |det J| f(F(t)) B_i(t) over one colour class of elements.
template <int D, int P>
__global__ __launch_bounds__(kBlock) void k_load(Tables T, GeomDesc g, RhsDesc rhs, double* __restrict__ b,
                                                 int c1, int c2, int c3, int m1, int m2) {
  constexpr int Q = P + 1, L = P + 1;
  constexpr int Q3 = (D == 3) ? Q : 1;
  constexpr int L3 = (D == 3) ? L : 1;
  constexpr int NQ = Q * Q * Q3;
  __shared__ double sg[NQ];
  __shared__ double sV[3][Q][L];
  int bid = blockIdx.x;
  const int j1 = bid % m1;
  bid /= m1;
  const int j2 = bid % m2;
  const int j3 = bid / m2;
  const int e[3] = {c1 + j1 * (P + 1), c2 + j2 * (P + 1), (D == 3) ? c3 + j3 * (P + 1) : 0};
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 3 * Q * L; idx += kBlock) {
    const int l = idx / (Q * L), t = (idx / L) % Q, a = idx % L;
    sV[l][t][a] = (l < D) ? T.val[l][(e[l] * Q + t) * L + a] : ((t == 0 && a == 0) ? 1.0 : 0.0);
  }
  for (int t = tid; t < NQ; t += kBlock) {
    const int t1 = t % Q, t2 = (t / Q) % Q, t3 = t / (Q * Q);
    double xi[3] = {T.qx[0][e[0] * Q + t1], T.qx[1][e[1] * Q + t2], 0.0};
    double w = T.qw[0][e[0] * Q + t1] * T.qw[1][e[1] * Q + t2];
    if (D == 3) {
      xi[2] = T.qx[2][e[2] * Q + t3];
      w *= T.qw[2][e[2] * Q + t3];
    }
    double x[3], J[3][3], A[3][3];
    map_eval<D>(g, xi, x, J);
    const double det = adjugate<D>(J, A);
    sg[t] = w * fabs(det) * rhs_eval<D>(rhs, x);
  }
  __syncthreads();
  for (int idx = tid; idx < L * L * L3; idx += kBlock) {
    const int a1 = idx % L, a2 = (idx / L) % L, a3 = idx / (L * L);
    const int r1 = T.first[0][e[0]] + a1 - 1, r2 = T.first[1][e[1]] + a2 - 1;
    const int r3 = (D == 3) ? T.first[2][e[2]] + a3 - 1 : 0;
    if (r1 < 0 || r1 >= T.n[0] || r2 < 0 || r2 >= T.n[1] || r3 < 0 || r3 >= T.n[2]) continue;
    double s = 0.0;
    for (int t = 0; t < NQ; ++t) {
      const int t1 = t % Q, t2 = (t / Q) % Q, t3 = t / (Q * Q);
      s += sg[t] * sV[0][t1][a1] * sV[1][t2][a2] * sV[2][t3][a3];
    }
    b[r1 + (long long)T.n[0] * (r2 + (long long)T.n[1] * r3)] += s;
  }
}

// Per-dof geometry/coefficient statistics for the learned scaling, without
// assembling A: the same Gauss-point values as k_assemble's feature channels
// (w G's six entries, w kappa, w), summed into acc by feature_sums.
template <int D, int P>
__global__ __launch_bounds__(kBlock) void k_features(Tables T, GeomDesc g, double* __restrict__ acc, int c1, int c2,
                                                     int c3, int m1, int m2) {
  constexpr int Q = P + 1, L = P + 1;
  constexpr int Q3 = (D == 3) ? Q : 1;
  constexpr int NQ = Q * Q * Q3;
  __shared__ double sf[8][NQ];
  __shared__ double sV[3][Q][L];
  __shared__ double sF1[8 * L * Q * Q3], sF2[8 * L * L * Q3];
  __shared__ int sFirst[3];
  int bid = blockIdx.x;
  const int j1 = bid % m1;
  bid /= m1;
  const int j2 = bid % m2;
  const int j3 = bid / m2;
  const int e[3] = {c1 + j1 * (P + 1), c2 + j2 * (P + 1), (D == 3) ? c3 + j3 * (P + 1) : 0};
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 3 * Q * L; idx += kBlock) {
    const int l = idx / (Q * L), t = (idx / L) % Q, a = idx % L;
    sV[l][t][a] = (l < D) ? T.val[l][(e[l] * Q + t) * L + a] : ((t == 0 && a == 0) ? 1.0 : 0.0);
  }
  if (tid < 3) sFirst[tid] = (tid < D) ? T.first[tid][e[tid]] : 1;
  for (int t = tid; t < NQ; t += kBlock) {
    const int t1 = t % Q, t2 = (t / Q) % Q, t3 = t / (Q * Q);
    double xi[3] = {T.qx[0][e[0] * Q + t1], T.qx[1][e[1] * Q + t2], 0.0};
    double w = T.qw[0][e[0] * Q + t1] * T.qw[1][e[1] * Q + t2];
    if (D == 3) {
      xi[2] = T.qx[2][e[2] * Q + t3];
      w *= T.qw[2][e[2] * Q + t3];
    }
    double x[3], J[3][3], A[3][3] = {};
    map_eval<D>(g, xi, x, J);
    const double det = fabs(adjugate<D>(J, A));
    double G[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int k = 0; k < D; ++k) s += A[a][k] * A[b][k];
        G[a][b] = (a < D && b < D) ? s / det : 0.0;
      }
    sf[0][t] = w * G[0][0];
    sf[1][t] = w * G[1][1];
    sf[2][t] = w * G[2][2];
    sf[3][t] = w * G[0][1];
    sf[4][t] = w * G[0][2];
    sf[5][t] = w * G[1][2];
    sf[6][t] = w * kappa_eval(g, x);
    sf[7][t] = w;
  }
  __syncthreads();
  feature_sums<D, P, 8>(0, &sf[0][0], sV, sFirst, T, sF1, sF2, acc);
}

// Extreme eigenvalues of a symmetric positive definite 2x2 / 3x3 matrix.
// 2x2: closed form, the small one as det / large (no cancellation).  3x3:
// cyclic Jacobi rotations (each zeroes one off-diagonal pair; the diagonal
// converges quadratically to the eigenvalues, accurate to roundoff also for
// repeated eigenvalues, where closed forms of the cubic lose half the digits).
__device__ inline void sym_extremes(int d, const double Q[3][3], double& lo, double& hi) {
  if (d == 2) {
    const double m = 0.5 * (Q[0][0] + Q[1][1]), h = 0.5 * (Q[0][0] - Q[1][1]);
    hi = m + sqrt(h * h + Q[0][1] * Q[0][1]);
    lo = (Q[0][0] * Q[1][1] - Q[0][1] * Q[0][1]) / hi;
    return;
  }
  double a[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a[i][j] = Q[i][j];
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= 1e-36 * dia) break;
    for (int k = 0; k < 3; ++k) {
      const int p = k == 2 ? 1 : 0, q = k == 0 ? 1 : 2;
      const double apq = a[p][q];
      if (fabs(apq) <= 1e-300) continue;
      // rotation angle with tan(2 phi) = 2 a_pq / (a_qq - a_pp); t = tan(phi), the smaller root
      const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.0;
      const int r = 3 - p - q;
      const double arp = a[r][p], arq = a[r][q];
      a[r][p] = a[p][r] = c * arp - s * arq;
      a[r][q] = a[q][r] = s * arp + c * arq;
    }
  }
  lo = fmin(a[0][0], fmin(a[1][1], a[2][2]));
  hi = fmax(a[0][0], fmax(a[1][1], a[2][2]));
}

// min / max over the Gauss points of the extreme eigenvalues of
// Q = kappa |det J| J^-1 J^-T (Sec. 2.1 eq. Q), and the max over the points of
// the local ratio lambda_max(Q(x)) / lambda_min(Q(x)).  Grid-stride over all
// points (nq[l] = points along direction l, flat index i1 + nq0 (i2 + nq1 i3));
// per block part[blockIdx.x] = min, part[G + blockIdx.x] = max and
// part[2 G + blockIdx.x] = max ratio (G = gridDim.x).
template <int D>
__global__ __launch_bounds__(kBlock) void k_qbounds(const double* __restrict__ qx0, const double* __restrict__ qx1,
                                                    const double* __restrict__ qx2, GeomDesc g, int nq0, int nq1,
                                                    int nq2, double* __restrict__ part) {
  double lo = INFINITY, hi = -INFINITY, loc = 0.0;
  const long long total = (long long)nq0 * nq1 * nq2;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total; i += (long long)gridDim.x * kBlock) {
    const int i1 = (int)(i % nq0);
    const long long rest = i / nq0;
    const int i2 = (int)(rest % nq1), i3 = (int)(rest / nq1);
    const double xi[3] = {qx0[i1], qx1[i2], D == 3 ? qx2[i3] : 0.0};
    double x[3], J[3][3], A[3][3] = {};
    map_eval<D>(g, xi, x, J);
    const double det = fabs(adjugate<D>(J, A));
    const double k = kappa_eval(g, x) / det;
    double Q[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int l = 0; l < D; ++l) s += A[a][l] * A[b][l];
        Q[a][b] = k * s;
      }
    double l0, l1;
    sym_extremes(D, Q, l0, l1);
    lo = fmin(lo, l0);
    hi = fmax(hi, l1);
    loc = fmax(loc, l1 / l0);
  }
  // min / max are exact: any reduction order gives the same result
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_down(lo, off, 64));
    hi = fmax(hi, __shfl_down(hi, off, 64));
    loc = fmax(loc, __shfl_down(loc, off, 64));
  }
  __shared__ double slo[kBlock / 64], shi[kBlock / 64], sloc[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    slo[wid] = lo;
    shi[wid] = hi;
    sloc[wid] = loc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      lo = fmin(lo, slo[w]);
      hi = fmax(hi, shi[w]);
      loc = fmax(loc, sloc[w]);
    }
    part[blockIdx.x] = lo;
    part[gridDim.x + blockIdx.x] = hi;
    part[2 * gridDim.x + blockIdx.x] = loc;
  }
}

__global__ void k_minmax(const double* __restrict__ part, int count, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo = INFINITY, hi = -INFINITY, loc = 0.0;
  for (int k = 0; k < count; ++k) {
    lo = fmin(lo, part[k]);
    hi = fmax(hi, part[count + k]);
    loc = fmax(loc, part[2 * count + k]);
  }
  out[0] = lo;
  out[1] = hi;
  out[2] = loc;
}

// feat[i] = (acc[i][0..6] / acc[i][7], p) in FP32
__global__ void k_features_finish(const double* __restrict__ acc, float* __restrict__ feat, long long N, int p) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double inv = 1.0 / acc[8 * i + 7];
  for (int ch = 0; ch < 7; ++ch) feat[8 * i + ch] = (float)(acc[8 * i + ch] * inv);
  feat[8 * i + 7] = (float)p;
}

// diag(P)_i = sum_j K_j[i_j, i_j] prod_{l != j} M_l[i_l, i_l]  (Sec. 3 Kronecker sum)
__device__ inline double diagP_at(const double* m1, const double* k1, const double* m2, const double* k2,
                                  const double* m3, const double* k3, int n1, int n2, int dim, long long i) {
  const int i1 = (int)(i % n1);
  const long long t = i / n1;
  const int i2 = (int)(t % n2), i3 = (int)(t / n2);
  if (dim == 2) return k1[i1] * m2[i2] + m1[i1] * k2[i2];
  return k1[i1] * m2[i2] * m3[i3] + m1[i1] * k2[i2] * m3[i3] + m1[i1] * m2[i2] * k3[i3];
}

__global__ void k_diagP(const double* m1, const double* k1, const double* m2, const double* k2,
                        const double* m3, const double* k3, int n1, int n2, long long N, int dim,
                        double* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = diagP_at(m1, k1, m2, k2, m3, k3, n1, n2, dim, i);
}

// a fill kernel instead of a memset: callers may capture these launches into graphs
__global__ void k_zero(double* __restrict__ p, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

__global__ void k_copy_plane(const double* __restrict__ src, double* __restrict__ dst, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[i] = src[i];
}

Tables make_tables(const igafd_ctx* c) {
  Tables T{};
  for (int l = 0; l < 3; ++l) {
    T.first[l] = c->ddir[l].elem_first;
    T.qx[l] = c->ddir[l].qx;
    T.qw[l] = c->ddir[l].qw;
    T.val[l] = c->ddir[l].val;
    T.der[l] = c->ddir[l].der;
    T.n[l] = c->n[l];
  }
  return T;
}

template <int D, int P>
igafd_status launch_assemble(igafd_ctx* c, double* acc) {
  const Tables T = make_tables(c);
  const int nel[3] = {c->ddir[0].nel, c->ddir[1].nel, D == 3 ? c->ddir[2].nel : 1};
  const int C3 = (D == 3) ? P + 1 : 1;
  for (int c3 = 0; c3 < C3; ++c3)
    for (int c2 = 0; c2 <= P; ++c2)
      for (int c1 = 0; c1 <= P; ++c1) {
        const int m1 = c1 < nel[0] ? (nel[0] - c1 + P) / (P + 1) : 0;
        const int m2 = c2 < nel[1] ? (nel[1] - c2 + P) / (P + 1) : 0;
        const int m3 = (D == 3) ? (c3 < nel[2] ? (nel[2] - c3 + P) / (P + 1) : 0) : 1;
        const long long blocks = (long long)m1 * m2 * m3;
        if (blocks == 0) continue;
        if (acc)
          hipLaunchKernelGGL((k_assemble<D, P, 1>), dim3((unsigned)blocks), dim3(kBlock), 0, c->stream, T, c->geom,
                             c->band + c->halo, c->Ns, c1, c2, c3, m1, m2, c->dflag, acc);
        else
          hipLaunchKernelGGL((k_assemble<D, P, 0>), dim3((unsigned)blocks), dim3(kBlock), 0, c->stream, T, c->geom,
                             c->band + c->halo, c->Ns, c1, c2, c3, m1, m2, c->dflag, nullptr);
        IGAFD_HIP_CHECK(hipGetLastError());
      }
  return IGAFD_OK;
}

template <int D, int P>
igafd_status launch_load(igafd_ctx* c, RhsDesc rhs, double* b) {
  const Tables T = make_tables(c);
  const int nel[3] = {c->ddir[0].nel, c->ddir[1].nel, D == 3 ? c->ddir[2].nel : 1};
  const int C3 = (D == 3) ? P + 1 : 1;
  for (int c3 = 0; c3 < C3; ++c3)
    for (int c2 = 0; c2 <= P; ++c2)
      for (int c1 = 0; c1 <= P; ++c1) {
        const int m1 = c1 < nel[0] ? (nel[0] - c1 + P) / (P + 1) : 0;
        const int m2 = c2 < nel[1] ? (nel[1] - c2 + P) / (P + 1) : 0;
        const int m3 = (D == 3) ? (c3 < nel[2] ? (nel[2] - c3 + P) / (P + 1) : 0) : 1;
        const long long blocks = (long long)m1 * m2 * m3;
        if (blocks == 0) continue;
        hipLaunchKernelGGL((k_load<D, P>), dim3((unsigned)blocks), dim3(kBlock), 0, c->stream, T, c->geom, rhs, b,
                           c1, c2, c3, m1, m2);
        IGAFD_HIP_CHECK(hipGetLastError());
      }
  return IGAFD_OK;
}

template <int D, int P>
igafd_status launch_features(igafd_ctx* c, double* acc) {
  const Tables T = make_tables(c);
  const int nel[3] = {c->ddir[0].nel, c->ddir[1].nel, D == 3 ? c->ddir[2].nel : 1};
  const int C3 = (D == 3) ? P + 1 : 1;
  for (int c3 = 0; c3 < C3; ++c3)
    for (int c2 = 0; c2 <= P; ++c2)
      for (int c1 = 0; c1 <= P; ++c1) {
        const int m1 = c1 < nel[0] ? (nel[0] - c1 + P) / (P + 1) : 0;
        const int m2 = c2 < nel[1] ? (nel[1] - c2 + P) / (P + 1) : 0;
        const int m3 = (D == 3) ? (c3 < nel[2] ? (nel[2] - c3 + P) / (P + 1) : 0) : 1;
        const long long blocks = (long long)m1 * m2 * m3;
        if (blocks == 0) continue;
        hipLaunchKernelGGL((k_features<D, P>), dim3((unsigned)blocks), dim3(kBlock), 0, c->stream, T, c->geom, acc,
                           c1, c2, c3, m1, m2);
        IGAFD_HIP_CHECK(hipGetLastError());
      }
  return IGAFD_OK;
}

template <template <int, int> class F, typename... Args>
igafd_status dispatch(int dim, int p, Args... args) {
  switch (dim * 10 + p) {
#define IGAFD_CASE(D, P) \
  case D * 10 + P:       \
    return F<D, P>::run(args...);
    IGAFD_CASE(2, 1) IGAFD_CASE(2, 2) IGAFD_CASE(2, 3) IGAFD_CASE(2, 4) IGAFD_CASE(2, 5) IGAFD_CASE(2, 6)
    IGAFD_CASE(3, 1) IGAFD_CASE(3, 2) IGAFD_CASE(3, 3) IGAFD_CASE(3, 4) IGAFD_CASE(3, 5) IGAFD_CASE(3, 6)
#undef IGAFD_CASE
    default:
      set_error("unsupported dimension/degree");
      return IGAFD_ERR_ARG;
  }
}

template <int D, int P>
struct AssembleOp {
  static igafd_status run(igafd_ctx* c, double* acc) { return launch_assemble<D, P>(c, acc); }
};
template <int D, int P>
struct FeatureOp {
  static igafd_status run(igafd_ctx* c, double* acc) { return launch_features<D, P>(c, acc); }
};
template <int D, int P>
struct LoadOp {
  static igafd_status run(igafd_ctx* c, RhsDesc f, double* b) { return launch_load<D, P>(c, f, b); }
};

}  // namespace

igafd_status assemble_band(igafd_ctx* c, bool with_features) {
  IGAFD_HIP_CHECK(hipMemsetAsync(c->band, 0, sizeof(double) * c->H * c->Ns, c->stream));
  IGAFD_HIP_CHECK(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
  double* acc = nullptr;
  if (with_features) {  // feature sums (8 per dof) assembled with A, kept as FP32 features
    IGAFD_HIP_CHECK(hipMalloc((void**)&acc, sizeof(double) * 8 * (size_t)c->N));
    IGAFD_HIP_CHECK(hipMalloc((void**)&c->feat, sizeof(float) * 8 * (size_t)c->N));
    IGAFD_HIP_CHECK(hipMemsetAsync(acc, 0, sizeof(double) * 8 * (size_t)c->N, c->stream));
  }
  igafd_status st = dispatch<AssembleOp>(c->dim, c->p, c, acc);
  if (st == IGAFD_OK && acc) {
    const unsigned blocks = (unsigned)((c->N + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_features_finish, dim3(blocks), dim3(kBlock), 0, c->stream, acc, c->feat, c->N, c->p);
    if (hipGetLastError() != hipSuccess) {
      set_error("feature finish kernel failed");
      st = IGAFD_ERR_HIP;
    }
  }
  if (acc) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(acc);
  }
  if (st != IGAFD_OK) return st;
  int flag = 0;
  IGAFD_HIP_CHECK(hipMemcpyAsync(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  IGAFD_HIP_CHECK(hipStreamSynchronize(c->stream));
  if (flag) {
    set_error("det J <= 0 at a quadrature point");
    return IGAFD_ERR_GEOMETRY;
  }
  return IGAFD_OK;
}

igafd_status assemble_load(igafd_ctx* c, int rhs_kind, const double* params, int nparams, double* b) {
  if (rhs_kind < IGAFD_RHS_SINPROD || rhs_kind > IGAFD_RHS_ONE) {
    set_error("unknown right-hand side kind");
    return IGAFD_ERR_ARG;
  }
  RhsDesc f{};
  f.kind = rhs_kind;
  f.amp = rhs_kind == IGAFD_RHS_SINPROD ? c->dim * M_PI * M_PI : 1.0;
  for (int l = 0; l < 3; ++l) f.k[l] = 1.0;
  const int want = rhs_kind == IGAFD_RHS_SINPROD ? 1 + c->dim : 1;
  if (nparams != 0) {  // NULL / 0 keeps the defaults
    if (!params || nparams != want) {
      set_error("right-hand side parameters: expected " + std::to_string(want) + " values");
      return IGAFD_ERR_ARG;
    }
    f.amp = params[0];
    for (int l = 1; l < nparams; ++l) f.k[l - 1] = params[l];
  }
  IGAFD_HIP_CHECK(hipMemsetAsync(b, 0, sizeof(double) * c->N, c->stream));
  return dispatch<LoadOp>(c->dim, c->p, c, f, b);
}

igafd_status spectral_bounds(igafd_ctx* c, double* qmin, double* qmax, double* qloc) {
  if (!c->bounds_valid) {
    const int nq0 = c->dir[0].nel * c->dir[0].q, nq1 = c->dir[1].nel * c->dir[1].q;
    const int nq2 = c->dim == 3 ? c->dir[2].nel * c->dir[2].q : 1;
    // partial buffer: 2 * npartial doubles = blocks (min, max, ratio) triples + the result
    int blocks = (2 * c->npartial - 3) / 3;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) {
      set_error("internal: partial-sum buffer too small for the spectral bounds");
      return IGAFD_ERR_ARG;
    }
    double* out = c->partial + 3 * blocks;
    if (c->dim == 3)
      hipLaunchKernelGGL(k_qbounds<3>, dim3(blocks), dim3(kBlock), 0, c->stream, c->ddir[0].qx, c->ddir[1].qx,
                         c->ddir[2].qx, c->geom, nq0, nq1, nq2, c->partial);
    else
      hipLaunchKernelGGL(k_qbounds<2>, dim3(blocks), dim3(kBlock), 0, c->stream, c->ddir[0].qx, c->ddir[1].qx,
                         c->ddir[1].qx, c->geom, nq0, nq1, 1, c->partial);
    IGAFD_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(64), 0, c->stream, c->partial, blocks, out);
    IGAFD_HIP_CHECK(hipGetLastError());
    double h[3];
    IGAFD_HIP_CHECK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    IGAFD_HIP_CHECK(hipStreamSynchronize(c->stream));
    c->qmin = h[0];
    c->qmax = h[1];
    c->qloc = h[2];
    c->bounds_valid = true;
  }
  if (qmin) *qmin = c->qmin;
  if (qmax) *qmax = c->qmax;
  if (qloc) *qloc = c->qloc;
  return IGAFD_OK;
}

igafd_status diagonals(igafd_ctx* c, double* dA, double* dP) {
  const unsigned blocks = (unsigned)((c->N + kBlock - 1) / kBlock);
  if (dA) {  // plane 0 of the band is the diagonal
    hipLaunchKernelGGL(k_copy_plane, dim3(blocks), dim3(kBlock), 0, c->stream, c->band + c->halo, dA, c->N);
    IGAFD_HIP_CHECK(hipGetLastError());
  }
  if (dP) {
    const DevDir* d = c->ddir;
    hipLaunchKernelGGL(k_diagP, dim3(blocks), dim3(kBlock), 0, c->stream, d[0].diagM, d[0].diagK, d[1].diagM,
                       d[1].diagK, d[2].diagM, d[2].diagK, c->n[0], c->n[1], c->N, c->dim, dP);
    IGAFD_HIP_CHECK(hipGetLastError());
  }
  return IGAFD_OK;
}

igafd_status features(igafd_ctx* c, float* feat) {
  if (c->feat) {  // assembled with A at setup
    IGAFD_HIP_CHECK(
        hipMemcpyAsync(feat, c->feat, sizeof(float) * 8 * (size_t)c->N, hipMemcpyDeviceToDevice, c->stream));
    return IGAFD_OK;
  }
  double* acc = nullptr;
  IGAFD_HIP_CHECK(hipMalloc((void**)&acc, sizeof(double) * 8 * (size_t)c->N));
  igafd_status st = features_into(c, acc, feat);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(acc);
  return st;
}

igafd_status features_into(igafd_ctx* c, double* acc, float* feat) {
  const unsigned blocks = (unsigned)((c->N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((8 * c->N + kBlock - 1) / kBlock)), dim3(kBlock), 0, c->stream, acc,
                     8 * c->N);
  IGAFD_HIP_CHECK(hipGetLastError());
  igafd_status st = dispatch<FeatureOp>(c->dim, c->p, c, acc);
  if (st != IGAFD_OK) return st;
  hipLaunchKernelGGL(k_features_finish, dim3(blocks), dim3(kBlock), 0, c->stream, acc, feat, c->N, c->p);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

// t_i = 1/2 log(P_ii / A_ii) (log = 1) or S_i = sqrt(P_ii / A_ii) (log = 0),
// diag(P) from the univariate diagonals (Sec. 3 Kronecker sum)
__global__ void k_diag_ratio(const double* __restrict__ band0, const double* m1, const double* k1, const double* m2,
                             const double* k2, const double* m3, const double* k3, int n1, int n2, long long N,
                             int dim, int log_form, float* __restrict__ t, double* __restrict__ S) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double dP = diagP_at(m1, k1, m2, k2, m3, k3, n1, n2, dim, i);
  if (log_form)
    t[i] = (float)(0.5 * log(dP / band0[i]));
  else
    S[i] = sqrt(dP / band0[i]);
}

igafd_status scaling_targets(igafd_ctx* c, float* t) {
  const unsigned blocks = (unsigned)((c->N + kBlock - 1) / kBlock);
  const DevDir* d = c->ddir;
  hipLaunchKernelGGL(k_diag_ratio, dim3(blocks), dim3(kBlock), 0, c->stream, c->band + c->halo, d[0].diagM,
                     d[0].diagK, d[1].diagM, d[1].diagK, d[2].diagM, d[2].diagK, c->n[0], c->n[1], c->N, c->dim, 1, t,
                     nullptr);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

igafd_status diag_ratio_scaling(igafd_ctx* c, double* S) {
  const unsigned blocks = (unsigned)((c->N + kBlock - 1) / kBlock);
  const DevDir* d = c->ddir;
  hipLaunchKernelGGL(k_diag_ratio, dim3(blocks), dim3(kBlock), 0, c->stream, c->band + c->halo, d[0].diagM,
                     d[0].diagK, d[1].diagM, d[1].diagK, d[2].diagM, d[2].diagK, c->n[0], c->n[1], c->N, c->dim, 0,
                     nullptr, S);
  IGAFD_HIP_CHECK(hipGetLastError());
  return IGAFD_OK;
}

}  // namespace igafd

// Host-side univariate setup: knot validation, Gauss-Legendre rule, B-spline
// values at the Gauss points, the 1D mass/stiffness matrices and their
// generalised eigendecomposition.
//
// Paper Sec. 2.1 (eq. knot-vector, eq. cox-deboor-1/2, eq. Vh), Sec. 3 (the
// univariate M_d, K_d) and Sec. 4.1 (generalised eigenproblem by Cholesky of M,
// symmetric eigendecomposition of L^-1 K L^-T, U = L^-T Ut).  The symmetric
// eigensolver is Householder tridiagonalisation plus implicit shifted QR.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

namespace igafd {

namespace {

// Legendre polynomials P_q(z) and P_{q-1}(z) by the three-term recurrence.
void legendre(int q, double z, double* pq, double* pqm1) {
  double p0 = 1.0, p1 = z;
  for (int k = 2; k <= q; ++k) {
    const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *pq = p1;
  *pqm1 = p0;
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on P_q with
// P_q'(z) = q (z P_q - P_{q-1}) / (z^2 - 1).
void gauss_legendre(int q, double* x, double* w) {
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double pq = 0.0, pqm1 = 0.0;
    for (int it = 0; it < 100; ++it) {
      legendre(q, z, &pq, &pqm1);
      const double dz = pq / (q * (z * pq - pqm1) / (z * z - 1.0));
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre(q, z, &pq, &pqm1);
    const double dp = q * (z * pq - pqm1) / (z * z - 1.0);
    x[q - 1 - i] = z;
    w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Values and first derivatives of the p+1 B-splines B_{k-p..k} that are
// nonzero on the span [t_k, t_{k+1}), at x in that span.  The degree is raised
// one step at a time with the two-term recursion (0/0 = 0); the derivative
// combines the degree p-1 values.
void span_basis(const double* t, int p, int k, double x, double* N, double* dN) {
  double cur[kMaxDegree + 2], nxt[kMaxDegree + 2], low[kMaxDegree + 2];
  cur[0] = 1.0;
  low[0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    if (j == p)
      for (int i = 0; i < j; ++i) low[i] = cur[i];
    for (int i = 0; i <= j; ++i) {
      const int g = k - j + i;  // B_{g,j}
      double v = 0.0;
      if (i >= 1) {
        const double den = t[g + j] - t[g];
        if (den > 0.0) v += (x - t[g]) / den * cur[i - 1];
      }
      if (i <= j - 1) {
        const double den = t[g + j + 1] - t[g + 1];
        if (den > 0.0) v += (t[g + j + 1] - x) / den * cur[i];
      }
      nxt[i] = v;
    }
    for (int i = 0; i <= j; ++i) cur[i] = nxt[i];
  }
  for (int i = 0; i <= p; ++i) {
    N[i] = cur[i];
    const int g = k - p + i;
    double d = 0.0;
    if (i >= 1) {
      const double den = t[g + p] - t[g];
      if (den > 0.0) d += p / den * low[i - 1];
    }
    if (i <= p - 1) {
      const double den = t[g + p + 1] - t[g + 1];
      if (den > 0.0) d -= p / den * low[i];
    }
    dN[i] = d;
  }
}

// Runs fn(lo, hi) on contiguous chunks of [0, n) on up to 16 host threads
// (serially when n < 2 * min_chunk).
template <class F>
void parallel_rows(int n, int min_chunk, const F& fn) {
  const unsigned hw = std::thread::hardware_concurrency();
  const int T = (int)std::max(1u, std::min(16u, hw));
  const int chunks = std::min(T, n / std::max(1, min_chunk));
  if (chunks <= 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(chunks);
  for (int t = 0; t < chunks; ++t)
    th.emplace_back(fn, (int)((long long)n * t / chunks), (int)((long long)n * (t + 1) / chunks));
  for (auto& x : th) x.join();
}

// Largest |i - j| with A_ij != 0 (A n x n, row-major).
int bandwidth(const std::vector<double>& A, int n) {
  int bw = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (A[(size_t)i * n + j] != 0.0 || A[(size_t)j * n + i] != 0.0) {
        bw = std::max(bw, i - j);
        break;
      }
  return bw;
}

// Cholesky A = L L^T of a band matrix (bandwidth bw; lower factor in place,
// row-major, upper part zeroed).  The factor keeps the band.  False if not SPD.
bool cholesky(std::vector<double>& A, int n, int bw) {
  for (int j = 0; j < n; ++j) {
    double* aj = &A[(size_t)j * n];
    const int k0 = std::max(0, j - bw);
    double s = aj[j];
    for (int k = k0; k < j; ++k) s -= aj[k] * aj[k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    aj[j] = ljj;
    for (int i = j + 1; i <= std::min(n - 1, j + bw); ++i) {
      double* ai = &A[(size_t)i * n];
      double v = ai[j];
      for (int k = std::max(k0, i - bw); k < j; ++k) v -= ai[k] * aj[k];
      ai[j] = v / ljj;
    }
    for (int k = j + 1; k < n; ++k) aj[k] = 0.0;
  }
  return true;
}

// X <- L^-1 X for a band lower factor L (forward substitution on whole rows).
void forward_rows(const std::vector<double>& L, int n, int bw, std::vector<double>& X) {
  for (int i = 0; i < n; ++i) {
    double* xi = &X[(size_t)i * n];
    for (int k = std::max(0, i - bw); k < i; ++k) {
      const double l = L[(size_t)i * n + k];
      const double* xk = &X[(size_t)k * n];
      for (int j = 0; j < n; ++j) xi[j] -= l * xk[j];
    }
    const double d = L[(size_t)i * n + i];
    for (int j = 0; j < n; ++j) xi[j] /= d;
  }
}

// Symmetric eigensolver: Householder reduction to tridiagonal form followed by
// implicit QR steps with the Wilkinson shift (Golub & Van Loan, Sec. 8.3).
// S (n x n, row-major) is destroyed; on return lam holds the eigenvalues in
// ascending order and V the orthonormal eigenvectors as columns (V[i][k]).
// The QR steps run on the tridiagonal alone; their plane rotations are
// recorded and applied to V afterwards, a block of rows at a time.
void symmetric_eig(std::vector<double>& S, int n, std::vector<double>& lam, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), pv(n);
  constexpr int kMinRows = 128;
  // 1. S = Q T Q^T: reflector k zeroes column k below the subdiagonal
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = S[k+1:, k]
    double nx = 0.0;
    for (int i = 0; i < m; ++i) nx += S[(size_t)(k + 1 + i) * n + k] * S[(size_t)(k + 1 + i) * n + k];
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double x0 = S[(size_t)(k + 1) * n + k];
    const double alpha = x0 >= 0 ? -nx : nx;
    for (int i = 0; i < m; ++i) v[i] = S[(size_t)(k + 1 + i) * n + k];
    v[0] -= alpha;
    double nv = 0.0;
    for (int i = 0; i < m; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    if (nv == 0.0) continue;
    for (int i = 0; i < m; ++i) v[i] /= nv;
    // trailing block B <- H B H = B - 2 v w^T - 2 w v^T, w = B v - (v^T B v) v
    parallel_rows(m, kMinRows, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i) {
        const double* row = &S[(size_t)(k + 1 + i) * n + k + 1];
        double t = 0.0;
        for (int j = 0; j < m; ++j) t += row[j] * v[j];
        pv[i] = t;
      }
    });
    double cvp = 0.0;
    for (int i = 0; i < m; ++i) cvp += v[i] * pv[i];
    for (int i = 0; i < m; ++i) pv[i] -= cvp * v[i];
    parallel_rows(m, kMinRows, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i) {
        double* row = &S[(size_t)(k + 1 + i) * n + k + 1];
        const double vi = 2.0 * v[i], pi = 2.0 * pv[i];
        for (int j = 0; j < m; ++j) row[j] -= vi * pv[j] + pi * v[j];
      }
    });
    S[(size_t)(k + 1) * n + k] = S[(size_t)k * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) S[(size_t)(k + 1 + i) * n + k] = S[(size_t)k * n + k + 1 + i] = 0.0;
    // V <- V H on columns k+1..n-1
    parallel_rows(n, kMinRows, [&](int lo, int hi) {
      for (int r = lo; r < hi; ++r) {
        double* row = &V[(size_t)r * n + k + 1];
        double t = 0.0;
        for (int j = 0; j < m; ++j) t += row[j] * v[j];
        t *= 2.0;
        for (int j = 0; j < m; ++j) row[j] -= t * v[j];
      }
    });
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = S[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = S[(size_t)(i + 1) * n + i];
  // 2. implicit QR steps on unreduced blocks [lo, hi] of the tridiagonal T;
  // rotation j acts on columns (rk[j], rk[j] + 1) of V
  std::vector<int> rk;
  std::vector<double> rc, rs;
  const double eps = 2.2e-16;
  int hi = n - 1, guard = 0;
  while (hi > 0 && guard < 100 * n) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    ++guard;
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    // Wilkinson shift: eigenvalue of the trailing 2x2 closer to d[hi]
    const double delta = 0.5 * (d[hi - 1] - d[hi]);
    const double eh = e[hi - 1];
    const double den = delta + (delta >= 0 ? 1.0 : -1.0) * std::sqrt(delta * delta + eh * eh);
    const double mu = d[hi] - eh * eh / den;
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      // rotation in the (k, k+1) plane taking (x, z) to (r, 0)
      const double r = std::hypot(x, z);
      const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
      if (k > lo) e[k - 1] = r;  // (x, z) were (e[k-1], bulge)
      const double a = d[k], b = e[k], cc = d[k + 1];
      d[k] = c * c * a + 2.0 * c * s * b + s * s * cc;
      d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * cc;
      e[k] = c * s * (cc - a) + (c * c - s * s) * b;
      if (k + 1 < hi) {
        const double next = e[k + 1];
        x = e[k];
        z = s * next;        // new bulge at (k, k+2)
        e[k + 1] = c * next;
      }
      rk.push_back(k);
      rc.push_back(c);
      rs.push_back(s);
    }
  }
  // 3. V <- V G_1 G_2 ...: blocks of B rows, stored transposed so that one
  // rotation updates two contiguous runs of B values
  constexpr int B = 32;
  const size_t nrot = rk.size();
  parallel_rows((n + B - 1) / B, 1, [&](int blo, int bhi) {
    std::vector<double> T((size_t)n * B);
    for (int blk = blo; blk < bhi; ++blk) {
      const int r0 = blk * B, nb = std::min(B, n - r0);
      for (int j = 0; j < nb; ++j)
        for (int k = 0; k < n; ++k) T[(size_t)k * B + j] = V[(size_t)(r0 + j) * n + k];
      for (size_t q = 0; q < nrot; ++q) {
        double* a = &T[(size_t)rk[q] * B];
        double* b = a + B;
        const double c = rc[q], s = rs[q];
        for (int j = 0; j < B; ++j) {
          const double va = a[j], vb = b[j];
          a[j] = c * va + s * vb;
          b[j] = -s * va + c * vb;
        }
      }
      for (int j = 0; j < nb; ++j)
        for (int k = 0; k < n; ++k) V[(size_t)(r0 + j) * n + k] = T[(size_t)k * B + j];
    }
  });
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  lam.resize(n);
  std::vector<double> Vs((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    lam[k] = d[order[k]];
    for (int i = 0; i < n; ++i) Vs[(size_t)i * n + k] = V[(size_t)i * n + order[k]];
  }
  V.swap(Vs);
}

}  // namespace

igafd_status build_direction(int p, int q, int nknots, const double* knots, Dir1D* out, bool eig) {
  if (p < 1 || p > kMaxDegree) {
    set_error("degree must be in 1.." + std::to_string(kMaxDegree));
    return IGAFD_ERR_ARG;
  }
  if (q != p + 1) {
    set_error("the library integrates with p+1 Gauss points per element and direction");
    return IGAFD_ERR_ARG;
  }
  if (!knots || nknots < 2 * p + 2) {
    set_error("knot vector too short for the degree");
    return IGAFD_ERR_ARG;
  }
  const double* t = knots;
  for (int i = 0; i + 1 < nknots; ++i)
    if (!(t[i] <= t[i + 1])) {
      set_error("knots must be nondecreasing");
      return IGAFD_ERR_ARG;
    }
  for (int i = 0; i <= p; ++i)
    if (t[i] != 0.0 || t[nknots - 1 - i] != 1.0) {
      set_error("knot vector must be open on [0,1]");
      return IGAFD_ERR_ARG;
    }
  if (t[p + 1] == 0.0 || t[nknots - p - 2] == 1.0) {
    set_error("end knots repeated more than p+1 times");
    return IGAFD_ERR_ARG;
  }
  for (int i = p + 1; i < nknots - p - 1;) {
    int j = i;
    while (j < nknots - p - 1 && t[j] == t[i]) ++j;
    if (j - i > p) {
      set_error("interior knot multiplicity exceeds p");
      return IGAFD_ERR_ARG;
    }
    i = j;
  }
  Dir1D& d = *out;
  d.p = p;
  d.q = q;
  d.knots.assign(t, t + nknots);
  d.m = nknots - p - 1;
  d.n = d.m - 2;
  if (d.n < 1) {
    set_error("no interior basis functions");
    return IGAFD_ERR_ARG;
  }
  std::vector<double> gx(q), gw(q);
  gauss_legendre(q, gx.data(), gw.data());
  d.elem_first.clear();
  d.qx.clear();
  d.qw.clear();
  d.val.clear();
  d.der.clear();
  for (int k = p; k < d.m; ++k) {
    if (!(t[k] < t[k + 1])) continue;
    d.elem_first.push_back(k - p);
    const double a = t[k], b = t[k + 1];
    for (int s = 0; s < q; ++s) {
      const double x = a + 0.5 * (b - a) * (gx[s] + 1.0);
      d.qx.push_back(x);
      d.qw.push_back(0.5 * (b - a) * gw[s]);
      double N[kMaxDegree + 1], dN[kMaxDegree + 1];
      span_basis(t, p, k, x, N, dN);
      for (int i = 0; i <= p; ++i) {
        d.val.push_back(N[i]);
        d.der.push_back(dN[i]);
      }
    }
  }
  d.nel = (int)d.elem_first.size();
  const int n = d.n;
  d.M.assign((size_t)n * n, 0.0);
  d.K.assign((size_t)n * n, 0.0);
  for (int e = 0; e < d.nel; ++e) {
    for (int s = 0; s < q; ++s) {
      const double w = d.qw[e * q + s];
      const double* v = &d.val[(e * q + s) * (p + 1)];
      const double* dv = &d.der[(e * q + s) * (p + 1)];
      for (int a = 0; a <= p; ++a) {
        const int ia = d.elem_first[e] + a - 1;
        if (ia < 0 || ia >= n) continue;
        for (int b = 0; b <= p; ++b) {
          const int ib = d.elem_first[e] + b - 1;
          if (ib < 0 || ib >= n) continue;
          d.M[ia * n + ib] += w * v[a] * v[b];
          d.K[ia * n + ib] += w * dv[a] * dv[b];
        }
      }
    }
  }
  d.U.clear();
  d.lam.clear();
  if (!eig) return IGAFD_OK;
  // generalised eigendecomposition K U = M U D, U^T M U = I
  const int bw = bandwidth(d.M, n);
  std::vector<double> L = d.M;
  if (!cholesky(L, n, bw)) {
    set_error("Cholesky of the 1D mass matrix failed");
    return IGAFD_ERR_NOT_SPD;
  }
  // S = L^-1 K L^-T = L^-1 (L^-1 K)^T (K symmetric)
  std::vector<double> X = d.K;
  forward_rows(L, n, bw, X);
  std::vector<double> S((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[(size_t)j * n + i] = X[(size_t)i * n + j];
  forward_rows(L, n, bw, S);
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = 0.5 * (S[(size_t)i * n + j] + S[(size_t)j * n + i]);
      S[(size_t)i * n + j] = S[(size_t)j * n + i] = s;
    }
  std::vector<double> Ut;
  symmetric_eig(S, n, d.lam, Ut);
  // U = L^-T Ut: backward substitution on whole rows, L^T upper with band bw
  d.U = Ut;
  for (int i = n - 1; i >= 0; --i) {
    double* ui = &d.U[(size_t)i * n];
    for (int k = i + 1; k <= std::min(n - 1, i + bw); ++k) {
      const double l = L[(size_t)k * n + i];
      const double* uk = &d.U[(size_t)k * n];
      for (int j = 0; j < n; ++j) ui[j] -= l * uk[j];
    }
    const double dd = L[(size_t)i * n + i];
    for (int j = 0; j < n; ++j) ui[j] /= dd;
  }
  return IGAFD_OK;
}

}  // namespace igafd

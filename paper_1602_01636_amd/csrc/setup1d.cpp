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

// Dense Cholesky A = L L^T (lower, row-major, in place).  False if not SPD.
bool cholesky(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    A[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = v / ljj;
    }
    for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
  }
  return true;
}

// Symmetric eigensolver: Householder reduction to tridiagonal form followed by
// implicit QR steps with the Wilkinson shift (Golub & Van Loan, Sec. 8.3).
// S (n x n, row-major) is destroyed; on return lam holds the eigenvalues in
// ascending order and V the orthonormal eigenvectors as columns (V[i][k]).
void symmetric_eig(std::vector<double>& S, int n, std::vector<double>& lam, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), pv(n);
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
    for (int i = 0; i < m; ++i) {
      double t = 0.0;
      for (int j = 0; j < m; ++j) t += S[(size_t)(k + 1 + i) * n + k + 1 + j] * v[j];
      pv[i] = t;
    }
    double cvp = 0.0;
    for (int i = 0; i < m; ++i) cvp += v[i] * pv[i];
    for (int i = 0; i < m; ++i) pv[i] -= cvp * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j)
        S[(size_t)(k + 1 + i) * n + k + 1 + j] -= 2.0 * (v[i] * pv[j] + pv[i] * v[j]);
    S[(size_t)(k + 1) * n + k] = S[(size_t)k * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) S[(size_t)(k + 1 + i) * n + k] = S[(size_t)k * n + k + 1 + i] = 0.0;
    // V <- V H on columns k+1..n-1
    for (int r = 0; r < n; ++r) {
      double t = 0.0;
      for (int j = 0; j < m; ++j) t += V[(size_t)r * n + k + 1 + j] * v[j];
      for (int j = 0; j < m; ++j) V[(size_t)r * n + k + 1 + j] -= 2.0 * t * v[j];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = S[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = S[(size_t)(i + 1) * n + i];
  // 2. implicit QR steps on unreduced blocks [lo, hi] of the tridiagonal T
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
      for (int row = 0; row < n; ++row) {
        double* Vr = &V[(size_t)row * n];
        const double vk = Vr[k], vk1 = Vr[k + 1];
        Vr[k] = c * vk + s * vk1;
        Vr[k + 1] = -s * vk + c * vk1;
      }
    }
  }
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

igafd_status build_direction(int p, int q, int nknots, const double* knots, Dir1D* out) {
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
  // generalised eigendecomposition K U = M U D, U^T M U = I
  std::vector<double> L = d.M;
  if (!cholesky(L, n)) {
    set_error("Cholesky of the 1D mass matrix failed");
    return IGAFD_ERR_NOT_SPD;
  }
  // X = L^-1 K (forward substitution on each column), then S = X L^-T
  std::vector<double> X = d.K;
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = X[i * n + c];
      for (int k = 0; k < i; ++k) v -= L[i * n + k] * X[k * n + c];
      X[i * n + c] = v / L[i * n + i];
    }
  std::vector<double> S((size_t)n * n);
  for (int r = 0; r < n; ++r)  // row r of S solves L s = X[r,:]^T  (S = X L^-T)
    for (int i = 0; i < n; ++i) {
      double v = X[r * n + i];
      for (int k = 0; k < i; ++k) v -= L[i * n + k] * S[r * n + k];
      S[r * n + i] = v / L[i * n + i];
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double s = 0.5 * (S[i * n + j] + S[j * n + i]);
      S[i * n + j] = S[j * n + i] = s;
    }
  std::vector<double> Ut;
  symmetric_eig(S, n, d.lam, Ut);
  // U = L^-T Ut: back substitution with L^T on each column
  d.U.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double v = Ut[i * n + c];
      for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * d.U[k * n + c];
      d.U[i * n + c] = v / L[i * n + i];
    }
  return IGAFD_OK;
}

}  // namespace igafd

// Host eigensolvers for the Lanczos matrix and the Rayleigh-Ritz
// projection.  Symmetric tridiagonal: the implicit QL algorithm with
// Wilkinson-type shifts (Dubrulle, Martin and Wilkinson, Numer. Math. 12,
// 1968, the procedure known as imtql2).  Dense symmetric: Householder
// reduction to tridiagonal form (Golub and Van Loan, Sec. 8.3) followed by
// the tridiagonal solver.  Both run in O(n^3); the work on the rows of the
// eigenvector matrix (and of the matrix being reduced) is shared among the
// host's threads with OpenMP once n reaches the thousands that thousands of
// wanted pairs bring (about 3,000 Lanczos vectors for 1,500 pairs).  Each
// QL sweep first computes its rotations and then applies them row by row,
// every row in the same order as a rotation-by-rotation update would.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

#include "eig.hpp"

namespace polfed {

namespace {

// Rows updated per thread below which a loop stays serial.
constexpr long kParWork = 1L << 16;

// Applies the rotations of one QL sweep, recorded for i = i_hi down to
// i_lo, to every row of Z: (z_i, z_{i+1}) <- (c z_i - s z_{i+1}, s z_i + c z_{i+1}).
void apply_sweep(int n, std::vector<double>& Z, int nz, int i_hi, int i_lo,
                 const std::vector<double>& cs, const std::vector<double>& sn) {
  if (i_hi < i_lo) return;
  const long work = (long)nz * (i_hi - i_lo + 1);
#pragma omp parallel for schedule(static) if (work > kParWork)
  for (int k = 0; k < nz; ++k) {
    double* zk = &Z[(size_t)k * n];
    for (int i = i_hi; i >= i_lo; --i) {
      const double c = cs[i], s = sn[i];
      const double zf = zk[i + 1];
      zk[i + 1] = s * zk[i] + c * zf;
      zk[i] = c * zk[i] - s * zf;
    }
  }
}

}  // namespace

void tridiag_eig(int n, std::vector<double>& d, std::vector<double> e,
                 std::vector<double>& Z, int nz) {
  if (n <= 0) return;
  e.resize(n, 0.0);
  e[n - 1] = 0.0;
  const double eps = 2.220446049250313e-16;
  std::vector<double> cs(n), sn(n);
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 200) throw std::runtime_error("tridiagonal QL did not converge");
      // shift from the leading 2x2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // underflow: split and restart
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        cs[i] = c;
        sn[i] = s;
      }
      // the rotations of this sweep: i = m - 1 down to the last one done
      apply_sweep(n, Z, nz, m - 1, deflated ? i + 1 : l, cs, sn);
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // ascending order, columns of Z alike
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  std::vector<double> d2(n), Z2((size_t)nz * n);
  for (int j = 0; j < n; ++j) {
    d2[j] = d[idx[j]];
    for (int k = 0; k < nz; ++k) Z2[(size_t)k * n + j] = Z[(size_t)k * n + idx[j]];
  }
  d.swap(d2);
  Z.swap(Z2);
}

namespace {

// Householder reduction of the symmetric row-major a to tridiagonal form,
// a = Q T Q^T; Q keeps only its rows q0..n-1 ((n - q0) x n, row-major),
// which start as the matching rows of the identity.
void tridiagonalize(int n, std::vector<double>& a, std::vector<double>& Q, int q0,
                    std::vector<double>& d, std::vector<double>& e) {
  const int nq = n - q0;
  Q.assign((size_t)nq * n, 0.0);
  for (int i = 0; i < nq; ++i) Q[(size_t)i * n + q0 + i] = 1.0;
  std::vector<double> v(n), p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double xn = 0;
    for (int i = 0; i < m; ++i) xn += a[(size_t)(k + 1 + i) * n + k] * a[(size_t)(k + 1 + i) * n + k];
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double x0 = a[(size_t)(k + 1) * n + k];
    const double alpha = x0 >= 0 ? -xn : xn;
    for (int i = 0; i < m; ++i) v[i] = a[(size_t)(k + 1 + i) * n + k];
    v[0] -= alpha;
    double vv = 0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // p = beta * A_sub v
    const bool par = (long)m * m > kParWork;
#pragma omp parallel for schedule(static) if (par)
    for (int i = 0; i < m; ++i) {
      double t = 0;
      const double* row = &a[(size_t)(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) t += row[j] * v[j];
      p[i] = beta * t;
    }
    double vp = 0;
    for (int i = 0; i < m; ++i) vp += v[i] * p[i];
    const double Kc = 0.5 * beta * vp;
    for (int i = 0; i < m; ++i) q[i] = p[i] - Kc * v[i];
#pragma omp parallel for schedule(static) if (par)
    for (int i = 0; i < m; ++i) {
      double* row = &a[(size_t)(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * q[j] + q[i] * v[j];
    }
    a[(size_t)(k + 1) * n + k] = alpha;
    a[(size_t)k * n + (k + 1)] = alpha;
    for (int i = 1; i < m; ++i) {
      a[(size_t)(k + 1 + i) * n + k] = 0.0;
      a[(size_t)k * n + (k + 1 + i)] = 0.0;
    }
    // Q <- Q H on columns k+1..n-1
#pragma omp parallel for schedule(static) if ((long)nq * m > kParWork)
    for (int r = 0; r < nq; ++r) {
      double* qr = &Q[(size_t)r * n + (k + 1)];
      double t = 0;
      for (int j = 0; j < m; ++j) t += qr[j] * v[j];
      t *= beta;
      for (int j = 0; j < m; ++j) qr[j] -= t * v[j];
    }
  }
  d.assign(n, 0.0);
  e.assign(n > 1 ? n - 1 : 0, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)(i + 1) * n + i];
}

std::vector<double> symmetric_copy(int n, const std::vector<double>& A) {
  std::vector<double> a((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      a[(size_t)i * n + j] = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
  return a;
}

}  // namespace

void sym_eig(int n, std::vector<double>& A, std::vector<double>& w,
             std::vector<double>& Zout) {
  // Work row-major on a symmetric copy (A is col-major; symmetric anyway).
  std::vector<double> a = symmetric_copy(n, A), Q, d, e;
  tridiagonalize(n, a, Q, 0, d, e);
  tridiag_eig(n, d, e, Q, n);  // Q rows: components, columns: eigenvectors
  w = d;
  Zout.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Zout[(size_t)j * n + i] = Q[(size_t)i * n + j];
}

void sym_eig_tail(int n, const std::vector<double>& A, int r, std::vector<double>& w,
                  std::vector<double>& Ztail) {
  std::vector<double> a = symmetric_copy(n, A), d, e;
  r = std::min(std::max(r, 1), n);
  tridiagonalize(n, a, Ztail, n - r, d, e);
  tridiag_eig(n, d, e, Ztail, r);
  w = d;
}

}  // namespace polfed

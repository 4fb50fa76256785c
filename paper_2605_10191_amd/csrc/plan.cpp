// Filter plan (Secs. 3.2, 4.1 and 4.2 of the paper), host side.
//
// With c_0 = 1, c_n = 2 cos(n phi), phi = arccos(lambda~) (eq.
// transformationCoefficients) and x = cos(theta),
//   sum_{n=0}^{K} c_n T_n(x) = [D_K(theta - phi) + D_K(theta + phi)] / 2,
// where D_K(u) = 1 + 2 sum_{n=1}^{K} cos(n u) = sin((K + 1/2) u) / sin(u / 2)
// is the Dirichlet kernel; chi is the same sum at theta = phi.  So the
// normalized filter of eq. transformation has the closed form
//   P(cos theta) = [D_K(theta - phi) + D_K(theta + phi)] / [D_K(0) + D_K(2 phi)],
// evaluated here in O(1), which makes the bisection of eq. condition_for_K
// cheap at any K.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace polfed {

static double dirichlet(int K, double u) {
  // D_K is even and 2 pi periodic: fold u into [0, pi]
  u = std::fabs(std::remainder(u, 2.0 * M_PI));
  if (u == 0.0) return 2.0 * K + 1.0;
  return std::sin((K + 0.5) * u) / std::sin(0.5 * u);
}

double filter_value_closed(double lambda_t, int K, double x) {
  x = std::min(1.0, std::max(-1.0, x));
  const double phi = std::acos(std::min(1.0, std::max(-1.0, lambda_t)));
  const double th = std::acos(x);
  const double num = dirichlet(K, th - phi) + dirichlet(K, th + phi);
  const double den = dirichlet(K, 0.0) + dirichlet(K, 2.0 * phi);
  return num / den;
}

void filter_coefficients(double lambda_t, int K, double* a) {
  const double phi = std::acos(std::min(1.0, std::max(-1.0, lambda_t)));
  const double chi = 0.5 * (dirichlet(K, 0.0) + dirichlet(K, 2.0 * phi));
  a[0] = 1.0 / chi;
  for (int n = 1; n <= K; ++n) a[n] = 2.0 * std::cos(n * phi) / chi;
}

// Divided difference of a Chebyshev series p(x) = sum_{n=0}^{K} a_n T_n(x)
// at theta: Q(x) = (p(x) - p(theta)) / (x - theta), a polynomial of degree
// K - 1.  With the Clenshaw intermediates at theta,
//   b_{K+1} = b_{K+2} = 0,  b_k = a_k + 2 theta b_{k+1} - b_{k+2},
// one has b_k = sum_{n >= k} a_n U_{n-k}(theta), and expanding
// (T_n(x) - T_n(theta)) / (x - theta) in U_k(x) with T-valued weights, then
// U_k in T_j, telescopes to
//   Q(x) = b_1 T_0(x) + 2 sum_{j=1}^{K-1} b_{j+1} T_j(x),
// while p(theta) = a_0 + theta b_1 - b_2.  q receives K coefficients
// (none for K = 0, where Q = 0).
void filter_quotient(const double* a, int K, double theta, double* q, double* p_theta) {
  double b1 = 0.0, b2 = 0.0;  // b_{k+1}, b_{k+2}
  for (int k = K; k >= 1; --k) {
    const double bk = a[k] + 2.0 * theta * b1 - b2;
    b2 = b1;
    b1 = bk;
    if (k >= 2) q[k - 1] = 2.0 * bk;  // q_{k-1} = 2 b_k
    else if (K >= 1) q[0] = bk;       // q_0 = b_1
  }
  if (p_theta) *p_theta = a[0] + theta * b1 - b2;
}

static bool meets_cutoff(int K, double lt, double delta, double omega) {
  const double lo = filter_value_closed(lt, K, lt - delta);
  const double hi = filter_value_closed(lt, K, lt + delta);
  return std::min(lo, hi) >= omega;
}

// Largest K with min P^K(lambda~ +- delta) >= Omega (eq. condition_for_K),
// bisection from the bracket [K_approx / 2, 2 K_approx] of Sec. 4.2, widened
// when the estimate misses.
static int choose_K(double lt, double delta, double omega, double K0) {
  const int64_t cap = 100000000;
  int64_t lo = std::max<int64_t>(1, (int64_t)std::floor(K0 / 2));
  int64_t hi = std::max<int64_t>(lo + 1, (int64_t)std::ceil(2 * K0));
  while (lo > 1 && !meets_cutoff((int)lo, lt, delta, omega)) lo = std::max<int64_t>(1, lo / 2);
  if (!meets_cutoff((int)lo, lt, delta, omega)) return 1;
  while (meets_cutoff((int)hi, lt, delta, omega)) {
    lo = hi;
    hi = 2 * hi;
    if (hi > cap) return (int)cap;
  }
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (meets_cutoff((int)mid, lt, delta, omega)) lo = mid;
    else hi = mid;
  }
  return (int)lo;
}

int expected_krylov_dim(int howmany, int blocksize, double eta) {
  return (int)std::ceil((20.427 * blocksize + 1.696 * howmany) * eta);
}

polfed_plan make_plan(int64_t D, double E_min, double E_max, double pad,
                      double lambda, double tr1, double tr2, int n_window,
                      double omega, int K_override, const double* kpm_mu, int kpm_n) {
  REQUIRE(D >= 1, "plan: empty operator");
  REQUIRE(std::isfinite(E_min) && std::isfinite(E_max) && E_max > E_min,
          "plan: need finite E_min < E_max");
  REQUIRE(pad >= 0 && std::isfinite(pad), "plan: bad pad");
  REQUIRE(std::isfinite(lambda), "plan: non-finite target");
  REQUIRE(n_window >= 1, "plan: n_window must be >= 1");
  if (!(omega > 0)) omega = kOmegaDefault;
  REQUIRE(omega < 1.0, "plan: cutoff must lie below 1");
  polfed_plan p{};
  const double w = E_max - E_min;
  const double lo = E_min - pad * w, hi = E_max + pad * w;
  p.E_c = 0.5 * (hi + lo);
  p.dE = 0.5 * (hi - lo);
  p.lambda_t = (lambda - p.E_c) / p.dE;
  REQUIRE(p.lambda_t > -1.0 && p.lambda_t < 1.0, "plan: target outside the spectrum");
  p.mu_t = (tr1 - p.E_c) / p.dE;
  p.Gamma_t = std::sqrt(std::max(tr2 - tr1 * tr1, 0.0)) / p.dE;
  if (!(p.Gamma_t > 0)) p.Gamma_t = 1e-300;
  const double z = (p.lambda_t - p.mu_t) / p.Gamma_t;
  p.rho = (double)D / (std::sqrt(2.0 * M_PI) * p.Gamma_t) * std::exp(-0.5 * z * z);
  if (kpm_n > 0) {
    // KPM density at the target (Sec. 4.1 eq. dos_kpm); a stochastic
    // estimate that is not positive there leaves the Gaussian one
    double r = 0;
    kpm_density(kpm_mu, kpm_n, &p.lambda_t, 1, &r);
    if (r > 0 && std::isfinite(r)) p.rho = r;
  }
  p.delta = n_window / (2.0 * p.rho);
  p.K_approx = 2.655 * std::sqrt(std::max(0.0, 1.0 - p.lambda_t * p.lambda_t)) / p.delta;
  if (K_override > 0) {
    p.K = K_override;
  } else if (!(p.rho > 0) || !std::isfinite(p.delta)) {
    p.K = 1;  // no density at the target: the lowest order will do
  } else {
    p.K = choose_K(p.lambda_t, p.delta, omega, p.K_approx);
  }
  return p;
}

}  // namespace polfed

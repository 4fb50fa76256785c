// Kernel polynomial method for the density of states (Sec. 4.1 eq. dos_kpm
// and App. B): stochastic Chebyshev moments mu_n = Tr T_n(H~), estimated as
// the mean over R random vectors r of <r|T_n(H~)|r>, and the Jackson-damped
// density rho_KPM(x) = [mu_0 g_0 + 2 sum_{n>=1} mu_n g_n T_n(x)] /
// (pi sqrt(1 - x^2)).  The recurrence t_{n+1} = 2 H~ t_n - t_{n-1} is the
// fused Clenshaw step with a = 0 (out = sigma H t_n + tau t_n - t_{n-1},
// written over t_{n-1}), so the moments run on the same kernels as the filter.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace polfed {

void kpm_moments(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE, int N, int R,
                 const double* rvecs, uint64_t seed, double* mu) {
  REQUIRE(N >= 1 && R >= 1, "kpm: need N >= 1 moments and R >= 1 vectors");
  REQUIRE(dE > 0 && std::isfinite(dE) && std::isfinite(E_c), "kpm: need finite E_c, dE > 0");
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  const size_t nd = (size_t)std::max<int64_t>(D, 1);
  DevBuf r(nd * sizeof(double)), ta(nd * sizeof(double)), tb(nd * sizeof(double)),
      dots((size_t)N * R * sizeof(double)), part(8192 * sizeof(double));
  for (int c = 0; c < R; ++c) {
    const double* rv;
    if (rvecs) {
      rv = rvecs + (size_t)c * D;
    } else {
      // uniform on [-sqrt 3, sqrt 3): zero mean, unit variance
      dev_random(s, D, seed + (uint64_t)c, r.as<double>());
      dev_axpby(s, D, 0.0, r.as<double>(), std::sqrt(3.0), r.as<double>());
      rv = r.as<double>();
    }
    double* out = dots.as<double>() + (size_t)c * N;
    // t_0 = r
    dev_dot(s, D, rv, rv, part.as<double>(), 1024, out, 0);
    if (N == 1) continue;
    // t_1 = H~ r into ta
    op_step<double>(s, op, 1.0 / dE, -E_c / dE, 0.0, nullptr, rv, nullptr, ta.as<double>());
    dev_dot(s, D, rv, ta.as<double>(), part.as<double>(), 1024, out + 1, 0);
    // t_{n+1} = 2 H~ t_n - t_{n-1}: cur = t_n, prev = t_{n-1} (prev is
    // overwritten); t_0 is r itself, so the first update writes to tb
    const double* cur = ta.as<double>();
    const double* prev = rv;
    for (int n = 2; n < N; ++n) {
      double* nxt = (prev == rv) ? tb.as<double>() : const_cast<double*>(prev);
      op_step<double>(s, op, 2.0 / dE, -2.0 * E_c / dE, 0.0, nullptr, cur, prev, nxt);
      dev_dot(s, D, rv, nxt, part.as<double>(), 1024, out + n, 0);
      prev = cur;
      cur = nxt;
    }
  }
  std::vector<double> h((size_t)N * R);
  HIPC(hipMemcpyAsync(h.data(), dots.get(), h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  for (int n = 0; n < N; ++n) {
    double acc = 0;
    for (int c = 0; c < R; ++c) acc += h[(size_t)c * N + n];
    mu[n] = acc / R;
  }
}

// Jackson factors g_n for N moments (App. B eq. kernels_jackson_and_lorenz).
static double jackson(int n, int N) {
  const double a = M_PI / (N + 1);
  return ((N - n + 1) * std::cos(a * n) + std::sin(a * n) / std::tan(a)) / (N + 1);
}

void kpm_density(const double* mu, int N, const double* x, int nx, double* rho) {
  REQUIRE(N >= 1, "kpm: need N >= 1 moments");
  std::vector<double> c(N);
  for (int n = 0; n < N; ++n) c[n] = (n == 0 ? 1.0 : 2.0) * mu[n] * jackson(n, N);
  for (int j = 0; j < nx; ++j) {
    const double t = x[j];
    REQUIRE(t > -1.0 && t < 1.0, "kpm: evaluation points must lie in (-1, 1)");
    // sum_n c_n T_n(t) by Clenshaw's recurrence
    double b1 = 0, b2 = 0;
    for (int n = N - 1; n >= 1; --n) {
      const double b = c[n] + 2.0 * t * b1 - b2;
      b2 = b1;
      b1 = b;
    }
    const double sum = c[0] + t * b1 - b2;
    rho[j] = sum / (M_PI * std::sqrt(1.0 - t * t));
  }
}

double kpm_maxdos(const double* mu, int N, double lo, double hi) {
  constexpr int kGrid = 4096;
  std::vector<double> x;
  for (int j = 0; j < kGrid; ++j) {
    const double t = std::cos(M_PI * (j + 0.5) / kGrid);
    if (t >= lo && t <= hi) x.push_back(t);
  }
  REQUIRE(!x.empty(), "kpm: empty search interval");
  std::vector<double> rho(x.size());
  kpm_density(mu, N, x.data(), (int)x.size(), rho.data());
  return x[std::max_element(rho.begin(), rho.end()) - rho.begin()];
}

}  // namespace polfed

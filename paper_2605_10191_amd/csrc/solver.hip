// POLFED driver on one GPU (Sec. 4.6 of the paper): spectral bounds by
// Lanczos, the filter plan, Lanczos on P(H~) with the Clenshaw filter and
// full reorthogonalization (classical Gram-Schmidt, two passes), periodic
// convergence checks on the tridiagonal Lanczos matrix, and the extraction
// u = V t refined by Rayleigh-Ritz with H.
//
// Everything of size D stays on the device.  The host sees only the Lanczos
// coefficients (copied at the periodic checks) and the small projected
// matrices of the extraction.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>
#include <string>

#include "internal.hpp"
#include "solve_run.hpp"

namespace polfed {

bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("POLFED_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

int pattern_choice(const polfed_op* op, const std::string& what) {
  if (!op || op->pattern_key.empty()) return -1;
  std::lock_guard<std::mutex> lk(op->ctx->tune_mu);
  auto it = op->ctx->pattern_tuned.find(op->pattern_key + "|" + what);
  return it == op->ctx->pattern_tuned.end() ? -1 : it->second;
}

void pattern_choice_set(const polfed_op* op, const std::string& what, int v) {
  if (!op || op->pattern_key.empty()) return;
  std::lock_guard<std::mutex> lk(op->ctx->tune_mu);
  op->ctx->pattern_tuned[op->pattern_key + "|" + what] = v;
}

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Algorithmic HBM bytes of one Clenshaw step on one vector: v, b1, b2 read
// and out written, plus the matrix stream of CSR storage.
double step_bytes(const polfed_op* op, int precision) {
  const double w = precision == POLFED_FP32 ? 4.0 : 8.0;
  double b = 4.0 * w * (double)op->D;
  if (op->model == Model::Qrem) b += w * (double)op->D;  // the energies E_a
  if (op->storage == POLFED_CSR) {
    // column index plus the value, its one-byte code, or nothing (one value)
    const double per = op->ncode == 1 ? 4.0 : (op->ncode > 1 ? 5.0 : w + 4.0);
    b += (double)op->nnz * per + 8.0 * (double)(op->D + 1) + w * (double)op->D;
  }
  return b;
}

// ------------------------------------------------------- filter apply ----

template <typename T>
__global__ void k_scale_t(int64_t n, T a, const T* x, T* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

template <typename T>
static void scale_t(hipStream_t s, int64_t n, T a, const T* x, T* y) {
  if (!n) return;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256));
  hipLaunchKernelGGL((k_scale_t<T>), dim3(g), dim3(256), 0, s, n, a, x, y);
  HIPC(hipGetLastError());
}

// w = P(H~) v, eq. clenshaw_chebyshev_prod: b_{K+1} = b_{K+2} = 0,
// b_i = a_i v + 2 H~ b_{i+1} - b_{i+2} for i = K..1, then
// w = a_0 v + H~ b_1 - b_2.  b_i overwrites b_{i+2} in place, so two buffers
// carry the recurrence.
template <typename T>
void filter_apply_on(hipStream_t s, const polfed_op* op, double E_c, double dE,
                     const double* a, int K, const T* v, T* w, T* bufA, T* bufB) {
  const int64_t D = op->D;
  const T sigma = (T)(2.0 / dE), tau = (T)(-2.0 * E_c / dE);
  if (K == 0) {
    scale_t<T>(s, D, (T)a[0], v, w);
    return;
  }
  scale_t<T>(s, D, (T)a[K], v, bufA);  // b_K
  const T* cur = bufA;                  // b_{i+1}
  T* prev = nullptr;                    // b_{i+2}
  for (int i = K - 1; i >= 1; --i) {
    T* out = prev ? prev : bufB;
    op_step<T>(s, op, sigma, tau, (T)a[i], v, cur, prev, out);
    prev = const_cast<T*>(cur);
    cur = out;
  }
  op_step<T>(s, op, (T)(0.5 * sigma), (T)(0.5 * tau), (T)a[0], v, cur, prev, w);
}

template <typename T>
void filter_apply(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE,
                  const double* a, int K, const T* v, T* w, T* bufA, T* bufB) {
  filter_apply_on<T>(ctx->stream, op, E_c, dE, a, K, v, w, bufA, bufB);
}

template void filter_apply_on<double>(hipStream_t, const polfed_op*, double, double,
                                      const double*, int, const double*, double*, double*,
                                      double*);
template void filter_apply_on<float>(hipStream_t, const polfed_op*, double, double,
                                     const double*, int, const float*, float*, float*,
                                     float*);
template void filter_apply<double>(polfed_ctx*, const polfed_op*, double, double,
                                   const double*, int, const double*, double*,
                                   double*, double*);
template void filter_apply<float>(polfed_ctx*, const polfed_op*, double, double,
                                  const double*, int, const float*, float*, float*,
                                  float*);

// ------------------------------------------------------------ Lanczos ----

namespace {

// w <- w - V V^T w twice over the first k1 basis vectors; the first column
// projection of each pass adds up alpha[k]; then beta_next = ||w|| and
// v_next = w / beta_next.
void cgs2_raw(hipStream_t s, int64_t D, int k1, const double* V, double* w,
              double* c, double* partial, int64_t nseg, int* flag, double* alpha_k,
              double* beta_next, double* v_next) {
  for (int pass = 0; pass < 2; ++pass) {
    dev_gemv_t(s, D, k1, V, D, w, partial, nseg, c, alpha_k, pass);
    dev_gemv_n_sub(s, D, k1, V, D, c, w);
  }
  dev_dot(s, D, w, w, partial, 1024, beta_next, 1);
  dev_scale_into(s, D, w, beta_next, v_next, flag);
}

void cgs2_normalize(hipStream_t s, int64_t D, int k1, const Basis& B, Ws& ws,
                    double* alpha_k, double* beta_next, double* v_next) {
  cgs2_raw(s, D, k1, B.V.as<double>(), ws.w.as<double>(), ws.c.as<double>(),
           ws.partial.as<double>(), ws.nseg, ws.flag.as<int>(), alpha_k, beta_next,
           v_next);
}

void normalize_into(hipStream_t s, int64_t D, const double* x, Ws& ws, double* out) {
  double* nrm = ws.scal.as<double>();
  dev_dot(s, D, x, x, ws.partial.as<double>(), 1024, nrm, 1);
  dev_scale_into(s, D, x, nrm, out, ws.flag.as<int>());
}

// Lanczos breakdown at step k (the Krylov space of the start vector is an
// invariant subspace): v_k becomes a random unit vector orthogonal to
// v_0..v_{k-1}, and beta_k = 0 decouples the Lanczos matrix there.
void restart_random(hipStream_t s, int64_t D, int k, const Basis& B, Ws& ws, uint64_t seed) {
  double* w = ws.w.as<double>();
  dev_random(s, D, seed, w);
  double* junk = ws.scal.as<double>() + 8;
  for (int pass = 0; pass < 2; ++pass) {
    dev_gemv_t(s, D, k, B.V.as<double>(), D, w, ws.partial.as<double>(), ws.nseg,
               ws.c.as<double>(), junk, 0);
    dev_gemv_n_sub(s, D, k, B.V.as<double>(), D, ws.c.as<double>(), w);
  }
  const double zero = 0.0;
  HIPC(hipMemcpyAsync(ws.beta.as<double>() + k, &zero, sizeof(double), hipMemcpyHostToDevice, s));
  normalize_into(s, D, w, ws, B.col(k));
  HIPC(hipMemsetAsync(ws.flag.get(), 0, sizeof(int), s));
  HIPC(hipStreamSynchronize(s));
}

// First breakdown at an index in [from, k]: beta_i below 1e-13 times the
// largest Lanczos coefficient before it; -1 if none.
int first_breakdown(int from, int k, const std::vector<double>& al,
                    const std::vector<double>& be, double floor_scale) {
  double scale = floor_scale;
  for (int i = 1; i <= k; ++i) {
    scale = std::max({scale, std::fabs(al[i - 1]), i > 1 ? be[i - 1] : 0.0});
    if (i >= from && be[i] <= 1e-13 * scale) return i;
  }
  return -1;
}

void apply_H(hipStream_t s, const polfed_op* op, const double* x, double* y) {
  op_step<double>(s, op, 1.0, 0.0, 0.0, nullptr, x, nullptr, y);
}

// Tridiagonal Lanczos matrix from alpha[0..m) and beta[1..m).
void ritz_last(int m, const std::vector<double>& al, const std::vector<double>& be,
               std::vector<double>& theta, std::vector<double>& zlast) {
  theta.assign(al.begin(), al.begin() + m);
  std::vector<double> e(m > 1 ? m - 1 : 0);
  for (int i = 0; i + 1 < m; ++i) e[i] = be[i + 1];
  std::vector<double> Z((size_t)m, 0.0);
  Z[m - 1] = 1.0;  // track the last component only
  tridiag_eig(m, theta, e, Z, 1);
  zlast = Z;
}

void ritz_full(int m, const std::vector<double>& al, const std::vector<double>& be,
               std::vector<double>& theta, std::vector<double>& Y /* m x m row-major */) {
  theta.assign(al.begin(), al.begin() + m);
  std::vector<double> e(m > 1 ? m - 1 : 0);
  for (int i = 0; i + 1 < m; ++i) e[i] = be[i + 1];
  Y.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Y[(size_t)i * m + i] = 1.0;
  tridiag_eig(m, theta, e, Y, m);
}

template <typename T>
void dcopy_async(hipStream_t s, T* dst, const T* src, size_t n, hipMemcpyKind k) {
  if (n) HIPC(hipMemcpyAsync(dst, src, n * sizeof(T), k, s));
}

}  // namespace

void bounds(polfed_ctx* ctx, const polfed_op* op, const double* x0, double tol,
            int max_iter, double* E_min, double* E_max, int* iters) {
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  REQUIRE(D >= 1, "bounds: empty operator");
  if (!(tol > 0)) tol = 1e-10;
  if (max_iter <= 0) max_iter = 300;
  const int cap = (int)std::min<int64_t>(max_iter, D);
  Basis B;
  B.ensure(s, D, cap, 0);
  Ws ws;
  ws.init(s, D, cap + 1, false);
  normalize_into(s, D, x0, ws, B.col(0));
  std::vector<double> al(cap + 1), be(cap + 2);
  double lo = 0, hi = 0;
  int k = 0, restarts = 0, brk_from = 1;
  for (;;) {
    apply_H(s, op, B.col(k), ws.w.as<double>());
    cgs2_normalize(s, D, k + 1, B, ws, ws.alpha.as<double>() + k,
                   ws.beta.as<double>() + k + 1, B.col(k + 1));
    ++k;
    const bool last = k >= cap;
    if (k % 10 == 0 || last) {
      HIPC(hipMemcpyAsync(al.data(), ws.alpha.get(), k * sizeof(double),
                          hipMemcpyDeviceToHost, s));
      HIPC(hipMemcpyAsync(be.data(), ws.beta.get(), (k + 1) * sizeof(double),
                          hipMemcpyDeviceToHost, s));
      HIPC(hipStreamSynchronize(s));
      for (int i = 0; i < k; ++i)
        if (!std::isfinite(al[i]) || !std::isfinite(be[i + 1]))
          fail(POLFED_ERR_INVALID, "bounds: non-finite Lanczos coefficient");
      // a start vector inside an invariant subspace: continue from a random
      // direction orthogonal to it, so that the bounds cover the spectrum
      const int kb = first_breakdown(brk_from, k, al, be, 0.0);
      if (kb > 0 && kb < cap && restarts < 8) {
        ++restarts;
        k = kb;
        restart_random(s, D, k, B, ws, 0xB0D5ULL + (uint64_t)restarts);
        brk_from = k + 1;
        continue;
      }
      std::vector<double> th, zl;
      ritz_last(k, al, be, th, zl);
      lo = th.front();
      hi = th.back();
      const double r_lo = std::fabs(be[k] * zl.front()), r_hi = std::fabs(be[k] * zl.back());
      const double width = std::max(hi - lo, 1e-300);
      const bool brk = be[k] <= 1e-13 * std::max(std::fabs(lo), std::fabs(hi));
      if ((r_lo <= tol * width && r_hi <= tol * width) || last || brk) break;
    }
  }
  *E_min = lo;
  *E_max = hi;
  if (iters) *iters = k;
}

// ------------------------------------------------------------- solve ----

namespace {

int buffer_size(int n_ev) { return std::max(10, (int)std::ceil(0.2 * n_ev)); }

double target_energy(int kind, double target, double E_min, double E_max, double mean) {
  switch (kind) {
    case POLFED_TARGET_ABSOLUTE: return target;
    case POLFED_TARGET_RESCALED: return 0.5 * (E_max + E_min) + target * 0.5 * (E_max - E_min);
    case POLFED_TARGET_NORMALIZED: return E_min + target * (E_max - E_min);
    case POLFED_TARGET_MAXDOS: return mean;  // peak of the Gaussian DOS estimate
    case POLFED_TARGET_OFFSET: {
      // from the DOS peak toward an edge, linearly in rescaled coordinates
      REQUIRE(target >= -1.0 && target <= 1.0, "offset target must lie in [-1, 1]");
      const double c = 0.5 * (E_max + E_min), h = 0.5 * (E_max - E_min);
      const double em = (mean - c) / h;
      const double e = target >= 0 ? em + target * (1.0 - em) : em + target * (1.0 + em);
      return c + e * h;
    }
  }
  fail(POLFED_ERR_INVALID, "unknown target kind");
}

}  // namespace

void rayleigh_ritz(hipStream_t s, int64_t D, int n, const double* U, const double* HU,
                   int64_t nseg, Extracted& ex) {
  DevBuf dG((size_t)n * n * sizeof(double));
  DevBuf part((size_t)nseg * n * sizeof(double) + 8192 * sizeof(double));
  dev_gemm_tn(s, D, n, n, U, D, HU, D, dG.as<double>(), n);
  std::vector<double> w;
  DevBuf dZ, dE((size_t)n * sizeof(double)), dR((size_t)n * sizeof(double));
  std::vector<double> G((size_t)n * n);
  dcopy_async(s, G.data(), dG.as<double>(), G.size(), hipMemcpyDeviceToHost);
  HIPC(hipStreamSynchronize(s));
  // symmetrize: G is symmetric up to rounding
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const double m = 0.5 * (G[(size_t)i * n + j] + G[(size_t)j * n + i]);
      G[(size_t)i * n + j] = G[(size_t)j * n + i] = m;
    }
  std::vector<double> Z;
  sym_eig(n, G, w, Z);
  dZ = std::move(dG);
  dcopy_async(s, dZ.as<double>(), Z.data(), Z.size(), hipMemcpyHostToDevice);
  dcopy_async(s, dE.as<double>(), w.data(), w.size(), hipMemcpyHostToDevice);
  DevBuf U2((size_t)D * n * sizeof(double)), HU2((size_t)D * n * sizeof(double));
  dev_gemm_nn(s, D, n, n, U, D, dZ.as<double>(), n, U2.as<double>(), D, false);
  dev_gemm_nn(s, D, n, n, HU, D, dZ.as<double>(), n, HU2.as<double>(), D, false);
  dev_resid(s, D, n, U2.as<double>(), HU2.as<double>(), dE.as<double>(), part.as<double>(),
            nseg, dR.as<double>());
  ex.res.resize(n);
  dcopy_async(s, ex.res.data(), dR.as<double>(), (size_t)n, hipMemcpyDeviceToHost);
  HIPC(hipStreamSynchronize(s));
  ex.E = w;
  ex.U2 = std::move(U2);
  ex.HU2 = std::move(HU2);
}

// The n_ev pairs nearest lambda, ordered by (|E - lambda|, E), once they are
// all accepted, and the check that no nearer eigenvalue can be missing: the
// filter at the farthest selected energy must not fall below the smallest
// converged P-Ritz value theta_min.
void select_pairs(Extracted& ex, double lam, int n_ev, double tol_resid, double theta_min,
                  const polfed_plan& pl) {
  const int n = (int)ex.E.size();
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double da = std::fabs(ex.E[a] - lam), db = std::fabs(ex.E[b] - lam);
    if (da != db) return da < db;
    return ex.E[a] < ex.E[b];
  });
  // the leading accepted run of the n_ev nearest Ritz pairs: a pair nearer
  // to lambda than an accepted one but not converged yet is not skipped (the
  // selection would otherwise take a farther pair in its place, and the
  // completeness test, which argues only about the extracted values, would
  // not notice)
  std::vector<int> ok;
  for (int q = 0; q < std::min(n_ev, n); ++q) {
    if (ex.res[order[q]] > tol_resid) break;
    ok.push_back(order[q]);
  }
  ex.sel = ok;
  ex.complete = false;
  if ((int)ok.size() == n_ev && n_ev > 0) {
    double d = 0;
    for (int j : ok) d = std::max(d, std::fabs(ex.E[j] - lam));
    d /= pl.dE;
    const double pm = filter_value_closed(pl.lambda_t, pl.K, pl.lambda_t - d);
    const double pp = filter_value_closed(pl.lambda_t, pl.K, pl.lambda_t + d);
    ex.complete = std::min(pm, pp) >= theta_min;
  }
}

namespace {

// u = V t for the selected Ritz vectors, Rayleigh-Ritz with H on their span
// and residual norms.
Extracted extract(polfed_ctx* ctx, const polfed_op* op, const Basis& B, Ws& ws, int m,
                  const DevBuf& dY /* m x n col-major, device */, int n) {
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  Extracted ex;
  DevBuf U((size_t)D * n * sizeof(double)), HU((size_t)D * n * sizeof(double));
  dev_gemm_nn(s, D, m, n, B.V.as<double>(), D, dY.as<double>(), m, U.as<double>(), D, false);
  for (int j = 0; j < n; ++j) apply_H(s, op, U.as<double>() + (size_t)j * D, HU.as<double>() + (size_t)j * D);
  rayleigh_ritz(s, D, n, U.as<double>(), HU.as<double>(), ws.nseg, ex);
  return ex;
}


}  // namespace

void extract_pairs(polfed_ctx* ctx, const polfed_op* op, const double* V, int m,
                   const double* T, int n, double* E, double* U2, double* resid) {
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  const int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(256, (D + 8191) / 8192));
  DevBuf U((size_t)D * n * sizeof(double)), HU((size_t)D * n * sizeof(double));
  dev_gemm_nn(s, D, m, n, V, D, T, m, U.as<double>(), D, false);
  for (int j = 0; j < n; ++j)
    apply_H(s, op, U.as<double>() + (size_t)j * D, HU.as<double>() + (size_t)j * D);
  Extracted ex;
  rayleigh_ritz(s, D, n, U.as<double>(), HU.as<double>(), nseg, ex);
  dcopy_async(s, E, ex.E.data(), (size_t)n, hipMemcpyHostToDevice);
  dcopy_async(s, resid, ex.res.data(), (size_t)n, hipMemcpyHostToDevice);
  HIPC(hipMemcpyAsync(U2, ex.U2.get(), (size_t)D * n * sizeof(double), hipMemcpyDeviceToDevice,
                      s));
  HIPC(hipStreamSynchronize(s));
}

// ---------------------------------------------------------- SolveRun ----

void SolveRun::setup(polfed_ctx* c, const polfed_op* o, const polfed_params& prm,
                     const double* x0, double* ev, double* vecs, double* res, int* nf) {
  ctx = c;
  op = o;
  p = prm;
  evals = ev;
  evecs = vecs;
  resid = res;
  n_found = nf;
  hipStream_t s = ctx->stream;
  t_start = now_seconds();
  const int64_t D = op->D;
  REQUIRE(D >= 1, "solve: empty operator");
  REQUIRE(p.n_ev >= 1 && p.n_ev <= D, "solve: need 1 <= n_ev <= D");
  p.precision = resolve_precision(s, op, p.precision);
  REQUIRE(p.precision == POLFED_FP64 || p.precision == POLFED_FP32, "solve: bad precision");
  REQUIRE(x0 && evals && evecs && resid && n_found, "solve: null buffer");
  this->s = std::max(1, p.block_size);
  REQUIRE(this->s <= 64, "solve: block_size must lie in 0..64");
  REQUIRE(this->s == 1 || D >= 2 * (int64_t)this->s,
          "solve: block Lanczos needs D >= 2 block_size");
  static std::atomic<uint64_t> next_uid{1};
  uid = next_uid.fetch_add(1);
  fp32 = p.precision == POLFED_FP32;
  tol_resid = p.tol_resid > 0 ? p.tol_resid : 1e-8;
  tol_ritz = 1e-10;
  const double pad = p.bound_pad > 0 ? p.bound_pad : 1e-3;
  const double eta = p.eta > 0 ? p.eta : 1.5;
  R = polfed_report{};
  R.precision = p.precision;
  *n_found = 0;

  // 1. spectral bounds
  double E_min = p.E_min, E_max = p.E_max;
  double t0 = now_seconds();
  if (!(E_max > E_min)) {
    int it = 0;
    bounds(ctx, op, x0, 1e-10, 300, &E_min, &E_max, &it);
  }
  R.t_bounds = now_seconds() - t0;
  R.E_min = E_min;
  R.E_max = E_max;

  // 2-3. trace moments, DOS, window, K, coefficients
  t0 = now_seconds();
  DevBuf two(2 * sizeof(double)), mpart(2 * 4096 * sizeof(double));
  op_moments(s, op, two.as<double>(), mpart.as<double>(), 4096);
  double tr[2];
  HIPC(hipMemcpyAsync(tr, two.get(), sizeof tr, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  const double tr1 = tr[0] / (double)D, tr2 = tr[1] / (double)D;
  // KPM density of states (Sec. 4.1) in the rescaled coordinates of the
  // padded bounds, when asked for: it sets the window and the maxdos point
  std::vector<double> kmu;
  double peak = tr1;  // maxdos point: the Gaussian estimate's mean by default
  if (p.kpm_moments > 0) {
    const double w = E_max - E_min, lo = E_min - pad * w, hi = E_max + pad * w;
    const double Ec = 0.5 * (hi + lo), dEk = 0.5 * (hi - lo);
    kmu.resize(p.kpm_moments);
    kpm_moments(ctx, op, Ec, dEk, p.kpm_moments, p.kpm_vectors > 0 ? p.kpm_vectors : 100,
                nullptr, kKpmSeed, kmu.data());
    peak = Ec + dEk * kpm_maxdos(kmu.data(), p.kpm_moments, (E_min + 0.05 * w - Ec) / dEk,
                                 (E_max - 0.05 * w - Ec) / dEk);
  }
  lam = target_energy(p.target_kind, p.target, E_min, E_max, peak);
  // FP32 bulk keeps twice the buffer: the window edge moves away from the
  // wanted pairs, whose refinement then converges in about two sweeps (the
  // wider window also lowers K, so the Lanczos work stays about the same)
  n_want = (int)std::min<int64_t>(D, p.n_ev + (fp32 ? 2 : 1) * buffer_size(p.n_ev));
  n_want0 = n_want;
  pl = make_plan(D, E_min, E_max, pad, lam, tr1, tr2, n_want, p.omega, p.K_override,
                 kmu.empty() ? nullptr : kmu.data(), (int)kmu.size());
  a.assign(pl.K + 1, 0.0);
  filter_coefficients(pl.lambda_t, pl.K, a.data());
  // An FP32 recurrence carries a relative error of a few times sqrt(K) unit
  // roundoffs; the Lanczos check stops at ten times that level and the
  // refinement takes the pairs the rest of the way.
  if (fp32) tol_ritz = std::max(1e-10, 10.0 * 4.0 * std::sqrt((double)pl.K) * 6e-8);
  R.t_plan = now_seconds() - t0;
  R.lambda = lam;
  R.lambda_t = pl.lambda_t;
  R.E_c = pl.E_c;
  R.dE = pl.dE;
  R.delta = pl.delta;
  R.rho = pl.rho;
  R.K = pl.K;

  // 4. filtered (block) Lanczos state; in block mode every count of basis
  // vectors is a whole number of blocks
  const int bs = this->s;
  auto whole = [bs](int64_t n) { return (int)(((n + bs - 1) / bs) * bs); };
  M_alloc = whole(expected_krylov_dim(n_want, bs, eta));
  M_max = (int)std::min<int64_t>(D, p.max_iter > 0 ? p.max_iter : 4 * (int64_t)M_alloc);
  if (bs > 1) M_max = (int)((std::min<int64_t>(M_max, D - bs) / bs) * bs);
  cap = std::min(M_alloc, M_max);
  R.M_alloc = M_alloc;
  B.ensure(s, D, cap + 2 * bs - 1, 0);
  ws.init(s, D, cap + 2 * bs, fp32);
  if (bs == 1) {
    normalize_into(s, D, x0, ws, B.col(0));
  } else {
    block_start(s, D, bs, x0, B.V.as<double>(), ws.w.as<double>(), ws.c.as<double>(),
                ws.partial.as<double>(), ws.nseg, ws.flag.as<int>(), ws.scal.as<double>());
    bw.init(ctx, op, bs, fp32, pl, a.data());
    grow_band(cap / bs + 1);
  }
  check_every = whole(std::max(10, (int)std::ceil(0.05 * M_alloc)));
  next_check = std::min(whole(n_want), M_max);
  k = 0;
  brk_from = 1;
  early_lead = 0;
  done = false;
  status = POLFED_NOT_CONVERGED;
  restart_seed = 0x5EEDULL;
  sbytes = step_bytes(op, p.precision);
}

size_t SolveRun::bytes_at(int64_t D_, int m, int n, bool f32) {
  const size_t D = (size_t)std::max<int64_t>(D_, 1), vec = D * 8, M = (size_t)m, N = (size_t)n;
  const size_t nseg = (size_t)std::max<int64_t>(1, std::min<int64_t>(256, (D_ + 8191) / 8192));
  // basis (M + 2 columns) and the coefficient and partial-sum arrays
  size_t b = (M + 2) * vec + (nseg * (M + 1) + 8192 + 3 * (M + 2)) * 8;
  // w, the filter's two recurrence buffers, the FP32 copies of v and w,
  // and the fixed graph input (FP64)
  b += vec + (f32 ? 4 * D * 4 : 3 * vec);
  // check and extraction: the tridiagonal eigenvectors (M x M), the chosen
  // ones (M x n), the projected matrix and its eigenvectors, partial sums,
  // the split sums of the projection product
  b += (M * M + M * N + 2 * N * N + nseg * N + 8192) * 8 + gemm_tn_workspace(D_, n, n);
  // FP64: U, HU, U2, HU2.  FP32 refinement: the extracted U2, HU2, four
  // FP32 blocks, five FP64 blocks and the next Rayleigh-Ritz generation;
  // then the two FP64 recurrence buffers of the FP64 fallback.
  b += f32 ? 11 * N * vec + 2 * vec : 4 * N * vec;
  return b;
}

size_t SolveRun::footprint(const polfed_op* op, const polfed_params& p) {
  const int n_ev = std::max(1, p.n_ev);
  const bool f32 = p.precision == POLFED_FP32;
  const int g = (f32 ? 2 : 1) * buffer_size(n_ev);
  const int n_want = (int)std::min<int64_t>(op->D, n_ev + g);
  const int M = (int)std::min<int64_t>(op->D, expected_krylov_dim(n_want, 1, p.eta > 0 ? p.eta : 1.5));
  size_t b = bytes_at(op->D, M, n_want, f32);
  if (!(p.E_max > p.E_min)) {
    // the bounds Lanczos before it: its basis of up to 300 steps, w and the
    // two recurrence buffers of its work space
    const size_t D = (size_t)std::max<int64_t>(op->D, 1);
    const size_t cap = (size_t)std::min<int64_t>(300, op->D);
    b = std::max(b, (cap + 2 + 3) * D * 8 + (cap + 2) * 8 * 3 + 8192 * 8 * 2);
  }
  return b;
}

bool SolveRun::reserve(size_t bytes) {
  if (!take) return true;
  if (granted >= bytes) {
    granted -= bytes;
    return true;
  }
  if (!take(bytes - granted)) {
    want = bytes;
    return false;
  }
  granted = 0;
  return true;
}

void SolveRun::resume() {
  if (!want) return;
  if (!take(want - std::min(want, granted))) return;
  granted = want;
  want = 0;
  const auto what = pend;
  pend = kPendNone;
  if (what == kPendGrow) {
    step_tail();
  } else if (what == kPendWant) {
    granted = 0;
    n_want = pend_n_want;
  }
}

void SolveRun::filter_self() {
  if (this->s > 1) {
    filter_block();
    return;
  }
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  if (mode == kTimeDirect && (p.graph == 2 || pl.K < 8 || pl.K > kGraphMaxSteps)) mode = kDirect;
  if (mode == kTimeDirect && p.graph == 1) mode = kGraph;
  const bool use_graph = mode == kTimeGraph || mode == kGraph;
  if (use_graph && !graph.ready()) {
    if (!fp32) vst.alloc((size_t)std::max<int64_t>(D, 1) * sizeof(double));
    op_tune(s, op, fp32);
    graph.capture(ctx->cap_stream, [&](hipStream_t cs) {
      if (fp32)
        filter_apply_on<float>(cs, op, pl.E_c, pl.dE, a.data(), pl.K, ws.v32.as<float>(),
                               ws.w32.as<float>(), ws.bA.as<float>(), ws.bB.as<float>());
      else
        filter_apply_on<double>(cs, op, pl.E_c, pl.dE, a.data(), pl.K, vst.as<double>(),
                                ws.w.as<double>(), ws.bA.as<double>(), ws.bB.as<double>());
    });
  }
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  HIPC(hipEventRecord(e0, s));
  if (fp32) dev_copy_d2f(s, D, B.col(k), ws.v32.as<float>());
  if (use_graph) {
    if (!fp32)
      HIPC(hipMemcpyAsync(vst.get(), B.col(k), (size_t)D * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    graph.launch(s);
  } else if (fp32) {
    filter_apply<float>(ctx, op, pl.E_c, pl.dE, a.data(), pl.K, ws.v32.as<float>(),
                        ws.w32.as<float>(), ws.bA.as<float>(), ws.bB.as<float>());
  } else {
    filter_apply<double>(ctx, op, pl.E_c, pl.dE, a.data(), pl.K, B.col(k), ws.w.as<double>(),
                         ws.bA.as<double>(), ws.bB.as<double>());
  }
  if (fp32) dev_copy_f2d(s, D, ws.w32.as<float>(), ws.w.as<double>());
  HIPC(hipEventRecord(e1, s));
  fev.emplace_back(e0, e1);
  R.filter_steps += pl.K;
  R.filter_bytes += pl.K * step_bytes(op, fp32 ? POLFED_FP32 : POLFED_FP64);
  // autotuning: the first application runs direct, the second as a graph;
  // the faster way serves the rest of the solve
  if (mode == kTimeDirect || mode == kTimeGraph) {
    HIPC(hipEventSynchronize(e1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, e0, e1));
    if (mode == kTimeDirect) {
      t_direct_ms = ms;
      mode = kTimeGraph;
    } else {
      mode = ms < t_direct_ms ? kGraph : kDirect;
      if (mode == kDirect) graph.reset();
      if (verbose())
        std::fprintf(stderr, "[polfed] filter K=%d: direct %.3f ms, graph %.3f ms -> %s\n", pl.K,
                     t_direct_ms, ms, mode == kGraph ? "graph" : "direct");
    }
  }
}

void SolveRun::drain() {
  auto one = [](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& acc) {
    for (auto& pr : v) {
      float ms = 0;
      HIPC(hipEventElapsedTime(&ms, pr.first, pr.second));
      acc += 1e-3 * ms;
      HIPC(hipEventDestroy(pr.first));
      HIPC(hipEventDestroy(pr.second));
    }
    v.clear();
  };
  one(fev, R.t_filter);
  one(rev, R.t_reorth);
}

SolveRun::~SolveRun() {
  for (auto* v : {&fev, &rev})
    for (auto& pr : *v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
}

// Full reorthogonalization of w = P(H~) v_k against the basis (CGS2), then
// the periodic convergence check (eq. lan_criterion), extraction and the
// completeness test once the check passes.
void SolveRun::advance() {
  if (this->s > 1) {
    advance_block();
    return;
  }
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  hipEvent_t r0, r1;
  HIPC(hipEventCreate(&r0));
  HIPC(hipEventCreate(&r1));
  HIPC(hipEventRecord(r0, s));
  cgs2_normalize(s, D, k + 1, B, ws, ws.alpha.as<double>() + k, ws.beta.as<double>() + k + 1,
                 B.col(k + 1));
  HIPC(hipEventRecord(r1, s));
  rev.emplace_back(r0, r1);
  ++k;
  step_tail();
}

void SolveRun::step_tail() {
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  if (k >= cap && cap < M_max) {
    const int ncap = std::min(M_max, (int)std::ceil(1.25 * cap) + 1);
    // the larger basis is allocated before the old one is freed
    const size_t old_basis = (size_t)D * (B.cap + 1) * 8;
    const size_t more = bytes_at(D, ncap, n_want, fp32) - bytes_at(D, cap, n_want, fp32);
    if (!reserve(more + old_basis)) {
      pend = kPendGrow;
      return;
    }
    B.ensure(s, D, ncap, k + 1);
    ws.grow(s, ncap + 1);
    cap = ncap;
    if (give) give(old_basis);
  }
  if (k < next_check && k < M_max) return;

  const double tc = now_seconds();
  std::vector<double> al(k), be(k + 1);
  HIPC(hipMemcpyAsync(al.data(), ws.alpha.get(), k * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(be.data(), ws.beta.get(), (k + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  drain();
  for (int i = 0; i < k; ++i)
    if (!std::isfinite(al[i]) || std::fabs(al[i]) > 4.0 || !std::isfinite(be[i + 1]))
      fail(POLFED_ERR_BOUNDS, "filter blow-up: Lanczos coefficient " + std::to_string(al[i]) +
                                  " at step " + std::to_string(i) +
                                  " (spectral bounds too tight?)");
  // breakdown: restart from the first vanishing beta with a random vector
  // (the zero beta of an earlier restart is not one)
  const int kb = first_breakdown(brk_from, k, al, be, 1.0);
  if (kb > 0 && kb < M_max) {
    if (R.restarts >= 8) fail(POLFED_ERR_BREAKDOWN, "Lanczos breakdown: too many restarts");
    ++R.restarts;
    k = kb;
    restart_random(s, D, k, B, ws, restart_seed++);
    brk_from = k + 1;
    next_check = k + 1;
    R.t_check += now_seconds() - tc;
    return;
  }
  ++R.checks;
  std::vector<double> th, zl;
  ritz_last(k, al, be, th, zl);
  std::vector<int> order(k);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return th[x] > th[y]; });
  const int nw = std::min(n_want, k);
  double thmax = 0;
  for (double t : th) thmax = std::max(thmax, std::fabs(t));
  bool conv = true;
  double est_max = 0;
  int lead = 0;  // leading run of converged Ritz values, from the largest
  for (int j = 0; j < k; ++j) {
    const double e = std::fabs(be[k] * zl[order[j]]);
    const bool ok_j = e <= tol_ritz * std::max(1.0, thmax);
    if (j < nw) {
      est_max = std::max(est_max, e);
      if (!ok_j) conv = false;
    }
    if (ok_j && lead == j) ++lead;
    if (!ok_j && j >= nw) break;
  }
  const bool early = !conv && early_ready(lead);
  if (verbose())
    std::fprintf(stderr, "[polfed] check k=%d n_want=%d max |beta z|=%.2e tol=%.1e conv=%d lead=%d\n",
                 k, n_want, est_max, tol_ritz, (int)conv, lead);
  R.t_check += now_seconds() - tc;
  if (conv || k >= M_max || early) {
    std::vector<double> thf;
    DevBuf dC;  // eigenvectors of the tridiagonal matrix, k x k col-major
    {
      std::vector<double> Y;
      ritz_full(k, al, be, thf, Y);
      std::vector<double> Yc((size_t)k * k);
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Yc[(size_t)j * k + i] = Y[(size_t)i * k + j];
      upload(dC, Yc.data(), Yc.size(), s);
    }
    if (conv || k >= M_max) {
      if (conclude(thf, dC, nw, false)) return;
    } else if (conclude(thf, dC, lead, true)) {
      return;
    }
  }
  next_check = k + check_every;
}

// An extraction before all n_want leading Ritz values have converged: once
// a leading run of converged values covers N_ev plus half the buffer, their
// pairs may already hold the N_ev nearest the target and pass the
// completeness test.  Tried again only after the run has grown by a
// twentieth of N_ev (at least 5).  FP64 filter only: an FP32 run refines at
// its extraction instead.
bool SolveRun::early_ready(int lead) {
  if (fp32) return false;
  const int need = p.n_ev + (n_want0 - p.n_ev + 1) / 2;
  if (lead < need || lead >= std::min(n_want, k)) return false;
  if (lead < early_lead + std::max(5, p.n_ev / 20)) return false;
  early_lead = lead;
  return true;
}

// After a passed check (or at the Krylov limit): the n_want largest Ritz
// values of P(H~) and their vectors u = V t, Rayleigh-Ritz with H, the
// selection and the completeness test; refinement of an FP32-filtered run.
bool SolveRun::conclude(const std::vector<double>& thf, const DevBuf& dC, int nw, bool early) {
  hipStream_t s = ctx->stream;
  const double tx = now_seconds();
  nw = std::min(nw, k);
  // pick the n_want largest
  std::vector<int> ord(k);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return thf[x] > thf[y]; });
  DevBuf dY((size_t)k * nw * sizeof(double));
  for (int j = 0; j < nw; ++j)
    dcopy_async(s, dY.as<double>() + (size_t)j * k, dC.as<double>() + (size_t)ord[j] * k,
                (size_t)k, hipMemcpyDeviceToDevice);
  const double theta_min = thf[ord[nw - 1]];
  Extracted ex = extract(ctx, op, B, ws, k, dY, nw);
  select_pairs(ex, lam, p.n_ev, tol_resid, theta_min, pl);
  R.t_extract += now_seconds() - tx;
  if (verbose()) {
    int acc = 0;
    for (double r : ex.res) acc += r <= tol_resid;
    std::fprintf(stderr,
                 "[polfed] extract k=%d vectors=%d%s accepted=%d selected=%d complete=%d "
                 "theta_min=%.4f\n",
                 k, nw, early ? " (early)" : "", acc, (int)ex.sel.size(), (int)ex.complete,
                 theta_min);
  }
  if (early) {
    // not finished yet: the iteration goes on to the regular check
    if ((int)ex.sel.size() == p.n_ev && ex.complete) {
      emit(ex, POLFED_OK);
      return true;
    }
    return false;
  }
  if (fp32 && !((int)ex.sel.size() == p.n_ev && ex.complete)) {
    const double tr = now_seconds();
    refine(*this, ex, theta_min);
    R.t_refine += now_seconds() - tr;
  }
  const bool ok = (int)ex.sel.size() == p.n_ev && ex.complete;
  if (ok || k >= M_max) {
    emit(ex, ok ? POLFED_OK : POLFED_NOT_CONVERGED);
    return true;
  }
  // The Ritz vectors of an FP32-filtered run stop improving once Lanczos
  // has reached the FP32 noise level, so a refinement that did not finish
  // will not finish later either: the solve is completed in FP64.
  if (fp32 && !ok) {
    fallback_fp64();
    return true;
  }
  if ((int)ex.sel.size() == p.n_ev && !ex.complete) {
    const int nw2 = std::min(M_max, n_want + std::max(10, n_want / 5));
    if (reserve(bytes_at(op->D, cap, nw2, fp32) - bytes_at(op->D, cap, n_want, fp32))) {
      n_want = nw2;
    } else {
      pend = kPendWant;
      pend_n_want = nw2;
    }
  }
  return false;
}

// Restarts the filtered Lanczos iteration from v_0 with the FP64 filter (the
// bounds, plan and basis allocation are kept).
void SolveRun::fallback_fp64() {
  const int64_t D = op->D;
  fp32 = false;
  // the FP64 restart keeps the plan (and window) of the FP32 run
  R.fp32_fallback = 1;
  tol_ritz = 1e-10;
  graph.reset();
  mode = (p.graph == 2 || pl.K < 8 || pl.K > kGraphMaxSteps) ? kDirect
                                                             : (p.graph == 1 ? kGraph : kTimeDirect);
  ws.bA.alloc((size_t)std::max<int64_t>(D, 1) * sizeof(double));
  ws.bB.alloc((size_t)std::max<int64_t>(D, 1) * sizeof(double));
  k = 0;
  brk_from = 1;
  early_lead = 0;
  n_want = n_want0;
  next_check = std::min(((n_want + s - 1) / s) * s, M_max);
  // block mode: the start block (columns 0..s-1) is kept; the filter
  // buffers change precision
  if (s > 1) bw.init(ctx, op, s, false, pl, a.data());
  if (verbose()) std::fprintf(stderr, "[polfed] FP32 refinement stalled: restarting in FP64\n");
}

// Copies the selected pairs to the caller's buffers and finishes the run.
void SolveRun::emit(const Extracted& ex, polfed_status st) {
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  const int nf = (int)ex.sel.size();
  std::vector<double> Eo(nf), Ro(nf);
  for (int j = 0; j < nf; ++j) {
    Eo[j] = ex.E[ex.sel[j]];
    Ro[j] = ex.res[ex.sel[j]];
    dcopy_async(s, evecs + (size_t)j * D, ex.U2.as<double>() + (size_t)ex.sel[j] * D, (size_t)D,
                hipMemcpyDeviceToDevice);
  }
  dcopy_async(s, evals, Eo.data(), (size_t)nf, hipMemcpyHostToDevice);
  dcopy_async(s, resid, Ro.data(), (size_t)nf, hipMemcpyHostToDevice);
  HIPC(hipStreamSynchronize(s));
  *n_found = nf;
  R.n_converged = nf;
  status = st;
  finish();
}

void SolveRun::finish() {
  drain();
  R.iters = k;
  R.n_want = n_want;
  R.filter_GBps = R.t_filter > 0 ? R.filter_bytes / R.t_filter / 1e9 : 0;
  R.t_total = now_seconds() - t_start;
  done = true;
  // the basis and work vectors are not needed any more
  B = Basis{};
  ws = Ws{};
  bw = BlockWs{};
  band = DevBuf{};
  band_blocks = 0;
}

polfed_status solve(polfed_ctx* ctx, const polfed_op* op, const polfed_params& p,
                    const double* x0, double* evals, double* evecs, double* resid,
                    int* n_found, polfed_report* rep) {
  SolveRun run;
  TallyScope ts(&run.tally);
  run.setup(ctx, op, p, x0, evals, evecs, resid, n_found);
  while (!run.done) {
    run.filter_self();
    run.advance();
  }
  run.R.mem_peak = (double)run.tally.peak;
  if (rep) *rep = run.R;
  return run.status;
}

// ---------------------------------------------- single Lanczos step (API) ----

void* ctx_scratch(polfed_ctx* ctx, int slot, size_t bytes) {
  DevBuf& b = ctx->ws[slot];
  TallyScope untallied(nullptr);  // held by the context
  if (b.bytes() < bytes) b.alloc(bytes);
  return b.get();
}

void lanczos_step(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE,
                  const double* a, int K, double* V, int k, double* alpha,
                  double* beta, int precision) {
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  const size_t nd = (size_t)std::max<int64_t>(D, 1);
  double* w = static_cast<double*>(ctx_scratch(ctx, 0, nd * sizeof(double)));
  const int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(256, (D + 8191) / 8192));
  double* c = static_cast<double*>(ctx_scratch(ctx, 1, (size_t)(k + 2) * sizeof(double)));
  double* part = static_cast<double*>(
      ctx_scratch(ctx, 2, ((size_t)nseg * (k + 2) + 8192) * sizeof(double)));
  int* flag = static_cast<int*>(ctx_scratch(ctx, 3, 64));
  double* vk = V + (size_t)k * D;
  if (precision == POLFED_FP32) {
    float* v32 = static_cast<float*>(ctx_scratch(ctx, 4, nd * sizeof(float)));
    float* w32 = static_cast<float*>(ctx_scratch(ctx, 5, nd * sizeof(float)));
    float* bA = static_cast<float*>(ctx_scratch(ctx, 6, nd * sizeof(float)));
    float* bB = static_cast<float*>(ctx_scratch(ctx, 7, nd * sizeof(float)));
    dev_copy_d2f(s, D, vk, v32);
    filter_apply<float>(ctx, op, E_c, dE, a, K, v32, w32, bA, bB);
    dev_copy_f2d(s, D, w32, w);
  } else {
    double* bA = static_cast<double*>(ctx_scratch(ctx, 6, nd * sizeof(double)));
    double* bB = static_cast<double*>(ctx_scratch(ctx, 7, nd * sizeof(double)));
    filter_apply<double>(ctx, op, E_c, dE, a, K, vk, w, bA, bB);
  }
  cgs2_raw(s, D, k + 1, V, w, c, part, nseg, flag, alpha, beta, V + (size_t)(k + 1) * D);
}

// Times `iters` back-to-back launches of the fused step kernel with a pair
// of HIP events around each launch on the context stream.
int resolve_precision(hipStream_t s, const polfed_op* op, int precision) {
  if (precision != POLFED_PRECISION_AUTO) return precision;
  if (op->auto_precision >= 0) return op->auto_precision;
  // operators sharing the off-diagonal pattern and the storage run the same
  // kernels at the same speed: one timing per pattern and device
  static std::mutex mu;
  static std::map<std::string, int> by_pattern;
  const std::string key =
      op->pattern_key.empty()
          ? std::string()
          : std::to_string(op->ctx->device) + "|" + std::to_string(op->storage) + "|" +
                op->pattern_key;
  if (!key.empty()) {
    std::lock_guard<std::mutex> lk(mu);
    const auto it = by_pattern.find(key);
    if (it != by_pattern.end()) return op->auto_precision = it->second;
  }
  const int64_t D = op->D;
  const size_t nd = (size_t)std::max<int64_t>(D, 1);
  DevBuf v(nd * 8), b1(nd * 8), b2(nd * 8);
  HIPC(hipMemsetAsync(v.get(), 0, nd * 8, s));
  HIPC(hipMemsetAsync(b1.get(), 0, nd * 8, s));
  HIPC(hipMemsetAsync(b2.get(), 0, nd * 8, s));
  auto step = [&](hipStream_t st, bool f32) {
    if (f32)
      op_step<float>(st, op, 0.1f, 0.0f, 0.0f, v.as<float>(), b1.as<float>(), b2.as<float>(),
                     b2.as<float>());
    else
      op_step<double>(st, op, 0.1, 0.0, 0.0, v.as<double>(), b1.as<double>(), b2.as<double>(),
                      b2.as<double>());
  };
  // the first steps pick the kernel variants (timed on s, outside any capture)
  step(s, false);
  step(s, true);
  HIPC(hipStreamSynchronize(s));
  const float t64 = replay_time_us([&](hipStream_t st) { step(st, false); }, 20);
  const float t32 = replay_time_us([&](hipStream_t st) { step(st, true); }, 20);
  op->auto_precision = t32 < 0.7f * t64 ? POLFED_FP32 : POLFED_FP64;
  if (!key.empty()) {
    std::lock_guard<std::mutex> lk(mu);
    by_pattern.emplace(key, op->auto_precision);
  }
  if (verbose())
    std::fprintf(stderr, "[polfed] precision auto: step %.2f us FP64, %.2f us FP32 -> %s\n",
                 t64, t32, op->auto_precision == POLFED_FP32 ? "FP32 bulk" : "FP64");
  return op->auto_precision;
}

void profile_step(polfed_ctx* ctx, const polfed_op* op, int precision, int iters,
                  double* avg_ms, double* min_ms) {
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  const size_t nd = (size_t)std::max<int64_t>(D, 1);
  DevBuf v(nd * 8), b1(nd * 8), b2(nd * 8);
  dev_random(s, D, 11, v.as<double>());
  dev_random(s, D, 12, b1.as<double>());
  dev_random(s, D, 13, b2.as<double>());
  if (precision == POLFED_FP32) {
    DevBuf t(nd * 4);
    for (DevBuf* b : {&v, &b1, &b2}) {
      dev_copy_d2f(s, D, b->as<double>(), t.as<float>());
      HIPC(hipMemcpyAsync(b->get(), t.get(), nd * 4, hipMemcpyDeviceToDevice, s));
    }
    HIPC(hipStreamSynchronize(s));
  }
  const double sigma = 0.1, tau = -0.01, a = 1e-3;
  auto launch = [&]() {
    if (precision == POLFED_FP32)
      op_step<float>(s, op, (float)sigma, (float)tau, (float)a, v.as<float>(), b1.as<float>(),
                     b2.as<float>(), b2.as<float>());
    else
      op_step<double>(s, op, sigma, tau, a, v.as<double>(), b1.as<double>(), b2.as<double>(),
                      b2.as<double>());
  };
  // mean: one event pair around iters back-to-back launches, as the
  // recurrence runs them; min: event pairs around single launches
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  launch();
  HIPC(hipEventRecord(e0, s));
  for (int i = 0; i < iters; ++i) launch();
  HIPC(hipEventRecord(e1, s));
  HIPC(hipEventSynchronize(e1));
  float total = 0;
  HIPC(hipEventElapsedTime(&total, e0, e1));
  double mn = 1e300;
  for (int i = 0; i < std::min(iters, 20); ++i) {
    HIPC(hipEventRecord(e0, s));
    launch();
    HIPC(hipEventRecord(e1, s));
    HIPC(hipEventSynchronize(e1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, e0, e1));
    mn = std::min(mn, (double)ms);
  }
  HIPC(hipEventDestroy(e0));
  HIPC(hipEventDestroy(e1));
  const double sum = total;
  *avg_ms = iters ? sum / iters : 0;
  *min_ms = iters ? mn : 0;
}

}  // namespace polfed

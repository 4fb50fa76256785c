// FP64-accurate refinement of the Ritz pairs of a Lanczos run whose filter
// recurrence ran in FP32.
//
// The Ritz vectors u_j (Rayleigh-Ritz with H in FP64) carry errors at the
// rounding level of the FP32 filter.  A sweep of filtered subspace iteration,
// w_j = P(H~) u_j, damps them (P is small away from the target window); it is
// evaluated as
//     P(H~) u_j = P(t_j) u_j + Q_j(H~) r_j,    r_j = (H~ - t_j) u_j,
// with t_j = (E_j - E_c) / dE and Q_j the divided difference of P at t_j.
// r_j is formed in FP64 and is small, so running the FP32 recurrence on it
// (the bulk of the work) perturbs w_j only at the level of the FP32 filter
// error times ||r_j||, far below the error the sweep removes.  The w_j are
// orthonormalized (Cholesky QR, twice) and Rayleigh-Ritz with H in FP64 gives
// the next pairs.  Sweeps repeat until the n_ev pairs nearest the target meet
// the residual tolerance.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "internal.hpp"
#include "solve_run.hpp"

namespace polfed {

// r[:, j] = (HU[:, j] - E[j] U[:, j]) * scale, rounded to FP32
__global__ void k_resid_f32(int64_t D, int n, const double* __restrict__ U,
                            const double* __restrict__ HU, const double* __restrict__ E,
                            double scale, float* __restrict__ r) {
  const int64_t total = D * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double e = E[i / D];
    r[i] = (float)((HU[i] - e * U[i]) * scale);
  }
}

// W[:, j] = p[j] U[:, j] + Z[:, j]
__global__ void k_combine(int64_t D, int n, const double* __restrict__ U,
                          const double* __restrict__ p, const float* __restrict__ Z,
                          double* __restrict__ W) {
  const int64_t total = D * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x)
    W[i] = p[i / D] * U[i] + (double)Z[i];
}

static unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(16384, (n + 255) / 256));
}

// W <- W R^{-1} with W^T W = R^T R (Cholesky); tmp: D x n scratch.
static void cholqr(hipStream_t s, int64_t D, int n, DevBuf& W, DevBuf& tmp) {
  DevBuf dG((size_t)n * n * sizeof(double));
  dev_gemm_tn(s, D, n, n, W.as<double>(), D, W.as<double>(), D, dG.as<double>(), n);
  std::vector<double> G((size_t)n * n);
  HIPC(hipMemcpyAsync(G.data(), dG.get(), G.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  // upper R, col-major: R[i + j n], i <= j
  std::vector<double> R((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i <= j; ++i) {
      double acc = G[(size_t)i + (size_t)j * n];
      for (int k = 0; k < i; ++k) acc -= R[(size_t)k + (size_t)i * n] * R[(size_t)k + (size_t)j * n];
      if (i == j) {
        if (!(acc > 0)) fail(POLFED_ERR_BREAKDOWN, "refinement: subspace lost rank");
        R[(size_t)j + (size_t)j * n] = std::sqrt(acc);
      } else {
        R[(size_t)i + (size_t)j * n] = acc / R[(size_t)i + (size_t)i * n];
      }
    }
  }
  // Rinv, upper triangular, by back substitution column by column
  std::vector<double> Ri((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Ri[(size_t)j + (size_t)j * n] = 1.0 / R[(size_t)j + (size_t)j * n];
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0;
      for (int k = i + 1; k <= j; ++k) acc += R[(size_t)i + (size_t)k * n] * Ri[(size_t)k + (size_t)j * n];
      Ri[(size_t)i + (size_t)j * n] = -acc / R[(size_t)i + (size_t)i * n];
    }
  }
  DevBuf dRi;
  upload(dRi, Ri.data(), Ri.size(), s);
  dev_gemm_nn(s, D, n, n, W.as<double>(), D, dRi.as<double>(), n, tmp.as<double>(), D, false);
  std::swap(W, tmp);
  HIPC(hipStreamSynchronize(s));
}

// Columns of X (D x n) listed in idx, packed into Y (D x idx.size()).
static void gather_cols(hipStream_t s, int64_t D, const double* X, const std::vector<int>& idx,
                        double* Y) {
  for (size_t c = 0; c < idx.size(); ++c)
    HIPC(hipMemcpyAsync(Y + c * D, X + (size_t)idx[c] * D, (size_t)D * sizeof(double),
                        hipMemcpyDeviceToDevice, s));
}

void refine(SolveRun& run, Extracted& ex, double theta_min) {
  polfed_ctx* ctx = run.ctx;
  const polfed_op* op = run.op;
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  const int n = (int)ex.E.size();
  const polfed_plan& pl = run.pl;
  const int K = pl.K;
  // Sweeps filter only the pairs not yet locked; a pair locks once its
  // residual is a tenth of the tolerance, so the slow tail of a few pairs
  // near the window edge costs a few filters per sweep.
  constexpr int kStall = 4;
  const int kMaxSweeps = run.p.refine_max > 0 ? run.p.refine_max : (run.p.refine_max < 0 ? 0 : 16);
  int best = -1, since_best = 0;
  const double lock_tol = 0.1 * run.tol_resid;
  if (n == 0) return;
  const size_t n32 = (size_t)D * n * sizeof(float), n64 = (size_t)D * n * sizeof(double);
  DevBuf r32(n32), z32(n32), bA(n32), bB(n32), Ua(n64), HUa(n64), W(n64), HW(n64), tmp(n64),
      dE, dP;
  const bool batched = op->model == Model::Chain && !op->pattern_key.empty() && op->split_nseg > 0;
  std::vector<std::vector<double>> q(n, std::vector<double>(std::max(K, 1)));
  std::vector<double> pv(n);
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if ((int)ex.sel.size() == run.p.n_ev && ex.complete) break;
    ++run.R.refine_sweeps;
    std::vector<int> act, lock;
    for (int j = 0; j < n; ++j) (ex.res[j] <= lock_tol ? lock : act).push_back(j);
    if (act.empty()) break;
    const int na = (int)act.size();
    // active pairs, packed
    std::vector<double> Ea(na);
    for (int c = 0; c < na; ++c) Ea[c] = ex.E[act[c]];
    gather_cols(s, D, ex.U2.as<double>(), act, Ua.as<double>());
    gather_cols(s, D, ex.HU2.as<double>(), act, HUa.as<double>());
    // divided differences of P at their Ritz values
    for (int c = 0; c < na; ++c) {
      const double t = (Ea[c] - pl.E_c) / pl.dE;
      filter_quotient(run.a.data(), K, t, q[c].data(), &pv[c]);
    }
    upload(dE, Ea.data(), (size_t)na, s);
    upload(dP, pv.data(), (size_t)na, s);
    hipLaunchKernelGGL(k_resid_f32, dim3(grid_for(D * na)), dim3(256), 0, s, D, na,
                       Ua.as<double>(), HUa.as<double>(), dE.as<double>(), 1.0 / pl.dE,
                       r32.as<float>());
    HIPC(hipGetLastError());
    // z_c = Q_c(H~) r_c in FP32
    if (K == 0) {
      dev_fillf(s, D * na, 0.0f, z32.as<float>());
    } else if (batched) {
      std::vector<const polfed_op*> ops(na, op);
      std::vector<double> Ec(na, pl.E_c), dEv(na, pl.dE);
      ChainBatch bt;
      bt.init(ctx, ops.data(), na);
      bt.set_scale(Ec.data(), dEv.data());
      std::vector<const double*> qp(na);
      std::vector<int> Kq(na, K - 1);
      for (int c = 0; c < na; ++c) qp[c] = q[c].data();
      BatchCoef co;
      co.set(s, na, qp.data(), Kq.data());
      filter_apply_batch<float>(ctx, bt, co, r32.as<float>(), z32.as<float>(), bA.as<float>(),
                                bB.as<float>());
    } else {
      for (int c = 0; c < na; ++c)
        filter_apply<float>(ctx, op, pl.E_c, pl.dE, q[c].data(), K - 1,
                            r32.as<float>() + (size_t)c * D, z32.as<float>() + (size_t)c * D,
                            bA.as<float>(), bB.as<float>());
    }
    // W = [locked pairs | P(t_c) u_c + z_c]
    gather_cols(s, D, ex.U2.as<double>(), lock, W.as<double>());
    double* Wa = W.as<double>() + lock.size() * (size_t)D;
    hipLaunchKernelGGL(k_combine, dim3(grid_for(D * na)), dim3(256), 0, s, D, na,
                       Ua.as<double>(), dP.as<double>(), z32.as<float>(), Wa);
    HIPC(hipGetLastError());
    cholqr(s, D, n, W, tmp);
    cholqr(s, D, n, W, tmp);
    for (int j = 0; j < n; ++j)
      op_step<double>(s, op, 1.0, 0.0, 0.0, nullptr, W.as<double>() + (size_t)j * D, nullptr,
                      HW.as<double>() + (size_t)j * D);
    rayleigh_ritz(s, D, n, W.as<double>(), HW.as<double>(), run.ws.nseg, ex);
    select_pairs(ex, run.lam, run.p.n_ev, run.tol_resid, theta_min, pl);
    int n_acc = 0;
    for (double x : ex.res) n_acc += x <= run.tol_resid;
    if (n_acc > best) {
      best = n_acc;
      since_best = 0;
    } else if (++since_best >= kStall) {
      break;  // stalled: the caller falls back to the FP64 filter
    }
    if (verbose()) {
      int acc = 0;
      double rmax = 0;
      for (double x : ex.res) acc += x <= run.tol_resid;
      for (int j : ex.sel) rmax = std::max(rmax, ex.res[j]);
      std::fprintf(stderr,
                   "[polfed] refine sweep %d: filtered=%d accepted=%d selected=%d complete=%d "
                   "max sel res=%.1e\n",
                   sweep, na, acc, (int)ex.sel.size(), (int)ex.complete, rmax);
    }
  }
}

}  // namespace polfed

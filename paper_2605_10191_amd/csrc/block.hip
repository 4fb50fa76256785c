// Block Lanczos on the filtered operator (Sec. 2.2 with the filter of Sec.
// 4.3): the filter P(H~) of a block of s Krylov vectors, the orthogonalization
// of the filtered block against the whole basis with the QR that gives the
// next block and B_{j+1}, the block tridiagonal Lanczos matrix and the block
// convergence check of eq. blocklan_criterion.
//
// The filter of a chain operator runs as one multi-column Clenshaw recurrence
// with every column on the same operator, so each step decodes a row segment
// once for all s columns.  The orthogonalization works column by column:
// two passes of classical Gram-Schmidt against all earlier basis vectors,
// the new block's earlier columns included, then normalization, which is the
// Gram-Schmidt QR of the orthogonalized block (positive diagonal of B_{j+1}).
// The passes against the existing basis are tall-skinny block products
// (C = V^T W, W -= V C, twice), so each block step reads the basis four times
// (per 8 columns) instead of four times per column.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

#include "internal.hpp"
#include "solve_run.hpp"

namespace polfed {

// --------------------------------------------------------- block filter ----

void BlockWs::init(polfed_ctx* ctx, const polfed_op* op, int s_, bool fp32_,
                   const polfed_plan& pl, const double* a) {
  s = s_;
  D = op->D;
  fp32 = fp32_;
  const size_t n = (size_t)std::max<int64_t>(D, 1) * s;
  w.alloc(n * sizeof(double));
  save.alloc(n * sizeof(double));
  const size_t tb = fp32 ? sizeof(float) : sizeof(double);
  bA.alloc(n * tb);
  bB.alloc(n * tb);
  if (fp32) {
    v32.alloc(n * sizeof(float));
    w32.alloc(n * sizeof(float));
  } else {
    v32 = DevBuf{};
    w32 = DevBuf{};
  }
  batched = op->model == Model::Chain && !op->pattern_key.empty() && op->split_nseg > 0;
  if (batched) {
    std::vector<const polfed_op*> ops(s, op);
    std::vector<double> Ec(s, pl.E_c), dE(s, pl.dE);
    std::vector<const double*> ap(s, a);
    std::vector<int> K(s, pl.K);
    bt.init(ctx, ops.data(), s);
    bt.set_scale(Ec.data(), dE.data());
    co.set(ctx->stream, s, ap.data(), K.data());
    // the step kernel is picked before a graph records the recurrence
    if (fp32)
      (void)batch_variant<float>(ctx->stream, bt);
    else
      (void)batch_variant<double>(ctx->stream, bt);
  }
}

template <typename T>
__global__ void k_scale_block(int64_t n, T a, const T* __restrict__ x, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

// The Clenshaw recurrence of eq. clenshaw_chebyshev_prod for the n columns
// of a QREM block at once, on the multi-column step (same sequence of
// operations as the single-column filter, column by column).
template <typename T>
static void qrem_filter_block(hipStream_t st, const polfed_op* op, const polfed_plan& pl,
                              const double* a, int n, const T* X, T* Wout, T* bA, T* bB) {
  const int64_t D = op->D, tot = D * n;
  const int K = pl.K;
  const T sigma = (T)(2.0 / pl.dE), tau = (T)(-2.0 * pl.E_c / pl.dE);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (tot + 255) / 256));
  if (K == 0) {
    hipLaunchKernelGGL((k_scale_block<T>), dim3(g), dim3(256), 0, st, tot, (T)a[0], X, Wout);
    HIPC(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL((k_scale_block<T>), dim3(g), dim3(256), 0, st, tot, (T)a[K], X, bA);
  HIPC(hipGetLastError());
  const T* cur = bA;
  T* prev = nullptr;
  for (int i = K - 1; i >= 1; --i) {
    T* o = prev ? prev : bB;
    qrem_step_multi<T>(st, op, n, sigma, tau, (T)a[i], X, cur, prev, o);
    prev = const_cast<T*>(cur);
    cur = o;
  }
  qrem_step_multi<T>(st, op, n, (T)(0.5 * sigma), (T)(0.5 * tau), (T)a[0], X, cur, prev, Wout);
}

template <typename T>
void block_filter_on(hipStream_t st, const polfed_op* op, BlockWs& bw, const polfed_plan& pl,
                     const double* a, const T* X, T* W) {
  T* bA = (T*)bw.bA.get();
  T* bB = (T*)bw.bB.get();
  if (bw.batched) {
    filter_apply_batch_on<T>(st, bw.bt, bw.co, X, W, bA, bB);
    return;
  }
  if (op->model == Model::Qrem && op->L >= 10) {
    qrem_filter_block<T>(st, op, pl, a, bw.s, X, W, bA, bB);
    return;
  }
  const int64_t D = bw.D;
  for (int c = 0; c < bw.s; ++c)
    filter_apply_on<T>(st, op, pl.E_c, pl.dE, a, pl.K, X + (size_t)c * D, W + (size_t)c * D, bA,
                       bB);
}

template void block_filter_on<double>(hipStream_t, const polfed_op*, BlockWs&,
                                      const polfed_plan&, const double*, const double*,
                                      double*);
template void block_filter_on<float>(hipStream_t, const polfed_op*, BlockWs&,
                                     const polfed_plan&, const double*, const float*, float*);

// ------------------------------------------------- block orthogonalization ----

// A (s x s) = (pass 0) or += (pass 1) rows row0..row0+s-1 of the ldc x s
// coefficient block C.
__global__ void k_take_rows(const double* __restrict__ C, int ldc, int row0, int s, int pass,
                            double* __restrict__ A) {
  for (int i = threadIdx.x; i < s * s; i += blockDim.x) {
    const int r = i % s, col = i / s;
    const double v = C[row0 + r + (size_t)col * ldc];
    A[i] = pass ? A[i] + v : v;
  }
}

// Column col of Bn: rows 0..col-1 = (pass 0) or += (pass 1) c[0..col); the
// first pass also zeroes the rows below the diagonal.
__global__ void k_r_col(const double* __restrict__ c, int s, int col, int pass,
                        double* __restrict__ Bn) {
  for (int r = threadIdx.x; r < s; r += blockDim.x) {
    double* d = Bn + r + (size_t)col * s;
    if (r < col)
      *d = pass ? *d + c[r] : c[r];
    else if (r > col && pass == 0)
      *d = 0.0;
  }
}

namespace {

// w <- w - V V^T w over the first k1 columns, twice; the coefficients of the
// last pass stay in c
void cgs2_plain(hipStream_t st, int64_t D, int k1, const double* V, double* w, double* c,
                double* partial, int64_t nseg) {
  for (int pass = 0; pass < 2; ++pass) {
    dev_gemv_t(st, D, k1, V, D, w, partial, nseg, c, nullptr, 0);
    dev_gemv_n_sub(st, D, k1, V, D, c, w);
  }
}

}  // namespace

int block_orth(hipStream_t st, int64_t D, int k, int s, double* V, double* W, double* save,
               double* c, double* partial, int64_t nseg, int* flag, double* scal, double* A,
               double* Bn, double* Cb, uint64_t& seed) {
  const int kb = k + s;  // basis columns before the new block
  // block Gram-Schmidt against all kb columns, two passes, as tall-skinny
  // products: C = V^T W, W -= V C; the rows of the current block sum to A
  for (int pass = 0; pass < 2; ++pass) {
    dev_block_gs_pass(st, D, kb, V, W, s, partial, nseg, Cb);
    hipLaunchKernelGGL(k_take_rows, dim3(1), dim3(256), 0, st, Cb, kb, k, s, pass, A);
    HIPC(hipGetLastError());
  }
  HIPC(hipMemcpyAsync(save, W, (size_t)D * s * sizeof(double), hipMemcpyDeviceToDevice, st));
  const double* Vn = V + (size_t)kb * D;  // the new block
  int c0 = 0, replaced = 0;
  std::vector<double> Bh((size_t)s * s);
  for (;;) {
    // inside the block: column col against the new columns 0..col-1 (two
    // passes), then normalized into column kb + col
    for (int col = c0; col < s; ++col) {
      double* w = W + (size_t)col * D;
      for (int pass = 0; pass < 2; ++pass) {
        if (col > 0) dev_gemv_t(st, D, col, Vn, D, w, partial, nseg, c, nullptr, 0);
        hipLaunchKernelGGL(k_r_col, dim3(1), dim3(64), 0, st, c, s, col, pass, Bn);
        HIPC(hipGetLastError());
        if (col > 0) dev_gemv_n_sub(st, D, col, Vn, D, c, w);
      }
      double* rcc = Bn + col + (size_t)col * s;
      dev_dot(st, D, w, w, partial, 1024, rcc, 1);
      dev_scale_into(st, D, w, rcc, V + (size_t)(kb + col) * D, flag);
    }
    HIPC(hipMemcpyAsync(Bh.data(), Bn, Bh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    int bad = -1;
    for (int col = c0; col < s; ++col) {
      const double r = Bh[(size_t)col + (size_t)col * s];
      if (!std::isfinite(r))
        fail(POLFED_ERR_BOUNDS, "filter blow-up: non-finite block norm (spectral bounds too tight?)");
      if (r <= 1e-13) {
        bad = col;
        break;
      }
    }
    if (bad < 0) break;
    if (++replaced > 4 * s) fail(POLFED_ERR_BREAKDOWN, "block Lanczos breakdown: too many restarts");
    // The block lost rank at column `bad`: its direction is a random unit
    // vector orthogonal to the basis, with a zero entry on the diagonal of
    // Bn (W's column lies in the span of the earlier ones).
    const int k1 = kb + bad;
    double* w = W + (size_t)bad * D;
    dev_random(st, D, seed++, w);
    cgs2_plain(st, D, k1, V, w, c, partial, nseg);
    dev_dot(st, D, w, w, partial, 1024, scal, 1);
    dev_scale_into(st, D, w, scal, V + (size_t)k1 * D, flag);
    const double zero = 0.0;
    HIPC(hipMemcpyAsync(Bn + bad + (size_t)bad * s, &zero, sizeof(double), hipMemcpyHostToDevice,
                        st));
    HIPC(hipMemsetAsync(flag, 0, sizeof(int), st));
    // the later columns start again from their state after the block passes
    c0 = bad + 1;
    if (c0 < s)
      HIPC(hipMemcpyAsync(W + (size_t)c0 * D, save + (size_t)c0 * D,
                          (size_t)D * (s - c0) * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPC(hipStreamSynchronize(st));
    if (c0 >= s) break;
  }
  return replaced;
}

void block_start(hipStream_t st, int64_t D, int s, const double* X0, double* V, double* w,
                 double* c, double* partial, int64_t nseg, int* flag, double* scal) {
  std::vector<double> nrm(2);
  for (int col = 0; col < s; ++col) {
    HIPC(hipMemcpyAsync(w, X0 + (size_t)col * D, (size_t)D * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
    dev_dot(st, D, w, w, partial, 1024, scal, 1);
    cgs2_plain(st, D, col, V, w, c, partial, nseg);
    dev_dot(st, D, w, w, partial, 1024, scal + 1, 1);
    HIPC(hipMemcpyAsync(nrm.data(), scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    REQUIRE(std::isfinite(nrm[0]) && nrm[0] > 0 && nrm[1] > 1e-10 * nrm[0],
            "solve: the start block x0 must have full rank");
    dev_scale_into(st, D, w, scal + 1, V + (size_t)col * D, flag);
  }
  HIPC(hipStreamSynchronize(st));
}

// ------------------------------------------------------ SolveRun, s > 1 ----

void SolveRun::grow_band(int blocks) {
  if (blocks <= band_blocks) return;
  const size_t per = (size_t)2 * s * s;
  DevBuf nb(per * blocks * sizeof(double));
  if (band_blocks > 0)
    HIPC(hipMemcpyAsync(nb.get(), band.get(), per * band_blocks * sizeof(double),
                        hipMemcpyDeviceToDevice, ctx->stream));
  HIPC(hipStreamSynchronize(ctx->stream));
  band = std::move(nb);
  band_blocks = blocks;
}

// P(H~) V_j for the current block (columns k..k+s-1) into bw.w, by direct
// launches or a graph replay, chosen like the single-vector filter.
void SolveRun::filter_block() {
  hipStream_t st = ctx->stream;
  const int64_t D = op->D;
  const size_t n = (size_t)D * s;
  if (mode == kTimeDirect && (p.graph == 2 || pl.K < 8 || pl.K > kGraphMaxSteps)) mode = kDirect;
  if (mode == kTimeDirect && p.graph == 1) mode = kGraph;
  const bool use_graph = mode == kTimeGraph || mode == kGraph;
  if (use_graph && !graph.ready()) {
    if (!fp32) bw.vin.alloc(n * sizeof(double));
    graph.capture(ctx->cap_stream, [&](hipStream_t cs) {
      if (fp32)
        block_filter_on<float>(cs, op, bw, pl, a.data(), bw.v32.as<float>(), bw.w32.as<float>());
      else
        block_filter_on<double>(cs, op, bw, pl, a.data(), bw.vin.as<double>(),
                                bw.w.as<double>());
    });
  }
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  HIPC(hipEventRecord(e0, st));
  const double* Vj = B.col(k);
  if (fp32) dev_copy_d2f(st, (int64_t)n, Vj, bw.v32.as<float>());
  if (use_graph) {
    if (!fp32)
      HIPC(hipMemcpyAsync(bw.vin.get(), Vj, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    graph.launch(st);
  } else if (fp32) {
    block_filter_on<float>(st, op, bw, pl, a.data(), bw.v32.as<float>(), bw.w32.as<float>());
  } else {
    block_filter_on<double>(st, op, bw, pl, a.data(), Vj, bw.w.as<double>());
  }
  if (fp32) dev_copy_f2d(st, (int64_t)n, bw.w32.as<float>(), bw.w.as<double>());
  HIPC(hipEventRecord(e1, st));
  fev.emplace_back(e0, e1);
  R.filter_steps += (double)pl.K * s;
  R.filter_bytes += (double)pl.K * s * step_bytes(op, fp32 ? POLFED_FP32 : POLFED_FP64);
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
        std::fprintf(stderr, "[polfed] block filter s=%d K=%d: direct %.3f ms, graph %.3f ms -> %s\n",
                     s, pl.K, t_direct_ms, ms, mode == kGraph ? "graph" : "direct");
    }
  }
}

// Orthogonalization and QR of the filtered block, then, at the periodic
// checks, the block tridiagonal H_L (diagonal blocks A_j symmetrized,
// B_{j+1} below and B_{j+1}^T above), its eigenvalues and the last block of
// every eigenvector, and the residual estimate ||B_{m+1} tau_mj|| (eq.
// blocklan_criterion) for the n_want largest Ritz values of P(H~).
void SolveRun::advance_block() {
  hipStream_t st = ctx->stream;
  const int64_t D = op->D;
  const size_t ss = (size_t)s * s;
  const int j = k / s;
  grow_band(j + 2);
  double* Aj = band.as<double>() + 2 * ss * j;
  hipEvent_t r0, r1;
  HIPC(hipEventCreate(&r0));
  HIPC(hipEventCreate(&r1));
  HIPC(hipEventRecord(r0, st));
  const size_t cb_need = (size_t)(k + s) * s * sizeof(double);
  if (bw.cb.bytes() < cb_need) bw.cb.alloc(std::max(cb_need, (size_t)(cap + 2 * s) * s * sizeof(double)));
  // partials: 8 columns of coefficients per row segment and basis vector
  const size_t part_need = ((size_t)ws.nseg * (k + 2 * s + 1) * 8 + 8192) * sizeof(double);
  if (bw.part.bytes() < part_need)
    bw.part.alloc(std::max(part_need, ((size_t)ws.nseg * (cap + 2 * s + 1) * 8 + 8192) * sizeof(double)));
  R.restarts += block_orth(st, D, k, s, B.V.as<double>(), bw.w.as<double>(),
                           bw.save.as<double>(), ws.c.as<double>(), bw.part.as<double>(),
                           ws.nseg, ws.flag.as<int>(), ws.scal.as<double>(), Aj, Aj + ss,
                           bw.cb.as<double>(), restart_seed);
  HIPC(hipEventRecord(r1, st));
  rev.emplace_back(r0, r1);
  k += s;
  if (k >= cap && cap < M_max) {
    const int ncap = std::min(M_max, (((int)std::ceil(1.25 * cap) + 1 + s - 1) / s) * s);
    B.ensure(st, D, ncap + 2 * s - 1, k + s);
    ws.grow(st, ncap + 2 * s);
    cap = ncap;
  }
  if (k < next_check && k < M_max) return;

  const double tc = now_seconds();
  const int m = k / s;
  std::vector<double> band_h(2 * ss * m);
  HIPC(hipMemcpyAsync(band_h.data(), band.get(), band_h.size() * sizeof(double),
                      hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  drain();
  for (double x : band_h)
    if (!std::isfinite(x) || std::fabs(x) > 4.0)
      fail(POLFED_ERR_BOUNDS, "filter blow-up: block Lanczos coefficient " + std::to_string(x) +
                                  " (spectral bounds too tight?)");
  ++R.checks;
  // H_L, column-major k x k (symmetric)
  std::vector<double> H((size_t)k * k, 0.0);
  for (int b = 0; b < m; ++b) {
    const double* A = band_h.data() + 2 * ss * b;
    const double* Bn = A + ss;
    for (int c = 0; c < s; ++c)
      for (int i = 0; i < s; ++i)
        H[(size_t)(b * s + i) + (size_t)(b * s + c) * k] =
            0.5 * (A[i + (size_t)c * s] + A[c + (size_t)i * s]);
    if (b + 1 < m)
      for (int c = 0; c < s; ++c)
        for (int i = 0; i <= c; ++i) {
          const double v = Bn[i + (size_t)c * s];
          H[(size_t)((b + 1) * s + i) + (size_t)(b * s + c) * k] = v;
          H[(size_t)(b * s + c) + (size_t)((b + 1) * s + i) * k] = v;
        }
  }
  const double* Blast = band_h.data() + 2 * ss * (m - 1) + ss;
  std::vector<double> th, Zt;
  sym_eig_tail(k, H, s, th, Zt);
  std::vector<int> order(k);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return th[x] > th[y]; });
  const int nw = std::min(n_want, k);
  double thmax = 0;
  for (double t : th) thmax = std::max(thmax, std::fabs(t));
  bool conv = true;
  double est_max = 0;
  int lead = 0;  // leading run of converged Ritz values, from the largest
  for (int q = 0; q < k; ++q) {
    const int jj = order[q];
    double e2 = 0;
    for (int i = 0; i < s; ++i) {
      double acc = 0;
      for (int c = i; c < s; ++c) acc += Blast[i + (size_t)c * s] * Zt[(size_t)c * k + jj];
      e2 += acc * acc;
    }
    const double e = std::sqrt(e2);
    const bool ok_q = e <= tol_ritz * std::max(1.0, thmax);
    if (q < nw) {
      est_max = std::max(est_max, e);
      if (!ok_q) conv = false;
    }
    if (ok_q && lead == q) ++lead;
    if (!ok_q && q >= nw) break;
  }
  const bool early = !conv && early_ready(lead);
  if (verbose())
    std::fprintf(stderr,
                 "[polfed] block check k=%d s=%d n_want=%d max |B tau|=%.2e tol=%.1e conv=%d "
                 "lead=%d\n",
                 k, s, n_want, est_max, tol_ritz, (int)conv, lead);
  R.t_check += now_seconds() - tc;
  if (conv || k >= M_max || early) {
    const bool full = conv || k >= M_max;
    const int take = full ? nw : lead;
    std::vector<double> thf, Z;
    sym_eig(k, H, thf, Z);
    DevBuf dZ;
    upload(dZ, Z.data(), Z.size(), st);
    if (conclude(thf, dZ, take, !full)) return;
  }
  next_check = k + check_every;
}

// --------------------------------------------------- single block step (API) ----

void block_lanczos_step(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE,
                        const double* a, int K, double* V, int k, int s, double* A,
                        double* Bn, int precision) {
  hipStream_t st = ctx->stream;
  const int64_t D = op->D;
  polfed_plan pl{};
  pl.E_c = E_c;
  pl.dE = dE;
  pl.K = K;
  const bool f32 = precision == POLFED_FP32;
  BlockWs bw;
  bw.init(ctx, op, s, f32, pl, a);
  const double* Vj = V + (size_t)k * D;
  const size_t n = (size_t)D * s;
  if (f32) {
    dev_copy_d2f(st, (int64_t)n, Vj, bw.v32.as<float>());
    block_filter_on<float>(st, op, bw, pl, a, bw.v32.as<float>(), bw.w32.as<float>());
    dev_copy_f2d(st, (int64_t)n, bw.w32.as<float>(), bw.w.as<double>());
  } else {
    block_filter_on<double>(st, op, bw, pl, a, Vj, bw.w.as<double>());
  }
  const int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(256, (D + 8191) / 8192));
  DevBuf c((size_t)(k + 2 * s + 1) * sizeof(double)),
      part(((size_t)nseg * (k + 2 * s + 1) * 8 + 8192) * sizeof(double)), flag(64),
      scal(8 * sizeof(double));
  HIPC(hipMemsetAsync(flag.get(), 0, 64, st));
  uint64_t seed = 0xB10CULL + (uint64_t)k;
  DevBuf cb((size_t)(k + s) * s * sizeof(double));
  block_orth(st, D, k, s, V, bw.w.as<double>(), bw.save.as<double>(), c.as<double>(),
             part.as<double>(), nseg, flag.as<int>(), scal.as<double>(), A, Bn, cb.as<double>(),
             seed);
  HIPC(hipStreamSynchronize(st));
}

}  // namespace polfed

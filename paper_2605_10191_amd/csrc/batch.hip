// Multi-column filter P(H~_c) v_c for a batch of chain realizations that
// share the off-diagonal pattern, and the batched solve built on it: every
// realization runs its own filtered Lanczos iteration (its own bounds, plan,
// Krylov basis and checks), while the filter of all unfinished
// realizations is one multi-column Clenshaw recurrence.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <memory>

#include "internal.hpp"
#include "solve_run.hpp"

namespace polfed {

template <typename T>
__global__ void k_scale_cols(int64_t D, int nb, const T* __restrict__ a, const T* v, T* y) {
  const int64_t n = D * nb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i / D] * v[i];
}

template <typename T>
static void scale_cols(hipStream_t s, int64_t D, int nb, const T* a, const T* v, T* y) {
  const int64_t n = D * nb;
  if (!n) return;
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256));
  hipLaunchKernelGGL((k_scale_cols<T>), dim3(g), dim3(256), 0, s, D, nb, a, v, y);
  HIPC(hipGetLastError());
}

// y (interleaved: element (r, c) at r nb + c) = a_c v_c, v column-major.
template <typename T>
__global__ void k_scale_ilv(int64_t D, int nb, const T* __restrict__ a, const T* v, T* y) {
  const int64_t n = D * nb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / nb;
    const int c = (int)(i - r * nb);
    y[i] = a[c] * v[(int64_t)c * D + r];
  }
}

void BatchCoef::set(hipStream_t s, int nb_, const double* const* a, const int* K) {
  nb = nb_;
  Kmax = 0;
  for (int c = 0; c < nb; ++c) {
    REQUIRE(K[c] >= 0, "batch filter: need K >= 0");
    Kmax = std::max(Kmax, K[c]);
  }
  std::vector<double> A((size_t)(Kmax + 1) * nb, 0.0);
  for (int c = 0; c < nb; ++c)
    for (int i = 0; i <= K[c]; ++i) A[(size_t)i * nb + c] = a[c][i];
  host = A;
  this->K.assign(K, K + nb);
  upload(dK, this->K.data(), this->K.size(), s);
  std::vector<float> A32(A.begin(), A.end());
  upload(d64, A.data(), A.size(), s);
  upload(d32, A32.data(), A32.size(), s);
  HIPC(hipStreamSynchronize(s));
}

// Clenshaw recurrence of eq. clenshaw_chebyshev_prod for all columns at once.
// A column whose order K_c is below the batch maximum has zero coefficients
// above K_c, so its b_i stay zero until i = K_c.
template <typename T>
void filter_apply_batch_on(hipStream_t s, const ChainBatch& bt, const BatchCoef& co,
                           const T* v, T* w, T* bufA, T* bufB) {
  const int64_t D = bt.ops[0]->D;
  const int nb = bt.nb;
  REQUIRE(co.nb == nb, "batch filter: coefficient table of another batch");
  const T* A = (const T*)(sizeof(T) == 8 ? co.d64.get() : co.d32.get());
  const int K = co.Kmax;
  if (K == 0) {
    scale_cols<T>(s, D, nb, A, v, w);
    return;
  }
  // the recurrence blocks take the tuned kernel's layout; v and w stay
  // column-major
  const int var = batch_variant<T>(s, bt);
  if (var == 5) {
    chain_lds_filter<T>(s, bt, A, co.dK.as<int>(), v, w);
    return;
  }
  if (var == 4) {
    // every column its own recurrence with its operator's tuned kernel
    std::vector<double> ac;
    for (int c = 0; c < nb; ++c) {
      ac.resize((size_t)co.K[c] + 1);
      for (int i = 0; i <= co.K[c]; ++i) ac[i] = co.host[(size_t)i * nb + c];
      filter_apply_on<T>(s, bt.ops[c], bt.E_c[c], bt.dE[c], ac.data(), co.K[c],
                         v + (size_t)c * D, w + (size_t)c * D, bufA + (size_t)c * D,
                         bufB + (size_t)c * D);
    }
    return;
  }
  const bool ilv = var >= 2;
  if (ilv) {
    const int64_t n = D * nb;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256));
    hipLaunchKernelGGL((k_scale_ilv<T>), dim3(g), dim3(256), 0, s, D, nb, A + (size_t)K * nb, v,
                       bufA);
    HIPC(hipGetLastError());
  } else {
    scale_cols<T>(s, D, nb, A + (size_t)K * nb, v, bufA);
  }
  const T* cur = bufA;
  T* prev = nullptr;
  for (int i = K - 1; i >= 1; --i) {
    T* out = prev ? prev : bufB;
    chain_batch_step_var<T>(s, bt, var, false, A + (size_t)i * nb, v, true, cur, prev, out, !ilv);
    prev = const_cast<T*>(cur);
    cur = out;
  }
  chain_batch_step_var<T>(s, bt, var, true, A, v, true, cur, prev, w, true);
}

template <typename T>
void filter_apply_batch(polfed_ctx* ctx, const ChainBatch& bt, const BatchCoef& co,
                        const T* v, T* w, T* bufA, T* bufB) {
  filter_apply_batch_on<T>(ctx->stream, bt, co, v, w, bufA, bufB);
}

template void filter_apply_batch<double>(polfed_ctx*, const ChainBatch&, const BatchCoef&,
                                         const double*, double*, double*, double*);
template void filter_apply_batch<float>(polfed_ctx*, const ChainBatch&, const BatchCoef&,
                                        const float*, float*, float*, float*);

bool BatchFilter::same_members(const std::vector<SolveRun*>& runs) const {
  if (runs.size() != ids.size()) return false;
  for (size_t i = 0; i < runs.size(); ++i)
    if (runs[i] != members[i] || runs[i]->uid != ids[i]) return false;
  return true;
}

void BatchFilter::drain() {
  for (auto& pd : pending) {
    HIPC(hipEventSynchronize(pd.e1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, pd.e0, pd.e1));
    for (auto* r : pd.runs) r->R.t_filter += 1e-3 * ms / (double)pd.runs.size();
    HIPC(hipEventDestroy(pd.e0));
    HIPC(hipEventDestroy(pd.e1));
  }
  pending.clear();
}

void BatchFilter::forget() {
  for (auto& pd : pending) {
    (void)hipEventDestroy(pd.e0);
    (void)hipEventDestroy(pd.e1);
  }
  pending.clear();
}

BatchFilter::~BatchFilter() { forget(); }

std::string BatchFilter::graph_choice_key() const {
  int lg = 0;
  while ((2 << lg) <= std::max(co.Kmax, 1)) ++lg;
  return "bgraph" + std::to_string(co.nb) + (fp32 ? "|32|" : "|64|") + std::to_string(lg);
}

void BatchFilter::form(polfed_ctx* c, const std::vector<SolveRun*>& runs) {
  drain();
  ctx = c;
  members = runs;
  ids.clear();
  for (auto* r : runs) ids.push_back(r->uid);
  const int nb = (int)runs.size();
  std::vector<const polfed_op*> ops(nb);
  std::vector<double> Ec(nb), dE(nb);
  std::vector<const double*> a(nb);
  std::vector<int> K(nb);
  fp32 = runs[0]->fp32;
  for (int i = 0; i < nb; ++i) {
    REQUIRE(runs[i]->fp32 == fp32, "batch: members must share the precision");
    ops[i] = runs[i]->op;
    Ec[i] = runs[i]->pl.E_c;
    dE[i] = runs[i]->pl.dE;
    a[i] = runs[i]->a.data();
    K[i] = runs[i]->pl.K;
  }
  bt.init(c, ops.data(), nb);
  bt.set_scale(Ec.data(), dE.data());
  co.set(c->stream, nb, a.data(), K.data());
  // the step kernel is picked before run() records the recurrence
  if (fp32)
    (void)batch_variant<float>(c->stream, bt);
  else
    (void)batch_variant<double>(c->stream, bt);
  graph.reset();
  graph_pref = runs[0]->p.graph;
  mode = kTimeDirect;
  if (graph_pref == 2 || co.Kmax < 8 || co.Kmax > kGraphMaxSteps) mode = kDirect;
  if (graph_pref == 1 && mode == kTimeDirect) mode = kGraph;
  if (mode == kTimeDirect) {
    // the way an earlier batch of this pattern, width, precision and order
    // (to a factor of two) chose
    const int v = pattern_choice(ops[0], graph_choice_key());
    if (v >= 0) mode = v == 1 ? kGraph : kDirect;
  }
  const int64_t D = ops[0]->D;
  const size_t tb = fp32 ? sizeof(float) : sizeof(double);
  const size_t need = (size_t)D * nb * tb;
  if (vb.bytes() < need) {
    vb.alloc(need);
    wb.alloc(need);
    bA.alloc(need);
    bB.alloc(need);
  }
}

// One filter application for every member: gather v_k of each member into
// the block, run the recurrence, scatter P(H~) v_k into each member's w.
// Only the two applications that choose between direct launches and a graph
// wait for the device; the others are timed when drained.
void BatchFilter::run() {
  hipStream_t s = ctx->stream;
  const int nb = (int)members.size();
  const int64_t D = bt.ops[0]->D;
  const bool use_graph = mode == kTimeGraph || mode == kGraph;
  if (use_graph && !graph.ready())
    graph.capture(ctx->cap_stream, [&](hipStream_t cs) {
      if (fp32)
        filter_apply_batch_on<float>(cs, bt, co, vb.as<float>(), wb.as<float>(), bA.as<float>(),
                                     bB.as<float>());
      else
        filter_apply_batch_on<double>(cs, bt, co, vb.as<double>(), wb.as<double>(),
                                      bA.as<double>(), bB.as<double>());
    });
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  HIPC(hipEventRecord(e0, s));
  for (int i = 0; i < nb; ++i) {
    if (fp32)
      dev_copy_d2f(s, D, members[i]->vec(), vb.as<float>() + (size_t)i * D);
    else
      HIPC(hipMemcpyAsync(vb.as<double>() + (size_t)i * D, members[i]->vec(),
                          (size_t)D * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  if (use_graph)
    graph.launch(s);
  else if (fp32)
    filter_apply_batch<float>(ctx, bt, co, vb.as<float>(), wb.as<float>(), bA.as<float>(),
                              bB.as<float>());
  else
    filter_apply_batch<double>(ctx, bt, co, vb.as<double>(), wb.as<double>(),
                               bA.as<double>(), bB.as<double>());
  for (int i = 0; i < nb; ++i) {
    if (fp32)
      dev_copy_f2d(s, D, wb.as<float>() + (size_t)i * D, members[i]->wbuf());
    else
      HIPC(hipMemcpyAsync(members[i]->wbuf(), wb.as<double>() + (size_t)i * D,
                          (size_t)D * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  HIPC(hipEventRecord(e1, s));
  for (auto* r : members) {
    r->R.filter_steps += r->pl.K;
    r->R.filter_bytes += r->pl.K * (fp32 ? 16.0 : 32.0) * (double)D;
  }
  if (mode != kTimeDirect && mode != kTimeGraph) {
    pending.push_back({e0, e1, members});
    return;
  }
  HIPC(hipEventSynchronize(e1));
  float ms = 0;
  HIPC(hipEventElapsedTime(&ms, e0, e1));
  HIPC(hipEventDestroy(e0));
  HIPC(hipEventDestroy(e1));
  const double t = 1e-3 * ms;
  if (mode == kTimeDirect) {
    t_direct_ms = ms;
    mode = kTimeGraph;
  } else if (mode == kTimeGraph) {
    mode = ms < t_direct_ms ? kGraph : kDirect;
    if (mode == kDirect) graph.reset();
    pattern_choice_set(bt.ops[0], graph_choice_key(), mode == kGraph ? 1 : 0);
    if (verbose())
      std::fprintf(stderr, "[polfed] batch filter nb=%d K=%d: direct %.3f ms, graph %.3f ms -> %s\n",
                   nb, co.Kmax, t_direct_ms, ms, mode == kGraph ? "graph" : "direct");
  }
  for (auto* r : members) r->R.t_filter += t / nb;
}

polfed_status solve_batch(polfed_ctx* ctx, int B, const polfed_op* const* ops,
                          const polfed_params& p, const double* const* x0,
                          double* const* evals, double* const* evecs, double* const* resid,
                          int* n_found, polfed_report* rep) {
  REQUIRE(B >= 1, "solve_batch: need B >= 1");
  REQUIRE(ops && x0 && evals && evecs && resid && n_found, "solve_batch: null array");
  REQUIRE(p.block_size <= 1, "solve_batch: block Lanczos (block_size > 1) runs through polfed_solve only");
  for (int i = 0; i < B; ++i) {
    REQUIRE(ops[i] && ops[i]->ctx == ctx, "solve_batch: operator missing or of another context");
    REQUIRE(ops[i]->model == Model::Chain && !ops[i]->pattern_key.empty() &&
                ops[i]->pattern_key == ops[0]->pattern_key,
            "solve_batch: operators must be chains sharing the off-diagonal pattern");
  }
  // one precision for the whole batch: the operators share the pattern, so
  // the first one's timing stands for all
  polfed_params q = p;
  q.precision = resolve_precision(ctx->stream, ops[0], p.precision);
  std::vector<std::unique_ptr<SolveRun>> runs;
  for (int i = 0; i < B; ++i) {
    runs.emplace_back(new SolveRun());
    runs.back()->setup(ctx, ops[i], q, x0[i], evals[i], evecs[i], resid[i], &n_found[i]);
  }
  // one batched filter per precision: an FP32-bulk run whose refinement
  // stalls continues with the FP64 filter
  BatchFilter bf[2];
  for (;;) {
    std::vector<SolveRun*> now[2];
    for (auto& r : runs)
      if (!r->done) now[r->fp32 ? 1 : 0].push_back(r.get());
    if (now[0].empty() && now[1].empty()) break;
    for (int g = 0; g < 2; ++g) {
      if (now[g].empty()) continue;
      if (!bf[g].same_members(now[g])) bf[g].form(ctx, now[g]);
      bf[g].run();
      for (auto* r : now[g]) r->advance();
    }
  }
  for (auto& f : bf) f.drain();
  polfed_status st = POLFED_OK;
  for (int i = 0; i < B; ++i) {
    polfed_report& R = runs[i]->R;
    R.filter_GBps = R.t_filter > 0 ? R.filter_bytes / R.t_filter / 1e9 : 0;
    if (rep) rep[i] = R;
    if (runs[i]->status != POLFED_OK) st = POLFED_NOT_CONVERGED;
  }
  return st;
}

}  // namespace polfed

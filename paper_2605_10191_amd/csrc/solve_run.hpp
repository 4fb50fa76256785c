// Resumable POLFED solve: the per-realization state of the filtered Lanczos
// iteration, driven either one column at a time or by a multi-column filter
// shared with other realizations.
#pragma once
#include <functional>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace polfed {

struct Basis {
  int64_t D = 0;
  int cap = 0;  // columns available beyond v_0: V holds cap + 1 vectors
  DevBuf V;
  void ensure(hipStream_t s, int64_t D_, int need_cap, int keep_cols) {
    if (need_cap <= cap && D_ == D) return;
    DevBuf nv((size_t)D_ * (need_cap + 1) * sizeof(double));
    if (keep_cols > 0)
      HIPC(hipMemcpyAsync(nv.get(), V.get(), (size_t)D_ * keep_cols * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    V = std::move(nv);
    D = D_;
    cap = need_cap;
  }
  double* col(int j) const { return V.as<double>() + (size_t)j * D; }
};

struct Ws {
  DevBuf w, c, partial, scal, flag, alpha, beta, bA, bB, v32, w32;
  int64_t nseg = 0;
  int coef_cap = 0;
  void init(hipStream_t s, int64_t D, int max_cols, bool fp32) {
    w.alloc(std::max<int64_t>(D, 1) * sizeof(double));
    nseg = std::max<int64_t>(1, std::min<int64_t>(256, (D + 8191) / 8192));
    grow(s, max_cols);
    scal.alloc(64 * sizeof(double));
    flag.alloc(sizeof(int));
    HIPC(hipMemsetAsync(flag.get(), 0, sizeof(int), s));
    const size_t tb = fp32 ? sizeof(float) : sizeof(double);
    bA.alloc(std::max<int64_t>(D, 1) * tb);
    bB.alloc(std::max<int64_t>(D, 1) * tb);
    if (fp32) {
      v32.alloc(std::max<int64_t>(D, 1) * sizeof(float));
      w32.alloc(std::max<int64_t>(D, 1) * sizeof(float));
    }
  }
  void grow(hipStream_t s, int max_cols) {
    if (max_cols <= coef_cap) return;
    DevBuf na((size_t)(max_cols + 1) * sizeof(double)), nb((size_t)(max_cols + 2) * sizeof(double));
    if (coef_cap > 0) {
      HIPC(hipMemcpyAsync(na.get(), alpha.get(), (size_t)(coef_cap + 1) * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
      HIPC(hipMemcpyAsync(nb.get(), beta.get(), (size_t)(coef_cap + 2) * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
      HIPC(hipStreamSynchronize(s));
    }
    alpha = std::move(na);
    beta = std::move(nb);
    c.alloc((size_t)(max_cols + 1) * sizeof(double));
    partial.alloc((size_t)nseg * (max_cols + 1) * sizeof(double) + 8192 * sizeof(double));
    coef_cap = max_cols;
  }
};

// Ritz pairs of H on a subspace: U2 (D x n, orthonormal), HU2 = H U2, E,
// residual norms, and the selection made from them.
struct Extracted {
  std::vector<double> E, res;
  std::vector<int> sel;  // chosen columns of U2, ordered by (|E - lambda|, E)
  bool complete = false;
  DevBuf U2, HU2;
};

// Rayleigh-Ritz of H on span(U) (U orthonormal D x n, HU = H U).
void rayleigh_ritz(hipStream_t s, int64_t D, int n, const double* U, const double* HU,
                   int64_t nseg, Extracted& ex);
void select_pairs(Extracted& ex, double lam, int n_ev, double tol_resid, double theta_min,
                  const polfed_plan& pl);

double step_bytes(const polfed_op* op, int precision);

// Device coefficient table [(Kmax + 1)][nb] of a multi-column filter; column
// c is zero above its own order K[c].
struct BatchCoef {
  DevBuf d64, d32;
  int nb = 0, Kmax = 0;
  std::vector<double> host;  // (Kmax + 1) x nb, column c of row i = a_c[i]
  std::vector<int> K;        // each column's own order
  DevBuf dK;                 // the same on the device (int32)
  void set(hipStream_t s, int nb, const double* const* a, const int* K);
};

// Device state of the block filter and block orthogonalization (block
// Lanczos, Sec. 2.2): the filtered block W, a copy of it for the repair of a
// rank-deficient block, the filter buffers and, for chain operators, the
// multi-column recurrence with every column on the same operator.
struct BlockWs {
  int s = 0;
  int64_t D = 0;
  bool fp32 = false, batched = false;
  DevBuf w, save, vin;     // D x s FP64
  DevBuf cb;               // (k + s) x s block Gram-Schmidt coefficients
  DevBuf part;             // reduction partials of the block products
  DevBuf v32, w32;         // D x s FP32 (FP32 filter)
  DevBuf bA, bB;           // D x s of the filter precision
  ChainBatch bt;
  BatchCoef co;
  void init(polfed_ctx* ctx, const polfed_op* op, int s, bool fp32, const polfed_plan& pl,
            const double* a);
};

// W = P(H~) X for the D x s block X (columns contiguous), into W.
template <typename T>
void block_filter_on(hipStream_t st, const polfed_op* op, BlockWs& bw, const polfed_plan& pl,
                     const double* a, const T* X, T* W);

// Orthogonalizes the filtered block W (D x s, overwritten) against basis
// columns [0, k + s) of V and writes the next block into columns
// [k + s, k + 2s): two passes of block Gram-Schmidt against [0, k + s)
// (tall-skinny products through Cb, (k + s) x s), then, column by column,
// two passes against the new block's earlier columns and normalization.
// The summed projections onto the current block give A (s x s, col-major);
// those onto the new columns and the norms give the upper triangular Bn.
// save: D x s scratch; c, partial: coefficient scratch for k + 2s columns;
// scal: 8 device doubles.  Returns the number of rank-deficient columns
// replaced by random directions.
int block_orth(hipStream_t st, int64_t D, int k, int s, double* V, double* W, double* save,
               double* c, double* partial, int64_t nseg, int* flag, double* scal, double* A,
               double* Bn, double* Cb, uint64_t& seed);

// Orthonormal start block: Gram-Schmidt QR (two passes per column) of the
// D x s block X0 into columns [0, s) of V; fails on a rank-deficient X0.
void block_start(hipStream_t st, int64_t D, int s, const double* X0, double* V, double* w,
                 double* c, double* partial, int64_t nseg, int* flag, double* scal);

struct SolveRun {
  // device bytes held by this solve's own buffers (declared first, so it
  // outlives every buffer member that counts toward it)
  MemTally tally;
  // inputs
  polfed_ctx* ctx = nullptr;
  const polfed_op* op = nullptr;
  polfed_params p{};
  double* evals = nullptr;
  double* evecs = nullptr;
  double* resid = nullptr;
  int* n_found = nullptr;
  // plan
  bool fp32 = false;
  double tol_resid = 1e-8, tol_ritz = 1e-10, lam = 0, sbytes = 0, t_start = 0;
  polfed_plan pl{};
  std::vector<double> a;  // filter coefficients a_0..a_K
  // Lanczos state
  int n_want = 0, n_want0 = 0, M_alloc = 0, M_max = 0, cap = 0, check_every = 0,
      next_check = 0, k = 0;
  uint64_t restart_seed = 0;
  int brk_from = 1;  // breakdowns are searched from this Lanczos index on
  Basis B;
  Ws ws;
  polfed_report R{};
  polfed_status status = POLFED_NOT_CONVERGED;
  bool done = false;
  uint64_t uid = 0;  // unique per setup(), identifies the solve in a batch
  std::vector<std::pair<hipEvent_t, hipEvent_t>> fev, rev;
  // filter launch mode: direct launches or one graph replay per application
  GraphExec graph;
  DevBuf vst;  // FP64: fixed copy of v_k read by the graph
  enum { kTimeDirect, kTimeGraph, kDirect, kGraph } mode = kTimeDirect;
  float t_direct_ms = 0;
  // block Lanczos (s > 1): band holds [A_j | B_{j+1}] (2 s^2 doubles) for
  // every block step j; the filtered block lives in bw.w
  int s = 1;
  DevBuf band;
  int band_blocks = 0;
  BlockWs bw;

  SolveRun() = default;
  SolveRun(const SolveRun&) = delete;
  SolveRun& operator=(const SolveRun&) = delete;
  ~SolveRun();
  // bounds, plan, basis allocation, v_0 = x0 / ||x0||
  void setup(polfed_ctx* c, const polfed_op* o, const polfed_params& prm, const double* x0,
             double* ev, double* vecs, double* res, int* nf);
  // Largest device bytes a solve of this operator holds when its Krylov
  // space stays within the expected size and n_want does not grow: the
  // bounds Lanczos (unless the bounds are given), then the basis, work and
  // filter vectors, and the larger of the extraction (FP64) and the FP32
  // refinement with its FP64 fallback.
  static size_t footprint(const polfed_op* op, const polfed_params& p);
  // the same for m basis columns and n wanted pairs
  static size_t bytes_at(int64_t D, int m, int n, bool fp32);
  // Served solves: bytes beyond the admission's footprint (a basis grown
  // past the expected size, a larger n_want) are asked for through take()
  // before they are allocated; bytes no longer held go back through give().
  // Both are empty outside the server.  A refused request blocks the solve
  // (no filter runs for it) until resume() obtains the bytes.
  std::function<bool(size_t)> take;
  std::function<void(size_t)> give;
  size_t want = 0;     // bytes a blocked solve waits for
  size_t granted = 0;  // bytes obtained ahead of the allocation that needs them
  enum { kPendNone, kPendGrow, kPendWant } pend = kPendNone;
  int pend_n_want = 0;
  bool blocked() const { return want > 0; }
  bool reserve(size_t bytes);  // false: blocked, want = bytes
  void resume();               // retries a blocked request, then continues
  void step_tail();            // basis growth and the periodic check
  const double* vec() const { return B.col(k); }  // v_k, the vector to filter
  double* wbuf() const { return ws.w.as<double>(); }  // where P(H~) v_k goes
  void filter_self();  // single-column filter of v_k into wbuf()
  void advance();      // CGS2, k += 1, periodic check; sets done when finished
  void filter_block();   // block mode: P(H~) of the current block into bw.w
  void advance_block();  // block mode: orthogonalization, QR, k += s, check
  // extraction from the Ritz pairs of a passed check (values thf, vectors
  // in the columns of the device k x k matrix dC), refinement, completion
  // test; true when the run finished or restarted (no further check
  // scheduling)
  // the nw Ritz vectors of the largest values are extracted; early: the
  // check has not passed yet, so a failure only returns false
  bool conclude(const std::vector<double>& thf, const DevBuf& dC, int nw, bool early);
  bool early_ready(int lead);  // whether to try an early extraction now
  int early_lead = 0;          // leading converged run at the last early try
  void grow_band(int blocks);
  void emit(const Extracted& ex, polfed_status st);
  void fallback_fp64();  // restart the Lanczos iteration with the FP64 filter
  void finish();
  void drain();
};

// FP64-accurate refinement of the Ritz pairs of an FP32-filtered run (ex is
// updated in place, selection included).
void refine(SolveRun& run, Extracted& ex, double theta_min);

template <typename T>
void filter_apply_batch(polfed_ctx* ctx, const ChainBatch& bt, const BatchCoef& co,
                        const T* v, T* w, T* bufA, T* bufB);
template <typename T>
void filter_apply_batch_on(hipStream_t s, const ChainBatch& bt, const BatchCoef& co,
                           const T* v, T* w, T* bufA, T* bufB);

// The multi-column filter shared by a set of running solves.
struct BatchFilter {
  polfed_ctx* ctx = nullptr;
  int graph_pref = 0;  // polfed_params.graph of the members
  GraphExec graph;
  enum { kTimeDirect, kTimeGraph, kDirect, kGraph } mode = kTimeDirect;
  float t_direct_ms = 0;
  std::vector<SolveRun*> members;
  std::vector<uint64_t> ids;  // uid of each member when the batch was formed
  // true when runs are exactly the members the tables were built for
  bool same_members(const std::vector<SolveRun*>& runs) const;
  std::string graph_choice_key() const;
  bool fp32 = false;
  ChainBatch bt;
  BatchCoef co;
  DevBuf vb, wb, bA, bB;  // D x nb blocks
  // filter applications whose timing is still to be read: events and the
  // members they served (alive until drain(), which callers invoke before a
  // member is retired or the batch is re-formed)
  struct Pending {
    hipEvent_t e0, e1;
    std::vector<SolveRun*> runs;
  };
  std::vector<Pending> pending;
  void form(polfed_ctx* c, const std::vector<SolveRun*>& runs);
  void run();    // filters v_k of every member into its w (asynchronous)
  void drain();   // adds the finished applications' time to the members
  void forget();  // drops the pending timings (after an error)
  ~BatchFilter();
};

}  // namespace polfed

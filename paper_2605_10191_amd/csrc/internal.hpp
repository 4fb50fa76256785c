// Internal declarations of the POLFED HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <stdexcept>
#include <map>
#include <string>
#include <vector>

#include "../../include/polfed.h"

namespace polfed {

// ------------------------------------------------------------ errors ----

struct Error : std::runtime_error {
  polfed_status code;
  Error(polfed_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(polfed_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPC(x) ::polfed::hip_check((x), #x, __FILE__, __LINE__)
#define REQUIRE(cond, msg)                                        \
  do {                                                            \
    if (!(cond)) ::polfed::fail(POLFED_ERR_INVALID, (msg));       \
  } while (0)

// --------------------------------------------------- device buffers ----

// Device bytes held by a set of buffers: the current total and its peak.
// A buffer counts toward the tally that was active on its thread when it
// was allocated, until it is released (wherever that happens).
struct MemTally {
  size_t cur = 0, peak = 0;
};
extern thread_local MemTally* g_mem_tally;
// Makes t the active tally of this thread for the scope's lifetime.
struct TallyScope {
  MemTally* prev;
  explicit TallyScope(MemTally* t) : prev(g_mem_tally) { g_mem_tally = t; }
  ~TallyScope() { g_mem_tally = prev; }
  TallyScope(const TallyScope&) = delete;
  TallyScope& operator=(const TallyScope&) = delete;
};

// Owning device allocation (library-internal workspaces and tables).
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_), cap_(o.cap_), dev_(o.dev_), t_(o.t_) {
    o.p_ = nullptr;
    o.n_ = 0;
    o.cap_ = 0;
    o.t_ = nullptr;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_;
      n_ = o.n_;
      cap_ = o.cap_;
      dev_ = o.dev_;
      t_ = o.t_;
      o.p_ = nullptr;
      o.n_ = 0;
      o.cap_ = 0;
      o.t_ = nullptr;
    }
    return *this;
  }
  void alloc(size_t bytes);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t bytes() const { return n_; }
 private:
  void* p_ = nullptr;
  size_t n_ = 0;    // bytes asked for
  size_t cap_ = 0;  // bytes of the block (its cache bucket)
  int dev_ = 0;
  MemTally* t_ = nullptr;
};

// Streams the library queues work on, per device: a released device block
// is reused only after every registered stream has passed the release.
void register_stream(int dev, hipStream_t s);
void unregister_stream(int dev, hipStream_t s);

// A sequence of launches recorded once on a capture stream and replayed as
// one HIP graph on any stream.  The recorded launches keep their arguments,
// so everything they touch must stay at the same addresses between replays.
class GraphExec {
 public:
  GraphExec() = default;
  GraphExec(const GraphExec&) = delete;
  GraphExec& operator=(const GraphExec&) = delete;
  ~GraphExec() { reset(); }
  bool ready() const { return exec_ != nullptr; }
  void reset();
  // record(s) issues the launches on stream s (kernels only: no memset,
  // copy, allocation or synchronization)
  template <class F>
  void capture(hipStream_t cap, F&& record) {
    reset();
    begin(cap);
    try {
      record(cap);
    } catch (...) {
      abort(cap);
      throw;
    }
    end(cap);
  }
  void launch(hipStream_t s);
 private:
  void begin(hipStream_t cap);
  void end(hipStream_t cap);
  void abort(hipStream_t cap);
  hipGraphExec_t exec_ = nullptr;
};

// Set on the server's threads: they capture no graphs.  A stream capture on
// one thread can be invalidated by HIP calls other threads make meanwhile,
// and the server's rounds run side by side on several threads.
extern thread_local bool g_no_capture;

// Average run time in microseconds of one call of launch(stream), taken from
// a replay of a graph of `reps` calls on a private stream (on a thread that
// captures no graphs: from `reps` eager launches, which at small kernel sizes
// also time the host's launch gaps).  Between eager
// launches the host leaves gaps longer than a small kernel's own run time, so
// an eager timing would not tell kernel variants apart at small sizes; a
// replay runs the kernels back to back, as the filter's graphs do.  The caller
// synchronizes whatever stream produced the data the launches read.
template <class F>
float replay_time_us(F&& launch, int reps) {
  struct Timing {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timing() {
      if (s) (void)hipStreamSynchronize(s);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (s) (void)hipStreamDestroy(s);
    }
  };
  GraphExec g;  // destroyed after the stream has drained
  Timing t;
  HIPC(hipStreamCreateWithFlags(&t.s, hipStreamNonBlocking));
  HIPC(hipEventCreate(&t.e0));
  HIPC(hipEventCreate(&t.e1));
  launch(t.s);  // any first-call work outside the capture
  if (g_no_capture) {
    HIPC(hipEventRecord(t.e0, t.s));
    for (int i = 0; i < reps; ++i) launch(t.s);
    HIPC(hipEventRecord(t.e1, t.s));
    HIPC(hipEventSynchronize(t.e1));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, t.e0, t.e1));
    return 1e3f * ms / (float)reps;
  }
  g.capture(t.s, [&](hipStream_t c) {
    for (int i = 0; i < reps; ++i) launch(c);
  });
  g.launch(t.s);
  HIPC(hipEventRecord(t.e0, t.s));
  g.launch(t.s);
  HIPC(hipEventRecord(t.e1, t.s));
  HIPC(hipEventSynchronize(t.e1));
  float ms = 0;
  HIPC(hipEventElapsedTime(&ms, t.e0, t.e1));
  return 1e3f * ms / (float)reps;
}

template <class T>
void upload(DevBuf& b, const T* host, size_t n, hipStream_t s) {
  b.alloc(n * sizeof(T) > 0 ? n * sizeof(T) : 16);
  if (n) HIPC(hipMemcpyAsync(b.get(), host, n * sizeof(T), hipMemcpyHostToDevice, s));
}

// ------------------------------------------------------- model structs ----

constexpr int kBinomN = 33;  // binomial table C(n, k), 0 <= n, k <= 32

// Random-field / t-V chain in a fixed particle-number sector, matrix-free.
// Diagonal: vzz * #(occupied nearest-neighbour pairs) + c0 + sum_i f_i n_i,
// with the site sum read from four byte-indexed tables.  Hopping on an
// internal bond has amplitude t_in, on the periodic bond t_pb.
struct ChainDev {
  int L, N, periodic, Lb;
  int64_t D;
  double t_in, t_pb, vzz, c0;
  const double* ftab;      // [4][256] partial field sums (FP64)
  const float* ftab32;     // same in FP32
  const uint32_t* binom;   // [kBinomN][kBinomN]
  const int32_t* hi_off;   // ranks of the first state of each high part
  const int32_t* lo_rank;  // rank of a low part among equal-popcount ones
};

// Split layout of the chain kernel (state = hi << Lb | lo, rows of one hi
// contiguous): one wavefront per segment of a block, described by a
// 128-byte record of wave-uniform data:
//   [0] first row  [1] rows  [2] index of its first low part  [3] flags
//   (bit 0: lowest high bit, bit 1: top high bit, bits 2-11: rows of the
//   block, bits 12-21: position of the segment in its block)  [4] high bonds
//   that cannot hop  [5] row offset of the joining bond  [6] of the periodic
//   bond  [8..9] high-part diagonal (double)  [10..31] row offsets of the
//   hops inside the high part (0 where no hop).
constexpr int kChainLoBits = 10;      // Lb = min(10, L / 2); blocks <= 252 rows
constexpr int kChainSegRows = 128;   // rows per wavefront segment
constexpr int kChainStageRows = 256;  // LDS rows staged per wavefront
constexpr int kChainBlocksPerCU = 4;  // persistent blocks per compute unit
constexpr int kBatchMaxCols = 16;     // columns per multi-column launch
// A filter of more Clenshaw steps than this runs as direct launches: a graph
// of that many kernel nodes costs more to build than it saves.
constexpr int kGraphMaxSteps = 65536;
// Tile kernel: a workgroup stages 2^KT consecutive high-part blocks in LDS.
// KT is chosen so that there are at least 512 tiles; 0 = no tile kernel.
constexpr int chain_tile_bits(int L) {
  const int Lb = (L / 2 < 10) ? L / 2 : 10;
  const int Lh = L - Lb;
  const int kt = Lh - 9 < 5 ? Lh - 9 : 5;
  return (L >= 22 && kt >= 2) ? kt : 0;
}
constexpr int kTileThreads = 512;
constexpr size_t kLdsPerCU = 160 * 1024;
constexpr int kChainRecWords = 32;
constexpr int kChainMaxHighBonds = kChainRecWords - 10;
// bytes of the packed LDS image of the low-part tables, per low part lo:
// 16 bytes of block positions (the Lb-1 low-bond neighbours, own position
// where a bond cannot hop; then lo_rank of lo with its top bit flipped and of
// lo with bit 0 flipped), the low-part diagonal (T) and the low-part list
// (uint16).  16-byte multiple.
constexpr int chain_blob_bytes(int nlo, int tbytes) {
  return ((nlo * (16 + tbytes + 2)) + 15) / 16 * 16;
}
struct ChainSplitDev {
  int64_t D;
  int N, periodic;
  double t_in, t_pb, vzz;
  const void* blob64;  // packed LDS image, FP64 diagonal
  const void* blob32;  // same with FP32 diagonal
  const void* blobl64;  // the same tables in low-part list order (FP64)
  const void* blobl32;  // (FP32)
  const int32_t* rec;
  int64_t nseg;
};

constexpr int kQsunMaxL = 31;
// Quantum sun in the full space: index = dot_state << L | outer_bits.
struct QsunDev {
  int N, L;
  int64_t D;
  double c0;
  const double* hdot;     // [2^N][2^N]
  const double* ftab;     // [4][256] outer field sums (FP64)
  const float* ftab32;
  uint32_t ray_mask[kQsunMaxL];
  double ray_amp[kQsunMaxL];
};

// CSR with the diagonal split off.  Rows are grouped in blocks whose
// off-diagonal entries fit the LDS stage of the CSR kernel.
struct CsrDev {
  int64_t D;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
  const float* val32;
  const double* diag;
  const float* diag32;
  const int64_t* blk_row;  // [nblk + 1]
  int64_t nblk;
  // optimized mapping: off-diagonal values from a table of ncode distinct
  // values, by one byte per entry (code), or the single value vtab[0]
  // (ncode = 1, no code array); ncode = 0: the val arrays
  int ncode;
  const uint8_t* code;
  const double* vtab;
  const float* vtab32;
};

enum class Model { Chain, Qsun, Csr, Qrem };

}  // namespace polfed

// Opaque handles of the C ABI.
namespace polfed {
struct Server;
}

struct polfed_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  int n_cu = 256;
  std::mutex mu;  // serializes calls that use the shared workspaces
  // API calls waiting for mu (the server thread lets them in between rounds)
  std::atomic<int> api_waiting{0};
  // held shared by the server's rounds in flight, exclusively by calls that
  // may use or change operators those rounds use
  std::shared_mutex serve_mu;
  // the autotuners' choices, shared by the operators of one chain pattern
  // (same kernels and tables, only the diagonal differs): key
  // "<pattern>|<what>"; guarded by tune_mu
  std::mutex tune_mu;
  std::map<std::string, int> pattern_tuned;
  // reusable workspaces
  polfed::DevBuf scratch_red;  // reduction partials
  polfed::DevBuf scratch_scalar;
  polfed::DevBuf binom;  // binomial table for the basis calls
  polfed::DevBuf ws[8];  // scratch of the single-step entry points
  polfed::Server* server = nullptr;
};

namespace polfed {
// Lock of a context for an API call.  The call announces itself before it
// blocks: the server thread takes the lock between its rounds and, as
// std::mutex is not fair, would otherwise take it again at once and keep a
// caller (say, one building the next request's operator) waiting.  A call
// that may use or change existing operators (kOps) also waits for the
// server's rounds in flight; one that only builds new objects (kBuild) does
// not.
class CtxLock {
 public:
  enum Kind { kOps, kBuild };
  explicit CtxLock(polfed_ctx* c, Kind kind = kOps) : c_(c) {
    c_->api_waiting.fetch_add(1);
    try {
      c_->mu.lock();
    } catch (...) {
      c_->api_waiting.fetch_sub(1);  // else the server would wait for ever
      throw;
    }
    c_->api_waiting.fetch_sub(1);
    if (kind == kOps) {
      try {
        c_->serve_mu.lock();
      } catch (...) {
        c_->mu.unlock();
        throw;
      }
      ops_ = true;
    }
  }
  ~CtxLock() {
    if (ops_) c_->serve_mu.unlock();
    c_->mu.unlock();
  }
  CtxLock(const CtxLock&) = delete;
  CtxLock& operator=(const CtxLock&) = delete;
 private:
  polfed_ctx* c_;
  bool ops_ = false;
};
}  // namespace polfed

struct polfed_op {
  polfed_ctx* ctx = nullptr;
  polfed::Model model = polfed::Model::Chain;
  int storage = POLFED_MATRIX_FREE;
  int64_t D = 0;
  // chain parameters (host copy) and tables
  int L = 0, N = 0, periodic = 0;
  double t_in = 0, t_pb = 0, vzz = 0, c0 = 0;
  std::vector<double> site_f;  // f_i
  // quantum sun (host copy)
  int N_dot = 0;
  std::vector<double> hdot;
  std::vector<uint32_t> ray_mask;
  std::vector<double> ray_amp;
  // quantum random energy model: transverse field and exact trace moments
  // (sums over the space); the energies are the diagonal d_diag / d_diag32
  double qrem_gamma = 0;
  double qrem_tr[2] = {0, 0};
  // pattern key: operators with equal keys share the off-diagonal pattern
  std::string pattern_key;
  polfed::DevBuf d_ftab, d_ftab32, d_binom, d_hi_off, d_lo_rank, d_hdot;
  // split layout of the chain kernel
  int split_Lb = 0;
  int64_t split_nseg = 0;
  polfed::DevBuf d_blob64, d_blob32, d_blobl64, d_blobl32, d_rec;
  // tile-kernel tables for three tile sizes (bits KT, KT - 1, KT - 2)
  struct Tiles {
    int bits = 0, max_rows = 0, n = 0;
    polfed::DevBuf d;  // [n][4]: first row, rows, first segment, segments
  } tiles[3];
  // host copies of the split layout's block offsets and first segments
  // (2^(L - Lb) + 1 entries each), for building more tile tables
  std::vector<int32_t> split_hi_off, split_seg_of_hi;
  // tables of the staged-tile kernel, per (tile bits, wrap): the non-empty
  // tiles, each [first row, rows, first segment, segments] for its low run
  // and (wrapped tiles) its top run; LDS rows of the largest tile with every
  // run rounded up to whole staging chunks of 128 (FP64) and 256 (FP32) rows
  struct WTiles {
    int kt = 0, wrap = 0, n = 0;
    int buf_rows[2] = {0, 0};
    int rec_slots = 0;  // segment records of the largest tile, runs padded to 8
    polfed::DevBuf d;
  };
  mutable std::map<int, WTiles> wtiles;
  // multi-column step variant per (batch width, precision), by timing
  mutable std::map<int, int> batch_tuned;
  // step-kernel variant picked by timing on first use, per precision
  // (-1: not tuned yet, 0: segment kernel, 1 + i: tile kernel tiles[i])
  mutable int tuned[2] = {-1, -1};
  // POLFED_PRECISION_AUTO resolved for this operator (-1: not timed yet)
  mutable int auto_precision = -1;
  std::vector<double> split_dseg;  // uniform diagonal part of each segment
  std::vector<double> split_fab;   // field sums of low bits 0-4 | 5-9
  polfed::ChainSplitDev chain_split() const;
  // CSR copy
  bool has_csr = false;
  int64_t nnz = -1;
  polfed::DevBuf d_rowptr, d_col, d_val, d_val32, d_diag, d_diag32, d_blk;
  int64_t nblk = 0;
  // optimized mapping (polfed_op_optimize_mapping): value table and codes
  int ncode = 0;
  polfed::DevBuf d_code, d_vtab, d_vtab32;
  polfed::ChainDev chain() const;
  polfed::QsunDev qsun() const;
  polfed::CsrDev csr() const;
};

namespace polfed {

// ------------------------------------------------------------ basis ----
const uint32_t* host_binom();  // host table [kBinomN][kBinomN]
int64_t binom64(int n, int k);
void basis_enumerate(hipStream_t s, int L, int N, int64_t D, uint32_t* states,
                     const uint32_t* d_binom);
void basis_rank(hipStream_t s, int L, int N, const uint32_t* states, int64_t n,
                int64_t* ranks, const uint32_t* d_binom);
void basis_unrank(hipStream_t s, int L, int N, int64_t D, const int64_t* ranks,
                  int64_t n, uint32_t* states, const uint32_t* d_binom);
// Tables for ranking through the split state = hi << Lb | lo.
void build_split_rank_tables(int L, int N, int Lb, std::vector<int32_t>& hi_off,
                             std::vector<int32_t>& lo_rank);

// A batch of chain operators that share the off-diagonal pattern; column i
// of every vector block belongs to ops[i].
struct ChainBatch {
  polfed_ctx* ctx = nullptr;
  std::vector<const polfed_op*> ops;
  int nb = 0;
  DevBuf fab64, fab32;    // [nb][64] low-bit field sums (bits 0-4 | 5-9)
  DevBuf dseg64, dseg32;  // [nseg][nb] uniform diagonal part per segment
  DevBuf sc64, sc32;      // [2][nb] sigma = 2/dE, tau = -2 E_c/dE
  std::vector<double> E_c, dE;  // host copies of each column's rescaling
  void init(polfed_ctx* c, const polfed_op* const* o, int n);
  void set_scale(const double* E_c, const double* dE);
};
// out_c = a_c v_c + h (sigma_c H_c b1_c + tau_c b1_c) - b2_c for every
// column, h = 1/2 on the closing step; acoef: device [nb] (null: no v term);
// blocks are column-major with column stride ld; out may alias b2.
template <typename T>
void chain_batch_step(hipStream_t s, const ChainBatch& bt, int64_t ld, bool final_step,
                      const T* acoef, const T* v, const T* b1, const T* b2, T* out);
// The multi-column step kernel picked by timing for this batch width and
// precision (kept per operator pattern): 0, 1 column-major blocks (16 or 8
// columns per launch), 2, 3 interleaved blocks (element (r, c) at r nb + c;
// 2 or 4 workgroups per compute unit), 4 column-major blocks with every
// column stepped by its operator's own tuned single-column kernel (the
// staged-tile kernels of long chains), 5 the LDS-resident whole filter
// (one workgroup per column; short chains).  Not while the stream is
// captured (returns 0 then, without keeping it).
template <typename T>
int batch_variant(hipStream_t s, const ChainBatch& bt);
// Variant 5: the whole filter of every column in LDS (one workgroup per
// column, a barrier between steps), for short chains.  A: (Kmax + 1) x nb
// coefficients, Kc: device int32 orders; v, w column-major D x nb.
template <typename T>
bool chain_lds_filter_fits(const polfed_op* op0);
template <typename T>
void chain_lds_filter(hipStream_t s, const ChainBatch& bt, const T* A, const int* Kc, const T* v,
                      T* w);
// One step with variant var; v column-major (column stride D) when vcm,
// else in the variant's layout; out column-major when ocm.
template <typename T>
void chain_batch_step_var(hipStream_t s, const ChainBatch& bt, int var, bool final_step,
                          const T* acoef, const T* v, bool vcm, const T* b1, const T* b2,
                          T* out, bool ocm);

// ----------------------------------------------------------- operators ----
// Fused Clenshaw step for every operator kind and precision:
//   out = a * v + sigma * (H b1) + tau * b1 - (b2 ? b2 : 0)
// v may be null (a ignored); out may alias b2.
template <typename T>
void op_step(hipStream_t s, const polfed_op* op, T sigma, T tau, T a,
             const T* v, const T* b1, const T* b2, T* out);
// Runs the step-kernel tuner of a matrix-free chain or QREM operator for one
// precision (one eager step on scratch vectors, on s) if it has not run yet.
// The tuners time launches and cannot run inside a stream capture, so every
// caller that records the recurrence into a graph calls this first.
void op_tune(hipStream_t s, const polfed_op* op, bool fp32);
void op_moments(hipStream_t s, const polfed_op* op, double* d_two, double* partial,
                int64_t npart);
// Split-layout chain step; false when no instantiation covers op->L.
template <typename T>
bool chain_split_step(hipStream_t s, const polfed_op* op, T sigma, T tau, T a,
                      const T* v, const T* b1, const T* b2, T* out);
void build_chain_split(polfed_op* op);
// Whether staged-tile variant var of the chain step exists for op at this
// precision (chain length, tile table and LDS footprint).
bool chain_wt_exists(const polfed_op* op, int var, bool fp32);
constexpr int kChainVariants = 10;  // variants 0 .. 9
// Fused Clenshaw step of the quantum random energy model (hypercube stencil).
template <typename T>
void qrem_step(hipStream_t s, const polfed_op* op, T sigma, T tau, T a, const T* v, const T* b1,
               const T* b2, T* out);
int qrem_tile_bits(int L);
// The step for n columns of one QREM operator (blocks of column stride D);
// every column equals the single-column step's result.  L >= 10.
template <typename T>
void qrem_step_multi(hipStream_t s, const polfed_op* op, int n, T sigma, T tau, T a, const T* v,
                     const T* b1, const T* b2, T* out);
void materialize_csr(polfed_ctx* ctx, polfed_op* op);

// ---------------------------------------------------------------- blas ----
int64_t red_blocks(int64_t n);
void dev_dot(hipStream_t s, int64_t n, const double* x, const double* y,
             double* partial, int64_t npart, double* out, int sqrt_out);
void dev_gemv_t(hipStream_t s, int64_t D, int k, const double* V, int64_t ld,
                const double* w, double* partial, int64_t nseg, double* c,
                double* tail, int tail_add);
void dev_gemv_n_sub(hipStream_t s, int64_t D, int k, const double* V, int64_t ld,
                    const double* c, double* w);
void dev_scale_into(hipStream_t s, int64_t D, const double* w,
                    const double* beta, double* out, int* flag);
void dev_axpby(hipStream_t s, int64_t n, double a, const double* x, double b,
               double* y);
void dev_copy_d2f(hipStream_t s, int64_t n, const double* x, float* y);
void dev_copy_f2d(hipStream_t s, int64_t n, const float* x, double* y);
void dev_fill(hipStream_t s, int64_t n, double v, double* y);
void dev_fillf(hipStream_t s, int64_t n, float v, float* y);
void dev_random(hipStream_t s, int64_t n, uint64_t seed, double* y);
// Blocks of at least this many columns take the MFMA products.
constexpr int kMfmaMinCols = 16;
// One block Gram-Schmidt pass: C = V^T W (k x n, ld k), W -= V C, for the
// D x n block W against the first k columns of V (ld D): the vector-unit
// tall-skinny kernels (8 columns per pass, V read once per product) below
// kMfmaMinCols columns, the MFMA products from there on.
// partial: nseg * k * 8.
void dev_block_gs_pass(hipStream_t s, int64_t D, int k, const double* V, double* W, int n,
                       double* partial, int64_t nseg, double* C);
// u_j = V t_j for the n columns of T, Rayleigh-Ritz with H on their span
// (E ascending, U2 = U Z, residual norms); device inputs and outputs.
void extract_pairs(polfed_ctx* ctx, const polfed_op* op, const double* V, int m,
                   const double* T, int n, double* E, double* U2, double* resid);
// MFMA products of tall matrices (gemm.hip).  C (D x n, ldc) = A (D x m,
// lda) B (m x n, ldb), or C -= A B with sub.
void dev_gemm_nn(hipStream_t s, int64_t D, int m, int n, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc, bool sub);
// G (n1 x n2, ldg) = A^T B, A: D x n1 (lda), B: D x n2 (ldb); allocates its
// split-sum workspace of gemm_tn_workspace(D, n1, n2) bytes.
void dev_gemm_tn(hipStream_t s, int64_t D, int n1, int n2, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* G, int64_t ldg);
int gemm_tn_splits(int64_t D, int n1, int n2);
size_t gemm_tn_workspace(int64_t D, int n1, int n2);
// res[j] = || HU[:, j] - E[j] U[:, j] ||
void dev_resid(hipStream_t s, int64_t D, int n, const double* U,
               const double* HU, const double* E, double* partial, int64_t nseg,
               double* res);

// ------------------------------------------------------- host eigen ----
}  // namespace polfed
#include "eig.hpp"
namespace polfed {

// ----------------------------------------------------------------- kpm ----
// mu[0..N) = mean over R vectors of <r|T_n(H~)|r>; rvecs: device D x R, or
// null for vectors drawn from the counter-based generator of dev_random
// (vector c with seed + c), scaled to unit variance.
void kpm_moments(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE, int N, int R,
                 const double* rvecs, uint64_t seed, double* mu);
void kpm_density(const double* mu, int N, const double* x, int nx, double* rho);
// argmax of the KPM density over the Chebyshev nodes of 4096 that lie in [lo, hi]
double kpm_maxdos(const double* mu, int N, double lo, double hi);
constexpr uint64_t kKpmSeed = 0x4B504DULL;  // random vectors of the KPM DOS of a solve

// ---------------------------------------------------------------- plan ----
double filter_value_closed(double lambda_t, int K, double x);
void filter_coefficients(double lambda_t, int K, double* a);
void filter_quotient(const double* a, int K, double theta, double* q, double* p_theta);
polfed_plan make_plan(int64_t D, double E_min, double E_max, double pad,
                      double lambda, double tr1, double tr2, int n_window,
                      double omega, int K_override, const double* kpm_mu = nullptr,
                      int kpm_n = 0);
constexpr double kOmegaDefault = 0.17612720216036546;  // sin(2.655)/2.655
int expected_krylov_dim(int howmany, int blocksize, double eta);

// ---------------------------------------------------------------- solve ----
// as filter_apply, on an explicit stream (graph capture)
template <typename T>
void filter_apply_on(hipStream_t s, const polfed_op* op, double E_c, double dE,
                     const double* a, int K, const T* v, T* w, T* bufA, T* bufB);
template <typename T>
void filter_apply(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE,
                  const double* a, int K, const T* v, T* w, T* bufA, T* bufB);
void bounds(polfed_ctx* ctx, const polfed_op* op, const double* x0, double tol,
            int max_iter, double* E_min, double* E_max, int* iters);
polfed_status solve(polfed_ctx* ctx, const polfed_op* op, const polfed_params& p,
                    const double* x0, double* evals, double* evecs,
                    double* resid, int* n_found, polfed_report* rep);
polfed_status solve_batch(polfed_ctx* ctx, int B, const polfed_op* const* ops,
                          const polfed_params& p, const double* const* x0,
                          double* const* evals, double* const* evecs,
                          double* const* resid, int* n_found,
                          polfed_report* rep);
double now_seconds();
bool verbose();  // POLFED_VERBOSE set: solver diagnostics on stderr
// A tuner's choice `what` for the operator's chain pattern on its context
// (-1: none yet, or the operator has no pattern), and its record.
int pattern_choice(const polfed_op* op, const std::string& what);
void pattern_choice_set(const polfed_op* op, const std::string& what, int v);
void* ctx_scratch(polfed_ctx* ctx, int slot, size_t bytes);
void lanczos_step(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE,
                  const double* a, int K, double* V, int k, double* alpha,
                  double* beta, int precision);
void block_lanczos_step(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE,
                        const double* a, int K, double* V, int k, int s, double* A,
                        double* Bn, int precision);
// POLFED_PRECISION_AUTO: FP32 when the operator's FP32 Clenshaw step runs in
// under 0.7 of the FP64 step's time, else FP64; timed once per operator, or
// per off-diagonal pattern and storage for chains, and kept.  Any other
// precision is returned unchanged.  Synchronizes s when it times.
int resolve_precision(hipStream_t s, const polfed_op* op, int precision);
void profile_step(polfed_ctx* ctx, const polfed_op* op, int precision, int iters,
                  double* avg_ms, double* min_ms);

}  // namespace polfed

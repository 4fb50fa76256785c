// extern "C" entry points of polfed.h: argument checks, error capture and
// dispatch to the library internals.  No exception crosses this boundary.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "internal.hpp"
#include "solve_run.hpp"

namespace polfed {

polfed_op* make_xxz(polfed_ctx*, int, int, double, double, const double*, int);
polfed_op* make_tv(polfed_ctx*, int, int, double, double, const double*, int);
polfed_op* make_qsun(polfed_ctx*, int, int, const double*, double, double, double,
                     const double*, const int32_t*, const double*);
polfed_op* make_csr(polfed_ctx*, int64_t, const int64_t*, const int32_t*, const double*);
polfed_op* make_qrem(polfed_ctx*, int, const double*, double);
polfed_op* make_spin_chain(polfed_ctx*, int, int, int, const double*, const double*,
                           const double*, int);
int optimize_mapping(polfed_ctx*, polfed_op*);
polfed_status serve_start(polfed_ctx*, size_t, int);
polfed_status serve_submit(polfed_ctx*, const polfed_op*, const polfed_params*,
                           const double*, double*, double*, double*, polfed_req**);
polfed_status req_poll(polfed_req*, int*);
polfed_status req_wait(polfed_req*, int*, polfed_report*);
polfed_status req_destroy(polfed_req*);
polfed_status serve_stop(polfed_ctx*);

namespace {
thread_local std::string g_err;
}

[[noreturn]] void fail(polfed_status code, const std::string& msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  const char* base = std::strrchr(file, '/');
  std::string m = std::string(what) + " failed: " + hipGetErrorString(e) + " (" +
                  (base ? base + 1 : file) + ":" + std::to_string(line) + ")";
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    throw Error(POLFED_ERR_OOM, m);
  throw Error(POLFED_ERR_HIP, m);
}

thread_local MemTally* g_mem_tally = nullptr;
thread_local bool g_no_capture = false;

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) HIPC(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// ------------------------------------------------------ device memory ----
// hipFree waits until everything queued on the device has finished, so a
// buffer released in the middle of other streams' work (a server round, a
// retiring request) would stall all of them.  Released blocks are therefore
// kept per device and handed out again once the device has passed the
// release: at release an event is recorded on every stream the library
// queues work on, and a cached block is reused only when all its events have
// completed.  Blocks go back to hipFree only when the cache would exceed its
// cap, or to make room when an allocation fails.  Sizes are rounded to
// buckets (powers of two up to 1 MiB, then 2 MiB multiples) so that blocks
// of a repeating workload fit each other.
namespace {
// A fence event and the stream it was recorded on.  Events never outlive
// their stream: when a stream is unregistered (after its work has drained,
// before it is destroyed), the events recorded on it are destroyed.
struct Fence {
  hipStream_t s;
  hipEvent_t e;
};
struct CachedBlock {
  void* p;
  std::vector<Fence> fence;
};
struct DevicePool {
  std::mutex mu;
  std::vector<hipStream_t> streams;  // work streams (one entry per registration)
  std::multimap<size_t, CachedBlock> blocks;  // by bucket size
  std::vector<Fence> spare;                  // events of reused blocks (s: last stream)
  size_t cached = 0, cap = 0;
};

DevicePool& device_pool(int dev) {
  static std::mutex m;
  // never destroyed: blocks cached at exit are returned with the process
  static auto* pools = new std::map<int, DevicePool*>();
  std::lock_guard<std::mutex> lk(m);
  DevicePool*& p = (*pools)[dev];
  if (!p) {
    p = new DevicePool();
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      tot = (size_t)16 << 30;
    }
    p->cap = std::min<size_t>(tot / 8, (size_t)32 << 30);
  }
  return *p;
}

size_t bucket_of(size_t b) {
  if (b <= 256) return 256;
  if (b <= ((size_t)1 << 20)) {
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t g = (size_t)2 << 20;
  return (b + g - 1) / g * g;
}

// Makes dev current for the scope without throwing (release paths run in
// destructors).
struct QuietDevice {
  int prev = -1;
  explicit QuietDevice(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
    (void)hipGetLastError();
  }
  ~QuietDevice() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

bool fence_passed(const CachedBlock& c) {
  for (const Fence& f : c.fence) {
    const hipError_t q = hipEventQuery(f.e);
    if (q == hipSuccess) continue;
    (void)hipGetLastError();  // a pending event is no error of a later call
    return false;
  }
  return true;
}

// Frees every cached block once its fence has passed (pool lock held).  No
// device-wide synchronization: on another thread, that would invalidate a
// graph capture in progress (and fail itself).
void flush_pool(DevicePool& P) {
  for (auto& kv : P.blocks) {
    for (const Fence& f : kv.second.fence) {
      (void)hipEventSynchronize(f.e);
      P.spare.push_back(f);
    }
    (void)hipFree(kv.second.p);
  }
  P.blocks.clear();
  P.cached = 0;
  (void)hipGetLastError();
}
}  // namespace

void register_stream(int dev, hipStream_t s) {
  QuietDevice g(dev);
  DevicePool& P = device_pool(dev);
  std::lock_guard<std::mutex> lk(P.mu);
  P.streams.push_back(s);
}

void unregister_stream(int dev, hipStream_t s) {
  QuietDevice g(dev);
  DevicePool& P = device_pool(dev);
  std::lock_guard<std::mutex> lk(P.mu);
  auto it = std::find(P.streams.begin(), P.streams.end(), s);
  if (it != P.streams.end()) P.streams.erase(it);
  if (std::find(P.streams.begin(), P.streams.end(), s) == P.streams.end()) {
    // the stream's work has drained (callers synchronize it first): its
    // fence events have completed and are destroyed while it still exists
    for (auto& kv : P.blocks) {
      auto& fv = kv.second.fence;
      for (const Fence& f : fv)
        if (f.s == s) (void)hipEventDestroy(f.e);
      fv.erase(std::remove_if(fv.begin(), fv.end(), [&](const Fence& f) { return f.s == s; }),
               fv.end());
    }
    for (const Fence& f : P.spare)
      if (f.s == s) (void)hipEventDestroy(f.e);
    P.spare.erase(std::remove_if(P.spare.begin(), P.spare.end(),
                                 [&](const Fence& f) { return f.s == s; }),
                  P.spare.end());
    (void)hipGetLastError();
  }
  // the last stream gone: nothing of the library runs on the device any
  // more, so the cached blocks go back to the device
  if (P.streams.empty()) flush_pool(P);
}

void DevBuf::alloc(size_t bytes) {
  release();
  if (bytes == 0) bytes = 16;
  const size_t cap = bucket_of(bytes);
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  DevicePool& P = device_pool(dev);
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(P.mu);
    auto range = P.blocks.equal_range(cap);
    for (auto it = range.first; it != range.second; ++it)
      if (fence_passed(it->second)) {
        p = it->second.p;
        for (const Fence& f : it->second.fence) P.spare.push_back(f);
        P.blocks.erase(it);
        P.cached -= cap;
        break;
      }
  }
  if (!p) {
    hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      {
        std::lock_guard<std::mutex> lk(P.mu);
        flush_pool(P);
      }
      e = hipMalloc(&p, cap);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(POLFED_ERR_OOM, "device allocation of " + std::to_string(bytes) +
                                      " bytes failed: " + hipGetErrorString(e));
    }
  }
  p_ = p;
  n_ = bytes;
  cap_ = cap;
  dev_ = dev;
  t_ = g_mem_tally;
  if (t_) {
    t_->cur += bytes;
    t_->peak = std::max(t_->peak, t_->cur);
  }
}

void DevBuf::release() {
  if (p_) {
    if (t_) t_->cur -= n_;
    QuietDevice g(dev_);
    DevicePool& P = device_pool(dev_);
    bool cached = false;
    {
      std::lock_guard<std::mutex> lk(P.mu);
      if (P.cached + cap_ <= P.cap) {
        CachedBlock c{p_, {}};
        bool ok = true;
        std::vector<hipStream_t> seen;
        for (hipStream_t s : P.streams) {
          if (std::find(seen.begin(), seen.end(), s) != seen.end()) continue;
          seen.push_back(s);
          // a stream being captured takes no event: its work is a graph
          // that can run later, so the block goes back to hipFree
          hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
          if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
            (void)hipGetLastError();
            ok = false;
            break;
          }
          hipEvent_t e = nullptr;
          if (!P.spare.empty()) {
            e = P.spare.back().e;
            P.spare.pop_back();
          } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            ok = false;
            break;
          }
          c.fence.push_back({s, e});
          if (hipEventRecord(e, s) != hipSuccess) {
            (void)hipGetLastError();
            ok = false;
            break;
          }
        }
        if (ok) {
          P.blocks.emplace(cap_, std::move(c));
          P.cached += cap_;
          cached = true;
        } else {
          for (const Fence& f : c.fence) P.spare.push_back(f);
        }
      }
    }
    if (!cached) (void)hipFree(p_);
  }
  p_ = nullptr;
  n_ = 0;
  cap_ = 0;
  t_ = nullptr;
}

void GraphExec::reset() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  exec_ = nullptr;
}

void GraphExec::begin(hipStream_t cap) {
  REQUIRE(!g_no_capture, "graph capture on a thread that captures no graphs (a server thread)");
  HIPC(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
}

void GraphExec::end(hipStream_t cap) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamEndCapture(cap, &g));
  const hipError_t e = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) exec_ = nullptr;
  HIPC(e);
}

void GraphExec::abort(hipStream_t cap) {
  hipGraph_t g = nullptr;
  (void)hipStreamEndCapture(cap, &g);
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}

void GraphExec::launch(hipStream_t s) {
  REQUIRE(exec_ != nullptr, "graph not captured");
  HIPC(hipGraphLaunch(exec_, s));
}

template <class F>
polfed_status guarded(F&& f) {
  try {
    g_err.clear();
    // hipGetLastError is per-thread state that any earlier HIP call of the
    // caller (another library, the framework) may have left set; the launch
    // checks inside this call must only see errors of this call
    (void)hipGetLastError();
    return f();
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return POLFED_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return POLFED_ERR_INVALID;
  } catch (...) {
    g_err = "unknown error";
    return POLFED_ERR_INVALID;
  }
}


}  // namespace polfed

using namespace polfed;

#define CTX_OK(ctx) REQUIRE((ctx) != nullptr, "null context")

extern "C" {

int polfed_version(void) { return 10100; }

const char* polfed_last_error(void) { return g_err.c_str(); }

// ----------------------------------------- allocation-free filter scratch
//
// The two recurrence buffers of polfed_filter_apply_noalloc live in this
// file-scope device array.  In host code its name is only a host-side stand-in:
// the device address is looked up once per device, with that device current,
// when a context is created on it, and only that address is ever passed to
// kernels and copies.  Every call on a device shares the device's array.
constexpr size_t kNoAllocScratchBytes = (size_t)48 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of the scratch array on the current device (device).
void* resolve_scratch(int device) {
  REQUIRE(device >= 0 && device < kMaxDevices, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    HIPC(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    REQUIRE(ptr != nullptr, "no device address for the filter scratch array");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}
}  // namespace

polfed_status polfed_create(int device, void* hip_stream, polfed_ctx** out) {
  return guarded([&]() -> polfed_status {
    REQUIRE(out != nullptr, "null output handle");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
      (void)hipGetLastError();
      fail(POLFED_ERR_NODEVICE, "no HIP device visible");
    }
    REQUIRE(device >= 0 && device < n, "device index out of range");
    DeviceGuard g(device);
    auto ctx = std::make_unique<polfed_ctx>();
    ctx->device = device;
    // NULL: ordered with the device's null stream (torch's default stream)
    // through a blocking stream of the context's own; work queued on the
    // null stream itself while another thread captures a graph can
    // invalidate that capture
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    if (!ctx->stream) {
      HIPC(hipStreamCreateWithFlags(&ctx->stream, hipStreamDefault));
      ctx->own_stream = true;
    }
    HIPC(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    register_stream(device, ctx->stream);
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, device));
    ctx->n_cu = prop.multiProcessorCount;
    (void)resolve_scratch(device);  // device is current here
    *out = ctx.release();
    return POLFED_OK;
  });
}

polfed_status polfed_destroy(polfed_ctx* ctx) {
  return guarded([&]() -> polfed_status {
    if (!ctx) return POLFED_OK;
    if (ctx->server) (void)serve_stop(ctx);
    {
      DeviceGuard g(ctx->device);
      (void)hipStreamSynchronize(ctx->stream);
      ctx->scratch_red.release();
      ctx->scratch_scalar.release();
      ctx->binom.release();
      for (auto& b : ctx->ws) b.release();
      unregister_stream(ctx->device, ctx->stream);
      if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
      if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    }
    delete ctx;
    return POLFED_OK;
  });
}

polfed_status polfed_sync(polfed_ctx* ctx) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    DeviceGuard g(ctx->device);
    HIPC(hipStreamSynchronize(ctx->stream));
    return POLFED_OK;
  });
}

// ---------------------------------------------------------------- basis

polfed_status polfed_basis_dim(int L, int N, int64_t* D) {
  return guarded([&]() -> polfed_status {
    REQUIRE(D != nullptr, "null output");
    REQUIRE(L >= 1 && L <= 32 && N >= 0 && N <= L, "need 1 <= L <= 32, 0 <= N <= L");
    *D = binom64(L, N);
    return POLFED_OK;
  });
}

namespace {
const uint32_t* ctx_binom(polfed_ctx* ctx) {
  if (!ctx->binom.get()) {
    upload(ctx->binom, host_binom(), (size_t)kBinomN * kBinomN, ctx->stream);
    HIPC(hipStreamSynchronize(ctx->stream));
  }
  return ctx->binom.as<uint32_t>();
}
}  // namespace

polfed_status polfed_basis_enumerate(polfed_ctx* ctx, int L, int N, uint32_t* states) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(L >= 1 && L <= 32 && N >= 0 && N <= L, "need 1 <= L <= 32, 0 <= N <= L");
    const int64_t D = binom64(L, N);
    REQUIRE(D < (int64_t(1) << 31), "sector too large");
    REQUIRE(states != nullptr || D == 0, "null states");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    basis_enumerate(ctx->stream, L, N, D, states, ctx_binom(ctx));
    return POLFED_OK;
  });
}

polfed_status polfed_basis_rank(polfed_ctx* ctx, int L, int N, const uint32_t* states,
                                int64_t n, int64_t* ranks) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(L >= 1 && L <= 32 && N >= 0 && N <= L, "need 1 <= L <= 32, 0 <= N <= L");
    REQUIRE(n >= 0, "negative count");
    REQUIRE(n == 0 || (states && ranks), "null array");
    REQUIRE(binom64(L, N) < (int64_t(1) << 31), "sector too large");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    basis_rank(ctx->stream, L, N, states, n, ranks, ctx_binom(ctx));
    return POLFED_OK;
  });
}

polfed_status polfed_basis_unrank(polfed_ctx* ctx, int L, int N, const int64_t* ranks,
                                  int64_t n, uint32_t* states) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(L >= 1 && L <= 32 && N >= 0 && N <= L, "need 1 <= L <= 32, 0 <= N <= L");
    REQUIRE(n >= 0, "negative count");
    REQUIRE(n == 0 || (states && ranks), "null array");
    const int64_t D = binom64(L, N);
    REQUIRE(D < (int64_t(1) << 31), "sector too large");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    basis_unrank(ctx->stream, L, N, D, ranks, n, states, ctx_binom(ctx));
    return POLFED_OK;
  });
}

// ------------------------------------------------------------ operators

polfed_status polfed_op_xxz(polfed_ctx* ctx, int L, int n_up, double J, double Delta,
                            const double* h, int periodic, polfed_op** out) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(out, "null output handle");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    *out = make_xxz(ctx, L, n_up, J, Delta, h, periodic);
    return POLFED_OK;
  });
}

polfed_status polfed_op_tv(polfed_ctx* ctx, int L, int n_part, double t, double V,
                           const double* eps, int periodic, polfed_op** out) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(out, "null output handle");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    *out = make_tv(ctx, L, n_part, t, V, eps, periodic);
    return POLFED_OK;
  });
}

polfed_status polfed_op_qsun(polfed_ctx* ctx, int N_dot, int L, const double* A,
                             double gamma, double g0, double alpha, const double* u,
                             const int32_t* n_of_j, const double* h, polfed_op** out) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(out, "null output handle");
    *out = nullptr;
    REQUIRE(std::isfinite(gamma) && std::isfinite(g0) && std::isfinite(alpha) && alpha > 0,
            "qsun: need finite gamma, g0 and alpha > 0");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    *out = make_qsun(ctx, N_dot, L, A, gamma, g0, alpha, u, n_of_j, h);
    return POLFED_OK;
  });
}

polfed_status polfed_op_qrem(polfed_ctx* ctx, int L, const double* E, double Gamma,
                             polfed_op** out) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(out, "null output handle");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    *out = make_qrem(ctx, L, E, Gamma);
    return POLFED_OK;
  });
}

polfed_status polfed_op_spin_chain(polfed_ctx* ctx, int L, int N, int R, const double* J,
                                   const double* Delta, const double* h, int periodic,
                                   polfed_op** out) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(out, "null output handle");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    *out = make_spin_chain(ctx, L, N, R, J, Delta, h, periodic);
    return POLFED_OK;
  });
}

polfed_status polfed_op_optimize_mapping(polfed_ctx* ctx, polfed_op* op, int* n_values) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    const int n = optimize_mapping(ctx, op);
    if (n_values) *n_values = n;
    return POLFED_OK;
  });
}

polfed_status polfed_op_csr(polfed_ctx* ctx, int64_t D, const int64_t* rowptr,
                            const int32_t* col, const double* val, polfed_op** out) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(out, "null output handle");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    *out = make_csr(ctx, D, rowptr, col, val);
    return POLFED_OK;
  });
}

polfed_status polfed_op_materialize_csr(polfed_ctx* ctx, polfed_op* op) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    materialize_csr(ctx, op);
    return POLFED_OK;
  });
}

polfed_status polfed_op_set_storage(polfed_op* op, int storage) {
  return guarded([&]() -> polfed_status {
    REQUIRE(op, "null operator");
    if (storage == POLFED_CSR) {
      REQUIRE(op->has_csr, "operator has no CSR copy (call polfed_op_materialize_csr)");
    } else {
      REQUIRE(storage == POLFED_MATRIX_FREE, "unknown storage");
      REQUIRE(op->model != Model::Csr, "CSR operator has no matrix-free form");
    }
    op->storage = storage;
    return POLFED_OK;
  });
}

polfed_status polfed_op_set_kernel(polfed_op* op, int precision, int variant, int* chosen) {
  return guarded([&]() -> polfed_status {
    REQUIRE(op, "null operator");
    REQUIRE(precision == POLFED_FP64 || precision == POLFED_FP32, "unknown precision");
    const int pi = precision == POLFED_FP64 ? 0 : 1;
    if (variant == -2) {  // query only
      if (chosen) *chosen = op->tuned[pi];
      return POLFED_OK;
    }
    if (op->model == Model::Qrem) {
      REQUIRE(variant == -1 || (variant >= 1 && variant <= std::min(op->L, 12)),
              "qrem: tile bits must be -1 or 1 .. min(L, 12)");
      op->tuned[pi] = variant;
      if (chosen) *chosen = op->tuned[pi];
      return POLFED_OK;
    }
    REQUIRE(variant >= -1 && variant < kChainVariants,
            "variant must be -2 .. " + std::to_string(kChainVariants - 1));
    if (variant > 0) {
      REQUIRE(op->model == Model::Chain && op->split_nseg > 0,
              "step-kernel variants exist only for matrix-free chains");
      if (variant <= 2 || variant == 5)
        REQUIRE(op->tiles[variant == 5 ? 2 : variant - 1].n > 0,
                "no tile kernel of this size for this chain length");
      if (variant >= 6)
        REQUIRE(chain_wt_exists(op, variant, pi == 1),
                "no staged-tile kernel of this shape for this chain length and precision");
    }
    op->tuned[pi] = variant;
    if (chosen) *chosen = op->tuned[pi];
    return POLFED_OK;
  });
}

polfed_status polfed_op_set_batch_kernel(polfed_op* op, int B, int precision, int variant,
                                         int* chosen) {
  return guarded([&]() -> polfed_status {
    REQUIRE(op, "null operator");
    REQUIRE(op->model == Model::Chain && op->split_nseg > 0 && !op->pattern_key.empty(),
            "multi-column kernels exist only for matrix-free chains");
    REQUIRE(B >= 1, "need B >= 1");
    REQUIRE(precision == POLFED_FP64 || precision == POLFED_FP32, "unknown precision");
    REQUIRE(variant >= -2 && variant < 8, "variant must be -2 .. 7");
    if (variant == 4) REQUIRE(op->L >= 22, "variant 4 needs a chain of L >= 22");
    if (variant == 5)
      REQUIRE(precision == POLFED_FP64 ? chain_lds_filter_fits<double>(op)
                                       : chain_lds_filter_fits<float>(op),
              "variant 5: two vectors of this chain do not fit the LDS");
    const int key = B * 2 + (precision == POLFED_FP64 ? 0 : 1);
    if (variant == -1) op->batch_tuned.erase(key);
    if (variant >= 0) {
      if (variant >= 2)
        REQUIRE((uint64_t)op->D * (uint64_t)B * (precision == POLFED_FP64 ? 8 : 4) <
                    (uint64_t(1) << 32) - 64,
                "interleaved blocks of this size exceed 4 GiB");
      if (variant >= 6) {
        const int groups = (int)(((size_t)B * (precision == POLFED_FP64 ? 8 : 4) + 15) / 16);
        REQUIRE(groups <= 16, "variants 6 and 7: at most 16 lanes per row (32 FP64 or 64 FP32 "
                              "columns)");
      }
      op->batch_tuned[key] = variant;
    }
    if (chosen) {
      const auto it = op->batch_tuned.find(key);
      *chosen = it == op->batch_tuned.end() ? -1 : it->second;
    }
    return POLFED_OK;
  });
}

polfed_status polfed_op_dim(const polfed_op* op, int64_t* D) {
  return guarded([&]() -> polfed_status {
    REQUIRE(op && D, "null argument");
    *D = op->D;
    return POLFED_OK;
  });
}

polfed_status polfed_op_nnz(const polfed_op* op, int64_t* nnz) {
  return guarded([&]() -> polfed_status {
    REQUIRE(op && nnz, "null argument");
    *nnz = op->has_csr ? op->nnz : -1;
    return POLFED_OK;
  });
}

polfed_status polfed_op_export_csr(polfed_ctx* ctx, const polfed_op* op, int64_t* rowptr,
                                   int32_t* col, double* val, double* diag) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    REQUIRE(op->has_csr, "operator has no CSR copy");
    REQUIRE(rowptr && diag && (op->nnz == 0 || (col && val)), "null buffer");
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    HIPC(hipMemcpyAsync(rowptr, op->d_rowptr.get(), (op->D + 1) * sizeof(int64_t),
                        hipMemcpyDeviceToDevice, s));
    if (op->nnz) {
      HIPC(hipMemcpyAsync(col, op->d_col.get(), op->nnz * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
      HIPC(hipMemcpyAsync(val, op->d_val.get(), op->nnz * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    }
    if (op->D)
      HIPC(hipMemcpyAsync(diag, op->d_diag.get(), op->D * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    return POLFED_OK;
  });
}

polfed_status polfed_op_destroy(polfed_op* op) {
  return guarded([&]() -> polfed_status {
    if (!op) return POLFED_OK;
    DeviceGuard g(op->ctx->device);
    (void)hipStreamSynchronize(op->ctx->stream);
    delete op;
    return POLFED_OK;
  });
}

polfed_status polfed_op_apply(polfed_ctx* ctx, const polfed_op* op, const double* x,
                              double* y) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    REQUIRE(op->D == 0 || (x && y), "null vector");
    REQUIRE(x != y, "x and y must not overlap");
    DeviceGuard g(ctx->device);
    op_step<double>(ctx->stream, op, 1.0, 0.0, 0.0, nullptr, x, nullptr, y);
    return POLFED_OK;
  });
}

polfed_status polfed_op_moments(polfed_ctx* ctx, const polfed_op* op, double* tr1,
                                double* tr2) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    REQUIRE(tr1 && tr2, "null output");
    REQUIRE(op->D >= 1, "empty operator");
    DeviceGuard g(ctx->device);
    DevBuf two(2 * sizeof(double)), part(2 * 4096 * sizeof(double));
    op_moments(ctx->stream, op, two.as<double>(), part.as<double>(), 4096);
    double t[2];
    HIPC(hipMemcpyAsync(t, two.get(), sizeof t, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    *tr1 = t[0] / (double)op->D;
    *tr2 = t[1] / (double)op->D;
    return POLFED_OK;
  });
}

// ------------------------------------------------------------- filter

polfed_status polfed_make_plan(int64_t D, double E_min, double E_max, double pad,
                               double lambda, double tr1, double tr2, int n_window,
                               double omega, int K_override, polfed_plan* out) {
  return guarded([&]() -> polfed_status {
    REQUIRE(out, "null output");
    *out = make_plan(D, E_min, E_max, pad, lambda, tr1, tr2, n_window, omega, K_override);
    return POLFED_OK;
  });
}

polfed_status polfed_filter_coefficients(double lambda_t, int K, double* a) {
  return guarded([&]() -> polfed_status {
    REQUIRE(a, "null output");
    REQUIRE(K >= 0, "K must be >= 0");
    REQUIRE(lambda_t >= -1.0 && lambda_t <= 1.0, "lambda~ must lie in [-1, 1]");
    filter_coefficients(lambda_t, K, a);
    return POLFED_OK;
  });
}

polfed_status polfed_filter_quotient(const double* a, int K, double theta, double* q,
                                     double* p_theta) {
  return guarded([&]() -> polfed_status {
    REQUIRE(K >= 0 && a && (K == 0 || q), "need K >= 0, a[K+1] and q[K]");
    REQUIRE(std::isfinite(theta), "theta must be finite");
    filter_quotient(a, K, theta, q, p_theta);
    return POLFED_OK;
  });
}

polfed_status polfed_filter_value(double lambda_t, int K, const double* x, int64_t n,
                                  double* out) {
  return guarded([&]() -> polfed_status {
    REQUIRE(n >= 0 && (n == 0 || (x && out)), "null array");
    REQUIRE(K >= 0, "K must be >= 0");
    REQUIRE(lambda_t >= -1.0 && lambda_t <= 1.0, "lambda~ must lie in [-1, 1]");
    for (int64_t i = 0; i < n; ++i) out[i] = filter_value_closed(lambda_t, K, x[i]);
    return POLFED_OK;
  });
}

static void check_step_args(polfed_ctx* ctx, const polfed_op* op, double dE, int precision) {
  CTX_OK(ctx);
  REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
  REQUIRE(precision == POLFED_FP64 || precision == POLFED_FP32, "unknown precision");
  REQUIRE(std::isfinite(dE) && dE > 0, "dE must be finite and positive");
}

polfed_status polfed_filter_apply(polfed_ctx* ctx, const polfed_op* op, double E_c,
                                  double dE, const double* a, int K, const void* v, void* w,
                                  int precision) {
  return guarded([&]() -> polfed_status {
    check_step_args(ctx, op, dE, precision);
    REQUIRE(std::isfinite(E_c), "E_c must be finite");
    REQUIRE(K >= 0 && a, "need K >= 0 and coefficients a[K+1]");
    REQUIRE(op->D == 0 || (v && w), "null vector");
    REQUIRE(v != w, "v and w must not overlap");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    const int64_t D = op->D;
    if (precision == POLFED_FP64) {
      DevBuf A(std::max<int64_t>(D, 1) * sizeof(double)), Bb(std::max<int64_t>(D, 1) * sizeof(double));
      filter_apply<double>(ctx, op, E_c, dE, a, K, static_cast<const double*>(v),
                           static_cast<double*>(w), A.as<double>(), Bb.as<double>());
      HIPC(hipStreamSynchronize(ctx->stream));
    } else {
      DevBuf A(std::max<int64_t>(D, 1) * sizeof(float)), Bb(std::max<int64_t>(D, 1) * sizeof(float));
      filter_apply<float>(ctx, op, E_c, dE, a, K, static_cast<const float*>(v),
                          static_cast<float*>(w), A.as<float>(), Bb.as<float>());
      HIPC(hipStreamSynchronize(ctx->stream));
    }
    return POLFED_OK;
  });
}

polfed_status polfed_filter_apply_noalloc(polfed_ctx* ctx, const polfed_op* op, double E_c,
                                          double dE, const double* a, int K, const void* v,
                                          void* w, int precision) {
  return guarded([&]() -> polfed_status {
    check_step_args(ctx, op, dE, precision);
    REQUIRE(std::isfinite(E_c), "E_c must be finite");
    REQUIRE(K >= 0 && a, "need K >= 0 and coefficients a[K+1]");
    REQUIRE(op->D == 0 || (v && w), "null vector");
    REQUIRE(v != w, "v and w must not overlap");
    const int64_t D = op->D;
    const size_t tb = precision == POLFED_FP64 ? sizeof(double) : sizeof(float);
    if ((size_t)std::max<int64_t>(D, 1) * tb > kNoAllocScratchBytes / 2)
      fail(POLFED_ERR_INVALID,
           "filter_apply_noalloc: the two recurrence vectors of D = " + std::to_string(D) +
               " rows need " + std::to_string(2 * (size_t)D * tb) +
               " bytes, more than the " + std::to_string(kNoAllocScratchBytes) +
               "-byte scratch array");
    // the step kernel must be chosen already: its timing allocates
    const int pi = precision == POLFED_FP64 ? 0 : 1;
    if (op->storage != POLFED_CSR &&
        ((op->model == Model::Chain && op->split_nseg > 0 && op->tuned[pi] < 0) ||
         (op->model == Model::Qrem && op->L >= 12 && op->tuned[pi] < 1)))
      fail(POLFED_ERR_INVALID,
           "filter_apply_noalloc: the operator's step kernel for this precision is not chosen "
           "yet; run one step, filter or solve in this precision, or pick it with "
           "polfed_op_set_kernel, first");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    unsigned char* base = static_cast<unsigned char*>(resolve_scratch(ctx->device));
    const size_t half = kNoAllocScratchBytes / 2;
    if (precision == POLFED_FP64)
      filter_apply<double>(ctx, op, E_c, dE, a, K, static_cast<const double*>(v),
                           static_cast<double*>(w), reinterpret_cast<double*>(base),
                           reinterpret_cast<double*>(base + half));
    else
      filter_apply<float>(ctx, op, E_c, dE, a, K, static_cast<const float*>(v),
                          static_cast<float*>(w), reinterpret_cast<float*>(base),
                          reinterpret_cast<float*>(base + half));
    return POLFED_OK;
  });
}

polfed_status polfed_clenshaw_step(polfed_ctx* ctx, const polfed_op* op, double E_c,
                                   double dE, double a_i, const void* v, const void* b1,
                                   void* b2, int precision, int final) {
  return guarded([&]() -> polfed_status {
    check_step_args(ctx, op, dE, precision);
    REQUIRE(std::isfinite(E_c) && std::isfinite(a_i), "non-finite scalar");
    REQUIRE(op->D == 0 || (v && b1 && b2), "null vector");
    REQUIRE(b1 != b2 && b1 != v, "b1 must not overlap v or b2");
    DeviceGuard g(ctx->device);
    const double f = final ? 0.5 : 1.0;
    const double sigma = f * 2.0 / dE, tau = -f * 2.0 * E_c / dE;
    if (precision == POLFED_FP64)
      op_step<double>(ctx->stream, op, sigma, tau, a_i, static_cast<const double*>(v),
                      static_cast<const double*>(b1), static_cast<const double*>(b2),
                      static_cast<double*>(b2));
    else
      op_step<float>(ctx->stream, op, (float)sigma, (float)tau, (float)a_i,
                     static_cast<const float*>(v), static_cast<const float*>(b1),
                     static_cast<const float*>(b2), static_cast<float*>(b2));
    return POLFED_OK;
  });
}

// ------------------------------------------------ extraction and products

polfed_status polfed_extract(polfed_ctx* ctx, const polfed_op* op, const double* V, int m,
                             const double* T, int n, double* E, double* U2, double* resid) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    REQUIRE(m >= 1 && n >= 1 && n <= m && m <= op->D, "extract: need 1 <= n <= m <= D");
    REQUIRE(V && T && E && U2 && resid, "extract: null buffer");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    extract_pairs(ctx, op, V, m, T, n, E, U2, resid);
    return POLFED_OK;
  });
}

polfed_status polfed_gemm_nn(polfed_ctx* ctx, int64_t D, int m, int n, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                             int subtract) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(D >= 0 && m >= 0 && n >= 0, "gemm: negative size");
    REQUIRE(lda >= std::max<int64_t>(D, 1) && ldc >= std::max<int64_t>(D, 1) &&
                ldb >= std::max(m, 1),
            "gemm: leading dimension too small");
    REQUIRE(D == 0 || n == 0 || ((m == 0 || (A && B)) && C), "gemm: null buffer");
    REQUIRE(m > 0 || subtract || D == 0 || n == 0, "gemm: empty inner dimension");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    dev_gemm_nn(ctx->stream, D, m, n, A, lda, B, ldb, C, ldc, subtract != 0);
    return POLFED_OK;
  });
}

polfed_status polfed_gemm_tn(polfed_ctx* ctx, int64_t D, int n1, int n2, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double* G, int64_t ldg) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(D >= 0 && n1 >= 0 && n2 >= 0, "gemm: negative size");
    REQUIRE(lda >= std::max<int64_t>(D, 1) && ldb >= std::max<int64_t>(D, 1) &&
                ldg >= std::max(n1, 1),
            "gemm: leading dimension too small");
    REQUIRE(n1 == 0 || n2 == 0 || (A && B && G), "gemm: null buffer");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx, CtxLock::kBuild);
    dev_gemm_tn(ctx->stream, D, n1, n2, A, lda, B, ldb, G, ldg);
    return POLFED_OK;
  });
}

// ----------------------------------------------------- multi-column filter

static void check_batch_args(polfed_ctx* ctx, int B, const polfed_op* const* ops,
                             const double* E_c, const double* dE, int precision) {
  CTX_OK(ctx);
  REQUIRE(B >= 1 && ops && E_c && dE, "batch: need B >= 1 and arrays ops, E_c, dE");
  REQUIRE(precision == POLFED_FP64 || precision == POLFED_FP32, "unknown precision");
  for (int i = 0; i < B; ++i) {
    REQUIRE(ops[i] && ops[i]->ctx == ctx, "batch: operator missing or from another context");
    REQUIRE(std::isfinite(E_c[i]) && std::isfinite(dE[i]) && dE[i] > 0,
            "batch: E_c must be finite and dE finite and positive");
  }
}

polfed_status polfed_filter_apply_batch(polfed_ctx* ctx, int B, const polfed_op* const* ops,
                                        const double* E_c, const double* dE,
                                        const double* const* a, const int* K, const void* v,
                                        void* w, int precision) {
  return guarded([&]() -> polfed_status {
    check_batch_args(ctx, B, ops, E_c, dE, precision);
    REQUIRE(a && K, "batch: need coefficient arrays a and orders K");
    for (int i = 0; i < B; ++i) REQUIRE(a[i] && K[i] >= 0, "batch: need K >= 0 and a[K+1]");
    REQUIRE(v && w && v != w, "batch: null or overlapping vector blocks");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    ChainBatch bt;
    bt.init(ctx, ops, B);
    bt.set_scale(E_c, dE);
    BatchCoef co;
    co.set(ctx->stream, B, a, K);
    const size_t n = (size_t)ops[0]->D * B;
    if (precision == POLFED_FP64) {
      DevBuf A(n * sizeof(double)), Bb(n * sizeof(double));
      filter_apply_batch<double>(ctx, bt, co, static_cast<const double*>(v),
                                 static_cast<double*>(w), A.as<double>(), Bb.as<double>());
      HIPC(hipStreamSynchronize(ctx->stream));
    } else {
      DevBuf A(n * sizeof(float)), Bb(n * sizeof(float));
      filter_apply_batch<float>(ctx, bt, co, static_cast<const float*>(v),
                                static_cast<float*>(w), A.as<float>(), Bb.as<float>());
      HIPC(hipStreamSynchronize(ctx->stream));
    }
    return POLFED_OK;
  });
}

polfed_status polfed_clenshaw_step_batch(polfed_ctx* ctx, int B, const polfed_op* const* ops,
                                         const double* E_c, const double* dE,
                                         const double* a_i, const void* v, const void* b1,
                                         void* b2, int precision, int final) {
  return guarded([&]() -> polfed_status {
    check_batch_args(ctx, B, ops, E_c, dE, precision);
    REQUIRE(a_i, "batch: need coefficients a_i[B]");
    for (int i = 0; i < B; ++i) REQUIRE(std::isfinite(a_i[i]), "batch: non-finite a_i");
    REQUIRE(v && b1 && b2, "batch: null vector block");
    REQUIRE(b1 != b2 && b1 != v, "batch: b1 must not overlap v or b2");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    ChainBatch bt;
    bt.init(ctx, ops, B);
    bt.set_scale(E_c, dE);
    const int64_t D = ops[0]->D;
    if (precision == POLFED_FP64) {
      DevBuf ad;
      upload(ad, a_i, (size_t)B, ctx->stream);
      chain_batch_step<double>(ctx->stream, bt, D, final != 0, ad.as<double>(),
                               static_cast<const double*>(v), static_cast<const double*>(b1),
                               static_cast<const double*>(b2), static_cast<double*>(b2));
      HIPC(hipStreamSynchronize(ctx->stream));
    } else {
      std::vector<float> af(a_i, a_i + B);
      DevBuf ad;
      upload(ad, af.data(), af.size(), ctx->stream);
      chain_batch_step<float>(ctx->stream, bt, D, final != 0, ad.as<float>(),
                              static_cast<const float*>(v), static_cast<const float*>(b1),
                              static_cast<const float*>(b2), static_cast<float*>(b2));
      HIPC(hipStreamSynchronize(ctx->stream));
    }
    return POLFED_OK;
  });
}

// ------------------------------------------------------------- Lanczos

polfed_status polfed_bounds(polfed_ctx* ctx, const polfed_op* op, const double* x0,
                            double tol, int max_iter, double* E_min, double* E_max) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    REQUIRE(x0 && E_min && E_max, "null argument");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    bounds(ctx, op, x0, tol, max_iter, E_min, E_max, nullptr);
    return POLFED_OK;
  });
}

polfed_status polfed_lanczos_step(polfed_ctx* ctx, const polfed_op* op, double E_c,
                                  double dE, const double* a, int K, double* V, int k,
                                  double* alpha, double* beta, int precision) {
  return guarded([&]() -> polfed_status {
    check_step_args(ctx, op, dE, precision);
    REQUIRE(std::isfinite(E_c), "E_c must be finite");
    REQUIRE(K >= 0 && a, "need K >= 0 and coefficients a[K+1]");
    REQUIRE(k >= 0 && k + 1 < op->D + 1, "need 0 <= k and k + 1 <= D");
    REQUIRE(V && alpha && beta, "null buffer");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    lanczos_step(ctx, op, E_c, dE, a, K, V, k, alpha, beta, precision);
    return POLFED_OK;
  });
}

polfed_status polfed_kpm_moments(polfed_ctx* ctx, const polfed_op* op, double E_c, double dE,
                                 int N, int R, const double* r, uint64_t seed, double* mu) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    REQUIRE(mu, "null output");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    kpm_moments(ctx, op, E_c, dE, N, R, r, seed, mu);
    return POLFED_OK;
  });
}

polfed_status polfed_kpm_density(const double* mu, int N, const double* x, int nx, double* rho) {
  return guarded([&]() -> polfed_status {
    REQUIRE(mu && x && rho && nx >= 0, "null argument");
    kpm_density(mu, N, x, nx, rho);
    return POLFED_OK;
  });
}

polfed_status polfed_block_lanczos_step(polfed_ctx* ctx, const polfed_op* op, double E_c,
                                        double dE, const double* a, int K, double* V, int k,
                                        int s, double* A, double* Bn, int precision) {
  return guarded([&]() -> polfed_status {
    check_step_args(ctx, op, dE, precision);
    REQUIRE(std::isfinite(E_c), "E_c must be finite");
    REQUIRE(K >= 0 && a, "need K >= 0 and coefficients a[K+1]");
    REQUIRE(s >= 1 && s <= 64, "need 1 <= s <= 64");
    REQUIRE(k >= 0 && k % s == 0 && (int64_t)k + 2 * s <= op->D,
            "need k >= 0 a multiple of s and k + 2 s <= D");
    REQUIRE(V && A && Bn, "null buffer");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    block_lanczos_step(ctx, op, E_c, dE, a, K, V, k, s, A, Bn, precision);
    return POLFED_OK;
  });
}

polfed_status polfed_profile_step(polfed_ctx* ctx, const polfed_op* op, int precision,
                                  int iters, double* avg_ms, double* min_ms) {
  return guarded([&]() -> polfed_status {
    check_step_args(ctx, op, 1.0, precision);
    REQUIRE(iters >= 1 && iters <= 100000, "need 1 <= iters <= 100000");
    REQUIRE(avg_ms && min_ms, "null output");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    profile_step(ctx, op, precision, iters, avg_ms, min_ms);
    return POLFED_OK;
  });
}

polfed_status polfed_params_default(polfed_params* p) {
  return guarded([&]() -> polfed_status {
    REQUIRE(p, "null params");
    std::memset(p, 0, sizeof *p);
    p->target_kind = POLFED_TARGET_NORMALIZED;
    p->target = 0.5;
    p->n_ev = 20;
    p->precision = POLFED_FP64;
    p->eta = 1.5;
    p->tol_resid = 1e-8;
    p->bound_pad = 1e-3;
    return POLFED_OK;
  });
}

polfed_status polfed_solve(polfed_ctx* ctx, const polfed_op* op, const polfed_params* params,
                           const double* x0, double* evals, double* evecs, double* resid,
                           int* n_found, polfed_report* rep) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(op && op->ctx == ctx, "operator missing or from another context");
    REQUIRE(params, "null params");
    if (n_found) *n_found = 0;
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    return solve(ctx, op, *params, x0, evals, evecs, resid, n_found, rep);
  });
}

polfed_status polfed_solve_batch(polfed_ctx* ctx, int B, const polfed_op* const* ops,
                                 const polfed_params* params, const double* const* x0,
                                 double* const* evals, double* const* evecs,
                                 double* const* resid, int* n_found, polfed_report* rep) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    REQUIRE(B >= 1 && ops && params && x0 && evals && evecs && resid && n_found,
            "null argument");
    for (int i = 0; i < B; ++i) REQUIRE(ops[i] && ops[i]->ctx == ctx, "bad operator");
    DeviceGuard g(ctx->device);
    CtxLock lk(ctx);
    return solve_batch(ctx, B, ops, *params, x0, evals, evecs, resid, n_found, rep);
  });
}

// ------------------------------------------------------------- serving

polfed_status polfed_serve_start(polfed_ctx* ctx, size_t hbm_budget_bytes, int max_cols) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    return serve_start(ctx, hbm_budget_bytes, max_cols);
  });
}

polfed_status polfed_submit(polfed_ctx* ctx, const polfed_op* op, const polfed_params* params,
                            const double* x0, double* evals, double* evecs, double* resid,
                            polfed_req** out) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    return serve_submit(ctx, op, params, x0, evals, evecs, resid, out);
  });
}

polfed_status polfed_poll(polfed_req* req, int* done) {
  return guarded([&]() -> polfed_status { return req_poll(req, done); });
}

polfed_status polfed_wait(polfed_req* req, int* n_found, polfed_report* rep) {
  return guarded([&]() -> polfed_status { return req_wait(req, n_found, rep); });
}

polfed_status polfed_req_destroy(polfed_req* req) {
  return guarded([&]() -> polfed_status { return req_destroy(req); });
}

polfed_status polfed_serve_stop(polfed_ctx* ctx) {
  return guarded([&]() -> polfed_status {
    CTX_OK(ctx);
    return serve_stop(ctx);
  });
}

}  // extern "C"

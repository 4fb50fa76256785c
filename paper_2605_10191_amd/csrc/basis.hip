// Sector basis of L-bit strings with N set bits (App. A, U(1) sector),
// ranked in ascending integer order.  The rank of s is the combinadic
// sum_k binom(p_k, k) over its set-bit positions p_1 < ... < p_N: the number
// of sector states below s.
#include "internal.hpp"

namespace polfed {

namespace {
struct BinomTable {
  uint32_t c[kBinomN * kBinomN];
  BinomTable() {
    for (int n = 0; n < kBinomN; ++n)
      for (int k = 0; k < kBinomN; ++k) {
        uint64_t v;
        if (k == 0) v = 1;
        else if (n == 0) v = 0;
        else v = (uint64_t)c[(n - 1) * kBinomN + k - 1] + c[(n - 1) * kBinomN + k];
        // entries that do not fit 32 bits are never used as ranks (D < 2^31)
        c[n * kBinomN + k] = v > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)v;
      }
  }
};
const BinomTable& table() {
  static BinomTable t;
  return t;
}
}  // namespace

const uint32_t* host_binom() { return table().c; }

int64_t binom64(int n, int k) {
  if (k < 0 || n < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

__device__ __forceinline__ uint32_t rank_of(uint32_t s, const uint32_t* B) {
  uint32_t r = 0;
  int k = 1;
  while (s) {
    int p = __ffs(s) - 1;
    r += B[p * kBinomN + k];
    ++k;
    s &= s - 1;
  }
  return r;
}

__device__ __forceinline__ uint32_t unrank_of(uint32_t r, int L, int N,
                                              const uint32_t* B) {
  uint32_t s = 0;
  int k = N;
  for (int p = L - 1; p >= 0 && k > 0; --p) {
    uint32_t c = B[p * kBinomN + k];
    if (r >= c) {
      s |= 1u << p;
      r -= c;
      --k;
    }
  }
  return s;
}

__global__ void k_enumerate(int L, int N, int64_t D, uint32_t* states,
                            const uint32_t* B) {
  const int chunk = 16;
  int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * chunk;
  if (r0 >= D) return;
  uint32_t s = unrank_of((uint32_t)r0, L, N, B);
  for (int j = 0; j < chunk && r0 + j < D; ++j) {
    states[r0 + j] = s;
    if (s) {  // next combination with the same popcount (Gosper)
      uint32_t t = s | (s - 1);
      s = (t + 1) | (((~t & (0u - ~t)) - 1) >> (__ffs(s)));
    }
  }
}

__global__ void k_rank(int L, int N, const uint32_t* states, int64_t n,
                       int64_t* ranks, const uint32_t* B) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t s = states[i];
  bool ok = __popc(s) == N && (L == 32 || (s >> L) == 0);
  ranks[i] = ok ? (int64_t)rank_of(s, B) : -1;
}

__global__ void k_unrank(int L, int N, int64_t D, const int64_t* ranks,
                         int64_t n, uint32_t* states, const uint32_t* B) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t r = ranks[i];
  states[i] = (r < 0 || r >= D) ? 0xFFFFFFFFu : unrank_of((uint32_t)r, L, N, B);
}

static unsigned grid_for(int64_t n, int per_block) {
  int64_t g = (n + per_block - 1) / per_block;
  return (unsigned)(g > 0 ? g : 1);
}

void basis_enumerate(hipStream_t s, int L, int N, int64_t D, uint32_t* states,
                     const uint32_t* d_binom) {
  if (D == 0) return;
  hipLaunchKernelGGL(k_enumerate, dim3(grid_for(D, 256 * 16)), dim3(256), 0, s,
                     L, N, D, states, d_binom);
  HIPC(hipGetLastError());
}

void basis_rank(hipStream_t s, int L, int N, const uint32_t* states, int64_t n,
                int64_t* ranks, const uint32_t* d_binom) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_rank, dim3(grid_for(n, 256)), dim3(256), 0, s, L, N,
                     states, n, ranks, d_binom);
  HIPC(hipGetLastError());
}

void basis_unrank(hipStream_t s, int L, int N, int64_t D, const int64_t* ranks,
                  int64_t n, uint32_t* states, const uint32_t* d_binom) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_unrank, dim3(grid_for(n, 256)), dim3(256), 0, s, L, N,
                     D, ranks, n, states, d_binom);
  HIPC(hipGetLastError());
}

// state = hi << Lb | lo.  Ascending state order is ascending (hi, lo), so
// rank(state) = hi_off[hi] + lo_rank[lo], where hi_off[hi] counts sector
// states with a smaller high part and lo_rank[lo] counts the low parts below
// lo with the same popcount.
void build_split_rank_tables(int L, int N, int Lb, std::vector<int32_t>& hi_off,
                             std::vector<int32_t>& lo_rank) {
  const int Lh = L - Lb;
  lo_rank.assign((size_t)1 << Lb, 0);
  std::vector<int32_t> seen(Lb + 1, 0);
  for (uint32_t lo = 0; lo < (1u << Lb); ++lo) {
    int p = __builtin_popcount(lo);
    lo_rank[lo] = seen[p]++;
  }
  hi_off.assign((size_t)1 << Lh, 0);
  int64_t acc = 0;
  for (uint32_t hi = 0; hi < (1u << Lh); ++hi) {
    hi_off[hi] = (int32_t)acc;
    int need = N - __builtin_popcount(hi);
    if (need >= 0 && need <= Lb) acc += binom64(Lb, need);
  }
}

}  // namespace polfed

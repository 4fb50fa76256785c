// Dense vector and tall-skinny kernels of the Lanczos iteration: reductions,
// the two products of classical Gram-Schmidt (c = V^T w, w -= V c), scaling,
// conversions, and the small GEMMs of the eigenpair extraction.  All FP64;
// every reduction has a fixed order (block partials, then one block), so
// results do not depend on timing.
#include <algorithm>

#include "internal.hpp"

namespace polfed {

constexpr int kTB = 256;  // threads per block of these kernels

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

// Sums x over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_reduce(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = x;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

int64_t red_blocks(int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(1024, (n + kTB * 4 - 1) / (kTB * 4)));
}

__global__ __launch_bounds__(kTB) void k_dot_partial(int64_t n, const double* x,
                                                     const double* y, double* part) {
  __shared__ double red[kTB / 64];
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  const double t = block_reduce(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kTB) void k_sum_partials(const double* part, int64_t n,
                                                      double* out, int sqrt_out) {
  __shared__ double red[kTB / 64];
  double acc = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  const double t = block_reduce(acc, red);
  if (threadIdx.x == 0) out[0] = sqrt_out ? sqrt(t) : t;
}

void dev_dot(hipStream_t s, int64_t n, const double* x, const double* y,
             double* partial, int64_t npart, double* out, int sqrt_out) {
  const int64_t g = std::min(npart, red_blocks(n));
  hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)g), dim3(kTB), 0, s, n, x, y, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kTB), 0, s, partial, g, out, sqrt_out);
  HIPC(hipGetLastError());
}

// ---- c = V^T w over k columns: grid (column groups of 8, row segments) ----
constexpr int kCols = 8;

__global__ __launch_bounds__(kTB) void k_gemv_t(int64_t D, int k, const double* V,
                                                int64_t ld, const double* w,
                                                int64_t seg_len, int64_t nseg,
                                                double* part) {
  __shared__ double red[kCols][kTB / 64];
  const int j0 = blockIdx.x * kCols;
  const int64_t seg = blockIdx.y;
  const int64_t r0 = seg * seg_len, r1 = std::min<int64_t>(D, r0 + seg_len);
  double acc[kCols];
#pragma unroll
  for (int q = 0; q < kCols; ++q) acc[q] = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const double wr = w[r];
#pragma unroll
    for (int q = 0; q < kCols; ++q)
      if (j0 + q < k) acc[q] += V[r + (int64_t)(j0 + q) * ld] * wr;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kCols; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) red[q][wid] = t;
  }
  __syncthreads();
  if (threadIdx.x < kCols && j0 + (int)threadIdx.x < k) {
    double t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[threadIdx.x][i];
    part[(int64_t)(j0 + threadIdx.x) * nseg + seg] = t;
  }
}

// c[j] = sum of the partials of column j; the last column's value is also
// stored to (or added to) *tail, which carries the Lanczos alpha_k.
__global__ void k_reduce_cols(const double* part, int64_t nseg, int k, double* c,
                              double* tail, int tail_add) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double t = 0;
  for (int64_t s = 0; s < nseg; ++s) t += part[(int64_t)j * nseg + s];
  c[j] = t;
  if (tail && j == k - 1) tail[0] = tail_add ? tail[0] + t : t;
}

static int64_t seg_len_for(int64_t D, int64_t nseg) {
  int64_t len = (D + nseg - 1) / nseg;
  return std::max<int64_t>(kTB, ((len + kTB - 1) / kTB) * kTB);
}

void dev_gemv_t(hipStream_t s, int64_t D, int k, const double* V, int64_t ld,
                const double* w, double* partial, int64_t nseg, double* c,
                double* tail, int tail_add) {
  if (k <= 0) return;
  const int64_t len = seg_len_for(D, nseg);
  const int64_t ns = std::max<int64_t>(1, (D + len - 1) / len);
  dim3 grid((unsigned)((k + kCols - 1) / kCols), (unsigned)ns);
  hipLaunchKernelGGL(k_gemv_t, grid, dim3(kTB), 0, s, D, k, V, ld, w, len, ns, partial);
  hipLaunchKernelGGL(k_reduce_cols, dim3((unsigned)((k + 63) / 64)), dim3(64), 0, s,
                     partial, ns, k, c, tail, tail_add);
  HIPC(hipGetLastError());
}

// ---- tall-skinny block products: C = V^T W and W -= V C for W of S <= 8
// columns (block Gram-Schmidt); V is read once per product ----
template <int S>
__global__ __launch_bounds__(kTB) void k_gemm_tn_tall(int64_t D, int k, const double* V,
                                                      const double* W, int64_t seg_len,
                                                      int64_t nseg, double* part) {
  __shared__ double red[kCols * S][kTB / 64];
  const int j0 = blockIdx.x * kCols;
  const int64_t seg = blockIdx.y;
  const int64_t r0 = seg * seg_len, r1 = std::min<int64_t>(D, r0 + seg_len);
  double acc[kCols][S];
#pragma unroll
  for (int q = 0; q < kCols; ++q)
#pragma unroll
    for (int j = 0; j < S; ++j) acc[q][j] = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    double w[S];
#pragma unroll
    for (int j = 0; j < S; ++j) w[j] = W[r + (int64_t)j * D];
#pragma unroll
    for (int q = 0; q < kCols; ++q)
      if (j0 + q < k) {
        const double x = V[r + (int64_t)(j0 + q) * D];
#pragma unroll
        for (int j = 0; j < S; ++j) acc[q][j] += x * w[j];
      }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kCols; ++q)
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const double t = wave_sum(acc[q][j]);
      if (lane == 0) red[q * S + j][wid] = t;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < kCols * S; i += blockDim.x) {
    const int q = i / S, j = i % S;
    if (j0 + q < k) {
      double t = 0;
      for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) t += red[i][w2];
      // column-major k x S result: entry (j0 + q, j)
      part[((int64_t)j * k + j0 + q) * nseg + seg] = t;
    }
  }
}

template <int S>
__global__ __launch_bounds__(kTB) void k_gemm_nn_sub_tall(int64_t D, int k, const double* V,
                                                          const double* C, double* W) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  double acc[S];
#pragma unroll
  for (int j = 0; j < S; ++j) acc[j] = 0;
  for (int i = 0; i < k; ++i) {
    const double x = V[r + (int64_t)i * D];
#pragma unroll
    for (int j = 0; j < S; ++j) acc[j] += x * C[i + (int64_t)j * k];
  }
#pragma unroll
  for (int j = 0; j < S; ++j) W[r + (int64_t)j * D] -= acc[j];
}

template <int S>
static void tall_pass(hipStream_t s, int64_t D, int k, const double* V, double* W,
                      double* partial, int64_t nseg, double* C) {
  const int64_t len = seg_len_for(D, nseg);
  const int64_t ns = std::max<int64_t>(1, (D + len - 1) / len);
  dim3 grid((unsigned)((k + kCols - 1) / kCols), (unsigned)ns);
  hipLaunchKernelGGL(k_gemm_tn_tall<S>, grid, dim3(kTB), 0, s, D, k, V, W, len, ns, partial);
  hipLaunchKernelGGL(k_reduce_cols, dim3((unsigned)((k * S + 63) / 64)), dim3(64), 0, s, partial,
                     ns, k * S, C, nullptr, 0);
  hipLaunchKernelGGL(k_gemm_nn_sub_tall<S>, dim3((unsigned)((D + kTB - 1) / kTB)), dim3(kTB), 0,
                     s, D, k, V, C, W);
  HIPC(hipGetLastError());
}

// One Gram-Schmidt pass of the D x n block W against the first k columns of
// V: C = V^T W (k x n col-major, ld k), W -= V C, in chunks of 8 columns.
// partial: nseg * k * 8 doubles.
void dev_block_gs_pass(hipStream_t s, int64_t D, int k, const double* V, double* W, int n,
                       double* partial, int64_t nseg, double* C) {
  if (k <= 0 || D == 0) return;
  if (n >= kMfmaMinCols) {
    // a wide block: both products on the matrix cores
    dev_gemm_tn(s, D, k, n, V, D, W, D, C, k);
    dev_gemm_nn(s, D, k, n, V, D, C, k, W, D, true);
    return;
  }
  for (int j0 = 0; j0 < n; j0 += 8) {
    const int m = std::min(8, n - j0);
    double* Wc = W + (int64_t)j0 * D;
    double* Cc = C + (int64_t)j0 * k;
    switch (m) {
#define POLFED_CASE(S) \
  case S:              \
    tall_pass<S>(s, D, k, V, Wc, partial, nseg, Cc); \
    break;
      POLFED_CASE(1) POLFED_CASE(2) POLFED_CASE(3) POLFED_CASE(4)
      POLFED_CASE(5) POLFED_CASE(6) POLFED_CASE(7) POLFED_CASE(8)
#undef POLFED_CASE
    }
  }
}

// ---- w -= V c ----
__global__ __launch_bounds__(kTB) void k_gemv_n_sub(int64_t D, int k, const double* V,
                                                    int64_t ld, const double* c,
                                                    double* w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  double acc = 0;
  for (int j = 0; j < k; ++j) acc += V[r + (int64_t)j * ld] * c[j];
  w[r] -= acc;
}

void dev_gemv_n_sub(hipStream_t s, int64_t D, int k, const double* V, int64_t ld,
                    const double* c, double* w) {
  if (k <= 0 || D == 0) return;
  hipLaunchKernelGGL(k_gemv_n_sub, dim3((unsigned)((D + kTB - 1) / kTB)), dim3(kTB), 0,
                     s, D, k, V, ld, c, w);
  HIPC(hipGetLastError());
}

// ---- out = w / beta; a vanishing beta (breakdown) leaves zeros and raises flag ----
__global__ void k_scale_into(int64_t D, const double* w, const double* beta,
                             double* out, int* flag) {
  const double b = beta[0];
  const bool ok = b > 1e-300 && isfinite(b);
  const double inv = ok ? 1.0 / b : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = w[i] * inv;
  if (!ok && flag && blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 1;
}

static unsigned stream_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kTB - 1) / kTB));
}

void dev_scale_into(hipStream_t s, int64_t D, const double* w, const double* beta,
                    double* out, int* flag) {
  hipLaunchKernelGGL(k_scale_into, dim3(stream_grid(D)), dim3(kTB), 0, s, D, w, beta,
                     out, flag);
  HIPC(hipGetLastError());
}

__global__ void k_axpby(int64_t n, double a, const double* x, double b, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}
void dev_axpby(hipStream_t s, int64_t n, double a, const double* x, double b,
               double* y) {
  if (!n) return;
  hipLaunchKernelGGL(k_axpby, dim3(stream_grid(n)), dim3(kTB), 0, s, n, a, x, b, y);
  HIPC(hipGetLastError());
}

__global__ void k_cvt_d2f(int64_t n, const double* x, float* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void k_cvt_f2d(int64_t n, const float* x, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}
void dev_copy_d2f(hipStream_t s, int64_t n, const double* x, float* y) {
  if (!n) return;
  hipLaunchKernelGGL(k_cvt_d2f, dim3(stream_grid(n)), dim3(kTB), 0, s, n, x, y);
  HIPC(hipGetLastError());
}
void dev_copy_f2d(hipStream_t s, int64_t n, const float* x, double* y) {
  if (!n) return;
  hipLaunchKernelGGL(k_cvt_f2d, dim3(stream_grid(n)), dim3(kTB), 0, s, n, x, y);
  HIPC(hipGetLastError());
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}
void dev_fill(hipStream_t s, int64_t n, double v, double* y) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill<double>, dim3(stream_grid(n)), dim3(kTB), 0, s, n, v, y);
  HIPC(hipGetLastError());
}
void dev_fillf(hipStream_t s, int64_t n, float v, float* y) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill<float>, dim3(stream_grid(n)), dim3(kTB), 0, s, n, v, y);
  HIPC(hipGetLastError());
}

// Counter-based uniform draws in [-1, 1): splitmix64 of (seed, index).
__global__ void k_random(int64_t n, uint64_t seed, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    y[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}
void dev_random(hipStream_t s, int64_t n, uint64_t seed, double* y) {
  if (!n) return;
  hipLaunchKernelGGL(k_random, dim3(stream_grid(n)), dim3(kTB), 0, s, n, seed, y);
  HIPC(hipGetLastError());
}

// ---- residual norms ----
__global__ __launch_bounds__(kTB) void k_resid(int64_t D, int n, const double* U,
                                               const double* HU, const double* E,
                                               int64_t seg_len, int64_t nseg,
                                               double* part) {
  __shared__ double red[kTB / 64];
  const int j = blockIdx.x;
  const int64_t seg = blockIdx.y;
  const int64_t r0 = seg * seg_len, r1 = std::min<int64_t>(D, r0 + seg_len);
  const double e = E[j];
  double acc = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const double d = HU[r + (int64_t)j * D] - e * U[r + (int64_t)j * D];
    acc += d * d;
  }
  const double t = block_reduce(acc, red);
  if (threadIdx.x == 0) part[(int64_t)j * nseg + seg] = t;
}

__global__ void k_reduce_cols_sqrt(const double* part, int64_t nseg, int n, double* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double t = 0;
  for (int64_t s = 0; s < nseg; ++s) t += part[(int64_t)j * nseg + s];
  out[j] = sqrt(t);
}

void dev_resid(hipStream_t s, int64_t D, int n, const double* U, const double* HU,
               const double* E, double* partial, int64_t nseg, double* res) {
  if (!n) return;
  const int64_t len = seg_len_for(D, nseg);
  const int64_t ns = std::max<int64_t>(1, (D + len - 1) / len);
  hipLaunchKernelGGL(k_resid, dim3((unsigned)n, (unsigned)ns), dim3(kTB), 0, s, D, n, U,
                     HU, E, len, ns, partial);
  hipLaunchKernelGGL(k_reduce_cols_sqrt, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s,
                     partial, ns, n, res);
  HIPC(hipGetLastError());
}

}  // namespace polfed

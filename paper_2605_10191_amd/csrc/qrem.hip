// Quantum random energy model (eq. qrem of App. A) on the full 2^L space:
//   H = sum_a E_a |a><a| - Gamma sum_i sigma^x_i,
// sigma^x_i flipping bit i of the state index.  The fused Clenshaw step
//   out = a v + sigma (H b1) + tau b1 - b2
// is a hypercube stencil: row r needs b1 at r ^ 2^i for every bit i.
//
// A workgroup takes a tile of 2^TB consecutive rows and stages that tile of
// b1 in LDS, so the flips of bits 1..TB-1 read LDS.  The flip of a higher bit
// i moves the whole tile to tile ^ 2^(i-TB) at the same in-tile offset, so
// those reads are coalesced loads at a wave-uniform offset.  Each lane holds
// two adjacent rows (16-byte accesses in FP64), so the flip of bit 0 swaps
// the pair in registers.  Tiles are dealt to the XCDs in contiguous ranges
// (blockIdx.x % 8 is the XCD), so the flips of all but the top three tile
// bits stay inside one XCD's L2.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "chain_dev.hpp"
#include "internal.hpp"

namespace polfed {

constexpr int kQremThreads = 512;
constexpr int kQremMaxTileBits = 12;

template <typename T, int TB>
__global__ __launch_bounds__(kQremThreads) void k_qrem_step(
    int L, int64_t ntiles, int nxcd, T gamma, T sigma, T tau, T a, const T* __restrict__ E,
    const T* __restrict__ v, const T* __restrict__ b1, const T* b2, T* out, uint32_t vbytes) {
  constexpr int NP = 1 << (TB - 1);  // row pairs per tile
  constexpr int PPT = NP > kQremThreads ? NP / kQremThreads : 1;  // pairs per thread
  constexpr uint32_t W = sizeof(T);
  __shared__ __attribute__((aligned(16))) T tile[2 * NP];
  const rsrc_t rb1 = make_rsrc(b1, vbytes), rE = make_rsrc(E, vbytes);
  const rsrc_t rv = make_rsrc(v ? v : b1, v ? vbytes : 0);
  const rsrc_t rb2 = make_rsrc(b2 ? b2 : b1, b2 ? vbytes : 0);
  const rsrc_t ro = make_rsrc(out, vbytes);
  const int xcd = blockIdx.x % nxcd;
  const int64_t per_xcd = gridDim.x / nxcd;
  const int64_t t_end = ntiles * (xcd + 1) / nxcd;
  for (int64_t t = ntiles * xcd / nxcd + blockIdx.x / nxcd; t < t_end; t += per_xcd) {
    const uint32_t toff = (uint32_t)uniform((int)(t << TB)) * W;  // byte offset of the tile
    T x[PPT][2];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int q = threadIdx.x + j * kQremThreads;
      if (q < NP) {
        bload2<T>(rb1, (uint32_t)(2 * q) * W, toff, x[j][0], x[j][1]);
        tile[2 * q] = x[j][0];
        tile[2 * q + 1] = x[j][1];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int q = threadIdx.x + j * kQremThreads;
      if (q < NP) {
        const uint32_t vo = (uint32_t)(2 * q) * W;
        // bit 0: the other row of the pair
        T s0 = x[j][1], s1 = x[j][0];
        // bits 1..TB-1: the pair q ^ 2^(i-1) of this tile, in LDS
#pragma unroll
        for (int i = 1; i < TB; ++i) {
          const int p = q ^ (1 << (i - 1));
          s0 += tile[2 * p];
          s1 += tile[2 * p + 1];
        }
        // bits TB..L-1: the same pair of tile t ^ 2^(i-TB)
#pragma unroll 4
        for (int i = TB; i < L; ++i) {
          const uint32_t po = (uint32_t)uniform((int)((t ^ ((int64_t)1 << (i - TB))) << TB)) * W;
          T g0, g1;
          bload2<T>(rb1, vo, po, g0, g1);
          s0 += g0;
          s1 += g1;
        }
        T e0, e1, v0 = T(0), v1 = T(0), c0 = T(0), c1 = T(0);
        bload2<T, kAuxNT>(rE, vo, toff, e0, e1);
        if (v) bload2<T, kAuxNT>(rv, vo, toff, v0, v1);
        if (b2) bload2<T, kAuxNT>(rb2, vo, toff, c0, c1);
        const T h0 = e0 * x[j][0] - gamma * s0, h1 = e1 * x[j][1] - gamma * s1;
        const T o0 = a * v0 + sigma * h0 + tau * x[j][0] - c0;
        const T o1 = a * v1 + sigma * h1 + tau * x[j][1] - c1;
        bstore2<kAuxNT>(o0, o1, ro, vo, toff);
      }
    }
    __syncthreads();
  }
}

// The same step for NC columns of one operator (block Lanczos): column c of
// the D x NC blocks (column stride D) gets out_c = a v_c + sigma H b1_c +
// tau b1_c - b2_c.  The tile, index arithmetic and the energies are shared;
// each column keeps its own gathers.  Per column the sums run in the same
// order as in k_qrem_step, so each column equals the single-column result.
template <typename T, int TB, int NC>
__global__ __launch_bounds__(kQremThreads) void k_qrem_step_multi(
    int L, int64_t ntiles, int nxcd, T gamma, T sigma, T tau, T a, const T* __restrict__ E,
    const T* __restrict__ v, const T* __restrict__ b1, const T* b2, T* out, int64_t D) {
  constexpr int NP = 1 << (TB - 1);
  constexpr int PPT = NP > kQremThreads ? NP / kQremThreads : 1;
  constexpr uint32_t W = sizeof(T);
  __shared__ __attribute__((aligned(16))) T tile[NC][2 * NP];
  const uint32_t vbytes = (uint32_t)(D * W);
  const rsrc_t rE = make_rsrc(E, vbytes);
  const int xcd = blockIdx.x % nxcd;
  const int64_t per_xcd = gridDim.x / nxcd;
  const int64_t t_end = ntiles * (xcd + 1) / nxcd;
  for (int64_t t = ntiles * xcd / nxcd + blockIdx.x / nxcd; t < t_end; t += per_xcd) {
    const uint32_t toff = (uint32_t)uniform((int)(t << TB)) * W;
    T x[NC][PPT][2];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const rsrc_t rb1 = make_rsrc(b1 + (size_t)c * D, vbytes);
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        const int q = threadIdx.x + j * kQremThreads;
        if (q < NP) {
          bload2<T>(rb1, (uint32_t)(2 * q) * W, toff, x[c][j][0], x[c][j][1]);
          tile[c][2 * q] = x[c][j][0];
          tile[c][2 * q + 1] = x[c][j][1];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int q = threadIdx.x + j * kQremThreads;
      if (q < NP) {
        const uint32_t vo = (uint32_t)(2 * q) * W;
        T e0, e1;
        bload2<T, kAuxNT>(rE, vo, toff, e0, e1);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const rsrc_t rb1 = make_rsrc(b1 + (size_t)c * D, vbytes);
          T s0 = x[c][j][1], s1 = x[c][j][0];
#pragma unroll
          for (int i = 1; i < TB; ++i) {
            const int p = q ^ (1 << (i - 1));
            s0 += tile[c][2 * p];
            s1 += tile[c][2 * p + 1];
          }
#pragma unroll 4
          for (int i = TB; i < L; ++i) {
            const uint32_t po =
                (uint32_t)uniform((int)((t ^ ((int64_t)1 << (i - TB))) << TB)) * W;
            T g0, g1;
            bload2<T>(rb1, vo, po, g0, g1);
            s0 += g0;
            s1 += g1;
          }
          T v0 = T(0), v1 = T(0), c0 = T(0), c1 = T(0);
          if (v) bload2<T, kAuxNT>(make_rsrc(v + (size_t)c * D, vbytes), vo, toff, v0, v1);
          if (b2) bload2<T, kAuxNT>(make_rsrc(b2 + (size_t)c * D, vbytes), vo, toff, c0, c1);
          const T h0 = e0 * x[c][j][0] - gamma * s0, h1 = e1 * x[c][j][1] - gamma * s1;
          const T o0 = a * v0 + sigma * h0 + tau * x[c][j][0] - c0;
          const T o1 = a * v1 + sigma * h1 + tau * x[c][j][1] - c1;
          bstore2<kAuxNT>(o0, o1, make_rsrc(out + (size_t)c * D, vbytes), vo, toff);
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int TB>
static void launch_qrem(hipStream_t s, const polfed_op* op, T sigma, T tau, T a, const T* v,
                        const T* b1, const T* b2, T* out) {
  const int64_t ntiles = op->D >> TB;
  const int per_cu = std::max(1, (int)(2048 / kQremThreads));
  int64_t grid = std::min<int64_t>(ntiles, (int64_t)op->ctx->n_cu * per_cu);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  const bool f64 = sizeof(T) == 8;
  const T* E = (const T*)(f64 ? op->d_diag.get() : op->d_diag32.get());
  hipLaunchKernelGGL((k_qrem_step<T, TB>), dim3((unsigned)std::max<int64_t>(grid, 1)),
                     dim3(kQremThreads), 0, s, op->L, ntiles, nxcd, (T)op->qrem_gamma, sigma,
                     tau, a, E, v, b1, b2, out, (uint32_t)(op->D * sizeof(T)));
  HIPC(hipGetLastError());
}

// Default tile bits: up to 2^12 rows per tile, keeping at least 512 tiles
// (two per CU) from L = 15 on; short chains use tiles of 64 rows.
int qrem_tile_bits(int L) { return std::min({L, kQremMaxTileBits, std::max(L - 9, 6)}); }

template <typename T>
static void launch_tb(hipStream_t s, const polfed_op* op, int tb, T sigma, T tau, T a, const T* v,
                      const T* b1, const T* b2, T* out) {
  switch (tb) {
#define POLFED_CASE(TB)                                           \
  case TB:                                                        \
    launch_qrem<T, TB>(s, op, sigma, tau, a, v, b1, b2, out); \
    break;
    POLFED_CASE(1) POLFED_CASE(2) POLFED_CASE(3) POLFED_CASE(4) POLFED_CASE(5) POLFED_CASE(6)
    POLFED_CASE(7) POLFED_CASE(8) POLFED_CASE(9) POLFED_CASE(10) POLFED_CASE(11)
    POLFED_CASE(12)
#undef POLFED_CASE
    default: fail(POLFED_ERR_INVALID, "qrem: bad tile size");
  }
}

// Tile size picked by timing: the default and its two neighbours, a replay
// of 20 launches each on scratch vectors, at the first step of an operator in each
// precision (not while the stream is being captured).
template <typename T>
static int tuned_tile_bits(hipStream_t s, const polfed_op* op) {
  const int pi = sizeof(T) == 8 ? 0 : 1;
  if (op->tuned[pi] >= 1) return op->tuned[pi];
  const int t0 = qrem_tile_bits(op->L);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPC(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone || op->L < 12) return t0;
  const size_t n = (size_t)op->D;
  DevBuf bv(n * sizeof(T)), bb1(n * sizeof(T)), bb2(n * sizeof(T));
  HIPC(hipMemsetAsync(bv.get(), 0, n * sizeof(T), s));
  HIPC(hipMemsetAsync(bb1.get(), 0, n * sizeof(T), s));
  HIPC(hipMemsetAsync(bb2.get(), 0, n * sizeof(T), s));
  HIPC(hipStreamSynchronize(s));  // the operator's tables and the scratch vectors
  int best = t0;
  float best_us = 1e30f;
  for (int tb = t0 - 1; tb <= t0 + 1; ++tb) {
    if (tb < 1 || tb > std::min(op->L, kQremMaxTileBits)) continue;
    const float us = replay_time_us(
        [&](hipStream_t ts) {
          launch_tb<T>(ts, op, tb, T(0.1), T(0), T(0), bv.as<T>(), bb1.as<T>(), bb2.as<T>(),
                       bb2.as<T>());
        },
        20);
    if (verbose())
      std::fprintf(stderr, "[polfed] qrem step L=%d %s tile bits %d: %.2f us\n", op->L,
                   sizeof(T) == 8 ? "fp64" : "fp32", tb, us);
    if (us < best_us) {
      best_us = us;
      best = tb;
    }
  }
  HIPC(hipStreamSynchronize(s));
  return op->tuned[pi] = best;
}

template <typename T>
void qrem_step(hipStream_t s, const polfed_op* op, T sigma, T tau, T a, const T* v, const T* b1,
               const T* b2, T* out) {
  launch_tb<T>(s, op, tuned_tile_bits<T>(s, op), sigma, tau, a, v, b1, b2, out);
}

template <typename T, int NC>
static void launch_multi(hipStream_t s, const polfed_op* op, T sigma, T tau, T a, const T* v,
                         const T* b1, const T* b2, T* out) {
  constexpr int TB = 10;  // 8 KB of FP64 rows per column and tile
  const int64_t ntiles = op->D >> TB;
  const int per_cu = std::max(1, (int)(2048 / kQremThreads));
  int64_t grid = std::min<int64_t>(ntiles, (int64_t)op->ctx->n_cu * per_cu);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  const bool f64 = sizeof(T) == 8;
  const T* E = (const T*)(f64 ? op->d_diag.get() : op->d_diag32.get());
  hipLaunchKernelGGL((k_qrem_step_multi<T, TB, NC>), dim3((unsigned)std::max<int64_t>(grid, 1)),
                     dim3(kQremThreads), 0, s, op->L, ntiles, nxcd, (T)op->qrem_gamma, sigma, tau,
                     a, E, v, b1, b2, out, op->D);
  HIPC(hipGetLastError());
}

template <typename T>
void qrem_step_multi(hipStream_t s, const polfed_op* op, int n, T sigma, T tau, T a, const T* v,
                     const T* b1, const T* b2, T* out) {
  REQUIRE(op->L >= 10, "qrem: the multi-column step needs L >= 10");
  const int64_t D = op->D;
  for (int c0 = 0; c0 < n;) {
    const int m = n - c0 >= 4 ? 4 : (n - c0 >= 2 ? 2 : 1);
    const size_t o = (size_t)c0 * D;
    const T* vc = v ? v + o : nullptr;
    const T* b2c = b2 ? b2 + o : nullptr;
    if (m == 4)
      launch_multi<T, 4>(s, op, sigma, tau, a, vc, b1 + o, b2c, out + o);
    else if (m == 2)
      launch_multi<T, 2>(s, op, sigma, tau, a, vc, b1 + o, b2c, out + o);
    else
      launch_multi<T, 1>(s, op, sigma, tau, a, vc, b1 + o, b2c, out + o);
    c0 += m;
  }
}

template void qrem_step_multi<double>(hipStream_t, const polfed_op*, int, double, double, double,
                                      const double*, const double*, const double*, double*);
template void qrem_step_multi<float>(hipStream_t, const polfed_op*, int, float, float, float,
                                     const float*, const float*, const float*, float*);

template void qrem_step<double>(hipStream_t, const polfed_op*, double, double, double,
                                const double*, const double*, const double*, double*);
template void qrem_step<float>(hipStream_t, const polfed_op*, float, float, float, const float*,
                               const float*, const float*, float*);

__global__ void k_qrem_d2f(int64_t n, const double* x, float* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

polfed_op* make_qrem(polfed_ctx* ctx, int L, const double* E, double gamma) {
  REQUIRE(L >= 2 && L <= 28, "qrem: need 2 <= L <= 28");
  REQUIRE(E, "qrem: missing energies");
  REQUIRE(std::isfinite(gamma), "qrem: non-finite Gamma");
  const int64_t D = (int64_t)1 << L;
  auto op = std::make_unique<polfed_op>();
  op->ctx = ctx;
  op->model = Model::Qrem;
  op->L = L;
  op->D = D;
  op->qrem_gamma = gamma;
  // exact trace moments: Tr H / D = mean E, Tr H^2 / D = mean E^2 + L Gamma^2
  double s1 = 0, s2 = 0;
  for (int64_t i = 0; i < D; ++i) {
    REQUIRE(std::isfinite(E[i]), "qrem: non-finite energy");
    s1 += E[i];
    s2 += E[i] * E[i];
  }
  op->qrem_tr[0] = s1;
  op->qrem_tr[1] = s2 + (double)D * L * gamma * gamma;
  op->nnz = D * L;
  hipStream_t s = ctx->stream;
  upload(op->d_diag, E, (size_t)D, s);
  op->d_diag32.alloc((size_t)D * sizeof(float));
  hipLaunchKernelGGL(k_qrem_d2f, dim3(1024), dim3(256), 0, s, D, op->d_diag.as<double>(),
                     op->d_diag32.as<float>());
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(s));
  return op.release();
}

}  // namespace polfed

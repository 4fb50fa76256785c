// Hamiltonian operators and the fused Clenshaw step (the hot kernel).
//
// One Clenshaw step of eq. clenshaw_chebyshev_prod with the rescaling of
// eq. rescaledMatrix folded in (2 H~ b = sigma H b + tau b, sigma = 2/dE,
// tau = -2 E_c/dE) is
//     out = a_i v + sigma (H b1) + tau b1 - b2,
// and the same kernel with (sigma/2, tau/2) is the closing step
// a_0 v + H~ b_1 - b_2.  Each kernel reads v, b1 (own rows plus gathered
// neighbours), b2 and writes out = b2 in place: one pass over HBM per step.
//
// Matrix-free operators generate H from the state bits (the "specialized
// mapping" of Sec. 4.5 / 5.7): for the chain models a lane owns ROWS
// consecutive sector states, unranks the first one and steps to the next
// with the next-combination bit trick; a hop of the particle at site b to
// b+1 changes the combinadic rank by +binom(b, m) (m = particles below b),
// the reverse hop by -binom(b, m); only the periodic bond needs the split
// rank tables.  The diagonal is generated from popcounts and byte tables of
// the fields, so neither the basis nor the diagonal is read from HBM.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>

#include "internal.hpp"

namespace polfed {

// ------------------------------------------------------------- helpers ----

template <typename T>
struct Tab;
template <>
struct Tab<double> {
  __host__ __device__ static const double* chain(const ChainDev& c) { return c.ftab; }
  __host__ __device__ static const double* qsun(const QsunDev& q) { return q.ftab; }
  __host__ __device__ static const double* val(const CsrDev& m) { return m.val; }
  __host__ __device__ static const double* diag(const CsrDev& m) { return m.diag; }
  __host__ __device__ static const double* vtab(const CsrDev& m) { return m.vtab; }
};
template <>
struct Tab<float> {
  __host__ __device__ static const float* chain(const ChainDev& c) { return c.ftab32; }
  __host__ __device__ static const float* qsun(const QsunDev& q) { return q.ftab32; }
  __host__ __device__ static const float* val(const CsrDev& m) { return m.val32; }
  __host__ __device__ static const float* diag(const CsrDev& m) { return m.diag32; }
  __host__ __device__ static const float* vtab(const CsrDev& m) { return m.vtab32; }
};

// Off-diagonal value of entry e: from the value array, or (MAPPED) from the
// table of an optimized mapping, by a one-byte code per entry or, for a
// single value, without any per-entry data.
template <typename T, bool MAPPED>
__device__ __forceinline__ T csr_value(const CsrDev& m, const T* val, const T* vt, int64_t e) {
  if constexpr (MAPPED) {
    if (m.ncode == 1) return vt[0];
    return vt[m.code[e]];
  } else {
    return val[e];
  }
}

using u32x4 = __attribute__((ext_vector_type(4))) uint32_t;

template <typename T, int ROWS>
__device__ __forceinline__ void vload(const T* p, T (&x)[ROWS]) {
  static_assert((sizeof(T) * ROWS) % 16 == 0, "16-byte vector rows");
  constexpr int NV = sizeof(T) * ROWS / 16;
  u32x4 t[NV];
  const u32x4* q = reinterpret_cast<const u32x4*>(p);
#pragma unroll
  for (int i = 0; i < NV; ++i) t[i] = q[i];
  __builtin_memcpy(x, t, sizeof(T) * ROWS);
}

template <typename T, int ROWS>
__device__ __forceinline__ void vstore(T* p, const T (&x)[ROWS]) {
  constexpr int NV = sizeof(T) * ROWS / 16;
  u32x4 t[NV];
  __builtin_memcpy(t, x, sizeof(T) * ROWS);
  u32x4* q = reinterpret_cast<u32x4*>(p);
#pragma unroll
  for (int i = 0; i < NV; ++i) q[i] = t[i];
}

__device__ __forceinline__ uint32_t next_comb(uint32_t s) {
  uint32_t t = s | (s - 1);
  return (t + 1) | (((~t & (0u - ~t)) - 1) >> (__ffs(s)));
}

__device__ __forceinline__ uint32_t unrank_lds(uint32_t r, int L, int N,
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

template <typename T>
__device__ __forceinline__ T field_sum(const T* f, uint32_t s) {
  return f[s & 255u] + f[256 + ((s >> 8) & 255u)] + f[512 + ((s >> 16) & 255u)] +
         f[768 + (s >> 24)];
}

// Row r of H applied to b1, for the chain in state s (rank r).
template <typename T>
__device__ __forceinline__ T chain_row(const ChainDev& c, const T* sf,
                                       const uint32_t* sB, uint32_t s, int32_t r,
                                       T b_own, const T* __restrict__ b1) {
  const int L = c.L;
  const uint32_t pairs = s & (s >> 1);
  const uint32_t top = s >> (L - 1);
  int n11 = __popc(pairs) + (c.periodic ? (int)(top & s & 1u) : 0);
  T dg = (T)c.vzz * (T)n11 + (T)c.c0 + field_sum(sf, s);
  const uint32_t x = (s ^ (s >> 1)) & ((1u << (L - 1)) - 1u);
  T hop = 0;
  int m = 0;
  for (int b = 0; b < L - 1; ++b) {
    const uint32_t sb = (s >> b) & 1u;
    if ((x >> b) & 1u) {
      const int32_t d = (int32_t)sB[b * kBinomN + m];
      hop += b1[r + (sb ? d : -d)];
    }
    m += (int)sb;
  }
  T acc = dg * b_own + (T)c.t_in * hop;
  if (c.periodic && ((top ^ s) & 1u)) {
    const uint32_t sp = s ^ (1u | (1u << (L - 1)));
    const int32_t nr =
        c.hi_off[sp >> c.Lb] + c.lo_rank[sp & ((1u << c.Lb) - 1u)];
    acc += (T)c.t_pb * b1[nr];
  }
  return acc;
}

// ------------------------------------------------------ chain kernel ----

template <typename T, int ROWS>
__global__ __launch_bounds__(256) void k_chain_step(
    ChainDev c, T sigma, T tau, T a, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out, int vec_ok) {
  __shared__ T sf[1024];
  __shared__ uint32_t sB[kBinomN * kBinomN];
  const T* ft = Tab<T>::chain(c);
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) sf[i] = ft[i];
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += blockDim.x)
    sB[i] = c.binom[i];
  __syncthreads();
  const int64_t per_block = (int64_t)blockDim.x * ROWS;
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < c.D;
       base += (int64_t)gridDim.x * per_block) {
    const int64_t r0 = base + (int64_t)threadIdx.x * ROWS;
    if (r0 >= c.D) continue;
    const bool full = vec_ok && (r0 + ROWS <= c.D);
    T vv[ROWS], bo[ROWS], bt[ROWS], res[ROWS];
    if (full) {
      vload<T, ROWS>(b1 + r0, bo);
      if (v) vload<T, ROWS>(v + r0, vv);
      if (b2) vload<T, ROWS>(b2 + r0, bt);
    } else {
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        const bool in = r0 + j < c.D;
        bo[j] = in ? b1[r0 + j] : T(0);
        vv[j] = (in && v) ? v[r0 + j] : T(0);
        bt[j] = (in && b2) ? b2[r0 + j] : T(0);
      }
    }
    uint32_t s = unrank_lds((uint32_t)r0, c.L, c.N, sB);
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      T o = 0;
      if (r0 + j < c.D) {
        const T acc = chain_row<T>(c, sf, sB, s, (int32_t)(r0 + j), bo[j], b1);
        o = sigma * acc + tau * bo[j];
        if (v) o += a * vv[j];
        if (b2) o -= bt[j];
        s = next_comb(s);
      }
      res[j] = o;
    }
    if (full) {
      vstore<T, ROWS>(out + r0, res);
    } else {
#pragma unroll
      for (int j = 0; j < ROWS; ++j)
        if (r0 + j < c.D) out[r0 + j] = res[j];
    }
  }
}

// ------------------------------------------------------- qsun kernel ----

template <typename T, int ROWS>
__global__ __launch_bounds__(256) void k_qsun_step(
    QsunDev q, T sigma, T tau, T a, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out, int vec_ok) {
  extern __shared__ unsigned char smem_raw[];
  T* sf = reinterpret_cast<T*>(smem_raw);  // 1024 field entries
  T* sh = sf + 1024;                        // 2^N x 2^N dot matrix
  const int nd = 1 << q.N;
  const T* ft = Tab<T>::qsun(q);
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) sf[i] = ft[i];
  for (int i = threadIdx.x; i < nd * nd; i += blockDim.x) sh[i] = (T)q.hdot[i];
  __syncthreads();
  const uint32_t omask = (1u << q.L) - 1u;
  const int64_t per_block = (int64_t)blockDim.x * ROWS;
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < q.D;
       base += (int64_t)gridDim.x * per_block) {
    const int64_t r0 = base + (int64_t)threadIdx.x * ROWS;
    if (r0 >= q.D) continue;
    const bool full = vec_ok && (r0 + ROWS <= q.D);
    T vv[ROWS], bo[ROWS], bt[ROWS], res[ROWS];
    if (full) {
      vload<T, ROWS>(b1 + r0, bo);
      if (v) vload<T, ROWS>(v + r0, vv);
      if (b2) vload<T, ROWS>(b2 + r0, bt);
    } else {
#pragma unroll
      for (int j = 0; j < ROWS; ++j) {
        const bool in = r0 + j < q.D;
        bo[j] = in ? b1[r0 + j] : T(0);
        vv[j] = (in && v) ? v[r0 + j] : T(0);
        bt[j] = (in && b2) ? b2[r0 + j] : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      T o = 0;
      const int64_t r = r0 + j;
      if (r < q.D) {
        const uint32_t idx = (uint32_t)r;
        const uint32_t d = idx >> q.L, ob = idx & omask;
        const T* hrow = sh + d * nd;
        T acc = ((T)q.c0 + field_sum(sf, ob)) * bo[j];
        for (int dp = 0; dp < nd; ++dp) {
          const uint32_t col = ((uint32_t)dp << q.L) | ob;
          acc += hrow[dp] * (dp == (int)d ? bo[j] : b1[col]);
        }
        for (int jj = 0; jj < q.L; ++jj) acc += (T)q.ray_amp[jj] * b1[idx ^ q.ray_mask[jj]];
        o = sigma * acc + tau * bo[j];
        if (v) o += a * vv[j];
        if (b2) o -= bt[j];
      }
      res[j] = o;
    }
    if (full) {
      vstore<T, ROWS>(out + r0, res);
    } else {
#pragma unroll
      for (int j = 0; j < ROWS; ++j)
        if (r0 + j < q.D) out[r0 + j] = res[j];
    }
  }
}

// -------------------------------------------------------- CSR kernel ----
// Each block owns a run of rows whose off-diagonal entries (at most
// kCsrStage) are first staged into LDS with coalesced loads; each lane then
// walks its rows out of LDS and gathers b1.  A row longer than the stage is
// a block of its own and is reduced across the block from global memory.
constexpr int kCsrStage = 3072;
constexpr int kCsrRowsPerBlock = 512;

template <typename T>
__device__ __forceinline__ T block_sum(T x, T* red) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = x;
  __syncthreads();
  T tot = 0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) tot += red[i];
  return tot;
}

template <typename T, bool MAPPED>
__global__ __launch_bounds__(256) void k_csr_step(
    CsrDev m, T sigma, T tau, T a, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out) {
  // the mapped variant stages one-byte codes instead of values, which
  // leaves room for more workgroups per CU
  using Stage = std::conditional_t<MAPPED, uint8_t, T>;
  __shared__ int32_t scol[kCsrStage];
  __shared__ Stage sval[kCsrStage];
  __shared__ T red[8];
  __shared__ T stab[MAPPED ? 256 : 1];  // value table of an optimized mapping
  const int64_t blk = blockIdx.x;
  const int64_t rb = m.blk_row[blk], re = m.blk_row[blk + 1];
  const int64_t z0 = m.rowptr[rb], z1 = m.rowptr[re];
  const T* val = Tab<T>::val(m);
  const T* dia = Tab<T>::diag(m);
  if constexpr (MAPPED) {
    const T* vg = Tab<T>::vtab(m);
    for (int i = threadIdx.x; i < m.ncode; i += blockDim.x) stab[i] = vg[i];
    __syncthreads();
  }
  const T* vt = stab;
  if (z1 - z0 <= kCsrStage) {
    for (int64_t i = threadIdx.x; i < z1 - z0; i += blockDim.x) {
      scol[i] = m.col[z0 + i];
      if constexpr (MAPPED)
        sval[i] = m.ncode == 1 ? (uint8_t)0 : m.code[z0 + i];
      else
        sval[i] = val[z0 + i];
    }
    __syncthreads();
    for (int64_t r = rb + threadIdx.x; r < re; r += blockDim.x) {
      const int64_t e0 = m.rowptr[r] - z0, e1 = m.rowptr[r + 1] - z0;
      const T bo = b1[r];
      T acc = dia[r] * bo;
      for (int64_t e = e0; e < e1; ++e) {
        T x;
        if constexpr (MAPPED)
          x = vt[sval[e]];
        else
          x = sval[e];
        acc += x * b1[scol[e]];
      }
      T o = sigma * acc + tau * bo;
      if (v) o += a * v[r];
      if (b2) o -= b2[r];
      out[r] = o;
    }
  } else {
    // a single long row
    T part = 0;
    for (int64_t e = z0 + threadIdx.x; e < z1; e += blockDim.x)
      part += csr_value<T, MAPPED>(m, val, vt, e) * b1[m.col[e]];
    const T tot = block_sum(part, red);
    if (threadIdx.x == 0) {
      const T bo = b1[rb];
      T o = sigma * (tot + dia[rb] * bo) + tau * bo;
      if (v) o += a * v[rb];
      if (b2) o -= b2[rb];
      out[rb] = o;
    }
  }
}

// ------------------------------------------------------------ dispatch ----

static int grid_cap(const polfed_op* op) {
  return std::max(1, op->ctx->n_cu) * 8;
}

static bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

template <typename T>
void op_step(hipStream_t s, const polfed_op* op, T sigma, T tau, T a,
             const T* v, const T* b1, const T* b2, T* out) {
  if (op->D == 0) return;
  if (op->storage == POLFED_CSR) {
    CsrDev m = op->csr();
    if (m.ncode > 0)
      hipLaunchKernelGGL((k_csr_step<T, true>), dim3((unsigned)m.nblk), dim3(256), 0, s, m, sigma,
                         tau, a, v, b1, b2, out);
    else
      hipLaunchKernelGGL((k_csr_step<T, false>), dim3((unsigned)m.nblk), dim3(256), 0, s, m,
                         sigma, tau, a, v, b1, b2, out);
    HIPC(hipGetLastError());
    return;
  }
  const int vec_ok = aligned16(b1) && aligned16(out) && (!v || aligned16(v)) &&
                     (!b2 || aligned16(b2));
  constexpr int ROWS = sizeof(T) == 8 ? 4 : 8;
  const int64_t tiles = (op->D + 256 * ROWS - 1) / (256 * ROWS);
  const unsigned grid = (unsigned)std::min<int64_t>(tiles, grid_cap(op));
  if (op->model == Model::Chain) {
    if (chain_split_step<T>(s, op, sigma, tau, a, v, b1, b2, out)) return;
    hipLaunchKernelGGL((k_chain_step<T, ROWS>), dim3(grid), dim3(256), 0, s,
                       op->chain(), sigma, tau, a, v, b1, b2, out, vec_ok);
  } else if (op->model == Model::Qrem) {
    qrem_step<T>(s, op, sigma, tau, a, v, b1, b2, out);
    return;
  } else if (op->model == Model::Qsun) {
    constexpr int QROWS = sizeof(T) == 8 ? 2 : 4;
    const int64_t qt = (op->D + 256 * QROWS - 1) / (256 * QROWS);
    const unsigned qg = (unsigned)std::min<int64_t>(qt, grid_cap(op));
    const size_t nd = (size_t)1 << op->N_dot;
    const size_t shm = (1024 + nd * nd) * sizeof(T);
    hipLaunchKernelGGL((k_qsun_step<T, QROWS>), dim3(qg), dim3(256), shm, s,
                       op->qsun(), sigma, tau, a, v, b1, b2, out, vec_ok);
  } else {
    fail(POLFED_ERR_INVALID, "operator has no matrix-free form; use CSR storage");
  }
  HIPC(hipGetLastError());
}

template void op_step<double>(hipStream_t, const polfed_op*, double, double,
                              double, const double*, const double*,
                              const double*, double*);
template void op_step<float>(hipStream_t, const polfed_op*, float, float, float,
                             const float*, const float*, const float*, float*);

void op_tune(hipStream_t s, const polfed_op* op, bool fp32) {
  if (op->D == 0 || op->storage == POLFED_CSR) return;
  const int pi = fp32 ? 1 : 0;
  // (the QREM tuner skips chains shorter than 12 sites)
  const bool untuned = op->model == Model::Qrem    ? (op->tuned[pi] < 1 && op->L >= 12)
                       : op->model == Model::Chain ? (op->tuned[pi] < 0 && op->split_nseg > 0)
                                                   : false;
  if (!untuned) return;
  const size_t bytes = (size_t)op->D * (fp32 ? sizeof(float) : sizeof(double));
  DevBuf b1(bytes), out(bytes);
  HIPC(hipMemsetAsync(b1.get(), 0, bytes, s));
  if (fp32)
    op_step<float>(s, op, 0.0f, 0.0f, 0.0f, nullptr, b1.as<float>(), nullptr, out.as<float>());
  else
    op_step<double>(s, op, 0.0, 0.0, 0.0, nullptr, b1.as<double>(), nullptr, out.as<double>());
  HIPC(hipStreamSynchronize(s));
}

// ------------------------------------------------------------ moments ----
// Per row: diag and (diag^2 + sum of squared off-diagonal entries).

__device__ __forceinline__ void block_sum2(double& x, double& y, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    x += __shfl_down(x, off, 64);
    y += __shfl_down(y, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wid] = x;
    red[2 * wid + 1] = y;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sx = 0, sy = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      sx += red[2 * i];
      sy += red[2 * i + 1];
    }
    x = sx;
    y = sy;
  }
}

__global__ __launch_bounds__(256) void k_moments_chain(ChainDev c, double* part) {
  __shared__ double red[16];
  __shared__ uint32_t sB[kBinomN * kBinomN];
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += blockDim.x) sB[i] = c.binom[i];
  __syncthreads();
  double s1 = 0, s2 = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < c.D;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s = unrank_lds((uint32_t)r, c.L, c.N, sB);
    const int L = c.L;
    const uint32_t top = s >> (L - 1);
    const int n11 = __popc(s & (s >> 1)) + (c.periodic ? (int)(top & s & 1u) : 0);
    const double dg = c.vzz * n11 + c.c0 + field_sum(c.ftab, s);
    const int nhop = __popc((s ^ (s >> 1)) & ((1u << (L - 1)) - 1u));
    const int npb = (c.periodic && ((top ^ s) & 1u)) ? 1 : 0;
    s1 += dg;
    s2 += dg * dg + nhop * c.t_in * c.t_in + npb * c.t_pb * c.t_pb;
  }
  block_sum2(s1, s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

__global__ __launch_bounds__(256) void k_moments_qsun(QsunDev q, double* part) {
  __shared__ double red[16];
  const int nd = 1 << q.N;
  double off2 = 0;
  for (int j = 0; j < q.L; ++j) off2 += q.ray_amp[j] * q.ray_amp[j];
  double s1 = 0, s2 = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < q.D;
       r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t idx = (uint32_t)r;
    const uint32_t d = idx >> q.L, ob = idx & ((1u << q.L) - 1u);
    const double dg = q.hdot[d * nd + d] + q.c0 + field_sum(q.ftab, ob);
    double o2 = off2;
    for (int dp = 0; dp < nd; ++dp)
      if (dp != (int)d) o2 += q.hdot[d * nd + dp] * q.hdot[d * nd + dp];
    s1 += dg;
    s2 += dg * dg + o2;
  }
  block_sum2(s1, s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

__global__ __launch_bounds__(256) void k_moments_csr(CsrDev m, double* part) {
  __shared__ double red[16];
  double s1 = 0, s2 = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m.D;
       r += (int64_t)gridDim.x * blockDim.x) {
    const double dg = m.diag[r];
    double o2 = 0;
    for (int64_t e = m.rowptr[r]; e < m.rowptr[r + 1]; ++e) o2 += m.val[e] * m.val[e];
    s1 += dg;
    s2 += dg * dg + o2;
  }
  block_sum2(s1, s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

__global__ void k_sum_pairs(const double* part, int64_t n, double* out) {
  __shared__ double red[16];
  double x = 0, y = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    x += part[2 * i];
    y += part[2 * i + 1];
  }
  block_sum2(x, y, red);
  if (threadIdx.x == 0) {
    out[0] = x;
    out[1] = y;
  }
}

void op_moments(hipStream_t s, const polfed_op* op, double* d_two, double* partial,
                int64_t npart) {
  const unsigned g = (unsigned)std::max<int64_t>(
      1, std::min<int64_t>(npart, (op->D + 255) / 256));
  if (op->model == Model::Qrem) {
    // exact moments, summed on the host when the energies were uploaded
    HIPC(hipMemcpyAsync(d_two, op->qrem_tr, 2 * sizeof(double), hipMemcpyHostToDevice, s));
    return;
  }
  if (op->storage == POLFED_CSR || op->model == Model::Csr) {
    hipLaunchKernelGGL(k_moments_csr, dim3(g), dim3(256), 0, s, op->csr(), partial);
  } else if (op->model == Model::Chain) {
    hipLaunchKernelGGL(k_moments_chain, dim3(g), dim3(256), 0, s, op->chain(), partial);
  } else {
    hipLaunchKernelGGL(k_moments_qsun, dim3(g), dim3(256), 0, s, op->qsun(), partial);
  }
  HIPC(hipGetLastError());
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, s, partial, (int64_t)g, d_two);
  HIPC(hipGetLastError());
}

// ---------------------------------------------------- CSR materialization ----

__global__ void k_count_chain(ChainDev c, int32_t* cnt) {
  __shared__ uint32_t sB[kBinomN * kBinomN];
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += blockDim.x) sB[i] = c.binom[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.D) return;
  const uint32_t s = unrank_lds((uint32_t)r, c.L, c.N, sB);
  const uint32_t top = s >> (c.L - 1);
  int n = __popc((s ^ (s >> 1)) & ((1u << (c.L - 1)) - 1u));
  if (c.periodic && ((top ^ s) & 1u)) ++n;
  cnt[r] = n;
}

__device__ void sort_row(int32_t* col, double* val, int n) {
  for (int i = 1; i < n; ++i) {
    int32_t c = col[i];
    double x = val[i];
    int j = i - 1;
    while (j >= 0 && col[j] > c) {
      col[j + 1] = col[j];
      val[j + 1] = val[j];
      --j;
    }
    col[j + 1] = c;
    val[j + 1] = x;
  }
}

__global__ void k_fill_chain(ChainDev c, const int64_t* rowptr, int32_t* col,
                             double* val, double* diag) {
  __shared__ uint32_t sB[kBinomN * kBinomN];
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += blockDim.x) sB[i] = c.binom[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= c.D) return;
  const int L = c.L;
  const uint32_t s = unrank_lds((uint32_t)r, L, c.N, sB);
  const uint32_t top = s >> (L - 1);
  const int n11 = __popc(s & (s >> 1)) + (c.periodic ? (int)(top & s & 1u) : 0);
  diag[r] = c.vzz * n11 + c.c0 + field_sum(c.ftab, s);
  int32_t* cp = col + rowptr[r];
  double* vp = val + rowptr[r];
  int n = 0, m = 0;
  const uint32_t x = (s ^ (s >> 1)) & ((1u << (L - 1)) - 1u);
  for (int b = 0; b < L - 1; ++b) {
    const uint32_t sb = (s >> b) & 1u;
    if ((x >> b) & 1u) {
      const int32_t d = (int32_t)sB[b * kBinomN + m];
      cp[n] = (int32_t)r + (sb ? d : -d);
      vp[n] = c.t_in;
      ++n;
    }
    m += (int)sb;
  }
  if (c.periodic && ((top ^ s) & 1u)) {
    const uint32_t sp = s ^ (1u | (1u << (L - 1)));
    cp[n] = c.hi_off[sp >> c.Lb] + c.lo_rank[sp & ((1u << c.Lb) - 1u)];
    vp[n] = c.t_pb;
    ++n;
  }
  sort_row(cp, vp, n);
}

__global__ void k_fill_qsun(QsunDev q, const int64_t* rowptr, int32_t* col,
                            double* val, double* diag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= q.D) return;
  const int nd = 1 << q.N;
  const uint32_t idx = (uint32_t)r, d = idx >> q.L, ob = idx & ((1u << q.L) - 1u);
  diag[r] = q.hdot[d * nd + d] + q.c0 + field_sum(q.ftab, ob);
  int32_t* cp = col + rowptr[r];
  double* vp = val + rowptr[r];
  int n = 0;
  for (int dp = 0; dp < nd; ++dp) {
    if (dp == (int)d) continue;
    cp[n] = (int32_t)(((uint32_t)dp << q.L) | ob);
    vp[n] = q.hdot[d * nd + dp];
    ++n;
  }
  for (int j = 0; j < q.L; ++j) {
    cp[n] = (int32_t)(idx ^ q.ray_mask[j]);
    vp[n] = q.ray_amp[j];
    ++n;
  }
  sort_row(cp, vp, n);
}

__global__ void k_d2f(int64_t n, const double* x, float* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

static void csr_blocks(const std::vector<int64_t>& rowptr, int64_t D,
                       std::vector<int64_t>& blk) {
  blk.clear();
  int64_t r = 0;
  blk.push_back(0);
  while (r < D) {
    int64_t e = r, nz = 0;
    while (e < D && e - r < kCsrRowsPerBlock) {
      const int64_t len = rowptr[e + 1] - rowptr[e];
      if (nz + len > kCsrStage) break;
      nz += len;
      ++e;
    }
    if (e == r) e = r + 1;  // a row longer than the LDS stage
    blk.push_back(e);
    r = e;
  }
}

static void finish_csr(polfed_ctx* ctx, polfed_op* op,
                       const std::vector<int64_t>& h_rowptr) {
  hipStream_t s = ctx->stream;
  const int64_t nnz = h_rowptr[op->D];
  op->d_val32.alloc(std::max<int64_t>(nnz, 1) * sizeof(float));
  op->d_diag32.alloc(std::max<int64_t>(op->D, 1) * sizeof(float));
  const unsigned g = 1024;
  if (nnz)
    hipLaunchKernelGGL(k_d2f, dim3(g), dim3(256), 0, s, nnz,
                       op->d_val.as<double>(), op->d_val32.as<float>());
  if (op->D)
    hipLaunchKernelGGL(k_d2f, dim3(g), dim3(256), 0, s, op->D,
                       op->d_diag.as<double>(), op->d_diag32.as<float>());
  HIPC(hipGetLastError());
  std::vector<int64_t> blk;
  csr_blocks(h_rowptr, op->D, blk);
  op->nblk = (int64_t)blk.size() - 1;
  upload(op->d_blk, blk.data(), blk.size(), s);
  op->nnz = nnz;
  op->has_csr = true;
  HIPC(hipStreamSynchronize(s));
}

void materialize_csr(polfed_ctx* ctx, polfed_op* op) {
  if (op->model == Model::Csr || op->has_csr) return;
  REQUIRE(op->model != Model::Qrem, "qrem: no CSR copy is offered (the operator is matrix-free)");
  hipStream_t s = ctx->stream;
  const int64_t D = op->D;
  std::vector<int64_t> rp(D + 1, 0);
  op->d_diag.alloc(std::max<int64_t>(D, 1) * sizeof(double));
  const unsigned g = (unsigned)std::max<int64_t>(1, (D + 255) / 256);
  if (op->model == Model::Chain) {
    DevBuf cnt(std::max<int64_t>(D, 1) * sizeof(int32_t));
    hipLaunchKernelGGL(k_count_chain, dim3(g), dim3(256), 0, s, op->chain(),
                       cnt.as<int32_t>());
    HIPC(hipGetLastError());
    std::vector<int32_t> hc(D);
    if (D) HIPC(hipMemcpyAsync(hc.data(), cnt.get(), D * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int64_t r = 0; r < D; ++r) rp[r + 1] = rp[r] + hc[r];
  } else {
    const int64_t per = ((int64_t)1 << op->N_dot) - 1 + op->L;
    for (int64_t r = 0; r < D; ++r) rp[r + 1] = rp[r] + per;
  }
  const int64_t nnz = rp[D];
  upload(op->d_rowptr, rp.data(), rp.size(), s);
  op->d_col.alloc(std::max<int64_t>(nnz, 1) * sizeof(int32_t));
  op->d_val.alloc(std::max<int64_t>(nnz, 1) * sizeof(double));
  if (op->model == Model::Chain)
    hipLaunchKernelGGL(k_fill_chain, dim3(g), dim3(256), 0, s, op->chain(),
                       op->d_rowptr.as<int64_t>(), op->d_col.as<int32_t>(),
                       op->d_val.as<double>(), op->d_diag.as<double>());
  else
    hipLaunchKernelGGL(k_fill_qsun, dim3(g), dim3(256), 0, s, op->qsun(),
                       op->d_rowptr.as<int64_t>(), op->d_col.as<int32_t>(),
                       op->d_val.as<double>(), op->d_diag.as<double>());
  HIPC(hipGetLastError());
  finish_csr(ctx, op, rp);
}

// --------------------------------------------------------- op creation ----

static void field_tables(const std::vector<double>& f, int nbits,
                         std::vector<double>& tab) {
  tab.assign(1024, 0.0);
  for (int t = 0; t < 4; ++t)
    for (int e = 0; e < 256; ++e) {
      double acc = 0;
      for (int k = 0; k < 8; ++k) {
        const int site = 8 * t + k;
        if (((e >> k) & 1) && site < nbits) acc += f[site];
      }
      tab[t * 256 + e] = acc;
    }
}

static void upload_tables(polfed_op* op, const std::vector<double>& tab) {
  hipStream_t s = op->ctx->stream;
  upload(op->d_ftab, tab.data(), tab.size(), s);
  std::vector<float> tf(tab.begin(), tab.end());
  upload(op->d_ftab32, tf.data(), tf.size(), s);
}

// Chain in occupation form: diag = vzz * n11 + c0 + sum f_i n_i.
static polfed_op* make_chain(polfed_ctx* ctx, int L, int N, int periodic,
                             double t_in, double t_pb, double vzz, double c0,
                             const std::vector<double>& f, const std::string& key) {
  auto op = std::make_unique<polfed_op>();
  op->ctx = ctx;
  op->model = Model::Chain;
  op->L = L;
  op->N = N;
  op->periodic = periodic ? 1 : 0;
  op->D = binom64(L, N);
  op->t_in = t_in;
  op->t_pb = t_pb;
  op->vzz = vzz;
  op->c0 = c0;
  op->site_f = f;
  op->pattern_key = key;
  std::vector<double> tab;
  field_tables(f, L, tab);
  upload_tables(op.get(), tab);
  hipStream_t s = ctx->stream;
  upload(op->d_binom, host_binom(), (size_t)kBinomN * kBinomN, s);
  std::vector<int32_t> hi, lo;
  build_split_rank_tables(L, N, L / 2, hi, lo);
  upload(op->d_hi_off, hi.data(), hi.size(), s);
  upload(op->d_lo_rank, lo.data(), lo.size(), s);
  HIPC(hipStreamSynchronize(s));
  if (L >= 4 && L <= 28) build_chain_split(op.get());
  return op.release();
}

polfed_op* make_xxz(polfed_ctx* ctx, int L, int n_up, double J, double Delta,
                    const double* h, int periodic) {
  REQUIRE(L >= 2 && L <= 32, "XXZ: need 2 <= L <= 32");
  REQUIRE(!periodic || L >= 3, "XXZ: periodic chain needs L >= 3");
  REQUIRE(n_up >= 0 && n_up <= L, "XXZ: need 0 <= n_up <= L");
  REQUIRE(h != nullptr, "XXZ: fields h[L] missing");
  REQUIRE(binom64(L, n_up) < (int64_t(1) << 31), "XXZ: sector too large");
  for (int i = 0; i < L; ++i) REQUIRE(std::isfinite(h[i]), "XXZ: non-finite field");
  REQUIRE(std::isfinite(J) && std::isfinite(Delta), "XXZ: non-finite coupling");
  // S^z_i S^z_j = n_i n_j - (n_i + n_j)/2 + 1/4 and S^z_i = n_i - 1/2.
  std::vector<double> f(L, 0.0);
  double c0 = 0.0;
  const int nb = periodic ? L : L - 1;
  for (int i = 0; i < L; ++i) {
    f[i] += h[i];
    c0 -= 0.5 * h[i];
  }
  for (int b = 0; b < nb; ++b) {
    const int i = b, j = (b + 1) % L;
    f[i] -= 0.5 * J * Delta;
    f[j] -= 0.5 * J * Delta;
    c0 += 0.25 * J * Delta;
  }
  char key[128];
  snprintf(key, sizeof key, "chain:%d:%d:%d:%.17g:%.17g:%.17g", L, n_up, periodic,
           0.5 * J, 0.5 * J, J * Delta);
  return make_chain(ctx, L, n_up, periodic, 0.5 * J, 0.5 * J, J * Delta, c0, f, key);
}

polfed_op* make_tv(polfed_ctx* ctx, int L, int n_part, double t, double V,
                   const double* eps, int periodic) {
  REQUIRE(L >= 2 && L <= 32, "t-V: need 2 <= L <= 32");
  REQUIRE(!periodic || L >= 3, "t-V: periodic chain needs L >= 3");
  REQUIRE(n_part >= 0 && n_part <= L, "t-V: need 0 <= n_part <= L");
  REQUIRE(eps != nullptr, "t-V: on-site energies eps[L] missing");
  REQUIRE(binom64(L, n_part) < (int64_t(1) << 31), "t-V: sector too large");
  for (int i = 0; i < L; ++i) REQUIRE(std::isfinite(eps[i]), "t-V: non-finite eps");
  REQUIRE(std::isfinite(t) && std::isfinite(V), "t-V: non-finite coupling");
  std::vector<double> f(eps, eps + L);
  // Hopping across the periodic bond passes the other n_part - 1 fermions.
  const double sign = ((n_part - 1) % 2 == 0) ? 1.0 : -1.0;
  char key[128];
  snprintf(key, sizeof key, "chain:%d:%d:%d:%.17g:%.17g:%.17g", L, n_part, periodic,
           -t, -t * sign, V);
  return make_chain(ctx, L, n_part, periodic, -t, -t * sign, V, 0.0, f, key);
}

polfed_op* make_qsun(polfed_ctx* ctx, int N, int L, const double* A, double gamma,
                     double g0, double alpha, const double* u, const int32_t* n_of_j,
                     const double* h) {
  REQUIRE(N >= 1 && N <= 6, "qsun: need 1 <= N_dot <= 6");
  REQUIRE(L >= 1 && N + L <= 31 && L <= kQsunMaxL, "qsun: need L >= 1, N_dot + L <= 31");
  REQUIRE(A && u && n_of_j && h, "qsun: missing parameter array");
  const int nd = 1 << N;
  auto op = std::make_unique<polfed_op>();
  op->ctx = ctx;
  op->model = Model::Qsun;
  op->N_dot = N;
  op->L = L;
  op->D = (int64_t)1 << (N + L);
  op->hdot.assign((size_t)nd * nd, 0.0);
  const double scale = gamma / std::sqrt(2.0 * (nd + 1.0));
  for (int i = 0; i < nd; ++i)
    for (int j = 0; j < nd; ++j) {
      REQUIRE(std::isfinite(A[i * nd + j]), "qsun: non-finite A");
      op->hdot[i * nd + j] = scale * (A[i * nd + j] + A[j * nd + i]);
    }
  op->ray_mask.resize(L);
  op->ray_amp.resize(L);
  std::vector<double> f(L);
  double c0 = 0;
  for (int j = 0; j < L; ++j) {
    REQUIRE(n_of_j[j] >= 0 && n_of_j[j] < N, "qsun: n_of_j out of range");
    REQUIRE(std::isfinite(u[j]) && std::isfinite(h[j]), "qsun: non-finite u or h");
    op->ray_mask[j] = (1u << (L + n_of_j[j])) | (1u << j);
    op->ray_amp[j] = 0.25 * g0 * std::pow(alpha, u[j]);
    f[j] = h[j];
    c0 -= 0.5 * h[j];
  }
  op->c0 = c0;
  op->site_f = f;
  op->pattern_key = "";  // batching of qsun realizations is not offered
  std::vector<double> tab;
  field_tables(f, L, tab);
  upload_tables(op.get(), tab);
  upload(op->d_hdot, op->hdot.data(), op->hdot.size(), ctx->stream);
  HIPC(hipStreamSynchronize(ctx->stream));
  return op.release();
}

// The optimized mapping (Sec. 5.6): the off-diagonal values of a CSR copy
// are replaced by a table of their distinct values and one byte per entry
// (none when all are equal), cutting the matrix stream from 12 to 5 (or 4)
// bytes per entry.  More than 256 distinct values leave the operator as it
// is.  Returns the number of distinct values.
int optimize_mapping(polfed_ctx* ctx, polfed_op* op) {
  REQUIRE(op->has_csr, "optimize_mapping: the operator has no CSR copy");
  hipStream_t s = ctx->stream;
  const int64_t nnz = op->nnz;
  std::vector<double> v((size_t)std::max<int64_t>(nnz, 0));
  if (nnz) HIPC(hipMemcpyAsync(v.data(), op->d_val.get(), nnz * sizeof(double),
                               hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  std::vector<double> tab;
  std::vector<uint8_t> code((size_t)std::max<int64_t>(nnz, 0));
  for (int64_t e = 0; e < nnz; ++e) {
    int c = 0;
    while (c < (int)tab.size() && std::memcmp(&tab[c], &v[e], sizeof(double)) != 0) ++c;
    if (c == (int)tab.size()) {
      if (tab.size() == 256) return 257;  // too many: unchanged
      tab.push_back(v[e]);
    }
    code[e] = (uint8_t)c;
  }
  if (tab.empty()) return 0;
  std::vector<float> tab32(tab.begin(), tab.end());
  upload(op->d_vtab, tab.data(), tab.size(), s);
  upload(op->d_vtab32, tab32.data(), tab32.size(), s);
  if (tab.size() > 1) upload(op->d_code, code.data(), code.size(), s);
  HIPC(hipStreamSynchronize(s));
  op->ncode = (int)tab.size();
  return op->ncode;
}

polfed_op* make_csr(polfed_ctx* ctx, int64_t D, const int64_t* rowptr, const int32_t* col,
                    const double* val);

// Spin-1/2 chain with couplings of range 1..R (eqs. xxz, j1j2, j1j2j3 of
// App. A) in the sector of N up spins, built on the host as a CSR matrix:
// a bond (i, i + r) flips the antiparallel pair with amplitude J_r / 2 and
// adds J_r Delta_r (b_i - 1/2)(b_j - 1/2) to the diagonal.
polfed_op* make_spin_chain(polfed_ctx* ctx, int L, int N, int R, const double* J,
                           const double* Delta, const double* h, int periodic) {
  REQUIRE(L >= 2 && L <= 24 && N >= 0 && N <= L, "spin chain: need 2 <= L <= 24, 0 <= N <= L");
  REQUIRE(R >= 1 && R <= 8 && J && Delta && h, "spin chain: need 1 <= R <= 8 and parameters");
  REQUIRE(!periodic || L > 2 * R, "spin chain: periodic bonds need L > 2 R");
  const int64_t D = binom64(L, N);
  std::vector<uint32_t> st;
  st.reserve((size_t)D);
  for (uint32_t x = 0; x < (1u << L); ++x)
    if (__builtin_popcount(x) == N) st.push_back(x);
  std::vector<int64_t> rp((size_t)D + 1, 0);
  std::vector<int32_t> col;
  std::vector<double> val;
  col.reserve((size_t)D * (R * L + 1));
  val.reserve((size_t)D * (R * L + 1));
  for (int64_t k = 0; k < D; ++k) {
    const uint32_t x = st[(size_t)k];
    double dg = 0;
    for (int i = 0; i < L; ++i) dg += h[i] * ((double)((x >> i) & 1u) - 0.5);
    for (int r = 1; r <= R; ++r)
      for (int i = 0; i < L; ++i) {
        int j = i + r;
        if (j >= L) {
          if (!periodic) continue;
          j -= L;
        }
        const int bi = (x >> i) & 1u, bj = (x >> j) & 1u;
        dg += J[r - 1] * Delta[r - 1] * ((double)bi - 0.5) * ((double)bj - 0.5);
        if (bi != bj) {
          const uint32_t y = x ^ ((1u << i) | (1u << j));
          const int64_t c = std::lower_bound(st.begin(), st.end(), y) - st.begin();
          col.push_back((int32_t)c);
          val.push_back(0.5 * J[r - 1]);
        }
      }
    col.push_back((int32_t)k);
    val.push_back(dg);
    rp[(size_t)k + 1] = (int64_t)col.size();
  }
  polfed_op* op = make_csr(ctx, D, rp.data(), col.data(), val.data());
  op->L = L;
  op->N = N;
  op->periodic = periodic;
  return op;
}

polfed_op* make_csr(polfed_ctx* ctx, int64_t D, const int64_t* rowptr,
                    const int32_t* col, const double* val) {
  REQUIRE(D >= 0 && D < (int64_t(1) << 31), "CSR: need 0 <= D < 2^31");
  REQUIRE(rowptr && (D == 0 || (col && val)) , "CSR: missing array");
  REQUIRE(rowptr[0] == 0, "CSR: rowptr[0] must be 0");
  auto op = std::make_unique<polfed_op>();
  op->ctx = ctx;
  op->model = Model::Csr;
  op->storage = POLFED_CSR;
  op->D = D;
  std::vector<int64_t> rp(D + 1, 0);
  std::vector<int32_t> c;
  std::vector<double> v, dg(D, 0.0);
  c.reserve(rowptr[D]);
  v.reserve(rowptr[D]);
  for (int64_t r = 0; r < D; ++r) {
    REQUIRE(rowptr[r + 1] >= rowptr[r], "CSR: rowptr not monotone");
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      REQUIRE(col[e] >= 0 && col[e] < D, "CSR: column index out of range");
      REQUIRE(std::isfinite(val[e]), "CSR: non-finite value");
      if (col[e] == r) {
        dg[r] += val[e];
      } else {
        c.push_back(col[e]);
        v.push_back(val[e]);
      }
    }
    rp[r + 1] = (int64_t)c.size();
  }
  hipStream_t s = ctx->stream;
  upload(op->d_rowptr, rp.data(), rp.size(), s);
  upload(op->d_col, c.data(), c.size(), s);
  upload(op->d_val, v.data(), v.size(), s);
  upload(op->d_diag, dg.data(), dg.size(), s);
  finish_csr(ctx, op.get(), rp);
  return op.release();
}

}  // namespace polfed

// ------------------------------------------------- device views of ops ----

polfed::ChainDev polfed_op::chain() const {
  polfed::ChainDev c{};
  c.L = L;
  c.N = N;
  c.periodic = periodic;
  c.Lb = L / 2;
  c.D = D;
  c.t_in = t_in;
  c.t_pb = t_pb;
  c.vzz = vzz;
  c.c0 = c0;
  c.ftab = d_ftab.as<double>();
  c.ftab32 = d_ftab32.as<float>();
  c.binom = d_binom.as<uint32_t>();
  c.hi_off = d_hi_off.as<int32_t>();
  c.lo_rank = d_lo_rank.as<int32_t>();
  return c;
}

polfed::QsunDev polfed_op::qsun() const {
  polfed::QsunDev q{};
  q.N = N_dot;
  q.L = L;
  q.D = D;
  q.c0 = c0;
  q.hdot = d_hdot.as<double>();
  q.ftab = d_ftab.as<double>();
  q.ftab32 = d_ftab32.as<float>();
  for (int j = 0; j < L && j < polfed::kQsunMaxL; ++j) {
    q.ray_mask[j] = ray_mask[j];
    q.ray_amp[j] = ray_amp[j];
  }
  return q;
}

polfed::CsrDev polfed_op::csr() const {
  polfed::CsrDev m{};
  m.D = D;
  m.rowptr = d_rowptr.as<int64_t>();
  m.col = d_col.as<int32_t>();
  m.val = d_val.as<double>();
  m.val32 = d_val32.as<float>();
  m.diag = d_diag.as<double>();
  m.diag32 = d_diag32.as<float>();
  m.blk_row = d_blk.as<int64_t>();
  m.nblk = nblk;
  m.ncode = ncode;
  m.code = d_code.as<uint8_t>();
  m.vtab = d_vtab.as<double>();
  m.vtab32 = d_vtab32.as<float>();
  return m;
}

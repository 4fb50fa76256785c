// Device helpers shared by the single- and multi-column chain kernels.
#pragma once
#include "internal.hpp"

namespace polfed {

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Orders the LDS accesses of a wavefront around a staging step.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-uniform data of one segment (see the record layout).
template <int NH>
struct SegRec {
  int row0, len, lidx, flags, n_idle_h, d_join, d_pbc;
  double dhi;
  int dh[NH > 0 ? NH : 1];
};

template <int NH>
__device__ __forceinline__ SegRec<NH> load_rec(const int32_t* rec) {
  SegRec<NH> r;
  r.row0 = uniform(rec[0]);
  r.len = uniform(rec[1]);
  r.lidx = uniform(rec[2]);
  r.flags = uniform(rec[3]);
  r.n_idle_h = uniform(rec[4]);
  r.d_join = uniform(rec[5]);
  r.d_pbc = uniform(rec[6]);
  int dw[2] = {uniform(rec[8]), uniform(rec[9])};
  __builtin_memcpy(&r.dhi, dw, sizeof(double));
#pragma unroll
  for (int b = 0; b < NH; ++b) r.dh[b] = uniform(rec[10 + b]);
  return r;
}

// Buffer accesses: a 128-bit resource for each vector, a per-lane 32-bit
// byte offset (VGPR) and a wave-uniform byte offset (SGPR), so gathers at
// uniform row offsets need no per-lane address arithmetic.  Accesses beyond
// the resource's size return 0 / are dropped by the hardware.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kAuxNT = 2;  // non-temporal cache policy

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
template <typename T, int AUX = 0>
__device__ __forceinline__ T bload(rsrc_t r, uint32_t vo, uint32_t so) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, AUX));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, AUX));
}
// Two consecutive elements in one 16-byte access (8-byte alignment suffices
// for buffer accesses).
template <typename T, int AUX = 0>
__device__ __forceinline__ void bload2(rsrc_t r, uint32_t vo, uint32_t so, T& x0, T& x1) {
  if constexpr (sizeof(T) == 8) {
    using d2 = __attribute__((ext_vector_type(2))) double;
    const d2 d = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, AUX));
    x0 = d[0];
    x1 = d[1];
  } else {
    using f2 = __attribute__((ext_vector_type(2))) float;
    const f2 d = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, AUX));
    x0 = d[0];
    x1 = d[1];
  }
}
template <int AUX, typename T>
__device__ __forceinline__ void bstore2(T x0, T x1, rsrc_t r, uint32_t vo, uint32_t so) {
  if constexpr (sizeof(T) == 8) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned int;
    using d2 = __attribute__((ext_vector_type(2))) double;
    const d2 d = {x0, x1};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, d), r, vo, so, AUX);
  } else {
    using u2 = __attribute__((ext_vector_type(2))) unsigned int;
    using f2 = __attribute__((ext_vector_type(2))) float;
    const f2 d = {x0, x1};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, d), r, vo, so, AUX);
  }
}
template <int AUX, typename T>
__device__ __forceinline__ void bstore(T x, rsrc_t r, uint32_t vo, uint32_t so) {
  using u2 = __attribute__((ext_vector_type(2))) unsigned int;
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, vo, so, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, vo, so, AUX);
}

}  // namespace polfed

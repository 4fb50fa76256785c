// Multi-column fused Clenshaw step for a batch of chain operators that share
// the off-diagonal pattern (same L, N, boundary and couplings) and differ in
// their on-site fields.  Column c of every vector block belongs to operator
// c; the step computes, for each column,
//     out_c = a_c v_c + h sigma_c (H_c b1_c) + h tau_c b1_c - b2_c
// with h = 1, or 1/2 on the closing Clenshaw step.
//
// The row decoding of the split layout (low part, neighbour positions,
// activity of the joining and periodic bonds, the interaction part of the
// diagonal) is done once per segment and reused by every column.  Each lane
// holds two adjacent rows, so the coalesced accesses move both in one
// 16-byte instruction.  Only the
// field part of the diagonal is per column: the sum over the low bits comes
// from two 32-entry LDS tables per column (bits 0-4 and 5-9) and the sum over
// the high bits plus the constant is one wave-uniform value per segment and
// column.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>

#include "chain_dev.hpp"
#include "internal.hpp"

namespace polfed {

template <typename T, int L>
__global__ __launch_bounds__(256) void k_chain_split_batch(
    ChainSplitDev c, int nb, int col0, int ncols, int64_t ld, T half,
    const T* __restrict__ fab, const T* __restrict__ dseg, const T* __restrict__ sc,
    const T* __restrict__ acoef, const T* __restrict__ v, const T* __restrict__ b1,
    const T* b2, T* out, int nxcd, const int32_t* __restrict__ recs) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int Lh = L - Lb;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = Lh - 1;
  constexpr int NL = Lb - 1;
  constexpr int SPL2 = kChainStageRows / 128;  // staged row pairs per lane
  constexpr int BLOB = chain_blob_bytes(NLO, (int)sizeof(T));
  constexpr int CHUNKS = BLOB / 16;
  constexpr uint32_t TB = sizeof(T);
  using u4 = __attribute__((ext_vector_type(4))) uint32_t;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  {
    const u4* src = reinterpret_cast<const u4*>(sizeof(T) == 8 ? c.blob64 : c.blob32);
    u4* dst = reinterpret_cast<u4*>(smem);
    constexpr int PER = (CHUNKS + 255) / 256;
    u4 tmp[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < CHUNKS) tmp[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < CHUNKS) dst[i] = tmp[k];
    }
  }
  T* s_fab = reinterpret_cast<T*>(smem + BLOB);
  for (int i = threadIdx.x; i < ncols * 64; i += 256) s_fab[i] = fab[(int64_t)col0 * 64 + i];
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(smem + 16 * NLO + TB * NLO);
  T* stage = s_fab + ncols * 64 + (threadIdx.x >> 6) * kChainStageRows;
  __syncthreads();

  const int xcd = blockIdx.x % nxcd;
  const int blocks_x = gridDim.x / nxcd;
  const int64_t s_begin = c.nseg * xcd / nxcd, s_end = c.nseg * (xcd + 1) / nxcd;
  const int wpb = blockDim.x >> 6;
  const int64_t wstride = (int64_t)blocks_x * wpb;
  const int lane = threadIdx.x & 63;
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  const uint32_t vbytes = (uint32_t)(c.D * TB);
  int64_t si = s_begin + (int64_t)(blockIdx.x / nxcd) * wpb + uniform(threadIdx.x >> 6);
  if (si >= s_end) return;
  for (; si < s_end; si += wstride) {
    const SegRec<NH> cur = load_rec<NH>(recs + (int64_t)uniform((int)si) * kChainRecWords);
    const int hi0 = cur.flags & 1, hitop = (cur.flags >> 1) & 1;
    const int bs = (cur.flags >> 2) & 1023, st = (cur.flags >> 12) & 1023;
    const int blk0 = cur.row0 - st;
    const uint32_t so_blk = (uint32_t)blk0 * TB, so_row = (uint32_t)cur.row0 * TB;
    // per-row decoding shared by all columns: lane l holds the adjacent rows
    // 2l and 2l + 1 (clamped into the segment)
    int jj[2], lo[2], gj[2], gp[2];
    u4 np[2];
    bool act_j[2], act_p[2];
    T zz[2], nidle[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      jj[i] = min(2 * lane + i, cur.len - 1);
      const int l = s_lo[cur.lidx + jj[i]];
      lo[i] = l;
      np[i] = s_np[l];
      act_j[i] = ((l >> (Lb - 1)) & 1) != hi0;
      act_p[i] = c.periodic && ((l & 1) != hitop);
      const int rj = (int)((np[i][2] >> 8) & 255u);
      const int rp = (int)((np[i][2] >> 16) & 255u);
      gj[i] = blk0 + cur.d_join + rj;
      gp[i] = blk0 + cur.d_pbc + rp;
      const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
      nidle[i] = (T)(NL - __popc(xlo));
      const int n11x = ((l >> (Lb - 1)) & 1 & hi0) + (c.periodic ? (hitop & l & 1) : 0);
      zz[i] = vzz * (T)(__popc(l & (l >> 1)) + n11x);
    }
    const uint32_t pair_off = (uint32_t)(2 * lane) * TB;
    const int r0 = 2 * lane;
#pragma unroll 1
    for (int cc = 0; cc < ncols; ++cc) {
      const int col = col0 + cc;
      const int64_t coff = (int64_t)col * ld;
      const T sig = sc[col] * half, ta = sc[nb + col] * half;
      const T ac = acoef ? acoef[col] : T(0);
      const T dsg = dseg[si * nb + col];
      const rsrc_t rb1 = make_rsrc(b1 + coff, vbytes);
      const rsrc_t rv = make_rsrc(v ? v + coff : nullptr, v ? vbytes : 0);
      const rsrc_t rb2 = make_rsrc(b2 ? b2 + coff : nullptr, b2 ? vbytes : 0);
      const rsrc_t rout = make_rsrc(out + coff, vbytes);
      T sg[SPL2][2];
#pragma unroll
      for (int m = 0; m < SPL2; ++m) {
        if (128 * m < bs)
          bload2<T>(rb1, pair_off + (uint32_t)(128 * m) * TB, so_blk, sg[m][0], sg[m][1]);
        else
          sg[m][0] = sg[m][1] = T(0);
      }
      T g_hi[NH > 0 ? NH : 1][2], g_j[2], g_p[2], vv[2], bt[2];
#pragma unroll
      for (int b = 0; b < NH; ++b) {
        if (cur.dh[b] != 0)
          bload2<T>(rb1, pair_off, (uint32_t)(cur.row0 + cur.dh[b]) * TB, g_hi[b][0], g_hi[b][1]);
        else
          g_hi[b][0] = g_hi[b][1] = T(0);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        g_j[i] = act_j[i] ? bload<T>(rb1, (uint32_t)gj[i] * TB, 0) : T(0);
        g_p[i] = act_p[i] ? bload<T>(rb1, (uint32_t)gp[i] * TB, 0) : T(0);
      }
      if (v)
        bload2<T, kAuxNT>(rv, pair_off, so_row, vv[0], vv[1]);
      else
        vv[0] = vv[1] = T(0);
      if (b2)
        bload2<T, kAuxNT>(rb2, pair_off, so_row, bt[0], bt[1]);
      else
        bt[0] = bt[1] = T(0);
      wave_sync();  // the previous column's (or segment's) LDS reads are done
#pragma unroll
      for (int m = 0; m < SPL2; ++m) {
        const int r = 128 * m + 2 * lane;
        if (r < bs) {
          stage[r] = sg[m][0];
          if (r + 1 < bs) stage[r + 1] = sg[m][1];
        }
      }
      wave_sync();
      const T* fa = s_fab + cc * 64;
      T o[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int l = lo[i];
        const T bo = stage[st + jj[i]];
        T hop = 0;
#pragma unroll
        for (int b = 0; b < NL; ++b) hop += stage[(np[i][b >> 2] >> (8 * (b & 3))) & 255u];
#pragma unroll
        for (int b = 0; b < NH; ++b) hop += g_hi[b][i];
        hop -= nidle[i] * bo;
        hop += act_j[i] ? g_j[i] : T(0);
        const T dg = zz[i] + fa[l & 31] + fa[32 + (l >> 5)] + dsg;
        const T acc = dg * bo + t_in * hop + (act_p[i] ? t_pb * g_p[i] : T(0));
        o[i] = sig * acc + ta * bo - bt[i];
        if (v) o[i] += ac * vv[i];
      }
      if (r0 + 1 < cur.len)
        bstore2<kAuxNT>(o[0], o[1], rout, pair_off, so_row);
      else if (r0 < cur.len)
        bstore<kAuxNT>(o[0], rout, pair_off, so_row);
    }
  }
}

// Interleaved multi-column step.  The recurrence blocks are stored with the
// columns of a row side by side: element (row r, column c) at X[r nb + c].
// A wavefront takes one (segment, column group) item, a group being the
// G = 16 / sizeof(T) columns (2 FP64, 4 FP32) that one 16-byte access moves
// for a row, and lane l holds rows l and l + 64 of the segment.  So every
// gather (uniform-offset high-part hops, the masked joining and periodic
// hops, the block staged in LDS for the low-part hops) serves G columns at
// once, and the columns of a batch run side by side on different
// wavefronts instead of one after another.  The start vectors v may be
// column-major (VCM, column stride D: the caller's block) and the output of
// the closing step column-major too (OCM).  A last group narrower than G
// (nb not a multiple of G) takes element-wise accesses.
template <typename T>
struct Grp {
  T x[16 / sizeof(T)];
};

template <typename T>
__device__ __forceinline__ Grp<T> gload(rsrc_t r, uint32_t row_bytes, uint32_t so, int w) {
  constexpr int G = 16 / sizeof(T);
  Grp<T> g;
  if (w == G) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned int;
    const u4 d = __builtin_amdgcn_raw_buffer_load_b128(r, row_bytes, so, 0);
    __builtin_memcpy(&g, &d, 16);
  } else {
#pragma unroll
    for (int c = 0; c < G; ++c)
      g.x[c] = c < w ? bload<T>(r, row_bytes + (uint32_t)(c * sizeof(T)), so) : T(0);
  }
  return g;
}

template <typename T>
__device__ __forceinline__ void gstore(const Grp<T>& g, rsrc_t r, uint32_t row_bytes, uint32_t so,
                                       int w) {
  constexpr int G = 16 / sizeof(T);
  if (w == G) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned int;
    u4 d;
    __builtin_memcpy(&d, &g, 16);
    __builtin_amdgcn_raw_buffer_store_b128(d, r, row_bytes, so, kAuxNT);
  } else {
#pragma unroll
    for (int c = 0; c < G; ++c)
      if (c < w) bstore<kAuxNT>(g.x[c], r, row_bytes + (uint32_t)(c * sizeof(T)), so);
  }
}

template <typename T, int L, bool VCM, bool OCM>
__global__ __launch_bounds__(256) void k_chain_ilv(
    ChainSplitDev c, int nb, T half, const T* __restrict__ fab, const T* __restrict__ dseg,
    const T* __restrict__ sc, const T* __restrict__ acoef, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out, int ngrp, int nxcd,
    const int32_t* __restrict__ recs) {
  constexpr int G = 16 / (int)sizeof(T);
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int Lh = L - Lb;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = Lh - 1;
  constexpr int NL = Lb - 1;
  constexpr int BLOB = chain_blob_bytes(NLO, (int)sizeof(T));
  constexpr int CHUNKS = BLOB / 16;
  constexpr uint32_t TB = sizeof(T);
  using u4 = __attribute__((ext_vector_type(4))) uint32_t;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  for (int i = threadIdx.x; i < CHUNKS; i += 256)
    reinterpret_cast<u4*>(smem)[i] =
        reinterpret_cast<const u4*>(sizeof(T) == 8 ? c.blobl64 : c.blobl32)[i];
  T* s_fab = reinterpret_cast<T*>(smem + BLOB);
  for (int i = threadIdx.x; i < nb * 64; i += 256) s_fab[i] = fab[i];
  // list-ordered tables: entry q describes the q-th low part of the list
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(smem + 16 * NLO + TB * NLO);
  // this wave's staging area: the segment's block, 256 rows of G columns
  Grp<T>* stage = reinterpret_cast<Grp<T>*>(
      reinterpret_cast<unsigned char*>(s_fab + ((nb * 64 + 1) & ~1)) +
      (size_t)(threadIdx.x >> 6) * kChainStageRows * 16);
  __syncthreads();

  const int xcd = blockIdx.x % nxcd;
  const int blocks_x = gridDim.x / nxcd;
  const int64_t nitem = c.nseg * ngrp;
  const int64_t i_begin = nitem * xcd / nxcd, i_end = nitem * (xcd + 1) / nxcd;
  const int wpb = blockDim.x >> 6;
  const int64_t wstride = (int64_t)blocks_x * wpb;
  const int lane = threadIdx.x & 63;
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  const uint32_t rowb = (uint32_t)nb * TB;  // bytes per row of a block
  const uint32_t blkbytes = (uint32_t)(c.D * rowb);
  const uint32_t cbytes = (uint32_t)(c.D * TB);  // one column-major column
  const rsrc_t rb1 = make_rsrc(b1, blkbytes), rb2 = make_rsrc(b2, b2 ? blkbytes : 0);
  const rsrc_t rv = make_rsrc(v, v ? (VCM ? (uint32_t)(c.D * nb * TB) : blkbytes) : 0);
  const rsrc_t rout = make_rsrc(out, OCM ? (uint32_t)(c.D * nb * TB) : blkbytes);
  int64_t it = i_begin + (int64_t)(blockIdx.x / nxcd) * wpb + uniform(threadIdx.x >> 6);
  for (; it < i_end; it += wstride) {
    const int64_t si = it / ngrp;
    const int g = (int)(it % ngrp);
    const int c0 = g * G, w = min(G, nb - c0);
    const uint32_t cb = (uint32_t)c0 * TB;  // byte offset of the group in a row
    const SegRec<NH> cur = load_rec<NH>(recs + (int64_t)uniform((int)si) * kChainRecWords);
    const int hi0 = cur.flags & 1, hitop = (cur.flags >> 1) & 1;
    const int bs = (cur.flags >> 2) & 1023, st = (cur.flags >> 12) & 1023;
    const int blk0 = cur.row0 - st;
    // per-column scalars of the group (padding columns repeat the last)
    T sig[G], ta[G], ac[G], dsg[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int col = min(c0 + q, nb - 1);
      sig[q] = sc[col] * half;
      ta[q] = sc[nb + col] * half;
      ac[q] = acoef ? acoef[col] : T(0);
      dsg[q] = dseg[si * nb + col];
    }
    // the block of b_{i+1} for the low-part hops: loads now, LDS later
    Grp<T> sg[kChainStageRows / 64];
#pragma unroll
    for (int m = 0; m < kChainStageRows / 64; ++m) {
      const int r = lane + 64 * m;
      sg[m] = gload<T>(rb1, (uint32_t)min(r, bs - 1) * rowb + cb, (uint32_t)blk0 * rowb, w);
    }
    int jj[2], lo[2], gj[2], gp[2];
    u4 np[2];
    bool act_j[2], act_p[2];
    T zz[2], nidle[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      jj[i] = min(lane + 64 * i, cur.len - 1);
      const int q = cur.lidx + jj[i];
      const int l = s_lo[q];
      lo[i] = l;
      np[i] = s_np[q];
      act_j[i] = ((l >> (Lb - 1)) & 1) != hi0;
      act_p[i] = c.periodic && ((l & 1) != hitop);
      gj[i] = blk0 + cur.d_join + (int)((np[i][2] >> 8) & 255u);
      gp[i] = blk0 + cur.d_pbc + (int)((np[i][2] >> 16) & 255u);
      const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
      nidle[i] = (T)(NL - __popc(xlo));
      const int n11x = ((l >> (Lb - 1)) & 1 & hi0) + (c.periodic ? (hitop & l & 1) : 0);
      zz[i] = vzz * (T)(__popc(l & (l >> 1)) + n11x);
    }
    Grp<T> g_hi[NH > 0 ? NH : 1][2], g_j[2], g_p[2], vv[2], bt[2];
#pragma unroll
    for (int b = 0; b < NH; ++b)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (cur.dh[b] != 0)
          g_hi[b][i] = gload<T>(rb1, (uint32_t)jj[i] * rowb + cb,
                                (uint32_t)(cur.row0 + cur.dh[b]) * rowb, w);
        else
          g_hi[b][i] = Grp<T>{};
      }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      g_j[i] = act_j[i] ? gload<T>(rb1, (uint32_t)gj[i] * rowb + cb, 0, w) : Grp<T>{};
      g_p[i] = act_p[i] ? gload<T>(rb1, (uint32_t)gp[i] * rowb + cb, 0, w) : Grp<T>{};
      const uint32_t row = (uint32_t)(cur.row0 + jj[i]);
      if (!v) {
        vv[i] = Grp<T>{};
      } else if (VCM) {
#pragma unroll
        for (int q = 0; q < G; ++q)
          vv[i].x[q] = q < w ? bload<T, kAuxNT>(rv, row * TB, (uint32_t)(c0 + q) * cbytes) : T(0);
      } else {
        vv[i] = gload<T>(rv, row * rowb + cb, 0, w);
      }
      bt[i] = b2 ? gload<T>(rb2, row * rowb + cb, 0, w) : Grp<T>{};
    }
    wave_sync();  // the previous item's LDS reads are done
#pragma unroll
    for (int m = 0; m < kChainStageRows / 64; ++m)
      if (lane + 64 * m < bs) stage[lane + 64 * m] = sg[m];
    wave_sync();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int l = lo[i];
      const Grp<T> bo = stage[st + jj[i]];
      Grp<T> nbv[NL > 0 ? NL : 1];
#pragma unroll
      for (int b = 0; b < NL; ++b) nbv[b] = stage[(np[i][b >> 2] >> (8 * (b & 3))) & 255u];
      Grp<T> o;
#pragma unroll
      for (int q = 0; q < G; ++q) {
        T hop = 0;
#pragma unroll
        for (int b = 0; b < NL; ++b) hop += nbv[b].x[q];
#pragma unroll
        for (int b = 0; b < NH; ++b) hop += g_hi[b][i].x[q];
        hop -= nidle[i] * bo.x[q];
        hop += act_j[i] ? g_j[i].x[q] : T(0);
        const T* fa = s_fab + min(c0 + q, nb - 1) * 64;
        const T dg = zz[i] + fa[l & 31] + fa[32 + (l >> 5)] + dsg[q];
        const T acc = dg * bo.x[q] + t_in * hop + (act_p[i] ? t_pb * g_p[i].x[q] : T(0));
        o.x[q] = sig[q] * acc + ta[q] * bo.x[q] - bt[i].x[q] + ac[q] * vv[i].x[q];
      }
      const uint32_t row = (uint32_t)(cur.row0 + jj[i]);
      if (lane + 64 * i >= cur.len) continue;  // a clamped repeat of the last row
      if (OCM) {
#pragma unroll
        for (int q = 0; q < G; ++q)
          if (q < w) bstore<kAuxNT>(o.x[q], rout, row * TB, (uint32_t)(c0 + q) * cbytes);
      } else {
        gstore<T>(o, rout, row * rowb + cb, 0, w);
      }
    }
  }
}

// Row-group multi-column step, on the interleaved layout (element (row r,
// column c) at X[r nb + c]).  The lpr = 2^lg_lpr lanes of a row group share
// one row, lane k of the group holding the row's columns kG .. kG + G - 1
// (one 16-byte access), so a wavefront reads 64 / lpr whole rows per access:
// every gather is contiguous, the row's own work (its low part, neighbour
// positions and diagonal) is done once per row group instead of once per
// column group, and the low-part neighbours, which lie in the row's block of
// at most 256 rows, are read from the L1 cache instead of an LDS stage.  A
// wavefront takes one (segment, chunk of 64 / lpr rows) item.  Lanes past
// the last column (nb below lpr G) load nothing and store nothing.  v may be
// column-major (vcm) and the output too (ocm), as in the interleaved kernel.
template <typename T, int L>
__global__ __launch_bounds__(256) void k_chain_rows(
    ChainSplitDev c, int nb, int lg_lpr, T half, const T* __restrict__ fab,
    const T* __restrict__ dseg, const T* __restrict__ sc, const T* __restrict__ acoef,
    const T* __restrict__ v, bool vcm, const T* __restrict__ b1, const T* b2, T* out, bool ocm,
    int nxcd, const int32_t* __restrict__ recs) {
  constexpr int G = 16 / (int)sizeof(T);
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int Lh = L - Lb;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = Lh - 1;
  constexpr int NL = Lb - 1;
  constexpr int BLOB = chain_blob_bytes(NLO, (int)sizeof(T));
  constexpr int CHUNKS = BLOB / 16;
  constexpr uint32_t TB = sizeof(T);
  using u4 = __attribute__((ext_vector_type(4))) uint32_t;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  for (int i = threadIdx.x; i < CHUNKS; i += 256)
    reinterpret_cast<u4*>(smem)[i] =
        reinterpret_cast<const u4*>(sizeof(T) == 8 ? c.blobl64 : c.blobl32)[i];
  T* s_fab = reinterpret_cast<T*>(smem + BLOB);
  for (int i = threadIdx.x; i < nb * 64; i += 256) s_fab[i] = fab[i];
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(smem + 16 * NLO + TB * NLO);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int rpw = 64 >> lg_lpr;          // rows per wavefront access
  const int nch = (kChainSegRows + rpw - 1) / rpw;  // chunks of a segment
  const int rl = lane >> lg_lpr;
  const int c0 = (lane & ((1 << lg_lpr) - 1)) * G;
  const int w = max(0, min(G, nb - c0));
  const uint32_t cb = (uint32_t)c0 * TB;
  T sig[G], ta[G], ac[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int col = min(c0 + q, nb - 1);
    sig[q] = sc[col] * half;
    ta[q] = sc[nb + col] * half;
    ac[q] = acoef ? acoef[col] : T(0);
  }
  const int xcd = blockIdx.x % nxcd;
  const int blocks_x = gridDim.x / nxcd;
  const int64_t nitem = c.nseg * nch;
  const int64_t i_begin = nitem * xcd / nxcd, i_end = nitem * (xcd + 1) / nxcd;
  const int wpb = blockDim.x >> 6;
  const int64_t wstride = (int64_t)blocks_x * wpb;
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  const uint32_t rowb = (uint32_t)nb * TB;
  const uint32_t blkbytes = (uint32_t)(c.D * rowb);
  const uint32_t cbytes = (uint32_t)(c.D * TB);
  const rsrc_t rb1 = make_rsrc(b1, blkbytes), rb2 = make_rsrc(b2, b2 ? blkbytes : 0);
  const rsrc_t rv = make_rsrc(v, v ? blkbytes : 0);
  const rsrc_t rout = make_rsrc(out, blkbytes);
  int64_t it = i_begin + (int64_t)(blockIdx.x / nxcd) * wpb + uniform(threadIdx.x >> 6);
  for (; it < i_end; it += wstride) {
    const int64_t si = it / nch;
    const int ch = (int)(it % nch);
    const SegRec<NH> cur = load_rec<NH>(recs + (int64_t)uniform((int)si) * kChainRecWords);
    if (ch * rpw >= cur.len) continue;  // wave-uniform: the segment is shorter
    const int hi0 = cur.flags & 1, hitop = (cur.flags >> 1) & 1;
    const int st = (cur.flags >> 12) & 1023;
    const int blk0 = cur.row0 - st;
    const int jr = ch * rpw + rl;
    const bool valid = jr < cur.len && w > 0;
    const int jj = min(jr, cur.len - 1);
    const int qd = cur.lidx + jj;
    const int l = s_lo[qd];
    const u4 np = s_np[qd];
    const bool act_j = ((l >> (Lb - 1)) & 1) != hi0;
    const bool act_p = c.periodic && ((l & 1) != hitop);
    const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
    const T nidle = (T)(NL - __popc(xlo));
    const int n11x = ((l >> (Lb - 1)) & 1 & hi0) + (c.periodic ? (hitop & l & 1) : 0);
    const T zz = vzz * (T)(__popc(l & (l >> 1)) + n11x);
    const uint32_t row = (uint32_t)(cur.row0 + jj);
    const int ww = valid ? w : 0;  // rows past the segment's end load nothing
    T dsg[G];
#pragma unroll
    for (int q = 0; q < G; ++q) dsg[q] = dseg[si * nb + min(c0 + q, nb - 1)];
    Grp<T> bo = gload<T>(rb1, row * rowb + cb, 0, ww);
    Grp<T> nbv[NL > 0 ? NL : 1], g_hi[NH > 0 ? NH : 1];
#pragma unroll
    for (int b = 0; b < NL; ++b)
      nbv[b] = gload<T>(rb1, (uint32_t)(blk0 + (int)((np[b >> 2] >> (8 * (b & 3))) & 255u)) * rowb + cb,
                        0, ww);
#pragma unroll
    for (int b = 0; b < NH; ++b)
      g_hi[b] = cur.dh[b] != 0 ? gload<T>(rb1, (uint32_t)jj * rowb + cb,
                                          (uint32_t)(cur.row0 + cur.dh[b]) * rowb, ww)
                               : Grp<T>{};
    const int gj = blk0 + cur.d_join + (int)((np[2] >> 8) & 255u);
    const int gp = blk0 + cur.d_pbc + (int)((np[2] >> 16) & 255u);
    const Grp<T> g_j = act_j ? gload<T>(rb1, (uint32_t)gj * rowb + cb, 0, ww) : Grp<T>{};
    const Grp<T> g_p = act_p ? gload<T>(rb1, (uint32_t)gp * rowb + cb, 0, ww) : Grp<T>{};
    Grp<T> vv{}, bt{};
    if (v) {
      if (vcm) {
#pragma unroll
        for (int q = 0; q < G; ++q)
          vv.x[q] = q < ww ? bload<T, kAuxNT>(rv, row * TB, (uint32_t)(c0 + q) * cbytes) : T(0);
      } else {
        vv = gload<T>(rv, row * rowb + cb, 0, ww);
      }
    }
    if (b2) bt = gload<T>(rb2, row * rowb + cb, 0, ww);
    Grp<T> o;
#pragma unroll
    for (int q = 0; q < G; ++q) {
      T hop = 0;
#pragma unroll
      for (int b = 0; b < NL; ++b) hop += nbv[b].x[q];
#pragma unroll
      for (int b = 0; b < NH; ++b) hop += g_hi[b].x[q];
      hop -= nidle * bo.x[q];
      hop += act_j ? g_j.x[q] : T(0);
      const T* fa = s_fab + min(c0 + q, nb - 1) * 64;
      const T dg = zz + fa[l & 31] + fa[32 + (l >> 5)] + dsg[q];
      const T acc = dg * bo.x[q] + t_in * hop + (act_p ? t_pb * g_p.x[q] : T(0));
      o.x[q] = sig[q] * acc + ta[q] * bo.x[q] - bt.x[q] + ac[q] * vv.x[q];
    }
    if (!valid) continue;
    if (ocm) {
#pragma unroll
      for (int q = 0; q < G; ++q)
        if (q < w) bstore<kAuxNT>(o.x[q], rout, row * TB, (uint32_t)(c0 + q) * cbytes);
    } else {
      gstore<T>(o, rout, row * rowb + cb, 0, w);
    }
  }
}

// LDS-resident filter for short chains: one workgroup per column runs that
// column's whole Clenshaw recurrence, b_K = a_K v, b_i = a_i v + 2 H~ b_{i+1}
// - b_{i+2} (i = K_c - 1 .. 1), w = a_0 v + H~ b_1 - b_2, with b_{i+1} and
// b_{i+2} both held in LDS (b_i overwrites b_{i+2} in place) and a
// workgroup barrier between steps: no launch per step and no global traffic
// but v (kept in LDS too where a third vector fits) and w.  The segment
// records, a row-to-segment map and the column's per-segment diagonal part
// sit in LDS as well, so the threads take rows, not segments: thread t
// handles rows t, t + 1024, ..., and every operand of a row (its segment's
// record, its low-part tables, the neighbours) is an LDS read, all issued
// before any is summed.  Fits where the vectors and tables fit the LDS
// (FP64 up to L = 14, FP32 up to L = 16 at half filling).
template <typename T, int L, bool VLDS>
__global__ __launch_bounds__(1024) void k_chain_lds_filter(
    ChainSplitDev c, int nb, const T* __restrict__ fab, const T* __restrict__ dseg,
    const T* __restrict__ sc, const T* __restrict__ A, const int* __restrict__ Kc,
    const T* __restrict__ v, T* __restrict__ w, const int32_t* __restrict__ recs) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int Lh = L - Lb;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = Lh - 1;
  constexpr int NL = Lb - 1;
  constexpr int BLOB = chain_blob_bytes(NLO, (int)sizeof(T));
  constexpr int CHUNKS = BLOB / 16;
  constexpr int RW = kChainRecWords;
  static_assert(10 + NH <= 20, "five 16-byte reads cover a record's used words");
  using u4 = __attribute__((ext_vector_type(4))) uint32_t;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int col = blockIdx.x;
  const int64_t D = c.D;
  const int nseg = (int)c.nseg;
  for (int i = threadIdx.x; i < CHUNKS; i += 1024)
    reinterpret_cast<u4*>(smem)[i] =
        reinterpret_cast<const u4*>(sizeof(T) == 8 ? c.blobl64 : c.blobl32)[i];
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(smem + 16 * NLO + sizeof(T) * NLO);
  T* s_fa = reinterpret_cast<T*>(smem + BLOB);
  if (threadIdx.x < 64) s_fa[threadIdx.x] = fab[(int64_t)col * 64 + threadIdx.x];
  // this column's uniform diagonal part per segment, the segment records,
  // the row-to-segment map, then the vectors
  T* s_dseg = s_fa + 64;
  for (int i = threadIdx.x; i < nseg; i += 1024) s_dseg[i] = dseg[(int64_t)i * nb + col];
  int32_t* s_rec = reinterpret_cast<int32_t*>(s_dseg + ((nseg + 1) & ~1));
  for (int i = threadIdx.x; i < nseg * RW / 4; i += 1024)
    reinterpret_cast<u4*>(s_rec)[i] = reinterpret_cast<const u4*>(recs)[i];
  uint16_t* s_rowseg = reinterpret_cast<uint16_t*>(s_rec + nseg * RW);
  T* bufX = reinterpret_cast<T*>(s_rowseg + ((D + 7) & ~int64_t(7)));
  T* bufY = bufX + D;
  T* s_v = bufY + D;
  const T* vg = v + (int64_t)col * D;
  if (VLDS)
    for (int64_t r = threadIdx.x; r < D; r += 1024) s_v[r] = vg[r];
  const T* vc = VLDS ? s_v : vg;
  const int K = Kc[col];
  const T sig = sc[col], tau = sc[nb + col];
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  __syncthreads();  // records in LDS
  for (int si = threadIdx.x; si < nseg; si += 1024) {
    const int row0 = s_rec[si * RW], len = s_rec[si * RW + 1];
    for (int j = 0; j < len; ++j) s_rowseg[row0 + j] = (uint16_t)si;
  }
  // b_K = a_K v, b_{K+1} = 0
  const T aK = A[(int64_t)K * nb + col];
  for (int64_t r = threadIdx.x; r < D; r += 1024) {
    bufX[r] = aK * vg[r];
    bufY[r] = T(0);
  }
  __syncthreads();
  T* cur = bufX;  // b_{i+1}
  T* prv = bufY;  // b_{i+2}, overwritten by b_i
  T a_next = K >= 1 ? A[(int64_t)(K - 1) * nb + col] : T(0);
  for (int i = K - 1; i >= 0; --i) {
    const bool last = i == 0;
    const T h = last ? T(0.5) : T(1);
    // this step's coefficient was read one step ahead
    const T ai = a_next;
    if (i >= 1) a_next = A[(int64_t)(i - 1) * nb + col];
    for (int64_t r = threadIdx.x; r < D; r += 1024) {
      const int si = s_rowseg[r];
      const u4* rq = reinterpret_cast<const u4*>(s_rec + si * RW);
      const u4 w0 = rq[0], w1 = rq[1], w2 = rq[2], w3 = rq[3], w4 = rq[4];
      const int row0 = (int)w0[0], lidx = (int)w0[2], flags = (int)w0[3];
      const int d_join = (int)w1[1], d_pbc = (int)w1[2];
      int dh[NH > 0 ? NH : 1];
#pragma unroll
      for (int b = 0; b < NH; ++b) {
        const int k = 10 + b;  // word k of the record
        const u4 q4 = k < 12 ? w2 : (k < 16 ? w3 : w4);
        dh[b] = (int)q4[k & 3];
      }
      const int hi0 = flags & 1, hitop = (flags >> 1) & 1, st = (flags >> 12) & 1023;
      const int jj = (int)r - row0, blk0 = row0 - st;
      const int q = lidx + jj;
      const int l = s_lo[q];
      const u4 np = s_np[q];
      // every operand first, then the sums
      const T bo = cur[r], bp = prv[r], vr = vc[r], dsg = s_dseg[si];
      T nbv[NL > 0 ? NL : 1], hv[NH > 0 ? NH : 1];
#pragma unroll
      for (int b = 0; b < NL; ++b) nbv[b] = cur[blk0 + (int)((np[b >> 2] >> (8 * (b & 3))) & 255u)];
#pragma unroll
      for (int b = 0; b < NH; ++b) hv[b] = cur[r + dh[b]];  // an idle bond reads the row itself
      const bool act_j = ((l >> (Lb - 1)) & 1) != hi0;
      const bool act_p = c.periodic && ((l & 1) != hitop);
      const T tj = cur[min(blk0 + d_join + (int)((np[2] >> 8) & 255u), (int)D - 1)];
      const T tp = cur[min(blk0 + d_pbc + (int)((np[2] >> 16) & 255u), (int)D - 1)];
      T hop = 0;
#pragma unroll
      for (int b = 0; b < NL; ++b) hop += nbv[b];
      const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
      hop -= (T)(NL - __popc(xlo)) * bo;
#pragma unroll
      for (int b = 0; b < NH; ++b) hop += dh[b] != 0 ? hv[b] : T(0);
      hop += act_j ? tj : T(0);
      const int n11x = ((l >> (Lb - 1)) & 1 & hi0) + (c.periodic ? (hitop & l & 1) : 0);
      const T dg =
          vzz * (T)(__popc(l & (l >> 1)) + n11x) + s_fa[l & 31] + s_fa[32 + (l >> 5)] + dsg;
      const T acc = dg * bo + t_in * hop + (act_p ? t_pb * tp : T(0));
      const T o = h * (sig * acc + tau * bo) - bp + ai * vr;
      if (last)
        w[(int64_t)col * D + r] = o;
      else
        prv[r] = o;
    }
    __syncthreads();  // b_i complete before it is read as b_{i+1}
    T* t = cur;
    cur = prv;
    prv = t;
  }
  if (K == 0)
    for (int64_t r = threadIdx.x; r < D; r += 1024) w[(int64_t)col * D + r] = A[col] * vg[r];
}

// LDS bytes of the resident filter with nv vectors of D in LDS.
template <typename T>
size_t lds_filter_bytes(const polfed_op* op0, int nv = 2) {
  const int Lb = std::min(kChainLoBits, op0->L / 2);
  return chain_blob_bytes(1 << Lb, (int)sizeof(T)) + 64 * sizeof(T) +
         (size_t)((op0->split_nseg + 1) & ~int64_t(1)) * sizeof(T) +
         (size_t)op0->split_nseg * kChainRecWords * 4 + (size_t)((op0->D + 7) & ~int64_t(7)) * 2 +
         (size_t)nv * op0->D * sizeof(T);
}

template <typename T>
bool chain_lds_filter_fits(const polfed_op* op0) {
  return op0->L <= 16 && op0->split_nseg > 0 && lds_filter_bytes<T>(op0) <= kLdsPerCU &&
         op0->split_Lb <= 8;
}

template <typename T>
void chain_lds_filter(hipStream_t s, const ChainBatch& bt, const T* A, const int* Kc, const T* v,
                      T* w) {
  const polfed_op* op0 = bt.ops[0];
  REQUIRE(chain_lds_filter_fits<T>(op0), "batch: chain too long for the LDS-resident filter");
  const bool f64 = sizeof(T) == 8;
  ChainSplitDev c = op0->chain_split();
  const T* fab = (const T*)(f64 ? bt.fab64.get() : bt.fab32.get());
  const T* dseg = (const T*)(f64 ? bt.dseg64.get() : bt.dseg32.get());
  const T* sc = (const T*)(f64 ? bt.sc64.get() : bt.sc32.get());
  const bool vlds = lds_filter_bytes<T>(op0, 3) <= kLdsPerCU;
  const size_t shm = lds_filter_bytes<T>(op0, vlds ? 3 : 2);
  switch (op0->L) {
#define POLFED_CASE(LL)                                                                         \
  case LL:                                                                                      \
    if (vlds)                                                                                   \
      hipLaunchKernelGGL((k_chain_lds_filter<T, LL, true>), dim3((unsigned)bt.nb), dim3(1024),  \
                         shm, s, c, bt.nb, fab, dseg, sc, A, Kc, v, w, c.rec);                  \
    else                                                                                        \
      hipLaunchKernelGGL((k_chain_lds_filter<T, LL, false>), dim3((unsigned)bt.nb), dim3(1024), \
                         shm, s, c, bt.nb, fab, dseg, sc, A, Kc, v, w, c.rec);                  \
    break;
    POLFED_CASE(4) POLFED_CASE(5) POLFED_CASE(6) POLFED_CASE(7) POLFED_CASE(8)
    POLFED_CASE(9) POLFED_CASE(10) POLFED_CASE(11) POLFED_CASE(12) POLFED_CASE(13)
    POLFED_CASE(14) POLFED_CASE(15) POLFED_CASE(16)
#undef POLFED_CASE
    default: fail(POLFED_ERR_INVALID, "batch: chain too long for the LDS-resident filter");
  }
  HIPC(hipGetLastError());
}

template bool chain_lds_filter_fits<double>(const polfed_op*);
template bool chain_lds_filter_fits<float>(const polfed_op*);
template void chain_lds_filter<double>(hipStream_t, const ChainBatch&, const double*, const int*,
                                       const double*, double*);
template void chain_lds_filter<float>(hipStream_t, const ChainBatch&, const float*, const int*,
                                      const float*, float*);

static int batch_bpc_fit(size_t shm) { return std::max(1, (int)(kLdsPerCU / shm)); }

template <typename T, int L>
static void launch_ilv(hipStream_t s, const polfed_op* op0, const ChainBatch& bt, int bpc, T half,
                       const T* acoef, const T* v, bool vcm, const T* b1, const T* b2, T* out,
                       bool ocm) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int G = 16 / (int)sizeof(T);
  const size_t shm = chain_blob_bytes(1 << Lb, (int)sizeof(T)) +
                     (size_t)((bt.nb * 64 + 1) & ~1) * sizeof(T) + 4 * kChainStageRows * 16;
  bpc = std::max(1, std::min(bpc, batch_bpc_fit(shm)));
  ChainSplitDev c = op0->chain_split();
  const int ngrp = (bt.nb + G - 1) / G;
  const int64_t items = c.nseg * ngrp;
  int64_t grid = std::min<int64_t>((items + 3) / 4, (int64_t)op0->ctx->n_cu * bpc);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  grid = std::max<int64_t>(grid, 1);
  const bool f64 = sizeof(T) == 8;
  const T* fab = (const T*)(f64 ? bt.fab64.get() : bt.fab32.get());
  const T* dseg = (const T*)(f64 ? bt.dseg64.get() : bt.dseg32.get());
  const T* sc = (const T*)(f64 ? bt.sc64.get() : bt.sc32.get());
#define POLFED_ILV(VC, OC)                                                                   \
  hipLaunchKernelGGL((k_chain_ilv<T, L, VC, OC>), dim3((unsigned)grid), dim3(256), shm, s, c, \
                     bt.nb, half, fab, dseg, sc, acoef, v, b1, b2, out, ngrp, nxcd, c.rec)
  if (vcm && ocm)
    POLFED_ILV(true, true);
  else if (vcm)
    POLFED_ILV(true, false);
  else if (ocm)
    POLFED_ILV(false, true);
  else
    POLFED_ILV(false, false);
#undef POLFED_ILV
  HIPC(hipGetLastError());
}

// lanes per row: the columns' 16-byte groups rounded up to a power of two
static int rows_lg_lpr(int nb, size_t tb) {
  const int groups = (int)((nb * tb + 15) / 16);
  int lg = 0;
  while ((1 << lg) < groups) ++lg;
  return lg;
}
constexpr int kRowsMaxLgLpr = 4;  // at most 16 lanes per row

template <typename T, int L>
static void launch_rows(hipStream_t s, const polfed_op* op0, const ChainBatch& bt, int bpc, T half,
                        const T* acoef, const T* v, bool vcm, const T* b1, const T* b2, T* out,
                        bool ocm) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  const size_t shm = chain_blob_bytes(1 << Lb, (int)sizeof(T)) + (size_t)bt.nb * 64 * sizeof(T);
  bpc = std::max(1, std::min(bpc, batch_bpc_fit(shm)));
  const int lg = rows_lg_lpr(bt.nb, sizeof(T));
  ChainSplitDev c = op0->chain_split();
  const int rpw = 64 >> lg;
  const int64_t items = c.nseg * ((kChainSegRows + rpw - 1) / rpw);
  int64_t grid = std::min<int64_t>((items + 3) / 4, (int64_t)op0->ctx->n_cu * bpc);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  grid = std::max<int64_t>(grid, 1);
  const bool f64 = sizeof(T) == 8;
  hipLaunchKernelGGL((k_chain_rows<T, L>), dim3((unsigned)grid), dim3(256), shm, s, c, bt.nb, lg,
                     half, (const T*)(f64 ? bt.fab64.get() : bt.fab32.get()),
                     (const T*)(f64 ? bt.dseg64.get() : bt.dseg32.get()),
                     (const T*)(f64 ? bt.sc64.get() : bt.sc32.get()), acoef, v, vcm, b1, b2, out,
                     ocm, nxcd, c.rec);
  HIPC(hipGetLastError());
}

template <typename T, int L>
static void launch_batch(hipStream_t s, const polfed_op* op0, const ChainBatch& bt,
                         int col0, int ncols, int64_t ld, int bpc, T half, const T* acoef,
                         const T* v, const T* b1, const T* b2, T* out) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int NLO = 1 << Lb;
  const size_t shm = chain_blob_bytes(NLO, (int)sizeof(T)) +
                     (size_t)ncols * 64 * sizeof(T) + 4 * kChainStageRows * sizeof(T);
  bpc = std::max(1, std::min(bpc, batch_bpc_fit(shm)));
  ChainSplitDev c = op0->chain_split();
  const int64_t blocks_needed = (c.nseg + 3) / 4;
  int64_t grid = std::min<int64_t>(blocks_needed, (int64_t)op0->ctx->n_cu * bpc);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  grid = std::max<int64_t>(grid, 1);
  const bool f64 = sizeof(T) == 8;
  hipLaunchKernelGGL((k_chain_split_batch<T, L>), dim3((unsigned)grid), dim3(256), shm, s, c,
                     bt.nb, col0, ncols, ld, half,
                     (const T*)(f64 ? bt.fab64.get() : bt.fab32.get()),
                     (const T*)(f64 ? bt.dseg64.get() : bt.dseg32.get()),
                     (const T*)(f64 ? bt.sc64.get() : bt.sc32.get()), acoef, v, b1, b2, out,
                     nxcd, c.rec);
  HIPC(hipGetLastError());
}

void ChainBatch::init(polfed_ctx* c, const polfed_op* const* o, int n) {
  REQUIRE(n >= 1, "batch: need at least one operator");
  ctx = c;
  nb = n;
  ops.assign(o, o + n);
  const polfed_op* op0 = ops[0];
  for (int i = 0; i < n; ++i) {
    REQUIRE(ops[i] != nullptr, "batch: null operator");
    REQUIRE(ops[i]->model == Model::Chain && !ops[i]->pattern_key.empty(),
            "batch: operators must be XXZ or t-V chains");
    REQUIRE(ops[i]->pattern_key == op0->pattern_key,
            "batch: operators must share the off-diagonal pattern (model, L, N, boundary, "
            "couplings)");
    REQUIRE(ops[i]->ctx == op0->ctx, "batch: operators belong to different contexts");
  }
  REQUIRE(op0->split_nseg > 0, "batch: chain length outside 4..28");
  const int64_t nseg = op0->split_nseg;
  std::vector<double> fab((size_t)n * 64), dseg((size_t)nseg * n);
  for (int i = 0; i < n; ++i) {
    std::copy(ops[i]->split_fab.begin(), ops[i]->split_fab.end(), fab.begin() + (size_t)i * 64);
    for (int64_t q = 0; q < nseg; ++q) dseg[(size_t)q * n + i] = ops[i]->split_dseg[q];
  }
  hipStream_t s = ctx->stream;
  upload(fab64, fab.data(), fab.size(), s);
  upload(dseg64, dseg.data(), dseg.size(), s);
  std::vector<float> f32(fab.begin(), fab.end()), d32(dseg.begin(), dseg.end());
  upload(fab32, f32.data(), f32.size(), s);
  upload(dseg32, d32.data(), d32.size(), s);
  sc64.alloc((size_t)2 * n * sizeof(double));
  sc32.alloc((size_t)2 * n * sizeof(float));
  HIPC(hipStreamSynchronize(s));
}

void ChainBatch::set_scale(const double* E_c, const double* dE) {
  std::vector<double> sc(2 * (size_t)nb);
  for (int i = 0; i < nb; ++i) {
    REQUIRE(dE[i] > 0 && std::isfinite(dE[i]) && std::isfinite(E_c[i]),
            "batch: need finite E_c and dE > 0");
    sc[i] = 2.0 / dE[i];
    sc[nb + i] = -2.0 * E_c[i] / dE[i];
  }
  std::vector<float> s32(sc.begin(), sc.end());
  this->E_c.assign(E_c, E_c + nb);
  this->dE.assign(dE, dE + nb);
  hipStream_t s = ctx->stream;
  HIPC(hipMemcpyAsync(sc64.get(), sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(sc32.get(), s32.data(), s32.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIPC(hipStreamSynchronize(s));
}

// Multi-column step variants: 0 and 1 the column-major kernel with 16 and
// 8 columns per launch, 2 and 3 the interleaved kernel with 2 and 4
// workgroups per compute unit, 4 each column by its operator's own kernel,
// 5 the LDS-resident whole filter, 6 and 7 the row-group kernel with 4 and
// 8 workgroups per compute unit.
constexpr int kBatchVariants = 8;

static bool interleaved_fits(const ChainBatch& bt, size_t tb) {
  return (uint64_t)bt.ops[0]->D * (uint64_t)bt.nb * tb < (uint64_t(1) << 32) - 64;
}

static bool rows_fit(const ChainBatch& bt, size_t tb) {
  return interleaved_fits(bt, tb) && rows_lg_lpr(bt.nb, tb) <= kRowsMaxLgLpr;
}

template <typename T>
static void batch_step_var(hipStream_t s, const ChainBatch& bt, int var, bool final_step,
                           const T* acoef, const T* v, bool vcm, const T* b1, const T* b2,
                           T* out, bool ocm) {
  const polfed_op* op0 = bt.ops[0];
  const T half = final_step ? T(0.5) : T(1);
  const int64_t ld = op0->D;
  if (var == 4) {
    // column by column with each operator's single-column kernel; the
    // per-column scalars are host values (the filter passes them through
    // batch_step_cols), here the timing step of the tuner
    for (int c = 0; c < bt.nb; ++c)
      op_step<T>(s, bt.ops[c], half * (T)(2.0 / bt.dE[c]), half * (T)(-2.0 * bt.E_c[c] / bt.dE[c]),
                 T(0), v + (size_t)c * ld, b1 + (size_t)c * ld, b2 ? b2 + (size_t)c * ld : nullptr,
                 out + (size_t)c * ld);
    return;
  }
  if (var == 6 || var == 7) {
    const int bpc = var == 6 ? 4 : 8;
    switch (op0->L) {
#define POLFED_CASE(LL)                                                                     \
  case LL:                                                                                  \
    launch_rows<T, LL>(s, op0, bt, bpc, half, acoef, v, vcm, b1, b2, out, ocm);             \
    break;
      POLFED_CASE(4) POLFED_CASE(5) POLFED_CASE(6) POLFED_CASE(7) POLFED_CASE(8)
      POLFED_CASE(9) POLFED_CASE(10) POLFED_CASE(11) POLFED_CASE(12) POLFED_CASE(13)
      POLFED_CASE(14) POLFED_CASE(15) POLFED_CASE(16) POLFED_CASE(17) POLFED_CASE(18)
      POLFED_CASE(19) POLFED_CASE(20) POLFED_CASE(21) POLFED_CASE(22) POLFED_CASE(23)
      POLFED_CASE(24) POLFED_CASE(25) POLFED_CASE(26) POLFED_CASE(27) POLFED_CASE(28)
#undef POLFED_CASE
      default: fail(POLFED_ERR_INVALID, "batch: chain length outside 4..28");
    }
    return;
  }
  if (var >= 2) {
    const int bpc = var == 2 ? 2 : 4;
    switch (op0->L) {
#define POLFED_CASE(LL)                                                                     \
  case LL:                                                                                  \
    launch_ilv<T, LL>(s, op0, bt, bpc, half, acoef, v, vcm, b1, b2, out, ocm);              \
    break;
      POLFED_CASE(4) POLFED_CASE(5) POLFED_CASE(6) POLFED_CASE(7) POLFED_CASE(8)
      POLFED_CASE(9) POLFED_CASE(10) POLFED_CASE(11) POLFED_CASE(12) POLFED_CASE(13)
      POLFED_CASE(14) POLFED_CASE(15) POLFED_CASE(16) POLFED_CASE(17) POLFED_CASE(18)
      POLFED_CASE(19) POLFED_CASE(20) POLFED_CASE(21) POLFED_CASE(22) POLFED_CASE(23)
      POLFED_CASE(24) POLFED_CASE(25) POLFED_CASE(26) POLFED_CASE(27) POLFED_CASE(28)
#undef POLFED_CASE
      default: fail(POLFED_ERR_INVALID, "batch: chain length outside 4..28");
    }
    return;
  }
  const int per = var == 0 ? 16 : 8;
  for (int col0 = 0; col0 < bt.nb; col0 += per) {
    const int ncols = std::min(per, bt.nb - col0);
    switch (op0->L) {
#define POLFED_CASE(LL)                                                                     \
  case LL:                                                                                  \
    launch_batch<T, LL>(s, op0, bt, col0, ncols, ld, kChainBlocksPerCU, half, acoef, v, b1, \
                        b2, out);                                                           \
    break;
      POLFED_CASE(4) POLFED_CASE(5) POLFED_CASE(6) POLFED_CASE(7) POLFED_CASE(8)
      POLFED_CASE(9) POLFED_CASE(10) POLFED_CASE(11) POLFED_CASE(12) POLFED_CASE(13)
      POLFED_CASE(14) POLFED_CASE(15) POLFED_CASE(16) POLFED_CASE(17) POLFED_CASE(18)
      POLFED_CASE(19) POLFED_CASE(20) POLFED_CASE(21) POLFED_CASE(22) POLFED_CASE(23)
      POLFED_CASE(24) POLFED_CASE(25) POLFED_CASE(26) POLFED_CASE(27) POLFED_CASE(28)
#undef POLFED_CASE
      default: fail(POLFED_ERR_INVALID, "batch: chain length outside 4..28");
    }
  }
}

template <typename T>
void chain_batch_step(hipStream_t s, const ChainBatch& bt, int64_t ld, bool final_step,
                      const T* acoef, const T* v, const T* b1, const T* b2, T* out) {
  REQUIRE(ld == bt.ops[0]->D, "batch: column stride must be D");
  batch_step_var<T>(s, bt, 0, final_step, acoef, v, true, b1, b2, out, true);
}

template <typename T>
int batch_variant(hipStream_t s, const ChainBatch& bt) {
  const polfed_op* op0 = bt.ops[0];
  const int key = bt.nb * 2 + (sizeof(T) == 8 ? 0 : 1);
  {
    auto it = op0->batch_tuned.find(key);
    if (it != op0->batch_tuned.end()) return it->second;
  }
  // an earlier choice for this chain pattern (any operator of it)
  const std::string pkey = "batch" + std::to_string(bt.nb) + (sizeof(T) == 8 ? "|64" : "|32");
  {
    const int v = pattern_choice(op0, pkey);
    if (v >= 0) return op0->batch_tuned[key] = v;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPC(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return 0;  // tuned before any capture
  TallyScope untallied(nullptr);
  const size_t n = (size_t)std::max<int64_t>(op0->D, 1) * bt.nb;
  DevBuf bv(n * sizeof(T)), b1(n * sizeof(T)), b2(n * sizeof(T)), ac(bt.nb * sizeof(T));
  HIPC(hipMemsetAsync(bv.get(), 0, n * sizeof(T), s));
  HIPC(hipMemsetAsync(b1.get(), 0, n * sizeof(T), s));
  HIPC(hipMemsetAsync(b2.get(), 0, n * sizeof(T), s));
  HIPC(hipMemsetAsync(ac.get(), 0, bt.nb * sizeof(T), s));
  HIPC(hipStreamSynchronize(s));
  int best = 0;
  float best_us = 1e30f;
  for (int var = 0; var < kBatchVariants; ++var) {
    if ((var == 2 || var == 3) && !interleaved_fits(bt, sizeof(T))) continue;
    if ((var == 6 || var == 7) && !rows_fit(bt, sizeof(T))) continue;
    if (var == 1 && bt.nb <= 8) continue;  // the same launches as variant 0
    if (var == 4) {
      // only where a single-column tile kernel exists (L >= 22); each
      // operator picks its own kernel first, outside any capture
      if (op0->L < 22) continue;
      for (int c = 0; c < bt.nb; ++c) op_tune(s, bt.ops[c], sizeof(T) == 4);
    }
    if (var == 5) {
      // the whole filter: time 16 steps, compare per step
      if (!chain_lds_filter_fits<T>(op0)) continue;
      constexpr int K5 = 16;
      DevBuf A5((size_t)(K5 + 1) * bt.nb * sizeof(T)), K5d(bt.nb * sizeof(int));
      HIPC(hipMemsetAsync(A5.get(), 0, A5.bytes(), s));
      std::vector<int> kh(bt.nb, K5);
      HIPC(hipMemcpyAsync(K5d.get(), kh.data(), kh.size() * sizeof(int), hipMemcpyHostToDevice, s));
      HIPC(hipStreamSynchronize(s));
      const float us = replay_time_us(
                           [&](hipStream_t ts) {
                             chain_lds_filter<T>(ts, bt, A5.as<T>(), K5d.as<int>(), bv.as<T>(),
                                                 b2.as<T>());
                           },
                           4) /
                       K5;
      if (verbose())
        std::fprintf(stderr, "[polfed] batch step L=%d nb=%d %s variant 5: %.2f us per step\n",
                     op0->L, bt.nb, sizeof(T) == 8 ? "fp64" : "fp32", us);
      if (us < best_us) {
        best_us = us;
        best = 5;
      }
      continue;
    }
    const float us = replay_time_us(
        [&](hipStream_t ts) {
          batch_step_var<T>(ts, bt, var, false, ac.as<T>(), bv.as<T>(), true, b1.as<T>(),
                            b2.as<T>(), b2.as<T>(), false);
        },
        10);
    if (verbose())
      std::fprintf(stderr, "[polfed] batch step L=%d nb=%d %s variant %d: %.2f us\n", op0->L,
                   bt.nb, sizeof(T) == 8 ? "fp64" : "fp32", var, us);
    if (us < best_us) {
      best_us = us;
      best = var;
    }
  }
  HIPC(hipStreamSynchronize(s));
  pattern_choice_set(op0, pkey, best);
  op0->batch_tuned[key] = best;
  return best;
}

template <typename T>
void chain_batch_step_var(hipStream_t s, const ChainBatch& bt, int var, bool final_step,
                          const T* acoef, const T* v, bool vcm, const T* b1, const T* b2,
                          T* out, bool ocm) {
  batch_step_var<T>(s, bt, var, final_step, acoef, v, vcm, b1, b2, out, ocm);
}

template int batch_variant<double>(hipStream_t, const ChainBatch&);
template int batch_variant<float>(hipStream_t, const ChainBatch&);
template void chain_batch_step_var<double>(hipStream_t, const ChainBatch&, int, bool,
                                           const double*, const double*, bool, const double*,
                                           const double*, double*, bool);
template void chain_batch_step_var<float>(hipStream_t, const ChainBatch&, int, bool,
                                          const float*, const float*, bool, const float*,
                                          const float*, float*, bool);
template void chain_batch_step<double>(hipStream_t, const ChainBatch&, int64_t, bool,
                                       const double*, const double*, const double*,
                                       const double*, double*);
template void chain_batch_step<float>(hipStream_t, const ChainBatch&, int64_t, bool,
                                      const float*, const float*, const float*,
                                      const float*, float*);

}  // namespace polfed

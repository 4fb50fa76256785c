// Fused Clenshaw step for the chain models (XXZ, t-V) in a particle-number
// sector, laid out for wave64 execution.
//
// A state is split as s = hi << Lb | lo.  States in ascending order are
// grouped by hi, and the rows of one hi form a contiguous block of
// binom(Lb, N - popcount(hi)) rows (at most 252 for Lb = 10) whose low parts
// run through the Lb-bit strings of that popcount in ascending order, so
//     rank(s) = hi_off[hi] + lo_rank[lo]
// and the position of a row inside its block is lo_rank[lo].
//
// Each wavefront processes a segment of one block (up to 128 rows, lanes on
// consecutive rows; a block of more rows is split into two segments, which
// both stage it: one segment per block, processed in two passes, measured
// slower since the second pass waits for the first).  Within a wavefront hi is uniform, hence:
//   - a hop inside the low part stays in the block.  The wavefront stages
//     the block's b_{i+1} entries in LDS once (coalesced) and reads those
//     neighbours from LDS at position lo_rank[lo'];
//   - a hop across a bond inside the high part moves to row r + d with a
//     wave-uniform d = hi_off[hi'] - hi_off[hi]: fully coalesced gathers;
//   - the bond joining the two parts and the periodic bond land in another
//     block at r + d + lo_rank[lo'] - lo_rank[lo] (d uniform);
//   - the diagonal is DLO[lo] (LDS) + a uniform high part + two cross terms.
// All wave-uniform data of a segment (offsets, flags, diagonal part) is
// precomputed into a 128-byte record read with scalar loads.  A high-part
// bond whose two bits are equal in the segment's high part cannot hop: its
// gather is skipped by a wave-uniform branch; the joining and periodic
// gathers are masked per lane.  All gathers of a lane's rows are issued
// before any is consumed, so they are in flight together.
//
// Locality: the eight XCDs each sweep a contiguous eighth of the segments
// (workgroups are dispatched to the XCDs round robin), so most high-part
// gathers of an XCD stay in its own L2; the streamed vectors v, b2 and the
// output use non-temporal accesses so they do not evict the gathered one.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <tuple>
#include <utility>

#include "chain_dev.hpp"
#include "internal.hpp"

namespace polfed {

void build_chain_split(polfed_op* op) {
  const int L = op->L, N = op->N;
  const int Lb = std::min(kChainLoBits, L / 2), Lh = L - Lb;
  REQUIRE(Lh - 1 <= kChainMaxHighBonds, "chain: too many high bonds");
  const int nlo = 1 << Lb;
  // low parts: ranks within their popcount class, list grouped by popcount
  std::vector<int32_t> lo_rank(nlo), cnt(Lb + 1, 0), lo_base(Lb + 2, 0);
  for (int lo = 0; lo < nlo; ++lo) lo_rank[lo] = cnt[__builtin_popcount(lo)]++;
  for (int p = 0; p <= Lb; ++p) lo_base[p + 1] = lo_base[p] + cnt[p];
  std::vector<uint16_t> lolist(nlo);
  for (int lo = 0; lo < nlo; ++lo)
    lolist[lo_base[__builtin_popcount(lo)] + lo_rank[lo]] = (uint16_t)lo;
  // block positions of the low-bond neighbours (own position if no hop), then
  // the ranks of lo with its top bit and with bit 0 flipped (all < 256)
  std::vector<uint8_t> npos((size_t)nlo * 16, 0);
  for (int lo = 0; lo < nlo; ++lo) {
    uint8_t* q = &npos[(size_t)lo * 16];
    for (int b = 0; b + 1 < Lb; ++b) {
      const bool act = ((lo >> b) & 1) != ((lo >> (b + 1)) & 1);
      q[b] = (uint8_t)(act ? lo_rank[lo ^ (3 << b)] : lo_rank[lo]);
    }
    q[9] = (uint8_t)lo_rank[lo ^ (1 << (Lb - 1))];
    q[10] = (uint8_t)lo_rank[lo ^ 1];
  }
  std::vector<double> dlo(nlo);
  for (int lo = 0; lo < nlo; ++lo) {
    double f = op->vzz * __builtin_popcount(lo & (lo >> 1));
    for (int i = 0; i < Lb; ++i)
      if ((lo >> i) & 1) f += op->site_f[i];
    dlo[lo] = f;
  }
  // high parts: first row of each block
  const int64_t nhi = (int64_t)1 << Lh;
  std::vector<int32_t> hi_off(nhi + 1, 0);
  int64_t acc = 0;
  for (int64_t hi = 0; hi < nhi; ++hi) {
    hi_off[hi] = (int32_t)acc;
    const int need = N - __builtin_popcountll(hi);
    if (need >= 0 && need <= Lb) acc += cnt[need];
  }
  hi_off[nhi] = (int32_t)acc;
  // one record per segment
  std::vector<int32_t> rec;
  op->split_dseg.clear();
  for (int64_t hi = 0; hi < nhi; ++hi) {
    const int need = N - __builtin_popcountll(hi);
    if (need < 0 || need > Lb) continue;
    const int bs = cnt[need];
    const int hoff = hi_off[hi];
    double dhi = op->vzz * __builtin_popcountll(hi & (hi >> 1)) + op->c0;
    for (int i = 0; i < Lh; ++i)
      if ((hi >> i) & 1) dhi += op->site_f[Lb + i];
    int32_t w[kChainRecWords] = {0};
    int idle = 0;
    for (int b = 0; b + 1 < Lh; ++b) {
      const bool act = ((hi >> b) & 1) != ((hi >> (b + 1)) & 1);
      w[10 + b] = act ? hi_off[hi ^ (3LL << b)] - hoff : 0;
      idle += act ? 0 : 1;
    }
    w[4] = idle;
    w[5] = hi_off[hi ^ 1] - hoff;
    w[6] = hi_off[hi ^ (1LL << (Lh - 1))] - hoff;
    std::memcpy(&w[8], &dhi, sizeof(double));
    const int nseg_hi = (bs + kChainSegRows - 1) / kChainSegRows;
    op->split_dseg.insert(op->split_dseg.end(), nseg_hi, dhi);
    for (int st = 0; st < bs; st += kChainSegRows) {
      w[0] = hoff + st;
      w[1] = std::min(kChainSegRows, bs - st);
      w[2] = lo_base[need] + st;
      w[3] = (int32_t)((hi & 1) | (((hi >> (Lh - 1)) & 1) << 1) | (bs << 2) | (st << 12));
      rec.insert(rec.end(), w, w + kChainRecWords);
    }
  }
  // field sums over low bits 0-4 and 5-9 (per-column diagonals of a batch)
  op->split_fab.assign(64, 0.0);
  for (int e = 0; e < 32; ++e)
    for (int k = 0; k < 5; ++k)
      if ((e >> k) & 1) {
        if (k < Lb) op->split_fab[e] += op->site_f[k];
        if (5 + k < Lb) op->split_fab[32 + e] += op->site_f[5 + k];
      }
  hipStream_t s = op->ctx->stream;
  op->split_Lb = Lb;
  op->split_nseg = (int64_t)(rec.size() / kChainRecWords);
  // packed LDS images: [neighbour positions | diagonal of the low part (T) |
  // low-part list], indexed by the low part; then the same three tables
  // indexed by position p in the low-part list (entry p describes lolist[p]),
  // so that a row's tables are one lookup away from its list position
  for (int w = 0; w < 2; ++w) {
    const int tb = w == 0 ? 8 : 4;
    std::vector<unsigned char> blob(chain_blob_bytes(nlo, tb), 0);
    unsigned char* p = blob.data();
    for (int q = 0; q < nlo; ++q) std::memcpy(p + 16 * q, &npos[(size_t)lolist[q] * 16], 16);
    p += 16 * (size_t)nlo;
    for (int q = 0; q < nlo; ++q) {
      if (tb == 8) {
        std::memcpy(p + 8 * q, &dlo[lolist[q]], 8);
      } else {
        const float f = (float)dlo[lolist[q]];
        std::memcpy(p + 4 * q, &f, 4);
      }
    }
    std::memcpy(p + (size_t)tb * nlo, lolist.data(), 2 * (size_t)nlo);
    upload(w == 0 ? op->d_blobl64 : op->d_blobl32, blob.data(), blob.size(), s);
  }
  for (int w = 0; w < 2; ++w) {
    const int tb = w == 0 ? 8 : 4;
    std::vector<unsigned char> blob(chain_blob_bytes(nlo, tb), 0);
    unsigned char* p = blob.data();
    std::memcpy(p, npos.data(), npos.size());
    p += npos.size();
    for (int lo = 0; lo < nlo; ++lo) {
      if (tb == 8) {
        std::memcpy(p + 8 * lo, &dlo[lo], 8);
      } else {
        const float f = (float)dlo[lo];
        std::memcpy(p + 4 * lo, &f, 4);
      }
    }
    std::memcpy(p + (size_t)tb * nlo, lolist.data(), 2 * (size_t)nlo);
    upload(w == 0 ? op->d_blob64 : op->d_blob32, blob.data(), blob.size(), s);
  }
  upload(op->d_rec, rec.data(), rec.size(), s);
  // tiles of 2^KT consecutive high parts (segments are in ascending hi), for
  // the largest KT with at least 512 tiles and for KT - 1
  std::vector<int32_t> seg_of_hi(nhi + 1, 0);
  {
    int32_t sidx = 0;
    for (int64_t hi = 0; hi < nhi; ++hi) {
      seg_of_hi[hi] = sidx;
      const int need = N - __builtin_popcountll(hi);
      if (need >= 0 && need <= Lb) sidx += (cnt[need] + kChainSegRows - 1) / kChainSegRows;
    }
    seg_of_hi[nhi] = sidx;
  }
  op->split_hi_off = hi_off;
  op->split_seg_of_hi = seg_of_hi;
  op->wtiles.clear();
  const int KT = chain_tile_bits(L);
  for (int v = 0; v < 3; ++v) {
    auto& T = op->tiles[v];
    T = polfed_op::Tiles{};
    const int kt = KT - v;
    if (KT == 0 || kt < 2) continue;
    const int64_t nt = (int64_t)1 << (Lh - kt);
    std::vector<int32_t> tiles((size_t)nt * 4, 0);
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t h0 = t << kt, h1 = (t + 1) << kt;
      tiles[4 * t] = hi_off[h0];
      tiles[4 * t + 1] = hi_off[h1] - hi_off[h0];
      tiles[4 * t + 2] = seg_of_hi[h0];
      tiles[4 * t + 3] = seg_of_hi[h1] - seg_of_hi[h0];
      T.max_rows = std::max(T.max_rows, tiles[4 * t + 1]);
    }
    T.bits = kt;
    T.n = (int)nt;
    upload(T.d, tiles.data(), tiles.size(), s);
  }
  op->tuned[0] = op->tuned[1] = -1;
  HIPC(hipStreamSynchronize(s));
}

// HALVES = 2 splits every segment between two wavefronts (64 rows each, one
// row per lane): twice the independent wavefronts, each with half the
// dependent work, for chains too short to fill the chip.
template <typename T, int L, int HALVES = 1>
__global__ __launch_bounds__(256) void k_chain_split(
    ChainSplitDev c, T sigma, T tau, T a, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out, int nxcd,
    const int32_t* __restrict__ recs) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int Lh = L - Lb;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = Lh - 1;  // bonds inside the high part
  constexpr int NL = Lb - 1;  // bonds inside the low part
  constexpr int RPL = 2 / HALVES;               // rows per lane and pass
  constexpr int kPasses = kChainSegRows / 128;  // passes per segment
  constexpr int SPL = kChainStageRows / 64;  // staged rows per lane
  constexpr int BLOB = chain_blob_bytes(NLO, (int)sizeof(T));
  constexpr int CHUNKS = BLOB / 16;
  constexpr uint32_t TB = sizeof(T);
  using u4 = __attribute__((ext_vector_type(4))) uint32_t;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  {  // one vectorized, unrolled copy of the packed tables into LDS
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
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const T* s_dlo = reinterpret_cast<const T*>(smem + 16 * NLO);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(s_dlo + NLO);
  T* stage = reinterpret_cast<T*>(smem + BLOB) + (threadIdx.x >> 6) * kChainStageRows;
  __syncthreads();

  // this XCD's contiguous share of the segments
  const int xcd = blockIdx.x % nxcd;
  const int blocks_x = gridDim.x / nxcd;
  const int64_t nvirt = c.nseg * HALVES;  // (segment, half) work items
  const int64_t s_begin = nvirt * xcd / nxcd, s_end = nvirt * (xcd + 1) / nxcd;
  const int wpb = blockDim.x >> 6;
  const int64_t wstride = (int64_t)blocks_x * wpb;
  const int lane = threadIdx.x & 63;
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  const uint32_t vbytes = (uint32_t)(c.D * TB);
  const rsrc_t rb1 = make_rsrc(b1, vbytes), rv = make_rsrc(v, v ? vbytes : 0),
               rb2 = make_rsrc(b2, b2 ? vbytes : 0), rout = make_rsrc(out, vbytes);
  int64_t vi = s_begin + (int64_t)(blockIdx.x / nxcd) * wpb + uniform(threadIdx.x >> 6);
  if (vi >= s_end) return;
  for (; vi < s_end; vi += wstride) {
    const int64_t si = vi / HALVES;
    const int half = (int)(vi % HALVES);
    const SegRec<NH> cur = load_rec<NH>(recs + (int64_t)uniform((int)si) * kChainRecWords);
    if (half * 64 >= cur.len) continue;
    const int hi0 = cur.flags & 1, hitop = (cur.flags >> 1) & 1;
    const int bs = (cur.flags >> 2) & 1023, st = (cur.flags >> 12) & 1023;
    const int blk0 = cur.row0 - st;
    const uint32_t so_blk = (uint32_t)blk0 * TB, so_row = (uint32_t)cur.row0 * TB;
    // the block of b_{i+1} for the low-part hops: loads now, LDS later
    T stg[SPL];
#pragma unroll
    for (int m = 0; m < SPL; ++m)
      stg[m] = 64 * m < bs ? bload<T>(rb1, (uint32_t)min(lane + 64 * m, bs - 1) * TB, so_blk)
                           : T(0);
    // the segment's rows in passes of 128 (two rows per lane); the block is
    // staged in LDS by the first pass
    for (int pass = 0; pass < kPasses; ++pass) {
      const int p0 = pass * 128 + half * 64;
      if (p0 >= cur.len) break;
      // rows of this lane, clamped into the segment (a clamped lane repeats
      // the last row and stores the same value)
      int jj[RPL], lo[RPL];
      u4 np[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        jj[i] = min(p0 + lane + 64 * i, cur.len - 1);
        lo[i] = s_lo[cur.lidx + jj[i]];
        np[i] = s_np[lo[i]];
      }
      // global gathers: high-part hops at uniform offsets, joining and
      // periodic bonds, and the streamed v and b_{i+2}
      T g_hi[RPL][NH > 0 ? NH : 1], g_j[RPL], g_p[RPL], vv[RPL], bt[RPL];
      bool act_j[RPL], act_p[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const uint32_t off = (uint32_t)jj[i] * TB;
#pragma unroll
        for (int b = 0; b < NH; ++b)
          g_hi[i][b] = cur.dh[b] != 0
                           ? bload<T>(rb1, off, (uint32_t)(cur.row0 + cur.dh[b]) * TB)
                           : T(0);
        const int l = lo[i];
        act_j[i] = ((l >> (Lb - 1)) & 1) != hi0;
        act_p[i] = c.periodic && ((l & 1) != hitop);
        const int rj = (int)((np[i][2] >> 8) & 255u);   // byte 9
        const int rp = (int)((np[i][2] >> 16) & 255u);  // byte 10
        g_j[i] = act_j[i] ? bload<T>(rb1, (uint32_t)(blk0 + cur.d_join + rj) * TB, 0) : T(0);
        g_p[i] = act_p[i] ? bload<T>(rb1, (uint32_t)(blk0 + cur.d_pbc + rp) * TB, 0) : T(0);
        vv[i] = v ? bload<T, kAuxNT>(rv, off, so_row) : T(0);
        bt[i] = b2 ? bload<T, kAuxNT>(rb2, off, so_row) : T(0);
      }
      if (pass == 0) {
        wave_sync();  // the previous segment's LDS reads are done
#pragma unroll
        for (int m = 0; m < SPL; ++m)
          if (64 * m < bs) stage[min(lane + 64 * m, bs - 1)] = stg[m];
        wave_sync();
      }
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int l = lo[i];
        const T bo = stage[st + jj[i]];
        T hop = 0;
#pragma unroll
        for (int b = 0; b < NL; ++b) hop += stage[(np[i][b >> 2] >> (8 * (b & 3))) & 255u];
#pragma unroll
        for (int b = 0; b < NH; ++b) hop += g_hi[i][b];
        const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
        const int n_idle = NL - __popc(xlo);
        hop -= (T)n_idle * bo;
        hop += act_j[i] ? g_j[i] : T(0);
        const int lo_top = (l >> (Lb - 1)) & 1, lo0 = l & 1;
        const int n11x = (lo_top & hi0) + (c.periodic ? (hitop & lo0) : 0);
        const T dg = s_dlo[l] + (T)cur.dhi + vzz * (T)n11x;
        const T acc = dg * bo + t_in * hop + (act_p[i] ? t_pb * g_p[i] : T(0));
        T o = sigma * acc + tau * bo - bt[i];
        if (v) o += a * vv[i];
        bstore<kAuxNT>(o, rout, (uint32_t)jj[i] * TB, so_row);
      }
    }
  }
}

// Paired variant: lane l holds the adjacent rows 2l and 2l + 1 of a segment,
// so every coalesced access (block staging, high-part gathers, v, b_{i+2}
// and the store) moves both rows in one 16-byte instruction, halving the
// vector-memory instructions per row.  Loads past the segment's end read
// other rows (unused) or fall outside the buffer (read as 0); stores are
// guarded per row.
template <typename T, int L>
__global__ __launch_bounds__(256) void k_chain_pair(
    ChainSplitDev c, T sigma, T tau, T a, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out, int nxcd,
    const int32_t* __restrict__ recs) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int Lh = L - Lb;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = Lh - 1;
  constexpr int NL = Lb - 1;
  constexpr int SPL = kChainStageRows / 128;  // staged row pairs per lane
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
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const T* s_dlo = reinterpret_cast<const T*>(smem + 16 * NLO);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(s_dlo + NLO);
  T* stage = reinterpret_cast<T*>(smem + BLOB) + (threadIdx.x >> 6) * kChainStageRows;
  __syncthreads();

  const int xcd = blockIdx.x % nxcd;
  const int blocks_x = gridDim.x / nxcd;
  const int64_t s_begin = c.nseg * xcd / nxcd, s_end = c.nseg * (xcd + 1) / nxcd;
  const int wpb = blockDim.x >> 6;
  const int64_t wstride = (int64_t)blocks_x * wpb;
  const int lane = threadIdx.x & 63;
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  const uint32_t vbytes = (uint32_t)(c.D * TB);
  const rsrc_t rb1 = make_rsrc(b1, vbytes), rv = make_rsrc(v, v ? vbytes : 0),
               rb2 = make_rsrc(b2, b2 ? vbytes : 0), rout = make_rsrc(out, vbytes);
  int64_t si = s_begin + (int64_t)(blockIdx.x / nxcd) * wpb + uniform(threadIdx.x >> 6);
  if (si >= s_end) return;
  for (; si < s_end; si += wstride) {
    const SegRec<NH> cur = load_rec<NH>(recs + (int64_t)uniform((int)si) * kChainRecWords);
    const int hi0 = cur.flags & 1, hitop = (cur.flags >> 1) & 1;
    const int bs = (cur.flags >> 2) & 1023, st = (cur.flags >> 12) & 1023;
    const int blk0 = cur.row0 - st;
    const uint32_t so_blk = (uint32_t)blk0 * TB, so_row = (uint32_t)cur.row0 * TB;
    const uint32_t pair_off = (uint32_t)(2 * lane) * TB;
    // stage the block: pairs of rows
    T sg[SPL][2];
#pragma unroll
    for (int m = 0; m < SPL; ++m) {
      if (128 * m < bs)
        bload2<T>(rb1, pair_off + (uint32_t)(128 * m) * TB, so_blk, sg[m][0], sg[m][1]);
      else
        sg[m][0] = sg[m][1] = T(0);
    }
    // the lane's two rows, clamped into the segment
    int jj[2], lo[2];
    u4 np[2];
    bool act_j[2], act_p[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      jj[i] = min(2 * lane + i, cur.len - 1);
      lo[i] = s_lo[cur.lidx + jj[i]];
      np[i] = s_np[lo[i]];
      act_j[i] = ((lo[i] >> (Lb - 1)) & 1) != hi0;
      act_p[i] = c.periodic && ((lo[i] & 1) != hitop);
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
      const int rj = (int)((np[i][2] >> 8) & 255u);
      const int rp = (int)((np[i][2] >> 16) & 255u);
      g_j[i] = act_j[i] ? bload<T>(rb1, (uint32_t)(blk0 + cur.d_join + rj) * TB, 0) : T(0);
      g_p[i] = act_p[i] ? bload<T>(rb1, (uint32_t)(blk0 + cur.d_pbc + rp) * TB, 0) : T(0);
    }
    if (v)
      bload2<T, kAuxNT>(rv, pair_off, so_row, vv[0], vv[1]);
    else
      vv[0] = vv[1] = T(0);
    if (b2)
      bload2<T, kAuxNT>(rb2, pair_off, so_row, bt[0], bt[1]);
    else
      bt[0] = bt[1] = T(0);
    wave_sync();  // the previous segment's LDS reads are done
#pragma unroll
    for (int m = 0; m < SPL; ++m) {
      const int r = 128 * m + 2 * lane;
      if (r < bs) {
        stage[r] = sg[m][0];
        if (r + 1 < bs) stage[r + 1] = sg[m][1];
      }
    }
    wave_sync();
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
      const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
      hop -= (T)(NL - __popc(xlo)) * bo;
      hop += act_j[i] ? g_j[i] : T(0);
      const int lo_top = (l >> (Lb - 1)) & 1, lo0 = l & 1;
      const int n11x = (lo_top & hi0) + (c.periodic ? (hitop & lo0) : 0);
      const T dg = s_dlo[l] + (T)cur.dhi + vzz * (T)n11x;
      const T acc = dg * bo + t_in * hop + (act_p[i] ? t_pb * g_p[i] : T(0));
      o[i] = sigma * acc + tau * bo - bt[i];
      if (v) o[i] += a * vv[i];
    }
    const int r0 = 2 * lane;
    if (r0 + 1 < cur.len)
      bstore2<kAuxNT>(o[0], o[1], rout, pair_off, so_row);
    else if (r0 < cur.len)
      bstore<kAuxNT>(o[0], rout, pair_off, so_row);
  }
}

template <typename T, int L>
static void launch_pair(hipStream_t s, const polfed_op* op, T sigma, T tau, T a, const T* v,
                        const T* b1, const T* b2, T* out) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int NLO = 1 << Lb;
  const size_t shm = chain_blob_bytes(NLO, (int)sizeof(T)) + 4 * kChainStageRows * sizeof(T);
  const int bpc = std::max(1, std::min(kChainBlocksPerCU, (int)(kLdsPerCU / shm)));
  ChainSplitDev c = op->chain_split();
  const int64_t blocks_needed = (c.nseg + 3) / 4;
  int64_t grid = std::min<int64_t>(blocks_needed, (int64_t)op->ctx->n_cu * bpc);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  grid = std::max<int64_t>(grid, 1);
  hipLaunchKernelGGL((k_chain_pair<T, L>), dim3((unsigned)grid), dim3(256), shm, s, c, sigma,
                     tau, a, v, b1, b2, out, nxcd, c.rec);
  HIPC(hipGetLastError());
}

// Tile variant for long chains: a workgroup stages a whole tile of 2^KT
// consecutive high parts of b_{i+1} in LDS (one coalesced read of its rows),
// so the low-part hops, the joining bond (high bit 0) and the KT - 1 bonds
// inside the tile's high bits are LDS reads; only the bonds among the
// remaining high bits and the periodic bond gather from global memory.  The
// tile's segments are shared among the workgroup's wavefronts; each lane
// holds two adjacent rows, as in the paired kernel.
template <typename T, int L, int KT>
__global__ __launch_bounds__(kTileThreads) void k_chain_tile(
    ChainSplitDev c, T sigma, T tau, T a, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out, int nxcd, int ntiles,
    const int32_t* __restrict__ recs, const int32_t* __restrict__ tiles) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int Lh = L - Lb;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = Lh - 1;   // bonds inside the high part
  constexpr int NHL = KT - 1;  // of which inside the tile: b < NHL
  constexpr int NL = Lb - 1;
  constexpr int BLOB = chain_blob_bytes(NLO, (int)sizeof(T));
  constexpr int CHUNKS = BLOB / 16;
  constexpr uint32_t TB = sizeof(T);
  using u4 = __attribute__((ext_vector_type(4))) uint32_t;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  {
    const u4* src = reinterpret_cast<const u4*>(sizeof(T) == 8 ? c.blob64 : c.blob32);
    u4* dst = reinterpret_cast<u4*>(smem);
    for (int i = threadIdx.x; i < CHUNKS; i += kTileThreads) dst[i] = src[i];
  }
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const T* s_dlo = reinterpret_cast<const T*>(smem + 16 * NLO);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(s_dlo + NLO);
  T* s_tile = reinterpret_cast<T*>(smem + BLOB);

  const int xcd = blockIdx.x % nxcd;
  const int wg = blockIdx.x / nxcd, nwg = gridDim.x / nxcd;
  const int t_begin = (int)((int64_t)ntiles * xcd / nxcd);
  const int t_end = (int)((int64_t)ntiles * (xcd + 1) / nxcd);
  const int wave = uniform(threadIdx.x >> 6);
  constexpr int NW = kTileThreads / 64;
  const int lane = threadIdx.x & 63;
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  const uint32_t vbytes = (uint32_t)(c.D * TB);
  const rsrc_t rb1 = make_rsrc(b1, vbytes), rv = make_rsrc(v, v ? vbytes : 0),
               rb2 = make_rsrc(b2, b2 ? vbytes : 0), rout = make_rsrc(out, vbytes);
  for (int t = t_begin + wg; t < t_end; t += nwg) {
    const int trow0 = tiles[4 * t], trows = tiles[4 * t + 1];
    const int tseg0 = tiles[4 * t + 2], tnseg = tiles[4 * t + 3];
    __syncthreads();  // the previous tile's LDS reads are done (and the tables)
    {  // two rows per thread and access; rows past the tile are not stored
      constexpr int U = 4;
      const uint32_t so = (uint32_t)trow0 * TB;
      for (int i0 = 0; i0 < trows; i0 += 2 * U * kTileThreads) {
        T x[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + 2 * (u * kTileThreads + (int)threadIdx.x);
          if (i < trows)
            bload2<T>(rb1, (uint32_t)i * TB, so, x[u][0], x[u][1]);
          else
            x[u][0] = x[u][1] = T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = i0 + 2 * (u * kTileThreads + (int)threadIdx.x);
          if (i < trows) s_tile[i] = x[u][0];
          if (i + 1 < trows) s_tile[i + 1] = x[u][1];
        }
      }
    }
    __syncthreads();
    for (int si = tseg0 + wave; si < tseg0 + tnseg; si += NW) {
      const SegRec<NH> cur = load_rec<NH>(recs + (int64_t)uniform(si) * kChainRecWords);
      const int hi0 = cur.flags & 1, hitop = (cur.flags >> 1) & 1;
      const int st = (cur.flags >> 12) & 1023;
      const int blk0 = cur.row0 - st;
      const int lrow0 = cur.row0 - trow0, lblk0 = blk0 - trow0;
      const uint32_t so_row = (uint32_t)cur.row0 * TB;
      const uint32_t pair_off = (uint32_t)(2 * lane) * TB;
      // lane l holds the adjacent rows 2l and 2l + 1 (clamped into the segment)
      int jj[2], lo[2];
      u4 np[2];
      bool act_j[2], act_p[2];
      T g_hi[NH - NHL > 0 ? NH - NHL : 1][2], g_p[2], vv[2], bt[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        jj[i] = min(2 * lane + i, cur.len - 1);
        const int l = s_lo[cur.lidx + jj[i]];
        lo[i] = l;
        np[i] = s_np[l];
        act_j[i] = ((l >> (Lb - 1)) & 1) != hi0;
        act_p[i] = c.periodic && ((l & 1) != hitop);
      }
#pragma unroll
      for (int b = NHL; b < NH; ++b) {
        if (cur.dh[b] != 0)
          bload2<T>(rb1, pair_off, (uint32_t)(cur.row0 + cur.dh[b]) * TB, g_hi[b - NHL][0],
                    g_hi[b - NHL][1]);
        else
          g_hi[b - NHL][0] = g_hi[b - NHL][1] = T(0);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int rp = (int)((np[i][2] >> 16) & 255u);
        g_p[i] = act_p[i] ? bload<T>(rb1, (uint32_t)(blk0 + cur.d_pbc + rp) * TB, 0) : T(0);
      }
      if (v)
        bload2<T, kAuxNT>(rv, pair_off, so_row, vv[0], vv[1]);
      else
        vv[0] = vv[1] = T(0);
      if (b2)
        bload2<T, kAuxNT>(rb2, pair_off, so_row, bt[0], bt[1]);
      else
        bt[0] = bt[1] = T(0);
      T o[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int l = lo[i];
        const int lr = lrow0 + jj[i];
        const T bo = s_tile[lr];
        T hop = 0;
#pragma unroll
        for (int b = 0; b < NL; ++b)
          hop += s_tile[lblk0 + (int)((np[i][b >> 2] >> (8 * (b & 3))) & 255u)];
        const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
        hop -= (T)(NL - __popc(xlo)) * bo;
#pragma unroll
        for (int b = 0; b < NHL; ++b)
          if (cur.dh[b] != 0) hop += s_tile[lr + cur.dh[b]];
#pragma unroll
        for (int b = NHL; b < NH; ++b) hop += g_hi[b - NHL][i];
        const int rj = (int)((np[i][2] >> 8) & 255u);
        if (act_j[i]) hop += s_tile[lblk0 + cur.d_join + rj];
        const int lo_top = (l >> (Lb - 1)) & 1, lo0 = l & 1;
        const int n11x = (lo_top & hi0) + (c.periodic ? (hitop & lo0) : 0);
        const T dg = s_dlo[l] + (T)cur.dhi + vzz * (T)n11x;
        const T acc = dg * bo + t_in * hop + (act_p[i] ? t_pb * g_p[i] : T(0));
        o[i] = sigma * acc + tau * bo - bt[i];
        if (v) o[i] += a * vv[i];
      }
      const int r0 = 2 * lane;
      if (r0 + 1 < cur.len)
        bstore2<kAuxNT>(o[0], o[1], rout, pair_off, so_row);
      else if (r0 < cur.len)
        bstore<kAuxNT>(o[0], rout, pair_off, so_row);
    }
  }
}

// XCDs of the device: the staged-tile table carries this many ranges.
constexpr int kWtXcds = 8;

// Staged-tile kernel.  A tile is the set of rows whose state bits outside
// [0, Lb + KT) (and, for a wrapped tile, outside the top bit L - 1) are
// fixed: 2^WR runs of 2^KT consecutive high parts, each run a contiguous
// range of rows.  The workgroup copies the tile's rows of b_{i+1}, and the
// records of its segments, into LDS with direct-to-LDS buffer loads (one
// 16-byte load per lane fills 1 KB of LDS, no registers involved), so that
//   - the low-part hops, the joining bond and the KT - 1 bonds among the
//     tile's high bits read LDS;
//   - in a wrapped tile the periodic bond (L - 1, 0) reads LDS too: its
//     target differs in the top bit, so it lies in the tile's other run;
//   - only the bonds between the tile's high bits and the fixed middle
//     bits gather from global memory, at wave-uniform row offsets;
//   - a segment's record and its rows' low-part tables (in list order) are
//     LDS reads, so the global gathers of a segment start after two short
//     LDS round trips instead of a scalar load from global memory.
// With DB the next tile is staged into a second LDS buffer while the current
// one is processed.
template <typename T, int L, int KT, int WR, int DB, int NT>
__global__ __launch_bounds__(NT) void k_chain_wt(
    ChainSplitDev c, T sigma, T tau, T a, const T* __restrict__ v,
    const T* __restrict__ b1, const T* b2, T* out, int nxcd, int ntiles, int buf_rows,
    int rec_slots, const int32_t* __restrict__ recs, const int32_t* __restrict__ tiles) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int NLO = 1 << Lb;
  constexpr int NH = L - Lb - 1;  // bonds inside the high part
  constexpr int NHL = KT - 1;     // of which inside the tile: b < NHL
  constexpr int NL = Lb - 1;
  constexpr int BLOB = chain_blob_bytes(NLO, (int)sizeof(T));
  constexpr int CHUNKS = BLOB / 16;
  constexpr int CH = 1024 / (int)sizeof(T);  // rows per staging load of a wave
  constexpr int RB = kChainRecWords * 4;      // bytes per segment record
  constexpr int NW = NT / 64;
  constexpr uint32_t TB = sizeof(T);
  using u4 = __attribute__((ext_vector_type(4))) uint32_t;
  using lds_ptr = __attribute__((address_space(3))) void*;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  {
    const u4* src = reinterpret_cast<const u4*>(sizeof(T) == 8 ? c.blobl64 : c.blobl32);
    u4* dst = reinterpret_cast<u4*>(smem);
    for (int i = threadIdx.x; i < CHUNKS; i += NT) dst[i] = src[i];
  }
  // list-ordered tables: entry p describes the p-th low part of the list
  const u4* s_np = reinterpret_cast<const u4*>(smem);
  const T* s_dlo = reinterpret_cast<const T*>(smem + 16 * NLO);
  const uint16_t* s_lo = reinterpret_cast<const uint16_t*>(s_dlo + NLO);
  // per buffer: buf_rows rows of b_{i+1}, then rec_slots segment records
  const size_t buf_bytes = (size_t)buf_rows * TB + (size_t)rec_slots * RB;
  unsigned char* const s_b0 = smem + BLOB;
  unsigned char* const s_b1 = s_b0 + (DB ? buf_bytes : 0);

  const int xcd = blockIdx.x % nxcd;
  const int wg = blockIdx.x / nxcd, nwg = gridDim.x / nxcd;
  // the XCD's range of the tile table (row-balanced bounds after the
  // entries; one XCD takes them all)
  const int t_begin = nxcd == kWtXcds ? uniform(tiles[8 * ntiles + xcd]) : 0;
  const int t_end = nxcd == kWtXcds ? uniform(tiles[8 * ntiles + xcd + 1]) : ntiles;
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const T vzz = (T)c.vzz, t_in = (T)c.t_in, t_pb = (T)c.t_pb;
  const uint32_t vbytes = (uint32_t)(c.D * TB);
  const rsrc_t rb1 = make_rsrc(b1, vbytes), rv = make_rsrc(v, v ? vbytes : 0),
               rb2 = make_rsrc(b2, b2 ? vbytes : 0), rout = make_rsrc(out, vbytes),
               rrec = make_rsrc(recs, (uint32_t)(c.nseg * RB));
  // the tile's runs of rows and of segment records into a buffer, in chunks
  // of 1 KB dealt round robin to the waves; a run's last chunk spills into
  // the run's padding
  auto stage = [&](int t, unsigned char* buf) {
    const int32_t* tt = tiles + 8 * t;
    int rbase = 0, sbase = 0;
#pragma unroll
    for (int r = 0; r < (1 << WR); ++r) {
      const int row0 = tt[4 * r], rows = tt[4 * r + 1];
      const int seg0 = tt[4 * r + 2], nseg = tt[4 * r + 3];
      const int nch = (rows + CH - 1) / CH;
      for (int ch = wave; ch < nch; ch += NW)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rb1, (lds_ptr)(buf + (size_t)(rbase + ch * CH) * TB), 16,
            (uint32_t)(ch * CH) * TB + 16u * lane, (uint32_t)row0 * TB, 0, 0);
      const int nrc = (nseg + 7) / 8;
      for (int ch = wave; ch < nrc; ch += NW)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rrec, (lds_ptr)(buf + (size_t)buf_rows * TB + (size_t)(sbase + 8 * ch) * RB), 16,
            (uint32_t)(8 * ch * RB) + 16u * lane, (uint32_t)seg0 * RB, 0, 0);
      rbase += nch * CH;
      sbase += nrc * 8;
    }
  };
  int t = t_begin + wg;
  if (DB && t < t_end) stage(t, s_b0);
  for (int it = 0; t < t_end; t += nwg, ++it) {
    unsigned char* const cb = (DB && (it & 1)) ? s_b1 : s_b0;
    if (DB) {
      // this tile was requested one iteration ago; once every wave has it
      // (and is done with the other buffer), stage the next tile
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (t + nwg < t_end) stage(t + nwg, (it & 1) ? s_b0 : s_b1);
    } else {
      __syncthreads();  // the previous tile's LDS reads are done
      stage(t, s_b0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    const T* const cur_buf = reinterpret_cast<const T*>(cb);
    const int32_t* const s_rec = reinterpret_cast<const int32_t*>(cb + (size_t)buf_rows * TB);
    const int32_t* tt = tiles + 8 * t;
    const int r0row = tt[0], r0nseg = tt[3];
    const int r1row = WR ? tt[4] : 0, r1nseg = WR ? tt[7] : 0;
    const int base1 = WR ? ((tt[1] + CH - 1) / CH) * CH : 0;
    const int sbase1 = ((r0nseg + 7) / 8) * 8;
    const int nsegs = r0nseg + r1nseg;
    for (int j = wave; j < nsegs; j += NW) {
      const bool in1 = WR && j >= r0nseg;
      // LDS index = global row + shift (own run), + pshift (the other run)
      const int shift = in1 ? base1 - r1row : -r0row;
      const int pshift = in1 ? -r0row : base1 - r1row;
      const SegRec<NH> cur = load_rec<NH>(s_rec + (in1 ? sbase1 + j - r0nseg : j) * kChainRecWords);
      const int hi0 = cur.flags & 1, hitop = (cur.flags >> 1) & 1;
      const int st = (cur.flags >> 12) & 1023;
      const int blk0 = cur.row0 - st;
      const int lrow0 = cur.row0 + shift, lblk0 = blk0 + shift;
      const uint32_t so_row = (uint32_t)cur.row0 * TB;
      const uint32_t pair_off = (uint32_t)(2 * lane) * TB;
      // global gathers first: high-part hops at uniform offsets, the
      // periodic bond of an unwrapped tile, the streamed v and b_{i+2}
      T g_hi[NH - NHL > 0 ? NH - NHL : 1][2], vv[2], bt[2];
#pragma unroll
      for (int b = NHL; b < NH; ++b) {
        if (cur.dh[b] != 0)
          bload2<T>(rb1, pair_off, (uint32_t)(cur.row0 + cur.dh[b]) * TB, g_hi[b - NHL][0],
                    g_hi[b - NHL][1]);
        else
          g_hi[b - NHL][0] = g_hi[b - NHL][1] = T(0);
      }
      if (v)
        bload2<T, kAuxNT>(rv, pair_off, so_row, vv[0], vv[1]);
      else
        vv[0] = vv[1] = T(0);
      if (b2)
        bload2<T, kAuxNT>(rb2, pair_off, so_row, bt[0], bt[1]);
      else
        bt[0] = bt[1] = T(0);
      // the lane's rows 2 lane and 2 lane + 1 (clamped into the segment)
      int jj[2], lo[2];
      u4 np[2];
      T dl[2];
      bool act_j[2], act_p[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        jj[i] = min(2 * lane + i, cur.len - 1);
        const int q = cur.lidx + jj[i];
        lo[i] = s_lo[q];
        np[i] = s_np[q];
        dl[i] = s_dlo[q];
      }
      T g_p[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int l = lo[i];
        act_j[i] = ((l >> (Lb - 1)) & 1) != hi0;
        act_p[i] = c.periodic && ((l & 1) != hitop);
        if (!WR) {
          const int rp = (int)((np[i][2] >> 16) & 255u);
          g_p[i] = act_p[i] ? bload<T>(rb1, (uint32_t)(blk0 + cur.d_pbc + rp) * TB, 0) : T(0);
        }
      }
      // every LDS operand of both rows is read before any is summed (an
      // idle in-tile high bond reads the row itself and is masked; the
      // joining and periodic reads are clamped into the buffer and masked)
      T bo[2], nb[2][NL > 0 ? NL : 1], th[2][NHL > 0 ? NHL : 1], tj[2], tp[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int lr = lrow0 + jj[i];
        bo[i] = cur_buf[lr];
#pragma unroll
        for (int b = 0; b < NL; ++b)
          nb[i][b] = cur_buf[lblk0 + (int)((np[i][b >> 2] >> (8 * (b & 3))) & 255u)];
#pragma unroll
        for (int b = 0; b < NHL; ++b) th[i][b] = cur_buf[lr + cur.dh[b]];
        const int rj = (int)((np[i][2] >> 8) & 255u);
        tj[i] = cur_buf[min(lblk0 + cur.d_join + rj, buf_rows - 1)];
        if (WR) {
          const int rp = (int)((np[i][2] >> 16) & 255u);
          tp[i] = cur_buf[min(blk0 + cur.d_pbc + rp + pshift, buf_rows - 1)];
        }
      }
      T o[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int l = lo[i];
        T hop = 0;
#pragma unroll
        for (int b = 0; b < NL; ++b) hop += nb[i][b];
        const int xlo = (l ^ (l >> 1)) & ((1 << NL) - 1);
        hop -= (T)(NL - __popc(xlo)) * bo[i];
#pragma unroll
        for (int b = 0; b < NHL; ++b) hop += cur.dh[b] != 0 ? th[i][b] : T(0);
#pragma unroll
        for (int b = NHL; b < NH; ++b) hop += g_hi[b - NHL][i];
        hop += act_j[i] ? tj[i] : T(0);
        if (WR) g_p[i] = act_p[i] ? tp[i] : T(0);
        const int lo_top = (l >> (Lb - 1)) & 1, lo0 = l & 1;
        const int n11x = (lo_top & hi0) + (c.periodic ? (hitop & lo0) : 0);
        const T dg = dl[i] + (T)cur.dhi + vzz * (T)n11x;
        const T acc = dg * bo[i] + t_in * hop + (act_p[i] ? t_pb * g_p[i] : T(0));
        o[i] = sigma * acc + tau * bo[i] - bt[i];
        if (v) o[i] += a * vv[i];
      }
      const int r0 = 2 * lane;
      if (r0 + 1 < cur.len)
        bstore2<kAuxNT>(o[0], o[1], rout, pair_off, so_row);
      else if (r0 < cur.len)
        bstore<kAuxNT>(o[0], rout, pair_off, so_row);
    }
  }
}

// Staged-tile configurations: tile bits (below the largest tile bits of the
// chain), wrap, double buffer, threads per workgroup.
struct WtConf {
  int dkt, wrap, db, nt;
};
constexpr WtConf kWtConf[] = {
    {0, 1, 0, 1024},  // 6: largest wrapped tile, one buffer, 16 waves
    {1, 1, 1, 512},   // 7: half-size wrapped tile, two buffers, 8 waves
    {1, 1, 0, 512},   // 8: half-size wrapped tile, one buffer, 8 waves
    {0, 1, 1, 1024},  // 9: largest wrapped tile, two buffers (FP32 fits)
};
constexpr int kWtFirst = 6, kWtCount = (int)(sizeof(kWtConf) / sizeof(kWtConf[0]));

// Tile bits of the staged-tile kernel's largest tile at chain length L.
constexpr int chain_wt_bits(int L) {
  const int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  const int Lh = L - Lb;
  const int kt = Lh - 10 < 4 ? Lh - 10 : 4;
  return (L >= 20 && kt >= 2) ? kt : 0;
}

static const polfed_op::WTiles* wt_tables(const polfed_op* op, int kt, int wrap) {
  const int key = kt * 2 + wrap;
  auto it = op->wtiles.find(key);
  if (it != op->wtiles.end()) return it->second.n > 0 ? &it->second : nullptr;
  polfed_op::WTiles& W = op->wtiles[key];
  const int Lh = op->L - op->split_Lb;
  if (kt < 1 || Lh - kt - wrap < 3 || op->split_hi_off.empty()) return nullptr;
  const auto& ho = op->split_hi_off;
  const auto& so = op->split_seg_of_hi;
  const int64_t nt = (int64_t)1 << (Lh - kt - wrap);
  TallyScope untallied(nullptr);  // the table lives as long as the operator
  std::vector<int32_t> tab;
  std::vector<int64_t> tid;   // the tile index t of each entry
  std::vector<int> trows;     // its rows
  for (int64_t t = 0; t < nt; ++t) {
    int32_t e[8] = {0};
    int rows_tot = 0, bufr[2] = {0, 0}, slots = 0;
    for (int r = 0; r <= wrap; ++r) {
      const int64_t h0 = ((int64_t)r << (Lh - 1)) | (t << kt), h1 = h0 + ((int64_t)1 << kt);
      e[4 * r] = ho[h0];
      e[4 * r + 1] = ho[h1] - ho[h0];
      e[4 * r + 2] = so[h0];
      e[4 * r + 3] = so[h1] - so[h0];
      rows_tot += e[4 * r + 1];
      slots += ((e[4 * r + 3] + 7) / 8) * 8;
      for (int p = 0; p < 2; ++p) {
        const int ch = p == 0 ? 128 : 256;
        bufr[p] += ((e[4 * r + 1] + ch - 1) / ch) * ch;
      }
    }
    if (rows_tot == 0) continue;
    tab.insert(tab.end(), e, e + 8);
    tid.push_back(t);
    trows.push_back(rows_tot);
    for (int p = 0; p < 2; ++p) W.buf_rows[p] = std::max(W.buf_rows[p], bufr[p]);
    W.rec_slots = std::max(W.rec_slots, slots);
  }
  W.kt = kt;
  W.wrap = wrap;
  W.n = (int)(tab.size() / 8);
  // Order of the tiles and their split over the XCDs.  A hop across a bond
  // between two fixed bits of a tile swaps them, which keeps the popcount of
  // the fixed bits t; only the bonds at the ends of the fixed range change
  // it.  Tiles sorted by popcount(t), then by the popcount of the upper half
  // of t (swaps inside either half keep it), then by t, therefore keep most
  // of their global gathers inside a contiguous range of the table, and each
  // XCD takes such a range, cut where the rows (not the tiles) are balanced.
  // Hopping gathers sent to another XCD's range, counted over the sector:
  // 26.6% instead of 39.9% in plain t order at L = 24, 22.1% instead of
  // 33.2% at L = 26, 38.8% instead of 50.3% at L = 22.
  const int tbits = Lh - kt - wrap, thalf = (tbits + 1) / 2;
  std::vector<int> ord(W.n);
  std::iota(ord.begin(), ord.end(), 0);
  auto order_key = [&](int x) {
    const unsigned long long t = (unsigned long long)tid[x];
    return std::make_tuple(__builtin_popcountll(t), __builtin_popcountll(t >> (tbits - thalf)),
                           tid[x]);
  };
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int x, int y) { return order_key(x) < order_key(y); });
  std::vector<int32_t> sorted;
  sorted.reserve(tab.size() + kWtXcds + 1);
  int64_t rows_all = 0;
  for (int i : ord) {
    sorted.insert(sorted.end(), tab.begin() + 8 * (size_t)i, tab.begin() + 8 * (size_t)i + 8);
    rows_all += trows[i];
  }
  // XCD x takes entries [bound[x], bound[x + 1]): bound[x] is the first
  // entry whose rows before it reach x/8 of all rows
  int64_t cum = 0;
  int x = 1;
  sorted.push_back(0);
  for (int k = 0; k < W.n && x < kWtXcds; ++k) {
    while (x < kWtXcds && cum >= rows_all * x / kWtXcds) {
      sorted.push_back(k);
      ++x;
    }
    cum += trows[ord[k]];
  }
  while (x < kWtXcds) {
    sorted.push_back(W.n);
    ++x;
  }
  sorted.push_back(W.n);
  tab.swap(sorted);
  upload(W.d, tab.data(), tab.size(), op->ctx->stream);
  HIPC(hipStreamSynchronize(op->ctx->stream));
  return W.n > 0 ? &W : nullptr;
}

bool chain_wt_exists(const polfed_op* op, int var, bool fp32) {
  if (op->model != Model::Chain || op->split_nseg <= 0) return false;
  if (var < kWtFirst || var >= kWtFirst + kWtCount) return false;
  const WtConf C = kWtConf[var - kWtFirst];
  const int KT = chain_wt_bits(op->L) - C.dkt;
  if (chain_wt_bits(op->L) == 0 || KT < 1) return false;
  const polfed_op::WTiles* W = wt_tables(op, KT, C.wrap);
  if (!W) return false;
  const size_t tb = fp32 ? 4 : 8;
  const size_t shm = chain_blob_bytes(1 << op->split_Lb, (int)tb) +
                     (size_t)(C.db ? 2 : 1) * ((size_t)W->buf_rows[fp32 ? 1 : 0] * tb +
                                               (size_t)W->rec_slots * kChainRecWords * 4);
  return shm <= kLdsPerCU;
}

template <typename T, int L, int KT, int WR, int DB, int NT>
static bool launch_wt(hipStream_t s, const polfed_op* op, T sigma, T tau, T a, const T* v,
                      const T* b1, const T* b2, T* out) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  const polfed_op::WTiles* W = wt_tables(op, KT, WR);
  if (!W) return false;
  const int buf_rows = W->buf_rows[sizeof(T) == 8 ? 0 : 1];
  const size_t shm = chain_blob_bytes(1 << Lb, (int)sizeof(T)) +
                     (size_t)(DB ? 2 : 1) * ((size_t)buf_rows * sizeof(T) +
                                              (size_t)W->rec_slots * kChainRecWords * 4);
  if (shm > kLdsPerCU) return false;
  const int per_cu = std::max(1, std::min((int)(kLdsPerCU / shm), 2048 / NT));
  ChainSplitDev c = op->chain_split();
  int64_t grid = std::min<int64_t>(W->n, (int64_t)op->ctx->n_cu * per_cu);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % kWtXcds;
    nxcd = kWtXcds;
  }
  grid = std::max<int64_t>(grid, 1);
  hipLaunchKernelGGL((k_chain_wt<T, L, KT, WR, DB, NT>), dim3((unsigned)grid), dim3(NT), shm, s,
                     c, sigma, tau, a, v, b1, b2, out, nxcd, W->n, buf_rows, W->rec_slots,
                     c.rec, W->d.as<int32_t>());
  HIPC(hipGetLastError());
  return true;
}

template <typename T, int L, int I>
static bool launch_wt_conf(hipStream_t s, const polfed_op* op, T sigma, T tau, T a, const T* v,
                           const T* b1, const T* b2, T* out) {
  constexpr WtConf C = kWtConf[I];
  constexpr int KT = chain_wt_bits(L) - C.dkt;
  if constexpr (chain_wt_bits(L) == 0 || KT < 1) {
    return false;
  } else {
    return launch_wt<T, L, KT, C.wrap, C.db, C.nt>(s, op, sigma, tau, a, v, b1, b2, out);
  }
}

template <typename T, int L, int... I>
static bool launch_wt_any(hipStream_t s, const polfed_op* op, int i, T sigma, T tau, T a,
                          const T* v, const T* b1, const T* b2, T* out,
                          std::integer_sequence<int, I...>) {
  bool ok = false;
  ((i == I ? (ok = launch_wt_conf<T, L, I>(s, op, sigma, tau, a, v, b1, b2, out), 0) : 0), ...);
  return ok;
}

// Launch shape: kChainBlocksPerCU persistent blocks per CU, the blocks of a
// launch mapped XCD-contiguously once there are enough of them.

template <typename T, int L, int HALVES = 1>
static void launch_split(hipStream_t s, const polfed_op* op, T sigma, T tau, T a,
                         const T* v, const T* b1, const T* b2, T* out) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int NLO = 1 << Lb;
  constexpr int bpc = kChainBlocksPerCU;
  const size_t shm = chain_blob_bytes(NLO, (int)sizeof(T)) + 4 * kChainStageRows * sizeof(T);
  ChainSplitDev c = op->chain_split();
  const int64_t blocks_needed = (c.nseg * HALVES + 3) / 4;
  int64_t grid = std::min<int64_t>(blocks_needed, (int64_t)op->ctx->n_cu * bpc);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  grid = std::max<int64_t>(grid, 1);
  hipLaunchKernelGGL((k_chain_split<T, L, HALVES>), dim3((unsigned)grid), dim3(256), shm, s, c,
                     sigma, tau, a, v, b1, b2, out, nxcd, c.rec);
  HIPC(hipGetLastError());
}

template <typename T, int L, int KT>
static void launch_tile(hipStream_t s, const polfed_op* op, const polfed_op::Tiles& tl, T sigma,
                        T tau, T a, const T* v, const T* b1, const T* b2, T* out) {
  constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
  constexpr int NLO = 1 << Lb;
  const size_t shm = chain_blob_bytes(NLO, (int)sizeof(T)) + (size_t)tl.max_rows * sizeof(T);
  const int per_cu = std::max(1, (int)(kLdsPerCU / shm));
  ChainSplitDev c = op->chain_split();
  int64_t grid = std::min<int64_t>(tl.n, (int64_t)op->ctx->n_cu * per_cu);
  int nxcd = 1;
  if (grid >= 64) {
    grid -= grid % 8;
    nxcd = 8;
  }
  grid = std::max<int64_t>(grid, 1);
  hipLaunchKernelGGL((k_chain_tile<T, L, KT>), dim3((unsigned)grid), dim3(kTileThreads), shm, s, c,
                     sigma, tau, a, v, b1, b2, out, nxcd, tl.n, c.rec, tl.d.as<int32_t>());
  HIPC(hipGetLastError());
}

// Step-kernel variants of a chain: 0 = segment kernel, 1 + i = tile kernel
// with tiles[i].  Returns false for a variant that does not exist.
template <typename T, int L>
static bool launch_variant(hipStream_t s, const polfed_op* op, int var, T sigma, T tau, T a,
                           const T* v, const T* b1, const T* b2, T* out) {
  constexpr int KT = chain_tile_bits(L);
  if (var == 0) {
    launch_split<T, L>(s, op, sigma, tau, a, v, b1, b2, out);
    return true;
  }
  if (var == 3) {
    launch_pair<T, L>(s, op, sigma, tau, a, v, b1, b2, out);
    return true;
  }
  if (var == 4) {
    launch_split<T, L, 2>(s, op, sigma, tau, a, v, b1, b2, out);
    return true;
  }
  if (var >= kWtFirst && var < kWtFirst + kWtCount)
    return launch_wt_any<T, L>(s, op, var - kWtFirst, sigma, tau, a, v, b1, b2, out,
                               std::make_integer_sequence<int, kWtCount>{});
  if constexpr (KT >= 2) {
    constexpr int Lb = (L / 2 < kChainLoBits) ? L / 2 : kChainLoBits;
    if (var != 1 && var != 2 && var != 5) return false;
    const auto& tl = op->tiles[var == 5 ? 2 : var - 1];
    if (tl.n <= 0) return false;
    if (chain_blob_bytes(1 << Lb, (int)sizeof(T)) + (size_t)tl.max_rows * sizeof(T) > kLdsPerCU)
      return false;
    if (var == 1 && tl.bits == KT) {
      launch_tile<T, L, KT>(s, op, tl, sigma, tau, a, v, b1, b2, out);
      return true;
    }
    if constexpr (KT - 1 >= 2) {
      if (var == 2 && tl.bits == KT - 1) {
        launch_tile<T, L, KT - 1>(s, op, tl, sigma, tau, a, v, b1, b2, out);
        return true;
      }
    }
    if constexpr (KT - 2 >= 2) {
      if (var == 5 && tl.bits == KT - 2) {
        launch_tile<T, L, KT - 2>(s, op, tl, sigma, tau, a, v, b1, b2, out);
        return true;
      }
    }
  }
  return false;
}

// Picks the fastest variant for (op, precision) by replaying 20 launches of
// each on scratch vectors; not while the stream is being captured.  The
// choice is shared by the context's operators of the same chain pattern
// (same kernels and tables, other diagonals).
template <typename T, int L>
static int tuned_variant(hipStream_t s, const polfed_op* op) {
  const int pi = sizeof(T) == 8 ? 0 : 1;
  if (op->tuned[pi] >= 0) return op->tuned[pi];
  const std::string pkey = std::string(sizeof(T) == 8 ? "step64" : "step32");
  {
    const int v = pattern_choice(op, pkey);
    if (v >= 0) return op->tuned[pi] = v;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPC(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return 0;
  const size_t n = (size_t)op->D;
  DevBuf bv(n * sizeof(T)), bb1(n * sizeof(T)), bb2(n * sizeof(T));
  HIPC(hipMemsetAsync(bv.get(), 0, n * sizeof(T), s));
  HIPC(hipMemsetAsync(bb1.get(), 0, n * sizeof(T), s));
  HIPC(hipMemsetAsync(bb2.get(), 0, n * sizeof(T), s));
  HIPC(hipStreamSynchronize(s));  // the operator's tables and the scratch vectors
  int best = 0;
  float best_us = 1e30f;
  for (int var = 0; var < kWtFirst + kWtCount; ++var) {
    const bool ok = launch_variant<T, L>(s, op, var, T(0.1), T(0), T(0), bv.as<T>(),
                                         bb1.as<T>(), bb2.as<T>(), bb2.as<T>());
    if (!ok) continue;
    HIPC(hipStreamSynchronize(s));
    const float us = replay_time_us(
        [&](hipStream_t ts) {
          launch_variant<T, L>(ts, op, var, T(0.1), T(0), T(0), bv.as<T>(), bb1.as<T>(),
                               bb2.as<T>(), bb2.as<T>());
        },
        20);
    if (verbose())
      std::fprintf(stderr, "[polfed] chain step L=%d %s variant %d: %.2f us\n", L,
                   sizeof(T) == 8 ? "fp64" : "fp32", var, us);
    if (us < best_us) {
      best_us = us;
      best = var;
    }
  }
  HIPC(hipStreamSynchronize(s));
  pattern_choice_set(op, pkey, best);
  return op->tuned[pi] = best;
}

template <typename T>
bool chain_split_step(hipStream_t s, const polfed_op* op, T sigma, T tau, T a,
                      const T* v, const T* b1, const T* b2, T* out) {
  if (op->split_nseg <= 0) return false;
  switch (op->L) {
#define POLFED_CASE(LL)                                                                     \
  case LL:                                                                                  \
    if (!launch_variant<T, LL>(s, op, tuned_variant<T, LL>(s, op), sigma, tau, a, v, b1, b2, \
                               out))                                                        \
      launch_split<T, LL>(s, op, sigma, tau, a, v, b1, b2, out);                            \
    return true;
    POLFED_CASE(4) POLFED_CASE(5) POLFED_CASE(6) POLFED_CASE(7) POLFED_CASE(8)
    POLFED_CASE(9) POLFED_CASE(10) POLFED_CASE(11) POLFED_CASE(12) POLFED_CASE(13)
    POLFED_CASE(14) POLFED_CASE(15) POLFED_CASE(16) POLFED_CASE(17) POLFED_CASE(18)
    POLFED_CASE(19) POLFED_CASE(20) POLFED_CASE(21) POLFED_CASE(22) POLFED_CASE(23)
    POLFED_CASE(24) POLFED_CASE(25) POLFED_CASE(26) POLFED_CASE(27) POLFED_CASE(28)
#undef POLFED_CASE
    default: return false;
  }
}

template bool chain_split_step<double>(hipStream_t, const polfed_op*, double, double, double,
                                       const double*, const double*, const double*, double*);
template bool chain_split_step<float>(hipStream_t, const polfed_op*, float, float, float,
                                      const float*, const float*, const float*, float*);

}  // namespace polfed

polfed::ChainSplitDev polfed_op::chain_split() const {
  polfed::ChainSplitDev c{};
  c.D = D;
  c.N = N;
  c.periodic = periodic;
  c.t_in = t_in;
  c.t_pb = t_pb;
  c.vzz = vzz;
  c.blob64 = d_blob64.get();
  c.blob32 = d_blob32.get();
  c.blobl64 = d_blobl64.get();
  c.blobl32 = d_blobl32.get();
  c.rec = d_rec.as<int32_t>();
  c.nseg = split_nseg;
  return c;
}

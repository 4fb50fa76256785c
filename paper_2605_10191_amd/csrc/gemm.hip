// FP64 products of tall matrices on the matrix cores (v_mfma_f64_16x16x4f64).
//
// The extraction of Sec. 4.3 forms u_i = V t_i for the selected Ritz vectors
// (a D x m basis times an m x n coefficient block), the projection of H on
// their span (an n x n product with inner dimension D) and the rotations of
// the Rayleigh-Ritz step; a block Gram-Schmidt pass of Sec. 2.2 forms
// C = V^T W and W -= V C.  All are dense FP64 contractions with one very
// long dimension D, so they run as 64 x 64 output tiles on the MFMA units:
//   - nn:  C (D x n) = A (D x m) B (m x n), or C -= A B; one workgroup per
//          64 x 64 tile of C, the inner dimension m in chunks of 32 staged
//          in LDS;
//   - tn:  G (n1 x n2) = A^T B with A (D x n1), B (D x n2); the long inner
//          dimension D is split over workgroups (at least 2,048 rows each),
//          whose partial tiles are summed in a fixed order by a second
//          kernel, so the result does not depend on timing.
// Each of the four waves of a workgroup computes a 32 x 32 quarter of the
// tile as 2 x 2 MFMA blocks of 16 x 16.  The MFMA's M index runs over the
// output columns and its N index over the output rows, so that the 16 lanes
// of a group hold consecutive rows of one column and every store of a wave
// writes 128-byte runs of four columns.
//
// Lane layout of v_mfma_f64_16x16x4f64 (wave64, checked on the device):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of the 16 x 4 and
// 4 x 16 operands and receives C[l / 16 + 4 r][l % 16], r = 0..3, of the
// 16 x 16 result.
#include <algorithm>

#include "internal.hpp"

namespace polfed {

namespace {

using d4 = __attribute__((ext_vector_type(4))) double;
constexpr int kT = 64;       // output tile edge
constexpr int kKC = 32;      // inner chunk staged per iteration
constexpr int kPad = 2;      // LDS row padding (doubles)
constexpr int kTnMinRows = 2048;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The 2 x 2 blocks of a wave: MFMA A operand from sM ([k][M index]), B
// operand from sN ([k][N index]), over one staged chunk of kKC.
__device__ __forceinline__ void mfma_chunk(const double (*sM)[kT + kPad],
                                           const double (*sN)[kT + kPad], int wm, int wn,
                                           int lane, d4 (&acc)[2][2]) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < kKC; ks += 4) {
    double a[2], b[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      a[q] = sM[ks + lk][wm * 32 + q * 16 + li];
      b[q] = sN[ks + lk][wn * 32 + q * 16 + li];
    }
#pragma unroll
    for (int qm = 0; qm < 2; ++qm)
#pragma unroll
      for (int qn = 0; qn < 2; ++qn) acc[qm][qn] = mfma(a[qm], b[qn], acc[qm][qn]);
  }
}

// C = A B (SUB: C -= A B).  Tile (blockIdx.x: 64 rows of D, blockIdx.y: 64
// columns of n); MFMA M = columns of C, N = rows of C, K = m.
template <bool SUB>
__global__ __launch_bounds__(256) void k_gemm_nn(int64_t D, int m, int n, const double* A,
                                                 int64_t lda, const double* B, int64_t ldb,
                                                 double* C, int64_t ldc) {
  __shared__ double sA[kKC][kT + kPad];  // [k][row]
  __shared__ double sB[kKC][kT + kPad];  // [k][col]
  const int64_t I0 = (int64_t)blockIdx.x * kT;
  const int J0 = blockIdx.y * kT;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wn = w & 1, wm = w >> 1;  // wave's row half (N) and column half (M)
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
  for (int k0 = 0; k0 < m; k0 += kKC) {
    // A chunk: 64 rows x 32 k, coalesced along the rows of each column
#pragma unroll
    for (int q = 0; q < kT * kKC / 256; ++q) {
      const int idx = t + 256 * q, kk = idx / kT, ii = idx % kT;
      const int64_t r = I0 + ii;
      const int k = k0 + kk;
      sA[kk][ii] = (r < D && k < m) ? A[r + (int64_t)k * lda] : 0.0;
    }
    // B chunk: 32 k x 64 columns, coalesced along k within a column
#pragma unroll
    for (int q = 0; q < kT * kKC / 256; ++q) {
      const int idx = t + 256 * q, kk = idx % kKC, jj = idx / kKC;
      const int j = J0 + jj, k = k0 + kk;
      sB[kk][jj] = (j < n && k < m) ? B[k + (int64_t)j * ldb] : 0.0;
    }
    __syncthreads();
    mfma_chunk(sB, sA, wm, wn, lane, acc);
    __syncthreads();
  }
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int qm = 0; qm < 2; ++qm)
#pragma unroll
    for (int qn = 0; qn < 2; ++qn) {
      const int64_t r = I0 + wn * 32 + qn * 16 + li;
      if (r >= D) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = J0 + wm * 32 + qm * 16 + lk + 4 * e;
        if (j < n) {
          double* p = C + r + (int64_t)j * ldc;
          if (SUB)
            *p -= acc[qm][qn][e];
          else
            *p = acc[qm][qn][e];
        }
      }
    }
}

// Partial G tiles: part[z] (n1 x n2, col-major) = A^T B over the rows of
// split z.  MFMA M = columns of A (rows of G), N = columns of B, K = rows.
__global__ __launch_bounds__(256) void k_gemm_tn(int64_t D, int n1, int n2, const double* A,
                                                 int64_t lda, const double* B, int64_t ldb,
                                                 int64_t rows_per, double* part) {
  __shared__ double sA[kKC][kT + kPad];  // [row][col of A]
  __shared__ double sB[kKC][kT + kPad];  // [row][col of B]
  const int J1 = blockIdx.x * kT, J2 = blockIdx.y * kT;
  const int64_t r0 = (int64_t)blockIdx.z * rows_per;
  const int64_t r1 = std::min<int64_t>(D, r0 + rows_per);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wn = w & 1, wm = w >> 1;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
  for (int64_t k0 = r0; k0 < r1; k0 += kKC) {
#pragma unroll
    for (int q = 0; q < kT * kKC / 256; ++q) {
      const int idx = t + 256 * q, kk = idx % kKC, jj = idx / kKC;
      const int64_t r = k0 + kk;
      const int j1 = J1 + jj, j2 = J2 + jj;
      sA[kk][jj] = (r < r1 && j1 < n1) ? A[r + (int64_t)j1 * lda] : 0.0;
      sB[kk][jj] = (r < r1 && j2 < n2) ? B[r + (int64_t)j2 * ldb] : 0.0;
    }
    __syncthreads();
    mfma_chunk(sA, sB, wm, wn, lane, acc);
    __syncthreads();
  }
  const int li = lane & 15, lk = lane >> 4;
  double* P = part + (int64_t)blockIdx.z * n1 * n2;
#pragma unroll
  for (int qm = 0; qm < 2; ++qm)
#pragma unroll
    for (int qn = 0; qn < 2; ++qn) {
      const int j2 = J2 + wn * 32 + qn * 16 + li;
      if (j2 >= n2) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j1 = J1 + wm * 32 + qm * 16 + lk + 4 * e;
        if (j1 < n1) P[j1 + (int64_t)j2 * n1] = acc[qm][qn][e];
      }
    }
}

// G (ldg) = sum over the splits of part, in split order.
__global__ void k_sum_splits(int n1, int n2, int nsplit, const double* part, double* G,
                             int64_t ldg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ne = (int64_t)n1 * n2;
  if (e >= ne) return;
  double s = 0;
  for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * ne + e];
  G[(e % n1) + (e / n1) * ldg] = s;
}

}  // namespace

int gemm_tn_splits(int64_t D, int n1, int n2) {
  const int64_t tiles = (int64_t)((n1 + kT - 1) / kT) * ((n2 + kT - 1) / kT);
  int64_t z = (1024 + tiles - 1) / std::max<int64_t>(tiles, 1);
  z = std::min<int64_t>(z, std::max<int64_t>(1, D / kTnMinRows));
  return (int)std::max<int64_t>(1, std::min<int64_t>(z, 256));
}

size_t gemm_tn_workspace(int64_t D, int n1, int n2) {
  return (size_t)gemm_tn_splits(D, n1, n2) * (size_t)n1 * (size_t)n2 * sizeof(double);
}

void dev_gemm_nn(hipStream_t s, int64_t D, int m, int n, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc, bool sub) {
  if (D <= 0 || n <= 0) return;
  if (m <= 0) {
    REQUIRE(sub, "gemm: empty inner dimension");
    return;  // C -= 0
  }
  REQUIRE((D + kT - 1) / kT < (int64_t(1) << 31), "gemm: too many rows");
  const dim3 grid((unsigned)((D + kT - 1) / kT), (unsigned)((n + kT - 1) / kT));
  if (sub)
    hipLaunchKernelGGL(k_gemm_nn<true>, grid, dim3(256), 0, s, D, m, n, A, lda, B, ldb, C, ldc);
  else
    hipLaunchKernelGGL(k_gemm_nn<false>, grid, dim3(256), 0, s, D, m, n, A, lda, B, ldb, C, ldc);
  HIPC(hipGetLastError());
}

void dev_gemm_tn(hipStream_t s, int64_t D, int n1, int n2, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* G, int64_t ldg) {
  if (n1 <= 0 || n2 <= 0) return;
  const int z = gemm_tn_splits(D, n1, n2);
  const int64_t rows_per = std::max<int64_t>(1, (D + z - 1) / z);
  DevBuf part(gemm_tn_workspace(D, n1, n2));
  const dim3 grid((unsigned)((n1 + kT - 1) / kT), (unsigned)((n2 + kT - 1) / kT), (unsigned)z);
  hipLaunchKernelGGL(k_gemm_tn, grid, dim3(256), 0, s, D, n1, n2, A, lda, B, ldb, rows_per,
                     part.as<double>());
  const int64_t ne = (int64_t)n1 * n2;
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, n1, n2,
                     z, part.as<double>(), G, ldg);
  HIPC(hipGetLastError());
}

}  // namespace polfed

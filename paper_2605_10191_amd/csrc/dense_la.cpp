// Dense linear algebra of the Lanczos bookkeeping on the device, through
// rocBLAS and rocSOLVER: the products of the basis with small coefficient
// matrices (extraction u = V t, Rayleigh-Ritz), and the symmetric and
// tridiagonal eigenproblems once they are too large for the host solvers
// (their cost grows as n^3, and n reaches the thousands when thousands of
// pairs are wanted).  The filter and the Gram-Schmidt passes do not use
// these libraries.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <string>
#include <unordered_map>

#include "internal.hpp"

namespace polfed {

namespace {

void rbc(rocblas_status st, const char* what) {
  // the libraries report through their status; HIP's per-thread last-error
  // state they may leave behind is not an error of this library's launches
  (void)hipGetLastError();
  if (st != rocblas_status_success)
    fail(POLFED_ERR_HIP, std::string(what) + ": " + rocblas_status_to_string(st));
}

// One handle per thread and device, bound to the caller's stream.
rocblas_handle handle_for(hipStream_t s) {
  thread_local std::unordered_map<int, rocblas_handle> handles;
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  auto it = handles.find(dev);
  if (it == handles.end()) {
    rocblas_handle h = nullptr;
    rbc(rocblas_create_handle(&h), "rocblas_create_handle");
    it = handles.emplace(dev, h).first;
  }
  rbc(rocblas_set_stream(it->second, s), "rocblas_set_stream");
  return it->second;
}

void check_info(hipStream_t s, const rocblas_int* d_info, const char* what) {
  rocblas_int info = 0;
  HIPC(hipMemcpyAsync(&info, d_info, sizeof info, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  if (info != 0) fail(POLFED_ERR_INVALID, std::string(what) + " did not converge");
}

}  // namespace

void dev_gemm_nn(hipStream_t s, int64_t D, int m, int n, const double* A, int64_t lda,
                 const double* B, double* C, int64_t ldc) {
  if (!D || !n) return;
  REQUIRE(D < (int64_t(1) << 31) && lda < (int64_t(1) << 31), "gemm: dimension too large");
  const double one = 1.0, zero = 0.0;
  rbc(rocblas_dgemm(handle_for(s), rocblas_operation_none, rocblas_operation_none, (rocblas_int)D,
                    n, m, &one, A, (rocblas_int)lda, B, m, &zero, C, (rocblas_int)ldc),
      "rocblas_dgemm");
}

void dev_gemm_tn(hipStream_t s, int64_t D, int n, const double* A, const double* B,
                 double* /*partial*/, int64_t /*nseg*/, double* G) {
  if (!n) return;
  REQUIRE(D < (int64_t(1) << 31), "gemm: dimension too large");
  const double one = 1.0, zero = 0.0;
  rbc(rocblas_dgemm(handle_for(s), rocblas_operation_transpose, rocblas_operation_none, n, n,
                    (rocblas_int)D, &one, A, (rocblas_int)D, B, (rocblas_int)D, &zero, G, n),
      "rocblas_dgemm");
}

void dev_dgemm(hipStream_t s, bool ta, bool tb, int m, int n, int64_t k, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
               double* C, int64_t ldc) {
  if (m <= 0 || n <= 0) return;
  REQUIRE(k < (int64_t(1) << 31) && lda < (int64_t(1) << 31) && ldb < (int64_t(1) << 31) &&
              ldc < (int64_t(1) << 31),
          "gemm: dimension too large");
  rbc(rocblas_dgemm(handle_for(s), ta ? rocblas_operation_transpose : rocblas_operation_none,
                    tb ? rocblas_operation_transpose : rocblas_operation_none, m, n,
                    (rocblas_int)k, &alpha, A, (rocblas_int)lda, B, (rocblas_int)ldb, &beta, C,
                    (rocblas_int)ldc),
      "rocblas_dgemm");
}

void dev_syevd(hipStream_t s, int n, double* A, double* w) {
  if (n <= 0) return;
  DevBuf e((size_t)n * sizeof(double)), info(sizeof(rocblas_int));
  rbc(rocsolver_dsyevd(handle_for(s), rocblas_evect_original, rocblas_fill_lower, n, A, n, w,
                       e.as<double>(), info.as<rocblas_int>()),
      "rocsolver_dsyevd");
  check_info(s, info.as<rocblas_int>(), "rocsolver_dsyevd");
}

void dev_stedc(hipStream_t s, int n, double* d, double* e, double* C) {
  if (n <= 0) return;
  DevBuf info(sizeof(rocblas_int));
  rbc(rocsolver_dstedc(handle_for(s), rocblas_evect_tridiagonal, n, d, e, C, n,
                       info.as<rocblas_int>()),
      "rocsolver_dstedc");
  check_info(s, info.as<rocblas_int>(), "rocsolver_dstedc");
}

}  // namespace polfed

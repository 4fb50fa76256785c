/*
 * polfed.h -- C ABI of the MI355X POLFED library (polynomially filtered exact
 * diagonalization of sparse many-body Hamiltonians).
 *
 * Problem statement (paper, Sec. 4.6): given a sparse Hamiltonian H, a target
 * energy lambda and a number of eigenpairs N_ev, return the N_ev eigenpairs
 * of H nearest lambda.  The method (Secs. 3.2, 4.1-4.4) rescales H to
 * H~ = (H - E_c)/dE (eq. rescaledMatrix), builds the Chebyshev delta filter
 * P(H~) = (1/chi) sum_{n=0}^{K} c_n T_n(H~) (eqs. transformation and
 * transformationCoefficients), and runs Lanczos on P(H~) with full
 * reorthogonalization, applying P(H~) by the Clenshaw recurrence
 * (eq. clenshaw_chebyshev_prod): K sparse mat-vecs per Lanczos step.
 *
 * Conventions shared by every call
 *  - Every function returns a polfed_status: 0 = OK, > 0 warning, < 0 error.
 *    No function throws or aborts.  After an error, polfed_last_error()
 *    returns a message for the calling thread (owned by the library, valid
 *    until the next call on that thread).
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory on the context's device (e.g. torch tensor data_ptr()).
 *  - Vectors are contiguous; blocks of vectors are column-major with leading
 *    dimension D (column j starts at j*D).
 *  - Work is ordered on the context's HIP stream.  Calls that return results
 *    in host memory synchronize that stream; calls that only write device
 *    buffers are asynchronous unless stated otherwise.
 *  - Ownership: the library owns contexts, operators and requests and frees
 *    them in the matching destroy call.  Arrays passed in are borrowed: input
 *    arrays are copied before the call returns, caller-owned output buffers
 *    must stay alive until the call (or, for serving, the request) finishes.
 *  - Many-body bit convention: site j = 1..L is bit j-1 of a state integer;
 *    an up spin / occupied site is a set bit.
 */
#ifndef POLFED_H
#define POLFED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  POLFED_OK = 0,
  POLFED_NOT_CONVERGED = 1,  /* partial result: *n_found pairs are valid */
  POLFED_ERR_INVALID = -1,   /* bad argument (message says which) */
  POLFED_ERR_OOM = -2,       /* device allocation failed */
  POLFED_ERR_HIP = -3,       /* HIP runtime error (message has the code) */
  POLFED_ERR_BOUNDS = -4,    /* filter blow-up: spectral bounds too tight */
  POLFED_ERR_BREAKDOWN = -5, /* Lanczos breakdown that could not be resumed */
  POLFED_ERR_BUSY = -6,      /* serving not started / already running */
  POLFED_ERR_NODEVICE = -7,  /* no HIP device visible */
  POLFED_ERR_REJECTED = -8   /* serving: request larger than the HBM budget */
} polfed_status;

enum { POLFED_FP64 = 0, POLFED_FP32 = 1 };        /* Clenshaw precision */
/* polfed_params.precision only (solves, batches, served requests): FP32 bulk
 * filtering with FP64 refinement when the operator's FP32 Clenshaw step runs
 * in less than 0.7 of the FP64 step's time, else FP64.  The two steps are
 * timed (graph replays of 20 launches on scratch vectors, eager launches on
 * the server's threads; about 3 D-vectors of device memory for the
 * duration) at the first such solve of an operator,
 * or of any chain operator with the same off-diagonal pattern and storage on
 * the device, and the choice is kept; polfed_report.precision says which
 * ran.  The refinement costs about 40% of the FP32 filter time, so FP32 bulk
 * only pays where the step is bound by bytes rather than by latency. */
enum { POLFED_PRECISION_AUTO = 2 };
enum { POLFED_MATRIX_FREE = 0, POLFED_CSR = 1 };  /* operator storage */
enum {
  POLFED_TARGET_ABSOLUTE = 0,   /* target is lambda itself */
  POLFED_TARGET_RESCALED = 1,   /* target is lambda~ in [-1, 1] of [E_min, E_max] */
  POLFED_TARGET_NORMALIZED = 2, /* target is (lambda - E_min)/(E_max - E_min) */
  POLFED_TARGET_MAXDOS = 3,     /* the maximum of the density-of-states estimate
                                   (Sec. 5.4): the mean Tr H / D for the
                                   Gaussian estimate; target is ignored */
  POLFED_TARGET_OFFSET = 4      /* target = eta in [-1, 1]: from the maxdos point
                                   toward the upper (eta > 0) or lower edge,
                                   linearly in rescaled coordinates (Sec. 5.4) */
};

typedef struct polfed_ctx polfed_ctx;
typedef struct polfed_op polfed_op;
typedef struct polfed_req polfed_req;

/* ---------------------------------------------------------------- context */

/* Library version (major * 10000 + minor * 100 + patch).  10100 added
 * POLFED_PRECISION_AUTO and polfed_report.precision (the report grew by one
 * int: callers built against an older header pass a smaller struct). */
int polfed_version(void);
/* Text of the last error on the calling thread ("" after a success); owned
 * by the library, valid until the thread's next call. */
const char* polfed_last_error(void);

/* Creates a context on HIP device `device`.  `hip_stream` is the hipStream_t
 * the context borrows for all its work.  NULL asks for ordering with the
 * device's null stream (e.g. torch's default stream): the context then
 * creates a blocking stream of its own, which the null stream and it wait on
 * each other through (the library queues nothing on the null stream itself,
 * which would break the graph captures its server runs beside it).  Fails
 * with POLFED_ERR_NODEVICE when no GPU is visible. */
polfed_status polfed_create(int device, void* hip_stream, polfed_ctx** out);
/* Stops a running server, waits for the context's work and frees the
 * context; its operators must not be used afterwards (NULL is a no-op). */
polfed_status polfed_destroy(polfed_ctx* ctx);
/* Waits for all work queued on the context's stream. */
polfed_status polfed_sync(polfed_ctx* ctx);

/* ------------------------------------------------------------------ basis
 * Sector of L-bit strings with N set bits (the U(1) sector of App. A), in
 * ascending integer order; the rank of a state is its position.  The library
 * computes ranks with the combinadic rank(s) = sum_k binom(p_k, k) over the
 * set-bit positions p_1 < ... < p_N, which equals that position.
 * 1 <= L <= 32, 0 <= N <= L. */

/* Host only: D = binom(L, N). */
polfed_status polfed_basis_dim(int L, int N, int64_t* D);
/* Writes all D states, ascending, to device array states[D]. */
polfed_status polfed_basis_enumerate(polfed_ctx* ctx, int L, int N,
                                     uint32_t* states);
/* ranks[i] = rank of states[i] (device arrays, n entries); a state that is
 * not in the sector (wrong popcount or bits >= L) gets rank -1. */
polfed_status polfed_basis_rank(polfed_ctx* ctx, int L, int N,
                                const uint32_t* states, int64_t n,
                                int64_t* ranks);
/* states[i] = state of rank ranks[i] (device arrays); ranks outside [0, D)
 * give 0xFFFFFFFF. */
polfed_status polfed_basis_unrank(polfed_ctx* ctx, int L, int N,
                                  const int64_t* ranks, int64_t n,
                                  uint32_t* states);

/* -------------------------------------------------------------- operators
 * All parameter arrays are host arrays, copied at creation.  Matrix-free
 * operators generate matrix elements from the state bits on the fly; a CSR
 * copy can be built on the device with polfed_op_materialize_csr. */

/* Random-field XXZ chain, App. A eq. (xxz):
 *   H = J sum_i (S^x_i S^x_{i+1} + S^y_i S^y_{i+1} + Delta S^z_i S^z_{i+1})
 *       + sum_i h_i S^z_i,   S = sigma/2,
 * in the sector with n_up up spins; h[L]; periodic != 0 adds bond (L, 1).
 * 3 <= L <= 32 for periodic chains, 2 <= L <= 32 otherwise. */
polfed_status polfed_op_xxz(polfed_ctx* ctx, int L, int n_up, double J,
                            double Delta, const double* h, int periodic,
                            polfed_op** out);
/* Spinless fermions (not a model of the paper):
 *   H = -t sum_i (c^dag_i c_{i+1} + h.c.) + V sum_i n_i n_{i+1}
 *       + sum_i eps_i n_i
 * with Jordan-Wigner ordering by site; the periodic bond carries the string
 * sign (-1)^(n_part - 1).  eps[L]. */
polfed_status polfed_op_tv(polfed_ctx* ctx, int L, int n_part, double t,
                           double V, const double* eps, int periodic,
                           polfed_op** out);
/* Quantum sun, App. A eq. (qsun), full 2^(N_dot+L) space:
 *   H = H_dot (x) I + g0 sum_j alpha^{u_j} S^x_{n(j)} S^x_j + sum_j h_j S^z_j,
 *   H_dot = gamma (A + A^T) / sqrt(2 (2^N_dot + 1))   (App. A normalization).
 * A: 2^N_dot x 2^N_dot row-major host matrix of the raw normal draws;
 * u[L], n_of_j[L] (dot spin 0..N_dot-1 coupled to outer spin j), h[L].
 * Dot spin k is bit L+k of the state index, outer spin j is bit j-1.
 * 1 <= N_dot <= 6, 1 <= L, N_dot + L <= 31. */
polfed_status polfed_op_qsun(polfed_ctx* ctx, int N_dot, int L,
                             const double* A, double gamma, double g0,
                             double alpha, const double* u,
                             const int32_t* n_of_j, const double* h,
                             polfed_op** out);
/* Quantum random energy model, eq. (qrem) of App. A, on the full 2^L space:
 * H = sum_a E[a] |a><a| - Gamma sum_i sigma^x_i, sigma^x_i flipping bit i
 * of the state index a.  E: host array [2^L], copied.  2 <= L <= 28.
 * Matrix-free only (no CSR copy). */
polfed_status polfed_op_qrem(polfed_ctx* ctx, int L, const double* E, double Gamma,
                             polfed_op** out);
/* Spin-1/2 chain with couplings of range r = 1..R (App. A: eq. xxz for
 * R = 1, eq. j1j2 for R = 2, eq. j1j2j3 for R = 3):
 * H = sum_r J[r-1] sum_i (S^x_i S^x_{i+r} + S^y_i S^y_{i+r}
 *     + Delta[r-1] S^z_i S^z_{i+r}) + sum_i h[i] S^z_i,
 * in the sector of N up spins (site i is bit i, ascending order), built as
 * a CSR operator (host arrays J[R], Delta[R], h[L] copied).  Periodic bonds
 * wrap around and need L > 2R.  2 <= L <= 24, 1 <= R <= 8. */
polfed_status polfed_op_spin_chain(polfed_ctx* ctx, int L, int N, int R, const double* J,
                                   const double* Delta, const double* h, int periodic,
                                   polfed_op** out);
/* Optimized mapping (Sec. 5.6): replaces the off-diagonal values of the
 * operator's CSR copy by a table of the distinct values and a one-byte code
 * per entry (no code at all when every value is the same), so the filter
 * reads 5 (or 4) instead of 12 bytes per entry.  With more than 256 distinct
 * values the operator is left as it is.  *n_values (may be NULL) gets the
 * number of distinct values found (257 meaning "more than 256"). */
polfed_status polfed_op_optimize_mapping(polfed_ctx* ctx, polfed_op* op, int* n_values);
/* Generic symmetric sparse matrix in CSR (host arrays, copied): rowptr[D+1]
 * (int64), col[nnz] (int32, any order within a row), val[nnz].  Diagonal
 * entries may appear; they are split off internally.  Symmetry is the
 * caller's promise (not checked).  D < 2^31. */
polfed_status polfed_op_csr(polfed_ctx* ctx, int64_t D, const int64_t* rowptr,
                            const int32_t* col, const double* val,
                            polfed_op** out);
/* Builds the device CSR copy of a matrix-free operator (off-diagonal part in
 * CSR, diagonal separate).  No-op for CSR operators. */
polfed_status polfed_op_materialize_csr(polfed_ctx* ctx, polfed_op* op);
/* Chooses which representation the filter uses (POLFED_MATRIX_FREE needs a
 * model operator; POLFED_CSR needs a CSR copy). */
polfed_status polfed_op_set_storage(polfed_op* op, int storage);
/* Step-kernel variant of a matrix-free chain (XXZ, t-V) in one precision:
 * -1 = pick by timing on the next step (the default), 0 = segment kernel,
 * 1 = tile kernel with the largest tile, 2 = tile kernel with half that tile,
 * 3 = segment kernel with two adjacent rows per lane (16-byte accesses),
 * 4 = segment kernel with each segment split between two wavefronts,
 * 5 = tile kernel with a quarter of the largest tile;
 * 6 .. 9 = staged-tile kernel (the tile's rows and segment records copied
 * to LDS by direct-to-LDS loads; the tile also spans the top state bit, so
 * the periodic bond is an LDS read): 6 the largest tile with one buffer and
 * 1024 threads, 7 half that tile with two buffers (the next tile is staged
 * while the current one is processed) and 512 threads, 8 half that tile
 * with one buffer, 9 the largest tile with two buffers (where the LDS holds
 * them, FP32);
 * -2 only reports the variant in use.
 * A variant that does not exist for the chain length and precision (tiles
 * need L >= 22) gives POLFED_ERR_INVALID.  For a quantum random energy model the variant is
 * the tile size in bits (rows per LDS tile = 2^variant), 1 .. min(L, 12), or
 * -1 to pick among the default and its neighbours by timing.  *chosen (may
 * be NULL) receives the variant in use after the call (-1 while not tuned
 * yet). */
polfed_status polfed_op_set_kernel(polfed_op* op, int precision, int variant, int* chosen);
/* Multi-column step kernel of batches of B chain realizations that share the
 * pattern of op (the batch's first operator), in one precision: -1 = pick by
 * timing at the next batched filter (the default), 0 / 1 = column-major
 * blocks with 16 / 8 columns per launch, 2 / 3 = interleaved blocks (the B
 * columns of a row side by side, one 16-byte access per row and 2 FP64 or 4
 * FP32 columns; 2 / 4 workgroups per compute unit), 4 = every column
 * stepped by its own operator's tuned single-column kernel (the staged-tile
 * kernels, L >= 22), 5 = the LDS-resident filter (one workgroup per column
 * runs the column's whole recurrence with both Clenshaw vectors in LDS and
 * a barrier between steps; where two vectors fit: FP64 to L = 14, FP32 to
 * L = 16 at half filling), 6 / 7 = row-group kernel on the interleaved
 * blocks (the 16-byte column groups of a row on neighbouring lanes, so a
 * wavefront reads whole rows; up to 32 FP64 or 64 FP32 columns; 4 / 8
 * workgroups per compute unit); -2 only reports.  A batch whose pattern was
 * timed before (any operator of it, same width and precision) takes that
 * pick without timing again.
 * *chosen (may be NULL) receives the variant in use (-1 while not tuned). */
polfed_status polfed_op_set_batch_kernel(polfed_op* op, int B, int precision, int variant,
                                         int* chosen);
/* Dimension D of the operator's space (sector or full space). */
polfed_status polfed_op_dim(const polfed_op* op, int64_t* D);
/* Off-diagonal nnz of the CSR copy (-1 if there is none). */
polfed_status polfed_op_nnz(const polfed_op* op, int64_t* nnz_offdiag);
/* Copies the CSR copy to caller device buffers: rowptr[D+1], col[nnz],
 * val[nnz] (off-diagonal part, rows sorted by column) and diag[D]. */
polfed_status polfed_op_export_csr(polfed_ctx* ctx, const polfed_op* op,
                                   int64_t* rowptr, int32_t* col, double* val,
                                   double* diag);
/* Frees the operator and its device tables (NULL is a no-op). */
polfed_status polfed_op_destroy(polfed_op* op);
/* y = H x (device vectors of length D, FP64). */
polfed_status polfed_op_apply(polfed_ctx* ctx, const polfed_op* op,
                              const double* x, double* y);
/* Exact trace moments Tr H / D and Tr H^2 / D (host results; synchronizes).
 * They fix the mean and width of the Gaussian DOS, eq. (dos_gaussian). */
polfed_status polfed_op_moments(polfed_ctx* ctx, const polfed_op* op,
                                double* tr1, double* tr2);

/* ------------------------------------------------------ filter (host side) */

/* Plan of the filter (Secs. 4.1-4.2), computed on the host from the bounds,
 * the trace moments and the target. */
typedef struct {
  double E_c, dE;      /* eq. rescaledMatrix, from the padded bounds */
  double lambda_t;     /* rescaled target */
  double mu_t, Gamma_t;/* Gaussian DOS mean and width, rescaled */
  double rho;          /* DOS at the target, eq. dos_gaussian */
  double delta;        /* window half-width, eq. Nev */
  double K_approx;     /* eq. K_approx */
  int K;               /* order from eq. condition_for_K */
} polfed_plan;

/* n_window eigenvalues in the window; omega <= 0 selects the default cutoff
 * sin(2.655)/2.655; K_override > 0 skips the bisection.  D is the matrix
 * dimension; pad widens [E_min, E_max] by pad*(E_max-E_min) on each side. */
polfed_status polfed_make_plan(int64_t D, double E_min, double E_max,
                               double pad, double lambda, double tr1,
                               double tr2, int n_window, double omega,
                               int K_override, polfed_plan* out);
/* a[0..K] = c_n / chi (eqs. transformation, transformationCoefficients). */
polfed_status polfed_filter_coefficients(double lambda_t, int K, double* a);
/* out[i] = P^K_{lambda~}(x[i]) by its closed form (host arrays). */
polfed_status polfed_filter_value(double lambda_t, int K, const double* x,
                                  int64_t n, double* out);

/* Divided difference of the Chebyshev series p = sum_{n<=K} a_n T_n at theta:
 * q[0..K-1] are the Chebyshev coefficients of (p(x) - p(theta)) / (x - theta)
 * and *p_theta = p(theta) (may be NULL).  Used by the FP32 refinement, where
 * P(H~) u = P(theta) u + Q(H~) (H~ - theta) u moves only the small residual
 * through the low-precision recurrence.  Host arrays; K >= 0 (q unused for
 * K = 0). */
polfed_status polfed_filter_quotient(const double* a, int K, double theta,
                                     double* q, double* p_theta);

/* ------------------------------------------------------- filter (device) */

/* w = P(H~) v by the Clenshaw recurrence, eq. clenshaw_chebyshev_prod, with
 * H~ = (H - E_c)/dE; a[0..K] host coefficients.  v, w: device vectors of
 * length D in the chosen precision (double for POLFED_FP64, float for
 * POLFED_FP32); v and w must not overlap.  K >= 0. */
polfed_status polfed_filter_apply(polfed_ctx* ctx, const polfed_op* op,
                                  double E_c, double dE, const double* a,
                                  int K, const void* v, void* w,
                                  int precision);
/* The same filter application for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the two recurrence buffers come from a static device
 * scratch array of 48 MiB that each GPU the library runs on holds until the
 * process ends, so D is limited to 3,145,728 rows in FP64 and 6,291,456 in
 * FP32 (larger D gives POLFED_ERR_INVALID).  The operator's step kernel must
 * already be chosen in this precision (by an earlier step, filter or solve,
 * or polfed_op_set_kernel), since choosing it times launches on scratch
 * vectors; otherwise POLFED_ERR_INVALID.  Asynchronous on the context's
 * stream, no allocation and no synchronization.  Every call on a GPU uses
 * that GPU's one scratch array: calls that overlap on one GPU (two contexts
 * or streams, or threads) race and give wrong results. */
polfed_status polfed_filter_apply_noalloc(polfed_ctx* ctx, const polfed_op* op,
                                          double E_c, double dE, const double* a,
                                          int K, const void* v, void* w,
                                          int precision);
/* One fused Clenshaw step (the hot kernel), in place on b2:
 *   b2 <- a_i v + 2 H~ b1 - b2            (final == 0)
 *   b2 <- a_i v +   H~ b1 - b2            (final != 0, the closing step)
 * Device vectors of length D in the chosen precision; b1 must not overlap
 * v or b2. */
polfed_status polfed_clenshaw_step(polfed_ctx* ctx, const polfed_op* op,
                                   double E_c, double dE, double a_i,
                                   const void* v, const void* b1, void* b2,
                                   int precision, int final);

/* Multi-column filter for B chain operators that share the off-diagonal
 * pattern (same model, L, N, boundary and couplings; on-site fields may
 * differ): column c of the device blocks v and w (D x B, column-major,
 * column stride D, in the chosen precision) gets
 *     w_c = P_c(H~_c) v_c,   H~_c = (H_c - E_c[c]) / dE[c],
 * with the Chebyshev coefficients a[c][0..K[c]] (host arrays) evaluated by
 * the Clenshaw recurrence of eq. clenshaw_chebyshev_prod as one recurrence
 * of max K[c] steps over all columns.  Synchronizes.  Operators of another
 * pattern or outside L = 4..28 give POLFED_ERR_INVALID. */
polfed_status polfed_filter_apply_batch(polfed_ctx* ctx, int B,
                                        const polfed_op* const* ops,
                                        const double* E_c, const double* dE,
                                        const double* const* a, const int* K,
                                        const void* v, void* w, int precision);
/* One multi-column Clenshaw step, in place on the block b2 (D x B):
 *   b2_c <- a_i[c] v_c + 2 H~_c b1_c - b2_c   (final == 0)
 *   b2_c <- a_i[c] v_c +   H~_c b1_c - b2_c   (final != 0)
 * a_i: host [B].  Synchronizes. */
polfed_status polfed_clenshaw_step_batch(polfed_ctx* ctx, int B,
                                         const polfed_op* const* ops,
                                         const double* E_c, const double* dE,
                                         const double* a_i, const void* v,
                                         const void* b1, void* b2, int precision,
                                         int final);

/* --------------------------------------------------------------- Lanczos */

/* Spectral extremes by plain Lanczos on H with full reorthogonalization
 * (Sec. 3.2), started from device vector x0[D] (need not be normalized).
 * Stops when both extreme Ritz residuals are below tol*(E_max-E_min) or
 * after max_iter steps.  Host results; synchronizes. */
polfed_status polfed_bounds(polfed_ctx* ctx, const polfed_op* op,
                            const double* x0, double tol, int max_iter,
                            double* E_min, double* E_max);

/* One Lanczos step on the filtered operator (Sec. 4.3 with block size 1):
 * w = P(H~) v_k by the Clenshaw filter (a[0..K], host), full
 * reorthogonalization of w against v_0..v_k by classical Gram-Schmidt
 * applied twice, *alpha = v_k^T P(H~) v_k, *beta = ||w||, v_{k+1} = w / beta.
 * V: device basis, column-major D x (k+2), columns 0..k orthonormal; column
 * k+1 is written.  alpha, beta: device scalars.  precision selects the
 * Clenshaw arithmetic (the basis is FP64 either way).  Asynchronous. */
polfed_status polfed_lanczos_step(polfed_ctx* ctx, const polfed_op* op,
                                  double E_c, double dE, const double* a,
                                  int K, double* V, int k, double* alpha,
                                  double* beta, int precision);
/* Extraction (Sec. 4.3): the Ritz vectors u_j = V t_j of the selected
 * eigenvectors t_j of the Lanczos matrix, then Rayleigh-Ritz with H on their
 * span (the reading of Sec. 4.3's per-vector energies for a subspace):
 * G = U^T H U (symmetrized), G = Z diag(E) Z^T, U2 = U Z, and the residuals
 * ||H u2_j - E_j u2_j||.  V: device D x m column-major (ld D), orthonormal
 * columns; T: device m x n column-major (ld m), orthonormal columns.  E[n]
 * ascending, U2 (D x n, ld D), resid[n]: device outputs, caller-owned.  The
 * products run on the matrix cores (MFMA), the n x n eigenproblem on the
 * host.  Synchronizes. */
polfed_status polfed_extract(polfed_ctx* ctx, const polfed_op* op, const double* V, int m,
                             const double* T, int n, double* E, double* U2, double* resid);
/* The products of the extraction and of block Gram-Schmidt, exposed for
 * parity tests and profiling (device column-major FP64 arrays with leading
 * dimensions; D >= 0, sizes >= 0):
 *   polfed_gemm_nn:  C (D x n) = A (D x m) B (m x n), or C -= A B when
 *                    subtract is nonzero;
 *   polfed_gemm_tn:  G (n1 x n2) = A^T B with A (D x n1), B (D x n2); the
 *                    sum over D is split over workgroups and the partial
 *                    results are added in a fixed order (deterministic).
 * Asynchronous on the context's stream. */
polfed_status polfed_gemm_nn(polfed_ctx* ctx, int64_t D, int m, int n, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                             int subtract);
polfed_status polfed_gemm_tn(polfed_ctx* ctx, int64_t D, int n1, int n2, const double* A,
                             int64_t lda, const double* B, int64_t ldb, double* G, int64_t ldg);

/* One block Lanczos step on the filtered operator (Sec. 2.2, eq.
 * block_lanczos_reocurrence, with the filter of Sec. 4.3): W = P(H~) V_j
 * for the current block V_j = columns k..k+s-1 of V (one multi-column
 * Clenshaw recurrence for chain operators, s single ones otherwise), full
 * reorthogonalization of W against columns 0..k+s-1 and its QR, which gives
 * the next block (columns k+s..k+2s-1, written) and B_{j+1}.  W gets two
 * passes of block Gram-Schmidt against columns 0..k+s-1 (tall-skinny
 * products); then column c gets two passes against the new block's columns
 * 0..c-1 and is normalized (a Gram-Schmidt QR, positive diagonal).
 * V: device basis, column-major D x (k+2s), columns 0..k+s-1 orthonormal,
 * k a multiple of s, 1 <= s <= 64 and k + 2s <= D.
 * A: device s x s column-major, A_j = V_j^T P(H~) V_j (as computed; not
 * symmetrized).  Bn: device s x s column-major, upper triangular B_{j+1}.
 * A column of W that has lost rank (norm <= 1e-13) is replaced by a random
 * unit vector orthogonal to the basis, with a zero diagonal entry in Bn.
 * precision selects the Clenshaw arithmetic.  Synchronizes (the diagonal of
 * Bn is inspected on the host). */
polfed_status polfed_block_lanczos_step(polfed_ctx* ctx, const polfed_op* op,
                                        double E_c, double dE, const double* a,
                                        int K, double* V, int k, int s, double* A,
                                        double* Bn, int precision);
/* Kernel polynomial method (Sec. 4.1 eq. dos_kpm, App. B): mu[n] for
 * n < N, the mean over R vectors r of <r| T_n(H~) |r> with H~ = (H - E_c)/dE,
 * by the three-term Chebyshev recurrence on the fused step kernel (FP64).
 * r: device D x R column-major, or NULL: then vector c (0 <= c < R) has
 * entries sqrt(3) (2 u - 1), u = (z >> 11) / 2^53 for the splitmix64 output
 * z of seed + c at counter i + 1 (zero mean, unit variance).  mu: host [N].
 * Synchronizes. */
polfed_status polfed_kpm_moments(polfed_ctx* ctx, const polfed_op* op, double E_c,
                                 double dE, int N, int R, const double* r, uint64_t seed,
                                 double* mu);
/* The Jackson-damped KPM density rho(x) = [mu_0 g_0 + 2 sum_{n=1}^{N-1}
 * mu_n g_n T_n(x)] / (pi sqrt(1 - x^2)) at nx host points x in (-1, 1).
 * Host only. */
polfed_status polfed_kpm_density(const double* mu, int N, const double* x, int nx,
                                 double* rho);
/* Measurement helper: times `iters` back-to-back launches of the fused
 * Clenshaw step kernel on scratch vectors with one pair of HIP events on the
 * context stream (mean = elapsed / iters, the rate of a running recurrence)
 * and up to 20 single launches each between its own event pair (minimum).
 * Milliseconds, host results; synchronizes. */
polfed_status polfed_profile_step(polfed_ctx* ctx, const polfed_op* op,
                                  int precision, int iters, double* avg_ms,
                                  double* min_ms);

typedef struct {
  int target_kind;     /* POLFED_TARGET_* */
  double target;
  int n_ev;            /* N_ev >= 1 */
  int precision;       /* POLFED_FP64, POLFED_FP32 for the bulk filter, or
                          POLFED_PRECISION_AUTO */
  int K_override;      /* 0: plan K */
  double omega;        /* 0: default cutoff */
  double eta;          /* 0: 1.5, over-allocation of the Krylov basis */
  double tol_resid;    /* 0: 1e-8, accepted ||H u - E u|| */
  double bound_pad;    /* 0: 1e-3 */
  int max_iter;        /* 0: 4 * expectedkrylovdim */
  double E_min, E_max; /* both 0: compute the bounds */
  int graph;           /* filter recurrence as one HIP graph: 0 = pick the
                          faster of direct launches and graph replay on the
                          first two filter applications (a multi-column
                          filter reuses the pick of an earlier batch of the
                          same chain pattern, width, precision and order to a
                          factor of two), 1 = always graph, 2 = never.
                          Served requests always launch directly (the
                          server's threads capture no graphs: a device
                          synchronization or synchronous copy on another
                          thread would invalidate the capture). */
  int refine_max;      /* FP32 bulk: at most this many refinement sweeps
                          (0: 16; -1: none); a refinement that stalls or
                          runs out hands the solve to the FP64 filter */
  int block_size;      /* 0 or 1: Lanczos; s in 2..64: block Lanczos with
                          blocks of s vectors (Sec. 2.2), polfed_solve only */
  int kpm_moments;     /* 0: Gaussian DOS from the traces; N > 0: KPM DOS
                          (Sec. 4.1 eq. dos_kpm, Jackson kernel) with N
                          moments, for the window and the maxdos point */
  int kpm_vectors;     /* KPM: random vectors (0: 100); drawn as in
                          polfed_kpm_moments with r = NULL and seed 0x4B504D */
} polfed_params;

typedef struct {
  double E_min, E_max, lambda, lambda_t, E_c, dE, delta, rho;
  int K, M_alloc, iters, n_want, n_converged, checks, restarts, refine_sweeps;
  double t_bounds, t_plan, t_filter, t_reorth, t_check, t_extract, t_refine,
      t_total;           /* seconds */
  double filter_steps;   /* Clenshaw steps executed */
  double filter_bytes;   /* algorithmic HBM bytes of those steps */
  double filter_GBps;    /* filter_bytes / t_filter / 1e9 */
  double t_queue;        /* served requests: submission to admission (s) */
  double t_latency;      /* served requests: submission to result (s) */
  int fp32_fallback;     /* 1: the FP32-bulk refinement stalled and the solve
                            was completed by the FP64 filter */
  int precision;         /* POLFED_FP64 or POLFED_FP32: the filter precision
                            the solve started in (the resolved choice for
                            POLFED_PRECISION_AUTO) */
  double mem_peak;       /* largest device bytes the solve's own buffers held
                            at once (operator tables and the server's shared
                            batch buffers not included) */
  double mem_reserved;   /* served requests: the most device bytes reserved
                            for the request against the server's budget
                            (admission estimate plus later grants); 0 for
                            polfed_solve */
} polfed_report;

/* Defaults: normalized target 0.5, 20 pairs, FP64, eta 1.5, residual
 * tolerance 1e-8, bound pad 1e-3; every other field 0 (automatic). */
polfed_status polfed_params_default(polfed_params* p);

/* Synchronous solve.  x0: device start vector [D], or with block_size s > 1
 * the start block, column-major D x s of full rank (orthonormalized by a
 * Gram-Schmidt QR, Sec. 2.2).  Outputs are caller
 * device buffers: evals[n_ev], evecs[D * n_ev] (column-major, unit norm),
 * resid[n_ev] = ||H u - E u||, ordered by (|E - lambda|, E).  *n_found gets
 * the number of valid pairs (n_ev on POLFED_OK, fewer with
 * POLFED_NOT_CONVERGED).  rep may be NULL. */
polfed_status polfed_solve(polfed_ctx* ctx, const polfed_op* op,
                           const polfed_params* params, const double* x0,
                           double* evals, double* evecs, double* resid,
                           int* n_found, polfed_report* rep);

/* Batched solve of B realizations that share the off-diagonal pattern (same
 * model, L, N and couplings, different diagonal fields): the filter runs as
 * one multi-column recurrence.  Arrays of B pointers; each entry as in
 * polfed_solve.  n_found[B], rep[B] (rep may be NULL).  block_size must be
 * 0 or 1. */
polfed_status polfed_solve_batch(polfed_ctx* ctx, int B,
                                 const polfed_op* const* ops,
                                 const polfed_params* params,
                                 const double* const* x0,
                                 double* const* evals, double* const* evecs,
                                 double* const* resid, int* n_found,
                                 polfed_report* rep);

/* --------------------------------------------------------------- serving
 * Continuous batching: requests are admitted while the HBM their Krylov
 * bases need fits the budget and a column slot is free; admitted requests of
 * the same operator class (same chain pattern and precision) share one
 * multi-column filter recurrence, and each leaves the batch as soon as it
 * converges.  Each class runs its rounds (recurrence, then every member's
 * Lanczos step) on its own stream at its own pace. */
polfed_status polfed_serve_start(polfed_ctx* ctx, size_t hbm_budget_bytes,
                                 int max_cols);
/* Queues a solve; op, x0 and the output buffers must stay alive until
 * polfed_wait returns.  Requests whose footprint exceeds the budget are
 * rejected (POLFED_ERR_REJECTED); block_size must be 0 or 1.  With
 * POLFED_PRECISION_AUTO the precision is chosen at admission and the request
 * reserves the larger of the two footprints.  Calls on ctx from other
 * threads while the server runs: those that only build new objects (basis
 * calls, operator constructors, polfed_gemm_nn/tn) run beside the server's
 * rounds; the others wait until the rounds in flight have ended (at most one
 * round of each group) and run before the next ones start. */
polfed_status polfed_submit(polfed_ctx* ctx, const polfed_op* op,
                            const polfed_params* params, const double* x0,
                            double* evals, double* evecs, double* resid,
                            polfed_req** out);
/* *done = 1 once the request has finished (does not block). */
polfed_status polfed_poll(polfed_req* req, int* done);
/* Blocks until the request finished; returns its solve status. */
polfed_status polfed_wait(polfed_req* req, int* n_found, polfed_report* rep);
/* Frees a finished request (POLFED_ERR_BUSY while it still runs; NULL is a
 * no-op). */
polfed_status polfed_req_destroy(polfed_req* req);
/* Finishes every submitted request, then stops the scheduler. */
polfed_status polfed_serve_stop(polfed_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* POLFED_H */

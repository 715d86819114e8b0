/*
 * rtucker.h -- randomized Tucker decomposition with Kronecker-structured sketches
 * on AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * Method: Minster, Li, Ballard, "Parallel Randomized Tucker Decomposition
 * Algorithms" (arXiv 2211.13028).  Notation: a d-way tensor X of size
 * I_1 x ... x I_d, target ranks r_n, oversampling p, ell_n = r_n + p,
 * Kronecker factors Phi_k (s_k x I_k) of the sketch, sketch width
 * ltilde_n = prod_{k != n} s_k.
 *
 * Conventions shared by every entry point
 *  - Tensors are dense, contiguous, C order (last index fastest).  A mode-n
 *    unfolding X_(n) is the I_n x (N / I_n) row-major matrix whose row i holds
 *    the slice i_n = i flattened in C order.  (The paper unfolds column-major;
 *    the two differ by a column permutation, which changes no range, rank or
 *    singular value; in C order the Kronecker factors of a multi-TTM appear in
 *    ascending mode order.)
 *  - Matrices are row-major.
 *  - Pointers named "device" must be device memory of the current HIP device;
 *    the caller owns all of them.  The library never allocates device memory:
 *    scratch space is the caller's workspace `ws` of `ws_bytes` bytes (256-byte
 *    aligned), whose required size the matching *_workspace query returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every compute entry point validates its arguments on the host, then only
 *    enqueues work on `stream` and returns: it does not synchronise, unless
 *    stated otherwise.
 *  - Results are bitwise reproducible for identical inputs and launch sizes
 *    (fixed-order reductions, no floating-point atomics).
 *  - Errors are returned as rt_status codes (never exceptions); on error no
 *    work has been enqueued, except RT_EHIP, which reports a failed HIP call.
 */
#ifndef RTUCKER_H
#define RTUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_MAX_D 8

typedef enum {
  RT_OK = 0,
  RT_EINVAL = -1,     /* bad scalar argument, NULL pointer, bad mode mask */
  RT_ESHAPE = -2,     /* dimensions, ranks or sketch sizes inconsistent or beyond limits */
  RT_EDTYPE = -3,     /* dtype not supported by this entry point */
  RT_EWORKSPACE = -4, /* workspace NULL, misaligned or smaller than the query's answer */
                      /* (-5 is not used: rtucker_rel_error counts non-finite input
                          entries in its device output instead, since it does not
                          synchronise) */
  RT_EHIP = -6,       /* a HIP runtime call failed */
  RT_ENOTCONVERGED = -7 /* an iterative eigensolver stopped at its iteration limit
                           (rtucker_sthosvd; the outputs hold its last iterate) */
} rt_status;

typedef enum {
  RT_F64 = 0,    /* IEEE binary64 */
  RT_F32 = 1,    /* IEEE binary32 */
  RT_BF16 = 2,   /* bfloat16 (binary32 with 8 significant bits) */
  RT_F8E4M3 = 3  /* OCP FP8 E4M3 ("e4m3fn": bias 7, max 448, no infinities) */
} rt_dtype;

typedef enum {
  RT_RHKRON = 0,          /* randomized HOSVD with Kronecker factor reuse (Alg. 4.4, Sec. 4.3) */
  RT_RSTHKRON = 1,        /* randomized STHOSVD with Kronecker products (Alg. 4.3, Sec. 4.2) */
  RT_RHKRON_NOREUSE = 2   /* randomized HOSVD with an independent Kronecker factor set per
                             mode (App. A); subranks as the d x d matrix of Alg. 4.3 */
} rt_algo;

/* A dense C-order tensor in device memory. */
typedef struct {
  int32_t d;                /* order, 2..RT_MAX_D */
  int64_t dims[RT_MAX_D];   /* I_1..I_d (entries past d ignored) */
  rt_dtype dtype;
  const void* data;         /* device pointer */
} rt_tensor;

/* Human-readable name of a status code (static string). */
const char* rtucker_status_string(int status);

/* Library version string (static). */
const char* rtucker_version(void);

/* ------------------------------------------------------------------ sizes
 * Sketch sizes (Sec. 4.2 and 4.3, "choosing subranks").  Host only.
 *  RT_RHKRON:   s_out[d]:  s_i = ceil((prod_j ell_j)^(1/(d-1)) / ell_i), computed
 *               exactly in integers (least s with (s*ell_i)^(d-1) >= prod ell).
 *  RT_RSTHKRON, RT_RHKRON_NOREUSE: s_out[d*d] (row-major S, diagonal 1): row j
 *               holds d-1 integer factors of ell_j, each >= 2; when ell_j has no
 *               such split, ell_j is raised to the least value that has one (extra
 *               oversampling); the most balanced split (smallest largest factor) is
 *               taken and assigned to modes k != j in ascending order, largest first.
 * Fails with RT_ESHAPE if r_n > I_n, and if any s_k exceeds the mode size it
 * will be applied to (I_k; for RT_RSTHKRON and k < j the truncated size). */
int rtucker_sketch_sizes(int32_t d, const int64_t* dims, const int32_t* r, int32_t p,
                         rt_algo algo, int64_t* s_out);

/* ------------------------------------------------------------------ sketch
 * All-at-once sketch multi-TTM (Alg. 4.4 sketch step; Sec. 4.4 dimension tree):
 *   Y_n = X x_{k != n} Phi_k, returned as its mode-n unfolding, for every mode n
 *   whose bit is set in mode_mask.
 *  X:       d >= 2; dtype F64, F32, BF16 or F8E4M3.  The arithmetic runs in the
 *           dtype of X: each Phi_k is rounded (to nearest even) to that dtype;
 *           products accumulate in binary32 (binary64 when X is F64).  X is read
 *           once for all requested modes.
 *  phi[k]:  device, binary64, s_k x I_k row-major, for every k (a factor that no
 *           requested mode uses may be NULL).
 *  s[k]:    subranks, 1 <= s_k <= I_k.
 *  Y[n]:    device, I_n x ltilde_n row-major, column index = C-order index of
 *           (c_k, k != n ascending); binary64 when X is F64, else binary32.
 *           Y[n] may be NULL for modes not in mode_mask.
 *  ws:      at least rtucker_sketch_workspace() bytes. */
int rtucker_sketch_workspace(const rt_tensor* X, const int64_t* s, uint32_t mode_mask,
                             size_t* bytes);
int rtucker_sketch(const rt_tensor* X, const double* const* phi, const int64_t* s,
                   uint32_t mode_mask, void* const* Y, void* ws, size_t ws_bytes, void* stream);

/* The single streaming pass of that sketch: the two children of the root of the
 * dimension tree (Sec. 4.4), computed together in one read of X,
 *   Z = X x_d Phi_d          (dims of X with the last mode replaced by s_last)
 *   W = X x_{d-1} Phi_{d-1}  (dims of X with mode d-1 replaced by s_prev)
 * with the same operand rounding and accumulation as rtucker_sketch.  Every
 * sketch of a mode is Z or W contracted further by small factors.
 *  phi_prev: device binary64 s_prev x I_{d-1}; phi_last: s_last x I_d.
 *  Z, W: device, compute type (binary64 for F64 X, else binary32), C order;
 *  either may be NULL (not computed; its factor may then be NULL too).
 *  ws: at least rtucker_sketch_pass_workspace() bytes (sized for both outputs). */
int rtucker_sketch_pass_workspace(const rt_tensor* X, int64_t s_prev, int64_t s_last, size_t* bytes);
int rtucker_sketch_pass(const rt_tensor* X, const double* phi_prev, int64_t s_prev,
                        const double* phi_last, int64_t s_last, void* Z, void* W, void* ws,
                        size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ QR
 * Thin QR of a tall-skinny sketch (range-finder QR, Alg. 2.3): Y = Q R in
 * binary64 with diag(R) >= 0, so Q is unique when Y has full column rank.
 * Method: CholeskyQR2 (Gram matrix, Cholesky factor, Q = Y R^-1, twice); when a
 * Cholesky pivot falls below 1e-13 of the largest diagonal entry (Y numerically
 * rank deficient) the call switches, on the device, to Householder reflections
 * (tall-skinny QR), for which Q is an orthonormal basis whose leading columns
 * span range(Y).
 *  Y: device, m x n row-major, dtype F32 or F64 (read, widened to binary64).
 *  Q: device, binary64, m x c row-major, c = min(m, n).
 *  R: device, binary64, c x n row-major (upper triangular), or NULL.
 * Limits: 1 <= n <= 64 (RT_ESHAPE beyond), m >= 1. */
int rtucker_qr_workspace(int64_t m, int64_t n, size_t* bytes);
int rtucker_qr(int64_t m, int64_t n, const void* Y, rt_dtype y_dtype, double* Q, double* R,
               void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ core
 * Core multi-TTM (Alg. 4.4 core step): G = X x_k U_k^T over the modes k in
 * mode_mask (a single bit gives one TTM, as in each step of Alg. 4.3).
 *  U[k]: device, binary64, I_k x l_k row-major (orthonormal columns in the
 *        method, but any matrix is accepted), for k in mode_mask.
 *  l[k]: number of columns of U[k], 1 <= l_k <= 64.
 *  G:    device; dims l_k for k in mode_mask and I_k otherwise; binary64 when X
 *        is F64, else binary32.
 *  Arithmetic: modes are contracted largest first (ties: lower mode first).  The
 *  first contraction reads X in its own dtype (F64, F32 or BF16) with U rounded
 *  to that dtype and binary32 accumulation (binary64 for F64); later ones run on
 *  the binary32 (binary64) intermediate with U rounded to binary32 (binary64). */
int rtucker_core_workspace(const rt_tensor* X, const int64_t* l, uint32_t mode_mask,
                           size_t* bytes);
int rtucker_core(const rt_tensor* X, const double* const* U, const int64_t* l,
                 uint32_t mode_mask, void* G, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ decompose
 * Full randomized Tucker decomposition [G; U_1..U_d] of X at ranks r with
 * oversampling p (Alg. 4.3 or Alg. 4.4): sketches, QR, core, then the holistic
 * truncation STHOSVD(G_hat, r) in mode order 1..d (Sec. 4.1) computed in
 * binary64 (Gram matrix of each core unfolding, its r_j leading eigenvectors by
 * Householder tridiagonalisation, bisection and inverse iteration, with one-sided
 * Jacobi as the fallback), and U_j = U_hat_j V_j.
 *  X:        dtype F64, F32 or BF16.
 *  X_sketch: NULL, or a tensor with X's dims used for the sketch instead of X
 *            (e.g. an F8E4M3 copy); RT_RHKRON only.
 *  Sketch passes over X: one for RT_RHKRON (all modes, dimension tree), one per mode for
 *  RT_RHKRON_NOREUSE, one per step on the shrinking core for RT_RSTHKRON.
 *  r[d], p:  1 <= r_n <= min(I_n, ltilde_n), p >= 0.
 *  s:        RT_RHKRON: d subranks; RT_RSTHKRON, RT_RHKRON_NOREUSE: d*d row-major
 *            subrank matrix (diagonal ignored); NULL = rtucker_sketch_sizes().  Must
 *            satisfy ltilde_n >= r_n + p.
 *  phi:      device binary64 random factors (Gaussian, or SRHT from
 *            rtucker_srht_factor).  RT_RHKRON: phi[k] is s_k x I_k.
 *            RT_RSTHKRON: phi[j*d + k] (k != j) is s_{j,k} x n_k with n_k = c_k
 *            for k < j and I_k for k > j, where c_k = min(I_k, ltilde_k) is the
 *            truncated size of mode k.  RT_RHKRON_NOREUSE: phi[j*d + k] (k != j) is
 *            s_{j,k} x I_k.
 *  G:        device binary64, r_1 x ... x r_d.
 *  U[j]:     device binary64, I_j x r_j.  Columns ordered by decreasing singular
 *            value of the core unfolding; each column's largest-magnitude entry
 *            of V_j is positive.
 * Limits: ltilde_n clipped to I_n must be <= 64. */
int rtucker_decompose_workspace(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r,
                                int32_t p, const int64_t* s, rt_algo algo, size_t* bytes);
int rtucker_decompose(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r, int32_t p,
                      const int64_t* s, rt_algo algo, const double* const* phi, double* G,
                      double* const* U, void* ws, size_t ws_bytes, void* stream);

/* The same decomposition with its time split by phase (the breakdown of Sec. 7.5-7.6
 * in the paper's own terms): an event is recorded on `stream` at each phase boundary,
 * the call synchronises `stream`, and phase_ms (host, 4 floats) receives the device
 * time in milliseconds of
 *   [0] sketch (operand rounding, the streaming pass and the tree contractions),
 *   [1] QR of the sketches, [2] core multi-TTM, [3] truncation (STHOSVD of the core and
 *   U_j = U_hat_j V_j),
 * summed over the steps of Alg. 4.3 for RT_RSTHKRON.  Results equal rtucker_decompose's
 * bit for bit.  RT_EINVAL if phase_ms is NULL. */
int rtucker_decompose_phases(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r,
                             int32_t p, const int64_t* s, rt_algo algo, const double* const* phi,
                             double* G, double* const* U, void* ws, size_t ws_bytes, void* stream,
                             float* phase_ms);

/* Allocation-free form of rtucker_decompose, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments and results as rtucker_decompose without ws/ws_bytes:
 * the workspace is a static device array of the library, RTUCKER_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per GPU, held until the process ends (enough for, e.g., 256^3 binary32 at
 * ranks 16).  The call allocates nothing and copies nothing from the host; its first
 * call on a device looks up that device's array.  Every call on one GPU uses the same
 * array, so calls that overlap on one GPU (concurrent streams or threads) race; calls
 * ordered on one stream do not.  No part of the array needs clearing between calls:
 * every kernel initialises what it reads.
 * RT_EWORKSPACE if rtucker_decompose_workspace() exceeds the array; RT_EHIP if the
 * array's address cannot be obtained. */
#define RTUCKER_NOALLOC_SCRATCH_BYTES (64ull << 20)
int rtucker_decompose_noalloc(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r,
                              int32_t p, const int64_t* s, rt_algo algo, const double* const* phi,
                              double* G, double* const* U, void* stream);

/* ------------------------------------------------------------------ deterministic STHOSVD
 * The deterministic sequentially truncated HOSVD (Alg. 2.2) of X at ranks r, the baseline
 * the randomized algorithms are compared with (Sec. 7.4-7.5): for j = 1..d, V_j = the r_j
 * leading eigenvectors of the Gram matrix of the current tensor's mode-j unfolding
 * (products of the binary32 or binary64 entries accumulated in binary64: a binary32 Gram
 * matrix would lose the trailing eigenvalues, whose sum is the squared error), then the
 * tensor is contracted with V_j^T in mode j.  G = the final tensor, U_j = V_j.
 * Eigenvectors: the one-workgroup solver of the truncation for I_j <= 64; for larger
 * modes subspace iteration on 64 vectors with Rayleigh-Ritz every 4 iterations until
 * max_i ||M v_i - theta_i v_i|| <= 1e-12 theta_1 (at most 400 iterations; the host reads
 * one value per check).  Columns in decreasing eigenvalue order, each column's
 * largest-magnitude entry positive.
 *  X: F64 or F32.  r[j] <= I_j, and r[j] <= 32 when I_j > 64 (<= 64 otherwise).
 *  G: device binary64 r_1 x ... x r_d.  U[j]: device binary64 I_j x r_j.
 *  iterations (host, nullable): subspace iterations summed over the modes.
 *  Synchronises `stream`.  RT_ENOTCONVERGED when a mode hit the iteration limit. */
int rtucker_sthosvd_workspace(const rt_tensor* X, const int32_t* r, size_t* bytes);
int rtucker_sthosvd(const rt_tensor* X, const int32_t* r, double* G, double* const* U,
                    int32_t* iterations, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ error
 * Squared norms for the relative reconstruction error (Sec. 5), in binary64 on
 * the device, by explicit residual (no cancellation-prone identity):
 *   out[0] = ||X - G x_1 U_1 ... x_d U_d||^2,  out[1] = ||X||^2,
 *   out[2] = ||G||^2,  out[3] = number of non-finite (NaN or +-Inf) entries of X,
 *   as a double.  Non-finite entries are left out of out[0] and out[1], so a
 *   caller that finds out[3] > 0 knows the two norms cover the finite part only.
 *  G: device binary64 r_1 x ... x r_d; U[j]: device binary64 I_j x r_j.
 *  out: device, 4 doubles.  X: dtype F64, F32 or BF16. */
int rtucker_rel_error_workspace(const rt_tensor* X, const int32_t* r, size_t* bytes);
int rtucker_rel_error(const rt_tensor* X, const double* G, const int32_t* r,
                      const double* const* U, double* out, void* ws, size_t ws_bytes,
                      void* stream);

/* ------------------------------------------------------------------ precision
 * Elementwise conversion dst[i] = round(src[i] * 2^scale_exp) to dst_dtype with
 * round-to-nearest-even.  F8E4M3 saturates finite values to +-448 and maps NaN
 * or Inf to NaN (0x7f/0xff); BF16 and F32 overflow to Inf.
 *  src_dtype: F64 or F32.  dst_dtype: F32, BF16 or F8E4M3.  n >= 0. */
int rtucker_convert(const void* src, rt_dtype src_dtype, void* dst, rt_dtype dst_dtype,
                    int64_t n, int32_t scale_exp, void* stream);

/* ------------------------------------------------------------------ SRHT factors
 * A subsampled randomized Hadamard factor of the Kronecker sketch (Sec. 5.1):
 *   Phi = (R H D)[:, :n],  phi[i*n + j] = signs[j] * H[rows[i]][j] / sqrt(N),
 * with N the least power of two >= n (a mode of size n is read as zero-padded to N),
 * H the N x N Walsh-Hadamard matrix in Sylvester order (H[a][b] = (-1)^popcount(a & b)),
 * D = diag(signs) and R the selection of rows.  The result is a binary64 s x n row-major
 * matrix, usable as phi[k] of rtucker_sketch / rtucker_decompose.
 *  rows:  device, s distinct int64 in [0, N) (not checked: an index outside gives a
 *         wrong factor, never an access outside the buffers);
 *  signs: device, n binary64 values +-1;  phi: device, s x n binary64.
 *  RT_ESHAPE unless 1 <= s <= N and n >= 1. */
int rtucker_srht_factor(int64_t n, int64_t s, const int64_t* rows, const double* signs, double* phi,
                        void* stream);

/* The SRHT sketch of the contiguous last mode by a fast Walsh-Hadamard transform:
 *   Z = X x_d Phi  with Phi = (R H D)[:, :Q] as in rtucker_srht_factor (Q = I_d),
 * in O(log N) operations per entry of X instead of s.  Each fiber of Q values is signed,
 * zero-padded to N, transformed, scaled by 1/sqrt(N) and sampled at `rows`.
 *  X: F32, 1 <= d <= 8, any sizes, Q <= 4096 (N <= 4096); Z: device binary32, X's dims
 *  with the last replaced by s, C order.  1 <= s <= min(64, N).  rows: device int64,
 *  s distinct values in [0, N) (reduced modulo N, not checked); signs: device binary64,
 *  Q values +-1.  Arithmetic in binary32. */
int rtucker_srht_sketch_last(const rt_tensor* X, int64_t s, const int64_t* rows, const double* signs,
                             float* Z, void* stream);

/* ------------------------------------------------------------------ adjoint
 * Plain multi-TTM and its adjoint pieces, for differentiation (Sec. 2.1
 * multi-TTM; the adjoint of Y = X x_k A_k is dX = dY x_k A_k^T and
 * dA_n = dY_(n) Z_(n)^T with Z = X x_{k != n} A_k).
 *
 * rtucker_multi_ttm: Y = X x_k op(A_k) for k in mode_mask, where op(A) = A
 *  (A_k: m_k x I_k) or, with transpose != 0, op(A) = A^T (A_k: I_k x m_k).
 *  X, A_k, Y share one dtype, F32 or F64; arithmetic in that dtype.  Y dims:
 *  m_k for k in mode_mask, I_k otherwise.  1 <= m_k <= 256.
 * rtucker_mode_contract: out[i][j] = sum over all indices except mode n of
 *  P[.., i, ..] * Q[.., j, ..]  (= P_(n) Q_(n)^T).  P, Q: same dtype (F32 or
 *  F64), same dims except mode n.  out: device, P.dims[n] x Q.dims[n], that dtype.
 *  With accumulate != 0 the result is added to what out holds (out += ...), so
 *  the two contributions to a factor used twice sum without another call.
 * rtucker_sq_residual: R = A - B elementwise (R may be NULL) and
 *  out[0] = sum (A - B)^2 accumulated in binary64.  A, B (and R): same dims and
 *  dtype, F32 or F64; out: device, 1 double.  ws: device, >= 8192 bytes,
 *  256-byte aligned (partial sums of the fixed-order reduction).
 * rtucker_scaled_diff: out = alpha * g[0] * (A - B) elementwise, the adjoint of
 *  the squared residual (dA = 2 g R, dB = -2 g R) and of its projected form.
 *  g: device binary64 scalar or NULL (= 1); B: NULL means 0.  A, B, out: same
 *  dims and dtype (F32 or F64); out may alias A or B. */
int rtucker_multi_ttm_workspace(const rt_tensor* X, const int64_t* m, uint32_t mode_mask,
                                size_t* bytes);
int rtucker_multi_ttm(const rt_tensor* X, const void* const* A, const int64_t* m,
                      uint32_t mode_mask, int32_t transpose, void* Y, void* ws, size_t ws_bytes,
                      void* stream);
int rtucker_mode_contract(const rt_tensor* P, const rt_tensor* Q, int32_t n, int32_t accumulate,
                          void* out, void* ws, size_t ws_bytes, void* stream);
int rtucker_mode_contract_workspace(const rt_tensor* P, const rt_tensor* Q, int32_t n,
                                    size_t* bytes);
int rtucker_sq_residual(const rt_tensor* A, const void* B, void* R, double* out, void* ws,
                        size_t ws_bytes, void* stream);
int rtucker_scaled_diff(const rt_tensor* A, const void* B, const double* g, double alpha, void* out,
                        void* stream);

/* ------------------------------------------------------------------ batched
 * Batched factor-reuse decomposition of many independent 3-way tensors of
 * different sizes (Alg. 4.4, Sec. 4.3, applied to each tensor): every phase
 * (operand rounding, sketch pass, sketch contractions, QR, core contractions,
 * truncation Gram / eigensolver / contractions) runs for all tensors in one
 * grouped launch, about 25 launches whatever the batch size.
 * Per item: X (device, dtype of the batch, dims[3]), r[3], s[3] (subranks;
 * 0 entries = formula), phi[3] (device binary64 s_k x I_k), G (device binary64
 * r1 x r2 x r3), U[3] (device binary64 I_k x r_k).
 *  dtype: F32 or BF16.  count >= 1.  Limits per item: I_k <= 256, s_k <= 8,
 *  sketch widths prod_{k != n} s_k <= 64 and >= r_n + p.
 *  Workspace: rtucker_decompose_batched_workspace (independent of tuning); the
 *  first part of it holds the job tables.
 * rtucker_decompose_batched: writes the job tables into ws (a blocking host to
 *  device copy) and enqueues all phases on `stream`.
 * rtucker_decompose_batched_upload: only writes the job tables (blocking).
 * rtucker_decompose_batched_launch: only enqueues the kernels, reading the
 *  tables left in ws by an upload with the same arguments.  It copies nothing
 *  from the host and allocates nothing, so it can be captured in a graph.
 * rtucker_decompose_batched_autotune: times the whole batch for each pair of a
 *  row tile of the vector-ALU core contractions (8, 16, 32 rows) and a number of
 *  slabs that a wave of the sketch pass takes in turn (at most 1, 2 or 4), keeps
 *  the fastest for this batch signature (sizes, ranks, subranks, p, dtype) for the
 *  rest of the process, writes chosen[0] = row tile and chosen[1] = slabs
 *  (chosen: nullable, 2 int32), and leaves the matching tables in ws.  It
 *  synchronises `stream`.  When the environment variable RTUCKER_TUNE_CACHE names
 *  a file, the choice is also appended to it ("<signature key, 16 hex digits>
 *  <row tile> <slabs>" per line), and every batched call of a process that has the
 *  variable set reads the file once per path before it looks a signature up, so a
 *  later process starts tuned; lines that do not parse are skipped.  The slabs
 *  setting does not change any result; the row tile changes the summation order
 *  of the vector-ALU contractions only.
 * rtucker_decompose_batched_tuning: host only; the setting the batched calls would
 *  use now for this signature (the cache, else the defaults 16 and 4): tuning[0] =
 *  row tile, tuning[1] = slabs, and *key = the signature key of the cache file. */
typedef struct {
  const void* X;
  int64_t dims[3];
  int32_t r[3];
  int64_t s[3];
  const double* phi[3];
  double* G;
  double* U[3];
} rt_batch_item;

int rtucker_decompose_batched_workspace(int32_t count, const rt_batch_item* items, int32_t p,
                                        rt_dtype dtype, size_t* bytes);
int rtucker_decompose_batched(int32_t count, const rt_batch_item* items, int32_t p,
                              rt_dtype dtype, void* ws, size_t ws_bytes, void* stream);
int rtucker_decompose_batched_upload(int32_t count, const rt_batch_item* items, int32_t p,
                                     rt_dtype dtype, void* ws, size_t ws_bytes, void* stream);
int rtucker_decompose_batched_launch(int32_t count, const rt_batch_item* items, int32_t p,
                                     rt_dtype dtype, void* ws, size_t ws_bytes, void* stream);
int rtucker_decompose_batched_autotune(int32_t count, const rt_batch_item* items, int32_t p,
                                       rt_dtype dtype, void* ws, size_t ws_bytes, void* stream,
                                       int32_t* chosen);
int rtucker_decompose_batched_tuning(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype,
                                     int32_t* tuning, uint64_t* key);

#ifdef __cplusplus
}
#endif

#endif /* RTUCKER_H */

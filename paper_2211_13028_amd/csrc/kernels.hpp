// Internal launchers of rtucker's HIP kernels (not part of the C ABI).
// Every launcher enqueues on `st` and returns the launch status.
#pragma once

#include "common.hpp"

namespace rt {

// ------------------------------------------------------------------ k_basic.hip
// dst[i] = round(src[i] * 2^scale_exp) (RNE); see rtucker_convert.
// Phi = (R H D)[:, :n] for a subsampled randomized Hadamard factor: phi[i*n + j] =
// signs[j] * (-1)^popcount(rows[i] & j) * inv_sqrt_N
hipError_t launch_srht_factor(int64_t n, int64_t s, const int64_t* rows, const double* signs, double inv_sqrt_N,
                              double* phi, hipStream_t st);
// Z = X x_last (R H D)[:, :Q] by a fast Walsh-Hadamard transform per fiber (Q <= 4096)
bool srht_last_ok(int64_t Q, int64_t s);
hipError_t launch_srht_last(const float* X, int64_t fibers, int64_t Q, const int64_t* rows, const double* signs,
                            int64_t s, float* Z, hipStream_t st);
hipError_t launch_convert(const void* src, rt_dtype sdt, void* dst, rt_dtype ddt, int64_t n,
                          int scale_exp, hipStream_t st);

// Prepare a compute operand from a binary64 matrix:
//   out(i, k) for i < m, k < K, row-major m x K, stored as `store` with values
//   rounded to `round_to` (RNE).  src is m x K row-major (trans == false) or
//   K x m row-major (trans == true).  Rows i >= m up to m_pad are zero-filled.
//   store: RT_F64, RT_F32 (value rounded to round_to, kept in binary32),
//   RT_BF16 (bit patterns; round_to BF16, or F8E4M3 whose values bfloat16 holds exactly)
//   or RT_F8E4M3 (bit patterns; round_to must be F8E4M3).
hipError_t launch_prep_matrix(const double* src, int64_t m, int64_t K, bool trans, rt_dtype round_to,
                              rt_dtype store, int64_t m_pad, void* dst, hipStream_t st);

// Several launch_prep_matrix jobs in one launch.
struct PrepTask {
  const double* src;
  int64_t m, K, m_pad;
  bool trans;
  rt_dtype round_to, store;
  void* dst;
};
constexpr int kMaxPrepTasks = 16;
struct PrepTable {
  PrepTask t[kMaxPrepTasks];
};
hipError_t launch_prep_batch(const PrepTask* tasks, int count, hipStream_t st);

// dst (m_pad x K row-major, binary32) = src (m x K, or K x m with trans), rows >= m zero.
hipError_t launch_pack_f32(const float* src, int64_t m, int64_t K, bool trans, int64_t m_pad, float* dst,
                           hipStream_t st);

// dst[i * (A*B) + a*B + b] = src[a*m*B + i*B + b]   (mode-n unfolding of an (A, m, B) view)
hipError_t launch_unfold(const void* src, size_t esize, int64_t A, int64_t m, int64_t B, void* dst,
                         hipStream_t st);

// Elementwise R = A - B (R may be null) and out[0] = sum (A-B)^2 in binary64, deterministic.
size_t sq_residual_ws(int64_t n);
hipError_t launch_sq_residual(const void* a, const void* b, void* r, rt_dtype dt, int64_t n,
                              double* out, void* ws, hipStream_t st);
// out[i] = alpha * g[0] * (a[i] - b[i]) in dt (F32 or F64); g null means 1, b null means 0.
hipError_t launch_scaled_diff(const void* a, const void* b, const double* g, double alpha, rt_dtype dt,
                              int64_t n, void* out, hipStream_t st);

// ------------------------------------------------------------------ k_ttm.hip
// Y[a, i, b] = sum_k M[i*K + k] * X[a, k, b] for i < m.
//  X dtype xdt; M and Y in the compute type: binary64 if xdt == RT_F64, else binary32.
//  With mtrans, M is stored K x m row-major (M[k*m + i]) instead.
//  When A*B is small the contraction is split over K and `ws` (ttm_generic_ws bytes)
//  holds the partial sums, added in a fixed order.
size_t ttm_generic_ws(rt_dtype xdt, int64_t A, int64_t K, int64_t B, int64_t m);
hipError_t launch_ttm_generic(const void* X, rt_dtype xdt, int64_t A, int64_t K, int64_t B,
                              const void* M, int64_t m, void* Y, void* ws, hipStream_t st,
                              bool mtrans = false);

// MFMA path for X in binary32 or bfloat16 (binary32 accumulation, binary32 output).
//  Operand Mop prepared by launch_prep_matrix with store = xdt (F32 or BF16),
//  m_pad = ttm_mfma_mpad(m).  Requires ttm_mfma_ok().
//  Split-K partial sums use `ws` (ttm_mfma_ws bytes) when the output is too small to fill the chip.
bool ttm_mfma_ok(rt_dtype xdt, int64_t A, int64_t K, int64_t B, int64_t m);
int64_t ttm_mfma_mpad(int64_t m);
size_t ttm_mfma_ws(rt_dtype xdt, int64_t A, int64_t K, int64_t B, int64_t m);
hipError_t launch_ttm_mfma_ws(const void* X, rt_dtype xdt, int64_t A, int64_t K, int64_t B,
                              const void* Mop, int64_t m, float* Y, void* ws, hipStream_t st);

// Several independent binary32 contractions (X binary32, M packed as above) in one kernel
// launch plus one launch for their split sums; jobs whose tile count or M alignment differ
// from the first job's run as separate launches.
constexpr int kMaxF32Group = 8;
struct F32Contraction {
  const float* X;
  int64_t A, K, B;
  const float* Mop;
  int64_t m;
  float* Y;
  void* ws;  // ttm_mfma_ws(RT_F32, A, K, B, m) bytes
};
hipError_t launch_ttm_mfma_f32_group(const F32Contraction* c, int count, hipStream_t st);

// Matrix-core contraction of the last mode (B == 1): Y[a, i] = sum_k X[a, k] Mop[i, k],
// X binary32 A x K row-major, Mop packed to ttm_mfma_mpad(m) rows; K % 4 == 0, m <= 64.
// With Y64 given, the result is written as binary64 there instead (the binary32 sum of
// the split parts, widened exactly), and Y is not used; the workspace query then needs
// f64_out set.
bool ttm_mfma_last_ok(int64_t A, int64_t K, int64_t m);
size_t ttm_mfma_last_ws(int64_t A, int64_t K, int64_t m, bool f64_out = false);
hipError_t launch_ttm_mfma_last(const float* X, int64_t A, int64_t K, const float* Mop, int64_t m, float* Y,
                                void* ws, hipStream_t st, double* Y64 = nullptr);

// ------------------------------------------------------------------ k_sketch.hip
// First level of the sketch dimension tree over X viewed as (A, P, Q):
//   Z[a, p, c] = sum_q X[a,p,q] phiQ[c,q]     (A x P x sQ)
//   W[a, c, q] = sum_p phiP[c,p] X[a,p,q]     (A x sP x Q)
// phiP/phiQ: compute type (binary64 for F64 X, else binary32 holding values
// already rounded to X's dtype), row-major sP x P and sQ x Q.
// Either output may be skipped (null).  Z/W in the compute type.
// bfloat16 or FP8 e4m3 X with P, Q multiples of 8 runs on matrix cores (plan.mfma)
// and also needs phiP16 / phiQ16: the factors rounded to X's dtype, stored as
// bfloat16 (exact), zero-padded to 16 rows.
struct ZWPlan {
  int64_t qblocks, pblocks, rows_per_block;
  size_t ws_bytes;
  bool mfma;
};
ZWPlan sketch_zw_plan(rt_dtype xdt, int64_t A, int64_t P, int64_t Q, int64_t sP, int64_t sQ,
                      bool needZ, bool needW);
bool sketch_zw_ok(rt_dtype xdt, int64_t sP, int64_t sQ);
hipError_t launch_sketch_zw(const void* X, rt_dtype xdt, int64_t A, int64_t P, int64_t Q,
                            const void* phiP, int64_t sP, const void* phiQ, int64_t sQ,
                            const void* phiP16, const void* phiQ16, void* Z, void* W,
                            const ZWPlan& plan, void* ws, hipStream_t st);

// ------------------------------------------------------------------ k_qr.hip
// Thin Householder QR (binary64) of matrices given as (A, m, B) views:
// element (i, j = a*B + b) at Y[a*m*B + i*B + b]; n = A*B <= 64 columns.
struct QRJob {
  const void* Y;
  int64_t A, m, B;
  double* Q;  // m x min(m, n) row-major
  double* R;  // min(m, n) x n row-major, may be null
};
constexpr int kMaxQRJobs = 8;
constexpr int kMaxQRCols = 64;
size_t qr_ws(const QRJob* jobs, int count);
hipError_t launch_qr(const QRJob* jobs, int count, rt_dtype ydt, void* ws, hipStream_t st);
// Orthonormal basis Q (m x n, m >= n) of the columns of a binary64 m x n matrix Y that may
// be ill-conditioned or numerically rank-deficient (the subspace iteration's M Q): two
// shifted Cholesky QR passes into T (m x n scratch), then CholeskyQR2 of T (Householder
// if that breaks down).  ws: orth_ws(m, n) bytes.
size_t orth_ws(int64_t m, int n);
hipError_t launch_orth(const double* Y, int64_t m, int n, double* T, double* Q, void* ws, hipStream_t st);

// ------------------------------------------------------------------ k_eig.hip
// out[i][j] = sum_{a,b} P[a,i,b] * Q[a,j,b], P: (A, mP, B), Q: (A, mQ, B); same dtype
// (F32 or F64); out in that dtype, mP x mQ row-major; deterministic two-stage sum.
size_t mode_contract_ws(rt_dtype dt, int64_t A, int64_t mP, int64_t mQ, int64_t B);
// With accumulate, out += P_(n) Q_(n)^T instead.
hipError_t launch_mode_contract(const void* P, const void* Q, rt_dtype dt, int64_t A, int64_t mP,
                                int64_t mQ, int64_t B, void* out, void* ws, hipStream_t st,
                                bool accumulate = false);

// out = X_(n) X_(n)^T (m x m, binary64) of a binary32 (A, m, B) view, accumulated in binary64
size_t gram_wide_ws(int64_t A, int64_t m, int64_t B);
hipError_t launch_gram_wide(const float* X, int64_t A, int64_t m, int64_t B, double* out, void* ws,
                            hipStream_t st);

// Leading eigenpairs (binary64) of a symmetric positive semidefinite n x n matrix
// (n <= 64): Householder tridiagonalisation, multisection and inverse iteration for
// r <= 32, one-sided Jacobi on a pivoted Cholesky factor otherwise or when the first
// method's orthogonality / residual checks fail.  V (n x r row-major) = eigenvectors
// of the r largest eigenvalues, in decreasing order, each column's largest-magnitude
// entry (first on ties) made positive.  evals (may be null): those r eigenvalues.
// C = A B for up to kMaxSmallGemm binary64 jobs in one launch (row-major; A: m x k,
// B: k x n, k, n <= 64), 64 rows of C per workgroup: the factor updates U_j = U_hat_j V_j
// and the truncation's last-mode contraction.
constexpr int kMaxSmallGemm = 8;
struct SmallGemmJob {
  const double* A;
  const double* B;
  double* C;
  int64_t m;
  int32_t k, n;
};
hipError_t launch_small_gemm_f64(const SmallGemmJob* jobs, int count, hipStream_t st);
hipError_t launch_sym_eig_top(const double* M, int64_t n, int64_t r, double* V, double* evals,
                              hipStream_t st);
// subspace iteration pieces for Gram matrices larger than 64 x 64 (deterministic STHOSVD):
// a fixed pseudo-random n x b start block; max_i ||(M V)_i - theta_i V_i|| / theta_0 of
// Ritz pairs (r <= 64); the sign rule (largest-magnitude entry positive) on n x r columns
hipError_t launch_subspace_start(double* Q, int64_t n, int b, hipStream_t st);
hipError_t launch_ritz_residual(const double* MV, const double* V, const double* theta, int64_t n, int r,
                                double* out, hipStream_t st);
hipError_t launch_column_sign(double* V, int64_t n, int r, hipStream_t st);

// ------------------------------------------------------------------ k_norm.hip
// Residual of X viewed as (I1, Brest) against U1 (I1 x r1) times T (r1 x Brest),
// both binary64: out[0] += ||X - U1 T||^2, out[1] = ||X||^2, out[3] = #nonfinite(X);
// out[2] is left to the caller.  Deterministic.
size_t recon_residual_ws(int64_t I1, int64_t Brest);
hipError_t launch_recon_residual(const void* X, rt_dtype xdt, int64_t I1, int64_t Brest,
                                 const double* U1, const double* T, int64_t r1, double* out,
                                 void* ws, hipStream_t st);
// out[2] = ||G||^2 for a binary64 array of n values.
hipError_t launch_sumsq_f64(const double* g, int64_t n, double* out_slot, hipStream_t st);

// ------------------------------------------------------------------ grouped launches
// For the batched decomposition: each launcher below runs many independent jobs
// of one kind in a single launch.  The job table lives in device memory; job j
// owns the workgroups [blk0_j, blk0_j + blocks_j) of a flat grid.  Where jobs
// own many workgroups, a device map blkjob[workgroup] = job replaces a search.

// k_basic.hip: operand rounding (PrepTask per job, blockIdx.y = job) and
// binary32 -> binary64 copies.
hipError_t launch_prep_grouped(const PrepTask* tasks, int count, int64_t max_elems, hipStream_t st);
struct GCopyJob {
  const float* src;
  double* dst;
  int64_t n;
};
hipError_t launch_copy_f64_grouped(const GCopyJob* jobs, int count, int64_t max_elems, hipStream_t st);

// k_ttm.hip: generic TTM jobs (as launch_ttm_generic, no split-K).  Each job's
// workgroups cover ceil(A*B / 64) column blocks times ceil(m / mt) row tiles
// (column-block major, so the tiles of one column block run together).
struct GTtmJob {
  const void* X;
  const void* M;
  void* Y;
  int64_t A, K, B, m;
  int64_t blk0, colblocks, mtiles;
  int32_t mtrans, pad;
};
int64_t ttm_grouped_blocks(int64_t A, int64_t B, int64_t m, int mt);
hipError_t launch_ttm_grouped(const GTtmJob* jobs, const int32_t* blkjob, int count, int64_t total_blocks,
                              rt_dtype xdt, int mt, hipStream_t st);

// First sketch level (Z = X x_3 PhiQ: A x P x sQ, W = X x_2 PhiP: A x sP x Q) of one 3-way
// tensor (A, P, Q) of a batch; Q <= 256, s <= 16, operands binary32; Z or W may be null.
// Workgroups blk0 .. of the job each take a run of 4 spb slabs.
struct GZwJob {
  const void* X;
  const float* phiP;
  const float* phiQ;
  float* Z;
  float* W;
  int64_t A, P, Q;
  int64_t blk0;
  int32_t sP, sQ;
  int32_t spb, pad;
};
// k_batch.hip: the same first sketch level for binary32 or bfloat16 tensors on 256-thread
// workgroups (four waves, each walking every fourth slab of the workgroup's run of
// 4 spb slabs), jobs grouped by column class ng = zw_batch_class(Q) in {4, 8, 12, 16}
// (16 ng >= Q); every job of one launch has the launch's class.
int zw_batch_class(int64_t Q);
hipError_t launch_zw_batch(const GZwJob* jobs, const int32_t* blkjob, int64_t total_blocks, int ng, rt_dtype xdt,
                           hipStream_t st);
// k_batch.hip: core contractions of every tensor of a batch on matrix cores,
// Y = X x_k M for (A, K, B) views with B == 1 (rows = true) or B >= 16 (rows = false),
// K <= 256, m <= 16 mt (ttm_batch_fits); binary32 or bfloat16 X, binary32 M (bfloat16
// values for bfloat16 X) and Y.  A job has colblocks = ttm_batch_units(A, B) units (one
// wave each, B == 1: 16-row tiles), taking ttm_batch_blocks(A, B) workgroups from blk0 on;
// blkjob maps workgroups to jobs.
int64_t ttm_batch_units(int64_t A, int64_t B);
int64_t ttm_batch_blocks(int64_t A, int64_t B);
int64_t ttm_batch_row_tiles(int64_t A, int64_t B);  // the job's mtiles (B == 1: units per wave)
bool ttm_batch_fits(int64_t K, int64_t B, int64_t m);
hipError_t launch_ttm_batch(const GTtmJob* jobs, const int32_t* blkjob, int64_t total_blocks, int mt, bool rows,
                            rt_dtype xdt, hipStream_t st);

// k_qr.hip: thin Householder QR of (A, m, B) views with m <= 256 rows and
// n = A*B <= 64 columns, one workgroup per job; Q: m x qcols (qcols = min(m, n)).
// With flag set, a job runs only when *flag != 0 (the Householder fallback of CholeskyQR2).
struct GQrJob {
  const void* Y;
  int64_t A, m, B;
  double* Q;
  int32_t n, qcols;
  const int32_t* flag;
};
hipError_t launch_qr_grouped(const GQrJob* jobs, int count, rt_dtype ydt, hipStream_t st);
// CholeskyQR2 of (A, m, B) views with m >= n = A*B <= 64 (the single-decomposition
// path's fast QR), many jobs per launch.  Per job: part = 2 x chunks x 64 x 64
// binary64 (chunks = ceil(m / 64)), R1, R2: 64 x 64, Q1: m x n, Q: m x n (ld n),
// Rout (may be null): n x n, flag: set to 1 when a Cholesky pivot breaks down (the
// job must then be redone by the Householder kernel).  shift1 / shift2 > 0 make the
// pass-1 / pass-2 factorisation a shifted one, of G + shift * trace(G) * I (zero: plain).
struct GCholQRJob {
  const void* Y;
  int64_t A, m, B;
  int32_t n;
  double* part;
  int32_t chunks;
  double* R1;  // 2 x 64 x 64: R1, then R1^-1
  double* R2;  // 2 x 64 x 64: R2, then R2^-1
  double* Q1;
  double* Q;
  double* Rout;
  int32_t* flag;
  double shift1, shift2;
};
// cols (32 or 64): every job of the launch has n <= cols, and its buffers are read with
// cols in place of 64 (part: 2 x chunks x cols x cols, R1 / R2: 2 x cols x cols), so
// 64-column allocations serve both widths.
hipError_t launch_cholqr2_grouped(const GCholQRJob* jobs, int count, int max_chunks, rt_dtype ydt, hipStream_t st,
                                  int cols = 64);

// k_eig.hip: Gram matrices out = G_(n) G_(n)^T of binary64 (A, m, B) views
// (m <= 64), and the eigensolver of launch_sym_eig_top, one workgroup per job.
struct GGramJob {
  const double* G;
  double* out;
  int64_t A, m, B;
};
// max_m: the largest m of the jobs (<= 64); at most 32 selects the small-core kernel (A B < 2^31)
hipError_t launch_gram_grouped(const GGramJob* jobs, int count, hipStream_t st, int max_m = 64);
struct GEigJob {
  const double* M;
  double* V;
  int32_t n, r;
};
// max_r: the largest r of the jobs; at most 16 selects the half-scratch variant
hipError_t launch_eig_grouped(const GEigJob* jobs, int count, hipStream_t st, int max_r = 32);

}  // namespace rt

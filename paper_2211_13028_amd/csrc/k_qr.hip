// Thin QR of tall-skinny sketches in binary64 (the range finder's QR step,
// Alg. 2.3), Householder reflections with diag(R) >= 0.
//
// Design: a block of up to 256 rows x 64 columns lives in LDS (128 KiB of the
// 160 KiB a gfx950 CU has) and one 256-thread workgroup factors it with
// Householder reflections (two barriers per reflection) and then forms its
// explicit Q in place (backward accumulation).  Taller matrices use a TSQR
// tree: independent 256-row blocks, their stacked R factors factored again,
// and Q = blockdiag(Q_b) * Q_top, so several CUs share the work.
#include <vector>

#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kRowsMax = 256;
constexpr int kCols = kMaxQRCols;  // 64
constexpr int kQRThreads = 256;
constexpr int kMaxTasks = 24;

struct QRTask {
  const void* src;   // (A, m, B) view, element (i, j=a*B+b) at a*m*B + i*B + b
  int64_t A, m, B;
  int64_t row0;      // first row of the block
  int32_t rows;      // rows in the block (<= 256)
  int32_t n;         // columns (= A*B <= 64)
  double* Q;         // rows x qcols, leading dimension ldq
  int32_t ldq, qcols;
  double* R;         // rrows x n (leading dimension n), or null
  int32_t rrows;
  int32_t f64;       // source dtype (host-side grouping only)
  const int32_t* flag;  // null, or: run only when *flag != 0 (CholeskyQR2 fallback)
};

struct QRTaskTable {
  QRTask t[kMaxTasks];
};

// Offset of column j (< 64) of the mode unfolding of an (A, m, B) view: column j = a B + b
// starts at a m B + b and advances by B per row.  Each thread computes it once for its
// column; j < 64, so a 32-bit division does (and none when B > j).
__device__ __forceinline__ int64_t col_offset(int j, int64_t m, int64_t B) {
  const int a = (B > j) ? 0 : j / static_cast<int>(B);
  return static_cast<int64_t>(a) * m * B + (j - static_cast<int64_t>(a) * B);
}

template <typename TY>
__device__ __forceinline__ void small_qr_body(const QRTask& T) {
  __shared__ double Y[kRowsMax * kCols];
  __shared__ double sh_nrm[4];
  __shared__ double sh_dot[4][kCols];
  __shared__ double sh_vk[kCols];
  __shared__ double sh_beta[kCols];
  __shared__ double sh_sgn[kCols];

  const int lane = threadIdx.x % kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int rows = T.rows, n = T.n;
  const int c = rows < n ? rows : n;
  const TY* src = static_cast<const TY*>(T.src);

  // load (zero padded), coalesced along the source's contiguous index; a thread keeps one
  // column (kQRThreads is a multiple of kCols)
  static_assert(kQRThreads % kCols == 0, "one column per thread in the load");
  const int lj = static_cast<int>(threadIdx.x) % kCols;
  const TY* scol = src + col_offset(lj, T.m, T.B) + T.row0 * T.B;
  for (int idx = threadIdx.x; idx < kRowsMax * kCols; idx += kQRThreads) {
    const int r = idx / kCols, j = lj;
    double v = 0.0;
    if (r < rows && j < n) v = static_cast<double>(scol[r * T.B]);
    Y[r * kCols + j] = v;
  }
  __syncthreads();
  const int r_lo = w * 64, r_hi = (w * 64 + 64 < rows) ? w * 64 + 64 : rows;
  // norm partials of column 0
  if (lane == 0) {
    double s = 0.0;
    for (int r = r_lo; r < r_hi; ++r) s += Y[r * kCols] * Y[r * kCols];
    sh_nrm[w] = s;
  }
  __syncthreads();

  // ---------------- factorization
  for (int k = 0; k < c; ++k) {
    const double sigma = sh_nrm[0] + sh_nrm[1] + sh_nrm[2] + sh_nrm[3];
    const double xkk = Y[k * kCols + k];
    double alpha = 0.0, vk = 0.0, beta = 0.0;
    if (sigma > 0.0) {
      alpha = -copysign(sqrt(sigma), xkk);
      vk = xkk - alpha;
      beta = 1.0 / (sigma - alpha * xkk);
    }
    const int j = lane;
    const int rs = (k > r_lo) ? k : r_lo;
    // dot products w_j = v^T Y[:, j] over this wave's rows
    if (beta != 0.0 && j > k && j < n) {
      double p = 0.0;
      for (int r = rs; r < r_hi; ++r) {
        const double v = (r == k) ? vk : Y[r * kCols + k];
        p = fma(v, Y[r * kCols + j], p);
      }
      sh_dot[w][j] = p;
    }
    __syncthreads();
    if (beta != 0.0 && j > k && j < n) {
      const double wj = beta * (sh_dot[0][j] + sh_dot[1][j] + sh_dot[2][j] + sh_dot[3][j]);
      double s = 0.0;
      for (int r = rs; r < r_hi; ++r) {
        const double v = (r == k) ? vk : Y[r * kCols + k];
        const double y = fma(-wj, v, Y[r * kCols + j]);
        Y[r * kCols + j] = y;
        if (j == k + 1 && r >= k + 1) s = fma(y, y, s);
      }
      if (j == k + 1) sh_nrm[w] = s;
    } else if (j == k + 1 && j < n) {
      double s = 0.0;
      const int rs1 = (k + 1 > r_lo) ? k + 1 : r_lo;
      for (int r = rs1; r < r_hi; ++r) s = fma(Y[r * kCols + j], Y[r * kCols + j], s);
      sh_nrm[w] = s;
    }
    if (threadIdx.x == 0) {
      sh_vk[k] = vk;
      sh_beta[k] = beta;
      sh_sgn[k] = (alpha < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) Y[k * kCols + k] = alpha;  // R_kk; v_k kept in sh_vk
    __syncthreads();
  }

  // ---------------- write R (sign-normalised rows), then clear it from Y
  if (T.R) {
    for (int idx = threadIdx.x; idx < T.rrows * n; idx += kQRThreads) {
      const int i = idx / n, jj = idx % n;
      double v = 0.0;
      if (i < c && jj >= i) v = sh_sgn[i] * Y[i * kCols + jj];
      T.R[static_cast<int64_t>(i) * n + jj] = v;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kRowsMax * kCols; idx += kQRThreads) {
    const int r = idx / kCols, jj = idx % kCols;
    if (jj >= c || r <= jj) {
      if (!(jj < c && r == jj)) Y[idx] = 0.0;  // diagonal rewritten below
    }
  }
  __syncthreads();

  // ---------------- explicit Q in place: Q = H_0 ... H_{c-1} [I; 0]
  for (int k = c - 1; k >= 0; --k) {
    const double vk = sh_vk[k], beta = sh_beta[k];
    const int j = lane;
    const int rs = (k + 1 > r_lo) ? k + 1 : r_lo;
    if (j > k && j < c) {
      double p = 0.0;
      for (int r = rs; r < r_hi; ++r) p = fma(Y[r * kCols + k], Y[r * kCols + j], p);
      sh_dot[w][j] = p;
    }
    __syncthreads();
    if (j > k && j < c) {
      const double wj = beta * (sh_dot[0][j] + sh_dot[1][j] + sh_dot[2][j] + sh_dot[3][j]);
      for (int r = rs; r < r_hi; ++r) Y[r * kCols + j] = fma(-wj, Y[r * kCols + k], Y[r * kCols + j]);
      if (k >= r_lo && k < r_hi) Y[k * kCols + j] = -wj * vk;
    }
    __syncthreads();
    // column k = H_k e_k
    if (j == k) {
      for (int r = (k + 1 > r_lo ? k + 1 : r_lo); r < r_hi; ++r) Y[r * kCols + k] = -beta * vk * Y[r * kCols + k];
      if (k >= r_lo && k < r_hi) Y[k * kCols + k] = 1.0 - beta * vk * vk;
    }
    __syncthreads();
  }

  // ---------------- write Q (sign-normalised columns, zero beyond c)
  for (int idx = threadIdx.x; idx < rows * T.qcols; idx += kQRThreads) {
    const int r = idx / T.qcols, jj = idx % T.qcols;
    const double v = (jj < c) ? sh_sgn[jj] * Y[r * kCols + jj] : 0.0;
    T.Q[static_cast<int64_t>(r) * T.ldq + jj] = v;
  }
}

template <typename TY>
__global__ __launch_bounds__(kQRThreads) void small_qr_kernel(QRTaskTable tab) {
  const QRTask& T = tab.t[blockIdx.x];
  if (T.flag && *T.flag == 0) return;
  small_qr_body<TY>(T);
}

// one job per workgroup, jobs in device memory (batched decomposition)
template <typename TY>
__global__ __launch_bounds__(kQRThreads) void small_qr_grouped_kernel(const GQrJob* __restrict__ jobs) {
  const GQrJob J = jobs[blockIdx.x];
  if (J.flag && *J.flag == 0) return;
  QRTask T;
  T.src = J.Y;
  T.A = J.A;
  T.m = J.m;
  T.B = J.B;
  T.row0 = 0;
  T.rows = static_cast<int32_t>(J.m);
  T.n = J.n;
  T.Q = J.Q;
  T.ldq = J.qcols;
  T.qcols = J.qcols;
  T.R = nullptr;
  T.rrows = 0;
  T.f64 = 0;
  T.flag = nullptr;
  small_qr_body<TY>(T);
}

struct CombineTask {
  const double* Qb;  // rows x n (ld n)
  const double* Q2;  // n x n block (ld n)
  double* Q;         // rows x n (leading dimension ldq)
  int32_t rows, n, ldq;
  const int32_t* flag;
};
struct CombineTable {
  CombineTask t[kMaxTasks];
};

// Q[r][j] = sum_t Qb[r][t] Q2[t][j]
__global__ __launch_bounds__(256) void qr_combine_kernel(CombineTable tab) {
  const CombineTask& T = tab.t[blockIdx.y];
  if (T.flag && *T.flag == 0) return;
  const int64_t total = static_cast<int64_t>(T.rows) * T.n;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * 256) {
    const int r = static_cast<int>(idx / T.n), jj = static_cast<int>(idx % T.n);
    double s = 0.0;
    for (int t = 0; t < T.n; ++t) s = fma(T.Qb[static_cast<int64_t>(r) * T.n + t], T.Q2[static_cast<int64_t>(t) * T.n + jj], s);
    T.Q[static_cast<int64_t>(r) * T.ldq + jj] = s;
  }
}

// ------------------------------------------------------------------ CholeskyQR2
// Fast path for well-conditioned sketches: G = Y^T Y, Y = Q1 R1 (R1 = chol(G)),
// then the same on Q1, Q = Q1 R2^-1, R = R2 R1 (diag(R) > 0 by construction).
// Two passes restore orthogonality to rounding level when cond(Y) is below
// about 1e7.  A Cholesky pivot below 1e-13 of the largest diagonal entry flags
// the job, and the Householder path (launched conditionally) recomputes it.
constexpr int kGramRows = 64;

using CJob = GCholQRJob;
struct CJobTable {
  CJob t[kMaxQRJobs];
};
// job access for the by-value table of a single decomposition and for a job
// array in device memory (batched decomposition)
struct CTabVal {
  CJobTable v;
  __device__ const CJob& operator[](int i) const { return v.t[i]; }
};
struct CTabPtr {
  const CJob* p;
  __device__ const CJob& operator[](int i) const { return p[i]; }
};


// partial Gram of one 64-row chunk of Y (first pass); C (32 or 64) bounds the columns and
// thread (ty, tx) owns a (C / 16) x (C / 16) block of the C x C partial
template <typename TY, typename TAB, int C = kCols>
__global__ __launch_bounds__(256) void cq_gram_kernel(TAB tab) {
  constexpr int kO = C / 16;
  constexpr int kStep = 256 / C;  // rows between a thread's loads
  __shared__ double sy[kGramRows][C + 1];
  const CJob& J = tab[blockIdx.y];
  if (static_cast<int>(blockIdx.x) >= J.chunks) return;
  // the breakdown flag of the job starts cleared (every later kernel reads it)
  if (blockIdx.x == 0 && threadIdx.x == 0) *J.flag = 0;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kGramRows;
  // thread: column j of rows rr0 + kStep q; every load is issued before the first LDS store
  constexpr int kPer = kGramRows * C / 256;
  const int j = static_cast<int>(threadIdx.x) % C, rr0 = static_cast<int>(threadIdx.x) / C;
  const TY* ys = static_cast<const TY*>(J.Y) + col_offset(j, J.m, J.B);
  double yv[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int64_t r = r0 + rr0 + kStep * q;
    yv[q] = (r < J.m && j < J.n) ? static_cast<double>(ys[r * J.B]) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) sy[rr0 + kStep * q][j] = yv[q];
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[kO][kO] = {};
  for (int rr = 0; rr < kGramRows; ++rr) {
    double a[kO], b[kO];
#pragma unroll
    for (int u = 0; u < kO; ++u) { a[u] = sy[rr][ty * kO + u]; b[u] = sy[rr][tx * kO + u]; }
#pragma unroll
    for (int u = 0; u < kO; ++u)
#pragma unroll
      for (int v = 0; v < kO; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
  double* out = J.part + static_cast<int64_t>(blockIdx.x) * C * C;
#pragma unroll
  for (int u = 0; u < kO; ++u)
#pragma unroll
    for (int v = 0; v < kO; ++v) out[(ty * kO + u) * C + tx * kO + v] = acc[u][v];
}


// Sum the partial Grams (fixed order), factor G = R^T R (upper R) and form R^-1: the
// symmetric elimination on [G | I] turns the left block into R and the right block into
// R^-T.  W = NT / 64 waves (eight for one matrix per launch, measured 4 % faster than four; four
// in the batched launches, where many workgroups share the CUs); thread (wave w, lane j) keeps
// column j of rows C/W w .. C/W (w + 1) - 1 of both blocks in registers for the whole factorisation (C = 32: lanes 32 .. 63 hold no
// column and store nothing).  After each step the wave that
// owns the next pivot row stores all its C/W rows to LDS (static register indices; rows
// that are not being eliminated keep their values, so concurrent readers of the current
// row see the same bits), and a step touches LDS only for reads of that row.  Every wave keeps the diagonal in registers (lane j:
// G[j][j], updated with the same rounding as the matrix).  R goes to the first C^2
// doubles of the job's R1 / R2 buffer, R^-1 to the second.
template <typename TAB, int C = kCols, int NT = 256>
__global__ __launch_bounds__(NT) void cq_chol_kernel(TAB tab, int second) {
  constexpr int kW = NT / kWave;
  constexpr int kRows = C / kW;
  __shared__ __align__(16) double fullL[C][kWave];  // the rows of the owner of the next row
  __shared__ __align__(16) double fullR[C][kWave];
  __shared__ double Rs[C][C + 1];
  __shared__ double Xs[C][C + 1];
  const CJob& J = tab[blockIdx.x];
  if (*J.flag) return;  // cleared by cq_gram_kernel before the first pass
  const int n = J.n;
  const int lane = static_cast<int>(threadIdx.x) % kWave, wv = static_cast<int>(threadIdx.x) / kWave;
  const double* part = J.part + (second ? static_cast<int64_t>(J.chunks) * C * C : 0);
  double gl[kRows], gr[kRows];
#pragma unroll
  for (int t = 0; t < kRows; ++t) gl[t] = 0.0;
  // chunk partials in chunk order; the loads of two chunks are in flight together
#pragma unroll 2
  for (int c = 0; c < J.chunks; ++c) {
    const double* pc = part + static_cast<int64_t>(c) * C * C + kRows * wv * C + (lane < C ? lane : 0);
    double v[kRows];
#pragma unroll
    for (int t = 0; t < kRows; ++t) v[t] = lane < C ? pc[t * C] : 0.0;
#pragma unroll
    for (int t = 0; t < kRows; ++t) gl[t] += v[t];
  }
#pragma unroll
  for (int t = 0; t < kRows; ++t) gr[t] = (kRows * wv + t == lane) ? 1.0 : 0.0;
  for (int idx = threadIdx.x; idx < C * (C + 1); idx += NT) {
    (&Rs[0][0])[idx] = 0.0;
    (&Xs[0][0])[idx] = 0.0;
  }
#pragma unroll
  for (int t = 0; t < kRows; ++t) {
    fullL[kRows * wv + t][lane] = gl[t];
    fullR[kRows * wv + t][lane] = gr[t];
  }
  __syncthreads();
  const double shift = second ? J.shift2 : J.shift1;
  if (shift > 0.0) {
    // shifted Cholesky QR: factor G + s I, s = shift * trace(G).  Its pivots are at least
    // s, so it cannot break down, and Y R^-1 spans the columns of Y with a condition
    // number of order 1 / sqrt(shift) at worst (Fukaya et al., SIAM J. Sci. Comput. 2020)
    double tr = (lane < n) ? fullL[lane][lane] : 0.0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) tr += __shfl_xor(tr, off);  // same bits in every lane
    const double sh = shift * tr;
    __syncthreads();  // every wave has read the diagonal
#pragma unroll
    for (int t = 0; t < kRows; ++t)
      if (kRows * wv + t == lane && lane < n) {
        gl[t] += sh;
        fullL[lane][lane] = gl[t];
      }
    __syncthreads();
  }
  double dj = (lane < n) ? fullL[lane][lane] : 0.0;
  double dmax = dj;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  bool broke = false;
  // the loop is unrolled over k, so the owner of the next pivot row stores that row alone
  // (its register slot is static), and the other steps' stores are skipped
#pragma clang loop unroll(full)
  for (int k = 0; k < C; ++k) {
    if (k >= n || broke) continue;  // uniform
    const double lk = fullL[k][lane], rk = fullR[k][lane];
    double li[kRows];
#pragma unroll
    for (int t = 0; t < kRows; t += 2) {
      const double2 q = *reinterpret_cast<const double2*>(&fullL[k][kRows * wv + t]);
      li[t] = q.x;
      li[t + 1] = q.y;
    }
    const double d = __longlong_as_double(
        (static_cast<long long>(__builtin_amdgcn_readlane(static_cast<int>(__double_as_longlong(dj) >> 32), k)) << 32) |
        static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(__double_as_longlong(dj) & 0xffffffff), k)));
    if (!(d > 1e-13 * dmax) || !(dmax > 0.0)) {  // uniform: every lane holds the same d
      broke = true;
      continue;
    }
    const double inv_s = rsq_refined(d);
    const double lj = lk * inv_s, xj = rk * inv_s;
    if (wv == 0 && lane < n) {
      if (lane >= k) Rs[k][lane] = lj;  // lane == k: d / sqrt(d)
      Xs[lane][k] = xj;
    }
    // every row is updated: rows up to k are final (R and R^-1 took them at their own
    // step) and are never read again, so no per-row test is needed
#pragma unroll
    for (int t = 0; t < kRows; ++t) {
      const double mult = li[t] * inv_s;
      gl[t] = fma(-mult, lj, gl[t]);
      gr[t] = fma(-mult, xj, gr[t]);
    }
    if (lane > k) dj = fma(-lj, lj, dj);
    if (k + 1 < n && wv == (k + 1) / kRows) {
      fullL[k + 1][lane] = gl[(k + 1) % kRows];
      fullR[k + 1][lane] = gr[(k + 1) % kRows];
    }
    __syncthreads();
  }
  if (broke) {
    if (threadIdx.x == 0) *J.flag = 1;
    return;
  }
  double* R = second ? J.R2 : J.R1;
  for (int idx = threadIdx.x; idx < C * C; idx += NT) {
    const int i = idx / C, j = idx % C;
    const bool in = i < n && j < n && j >= i;
    R[idx] = in ? Rs[i][j] : 0.0;
    R[C * C + idx] = in ? Xs[i][j] : 0.0;
  }
  if (second && J.Rout) {
    // R = R2 R1 with R1 staged in LDS (the inverse array is free now)
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * C; idx += NT) Xs[idx / C][idx % C] = J.R1[idx];
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * n; idx += NT) {
      const int i = idx / n, j = idx % n;
      double s0 = 0.0, s1 = 0.0;
      int t = i;
      for (; t + 1 <= j; t += 2) {
        s0 = fma(Rs[i][t], Xs[t][j], s0);
        s1 = fma(Rs[i][t + 1], Xs[t + 1][j], s1);
      }
      if (t <= j) s0 = fma(Rs[i][t], Xs[t][j], s0);
      J.Rout[idx] = (j >= i) ? s0 + s1 : 0.0;
    }
  }
}

// 64 rows of Q = Y R^-1 per workgroup as a product with the explicit inverse from
// cq_chol_kernel (4 x C/16 outputs per thread); the first pass also stores Q1 and the
// partial Gram of its rows
template <typename TY, typename TAB, int C = kCols>
__global__ __launch_bounds__(256) void cq_apply_kernel(TAB tab, int second) {
  constexpr int kS = C + 2;  // even row stride keeps the double2 reads aligned
  constexpr int kO = C / 16;
  constexpr int kStep = 256 / C;
  __shared__ __align__(16) double sy[kGramRows][kS];
  __shared__ __align__(16) double sx[C][kS];
  const CJob& J = tab[blockIdx.y];
  if (static_cast<int>(blockIdx.x) >= J.chunks) return;
  if (*J.flag) return;
  const int n = J.n;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kGramRows;
  const double* Xg = (second ? J.R2 : J.R1) + C * C;
  {
    // thread: column j of rows rr0 + kStep q (of the Y chunk, and of R^-1 for rows below
    // C); every load is issued before the first LDS store
    constexpr int kPer = kGramRows * C / 256;
    constexpr int kPerX = C * C / 256;
    const int j = static_cast<int>(threadIdx.x) % C, rr0 = static_cast<int>(threadIdx.x) / C;
    const TY* ys = static_cast<const TY*>(J.Y) + col_offset(j, J.m, J.B);
    double yv[kPer], xv[kPerX];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int64_t r = r0 + rr0 + kStep * q;
      double v = 0.0;
      if (r < J.m && j < n) v = second ? J.Q1[r * n + j] : static_cast<double>(ys[r * J.B]);
      yv[q] = v;
    }
#pragma unroll
    for (int q = 0; q < kPerX; ++q) xv[q] = Xg[(rr0 + kStep * q) * C + j];
#pragma unroll
    for (int q = 0; q < kPer; ++q) sy[rr0 + kStep * q][j] = yv[q];
#pragma unroll
    for (int q = 0; q < kPerX; ++q) sx[rr0 + kStep * q][j] = xv[q];
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  {
    double acc[4][kO] = {};
#pragma unroll 4
    for (int t = 0; t < n; ++t) {
      double a[4], b[kO];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = sy[ty * 4 + u][t];
#pragma unroll
      for (int v = 0; v < kO; v += 2) {
        const double2 bv = *reinterpret_cast<const double2*>(&sx[t][tx * kO + v]);
        b[v] = bv.x;
        b[v + 1] = bv.y;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < kO; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < kO; ++v) sy[ty * 4 + u][tx * kO + v] = acc[u][v];
  }
  __syncthreads();
  double* out = second ? J.Q : J.Q1;
  for (int idx = threadIdx.x; idx < kGramRows * C; idx += 256) {
    const int rr = idx / C, j = idx % C;
    const int64_t r = r0 + rr;
    if (r < J.m && j < n) out[r * n + j] = sy[rr][j];
  }
  if (second) return;
  // partial Gram of these Q1 rows for the second pass (rows past m and columns past n
  // are zero: the inputs there were zero)
  double g[kO][kO] = {};
#pragma unroll 4
  for (int rr = 0; rr < kGramRows; ++rr) {
    double a[kO], b[kO];
#pragma unroll
    for (int v = 0; v < kO; v += 2) {
      const double2 av = *reinterpret_cast<const double2*>(&sy[rr][ty * kO + v]);
      const double2 bv = *reinterpret_cast<const double2*>(&sy[rr][tx * kO + v]);
      a[v] = av.x;
      a[v + 1] = av.y;
      b[v] = bv.x;
      b[v + 1] = bv.y;
    }
#pragma unroll
    for (int u = 0; u < kO; ++u)
#pragma unroll
      for (int v = 0; v < kO; ++v) g[u][v] = fma(a[u], b[v], g[u][v]);
  }
  double* gp = J.part + (static_cast<int64_t>(J.chunks) + blockIdx.x) * C * C;
#pragma unroll
  for (int u = 0; u < kO; ++u)
#pragma unroll
    for (int v = 0; v < kO; ++v) gp[(ty * kO + u) * C + tx * kO + v] = g[u][v];
}


// One matrix of the (recursive) TSQR plan.
struct Mat {
  const void* src;
  bool f64;
  int64_t A, m, B;
  int n;
  double* Q;  // m x qcols (ld ldq)
  int ldq, qcols;
  double* R;  // rrows x n or null
  int rrows;
  const int32_t* flag;
};

struct Bump {
  char* base;
  size_t off;
  void* take(size_t bytes) {
    const size_t o = align256(off);
    off = o + align256(bytes);
    return base ? base + o : nullptr;
  }
};

// Plans (and, when launch is true, enqueues) the QR of a set of matrices.
hipError_t qr_level(std::vector<Mat>& mats, bool launch, Bump& ws, hipStream_t st) {
  std::vector<QRTask> direct;
  std::vector<Mat> upper;               // stacked-R matrices of the next level
  std::vector<CombineTask> combine;     // filled after the upper level is planned
  struct Pending { Mat mat; double* Qb; double* Rs; int nb; };
  std::vector<Pending> pend;
  for (const Mat& M : mats) {
    if (M.m <= kRowsMax) {
      QRTask t;
      t.src = M.src; t.A = M.A; t.m = M.m; t.B = M.B; t.row0 = 0; t.rows = static_cast<int32_t>(M.m);
      t.n = M.n; t.Q = M.Q; t.ldq = M.ldq; t.qcols = M.qcols; t.R = M.R; t.rrows = M.rrows;
      t.f64 = M.f64 ? 1 : 0;
      t.flag = M.flag;
      direct.push_back(t);
    } else {
      const int nb = static_cast<int>(ceil_div(M.m, kRowsMax));
      Pending p;
      p.mat = M;
      p.nb = nb;
      p.Qb = static_cast<double*>(ws.take(static_cast<size_t>(M.m) * M.n * sizeof(double)));
      p.Rs = static_cast<double*>(ws.take(static_cast<size_t>(nb) * M.n * M.n * sizeof(double)));
      for (int b = 0; b < nb; ++b) {
        QRTask t;
        t.src = M.src; t.A = M.A; t.m = M.m; t.B = M.B; t.row0 = static_cast<int64_t>(b) * kRowsMax;
        const int64_t left = M.m - t.row0;
        t.rows = static_cast<int32_t>(left < kRowsMax ? left : kRowsMax);
        t.n = M.n;
        t.Q = p.Qb ? p.Qb + t.row0 * M.n : nullptr;
        t.ldq = M.n; t.qcols = M.n;
        t.R = p.Rs ? p.Rs + static_cast<int64_t>(b) * M.n * M.n : nullptr;
        t.rrows = M.n;
        t.f64 = M.f64 ? 1 : 0;
        t.flag = M.flag;
        direct.push_back(t);
      }
      pend.push_back(p);
    }
  }
  // launch this level's block factorizations (grouped by input dtype)
  if (launch) {
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<QRTask> sel;
      for (size_t i = 0; i < direct.size(); ++i)
        if ((pass == 1) == (direct[i].f64 != 0)) sel.push_back(direct[i]);
      for (size_t i0 = 0; i0 < sel.size(); i0 += kMaxTasks) {
        QRTaskTable tab;
        const size_t cnt = (sel.size() - i0 < static_cast<size_t>(kMaxTasks)) ? sel.size() - i0 : kMaxTasks;
        for (size_t i = 0; i < cnt; ++i) tab.t[i] = sel[i0 + i];
        if (pass == 1)
          small_qr_kernel<double><<<static_cast<unsigned>(cnt), kQRThreads, 0, st>>>(tab);
        else
          small_qr_kernel<float><<<static_cast<unsigned>(cnt), kQRThreads, 0, st>>>(tab);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
  }
  if (pend.empty()) return hipSuccess;
  // next level: QR of the stacked R factors, then Q = blockdiag(Qb) * Q2
  std::vector<double*> q2(pend.size());
  for (size_t i = 0; i < pend.size(); ++i) {
    const Pending& p = pend[i];
    Mat U;
    U.src = p.Rs; U.f64 = true; U.A = 1; U.m = static_cast<int64_t>(p.nb) * p.mat.n; U.B = p.mat.n;
    U.n = p.mat.n;
    q2[i] = static_cast<double*>(ws.take(static_cast<size_t>(U.m) * U.n * sizeof(double)));
    U.Q = q2[i]; U.ldq = U.n; U.qcols = U.n;
    U.R = p.mat.R; U.rrows = p.mat.rrows;
    U.flag = p.mat.flag;
    upper.push_back(U);
  }
  hipError_t e = qr_level(upper, launch, ws, st);
  if (e != hipSuccess) return e;
  for (size_t i = 0; i < pend.size(); ++i) {
    const Pending& p = pend[i];
    for (int b = 0; b < p.nb; ++b) {
      CombineTask t;
      const int64_t row0 = static_cast<int64_t>(b) * kRowsMax;
      const int64_t left = p.mat.m - row0;
      t.rows = static_cast<int32_t>(left < kRowsMax ? left : kRowsMax);
      t.n = p.mat.n;
      t.Qb = p.Qb ? p.Qb + row0 * p.mat.n : nullptr;
      t.Q2 = q2[i] ? q2[i] + static_cast<int64_t>(b) * p.mat.n * p.mat.n : nullptr;
      t.Q = p.mat.Q ? p.mat.Q + row0 * p.mat.ldq : nullptr;
      t.ldq = p.mat.ldq;
      t.flag = p.mat.flag;
      combine.push_back(t);
    }
  }
  if (launch) {
    for (size_t i0 = 0; i0 < combine.size(); i0 += kMaxTasks) {
      CombineTable tab;
      const size_t cnt = (combine.size() - i0 < static_cast<size_t>(kMaxTasks)) ? combine.size() - i0 : kMaxTasks;
      for (size_t i = 0; i < cnt; ++i) tab.t[i] = combine[i0 + i];
      qr_combine_kernel<<<dim3(64, static_cast<unsigned>(cnt)), 256, 0, st>>>(tab);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// Plans (and, when launch is true, enqueues) the QR of a set of jobs:
// CholeskyQR2 with a Householder fallback for m >= n, Householder otherwise.
hipError_t qr_plan(const QRJob* jobs, int count, rt_dtype ydt, bool launch, Bump& ws, hipStream_t st,
                   double shift = 0.0) {
  std::vector<Mat> hh;
  CJobTable tab;
  int nc = 0;
  int max_chunks = 1;
  int64_t max_m = 1;
  for (int i = 0; i < count; ++i) {
    Mat M;
    M.src = jobs[i].Y; M.f64 = (ydt == RT_F64);
    M.A = jobs[i].A; M.m = jobs[i].m; M.B = jobs[i].B;
    M.n = static_cast<int>(jobs[i].A * jobs[i].B);
    const int c = static_cast<int>(M.m < M.n ? M.m : M.n);
    M.Q = jobs[i].Q; M.ldq = c; M.qcols = c;
    M.R = jobs[i].R; M.rrows = c;
    M.flag = nullptr;
    if (M.m >= M.n && nc < kMaxQRJobs) {
      CJob J;
      J.Y = M.src; J.A = M.A; J.m = M.m; J.B = M.B; J.n = M.n;
      J.chunks = static_cast<int32_t>(ceil_div(M.m, kGramRows));
      J.part = static_cast<double*>(ws.take(2 * static_cast<size_t>(J.chunks) * kCols * kCols * sizeof(double)));
      J.R1 = static_cast<double*>(ws.take(2 * kCols * kCols * sizeof(double)));  // R1, then R1^-1
      J.R2 = static_cast<double*>(ws.take(2 * kCols * kCols * sizeof(double)));  // R2, then R2^-1
      J.Q1 = static_cast<double*>(ws.take(static_cast<size_t>(M.m) * M.n * sizeof(double)));
      J.flag = static_cast<int32_t*>(ws.take(sizeof(int32_t)));
      J.Q = M.Q; J.Rout = M.R;
      J.shift1 = J.shift2 = shift;
      M.flag = J.flag;
      tab.t[nc++] = J;
      if (J.chunks > max_chunks) max_chunks = J.chunks;
      if (M.m > max_m) max_m = M.m;
    }
    hh.push_back(M);
  }
  if (launch && nc > 0) {
    const dim3 g1(max_chunks, nc);
    (void)max_m;
    const CTabVal tv{tab};
    if (ydt == RT_F64) {
      cq_gram_kernel<double><<<g1, 256, 0, st>>>(tv);
      cq_chol_kernel<CTabVal, kCols, 512><<<nc, 512, 0, st>>>(tv, 0);
      cq_apply_kernel<double><<<g1, 256, 0, st>>>(tv, 0);
    } else {
      cq_gram_kernel<float><<<g1, 256, 0, st>>>(tv);
      cq_chol_kernel<CTabVal, kCols, 512><<<nc, 512, 0, st>>>(tv, 0);
      cq_apply_kernel<float><<<g1, 256, 0, st>>>(tv, 0);
    }
    cq_chol_kernel<CTabVal, kCols, 512><<<nc, 512, 0, st>>>(tv, 1);
    cq_apply_kernel<double><<<g1, 256, 0, st>>>(tv, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return qr_level(hh, launch, ws, st);
}

}  // namespace

size_t qr_ws(const QRJob* jobs, int count) {
  Bump b{nullptr, 0};
  (void)qr_plan(jobs, count, RT_F32, false, b, nullptr);
  return align256(b.off);
}

hipError_t launch_qr(const QRJob* jobs, int count, rt_dtype ydt, void* ws, hipStream_t st) {
  Bump b{static_cast<char*>(ws), 0};
  return qr_plan(jobs, count, ydt, true, b, st);
}

size_t orth_ws(int64_t m, int n) {
  const QRJob job{nullptr, 1, m, n, nullptr, nullptr};
  return qr_ws(&job, 1);
}

hipError_t launch_orth(const double* Y, int64_t m, int n, double* T, double* Q, void* ws, hipStream_t st) {
  // shift factor 11 (m n + n (n + 1)) u of shifted Cholesky QR, applied to trace(G) >= ||Y||_2^2
  const double shift = 11.0 * (static_cast<double>(m) * n + static_cast<double>(n) * (n + 1)) * 0x1p-53;
  const QRJob pre{Y, 1, m, n, T, nullptr};
  Bump b{static_cast<char*>(ws), 0};
  hipError_t e = qr_plan(&pre, 1, RT_F64, true, b, st, shift);
  if (e != hipSuccess) return e;
  const QRJob fin{T, 1, m, n, Q, nullptr};
  Bump b2{static_cast<char*>(ws), 0};
  return qr_plan(&fin, 1, RT_F64, true, b2, st);
}

hipError_t launch_qr_grouped(const GQrJob* jobs, int count, rt_dtype ydt, hipStream_t st) {
  if (count == 0) return hipSuccess;
  if (ydt == RT_F64)
    small_qr_grouped_kernel<double><<<static_cast<unsigned>(count), kQRThreads, 0, st>>>(jobs);
  else
    small_qr_grouped_kernel<float><<<static_cast<unsigned>(count), kQRThreads, 0, st>>>(jobs);
  return hipGetLastError();
}

namespace {
template <int C>
void cholqr2_grouped(const CTabPtr tp, int count, int max_chunks, rt_dtype ydt, hipStream_t st) {
  const dim3 g1(static_cast<unsigned>(max_chunks), static_cast<unsigned>(count));
  if (ydt == RT_F64) {
    cq_gram_kernel<double, CTabPtr, C><<<g1, 256, 0, st>>>(tp);
    cq_chol_kernel<CTabPtr, C><<<count, 256, 0, st>>>(tp, 0);
    cq_apply_kernel<double, CTabPtr, C><<<g1, 256, 0, st>>>(tp, 0);
  } else {
    cq_gram_kernel<float, CTabPtr, C><<<g1, 256, 0, st>>>(tp);
    cq_chol_kernel<CTabPtr, C><<<count, 256, 0, st>>>(tp, 0);
    cq_apply_kernel<float, CTabPtr, C><<<g1, 256, 0, st>>>(tp, 0);
  }
  cq_chol_kernel<CTabPtr, C><<<count, 256, 0, st>>>(tp, 1);
  cq_apply_kernel<double, CTabPtr, C><<<g1, 256, 0, st>>>(tp, 1);
}
}  // namespace

hipError_t launch_cholqr2_grouped(const GCholQRJob* jobs, int count, int max_chunks, rt_dtype ydt, hipStream_t st,
                                  int cols) {
  if (count == 0) return hipSuccess;
  if (cols != 32 && cols != 64) return hipErrorInvalidValue;
  const CTabPtr tp{jobs};
  if (cols == 32)
    cholqr2_grouped<32>(tp, count, max_chunks, ydt, st);
  else
    cholqr2_grouped<64>(tp, count, max_chunks, ydt, st);
  return hipGetLastError();
}

}  // namespace rt

// Core truncation pieces (Alg. 2.2 applied to the small core, Sec. 4.1):
//  * mode contraction out = P_(n) Q_(n)^T on (A, m, B) views, which gives the
//    Gram matrix G_(j) G_(j)^T of the core (P = Q) and the adjoint dA_n;
//    fixed-order two-stage reduction, so results are bitwise reproducible;
//  * a symmetric eigensolver for the <= 64 x 64 Gram matrices, binary64, one
//    workgroup: Householder tridiagonalisation + multisection + inverse iteration
//    for up to 32 leading pairs, with one-sided Jacobi on a pivoted Cholesky factor
//    as the fallback (clusters, numerically zero eigenvalues, r > 32);
//  * the small binary64 products U_j = U_hat_j V_j of all modes in one launch.
#include "kernels.hpp"

namespace rt {

namespace {

// ------------------------------------------------------------------ mode contraction
constexpr int kMCTile = 64;
constexpr int kMCK = 16;
constexpr int kMCThreads = 256;

// one 64 x 64 output tile (rows i0.., columns j0..) summed over t in [t0, t1);
// thread (ty, tx) accumulates rows 4 ty.., columns 4 tx..  The operands of the next
// 16 t are loaded into registers while the current 16 are multiplied from LDS.
// (TIn: the operands' type, widened to T on load; T: LDS staging and accumulation)
template <typename T, typename TIn = T>
__device__ __forceinline__ void mode_contract_tile(const TIn* __restrict__ P, const TIn* __restrict__ Q, int64_t A,
                                                   int64_t mP, int64_t mQ, int64_t B, int64_t t0, int64_t t1,
                                                   int64_t i0, int64_t j0, T (&acc)[4][4]) {
  __shared__ T sP[kMCK][kMCTile + 1];
  __shared__ T sQ[kMCK][kMCTile + 1];
  (void)A;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;  // 4x4 outputs per thread
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
  // loading roles: each thread loads four (tt, ii) elements per 16 t, following memory
  // order: t fastest when rows of b are long (tt = lt, ii = li + 16 rep), the mode
  // index fastest otherwise (tt = lt + 4 rep, ii = li)
  const bool tfast = B >= kMCK;
  int lt, li;
  if (tfast) { lt = threadIdx.x % kMCK; li = threadIdx.x / kMCK; } else { li = threadIdx.x % kMCTile; lt = threadIdx.x / kMCTile; }
  // incremental (a, b) of this thread's first t, no division inside the loop
  int64_t ta = (t0 + lt) / B, tb = (t0 + lt) - ((t0 + lt) / B) * B;
  T pv[4], qv[4];
  auto load16 = [&](int64_t tbase) {
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int dt = tfast ? 0 : 4 * rep;
      const int ii = tfast ? li + 16 * rep : li;
      int64_t a = ta, b = tb + dt;
      while (b >= B) { b -= B; ++a; }
      const bool in = tbase + lt + dt < t1;
      pv[rep] = (in && i0 + ii < mP) ? static_cast<T>(P[a * mP * B + (i0 + ii) * B + b]) : T(0);
      qv[rep] = (in && j0 + ii < mQ) ? static_cast<T>(Q[a * mQ * B + (j0 + ii) * B + b]) : T(0);
    }
    tb += kMCK;
    while (tb >= B) { tb -= B; ++ta; }
  };
  load16(t0);
  for (int64_t tbase = t0; tbase < t1; tbase += kMCK) {
    __syncthreads();
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      const int tt = tfast ? lt : lt + 4 * rep;
      const int ii = tfast ? li + 16 * rep : li;
      sP[tt][ii] = pv[rep];
      sQ[tt][ii] = qv[rep];
    }
    __syncthreads();
    if (tbase + kMCK < t1) load16(tbase + kMCK);
#pragma unroll 4
    for (int tt = 0; tt < kMCK; ++tt) {
      T pr[4], qr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pr[u] = sP[tt][ty * 4 + u];
#pragma unroll
      for (int v = 0; v < 4; ++v) qr[v] = sQ[tt][tx * 4 + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(pr[u], qr[v], acc[u][v]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kMCThreads) void mode_contract_kernel(const T* __restrict__ P, const T* __restrict__ Q,
                                                                   int64_t A, int64_t mP, int64_t mQ, int64_t B,
                                                                   int64_t chunk, int tilesQ, T* __restrict__ part) {
  const int tile = blockIdx.x;
  const int ti = tile / tilesQ, tj = tile % tilesQ;
  const int64_t i0 = static_cast<int64_t>(ti) * kMCTile, j0 = static_cast<int64_t>(tj) * kMCTile;
  const int64_t total = A * B;
  const int64_t t0 = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t t1 = (t0 + chunk < total) ? t0 + chunk : total;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  T acc[4][4];
  mode_contract_tile<T>(P, Q, A, mP, mQ, B, t0, t1, i0, j0, acc);
  T* out = part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + tile) * kMCTile * kMCTile;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(ty * 4 + u) * kMCTile + tx * 4 + v] = acc[u][v];
}

// Gram matrix X_(n) X_(n)^T of a binary32 (A, m, B) view, accumulated in binary64 (the
// deterministic STHOSVD: a binary32 Gram matrix would bury the trailing eigenvalues, whose
// share of ||X||^2 is the squared error, under its rounding).  64 x 64 output tiles on or
// above the diagonal only (the reduction mirrors them), each summed over one chunk of t;
// binary64 16x16x4 matrix-core products of the widened (exact) binary32 values.
//  * operands stay binary32 in LDS (half the footprint: four workgroups per CU) and are
//    widened as they are read;
//  * the next 64 t are fetched into registers while the current 64 are multiplied;
//  * workgroups are numbered so that all tiles of one chunk run on one XCD (the hardware
//    deals consecutive workgroups round-robin to the eight XCDs), so each XCD's L2 holds
//    the rows its tiles share and X streams from HBM about once.
typedef double mc_f64x4 __attribute__((ext_vector_type(4)));
typedef float mc_f32x4v __attribute__((ext_vector_type(4)));
constexpr int kGWT = 64;                // t staged per round
constexpr int kGWStride = kGWT + 4;     // floats per LDS row: 16-byte rows, conflict-free column reads
constexpr int kXcds = 8;
// operand loads: kGWVec, 16-byte groups along t (B % 4 == 0, X 16-byte aligned; chunks are
// multiples of 64, so every group of four lies in one (a, b) row); kGWTFast, element loads with
// the lanes along t (B >= 64: a round crosses at most one row boundary); kGWRowFast,
// element loads with the lanes along the mode index (short rows, e.g. B = 1)
enum GWLoad { kGWVec = 0, kGWTFast = 1, kGWRowFast = 2 };
template <int LOAD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gram_wide_kernel(
    const float* __restrict__ X, int64_t A, int64_t m, int64_t B, int64_t chunk, int tiles1, int upper, int64_t work,
    double* __restrict__ part) {
  __shared__ __align__(16) float sP[kMCTile * kGWStride];
  __shared__ __align__(16) float sQ[kMCTile * kGWStride];
  // XCD-aware numbering: hardware workgroup h runs on XCD h % 8; logical id = XCD-major
  const int64_t per = static_cast<int64_t>(gridDim.x) / kXcds;
  const int64_t logical = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  if (logical >= work) return;
  const int c = static_cast<int>(logical / upper);
  int rem = static_cast<int>(logical % upper), ti = 0;
  while (rem >= tiles1 - ti) {  // row-major enumeration of the upper tiles
    rem -= tiles1 - ti;
    ++ti;
  }
  const int tj = ti + rem;
  const bool diag = ti == tj;  // P and Q blocks coincide: stage one
  const int64_t i0 = static_cast<int64_t>(ti) * kMCTile, j0 = static_cast<int64_t>(tj) * kMCTile;
  const int64_t total = A * B;
  const int64_t t0 = static_cast<int64_t>(c) * chunk;
  const int64_t t1 = (t0 + chunk < total) ? t0 + chunk : total;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int r16 = lane % 16, q = lane / 16;
  const int64_t nP = (m - i0 < kMCTile) ? m - i0 : kMCTile;
  const int64_t nQ = (m - j0 < kMCTile) ? m - j0 : kMCTile;
  const float* sQr = diag ? sP : sQ;
  mc_f64x4 acc[4];
#pragma unroll
  for (int js = 0; js < 4; ++js) acc[js] = mc_f64x4{0.0, 0.0, 0.0, 0.0};
  const int vt = 4 * (threadIdx.x % 16), vr = threadIdx.x / 16;  // kGWVec roles
  const int lt = threadIdx.x % kWave, lr = threadIdx.x / kWave;    // kGWTFast roles
  const int li = threadIdx.x % kMCTile, lq = threadIdx.x / kMCTile; // kGWRowFast roles
  mc_f32x4v pv[4], qv[4];
  auto fetch = [&](int64_t tb) {
    if constexpr (LOAD == kGWVec) {
      // thread -> rows tid / 16 + 16 rep, t 4 (tid % 16) .. + 3; tb and B are multiples
      // of 4, so a group of four never straddles a row boundary (a round may)
      const int64_t t = tb + vt;
      const bool tin = t < t1;
      const int64_t a = tin ? t / B : 0, b = tin ? t - (t / B) * B : 0;
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        const int ii = vr + 16 * rep;
        pv[rep] = (tin && ii < nP) ? *reinterpret_cast<const mc_f32x4v*>(X + a * m * B + (i0 + ii) * B + b)
                                   : mc_f32x4v{0.f, 0.f, 0.f, 0.f};
        qv[rep] = (tin && !diag && ii < nQ) ? *reinterpret_cast<const mc_f32x4v*>(X + a * m * B + (j0 + ii) * B + b)
                                            : mc_f32x4v{0.f, 0.f, 0.f, 0.f};
      }
    } else if constexpr (LOAD == kGWTFast) {
      // thread -> t = tb + tid % 64, rows tid / 64 + 4 k (a wave reads 64 consecutive t of a row)
      int64_t a = tb / B, b = tb - (tb / B) * B + lt;
      if (b >= B) {
        b -= B;
        ++a;
      }
      const bool tin = tb + lt < t1;
      // row ii = lr + 4 k: the lane's address advances by the uniform 4 B per k
      const float* pp = X + a * m * B + (i0 + lr) * B + b;
      const float* qp = X + a * m * B + (j0 + lr) * B + b;
      const int64_t step = 4 * B;
#pragma unroll
      for (int rep = 0; rep < 4; ++rep)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ii = lr + 4 * (4 * rep + e);
          pv[rep][e] = (tin && ii < nP) ? *pp : 0.f;
          qv[rep][e] = (tin && !diag && ii < nQ) ? *qp : 0.f;
          pp += step;
          qp += step;
        }
    } else {
      // thread -> row tid % 64, t = tb + tid / 64 + 4 k
#pragma unroll
      for (int rep = 0; rep < 4; ++rep)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t t = tb + lq + 4 * (4 * rep + e);
          const bool tin = t < t1;
          const int64_t a = tin ? t / B : 0, b = tin ? t - (t / B) * B : 0;
          pv[rep][e] = (tin && li < nP) ? X[a * m * B + (i0 + li) * B + b] : 0.f;
          qv[rep][e] = (tin && !diag && li < nQ) ? X[a * m * B + (j0 + li) * B + b] : 0.f;
        }
    }
  };
  auto stage = [&]() {
    if constexpr (LOAD == kGWVec) {
#pragma unroll
      for (int rep = 0; rep < 4; ++rep) {
        const int ii = vr + 16 * rep;
        *reinterpret_cast<mc_f32x4v*>(sP + ii * kGWStride + vt) = pv[rep];
        if (!diag) *reinterpret_cast<mc_f32x4v*>(sQ + ii * kGWStride + vt) = qv[rep];
      }
    } else if constexpr (LOAD == kGWTFast) {
#pragma unroll
      for (int rep = 0; rep < 4; ++rep)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ii = lr + 4 * (4 * rep + e);
          sP[ii * kGWStride + lt] = pv[rep][e];
          if (!diag) sQ[ii * kGWStride + lt] = qv[rep][e];
        }
    } else {
#pragma unroll
      for (int rep = 0; rep < 4; ++rep)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int tt = lq + 4 * (4 * rep + e);
          sP[li * kGWStride + tt] = pv[rep][e];
          if (!diag) sQ[li * kGWStride + tt] = qv[rep][e];
        }
    }
  };
  fetch(t0);
  for (int64_t tb = t0; tb < t1; tb += kGWT) {
    __syncthreads();
    stage();
    __syncthreads();
    if (tb + kGWT < t1) fetch(tb + kGWT);
    // every wave multiplies all four column tiles: rows past the matrix are zero in LDS,
    // so their products vanish, and the loop stays branch-free
#pragma unroll 4
    for (int k0 = 0; k0 < kGWT; k0 += 4) {
      const double av = static_cast<double>(sP[(16 * wave + r16) * kGWStride + k0 + q]);
#pragma unroll
      for (int js = 0; js < 4; ++js) {
        const double bv = static_cast<double>(sQr[(16 * js + r16) * kGWStride + k0 + q]);
        acc[js] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[js], 0, 0, 0);
      }
    }
  }
  if (16 * wave >= nP) return;
  // binary64 16x16x4 result layout: value v of lane (r16, q) is row q + 4 v, column r16
  double* out = part + (static_cast<int64_t>(c) * tiles1 * tiles1 + ti * tiles1 + tj) * kMCTile * kMCTile;
  const int njt = static_cast<int>((nQ + 15) / 16);
#pragma unroll
  for (int js = 0; js < 4; ++js)
    if (js < njt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(16 * wave + q + 4 * v) * kMCTile + 16 * js + r16] = acc[js][v];
    }
}

// out[i][j] (m x m) = sum over chunks of the upper tiles' partials, (i, j) below the diagonal
// tile read transposed from tile (j, i); 16 lanes per element, fixed order
__global__ __launch_bounds__(256) void gram_wide_reduce(const double* __restrict__ part, int nchunks, int tiles1,
                                                        int64_t m, double* __restrict__ out) {
  const int64_t total = m * m;
  const int sub = threadIdx.x % 16;
  const int64_t idx = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / 16;
  const bool valid = idx < total;
  double s = 0.0;
  if (valid) {
    int64_t i = idx / m, j = idx - (idx / m) * m;
    if (i / kMCTile > j / kMCTile) {
      const int64_t t = i;
      i = j;
      j = t;
    }
    const int tile = static_cast<int>((i / kMCTile) * tiles1 + (j / kMCTile));
    const int64_t off = (i % kMCTile) * kMCTile + (j % kMCTile);
    const int tiles = tiles1 * tiles1;
    for (int c = sub; c < nchunks; c += 16) s += part[(static_cast<int64_t>(c) * tiles + tile) * kMCTile * kMCTile + off];
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, 16);
  if (valid && sub == 0) out[idx] = s;
}

// Gram matrix of one binary64 (A, m, B) view per workgroup (m <= 64), batched
__global__ __launch_bounds__(kMCThreads) void gram_grouped_kernel(const GGramJob* __restrict__ jobs) {
  const GGramJob J = jobs[blockIdx.x];
  double acc[4][4];
  mode_contract_tile<double>(J.G, J.G, J.A, J.m, J.m, J.B, 0, J.A * J.B, 0, 0, acc);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = ty * 4 + u, j = tx * 4 + v;
      if (i < J.m && j < J.m) J.out[i * J.m + j] = acc[u][v];
    }
}

// Gram matrix of one binary64 (A, m, B) view per workgroup for m <= 32 (the cores of the
// batched decomposition).  The view is read 64 t = (a, b) at a time into an LDS stage (the
// next 64 t are in flight while the current ones are multiplied); thread (ty, tx) forms
// rows 2 ty, 2 ty + 1 and columns 2 tx, 2 tx + 1 of the 32 x 32 result, each entry a
// sequential fused sum over t in increasing order (so out[i][j] and out[j][i] agree
// bitwise).  A * B < 2^31.
constexpr int kGST = 64;                                  // t per stage
constexpr int kGSStride = 34;                             // even: 16-byte aligned pairs
constexpr int kGSPer = kGST * 32 / kMCThreads;            // values each thread loads per stage
__global__ __launch_bounds__(kMCThreads) void gram_small_grouped_kernel(const GGramJob* __restrict__ jobs) {
  __shared__ __align__(16) double sG[kGST][kGSStride];
  const GGramJob J = jobs[blockIdx.x];
  const uint32_t m = static_cast<uint32_t>(J.m), B = static_cast<uint32_t>(J.B);
  const uint32_t T = static_cast<uint32_t>(J.A * J.B);
  const int tid = threadIdx.x;
  // load roles, following memory order: t fastest when rows of b are long, the mode index
  // fastest otherwise
  const bool tfast = B >= static_cast<uint32_t>(kGST);
  const uint32_t lt = tfast ? tid % kGST : tid / 32, li = tfast ? tid / kGST : tid % 32;
  const uint32_t tstep = tfast ? 0 : kMCThreads / 32, istep = tfast ? kMCThreads / kGST : 0;
  double v[kGSPer];
  auto load = [&](uint32_t t0) {
#pragma unroll
    for (int q = 0; q < kGSPer; ++q) {
      const uint32_t t = t0 + lt + tstep * q, i = li + istep * q;
      const uint32_t a = t / B, b = t - a * B;
      v[q] = (t < T && i < m) ? J.G[(static_cast<int64_t>(a) * m + i) * B + b] : 0.0;
    }
  };
  const int tx = tid % 16, ty = tid / 16;
  double acc[2][2] = {};
  load(0);
  for (uint32_t t0 = 0; t0 < T; t0 += kGST) {
    __syncthreads();  // the previous stage has been read
#pragma unroll
    for (int q = 0; q < kGSPer; ++q) sG[lt + tstep * q][li + istep * q] = v[q];
    __syncthreads();
    if (t0 + kGST < T) load(t0 + kGST);
    const uint32_t tn = T - t0 < static_cast<uint32_t>(kGST) ? T - t0 : kGST;
#pragma unroll 4
    for (uint32_t tt = 0; tt < tn; ++tt) {
      const double2 a = *reinterpret_cast<const double2*>(&sG[tt][2 * ty]);
      const double2 b = *reinterpret_cast<const double2*>(&sG[tt][2 * tx]);
      acc[0][0] = fma(a.x, b.x, acc[0][0]);
      acc[0][1] = fma(a.x, b.y, acc[0][1]);
      acc[1][0] = fma(a.y, b.x, acc[1][0]);
      acc[1][1] = fma(a.y, b.y, acc[1][1]);
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const uint32_t i = 2 * ty + u, j = 2 * tx + w;
      if (i < m && j < m) J.out[i * m + j] = acc[u][w];
    }
}

// out = sum over chunks of the partial tiles: 16 lanes per output element, each
// summing every 16th chunk, then a fixed butterfly (deterministic order).
template <typename T>
__global__ __launch_bounds__(256) void mode_contract_reduce(const T* __restrict__ part, int nchunks, int tiles,
                                                            int tilesQ, int64_t mP, int64_t mQ, bool accumulate,
                                                            T* __restrict__ out) {
  const int64_t total = mP * mQ;
  const int sub = threadIdx.x % 16;
  const int64_t idx = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) / 16;
  const bool valid = idx < total;
  T s = T(0);
  int64_t i = 0, j = 0;
  if (valid) {
    i = idx / mQ;
    j = idx - i * mQ;
    const int tile = static_cast<int>((i / kMCTile) * tilesQ + (j / kMCTile));
    const int64_t off = (i % kMCTile) * kMCTile + (j % kMCTile);
    for (int c = sub; c < nchunks; c += 16) s += part[(static_cast<int64_t>(c) * tiles + tile) * kMCTile * kMCTile + off];
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, 16);
  if (valid && sub == 0) out[idx] = accumulate ? out[idx] + s : s;
}

// binary32 mode contraction on matrix cores.  A workgroup owns a 64 x 64 output
// tile and a range of the contracted index t = (a, b); it stages 32 t at a time
// of both operands in LDS (loads follow memory order: along b when rows are long,
// along the mode index otherwise) and each wave accumulates a 16 x 64 strip with
// 16x16x4 MFMAs.  Output: one 64 x 64 partial tile per (chunk, tile).
typedef float mc_f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMCT = 32;
constexpr int kMCStride = kMCT + 1;

__global__ __launch_bounds__(256) void mode_contract_mfma_kernel(const float* __restrict__ P,
                                                                 const float* __restrict__ Q, int64_t A, int64_t mP,
                                                                 int64_t mQ, int64_t B, int64_t chunk, int tilesQ,
                                                                 float* __restrict__ part) {
  __shared__ float sP[kMCTile * kMCStride];
  __shared__ float sQ[kMCTile * kMCStride];
  const int tile = blockIdx.x;
  const int ti = tile / tilesQ, tj = tile % tilesQ;
  const int64_t i0 = static_cast<int64_t>(ti) * kMCTile, j0 = static_cast<int64_t>(tj) * kMCTile;
  const int64_t total = A * B;
  const int64_t t0 = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t t1 = (t0 + chunk < total) ? t0 + chunk : total;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int r16 = lane % 16, q = lane / 16;
  const int64_t nP = (mP - i0 < kMCTile) ? mP - i0 : kMCTile;  // valid rows of this tile
  const int64_t nQ = (mQ - j0 < kMCTile) ? mQ - j0 : kMCTile;
  const int njt = static_cast<int>((nQ + 15) / 16);
  const bool wave_rows = 16 * wave < nP;
  mc_f32x4 acc[4];
#pragma unroll
  for (int js = 0; js < 4; ++js) acc[js] = mc_f32x4{0.f, 0.f, 0.f, 0.f};

  const bool tfast = B >= kMCT;
  // tfast: thread loads t = tb + (tid % 32) for rows tid/32 + 8 r;
  // otherwise: row tid % 64, t = tb + tid/64 + 4 r (consecutive threads: consecutive rows)
  const int lt = tfast ? threadIdx.x % kMCT : threadIdx.x / kMCTile;
  const int li = tfast ? threadIdx.x / kMCT : threadIdx.x % kMCTile;
  int64_t a = (t0 + lt) / B, b = (t0 + lt) - ((t0 + lt) / B) * B;
  const int64_t da = 4 / B, db = 4 % B;  // a step of 4 in t, for rows shorter than 32
  for (int64_t tb = t0; tb < t1; tb += kMCT) {
    __syncthreads();
    if (tfast) {
      const int64_t t = tb + lt;
      const bool tin = t < t1;
      const float* pp = P + a * mP * B + (i0 + li) * B + b;
      const float* qp = Q + a * mQ * B + (j0 + li) * B + b;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int ii = li + 8 * r;
        sP[ii * kMCStride + lt] = (tin && ii < nP) ? pp[static_cast<int64_t>(8 * r) * B] : 0.f;
        sQ[ii * kMCStride + lt] = (tin && ii < nQ) ? qp[static_cast<int64_t>(8 * r) * B] : 0.f;
      }
      b += kMCT;
      if (b >= B) { b -= B; ++a; }
    } else {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int tt = lt + 4 * r;
        const bool tin = tb + tt < t1;
        sP[li * kMCStride + tt] = (tin && li < nP) ? P[a * mP * B + (i0 + li) * B + b] : 0.f;
        sQ[li * kMCStride + tt] = (tin && li < nQ) ? Q[a * mQ * B + (j0 + li) * B + b] : 0.f;
        a += da;
        b += db;
        if (b >= B) { b -= B; ++a; }
      }
    }
    __syncthreads();
    // branch-free: rows past the matrix are zero in LDS (see the binary64 Gram kernel)
#pragma unroll
    for (int k0 = 0; k0 < kMCT; k0 += 4) {
      const float av = sP[(16 * wave + r16) * kMCStride + k0 + q];
#pragma unroll
      for (int js = 0; js < 4; ++js) {
        const float bv = sQ[(16 * js + r16) * kMCStride + k0 + q];
        acc[js] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[js], 0, 0, 0);
      }
    }
  }
  if (!wave_rows) return;
  float* out = part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + tile) * kMCTile * kMCTile;
#pragma unroll
  for (int js = 0; js < 4; ++js)
    if (js < njt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(16 * wave + 4 * q + v) * kMCTile + 16 * js + r16] = acc[js][v];
    }
}

struct MCPlan {
  int tilesP, tilesQ, nchunks;
  int64_t chunk;
};

MCPlan mc_plan(rt_dtype dt, int64_t A, int64_t mP, int64_t mQ, int64_t B) {
  MCPlan p;
  p.tilesP = static_cast<int>(ceil_div(mP, kMCTile));
  p.tilesQ = static_cast<int>(ceil_div(mQ, kMCTile));
  const int64_t total = A * B;
  // binary32 runs on matrix cores and is bound by the operand read: aim for
  // about 4 workgroups per CU; binary64 (small Gram matrices) keeps ~512
  const int64_t target = (dt == RT_F32) ? 1024 : 512;
  const int64_t gran = (dt == RT_F32) ? kMCT : kMCK;
  int64_t want = target / (p.tilesP * p.tilesQ);
  if (want < 1) want = 1;
  int64_t chunk = ceil_div(total, want);
  // binary64 (small Gram matrices): one or two rounds of 16 t per workgroup, so the
  // contraction is not a chain of load latencies; binary32 keeps 64 t or more
  const int64_t cmin = (dt == RT_F32) ? 64 : 16;
  if (chunk < cmin) chunk = cmin;
  chunk = ceil_div(chunk, gran) * gran;
  p.chunk = chunk;
  p.nchunks = static_cast<int>(ceil_div(total, chunk));
  if (p.nchunks < 1) p.nchunks = 1;
  return p;
}

// ------------------------------------------------------------------ eigensolver
// Eigenvectors of the symmetric positive semidefinite Gram matrix M = G_(j) G_(j)^T:
//  1. Cholesky with complete (diagonal) pivoting, M(p, p) = L L^T, taking at each
//     step the largest remaining diagonal entry; this is the R factor of a
//     column-pivoted QR of G_(j)^T, so L is strongly graded;
//  2. one-sided (Hestenes) Jacobi on the columns of L: rotate column pairs until
//     all are mutually orthogonal, so L V = U S with U the eigenvectors of M and
//     S^2 its eigenvalues (no V is accumulated: the rotated columns are U S).
// Jacobi on the transposed R factor of a pivoted QR converges in a few sweeps,
// and the left singular vectors of L are more accurate than eigenvectors of M
// computed directly.  One round applies the rotations of all disjoint pairs of
// the circle-method pairing; each pair is owned by a row of 16 lanes (4 rows of L
// each), so a round needs one barrier and two waves share each SIMD, which hides
// part of the latency of the dependent binary64 operations.  A round is bound by
// the dependent chain of one pair, so the rotation angle is found in binary32
// (any angle gives an exactly orthogonal rotation; a slightly wrong one only
// leaves a residual product of about 1e-7 of the old one, which later rotations
// remove) and only cos phi = 1 / sqrt(1 + tan^2 phi) is computed to full binary64
// accuracy, with sin phi = tan phi cos phi, so that c^2 + s^2 = 1 to rounding.
constexpr int kJN = 64;
constexpr int kJThreads = 512;
constexpr int kJWaves = kJThreads / kWave;
constexpr int kPairLanes = 16;
constexpr int kPairRows = kJN / kPairLanes;  // rows of a column per lane
constexpr int kMaxSweeps = 30;
constexpr int kLStride = 72;  // doubles per column of L in LDS (padding spreads banks)
constexpr int kAStride = 65;  // doubles per row of the working matrix

// DPP moves on the two halves of a binary64 value (every source lane used here
// lies inside the row, so bound_ctrl never takes effect and no old value is needed)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int64_t u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(u & 0xffffffff), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(u >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}
// sum over aligned groups of 16 lanes (a DPP row); every lane of a group gets bitwise the
// same value (each step adds a value to its partner's with the operands swapped, and
// addition commutes)
__device__ __forceinline__ double group16_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror: lane i <- lane 7-i within 8
  v += dpp_f64<0x140>(v);  // row_mirror: lane i <- lane 15-i within 16
  return v;
}
// three such sums, stage by stage, so that the three dependent chains overlap
__device__ __forceinline__ void group16_sum3(double& a, double& b, double& c) {
#define RT_STAGE(CTRL)                   \
  {                                      \
    const double da = dpp_f64<CTRL>(a);  \
    const double db = dpp_f64<CTRL>(b);  \
    const double dc = dpp_f64<CTRL>(c);  \
    a += da;                             \
    b += db;                             \
    c += dc;                             \
  }
  RT_STAGE(0xB1)
  RT_STAGE(0x4E)
  RT_STAGE(0x141)
  RT_STAGE(0x140)
#undef RT_STAGE
}


__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int64_t u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), lane);
  return __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}

// DPP broadcast of the last lane of a row into the rows of ROW_MASK (other rows keep v)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_bcast_f64(double v) {
  const int64_t u = __double_as_longlong(v);
  const int l = static_cast<int>(u & 0xffffffff), h = static_cast<int>(u >> 32);
  const int lo = __builtin_amdgcn_update_dpp(l, l, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(h, h, CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}

// argmax over the whole wave; every lane ends with the value and its lane.  The lane
// number (reversed) replaces the 6 lowest mantissa bits, so one binary64 max per step
// carries the index along; values that agree to 46 bits count as ties, which go to the
// lowest lane.  The returned value is the unmodified one of the chosen lane.
__device__ __forceinline__ void argmax64(double& v, int& idx) {
  const int lane = static_cast<int>(threadIdx.x % kWave);
  double k = __longlong_as_double((__double_as_longlong(v) & ~static_cast<int64_t>(63)) | (63 - lane));
  k = fmax(k, dpp_f64<0xB1>(k));   // quad_perm [1,0,3,2]
  k = fmax(k, dpp_f64<0x4E>(k));   // quad_perm [2,3,0,1]
  k = fmax(k, dpp_f64<0x141>(k));  // row_half_mirror
  k = fmax(k, dpp_f64<0x140>(k));  // row_mirror: every lane of a row holds the row's maximum
  k = fmax(k, dpp_bcast_f64<0x142, 0xA>(k));  // row_bcast:15 -> rows 1, 3
  k = fmax(k, dpp_bcast_f64<0x143, 0xC>(k));  // row_bcast:31 -> rows 2, 3 (row 3: all)
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(__double_as_longlong(k) & 0xffffffff), kWave - 1);
  idx = 63 - (lo & 63);
  v = readlane_f64(v, idx);
}


// Am: Schur complement during the Cholesky (original indices), kJN x kAStride;
// Lc: columns of L, Lc[col * kLStride + row] (original row order), kJN x kLStride.
__device__ __forceinline__ void eig_jacobi(const double* __restrict__ M, int n, int r, double* __restrict__ Vout,
                                           double* __restrict__ evals, double* __restrict__ Am,
                                           double* __restrict__ Lc) {
  __shared__ double nrm[kJN];
  __shared__ int active;
  __shared__ double tau2s;
  __shared__ int order[kJN];
  __shared__ double vtmp[kJN];
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wv = tid / kWave;
  for (int idx = tid; idx < kJN * kLStride; idx += kJThreads) Lc[idx] = 0.0;
  for (int idx = tid; idx < kJN * kAStride; idx += kJThreads) Am[idx] = 0.0;
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += kJThreads) {
    const int i = idx / n, j = idx - (idx / n) * n;
    Am[i * kAStride + j] = M[idx];
  }
  __syncthreads();
  // ---- 1. Cholesky with complete pivoting; column k of L is stored in original row order.
  //         Thread (wave w, lane j) owns column j on rows w, w + 8, ...  In a step the pivot
  //         column is only read; the pivot row is set to zero, so rows pivoted earlier give
  //         zero multipliers without any masking.  Every wave keeps the whole remaining
  //         diagonal in registers (lane j: entry j, updated with the same arithmetic as the
  //         matrix) and picks the next pivot itself, so a step needs a single barrier.
  double dj = (lane < n) ? Am[lane * kAStride + lane] : -1.0;
  double d = dj;
  int p = lane;
  argmax64(d, p);
  const double dmax = d;
  int nc = n;
  for (int k = 0; k < n; ++k) {
    if (!(d > 1e-300 && d > 1e-30 * dmax)) {
      nc = k;
      break;
    }
    const double inv = rsq_refined(d);
    // multipliers L[i][k] = A[i][p] / sqrt(d) (A[p][p] = d gives sqrt(d) on the pivot row)
    const double lj = Am[lane * kAStride + p] * inv;
    if (wv == 0 && lane < n) Lc[k * kLStride + lane] = lj;
    if (lane < n && lane != p) {
      // all loads first (the pivot column is not written in this step), then the stores
      double li[kJN / kJWaves], av[kJN / kJWaves];
#pragma unroll
      for (int t = 0; t < kJN / kJWaves; ++t) {
        li[t] = Am[(wv + kJWaves * t) * kAStride + p];
        av[t] = Am[(wv + kJWaves * t) * kAStride + lane];
      }
#pragma unroll
      for (int t = 0; t < kJN / kJWaves; ++t) {
        const int i = wv + kJWaves * t;
        Am[i * kAStride + lane] = (i == p) ? 0.0 : fma(-li[t] * inv, lj, av[t]);
      }
    }
    dj = (lane == p || dj < 0.0) ? -1.0 : fma(-lj, lj, dj);
    d = dj;
    p = lane;
    argmax64(d, p);
    __syncthreads();
  }
  // ---- 2. one-sided Jacobi on the nc columns of L; lane `sub` of a pair group owns rows 4*sub .. 4*sub+3
  const int N = nc + (nc & 1);
  const int half = N / 2;
  const int g = tid / kPairLanes, sub = tid % kPairLanes;
  const double tol = (n > 8 ? n : 8) * 2.220446049250313e-16;
  const double tol2 = tol * tol;
  // Near convergence a sweep squares the largest relative off-diagonal product, so a
  // sweep in which none exceeded 1e-9 leaves them all far below tol: the verifying sweep
  // that would rotate nothing is skipped.
  const double thr2 = 1e-18;
  // Only the r columns of largest norm are returned.  A pair of two columns that both
  // lie below the r-th largest norm only mixes directions inside the discarded subspace,
  // so it does not hold up the stopping test (it is still rotated).  tau2 is the r-th
  // largest squared norm, taken from the last round of the previous sweep, in which
  // every column is in a pair; sweep 0 counts every pair.
  double tau2 = 0.0;
  if (tid == 0) tau2s = 0.0;
  for (int sweep = 0; sweep < kMaxSweeps && N > 1; ++sweep) {
    if (tid == 0) active = 0;
    __syncthreads();
    if (sweep > 0) tau2 = tau2s;
    // circle-method positions of this group's pair, advanced without division
    int a_pos = (g == 0) ? 0 : g;                  // position g holds player g at round 0
    int b_pos = N - 1 - g;
    for (int round = 0; round < N - 1; ++round) {
      if (g < half) {
        const int pc = a_pos < b_pos ? a_pos : b_pos, qc = a_pos < b_pos ? b_pos : a_pos;
        double* xp = Lc + pc * kLStride + kPairRows * sub;
        double* yp = Lc + qc * kLStride + kPairRows * sub;
        double2 x2[kPairRows / 2], y2[kPairRows / 2];
#pragma unroll
        for (int t = 0; t < kPairRows / 2; ++t) {
          x2[t] = reinterpret_cast<const double2*>(xp)[t];
          y2[t] = reinterpret_cast<const double2*>(yp)[t];
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int t = 0; t < kPairRows / 2; ++t) {
          al = fma(x2[t].x, x2[t].x, al); al = fma(x2[t].y, x2[t].y, al);
          be = fma(y2[t].x, y2[t].x, be); be = fma(y2[t].y, y2[t].y, be);
          ga = fma(x2[t].x, y2[t].x, ga); ga = fma(x2[t].y, y2[t].y, ga);
        }
        group16_sum3(al, be, ga);
        if (round == N - 2 && sub == 0) {
          nrm[pc] = al;
          nrm[qc] = be;
        }
        // rotate unless the pair is orthogonal to the rounding level of an n-term dot product
        if (fabs(ga) > 1e-300 && ga * ga > tol2 * (al * be)) {
          // tan(2 phi) = v / u with u = be - al, v = 2 ga; smallest rotation |phi| <= pi/4:
          //   |tan phi| = |v| / (|u| + sqrt(u^2 + v^2)),  sign = sign(u v) (+ for u = 0).
          // u and v are scaled exactly by a power of two to |.| <= 1 before going to binary32.
          const double u0 = be - al, v0 = 2.0 * ga;
          const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(u0), fabs(v0)));
          const float uf = static_cast<float>(__builtin_amdgcn_ldexp(fabs(u0), -ex));
          const float vf = static_cast<float>(__builtin_amdgcn_ldexp(fabs(v0), -ex));
          const float hf = __builtin_amdgcn_sqrtf(fmaf(uf, uf, vf * vf));
          const double t = static_cast<double>(vf * __builtin_amdgcn_rcpf(uf + hf));
          const double c = rsq_refined(fma(t, t, 1.0));
          double s = t * c;
          if ((u0 < 0.0) != (v0 < 0.0) && u0 != 0.0) s = -s;
#pragma unroll
          for (int q = 0; q < kPairRows / 2; ++q) {
            double2 nx, ny;
            nx.x = c * x2[q].x - s * y2[q].x;  nx.y = c * x2[q].y - s * y2[q].y;
            ny.x = s * x2[q].x + c * y2[q].x;  ny.y = s * x2[q].y + c * y2[q].y;
            reinterpret_cast<double2*>(xp)[q] = nx;
            reinterpret_cast<double2*>(yp)[q] = ny;
          }
          if (sub == 0 && ga * ga > thr2 * (al * be) && fmax(al, be) >= tau2) active = 1;
        }
      }
      // next round: every position except 0 advances by one player (wrapping N-1 -> 1)
      if (g != 0) a_pos = (a_pos == N - 1) ? 1 : a_pos + 1;
      b_pos = (b_pos == N - 1) ? 1 : b_pos + 1;
      __syncthreads();
    }
    if (!active) break;
    // r-th largest squared norm (ties: lower index first) for the next sweep's test
    if (tid < N) {
      const double li = nrm[tid];
      int rk = 0;
      for (int j = 0; j < N; ++j) {
        const double lj = nrm[j];
        rk += (lj > li || (lj == li && j < tid)) ? 1 : 0;
      }
      if (rk == r - 1) tau2s = li;
    }
    __syncthreads();
  }
  // ---- 3. norms, order (decreasing), normalised columns, sign rule
  if (tid < kJN) {
    double s = 0.0;
    if (tid < nc)
      for (int i = 0; i < n; ++i) s = fma(Lc[tid * kLStride + i], Lc[tid * kLStride + i], s);
    nrm[tid] = s;
  }
  __syncthreads();
  if (tid < n) {
    const int i = tid;
    const double li = nrm[i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = nrm[j];
      if (lj > li || (lj == li && j < i)) ++rk;
    }
    order[rk] = i;
  }
  __syncthreads();
  if (evals && tid < r) evals[tid] = nrm[order[tid]];
  if (tid == 0) {
    // columns beyond the numerical rank: complete with unit vectors orthogonalised
    // against the previous columns (modified Gram-Schmidt), so V stays orthonormal
    for (int k = 0; k < r; ++k) {
      const int col = order[k];
      if (nrm[col] > 0.0 && k < nc) continue;
      for (int e = 0; e < n; ++e) {
        double* v = vtmp;
        for (int i = 0; i < n; ++i) v[i] = (i == e) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass)
          for (int kk = 0; kk < k; ++kk) {
            const int cc = order[kk];
            const double inv = 1.0 / sqrt(nrm[cc]);
            double dp = 0.0;
            for (int i = 0; i < n; ++i) dp += Lc[cc * kLStride + i] * inv * v[i];
            for (int i = 0; i < n; ++i) v[i] -= dp * Lc[cc * kLStride + i] * inv;
          }
        double nv = 0.0;
        for (int i = 0; i < n; ++i) nv += v[i] * v[i];
        if (nv > 0.5) {
          for (int i = 0; i < n; ++i) Lc[col * kLStride + i] = v[i] / sqrt(nv);
          nrm[col] = 1.0;
          break;
        }
      }
    }
  }
  __syncthreads();
  if (tid < r) {
    const int k = tid, col = order[k];
    const double inv = 1.0 / sqrt(nrm[col]);
    // sign rule: largest |entry| (first on ties) positive
    double best = -1.0, sgn = 1.0;
    for (int x = 0; x < n; ++x) {
      const double v = Lc[col * kLStride + x];
      if (fabs(v) > best) { best = fabs(v); sgn = (v < 0.0) ? -1.0 : 1.0; }
    }
    for (int i = 0; i < n; ++i) Vout[i * r + k] = sgn * inv * Lc[col * kLStride + i];
  }
}

// ------------------------------------------------------------------ tridiagonal eigensolver
// The r <= 32 leading eigenpairs of the Gram matrix, in four phases on one workgroup:
//  1. Householder reduction to tridiagonal form, T = Q^T A Q with Q = H_0 ... H_{n-3};
//  2. the r largest eigenvalues of T by multisection: G lanes per eigenvalue evaluate the
//     Sturm count (sign changes of the leading principal minors, a three-term recurrence
//     rescaled by powers of two) at G interior points of its bracket, which shrinks
//     (G + 1)x per step (G = 16 for r <= 16, else 8, so at most four waves count);
//  3. eigenvectors of T by inverse iteration, one lane per eigenvalue: LU of T - lambda I
//     with partial pivoting (tiny pivots raised to eps |T|), two solves from a fixed
//     pseudo-random start vector;
//  4. one Loewdin step Z <- Z (I - E/2 + 3 E^2 / 8), E = Z^T Z - I, skipped when Z is
//     orthonormal to rounding already, then V = Q Z.
// The result is accepted only when ||E|| <= 1e-6 (the series is then exact to rounding)
// and every residual |T z - lambda z| is below 1e-12 |T|; otherwise, for example for
// repeated or numerically zero eigenvalues, whose inverse-iteration vectors are not
// independent, the caller falls back to the Jacobi solver.  The phases are sequential
// chains of about 50 steps each instead of the ~350 rounds of Jacobi sweeps.
constexpr int kTriMaxR = 32;
// Multisection widths: the Sturm counts are issue-bound, so the lane groups are sized to
// keep at most one counting wave per SIMD (r <= 16: 16 lanes, 17^14 > 2^57; r <= 32:
// 8 lanes, 9^18 > 2^57); either way the bracket reaches rounding level of |T|.
constexpr int kMsLanes = 256;
static_assert(16 * 16 <= kMsLanes && 8 * kTriMaxR <= kMsLanes && kMsLanes <= kJThreads,
              "one lane group per eigenvalue");
constexpr int kInvIters = 2;
// scratch region B (doubles): five n x RM arrays of the inverse iteration (RM: the bound on
// r); aliased by the per-wave vectors and partial sums of phase 1, by E and F of phase 4,
// and by the Jacobi L

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_rows_f64(double v, double old) {
  const int64_t u = __double_as_longlong(v), o = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(o & 0xffffffff), static_cast<int>(u & 0xffffffff),
                                             CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(o >> 32), static_cast<int>(u >> 32), CTRL,
                                             ROW_MASK, 0xF, false);
  return __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}
// sum / max over the whole wave; every lane of every wave gets bitwise the same value
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  v += dpp_rows_f64<0x142, 0xA>(v, 0.0);  // row_bcast:15 -> rows 1, 3
  v += dpp_rows_f64<0x143, 0xC>(v, 0.0);  // row_bcast:31 -> rows 2, 3
  return readlane_f64(v, kWave - 1);
}
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  v = fmax(v, dpp_rows_f64<0x142, 0xA>(v, v));
  v = fmax(v, dpp_rows_f64<0x143, 0xC>(v, v));
  return readlane_f64(v, kWave - 1);
}
__device__ __forceinline__ double rcp_refined(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
// fixed pseudo-random start value in [-1/2, 1/2) for row i of eigenvector m
// (32-bit integer finaliser of MurmurHash3)
__device__ __forceinline__ double start_value(int i, int m) {
  uint32_t h = static_cast<uint32_t>(i * 64 + m + 1);
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return static_cast<double>(h) * 0x1p-32 - 0.5;
}
// make LDS data written by other lanes of this wave visible to the next reads of this wave
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Number of eigenvalues of T below x: sign changes along the leading principal minors
// p_i = (d_i - x) p_{i-1} - e2_{i-1} p_{i-2}.  The arrays are padded past n - 1 with
// d = 2^200 and e2 = 0, where the minors keep their sign, so the loop runs in whole
// blocks of eight.  Two register buffers alternate (the loop is unrolled by two
// blocks), so the loads of the next block are in flight during a whole block of
// arithmetic; an exact power-of-two rescaling after each block keeps the minors in range.
constexpr int kStBlk = 8;
__device__ __forceinline__ uint32_t sign_word(double v) {
  return static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(v)) >> 32);
}
// (the sign changes are counted on the high words in vector registers: no mask round trips)
__device__ __forceinline__ void sturm_steps(const double (&dv)[kStBlk], const double (&ev)[kStBlk], double x,
                                            double& p0, double& p1, uint32_t& h1, uint32_t& cnt) {
#pragma unroll
  for (int t = 0; t < kStBlk; ++t) {
    const double p2 = fma(dv[t] - x, p1, -ev[t] * p0);
    const uint32_t h2 = sign_word(p2);
    cnt += (h2 ^ h1) >> 31;
    p0 = p1;
    p1 = p2;
    h1 = h2;
  }
  const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(p0), fabs(p1)));
  p0 = __builtin_amdgcn_ldexp(p0, -ex);
  p1 = __builtin_amdgcn_ldexp(p1, -ex);
}
__device__ __forceinline__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n,
                                           double x) {
  // A minor that is exactly zero counts with the sign bit it carries.  With e_{i-1} != 0
  // the next minor has the opposite sign of the one before the zero, so the pair of
  // transitions adds one change whichever sign the zero takes; a zero next to a split of
  // T (e = 0) can miscount, and the caller's residual check then rejects the eigenvalue.
  double p0 = 1.0, p1 = d[0] - x;
  uint32_t h1 = sign_word(p1);
  uint32_t cnt = h1 >> 31;
  double da[kStBlk], ea[kStBlk], db[kStBlk], eb[kStBlk];
#pragma unroll
  for (int t = 0; t < kStBlk; ++t) {
    da[t] = d[1 + t];
    ea[t] = e2[t];
  }
  for (int i = 1; i < n; i += 2 * kStBlk) {
#pragma unroll
    for (int t = 0; t < kStBlk; ++t) {
      db[t] = d[i + kStBlk + t];
      eb[t] = e2[i + kStBlk - 1 + t];
    }
    sturm_steps(da, ea, x, p0, p1, h1, cnt);
    if (i + kStBlk >= n) break;
#pragma unroll
    for (int t = 0; t < kStBlk; ++t) {
      da[t] = d[i + 2 * kStBlk + t];
      ea[t] = e2[i + 2 * kStBlk - 1 + t];
    }
    sturm_steps(db, eb, x, p0, p1, h1, cnt);
  }
  return static_cast<int>(cnt);
}

// Multisection for the r largest eigenvalues of T (d, e2 padded as sturm_count reads them):
// lanes G g .. G g + G - 1 bracket the g-th largest; ITERS steps shrink [lo, hi] by
// (G + 1)^ITERS.  lam[g] = the midpoint of the final bracket.
template <int G, int ITERS>
__device__ __forceinline__ void multisect(const double* __restrict__ d, const double* __restrict__ e2,
                                          const double* __restrict__ bounds, int n, int r,
                                          double* __restrict__ lam) {
  static_assert(kWave % G == 0 && G <= 32, "lane groups within a wave");
  const int tid = threadIdx.x;
  if (tid >= G * r) return;
  const int g = tid / G, sub = tid % G;
  const int target = n - 1 - g;  // count(x) > target  <=>  x above the g-th largest
  double a = bounds[0], b = bounds[1];
  const double cl = static_cast<double>(sub + 1) / (G + 1);
  for (int it = 0; it < ITERS; ++it) {
    const double wd = b - a;
    const int cnt = sturm_count(d, e2, n, fma(wd, cl, a));
    const unsigned long long bal = __ballot(cnt > target);
    const unsigned bits = static_cast<unsigned>(bal >> (G * (g % (kWave / G)))) & ((1u << G) - 1u);
    const int l = bits ? __builtin_ctz(bits) : G;
    const double na = (l == 0) ? a : fma(wd, static_cast<double>(l) / (G + 1), a);
    const double nb = (l == G) ? b : fma(wd, static_cast<double>(l + 1) / (G + 1), a);
    a = na;
    b = nb;
  }
  if (sub == 0) lam[g] = 0.5 * (a + b);
}

// Waves of the Householder reduction: eight (two per SIMD; measured 4 % faster than four)
// when the solve has its CU to itself (RM = 32), four when two solves share a CU (RM = 16).
constexpr int p1_waves(int rm) { return rm == 16 ? 4 : 8; }
constexpr int kP1MaxWaves = 8;

// Returns true (uniformly over the workgroup) when V and evals were written.  RM (32 or
// 16) bounds r: the scratch B holds 5 kJN RM doubles.
template <int RM>
__device__ __forceinline__ bool eig_tridiag(const double* __restrict__ M, int n, int r, double* __restrict__ Vout,
                                            double* __restrict__ evals, double* __restrict__ Am,
                                            double* __restrict__ B) {
  constexpr int kPad = kJN + 3 * kStBlk;  // tridiagonal arrays padded for the blocked Sturm loop
  constexpr int kP1Waves = p1_waves(RM);
  constexpr int kP1Cols = kJN / kP1Waves;  // matrix columns held in registers per wave
  __shared__ double dS[kPad], eS[kPad], e2S[kPad], tauS[kJN], lamS[kJN];
  __shared__ double bounds[3];
  __shared__ unsigned long long ebits, rbits;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
  // ---- load, scaled by the power of two that brings the largest diagonal entry to [1/2, 1)
  const double dmax = wave_max_f64(lane < n ? fabs(M[lane * n + lane]) : 0.0);
  if (!(dmax > 0.0) || !(dmax < 1e300)) return false;  // zero or non-finite: Jacobi path
  const int ex = __builtin_amdgcn_frexp_exp(dmax);
  // scratch in B: per-wave copies of v and w (in slot order, see below), partial products
  // and the published column, both double-buffered by the parity of the step
  double* vbuf = B;                               // [wave][kJN]
  double* wbuf = B + kP1Waves * kJN;              // [wave][kJN]
  double* part = B + 2 * kP1Waves * kJN;          // [2][wave][kJN]
  double* colbuf = B + 4 * kP1Waves * kJN;        // [2][kJN]
  for (int idx = tid; idx < kJN * kAStride; idx += kJThreads) Am[idx] = 0.0;
  if (tid == 0) {
    ebits = 0;
    rbits = 0;
  }
  // ---- 1. Householder tridiagonalisation on W = p1_waves(RM) waves.  Column j of the
  //         matrix lives in registers of wave j % W, slot j / W (lane = row), for the whole
  //         reduction.  The matrix-vector product and the rank-2 update touch LDS only for
  //         broadcast reads of v and w, which each wave stores in slot order (entry j at
  //         (j % W) (64 / W) + j / W); v stays in registers from the product to the update.
  //         Every wave keeps column k, the one the reflector of step k is formed from, in
  //         a register.  The wave that owns column k + 1 publishes it as it stands before
  //         step k, together with its partial products; after the step's one barrier every
  //         wave applies the step's rank-2 update to that copy with the same operands and
  //         the same fused operations as the owner, so all copies agree bitwise and no
  //         second barrier is needed.  The LDS areas written in a step alternate with the
  //         parity of k: a wave writes an area again only two steps later, after every wave
  //         has passed the barrier that follows its reads.  Rows and columns past n are zero
  //         and carry v = w = 0; finished columns (j <= k) see v_j = w_j = 0 and keep their
  //         values.
  const bool worker = wv < kP1Waves;
  const int slot_of_lane = (lane % kP1Waves) * kP1Cols + lane / kP1Waves;
  double ar[kP1Cols];
#pragma unroll
  for (int t = 0; t < kP1Cols; ++t) {
    const int j = kP1Waves * t + wv;
    ar[t] = (worker && lane < n && j < n) ? __builtin_amdgcn_ldexp(M[lane * n + j], -ex) : 0.0;
  }
  // column 0 goes through the slot that step 1 writes, so step 0's write cannot overtake it
  if (wv == 0) colbuf[kJN + lane] = ar[0];
  __syncthreads();
  double xc = worker ? colbuf[kJN + lane] : 0.0;  // column k
  for (int k = 0; k + 2 < n; ++k) {
    const bool live = lane > k && lane < n;
    double* partb = part + (k & 1) * (kP1Waves * kJN);
    double* colb = colbuf + (k & 1) * kJN;
    double sigma = 0.0, tk = 0.0, v = 0.0;
    double vv[kP1Cols];
    if (worker) {
      const double x = live ? xc : 0.0;
      sigma = wave_sum_f64((lane > k + 1 && lane < n) ? x * x : 0.0);
      const double alpha = readlane_f64(x, k + 1);
      double ek = alpha;
      v = (lane == k + 1) ? 1.0 : 0.0;
      double acc = 0.0;
      if (sigma != 0.0) {
        // H x = beta e_1 with beta = -sign(alpha) mu, mu = |x|; tau = 1 + |alpha| / mu and
        // v = x / (alpha - beta) = sign(alpha) x / (|alpha| + mu), v_{k+1} = 1
        const double s2 = fma(alpha, alpha, sigma);
        const double rs = rsq_refined(s2);
        const double mu = s2 * rs;
        ek = alpha >= 0.0 ? -mu : mu;
        tk = fma(fabs(alpha), rs, 1.0);
        const double sc = (alpha >= 0.0 ? 1.0 : -1.0) * rcp_refined(fabs(alpha) + mu);
        if (lane > k + 1 && lane < n) v = x * sc;
        double* myv = vbuf + wv * kJN;
        myv[slot_of_lane] = v;
        wave_lds_sync();
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int t = 0; t < kP1Cols; t += 2) {
          const double2 vj = *reinterpret_cast<const double2*>(myv + kP1Cols * wv + t);
          vv[t] = vj.x;
          vv[t + 1] = vj.y;
          a0 = fma(ar[t], vj.x, a0);
          a1 = fma(ar[t + 1], vj.y, a1);
        }
        acc = a0 + a1;
      }
      partb[wv * kJN + lane] = acc;
      if (wv == (k + 1) % kP1Waves) {  // column k + 1 before this step's update
        const int s = (k + 1) / kP1Waves;
#pragma unroll
        for (int t = 0; t < kP1Cols; ++t)
          if (t == s) colb[lane] = ar[t];
      }
      if (wv == 0) {
        const double dk = readlane_f64(xc, k);
        if (lane > k + 1 && lane < n) Am[lane * kAStride + k] = v;  // Householder vector below the subdiagonal
        if (lane == 0) {
          tauS[k] = tk;
          eS[k] = ek;
          dS[k] = dk;
        }
      }
    }
    __syncthreads();
    if (worker) {
      const double cb = colb[lane];
      double xn = cb;
      if (sigma != 0.0) {
        double p = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kP1Waves; ++w2) p += partb[w2 * kJN + lane];
        p = live ? tk * p : 0.0;
        const double K = 0.5 * tk * wave_sum_f64(p * v);
        const double w = fma(-K, v, p);
        double* myw = wbuf + wv * kJN;
        myw[slot_of_lane] = w;
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < kP1Cols; t += 2) {
          const double2 wj = *reinterpret_cast<const double2*>(myw + kP1Cols * wv + t);
          ar[t] = fma(-v, wj.x, fma(-w, vv[t], ar[t]));
          ar[t + 1] = fma(-v, wj.y, fma(-w, vv[t + 1], ar[t + 1]));
        }
        // column k + 1 after the update, formed exactly as its owner forms it
        const int sl = ((k + 1) % kP1Waves) * kP1Cols + (k + 1) / kP1Waves;
        xn = fma(-v, myw[sl], fma(-w, vbuf[wv * kJN + sl], cb));
      }
      xc = xn;
    }
  }
  // the last 2 x 2 block: column n - 2 is in xc; A[n-1][n-1] sits with its owner
  if (wv == (n - 1) % kP1Waves && lane == n - 1) {
    const int slot = (n - 1) / kP1Waves;
    double c = ar[0];
#pragma unroll
    for (int t = 1; t < kP1Cols; ++t) c = (t == slot) ? ar[t] : c;
    dS[n - 1] = c;
  }
  if (wv == 0) {
    const double d2 = readlane_f64(xc, n - 2), e2 = readlane_f64(xc, n - 1);
    if (lane == 0) {
      dS[n - 2] = d2;
      eS[n - 2] = e2;
    }
  }
  __syncthreads();
  for (int i = tid; i < kPad; i += kJThreads) {
    if (i >= n) dS[i] = 0x1p200;  // padding: the minors keep their sign (see sturm_count)
    e2S[i] = (i < n - 1) ? eS[i] * eS[i] : 0.0;
    if (i >= n - 1) eS[i] = 0.0;
  }
  if (wv == 0) {
    // Gershgorin interval and |T|
    const double el = (lane > 0 && lane < n) ? fabs(eS[lane - 1]) : 0.0;
    const double er = (lane < n - 1) ? fabs(eS[lane]) : 0.0;
    const double dl = lane < n ? dS[lane] : 0.0;
    const double lo = -wave_max_f64(lane < n ? -(dl - el - er) : -1e300);
    const double hi = wave_max_f64(lane < n ? dl + el + er : -1e300);
    const double tn = wave_max_f64(lane < n ? fmax(fabs(dl), er) : 0.0);
    if (lane == 0) {
      const double pad = 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + 0x1p-1000;
      bounds[0] = lo - pad;
      bounds[1] = hi + pad;
      bounds[2] = tn;
    }
  }
  __syncthreads();
  // ---- 2. multisection: group g brackets the g-th largest eigenvalue
  if (r > 16)
    multisect<8, 18>(dS, e2S, bounds, n, r, lamS);
  else
    multisect<16, 14>(dS, e2S, bounds, n, r, lamS);
  __syncthreads();
  // ---- 3. inverse iteration, lane m of wave 0 for eigenvalue m.  Loops run over rows with
  //         the row data for the next iterations loaded ahead (unrolled by four).
  auto F = [&](int f, int i, int m) -> double& { return B[(f * kJN + i) * RM + m]; };
  constexpr int IU0 = 0, U1 = 1, U2 = 2, ML = 3, ZZ = 4;
  if (wv == 0 && lane < r) {
    const int m = lane;
    const double lm = lamS[m];
    const double pert = 2.220446049250313e-16 * bounds[2];
    const double rpert = 1.0 / pert;
    double cd = dS[0] - lm, cs = eS[0];
    unsigned long long piv = 0;
#pragma unroll 4
    for (int i = 0; i + 1 < n; ++i) {
      const double sb = eS[i], nd = dS[i + 1] - lm, ns = eS[i + 1];  // eS is zero past n - 2
      const bool sw = fabs(sb) > fabs(cd);
      const double u0 = sw ? sb : cd;
      double ri = rcp_refined(u0);
      if (!(fabs(u0) >= pert)) ri = (u0 < 0.0) ? -rpert : rpert;  // tiny pivot raised to eps |T|
      const double mm = (sw ? cd : sb) * ri;
      F(IU0, i, m) = ri;
      F(U1, i, m) = sw ? nd : cs;
      F(U2, i, m) = sw ? ns : 0.0;
      F(ML, i, m) = mm;
      const double ncd = sw ? fma(-mm, nd, cs) : fma(-mm, cs, nd);
      cs = sw ? -mm * ns : ns;
      cd = ncd;
      piv |= static_cast<unsigned long long>(sw) << i;
    }
    {
      double ri = rcp_refined(cd);
      if (!(fabs(cd) >= pert)) ri = (cd < 0.0) ? -rpert : rpert;
      F(IU0, n - 1, m) = ri;
      F(U1, n - 1, m) = 0.0;
      F(U2, n - 1, m) = 0.0;
    }
    // Each solve reads the previous iterate scaled by 2^-ez (exact), where 2^ez brackets
    // its largest entry, so no separate rescaling pass is needed; the first forward
    // substitution takes the start vector as it goes.
    int ez = 0;
    for (int it = 0; it < kInvIters; ++it) {
      const auto rhs = [&](int i) {
        return it == 0 ? start_value(i, m) : __builtin_amdgcn_ldexp(F(ZZ, i, m), -ez);
      };
      double yi = rhs(0);
#pragma unroll 4
      for (int i = 0; i + 1 < n; ++i) {
        const double yn = rhs(i + 1), mm = F(ML, i, m);
        const bool sw = (piv >> i) & 1ull;
        F(ZZ, i, m) = sw ? yn : yi;
        yi = sw ? fma(-mm, yn, yi) : fma(-mm, yi, yn);
      }
      F(ZZ, n - 1, m) = yi;
      double z1 = 0.0, z2 = 0.0, mx = 0.0;
#pragma unroll 4
      for (int i = n - 1; i >= 0; --i) {
        const double zi = fma(-F(U1, i, m), z1, fma(-F(U2, i, m), z2, F(ZZ, i, m))) * F(IU0, i, m);
        F(ZZ, i, m) = zi;
        z2 = z1;
        z1 = zi;
        mx = fmax(mx, fabs(zi));
      }
      ez = (mx > 0.0) ? __builtin_amdgcn_frexp_exp(mx) : 0;
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
    for (int i = 0; i < n; ++i) {
      const double zi = __builtin_amdgcn_ldexp(F(ZZ, i, m), -ez);
      if (i & 1) s1 = fma(zi, zi, s1); else s0 = fma(zi, zi, s0);
    }
    const double ss = s0 + s1;
    const double inv = (ss > 0.0) ? rsq_refined(ss) : 0.0;
#pragma unroll 4
    for (int i = 0; i < n; ++i) F(ZZ, i, m) = __builtin_amdgcn_ldexp(F(ZZ, i, m), -ez) * inv;
  }
  __syncthreads();
  // ---- 4. orthogonality check E = Z^T Z - I (upper triangle) and residual check
  double* E = B;                          // r x r, stride (RM + 1) (the LU factors are dead now)
  double* Fm = B + RM * (RM + 1);   // I - E/2 + 3 E^2 / 8
  double emax = 0.0;
  for (int q = tid; q < r * r; q += kJThreads) {
    const int a = q / r, c = q - (q / r) * r;
    if (c < a) continue;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = 0;
#pragma unroll 2
    for (; i + 3 < n; i += 4) {
      s0 = fma(F(ZZ, i, a), F(ZZ, i, c), s0);
      s1 = fma(F(ZZ, i + 1, a), F(ZZ, i + 1, c), s1);
      s2 = fma(F(ZZ, i + 2, a), F(ZZ, i + 2, c), s2);
      s3 = fma(F(ZZ, i + 3, a), F(ZZ, i + 3, c), s3);
    }
    for (; i < n; ++i) s0 = fma(F(ZZ, i, a), F(ZZ, i, c), s0);
    const double eac = ((s0 + s1) + (s2 + s3)) - (a == c ? 1.0 : 0.0);
    E[a * (RM + 1) + c] = eac;
    E[c * (RM + 1) + a] = eac;
    emax = fmax(emax, fabs(eac));
  }
  constexpr int kPer = (kJN * RM + kJThreads - 1) / kJThreads;
  double rmax = 0.0;
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int q = tid + t * kJThreads;
    const int i = q / RM, m = q % RM;
    if (i < n && m < r) {
      double tz = fma(dS[i] - lamS[m], F(ZZ, i, m), 0.0);
      if (i > 0) tz = fma(eS[i - 1], F(ZZ, i - 1, m), tz);
      if (i + 1 < n) tz = fma(eS[i], F(ZZ, i + 1, m), tz);
      rmax = fmax(rmax, fabs(tz));
    }
  }
  if (!(emax <= 1.0)) emax = 1.0;  // NaN or large: rejected below
  if (!(rmax <= 1.0)) rmax = 1.0;
  // wave maxima first: one LDS atomic per wave instead of one per thread on a single word
  emax = wave_max_f64(emax);
  rmax = wave_max_f64(rmax);
  if (lane == 0) {
    atomicMax(&ebits, static_cast<unsigned long long>(__double_as_longlong(emax)));
    atomicMax(&rbits, static_cast<unsigned long long>(__double_as_longlong(rmax)));
  }
  __syncthreads();
  const double em = __longlong_as_double(static_cast<long long>(ebits));
  const double rm = __longlong_as_double(static_cast<long long>(rbits));
  if (!(em <= 1e-6 && rm <= 1e-12 * bounds[2])) return false;  // uniform
  if (em > 32.0 * 2.220446049250313e-16) {
    // one Loewdin step Z <- Z (I - E/2 + 3 E^2 / 8): orthonormal to O(|E|^3)
    for (int q = tid; q < r * r; q += kJThreads) {
      const int a = q / r, c = q - (q / r) * r;
      double sacc = 0.0;
      for (int b2 = 0; b2 < r; ++b2) sacc = fma(E[a * (RM + 1) + b2], E[b2 * (RM + 1) + c], sacc);
      Fm[a * (RM + 1) + c] = fma(0.375, sacc, fma(-0.5, E[a * (RM + 1) + c], a == c ? 1.0 : 0.0));
    }
    __syncthreads();
    double zn[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int q = tid + t * kJThreads;
      const int i = q / RM, m = q % RM;
      double sacc = 0.0;
      if (i < n && m < r)
        for (int c = 0; c < r; ++c) sacc = fma(F(ZZ, i, c), Fm[c * (RM + 1) + m], sacc);
      zn[t] = sacc;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int q = tid + t * kJThreads;
      const int i = q / RM, m = q % RM;
      if (i < n && m < r) F(ZZ, i, m) = zn[t];
    }
    __syncthreads();
  }
  // ---- 5. V = H_0 ... H_{n-3} Z: 16 lanes per column, 4 rows per lane, reflectors applied
  //         last to first, two per reduction round, with the next pair's entries loaded
  //         ahead; then the sign rule
  //         (largest |entry|, first on ties, positive) by a group argmax.
  {
    const int gm = tid / kPairLanes, sb = tid % kPairLanes;
    double zr[kPairRows];
#pragma unroll
    for (int t = 0; t < kPairRows; ++t) {
      const int row = kPairRows * sb + t;
      zr[t] = (gm < r && row < n) ? F(ZZ, row, gm) : 0.0;
    }
    const auto vload = [&](int k, double (&vr)[kPairRows]) {
#pragma unroll
      for (int t = 0; t < kPairRows; ++t) {
        const int row = kPairRows * sb + t;
        const double a = Am[row * kAStride + k];
        vr[t] = (row == k + 1) ? 1.0 : ((row > k + 1 && row < n) ? a : 0.0);
      }
    };
    // reflectors n - 3 .. 0; an odd one out goes first, the rest in pairs (k, k - 1):
    // with a = v_k^T z, b = v_{k-1}^T z and c = v_{k-1}^T v_k from one reduction round,
    // H_{k-1} H_k z = z - f_k v_k - f_{k-1} v_{k-1}, f_k = tau_k a,
    // f_{k-1} = tau_{k-1} (b - f_k c)
    int k = n - 3;
    if ((n - 2) & 1) {
      double vr[kPairRows];
      vload(k, vr);
      double sacc = 0.0;
#pragma unroll
      for (int t = 0; t < kPairRows; ++t) sacc = fma(vr[t], zr[t], sacc);
      const double f = tauS[k] * group16_sum(sacc);
#pragma unroll
      for (int t = 0; t < kPairRows; ++t) zr[t] = fma(-f, vr[t], zr[t]);
      --k;
    }
    double na[kPairRows], nb[kPairRows];
    double nta = 0.0, ntb = 0.0;
    if (k >= 1) {
      vload(k, na);
      vload(k - 1, nb);
      nta = tauS[k];
      ntb = tauS[k - 1];
    }
    for (; k >= 1; k -= 2) {
      double va[kPairRows], vb[kPairRows];
#pragma unroll
      for (int t = 0; t < kPairRows; ++t) {
        va[t] = na[t];
        vb[t] = nb[t];
      }
      const double ta = nta, tb = ntb;
      if (k >= 3) {
        vload(k - 2, na);
        vload(k - 3, nb);
        nta = tauS[k - 2];
        ntb = tauS[k - 3];
      }
      double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
      for (int t = 0; t < kPairRows; ++t) {
        a = fma(va[t], zr[t], a);
        b = fma(vb[t], zr[t], b);
        c = fma(vb[t], va[t], c);
      }
      group16_sum3(a, b, c);
      const double fa = ta * a;
      const double fb = tb * fma(-fa, c, b);
#pragma unroll
      for (int t = 0; t < kPairRows; ++t) zr[t] = fma(-fb, vb[t], fma(-fa, va[t], zr[t]));
    }
    // group argmax of |entry| with the first row on ties
    double best = -1.0;
    int brow = kJN;
    double bval = 0.0;
#pragma unroll
    for (int t = 0; t < kPairRows; ++t) {
      const int row = kPairRows * sb + t;
      if (row < n && fabs(zr[t]) > best) {
        best = fabs(zr[t]);
        brow = row;
        bval = zr[t];
      }
    }
#define RT_STEP(CTRL)                                                        \
  {                                                                          \
    const double ob = dpp_f64<CTRL>(best);                                   \
    const int orow = __builtin_amdgcn_mov_dpp(brow, CTRL, 0xF, 0xF, true);   \
    const double ov = dpp_f64<CTRL>(bval);                                   \
    if (ob > best || (ob == best && orow < brow)) {                          \
      best = ob;                                                             \
      brow = orow;                                                           \
      bval = ov;                                                             \
    }                                                                        \
  }
    RT_STEP(0xB1)
    RT_STEP(0x4E)
    RT_STEP(0x141)
    RT_STEP(0x140)
#undef RT_STEP
    const double sg = (bval < 0.0) ? -1.0 : 1.0;
    if (gm < r) {
#pragma unroll
      for (int t = 0; t < kPairRows; ++t) {
        const int row = kPairRows * sb + t;
        if (row < n) Vout[row * r + gm] = sg * zr[t];
      }
    }
  }
  if (evals && tid < r) evals[tid] = __builtin_amdgcn_ldexp(lamS[tid], ex);
  return true;
}

template <int RM>
__device__ __forceinline__ void eig_body(const double* __restrict__ M, int n, int r, double* __restrict__ Vout,
                                         double* __restrict__ evals) {
  __shared__ __align__(16) double Am[kJN * kAStride];
  static_assert(5 * kJN * RM >= kJN * kLStride, "Jacobi columns must fit the tridiagonal scratch");
  static_assert(5 * kJN * RM >= 4 * kP1MaxWaves * kJN + 2 * kJN, "phase-1 scratch must fit");
  __shared__ __align__(16) double B[5 * kJN * RM];
  if (n >= 3 && r <= RM) {
    if (eig_tridiag<RM>(M, n, r, Vout, evals, Am, B)) return;
    __syncthreads();
  }
  eig_jacobi(M, n, r, Vout, evals, Am, B);
}

__global__ __launch_bounds__(kJThreads) void eig_onesided_kernel(const double* __restrict__ M, int n, int r,
                                                                 double* __restrict__ Vout,
                                                                 double* __restrict__ evals) {
  eig_body<kTriMaxR>(M, n, r, Vout, evals);
}

// RM = 16 (every job r <= 16) halves the scratch, so two workgroups share a CU
template <int RM>
__global__ __launch_bounds__(kJThreads) void eig_grouped_kernel(const GEigJob* __restrict__ jobs) {
  const GEigJob J = jobs[blockIdx.x];
  eig_body<RM>(J.M, J.n, J.r, J.V, nullptr);
}

}  // namespace

size_t mode_contract_ws(rt_dtype dt, int64_t A, int64_t mP, int64_t mQ, int64_t B) {
  const MCPlan p = mc_plan(dt, A, mP, mQ, B);
  return align256(static_cast<size_t>(p.nchunks) * p.tilesP * p.tilesQ * kMCTile * kMCTile * dtype_size(dt));
}

namespace {
struct WidePlan {
  int tiles1;
  int upper;      // tiles on or above the diagonal
  int64_t chunk;  // t per workgroup, a multiple of 64
  int nchunks;
};
WidePlan wide_plan(int64_t A, int64_t m, int64_t B) {
  WidePlan p;
  p.tiles1 = static_cast<int>(ceil_div(m, kMCTile));
  p.upper = p.tiles1 * (p.tiles1 + 1) / 2;
  const int64_t total = A * B;
  // at most 4096 working workgroups (four rounds of four per CU, none left for a short
  // fifth), at least 64 t each
  int64_t want = 4096 / p.upper;
  if (want < 1) want = 1;
  int64_t chunk = ceil_div(total, want);
  if (chunk < kGWT) chunk = kGWT;
  chunk = ceil_div(chunk, kGWT) * kGWT;
  p.chunk = chunk;
  p.nchunks = static_cast<int>(ceil_div(total, chunk));
  if (p.nchunks < 1) p.nchunks = 1;
  return p;
}
}  // namespace

size_t gram_wide_ws(int64_t A, int64_t m, int64_t B) {
  const WidePlan p = wide_plan(A, m, B);
  return align256(static_cast<size_t>(p.nchunks) * p.tiles1 * p.tiles1 * kMCTile * kMCTile * sizeof(double));
}

hipError_t launch_gram_wide(const float* X, int64_t A, int64_t m, int64_t B, double* out, void* ws, hipStream_t st) {
  const WidePlan p = wide_plan(A, m, B);
  const int64_t work = static_cast<int64_t>(p.upper) * p.nchunks;
  const int64_t blocks = ceil_div(work, static_cast<int64_t>(kXcds)) * kXcds;  // whole XCD rows
  // 16-byte loads when rows hold whole groups of four and X is 16-byte aligned
  const bool vec = (B % 4 == 0) && (reinterpret_cast<uintptr_t>(X) & 15u) == 0;
  const unsigned nb = static_cast<unsigned>(blocks);
  double* part = static_cast<double*>(ws);
  if (vec)
    gram_wide_kernel<kGWVec><<<nb, kMCThreads, 0, st>>>(X, A, m, B, p.chunk, p.tiles1, p.upper, work, part);
  else if (B >= kGWT)
    gram_wide_kernel<kGWTFast><<<nb, kMCThreads, 0, st>>>(X, A, m, B, p.chunk, p.tiles1, p.upper, work, part);
  else
    gram_wide_kernel<kGWRowFast><<<nb, kMCThreads, 0, st>>>(X, A, m, B, p.chunk, p.tiles1, p.upper, work, part);
  const unsigned g2 = static_cast<unsigned>(ceil_div(m * m * 16, 256));
  gram_wide_reduce<<<g2, 256, 0, st>>>(static_cast<const double*>(ws), p.nchunks, p.tiles1, m, out);
  return hipGetLastError();
}

hipError_t launch_mode_contract(const void* P, const void* Q, rt_dtype dt, int64_t A, int64_t mP, int64_t mQ,
                                int64_t B, void* out, void* ws, hipStream_t st, bool accumulate) {
  const MCPlan p = mc_plan(dt, A, mP, mQ, B);
  const int tiles = p.tilesP * p.tilesQ;
  const dim3 grid(tiles, p.nchunks);
  const int64_t n = mP * mQ;
  const unsigned g2 = static_cast<unsigned>(ceil_div(n * 16, 256));
  if (dt == RT_F64) {
    mode_contract_kernel<double><<<grid, kMCThreads, 0, st>>>(static_cast<const double*>(P),
                                                              static_cast<const double*>(Q), A, mP, mQ, B, p.chunk,
                                                              p.tilesQ, static_cast<double*>(ws));
    mode_contract_reduce<double><<<g2, 256, 0, st>>>(static_cast<const double*>(ws), p.nchunks, tiles, p.tilesQ, mP,
                                                     mQ, accumulate, static_cast<double*>(out));
  } else {
    mode_contract_mfma_kernel<<<grid, 256, 0, st>>>(static_cast<const float*>(P), static_cast<const float*>(Q), A,
                                                    mP, mQ, B, p.chunk, p.tilesQ, static_cast<float*>(ws));
    mode_contract_reduce<float><<<g2, 256, 0, st>>>(static_cast<const float*>(ws), p.nchunks, tiles, p.tilesQ, mP,
                                                    mQ, accumulate, static_cast<float*>(out));
  }
  return hipGetLastError();
}

namespace {
struct SmallGemmTable {
  SmallGemmJob j[kMaxSmallGemm];
};
constexpr int kSGRows = 64;
constexpr int kSGStride = 66;  // even row stride keeps the double2 reads aligned
// 64 rows of C per workgroup, 4 x 4 outputs per thread, operands staged in LDS
__global__ __launch_bounds__(256) void small_gemm_f64_kernel(SmallGemmTable tab) {
  __shared__ __align__(16) double sa[kSGRows][kSGStride];
  __shared__ __align__(16) double sb[64][kSGStride];
  const SmallGemmJob& J = tab.j[blockIdx.y];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kSGRows;
  if (r0 >= J.m) return;
  // all global loads of both operands are issued before the first LDS store
  constexpr int kPer = kSGRows * 64 / 256;
  double va[kPer], vb[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int idx = static_cast<int>(threadIdx.x) + 256 * q;
    const int rr = idx / 64, c = idx % 64;
    va[q] = (r0 + rr < J.m && c < J.k) ? J.A[(r0 + rr) * J.k + c] : 0.0;
    vb[q] = (rr < J.k && c < J.n) ? J.B[static_cast<int64_t>(rr) * J.n + c] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int idx = static_cast<int>(threadIdx.x) + 256 * q;
    sa[idx / 64][idx % 64] = va[q];
    sb[idx / 64][idx % 64] = vb[q];
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
#pragma unroll 4
  for (int t = 0; t < J.k; ++t) {
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = sa[4 * ty + u][t];
    const double2 b0 = *reinterpret_cast<const double2*>(&sb[t][4 * tx]);
    const double2 b1 = *reinterpret_cast<const double2*>(&sb[t][4 * tx + 2]);
    const double b[4] = {b0.x, b0.y, b1.x, b1.y};
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = r0 + 4 * ty + u;
    if (r >= J.m) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * tx + v < J.n) J.C[r * J.n + 4 * tx + v] = acc[u][v];
  }
}
}  // namespace

hipError_t launch_small_gemm_f64(const SmallGemmJob* jobs, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxSmallGemm) return hipErrorInvalidValue;
  SmallGemmTable tab;
  int64_t mmax = 0;
  for (int i = 0; i < count; ++i) {
    if (jobs[i].k > 64 || jobs[i].n > 64 || jobs[i].k < 1 || jobs[i].n < 1) return hipErrorInvalidValue;
    tab.j[i] = jobs[i];
    if (jobs[i].m > mmax) mmax = jobs[i].m;
  }
  const dim3 grid(static_cast<unsigned>(ceil_div(mmax, kSGRows)), static_cast<unsigned>(count));
  small_gemm_f64_kernel<<<grid, 256, 0, st>>>(tab);
  return hipGetLastError();
}

// ------------------------------------------------------------------ subspace iteration pieces
// (eigenvectors of the large Gram matrices of the deterministic STHOSVD, n > 64)

// Q[i][c] = fixed pseudo-random start block (n x b), MurmurHash3 finaliser of (i, c)
__global__ __launch_bounds__(256) void subspace_start_kernel(double* __restrict__ Q, int64_t n, int b) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t >= n * b) return;
  uint32_t h = static_cast<uint32_t>(t * 2654435761ull + 12345u);
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  Q[t] = static_cast<double>(h) * 0x1p-32 - 0.5;
}

// out[0] = max_i ||MV[:, i] - theta_i V[:, i]|| / theta_0 (MV, V: n x r row-major), one
// workgroup: thread c % r sums column c over every (256 / r)-th row, fixed order
__global__ __launch_bounds__(256) void ritz_residual_kernel(const double* __restrict__ MV,
                                                            const double* __restrict__ V,
                                                            const double* __restrict__ theta, int64_t n, int r,
                                                            double* __restrict__ out) {
  __shared__ double part[256];
  const int t = threadIdx.x;
  const int per = 256 / r;  // row groups
  double acc = 0.0;
  const int c = t % r, g = t / r;
  if (g < per)
    for (int64_t i = g; i < n; i += per) {
      const double d = MV[i * r + c] - theta[c] * V[i * r + c];
      acc = fma(d, d, acc);
    }
  part[t] = (g < per) ? acc : 0.0;
  __syncthreads();
  if (t == 0) {
    double worst = 0.0;
    for (int cc = 0; cc < r; ++cc) {
      double s = 0.0;
      for (int gg = 0; gg < per; ++gg) s += part[gg * r + cc];
      worst = fmax(worst, sqrt(s));
    }
    out[0] = worst / fmax(fabs(theta[0]), 1e-300);
  }
}

// make every column's largest-magnitude entry (first on ties) positive; one wave per column
__global__ __launch_bounds__(64) void column_sign_kernel(double* __restrict__ V, int64_t n, int r) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  double best = -1.0;
  int64_t where = 0;
  for (int64_t i = lane; i < n; i += 64) {
    const double a = fabs(V[i * r + c]);
    if (a > best) { best = a; where = i; }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int64_t ow = __shfl_xor(where, off);
    if (ob > best || (ob == best && ow < where)) { best = ob; where = ow; }
  }
  const bool flip = V[where * r + c] < 0.0;
  if (flip)
    for (int64_t i = lane; i < n; i += 64) V[i * r + c] = -V[i * r + c];
}

hipError_t launch_subspace_start(double* Q, int64_t n, int b, hipStream_t st) {
  subspace_start_kernel<<<static_cast<unsigned>(ceil_div(n * b, 256)), 256, 0, st>>>(Q, n, b);
  return hipGetLastError();
}

hipError_t launch_ritz_residual(const double* MV, const double* V, const double* theta, int64_t n, int r,
                                double* out, hipStream_t st) {
  ritz_residual_kernel<<<1, 256, 0, st>>>(MV, V, theta, n, r, out);
  return hipGetLastError();
}

hipError_t launch_column_sign(double* V, int64_t n, int r, hipStream_t st) {
  column_sign_kernel<<<static_cast<unsigned>(r), 64, 0, st>>>(V, n, r);
  return hipGetLastError();
}

hipError_t launch_sym_eig_top(const double* M, int64_t n, int64_t r, double* V, double* evals, hipStream_t st) {
  eig_onesided_kernel<<<1, kJThreads, 0, st>>>(M, static_cast<int>(n), static_cast<int>(r), V, evals);
  return hipGetLastError();
}

hipError_t launch_gram_grouped(const GGramJob* jobs, int count, hipStream_t st, int max_m) {
  if (count == 0) return hipSuccess;
  if (max_m <= 32)
    gram_small_grouped_kernel<<<static_cast<unsigned>(count), kMCThreads, 0, st>>>(jobs);
  else
    gram_grouped_kernel<<<static_cast<unsigned>(count), kMCThreads, 0, st>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_eig_grouped(const GEigJob* jobs, int count, hipStream_t st, int max_r) {
  if (count == 0) return hipSuccess;
  if (max_r <= 16)
    eig_grouped_kernel<16><<<static_cast<unsigned>(count), kJThreads, 0, st>>>(jobs);
  else
    eig_grouped_kernel<kTriMaxR><<<static_cast<unsigned>(count), kJThreads, 0, st>>>(jobs);
  return hipGetLastError();
}

}  // namespace rt

// Core truncation pieces (Alg. 2.2 applied to the small core, Sec. 3.1):
//  * mode contraction out = P_(n) Q_(n)^T on (A, m, B) views, which gives the
//    Gram matrix G_(j) G_(j)^T of the core (P = Q) and the adjoint dA_n;
//    fixed-order two-stage reduction, so results are bitwise reproducible;
//  * a symmetric eigensolver for the <= 64 x 64 Gram matrices: parallel cyclic
//    Jacobi (round-robin pairing, all disjoint rotations of a round applied at
//    once as 2x2 block updates) in binary64, in one workgroup with the matrix and
//    the eigenvector accumulator in LDS.
#include "kernels.hpp"

namespace rt {

namespace {

// ------------------------------------------------------------------ mode contraction
constexpr int kMCTile = 64;
constexpr int kMCK = 16;
constexpr int kMCThreads = 256;

template <typename T>
__global__ __launch_bounds__(kMCThreads) void mode_contract_kernel(const T* __restrict__ P, const T* __restrict__ Q,
                                                                   int64_t A, int64_t mP, int64_t mQ, int64_t B,
                                                                   int64_t chunk, int tilesQ, T* __restrict__ part) {
  __shared__ T sP[kMCK][kMCTile + 1];
  __shared__ T sQ[kMCK][kMCTile + 1];
  const int tile = blockIdx.x;
  const int ti = tile / tilesQ, tj = tile % tilesQ;
  const int64_t i0 = static_cast<int64_t>(ti) * kMCTile, j0 = static_cast<int64_t>(tj) * kMCTile;
  const int64_t total = A * B;
  const int64_t t0 = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t t1 = (t0 + chunk < total) ? t0 + chunk : total;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;  // 4x4 outputs per thread
  T acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
  const bool tfast = B >= kMCK;  // choose the loading order that follows memory
  for (int64_t tb = t0; tb < t1; tb += kMCK) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kMCK * kMCTile; idx += kMCThreads) {
      int tt, ii;
      if (tfast) { tt = idx % kMCK; ii = idx / kMCK; } else { ii = idx % kMCTile; tt = idx / kMCTile; }
      const int64_t t = tb + tt;
      T pv = T(0), qv = T(0);
      if (t < t1) {
        const int64_t a = t / B, b = t - a * B;
        if (i0 + ii < mP) pv = P[a * mP * B + (i0 + ii) * B + b];
        if (j0 + ii < mQ) qv = Q[a * mQ * B + (j0 + ii) * B + b];
      }
      sP[tt][ii] = pv;
      sQ[tt][ii] = qv;
    }
    __syncthreads();
#pragma unroll 4
    for (int tt = 0; tt < kMCK; ++tt) {
      T pv[4], qv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pv[u] = sP[tt][ty * 4 + u];
#pragma unroll
      for (int v = 0; v < 4; ++v) qv[v] = sQ[tt][tx * 4 + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(pv[u], qv[v], acc[u][v]);
    }
  }
  T* out = part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + tile) * kMCTile * kMCTile;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(ty * 4 + u) * kMCTile + tx * 4 + v] = acc[u][v];
}

template <typename T>
__global__ __launch_bounds__(256) void mode_contract_reduce(const T* __restrict__ part, int nchunks, int tiles,
                                                            int tilesQ, int64_t mP, int64_t mQ, T* __restrict__ out) {
  const int64_t total = mP * mQ;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * 256) {
    const int64_t i = idx / mQ, j = idx - i * mQ;
    const int tile = static_cast<int>((i / kMCTile) * tilesQ + (j / kMCTile));
    const int64_t off = (i % kMCTile) * kMCTile + (j % kMCTile);
    T s = T(0);
    for (int c = 0; c < nchunks; ++c) s += part[(static_cast<int64_t>(c) * tiles + tile) * kMCTile * kMCTile + off];
    out[idx] = s;
  }
}

struct MCPlan {
  int tilesP, tilesQ, nchunks;
  int64_t chunk;
};

MCPlan mc_plan(int64_t A, int64_t mP, int64_t mQ, int64_t B) {
  MCPlan p;
  p.tilesP = static_cast<int>(ceil_div(mP, kMCTile));
  p.tilesQ = static_cast<int>(ceil_div(mQ, kMCTile));
  const int64_t total = A * B;
  int64_t want = 512 / (p.tilesP * p.tilesQ);
  if (want < 1) want = 1;
  int64_t chunk = ceil_div(total, want);
  if (chunk < 1024) chunk = 1024;
  chunk = ceil_div(chunk, kMCK) * kMCK;
  p.chunk = chunk;
  p.nchunks = static_cast<int>(ceil_div(total, chunk));
  if (p.nchunks < 1) p.nchunks = 1;
  return p;
}

// ------------------------------------------------------------------ Jacobi
constexpr int kJN = 64;
constexpr int kJThreads = 256;
constexpr int kMaxSweeps = 40;

__global__ __launch_bounds__(kJThreads) void jacobi_eig_kernel(const double* __restrict__ M, int n, int r,
                                                               double* __restrict__ Vout, double* __restrict__ evals) {
  __shared__ double Am[kJN][kJN + 1];
  __shared__ double Vm[kJN][kJN + 1];
  __shared__ double cs[kJN / 2], sn[kJN / 2];
  __shared__ int pp[kJN / 2], qq[kJN / 2];
  __shared__ int rotated;
  __shared__ int order[kJN];
  const int N = n + (n & 1);  // even number of players; index n is a zero dummy when n is odd
  const int half = N / 2;
  for (int idx = threadIdx.x; idx < kJN * kJN; idx += kJThreads) {
    const int i = idx / kJN, j = idx % kJN;
    Am[i][j] = (i < n && j < n) ? M[i * n + j] : 0.0;
    Vm[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps && N > 1; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < N - 1; ++round) {
      // phase 1: rotation of each disjoint pair (circle method pairing)
      if (threadIdx.x < half) {
        const int i = threadIdx.x;
        const int a = (i == 0) ? 0 : ((i - 1 + round) % (N - 1)) + 1;
        const int k2 = N - 1 - i;
        const int b = ((k2 - 1 + round) % (N - 1)) + 1;
        const int p = a < b ? a : b, q = a < b ? b : a;
        const double apq = Am[p][q], app = Am[p][p], aqq = Am[q][q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300 && fabs(apq) > 1e-16 * sqrt(fabs(app) * fabs(aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          rotated = 1;
        }
        cs[i] = c; sn[i] = s; pp[i] = p; qq[i] = q;
      }
      __syncthreads();
      // phase 2: A <- J^T A J as 2x2 blocks, V <- V J
      for (int blk = threadIdx.x; blk < half * half; blk += kJThreads) {
        const int P = blk / half, Qi = blk % half;
        const int p1 = pp[P], q1 = qq[P], p2 = pp[Qi], q2 = qq[Qi];
        const double c1 = cs[P], s1 = sn[P], c2 = cs[Qi], s2 = sn[Qi];
        const double m11 = Am[p1][p2], m12 = Am[p1][q2], m21 = Am[q1][p2], m22 = Am[q1][q2];
        // rows
        const double r11 = c1 * m11 - s1 * m21, r12 = c1 * m12 - s1 * m22;
        const double r21 = s1 * m11 + c1 * m21, r22 = s1 * m12 + c1 * m22;
        // columns
        double n11 = c2 * r11 - s2 * r12, n12 = s2 * r11 + c2 * r12;
        double n21 = c2 * r21 - s2 * r22, n22 = s2 * r21 + c2 * r22;
        if (P == Qi && s1 != 0.0) { n12 = 0.0; n21 = 0.0; }
        Am[p1][p2] = n11; Am[p1][q2] = n12; Am[q1][p2] = n21; Am[q1][q2] = n22;
      }
      for (int it = threadIdx.x; it < N * half; it += kJThreads) {
        const int x = it / half, P = it % half;
        const int p = pp[P], q = qq[P];
        const double c = cs[P], s = sn[P];
        const double vp = Vm[x][p], vq = Vm[x][q];
        Vm[x][p] = c * vp - s * vq;
        Vm[x][q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // order eigenvalues decreasing (ties by index)
  if (threadIdx.x < n) {
    const int i = threadIdx.x;
    const double li = Am[i][i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = Am[j][j];
      if (lj > li || (lj == li && j < i)) ++rank;
    }
    order[rank] = i;
  }
  __syncthreads();
  if (evals && threadIdx.x < n) evals[threadIdx.x] = Am[order[threadIdx.x]][order[threadIdx.x]];
  // output columns with the sign rule: largest |entry| (first on ties) positive
  if (threadIdx.x < r) {
    const int k = threadIdx.x, col = order[k];
    double best = -1.0, sgn = 1.0;
    for (int x = 0; x < n; ++x) {
      const double v = Vm[x][col];
      if (fabs(v) > best) { best = fabs(v); sgn = (v < 0.0) ? -1.0 : 1.0; }
    }
    for (int x = 0; x < n; ++x) Vout[x * r + k] = sgn * Vm[x][col];
  }
}

}  // namespace

size_t mode_contract_ws(rt_dtype dt, int64_t A, int64_t mP, int64_t mQ, int64_t B) {
  const MCPlan p = mc_plan(A, mP, mQ, B);
  return align256(static_cast<size_t>(p.nchunks) * p.tilesP * p.tilesQ * kMCTile * kMCTile * dtype_size(dt));
}

hipError_t launch_mode_contract(const void* P, const void* Q, rt_dtype dt, int64_t A, int64_t mP, int64_t mQ,
                                int64_t B, void* out, void* ws, hipStream_t st) {
  const MCPlan p = mc_plan(A, mP, mQ, B);
  const int tiles = p.tilesP * p.tilesQ;
  const dim3 grid(tiles, p.nchunks);
  const int64_t n = mP * mQ;
  const unsigned g2 = static_cast<unsigned>(ceil_div(n, 256) > 1024 ? 1024 : ceil_div(n, 256));
  if (dt == RT_F64) {
    mode_contract_kernel<double><<<grid, kMCThreads, 0, st>>>(static_cast<const double*>(P),
                                                              static_cast<const double*>(Q), A, mP, mQ, B, p.chunk,
                                                              p.tilesQ, static_cast<double*>(ws));
    mode_contract_reduce<double><<<g2, 256, 0, st>>>(static_cast<const double*>(ws), p.nchunks, tiles, p.tilesQ, mP,
                                                     mQ, static_cast<double*>(out));
  } else {
    mode_contract_kernel<float><<<grid, kMCThreads, 0, st>>>(static_cast<const float*>(P),
                                                             static_cast<const float*>(Q), A, mP, mQ, B, p.chunk,
                                                             p.tilesQ, static_cast<float*>(ws));
    mode_contract_reduce<float><<<g2, 256, 0, st>>>(static_cast<const float*>(ws), p.nchunks, tiles, p.tilesQ, mP,
                                                    mQ, static_cast<float*>(out));
  }
  return hipGetLastError();
}

hipError_t launch_sym_eig_top(const double* M, int64_t n, int64_t r, double* V, double* evals, hipStream_t st) {
  jacobi_eig_kernel<<<1, kJThreads, 0, st>>>(M, static_cast<int>(n), static_cast<int>(r), V, evals);
  return hipGetLastError();
}

}  // namespace rt

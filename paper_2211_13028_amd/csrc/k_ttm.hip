// Mode-k tensor-times-matrix on the (A, K, B) view of a C-order tensor:
//   Y[a, i, b] = sum_k M[i, k] X[a, k, b]
// (Sec. 2.1: the mode-k unfolding of X x_k M is M times the unfolding of X).
// No unfolding is materialised: for each a, X[a] is a row-major K x B matrix,
// so the contraction is a strided-batched GEMM whose HBM reads are whole rows.
//
//  * ttm_generic: VALU kernel for every dtype and shape (one output column per
//    thread, m split into register tiles, M chunks broadcast from LDS).
//  * ttm_mfma:   matrix-core kernel for binary32 / bfloat16 X and B % 4 == 0
//    (binary32) or B % 8 == 0 (bfloat16), m <= 64.  Each wave owns a 64 x 128
//    output tile (m padded to a multiple of 16) and streams X rows once; the
//    prepared M operand is read from L2.  bfloat16 operands are re-packed in
//    registers so that each lane holds 8 consecutive k of one column.
#include "kernels.hpp"

namespace rt {

namespace {

// ------------------------------------------------------------------ generic VALU
constexpr int kGenThreads = 256;
constexpr int kGenKC = 64;

// acc[ii] += sum over k in [kb, ke) of M(i0 + ii, k) X[a, k, b] for this thread's column
// (xp = &X[a, 0, b]).  A chunk of M is staged in LDS; its global loads are all issued
// into registers before the first LDS store, and X is read kXB rows at a time, so the
// loads of a chunk are in flight together instead of one latency each.
constexpr int kXB = 8;
static_assert(kGenKC % kXB == 0, "X blocks must tile the M chunk");
template <typename TX, typename TC, int MT>
__device__ __forceinline__ void generic_accumulate(const TX* __restrict__ xp, int64_t B, const TC* __restrict__ M,
                                                   int64_t m, int64_t K, int64_t i0, int64_t kb, int64_t ke,
                                                   bool mtrans, bool active, TC (&sM)[MT][kGenKC], TC (&acc)[MT]) {
  constexpr int kPer = MT * kGenKC / kWave;  // M elements per thread at the smallest block (one wave)
  const int nth = static_cast<int>(blockDim.x);
  for (int64_t k0 = kb; k0 < ke; k0 += kGenKC) {
    TC mv[kPer];
#pragma unroll
    for (int rep = 0; rep < kPer; ++rep) {
      const int t = static_cast<int>(threadIdx.x) + rep * nth;
      const int ii = t / kGenKC, kk = t % kGenKC;
      mv[rep] = (t < MT * kGenKC && i0 + ii < m && k0 + kk < ke)
                    ? (mtrans ? M[(k0 + kk) * m + i0 + ii] : M[(i0 + ii) * K + k0 + kk])
                    : TC(0);
    }
    __syncthreads();
#pragma unroll
    for (int rep = 0; rep < kPer; ++rep) {
      const int t = static_cast<int>(threadIdx.x) + rep * nth;
      if (t < MT * kGenKC) sM[t / kGenKC][t % kGenKC] = mv[rep];
    }
    __syncthreads();
    if (active) {
      const int kend = static_cast<int>((ke - k0) < kGenKC ? (ke - k0) : kGenKC);
      for (int kk0 = 0; kk0 < kend; kk0 += kXB) {
        TC xv[kXB];
#pragma unroll
        for (int u = 0; u < kXB; ++u)
          xv[u] = (kk0 + u < kend) ? static_cast<TC>(Load<TX>::get(xp, (k0 + kk0 + u) * B)) : TC(0);
#pragma unroll
        for (int u = 0; u < kXB; ++u)
#pragma unroll
          for (int ii = 0; ii < MT; ++ii) acc[ii] = fma(sM[ii][kk0 + u], xv[u], acc[ii]);
      }
    }
  }
}

template <typename TX, typename TC, int MT>
__global__ __launch_bounds__(kGenThreads) void ttm_generic_kernel(const TX* __restrict__ X, int64_t A, int64_t K,
                                                                  int64_t B, const TC* __restrict__ M, int64_t m,
                                                                  int64_t kper, bool mtrans, TC* __restrict__ Y) {
  __shared__ TC sM[MT][kGenKC];
  const int64_t col = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t i0 = static_cast<int64_t>(blockIdx.y) * MT;
  const int64_t kb = static_cast<int64_t>(blockIdx.z) * kper;
  const int64_t ke = (kb + kper < K) ? kb + kper : K;
  const bool active = col < A * B;
  const int64_t a = active ? col / B : 0;
  const int64_t b = active ? col - a * B : 0;
  TC acc[MT];
#pragma unroll
  for (int ii = 0; ii < MT; ++ii) acc[ii] = TC(0);
  generic_accumulate<TX, TC, MT>(X + a * K * B + b, B, M, m, K, i0, kb, ke, mtrans, active, sM, acc);
  if (active) {
    TC* y = Y + static_cast<int64_t>(blockIdx.z) * A * m * B;
#pragma unroll
    for (int ii = 0; ii < MT; ++ii)
      if (i0 + ii < m) y[a * m * B + (i0 + ii) * B + b] = acc[ii];
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void generic_sum_kernel(const TC* __restrict__ part, int ksplit, int64_t n,
                                                          TC* __restrict__ Y) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
    TC s = part[i];
    for (int k = 1; k < ksplit; ++k) s += part[k * n + i];
    Y[i] = s;
  }
}

// split K over grid.z when there are too few output columns to fill the chip
int generic_ksplit(int64_t A, int64_t K, int64_t B) {
  const int64_t cols = A * B;
  int ks = 1;
  while (cols * ks < 131072 && K / (2 * ks) >= 64 && ks < 64) ks *= 2;
  return ks;
}

template <typename TX, typename TC>
hipError_t generic_dispatch(const TX* X, int64_t A, int64_t K, int64_t B, const TC* M, int64_t m, TC* Y, TC* ws,
                            hipStream_t st, bool mtrans) {
  const int64_t cols = A * B;
  // few output columns: one-wave blocks, so that more CUs share the work
  const int threads = cols < 32768 ? kWave : kGenThreads;
  const unsigned gx = static_cast<unsigned>(ceil_div(cols, threads));
  const int ks = generic_ksplit(A, K, B);
  const int64_t kper = ceil_div(K, ks);
  TC* out = (ks > 1) ? ws : Y;
  if (m <= 4 || threads == kWave) {
    // (few output columns: 4-row tiles, so that more waves share the rows of m)
    const unsigned gy = static_cast<unsigned>(ceil_div(m, 4));
    ttm_generic_kernel<TX, TC, 4><<<dim3(gx, gy, ks), threads, 0, st>>>(X, A, K, B, M, m, kper, mtrans, out);
  } else if (m <= 8) {
    const unsigned gy = static_cast<unsigned>(ceil_div(m, 8));
    ttm_generic_kernel<TX, TC, 8><<<dim3(gx, gy, ks), threads, 0, st>>>(X, A, K, B, M, m, kper, mtrans, out);
  } else {
    const unsigned gy = static_cast<unsigned>(ceil_div(m, 16));
    ttm_generic_kernel<TX, TC, 16><<<dim3(gx, gy, ks), threads, 0, st>>>(X, A, K, B, M, m, kper, mtrans, out);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  const int64_t n = A * m * B;
  const unsigned g2 = static_cast<unsigned>(ceil_div(n, 256) > 4096 ? 4096 : ceil_div(n, 256));
  generic_sum_kernel<TC><<<g2, 256, 0, st>>>(out, ks, n, Y);
  return hipGetLastError();
}

// grouped form: job found by binary search over blk0; one wave per workgroup

template <typename TX, typename TC, int MT>
__global__ __launch_bounds__(kWave) void ttm_grouped_kernel(const GTtmJob* __restrict__ jobs,
                                                             const int32_t* __restrict__ blkjob) {
  __shared__ TC sM[MT][kGenKC];
  const int64_t blk = blockIdx.x;
  const GTtmJob J = jobs[blkjob[blk]];
  const int64_t local = blk - J.blk0;
  const int64_t cb = local / J.mtiles, mtile = local - cb * J.mtiles;
  const int64_t A = J.A, K = J.K, B = J.B, m = J.m;
  const TX* X = static_cast<const TX*>(J.X);
  const TC* M = static_cast<const TC*>(J.M);
  const int64_t col = cb * kWave + threadIdx.x;
  const int64_t i0 = mtile * MT;
  const bool active = col < A * B;
  const int64_t a = active ? col / B : 0;
  const int64_t b = active ? col - a * B : 0;
  TC acc[MT];
#pragma unroll
  for (int ii = 0; ii < MT; ++ii) acc[ii] = TC(0);
  // compact loops (few registers, several waves per SIMD for the many small jobs of a batch)
  const TX* xp = X + a * K * B + b;
  for (int64_t k0 = 0; k0 < K; k0 += kGenKC) {
    __syncthreads();
    for (int t = threadIdx.x; t < MT * kGenKC; t += kWave) {
      const int ii = t / kGenKC, kk = t % kGenKC;
      sM[ii][kk] = (i0 + ii < m && k0 + kk < K) ? (J.mtrans ? M[(k0 + kk) * m + i0 + ii] : M[(i0 + ii) * K + k0 + kk])
                                                : TC(0);
    }
    __syncthreads();
    if (active) {
      const int kend = static_cast<int>((K - k0) < kGenKC ? (K - k0) : kGenKC);
      for (int kk = 0; kk < kend; ++kk) {
        const TC x = static_cast<TC>(Load<TX>::get(xp, (k0 + kk) * B));
#pragma unroll
        for (int ii = 0; ii < MT; ++ii) acc[ii] = fma(sM[ii][kk], x, acc[ii]);
      }
    }
  }
  if (active) {
    TC* y = static_cast<TC*>(J.Y);
#pragma unroll
    for (int ii = 0; ii < MT; ++ii)
      if (i0 + ii < m) y[a * m * B + (i0 + ii) * B + b] = acc[ii];
  }
}

// ------------------------------------------------------------------ MFMA
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaThreads = 256;  // 4 waves, one 128-column unit each
constexpr int kUnitCols = 128;

// Work unit = (a, 128-column chunk, k-split part).  Y (or a split-K partial) is
// written for rows i < m only.
// One work unit (a wave) of the binary32 contraction; unit < A * chunks * ksplit.
// TAIL > 0 (with VM): rows 16 MT .. 16 MT + TAIL - 1 of M are not a whole 16-row matrix-core
// tile, and are multiplied on the vector ALU from the X values the lane already holds
// (m = 49 = 3 x 16 + 1 would otherwise pad a fourth tile: 31 % more matrix-core work).
template <int MT, bool VM, int TAIL = 0, int DEPTH = 3>
__device__ __forceinline__ void ttm_f32_unit(const float* __restrict__ X, int64_t A, int64_t K, int64_t B,
                                             const float* __restrict__ Mop, int64_t m, int64_t chunks, int ksplit,
                                             int64_t kper, float* __restrict__ Y, int64_t unit) {
  static_assert(TAIL == 0 || VM, "vector-ALU tail rows need K % 4 == 0");
  const int lane = threadIdx.x % kWave;
  const int ks = static_cast<int>(unit % ksplit);
  const int64_t ac = unit / ksplit;
  const int64_t a = ac / chunks;
  const int64_t b0 = (ac - a * chunks) * kUnitCols;
  const int j = lane % 16, q = lane / 16;
  const int64_t kbeg = ks * kper;
  const int64_t kend = (kbeg + kper < K) ? kbeg + kper : K;

  f32x4 acc[MT][2][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[mt][g][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const float* xa = X + a * K * B;
  const bool colok0 = (b0 + 4 * j) < B;
  const bool colok1 = (b0 + 64 + 4 * j) < B;
  // The wave takes k in blocks of 16.  Product s of a block sums over the four k that
  // lane groups q = 0..3 hold, k = k0 + 4 q + s, so a lane's share of the M tile for the
  // whole block is four consecutive k: one 16-byte load per tile when K % 4 == 0 (VM).
  // The lane loads the X rows k0 + 4 q + s (s = 0..3), columns b0 + 4 j .. and
  // b0 + 64 + 4 j ...  Loads carry no conditions: a row past kend reads row kend - 1 and
  // is zeroed before use, and a lane past B reads column b0 (its products land only in
  // output columns that are not stored).
  const int64_t c0off = colok0 ? b0 + 4 * j : b0, c1off = colok1 ? b0 + 64 + 4 * j : b0;
  const f32x4 zero4 = f32x4{0.f, 0.f, 0.f, 0.f};
  // DEPTH blocks in flight: set P holds the block DEPTH steps ahead of the one multiplied
  static_assert(DEPTH >= 1 && DEPTH <= 4, "one to four blocks ahead (four measured slower than three: registers)");
  f32x4 n0[DEPTH][4], n1[DEPTH][4];
  float nw[DEPTH][MT][4];
  f32x4 ntw[DEPTH][TAIL > 0 ? TAIL : 1];
  f32x4 tacc[TAIL > 0 ? TAIL : 1][2];
#pragma unroll
  for (int r = 0; r < TAIL; ++r) tacc[r][0] = tacc[r][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  const auto load_block = [&](int64_t k0, auto Pc) {
    constexpr int P = decltype(Pc)::value;
    const int64_t kl = k0 + 4 * q;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t kc = (kl + s < kend) ? kl + s : kend - 1;
      n0[P][s] = *reinterpret_cast<const f32x4*>(xa + kc * B + c0off);
      n1[P][s] = *reinterpret_cast<const f32x4*>(xa + kc * B + c1off);
    }
    if constexpr (VM) {
      // kl is a multiple of 4, so kl < kend <= K gives kl <= K - 4; a block past K reads
      // the last four k of the row instead (zeroed before use)
      const int64_t km = (kl <= K - 4) ? kl : K - 4;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(Mop + (mt * 16 + j) * K + km);
#pragma unroll
        for (int s = 0; s < 4; ++s) nw[P][mt][s] = v[s];
      }
#pragma unroll
      for (int r = 0; r < TAIL; ++r) ntw[P][r] = *reinterpret_cast<const f32x4*>(Mop + (MT * 16 + r) * K + km);
    } else {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int s = 0; s < 4; ++s) nw[P][mt][s] = Mop[(mt * 16 + j) * K + ((kl + s < kend) ? kl + s : kend - 1)];
    }
  };
  const auto block = [&](int64_t k0, auto Pc) {
    constexpr int P = decltype(Pc)::value;
    f32x4 y0[4], y1[4];
    float w[4][MT];
    f32x4 tw[TAIL > 0 ? TAIL : 1];
    const int64_t kl = k0 + 4 * q;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool kin = kl + s < kend;
      y0[s] = kin ? n0[P][s] : zero4;
      y1[s] = kin ? n1[P][s] : zero4;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) w[s][mt] = kin ? nw[P][mt][s] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < TAIL; ++r) tw[r] = ntw[P][r];
    // the block DEPTH steps ahead goes out before this block's products (the scheduler may
    // move neither the operand take-over below it nor it into the products)
    __builtin_amdgcn_sched_barrier(0);
    load_block(k0 + 16 * DEPTH, Pc);  // past kend: rows kend - 1 again, never used
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[mt][0][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[s][mt], y0[s][t], acc[mt][0][t], 0, 0, 0);
          acc[mt][1][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[s][mt], y1[s][t], acc[mt][1][t], 0, 0, 0);
        }
      }
    }
    // tail rows: the lane's four k of the block against its eight columns (y past kend
    // are zero, and the clamped loads of the tail rows are finite)
#pragma unroll
    for (int r = 0; r < TAIL; ++r)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          tacc[r][0][c] = fmaf(tw[r][s], y0[s][c], tacc[r][0][c]);
          tacc[r][1][c] = fmaf(tw[r][s], y1[s][c], tacc[r][1][c]);
        }
  };
  constexpr auto sets = std::make_integer_sequence<int, DEPTH>{};
  if (kbeg < kend) for_each_index([&](auto Pc) { load_block(kbeg + 16 * decltype(Pc)::value, Pc); }, sets);
  for (int64_t k0 = kbeg; k0 < kend; k0 += 16 * DEPTH)
    for_each_index(
        [&](auto Pc) {
          const int64_t kb = k0 + 16 * decltype(Pc)::value;
          if (kb < kend) block(kb, Pc);
        },
        sets);
  float* ya = Y + (static_cast<int64_t>(ks) * A + a) * m * B;
  // tail rows: the four lane groups q hold the partial sums of k = 4 q + s of every block;
  // add them in a fixed order (lane j collects groups 0..3) and store from group 0
#pragma unroll
  for (int r = 0; r < TAIL; ++r) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      f32x4 v = tacc[r][g];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float p1 = __shfl(v[c], j + 16), p2 = __shfl(v[c], j + 32), p3 = __shfl(v[c], j + 48);
        v[c] = ((v[c] + p1) + p2) + p3;
      }
      const int64_t i = MT * 16 + r;
      const int64_t c0 = b0 + 64 * g + 4 * j;
      if (q == 0 && i < m && c0 < B) *reinterpret_cast<f32x4*>(ya + i * B + c0) = v;
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = mt * 16 + 4 * q + v;
      if (i >= m) continue;
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int64_t c = b0 + 64 * g + 4 * j;
        if (c < B) {
          f32x4 o = f32x4{acc[mt][g][0][v], acc[mt][g][1][v], acc[mt][g][2][v], acc[mt][g][3][v]};
          *reinterpret_cast<f32x4*>(ya + i * B + c) = o;
        }
      }
    }
  }
}

template <int MT, bool VM, int TAIL = 0>
__global__ __launch_bounds__(kMfmaThreads) void ttm_mfma_f32_kernel(const float* __restrict__ X, int64_t A, int64_t K,
                                                                    int64_t B, const float* __restrict__ Mop,
                                                                    int64_t m, int64_t chunks, int ksplit,
                                                                    int64_t kper, float* __restrict__ Y) {
  const int64_t unit = static_cast<int64_t>(blockIdx.x) * (kMfmaThreads / kWave) + threadIdx.x / kWave;
  if (unit >= A * chunks * ksplit) return;
  ttm_f32_unit<MT, VM, TAIL>(X, A, K, B, Mop, m, chunks, ksplit, kper, Y, unit);
}

// The same for at most three 16-row tiles, held to 256 registers so that two waves share
// each SIMD: a wave has one block of X in flight besides the one it multiplies, so with one
// wave per SIMD (the compiler's choice otherwise: about 300 vector and matrix registers) the
// loads in flight per CU cover too little of the memory latency.  (With four tiles the
// limit would spill.)
template <int MT, bool VM, int TAIL = 0>
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(2))) void ttm_mfma_f32_occ2_kernel(
    const float* __restrict__ X, int64_t A, int64_t K, int64_t B, const float* __restrict__ Mop, int64_t m,
    int64_t chunks, int ksplit, int64_t kper, float* __restrict__ Y) {
  static_assert(MT <= 3, "four tiles do not fit two waves per SIMD");
  const int64_t unit = static_cast<int64_t>(blockIdx.x) * (kMfmaThreads / kWave) + threadIdx.x / kWave;
  if (unit >= A * chunks * ksplit) return;
  ttm_f32_unit<MT, VM, TAIL, 1>(X, A, K, B, Mop, m, chunks, ksplit, kper, Y, unit);
}

// The binary32 contraction with M staged in LDS, for plans without a split over k and
// K % 4 == 0 (rows 16 MT .. 16 MT + TAIL - 1 on the vector ALU as above).  The four waves
// of a workgroup take four consecutive units, which share the k loop, so M is staged once
// per workgroup in windows of kMWin k, double-buffered: every thread stages a share of the
// next window during each round of DEPTH 16-k blocks of the current one, and a barrier
// closes each window.  A lane's A operand (16 rows, four consecutive k) is then one 16-byte
// LDS read per tile; read from the caches instead, the 16 rows of a lane group touch 16
// cache lines per load, as many line accesses as the X loads themselves (the kernel ran
// 23 % faster in a timing build without the M loads).  Waves past the last unit run the
// loop on unit 0's data and store nothing.
constexpr int kMWin = 192;              // k per window: whole rounds of DEPTH 16-k blocks
// two waves per SIMD with two blocks of X in flight each (measured 10 % faster than one wave
// with three; three tiles plus two tail rows take one block, to stay within 256 registers)
constexpr int mlds_depth(int mt, int tail) { return (mt == 3 && tail == 2) ? 1 : 2; }
constexpr int kMWinStride = kMWin + 4;  // floats per staged row: 16-byte rows, rows four banks apart

template <int MT, int TAIL, int DEPTH, bool OCC2>
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(OCC2 ? 2 : 1))) void
ttm_mfma_f32_mlds_kernel(const float* __restrict__ X, int64_t A, int64_t K, int64_t B, const float* __restrict__ Mop,
                         int64_t m, int64_t chunks, float* __restrict__ Y) {
  constexpr int kRounds = kMWin / (16 * DEPTH);  // rounds of DEPTH blocks per window
  static_assert(kRounds * 16 * DEPTH == kMWin, "a window is whole rounds of DEPTH blocks");
  constexpr int kRows = 16 * MT + TAIL;
  constexpr int kF4 = kMWin / 4;        // 16-byte groups per staged row
  constexpr int kGroups = kRows * kF4;  // per window
  constexpr int kPer = (kGroups + kRounds * kMfmaThreads - 1) / (kRounds * kMfmaThreads);  // per thread and round
  __shared__ __align__(16) float sMw[2][kRows * kMWinStride];
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  const int64_t unit_raw = static_cast<int64_t>(blockIdx.x) * (kMfmaThreads / kWave) + tid / kWave;
  const bool active = unit_raw < A * chunks;
  const int64_t unit = active ? unit_raw : 0;
  const int64_t a = unit / chunks;
  const int64_t b0 = (unit - a * chunks) * kUnitCols;
  const int j = lane % 16, q = lane / 16;

  f32x4 acc[MT][2][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[mt][g][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 tacc[TAIL > 0 ? TAIL : 1][2];
#pragma unroll
  for (int r = 0; r < TAIL; ++r) tacc[r][0] = tacc[r][1] = f32x4{0.f, 0.f, 0.f, 0.f};

  const float* xa = X + a * K * B;
  const bool colok0 = (b0 + 4 * j) < B;
  const bool colok1 = (b0 + 64 + 4 * j) < B;
  const int64_t c0off = colok0 ? b0 + 4 * j : b0, c1off = colok1 ? b0 + 64 + 4 * j : b0;
  const f32x4 zero4 = f32x4{0.f, 0.f, 0.f, 0.f};
  f32x4 n0[DEPTH][4], n1[DEPTH][4];
  const auto load_block = [&](int64_t k0, auto Pc) {
    constexpr int P = decltype(Pc)::value;
    const int64_t kl = k0 + 4 * q;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t kc = (kl + s < K) ? kl + s : K - 1;
      n0[P][s] = *reinterpret_cast<const f32x4*>(xa + kc * B + c0off);
      n1[P][s] = *reinterpret_cast<const f32x4*>(xa + kc * B + c1off);
    }
  };
  // staging: group g of a window is row g / kF4, k = kw + 4 (g % kF4); zero past K
  f32x4 sv[kPer];
  const auto stage_load = [&](int64_t kw, int round) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int g = (round * kPer + i) * kMfmaThreads + tid;
      const int row = g / kF4, c4 = g - (g / kF4) * kF4;
      const int64_t k = kw + 4 * c4;
      sv[i] = (g < kGroups && k < K) ? *reinterpret_cast<const f32x4*>(Mop + row * K + k) : zero4;
    }
  };
  const auto stage_store = [&](int b, int round) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int g = (round * kPer + i) * kMfmaThreads + tid;
      const int row = g / kF4, c4 = g - (g / kF4) * kF4;
      if (g < kGroups) *reinterpret_cast<f32x4*>(&sMw[b][row * kMWinStride + 4 * c4]) = sv[i];
    }
  };
  int buf = 0;
  int64_t kw = 0;
  const auto block = [&](int64_t k0, auto Pc) {
    constexpr int P = decltype(Pc)::value;
    f32x4 y0[4], y1[4];
    float w[4][MT];
    f32x4 tw[TAIL > 0 ? TAIL : 1];
    const int64_t kl = k0 + 4 * q;
    const float* mw = &sMw[buf][kl - kw];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(mw + (mt * 16 + j) * kMWinStride);
#pragma unroll
      for (int s = 0; s < 4; ++s) w[s][mt] = v[s];  // zero past K (staged so)
    }
#pragma unroll
    for (int r = 0; r < TAIL; ++r) tw[r] = *reinterpret_cast<const f32x4*>(mw + (MT * 16 + r) * kMWinStride);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool kin = kl + s < K;
      y0[s] = kin ? n0[P][s] : zero4;
      y1[s] = kin ? n1[P][s] : zero4;
    }
    // the block DEPTH steps ahead goes out before this block's products
    __builtin_amdgcn_sched_barrier(0);
    load_block(k0 + 16 * DEPTH, Pc);  // past K: rows K - 1 again, never used
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc[mt][0][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[s][mt], y0[s][t], acc[mt][0][t], 0, 0, 0);
          acc[mt][1][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[s][mt], y1[s][t], acc[mt][1][t], 0, 0, 0);
        }
#pragma unroll
    for (int r = 0; r < TAIL; ++r)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          tacc[r][0][c] = fmaf(tw[r][s], y0[s][c], tacc[r][0][c]);
          tacc[r][1][c] = fmaf(tw[r][s], y1[s][c], tacc[r][1][c]);
        }
  };
  constexpr auto sets = std::make_integer_sequence<int, DEPTH>{};
  for_each_index([&](auto Pc) { load_block(16 * decltype(Pc)::value, Pc); }, sets);
  // window 0 before the loop
#pragma unroll
  for (int round = 0; round < kRounds; ++round) {
    stage_load(0, round);
    stage_store(0, round);
  }
  __syncthreads();
  for (int64_t k0 = 0; k0 < K; k0 += 16 * DEPTH) {
    const int round = static_cast<int>((k0 / (16 * DEPTH)) % kRounds);
    const bool more = kw + kMWin < K;
    if (more) stage_load(kw + kMWin, round);
    for_each_index(
        [&](auto Pc) {
          const int64_t kb = k0 + 16 * decltype(Pc)::value;
          if (kb < K) block(kb, Pc);
        },
        sets);
    if (more) stage_store(buf ^ 1, round);
    if (round == kRounds - 1 || k0 + 16 * DEPTH >= K) {
      __syncthreads();  // the window is read by every wave and the next one staged
      buf ^= 1;
      kw += kMWin;
    }
  }
  if (!active) return;
  float* ya = Y + a * m * B;
#pragma unroll
  for (int r = 0; r < TAIL; ++r) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      f32x4 v = tacc[r][g];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float p1 = __shfl(v[c], j + 16), p2 = __shfl(v[c], j + 32), p3 = __shfl(v[c], j + 48);
        v[c] = ((v[c] + p1) + p2) + p3;
      }
      const int64_t i = MT * 16 + r;
      const int64_t c0 = b0 + 64 * g + 4 * j;
      if (q == 0 && i < m && c0 < B) *reinterpret_cast<f32x4*>(ya + i * B + c0) = v;
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = mt * 16 + 4 * q + v;
      if (i >= m) continue;
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int64_t c = b0 + 64 * g + 4 * j;
        if (c < B) {
          f32x4 o = f32x4{acc[mt][g][0][v], acc[mt][g][1][v], acc[mt][g][2][v], acc[mt][g][3][v]};
          *reinterpret_cast<f32x4*>(ya + i * B + c) = o;
        }
      }
    }
  }
}

// Independent binary32 contractions of one shape class in one launch: job q owns the
// units [unit0_q, unit0_q + A_q chunks_q ksplit_q).
struct F32Job {
  const float* X;
  const float* Mop;
  float* out;
  int64_t A, K, B, m, chunks, kper, unit0;
  int ksplit;
};
struct F32JobTable {
  F32Job j[kMaxF32Group];
  int count;
};
template <int MT, bool VM>
__global__ __launch_bounds__(kMfmaThreads) void ttm_mfma_f32_grouped_kernel(F32JobTable tab) {
  const int64_t unit = static_cast<int64_t>(blockIdx.x) * (kMfmaThreads / kWave) + threadIdx.x / kWave;
  int q = 0;
  for (int t = 1; t < tab.count; ++t)
    if (unit >= tab.j[t].unit0) q = t;
  const F32Job& J = tab.j[q];
  const int64_t local = unit - J.unit0;
  if (local >= J.A * J.chunks * J.ksplit) return;
  ttm_f32_unit<MT, VM>(J.X, J.A, J.K, J.B, J.Mop, J.m, J.chunks, J.ksplit, J.kper, J.out, local);
}

// Split sums of several jobs in one launch: job q covers the flat indices [off_q, off_q + n_q).
struct SumJob {
  const float* part;
  float* Y;
  int64_t n, off;
  int ksplit;
};
struct SumJobTable {
  SumJob j[kMaxF32Group];
  int count;
};
__global__ __launch_bounds__(256) void sum_splits_grouped_kernel(SumJobTable tab, int64_t total) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; g < total; g += stride) {
    int q = 0;
    for (int t = 1; t < tab.count; ++t)
      if (g >= tab.j[t].off) q = t;
    const SumJob& J = tab.j[q];
    const int64_t i = g - J.off;
    float acc = J.part[i];
    for (int k = 1; k < J.ksplit; ++k) acc += J.part[k * J.n + i];
    J.Y[i] = acc;
  }
}

// Last-mode contraction (B == 1): Y[a, i] = sum_k X[a, k] M[i, k], a GEMM with
// the long contiguous rows of X as the reduction axis.  A wave owns 64 rows of X
// (four 16-row MFMA tiles) and reads them with 16-byte loads along k; the packed
// operand supplies the 16-row tiles of M.  Requires K % 4 == 0.
template <int MT>
__global__ __launch_bounds__(kMfmaThreads) void ttm_mfma_f32_last_kernel(const float* __restrict__ X, int64_t A,
                                                                         int64_t K, const float* __restrict__ Mop,
                                                                         int64_t m, int ksplit, int64_t kper,
                                                                         float* __restrict__ Y) {
  const int lane = threadIdx.x % kWave;
  const int64_t unit = static_cast<int64_t>(blockIdx.x) * (kMfmaThreads / kWave) + threadIdx.x / kWave;
  const int64_t groups = (A + 63) / 64;
  if (unit >= groups * ksplit) return;
  const int ks = static_cast<int>(unit % ksplit);
  const int64_t a0 = (unit / ksplit) * 64;
  const int r16 = lane % 16, q = lane / 16;
  const int64_t kbeg = ks * kper;
  const int64_t kend = (kbeg + kper < K) ? kbeg + kper : K;
  f32x4 acc[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int at = 0; at < 4; ++at) acc[mt][at] = f32x4{0.f, 0.f, 0.f, 0.f};
  // The next 16 k are loaded while the current ones are multiplied.  Loads carry no
  // conditions: k past kend reads the last four k of the range (zeroed before use; kbeg and
  // kend are multiples of 4), and a row past A reads row A - 1 (its products land only in
  // output rows that are not stored).
  f32x4 nx[4], nw[MT];
  const auto load = [&](int64_t k0) {
    const int64_t k = k0 + 4 * q;
    const int64_t kc = (k < kend) ? k : kend - 4;
#pragma unroll
    for (int at = 0; at < 4; ++at) {
      const int64_t a = a0 + 16 * at + r16;
      nx[at] = *reinterpret_cast<const f32x4*>(X + ((a < A) ? a : A - 1) * K + kc);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) nw[mt] = *reinterpret_cast<const f32x4*>(Mop + (16 * mt + r16) * K + kc);
  };
  if (kbeg < kend) load(kbeg);
  const f32x4 zero4 = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = kbeg; k0 < kend; k0 += 16) {
    const bool kin = k0 + 4 * q < kend;
    f32x4 xv[4], mv[MT];
#pragma unroll
    for (int at = 0; at < 4; ++at) xv[at] = kin ? nx[at] : zero4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) mv[mt] = kin ? nw[mt] : zero4;
    __builtin_amdgcn_sched_barrier(0);
    load(k0 + 16);  // past kend: clamped, never used
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int at = 0; at < 4; ++at)
          acc[mt][at] = __builtin_amdgcn_mfma_f32_16x16x4f32(mv[mt][c], xv[at][c], acc[mt][at], 0, 0, 0);
  }
  float* y = Y + static_cast<int64_t>(ks) * A * m;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int at = 0; at < 4; ++at) {
      const int64_t a = a0 + 16 * at + r16;
      if (a >= A) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = 16 * mt + 4 * q + v;
        if (i < m) y[a * m + i] = acc[mt][at][v];
      }
    }
}

__device__ __forceinline__ uint32_t pack_lo(uint32_t a, uint32_t b) { return (a & 0xffffu) | (b << 16); }
__device__ __forceinline__ uint32_t pack_hi(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }

template <int MT>
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(2))) void ttm_mfma_bf16_kernel(
    const bf16_t* __restrict__ X, int64_t A,
                                                                     int64_t K, int64_t B,
                                                                     const bf16_t* __restrict__ Mop, int64_t m,
                                                                     int64_t chunks, int ksplit, int64_t kper,
                                                                     float* __restrict__ Y) {
  const int lane = threadIdx.x % kWave;
  const int64_t unit = static_cast<int64_t>(blockIdx.x) * (kMfmaThreads / kWave) + threadIdx.x / kWave;
  const int64_t total = A * chunks * ksplit;
  if (unit >= total) return;
  const int ks = static_cast<int>(unit % ksplit);
  const int64_t ac = unit / ksplit;
  const int64_t a = ac / chunks;
  const int64_t b0 = (ac - a * chunks) * kUnitCols;
  const int j = lane % 16, q = lane / 16;
  const int64_t kbeg = ks * kper;
  const int64_t kend = (kbeg + kper < K) ? kbeg + kper : K;

  f32x4 acc[MT][8];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[mt][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  const bf16_t* xa = X + a * K * B;
  const int64_t col = b0 + 8 * j;
  const bool colok = col < B;
  // Lane loads rows k0 + 8q + t (t < 8) of columns col..col+7 and the matching 8 k of M.
  // The next 32 k are loaded while the current ones are multiplied.  Loads carry no
  // conditions: a block past kend reads the last 8 k of the range (zeroed before use; kbeg
  // and kend are multiples of 8), and a column block past B reads the last 8 columns (its
  // products land only in output columns that are not stored).
  const int64_t colc = colok ? col : B - 8;
  u32x4 rn[8], nw[MT];
  const auto load = [&](int64_t k0) {
    const int64_t k = k0 + 8 * q;
    const int64_t kc = (k < kend) ? k : kend - 8;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) nw[mt] = *reinterpret_cast<const u32x4*>(Mop + (mt * 16 + j) * K + kc);
#pragma unroll
    for (int t = 0; t < 8; ++t) rn[t] = *reinterpret_cast<const u32x4*>(xa + (kc + t) * B + colc);
  };
  if (kbeg < kend) load(kbeg);
  const u32x4 zero4 = u32x4{0u, 0u, 0u, 0u};
  for (int64_t k0 = kbeg; k0 < kend; k0 += 32) {
    const bool kin = k0 + 8 * q < kend;
    u32x4 r[8], mv[MT];
#pragma unroll
    for (int t = 0; t < 8; ++t) r[t] = kin ? rn[t] : zero4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) mv[mt] = kin ? nw[mt] : zero4;
    __builtin_amdgcn_sched_barrier(0);
    load(k0 + 32);  // past kend: clamped, never used
    __builtin_amdgcn_sched_barrier(0);
    // operand for column c (8 consecutive k of column col + c) is packed just before its
    // products, which keeps the register count low enough for two waves per SIMD
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      u32x4 op;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t lo = r[2 * w][c / 2], hi = r[2 * w + 1][c / 2];
        op[w] = (c % 2 == 0) ? pack_lo(lo, hi) : pack_hi(lo, hi);
      }
      const bf16x8 bv = __builtin_bit_cast(bf16x8, op);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        acc[mt][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, mv[mt]), bv, acc[mt][c], 0,
                                                             0, 0);
    }
  }
  float* ya = Y + (static_cast<int64_t>(ks) * A + a) * m * B;
  if (!colok) return;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = mt * 16 + 4 * q + v;
      if (i >= m) continue;
      f32x4 o0 = f32x4{acc[mt][0][v], acc[mt][1][v], acc[mt][2][v], acc[mt][3][v]};
      f32x4 o1 = f32x4{acc[mt][4][v], acc[mt][5][v], acc[mt][6][v], acc[mt][7][v]};
      *reinterpret_cast<f32x4*>(ya + i * B + col) = o0;
      *reinterpret_cast<f32x4*>(ya + i * B + col + 4) = o1;
    }
  }
}

// Y = sum of the split parts in part order (binary32), stored as TO
template <typename TO>
__global__ __launch_bounds__(256) void sum_splits_kernel(const float* __restrict__ part, int ksplit, int64_t n,
                                                         TO* __restrict__ Y) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
    float s = part[i];
    for (int k = 1; k < ksplit; ++k) s += part[k * n + i];
    Y[i] = static_cast<TO>(s);
  }
}

struct MfmaPlan {
  int64_t chunks;
  int ksplit;
  int64_t kper;
};

MfmaPlan mfma_plan(rt_dtype xdt, int64_t A, int64_t K, int64_t B, int64_t m) {
  MfmaPlan p;
  p.chunks = ceil_div(B, kUnitCols);
  const int64_t units = A * p.chunks;
  const int64_t kgran = (xdt == RT_BF16) ? 32 : 4;
  int ks = 1;
  // aim for >= 2048 waves (8 per CU) when K is long enough to split; short K
  // (>= 64 per part) is split too while the partial sums stay under a quarter
  // of the input read
  // (an input that stays in the caches may split down to 32 per part)
  const int64_t in_bytes = A * K * B * (xdt == RT_BF16 ? 2 : 4);
  const bool cached = in_bytes <= (int64_t(32) << 20);
  while (units * ks < 2048 && ks < 16) {
    const int64_t kp = K / (ks * 2);
    const int64_t part_bytes = 2 * ks * A * m * B * 4;
    if (kp >= 256 || (kp >= 64 && part_bytes * 4 <= in_bytes) || (cached && kp >= 32 && part_bytes <= in_bytes))
      ks *= 2;
    else
      break;
  }
  p.ksplit = ks;
  p.kper = ceil_div(ceil_div(K, ks), kgran) * kgran;
  return p;
}

}  // namespace

size_t ttm_generic_ws(rt_dtype xdt, int64_t A, int64_t K, int64_t B, int64_t m) {
  const int ks = generic_ksplit(A, K, B);
  if (ks == 1) return 0;
  return align256(static_cast<size_t>(ks) * A * m * B * (xdt == RT_F64 ? 8 : 4));
}

hipError_t launch_ttm_generic(const void* X, rt_dtype xdt, int64_t A, int64_t K, int64_t B, const void* M,
                              int64_t m, void* Y, void* ws, hipStream_t st, bool mtrans) {
  if (A * B == 0 || m == 0) return hipSuccess;
  switch (xdt) {
    case RT_F64:
      return generic_dispatch<double, double>(static_cast<const double*>(X), A, K, B,
                                              static_cast<const double*>(M), m, static_cast<double*>(Y),
                                              static_cast<double*>(ws), st, mtrans);
    case RT_F32:
      return generic_dispatch<float, float>(static_cast<const float*>(X), A, K, B, static_cast<const float*>(M),
                                            m, static_cast<float*>(Y), static_cast<float*>(ws), st, mtrans);
    case RT_BF16:
      return generic_dispatch<bf16_t, float>(static_cast<const bf16_t*>(X), A, K, B,
                                             static_cast<const float*>(M), m, static_cast<float*>(Y),
                                             static_cast<float*>(ws), st, mtrans);
    case RT_F8E4M3:
      return generic_dispatch<f8_t, float>(static_cast<const f8_t*>(X), A, K, B, static_cast<const float*>(M), m,
                                           static_cast<float*>(Y), static_cast<float*>(ws), st, mtrans);
  }
  return hipErrorInvalidValue;
}

int64_t ttm_mfma_mpad(int64_t m) { return ceil_div(m, 16) * 16; }

bool ttm_mfma_ok(rt_dtype xdt, int64_t A, int64_t K, int64_t B, int64_t m) {
  if (m < 1 || m > 64 || A < 1 || K < 1) return false;
  if (xdt == RT_F32) return B >= 64 && (B % 4) == 0;
  if (xdt == RT_BF16) return B >= 64 && (B % 8) == 0 && (K % 8) == 0;
  return false;
}

size_t ttm_mfma_ws(rt_dtype xdt, int64_t A, int64_t K, int64_t B, int64_t m) {
  const MfmaPlan p = mfma_plan(xdt, A, K, B, m);
  if (p.ksplit == 1) return 0;
  return align256(static_cast<size_t>(p.ksplit) * A * m * B * sizeof(float));
}

hipError_t launch_ttm_mfma_ws(const void* X, rt_dtype xdt, int64_t A, int64_t K, int64_t B, const void* Mop,
                              int64_t m, float* Y, void* ws, hipStream_t st) {
  const MfmaPlan p = mfma_plan(xdt, A, K, B, m);
  float* out = (p.ksplit == 1) ? Y : static_cast<float*>(ws);
  const int64_t units = A * p.chunks * p.ksplit;
  const unsigned grid = static_cast<unsigned>(ceil_div(units, kMfmaThreads / kWave));
  const int MT = static_cast<int>(ttm_mfma_mpad(m) / 16);
#define RT_LAUNCH_F32_K(KERNEL, MTV)                                                                        \
  if (K % 4 == 0)                                                                                           \
    KERNEL<MTV, true><<<grid, kMfmaThreads, 0, st>>>(static_cast<const float*>(X), A, K, B,                 \
                                                     static_cast<const float*>(Mop), m, p.chunks, p.ksplit,  \
                                                     p.kper, out);                                          \
  else                                                                                                      \
    KERNEL<MTV, false><<<grid, kMfmaThreads, 0, st>>>(static_cast<const float*>(X), A, K, B,                \
                                                      static_cast<const float*>(Mop), m, p.chunks, p.ksplit, \
                                                      p.kper, out)
#define RT_LAUNCH_F32(MTV) RT_LAUNCH_F32_K(ttm_mfma_f32_occ2_kernel, MTV)
#define RT_LAUNCH_BF16(MTV)                                                                                 \
  ttm_mfma_bf16_kernel<MTV><<<grid, kMfmaThreads, 0, st>>>(static_cast<const bf16_t*>(X), A, K, B,          \
                                                           static_cast<const bf16_t*>(Mop), m, p.chunks,    \
                                                           p.ksplit, p.kper, out)
  // rows past the last whole 16-row tile on the vector ALU when there are at most two
  const int tail = (K % 4 == 0 && m % 16 != 0 && m % 16 <= 2 && m > 16) ? static_cast<int>(m % 16) : 0;
  const int MTfull = static_cast<int>(m / 16);
#define RT_LAUNCH_F32_TAIL(MTV, TV)                                                                         \
  if (p.ksplit == 1)                                                                                         \
    ttm_mfma_f32_mlds_kernel<MTV, TV, mlds_depth(MTV, TV), true><<<grid, kMfmaThreads, 0, st>>>(             \
        static_cast<const float*>(X), A, K, B,                                                               \
                                                                     static_cast<const float*>(Mop), m,      \
                                                                     p.chunks, out);                         \
  else                                                                                                       \
    ttm_mfma_f32_kernel<MTV, true, TV><<<grid, kMfmaThreads, 0, st>>>(static_cast<const float*>(X), A, K, B, \
                                                                      static_cast<const float*>(Mop), m,     \
                                                                      p.chunks, p.ksplit, p.kper, out)
  if (xdt == RT_F32 && tail > 0) {
    if (MTfull == 1) {
      if (tail == 1) RT_LAUNCH_F32_TAIL(1, 1); else RT_LAUNCH_F32_TAIL(1, 2);
    } else if (MTfull == 2) {
      if (tail == 1) RT_LAUNCH_F32_TAIL(2, 1); else RT_LAUNCH_F32_TAIL(2, 2);
    } else {
      if (tail == 1) RT_LAUNCH_F32_TAIL(3, 1); else RT_LAUNCH_F32_TAIL(3, 2);
    }
  } else if (xdt == RT_F32) {
    switch (MT) {
      case 1: RT_LAUNCH_F32(1); break;
      case 2: RT_LAUNCH_F32(2); break;
      case 3: RT_LAUNCH_F32(3); break;
      default: RT_LAUNCH_F32_K(ttm_mfma_f32_kernel, 4); break;
    }
  } else {
    switch (MT) {
      case 1: RT_LAUNCH_BF16(1); break;
      case 2: RT_LAUNCH_BF16(2); break;
      case 3: RT_LAUNCH_BF16(3); break;
      default: RT_LAUNCH_BF16(4); break;
    }
  }
#undef RT_LAUNCH_F32
#undef RT_LAUNCH_F32_K
#undef RT_LAUNCH_F32_TAIL
#undef RT_LAUNCH_BF16
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.ksplit == 1) return e;
  const int64_t n = A * m * B;
  const unsigned g2 = static_cast<unsigned>(ceil_div(n, 256) > 8192 ? 8192 : ceil_div(n, 256));
  sum_splits_kernel<float><<<g2, 256, 0, st>>>(out, p.ksplit, n, Y);
  return hipGetLastError();
}

hipError_t launch_ttm_mfma_f32_group(const F32Contraction* c, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  // one launch needs one kernel instance: every job with the same tile count and M load
  int mt0 = -1;
  bool vm0 = true, same = count <= kMaxF32Group;
  for (int i = 0; i < count && same; ++i) {
    const int mt = static_cast<int>(ttm_mfma_mpad(c[i].m) / 16);
    const bool vm = c[i].K % 4 == 0;
    if (i == 0) {
      mt0 = mt;
      vm0 = vm;
    } else if (mt != mt0 || vm != vm0) {
      same = false;
    }
  }
  if (!same || count == 1) {
    for (int i = 0; i < count; ++i) {
      const hipError_t e =
          launch_ttm_mfma_ws(c[i].X, RT_F32, c[i].A, c[i].K, c[i].B, c[i].Mop, c[i].m, c[i].Y, c[i].ws, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  F32JobTable tab{};
  SumJobTable sums{};
  tab.count = count;
  int64_t units = 0, sum_total = 0;
  for (int i = 0; i < count; ++i) {
    const MfmaPlan p = mfma_plan(RT_F32, c[i].A, c[i].K, c[i].B, c[i].m);
    F32Job& J = tab.j[i];
    J.X = c[i].X;
    J.Mop = c[i].Mop;
    J.out = (p.ksplit == 1) ? c[i].Y : static_cast<float*>(c[i].ws);
    J.A = c[i].A; J.K = c[i].K; J.B = c[i].B; J.m = c[i].m;
    J.chunks = p.chunks;
    J.kper = p.kper;
    J.ksplit = p.ksplit;
    J.unit0 = units;
    units += c[i].A * p.chunks * p.ksplit;
    if (p.ksplit > 1) {
      SumJob& S = sums.j[sums.count++];
      S.part = J.out;
      S.Y = c[i].Y;
      S.n = c[i].A * c[i].m * c[i].B;
      S.off = sum_total;
      S.ksplit = p.ksplit;
      sum_total += S.n;
    }
  }
  const unsigned grid = static_cast<unsigned>(ceil_div(units, kMfmaThreads / kWave));
#define RT_LAUNCH_GROUP(MTV)                                                                     \
  if (vm0)                                                                                       \
    ttm_mfma_f32_grouped_kernel<MTV, true><<<grid, kMfmaThreads, 0, st>>>(tab);                  \
  else                                                                                           \
    ttm_mfma_f32_grouped_kernel<MTV, false><<<grid, kMfmaThreads, 0, st>>>(tab)
  switch (mt0) {
    case 1: RT_LAUNCH_GROUP(1); break;
    case 2: RT_LAUNCH_GROUP(2); break;
    case 3: RT_LAUNCH_GROUP(3); break;
    default: RT_LAUNCH_GROUP(4); break;
  }
#undef RT_LAUNCH_GROUP
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || sums.count == 0) return e;
  const unsigned g2 = static_cast<unsigned>(ceil_div(sum_total, 256) > 8192 ? 8192 : ceil_div(sum_total, 256));
  sum_splits_grouped_kernel<<<g2, 256, 0, st>>>(sums, sum_total);
  return hipGetLastError();
}

bool ttm_mfma_last_ok(int64_t A, int64_t K, int64_t m) { return A >= 1 && m >= 1 && m <= 64 && K >= 4 && K % 4 == 0; }

namespace {
struct LastPlan {
  int ksplit;
  int64_t kper;
};
LastPlan last_plan(int64_t A, int64_t K, int64_t m) {
  LastPlan p;
  const int64_t units = ceil_div(A, 64);
  int ks = 1;
  while (units * ks < 2048 && K / (ks * 2) >= 64 && ks < 16 && 2 * ks * A * m * 4 <= A * K * 4) ks *= 2;
  p.ksplit = ks;
  p.kper = ceil_div(ceil_div(K, ks), 16) * 16;
  return p;
}
}  // namespace

size_t ttm_mfma_last_ws(int64_t A, int64_t K, int64_t m, bool f64_out) {
  const LastPlan p = last_plan(A, K, m);
  return (p.ksplit == 1 && !f64_out) ? 0 : align256(static_cast<size_t>(p.ksplit) * A * m * sizeof(float));
}

hipError_t launch_ttm_mfma_last(const float* X, int64_t A, int64_t K, const float* Mop, int64_t m, float* Y,
                                void* ws, hipStream_t st, double* Y64) {
  const LastPlan p = last_plan(A, K, m);
  float* out = (p.ksplit == 1 && !Y64) ? Y : static_cast<float*>(ws);
  const int64_t units = ceil_div(A, 64) * p.ksplit;
  const unsigned grid = static_cast<unsigned>(ceil_div(units, kMfmaThreads / kWave));
  const int MT = static_cast<int>(ttm_mfma_mpad(m) / 16);
#define RT_LAUNCH_LAST(MTV) \
  ttm_mfma_f32_last_kernel<MTV><<<grid, kMfmaThreads, 0, st>>>(X, A, K, Mop, m, p.ksplit, p.kper, out)
  switch (MT) {
    case 1: RT_LAUNCH_LAST(1); break;
    case 2: RT_LAUNCH_LAST(2); break;
    case 3: RT_LAUNCH_LAST(3); break;
    default: RT_LAUNCH_LAST(4); break;
  }
#undef RT_LAUNCH_LAST
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || (p.ksplit == 1 && !Y64)) return e;
  const int64_t n = A * m;
  const unsigned g2 = static_cast<unsigned>(ceil_div(n, 256) > 8192 ? 8192 : ceil_div(n, 256));
  if (Y64)
    sum_splits_kernel<double><<<g2, 256, 0, st>>>(out, p.ksplit, n, Y64);
  else
    sum_splits_kernel<float><<<g2, 256, 0, st>>>(out, p.ksplit, n, Y);
  return hipGetLastError();
}

int64_t ttm_grouped_blocks(int64_t A, int64_t B, int64_t m, int mt) {
  return ceil_div(A * B, kWave) * ceil_div(m, mt);
}

hipError_t launch_ttm_grouped(const GTtmJob* jobs, const int32_t* blkjob, int count, int64_t total_blocks,
                              rt_dtype xdt, int mt, hipStream_t st) {
  if (count == 0 || total_blocks == 0) return hipSuccess;
  const unsigned g = static_cast<unsigned>(total_blocks);
#define RT_G(TX, TC, MTV) ttm_grouped_kernel<TX, TC, MTV><<<g, kWave, 0, st>>>(jobs, blkjob)
  // the row tile must be exactly the one the block counts were computed with
  if (mt != 8 && mt != 16 && mt != 32) return hipErrorInvalidValue;
  switch (xdt) {
    case RT_F64:
      if (mt == 8) RT_G(double, double, 8); else if (mt == 16) RT_G(double, double, 16); else RT_G(double, double, 32);
      break;
    case RT_F32:
      if (mt == 8) RT_G(float, float, 8); else if (mt == 16) RT_G(float, float, 16); else RT_G(float, float, 32);
      break;
    case RT_BF16:
      if (mt == 8) RT_G(bf16_t, float, 8); else if (mt == 16) RT_G(bf16_t, float, 16); else RT_G(bf16_t, float, 32);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef RT_G
  return hipGetLastError();
}

}  // namespace rt

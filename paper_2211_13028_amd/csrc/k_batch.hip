// Streaming kernels of the batched decomposition (many small 3-way tensors, one
// launch per step of Alg. 4.4 for the whole batch).
//
// First sketch level per tensor (the dimension-tree node of Sec. 4.4 that reads X):
//   Z = X x_3 Phi_3  (I1 x I2 x s3)      W = X x_2 Phi_2  (I1 x s2 x I3)
// in one pass over X.  A slab X[a] (P = I2 rows of Q = I3 contiguous values, Q <= 256)
// is the unit of work; a 256-thread workgroup takes a run of slabs of one tensor and its
// four waves take every fourth slab, independently (no barrier after the set-up).
// A wave walks its slabs in steps of 16 rows:
//  * lane (li, kg) = (lane % 16, lane / 16) loads rows pb + 4 t + kg (t < 4) at columns
//    16 g + li (g < NG = ceil(Q / 16)): 16 lanes read 64 consecutive bytes of a row.  The
//    next step's values are in flight while the current step is multiplied;
//  * W^T accumulates on matrix cores with the loaded values as the B operand
//    (A = Phi_2[c][p] of the lane's rows), one 16 x 16 tile per 16 columns;
//  * Z needs the rows as the A operand: the step is staged 64 columns at a time in the
//    wave's LDS area and read back row-wise; Phi_3 (zero-padded to 16 x 16 NG) sits in
//    LDS for the whole workgroup.
// Binary32 16x16x4 products for both input types (bfloat16 values widen exactly).
// (Reading each 16-row block as one flat run, 64 consecutive elements per load, and
// scattering it into an LDS tile read back for both products measured slower: 0.92 ms
// against 0.63 ms for the 192-column class of the 512-tensor batch.)
#include <type_traits>

#include "kernels.hpp"

namespace rt {

namespace {

typedef float bf32x4 __attribute__((ext_vector_type(4)));

constexpr int kBThreads = 256;
constexpr int kBWaves = kBThreads / kWave;
constexpr int kStageStride = 84;  // floats per staged row of 64 columns: = 20 mod 64, conflict-free
                                  // row-wise reads (lane li reads row li) with at most 2-way
                                  // conflicts on the column-wise stores

// Phi_3 rows in LDS: 16 NG columns (a multiple of 64) + 20, the same residue as the stage
__host__ __device__ constexpr int phi_stride(int ng) { return 16 * ng + 20; }

template <typename TX>
__device__ __forceinline__ float widen(TX v);
template <>
__device__ __forceinline__ float widen<float>(float v) { return v; }
template <>
__device__ __forceinline__ float widen<bf16_t>(bf16_t v) { return bf16_to_f32(v); }

// two waves per SIMD up to 192 columns; the widest class keeps its registers at one
template <typename TX, int NG>
__global__ __launch_bounds__(kBThreads, NG > 12 ? 1 : 2) void zw_batch_kernel(const GZwJob* __restrict__ jobs,
                                                               const int32_t* __restrict__ blkjob) {
  constexpr int S = phi_stride(NG);
  __shared__ float sPhi[16 * S];
  __shared__ float sStage[kBWaves][16 * kStageStride];
  const GZwJob J = jobs[blkjob[blockIdx.x]];
  const int64_t P = J.P, Q = J.Q, A = J.A;
  const int sP = J.sP, sQ = J.sQ;
  const bool needZ = J.Z != nullptr, needW = J.W != nullptr;
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int li = lane % 16, kg = lane / 16;
  const int64_t local = blockIdx.x - J.blk0;
  const int64_t a_first = local * kBWaves * J.spb + wave;
  const int64_t a_end = (local + 1) * kBWaves * J.spb < A ? (local + 1) * kBWaves * J.spb : A;
  const int steps = static_cast<int>((P + 15) / 16);
  float* st = sStage[wave];
  const gptr<const TX> X = global_ptr(static_cast<const TX*>(J.X));
  const gptr<const float> phiP = global_ptr(J.phiP);
  const gptr<float> Zo = global_ptr(J.Z), Wo = global_ptr(J.W);

  // column offsets and masks of the lane, fixed for the tensor (loads clamp to column Q - 1)
  uint32_t qoff[NG];
  bool qok[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int q = 16 * g + li;
    qok[g] = q < Q;
    qoff[g] = static_cast<uint32_t>(q < Q ? q : Q - 1);
  }

  const int pc_lane = li < sP ? li : sP - 1;

  // raw values of the next step (converted and masked when the step is taken over)
  TX rn[4][NG];
  float ppn[4];
  auto load = [&](int64_t a, int64_t pb) {
    const gptr<const TX> xa = X + a * P * Q;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t p = pb + 4 * t + kg;
      const uint32_t prow = static_cast<uint32_t>((p < P ? p : P - 1) * Q);
#pragma unroll
      for (int g = 0; g < NG; ++g) rn[t][g] = xa[prow + qoff[g]];
      ppn[t] = needW ? phiP[static_cast<int64_t>(pc_lane) * P + (p < P ? p : P - 1)] : 0.f;
    }
  };
  // the wave's first block is in flight while Phi_3 is staged
  if (a_first < a_end) load(a_first, 0);

  // Phi_3 (sQ x Q) zero-padded to 16 x 16 NG; without Z it is never read
  for (int idx = threadIdx.x; idx < 16 * S; idx += kBThreads) {
    const int c = idx / S, q = idx - (idx / S) * S;
    sPhi[idx] = (needZ && c < sQ && q < Q) ? global_ptr(J.phiQ)[static_cast<int64_t>(c) * Q + q] : 0.f;
  }
  __syncthreads();
  if (a_first >= a_end) return;

  bf32x4 wacc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) wacc[g] = bf32x4{0.f, 0.f, 0.f, 0.f};
  int64_t a = a_first;
  int step = 0;
  while (true) {
    const int64_t pb = static_cast<int64_t>(step) * 16;
    float r[4][NG], pp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool pin = pb + 4 * t + kg < P;
#pragma unroll
      for (int g = 0; g < NG; ++g) r[t][g] = (pin && qok[g]) ? widen<TX>(rn[t][g]) : 0.f;
      pp[t] = (pin && li < sP) ? ppn[t] : 0.f;
    }
    // next step: the following row block, or the first block of the wave's next slab
    const bool last_of_slab = step + 1 == steps;
    const int64_t a_next = last_of_slab ? a + kBWaves : a;
    const int step_next = last_of_slab ? 0 : step + 1;
    if (a_next < a_end) load(a_next, static_cast<int64_t>(step_next) * 16);
    if (needW) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int g = 0; g < NG; ++g) wacc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(pp[t], r[t][g], wacc[g], 0, 0, 0);
    }
    if (needZ) {
      // four accumulators in turn: the products of a step do not wait for each other
      bf32x4 zacc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) zacc[u] = bf32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int cb = 0; cb < (NG + 3) / 4; ++cb) {
        __builtin_amdgcn_wave_barrier();  // the previous block's reads of the stage stay above
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int gg = 0; gg < 4; ++gg)
            if (4 * cb + gg < NG) st[(4 * t + kg) * kStageStride + 16 * gg + li] = r[t][4 * cb + gg];
        __builtin_amdgcn_wave_barrier();  // cross-lane: stores before the reads below
#pragma unroll
        for (int kb = 0; kb < 16; ++kb) {
          if (16 * cb + kb >= 4 * NG) break;  // compile-time
          const float xv = st[li * kStageStride + 4 * kb + kg];
          const float bq = sPhi[li * S + 64 * cb + 4 * kb + kg];
          zacc[kb % 4] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv, bq, zacc[kb % 4], 0, 0, 0);
        }
      }
      const bf32x4 z = (zacc[0] + zacc[1]) + (zacc[2] + zacc[3]);
      if (li < sQ) {
        const gptr<float> zo = Zo + (a * P + pb) * sQ + li;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (pb + 4 * kg + v < P) zo[(4 * kg + v) * sQ] = z[v];
      }
    }
    if (last_of_slab) {
      if (needW) {
        const gptr<float> wo = Wo + a * sP * Q;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (4 * kg + v < sP && qok[g]) wo[(4 * kg + v) * Q + 16 * g + li] = wacc[g][v];
          wacc[g] = bf32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
      a = a_next;
      if (a >= a_end) break;
    }
    step = step_next;
  }
}

// bfloat16 X: the same pass with 16x16x16 bfloat16 products (binary32 accumulation; Phi_2 and
// Phi_3 hold bfloat16 values, so every product is exact and only the accumulation order
// differs from the binary32 path).  Lane (li, kg) loads rows pb + 4 kg + e (e < 4) at
// columns 16 g + li, four consecutive k of one column as the B operand of W^T (A = Phi_2[li]
// at the same rows); for Z the step is staged in binary32 as above and read back four
// consecutive columns of row li at a time (A), with Phi_3 kept in LDS as bfloat16 (B).  A
// quarter of the binary32 path's matrix-core instructions.
typedef short zb_s16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t zb_u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t zb_pack(uint32_t lo16, uint32_t hi16) { return lo16 | (hi16 << 16); }
__device__ __forceinline__ uint32_t zb_pack_f(float lo, float hi) {
  return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xffff0000u);
}

template <int NG>
__global__ __launch_bounds__(kBThreads, NG > 12 ? 1 : 2) void zw_batch_bf16_kernel(const GZwJob* __restrict__ jobs,
                                                                    const int32_t* __restrict__ blkjob) {
  constexpr int S16 = 16 * NG + 8;  // bfloat16 per Phi_3 row (8-byte reads stay aligned)
  __shared__ __align__(16) bf16_t sPhi16[16 * S16];
  __shared__ __align__(16) float sStage[kBWaves][16 * kStageStride];
  const GZwJob J = jobs[blkjob[blockIdx.x]];
  const int64_t P = J.P, Q = J.Q, A = J.A;
  const int sP = J.sP, sQ = J.sQ;
  const bool needZ = J.Z != nullptr, needW = J.W != nullptr;
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int li = lane % 16, kg = lane / 16;
  const int64_t local = blockIdx.x - J.blk0;
  const int64_t a_first = local * kBWaves * J.spb + wave;
  const int64_t a_end = (local + 1) * kBWaves * J.spb < A ? (local + 1) * kBWaves * J.spb : A;
  const int steps = static_cast<int>((P + 15) / 16);
  float* st = sStage[wave];
  const gptr<const bf16_t> X = global_ptr(static_cast<const bf16_t*>(J.X));
  const gptr<const float> phiP = global_ptr(J.phiP);
  const gptr<float> Zo = global_ptr(J.Z), Wo = global_ptr(J.W);
  uint32_t qoff[NG];
  bool qok[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int q = 16 * g + li;
    qok[g] = q < Q;
    qoff[g] = static_cast<uint32_t>(q < Q ? q : Q - 1);
  }
  const int pc_lane = li < sP ? li : sP - 1;
  // raw values of the next step: rows pb + 4 kg + e
  bf16_t rn[4][NG];
  float ppn[4];
  auto load = [&](int64_t a, int64_t pb) {
    const gptr<const bf16_t> xa = X + a * P * Q;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = pb + 4 * kg + e;
      const uint32_t prow = static_cast<uint32_t>((p < P ? p : P - 1) * Q);
#pragma unroll
      for (int g = 0; g < NG; ++g) rn[e][g] = xa[prow + qoff[g]];
      ppn[e] = needW ? phiP[static_cast<int64_t>(pc_lane) * P + (p < P ? p : P - 1)] : 0.f;
    }
  };
  if (a_first < a_end) load(a_first, 0);  // in flight while Phi_3 is staged
  for (int idx = threadIdx.x; idx < 16 * S16; idx += kBThreads) {
    const int c = idx / S16, q = idx - (idx / S16) * S16;
    const float v = (needZ && c < sQ && q < Q) ? global_ptr(J.phiQ)[static_cast<int64_t>(c) * Q + q] : 0.f;
    sPhi16[idx] = static_cast<bf16_t>(__float_as_uint(v) >> 16);
  }
  __syncthreads();
  if (a_first >= a_end) return;

  bf32x4 wacc[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) wacc[g] = bf32x4{0.f, 0.f, 0.f, 0.f};
  int64_t a = a_first;
  int step = 0;
  while (true) {
    const int64_t pb = static_cast<int64_t>(step) * 16;
    // operands of the step, zero past P, past Q and past s2: pairs of rows packed per word
    uint32_t rp[2][NG], pw[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool in0 = pb + 4 * kg + 2 * h < P, in1 = pb + 4 * kg + 2 * h + 1 < P;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const uint32_t lo = (in0 && qok[g]) ? static_cast<uint32_t>(rn[2 * h][g]) : 0u;
        const uint32_t hi = (in1 && qok[g]) ? static_cast<uint32_t>(rn[2 * h + 1][g]) : 0u;
        rp[h][g] = zb_pack(lo, hi);
      }
      const bool pl = li < sP;
      pw[h] = zb_pack_f((in0 && pl) ? ppn[2 * h] : 0.f, (in1 && pl) ? ppn[2 * h + 1] : 0.f);
    }
    const bool last_of_slab = step + 1 == steps;
    const int64_t a_next = last_of_slab ? a + kBWaves : a;
    const int step_next = last_of_slab ? 0 : step + 1;
    if (a_next < a_end) load(a_next, static_cast<int64_t>(step_next) * 16);
    if (needW) {
      const zb_s16x4 av = __builtin_bit_cast(zb_s16x4, zb_u32x2{pw[0], pw[1]});
#pragma unroll
      for (int g = 0; g < NG; ++g)
        wacc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
            av, __builtin_bit_cast(zb_s16x4, zb_u32x2{rp[0][g], rp[1][g]}), wacc[g], 0, 0, 0);
    }
    if (needZ) {
      bf32x4 zacc[2] = {bf32x4{0.f, 0.f, 0.f, 0.f}, bf32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int cb = 0; cb < (NG + 3) / 4; ++cb) {
        __builtin_amdgcn_wave_barrier();  // the previous block's reads of the stage stay above
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int gg = 0; gg < 4; ++gg)
            if (4 * cb + gg < NG)
              st[(4 * kg + e) * kStageStride + 16 * gg + li] =
                  __uint_as_float((rp[e / 2][4 * cb + gg] >> (16 * (e % 2))) << 16);
        __builtin_amdgcn_wave_barrier();  // cross-lane: stores before the reads below
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          if (4 * cb + kk >= NG) break;  // compile-time
          const bf32x4 xr = *reinterpret_cast<const bf32x4*>(st + li * kStageStride + 16 * kk + 4 * kg);
          const zb_u32x2 bq = *reinterpret_cast<const zb_u32x2*>(sPhi16 + li * S16 + 64 * cb + 16 * kk + 4 * kg);
          const zb_s16x4 xa4 = __builtin_bit_cast(zb_s16x4, zb_u32x2{zb_pack_f(xr[0], xr[1]), zb_pack_f(xr[2], xr[3])});
          zacc[kk % 2] =
              __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xa4, __builtin_bit_cast(zb_s16x4, bq), zacc[kk % 2], 0, 0, 0);
        }
      }
      const bf32x4 z = zacc[0] + zacc[1];
      if (li < sQ) {
        const gptr<float> zo = Zo + (a * P + pb) * sQ + li;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (pb + 4 * kg + v < P) zo[(4 * kg + v) * sQ] = z[v];
      }
    }
    if (last_of_slab) {
      if (needW) {
        const gptr<float> wo = Wo + a * sP * Q;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (4 * kg + v < sP && qok[g]) wo[(4 * kg + v) * Q + 16 * g + li] = wacc[g][v];
          wacc[g] = bf32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
      a = a_next;
      if (a >= a_end) break;
    }
    step = step_next;
  }
}

// ------------------------------------------------------------------ core contractions
// Y = X x_k M (Y[a][i][b] = sum_c M[i][c] X[a][c][b], X viewed as (A, K, B), M: m x K with
// m <= 16 MT, K <= 256) for every tensor of the batch, on matrix cores.  A wave owns one
// unit (B == 1: four); a workgroup works on one job.
//  * B >= 16 (a mode other than the last): unit = (a, 64 columns of b), all m rows.  M is
//    staged once per workgroup in LDS (zero past m and past K).  Lane (li, kg) loads
//    X[a][c][b0 + 16 j + li] (j < 4: 16 lanes read consecutive elements of a row) as the
//    B operand of four 16-column tiles:
//     - binary32 X: c = c0 + 4 s + kg (s < 4) per chunk of 16 c, 16x16x4 binary32 products
//       with A = M[16 t + li][c] read from LDS stored c-major;
//     - bfloat16 X: c = c0 + 8 kg + e (e < 8) per chunk of 32 c, packed in pairs for
//       16x16x32 bfloat16 products with A = M[16 t + li][c0 + 8 kg ..] (eight consecutive
//       bfloat16 of the LDS copy stored row-major; M holds bfloat16 values, so the products
//       are exact and only the binary32 accumulation order differs from the binary32 path).
//    The next chunk is in flight while the current one is multiplied; columns past B read
//    column B - 1 (their outputs are not stored) and rows past K are zeroed.
//  * B == 1 (the last mode): unit = 16 rows a, all m, up to four units per wave.  M is staged
//    in LDS as [c][16 MT].  Each 64-wide block of c is read row by row with the lanes
//    along c (256 consecutive bytes per row), staged in the wave's LDS area and read back
//    as the A operand X[a0 + li][c]; B = M[16 t + li][c].
// (Reading M from global memory, 16 rows of one lane group at a time, measured 15-20 %
// slower; three chunks in flight per wave instead of one measured slower.)
constexpr int kTStage = 68;  // floats per staged row of 64 c: = 4 mod 64, conflict-free row reads
constexpr int kTBMaxK = 256;
typedef __bf16 tb_bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t tb_u32x4 __attribute__((ext_vector_type(4)));

template <typename TX, int MT, bool ROWS>
__global__ __launch_bounds__(kBThreads, 2) void ttm_batch_kernel(const GTtmJob* __restrict__ jobs,
                                                                const int32_t* __restrict__ blkjob) {
  constexpr bool kBF = std::is_same<TX, bf16_t>::value;
  // LDS: M (B >= 16: binary32 [c][16 MT], or bfloat16 [16 MT][kMS]; B == 1: binary32
  // [c][16 MT]), then for B == 1 the per-wave stages
  constexpr int kLds = kTBMaxK * 16 * MT + (ROWS ? kBWaves * 16 * kTStage : 0);
  __shared__ __align__(16) float lds[kLds];
  float* const sM = lds;
  const GTtmJob J = jobs[blkjob[blockIdx.x]];
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int li = lane % 16, kg = lane / 16;
  const int64_t unit = (blockIdx.x - J.blk0) * kBWaves + wave;
  const int64_t K = J.K, B = J.B, m = J.m;
  const gptr<const TX> X = global_ptr(static_cast<const TX*>(J.X));
  const gptr<const float> M = global_ptr(static_cast<const float*>(J.M));
  const gptr<float> Y = global_ptr(static_cast<float*>(J.Y));
  if constexpr (!ROWS) {
    constexpr int kCh = kBF ? 32 : 16;      // c per chunk
    constexpr int kRows = kBF ? 8 : 4;      // rows per lane per chunk
    const int64_t Kp = (K + kCh - 1) / kCh * kCh;
    const int kMS = static_cast<int>(Kp) + 8;  // bfloat16 row stride: 16-byte rows
    const bool live = unit < J.colblocks;
    const int64_t nb = (B + 63) / 64;
    const int64_t a = live ? unit / nb : 0, b0 = live ? (unit - a * nb) * 64 : 0;
    const gptr<const TX> xa = X + a * K * B;
    int64_t col[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t b = b0 + 16 * j + li;
      col[j] = b < B ? b : B - 1;
    }
    // raw values of the next chunk: binary32 rows c0 + 4 e + kg; bfloat16 rows
    // c0 + 8 kg + 2 w, c0 + 8 kg + 2 w + 1 packed in one word (low half first)
    float xn[kBF ? 1 : 4][4];
    uint32_t xp[kBF ? 4 : 1][4];
    auto load = [&](int64_t c0) {
      if constexpr (kBF) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int64_t c = c0 + 8 * kg + 2 * w;
          const int64_t c1 = c < K ? c : K - 1, c2 = c + 1 < K ? c + 1 : K - 1;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            xp[w][j] = static_cast<uint32_t>(xa[c1 * B + col[j]]) | (static_cast<uint32_t>(xa[c2 * B + col[j]]) << 16);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t c = c0 + 4 * e + kg;
          const int64_t cc = c < K ? c : K - 1;
#pragma unroll
          for (int j = 0; j < 4; ++j) xn[e][j] = widen<TX>(xa[cc * B + col[j]]);
        }
      }
    };
    if (live) load(0);  // in flight while M is staged
    // stage M (zero past m and past K)
    const int64_t rows = 16 * MT;
    for (int64_t idx = threadIdx.x; idx < Kp * rows; idx += kBThreads) {
      const int64_t c = idx / rows, i = idx - c * rows;
      const float v = (c < K && i < m) ? M[i * K + c] : 0.f;
      if constexpr (kBF)
        reinterpret_cast<bf16_t*>(sM)[i * kMS + c] = static_cast<bf16_t>(__float_as_uint(v) >> 16);
      else
        sM[idx] = v;
    }
    __syncthreads();
    if (!live) return;
    bf32x4 acc[MT][4];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[t][j] = bf32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t c0 = 0; c0 < K; c0 += kCh) {
      const bool full = c0 + kCh <= K;  // uniform: only the last chunk has rows past K
      if constexpr (kBF) {
        // B operand of tile j: rows c0 + 8 kg + e of column j, element e (pairs packed)
        tb_u32x4 op[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            uint32_t v = xp[w][j];
            if (!full) {
              const int64_t c = c0 + 8 * kg + 2 * w;
              v &= (c < K ? 0x0000ffffu : 0u) | (c + 1 < K ? 0xffff0000u : 0u);
            }
            op[j][w] = v;
          }
        if (c0 + kCh < K) load(c0 + kCh);
        const bf16_t* mb = reinterpret_cast<const bf16_t*>(sM);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          const tb_u32x4 av = *reinterpret_cast<const tb_u32x4*>(mb + (16 * t + li) * kMS + c0 + 8 * kg);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(tb_bf16x8, av),
                                                                __builtin_bit_cast(tb_bf16x8, op[j]), acc[t][j], 0,
                                                                0, 0);
        }
      } else {
        float xv[4][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool cin = full || c0 + 4 * e + kg < K;
#pragma unroll
          for (int j = 0; j < 4; ++j) xv[e][j] = cin ? xn[e][j] : 0.f;
        }
        if (c0 + kCh < K) load(c0 + kCh);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float* mc = sM + (c0 + 4 * e + kg) * rows + li;
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            const float mv = mc[16 * t];
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(mv, xv[e][j], acc[t][j], 0, 0, 0);
          }
        }
      }
    }
    // D[i = 4 kg + v][b = li] of tile (t, j)
    const gptr<float> ya = Y + a * m * B;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t i = 16 * t + 4 * kg + v, b = b0 + 16 * j + li;
          if (i < m && b < B) ya[i * B + b] = acc[t][j][v];
        }
  } else {
    // B == 1: tiles of 16 rows a of the A x K matrix X.  A workgroup takes 4 U consecutive
    // tiles (U = J.mtiles, from ttm_batch_row_tiles); wave w takes tiles 4 u + w (u < U),
    // and the first block of its next tile is in flight during the last block of the
    // current one.
    const int64_t A = J.A;
    const int64_t U = J.mtiles;
    const int64_t tile0 = (blockIdx.x - J.blk0) * kBWaves * U + wave;
    const int64_t tile_end = J.colblocks;
    const int64_t rows = 16 * MT;
    float* st = lds + kTBMaxK * 16 * MT + wave * 16 * kTStage;
    TX xn[16];
    auto load = [&](int64_t a0, int64_t c0) {
      const int64_t c = c0 + lane;
      const int64_t cc = c < K ? c : K - 1;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t a = a0 + i < A ? a0 + i : A - 1;
        xn[i] = X[a * K + cc];
      }
    };
    if (tile0 < tile_end) load(tile0 * 16, 0);  // in flight while M is staged
    // stage M as [c][16 MT] (zero past m and past K, up to the next multiple of 64)
    const int64_t Kp = (K + 63) / 64 * 64;
    for (int64_t idx = threadIdx.x; idx < Kp * rows; idx += kBThreads) {
      const int64_t c = idx / rows, i = idx - c * rows;
      sM[idx] = (c < K && i < m) ? M[i * K + c] : 0.f;
    }
    __syncthreads();
    const int64_t tile_last = tile0 + kBWaves * (U - 1) < tile_end ? tile0 + kBWaves * (U - 1) : tile_end - 1;
    for (int64_t tile = tile0; tile <= tile_last; tile += kBWaves) {
      const int64_t a0 = tile * 16;
      bf32x4 acc[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[t] = bf32x4{0.f, 0.f, 0.f, 0.f};
      for (int64_t c0 = 0; c0 < K; c0 += 64) {
        const bool cin = c0 + lane < K;
        float xv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) xv[i] = (cin && a0 + i < A) ? widen<TX>(xn[i]) : 0.f;
        if (c0 + 64 < K)
          load(a0, c0 + 64);
        else if (tile + kBWaves <= tile_last)
          load(a0 + 16 * kBWaves, 0);
        __builtin_amdgcn_wave_barrier();  // the previous block's reads of the stage stay above
#pragma unroll
        for (int i = 0; i < 16; ++i) st[i * kTStage + lane] = xv[i];
        __builtin_amdgcn_wave_barrier();  // cross-lane: stores before the reads below
#pragma unroll 4
        for (int kk = 0; kk < 64; kk += 4) {
          const float av = st[li * kTStage + kk + kg];
          const float* mc = sM + (c0 + kk + kg) * rows + li;
#pragma unroll
          for (int t = 0; t < MT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, mc[16 * t], acc[t], 0, 0, 0);
        }
      }
      // D[a = a0 + 4 kg + v][i = 16 t + li]
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t a = a0 + 4 * kg + v, i = 16 * t + li;
          if (a < A && i < m) Y[a * m + i] = acc[t][v];
        }
    }
  }
}

}  // namespace

int zw_batch_class(int64_t Q) {
  const int ng = static_cast<int>((Q + 15) / 16);
  return ng <= 4 ? 4 : ng <= 8 ? 8 : ng <= 12 ? 12 : 16;
}

hipError_t launch_zw_batch(const GZwJob* jobs, const int32_t* blkjob, int64_t total_blocks, int ng, rt_dtype xdt,
                           hipStream_t st) {
  if (total_blocks == 0) return hipSuccess;
  const unsigned g = static_cast<unsigned>(total_blocks);
#define RT_ZWB(TX, N) zw_batch_kernel<TX, N><<<g, kBThreads, 0, st>>>(jobs, blkjob)
#define RT_ZWB_NG(TX)                 \
  switch (ng) {                       \
    case 4: RT_ZWB(TX, 4); break;     \
    case 8: RT_ZWB(TX, 8); break;     \
    case 12: RT_ZWB(TX, 12); break;   \
    case 16: RT_ZWB(TX, 16); break;   \
    default: return hipErrorInvalidValue; \
  }
  if (xdt == RT_F32) {
    RT_ZWB_NG(float)
  } else if (xdt == RT_BF16) {
    switch (ng) {
      case 4: zw_batch_bf16_kernel<4><<<g, kBThreads, 0, st>>>(jobs, blkjob); break;
      case 8: zw_batch_bf16_kernel<8><<<g, kBThreads, 0, st>>>(jobs, blkjob); break;
      case 12: zw_batch_bf16_kernel<12><<<g, kBThreads, 0, st>>>(jobs, blkjob); break;
      case 16: zw_batch_bf16_kernel<16><<<g, kBThreads, 0, st>>>(jobs, blkjob); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef RT_ZWB_NG
#undef RT_ZWB
  return hipGetLastError();
}

int64_t ttm_batch_units(int64_t A, int64_t B) { return B == 1 ? (A + 15) / 16 : A * ((B + 63) / 64); }
bool ttm_batch_fits(int64_t K, int64_t B, int64_t m) { return (B == 1 || B >= 16) && K <= kTBMaxK && m <= 64; }
int64_t ttm_batch_row_tiles(int64_t A, int64_t B) {
  if (B != 1) return 1;
  const int64_t units = ttm_batch_units(A, B);
  return units >= 1024 ? 4 : units >= 512 ? 2 : 1;  // long jobs: fewer M stagings per row
}
int64_t ttm_batch_blocks(int64_t A, int64_t B) {
  const int64_t per = kBWaves * ttm_batch_row_tiles(A, B);
  return (ttm_batch_units(A, B) + per - 1) / per;
}

hipError_t launch_ttm_batch(const GTtmJob* jobs, const int32_t* blkjob, int64_t total_blocks, int mt, bool rows,
                            rt_dtype xdt, hipStream_t st) {
  if (total_blocks == 0) return hipSuccess;
  const unsigned g = static_cast<unsigned>(total_blocks);
#define RT_TB(TX, N)                                                         \
  if (rows)                                                                  \
    ttm_batch_kernel<TX, N, true><<<g, kBThreads, 0, st>>>(jobs, blkjob);    \
  else                                                                       \
    ttm_batch_kernel<TX, N, false><<<g, kBThreads, 0, st>>>(jobs, blkjob)
#define RT_TB_MT(TX)                      \
  switch (mt) {                           \
    case 1: RT_TB(TX, 1); break;          \
    case 2: RT_TB(TX, 2); break;          \
    case 3: RT_TB(TX, 3); break;          \
    case 4: RT_TB(TX, 4); break;          \
    default: return hipErrorInvalidValue; \
  }
  if (xdt == RT_F32) {
    RT_TB_MT(float)
  } else if (xdt == RT_BF16) {
    RT_TB_MT(bf16_t)
  } else {
    return hipErrorInvalidValue;
  }
#undef RT_TB_MT
#undef RT_TB
  return hipGetLastError();
}

}  // namespace rt

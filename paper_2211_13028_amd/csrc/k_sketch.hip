// First level of the all-at-once sketch (Alg. 4.4 sketch step with the
// dimension tree of Sec. 4.4): one streaming pass over X, viewed as (A, P, Q)
// with P, Q the sizes of the last two modes, computes both
//   Z = X x_d Phi_d        (the node shared by every sketch that contracts mode d)
//   W = X x_{d-1} Phi_{d-1} (the node of the mode-d sketch)
// so X is read from HBM exactly once for all modes; every later contraction of
// the tree runs on Z or W, which are smaller by I_d/s_d and I_{d-1}/s_{d-1}.
//
// Layout: a 256-thread workgroup owns one slab X[a] (or a row range of it) and a
// range of up to 64*NQ columns.  Lane l holds columns q0 + l + 64*j (coalesced
// row reads), the matching Phi_Q entries in registers, and W accumulators for
// its columns; each row's Z values are reduced across the wave.  Phi_P[:, p]
// is wave-uniform (scalar loads).  Row ranges or column ranges split over
// several workgroups produce partial sums that a second kernel adds in a fixed
// order.
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kZWThreads = 256;
constexpr int kZWWaves = kZWThreads / kWave;

template <typename TX, typename TC, int NQ, int SMAX>
__global__ __launch_bounds__(kZWThreads) void sketch_zw_kernel(const TX* __restrict__ X, int64_t A, int64_t P,
                                                               int64_t Q, const TC* __restrict__ phiP, int sP,
                                                               const TC* __restrict__ phiQ, int sQ,
                                                               int64_t rows_per_block, int qblocks, int pblocks,
                                                               TC* __restrict__ Zo, TC* __restrict__ Wo) {
  extern __shared__ unsigned char zw_smem[];
  TC* sW = reinterpret_cast<TC*>(zw_smem);  // [waves][sP][64*NQ]
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t blk = blockIdx.x;
  const int qblk = static_cast<int>(blk % qblocks);
  const int64_t rest = blk / qblocks;
  const int pblk = static_cast<int>(rest % pblocks);
  const int64_t a = rest / pblocks;
  const int64_t q0 = static_cast<int64_t>(qblk) * 64 * NQ;
  const bool needZ = Zo != nullptr, needW = Wo != nullptr;

  TC phq[NQ][SMAX];
  TC wacc[NQ][SMAX];
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    const int64_t q = q0 + lane + 64 * j;
#pragma unroll
    for (int c = 0; c < SMAX; ++c) {
      phq[j][c] = (needZ && q < Q && c < sQ) ? phiQ[c * Q + q] : TC(0);
      wacc[j][c] = TC(0);
    }
  }
  const int64_t pbeg = static_cast<int64_t>(pblk) * rows_per_block;
  const int64_t pend = (pbeg + rows_per_block < P) ? pbeg + rows_per_block : P;
  const TX* xa = X + a * P * Q;
  TC* zrow = needZ ? Zo + (static_cast<int64_t>(qblk) * A + a) * P * sQ : nullptr;
  for (int64_t p = pbeg + wave; p < pend; p += kZWWaves) {
    TC x[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int64_t q = q0 + lane + 64 * j;
      x[j] = (q < Q) ? static_cast<TC>(Load<TX>::get(xa, p * Q + q)) : TC(0);
    }
    if (needW) {
#pragma unroll
      for (int c = 0; c < SMAX; ++c) {
        const TC f = (c < sP) ? phiP[c * P + p] : TC(0);
#pragma unroll
        for (int j = 0; j < NQ; ++j) wacc[j][c] = fma(f, x[j], wacc[j][c]);
      }
    }
    if (needZ) {
      TC z[SMAX];
#pragma unroll
      for (int c = 0; c < SMAX; ++c) {
        TC s = TC(0);
#pragma unroll
        for (int j = 0; j < NQ; ++j) s = fma(x[j], phq[j][c], s);
        z[c] = s;
      }
#pragma unroll
      for (int c = 0; c < SMAX; ++c)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) z[c] += __shfl_xor(z[c], off);
      // lane c stores z[c]
      TC mine = TC(0);
#pragma unroll
      for (int c = 0; c < SMAX; ++c)
        if (lane == c) mine = z[c];
      if (lane < sQ) zrow[p * sQ + lane] = mine;
    }
  }
  if (!needW) return;
  const int width = 64 * NQ;
#pragma unroll
  for (int j = 0; j < NQ; ++j)
#pragma unroll
    for (int c = 0; c < SMAX; ++c)
      if (c < sP) sW[(wave * sP + c) * width + lane + 64 * j] = wacc[j][c];
  __syncthreads();
  TC* wout = Wo + (static_cast<int64_t>(pblk) * A + a) * sP * Q;
  for (int idx = threadIdx.x; idx < sP * width; idx += kZWThreads) {
    const int c = idx / width, col = idx % width;
    const int64_t q = q0 + col;
    if (q >= Q) continue;
    TC s = TC(0);
    for (int w = 0; w < kZWWaves; ++w) s += sW[(w * sP + c) * width + col];
    wout[c * Q + q] = s;
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void sum_parts_kernel(const TC* __restrict__ part, int parts, int64_t n,
                                                        TC* __restrict__ out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
    TC s = part[i];
    for (int k = 1; k < parts; ++k) s += part[k * n + i];
    out[i] = s;
  }
}

// ------------------------------------------------------------------ bfloat16 / FP8 on matrix cores
// Same two contractions on MFMA (v_mfma_f32_16x16x32_bf16, binary32 accumulation).
// FP8 e4m3 data is widened exactly to bfloat16 as it is loaded, so it streams at
// one byte per element and multiplies as the FP8 values themselves.
// A workgroup of four waves covers 512 columns of a row range; wave w owns the
// 128 columns q0 + 128 w .. + 127 and all waves step through the rows together,
// 32 at a time:
//  * W^T tile: out[c][q] = sum_p PhiP[c][p] X[p][q].  Each lane loads an 8 x 8
//    block (8 rows, 8 consecutive columns, 16 bytes per row) and re-packs it in
//    registers into 8 operands holding 8 consecutive p of one column; the wave
//    keeps its 16 x 128 accumulator for the whole row range (no cross-wave sum).
//  * Z tile: out[p][c] = sum_q X[p][q] PhiQ[c][q] over the wave's 128 columns,
//    with the X rows staged row-major in the wave's LDS area as the A operand;
//    the four waves' partial Z rows are added in LDS in a fixed order, one
//    barrier per step (double-buffered partials).
// The next 32 rows are loaded while the current ones are used.  Rows beyond P and
// operand rows beyond s are zero.  Requires P % 8 == 0, Q % 8 == 0, s <= 8.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kZWColsMfma = 512;
constexpr int kTileStride = 136;  // bf16 per staged row: 128 columns + 8 padding (spreads LDS banks)

__device__ __forceinline__ u32x4 ld16(const bf16_t* p) { return *reinterpret_cast<const u32x4*>(p); }

// Raw loads of an 8-row x 8-column block (row t: 8 consecutive columns) and their
// widening to bfloat16 pairs.  The widening happens when a prefetched block is
// used, so the loads stay in flight across the previous step.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <typename TX>
struct BlockIO;

template <>
struct BlockIO<bf16_t> {
  typedef u32x4 raw_t;  // 8 bfloat16
  static __device__ __forceinline__ raw_t load(const bf16_t* p) { return *reinterpret_cast<const u32x4*>(p); }
  static __device__ __forceinline__ raw_t zero() { return u32x4{0u, 0u, 0u, 0u}; }
  static __device__ __forceinline__ u32x4 widen(raw_t v) { return v; }
};

// FP8 e4m3: 8 bytes per row, widened exactly to bfloat16 (every e4m3 value is a
// bfloat16 value) by the hardware conversion, so the products are the FP8 ones
template <>
struct BlockIO<f8_t> {
  typedef u32x2 raw_t;
  static __device__ __forceinline__ raw_t load(const f8_t* p) { return *reinterpret_cast<const u32x2*>(p); }
  static __device__ __forceinline__ raw_t zero() { return u32x2{0u, 0u}; }
  static __device__ __forceinline__ u32x4 widen(raw_t v) {
    return u32x4{__builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v[0], 1.0f, false)),
                 __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v[0], 1.0f, true)),
                 __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v[1], 1.0f, false)),
                 __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v[1], 1.0f, true))};
  }
};

template <typename TX>
__global__ __launch_bounds__(kZWThreads) __attribute__((amdgpu_waves_per_eu(3))) void sketch_zw_bf16_mfma_kernel(
    const TX* __restrict__ X, int64_t A, int64_t P, int64_t Q, const bf16_t* __restrict__ phiP, int sP,
    const bf16_t* __restrict__ phiQ, int sQ, int64_t rows_per_block, int qblocks, int pblocks,
    float* __restrict__ Zo, float* __restrict__ Wo) {
  __shared__ bf16_t tile[kZWWaves][32 * kTileStride];
  __shared__ float zpart[2][kZWWaves][32 * 16];
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t blk = blockIdx.x;
  const int qblk = static_cast<int>(blk % qblocks);
  const int64_t rest = blk / qblocks;
  const int pblk = static_cast<int>(rest % pblocks);
  const int64_t a = rest / pblocks;
  const int64_t q0 = static_cast<int64_t>(qblk) * kZWColsMfma;
  const int64_t qend = (q0 + kZWColsMfma < Q) ? q0 + kZWColsMfma : Q;
  const int64_t qw = q0 + 128 * wave;  // this wave's columns
  const bool needZ = Zo != nullptr, needW = Wo != nullptr;
  const int li = lane % 16, kg = lane / 16;
  const int64_t pbeg = static_cast<int64_t>(pblk) * rows_per_block;
  const int64_t pend = (pbeg + rows_per_block < P) ? pbeg + rows_per_block : P;
  const TX* xa = X + a * P * Q;
  bf16_t* my = tile[wave];
  const int64_t qc = qw + 8 * li;
  const bool colok = qc < qend;

  // loop-invariant PhiQ operands of the Z product: row c = li, 8 columns per k group
  u32x4 bq[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int64_t qk = qw + 32 * ks + 8 * kg;
    bq[ks] = (needZ && qk < qend) ? ld16(phiQ + static_cast<int64_t>(li) * Q + qk) : u32x4{0u, 0u, 0u, 0u};
  }
  f32x4 wacc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) wacc[c] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Lane (li, kg) loads rows p0 + 8 kg + t (t < 8), columns qc..qc+7.  Loads carry no
  // conditions: an 8-row group past pend reads the last 8 rows of the range and a column
  // group past qend the last 8 columns of the block (8-row groups lie wholly inside or
  // outside [pbeg, pend) because P % 8 == 0 and steps are 32 rows; Q % 8 == 0); such
  // values are zeroed when the block is taken over.
  const int64_t qcc = colok ? qc : qend - 8;
  // The PhiP operand of the W product (row c = li, columns pc .. pc + 7) comes with the
  // rows, clamped and zeroed the same way.
  typename BlockIO<TX>::raw_t rn[8];
  u32x4 ppn = u32x4{0u, 0u, 0u, 0u};
  const auto load = [&](int64_t pb) {
    const int64_t p = pb + 8 * kg;
    const int64_t pc = (p < pend) ? p : pend - 8;
    // without W the load reads an entry of PhiQ (in bounds: Z is then computed) and is unused
    ppn = ld16(needW ? phiP + static_cast<int64_t>(li) * P + pc : phiQ + static_cast<int64_t>(li) * Q + (qend - 8));
#pragma unroll
    for (int t = 0; t < 8; ++t) rn[t] = BlockIO<TX>::load(xa + (pc + t) * Q + qcc);
  };
  if (pbeg < pend) load(pbeg);
  int buf = 0;
  for (int64_t pb = pbeg; pb < pend; pb += 32) {
    const int64_t pc = pb + 8 * kg;
    const bool in = colok && pc < pend;
    u32x4 r[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const u32x4 w = BlockIO<TX>::widen(rn[t]);
      r[t] = in ? w : u32x4{0u, 0u, 0u, 0u};
    }
    const u32x4 pp = (pc < pend) ? ppn : u32x4{0u, 0u, 0u, 0u};
    __builtin_amdgcn_sched_barrier(0);
    load(pb + 32);  // past pend: clamped, never used
    __builtin_amdgcn_sched_barrier(0);
    if (needZ) {
      __builtin_amdgcn_wave_barrier();  // the previous step's reads of the staging area stay above
#pragma unroll
      for (int t = 0; t < 8; ++t) *reinterpret_cast<u32x4*>(my + (8 * kg + t) * kTileStride + 8 * li) = r[t];
      __builtin_amdgcn_wave_barrier();  // cross-lane: stores before the reads below
      f32x4 zacc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const u32x4 xr = *reinterpret_cast<const u32x4*>(my + (16 * mt + li) * kTileStride + 32 * ks + 8 * kg);
          zacc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, xr),
                                                              __builtin_bit_cast(bf16x8, bq[ks]), zacc[mt], 0, 0, 0);
        }
      // partial Z rows of this wave: D layout row 16 mt + 4 kg + v, column c = li
      float* zp = zpart[buf][wave];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) zp[(16 * mt + 4 * kg + v) * 16 + li] = zacc[mt][v];
      lds_barrier();  // the next rows' loads stay in flight
      // wave w finishes rows 8 w .. 8 w + 7 of the step: lane -> (row, c < 8)
      const int row = 8 * wave + lane / 8, c = lane % 8;
      const int64_t p = pb + row;
      float z = zpart[buf][0][row * 16 + c];
#pragma unroll
      for (int w = 1; w < kZWWaves; ++w) z += zpart[buf][w][row * 16 + c];
      if (c < sQ && p < pend) Zo[((static_cast<int64_t>(qblk) * A + a) * P + p) * sQ + c] = z;
      buf ^= 1;
    }
    if (needW) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        u32x4 op;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t lo = r[2 * w][c / 2], hi = r[2 * w + 1][c / 2];
          op[w] = (c % 2 == 0) ? ((lo & 0xffffu) | (hi << 16)) : ((lo >> 16) | (hi & 0xffff0000u));
        }
        wacc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, pp),
                                                          __builtin_bit_cast(bf16x8, op), wacc[c], 0, 0, 0);
      }
    }
  }
  if (!needW || !colok) return;
  // W^T accumulators: row cp = 4 kg + v, column qc + c
  float* wout = Wo + (static_cast<int64_t>(pblk) * A + a) * sP * Q;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int cp = 4 * kg + v;
    if (cp >= sP) continue;
    float* dst = wout + static_cast<int64_t>(cp) * Q + qc;
    *reinterpret_cast<f32x4*>(dst) = f32x4{wacc[0][v], wacc[1][v], wacc[2][v], wacc[3][v]};
    *reinterpret_cast<f32x4*>(dst + 4) = f32x4{wacc[4][v], wacc[5][v], wacc[6][v], wacc[7][v]};
  }
}

// ------------------------------------------------------------------ binary32 on matrix cores
// The same pass for binary32 X with v_mfma_f32_16x16x4f32.  Wave w owns 128
// columns; all waves step through 16 rows at a time.  Lane (li, kg) loads row
// 4t + kg of each row quad t as two 16-byte groups (columns 4 li.. and 64 + 4 li..):
//  * W^T: A = PhiP[c][p] (one value per lane), B = the loaded groups, component c
//    giving columns 4 n + c, so four MFMAs cover 64 columns per row quad;
//  * Z: the 16 x 128 tile is staged row-major in the wave's LDS area, 64 columns at a
//    time, and read back with lane (row li, 4 consecutive columns at 4 kg) as A; PhiQ is B, staged in LDS
//    once per workgroup when s <= 8 (read from the caches, the 16 rows of a lane group
//    touched 16 cache lines per load every step), else read from the caches.  Partial Z
//    rows are added across the waves in LDS (fixed order).
// Requires Q % 4 == 0; P, A arbitrary; s <= 16.
constexpr int kF32Stride = 68;  // floats per staged row: 64 + 4 padding (rows four banks apart)
constexpr int kPhiQRows = 8;                     // PhiQ rows kept in LDS (s <= 8)
constexpr int kPhiQStride = kZWColsMfma + 8;     // floats per row: 16-byte rows, rows 8 banks apart

template <bool QLDS>
__global__ __launch_bounds__(kZWThreads) __attribute__((amdgpu_waves_per_eu(3))) void sketch_zw_f32_mfma_kernel(
    const float* __restrict__ X, int64_t A, int64_t P, int64_t Q, const float* __restrict__ phiP, int sP,
    const float* __restrict__ phiQ, int sQ, int64_t rows_per_block, int qblocks, int pblocks,
    float* __restrict__ Zo, float* __restrict__ Wo) {
  __shared__ float tile[kZWWaves][16 * kF32Stride];
  __shared__ float zpart[2][kZWWaves][16 * 16];
  __shared__ __align__(16) float sPhiQ[QLDS ? kPhiQRows * kPhiQStride : 4];  // PhiQ rows < 8 of the block's columns
  __shared__ float sPhiP[QLDS ? 2 * 256 : 1];  // PhiP of a step, [parity][p - pb][c]
  const int lane = threadIdx.x % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t blk = blockIdx.x;
  const int qblk = static_cast<int>(blk % qblocks);
  const int64_t rest = blk / qblocks;
  const int pblk = static_cast<int>(rest % pblocks);
  const int64_t a = rest / pblocks;
  const int64_t q0 = static_cast<int64_t>(qblk) * kZWColsMfma;
  const int64_t qend = (q0 + kZWColsMfma < Q) ? q0 + kZWColsMfma : Q;
  const int64_t qw = q0 + 128 * wave;
  const bool needZ = Zo != nullptr, needW = Wo != nullptr;
  const int li = lane % 16, kg = lane / 16;
  const int64_t pbeg = static_cast<int64_t>(pblk) * rows_per_block;
  const int64_t pend = (pbeg + rows_per_block < P) ? pbeg + rows_per_block : P;
  const float* xa = X + a * P * Q;
  float* my = tile[wave];
  const int64_t qc[2] = {qw + 4 * li, qw + 64 + 4 * li};
  const bool ok[2] = {qc[0] < qend, qc[1] < qend};

  f32x4 wacc[2][4];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) wacc[j][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  // The next step's rows and PhiP values are loaded while the current step is multiplied.
  // Loads carry no per-lane conditions: a row past pend reads row pend - 1 and a column
  // group past qend the last group of the block (Q % 4 == 0); such values are zeroed when
  // the step is taken over.  Without W the PhiP load reads an entry of PhiQ (in bounds:
  // Z is then computed) and is unused.
  const int64_t qcc[2] = {ok[0] ? qc[0] : qend - 4, ok[1] ? qc[1] : qend - 4};
  f32x4 rn[4][2];
  float ppn[4];
  auto load_step = [&](int64_t pb) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t p = pb + 4 * t + kg;
      const int64_t pc = (p < pend) ? p : pend - 1;
      if constexpr (!QLDS)
        ppn[t] = *(needW ? phiP + static_cast<int64_t>(li) * P + pc : phiQ + static_cast<int64_t>(li) * Q + (qend - 4));
#pragma unroll
      for (int j = 0; j < 2; ++j) rn[t][j] = *reinterpret_cast<const f32x4*>(xa + pc * Q + qcc[j]);
    }
  };
  load_step(pbeg);  // in flight while PhiQ is staged
  // QLDS: the PhiP rows of a step are staged in LDS during the step before (thread: c = tid / 16,
  // p = pb + tid % 16, zero past pend), loaded one step earlier still; the Z path's barrier
  // of each step orders the stores before the next step's reads
  const int pc_c = threadIdx.x / 16, pc_p = threadIdx.x % 16;
  const auto phip_at = [&](int64_t pb) {
    const int64_t p = pb + pc_p;
    return (needW && p < pend) ? phiP[static_cast<int64_t>(pc_c) * P + p] : 0.f;
  };
  float pvn = 0.f;
  if constexpr (QLDS) {
    sPhiP[pc_p * 16 + pc_c] = phip_at(pbeg);
    pvn = phip_at(pbeg + 16);
  }
  // PhiQ (sQ <= 8) for the block's 512 columns in LDS, zero past sQ and past qend
  if (QLDS && needZ) {
    for (int g = threadIdx.x; g < kPhiQRows * (kZWColsMfma / 4); g += kZWThreads) {
      const int c = g / (kZWColsMfma / 4), q4 = 4 * (g % (kZWColsMfma / 4));
      f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
      if (c < sQ && q0 + q4 < qend) v = *reinterpret_cast<const f32x4*>(phiQ + static_cast<int64_t>(c) * Q + q0 + q4);
      *reinterpret_cast<f32x4*>(&sPhiQ[c * kPhiQStride + q4]) = v;
    }
  }
  __syncthreads();
  int buf = 0;
  for (int64_t pb = pbeg; pb < pend; pb += 16) {
    f32x4 r[4][2];
    float ppv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool pin = pb + 4 * t + kg < pend;
#pragma unroll
      for (int j = 0; j < 2; ++j) r[t][j] = (ok[j] && pin) ? rn[t][j] : f32x4{0.f, 0.f, 0.f, 0.f};
      if constexpr (QLDS)
        ppv[t] = pin ? sPhiP[buf * 256 + (4 * t + kg) * 16 + li] : 0.f;
      else
        ppv[t] = pin ? ppn[t] : 0.f;
    }
    if constexpr (QLDS) {
      sPhiP[(buf ^ 1) * 256 + pc_p * 16 + pc_c] = pvn;  // the next step's rows
      pvn = phip_at(pb + 32);
    }
    __builtin_amdgcn_sched_barrier(0);
    load_step(pb + 16);  // past pend: clamped, never used
    __builtin_amdgcn_sched_barrier(0);
    if (needW) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float pp = ppv[t];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int c = 0; c < 4; ++c)
            wacc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(pp, r[t][j][c], wacc[j][c], 0, 0, 0);
      }
    }
    if (needZ) {
      f32x4 zacc = f32x4{0.f, 0.f, 0.f, 0.f};
      // the 16 x 128 tile in two halves of 64 columns (a 16 x 64 stage per wave)
#pragma unroll
      for (int kb = 0; kb < 8; ++kb) {
        if (kb % 4 == 0) {
          __builtin_amdgcn_wave_barrier();  // the previous half's reads of the stage stay above
#pragma unroll
          for (int t = 0; t < 4; ++t)
            *reinterpret_cast<f32x4*>(my + (4 * t + kg) * kF32Stride + 4 * li) = r[t][kb / 4];
          __builtin_amdgcn_wave_barrier();  // cross-lane: stores before the reads below
        }
        // PhiQ[li][qw + 16 kb + 4 kg .. + 3]: a small operand re-read from the caches each step
        // (holding it in registers would cost the occupancy)
        const int64_t qk = qw + 16 * kb + 4 * kg;
        f32x4 bq;
        if constexpr (QLDS) {
          bq = *reinterpret_cast<const f32x4*>(&sPhiQ[(li & (kPhiQRows - 1)) * kPhiQStride + (qk - q0)]);
          if (li >= kPhiQRows) bq = f32x4{0.f, 0.f, 0.f, 0.f};
        } else {
          bq = *reinterpret_cast<const f32x4*>(phiQ + static_cast<int64_t>(li) * Q + ((qk < qend) ? qk : qend - 4));
          if (!(qk < qend)) bq = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        const f32x4 xr = *reinterpret_cast<const f32x4*>(my + li * kF32Stride + 16 * (kb % 4) + 4 * kg);
#pragma unroll
        for (int c = 0; c < 4; ++c) zacc = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[c], bq[c], zacc, 0, 0, 0);
      }
      float* zp = zpart[buf][wave];
#pragma unroll
      for (int v = 0; v < 4; ++v) zp[(4 * kg + v) * 16 + li] = zacc[v];
      lds_barrier();  // the next rows' loads stay in flight
      // wave w finishes rows 4 w .. 4 w + 3 of the step: lane -> (row, c)
      const int row = 4 * wave + lane / 16, c = lane % 16;
      const int64_t p = pb + row;
      float z = zpart[buf][0][row * 16 + c];
#pragma unroll
      for (int w = 1; w < kZWWaves; ++w) z += zpart[buf][w][row * 16 + c];
      if (c < sQ && p < pend) Zo[((static_cast<int64_t>(qblk) * A + a) * P + p) * sQ + c] = z;
      buf ^= 1;
    }
  }
  if (!needW) return;
  float* wout = Wo + (static_cast<int64_t>(pblk) * A + a) * sP * Q;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (!ok[j]) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cp = 4 * kg + v;
      if (cp < sP)
        *reinterpret_cast<f32x4*>(wout + static_cast<int64_t>(cp) * Q + qc[j]) =
            f32x4{wacc[j][0][v], wacc[j][1][v], wacc[j][2][v], wacc[j][3][v]};
    }
  }
}

int nq_max(rt_dtype xdt) { return xdt == RT_F64 ? 4 : 8; }

int pick_nq(rt_dtype xdt, int64_t Q) {
  const int64_t need = ceil_div(Q, 64);
  const int mx = nq_max(xdt);
  int nq = 1;
  while (nq < need && nq < mx) nq *= 2;
  return nq;
}

template <typename TX, typename TC>
hipError_t zw_dispatch(const TX* X, int64_t A, int64_t P, int64_t Q, const TC* phiP, int sP, const TC* phiQ, int sQ,
                       TC* Zo, TC* Wo, const ZWPlan& plan, int nq, hipStream_t st) {
  const int smax = (sP > sQ ? sP : sQ) <= 4 ? 4 : 8;
  const int64_t blocks = A * plan.pblocks * plan.qblocks;
  const size_t shmem = Wo ? static_cast<size_t>(kZWWaves) * sP * 64 * nq * sizeof(TC) : 0;
#define RT_ZW(NQV, SV)                                                                                        \
  sketch_zw_kernel<TX, TC, NQV, SV><<<static_cast<unsigned>(blocks), kZWThreads, shmem, st>>>(               \
      X, A, P, Q, phiP, sP, phiQ, sQ, plan.rows_per_block, static_cast<int>(plan.qblocks),                      \
      static_cast<int>(plan.pblocks), Zo, Wo)
  if (smax == 4) {
    switch (nq) {
      case 1: RT_ZW(1, 4); break;
      case 2: RT_ZW(2, 4); break;
      case 4: RT_ZW(4, 4); break;
      default: RT_ZW(8, 4); break;
    }
  } else {
    switch (nq) {
      case 1: RT_ZW(1, 8); break;
      case 2: RT_ZW(2, 8); break;
      case 4: RT_ZW(4, 8); break;
      default: RT_ZW(8, 8); break;
    }
  }
#undef RT_ZW
  return hipGetLastError();
}

}  // namespace

bool sketch_zw_ok(rt_dtype, int64_t sP, int64_t sQ) { return sP >= 1 && sQ >= 1 && sP <= 8 && sQ <= 8; }

ZWPlan sketch_zw_plan(rt_dtype xdt, int64_t A, int64_t P, int64_t Q, int64_t sP, int64_t sQ, bool needZ,
                      bool needW) {
  ZWPlan p;
  const bool mf16 = (xdt == RT_BF16 || xdt == RT_F8E4M3) && (P % 8 == 0) && (Q % 8 == 0) && P >= 32;
  const bool mf32 = (xdt == RT_F32) && (Q % 4 == 0) && P >= 16;
  p.mfma = mf16 || mf32;
  const int nq = pick_nq(xdt, Q);
  p.qblocks = p.mfma ? ceil_div(Q, kZWColsMfma) : ceil_div(Q, 64 * nq);
  if (p.mfma) {
    // Row split for the matrix-core pass: 768 workgroups are resident at once
    // (3 per CU).  Cost in units of "one row per resident workgroup":
    //   rows_per_block * max(1, workgroups / 768)  +  partial-W traffic of pb row ranges,
    // with the W partials (written and re-read, binary32) converted at the
    // 1 KiB of X that one row of 512 bfloat16 columns is.  A grid of at least one full
    // round streams at about the same rate whether its last round is full or not (the
    // pass is bound by HBM), so rounds count fractionally; a grid below one round is
    // bound by its longest workgroup.  (Counting the last round as full chose three row
    // ranges for 1024 x 1024 x 512 binary32, 20 us per decomposition slower than one.)
    const int64_t resident = 768;
    const int64_t step = mf32 ? 16 : 32;  // rows per step of the kernel
    const double row_bytes = static_cast<double>(resident) * kZWColsMfma * (mf32 ? 4 : 2);
    double best = 0.0;
    int64_t best_rows = 0;
    for (int64_t pb = 1; pb <= 64; ++pb) {
      const int64_t rows = ceil_div(ceil_div(P, pb), step) * step;
      const int64_t pbs = ceil_div(P, rows);
      if (pbs != pb || (pb > 1 && rows < 128)) continue;
      const int64_t wgs = A * p.qblocks * pb;
      const double rounds = wgs > resident ? static_cast<double>(wgs) / resident : 1.0;
      const double t = rounds * rows +
                       (pb > 1 && needW ? 2.0 * pb * A * sP * Q * 4.0 / row_bytes : 0.0);
      if (best_rows == 0 || t < best) {
        best = t;
        best_rows = rows;
      }
    }
    p.rows_per_block = best_rows ? best_rows : ceil_div(P, step) * step;
  } else {
    int64_t pb = 1;
    const int64_t target = 2048;
    if (A * p.qblocks < target) pb = ceil_div(target, A * p.qblocks);
    const int64_t maxpb = ceil_div(P, 16);  // keep at least 16 rows per block
    if (pb > maxpb) pb = maxpb;
    if (pb < 1) pb = 1;
    p.rows_per_block = ceil_div(P, pb);
  }
  p.pblocks = ceil_div(P, p.rows_per_block);
  const size_t esz = (xdt == RT_F64) ? 8 : 4;
  size_t ws = 0;
  if (needZ && p.qblocks > 1) ws += align256(static_cast<size_t>(p.qblocks) * A * P * sQ * esz);
  if (needW && p.pblocks > 1) ws += align256(static_cast<size_t>(p.pblocks) * A * sP * Q * esz);
  p.ws_bytes = ws;
  return p;
}

hipError_t launch_sketch_zw(const void* X, rt_dtype xdt, int64_t A, int64_t P, int64_t Q, const void* phiP, int64_t sP,
                            const void* phiQ, int64_t sQ, const void* phiP16, const void* phiQ16, void* Z, void* W,
                            const ZWPlan& plan, void* ws, hipStream_t st) {
  const int nq = pick_nq(xdt, Q);
  const size_t esz = (xdt == RT_F64) ? 8 : 4;
  char* wsp = static_cast<char*>(ws);
  void* zdst = Z;
  void* wdst = W;
  if (Z && plan.qblocks > 1) {
    zdst = wsp;
    wsp += align256(static_cast<size_t>(plan.qblocks) * A * P * sQ * esz);
  }
  if (W && plan.pblocks > 1) {
    wdst = wsp;
    wsp += align256(static_cast<size_t>(plan.pblocks) * A * sP * Q * esz);
  }
  hipError_t e;
  const int isP = static_cast<int>(sP), isQ = static_cast<int>(sQ);
  if (plan.mfma) {
    const int64_t blocks = A * plan.pblocks * plan.qblocks;
    if (xdt == RT_F32) {
      if (sQ <= kPhiQRows && zdst != nullptr)
        sketch_zw_f32_mfma_kernel<true><<<static_cast<unsigned>(blocks), kZWThreads, 0, st>>>(
            static_cast<const float*>(X), A, P, Q, static_cast<const float*>(phiP16), isP,
            static_cast<const float*>(phiQ16), isQ, plan.rows_per_block, static_cast<int>(plan.qblocks),
            static_cast<int>(plan.pblocks), static_cast<float*>(zdst), static_cast<float*>(wdst));
      else
        sketch_zw_f32_mfma_kernel<false><<<static_cast<unsigned>(blocks), kZWThreads, 0, st>>>(
            static_cast<const float*>(X), A, P, Q, static_cast<const float*>(phiP16), isP,
            static_cast<const float*>(phiQ16), isQ, plan.rows_per_block, static_cast<int>(plan.qblocks),
            static_cast<int>(plan.pblocks), static_cast<float*>(zdst), static_cast<float*>(wdst));
    }
    else if (xdt == RT_F8E4M3)
      sketch_zw_bf16_mfma_kernel<f8_t><<<static_cast<unsigned>(blocks), kZWThreads, 0, st>>>(
          static_cast<const f8_t*>(X), A, P, Q, static_cast<const bf16_t*>(phiP16), isP,
          static_cast<const bf16_t*>(phiQ16), isQ, plan.rows_per_block, static_cast<int>(plan.qblocks),
          static_cast<int>(plan.pblocks), static_cast<float*>(zdst), static_cast<float*>(wdst));
    else
      sketch_zw_bf16_mfma_kernel<bf16_t><<<static_cast<unsigned>(blocks), kZWThreads, 0, st>>>(
          static_cast<const bf16_t*>(X), A, P, Q, static_cast<const bf16_t*>(phiP16), isP,
          static_cast<const bf16_t*>(phiQ16), isQ, plan.rows_per_block, static_cast<int>(plan.qblocks),
          static_cast<int>(plan.pblocks), static_cast<float*>(zdst), static_cast<float*>(wdst));
    e = hipGetLastError();
  } else
  switch (xdt) {
    case RT_F64:
      e = zw_dispatch<double, double>(static_cast<const double*>(X), A, P, Q, static_cast<const double*>(phiP), isP,
                                      static_cast<const double*>(phiQ), isQ, static_cast<double*>(zdst),
                                      static_cast<double*>(wdst), plan, nq, st);
      break;
    case RT_F32:
      e = zw_dispatch<float, float>(static_cast<const float*>(X), A, P, Q, static_cast<const float*>(phiP), isP,
                                    static_cast<const float*>(phiQ), isQ, static_cast<float*>(zdst),
                                    static_cast<float*>(wdst), plan, nq, st);
      break;
    case RT_BF16:
      e = zw_dispatch<bf16_t, float>(static_cast<const bf16_t*>(X), A, P, Q, static_cast<const float*>(phiP), isP,
                                     static_cast<const float*>(phiQ), isQ, static_cast<float*>(zdst),
                                     static_cast<float*>(wdst), plan, nq, st);
      break;
    default:
      e = zw_dispatch<f8_t, float>(static_cast<const f8_t*>(X), A, P, Q, static_cast<const float*>(phiP), isP,
                                   static_cast<const float*>(phiQ), isQ, static_cast<float*>(zdst),
                                   static_cast<float*>(wdst), plan, nq, st);
      break;
  }
  if (e != hipSuccess) return e;
  // fixed-order sums of the partials
  if (Z && plan.qblocks > 1) {
    const int64_t n = A * P * sQ;
    const unsigned g = static_cast<unsigned>(ceil_div(n, 256) > 4096 ? 4096 : ceil_div(n, 256));
    if (xdt == RT_F64)
      sum_parts_kernel<double><<<g, 256, 0, st>>>(static_cast<const double*>(zdst), static_cast<int>(plan.qblocks), n,
                                                  static_cast<double*>(Z));
    else
      sum_parts_kernel<float><<<g, 256, 0, st>>>(static_cast<const float*>(zdst), static_cast<int>(plan.qblocks), n,
                                                 static_cast<float*>(Z));
  }
  if (W && plan.pblocks > 1) {
    const int64_t n = A * sP * Q;
    const unsigned g = static_cast<unsigned>(ceil_div(n, 256) > 4096 ? 4096 : ceil_div(n, 256));
    if (xdt == RT_F64)
      sum_parts_kernel<double><<<g, 256, 0, st>>>(static_cast<const double*>(wdst), static_cast<int>(plan.pblocks), n,
                                                  static_cast<double*>(W));
    else
      sum_parts_kernel<float><<<g, 256, 0, st>>>(static_cast<const float*>(wdst), static_cast<int>(plan.pblocks), n,
                                                 static_cast<float*>(W));
  }
  return hipGetLastError();
}

}  // namespace rt

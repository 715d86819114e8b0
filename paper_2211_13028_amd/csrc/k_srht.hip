// Subsampled randomized Hadamard sketch along the contiguous last mode (Sec. 5.1):
//   Z = X x_d Phi,  Phi = (R H D)[:, :Q]  (Q = I_d zero-padded to N = 2^m),
// by a fast Walsh-Hadamard transform of every fiber instead of a product with the
// dense s x Q factor.  One wave per fiber: lane l holds the N/64 entries l, l + 64, ...
// (each load instruction reads 64 consecutive values), so the transform's butterflies
// over the high index bits stay in registers and those over the six low bits are lane
// exchanges; the s sampled outputs are read back through LDS.
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kSrhtWaves = 4;

// make LDS data written by other lanes of this wave visible to the next reads of this wave
__device__ __forceinline__ void srht_wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// E = N / 64 entries per lane (N >= 64), or 1 for N < 64; F fibers per wave per iteration
// (several fibers' loads in flight at once for the short ones)
template <int E, int F>
__global__ __launch_bounds__(kSrhtWaves * kWave) void srht_last_kernel(const float* __restrict__ X, int64_t fibers,
                                                                        int Q, int N, const int64_t* __restrict__ rows,
                                                                        const double* __restrict__ signs, int s,
                                                                        float inv, float* __restrict__ Z) {
  __shared__ float buf[kSrhtWaves][F][64 * E];
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  float sg[E];
#pragma unroll
  for (int t = 0; t < E; ++t) {
    const int i = t * kWave + lane;
    sg[t] = (i < Q) ? static_cast<float>(signs[i]) : 0.f;
  }
  // the sampled row this lane reads back (lanes >= s read nothing); clamped into [0, N)
  const int row = (lane < s) ? static_cast<int>(rows[lane] & static_cast<int64_t>(N - 1)) : 0;
  const int64_t per_wave_iter = F;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * kSrhtWaves;
  for (int64_t f0 = (static_cast<int64_t>(blockIdx.x) * kSrhtWaves + wave) * per_wave_iter; f0 < fibers;
       f0 += waves * per_wave_iter) {
    float v[F][E];
#pragma unroll
    for (int u = 0; u < F; ++u) {
      const int64_t f = f0 + u;
      const float* x = X + ((f < fibers) ? f : 0) * static_cast<int64_t>(Q);
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int i = t * kWave + lane;
        v[u][t] = (f < fibers && i < Q) ? x[i] * sg[t] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < F; ++u) {
      // butterflies over the index bits held in registers (bit h of t)
#pragma unroll
      for (int h = 1; h < E; h <<= 1) {
#pragma unroll
        for (int t = 0; t < E; ++t) {
          if (t & h) continue;
          const float a = v[u][t], b = v[u][t + h];
          v[u][t] = a + b;
          v[u][t + h] = a - b;
        }
      }
      // butterflies over the lane bits: the partner's value by a lane exchange
      for (int m = 1; m < kWave && m < N; m <<= 1) {
#pragma unroll
        for (int t = 0; t < E; ++t) {
          const float o = __shfl_xor(v[u][t], m);
          v[u][t] = (lane & m) ? (o - v[u][t]) : (v[u][t] + o);
        }
      }
#pragma unroll
      for (int t = 0; t < E; ++t) buf[wave][u][t * kWave + lane] = v[u][t];
    }
    srht_wave_lds_sync();  // this wave's stores before its lanes read each other's entries
#pragma unroll
    for (int u = 0; u < F; ++u) {
      const int64_t f = f0 + u;
      const float z = buf[wave][u][row];
      if (f < fibers && lane < s) Z[f * s + lane] = z * inv;
    }
    srht_wave_lds_sync();  // the reads done before the next iteration's stores
  }
}

}  // namespace

bool srht_last_ok(int64_t Q, int64_t s) {
  int64_t N = 1;
  while (N < Q) N *= 2;
  return Q >= 1 && N <= 4096 && s >= 1 && s <= 64 && s <= N;
}

hipError_t launch_srht_last(const float* X, int64_t fibers, int64_t Q, const int64_t* rows, const double* signs,
                            int64_t s, float* Z, hipStream_t st) {
  int N = 1;
  while (N < Q) N *= 2;
  const float inv = static_cast<float>(1.0 / std::sqrt(static_cast<double>(N)));
  const int e = N >= kWave ? N / kWave : 1;
  const int F = e >= 16 ? 1 : (e >= 8 ? 2 : 4);  // at least about 2 KB of X per wave in flight
  const int64_t waves_needed = ceil_div(fibers, F);
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(ceil_div(waves_needed, kSrhtWaves), 256 * 16));
#define RT_SRHT(EV, FV)                                                                                         \
  srht_last_kernel<EV, FV><<<grid, kSrhtWaves * kWave, 0, st>>>(X, fibers, static_cast<int>(Q), N, rows,      \
                                                                signs, static_cast<int>(s), inv, Z)
  switch (e) {
    case 1: RT_SRHT(1, 4); break;
    case 2: RT_SRHT(2, 4); break;
    case 4: RT_SRHT(4, 4); break;
    case 8: RT_SRHT(8, 2); break;
    case 16: RT_SRHT(16, 1); break;
    case 32: RT_SRHT(32, 1); break;
    default: RT_SRHT(64, 1); break;
  }
#undef RT_SRHT
  return hipGetLastError();
}

}  // namespace rt

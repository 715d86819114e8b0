// Elementwise kernels: precision conversion, operand preparation, unfolding,
// squared residual.  Plain memory-bound grid-stride loops.
#include <algorithm>

#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kThreads = 256;
constexpr int kReduceBlocks = 1024;  // fixed grid of the deterministic reductions

__device__ __forceinline__ double load_as_f64(const void* p, rt_dtype dt, int64_t i) {
  switch (dt) {
    case RT_F64: return static_cast<const double*>(p)[i];
    case RT_F32: return static_cast<double>(static_cast<const float*>(p)[i]);
    case RT_BF16: return static_cast<double>(bf16_to_f32(static_cast<const bf16_t*>(p)[i]));
    default: return static_cast<double>(f8_to_f32(static_cast<const f8_t*>(p)[i]));
  }
}

// value of x after rounding to `fmt` (binary64 result, exact)
__device__ __forceinline__ double round_value(double x, rt_dtype fmt) {
  switch (fmt) {
    case RT_F64: return x;
    case RT_F32: return static_cast<double>(static_cast<float>(x));
    case RT_BF16: return static_cast<double>(bf16_to_f32(f64_to_bf16_bits(x)));
    default: return static_cast<double>(f8_to_f32(f64_to_f8_bits(x)));
  }
}

__device__ __forceinline__ void store_rounded(void* dst, rt_dtype store, rt_dtype fmt, int64_t i, double x) {
  switch (store) {
    case RT_F64: static_cast<double*>(dst)[i] = round_value(x, fmt); break;
    case RT_F32: static_cast<float*>(dst)[i] = static_cast<float>(round_value(x, fmt)); break;
    // a bfloat16 store of a value rounded to FP8 first is exact (matrix-core operands of FP8 data)
    case RT_BF16: static_cast<bf16_t*>(dst)[i] = f64_to_bf16_bits(fmt == RT_BF16 ? x : round_value(x, fmt)); break;
    default: static_cast<f8_t*>(dst)[i] = f64_to_f8_bits(x); break;
  }
}

__global__ __launch_bounds__(kThreads) void convert_kernel(const void* src, rt_dtype sdt, void* dst,
                                                           rt_dtype ddt, int64_t n, double scale) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const double x = load_as_f64(src, sdt, i) * scale;  // power-of-two scale: exact
    store_rounded(dst, ddt, ddt, i, x);
  }
}

// binary32 -> bfloat16 bits, round to nearest even: adding 0x7fff plus the lowest kept
// bit to the bit pattern and dropping 16 bits is exact RNE for every finite binary32
// value (subnormals included) and carries overflow into the infinity pattern.
__device__ __forceinline__ uint32_t f32_bits_to_bf16(uint32_t u) {
  if ((u & 0x7fffffffu) > 0x7f800000u) return ((u >> 16) & 0x8000u) | 0x7fc0u;  // NaN
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// The binary32 -> bfloat16 (or E4M3) cast of a whole tensor, the one pass that turns an
// FP32 input into the narrow operand of the precision form: each thread moves 4 x 16
// bytes per iteration (four independent loads in flight) and writes 4 x 8 (4 x 4) bytes.
constexpr int kCastVec = 4;  // float4 loads per thread per iteration

template <bool kF8> struct CastOut;
template <> struct CastOut<false> {
  typedef uint2 vec;  // four bfloat16 values
  __device__ static vec pack(float4 v) {
    const uint32_t a = f32_bits_to_bf16(__float_as_uint(v.x)), b = f32_bits_to_bf16(__float_as_uint(v.y));
    const uint32_t c = f32_bits_to_bf16(__float_as_uint(v.z)), d = f32_bits_to_bf16(__float_as_uint(v.w));
    return uint2{a | (b << 16), c | (d << 16)};
  }
  __device__ static void one(void* dst, int64_t i, float x) {
    static_cast<bf16_t*>(dst)[i] = static_cast<bf16_t>(f32_bits_to_bf16(__float_as_uint(x)));
  }
};
template <> struct CastOut<true> {
  typedef uint32_t vec;  // four E4M3 values (binary32 -> binary64 is exact, then one rounding)
  __device__ static vec pack(float4 v) {
    return static_cast<uint32_t>(f64_to_f8_bits(v.x)) | (static_cast<uint32_t>(f64_to_f8_bits(v.y)) << 8) |
           (static_cast<uint32_t>(f64_to_f8_bits(v.z)) << 16) | (static_cast<uint32_t>(f64_to_f8_bits(v.w)) << 24);
  }
  __device__ static void one(void* dst, int64_t i, float x) { static_cast<f8_t*>(dst)[i] = f64_to_f8_bits(x); }
};

template <bool kF8>
__global__ __launch_bounds__(kThreads) void cast_f32_kernel(const float4* __restrict__ src,
                                                             typename CastOut<kF8>::vec* __restrict__ dst,
                                                             int64_t nvec) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads * kCastVec;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads * kCastVec + threadIdx.x; base < nvec;
       base += stride) {
    float4 v[kCastVec];
#pragma unroll
    for (int u = 0; u < kCastVec; ++u) {
      const int64_t i = base + static_cast<int64_t>(u) * kThreads;
      v[u] = i < nvec ? src[i] : float4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < kCastVec; ++u) {
      const int64_t i = base + static_cast<int64_t>(u) * kThreads;
      if (i < nvec) dst[i] = CastOut<kF8>::pack(v[u]);
    }
  }
}

template <bool kF8>
__global__ __launch_bounds__(kThreads) void cast_f32_tail_kernel(const float* __restrict__ src, void* dst,
                                                                  int64_t off, int64_t n) {
  const int64_t i = off + static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) CastOut<kF8>::one(dst, i, src[i]);
}

template <bool kF8>
void launch_cast_f32(const float* src, void* dst, int64_t n, hipStream_t st) {
  const int64_t nvec = n / 4;
  if (nvec > 0) {
    // enough workgroups to fill every CU many times over; each thread then loops
    const int64_t per_block = static_cast<int64_t>(kThreads) * kCastVec;
    const int64_t blocks = std::min<int64_t>(ceil_div(nvec, per_block), 256 * 32);
    cast_f32_kernel<kF8><<<static_cast<unsigned>(blocks), kThreads, 0, st>>>(
        reinterpret_cast<const float4*>(src), static_cast<typename CastOut<kF8>::vec*>(dst), nvec);
  }
  if (n > nvec * 4) cast_f32_tail_kernel<kF8><<<1, kThreads, 0, st>>>(src, dst, nvec * 4, n);
}

__global__ __launch_bounds__(kThreads) void prep_kernel(const double* src, int64_t m, int64_t K, bool trans,
                                                        rt_dtype round_to, rt_dtype store, int64_t m_pad,
                                                        void* dst) {
  const int64_t total = m_pad * K;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / K, k = t - i * K;
    double x = 0.0;
    if (i < m) x = trans ? src[k * m + i] : src[i * K + k];
    store_rounded(dst, store, round_to, t, x);
  }
}

__global__ __launch_bounds__(kThreads) void prep_batch_kernel(PrepTable tab) {
  const PrepTask& T = tab.t[blockIdx.y];
  const int64_t total = T.m_pad * T.K;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / T.K, k = t - i * T.K;
    double x = 0.0;
    if (i < T.m) x = T.trans ? T.src[k * T.m + i] : T.src[i * T.K + k];
    store_rounded(T.dst, T.store, T.round_to, t, x);
  }
}

// f32 operand of the matrix-core TTM from a caller's f32 matrix: rows >= m zero
__global__ __launch_bounds__(kThreads) void pack_f32_kernel(const float* __restrict__ src, int64_t m, int64_t K,
                                                            bool trans, int64_t m_pad, float* __restrict__ dst) {
  const int64_t total = m_pad * K;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / K, k = t - i * K;
    dst[t] = (i < m) ? (trans ? src[k * m + i] : src[i * K + k]) : 0.f;
  }
}

__global__ __launch_bounds__(kThreads) void prep_grouped_kernel(const PrepTask* __restrict__ tasks) {
  const PrepTask T = tasks[blockIdx.y];
  const int64_t total = T.m_pad * T.K;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; t < total; t += stride) {
    const int64_t i = t / T.K, k = t - i * T.K;
    double x = 0.0;
    if (i < T.m) x = T.trans ? T.src[k * T.m + i] : T.src[i * T.K + k];
    store_rounded(T.dst, T.store, T.round_to, t, x);
  }
}

__global__ __launch_bounds__(kThreads) void copy_f64_grouped_kernel(const GCopyJob* __restrict__ jobs) {
  const GCopyJob J = jobs[blockIdx.y];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; t < J.n; t += stride)
    J.dst[t] = static_cast<double>(J.src[t]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void unfold_kernel(const T* src, int64_t A, int64_t m, int64_t B, T* dst) {
  const int64_t total = A * m * B;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; t < total; t += stride) {
    // t indexes the destination (i, a, b)
    const int64_t i = t / (A * B);
    const int64_t rem = t - i * (A * B);
    const int64_t a = rem / B, b = rem - a * B;
    dst[t] = src[a * m * B + i * B + b];
  }
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // fixed-order tree: wave shuffles then waves in order
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < kThreads / kWave; ++i) s += sh[i];
  }
  __syncthreads();
  return s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void sq_residual_kernel(const T* a, const T* b, T* r, int64_t n,
                                                               double* partial) {
  __shared__ double sh[kThreads / kWave];
  double acc = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const T d = a[i] - b[i];
    if (r) r[i] = d;
    acc += static_cast<double>(d) * static_cast<double>(d);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out = alpha * g[0] * (a - b); g and b may be null (then 1 and 0)
template <typename T>
__global__ __launch_bounds__(kThreads) void scaled_diff_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                               const double* __restrict__ g, double alpha,
                                                               int64_t n, T* __restrict__ out) {
  const T f = static_cast<T>(g ? alpha * g[0] : alpha);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const T d = b ? a[i] - b[i] : a[i];
    out[i] = f * d;
  }
}

__global__ __launch_bounds__(kThreads) void sum_partials_kernel(const double* partial, int count, double* out) {
  __shared__ double sh[kThreads / kWave];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += kThreads) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = s;
}

int grid_for(int64_t n) {
  const int64_t g = ceil_div(n, kThreads);
  return static_cast<int>(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

// Walsh-Hadamard entries in Sylvester order: H[i][j] = (-1)^popcount(i & j).  One thread
// per entry of the s x n factor (a few thousand entries).
__global__ __launch_bounds__(kThreads) void srht_factor_kernel(int64_t n, int64_t s, const int64_t* __restrict__ rows,
                                                                const double* __restrict__ signs, double inv,
                                                                double* __restrict__ phi) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (t >= n * s) return;
  const int64_t i = t / n, j = t - i * n;
  const uint64_t bits = static_cast<uint64_t>(rows[i]) & static_cast<uint64_t>(j);
  const double h = (__popcll(bits) & 1) ? -inv : inv;
  phi[t] = h * signs[j];
}

hipError_t launch_srht_factor(int64_t n, int64_t s, const int64_t* rows, const double* signs, double inv_sqrt_N,
                              double* phi, hipStream_t st) {
  srht_factor_kernel<<<static_cast<unsigned>(ceil_div(n * s, kThreads)), kThreads, 0, st>>>(n, s, rows, signs,
                                                                                            inv_sqrt_N, phi);
  return hipGetLastError();
}

hipError_t launch_convert(const void* src, rt_dtype sdt, void* dst, rt_dtype ddt, int64_t n, int scale_exp,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  // binary32 sources at 16-byte alignment take the vectorised cast (no scaling: the
  // E4M3 saturation would otherwise have to see the scaled value)
  const bool vec_src = sdt == RT_F32 && scale_exp == 0 && (reinterpret_cast<uintptr_t>(src) & 15u) == 0;
  if (vec_src && ddt == RT_BF16 && (reinterpret_cast<uintptr_t>(dst) & 7u) == 0) {
    launch_cast_f32<false>(static_cast<const float*>(src), dst, n, st);
    return hipGetLastError();
  }
  if (vec_src && ddt == RT_F8E4M3 && (reinterpret_cast<uintptr_t>(dst) & 3u) == 0) {
    launch_cast_f32<true>(static_cast<const float*>(src), dst, n, st);
    return hipGetLastError();
  }
  const double scale = ldexp(1.0, scale_exp);
  convert_kernel<<<grid_for(n), kThreads, 0, st>>>(src, sdt, dst, ddt, n, scale);
  return hipGetLastError();
}

hipError_t launch_prep_matrix(const double* src, int64_t m, int64_t K, bool trans, rt_dtype round_to,
                              rt_dtype store, int64_t m_pad, void* dst, hipStream_t st) {
  if (m_pad < m) m_pad = m;
  prep_kernel<<<grid_for(m_pad * K), kThreads, 0, st>>>(src, m, K, trans, round_to, store, m_pad, dst);
  return hipGetLastError();
}

hipError_t launch_prep_batch(const PrepTask* tasks, int count, hipStream_t st) {
  for (int i0 = 0; i0 < count; i0 += kMaxPrepTasks) {
    PrepTable tab;
    const int cnt = (count - i0 < kMaxPrepTasks) ? count - i0 : kMaxPrepTasks;
    int64_t most = 1;
    for (int i = 0; i < cnt; ++i) {
      tab.t[i] = tasks[i0 + i];
      const int64_t n = tasks[i0 + i].m_pad * tasks[i0 + i].K;
      if (n > most) most = n;
    }
    const int64_t g = ceil_div(most, kThreads);
    prep_batch_kernel<<<dim3(static_cast<unsigned>(g > 256 ? 256 : g), cnt), kThreads, 0, st>>>(tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pack_f32(const float* src, int64_t m, int64_t K, bool trans, int64_t m_pad, float* dst,
                           hipStream_t st) {
  if (m_pad < m) m_pad = m;
  pack_f32_kernel<<<grid_for(m_pad * K), kThreads, 0, st>>>(src, m, K, trans, m_pad, dst);
  return hipGetLastError();
}

hipError_t launch_prep_grouped(const PrepTask* tasks, int count, int64_t max_elems, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int64_t g = ceil_div(max_elems, kThreads);
  prep_grouped_kernel<<<dim3(static_cast<unsigned>(g > 64 ? 64 : (g < 1 ? 1 : g)), count), kThreads, 0, st>>>(tasks);
  return hipGetLastError();
}

hipError_t launch_copy_f64_grouped(const GCopyJob* jobs, int count, int64_t max_elems, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int64_t g = ceil_div(max_elems, kThreads);
  copy_f64_grouped_kernel<<<dim3(static_cast<unsigned>(g > 64 ? 64 : (g < 1 ? 1 : g)), count), kThreads, 0, st>>>(
      jobs);
  return hipGetLastError();
}

hipError_t launch_unfold(const void* src, size_t esize, int64_t A, int64_t m, int64_t B, void* dst,
                         hipStream_t st) {
  const int64_t n = A * m * B;
  if (n == 0) return hipSuccess;
  if (esize == 8)
    unfold_kernel<double><<<grid_for(n), kThreads, 0, st>>>(static_cast<const double*>(src), A, m, B,
                                                            static_cast<double*>(dst));
  else
    unfold_kernel<float><<<grid_for(n), kThreads, 0, st>>>(static_cast<const float*>(src), A, m, B,
                                                           static_cast<float*>(dst));
  return hipGetLastError();
}

size_t sq_residual_ws(int64_t) { return align256(kReduceBlocks * sizeof(double)); }

hipError_t launch_sq_residual(const void* a, const void* b, void* r, rt_dtype dt, int64_t n, double* out,
                              void* ws, hipStream_t st) {
  double* partial = static_cast<double*>(ws);
  if (dt == RT_F64)
    sq_residual_kernel<double><<<kReduceBlocks, kThreads, 0, st>>>(
        static_cast<const double*>(a), static_cast<const double*>(b), static_cast<double*>(r), n, partial);
  else
    sq_residual_kernel<float><<<kReduceBlocks, kThreads, 0, st>>>(
        static_cast<const float*>(a), static_cast<const float*>(b), static_cast<float*>(r), n, partial);
  sum_partials_kernel<<<1, kThreads, 0, st>>>(partial, kReduceBlocks, out);
  return hipGetLastError();
}

hipError_t launch_scaled_diff(const void* a, const void* b, const double* g, double alpha, rt_dtype dt, int64_t n,
                              void* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (dt == RT_F64)
    scaled_diff_kernel<double><<<grid_for(n), kThreads, 0, st>>>(static_cast<const double*>(a),
                                                                static_cast<const double*>(b), g, alpha, n,
                                                                static_cast<double*>(out));
  else
    scaled_diff_kernel<float><<<grid_for(n), kThreads, 0, st>>>(static_cast<const float*>(a),
                                                               static_cast<const float*>(b), g, alpha, n,
                                                               static_cast<float*>(out));
  return hipGetLastError();
}

}  // namespace rt

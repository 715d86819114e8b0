// Relative reconstruction error by explicit residual, in binary64 (Sec. 5):
// the host contracts all modes but the first into T = G x_2 U_2 ... x_d U_d
// (r1 x prod_{k>1} I_k), and this kernel streams X once, reconstructing each
// element as U_1[i, :] . T[:, b] and accumulating ||X - X_hat||^2, ||X||^2 and the
// count of non-finite entries.  Fixed-order reductions (bitwise reproducible).
#include "kernels.hpp"

namespace rt {

namespace {

constexpr int kRThreads = 256;
constexpr int kRowChunk = 32;

template <typename TX, int RMAX>
__global__ __launch_bounds__(kRThreads) void recon_residual_kernel(const TX* __restrict__ X, int64_t I1, int64_t Brest,
                                                                   const double* __restrict__ U1,
                                                                   const double* __restrict__ T, int r1,
                                                                   double* __restrict__ part) {
  __shared__ double sU[kRowChunk][RMAX];
  __shared__ double red[3][kRThreads / kWave];
  const int64_t b = static_cast<int64_t>(blockIdx.x) * kRThreads + threadIdx.x;
  const bool active = b < Brest;
  double t[RMAX];
#pragma unroll
  for (int a = 0; a < RMAX; ++a) t[a] = (active && a < r1) ? T[a * Brest + b] : 0.0;
  double s_res = 0.0, s_x = 0.0, s_bad = 0.0;
  for (int64_t i0 = 0; i0 < I1; i0 += kRowChunk) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kRowChunk * RMAX; idx += kRThreads) {
      const int ii = idx / RMAX, a = idx % RMAX;
      sU[ii][a] = (i0 + ii < I1 && a < r1) ? U1[(i0 + ii) * r1 + a] : 0.0;
    }
    __syncthreads();
    if (active) {
      const int iend = static_cast<int>((I1 - i0) < kRowChunk ? (I1 - i0) : kRowChunk);
      for (int ii = 0; ii < iend; ++ii) {
        double xh = 0.0;
#pragma unroll
        for (int a = 0; a < RMAX; ++a) xh = fma(sU[ii][a], t[a], xh);
        const double x = static_cast<double>(Load<TX>::get(X, (i0 + ii) * Brest + b));
        if (!isfinite(x)) {
          s_bad += 1.0;
        } else {
          const double d = x - xh;
          s_res = fma(d, d, s_res);
          s_x = fma(x, x, s_x);
        }
      }
    }
  }
  // fixed-order block reduction
  for (int off = 32; off >= 1; off >>= 1) {
    s_res += __shfl_xor(s_res, off);
    s_x += __shfl_xor(s_x, off);
    s_bad += __shfl_xor(s_bad, off);
  }
  const int w = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) { red[0][w] = s_res; red[1][w] = s_x; red[2][w] = s_bad; }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int i = 0; i < kRThreads / kWave; ++i) s += red[threadIdx.x][i];
    part[static_cast<int64_t>(blockIdx.x) * 3 + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void residual_finish_kernel(const double* __restrict__ part, int blocks,
                                                              double* __restrict__ out) {
  __shared__ double red[3][4];
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < blocks; i += 256)
    for (int k = 0; k < 3; ++k) s[k] += part[static_cast<int64_t>(i) * 3 + k];
  for (int k = 0; k < 3; ++k)
    for (int off = 32; off >= 1; off >>= 1) s[k] += __shfl_xor(s[k], off);
  if (threadIdx.x % kWave == 0)
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x / kWave] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
    out[0] = v[0];
    out[1] = v[1];
    out[3] = v[2];
  }
}

__global__ __launch_bounds__(256) void sumsq_kernel(const double* __restrict__ g, int64_t n, double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s = fma(g[i], g[i], s);
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

template <typename TX>
hipError_t dispatch(const TX* X, int64_t I1, int64_t Brest, const double* U1, const double* T, int64_t r1,
                    double* part, unsigned blocks, hipStream_t st) {
  const int r = static_cast<int>(r1);
  if (r <= 16)
    recon_residual_kernel<TX, 16><<<blocks, kRThreads, 0, st>>>(X, I1, Brest, U1, T, r, part);
  else if (r <= 32)
    recon_residual_kernel<TX, 32><<<blocks, kRThreads, 0, st>>>(X, I1, Brest, U1, T, r, part);
  else
    recon_residual_kernel<TX, 64><<<blocks, kRThreads, 0, st>>>(X, I1, Brest, U1, T, r, part);
  return hipGetLastError();
}

}  // namespace

size_t recon_residual_ws(int64_t, int64_t Brest) {
  return align256(static_cast<size_t>(ceil_div(Brest, kRThreads)) * 3 * sizeof(double));
}

hipError_t launch_recon_residual(const void* X, rt_dtype xdt, int64_t I1, int64_t Brest, const double* U1,
                                 const double* T, int64_t r1, double* out, void* ws, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>(ceil_div(Brest, kRThreads));
  double* part = static_cast<double*>(ws);
  hipError_t e;
  switch (xdt) {
    case RT_F64: e = dispatch(static_cast<const double*>(X), I1, Brest, U1, T, r1, part, blocks, st); break;
    case RT_F32: e = dispatch(static_cast<const float*>(X), I1, Brest, U1, T, r1, part, blocks, st); break;
    case RT_BF16: e = dispatch(static_cast<const bf16_t*>(X), I1, Brest, U1, T, r1, part, blocks, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  residual_finish_kernel<<<1, 256, 0, st>>>(part, static_cast<int>(blocks), out);
  return hipGetLastError();
}

hipError_t launch_sumsq_f64(const double* g, int64_t n, double* out_slot, hipStream_t st) {
  sumsq_kernel<<<1, 256, 0, st>>>(g, n, out_slot);
  return hipGetLastError();
}

}  // namespace rt

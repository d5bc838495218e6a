// libpdyn_peaks: the two machine rates that the roofline of the dynamics
// kernels is measured against, timed in the same run as the kernels
// (measurement only; not part of the dynamics library's C ABI).
//   peaks_fma   FP32 or FP64 vector FMA throughput: every lane runs kChains
//               independent FMA chains, so issue, not latency, bounds it. Built
//               like the dynamics kernels, with packed FP32 disabled, so each
//               FP32 FMA is one scalar v_fma per lane: the rate the dynamics
//               kernels can reach.
//   peaks_copy  HBM bandwidth: a grid-stride copy of 16-byte words between two
//               caller buffers larger than the last-level cache.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 16;

template <class T>
__global__ void __launch_bounds__(256) k_fma(int iters, T a0, T b0, T* out) {
  // per-lane coefficients, so that every FMA takes three vector-register operands
  const T a = a0 - (T)threadIdx.x * (T)1e-9;
  const T b = b0 * (T)(threadIdx.x + 1);
  T x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (T)(threadIdx.x + c);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = x[c] * a + b;
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  // a value only the host can tell apart, so the chains are not removed
  if (s == (T)-12345.678) out[0] = s;
}

__global__ void __launch_bounds__(256) k_copy(int64_t n16, const uint4* __restrict__ src, uint4* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// FMA chains: blocks x 256 threads, iters x kChains FMAs per thread (2 flop
// each). double_precision selects T. out: one element of T (device), written
// only in a case that never happens. Returns 0, or -4 if the launch failed.
int peaks_fma(int double_precision, int blocks, int iters, void* out, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (double_precision)
    hipLaunchKernelGGL(k_fma<double>, dim3(blocks), dim3(256), 0, s, iters, 0.999999, 1e-7,
                       static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_fma<float>, dim3(blocks), dim3(256), 0, s, iters, 0.999999f, 1e-7f,
                       static_cast<float*>(out));
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int peaks_fma_chains(void) { return kChains; }

// dst[0 .. bytes) = src[0 .. bytes); bytes a multiple of 16, both 16-byte aligned.
int peaks_copy(const void* src, void* dst, int64_t bytes, int blocks, void* stream) {
  if (bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16) return -1;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), bytes / 16,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst));
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"

// Device helpers for the gfx950 kernels: wave64 reductions and checked launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace tpo {

constexpr int kWave = 64;

#define TPO_HIP_CHECK(expr)                                                      \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw std::runtime_error(std::string("HIP error ") + hipGetErrorString(e_) \
                               + " at " + __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

#define TPO_LAUNCH_CHECK() TPO_HIP_CHECK(hipGetLastError())

inline unsigned ceil_div(int64_t a, int64_t b) { return static_cast<unsigned>((a + b - 1) / b); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Atomic max of a non-negative float stored as its bit pattern.
__device__ __forceinline__ void atomic_max_nonneg(uint32_t* addr, float v) {
  atomicMax(addr, __float_as_uint(v));
}

}  // namespace tpo

// Device helpers for the gfx950 kernels: wave64 reductions and checked launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
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

// OCP FP8 E4M3 (e4m3fn: exponent bias 7, 3 mantissa bits, subnormals below
// 2^-6, no infinities) code of a float, round to nearest even, saturating at
// +-448 (the largest finite value); NaN gives 0x7F.  Written from the
// format's definition; the same function serves device code and the
// library's host entry point tpo_e4m3_encode.
__host__ __device__ inline uint8_t e4m3_encode(float v) {
  const uint8_t sign = (v < 0.0f || (v == 0.0f && 1.0f / v < 0.0f)) ? 0x80 : 0x00;
  const float a = fabsf(v);
  if (!(a == a)) return 0x7F;
  if (a >= 448.0f) return static_cast<uint8_t>(sign | 0x7E);
  auto rne = [](float q) -> int {  // q >= 0, exact in float
    const float f = floorf(q);
    const float r = q - f;
    int i = static_cast<int>(f);
    if (r > 0.5f || (r == 0.5f && (i & 1))) ++i;
    return i;
  };
  int e;
  (void)frexpf(a, &e);  // a = m 2^e, m in [0.5, 1)
  int E = e - 1;        // a = (1 + f / 8) 2^E for a normal value
  if (a == 0.0f || E < -6) {
    // subnormal: a = f 2^-9, f in 0..7 (f = 8 is the smallest normal, 0x08)
    return static_cast<uint8_t>(sign | rne(a * 512.0f));
  }
  int f = rne((ldexpf(a, -E) - 1.0f) * 8.0f);
  if (f == 8) {
    f = 0;
    ++E;
  }
  if (E > 8 || (E == 8 && f > 6)) return static_cast<uint8_t>(sign | 0x7E);
  return static_cast<uint8_t>(sign | ((E + 7) << 3) | f);
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

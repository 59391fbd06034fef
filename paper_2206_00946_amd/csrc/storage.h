// Storage formats of the populations: FP64 (computed in double), FP32, FP16
// and BF16 (all three computed in float).  Narrow formats round to nearest,
// ties to even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

struct bf16 {
  uint16_t bits;
};

template <typename S>
struct Storage;

template <>
struct Storage<double> {
  using C = double;
  static __device__ __forceinline__ double load(const double* p) { return *p; }
  static __device__ __forceinline__ void store(double* p, double v) { *p = v; }
};

template <>
struct Storage<float> {
  using C = float;
  static __device__ __forceinline__ float load(const float* p) { return *p; }
  static __device__ __forceinline__ void store(float* p, float v) { *p = v; }
};

template <>
struct Storage<_Float16> {
  using C = float;
  static __device__ __forceinline__ float load(const _Float16* p) { return static_cast<float>(*p); }
  static __device__ __forceinline__ void store(_Float16* p, float v) { *p = static_cast<_Float16>(v); }
};

template <>
struct Storage<bf16> {
  using C = float;
  static __device__ __forceinline__ float load(const bf16* p) {
    return __uint_as_float(static_cast<uint32_t>(p->bits) << 16);
  }
  static __device__ __forceinline__ void store(bf16* p, float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
      p->bits = static_cast<uint16_t>((u >> 16) | 0x40u);  // keep NaN a NaN
      return;
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    p->bits = static_cast<uint16_t>(u >> 16);
  }
};

}  // namespace lbm

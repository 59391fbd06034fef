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
  // the hardware conversion (v_cvt_pk_bf16_f32: round to nearest even, NaN
  // stays NaN)
  static __device__ __forceinline__ void store(bf16* p, float v) {
    p->bits = __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
  }
};

// Raw buffer access: a descriptor over one uniform range (base, bytes) and a
// per-lane byte offset.  Offsets outside the range read 0 and drop stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_range(const void* base, unsigned bytes) {
  // word 3 of the descriptor for gfx9-family untyped 32-bit-format access
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename S>
struct Buf;

// voff: per-lane byte offset; soff: uniform byte offset (scalar operand)
template <>
struct Buf<double> {
  static __device__ __forceinline__ double load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  template <int CP = 0>
  static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, CP);
  }
};

template <>
struct Buf<float> {
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  template <int CP = 0>
  static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, CP);
  }
};

template <>
struct Buf<_Float16> {
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return static_cast<float>(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
  }
  template <int CP = 0>
  static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, static_cast<_Float16>(v)), r, voff,
                                          soff, CP);
  }
};

template <>
struct Buf<bf16> {
  static __device__ __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    bf16 h;
    h.bits = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    return Storage<bf16>::load(&h);
  }
  template <int CP = 0>
  static __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    bf16 h;
    Storage<bf16>::store(&h, v);
    __builtin_amdgcn_raw_buffer_store_b16(h.bits, r, voff, soff, CP);
  }
};

}  // namespace lbm

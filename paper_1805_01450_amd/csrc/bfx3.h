// BF16x3 scalar for the split-product precision form.
//
// A value is stored as an FP32 number.  A product x * y is formed the way a
// bf16 matrix unit with FP32 accumulation would form it from split operands:
// x = xh + xl with xh = bf16(x) and xl = bf16(x - xh) (round to nearest
// even), and likewise y; then x * y ~ xh*yh + (xh*yl + xl*yh) in FP32 (each
// bf16 x bf16 product is exact in FP32; the xl*yl term is dropped).  Sums and
// differences are plain FP32.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qgm {

__device__ __forceinline__ float bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

struct bfx3 {
  float v;
  __host__ __device__ bfx3() : v(0.0f) {}
  __host__ __device__ bfx3(float x) : v(x) {}
  __host__ __device__ bfx3(double x) : v((float)x) {}
  __host__ __device__ bfx3(int x) : v((float)x) {}
  __host__ __device__ explicit operator double() const { return (double)v; }
  __host__ __device__ bfx3& operator+=(bfx3 o) {
    v += o.v;
    return *this;
  }
};

__device__ __forceinline__ bfx3 operator+(bfx3 a, bfx3 b) { return bfx3(a.v + b.v); }
__device__ __forceinline__ bfx3 operator-(bfx3 a, bfx3 b) { return bfx3(a.v - b.v); }
__device__ __forceinline__ bfx3 operator*(bfx3 a, bfx3 b) {
  const float ah = bf16_rne(a.v), al = bf16_rne(a.v - ah);
  const float bh = bf16_rne(b.v), bl = bf16_rne(b.v - bh);
  return bfx3(ah * bh + (ah * bl + al * bh));
}

}  // namespace qgm

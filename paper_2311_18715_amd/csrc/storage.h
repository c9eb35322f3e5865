// Storage types of the stored basis columns and their conversions.
//
// double and float hold the columns directly; bf16 holds the upper 16 bits of
// an IEEE float (8-bit significand), rounded to nearest even on store (via
// FP32).  Residuals, projections and the matrix-core refold work in double
// (every stored value converts to double exactly).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace odmd {

struct bf16 {
  uint16_t bits;
};

template <typename TS> struct Storage;

typedef const __attribute__((address_space(1))) char* gbytes;   // global-memory byte address

__device__ inline uint64_t gload8(gbytes p) { return *(const __attribute__((address_space(1))) uint64_t*)p; }

// Rows per lane: a lane reads RPL consecutive rows of a column with one
// load, rows(p) (8 bytes for FP64 and FP32, so 16 lanes read a whole
// 128-byte line; 4 bytes for BF16, whose four-row loads kept too many rows
// live), or a single row with row(p), packed in a 64-bit value; elem(v, j)
// is row j of it.
template <> struct Storage<double> {
  static constexpr int RPL = 1;
  __device__ static uint64_t rows(gbytes p) { return gload8(p); }
  __device__ static uint64_t row(gbytes p) { return gload8(p); }
  __device__ static double elem(uint64_t v, int) { return __builtin_bit_cast(double, v); }
  __device__ static double gload(gbytes p) { return *(const __attribute__((address_space(1))) double*)p; }
  __device__ static double to_double(double v) { return v; }
  __device__ static double from_double(double v) { return v; }
};

template <> struct Storage<float> {
  static constexpr int RPL = 2;
  __device__ static uint64_t rows(gbytes p) { return gload8(p); }
  __device__ static uint64_t row(gbytes p) { return *(const __attribute__((address_space(1))) uint32_t*)p; }
  __device__ static float elem(uint64_t v, int j) { return __uint_as_float((uint32_t)(v >> (32 * j))); }
  __device__ static float gload(gbytes p) { return *(const __attribute__((address_space(1))) float*)p; }
  __device__ static double to_double(float v) { return (double)v; }
  __device__ static float from_double(double v) { return (float)v; }
};

template <> struct Storage<bf16> {
  static constexpr int RPL = 2;
  __device__ static uint64_t rows(gbytes p) { return *(const __attribute__((address_space(1))) uint32_t*)p; }
  __device__ static uint64_t row(gbytes p) { return *(const __attribute__((address_space(1))) uint16_t*)p; }
  __device__ static bf16 elem(uint64_t v, int j) { return bf16{(uint16_t)(v >> (16 * j))}; }
  __device__ static bf16 gload(gbytes p) {
    return bf16{*(const __attribute__((address_space(1))) uint16_t*)p};
  }
  __device__ static float to_float(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }
  __device__ static double to_double(bf16 v) { return (double)to_float(v); }
  // round to nearest even through FP32
  __device__ static bf16 from_float(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))   // NaN: keep it a NaN
      return bf16{(uint16_t)((u >> 16) | 0x0040u)};
    const uint32_t rounded = u + 0x7FFFu + ((u >> 16) & 1u);       // nearest, ties to even
    return bf16{(uint16_t)(rounded >> 16)};
  }
  __device__ static bf16 from_double(double v) { return from_float((float)v); }
};

}  // namespace odmd

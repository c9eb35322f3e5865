// Cross-lane FP64 reductions on the DPP network and the permlane swaps
// (CDNA4, wave64).  Every lane of a reduced group ends with the same value:
// each step adds the same two partial sums, in either order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace odmd {

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// sum over each 16-lane row: quad swaps, then the half-row and row mirrors
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_move<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141>(v);   // row_half_mirror
  v += dpp_move<0x140>(v);   // row_mirror
  return v;
}

__device__ __forceinline__ double row_prod(double v) {
  v *= dpp_move<0xB1>(v);
  v *= dpp_move<0x4E>(v);
  v *= dpp_move<0x141>(v);
  v *= dpp_move<0x140>(v);
  return v;
}

// v + the value of the same lane position in the neighbouring 16-lane row
// (rows 0 <-> 1, 2 <-> 3): the swap leaves own and partner value in its two
// outputs
__device__ __forceinline__ double add_row_pair(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  return __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32)) +
         __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}

// v + the value of the same lane position in the other 32-lane half
__device__ __forceinline__ double add_half_pair(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  return __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32)) +
         __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}

// sum over each 32-lane half
__device__ __forceinline__ double halfwave_sum(double v) { return add_row_pair(row_sum(v)); }

}  // namespace odmd

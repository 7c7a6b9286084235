// Wavefront-level helpers of the register-resident kernels: neighbour
// exchange across the 64 lanes by DPP, lane selection against a ballot mask,
// buffer resources with scalar row offsets, and wavefront sums.
#pragma once

#include <hip/hip_runtime.h>

namespace dz {

// lane i <- lane i - 1 (column x - 1); lane 0 receives 0 (bound_ctrl)
__device__ __forceinline__ float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
// lane i <- lane i + 1 (column x + 1); lane 63 receives 0 (bound_ctrl)
__device__ __forceinline__ float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

// Buffer resource of one plane: the row offset then travels in a scalar
// register and the lane's column offset is fixed, so no per-load address
// arithmetic is left in the vector ALU.  Word 3 is the gfx9-family default
// (32-bit dwords, no swizzle).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, static_cast<int>(bytes), 0x00020000);
}

// out where the lane's bit of `live` is set, else 0 (one v_cndmask).  The
// mask is uniform by construction; readfirstlane states that to the compiler,
// which must hold it in scalar registers for the instruction.
__device__ __forceinline__ float keep_lanes(float out, unsigned long long live) {
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(live));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(live >> 32));
  const unsigned long long m = (static_cast<unsigned long long>(hi) << 32) | lo;
  float r;
  asm volatile("v_cndmask_b32 %0, 0, %1, %2" : "=v"(r) : "v"(out), "s"(m));
  return r;
}

// Sum of a double over the 64 lanes; valid in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace dz

// Device helpers shared by the gfx950 kernels: element loads, wave-level
// reductions, and the register-tiled A^T B accumulation used for scatter
// and Gram matrices.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace cvx {

enum { DT_U16 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3, DT_U8 = 4 };


// Element storage types.
template <int DT> struct Elem;
template <> struct Elem<DT_U16>  { using T = uint16_t; };
template <> struct Elem<DT_F32>  { using T = float; };
template <> struct Elem<DT_BF16> { using T = uint16_t; };
template <> struct Elem<DT_F16>  { using T = uint16_t; };

template <int DT>
__device__ __forceinline__ float to_float(typename Elem<DT>::T v) {
  if constexpr (DT == DT_U16) {
    return (float)v;
  } else if constexpr (DT == DT_F32) {
    return v;
  } else if constexpr (DT == DT_BF16) {
    return __uint_as_float(((uint32_t)v) << 16);
  } else {
    _Float16 h = __builtin_bit_cast(_Float16, v);
    return (float)h;
  }
}

// Convert the low or high 16-bit half of a packed dword.
template <int DT>
__device__ __forceinline__ float half_lo(uint32_t d) { return to_float<DT>((uint16_t)(d & 0xffffu)); }
template <int DT>
__device__ __forceinline__ float half_hi(uint32_t d) { return to_float<DT>((uint16_t)(d >> 16)); }

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Synchronise the lanes of one wave on LDS written by other lanes of the
// same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Upper-triangular (bi <= bj) enumeration of 4x4 tiles of an nb x nb tile
// grid; returns false for blk >= nb (nb + 1) / 2.
__device__ __forceinline__ bool tri_tile(int blk, int nb, int& bi, int& bj) {
  int r = 0;
  int rem = blk;
  while (r < nb && rem >= nb - r) {
    rem -= nb - r;
    ++r;
  }
  if (r >= nb) return false;
  bi = r;
  bj = r + rem;
  return true;
}

// acc[4 i + j] += sum over rows r of A[r][4 bi + i] * Bm[r][4 bj + j].
// A and Bm are LDS row-major with leading dimensions that are multiples of 4.
__device__ __forceinline__ void tile_acc(const float* __restrict__ A, int lda,
                                         const float* __restrict__ Bm, int ldb,
                                         int bi, int bj, int r0, int r1, int rs,
                                         float acc[16]) {
  for (int r = r0; r < r1; r += rs) {
    const float4 a = *reinterpret_cast<const float4*>(A + r * lda + 4 * bi);
    const float4 b = *reinterpret_cast<const float4*>(Bm + r * ldb + 4 * bj);
    acc[0] = fmaf(a.x, b.x, acc[0]);   acc[1] = fmaf(a.x, b.y, acc[1]);
    acc[2] = fmaf(a.x, b.z, acc[2]);   acc[3] = fmaf(a.x, b.w, acc[3]);
    acc[4] = fmaf(a.y, b.x, acc[4]);   acc[5] = fmaf(a.y, b.y, acc[5]);
    acc[6] = fmaf(a.y, b.z, acc[6]);   acc[7] = fmaf(a.y, b.w, acc[7]);
    acc[8] = fmaf(a.z, b.x, acc[8]);   acc[9] = fmaf(a.z, b.y, acc[9]);
    acc[10] = fmaf(a.z, b.z, acc[10]); acc[11] = fmaf(a.z, b.w, acc[11]);
    acc[12] = fmaf(a.w, b.x, acc[12]); acc[13] = fmaf(a.w, b.y, acc[13]);
    acc[14] = fmaf(a.w, b.z, acc[14]); acc[15] = fmaf(a.w, b.w, acc[15]);
  }
}

// The linear stretch of [lo, hi] onto 0..levels as an affine map,
// q = floor(y s + o) clamped, with s = levels / (hi - lo) and
// o = 1/2 - lo s (a constant image maps to 0).  Every stretch in the
// library takes its map from here, so equal ranges give identical images.
__device__ __forceinline__ void stretch_map(float lo, float hi, float levels, float& s, float& o) {
  s = hi > lo ? levels / (hi - lo) : 0.f;
  o = fmaf(-lo, s, 0.5f);
}

// Ordered float <-> uint mapping so that unsigned integer min/max equals
// float min/max (for atomics-free reductions this is only used for keys).
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

}  // namespace cvx

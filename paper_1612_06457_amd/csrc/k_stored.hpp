// The fp16 intermediate of the one-read projection schedule, shared by the
// uint16 (matrix-core) and the other (vector-ALU) projection passes.
//
// Pass 1 finds each component's page range [a, b] and also stores every
// value y as h = fp16(y f) with f a power of two (planes of Pp values, Pp a
// multiple of 256).  Its last block derives the map of the stored values,
// q = floor(h s' + o) with s' = s / f exactly (q = floor(y s + o) is the
// map of the values themselves), and a bound on how far the stored values
// move the argument of the floor: rounding to fp16 moves y by at most
// 2^-11 |y| (2^-25 / f below fp16's normal range), and the map's FP32
// evaluation by a few units in its last place, so the move is at most
// s (M (2^-11 + 2^-22) + 2^-25 / f) + 2^-22 (s M + 1) with M = max(|a|, |b|).
// When that exceeds `limit` for a component, or a stored value could have
// overflowed, pass 2 re-reads the page (a flag uniform over the grid).
// Slots of range_dev: [16 + j] s', [24 + j] o, [32] the flag (as an
// unsigned), [40 + j] the bound.
#pragma once
#include "k_tile.hpp"

namespace cvx {

// The map of component j's stored values and its bound; returns true when
// pass 2 must re-read the page for it.  s, o: the map of the values.
__device__ __forceinline__ bool stored_map(float lo, float hi, float s, float o, float f, float limit, int j,
                                           float* __restrict__ range_dev) {
  range_dev[16 + j] = s / f;   // f a power of two: exact
  range_dev[24 + j] = o;
  const float M = fmaxf(fabsf(lo), fabsf(hi));
  float bound = 0.f;
  bool bad = !(M * f <= 32768.f);   // stored values stay far below fp16's largest, 65504
  if (hi > lo) {
    bound = s * (M * (0x1p-11f + 0x1p-22f) + 0x1p-25f / f) + 0x1p-22f * (s * M + 1.f);
    bad = bad || !(bound <= limit);
  }
  range_dev[40 + j] = bound;
  return bad;
}

__device__ __forceinline__ uint32_t quant_stored(float y, float s, float o) {
  float t = floorf(fmaf(y, s, o));
  t = fminf(fmaxf(t, 0.f), 255.f);
  return (uint32_t)t;
}

// Quantises the 16 stored values of one chunk (two 16-byte words) with the
// map of the stored values and writes them at pixel px of the plane dst
// (one 16-byte store when the plane rows allow, else byte by byte up to P).
__device__ __forceinline__ void quant_chunk(const u32x4& v0, const u32x4& v1, float s, float o, int64_t px,
                                            int64_t P, bool aligned, uint8_t* __restrict__ dst) {
  if (px >= P) return;
  // value 2 m + h of the chunk is half h of word m
  const uint32_t wd[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
  uint32_t qb[16];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    qb[2 * m] = quant_stored((float)__builtin_bit_cast(_Float16, (uint16_t)(wd[m] & 0xffffu)), s, o);
    qb[2 * m + 1] = quant_stored((float)__builtin_bit_cast(_Float16, (uint16_t)(wd[m] >> 16)), s, o);
  }
  u32x4 q;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    q[d] = qb[4 * d] | (qb[4 * d + 1] << 8) | (qb[4 * d + 2] << 16) | (qb[4 * d + 3] << 24);
  if (aligned && px + 16 <= P) {
    *reinterpret_cast<u32x4*>(dst + px) = q;
  } else {
    for (int e = 0; e < 16; ++e)
      if (px + e < P) dst[px + e] = (uint8_t)(q[e >> 2] >> (8 * (e & 3)));
  }
}

// Pass 2 from the stored fp16 planes: 16 values per lane and step, two
// steps' loads in flight (the second index clamped to the plane's last
// chunk, so no branch separates the loads).
__device__ __forceinline__ void stretch_stored(const _Float16* __restrict__ planes, int64_t Pp, int64_t P, int nc,
                                               const float* __restrict__ range_dev, uint8_t* __restrict__ images) {
  const int64_t cpp = Pp / 16;   // chunks per plane
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool aligned = (P % 16) == 0 && (reinterpret_cast<uintptr_t>(images) % 16) == 0;
  for (int j = 0; j < nc; ++j) {
    const float s = range_dev[16 + j], o = range_dev[24 + j];
    const u32x4* src = reinterpret_cast<const u32x4*>(planes + (int64_t)j * Pp);
    uint8_t* dst = images + (int64_t)j * P;
    for (int64_t i = t0; i < cpp; i += 2 * stride) {
      const int64_t i1 = i + stride < cpp ? i + stride : cpp - 1;
      const u32x4 a0 = __builtin_nontemporal_load(src + 2 * i);
      const u32x4 a1 = __builtin_nontemporal_load(src + 2 * i + 1);
      const u32x4 b0 = __builtin_nontemporal_load(src + 2 * i1);
      const u32x4 b1 = __builtin_nontemporal_load(src + 2 * i1 + 1);
      quant_chunk(a0, a1, s, o, 16 * i, P, aligned, dst);
      if (i + stride < cpp) quant_chunk(b0, b1, s, o, 16 * i1, P, aligned, dst);
    }
  }
}

}  // namespace cvx

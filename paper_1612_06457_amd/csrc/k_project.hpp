// Fused centre-project-stretch over every pixel of the page (paper
// Section 2: the regression coefficients multiply all bands of the whole
// page, and each float image is rescaled to 0..255 on its page-wide range).
//
// Both passes stream the band-interleaved cube once.  Each wave owns a tile
// of 64 "lane groups"; a lane group is the smallest run of whole pixels
// that is a whole number of dwords (two pixels for 16-bit elements and an
// odd band count, else one pixel), so a tile is 256 * S bytes with S the
// dwords per lane group.  The tile is fetched with coalesced 16-byte loads
// (all of a lane's loads issued back to back), stored into the wave's LDS
// slice, and each lane then reads its own S dwords; with S odd those reads
// hit distinct LDS banks.  Latency is covered by the other resident waves.
// y_j = sum_b W[b][j] (x_b - c_b) + off_j is accumulated in FP32 on the
// VALU (a streaming, HBM-bound pass with about 6 flop per byte: no matrix
// cores).  Pass 1 keeps running min/max per component; the last block to
// finish combines the block partials (all its threads, fixed assignment)
// and stores the affine map of the stretch, q = floor(y s + o) with
// s = 255 / (b - a), o = 1/2 - a s.  Pass 2 recomputes y bit for bit,
// quantises, clamps to 0..255 and writes planar bytes.
//
// BC > 0 instantiates the kernels for a fixed band count (fully unrolled
// band loops, exact chunk counts); BC = 0 takes the band count at run time.
// uint16 elements are converted with the exact float trick
// f = as_float(0x4b000000 | x) = 2^23 + x, and the per-band constant
// 2^23 + c_b (c_b an integer) is subtracted: one OR and one subtraction.
#pragma once
#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {
namespace proj {

constexpr int kMaxQ = 16;   // 16-byte chunks per lane per tile: 16 * S / 64 <= 16 for S <= 64

template <int DT>
struct Geo {
  static constexpr int esize = (DT == DT_F32) ? 4 : 2;
  static __device__ __host__ constexpr int g2(int B) { return (esize == 2 && (B & 1)) ? 2 : 1; }
  static __device__ __host__ constexpr int S(int B) { return (esize == 4 || (B & 1)) ? B : B / 2; }
};

// Element value minus the band centre.  For uint16 pages a.c holds
// 2^23 + c_b (exact) and the element is turned into 2^23 + x bit-wise.
template <int DT>
__device__ __forceinline__ float centred_lo(uint32_t d, float cb) {
  if constexpr (DT == DT_U16) {
    return __uint_as_float((d & 0xffffu) | 0x4b000000u) - cb;
  } else {
    return half_lo<DT>(d) - cb;
  }
}
template <int DT>
__device__ __forceinline__ float centred_hi(uint32_t d, float cb) {
  if constexpr (DT == DT_U16) {
    return __uint_as_float((d >> 16) | 0x4b000000u) - cb;
  } else {
    return half_hi<DT>(d) - cb;
  }
}

template <int NC>
__device__ __forceinline__ void accum(float (&acc)[NC], const ProjArgs& a, int b, float x) {
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = fmaf(a.w[b * NC + j], x, acc[j]);
}

// Issue the loads of wave tile t into registers (chunk j = lane + 64 q).
template <int BC, int DT>
__device__ __forceinline__ void load_tile(const unsigned char* __restrict__ base, int64_t total_bytes,
                                          int64_t t, int S, int lane, uint4 (&r)[kMaxQ]) {
  constexpr int SC = BC > 0 ? Geo<DT>::S(BC) : 0;
  const int Sx = BC > 0 ? SC : S;
  const int64_t tb = t * 256 * (int64_t)Sx;
  const int nchunk = 16 * Sx;
  const bool full = tb + 16 * (int64_t)nchunk <= total_bytes;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (64 * q < nchunk) {
      const int j = lane + 64 * q;
      if (j < nchunk) {
        const int64_t ob = tb + 16 * (int64_t)j;
        if (full || ob + 16 <= total_bytes) {
          r[q] = *reinterpret_cast<const uint4*>(base + ob);
        } else {
          uint16_t h[8];
#pragma unroll
          for (int e = 0; e < 8; ++e)
            h[e] = (ob + 2 * e + 2 <= total_bytes) ? *reinterpret_cast<const uint16_t*>(base + ob + 2 * e) : 0;
          r[q].x = h[0] | ((uint32_t)h[1] << 16);
          r[q].y = h[2] | ((uint32_t)h[3] << 16);
          r[q].z = h[4] | ((uint32_t)h[5] << 16);
          r[q].w = h[6] | ((uint32_t)h[7] << 16);
        }
      }
    }
  }
}

template <int BC, int DT>
__device__ __forceinline__ void store_tile(uint32_t* __restrict__ my, int S, int lane,
                                           const uint4 (&r)[kMaxQ]) {
  constexpr int SC = BC > 0 ? Geo<DT>::S(BC) : 0;
  const int nchunk = 16 * (BC > 0 ? SC : S);
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (64 * q < nchunk) {
      const int j = lane + 64 * q;
      if (j < nchunk) *reinterpret_cast<uint4*>(my + 4 * j) = r[q];
    }
  }
}

// y for the lane group at LDS dwords d[0..S): acc0 gets pixel 0, acc1 pixel 1.
template <int DT, int NC, int BC>
__device__ __forceinline__ void project_group(const uint32_t* __restrict__ d, int Brt,
                                              const ProjArgs& a, float (&acc0)[NC],
                                              float (&acc1)[NC]) {
  const int B = BC > 0 ? BC : Brt;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    acc0[j] = a.off[j];
    acc1[j] = a.off[j];
  }
  if constexpr (DT == DT_F32) {
#pragma unroll (BC > 0 ? 64 : 1)
    for (int b = 0; b < B; ++b) accum<NC>(acc0, a, b, __uint_as_float(d[b]) - a.c[b]);
  } else {
    if (!(B & 1)) {
#pragma unroll (BC > 0 ? 64 : 1)
      for (int q = 0; q < B / 2; ++q) {
        const uint32_t v = d[q];
        accum<NC>(acc0, a, 2 * q, centred_lo<DT>(v, a.c[2 * q]));
        accum<NC>(acc0, a, 2 * q + 1, centred_hi<DT>(v, a.c[2 * q + 1]));
      }
    } else {
      const int h = (B - 1) / 2;
#pragma unroll (BC > 0 ? 64 : 1)
      for (int q = 0; q < h; ++q) {
        const uint32_t v = d[q];
        accum<NC>(acc0, a, 2 * q, centred_lo<DT>(v, a.c[2 * q]));
        accum<NC>(acc0, a, 2 * q + 1, centred_hi<DT>(v, a.c[2 * q + 1]));
      }
      {
        const uint32_t v = d[h];
        accum<NC>(acc0, a, B - 1, centred_lo<DT>(v, a.c[B - 1]));
        accum<NC>(acc1, a, 0, centred_hi<DT>(v, a.c[0]));
      }
#pragma unroll (BC > 0 ? 64 : 1)
      for (int q = h + 1; q < B; ++q) {
        const uint32_t v = d[q];
        accum<NC>(acc1, a, 2 * q - B, centred_lo<DT>(v, a.c[2 * q - B]));
        accum<NC>(acc1, a, 2 * q + 1 - B, centred_hi<DT>(v, a.c[2 * q + 1 - B]));
      }
    }
  }
}

// Fixed band count: one pass over the bands reads the lane group's
// elements, W[b][0..NC) and c_b from LDS (W and c as broadcast loads, so
// they never occupy scalar registers) and updates both pixels.
template <int DT, int NC, int BC>
__device__ __forceinline__ void project_group_fixed(const uint32_t* __restrict__ d,
                                                    const float* __restrict__ wl,
                                                    const float* __restrict__ cl,
                                                    const float* __restrict__ ol, int z,
                                                    float (&acc0)[NC], float (&acc1)[NC]) {
  // z is zero, but opaque to the compiler: it keeps the W reads inside the
  // tile loop instead of hoisting all B x NC weights into registers
  wl += z;
  cl += z;
  ol += z;
  constexpr int G2 = Geo<DT>::g2(BC);
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    acc0[j] = ol[j];
    acc1[j] = ol[j];
  }
  // one pass over the bands per pixel of the lane group: each pass keeps
  // only a few bands of weights live
#pragma unroll
  for (int px = 0; px < G2; ++px) {
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const float4 w0 = *reinterpret_cast<const float4*>(wl + 8 * b);
      const float4 w1 = *reinterpret_cast<const float4*>(wl + 8 * b + 4);
      const float wv[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
      const float cb = cl[b];
      float x;
      if constexpr (DT == DT_F32) {
        x = __uint_as_float(d[b]) - cb;
      } else {
        const int e = px * BC + b;
        x = (e & 1) ? centred_hi<DT>(d[e >> 1], cb) : centred_lo<DT>(d[e >> 1], cb);
      }
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        if (px == 0) acc0[j] = fmaf(wv[j], x, acc0[j]);
        else acc1[j] = fmaf(wv[j], x, acc1[j]);
      }
      if ((b & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The tile loop shared by both passes: body(pix, g2, y0, y1) per lane group.
template <int DT, int NC, int BC, typename Body>
__device__ __forceinline__ void tile_loop(const void* __restrict__ cube, int Brt, int64_t P,
                                          const ProjArgs& a, uint32_t* __restrict__ lds, Body body) {
  const int B = BC > 0 ? BC : Brt;
  const int S = Geo<DT>::S(B), g2 = Geo<DT>::g2(B);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* my = lds + w * 64 * S;
  const int64_t tp = 64 * (int64_t)g2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * Geo<DT>::esize;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  // W (padded to 8 per band), the band centres and the offsets in LDS
  __shared__ __align__(16) float wl[kMaxB * 8];
  __shared__ float cl[kMaxB];
  __shared__ float ol[8];
  if constexpr (BC > 0) {
    for (int i = threadIdx.x; i < BC * 8; i += kBlock) {
      const int b = i >> 3, j = i & 7;
      wl[i] = (j < NC) ? a.w[b * NC + j] : 0.f;
    }
    for (int i = threadIdx.x; i < BC; i += kBlock) cl[i] = a.c[i];
    if (threadIdx.x < 8) ol[threadIdx.x] = (threadIdx.x < NC) ? a.off[threadIdx.x] : 0.f;
    __syncthreads();
  }
  for (int64_t t = (int64_t)blockIdx.x * kWaves + w; t < nt; t += stride) {
    {
      uint4 r[kMaxQ];
      load_tile<BC, DT>(base, total_bytes, t, S, lane, r);
      store_tile<BC, DT>(my, S, lane, r);
    }
    wave_lds_sync();
    float y0[NC], y1[NC];
    if constexpr (BC > 0) {
      int z = 0;
      asm volatile("" : "+v"(z));
      project_group_fixed<DT, NC, BC>(my + lane * S, wl, cl, ol, z, y0, y1);
    } else {
      project_group<DT, NC, BC>(my + lane * S, B, a, y0, y1);
    }
    body(t * tp + (int64_t)lane * g2, g2, y0, y1);
    wave_lds_sync();
  }
}

template <int DT, int NC, int BC>
__global__ __launch_bounds__(kBlock) void k_project_range(const void* __restrict__ cube, int B,
                                                          int64_t P, ProjArgs a,
                                                          float* __restrict__ part,
                                                          unsigned* __restrict__ ticket,
                                                          float* __restrict__ range_dev,
                                                          float* __restrict__ ab_dev) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float wred[kWaves][2 * NC];
  __shared__ bool am_last;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float mn[NC], mx[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    mn[j] = __builtin_inff();
    mx[j] = -__builtin_inff();
  }
  tile_loop<DT, NC, BC>(cube, B, P, a, lds, [&](int64_t pix, int g2, const float (&y0)[NC], const float (&y1)[NC]) {
    if (pix < P) {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        mn[j] = fminf(mn[j], y0[j]);
        mx[j] = fmaxf(mx[j], y0[j]);
      }
    }
    if (g2 == 2 && pix + 1 < P) {
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        mn[j] = fminf(mn[j], y1[j]);
        mx[j] = fmaxf(mx[j], y1[j]);
      }
    }
  });
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    mn[j] = wave_min(mn[j]);
    mx[j] = wave_max(mx[j]);
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      wred[w][j] = mn[j];
      wred[w][NC + j] = mx[j];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < NC; ++j) {
      float lo = wred[0][j], hi = wred[0][NC + j];
      for (int ww = 1; ww < kWaves; ++ww) {
        lo = fminf(lo, wred[ww][j]);
        hi = fmaxf(hi, wred[ww][NC + j]);
      }
      part[(int64_t)blockIdx.x * 2 * NC + j] = lo;
      part[(int64_t)blockIdx.x * 2 * NC + NC + j] = hi;
    }
    __threadfence();
    const unsigned prev = atomicAdd(ticket, 1u);
    am_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return;
  // last block: every thread folds a strided subset of the block partials
  __threadfence();
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    mn[j] = __builtin_inff();
    mx[j] = -__builtin_inff();
  }
  for (unsigned bk = threadIdx.x; bk < gridDim.x; bk += kBlock) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      mn[j] = fminf(mn[j], __builtin_nontemporal_load(part + (int64_t)bk * 2 * NC + j));
      mx[j] = fmaxf(mx[j], __builtin_nontemporal_load(part + (int64_t)bk * 2 * NC + NC + j));
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    mn[j] = wave_min(mn[j]);
    mx[j] = wave_max(mx[j]);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      wred[w][j] = mn[j];
      wred[w][NC + j] = mx[j];
    }
  }
  __syncthreads();
  if (threadIdx.x < NC) {
    const int j = threadIdx.x;
    float lo = wred[0][j], hi = wred[0][NC + j];
    for (int ww = 1; ww < kWaves; ++ww) {
      lo = fminf(lo, wred[ww][j]);
      hi = fmaxf(hi, wred[ww][NC + j]);
    }
    const float s = (hi > lo) ? 255.f / (hi - lo) : 0.f;
    range_dev[j] = s;
    range_dev[8 + j] = 0.5f - lo * s;
    ab_dev[2 * j] = lo;
    ab_dev[2 * j + 1] = hi;
  }
  if (threadIdx.x == 0) *ticket = 0u;
}

__device__ __forceinline__ uint32_t quant(float y, float s, float o) {
  float t = floorf(fmaf(y, s, o));
  t = fminf(fmaxf(t, 0.f), 255.f);
  return (uint32_t)t;
}

template <int DT, int NC, int BC>
__global__ __launch_bounds__(kBlock) void k_project_stretch(const void* __restrict__ cube, int B,
                                                            int64_t P, ProjArgs a,
                                                            const float* __restrict__ range_dev,
                                                            uint8_t* __restrict__ images) {
  extern __shared__ __align__(16) uint32_t lds[];
  float sc[NC], of[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    sc[j] = range_dev[j];
    of[j] = range_dev[8 + j];
  }
  const bool even = (P & 1) == 0;
  tile_loop<DT, NC, BC>(cube, B, P, a, lds, [&](int64_t pix, int g2, const float (&y0)[NC], const float (&y1)[NC]) {
    if (g2 == 2) {
      if (pix + 1 < P && even) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const uint32_t q = quant(y0[j], sc[j], of[j]) | (quant(y1[j], sc[j], of[j]) << 8);
          *reinterpret_cast<uint16_t*>(images + (int64_t)j * P + pix) = (uint16_t)q;
        }
      } else if (pix + 1 < P) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          images[(int64_t)j * P + pix] = (uint8_t)quant(y0[j], sc[j], of[j]);
          images[(int64_t)j * P + pix + 1] = (uint8_t)quant(y1[j], sc[j], of[j]);
        }
      } else if (pix < P) {
#pragma unroll
        for (int j = 0; j < NC; ++j) images[(int64_t)j * P + pix] = (uint8_t)quant(y0[j], sc[j], of[j]);
      }
    } else if (pix < P) {
#pragma unroll
      for (int j = 0; j < NC; ++j) images[(int64_t)j * P + pix] = (uint8_t)quant(y0[j], sc[j], of[j]);
    }
  });
}

inline size_t smem_bytes(int dtype, int B) {
  const int S = (dtype == DT_F32 || (B & 1)) ? B : B / 2;
  return (size_t)kWaves * 64 * S * 4;
}

// Launch both passes' kernels for one (DT, BC) with the exact component count.
template <int DT, int BC>
hipError_t range_bc(int nc, const void* cube, int B, int64_t P, const ProjArgs& a, int nblocks, float* part,
                    unsigned* ticket, float* range_dev, float* ab_dev, hipStream_t s) {
  const size_t sm = smem_bytes(DT, B);
#define CVX_RANGE(N)                                                                                          \
  case N:                                                                                                     \
    hipLaunchKernelGGL((k_project_range<DT, N, BC>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, a, part, \
                       ticket, range_dev, ab_dev);                                                            \
    break;
  switch (nc) {
    CVX_RANGE(1) CVX_RANGE(2) CVX_RANGE(3) CVX_RANGE(4) CVX_RANGE(5) CVX_RANGE(6) CVX_RANGE(7) CVX_RANGE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef CVX_RANGE
  return hipGetLastError();
}

template <int DT, int BC>
hipError_t stretch_bc(int nc, const void* cube, int B, int64_t P, const ProjArgs& a, int nblocks,
                      const float* range_dev, uint8_t* images, hipStream_t s) {
  const size_t sm = smem_bytes(DT, B);
#define CVX_STRETCH(N)                                                                                        \
  case N:                                                                                                     \
    hipLaunchKernelGGL((k_project_stretch<DT, N, BC>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, a,     \
                       range_dev, images);                                                                    \
    break;
  switch (nc) {
    CVX_STRETCH(1) CVX_STRETCH(2) CVX_STRETCH(3) CVX_STRETCH(4) CVX_STRETCH(5) CVX_STRETCH(6) CVX_STRETCH(7)
    CVX_STRETCH(8)
    default:
      return hipErrorInvalidValue;
  }
#undef CVX_STRETCH
  return hipGetLastError();
}

}  // namespace proj

// Per-translation-unit entry points (one per group of instantiations).
hipError_t project_range_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                 int nblocks, float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                 hipStream_t s);
hipError_t project_stretch_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                   int nblocks, const float* range_dev, uint8_t* images, hipStream_t s);
}  // namespace cvx

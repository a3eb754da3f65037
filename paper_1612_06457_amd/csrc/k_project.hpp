// Fused centre-project-stretch over every pixel of the page on the VALU
// (paper Section 2: the regression coefficients multiply all bands of the
// whole page, and each float image is rescaled to 0..255 on its page-wide
// range).  Used for float32 pages; 16-bit pages take the matrix-core
// kernels.
//
// Both passes stream the band-interleaved cube in wave tiles (k_tile.hpp);
// the next tile's loads are issued before the current one is computed.
// Each lane reads its own S dwords from LDS (with S odd those reads hit
// distinct banks), and each band's centre and weights as broadcast LDS
// reads of a per-block table.  y_j = sum_b W[b][j] (x_b - c_b) + off_j is accumulated
// in FP32.  Pass 1 keeps running min/max per component; the last block to
// finish combines the block partials (all its threads, fixed assignment)
// and stores the affine map of the stretch, q = floor(y s + o) with
// s = 255 / (b - a), o = 1/2 - a s.  Pass 2 recomputes y bit for bit,
// quantises, clamps to 0..255 and writes planar bytes.
#pragma once
#include <algorithm>

#include "k_stored.hpp"
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {
namespace proj {

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

typedef float f4v __attribute__((ext_vector_type(4)));

// 16-byte band records per band: the centre c_b, then W[b][0..NC), zero
// padded.
template <int NC>
constexpr int band_f4() { return (NC + 4) / 4; }

// The band records, staged once per block from the kernel arguments: in the
// band loop each band's centre and weights are then broadcast 16-byte LDS
// reads (scalar loads of the arguments at a runtime band index serialised
// that loop on the scalar cache).
template <int NC>
__device__ __forceinline__ void stage_bands(const ProjArgs& a, int B, f4v* __restrict__ rec) {
  constexpr int F = 4 * band_f4<NC>();
  for (int i = threadIdx.x; i < B * F; i += kBlock) {
    const int b = i / F, k = i - b * F;
    reinterpret_cast<float*>(rec)[i] = k == 0 ? a.c[b] : (k <= NC ? a.w[b * NC + k - 1] : 0.f);
  }
  __syncthreads();
}

template <int NC>
__device__ __forceinline__ void band(const f4v* __restrict__ rec, int b, float& c, float (&wv)[NC]) {
  constexpr int R = band_f4<NC>();
  f4v r[R];
#pragma unroll
  for (int k = 0; k < R; ++k) r[k] = rec[b * R + k];
  c = r[0][0];
#pragma unroll
  for (int j = 0; j < NC; ++j) wv[j] = r[(j + 1) >> 2][(j + 1) & 3];
}

template <int NC>
__device__ __forceinline__ void fma_band(float (&acc)[NC], const float (&wv)[NC], float x) {
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = fmaf(wv[j], x, acc[j]);
}

// y for the lane group at LDS dwords d[0..S): acc0 gets pixel 0, acc1 pixel
// 1; each pixel's bands are added in ascending order.
template <int DT, int NC>
__device__ __forceinline__ void project_group(const uint32_t* __restrict__ d, int B, const f4v* __restrict__ rec,
                                              const ProjArgs& a, float (&acc0)[NC], float (&acc1)[NC]) {
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    acc0[j] = a.off[j];
    acc1[j] = a.off[j];
  }
  float c, wv[NC];
  if constexpr (DT == DT_F32) {
    for (int b = 0; b < B; ++b) {
      band<NC>(rec, b, c, wv);
      fma_band<NC>(acc0, wv, __uint_as_float(d[b]) - c);
    }
  } else {
    if (!(B & 1)) {
      for (int q = 0; q < B / 2; ++q) {
        const uint32_t v = d[q];
        band<NC>(rec, 2 * q, c, wv);
        fma_band<NC>(acc0, wv, centred_lo<DT>(v, c));
        band<NC>(rec, 2 * q + 1, c, wv);
        fma_band<NC>(acc0, wv, centred_hi<DT>(v, c));
      }
    } else {
      // two pixels of B (odd) bands in 2B halves: pixel 0's band b is half
      // b, pixel 1's is half B + b, so one band record serves both pixels
      const int h = (B - 1) / 2;
      uint32_t carry = d[h];   // high half: pixel 1, band 0
      for (int q = 0; q < h; ++q) {
        const uint32_t v = d[q], nxt = d[h + q + 1];
        band<NC>(rec, 2 * q, c, wv);
        fma_band<NC>(acc0, wv, centred_lo<DT>(v, c));
        fma_band<NC>(acc1, wv, centred_hi<DT>(carry, c));
        band<NC>(rec, 2 * q + 1, c, wv);
        fma_band<NC>(acc0, wv, centred_hi<DT>(v, c));
        fma_band<NC>(acc1, wv, centred_lo<DT>(nxt, c));
        carry = nxt;
      }
      band<NC>(rec, B - 1, c, wv);
      fma_band<NC>(acc0, wv, centred_lo<DT>(d[h], c));
      fma_band<NC>(acc1, wv, centred_hi<DT>(carry, c));
    }
  }
}

// The tile loop shared by both passes: body(pix, g2, y0, y1) per lane group.
// Q 16-byte loads per lane hold a tile of S <= 4 Q dwords per lane group
// (fewer registers for narrower pages leave room for more waves).
template <int DT, int NC, int Q, typename Body>
__device__ __forceinline__ void tile_loop(const void* __restrict__ cube, int B, int64_t P,
                                          const ProjArgs& a, uint32_t* __restrict__ lds, Body body) {
  const int S = Geo<DT>::S(B), g2 = Geo<DT>::g2(B);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* my = lds + w * 64 * S;
  const int64_t tp = 64 * (int64_t)g2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * Geo<DT>::esize;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  __shared__ f4v rec[kMaxB * band_f4<NC>()];
  stage_bands<NC>(a, B, rec);
  for_each_tile<Q>(base, total_bytes, nt, S, my, [&](int64_t t) {
    float y0[NC], y1[NC];
    project_group<DT, NC>(my + lane * S, B, rec, a, y0, y1);
    body(t * tp + (int64_t)lane * g2, g2, y0, y1);
  });
}

// Pass 1; with H16 it also stores every value as fp16 (k_stored.hpp): the
// lane's pixel (or pair of pixels, one dword) in each plane, so a wave
// writes 64 consecutive pixels per plane; the last tile's pixels beyond P
// land in the planes' padding (Pp >= P rounded up to whole tiles).
template <int DT, int NC, bool H16, int Q>
__global__ __launch_bounds__(kBlock) void k_project_range(const void* __restrict__ cube, int B,
                                                          int64_t P, ProjArgs a,
                                                          float* __restrict__ part,
                                                          unsigned* __restrict__ ticket,
                                                          float* __restrict__ range_dev,
                                                          float* __restrict__ ab_dev, H16Args h,
                                                          _Float16* __restrict__ planes, int64_t Pp) {
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
  tile_loop<DT, NC, Q>(cube, B, P, a, lds, [&](int64_t pix, int g2, const float (&y0)[NC], const float (&y1)[NC]) {
    if constexpr (H16) {
      if (g2 == 2) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const uint32_t v = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(y0[j] * h.f[j])) |
                             ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(y1[j] * h.f[j])) << 16);
          *reinterpret_cast<uint32_t*>(planes + (int64_t)j * Pp + pix) = v;
        }
      } else {
#pragma unroll
        for (int j = 0; j < NC; ++j)
          *reinterpret_cast<uint16_t*>(planes + (int64_t)j * Pp + pix) =
              __builtin_bit_cast(uint16_t, (_Float16)(y0[j] * h.f[j]));
      }
    }
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
    float s, o;
    stretch_map(lo, hi, 255.f, s, o);
    range_dev[j] = s;
    range_dev[8 + j] = o;
    ab_dev[2 * j] = lo;
    ab_dev[2 * j + 1] = hi;
    if constexpr (H16) wred[0][j] = stored_map(lo, hi, s, o, h.f[j], h.limit, j, range_dev) ? 1.f : 0.f;
  }
  if constexpr (H16) {
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned flag = 0u;
      for (int j = 0; j < NC; ++j) flag |= wred[0][j] != 0.f ? 1u : 0u;
      reinterpret_cast<unsigned*>(range_dev)[32] = flag;
    }
  }
  if (threadIdx.x == 0) *ticket = 0u;
}

__device__ __forceinline__ uint32_t quant(float y, float s, float o) {
  float t = floorf(fmaf(y, s, o));
  t = fminf(fmaxf(t, 0.f), 255.f);
  return (uint32_t)t;
}

// Pass 2 from the page.
template <int DT, int NC, int Q>
__device__ __forceinline__ void stretch_page_valu(const void* __restrict__ cube, int B, int64_t P, const ProjArgs& a,
                                                  const float* __restrict__ range_dev, uint8_t* __restrict__ images,
                                                  uint32_t* __restrict__ lds) {
  float sc[NC], of[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    sc[j] = range_dev[j];
    of[j] = range_dev[8 + j];
  }
  const bool even = (P & 1) == 0;
  tile_loop<DT, NC, Q>(cube, B, P, a, lds, [&](int64_t pix, int g2, const float (&y0)[NC], const float (&y1)[NC]) {
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

template <int DT, int NC, int Q>
__global__ __launch_bounds__(kBlock) void k_project_stretch(const void* __restrict__ cube, int B,
                                                            int64_t P, ProjArgs a,
                                                            const float* __restrict__ range_dev,
                                                            uint8_t* __restrict__ images) {
  extern __shared__ __align__(16) uint32_t lds[];
  stretch_page_valu<DT, NC, Q>(cube, B, P, a, range_dev, images, lds);
}

// Pass 2 after a pass 1 that stored fp16 planes: from the planes, or from
// the page when pass 1 set the flag.
template <int DT, int NC, int Q>
__global__ __launch_bounds__(kBlock) void k_project_stretch_h16(const void* __restrict__ cube, int B,
                                                                int64_t P, ProjArgs a,
                                                                const float* __restrict__ range_dev,
                                                                const _Float16* __restrict__ planes, int64_t Pp,
                                                                uint8_t* __restrict__ images) {
  extern __shared__ __align__(16) uint32_t lds[];
  if (reinterpret_cast<const unsigned*>(range_dev)[32] != 0u) {
    stretch_page_valu<DT, NC, Q>(cube, B, P, a, range_dev, images, lds);
    return;
  }
  stretch_stored(planes, Pp, P, NC, range_dev, images);
}

// The FP32 component planes themselves: y[j][p] for every pixel, the same
// values the two passes above compute (lanes write consecutive pixels).
template <int DT, int NC, int Q>
__global__ __launch_bounds__(kBlock) void k_project_float(const void* __restrict__ cube, int B, int64_t P,
                                                          ProjArgs a, float* __restrict__ y) {
  extern __shared__ __align__(16) uint32_t lds[];
  tile_loop<DT, NC, Q>(cube, B, P, a, lds, [&](int64_t pix, int g2, const float (&y0)[NC], const float (&y1)[NC]) {
    if (pix < P) {
#pragma unroll
      for (int j = 0; j < NC; ++j) y[(int64_t)j * P + pix] = y0[j];
    }
    if (g2 == 2 && pix + 1 < P) {
#pragma unroll
      for (int j = 0; j < NC; ++j) y[(int64_t)j * P + pix + 1] = y1[j];
    }
  });
}

// 16-byte loads per lane for a tile of S dwords per lane group
inline int q_for(int dtype, int B) {
  const int S = (dtype == DT_F32 || (B & 1)) ? B : B / 2;
  return S <= 32 ? 8 : kMaxQ;
}

inline size_t smem_bytes(int dtype, int B) {
  const int S = (dtype == DT_F32 || (B & 1)) ? B : B / 2;
  return (size_t)kWaves * 64 * S * 4;
}

// The grid of a persistent pass: at most the blocks that are resident at
// once (a second round of blocks would run its tiles after the first with
// the device half idle), and at most nblocks.
inline int resident_grid(const void* kernel, size_t sm, int nblocks) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, sm) != hipSuccess || per < 1)
    return nblocks;
  return std::max(1, std::min(nblocks, per * ncu));
}

#define CVX_LAUNCH(KERNEL, SM, NB, S, ...)                                                     \
  do {                                                                                         \
    const int nb_ = resident_grid(reinterpret_cast<const void*>(&KERNEL), SM, NB);             \
    hipLaunchKernelGGL(KERNEL, dim3(nb_), dim3(kBlock), SM, S, __VA_ARGS__);                    \
  } while (0)

// Launch a pass's kernel for one element type with the exact component count.
template <int DT, bool H16 = false>
hipError_t range_nc(int nc, const void* cube, int B, int64_t P, const ProjArgs& a, int nblocks, float* part,
                    unsigned* ticket, float* range_dev, float* ab_dev, hipStream_t s, const H16Args& h = H16Args{},
                    _Float16* planes = nullptr, int64_t Pp = 0) {
  const size_t sm = smem_bytes(DT, B);
  const int q = q_for(DT, B);
#define CVX_RANGE(N)                                                                                          \
  case N:                                                                                                     \
    if (q == 8)                                                                                               \
      CVX_LAUNCH((k_project_range<DT, N, H16, 8>), sm, nblocks, s, cube, B, P, a, \
                         part, ticket, range_dev, ab_dev, h, planes, Pp);                                    \
    else                                                                                                      \
      CVX_LAUNCH((k_project_range<DT, N, H16, kMaxQ>), sm, nblocks, s, cube, B, P, \
                         a, part, ticket, range_dev, ab_dev, h, planes, Pp);                                 \
    break;
  switch (nc) {
    CVX_RANGE(1) CVX_RANGE(2) CVX_RANGE(3) CVX_RANGE(4) CVX_RANGE(5) CVX_RANGE(6) CVX_RANGE(7) CVX_RANGE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef CVX_RANGE
  return hipGetLastError();
}

template <int DT>
hipError_t stretch_nc(int nc, const void* cube, int B, int64_t P, const ProjArgs& a, int nblocks,
                      const float* range_dev, uint8_t* images, hipStream_t s) {
  const size_t sm = smem_bytes(DT, B);
  const int q = q_for(DT, B);
#define CVX_STRETCH(N)                                                                                        \
  case N:                                                                                                     \
    if (q == 8)                                                                                               \
      CVX_LAUNCH((k_project_stretch<DT, N, 8>), sm, nblocks, s, cube, B, P, a,    \
                         range_dev, images);                                                                  \
    else                                                                                                      \
      CVX_LAUNCH((k_project_stretch<DT, N, kMaxQ>), sm, nblocks, s, cube, B, P, a, \
                         range_dev, images);                                                                  \
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

template <int DT>
hipError_t stretch_h16_nc(int nc, const void* cube, int B, int64_t P, const ProjArgs& a, int nblocks,
                          const float* range_dev, const _Float16* planes, int64_t Pp, uint8_t* images,
                          hipStream_t s) {
  const size_t sm = smem_bytes(DT, B);
  const int q = q_for(DT, B);
#define CVX_STRETCH(N)                                                                                        \
  case N:                                                                                                     \
    if (q == 8)                                                                                               \
      CVX_LAUNCH((k_project_stretch_h16<DT, N, 8>), sm, nblocks, s, cube, B, P, a, \
                         range_dev, planes, Pp, images);                                                      \
    else                                                                                                      \
      CVX_LAUNCH((k_project_stretch_h16<DT, N, kMaxQ>), sm, nblocks, s, cube, B,   \
                         P, a, range_dev, planes, Pp, images);                                                \
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

template <int DT>
hipError_t float_nc(int nc, const void* cube, int B, int64_t P, const ProjArgs& a, int nblocks, float* y,
                    hipStream_t s) {
  const size_t sm = smem_bytes(DT, B);
  const int q = q_for(DT, B);
#define CVX_FLOAT(N)                                                                                          \
  case N:                                                                                                     \
    if (q == 8)                                                                                               \
      CVX_LAUNCH((k_project_float<DT, N, 8>), sm, nblocks, s, cube, B, P, a, y);  \
    else                                                                                                      \
      CVX_LAUNCH((k_project_float<DT, N, kMaxQ>), sm, nblocks, s, cube, B, P, a, y); \
    break;
  switch (nc) {
    CVX_FLOAT(1) CVX_FLOAT(2) CVX_FLOAT(3) CVX_FLOAT(4) CVX_FLOAT(5) CVX_FLOAT(6) CVX_FLOAT(7) CVX_FLOAT(8)
    default:
      return hipErrorInvalidValue;
  }
#undef CVX_FLOAT
  return hipGetLastError();
}

}  // namespace proj

// Per-translation-unit entry points (one per group of instantiations).
hipError_t project_range_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                 int nblocks, float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                 hipStream_t s);
hipError_t project_stretch_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                   int nblocks, const float* range_dev, uint8_t* images, hipStream_t s);
hipError_t project_float_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                 int nblocks, float* y, hipStream_t s);
hipError_t project_range_h16_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                     int nblocks, float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                     const H16Args& h, _Float16* planes, int64_t Pp, hipStream_t s);
hipError_t project_stretch_h16_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                       int nblocks, const float* range_dev, const _Float16* planes, int64_t Pp,
                                       uint8_t* images, hipStream_t s);
}  // namespace cvx

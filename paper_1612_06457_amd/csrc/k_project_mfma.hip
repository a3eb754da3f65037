// Fused centre-project-stretch on the matrix cores, for bf16 and fp16 pages
// (paper Section 2: the regression coefficients multiply every band of the
// whole page; each float image is rescaled to 0..255 on its page range).
// uint16 pages take k_project_u16.hip.
//
// The projection Y = (X - c) W is a dense contraction over the bands
// (K = B, N = components).  On gfx950 with packed FP32 off, the VALU form
// needs about 2 B C FMAs plus conversions per pixel, which competes with
// the HBM stream at C = 7; here v_mfma_f32_16x16x32_bf16 does the FMAs and
// the VALU only builds operands.
//
//   A (16 pixels x 32 bands): lane l holds pixel l % 16, bands
//       32 kb + 8 (l / 16) + t, t = 0..7, as (x - c) split exactly into
//       bf16 hi + lo (x - c has at most 16 significant bits for bf16 pages,
//       with c of the page's type);
//   B (32 bands x 16 components): W split into three bf16 terms
//       w1 + w2 + w3 (24 significant bits), held in registers for the
//       whole kernel;
//   C (16 pixels x 16 components): lane l holds pixels 4 (l / 16) + e,
//       component l % 16.
// Products hi w1 + hi w2 + hi w3 + lo w1 + lo w2 (the dropped lo w3 is
// below 2^-24 of the term) accumulate in FP32, like the VALU path.  fp16
// pages use a third term for x - c.
//
// The page is streamed in wave tiles by the prefetching driver of
// k_tile.hpp (coalesced 16-byte loads of 64 lane groups, the next tile's
// loads in flight while the current one is computed); each lane then reads
// its pixel's 8 bands per 32-band block from the wave's LDS slice.
// Pass 1 keeps per-lane min/max for its component and the last block folds
// the block partials; pass 2 quantises q = floor(y s + o), clamped, and
// writes 4 consecutive pixels of one component plane per lane.
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int DT>
struct PG {
  static __device__ __host__ constexpr int g2(int B) { return (B & 1) ? 2 : 1; }
  static __device__ __host__ constexpr int S(int B) { return (B & 1) ? B : B / 2; }
};

// x - c for element e of the tile (16-bit storage), as an exact float.
template <int DT>
__device__ __forceinline__ float centred(const uint16_t* __restrict__ tile, int e, float c) {
  return to_float<DT>(tile[e]) - c;
}

// Per-lane constant operands and centres for NKB 32-band blocks.
template <int NKB>
struct Ops {
  bf16x8 w1[NKB], w2[NKB], w3[NKB];
  float c[NKB][8];
  float off;
};

template <int DT, int NKB>
__device__ __forceinline__ void load_ops(const ProjArgs& a, int B, int nc, Ops<NKB>& o) {
  const int lane = __lane_id();
  const int j = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int b = 32 * kb + 8 * g + t;
      const float w = (b < B && j < nc) ? a.w[b * nc + j] : 0.f;
      const __bf16 h1 = (__bf16)w;
      const float r1 = w - (float)h1;
      const __bf16 h2 = (__bf16)r1;
      const __bf16 h3 = (__bf16)(r1 - (float)h2);
      o.w1[kb][t] = h1;
      o.w2[kb][t] = h2;
      o.w3[kb][t] = h3;
      o.c[kb][t] = (b < B) ? a.c[b] : 0.f;
    }
  }
  o.off = (j < nc) ? a.off[j] : 0.f;
}

// y for the 16 pixels starting at tile row p0: acc[e] = y(pixel p0 + 4 (l/16) + e, component l % 16)
template <int DT, int NKB>
__device__ __forceinline__ f32x4 project16(const uint16_t* __restrict__ tile, int p0, int B,
                                           const Ops<NKB>& o) {
  const int lane = __lane_id();
  const int i = lane & 15, g = lane >> 4;
  f32x4 acc = {o.off, o.off, o.off, o.off};
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    bf16x8 hi, lo, l2;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int b = 32 * kb + 8 * g + t;
      float v = 0.f;
      if (b < B) v = centred<DT>(tile, (p0 + i) * B + b, o.c[kb][t]);
      const __bf16 h = (__bf16)v;
      const float r = v - (float)h;
      const __bf16 m = (__bf16)r;
      hi[t] = h;
      lo[t] = m;
      if constexpr (DT == DT_F16) l2[t] = (__bf16)(r - (float)m);
    }
    acc = mma(hi, o.w1[kb], acc);
    acc = mma(hi, o.w2[kb], acc);
    acc = mma(hi, o.w3[kb], acc);
    acc = mma(lo, o.w1[kb], acc);
    acc = mma(lo, o.w2[kb], acc);
    if constexpr (DT == DT_F16) acc = mma(l2, o.w1[kb], acc);
  }
  return acc;
}

template <int DT, int NKB>
__global__ __launch_bounds__(kBlock) void k_range_mfma(const void* __restrict__ cube, int B, int64_t P, int nc,
                                                       ProjArgs a, float* __restrict__ part,
                                                       unsigned* __restrict__ ticket,
                                                       float* __restrict__ range_dev,
                                                       float* __restrict__ ab_dev) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float wred[kWaves][32];
  __shared__ bool am_last;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int S = PG<DT>::S(B), g2 = PG<DT>::g2(B);
  uint32_t* my = lds + w * 64 * S;
  const uint16_t* tile = reinterpret_cast<const uint16_t*>(my);
  const int tp = 64 * g2;                       // pixels per wave tile (multiple of 16)
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * 2;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  Ops<NKB> o;
  load_ops<DT, NKB>(a, B, nc, o);
  float mn = __builtin_inff(), mx = -__builtin_inff();
  const int g = lane >> 4;
  for_each_tile<8 * NKB>(base, total_bytes, nt, S, my, [&](int64_t t) {
    const int64_t pix0 = t * tp;
    for (int p0 = 0; p0 < tp; p0 += 16) {
      const f32x4 y = project16<DT, NKB>(tile, p0, B, o);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (pix0 + p0 + 4 * g + e < P) {
          mn = fminf(mn, y[e]);
          mx = fmaxf(mx, y[e]);
        }
      }
    }
  });
  // lanes with the same component (l % 16) hold disjoint pixels
  mn = fminf(mn, __shfl_xor(mn, 16, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
  mn = fminf(mn, __shfl_xor(mn, 32, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  if (lane < 16) {
    wred[w][lane] = mn;
    wred[w][16 + lane] = mx;
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int j = threadIdx.x;
    float lo = wred[0][j], hi = wred[0][16 + j];
    for (int ww = 1; ww < kWaves; ++ww) {
      lo = fminf(lo, wred[ww][j]);
      hi = fmaxf(hi, wred[ww][16 + j]);
    }
    part[(int64_t)blockIdx.x * 32 + j] = lo;
    part[(int64_t)blockIdx.x * 32 + 16 + j] = hi;
    __threadfence();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    am_last = (atomicAdd(ticket, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  // last block: thread (slice, component) folds a strided subset of partials
  const int j = threadIdx.x & 15, sl = threadIdx.x >> 4;
  float lo = __builtin_inff(), hi = -__builtin_inff();
  for (unsigned bk = sl; bk < gridDim.x; bk += kBlock / 16) {
    lo = fminf(lo, __builtin_nontemporal_load(part + (int64_t)bk * 32 + j));
    hi = fmaxf(hi, __builtin_nontemporal_load(part + (int64_t)bk * 32 + 16 + j));
  }
  // slices 0..15 -> combine: lanes j, j+16, j+32, j+48 of each wave, then waves
  lo = fminf(lo, __shfl_xor(lo, 16, 64));
  hi = fmaxf(hi, __shfl_xor(hi, 16, 64));
  lo = fminf(lo, __shfl_xor(lo, 32, 64));
  hi = fmaxf(hi, __shfl_xor(hi, 32, 64));
  __syncthreads();
  if (lane < 16) {
    wred[w][lane] = lo;
    wred[w][16 + lane] = hi;
  }
  __syncthreads();
  if (threadIdx.x < 16 && threadIdx.x < nc) {
    const int jj = threadIdx.x;
    float l2 = wred[0][jj], h2 = wred[0][16 + jj];
    for (int ww = 1; ww < kWaves; ++ww) {
      l2 = fminf(l2, wred[ww][jj]);
      h2 = fmaxf(h2, wred[ww][16 + jj]);
    }
    float s, o;
    stretch_map(l2, h2, 255.f, s, o);
    range_dev[jj] = s;
    range_dev[8 + jj] = o;
    ab_dev[2 * jj] = l2;
    ab_dev[2 * jj + 1] = h2;
  }
  if (threadIdx.x == 0) *ticket = 0u;
}

__device__ __forceinline__ uint32_t quant(float y, float s, float o) {
  float t = floorf(fmaf(y, s, o));
  t = fminf(fmaxf(t, 0.f), 255.f);
  return (uint32_t)t;
}

template <int DT, int NKB>
__global__ __launch_bounds__(kBlock) void k_stretch_mfma(const void* __restrict__ cube, int B, int64_t P, int nc,
                                                         ProjArgs a, const float* __restrict__ range_dev,
                                                         uint8_t* __restrict__ images) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int S = PG<DT>::S(B), g2 = PG<DT>::g2(B);
  uint32_t* my = lds + w * 64 * S;
  const uint16_t* tile = reinterpret_cast<const uint16_t*>(my);
  const int tp = 64 * g2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * 2;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  Ops<NKB> o;
  load_ops<DT, NKB>(a, B, nc, o);
  const int j = lane & 15, g = lane >> 4;
  const bool active = j < nc;
  const float sc = active ? range_dev[j] : 0.f;
  const float of = active ? range_dev[8 + j] : 0.f;
  uint8_t* plane = images + (int64_t)(active ? j : 0) * P;
  const bool aligned4 = (P & 3) == 0 && (reinterpret_cast<uintptr_t>(images) & 3) == 0;
  for_each_tile<8 * NKB>(base, total_bytes, nt, S, my, [&](int64_t t) {
    const int64_t pix0 = t * tp;
    for (int p0 = 0; p0 < tp; p0 += 16) {
      const f32x4 y = project16<DT, NKB>(tile, p0, B, o);
      if (active) {
        const int64_t p = pix0 + p0 + 4 * g;
        const uint32_t q = quant(y[0], sc, of) | (quant(y[1], sc, of) << 8) | (quant(y[2], sc, of) << 16) |
                           (quant(y[3], sc, of) << 24);
        if (aligned4 && p + 3 < P) {
          *reinterpret_cast<uint32_t*>(plane + p) = q;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (p + e < P) plane[p + e] = (uint8_t)(q >> (8 * e));
        }
      }
    }
  });
}

// The FP32 component planes: lane (g, j) stores the 4 consecutive pixels it
// holds of plane j as one 16-byte write.
template <int DT, int NKB>
__global__ __launch_bounds__(kBlock) void k_float_mfma(const void* __restrict__ cube, int B, int64_t P, int nc,
                                                       ProjArgs a, float* __restrict__ y) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int S = PG<DT>::S(B), g2 = PG<DT>::g2(B);
  uint32_t* my = lds + w * 64 * S;
  const uint16_t* tile = reinterpret_cast<const uint16_t*>(my);
  const int tp = 64 * g2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * 2;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  Ops<NKB> o;
  load_ops<DT, NKB>(a, B, nc, o);
  const int j = lane & 15, g = lane >> 4;
  const bool active = j < nc;
  float* plane = y + (int64_t)(active ? j : 0) * P;
  const bool aligned = (P & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0;
  for_each_tile<8 * NKB>(base, total_bytes, nt, S, my, [&](int64_t t) {
    const int64_t pix0 = t * tp;
    for (int p0 = 0; p0 < tp; p0 += 16) {
      const f32x4 v = project16<DT, NKB>(tile, p0, B, o);
      if (active) {
        const int64_t p = pix0 + p0 + 4 * g;
        if (aligned && p + 3 < P) {
          *reinterpret_cast<f32x4*>(plane + p) = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (p + e < P) plane[p + e] = v[e];
        }
      }
    }
  });
}

size_t smem(int B) { return (size_t)kWaves * 64 * ((B & 1) ? B : B / 2) * 4; }

template <int DT>
hipError_t range_dt(int nkb, const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks,
                    float* part, unsigned* ticket, float* range_dev, float* ab_dev, hipStream_t s) {
  if (nkb == 1)
    hipLaunchKernelGGL((k_range_mfma<DT, 1>), dim3(nblocks), dim3(kBlock), smem(B), s, cube, B, P, nc, a, part,
                       ticket, range_dev, ab_dev);
  else
    hipLaunchKernelGGL((k_range_mfma<DT, 2>), dim3(nblocks), dim3(kBlock), smem(B), s, cube, B, P, nc, a, part,
                       ticket, range_dev, ab_dev);
  return hipGetLastError();
}

template <int DT>
hipError_t stretch_dt(int nkb, const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks,
                      const float* range_dev, uint8_t* images, hipStream_t s) {
  if (nkb == 1)
    hipLaunchKernelGGL((k_stretch_mfma<DT, 1>), dim3(nblocks), dim3(kBlock), smem(B), s, cube, B, P, nc, a,
                       range_dev, images);
  else
    hipLaunchKernelGGL((k_stretch_mfma<DT, 2>), dim3(nblocks), dim3(kBlock), smem(B), s, cube, B, P, nc, a,
                       range_dev, images);
  return hipGetLastError();
}

template <int DT>
hipError_t float_dt(int nkb, const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks, float* y,
                    hipStream_t s) {
  if (nkb == 1)
    hipLaunchKernelGGL((k_float_mfma<DT, 1>), dim3(nblocks), dim3(kBlock), smem(B), s, cube, B, P, nc, a, y);
  else
    hipLaunchKernelGGL((k_float_mfma<DT, 2>), dim3(nblocks), dim3(kBlock), smem(B), s, cube, B, P, nc, a, y);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_project_range_mfma(int dtype, const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                     int nblocks, float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                     hipStream_t s) {
  const int nkb = (B + 31) / 32;
  switch (dtype) {
    case DT_BF16: return range_dt<DT_BF16>(nkb, cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, s);
    case DT_F16: return range_dt<DT_F16>(nkb, cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_project_stretch_mfma(int dtype, const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                       int nblocks, const float* range_dev, uint8_t* images, hipStream_t s) {
  const int nkb = (B + 31) / 32;
  switch (dtype) {
    case DT_BF16: return stretch_dt<DT_BF16>(nkb, cube, B, P, nc, a, nblocks, range_dev, images, s);
    case DT_F16: return stretch_dt<DT_F16>(nkb, cube, B, P, nc, a, nblocks, range_dev, images, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_project_float_mfma(int dtype, const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                     int nblocks, float* y, hipStream_t s) {
  const int nkb = (B + 31) / 32;
  switch (dtype) {
    case DT_BF16: return float_dt<DT_BF16>(nkb, cube, B, P, nc, a, nblocks, y, s);
    case DT_F16: return float_dt<DT_F16>(nkb, cube, B, P, nc, a, nblocks, y, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace cvx

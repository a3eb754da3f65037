// Rescaling of projected float images to 8 or 16 bits, from FP32 component
// planes y[j][p] (paper Section 2, the three rescaling paragraphs and the
// 8- and 16-bit outputs):
//   mode 1  the page-wide minimum and maximum of each component;
//   mode 2  the minimum and maximum over the training pixels;
//   mode 3  the p-th and (100 - p)-th percentiles (linear interpolation
//           between order statistics), values beyond them clamped.
// The quantisation is the definition q = floor(L (y - a) / (b - a) + 1/2),
// clamped to 0..L (L = 255 or 65535), evaluated in FP64 step by step.  Mode
// 1 here finds the same range as the fused projection passes (which use the
// FP32 affine form of the same map).
//
// Order statistics are found exactly by a most-significant-digit radix
// select on the order-preserving 32-bit keys of the FP32 values: three
// passes, of 11, 11 and 10 bits (2,048-bin histograms in LDS; one pass, a
// full read of the planes, fewer than with 8-bit digits).  A pass builds, per component and per wanted rank, the
// histogram of the current digit over the keys that share the digits found
// so far (ranks whose found digits coincide share one histogram); a small
// kernel then picks the digit that holds the rank and the rank left within
// it.  Integer counts only: the result is exact and independent of the
// launch shape.  Histograms are double-buffered so that each pick clears
// the buffer the next pass fills, and nothing is cleared by a memset.
//
// Also here: the RGB composite of three 8-bit planes (paper Section 2: the
// component with the clearest underwriting usually goes to the green
// channel; Section 4: the same plane may fill two channels).
#include <algorithm>
#include <type_traits>

#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

__device__ __forceinline__ float ord2f(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Lowest active lane of the wave.
__device__ __forceinline__ bool first_active() {
  return (int)__lane_id() == __ffsll((unsigned long long)__ballot(1)) - 1;
}

// Block (blockIdx.x, plane j = blockIdx.y) partial min/max of plane j over
// all P pixels, or over the pixels idx[0..n) when idx is non-NULL (an index
// outside 0..P-1 is skipped and sets the value 2 in *err).
// part[(j * gridDim.x + blockIdx.x) * 2 + {0, 1}] = {min, max}.
__global__ __launch_bounds__(kBlock) void k_plane_minmax(const float* __restrict__ y, int64_t P,
                                                         const int64_t* __restrict__ idx, int64_t n,
                                                         float* __restrict__ part, int32_t* __restrict__ err) {
  __shared__ float red[kWaves][2];
  const int j = blockIdx.y;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float* yj = y + (int64_t)j * P;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  float lo = __builtin_inff(), hi = -__builtin_inff();
  if (idx) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
      const int64_t q = idx[i];
      if (q < 0 || q >= P) {
        bad = true;
        continue;
      }
      const float v = yj[q];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
    if (bad) atomicOr(err, 2);
  } else if ((P & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
    const float4* y4 = reinterpret_cast<const float4*>(yj);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P / 4; i += stride) {
      const float4 v = y4[i];
      lo = fminf(fminf(lo, v.x), fminf(v.y, fminf(v.z, v.w)));
      hi = fmaxf(fmaxf(hi, v.x), fmaxf(v.y, fmaxf(v.z, v.w)));
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P; i += stride) {
      const float v = yj[i];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if (lane == 0) {
    red[w][0] = lo;
    red[w][1] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int ww = 1; ww < kWaves; ++ww) {
      lo = fminf(lo, red[ww][0]);
      hi = fmaxf(hi, red[ww][1]);
    }
    part[((int64_t)j * gridDim.x + blockIdx.x) * 2] = lo;
    part[((int64_t)j * gridDim.x + blockIdx.x) * 2 + 1] = hi;
  }
}

// sel[j][t] = {bits found so far, rank still wanted}; both histogram
// buffers (2 x nc x kSelTargets x kSelBins) cleared.
__global__ __launch_bounds__(kBlock) void k_select_init(int nc, uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3,
                                                        uint2* __restrict__ sel, uint32_t* __restrict__ hist) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nc * kSelTargets) {
    const int t = i % kSelTargets;
    sel[i] = make_uint2(0u, t == 0 ? r0 : t == 1 ? r1 : t == 2 ? r2 : r3);
  }
  const int nh = 2 * nc * kSelTargets * kSelBins;
  for (int e = i; e < nh; e += gridDim.x * kBlock) hist[e] = 0u;
}

// The target whose histogram target t uses in this pass: the first one whose
// found bits (all above this pass's digit) equal t's.
__device__ __forceinline__ int rep_of(const uint32_t (&pre)[kSelTargets], int t, int pass) {
  if (pass == 0) return 0;
  const int sh = sel_shift(pass) + sel_width(pass);
  for (int u = 0; u < t; ++u)
    if ((pre[u] >> sh) == (pre[t] >> sh)) return u;
  return t;
}

__device__ __forceinline__ void count_key(uint32_t* __restrict__ h, uint32_t key, int pass,
                                          const uint32_t (&pre)[kSelTargets], const bool (&own)[kSelTargets]) {
  const int shift = sel_shift(pass);
  const uint32_t digit = (key >> shift) & ((1u << sel_width(pass)) - 1u);
  const uint32_t d0 = __builtin_amdgcn_readfirstlane(digit);
  const bool uniform = __all(digit == d0);
#pragma unroll
  for (int t = 0; t < kSelTargets; ++t) {
    if (!own[t]) continue;
    const bool m = pass == 0 || ((key ^ pre[t]) >> (shift + sel_width(pass))) == 0u;
    if (uniform) {
      // the whole wave has one digit (typical of the leading digit): one add
      const unsigned cnt = (unsigned)__popcll((unsigned long long)__ballot(m));
      if (cnt && first_active()) atomicAdd(&h[t * kSelBins + d0], cnt);
    } else if (m) {
      atomicAdd(&h[t * kSelBins + digit], 1u);
    }
  }
}

// One radix pass over plane j = blockIdx.y into histogram buffer `hist`.
__global__ __launch_bounds__(kBlock) void k_select_hist(const float* __restrict__ y, int64_t P,
                                                        const uint2* __restrict__ sel, int pass,
                                                        uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kSelTargets * kSelBins];
  const int j = blockIdx.y;
  for (int i = threadIdx.x; i < kSelTargets * kSelBins; i += kBlock) h[i] = 0u;
  uint32_t pre[kSelTargets];
  bool own[kSelTargets];
#pragma unroll
  for (int t = 0; t < kSelTargets; ++t) pre[t] = sel[j * kSelTargets + t].x;
#pragma unroll
  for (int t = 0; t < kSelTargets; ++t) own[t] = rep_of(pre, t, pass) == t;
  __syncthreads();
  const float* yj = y + (int64_t)j * P;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if ((P & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
    const float4* y4 = reinterpret_cast<const float4*>(yj);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P / 4; i += stride) {
      const float4 v = y4[i];
      count_key(h, f2ord(v.x), pass, pre, own);
      count_key(h, f2ord(v.y), pass, pre, own);
      count_key(h, f2ord(v.z), pass, pre, own);
      count_key(h, f2ord(v.w), pass, pre, own);
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P; i += stride)
      count_key(h, f2ord(yj[i]), pass, pre, own);
  }
  __syncthreads();
  uint32_t* out = hist + (int64_t)j * kSelTargets * kSelBins;
  for (int i = threadIdx.x; i < kSelTargets * kSelBins; i += kBlock)
    if (h[i]) atomicAdd(&out[i], h[i]);
}

// Block j (one per plane), wave t (one per target): find the digit of the
// histogram `cur` that holds target t's rank, record it, and clear target
// t's row of `nxt` (the buffer the next pass fills).  Lane l holds bins
// 32 l .. 32 l + 31.
__global__ __launch_bounds__(kBlock) void k_select_pick(int pass, uint2* __restrict__ sel,
                                                        const uint32_t* __restrict__ cur,
                                                        uint32_t* __restrict__ nxt) {
  constexpr int kPerLane = kSelBins / 64;
  const int j = blockIdx.x, t = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t pre[kSelTargets];
#pragma unroll
  for (int u = 0; u < kSelTargets; ++u) pre[u] = sel[j * kSelTargets + u].x;
  const uint32_t want = sel[j * kSelTargets + t].y;
  __syncthreads();   // every wave has read sel before any wave updates it
  const int r = rep_of(pre, t, pass);
  const uint4* row = reinterpret_cast<const uint4*>(cur + ((int64_t)j * kSelTargets + r) * kSelBins + kPerLane * lane);
  uint32_t bins[kPerLane];
#pragma unroll
  for (int q = 0; q < kPerLane / 4; ++q) {
    const uint4 c = row[q];
    bins[4 * q] = c.x;
    bins[4 * q + 1] = c.y;
    bins[4 * q + 2] = c.z;
    bins[4 * q + 3] = c.w;
  }
  uint32_t mine = 0;
#pragma unroll
  for (int e = 0; e < kPerLane; ++e) mine += bins[e];
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const unsigned long long hit = __ballot(incl > want);
  const int L = hit ? __ffsll(hit) - 1 : 63;
  if (lane == L) {
    uint32_t below = incl - mine;
    int d = kPerLane * lane + kPerLane - 1;
    for (int e = 0; e < kPerLane; ++e) {
      if (below + bins[e] > want) {
        d = kPerLane * lane + e;
        break;
      }
      below += bins[e];
    }
    sel[j * kSelTargets + t] = make_uint2(pre[t] | ((uint32_t)d << sel_shift(pass)), want - below);
  }
  uint4* z = reinterpret_cast<uint4*>(nxt + ((int64_t)j * kSelTargets + t) * kSelBins + kPerLane * lane);
#pragma unroll
  for (int q = 0; q < kPerLane / 4; ++q) z[q] = make_uint4(0u, 0u, 0u, 0u);
}

// NumPy's linear interpolation between neighbouring order statistics, in
// the same operation order (no contraction).
__device__ double lerp_stat(double a, double b, double g) {
#pragma clang fp contract(off)
  const double d = b - a;
  return g < 0.5 ? a + d * g : b - d * (1.0 - g);
}

// Block j: the range (a_j, b_j) of plane j.  Modes 1 and 2 fold the nb
// block partials; mode 3 interpolates the four selected order statistics
// with weights g_lo and g_hi.
__global__ __launch_bounds__(64) void k_stretch_finish(int mode, int nb, const float* __restrict__ part,
                                                       const uint2* __restrict__ sel, double g_lo, double g_hi,
                                                       double* __restrict__ ab) {
  const int j = blockIdx.x, lane = threadIdx.x;
  double a, b;
  if (mode != 3) {
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int k = lane; k < nb; k += 64) {
      lo = fminf(lo, part[((int64_t)j * nb + k) * 2]);
      hi = fmaxf(hi, part[((int64_t)j * nb + k) * 2 + 1]);
    }
    a = wave_min(lo);
    b = wave_max(hi);
  } else {
    const uint2* sj = sel + j * kSelTargets;
    a = lerp_stat(ord2f(sj[0].x), ord2f(sj[1].x), g_lo);
    b = lerp_stat(ord2f(sj[2].x), ord2f(sj[3].x), g_hi);
  }
  if (lane == 0) {
    ab[2 * j] = a;
    ab[2 * j + 1] = b;
  }
}

// q = clamp(floor(L (y - a) / (b - a) + 1/2), 0, L) in FP64, operation by
// operation (no contraction), so the result is the exact definition's for
// the FP32 value y; q = 0 when b <= a.  FP64 runs at the FP32 rate on this
// chip and the pass is bound by memory, so the exact form costs nothing
// (an FP32 map floor(y s + o) loses up to |a| / (b - a) 2^-7 levels at 16
// bits).
template <int BITS>
__device__ __forceinline__ uint32_t quant64(float y, double a, double den) {
#pragma clang fp contract(off)
  constexpr double L = BITS == 8 ? 255.0 : 65535.0;
  if (!(den > 0.0)) return 0u;
  double t = floor(L * ((double)y - a) / den + 0.5);
  t = fmin(fmax(t, 0.0), L);
  return (uint32_t)t;
}

// Plane j = blockIdx.y: q = quant64(y) on the range of plane j, 4 pixels per
// thread step (one 16-byte read, one 4- or 8-byte write).
template <int BITS>
__global__ __launch_bounds__(kBlock) void k_stretch_planes(const float* __restrict__ y, int64_t P,
                                                           const double* __restrict__ ab, void* __restrict__ out) {
  using OutT = typename std::conditional<BITS == 8, uint8_t, uint16_t>::type;
  const int j = blockIdx.y;
  const double a = ab[2 * j], den = ab[2 * j + 1] - ab[2 * j];
  const float* yj = y + (int64_t)j * P;
  OutT* oj = reinterpret_cast<OutT*>(out) + (int64_t)j * P;
  const bool vec = (P & 3) == 0 && ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  const int64_t n4 = (P + 3) / 4;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kBlock) {
    const int64_t p = 4 * i;
    if (vec) {
      const float4 v = *reinterpret_cast<const float4*>(yj + p);
      const uint32_t q0 = quant64<BITS>(v.x, a, den), q1 = quant64<BITS>(v.y, a, den);
      const uint32_t q2 = quant64<BITS>(v.z, a, den), q3 = quant64<BITS>(v.w, a, den);
      if constexpr (BITS == 8) {
        *reinterpret_cast<uint32_t*>(oj + p) = q0 | (q1 << 8) | (q2 << 16) | (q3 << 24);
      } else {
        *reinterpret_cast<uint2*>(oj + p) = make_uint2(q0 | (q1 << 16), q2 | (q3 << 16));
      }
    } else {
      for (int e = 0; e < 4 && p + e < P; ++e) oj[p + e] = (OutT)quant64<BITS>(yj[p + e], a, den);
    }
  }
}

__device__ __forceinline__ uint32_t byte_of(uint32_t x, int i) { return (x >> (8 * i)) & 255u; }

// rgb[3 p + c] = channel c at pixel p (0 for a NULL channel), 4 pixels per
// thread step when every pointer is 4-byte aligned and P % 4 == 0.
__global__ __launch_bounds__(kBlock) void k_compose_rgb(const uint8_t* __restrict__ r, const uint8_t* __restrict__ g,
                                                        const uint8_t* __restrict__ b, int64_t P,
                                                        uint8_t* __restrict__ rgb) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(r) | reinterpret_cast<uintptr_t>(g) |
                       reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(rgb);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if ((P & 3) == 0 && (al & 3) == 0) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P / 4; i += stride) {
      const uint32_t R = r ? reinterpret_cast<const uint32_t*>(r)[i] : 0u;
      const uint32_t G = g ? reinterpret_cast<const uint32_t*>(g)[i] : 0u;
      const uint32_t B = b ? reinterpret_cast<const uint32_t*>(b)[i] : 0u;
      uint32_t* o = reinterpret_cast<uint32_t*>(rgb) + 3 * i;
      o[0] = byte_of(R, 0) | (byte_of(G, 0) << 8) | (byte_of(B, 0) << 16) | (byte_of(R, 1) << 24);
      o[1] = byte_of(G, 1) | (byte_of(B, 1) << 8) | (byte_of(R, 2) << 16) | (byte_of(G, 2) << 24);
      o[2] = byte_of(B, 2) | (byte_of(R, 3) << 8) | (byte_of(G, 3) << 16) | (byte_of(B, 3) << 24);
    }
  } else {
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P; p += stride) {
      rgb[3 * p + 0] = r ? r[p] : 0;
      rgb[3 * p + 1] = g ? g[p] : 0;
      rgb[3 * p + 2] = b ? b[p] : 0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0u;
}

int blocks_for(int64_t work, int64_t per_block, int cap) {
  const int64_t nb = (work + per_block - 1) / per_block;
  return (int)(nb < 1 ? 1 : (nb > cap ? cap : nb));
}

}  // namespace

int stretch_reduce_blocks(int64_t m, int nc, int num_cu) {
  return blocks_for(m, (int64_t)kBlock * 16, std::max(1, 8 * num_cu / std::max(1, nc)));
}

hipError_t launch_plane_minmax(const float* y, int64_t P, int nc, const int64_t* idx, int64_t n, int nb,
                               float* part, int32_t* err, hipStream_t s) {
  if (nc < 1 || nc > kMaxB || nb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plane_minmax, dim3(nb, nc), dim3(kBlock), 0, s, y, P, idx, n, part, err);
  return hipGetLastError();
}

hipError_t launch_select(const float* y, int64_t P, int nc, const uint32_t (&ranks)[kSelTargets], int nb,
                         uint2* sel, uint32_t* hist, hipStream_t s) {
  if (nc < 1 || nc > kMaxB || nb < 1) return hipErrorInvalidValue;
  const int nh = 2 * nc * kSelTargets * kSelBins;
  hipLaunchKernelGGL(k_select_init, dim3((nh + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nc, ranks[0], ranks[1],
                     ranks[2], ranks[3], sel, hist);
  const int64_t half = (int64_t)nc * kSelTargets * kSelBins;
  for (int pass = 0; pass < kSelPasses; ++pass) {
    uint32_t* cur = hist + (pass & 1) * half;
    uint32_t* nxt = hist + ((pass + 1) & 1) * half;
    hipLaunchKernelGGL(k_select_hist, dim3(nb, nc), dim3(kBlock), 0, s, y, P, (const uint2*)sel, pass, cur);
    hipLaunchKernelGGL(k_select_pick, dim3(nc), dim3(kBlock), 0, s, pass, sel, (const uint32_t*)cur, nxt);
  }
  return hipGetLastError();
}

hipError_t launch_stretch_finish(int mode, int nc, int nb, const float* part, const uint2* sel, double g_lo,
                                 double g_hi, double* ab, hipStream_t s) {
  if (nc < 1 || nc > kMaxB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stretch_finish, dim3(nc), dim3(64), 0, s, mode, nb, part, sel, g_lo, g_hi, ab);
  return hipGetLastError();
}

hipError_t launch_stretch_planes(const float* y, int64_t P, int nc, const double* ab, int bits, void* out,
                                 int num_cu, hipStream_t s) {
  if (nc < 1 || nc > kMaxB || (bits != 8 && bits != 16)) return hipErrorInvalidValue;
  const dim3 grid(blocks_for((P + 3) / 4, kBlock, std::max(1, 8 * num_cu / nc)), nc);
  if (bits == 8) hipLaunchKernelGGL(k_stretch_planes<8>, grid, dim3(kBlock), 0, s, y, P, ab, out);
  else hipLaunchKernelGGL(k_stretch_planes<16>, grid, dim3(kBlock), 0, s, y, P, ab, out);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(blocks_for(n, kBlock, 1024)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_compose_rgb(const uint8_t* r, const uint8_t* g, const uint8_t* b, int64_t P, uint8_t* rgb,
                              int num_cu, hipStream_t s) {
  hipLaunchKernelGGL(k_compose_rgb, dim3(blocks_for(P, 4 * kBlock, 8 * num_cu)), dim3(kBlock), 0, s, r, g, b, P,
                     rgb);
  return hipGetLastError();
}

}  // namespace cvx

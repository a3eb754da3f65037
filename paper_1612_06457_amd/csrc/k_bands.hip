// A page's band images, as read from a stack of per-band image files
// (paper Section 2: the 23 multispectral images of a page, 8-bit, one per
// illumination), laid band-sequentially (B planes of P pixels) are turned
// into the band-interleaved page the other kernels read (P rows of B
// elements).  8- and 16-bit bands become 16-bit elements (values kept), 32-bit
// float bands stay float.
//
// A block transposes a tile of kTilePix pixels x all B bands through LDS:
// each thread reads 4 consecutive pixels of one band (one 4- or 8-byte load,
// coalesced along the band), writes them into the pixel-major LDS tile, and
// the tile leaves as whole 16-byte chunks of the output rows.  The last,
// partial tile (and pages whose P is not a multiple of 4) go element by
// element.
#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

constexpr int kTilePix = 256;

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_bands_to_cube(const Tin* __restrict__ bands, int B, int64_t P,
                                                          Tout* __restrict__ cube) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Tout* tile = reinterpret_cast<Tout*>(lds_raw);   // kTilePix x B, pixel-major
  const int64_t p0 = (int64_t)blockIdx.x * kTilePix;
  const int npx = (int)min<int64_t>(kTilePix, P - p0);
  const bool whole = npx == kTilePix && (P & 3) == 0 && (reinterpret_cast<uintptr_t>(bands) & 15) == 0;
  if (whole) {
    // thread (band row r, quad i): pixels 4 i .. 4 i + 3 of band r
    const int i = threadIdx.x & 63;
    for (int b = threadIdx.x >> 6; b < B; b += kWaves) {
      const Tin* src = bands + (int64_t)b * P + p0 + 4 * i;
      Tin v[4];
      if constexpr (sizeof(Tin) == 1) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(src);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (Tin)((w >> (8 * q)) & 255u);
      } else if constexpr (sizeof(Tin) == 2) {
        const uint2 w = *reinterpret_cast<const uint2*>(src);
        v[0] = (Tin)(w.x & 0xffffu);
        v[1] = (Tin)(w.x >> 16);
        v[2] = (Tin)(w.y & 0xffffu);
        v[3] = (Tin)(w.y >> 16);
      } else {
        const float4 w = *reinterpret_cast<const float4*>(src);
        v[0] = w.x;
        v[1] = w.y;
        v[2] = w.z;
        v[3] = w.w;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) tile[(4 * i + q) * B + b] = (Tout)v[q];
    }
  } else {
    for (int e = threadIdx.x; e < B * kTilePix; e += kBlock) {
      const int b = e / kTilePix, i = e % kTilePix;
      if (i < npx) tile[i * B + b] = (Tout)bands[(int64_t)b * P + p0 + i];
    }
  }
  __syncthreads();
  Tout* dst = cube + p0 * B;
  const int nel = npx * B;
  if (whole && (reinterpret_cast<uintptr_t>(cube) & 15) == 0) {
    // kTilePix B elements = 16-byte chunks (kTilePix is a multiple of 8)
    constexpr int per = 16 / sizeof(Tout);
    for (int c = threadIdx.x; c < nel / per; c += kBlock)
      *reinterpret_cast<uint4*>(dst + per * c) = *reinterpret_cast<const uint4*>(tile + per * c);
  } else {
    for (int e = threadIdx.x; e < nel; e += kBlock) dst[e] = tile[e];
  }
}

// Small result regions to page-locked host memory, written by the kernel
// itself (16-byte stores when both ends allow).  A DMA copy would queue
// behind whatever large transfer the copy engines are busy with (for
// example the next page's upload), stalling the host's FP64 finish.
__global__ __launch_bounds__(kBlock) void k_copy_out(unsigned char* __restrict__ dst,
                                                     const unsigned char* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) == 0) {
    const int64_t n16 = n / 16;
    for (int64_t i = i0; i < n16; i += stride)
      reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
    for (int64_t i = 16 * n16 + i0; i < n; i += stride) dst[i] = src[i];
  } else {
    for (int64_t i = i0; i < n; i += stride) dst[i] = src[i];
  }
}

}  // namespace

hipError_t launch_copy_out(void* dst, const void* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t chunks = (n + 16 * kBlock - 1) / (16 * kBlock);
  const unsigned nb = (unsigned)(chunks < 64 ? chunks : 64);
  hipLaunchKernelGGL(k_copy_out, dim3(nb), dim3(kBlock), 0, s, (unsigned char*)dst, (const unsigned char*)src, n);
  return hipGetLastError();
}

hipError_t launch_bands_to_cube(int in_dtype, const void* bands, int B, int64_t P, void* cube, hipStream_t s) {
  if (B < 1 || B > kMaxB || P < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((P + kTilePix - 1) / kTilePix));
  switch (in_dtype) {
    case DT_U8:
      hipLaunchKernelGGL((k_bands_to_cube<uint8_t, uint16_t>), grid, dim3(kBlock), (size_t)kTilePix * B * 2, s,
                         (const uint8_t*)bands, B, P, (uint16_t*)cube);
      break;
    case DT_U16:
      hipLaunchKernelGGL((k_bands_to_cube<uint16_t, uint16_t>), grid, dim3(kBlock), (size_t)kTilePix * B * 2, s,
                         (const uint16_t*)bands, B, P, (uint16_t*)cube);
      break;
    case DT_F32:
      hipLaunchKernelGGL((k_bands_to_cube<float, float>), grid, dim3(kBlock), (size_t)kTilePix * B * 4, s,
                         (const float*)bands, B, P, (float*)cube);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cvx

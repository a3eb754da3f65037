// Page covariance (paper Section 2: PCA of the whole page) on the gfx950
// matrix cores: the augmented Gram of [x - s, 1] over all (or the masked)
// pixels with the compensated split of k_split.hpp.  The page is streamed in
// wave tiles (k_tile.hpp) with the next tile's loads in flight; each wave
// folds its FP32 tiles into FP64 after every wave tile, and the waves of a
// block combine in a fixed order into the packed partial layout.
//
// Shift: the mean of 64 pixels spread evenly over the page (rounded to the
// element type for 16-bit pages), summed in a fixed order by every block.
#include <type_traits>

#include "k_split.hpp"
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

template <int DT, int SPLIT, int NRB>
__global__ __launch_bounds__(kBlock) void k_pca_gram_mfma(const void* __restrict__ cube, int B, int64_t P,
                                                          const uint8_t* __restrict__ mask, float scale,
                                                          double* __restrict__ part,
                                                          double* __restrict__ shift_out) {
  constexpr int Q = 4 * NRB < kMaxQ ? 4 * NRB : kMaxQ;   // chunks per lane: S <= 16 NRB - 1 dwords
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float cs[kMaxB];
  __shared__ uint8_t vrow[kWaves][128];
  const int S = Geo<DT>::S(B), g2 = Geo<DT>::g2(B);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* my = lds + w * 64 * S;
  double* red = reinterpret_cast<double*>(lds);
  using T = typename Elem<DT>::T;
  const T* cx = reinterpret_cast<const T*>(cube);

  // shift: mean of 64 pixels spread evenly over the page, fixed order
  for (int b = threadIdx.x; b < B; b += kBlock) {
    float x[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = to_float<DT>(cx[((int64_t)i * P / 64) * B + b]);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 64; ++i) s += x[i];
    const float c = round_shift<DT>(s / 64.f);
    cs[b] = c;
    if (blockIdx.x == 0) shift_out[b] = (double)c;
  }
  __syncthreads();

  constexpr int NP = npairs(NRB);
  f32x4 acc[NP];
  double accd[NP][4];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[p][e] = 0.f;
      accd[p][e] = 0.0;
    }
  const int tp = 64 * g2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * (int64_t)Geo<DT>::esize;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  for_each_tile<Q>(base, total_bytes, nt, S, my, [&](int64_t t) {
    const int64_t pix0 = t * tp;
    // row validity (page end, mask), needed only for tiles not wholly taken
    const bool full = pix0 + tp <= P && mask == nullptr;
    if (!full) {
      for (int r = lane; r < tp; r += 64) {
        const int64_t p = pix0 + r;
        vrow[w][r] = (p < P && (mask == nullptr || mask[p] != 0)) ? 1 : 0;
      }
      wave_lds_sync();
    }
    auto ksteps = [&](auto whole) {
      constexpr bool WHOLE = decltype(whole)::value;
      auto get = [&](int r, int band) {
        float v = 0.f;
        if (WHOLE || vrow[w][r]) {
          if (band < B) {
            if constexpr (DT == DT_F32) v = (reinterpret_cast<const float*>(my)[r * B + band] - cs[band]) * scale;
            else v = (to_float<DT>(reinterpret_cast<const uint16_t*>(my)[r * B + band]) - cs[band]) * scale;
          } else if (band == B) {
            v = 1.f;
          }
        }
        return v;
      };
      for (int k0 = 0; k0 < tp; k0 += 32) kstep<SPLIT, NRB>(get, k0, acc);
    };
    if (full) ksteps(std::true_type{});
    else ksteps(std::false_type{});
    fold<NRB>(acc, accd);
  });
  __syncthreads();
  block_combine<NRB>(accd, B, scale, red, part + (int64_t)blockIdx.x * packed_doubles(B));
}

// uint16 pages: exact fp16 operands built with bit operations.  With
// x = 1024 h + l (h: 6 bits, l: 10 bits) and the integer shift
// c = 1024 c_h + c_l, v = (x - c) / 1024 = (h - c_h) + (l - c_l) / 1024:
// the fp16 with bits 0x6400 | h is 1024 + h and the one with bits
// 0x3c00 | l is 1 + l / 1024, so one AND-OR and one packed fp16 add give
// each term exactly, two pixels per dword.  Every product of two terms is
// exact in FP32 (at most 22 significant bits); the Gram of v is summed as
// H H + H L + L H + L L on v_mfma_f32_16x16x32_f16 and unscaled by 2^20 in
// FP64.  The ones column holds 1 in the L term.  Rows that hold no pixel
// (the page's end, the mask) are zeroed by a per-pixel mask, computed only
// for tiles that need it.
template <int NRB>
__global__ __launch_bounds__(kBlock) void k_pca_gram_u16(const void* __restrict__ cube, int B, int64_t P,
                                                         const uint8_t* __restrict__ mask,
                                                         double* __restrict__ part,
                                                         double* __restrict__ shift_out) {
  constexpr int Q = 4 * NRB < kMaxQ ? 4 * NRB : kMaxQ;   // chunks per lane: S <= 16 NRB - 1 dwords
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float cs[kMaxB];
  __shared__ uint8_t vrow[kWaves][128];
  const int S = Geo<DT_U16>::S(B), g2 = Geo<DT_U16>::g2(B);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  uint32_t* my = lds + w * 64 * S;
  double* red = reinterpret_cast<double*>(lds);
  const uint16_t* cx = reinterpret_cast<const uint16_t*>(cube);

  // shift: integer mean of 64 pixels spread evenly over the page, fixed order
  for (int b = threadIdx.x; b < B; b += kBlock) {
    float x[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = (float)cx[((int64_t)i * P / 64) * B + b];
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 64; ++i) s += x[i];
    const float c = rintf(s / 64.f);
    cs[b] = c;
    if (blockIdx.x == 0) shift_out[b] = (double)c;
  }
  __syncthreads();

  // per row block: this lane's band, its load column, the negated shift terms
  // and the masks that keep real bands and put 1 in the ones column
  U16Lane<NRB> ln;
  ln.init(B, cs, col);
  const U16Masks mk = make_u16_masks();

  constexpr int NP = npairs(NRB);
  f32x4 acc[NP];
  double accd[NP][4];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[p][e] = 0.f;
      accd[p][e] = 0.0;
    }
  const int tp = 64 * g2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * 2;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  for_each_tile<Q>(base, total_bytes, nt, S, my, [&](int64_t t) {
    const int64_t pix0 = t * tp;
    const bool full = pix0 + tp <= P && mask == nullptr;
    if (!full) {
      for (int r = lane; r < tp; r += 64) {
        const int64_t p = pix0 + r;
        vrow[w][r] = (p < P && (mask == nullptr || mask[p] != 0)) ? 1 : 0;
      }
      wave_lds_sync();
    }
    const uint16_t* tile = reinterpret_cast<const uint16_t*>(my);
    // whole tiles (the common case) build their operands with no row mask
    auto ksteps = [&](auto whole) {
      constexpr bool WHOLE = decltype(whole)::value;
      for (int k0 = 0; k0 < tp; k0 += 32) {
        f16x8 Hv[NRB], Lv[NRB];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          u32x4 H, L;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = k0 + 8 * grp + 2 * u;
            const uint32_t d =
                (uint32_t)tile[r * B + ln.bcol[rb]] | ((uint32_t)tile[(r + 1) * B + ln.bcol[rb]] << 16);
            uint32_t rm = 0xffffffffu;
            if constexpr (!WHOLE) rm = (vrow[w][r] ? 0x0000ffffu : 0u) | (vrow[w][r + 1] ? 0xffff0000u : 0u);
            uint32_t h, l;
            ln.terms(d, rb, rm, mk, h, l);
            H[u] = h;
            L[u] = l;
          }
          Hv[rb] = __builtin_bit_cast(f16x8, H);
          Lv[rb] = __builtin_bit_cast(f16x8, L);
        }
        u16_tile_products<NRB>(Hv, Lv, acc);
      }
    };
    if (full) ksteps(std::true_type{});
    else ksteps(std::false_type{});
    fold<NRB>(acc, accd);
  });
  __syncthreads();
  block_combine<NRB>(accd, B, 1.f / 1024.f, red, part + (int64_t)blockIdx.x * packed_doubles(B));
}

template <int DT, int SPLIT>
hipError_t pca_launch_dt(const void* cube, int B, int64_t P, const uint8_t* mask, int nblocks, double* part,
                         double* shift_out, hipStream_t s) {
  const int S = Geo<DT>::S(B);
  const size_t sm = std::max((size_t)kWaves * 64 * S * 4, packed_doubles(B) * 8);
  const float sc = prescale(DT, SPLIT);
  switch (nrb_for(B)) {
    case 2:
      hipLaunchKernelGGL((k_pca_gram_mfma<DT, SPLIT, 2>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, mask,
                         sc, part, shift_out);
      break;
    case 3:
      hipLaunchKernelGGL((k_pca_gram_mfma<DT, SPLIT, 3>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, mask,
                         sc, part, shift_out);
      break;
    default:
      hipLaunchKernelGGL((k_pca_gram_mfma<DT, SPLIT, 5>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, mask,
                         sc, part, shift_out);
      break;
  }
  return hipGetLastError();
}

hipError_t pca_launch_u16(const void* cube, int B, int64_t P, const uint8_t* mask, int nblocks, double* part,
                          double* shift_out, hipStream_t s) {
  const int S = Geo<DT_U16>::S(B);
  const size_t sm = std::max((size_t)kWaves * 64 * S * 4, packed_doubles(B) * 8);
  switch (nrb_for(B)) {
    case 2:
      hipLaunchKernelGGL((k_pca_gram_u16<2>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, mask, part,
                         shift_out);
      break;
    case 3:
      hipLaunchKernelGGL((k_pca_gram_u16<3>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, mask, part,
                         shift_out);
      break;
    default:
      hipLaunchKernelGGL((k_pca_gram_u16<5>), dim3(nblocks), dim3(kBlock), sm, s, cube, B, P, mask, part,
                         shift_out);
      break;
  }
  return hipGetLastError();
}

template <int SPLIT>
hipError_t pca_launch(int dtype, const void* cube, int B, int64_t P, const uint8_t* mask, int nblocks,
                      double* part, double* shift_out, hipStream_t s) {
  switch (dtype) {
    // uint16 pages: the exact bit-built operands whatever split was asked
    // (every product is exact either way)
    case DT_U16: return pca_launch_u16(cube, B, P, mask, nblocks, part, shift_out, s);
    case DT_F32: return pca_launch_dt<DT_F32, SPLIT>(cube, B, P, mask, nblocks, part, shift_out, s);
    case DT_BF16: return pca_launch_dt<DT_BF16, SPLIT>(cube, B, P, mask, nblocks, part, shift_out, s);
    case DT_F16: return pca_launch_dt<DT_F16, SPLIT>(cube, B, P, mask, nblocks, part, shift_out, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_pca_gram_mfma(int dtype, int split, const void* cube, int B, int64_t P, const uint8_t* mask,
                                int nblocks, double* part, double* shift_out, hipStream_t s) {
  if (B < 1 || B > kMaxB || nblocks < 1) return hipErrorInvalidValue;
  if (split == 0) return pca_launch<0>(dtype, cube, B, P, mask, nblocks, part, shift_out, s);
  return pca_launch<1>(dtype, cube, B, P, mask, nblocks, part, shift_out, s);
}

}  // namespace cvx

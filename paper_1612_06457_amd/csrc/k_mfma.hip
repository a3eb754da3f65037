// Page covariance (paper Section 2: PCA of the whole page) on the gfx950
// matrix cores: the augmented Gram of [x - s, 1] over all (or the masked)
// pixels.  The page is streamed in wave tiles (k_tile.hpp) with the next
// tile's loads in flight.  uint16 pages take exact int8 digit products
// (k_pca_gram_u16); the other element types take the compensated split of
// k_split.hpp, each wave folding its FP32 tiles into FP64 after every wave
// tile and the waves of a block combining in a fixed order.  Either way a
// block writes its partial in the packed layout of the fixed-order
// reduction.
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

// uint16 pages: an exact integer Gram on the int8 matrix cores.  Each
// x = 256 h + l is written y = x - 32896 = 256 (h - 128) + (l - 128): the
// high and the low byte with their top bit flipped are the two signed int8
// digits of y.  With digit vectors H and L,
//   y_i y_j = 65536 H_i H_j + 256 (H_i L_j + L_i H_j) + L_i L_j,
// and v_mfma_i32_16x16x64_i8 sums the three kinds of products over 64
// pixels per instruction in int32 with no rounding (each product is at most
// 2^14 in size).  The int32 tiles fold into FP64 every kFoldTiles wave
// tiles (at most 2^25 in size then); the sum is an integer below 2^53, so
// the fold is exact.  The ones column holds the digit pair (0, 1), whose
// value is 1.  Rows that hold no pixel (the page's end, the mask) get zero
// digits, value 0, ones column included.
//
// The waves of a block add their folds into one packed Gram in LDS; the
// sums stay integers below 2^53 while a block covers fewer than 2^22
// pixels, so they are exact in any order.  The block then moves the origin from
// 32896 to the shift c, still in exact integer arithmetic: with
// d = c - 32896 and u = [y, 1], [x - c, 1] = M u for M = [[I, -d], [0, 1]],
// so the Gram about c is M G M^T.  The block partial is then the same
// quantity, in the same packed layout, as that of every other Gram kernel.
//
// Operand layout: lane l holds band 16 rb + l % 16 of pixels
// k0 + 16 (l / 16) + s, s = 0..15, one byte each.  A and B take the same
// register, and the instruction pairs the k slots of A and B alike, so the
// pixel order inside a K step does not matter.  Reads of bands past B in
// the last row block (zeroed by a lane mask) may run up to 2 (16 NRB - B)
// bytes past a wave's tile: the launch pads LDS for that.
constexpr int kFoldTiles = 8;

// packed Gram doubles for the most bands: 4 x 4 tiles of the padded (B+1)^2
constexpr int kMaxPacked = ((kMaxB + 4) / 4) * ((kMaxB + 4) / 4 + 1) / 2 * 16;

// LDS of the wave tiles, with room for reads of bands past B after the last
inline size_t tile_area_bytes(int B) { return (size_t)kWaves * 64 * Geo<DT_U16>::S(B) * 4 + 128; }
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ i32x4 mma_i8(i32x4 a, i32x4 b, i32x4 c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// Row blocks whose 16 bands are real for every B this NRB serves (B + 1 in
// 17..32, 33..48 or 49..80 bands): these need no lane mask.
// Two waves per SIMD where the registers allow it without spilling (up to
// 48 padded bands: 256 registers).
template <int NRB>
constexpr int pca_u16_waves() { return NRB <= 3 ? 2 : 1; }

template <int NRB>
constexpr int full_rbs() { return NRB == 2 ? 0 : (NRB == 3 ? 2 : 3); }

template <int NRB>
__global__ __launch_bounds__(kBlock, (pca_u16_waves<NRB>())) void k_pca_gram_u16(const void* __restrict__ cube, int B, int64_t P,
                                                         const uint8_t* __restrict__ mask,
                                                         double* __restrict__ part,
                                                         double* __restrict__ shift_out) {
  constexpr int Q = 4 * NRB < kMaxQ ? 4 * NRB : kMaxQ;   // chunks per lane: S <= 16 NRB - 1 dwords
  constexpr int NF = full_rbs<NRB>();
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float cs[kMaxB];
  __shared__ __align__(4) uint8_t vrow[kWaves][128];
  __shared__ double red[kMaxPacked];
  const int S = Geo<DT_U16>::S(B), g2 = Geo<DT_U16>::g2(B);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  uint32_t* my = lds + w * 64 * S;
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

  // lane masks of the row blocks that may hold bands past B: keep real
  // bands, put the digit pair (0, 1) in the ones column
  uint32_t keep[NRB], ones[NRB];
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    const int band = 16 * rb + col;
    keep[rb] = band < B ? 0xffffffffu : 0u;
    ones[rb] = band == B ? 0x01010101u : 0u;
  }
  const uint32_t flip = 0x80808080u;

  // the block's packed Gram of [y, 1]: every fold adds integers below 2^53
  // into it, so the order of the adds does not matter
  const int D = B + 1, BP = (D + 3) & ~3, nb = BP / 4, L = nb * (nb + 1) / 2 * 16;
  for (int t = threadIdx.x; t < L; t += kBlock) red[t] = 0.0;
  constexpr int NP = npairs(NRB);
  i32x4 acc_hh[NP], acc_x[NP], acc_ll[NP];
  auto clear = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc_hh[p][e] = acc_x[p][e] = acc_ll[p][e] = 0;
  };
  clear();
  auto fold_i8 = [&]() __attribute__((always_inline)) {
    int p = 0;
#pragma unroll
    for (int ri = 0; ri < NRB; ++ri) {
#pragma unroll
      for (int rj = ri; rj < NRB; ++rj, ++p) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int I = 16 * ri + 4 * grp + e, J = 16 * rj + col;
          if ((I >> 2) <= (J >> 2) && I < D && J < D) {
            const int bi = I >> 2, bj = J >> 2;
            const double v = 65536.0 * (double)acc_hh[p][e] + 256.0 * (double)acc_x[p][e] + (double)acc_ll[p][e];
            atomicAdd(&red[(bi * nb - bi * (bi - 1) / 2 + (bj - bi)) * 16 + (I & 3) * 4 + (J & 3)], v);
          }
        }
      }
    }
    clear();
  };
  __syncthreads();
  const int tp = 64 * g2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * 2;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  const unsigned char* lane_base = reinterpret_cast<const unsigned char*>(my) + 2 * (16 * grp * B + col);
  int tiles = 0;
  for_each_tile<Q>(base, total_bytes, nt, S, my, [&](int64_t t) __attribute__((always_inline)) {
    const int64_t pix0 = t * tp;
    const bool full = pix0 + tp <= P && mask == nullptr;
    if (!full) {
      for (int r = lane; r < tp; r += 64) {
        const int64_t p = pix0 + r;
        vrow[w][r] = (p < P && (mask == nullptr || mask[p] != 0)) ? 1 : 0;
      }
      wave_lds_sync();
    }
    // whole tiles (the common case) build their operands with no row mask
    auto ksteps = [&](auto whole) __attribute__((always_inline)) {
      constexpr bool WHOLE = decltype(whole)::value;
      for (int k0 = 0; k0 < tp; k0 += 64) {
        i32x4 Hv[NRB], Lv[NRB];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const unsigned char* rp = lane_base + 2 * (k0 + 4 * q) * B;
          uint32_t rm = 0xffffffffu;
          if constexpr (!WHOLE)
            rm = 0xffu * *reinterpret_cast<const uint32_t*>(&vrow[w][k0 + 16 * grp + 4 * q]);
#pragma unroll
          for (int rb = 0; rb < NRB; ++rb) {
            const unsigned char* a = rp + 32 * rb;
            const uint32_t x0 = *reinterpret_cast<const uint16_t*>(a);
            const uint32_t x1 = *reinterpret_cast<const uint16_t*>(a + 2 * B);
            const uint32_t x2 = *reinterpret_cast<const uint16_t*>(a + 4 * B);
            const uint32_t x3 = *reinterpret_cast<const uint16_t*>(a + 6 * B);
            const uint32_t d01 = x0 | (x1 << 16), d23 = x2 | (x3 << 16);
            uint32_t h = __builtin_amdgcn_perm(d23, d01, 0x07050301u) ^ flip;
            uint32_t l = __builtin_amdgcn_perm(d23, d01, 0x06040200u) ^ flip;
            if (rb >= NF) {
              h &= keep[rb];
              l = (l & keep[rb]) | ones[rb];
            }
            if constexpr (!WHOLE) {
              h &= rm;
              l &= rm;
            }
            Hv[rb][q] = (int)h;
            Lv[rb][q] = (int)l;
          }
        }
        int p = 0;
#pragma unroll
        for (int ri = 0; ri < NRB; ++ri) {
#pragma unroll
          for (int rj = ri; rj < NRB; ++rj, ++p) {
            acc_ll[p] = mma_i8(Lv[ri], Lv[rj], acc_ll[p]);
            acc_x[p] = mma_i8(Hv[ri], Lv[rj], acc_x[p]);
            acc_x[p] = mma_i8(Lv[ri], Hv[rj], acc_x[p]);
            acc_hh[p] = mma_i8(Hv[ri], Hv[rj], acc_hh[p]);
          }
        }
      }
    };
    if (full) ksteps(std::true_type{});
    else ksteps(std::false_type{});
    if (++tiles == kFoldTiles) {
      fold_i8();
      tiles = 0;
    }
  });
  fold_i8();
  __syncthreads();

  // origin 32896 -> shift c: G' = M G M^T with M = [[I, -d], [0, 1]]
  auto at = [&](int I, int J) {   // packed index of (I, J), I <= J
    const int bi = I >> 2, bj = J >> 2;
    return (bi * nb - bi * (bi - 1) / 2 + (bj - bi)) * 16 + (I & 3) * 4 + (J & 3);
  };
  double* out = part + (int64_t)blockIdx.x * packed_doubles(B);
  const double n = red[at(B, B)];
  for (int t = threadIdx.x; t < L; t += kBlock) {
    int tix = t >> 4, bi = 0;
    while (tix >= nb - bi) {
      tix -= nb - bi;
      ++bi;
    }
    const int I = 4 * bi + ((t >> 2) & 3), J = 4 * (bi + tix) + (t & 3);
    double v = red[t];
    if (I < D && J < D) {
      const double di = I < B ? (double)cs[I] - 32896.0 : 0.0;
      const double dj = J < B ? (double)cs[J] - 32896.0 : 0.0;
      const double si = red[at(I, B)], sj = red[at(J, B)];
      v = v - di * sj - si * dj + di * dj * n;
    }
    out[t] = v;
  }
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
  const size_t sm = tile_area_bytes(B);
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

int pca_u16_blocks_per_cu(int B) {
  switch (nrb_for(B)) {
    case 2: return pca_u16_waves<2>();
    case 3: return pca_u16_waves<3>();
    default: return pca_u16_waves<5>();
  }
}

hipError_t launch_pca_gram_mfma(int dtype, int split, const void* cube, int B, int64_t P, const uint8_t* mask,
                                int nblocks, double* part, double* shift_out, hipStream_t s) {
  if (B < 1 || B > kMaxB || nblocks < 1) return hipErrorInvalidValue;
  if (split == 0) return pca_launch<0>(dtype, cube, B, P, mask, nblocks, part, shift_out, s);
  return pca_launch<1>(dtype, cube, B, P, mask, nblocks, part, shift_out, s);
}

}  // namespace cvx

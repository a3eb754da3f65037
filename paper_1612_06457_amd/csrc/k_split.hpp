// Compensated mixed-precision Gram accumulation on the gfx950 matrix cores,
// shared by the class-moment and page-covariance kernels.
//
// Same quantities as the FP32 path (per-class augmented Gram of
// [x - c_k, 1] over the training pixels, and the whole-page augmented Gram
// of [x - s, 1] for PCA), but the products run on MFMA: every value
// v = (x - c) * 2^e is split into a 16-bit head and tail, v = hi + lo with
// hi = round(v) and lo = round(v - hi) in bf16 (or fp16), and each
// 16 x 16 tile of the Gram accumulates hi hi^T + hi lo^T + lo hi^T + lo lo^T
// with v_mfma_f32_16x16x32_{bf16,f16} (32 pixels per instruction, FP32
// accumulation).  For 12-bit integer pages shifted by an integer, and for
// bf16/fp16 pages shifted by a value of the same type, the split is exact
// and so is every product: only the FP32 accumulation rounds.  Each wave
// folds its FP32 tiles into FP64 registers after every tile of at most 128
// pixels; the waves of a block then combine in a fixed order, and block
// partials use the same packed layout (upper-triangular 4 x 4 tiles of the
// padded (B+1) x (B+1) matrix) as the FP32 path, combined by the same
// fixed-order FP64 reduction.
//
// Operand layout of v_mfma_f32_16x16x32 (checked on the device): lane l
// holds A[l % 16][8 (l / 16) + t] and B[8 (l / 16) + t][l % 16] for
// t = 0..7, and C[4 (l / 16) + e][l % 16] for e = 0..3.  With A = X_ri^T
// and B = X_rj (X = pixels x bands, ri/rj 16-band row blocks) both operands
// are "pixel 8 (l / 16) + t, band 16 r + l % 16", so one pair of registers
// per row block feeds every tile of the Gram.
#pragma once
#include "k_common.hpp"

namespace cvx {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int SPLIT> struct SplitT;
template <> struct SplitT<0> {
  using V = bf16x8;
  using S = __bf16;
  static __device__ __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct SplitT<1> {
  using V = f16x8;
  using S = _Float16;
  static __device__ __forceinline__ f32x4 mma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Round a shift to the page's element type, so that x - c stays exact.
template <int DT>
__device__ __forceinline__ float round_shift(float c) {
  if constexpr (DT == DT_U16) {
    return rintf(c);
  } else if constexpr (DT == DT_BF16) {
    return (float)(__bf16)c;
  } else if constexpr (DT == DT_F16) {
    return (float)(_Float16)c;
  } else {
    return c;
  }
}

constexpr int npairs(int nrb) { return nrb * (nrb + 1) / 2; }

// Accumulate the 32-pixel K-step starting at pixel row k0.  get(r, band)
// returns the (shifted, prescaled) value of row r, band `band` < B, 1 for
// band == B and 0 beyond, or 0 for every band of a row that holds no pixel.
template <int SPLIT, int NRB, typename Get>
__device__ __forceinline__ void kstep(Get get, int k0, f32x4 (&acc)[npairs(NRB)]) {
  using ST = SplitT<SPLIT>;
  using V = typename ST::V;
  using S = typename ST::S;
  const int lane = __lane_id();
  const int col = lane & 15, grp = lane >> 4;
  V hi[NRB], lo[NRB];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int r = k0 + 8 * grp + t;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const float v = get(r, 16 * rb + col);
      const S h = (S)v;
      hi[rb][t] = h;
      lo[rb][t] = (S)(v - (float)h);
    }
  }
  int p = 0;
#pragma unroll
  for (int ri = 0; ri < NRB; ++ri) {
#pragma unroll
    for (int rj = ri; rj < NRB; ++rj, ++p) {
      acc[p] = ST::mma(hi[ri], hi[rj], acc[p]);
      acc[p] = ST::mma(hi[ri], lo[rj], acc[p]);
      acc[p] = ST::mma(lo[ri], hi[rj], acc[p]);
      acc[p] = ST::mma(lo[ri], lo[rj], acc[p]);
    }
  }
}

template <int NRB>
__device__ __forceinline__ void fold(f32x4 (&acc)[npairs(NRB)], double (&accd)[npairs(NRB)][4]) {
#pragma unroll
  for (int p = 0; p < npairs(NRB); ++p) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      accd[p][e] += (double)acc[p][e];
      acc[p][e] = 0.f;
    }
  }
}

// Add this wave's FP64 tiles, unscaled, into the block's packed partial red
// (waves in a fixed order), then write it out.  The packed layout holds the
// 4 x 4 tiles (bi <= bj) of the padded Gram, each tile complete.
template <int NRB>
__device__ __forceinline__ void block_combine(const double (&accd)[npairs(NRB)][4], int B, float scale,
                                              double* __restrict__ red, double* __restrict__ out) {
  const int BP = (B + 1 + 3) & ~3, nb = BP / 4, L = nb * (nb + 1) / 2 * 16;
  const int D = B + 1;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const double inv = 1.0 / (double)scale;
  for (int t = threadIdx.x; t < L; t += kBlock) red[t] = 0.0;
  __syncthreads();
  for (int ww = 0; ww < kWaves; ++ww) {
    if (w == ww) {
      int p = 0;
#pragma unroll
      for (int ri = 0; ri < NRB; ++ri) {
#pragma unroll
        for (int rj = ri; rj < NRB; ++rj, ++p) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int I = 16 * ri + 4 * (lane >> 4) + e, J = 16 * rj + (lane & 15);
            // a diagonal 4 x 4 tile keeps both triangles, like the FP32 path
            if ((I >> 2) <= (J >> 2) && I < D && J < D) {
              const int bi = I >> 2, bj = J >> 2;
              const int tix = bi * nb - bi * (bi - 1) / 2 + (bj - bi);
              double v = accd[p][e];
              if (I < B) v *= inv;
              if (J < B) v *= inv;
              red[tix * 16 + (I & 3) * 4 + (J & 3)] += v;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < L; t += kBlock) out[t] = red[t];
}

// Exact fp16 operands of uint16 values x about an integer shift
// c = 1024 c_h + c_l, two pixels per dword: with x = 1024 h + l,
// (x - c) / 1024 = (h - c_h) + (l - c_l) / 1024, where the fp16 with bits
// 0x6400 | h is 1024 + h and the one with bits 0x3c00 | l is 1 + l / 1024,
// so an AND-OR and one packed fp16 add give each term exactly.  Every
// product of two terms is exact in FP32 (at most 22 significant bits).  The
// bit masks sit in registers: VOP3 encodings on gfx9 take no literal.
struct U16Masks {
  uint32_t lo, hi, exp_l, exp_h;   // 0x03ff03ff, 0x003f003f, 0x3c003c00, 0x64006400
};
__device__ __forceinline__ U16Masks make_u16_masks() {
  U16Masks m{0x03ff03ffu, 0x003f003fu, 0x3c003c00u, 0x64006400u};
  asm volatile("" : "+v"(m.lo), "+v"(m.hi), "+v"(m.exp_l), "+v"(m.exp_h));
  return m;
}

__device__ __forceinline__ uint32_t pk_add_f16(uint32_t a, uint32_t b) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(h2, a) + __builtin_bit_cast(h2, b));
}

// Per lane and 16-band row block: the lane's band (16 rb + col), the column
// it loads (clamped to a real band), the negated shift terms, and the masks
// that keep real bands and put 1 in the ones column (band B).
template <int NRB>
struct U16Lane {
  int bcol[NRB];
  uint32_t nh[NRB], nl[NRB], keep[NRB], ones[NRB];
  __device__ __forceinline__ void init(int B, const float* __restrict__ cs, int col) {
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const int band = 16 * rb + col;
      bcol[rb] = band < B ? band : B - 1;
      const uint32_t c = band < B ? (uint32_t)cs[band] : 0u;
      const uint32_t h = __builtin_bit_cast(uint16_t, (_Float16)(-(1024.f + (float)(c >> 10))));
      const uint32_t l = __builtin_bit_cast(uint16_t, (_Float16)(-(1.f + (float)(c & 1023u) / 1024.f)));
      nh[rb] = h | (h << 16);
      nl[rb] = l | (l << 16);
      keep[rb] = band < B ? 0xffffffffu : 0u;
      ones[rb] = band == B ? 0x3c003c00u : 0u;
    }
  }
  // The H and L terms of the dword d (two pixels of this lane's band);
  // rowmask zeroes the halves of pixels that are not there.
  __device__ __forceinline__ void terms(uint32_t d, int rb, uint32_t rowmask, const U16Masks& mk, uint32_t& H,
                                        uint32_t& L) const {
    const uint32_t m = keep[rb] & rowmask, on = ones[rb] & rowmask;
    H = pk_add_f16(((d >> 10) & mk.hi) | mk.exp_h, nh[rb]) & m;
    L = (pk_add_f16((d & mk.lo) | mk.exp_l, nl[rb]) & m) | on;
  }
};

// Accumulate the 16 x 16 tile pairs of the Gram of v = H + L (per row block
// rb: Hv[rb], Lv[rb] in the k_split layout) on the fp16 matrix units.
template <int NRB>
__device__ __forceinline__ void u16_tile_products(const f16x8 (&Hv)[NRB], const f16x8 (&Lv)[NRB],
                                                  f32x4 (&acc)[npairs(NRB)]) {
  int p = 0;
#pragma unroll
  for (int ri = 0; ri < NRB; ++ri) {
#pragma unroll
    for (int rj = ri; rj < NRB; ++rj, ++p) {
      acc[p] = SplitT<1>::mma(Lv[ri], Lv[rj], acc[p]);   // smallest terms first
      acc[p] = SplitT<1>::mma(Hv[ri], Lv[rj], acc[p]);
      acc[p] = SplitT<1>::mma(Lv[ri], Hv[rj], acc[p]);
      acc[p] = SplitT<1>::mma(Hv[ri], Hv[rj], acc[p]);
    }
  }
}

// power-of-two prescale keeping split values inside the fp16 range with
// room for the tail (bf16 has the range of fp32; the scale is exact either way)
inline float prescale(int dtype, int split) {
  if (split == 0) return 1.f;
  if (dtype == DT_U16) return 1.f / 16.f;
  if (dtype == DT_BF16 || dtype == DT_F16) return 64.f;
  return 1.f;
}

// 16-band row blocks covering the B + 1 columns of the augmented Gram
inline int nrb_for(int B) {
  const int D = B + 1;
  if (D <= 32) return 2;
  if (D <= 48) return 3;
  return 5;
}

__host__ __device__ inline size_t packed_doubles(int B) {
  const int nb = (B + 4) / 4;
  return (size_t)nb * (nb + 1) / 2 * 16;
}

}  // namespace cvx

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

// Compensated mixed-precision scatter on the gfx950 matrix cores.
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
#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

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

template <int DT>
__device__ __forceinline__ float lds_elem(const void* tile, int e) {
  if constexpr (DT == DT_F32) {
    return reinterpret_cast<const float*>(tile)[e];
  } else {
    return to_float<DT>(reinterpret_cast<const uint16_t*>(tile)[e]);
  }
}

constexpr int npairs(int nrb) { return nrb * (nrb + 1) / 2; }

// Accumulate the 32-pixel K-step starting at pixel row k0 of an LDS tile
// (rows of B elements).  valid(r) tells whether row r holds a real pixel.
template <int DT, int SPLIT, int NRB, typename Valid>
__device__ __forceinline__ void kstep(const void* tile, int k0, int B, const float* __restrict__ cs,
                                      float scale, Valid valid, f32x4 (&acc)[npairs(NRB)]) {
  using ST = SplitT<SPLIT>;
  using V = typename ST::V;
  using S = typename ST::S;
  const int lane = __lane_id();
  const int col = lane & 15, grp = lane >> 4;
  V hi[NRB], lo[NRB];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int r = k0 + 8 * grp + t;
    const bool ok = valid(r);
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const int band = 16 * rb + col;
      float v = 0.f;
      if (ok) {
        if (band < B) v = (lds_elem<DT>(tile, r * B + band) - cs[band]) * scale;
        else if (band == B) v = 1.f;
      }
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

template <int DT>
__device__ __forceinline__ int tile_geometry(int B, int& S) {
  if (DT == DT_F32) {
    S = B;
    return 1;
  }
  if (B & 1) {
    S = B;
    return 2;
  }
  S = B / 2;
  return 1;
}

// Fetch wave tile t (64 lane groups) of the page into this wave's LDS slice.
__device__ __forceinline__ void fetch(const unsigned char* __restrict__ base, int64_t total_bytes,
                                      int64_t t, int S, uint32_t* __restrict__ my, int lane) {
  const int64_t tb = t * 256 * (int64_t)S;
  for (int j = lane; j < 16 * S; j += 64) {
    const int64_t ob = tb + 16 * (int64_t)j;
    uint4 v;
    if (ob + 16 <= total_bytes) {
      v = *reinterpret_cast<const uint4*>(base + ob);
    } else {
      uint16_t h[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        h[q] = (ob + 2 * q + 2 <= total_bytes) ? *reinterpret_cast<const uint16_t*>(base + ob + 2 * q) : 0;
      v.x = h[0] | ((uint32_t)h[1] << 16);
      v.y = h[2] | ((uint32_t)h[3] << 16);
      v.z = h[4] | ((uint32_t)h[5] << 16);
      v.w = h[6] | ((uint32_t)h[7] << 16);
    }
    *reinterpret_cast<uint4*>(my + 4 * j) = v;
  }
}

template <int DT, int SPLIT, int NRB>
__global__ __launch_bounds__(kBlock) void k_pca_gram_mfma(const void* __restrict__ cube, int B, int64_t P,
                                                          const uint8_t* __restrict__ mask, float scale,
                                                          double* __restrict__ part,
                                                          double* __restrict__ shift_out) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float cs[kMaxB];
  __shared__ float psum[kWaves][kMaxB];
  int S;
  const int g2 = tile_geometry<DT>(B, S);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* my = lds + w * 64 * S;
  double* red = reinterpret_cast<double*>(lds + kWaves * 64 * S);
  using T = typename Elem<DT>::T;
  const T* cx = reinterpret_cast<const T*>(cube);

  // shift: mean of 64 pixels spread evenly over the page, fixed order
  for (int b = lane; b < B; b += 64) {
    float s = 0.f;
    for (int i = w * 16; i < w * 16 + 16; ++i) s += to_float<DT>(cx[((int64_t)i * P / 64) * B + b]);
    psum[w][b] = s;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += kBlock) {
    const float c = round_shift<DT>((((psum[0][b] + psum[1][b]) + psum[2][b]) + psum[3][b]) / 64.f);
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
  const int64_t total_bytes = P * B * (int64_t)(DT == DT_F32 ? 4 : 2);
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  for (int64_t t = (int64_t)blockIdx.x * kWaves + w; t < nt; t += (int64_t)gridDim.x * kWaves) {
    fetch(base, total_bytes, t, S, my, lane);
    wave_lds_sync();
    const int64_t pix0 = t * tp;
    auto valid = [&](int r) {
      const int64_t p = pix0 + r;
      return p < P && (mask == nullptr || mask[p] != 0);
    };
    for (int k0 = 0; k0 < tp; k0 += 32) kstep<DT, SPLIT, NRB>(my, k0, B, cs, scale, valid, acc);
    fold<NRB>(acc, accd);
    wave_lds_sync();
  }
  block_combine<NRB>(accd, B, scale, red, part + (int64_t)blockIdx.x * (((B + 4) / 4) * ((B + 4) / 4 + 1) / 2 * 16));
}

template <int DT, int SPLIT, int NRB>
__global__ __launch_bounds__(kBlock) void k_class_moments_mfma(const void* __restrict__ cube, int B,
                                                               const int32_t* __restrict__ idx,
                                                               const int32_t* __restrict__ offsets, int G,
                                                               float scale, double* __restrict__ part,
                                                               double* __restrict__ shift_out) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float cs[kMaxB];
  __shared__ float psum[kWaves][kMaxB];
  constexpr int esz = (DT == DT_F32) ? 4 : 2;
  const int rowdw = (kChunk * B * esz + 3) / 4;          // dwords per wave tile of kChunk rows
  const int k = blockIdx.y, g = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* my = lds + w * rowdw;
  double* red = reinterpret_cast<double*>(lds + kWaves * rowdw + (kWaves * rowdw & 1));
  using T = typename Elem<DT>::T;
  const T* cx = reinterpret_cast<const T*>(cube);
  const int off = offsets[k];
  const int n = offsets[k + 1] - off;

  const int ns = n < 64 ? n : 64;
  for (int b = lane; b < B; b += 64) {
    float s = 0.f;
    const int i1 = (w * 16 + 16 < ns) ? w * 16 + 16 : ns;
    for (int i = w * 16; i < i1; ++i) s += to_float<DT>(cx[(int64_t)idx[off + i] * B + b]);
    psum[w][b] = s;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += kBlock) {
    const float s = ((psum[0][b] + psum[1][b]) + psum[2][b]) + psum[3][b];
    const float c = round_shift<DT>(ns > 0 ? s / (float)ns : 0.f);
    cs[b] = c;
    if (g == 0) shift_out[(int64_t)k * B + b] = (double)c;
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
  T* rows = reinterpret_cast<T*>(my);
  const int rpi = (64 / B) > 0 ? 64 / B : 1;              // rows gathered per wave instruction
  const int nch = (n + kChunk - 1) / kChunk;
  for (int ch = g * kWaves + w; ch < nch; ch += G * kWaves) {
    const int r0 = ch * kChunk;
    const int rows_here = (n - r0 < kChunk) ? n - r0 : kChunk;
    // gather rows: lane -> (row offset lane / B, band lane % B)
    const int lr = lane / B, lb = lane % B;
    int myp = -1;                                         // lane r: pixel of row r (and r + 64)
    int myp2 = -1;
    if (lane < rows_here) myp = idx[off + r0 + lane];
    if (lane + 64 < rows_here) myp2 = idx[off + r0 + lane + 64];
#pragma unroll 8
    for (int rr = 0; rr < kChunk; rr += rpi) {
      const int r = rr + lr;
      const int p1 = __shfl(myp, r & 63, 64);
      const int p2 = __shfl(myp2, r & 63, 64);
      const int p = (r < 64) ? p1 : p2;
      if (lr < rpi && r < kChunk) {
        for (int b = lb; b < B; b += 64) {
          T v = (T)0;
          if (r < rows_here) v = cx[(int64_t)p * B + b];
          rows[r * B + b] = v;
        }
      }
    }
    wave_lds_sync();
    auto valid = [&](int r) { return r < rows_here; };
    for (int k0 = 0; k0 < kChunk; k0 += 32) kstep<DT, SPLIT, NRB>(my, k0, B, cs, scale, valid, acc);
    fold<NRB>(acc, accd);
    wave_lds_sync();
  }
  const int nb = (B + 4) / 4;
  block_combine<NRB>(accd, B, scale, red, part + ((int64_t)k * G + g) * (nb * (nb + 1) / 2 * 16));
}

// power-of-two prescale keeping split values inside the fp16 range with
// room for the tail (bf16 has the range of fp32; the scale is exact either way)
float prescale(int dtype, int split) {
  if (split == 0) return 1.f;
  if (dtype == DT_U16) return 1.f / 16.f;
  if (dtype == DT_BF16 || dtype == DT_F16) return 64.f;
  return 1.f;
}

int nrb_for(int B) {
  const int D = B + 1;
  if (D <= 32) return 2;
  if (D <= 48) return 3;
  return 5;
}

size_t packed_doubles(int B) {
  const int nb = (B + 4) / 4;
  return (size_t)nb * (nb + 1) / 2 * 16;
}

template <int DT, int SPLIT>
hipError_t pca_launch_dt(int nrb, const void* cube, int B, int64_t P, const uint8_t* mask, int nblocks,
                         double* part, double* shift_out, size_t sm, float sc, hipStream_t s) {
  switch (nrb) {
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

template <int DT, int SPLIT>
hipError_t class_launch_dt(int nrb, const void* cube, int B, const int32_t* idx, const int32_t* offsets, int K,
                           int G, double* part, double* shift_out, size_t sm, float sc, hipStream_t s) {
  const dim3 grid(G, K);
  switch (nrb) {
    case 2:
      hipLaunchKernelGGL((k_class_moments_mfma<DT, SPLIT, 2>), grid, dim3(kBlock), sm, s, cube, B, idx, offsets, G,
                         sc, part, shift_out);
      break;
    case 3:
      hipLaunchKernelGGL((k_class_moments_mfma<DT, SPLIT, 3>), grid, dim3(kBlock), sm, s, cube, B, idx, offsets, G,
                         sc, part, shift_out);
      break;
    default:
      hipLaunchKernelGGL((k_class_moments_mfma<DT, SPLIT, 5>), grid, dim3(kBlock), sm, s, cube, B, idx, offsets, G,
                         sc, part, shift_out);
      break;
  }
  return hipGetLastError();
}

template <int SPLIT>
hipError_t pca_launch(int dtype, const void* cube, int B, int64_t P, const uint8_t* mask, int nblocks,
                      double* part, double* shift_out, hipStream_t s) {
  const int nrb = nrb_for(B);
  int S = (dtype == DT_F32) ? B : ((B & 1) ? B : B / 2);
  const size_t sm = (size_t)kWaves * 64 * S * 4 + packed_doubles(B) * 8;
  const float sc = prescale(dtype, SPLIT);
  switch (dtype) {
    case DT_U16: return pca_launch_dt<DT_U16, SPLIT>(nrb, cube, B, P, mask, nblocks, part, shift_out, sm, sc, s);
    case DT_F32: return pca_launch_dt<DT_F32, SPLIT>(nrb, cube, B, P, mask, nblocks, part, shift_out, sm, sc, s);
    case DT_BF16: return pca_launch_dt<DT_BF16, SPLIT>(nrb, cube, B, P, mask, nblocks, part, shift_out, sm, sc, s);
    case DT_F16: return pca_launch_dt<DT_F16, SPLIT>(nrb, cube, B, P, mask, nblocks, part, shift_out, sm, sc, s);
  }
  return hipErrorInvalidValue;
}

template <int SPLIT>
hipError_t class_launch(int dtype, const void* cube, int B, const int32_t* idx, const int32_t* offsets, int K,
                        int G, double* part, double* shift_out, hipStream_t s) {
  const int nrb = nrb_for(B);
  const int esz = dtype == DT_F32 ? 4 : 2;
  const int rowdw = (kChunk * B * esz + 3) / 4;
  const size_t sm = ((size_t)kWaves * rowdw + 1) * 4 + packed_doubles(B) * 8;
  const float sc = prescale(dtype, SPLIT);
  switch (dtype) {
    case DT_U16: return class_launch_dt<DT_U16, SPLIT>(nrb, cube, B, idx, offsets, K, G, part, shift_out, sm, sc, s);
    case DT_F32: return class_launch_dt<DT_F32, SPLIT>(nrb, cube, B, idx, offsets, K, G, part, shift_out, sm, sc, s);
    case DT_BF16: return class_launch_dt<DT_BF16, SPLIT>(nrb, cube, B, idx, offsets, K, G, part, shift_out, sm, sc, s);
    case DT_F16: return class_launch_dt<DT_F16, SPLIT>(nrb, cube, B, idx, offsets, K, G, part, shift_out, sm, sc, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_pca_gram_mfma(int dtype, int split, const void* cube, int B, int64_t P, const uint8_t* mask,
                                int nblocks, double* part, double* shift_out, hipStream_t s) {
  if (split == 0) return pca_launch<0>(dtype, cube, B, P, mask, nblocks, part, shift_out, s);
  return pca_launch<1>(dtype, cube, B, P, mask, nblocks, part, shift_out, s);
}

hipError_t launch_class_moments_mfma(int dtype, int split, const void* cube, int B, const int32_t* idx,
                                     const int32_t* offsets, int K, int G, double* part, double* shift_out,
                                     hipStream_t s) {
  if (split == 0) return class_launch<0>(dtype, cube, B, idx, offsets, K, G, part, shift_out, s);
  return class_launch<1>(dtype, cube, B, idx, offsets, K, G, part, shift_out, s);
}

}  // namespace cvx

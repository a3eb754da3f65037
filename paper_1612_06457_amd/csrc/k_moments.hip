// FP32 scatter accumulation (plain path): per-class augmented Gram
// matrices of [x - c_k, 1] over the training pixels, the whole-page Gram of
// [x - s, 1] for PCA, and the fixed-order FP64 combine of block partials.
//
// Paper Section 2: the within- and between-class covariance of the training
// points (CVA) and the covariance of the page (PCA).  The augmented Gram
// about a shift c gives n, sum (x - c) and sum (x - c)(x - c)^T in one
// product; the host turns those into the centred scatter exactly
// (sum (x - m)(x - m)^T = sum (x - c)(x - c)^T - n (m - c)(m - c)^T).  The
// shift is the mean of a few sample pixels (rounded to an integer for
// uint16 pages, so x - c stays exact), which keeps the FP32 sums short of
// cancellation.  Each thread accumulates a 4x4 tile in FP32 over one chunk
// of at most 128 rows and adds it into FP64 registers; block partials are
// combined in a fixed order, so results are bitwise repeatable.
#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

// Shared tail: accumulate the chunk xs (kChunk x BP, LDS) into acc / accd.
struct TileAssign {
  int bi, bj, slice, nslice, blk, nblk;
  bool active;
};

__device__ __forceinline__ TileAssign assign_tiles(int BP) {
  TileAssign t;
  const int nb = BP / 4;
  t.nblk = nb * (nb + 1) / 2;
  t.nslice = kBlock / t.nblk;
  t.blk = threadIdx.x % t.nblk;
  t.slice = threadIdx.x / t.nblk;
  t.bi = t.bj = 0;
  t.active = (t.slice < t.nslice) && tri_tile(t.blk, nb, t.bi, t.bj);
  return t;
}

// Combine the FP64 per-thread tiles across slices in a fixed order and
// write one block partial (nblk * 16 doubles).
__device__ __forceinline__ void write_partial(const TileAssign& ta, const double accd[16],
                                              double* __restrict__ red, double* __restrict__ out) {
  __syncthreads();
  if (ta.active)
    for (int e = 0; e < 16; ++e) red[(ta.slice * ta.nblk + ta.blk) * 16 + e] = accd[e];
  __syncthreads();
  for (int t = threadIdx.x; t < ta.nblk * 16; t += kBlock) {
    double s = 0.0;
    for (int sl = 0; sl < ta.nslice; ++sl) s += red[sl * ta.nblk * 16 + t];
    out[t] = s;
  }
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_class_moments(const typename Elem<DT>::T* __restrict__ cube,
                                                          int B, const int32_t* __restrict__ idx,
                                                          const int32_t* __restrict__ offsets, int G,
                                                          double* __restrict__ part,
                                                          double* __restrict__ shift_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* red = reinterpret_cast<double*>(smem_raw);
  __shared__ float cs[kMaxB];
  __shared__ float psum[kWaves][kMaxB];
  const int k = blockIdx.y, g = blockIdx.x;
  const int BP = (B + 1 + 3) & ~3;
  const int off = offsets[k];
  const int n = offsets[k + 1] - off;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;

  // shift: mean of the class's first min(64, n) pixels, fixed order
  const int ns = n < 64 ? n : 64;
  for (int b = lane; b < B; b += 64) {
    float s = 0.f;
    const int i1 = (w * 16 + 16 < ns) ? w * 16 + 16 : ns;
    for (int i = w * 16; i < i1; ++i) s += to_float<DT>(cube[(int64_t)idx[off + i] * B + b]);
    psum[w][b] = s;
  }
  __syncthreads();
  for (int b = tid; b < B; b += kBlock) {
    const float s = ((psum[0][b] + psum[1][b]) + psum[2][b]) + psum[3][b];
    float c = ns > 0 ? s / (float)ns : 0.f;
    if (DT == DT_U16) c = rintf(c);
    cs[b] = c;
    if (g == 0) shift_out[(int64_t)k * B + b] = (double)c;
  }
  __syncthreads();

  const TileAssign ta = assign_tiles(BP);
  float acc[16];
  double accd[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acc[e] = 0.f;
    accd[e] = 0.0;
  }
  const int nch = (n + kChunk - 1) / kChunk;
  for (int ch = g; ch < nch; ch += G) {
    const int rbase = ch * kChunk;
    int myp = -1;
    {
      const int pos = rbase + w * 32 + (lane & 31);
      if (lane < 32 && pos < n) myp = idx[off + pos];
    }
#pragma unroll 16
    for (int rr = 0; rr < 32; ++rr) {
      const int r = w * 32 + rr;
      const int p = __shfl(myp, rr, 64);
      for (int e = lane; e < BP; e += 64) {
        float v = 0.f;
        if (p >= 0) {
          if (e < B) v = to_float<DT>(cube[(int64_t)p * B + e]) - cs[e];
          else if (e == B) v = 1.f;
        }
        xs[r * BP + e] = v;
      }
    }
    __syncthreads();
    if (ta.active) tile_acc(xs, BP, xs, BP, ta.bi, ta.bj, ta.slice, kChunk, ta.nslice, acc);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      accd[e] += (double)acc[e];
      acc[e] = 0.f;
    }
  }
  write_partial(ta, accd, red, part + ((int64_t)k * G + g) * ta.nblk * 16);
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_pca_gram(const typename Elem<DT>::T* __restrict__ cube,
                                                     int B, int64_t P,
                                                     const uint8_t* __restrict__ mask,
                                                     double* __restrict__ part,
                                                     double* __restrict__ shift_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* xs = reinterpret_cast<float*>(smem_raw);
  double* red = reinterpret_cast<double*>(smem_raw);
  __shared__ float cs[kMaxB];
  __shared__ float psum[kWaves][kMaxB];
  const int BP = (B + 1 + 3) & ~3;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;

  // shift: mean of 64 pixels spread evenly over the page, fixed order
  for (int b = lane; b < B; b += 64) {
    float s = 0.f;
    for (int i = w * 16; i < w * 16 + 16; ++i) {
      const int64_t p = (int64_t)i * P / 64;
      s += to_float<DT>(cube[p * B + b]);
    }
    psum[w][b] = s;
  }
  __syncthreads();
  for (int b = tid; b < B; b += kBlock) {
    const float s = ((psum[0][b] + psum[1][b]) + psum[2][b]) + psum[3][b];
    float c = s / 64.f;
    if (DT == DT_U16) c = rintf(c);
    cs[b] = c;
    if (blockIdx.x == 0) shift_out[b] = (double)c;
  }
  __syncthreads();

  const TileAssign ta = assign_tiles(BP);
  float acc[16];
  double accd[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acc[e] = 0.f;
    accd[e] = 0.0;
  }
  const int64_t nch = (P + kChunk - 1) / kChunk;
  const int per = kChunk * B;                 // elements per chunk
  const int rstep = kBlock / B, bstep = kBlock % B;
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    const int64_t p0 = ch * kChunk;
    const int rows = (P - p0 < kChunk) ? (int)(P - p0) : kChunk;
    const int nel = rows * B;
    const typename Elem<DT>::T* src = cube + p0 * B;
    int r = tid / B, b = tid % B;
#pragma unroll 4
    for (int e = tid; e < per; e += kBlock) {
      float v = 0.f;
      if (e < nel && (mask == nullptr || mask[p0 + r])) v = to_float<DT>(src[e]) - cs[b];
      xs[r * BP + b] = v;
      r += rstep;
      b += bstep;
      if (b >= B) {
        b -= B;
        ++r;
      }
    }
    if (tid < kChunk) {
      const bool ok = tid < rows && (mask == nullptr || mask[p0 + tid]);
      xs[tid * BP + B] = ok ? 1.f : 0.f;
      for (int e = B + 1; e < BP; ++e) xs[tid * BP + e] = 0.f;
    }
    __syncthreads();
    if (ta.active) tile_acc(xs, BP, xs, BP, ta.bi, ta.bj, ta.slice, kChunk, ta.nslice, acc);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      accd[e] += (double)acc[e];
      acc[e] = 0.f;
    }
  }
  write_partial(ta, accd, red, part + (int64_t)blockIdx.x * ta.nblk * 16);
}

// 16 entries x 16 slices of g per block: slice j sums g = j, j + 16, ...
// (four independent chains in flight), then the 16 slice sums are added
// in slice order.  Fixed order throughout.
__global__ __launch_bounds__(kBlock) void k_reduce_part(const double* __restrict__ part, int nsets,
                                                        int G, int L, double* __restrict__ out) {
  __shared__ double red[16][17];
  const int s = blockIdx.y;
  const int tl = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int t = blockIdx.x * 16 + tl;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (t < L) {
    const double* src = part + (int64_t)s * G * L + t;
    int g = sl;
    for (; g + 48 < G; g += 64) {
      a0 += src[(int64_t)g * L];
      a1 += src[(int64_t)(g + 16) * L];
      a2 += src[(int64_t)(g + 32) * L];
      a3 += src[(int64_t)(g + 48) * L];
    }
    for (; g < G; g += 16) a0 += src[(int64_t)g * L];
  }
  red[sl][tl] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (threadIdx.x < 16 && t < L) {
    double acc = 0.0;
    for (int j = 0; j < 16; ++j) acc += red[j][tl];
    out[(int64_t)s * L + t] = acc;
  }
}

size_t scatter_smem(int B) {
  const int BP = (B + 1 + 3) & ~3;
  const int nb = BP / 4, nblk = nb * (nb + 1) / 2;
  const size_t a = (size_t)kChunk * BP * sizeof(float);
  const size_t b = (size_t)(kBlock / nblk) * nblk * 16 * sizeof(double);
  return a > b ? a : b;
}

}  // namespace

hipError_t launch_class_moments(int dtype, const void* cube, int B, const int32_t* idx,
                                const int32_t* offsets, int K, int G, double* part,
                                double* shift_out, hipStream_t s) {
  const dim3 grid(G, K);
  const size_t sm = scatter_smem(B);
  switch (dtype) {
    case DT_U16:
      hipLaunchKernelGGL(k_class_moments<DT_U16>, grid, dim3(kBlock), sm, s,
                         (const uint16_t*)cube, B, idx, offsets, G, part, shift_out);
      break;
    case DT_F32:
      hipLaunchKernelGGL(k_class_moments<DT_F32>, grid, dim3(kBlock), sm, s,
                         (const float*)cube, B, idx, offsets, G, part, shift_out);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(k_class_moments<DT_BF16>, grid, dim3(kBlock), sm, s,
                         (const uint16_t*)cube, B, idx, offsets, G, part, shift_out);
      break;
    case DT_F16:
      hipLaunchKernelGGL(k_class_moments<DT_F16>, grid, dim3(kBlock), sm, s,
                         (const uint16_t*)cube, B, idx, offsets, G, part, shift_out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pca_gram(int dtype, const void* cube, int B, int64_t P, const uint8_t* mask,
                           int nblocks, double* part, double* shift_out, hipStream_t s) {
  const size_t sm = scatter_smem(B);
  switch (dtype) {
    case DT_U16:
      hipLaunchKernelGGL(k_pca_gram<DT_U16>, dim3(nblocks), dim3(kBlock), sm, s,
                         (const uint16_t*)cube, B, P, mask, part, shift_out);
      break;
    case DT_F32:
      hipLaunchKernelGGL(k_pca_gram<DT_F32>, dim3(nblocks), dim3(kBlock), sm, s,
                         (const float*)cube, B, P, mask, part, shift_out);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(k_pca_gram<DT_BF16>, dim3(nblocks), dim3(kBlock), sm, s,
                         (const uint16_t*)cube, B, P, mask, part, shift_out);
      break;
    case DT_F16:
      hipLaunchKernelGGL(k_pca_gram<DT_F16>, dim3(nblocks), dim3(kBlock), sm, s,
                         (const uint16_t*)cube, B, P, mask, part, shift_out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_part(const double* part, int nsets, int G, int L, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((L + 15) / 16), nsets), dim3(kBlock), 0, s, part,
                     nsets, G, L, out);
  return hipGetLastError();
}

}  // namespace cvx

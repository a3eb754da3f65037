// FP32 scatter accumulation (plain path) for the whole-page Gram of
// [x - s, 1] (PCA), and the fixed-order FP64 combine of block partials
// (shared with the class moments of k_class.hip).
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
#include "k_gram.hpp"
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

// Block tiles of kChunk pixels (kChunk B elements: a multiple of 16 bytes)
// are streamed with the prefetching driver of k_tile.hpp; each is turned
// into the FP32 rows [x - s, 1] in LDS and accumulated by the block.
template <int DT, int Q>
__global__ __launch_bounds__(kBlock) void k_pca_gram(const typename Elem<DT>::T* __restrict__ cube,
                                                     int B, int64_t P,
                                                     const uint8_t* __restrict__ mask,
                                                     double* __restrict__ part,
                                                     double* __restrict__ shift_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int esz = DT == DT_F32 ? 4 : 2;
  const int BP = (B + 1 + 3) & ~3;
  const int tile_bytes = kChunk * B * esz;
  uint32_t* raw = reinterpret_cast<uint32_t*>(smem_raw);                       // the staged tile
  float* xs = reinterpret_cast<float*>(smem_raw + ((tile_bytes + 15) & ~15));  // kChunk x BP
  double* red = reinterpret_cast<double*>(smem_raw);
  __shared__ float cs[kMaxB];
  __shared__ uint8_t vrow[kChunk];
  const int tid = threadIdx.x;

  // shift: mean of 64 pixels spread evenly over the page, fixed order
  for (int b = tid; b < B; b += kBlock) {
    float x[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = to_float<DT>(cube[((int64_t)i * P / 64) * B + b]);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 64; ++i) s += x[i];
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
  const int rstep = kBlock / BP, bstep = kBlock % BP;
  const typename Elem<DT>::T* tile = reinterpret_cast<const typename Elem<DT>::T*>(raw);
  for_each_tile_n<Q, kBlock>(reinterpret_cast<const unsigned char*>(cube), P * B * (int64_t)esz, nch, tile_bytes,
                             raw, [&](int64_t ch) {
    const int64_t p0 = ch * kChunk;
    if (tid < kChunk) {
      const int64_t p = p0 + tid;
      vrow[tid] = (p < P && (mask == nullptr || mask[p] != 0)) ? 1 : 0;
    }
    __syncthreads();
    int r = tid / BP, b = tid % BP;
    for (int e = tid; e < kChunk * BP; e += kBlock) {
      float v = 0.f;
      if (vrow[r]) {
        if (b < B) v = to_float<DT>(tile[r * B + b]) - cs[b];
        else if (b == B) v = 1.f;
      }
      xs[e] = v;
      r += rstep;
      b += bstep;
      if (b >= BP) {
        b -= BP;
        ++r;
      }
    }
    __syncthreads();
    if (ta.active) tile_acc(xs, BP, xs, BP, ta.bi, ta.bj, ta.slice, kChunk, ta.nslice, acc);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      accd[e] += (double)acc[e];
      acc[e] = 0.f;
    }
  });
  write_partial(ta, accd, red, part + (int64_t)blockIdx.x * ta.nblk * 16);
}

// 16 entries x 16 slices of g per block: slice j sums g = j, j + 16, ...
// (four independent chains in flight), then the 16 slice sums are added
// in slice order.  Fixed order throughout.
//
// With hdr_bytes > 0, block (0, 0) also copies hdr_bytes (a multiple of 4)
// from hdr_src to hdr_dst: a fit's small results (counts, offsets, flags,
// shifts) then reach page-locked host memory in the same launch as its
// Gram, which the kernel writes there directly.
__global__ __launch_bounds__(kBlock) void k_reduce_part(const double* __restrict__ part, int nsets,
                                                        int G, int L, double* __restrict__ out,
                                                        const uint32_t* __restrict__ hdr_src,
                                                        uint32_t* __restrict__ hdr_dst, int64_t hdr_bytes) {
  __shared__ double red[16][17];
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int64_t i = threadIdx.x; i < hdr_bytes / 4; i += kBlock) hdr_dst[i] = hdr_src[i];
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

size_t pca_smem(int dtype, int B) {
  const int BP = (B + 1 + 3) & ~3;
  const int nb = BP / 4, nblk = nb * (nb + 1) / 2;
  const size_t tile = ((size_t)kChunk * B * (dtype == DT_F32 ? 4 : 2) + 15) & ~size_t(15);
  const size_t a = tile + (size_t)kChunk * BP * sizeof(float);
  const size_t b = (size_t)(kBlock / nblk) * nblk * 16 * sizeof(double);
  return a > b ? a : b;
}

// chunks per thread for a block tile: kChunk B esize / 16 / kBlock, rounded up to an instantiated bound
int pca_q(int dtype, int B) {
  const int chunks = kChunk * B * (dtype == DT_F32 ? 4 : 2) / 16;
  const int q = (chunks + kBlock - 1) / kBlock;
  return q <= 2 ? 2 : q <= 4 ? 4 : 8;
}

template <int DT>
hipError_t pca_dt(const void* cube, int B, int64_t P, const uint8_t* mask, int nblocks, double* part,
                  double* shift_out, hipStream_t s) {
  using T = typename Elem<DT>::T;
  const size_t sm = pca_smem(DT, B);
  switch (pca_q(DT, B)) {
    case 2:
      hipLaunchKernelGGL((k_pca_gram<DT, 2>), dim3(nblocks), dim3(kBlock), sm, s, (const T*)cube, B, P, mask, part,
                         shift_out);
      break;
    case 4:
      hipLaunchKernelGGL((k_pca_gram<DT, 4>), dim3(nblocks), dim3(kBlock), sm, s, (const T*)cube, B, P, mask, part,
                         shift_out);
      break;
    default:
      hipLaunchKernelGGL((k_pca_gram<DT, 8>), dim3(nblocks), dim3(kBlock), sm, s, (const T*)cube, B, P, mask, part,
                         shift_out);
      break;
  }
  return hipGetLastError();
}

}  // namespace


hipError_t launch_pca_gram(int dtype, const void* cube, int B, int64_t P, const uint8_t* mask,
                           int nblocks, double* part, double* shift_out, hipStream_t s) {
  if (B < 1 || B > kMaxB || nblocks < 1) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_U16: return pca_dt<DT_U16>(cube, B, P, mask, nblocks, part, shift_out, s);
    case DT_F32: return pca_dt<DT_F32>(cube, B, P, mask, nblocks, part, shift_out, s);
    case DT_BF16: return pca_dt<DT_BF16>(cube, B, P, mask, nblocks, part, shift_out, s);
    case DT_F16: return pca_dt<DT_F16>(cube, B, P, mask, nblocks, part, shift_out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_part(const double* part, int nsets, int G, int L, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((L + 15) / 16), nsets), dim3(kBlock), 0, s, part,
                     nsets, G, L, out, (const uint32_t*)nullptr, (uint32_t*)nullptr, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_reduce_part_out(const double* part, int nsets, int G, int L, double* out_host,
                                  const void* hdr_src, void* hdr_dst, int64_t hdr_bytes, hipStream_t s) {
  if (hdr_bytes % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_part, dim3((unsigned)((L + 15) / 16), nsets), dim3(kBlock), 0, s, part,
                     nsets, G, L, out_host, (const uint32_t*)hdr_src, (uint32_t*)hdr_dst, hdr_bytes);
  return hipGetLastError();
}

}  // namespace cvx

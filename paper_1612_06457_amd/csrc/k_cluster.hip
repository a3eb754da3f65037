// Cluster-separation indices of labelled points on a set of images (paper
// Section 3, Eqs. 1-5): for each class k the centroid A_k of the points'
// feature vectors (the values of n images at the point's pixel, Eq. 1's
// A_i) and the scatter S_k = mean over the class's points of ||X - A_k||_p
// (Eq. 1).  The host forms M_ij = ||A_i - A_j||_p (Eq. 2) and the indices
// of Eqs. 3 and 5 from these few numbers.
//
// The points arrive class-grouped from the label kernels (an index list and
// K + 1 offsets), so block (g, k) reads only class k's points.  Everything
// is FP64 and reduced in a fixed order (lane, wave, block, then the block
// partials by k_reduce_part), so the results are bitwise repeatable.
#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

constexpr int kFeat = 8;   // features per block in the centroid pass

template <int DT>
__device__ __forceinline__ double feature(const void* __restrict__ img, int64_t o) {
  if constexpr (DT == DT_U8) {
    return (double)reinterpret_cast<const uint8_t*>(img)[o];
  } else if constexpr (DT == DT_F32) {
    return (double)reinterpret_cast<const float*>(img)[o];
  } else {
    return (double)to_float<DT>(reinterpret_cast<const uint16_t*>(img)[o]);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block (g, k, c): sums over class k's points g, g + G, ... (in blocks of
// kBlock) of features kFeat c .. kFeat c + 7;
// part[(k * G + g) * L + kFeat c + e], L = kFeat * gridDim.z.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_cluster_sums(const void* __restrict__ img, int64_t P, int n,
                                                         const int32_t* __restrict__ idx,
                                                         const int32_t* __restrict__ off, double* __restrict__ part) {
  __shared__ double red[kWaves][kFeat];
  const int g = blockIdx.x, k = blockIdx.y, c = blockIdx.z, G = gridDim.x;
  const int L = kFeat * gridDim.z;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc[kFeat];
#pragma unroll
  for (int e = 0; e < kFeat; ++e) acc[e] = 0.0;
  const int beg = off[k], end = off[k + 1];
  for (int i = beg + g * kBlock + threadIdx.x; i < end; i += G * kBlock) {
    const int64_t q = idx[i];
#pragma unroll
    for (int e = 0; e < kFeat; ++e)
      if (kFeat * c + e < n) acc[e] += feature<DT>(img, (int64_t)(kFeat * c + e) * P + q);
  }
#pragma unroll
  for (int e = 0; e < kFeat; ++e) {
    const double v = wave_sum(acc[e]);
    if (lane == 0) red[w][e] = v;
  }
  __syncthreads();
  if (threadIdx.x < kFeat) {
    const int e = threadIdx.x;
    double s = red[0][e];
    for (int ww = 1; ww < kWaves; ++ww) s += red[ww][e];
    part[((int64_t)k * G + g) * L + kFeat * c + e] = s;
  }
}

// Block (g, k): sum of ||X - A_k||_p over class k's points g, g + G, ...;
// A_k = sums[k][.] / counts[k].  part[k * G + g].
template <int DT>
__global__ __launch_bounds__(kBlock) void k_cluster_scatter(const void* __restrict__ img, int64_t P, int n,
                                                            const int32_t* __restrict__ idx,
                                                            const int32_t* __restrict__ off,
                                                            const double* __restrict__ sums, int L,
                                                            const int64_t* __restrict__ counts, double p,
                                                            double* __restrict__ part) {
  __shared__ double A[kMaxB];
  __shared__ double red[kWaves];
  const int g = blockIdx.x, k = blockIdx.y, G = gridDim.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x < n) A[threadIdx.x] = sums[(int64_t)k * L + threadIdx.x] / (double)counts[k];
  __syncthreads();
  double acc = 0.0;
  const int beg = off[k], end = off[k + 1];
  for (int i = beg + g * kBlock + threadIdx.x; i < end; i += G * kBlock) {
    const int64_t q = idx[i];
    double s = 0.0;
    if (p == 2.0) {
      for (int f = 0; f < n; ++f) {
        const double d = feature<DT>(img, (int64_t)f * P + q) - A[f];
        s += d * d;
      }
      s = sqrt(s);
    } else if (p == 1.0) {
      for (int f = 0; f < n; ++f) s += fabs(feature<DT>(img, (int64_t)f * P + q) - A[f]);
    } else {
      for (int f = 0; f < n; ++f) s += pow(fabs(feature<DT>(img, (int64_t)f * P + q) - A[f]), p);
      s = pow(s, 1.0 / p);
    }
    acc += s;
  }
  acc = wave_sum(acc);
  if (lane == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = red[0];
    for (int ww = 1; ww < kWaves; ++ww) s += red[ww];
    part[(int64_t)k * G + g] = s;
  }
}

template <int DT>
hipError_t cluster_dt(const void* img, int64_t P, int n, const int32_t* idx, const int32_t* off,
                      const int64_t* counts, int K, int G, double p, double* part, double* sums, double* dsum,
                      hipStream_t s) {
  const int nfc = (n + kFeat - 1) / kFeat, L = kFeat * nfc;
  double* part2 = part + (int64_t)K * G * L;
  hipLaunchKernelGGL(k_cluster_sums<DT>, dim3(G, K, nfc), dim3(kBlock), 0, s, img, P, n, idx, off, part);
  hipError_t e = launch_reduce_part(part, K, G, L, sums, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cluster_scatter<DT>, dim3(G, K), dim3(kBlock), 0, s, img, P, n, idx, off,
                     (const double*)sums, L, counts, p, part2);
  return launch_reduce_part(part2, K, G, 1, dsum, s);
}

}  // namespace

int cluster_sum_len(int n) { return kFeat * ((n + kFeat - 1) / kFeat); }

hipError_t launch_cluster_moments(int dtype, const void* img, int64_t P, int n, const int32_t* idx,
                                  const int32_t* offsets, const int64_t* counts, int K, int G, double p,
                                  double* part, double* sums, double* dsum, hipStream_t s) {
  if (n < 1 || n > kMaxB || K < 1 || G < 1) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_U8: return cluster_dt<DT_U8>(img, P, n, idx, offsets, counts, K, G, p, part, sums, dsum, s);
    case DT_U16: return cluster_dt<DT_U16>(img, P, n, idx, offsets, counts, K, G, p, part, sums, dsum, s);
    case DT_F32: return cluster_dt<DT_F32>(img, P, n, idx, offsets, counts, K, G, p, part, sums, dsum, s);
    case DT_BF16: return cluster_dt<DT_BF16>(img, P, n, idx, offsets, counts, K, G, p, part, sums, dsum, s);
    case DT_F16: return cluster_dt<DT_F16>(img, P, n, idx, offsets, counts, K, G, p, part, sums, dsum, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace cvx

// Label bookkeeping: per-class counts and a class-grouped, raster-ordered
// list of training-pixel indices (paper Section 2: the analyst's input
// points per class).  Two passes over the int8 label map: per-tile class
// counts, then every tile computes its output offsets from the counts of
// the tiles before it and writes its indices in raster order.  Integer
// only, so the result is exact and independent of scheduling.
#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

// Load the labels of this thread's 4 consecutive pixels starting at p
// (p is a multiple of 4); out-of-range pixels read as -1.  Invalid label
// values are reported through `bad` and treated as -1.
__device__ __forceinline__ void load4(const int8_t* __restrict__ labels, int64_t p, int64_t end,
                                      int K, int v[4], bool& bad) {
  if (p + 3 < end) {
    const char4 c = *reinterpret_cast<const char4*>(labels + p);
    v[0] = c.x; v[1] = c.y; v[2] = c.z; v[3] = c.w;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = (p + s < end) ? (int)labels[p + s] : -1;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (v[s] < -1 || v[s] >= K) {
      bad = true;
      v[s] = -1;
    }
  }
}

// For the 4 x 64 pixels held by a wave (lane-major raster order), give each
// labelled slot its rank among the wave's pixels of the same class, and
// call fn(k, total) once per distinct class present (uniformly, all lanes).
template <typename Fn>
__device__ __forceinline__ void wave_rank(const int v[4], int rank[4], Fn fn) {
  const int lane = __lane_id();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned pending = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (v[s] >= 0) pending |= 1u << s;
  uint64_t lanes = __ballot(pending != 0);
  while (lanes) {
    const int leader = __ffsll((unsigned long long)lanes) - 1;
    int first = -1;
#pragma unroll
    for (int s = 3; s >= 0; --s)
      if (pending & (1u << s)) first = v[s];
    const int k = __shfl(first, leader, 64);
    const uint64_t b0 = __ballot(v[0] == k), b1 = __ballot(v[1] == k);
    const uint64_t b2 = __ballot(v[2] == k), b3 = __ballot(v[3] == k);
    const int before = __popcll(b0 & lt) + __popcll(b1 & lt) + __popcll(b2 & lt) + __popcll(b3 & lt);
    int run = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (v[s] == k) {
        rank[s] = before + run;
        ++run;
        pending &= ~(1u << s);
      }
    }
    fn(k, __popcll(b0) + __popcll(b1) + __popcll(b2) + __popcll(b3));
    lanes = __ballot(pending != 0);
  }
}

__global__ __launch_bounds__(kBlock) void k_label_count(const int8_t* __restrict__ labels, int64_t P,
                                                        int K, int32_t* __restrict__ tile_counts,
                                                        int32_t* __restrict__ err) {
  __shared__ int cnt[128];
  for (int i = threadIdx.x; i < 128; i += kBlock) cnt[i] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kLabelTile;
  const int64_t t1 = (t0 + kLabelTile < P) ? t0 + kLabelTile : P;
  const int lane = __lane_id();
  bool bad = false;
  for (int64_t base = t0; base < t1; base += 4 * kBlock) {
    int v[4], rank[4];
    load4(labels, base + 4 * threadIdx.x, t1, K, v, bad);
    wave_rank(v, rank, [&](int k, int total) {
      if (lane == 0) atomicAdd(&cnt[k], total);
    });
  }
  if (bad) atomicOr(err, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < K; i += kBlock) tile_counts[(int64_t)blockIdx.x * K + i] = cnt[i];
}

__global__ __launch_bounds__(kBlock) void k_label_index(const int8_t* __restrict__ labels, int64_t P,
                                                        int K, int nT,
                                                        const int32_t* __restrict__ tile_counts,
                                                        int32_t* __restrict__ idx,
                                                        int64_t* __restrict__ counts_out,
                                                        int32_t* __restrict__ offsets_out) {
  __shared__ int before[128], total[128], base[128];
  __shared__ int wcnt[kWaves][128];
  for (int i = threadIdx.x; i < 128; i += kBlock) {
    before[i] = 0;
    total[i] = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][i] = 0;
  }
  __syncthreads();
  const int t = blockIdx.x;
  for (int i = threadIdx.x; i < nT * K; i += kBlock) {
    const int tt = i / K, k = i - tt * K;
    const int c = tile_counts[i];
    if (c) {
      atomicAdd(&total[k], c);
      if (tt < t) atomicAdd(&before[k], c);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int off = 0;
    for (int k = 0; k < K; ++k) {
      const int tk = total[k];
      base[k] = off + before[k];
      if (t == 0) {
        counts_out[k] = tk;
        offsets_out[k] = off;
      }
      off += tk;
    }
    if (t == 0) offsets_out[K] = off;
  }
  __syncthreads();
  const int64_t t0 = (int64_t)t * kLabelTile;
  const int64_t t1 = (t0 + kLabelTile < P) ? t0 + kLabelTile : P;
  const int w = threadIdx.x >> 6, lane = __lane_id();
  for (int64_t rb = t0; rb < t1; rb += 4 * kBlock) {
    int v[4], rank[4] = {0, 0, 0, 0};
    bool bad = false;
    const int64_t p = rb + 4 * threadIdx.x;
    load4(labels, p, t1, K, v, bad);
    const int any = (v[0] >= 0) | (v[1] >= 0) | (v[2] >= 0) | (v[3] >= 0);
    if (!__syncthreads_or(any)) continue;
    wave_rank(v, rank, [&](int k, int tot) {
      if (lane == 0) wcnt[w][k] = tot;
    });
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = v[s];
      if (k >= 0) {
        int pos = base[k] + rank[s];
        for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][k];
        idx[pos] = (int32_t)(p + s);
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) {
      int add = 0;
#pragma unroll
      for (int ww = 0; ww < kWaves; ++ww) {
        add += wcnt[ww][k];
        wcnt[ww][k] = 0;
      }
      base[k] += add;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_label_count(const int8_t* labels, int64_t P, int K, int nT,
                              int32_t* tile_counts, int32_t* err_flag, hipStream_t s) {
  hipLaunchKernelGGL(k_label_count, dim3(nT), dim3(kBlock), 0, s, labels, P, K, tile_counts,
                     err_flag);
  return hipGetLastError();
}

hipError_t launch_label_index(const int8_t* labels, int64_t P, int K, int nT,
                              const int32_t* tile_counts, int32_t* idx, int64_t* counts_out,
                              int32_t* offsets_out, hipStream_t s) {
  hipLaunchKernelGGL(k_label_index, dim3(nT), dim3(kBlock), 0, s, labels, P, K, nT, tile_counts,
                     idx, counts_out, offsets_out);
  return hipGetLastError();
}

}  // namespace cvx

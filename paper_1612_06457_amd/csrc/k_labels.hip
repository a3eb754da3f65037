// Label bookkeeping: per-class counts and a class-grouped, raster-ordered
// list of training-pixel indices (paper Section 2: the analyst's input
// points per class).  Integer only, so the result is exact and independent
// of scheduling.
//
// Both kernels read the int8 label map in 16-byte chunks: a wave step covers
// 64 chunks = 1024 consecutive pixels, lane l holding pixels 16 l .. 16 l + 15.
// The labelled pixels of a step (a few percent of the page) are first
// compacted, in raster order, into a small per-wave LDS list; ranks within a
// class then come from one ballot per distinct class over that list.
//   k_label_count:  per-tile class counts (tile = 64 Ki pixels per block);
//   k_label_index:  every block derives its output offsets from the counts
//                   of the tiles before it; each wave walks its quarter of
//                   the tile with wave-private running offsets, so the main
//                   loop has no block barrier.
#include "k_common.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

constexpr int kSub = kLabelTile / kWaves;   // pixels per wave in a tile
constexpr int kStep = 64 * 16;              // pixels per wave step

// Load the 16 labels of chunk c (pixel 16 c ..) within [0, end); missing
// pixels read as -1 (0xff).
__device__ __forceinline__ uint4 load_chunk(const int8_t* __restrict__ labels, int64_t p, int64_t end) {
  if (p + 16 <= end) return *reinterpret_cast<const uint4*>(labels + p);
  uint32_t d[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t pp = p + 4 * q + b;
      const uint32_t byte = (pp < end) ? (uint32_t)(uint8_t)labels[pp] : 0xffu;
      v |= byte << (8 * b);
    }
    d[q] = v;
  }
  return make_uint4(d[0], d[1], d[2], d[3]);
}

// Bit i of the result is set when byte i (of the 16) is >= 0 (labelled).
// Sets `bad` when a negative byte is not -1.
__device__ __forceinline__ uint32_t labelled_mask(uint4 c, bool& bad) {
  const uint32_t d[4] = {c.x, c.y, c.z, c.w};
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t x = d[q];
    const uint32_t neg = x & 0x80808080u;
    const uint32_t y = ~x;                                            // -1 bytes -> 0
    const uint32_t nz = ((y & 0x7f7f7f7fu) + 0x7f7f7f7fu) | y;       // high bit: byte of y != 0
    if (nz & neg & 0x80808080u) bad = true;                           // negative but not -1
    const uint32_t pos = (~x) & 0x80808080u;                          // high bit: byte >= 0
    m |= ((pos >> 7) & 1u) << (4 * q) | ((pos >> 15) & 1u) << (4 * q + 1) |
         ((pos >> 23) & 1u) << (4 * q + 2) | ((pos >> 31) & 1u) << (4 * q + 3);
  }
  return m;
}

__device__ __forceinline__ int byte_at(uint4 c, int i) {
  const uint32_t d = (i < 4) ? c.x : (i < 8) ? c.y : (i < 12) ? c.z : c.w;
  return (int)(int8_t)((d >> (8 * (i & 3))) & 0xffu);
}

// Exclusive prefix over lanes of a per-lane count in 0..16, and the total.
__device__ __forceinline__ int lane_prefix(int c, int& total) {
  const int lane = __lane_id();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const uint64_t bb = __ballot((c >> b) & 1);
    pre += __popcll(bb & lt) << b;
    tot += __popcll(bb) << b;
  }
  total = tot;
  return pre;
}

// Compact the labelled pixels of one wave step into list[] (raster order):
// list entries are (pixel offset within the step) | (class << 16).
// Returns the number of entries (uniform).
__device__ __forceinline__ int compact_step(uint4 c, int K, uint32_t* __restrict__ list, bool& bad) {
  const int lane = __lane_id();
  uint32_t m = labelled_mask(c, bad);
  int total;
  int pos = lane_prefix(__popc(m), total);
  while (m) {
    const int i = __ffs(m) - 1;
    m &= m - 1;
    const int v = byte_at(c, i);
    if (v >= K) bad = true;
    list[pos++] = (uint32_t)(16 * lane + i) | ((uint32_t)(v < K ? v : 0) << 16);
  }
  return total;
}

__global__ __launch_bounds__(kBlock) void k_label_count(const int8_t* __restrict__ labels, int64_t P,
                                                        int K, int32_t* __restrict__ tile_counts,
                                                        int32_t* __restrict__ err) {
  __shared__ int cnt[128];
  __shared__ uint32_t lists[kWaves][kStep];
  for (int i = threadIdx.x; i < 128; i += kBlock) cnt[i] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* list = lists[w];
  const int64_t s0 = (int64_t)blockIdx.x * kLabelTile + (int64_t)w * kSub;
  const int64_t s1 = (s0 + kSub < P) ? s0 + kSub : P;
  bool bad = false;
  uint4 nxt = make_uint4(~0u, ~0u, ~0u, ~0u);
  if (s0 < s1) nxt = load_chunk(labels, s0 + 16 * lane, s1);
  for (int64_t st = s0; st < s1; st += kStep) {
    const uint4 cur = nxt;
    if (st + kStep < s1) nxt = load_chunk(labels, st + kStep + 16 * lane, s1);
    const int n = compact_step(cur, K, list, bad);
    if (n == 0) continue;
    wave_lds_sync();
    for (int b0 = 0; b0 < n; b0 += 64) {
      const int i = b0 + lane;
      const int k = (i < n) ? (int)(list[i] >> 16) : -1;
      uint64_t pending = __ballot(k >= 0);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int kk = __shfl(k, leader, 64);
        const uint64_t mk = __ballot(k == kk);
        if (lane == leader) atomicAdd(&cnt[kk], __popcll(mk));
        pending &= ~mk;
      }
    }
    wave_lds_sync();
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
  __shared__ int before[128], total[128];
  __shared__ int wcnt[kWaves][128];
  __shared__ int run[kWaves][128];
  __shared__ uint32_t lists[kWaves][kStep];
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
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* list = lists[w];
  const int64_t s0 = (int64_t)t * kLabelTile + (int64_t)w * kSub;
  const int64_t s1 = (s0 + kSub < P) ? s0 + kSub : P;
  bool bad = false;
  // per-wave class counts of this wave's quarter of the tile
  for (int64_t st = s0; st < s1; st += kStep) {
    const uint4 cur = load_chunk(labels, st + 16 * lane, s1);
    const int n = compact_step(cur, K, list, bad);
    if (n == 0) continue;
    wave_lds_sync();
    for (int b0 = 0; b0 < n; b0 += 64) {
      const int i = b0 + lane;
      const int k = (i < n) ? (int)(list[i] >> 16) : -1;
      uint64_t pending = __ballot(k >= 0);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int kk = __shfl(k, leader, 64);
        const uint64_t mk = __ballot(k == kk);
        if (lane == leader) wcnt[w][kk] += __popcll(mk);
        pending &= ~mk;
      }
    }
    wave_lds_sync();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int off = 0;
    for (int k = 0; k < K; ++k) {
      const int tk = total[k];
      int b = off + before[k];
      for (int ww = 0; ww < kWaves; ++ww) {
        run[ww][k] = b;
        b += wcnt[ww][k];
      }
      if (t == 0) {
        counts_out[k] = tk;
        offsets_out[k] = off;
      }
      off += tk;
    }
    if (t == 0) offsets_out[K] = off;
  }
  __syncthreads();
  // write indices in raster order with wave-private running offsets
  uint4 nxt = make_uint4(~0u, ~0u, ~0u, ~0u);
  if (s0 < s1) nxt = load_chunk(labels, s0 + 16 * lane, s1);
  for (int64_t st = s0; st < s1; st += kStep) {
    const uint4 cur = nxt;
    if (st + kStep < s1) nxt = load_chunk(labels, st + kStep + 16 * lane, s1);
    const int n = compact_step(cur, K, list, bad);
    if (n == 0) continue;
    wave_lds_sync();
    for (int b0 = 0; b0 < n; b0 += 64) {
      const int i = b0 + lane;
      const uint32_t e = (i < n) ? list[i] : 0u;
      const int k = (i < n) ? (int)(e >> 16) : -1;
      const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      uint64_t pending = __ballot(k >= 0);
      while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int kk = __shfl(k, leader, 64);
        const uint64_t mk = __ballot(k == kk);
        const int base = run[w][kk];
        if (k == kk) idx[base + __popcll(mk & lt)] = (int32_t)(st + (e & 0xffffu));
        wave_lds_sync();
        if (lane == leader) run[w][kk] = base + __popcll(mk);
        wave_lds_sync();
        pending &= ~mk;
      }
    }
    wave_lds_sync();
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

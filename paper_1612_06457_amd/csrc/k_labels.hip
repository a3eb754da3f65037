// Label bookkeeping: per-class counts and a class-grouped, raster-ordered
// list of training-pixel indices (paper Section 2: the analyst's input
// points per class).  Integer only, so the result is exact and independent
// of scheduling.
//
// Both kernels read the int8 label map in 16-byte chunks: a wave step covers
// 64 chunks = 1024 consecutive pixels, lane l holding pixels 16 l .. 16 l + 15.
// Steps are loaded four at a time (4 KiB per wave) with the next four in
// flight while the current ones are processed; the loads are unconditional
// (clamped to the wave's last whole group), and only the ragged end of a
// wave's range takes the byte-wise path.
// Counting adds each labelled pixel into LDS class counters.  For the index
// list, the labelled pixels of a step (a few percent of the page) are first
// compacted, in raster order, into a small per-wave LDS list; ranks within a
// class then come from one ballot per distinct class over that list.
//   k_label_count:  per-tile class counts (tile = 64 Ki pixels per block);
//   k_label_index:  every block derives its output offsets from the counts
//                   of the tiles before it; each wave walks its quarter of
//                   the tile with wave-private running offsets, so the main
//                   loop has no block barrier.
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

constexpr int kSub = kLabelTile / kWaves;   // pixels per wave in a tile
constexpr int kStep = 64 * 16;              // pixels per wave step
constexpr int kGroup = 4 * kStep;           // pixels per group of four steps

// Load the 16 labels of chunk c (pixel 16 c ..) within [0, end); missing
// pixels read as -1 (0xff).
__device__ __forceinline__ u32x4 load_chunk(const int8_t* __restrict__ labels, int64_t p, int64_t end) {
  if (p + 16 <= end) return *reinterpret_cast<const u32x4*>(labels + p);
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
  return u32x4{d[0], d[1], d[2], d[3]};
}

// The four steps of the group at st (whole, inside the map): chunk q of
// lane l is pixels st + kStep q + 16 l ...
__device__ __forceinline__ void load_group(const int8_t* __restrict__ labels, int64_t st, u32x4 (&g)[4]) {
  const int lane = __lane_id();
#pragma unroll
  for (int q = 0; q < 4; ++q) g[q] = *reinterpret_cast<const u32x4*>(labels + st + kStep * q + 16 * lane);
}

// Runs step(chunk, st) for the wave's steps over [s0, s1) in raster order.
template <typename Step>
__device__ __forceinline__ void for_each_step(const int8_t* __restrict__ labels, int64_t s0, int64_t s1, Step step) {
  const int lane = __lane_id();
  const int64_t ng = (s1 > s0) ? (s1 - s0) / kGroup : 0;
  if (ng > 0) {
    u32x4 nx[4];
    load_group(labels, s0, nx);
    for (int64_t i = 0; i < ng; ++i) {
      u32x4 cur[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) cur[q] = nx[q];
      load_group(labels, s0 + kGroup * (i + 1 < ng ? i + 1 : ng - 1), nx);
      __builtin_amdgcn_sched_barrier(0);   // keep the next group's loads ahead of the work
#pragma unroll
      for (int q = 0; q < 4; ++q) step(cur[q], s0 + kGroup * i + kStep * q);
    }
  }
  for (int64_t st = s0 + kGroup * ng; st < s1; st += kStep) step(load_chunk(labels, st + 16 * lane, s1), st);
}

// Bit i of the result is set when byte i (of the 16) is >= 0 (labelled).
// Sets `bad` when a negative byte is not -1.
__device__ __forceinline__ uint32_t labelled_mask(u32x4 c, bool& bad) {
  const uint32_t d[4] = {c[0], c[1], c[2], c[3]};
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

__device__ __forceinline__ int byte_at(u32x4 c, int i) {
  const uint32_t d = (i < 4) ? c[0] : (i < 8) ? c[1] : (i < 12) ? c[2] : c[3];
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

// Add the labelled pixels of a chunk into the LDS class counters cnt[].
__device__ __forceinline__ void count_chunk(u32x4 c, int K, int* __restrict__ cnt, bool& bad) {
  uint32_t m = labelled_mask(c, bad);
  while (m) {
    const int i = __ffs(m) - 1;
    m &= m - 1;
    const int v = byte_at(c, i);
    if (v < K) atomicAdd(&cnt[v], 1);
    else bad = true;
  }
}

// Compact the labelled pixels of one wave step into list[] (raster order):
// list entries are (pixel offset within the step) | (class << 16).
// Returns the number of entries (uniform).
__device__ __forceinline__ int compact_step(u32x4 c, int K, uint32_t* __restrict__ list, bool& bad) {
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
  for (int i = threadIdx.x; i < 128; i += kBlock) cnt[i] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t s0 = (int64_t)blockIdx.x * kLabelTile + (int64_t)w * kSub;
  const int64_t s1 = (s0 + kSub < P) ? s0 + kSub : P;
  bool bad = false;
  for_each_step(labels, s0, s1, [&](u32x4 cur, int64_t) { count_chunk(cur, K, cnt, bad); });
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
  {
    // thread i < m sums the entries i, i + m, ... of the nT x K counts, all
    // of class i % K (m a multiple of K), then adds its two sums into LDS
    const int m = K * (kBlock / K);
    if ((int)threadIdx.x < m) {
      const int k = threadIdx.x % K;
      int tot = 0, bef = 0;
      for (int i = threadIdx.x; i < nT * K; i += m) {
        const int c = tile_counts[i];
        tot += c;
        bef += (i / K < t) ? c : 0;
      }
      if (tot) atomicAdd(&total[k], tot);
      if (bef) atomicAdd(&before[k], bef);
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* list = lists[w];
  const int64_t s0 = (int64_t)t * kLabelTile + (int64_t)w * kSub;
  const int64_t s1 = (s0 + kSub < P) ? s0 + kSub : P;
  bool bad = false;
  // per-wave class counts of this wave's quarter of the tile
  for_each_step(labels, s0, s1, [&](u32x4 cur, int64_t) { count_chunk(cur, K, wcnt[w], bad); });
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
  for_each_step(labels, s0, s1, [&](u32x4 cur, int64_t st) {
    const int n = compact_step(cur, K, list, bad);
    if (n == 0) return;
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
  });
}

// Training points given as a list: the label kernels ran over the N point
// classes, so idx[0 .. total) holds positions in the list; replace each by
// its pixel, flagging (bit 2 of err) a pixel outside 0..P-1.
__global__ __launch_bounds__(kBlock) void k_points_to_pixels(const int64_t* __restrict__ pixels,
                                                             int32_t* __restrict__ idx,
                                                             const int32_t* __restrict__ offsets, int K,
                                                             int64_t P, int32_t* __restrict__ err) {
  const int64_t total = offsets[K];
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t p = pixels[idx[i]];
    const bool ok = p >= 0 && p < P;
    idx[i] = ok ? (int32_t)p : 0;
    bad |= !ok;
  }
  if (bad) atomicOr(err, 2);
}

}  // namespace

hipError_t launch_points_to_pixels(const int64_t* pixels, int32_t* idx, const int32_t* offsets, int K, int64_t N,
                                   int64_t P, int32_t* err_flag, int num_cu, hipStream_t s) {
  const int64_t need = (N + kBlock - 1) / kBlock;
  const int nb = (int)(need < (int64_t)num_cu * 8 ? (need > 0 ? need : 1) : (int64_t)num_cu * 8);
  hipLaunchKernelGGL(k_points_to_pixels, dim3(nb), dim3(kBlock), 0, s, pixels, idx, offsets, K, P, err_flag);
  return hipGetLastError();
}

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

// Label bookkeeping: per-class counts and a class-grouped, raster-ordered
// list of training-pixel indices (paper Section 2: the analyst's input
// points per class).  Integer only, so the result is exact and independent
// of scheduling.
//
// The label map is cut into wave tiles of kLabelWave entries (four wave
// steps).  A wave step covers 64 chunks of 16 bytes = 1024 consecutive
// entries, lane l holding entries 16 l .. 16 l + 15; a tile's four steps are
// loaded at once, and only the ragged end of the map takes the byte-wise
// path.  Small tiles give many waves, which is what these latency-bound
// passes need (the training pixels are a few percent of the page, scattered
// over it, so every step holds several classes).
//   k_label_count: class counts per wave tile, class-major (K rows of nW,
//                  each row padded to a multiple of four entries), with
//                  LDS counters private to the wave, and a row of flags
//                  for entries outside -1..K-1;
//   k_label_scan:  one block per class turns its row of counts into
//                  exclusive offsets within the class, and the class total;
//                  one more block turns the flags into the error flag;
//   k_label_index: each wave starts from its offsets (class base + its
//                  offset within the class), compacts the valid labelled
//                  entries of a step, in raster order, into a per-wave LDS
//                  list, and writes them with one ballot per distinct class
//                  of the list, the running offsets held in registers
//                  spread over the lanes (lane l: classes l and 64 + l).
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

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

// Bit i of the result is set when byte i (of the 16) is a class in 0..K-1.
// Sets `bad` for a byte outside -1..K-1.
__device__ __forceinline__ uint32_t valid_mask(u32x4 c, int K, bool& bad) {
  const uint32_t below = (uint32_t)(128 - K) * 0x01010101u;   // byte b < K <=> b + 128 - K < 128
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t x = c[q];
    const uint32_t neg = x & 0x80808080u;
    const uint32_t y = ~x;                                            // -1 bytes -> 0
    const uint32_t nz = ((y & 0x7f7f7f7fu) + 0x7f7f7f7fu) | y;       // high bit: byte of y != 0
    const uint32_t lt = ~((x & 0x7f7f7f7fu) + below) & 0x80808080u;  // high bit: low 7 bits < K
    const uint32_t ok = ~neg & lt;                                    // high bit: 0 <= byte < K
    if ((nz & neg) | (~neg & ~lt & 0x80808080u)) bad = true;         // negative but not -1, or >= K
    m |= ((ok >> 7) & 1u) << (4 * q) | ((ok >> 15) & 1u) << (4 * q + 1) |
         ((ok >> 23) & 1u) << (4 * q + 2) | ((ok >> 31) & 1u) << (4 * q + 3);
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

// Per-class values held across the wave's lanes: lane l keeps class l in
// lo and class 64 + l in hi (K <= 127).  v is uniform.  get() reads both
// registers of the owning lane and selects on the scalar side, so its result
// does not depend on which lanes are active; still, call it where the whole
// wave is.
struct LaneClasses {
  int lo = 0, hi = 0;
  __device__ __forceinline__ int get(int v) const {
    const int l = __builtin_amdgcn_readlane(lo, v & 63);
    const int h = __builtin_amdgcn_readlane(hi, v & 63);
    return v < 64 ? l : h;
  }
  __device__ __forceinline__ void add(int v, int n) {
    if (__lane_id() == (v & 63)) {
      if (v < 64) lo += n;
      else hi += n;
    }
  }
};

// Inclusive prefix sum over the wave's lanes.
__device__ __forceinline__ int wave_inclusive(int x) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__global__ __launch_bounds__(kBlock) void k_label_count(const int8_t* __restrict__ labels, int64_t P, int K,
                                                        int nW, int32_t* __restrict__ wave_counts) {
  __shared__ int cnt[kWaves][128];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wv = blockIdx.x * kWaves + w;
  int* my = cnt[w];
  my[lane] = 0;
  my[64 + lane] = 0;
  wave_lds_sync();
  if (wv >= nW) return;
  const int64_t s0 = (int64_t)wv * kLabelWave;
  const int64_t s1 = (s0 + kLabelWave < P) ? s0 + kLabelWave : P;
  bool bad = false;
  for_each_step(labels, s0, s1, [&](u32x4 cur, int64_t) {
    uint32_t m = valid_mask(cur, K, bad);
    while (m) {
      const int i = __ffs(m) - 1;
      m &= m - 1;
      atomicAdd(&my[byte_at(cur, i)], 1);
    }
  });
  wave_lds_sync();
  const int64_t ld = label_row_stride(nW);
  for (int k = lane; k < K; k += 64) wave_counts[(int64_t)k * ld + wv] = my[k];
  const bool any_bad = __ballot(bad) != 0;
  if (lane == 0) wave_counts[(int64_t)K * ld + wv] = any_bad ? 1 : 0;
}

// Block k < K: row k of the counts becomes exclusive offsets within the
// class (in place), and class_total[k] its sum.  Block K sums the row of
// flags the same way and sets the error flag from it.  Chunks of kScanThreads x
// kPer entries (one chunk covers a page of 67 M entries): each thread moves
// its kPer consecutive entries with 16-byte loads and stores (the rows are
// padded to a multiple of four entries), all in flight together, and the
// block scans the thread sums.  Entries past nW read as zero.
constexpr int kPer = 16;
constexpr int kScanThreads = 1024;
constexpr int kScanWaves = kScanThreads / 64;
__global__ __launch_bounds__(kScanThreads) void k_label_scan(int32_t* __restrict__ wave_counts, int nW, int K,
                                                             int32_t* __restrict__ class_total,
                                                             int32_t* __restrict__ err) {
  __shared__ int wsum[kScanWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ld = (int)label_row_stride(nW);
  int32_t* row = wave_counts + (int64_t)blockIdx.x * ld;
  int carry = 0;
  for (int c0 = 0; c0 < nW; c0 += kScanThreads * kPer) {
    const int j0 = c0 + (int)threadIdx.x * kPer;
    int v[kPer];
#pragma unroll
    for (int q = 0; q < kPer / 4; ++q) {
      const int j = j0 + 4 * q;
      const u32x4 x = j < ld ? *reinterpret_cast<const u32x4*>(row + j) : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
      for (int e = 0; e < 4; ++e) v[4 * q + e] = (j + e < nW) ? (int)x[e] : 0;
    }
    int sum = 0;
#pragma unroll
    for (int e = 0; e < kPer; ++e) sum += v[e];
    const int inc = wave_inclusive(sum);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int base = carry, tot = 0;
#pragma unroll
    for (int ww = 0; ww < kScanWaves; ++ww) {
      base += (ww < w) ? wsum[ww] : 0;
      tot += wsum[ww];
    }
    __syncthreads();
    int run = base + inc - sum;
#pragma unroll
    for (int q = 0; q < kPer / 4; ++q) {
      const int j = j0 + 4 * q;
      u32x4 o;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[e] = (uint32_t)run;
        run += v[4 * q + e];
      }
      if (j < ld) *reinterpret_cast<u32x4*>(row + j) = o;   // the padding takes values no one reads
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if ((int)blockIdx.x < K) {
      class_total[blockIdx.x] = carry;
    } else {
      err[0] = carry > 0 ? 1 : 0;
      err[1] = 0;
    }
  }
}

// Compact the valid labelled entries of one wave step into list[] (raster
// order): entries are (offset within the step) | (class << 16).  Returns
// their number (uniform).
__device__ __forceinline__ int compact_step(u32x4 c, int K, uint32_t* __restrict__ list) {
  const int lane = __lane_id();
  bool bad = false;   // reported by the count kernel
  uint32_t m = valid_mask(c, K, bad);
  int total;
  int pos = lane_prefix(__popc(m), total);
  while (m) {
    const int i = __ffs(m) - 1;
    m &= m - 1;
    list[pos++] = (uint32_t)(16 * lane + i) | ((uint32_t)byte_at(c, i) << 16);
  }
  return total;
}

__global__ __launch_bounds__(kBlock) void k_label_index(const int8_t* __restrict__ labels, int64_t P, int K,
                                                        int nW, const int32_t* __restrict__ wave_off,
                                                        const int32_t* __restrict__ class_total,
                                                        int32_t* __restrict__ idx,
                                                        int64_t* __restrict__ counts_out,
                                                        int32_t* __restrict__ offsets_out) {
  __shared__ uint32_t lists[kWaves][kStep];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wv = blockIdx.x * kWaves + w;
  // class bases (exclusive prefix of the totals), classes lane and 64 + lane
  const int t_lo = lane < K ? class_total[lane] : 0;
  const int t_hi = 64 + lane < K ? class_total[64 + lane] : 0;
  const int inc_lo = wave_inclusive(t_lo);
  const int sum_lo = __shfl(inc_lo, 63, 64);
  const int inc_hi = wave_inclusive(t_hi);
  const int base_lo = inc_lo - t_lo, base_hi = sum_lo + inc_hi - t_hi;
  if (blockIdx.x == 0 && w == 0) {
    if (lane < K) {
      counts_out[lane] = t_lo;
      offsets_out[lane] = base_lo;
    }
    if (64 + lane < K) {
      counts_out[64 + lane] = t_hi;
      offsets_out[64 + lane] = base_hi;
    }
    if (lane == 63) offsets_out[K] = sum_lo + inc_hi;
  }
  if (wv >= nW) return;
  LaneClasses at;
  const int64_t ld = label_row_stride(nW);
  at.lo = lane < K ? base_lo + wave_off[(int64_t)lane * ld + wv] : 0;
  at.hi = 64 + lane < K ? base_hi + wave_off[(int64_t)(64 + lane) * ld + wv] : 0;
  uint32_t* list = lists[w];
  const int64_t s0 = (int64_t)wv * kLabelWave;
  const int64_t s1 = (s0 + kLabelWave < P) ? s0 + kLabelWave : P;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for_each_step(labels, s0, s1, [&](u32x4 cur, int64_t st) {
    const int n = compact_step(cur, K, list);
    if (n == 0) return;
    wave_lds_sync();
    for (int b0 = 0; b0 < n; b0 += 64) {
      const int i = b0 + lane;
      const uint32_t e = (i < n) ? list[i] : 0u;
      const int k = (i < n) ? (int)(e >> 16) : -1;
      for (uint64_t pending = __ballot(k >= 0); pending;) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int kk = __builtin_amdgcn_readlane(k, leader);
        const uint64_t mk = __ballot(k == kk);
        const int base = at.get(kk);
        if (k == kk) idx[base + __popcll(mk & lt)] = (int32_t)(st + (e & 0xffffu));
        at.add(kk, __popcll(mk));
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

hipError_t launch_label_count(const int8_t* labels, int64_t P, int K, int nW, int32_t* wave_counts,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_label_count, dim3((nW + kWaves - 1) / kWaves), dim3(kBlock), 0, s, labels, P, K, nW,
                     wave_counts);
  return hipGetLastError();
}

hipError_t launch_label_scan(int32_t* wave_counts, int nW, int K, int32_t* class_total, int32_t* err_flag,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_label_scan, dim3(K + 1), dim3(kScanThreads), 0, s, wave_counts, nW, K, class_total,
                     err_flag);
  return hipGetLastError();
}

hipError_t launch_label_index(const int8_t* labels, int64_t P, int K, int nW, const int32_t* wave_off,
                              const int32_t* class_total, int32_t* idx, int64_t* counts_out, int32_t* offsets_out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_label_index, dim3((nW + kWaves - 1) / kWaves), dim3(kBlock), 0, s, labels, P, K, nW,
                     wave_off, class_total, idx, counts_out, offsets_out);
  return hipGetLastError();
}

}  // namespace cvx

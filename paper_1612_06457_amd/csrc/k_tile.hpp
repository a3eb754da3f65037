// Wave tiles of the band-interleaved page, shared by the projection passes.
//
// A wave owns a tile of 64 "lane groups"; a lane group is the smallest run
// of whole pixels that is a whole number of dwords (two pixels for 16-bit
// elements and an odd band count, else one pixel), so a tile is 256 S bytes
// with S the dwords per lane group.  A tile that lies wholly inside the page
// is fetched with coalesced 16-byte loads (chunk j = lane + 64 q) into
// registers, all issued back to back with no branch between them (a branch
// there makes the compiler wait for each load before the next), and
// stored into the wave's LDS slice later; this lets the next tile's loads
// be in flight while the current one is computed.  The page's last, partial
// tile is copied straight into LDS, element by element where it straddles
// the end, zero-filled beyond it, so no load leaves the page.
#pragma once
#include "k_common.hpp"

namespace cvx {

constexpr int kMaxQ = 16;   // 16-byte chunks per lane per tile: 16 S / 64 <= 16 for S <= 64

// A native 4-dword vector: loads and stores of it stay plain vector memory
// operations (HIP's uint4 is a union type whose copies become memcpy calls,
// which keep a register array of them in scratch memory).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int DT>
struct Geo {
  static constexpr int esize = (DT == DT_F32) ? 4 : 2;
  static __device__ __host__ constexpr int g2(int B) { return (esize == 2 && (B & 1)) ? 2 : 1; }
  static __device__ __host__ constexpr int S(int B) { return (esize == 4 || (B & 1)) ? B : B / 2; }
};

// Loads of a whole tile t (tile_bytes bytes, a multiple of 16) into
// registers, by the NT threads sharing the tile (Q >= tile_bytes / 16 NT),
// with no branch: a chunk index past the tile's last chunk is clamped to it
// (a re-read that the store below drops), so every register of r is written
// on every path and the array stays in registers.  STREAM marks the loads
// non-temporal: data read once (a page far larger than the caches) then
// does not displace other lines, and a streaming read measured about 10 %
// faster on this device (6.46 against 5.87 TB/s).  Operands that the next
// kernel reads again keep the default policy.
template <int Q, int NT = 64, bool STREAM = true>
__device__ __forceinline__ void load_tile(const unsigned char* __restrict__ base, int64_t t, int tile_bytes,
                                          int tid, u32x4 (&r)[Q]) {
  const unsigned char* tb = base + t * (int64_t)tile_bytes;
  const int last = tile_bytes / 16 - 1;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const u32x4* p = reinterpret_cast<const u32x4*>(tb + 16 * min(tid + NT * q, last));
    r[q] = STREAM ? __builtin_nontemporal_load(p) : *p;
  }
}

template <int Q, int NT = 64>
__device__ __forceinline__ void store_tile(uint32_t* __restrict__ my, int tile_bytes, int tid, const u32x4 (&r)[Q]) {
  const int nchunk = tile_bytes / 16;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = tid + NT * q;
    if (j < nchunk) *reinterpret_cast<u32x4*>(my + 4 * j) = r[q];
  }
}

// The partial last tile, straight into LDS (16-bit granularity at the end).
template <int NT = 64>
__device__ __forceinline__ void copy_partial_tile(const unsigned char* __restrict__ base, int64_t total_bytes,
                                                  int64_t t, int tile_bytes, int tid, uint32_t* __restrict__ my) {
  const int64_t tb = t * (int64_t)tile_bytes;
  const int nchunk = tile_bytes / 16;
  for (int j = tid; j < nchunk; j += NT) {
    const int64_t ob = tb + 16 * (int64_t)j;
    u32x4 v;
    if (ob + 16 <= total_bytes) {
      v = *reinterpret_cast<const u32x4*>(base + ob);
    } else {
      uint32_t h[8];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        h[e] = (ob + 2 * e + 2 <= total_bytes) ? *reinterpret_cast<const uint16_t*>(base + ob + 2 * e) : 0u;
      v = u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
    }
    *reinterpret_cast<u32x4*>(my + 4 * j) = v;
  }
}

template <int NT>
__device__ __forceinline__ void tile_sync() {
  if constexpr (NT == 64) wave_lds_sync();
  else __syncthreads();
}

// Runs compute(t) for the tiles t = first, first + stride, ... < nt of this
// wave (NT = 64: wave tiles, `my` the wave's LDS slice) or of this block
// (NT = kBlock), with tile t staged in `my` and the loads of the next tile
// in flight meanwhile.  The prefetch is unconditional (its tile index is
// clamped to a whole tile: past the end it re-reads the current, cache-hot
// one), because a conditional write to the register buffer makes the
// compiler keep that buffer in scratch memory.  A page shorter than one
// tile takes the plain path.  A scheduling barrier keeps the prefetch issued
// before the compute (the scheduler would otherwise sink it to the end of
// the loop body to reuse its registers).
template <int Q, int NT, bool STREAM = true, typename Compute>
__device__ __forceinline__ void for_each_tile_n(const unsigned char* __restrict__ base, int64_t total_bytes,
                                                int64_t nt, int tile_bytes, uint32_t* __restrict__ my,
                                                Compute compute) {
  static_assert(NT == 64 || NT == kBlock, "tiles belong to a wave or to the block");
  const int tid = NT == 64 ? (threadIdx.x & 63) : threadIdx.x;
  const int64_t stride = NT == 64 ? (int64_t)gridDim.x * kWaves : (int64_t)gridDim.x;
  int64_t t = NT == 64 ? (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6) : (int64_t)blockIdx.x;
  const int64_t nfull = total_bytes / tile_bytes;
  if (nfull == 0) {
    for (; t < nt; t += stride) {
      copy_partial_tile<NT>(base, total_bytes, t, tile_bytes, tid, my);
      tile_sync<NT>();
      compute(t);
      tile_sync<NT>();
    }
    return;
  }
  u32x4 r[Q];
  load_tile<Q, NT, STREAM>(base, t < nfull ? t : nfull - 1, tile_bytes, tid, r);
  for (; t < nt; t += stride) {
    if (t < nfull) store_tile<Q, NT>(my, tile_bytes, tid, r);
    else copy_partial_tile<NT>(base, total_bytes, t, tile_bytes, tid, my);
    tile_sync<NT>();
    const int64_t tn = t + stride;
    load_tile<Q, NT, STREAM>(base, tn < nfull ? tn : (t < nfull ? t : nfull - 1), tile_bytes, tid, r);
    __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the compute
    compute(t);
    tile_sync<NT>();
  }
}

// Wave tiles of 64 lane groups of S dwords.
template <int Q, bool STREAM = true, typename Compute>
__device__ __forceinline__ void for_each_tile(const unsigned char* __restrict__ base, int64_t total_bytes,
                                              int64_t nt, int S, uint32_t* __restrict__ my, Compute compute) {
  for_each_tile_n<Q, 64, STREAM>(base, total_bytes, nt, 256 * S, my, compute);
}

}  // namespace cvx

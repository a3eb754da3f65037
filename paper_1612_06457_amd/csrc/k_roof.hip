// Reference streams for measurement: every 16-byte chunk of a device
// buffer read once with non-temporal loads, eight in flight per thread
// (the access pattern of the page passes, without their arithmetic).  The
// read-only stream's rate is the read ceiling the page-streaming kernels
// are compared with; the mixed stream also writes a second buffer, spread
// evenly over the reads, so its rate is the ceiling for a pass that writes
// as it reads in the same proportion.  The loaded words are folded into one
// per thread, and a word that matches a value the caller chooses is written
// to `sink`, so no load can be dropped by the compiler.
#include <algorithm>

#include "k_tile.hpp"

namespace cvx {

namespace {

__global__ __launch_bounds__(kBlock) void k_stream_read(const u32x4* __restrict__ src, int64_t n, uint32_t key,
                                                        uint32_t* __restrict__ sink) {
  // a wave reads a contiguous tile of U x 64 chunks (lane l, load u: chunk
  // 64 u + l of the tile), then steps by the grid's waves
  constexpr int U = 8;
  constexpr int64_t TILE = U * 64;
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  uint32_t acc = 0u;
  for (int64_t t = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); t * TILE < n; t += nwaves) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = t * TILE + 64 * u + lane;
      v[u] = __builtin_nontemporal_load(src + (k < n ? k : n - 1));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u][0] ^ v[u][1] ^ v[u][2] ^ v[u][3];
  }
  if (acc == key) sink[0] = acc;
}

// Read tiles as above; after read tile t the wave writes the write tiles
// [t nw / nr, (t + 1) nw / nr) of dst (at most one, as nw <= nr) with
// non-temporal stores of the words it has just loaded.
__global__ __launch_bounds__(kBlock) void k_stream_mix(const u32x4* __restrict__ src, int64_t n,
                                                       u32x4* __restrict__ dst, int64_t m, uint32_t key,
                                                       uint32_t* __restrict__ sink) {
  constexpr int U = 8;
  constexpr int64_t TILE = U * 64;
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  const int64_t nr = (n + TILE - 1) / TILE, nw = (m + TILE - 1) / TILE;
  uint32_t acc = 0u;
  for (int64_t t = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); t < nr; t += nwaves) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = t * TILE + 64 * u + lane;
      v[u] = __builtin_nontemporal_load(src + (k < n ? k : n - 1));
    }
    const int64_t w0 = t * nw / nr, w1 = (t + 1) * nw / nr;
    if (w1 > w0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = w0 * TILE + 64 * u + lane;
        if (k < m) __builtin_nontemporal_store(v[u], dst + k);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u][0] ^ v[u][1] ^ v[u][2] ^ v[u][3];
  }
  if (acc == key) sink[0] = acc;
}

}  // namespace

hipError_t launch_stream_mix(const void* src, int64_t read_bytes, void* dst, int64_t write_bytes, uint32_t key,
                             uint32_t* sink, int num_cu, hipStream_t s) {
  const int64_t n = read_bytes / 16, m = write_bytes / 16;
  if (n < 1 || m < 0 || m > n) return hipErrorInvalidValue;
  const int64_t want = (n + 8 * 64 * kWaves - 1) / (8 * 64 * kWaves);
  const int nb = (int)std::min<int64_t>(want, (int64_t)num_cu * 8);
  hipLaunchKernelGGL(k_stream_mix, dim3(nb), dim3(kBlock), 0, s, reinterpret_cast<const u32x4*>(src), n,
                     reinterpret_cast<u32x4*>(dst), m, key, sink);
  return hipGetLastError();
}

hipError_t launch_stream_read(const void* src, int64_t bytes, uint32_t key, uint32_t* sink, int num_cu,
                              hipStream_t s) {
  const int64_t n = bytes / 16;
  if (n < 1) return hipErrorInvalidValue;
  const int64_t want = (n + 8 * 64 * kWaves - 1) / (8 * 64 * kWaves);   // blocks whose waves all get a tile
  const int nb = (int)std::min<int64_t>(want, (int64_t)num_cu * 8);
  hipLaunchKernelGGL(k_stream_read, dim3(nb), dim3(kBlock), 0, s, reinterpret_cast<const u32x4*>(src), n, key,
                     sink);
  return hipGetLastError();
}

}  // namespace cvx

// FP32 register-tiled Gram accumulation shared by the scatter kernels:
// thread (slice, tile) owns one upper-triangular 4 x 4 tile of the padded
// (B+1) x (B+1) Gram and every nslice-th row of a chunk; its FP32 tile is
// added into FP64 registers after each chunk, and a block's threads combine
// across slices in a fixed order.
#pragma once
#include "k_common.hpp"

namespace cvx {

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

}  // namespace cvx

// Fused centre-project-stretch for uint16 pages on the matrix cores (paper
// Section 2: the regression coefficients multiply every band of the whole
// page; each float image is rescaled to 0..255 on its page range).
//
// y_j = sum_b (x_b - c_b) W[b][j] + off_j with c_b an integer centre.  The
// contraction runs on v_mfma_f32_16x16x32_f16 with FP32 accumulation, and
// the operands are built exactly with bit operations, no conversions:
//
//   x = 1024 h + l (h: 6 bits, l: 10 bits), c = 1024 c_h + c_l.  The fp16
//   value with bits 0x6400 | l is 1024 + l exactly, so one AND-OR makes two
//   of them from a dword of two elements; likewise 1024 + h, and one packed
//   fp16 add of -(1024 + c_h) gives h - c_h (|.| <= 63) exactly.  Then
//   x - c = 1024 (h - c_h) + (1024 + l) - (1024 + c_l): the last term is a
//   constant per component, taken into the accumulator's start (the host
//   folds sum_b (1024 + c_l) W[b][j] into off_j in FP64).  The uncentred
//   1024 + l is at most 2047, no larger than the centred values the
//   accumulator carries anyway, so the FP32 rounding is of the same size.
//
//   A (16 rows x 32 slots): a row is one lane group (two pixels when B is
//   odd, so rows stay dword aligned; else one pixel).  Lane l holds row
//   l % 16 and, for K-block kb, the dwords q = 8 kb + 2 (l / 16) + {0, 1}
//   of that row: the l-parts of their four elements and then the h-parts.
//   Dwords past the row's end read the next row (or padding) and meet zero
//   weights; their transformed values are always finite.
//
//   B (32 slots x 16 columns): column n = 8 p + j is component j of pixel p
//   of the row.  The slot of element E (pixel E / B, band E % B) carries
//   W[band][j] for p = E / B (zero otherwise), times 1024 for the h-part.
//   The weights are scaled by a power of two per component (so the largest
//   is in [16, 32)) and split into three fp16 terms (33 significant bits;
//   the small terms may be subnormal, which costs at most 2^-29 of the
//   largest weight).  Products of fp16 values are exact in FP32.
//
//   C (16 rows x 16 columns): lane l holds rows 4 (l / 16) + e, column l % 16.
//
// The scaled sum is 2^s_j (y_j): pass 1 keeps min/max of it per column and
// the last block folds the block partials into the stretch map
// q = floor(y' s' + o), which equals the map on y exactly because scaling by
// 2^s_j is exact; the range reported to the host is scaled back.  Pass 2
// quantises and writes planar bytes (8 bytes per lane for two-pixel rows).
//
// Tiles are streamed as in the other projection kernels (k_tile.hpp), with
// the next tile's loads in flight while the current one is computed.  The
// constant operands live in a per-block LDS table.  Two waves per SIMD
// measured fastest: three (smaller tiles, or a register cap) and a second
// prefetched tile were both slower.
#include <algorithm>

#include "k_stored.hpp"
#include "k_tile.hpp"

namespace cvx {

namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mma(f16x8 a, f16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint32_t h16(_Float16 v) { return (uint32_t)__builtin_bit_cast(uint16_t, v); }

// The bit masks of the operand build, held in registers: VOP3 encodings on
// gfx9 take no literal operand, so with the masks as literals every AND-OR
// would be split into a VOP2 AND and a VOP2 OR.
struct Masks {
  uint32_t lo, hi, exp;   // 0x03ff03ff, 0x003f003f, 0x64006400
};
__device__ __forceinline__ Masks make_masks() {
  Masks m{0x03ff03ffu, 0x003f003fu, 0x64006400u};
  asm volatile("" : "+v"(m.lo), "+v"(m.hi), "+v"(m.exp));
  return m;
}

// 1024 + l and h - c_h for both elements of a data dword, as fp16 pairs.
__device__ __forceinline__ uint32_t low_part(uint32_t d, const Masks& m) { return (d & m.lo) | m.exp; }
__device__ __forceinline__ uint32_t high_part(uint32_t d, uint32_t nh, const Masks& m) {
  const f16x2 v = __builtin_bit_cast(f16x2, ((d >> 10) & m.hi) | m.exp);
  return __builtin_bit_cast(uint32_t, v + __builtin_bit_cast(f16x2, nh));
}

// v = t0 + t1 + t2 with each term the nearest fp16 to what is left.
__device__ __forceinline__ void split3(float v, _Float16& t0, _Float16& t1, _Float16& t2) {
  t0 = (_Float16)v;
  const float r = v - (float)t0;
  t1 = (_Float16)r;
  t2 = (_Float16)(r - (float)t1);
}

// Constant operands for NKB K-blocks, per lane, kept in LDS (the same for
// every wave of the block): the three fp16 terms of the scaled weights (B
// operand) and, per data dword pair, -(1024 + c_h) for both elements of
// each dword.
// 16-row blocks per wave tile (fewer rows per tile, for more blocks per CU,
// measured slower: the per-tile overhead grows faster than the overlap).
template <int NKB>
constexpr int row_blocks() { return 4; }

// The fp16 values of one wave tile staged by plane before their stores:
// dwords per plane row (16 RB G2 pixels, 2 per dword), padded so that the
// eight planes start 16 (two-pixel rows) or 8 banks apart.
template <int NKB>
__host__ __device__ constexpr int staged_row_dwords(int G2) {
  return 8 * row_blocks<NKB>() * G2 + (G2 == 2 ? 16 : 8);
}

// LDS dwords per wave: a tile (16 RB rows of S dwords), and at least the
// staged output of either pass (8 planes x 16 RB G2 pixels: bytes in the
// stretch pass, fp16 values in pass 1).
template <int NKB>
__host__ __device__ constexpr int slice_dwords(int S, int G2) {
  return 16 * row_blocks<NKB>() * S > 8 * staged_row_dwords<NKB>(G2) ? 16 * row_blocks<NKB>() * S
                                                                     : 8 * staged_row_dwords<NKB>(G2);
}

template <int NKB>
struct OpsTab {
  u32x4 w[NKB][3][64];
  u32x2 c[NKB][64];   // {nh(q0), nh(q1)}
};

// The kernel argument block copied into LDS by the whole block (one
// coalesced round of loads instead of many dependent per-lane ones).
__device__ __forceinline__ void stage_args(const ProjArgs& a, ProjArgs& sa) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&a);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&sa);
  for (int i = threadIdx.x; i < (int)(sizeof(ProjArgs) / 4); i += kBlock) dst[i] = src[i];
  __syncthreads();
}

// a.c holds 2^23 + c_b (c_b a non-negative integer), so its low 23 bits are
// c_b.  The first wave fills the table; every lane returns its
// accumulator start (off_j scaled).
template <int NKB, int G2>
__device__ __forceinline__ float build_ops(const ProjArgs& a, int B, int nc, OpsTab<NKB>& tab) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, g = lane >> 4;
  const int p = col >> 3, j = col & 7;
  const bool live = p < G2 && j < nc;
  const float sc = live ? a.scale[j] : 0.f;
  if (threadIdx.x < 64) {
    const int nel = G2 * B;
    for (int kb = 0; kb < NKB; ++kb) {
      f16x8 w[3];
      uint32_t cv[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int q = 8 * kb + 2 * g + u;
        uint32_t nhv = 0;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int E = 2 * q + hh;
          uint32_t cb = 0;
          float wv = 0.f;
          if (E < nel) {
            const int pix = E >= B ? 1 : 0;
            const int b = E - pix * B;
            cb = __float_as_uint(a.c[b]) & 0x7fffffu;
            if (live && pix == p) wv = a.w[b * nc + j] * sc;
          }
          nhv |= h16((_Float16)(-(float)(1024u + (cb >> 10)))) << (16 * hh);
          _Float16 t0, t1, t2;
          split3(wv, t0, t1, t2);
          w[0][2 * u + hh] = t0;
          w[1][2 * u + hh] = t1;
          w[2][2 * u + hh] = t2;
          split3(1024.f * wv, t0, t1, t2);
          w[0][4 + 2 * u + hh] = t0;
          w[1][4 + 2 * u + hh] = t1;
          w[2][4 + 2 * u + hh] = t2;
        }
        cv[u] = nhv;
      }
#pragma unroll
      for (int m = 0; m < 3; ++m) tab.w[kb][m][lane] = __builtin_bit_cast(u32x4, w[m]);
      tab.c[kb][lane] = u32x2{cv[0], cv[1]};
    }
  }
  __syncthreads();
  return live ? a.off[j] * sc : 0.f;
}

// The RB 16 x 16 output blocks of a wave tile: acc[rb] for rows
// 16 rb + (lane % 16), rp = that row's start + 2 (lane / 16) for rb = 0.
// The blocks' products are interleaved so that consecutive MFMAs are
// independent.
template <int NKB, int RB>
__device__ __forceinline__ void project_tile(const uint32_t* __restrict__ rp, int S, const OpsTab<NKB>& tab,
                                             float acc0, const Masks& mk, f32x4 (&acc)[RB]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = f32x4{acc0, acc0, acc0, acc0};
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    const u32x2 cv = tab.c[kb][lane];
    f16x8 A[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const uint32_t* q = rp + 16 * rb * S + 8 * kb;
      const uint32_t d0 = q[0], d1 = q[1];
      u32x4 v;
      v[0] = low_part(d0, mk);
      v[1] = low_part(d1, mk);
      v[2] = high_part(d0, cv[0], mk);
      v[3] = high_part(d1, cv[1], mk);
      A[rb] = __builtin_bit_cast(f16x8, v);
    }
#pragma unroll
    for (int m = 2; m >= 0; --m) {   // smallest terms first
      const f16x8 wm = __builtin_bit_cast(f16x8, tab.w[kb][m][lane]);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = mma(A[rb], wm, acc[rb]);
    }
  }
}

// Tile loop shared by both passes: body(t, acc[RB]) per wave tile of
// 16 RB rows (lane groups), acc[rb] holding rows 16 rb + 4 (lane / 16) + e.
template <int NKB, int G2, typename Body>
__device__ __forceinline__ void run_tiles(const void* __restrict__ cube, int B, int64_t P, const OpsTab<NKB>& tab,
                                          float acc0, uint32_t* __restrict__ lds, Body body) {
  constexpr int RB = row_blocks<NKB>();
  constexpr int TR = 16 * RB;                  // rows per wave tile
  constexpr int Q = (TR * 8 * NKB + 255) / 256;  // 16-byte chunks per lane: TR S / 4 / 64, S <= 8 NKB
  const int S = G2 == 2 ? B : B / 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* my = lds + w * slice_dwords<NKB>(S, G2);
  const int64_t tp = TR * G2;
  const int64_t nt = (P + tp - 1) / tp;
  const int64_t total_bytes = P * B * 2;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(cube);
  const uint32_t* rp = my + (lane & 15) * S + 2 * (lane >> 4);
  const Masks mk = make_masks();
  for_each_tile_n<Q, 64>(base, total_bytes, nt, TR * S * 4, my, [&](int64_t t) {
    f32x4 acc[RB];
    project_tile<NKB, RB>(rp, S, tab, acc0, mk, acc);
    body(t, acc);
  });
}

// Four consecutive pixels of this lane's component plane from the tile's
// row block rb: for two-pixel rows the partner lane l ^ 8 holds the other
// pixel of each row, and the two lanes swap halves; *px receives the first
// pixel's index.
template <int G2>
__device__ __forceinline__ f32x4 four_pixels(const f32x4& acc, int g, int p, int rb, int64_t pb, int64_t* px) {
  if constexpr (G2 == 2) {
    const float s0 = p == 0 ? acc[2] : acc[0];
    const float s1 = p == 0 ? acc[3] : acc[1];
    const float r0 = __shfl_xor(s0, 8, 64), r1 = __shfl_xor(s1, 8, 64);
    *px = pb + 2 * (16 * rb + 4 * g) + 4 * p;
    return p == 0 ? f32x4{acc[0], r0, acc[1], r1} : f32x4{r0, acc[2], r1, acc[3]};
  } else {
    *px = pb + 16 * rb + 4 * g;
    return acc;
  }
}

// Pass 1.  With H16 it also stores every component value as fp16 of the
// scaled sum times a power of two f_j (planes of Pp >= P values, Pp a
// multiple of 256, so whole tiles are stored without a bound check), and
// the last block derives the map of those stored values: q = floor(h s' + o)
// with s' = s / f_j exact, and a bound on how far the stored values move
// the argument of the floor (rounding to fp16: 2^-11 relative, 2^-25
// absolute below fp16's normal range; FP32 rounding of the map).  If the
// bound exceeds h.limit for some component, or a stored value could have
// overflowed, the flag in range_dev[32] tells pass 2 to re-read the page.
template <int NKB, int G2, bool H16>
__global__ __launch_bounds__(kBlock, NKB <= 5 ? 2 : 1) void k_range_u16(const void* __restrict__ cube, int B, int64_t P, int nc,
                                                      ProjArgs a, float* __restrict__ part,
                                                      unsigned* __restrict__ ticket, float* __restrict__ range_dev,
                                                      float* __restrict__ ab_dev, H16Args h,
                                                      _Float16* __restrict__ planes, int64_t Pp) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ float wred[kWaves][16];
  __shared__ bool am_last;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, p = (lane & 15) >> 3, jc = lane & 7;
  const bool live = p < G2 && jc < nc;
  constexpr int RB = row_blocks<NKB>();
  ProjArgs& sa = *reinterpret_cast<ProjArgs*>(lds);   // set-up only: the tiles reuse it
  stage_args(a, sa);
  __shared__ OpsTab<NKB> tab;
  const float acc0 = build_ops<NKB, G2>(sa, B, nc, tab);
  const float inv = 1.f / sa.scale[threadIdx.x & 7];   // a power of two: exact
  __syncthreads();
  const float hf = H16 ? h.f[jc] : 0.f;
  float mn = __builtin_inff(), mx = -__builtin_inff();
  // the wave's LDS slice: the tile, then (once the tile has been read) the
  // tile's fp16 values, plane by plane, so that each plane's run of
  // TPX = 16 RB G2 values leaves with 16-byte stores of whole 128-byte lines
  constexpr int TPX = 16 * RB * G2, PW = staged_row_dwords<NKB>(G2), LPP = TPX / 8, PPI = 64 / LPP;
  uint32_t* stg = lds + w * slice_dwords<NKB>(G2 == 2 ? B : B / 2, G2);
  run_tiles<NKB, G2>(cube, B, P, tab, acc0, lds, [&](int64_t t, const f32x4 (&acc)[RB]) {
    const int64_t pb = t * TPX;
    if constexpr (H16) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        int64_t px;
        const f32x4 v = four_pixels<G2>(acc[rb], g, p, rb, pb, &px);
        const uint32_t lo = h16((_Float16)(v[0] * hf)) | (h16((_Float16)(v[1] * hf)) << 16);
        const uint32_t hi = h16((_Float16)(v[2] * hf)) | (h16((_Float16)(v[3] * hf)) << 16);
        if (live) *reinterpret_cast<u32x2*>(stg + jc * PW + (int)(px - pb) / 2) = u32x2{lo, hi};
      }
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < 8 / PPI; ++i) {
        const int q = i * PPI + lane / LPP, c = lane % LPP;
        if (q < nc)
          __builtin_nontemporal_store(*reinterpret_cast<const u32x4*>(stg + q * PW + 4 * c),
                                      reinterpret_cast<u32x4*>(planes + (int64_t)q * Pp + pb + 8 * c));
      }
    }
    if (pb + 16 * RB * G2 <= P) {   // whole tile: every row is a pixel
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          mn = fminf(mn, acc[rb][e]);
          mx = fmaxf(mx, acc[rb][e]);
        }
    } else {
      const int left = (int)(P - pb);   // pixels of the tile inside the page
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if ((16 * rb + 4 * g + e) * G2 + p < left) {
            mn = fminf(mn, acc[rb][e]);
            mx = fmaxf(mx, acc[rb][e]);
          }
    }
  });
  // lanes holding the same component: l ^ 8 (other pixel of the row, if
  // any), l ^ 16, l ^ 32 (other rows)
  if (G2 == 2) {
    mn = fminf(mn, __shfl_xor(mn, 8, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 8, 64));
  }
  mn = fminf(mn, __shfl_xor(mn, 16, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
  mn = fminf(mn, __shfl_xor(mn, 32, 64));
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  if (lane < 8) {
    wred[w][lane] = mn;
    wred[w][8 + lane] = mx;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int j = threadIdx.x;
    float lo = wred[0][j], hi = wred[0][8 + j];
    for (int ww = 1; ww < kWaves; ++ww) {
      lo = fminf(lo, wred[ww][j]);
      hi = fmaxf(hi, wred[ww][8 + j]);
    }
    part[(int64_t)blockIdx.x * 16 + j] = lo;
    part[(int64_t)blockIdx.x * 16 + 8 + j] = hi;
    __threadfence();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    am_last = (atomicAdd(ticket, 1u) == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  // last block: thread (slice, component) folds a strided subset of partials
  const int j = threadIdx.x & 7, sl = threadIdx.x >> 3;
  float lo = __builtin_inff(), hi = -__builtin_inff();
  for (unsigned bk = sl; bk < gridDim.x; bk += kBlock / 8) {
    lo = fminf(lo, __builtin_nontemporal_load(part + (int64_t)bk * 16 + j));
    hi = fmaxf(hi, __builtin_nontemporal_load(part + (int64_t)bk * 16 + 8 + j));
  }
  lo = fminf(lo, __shfl_xor(lo, 8, 64));
  hi = fmaxf(hi, __shfl_xor(hi, 8, 64));
  lo = fminf(lo, __shfl_xor(lo, 16, 64));
  hi = fmaxf(hi, __shfl_xor(hi, 16, 64));
  lo = fminf(lo, __shfl_xor(lo, 32, 64));
  hi = fmaxf(hi, __shfl_xor(hi, 32, 64));
  __syncthreads();
  if (lane < 8) {
    wred[w][lane] = lo;
    wred[w][8 + lane] = hi;
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    const int jj = threadIdx.x;
    float l2 = wred[0][jj], h2 = wred[0][8 + jj];
    for (int ww = 1; ww < kWaves; ++ww) {
      l2 = fminf(l2, wred[ww][jj]);
      h2 = fmaxf(h2, wred[ww][8 + jj]);
    }
    float s, o;
    stretch_map(l2, h2, 255.f, s, o);
    range_dev[jj] = s;
    range_dev[8 + jj] = o;
    ab_dev[2 * jj] = l2 * inv;
    ab_dev[2 * jj + 1] = h2 * inv;
    if constexpr (H16) wred[0][jj] = stored_map(l2, h2, s, o, h.f[jj], h.limit, jj, range_dev) ? 1.f : 0.f;
  }
  if constexpr (H16) {
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned flag = 0u;
      for (int jj = 0; jj < nc; ++jj) flag |= wred[0][jj] != 0.f ? 1u : 0u;
      reinterpret_cast<unsigned*>(range_dev)[32] = flag;
    }
  }
  if (threadIdx.x == 0) *ticket = 0u;
}

__device__ __forceinline__ uint32_t quant(float y, float s, float o) {
  float t = floorf(fmaf(y, s, o));
  t = fminf(fmaxf(t, 0.f), 255.f);
  return (uint32_t)t;
}

// Pass 2 from the page: the quantised bytes of a wave tile are gathered per
// component plane in LDS (8 planes x the tile's pixels, in the wave's own
// tile slice) and written as 16-byte chunks, so each plane receives whole
// segments.
template <int NKB, int G2>
__device__ __forceinline__ void stretch_page(const void* __restrict__ cube, int B, int64_t P, int nc,
                                             const ProjArgs& a, const float* __restrict__ range_dev,
                                             uint8_t* __restrict__ images, uint32_t* __restrict__ lds) {
  constexpr int RB = row_blocks<NKB>();
  constexpr int TP = 16 * RB * G2;   // pixels per wave tile
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15, p = col >> 3, j = col & 7;
  const bool live = p < G2 && j < nc;
  const bool writer = p == 0 && j < nc;
  ProjArgs& sa = *reinterpret_cast<ProjArgs*>(lds);   // set-up only: the tiles reuse it
  stage_args(a, sa);
  __shared__ OpsTab<NKB> tab;
  const float acc0 = build_ops<NKB, G2>(sa, B, nc, tab);
  __syncthreads();
  const float sc = live ? range_dev[j] : 0.f;
  const float of = live ? range_dev[8 + j] : 0.f;
  // the output bytes of a tile are staged in the wave's own LDS slice,
  // whose tile data is all in registers by then
  const int S = G2 == 2 ? B : B / 2;
  uint8_t* ow = reinterpret_cast<uint8_t*>(lds + w * slice_dwords<NKB>(S, G2));
  const int jj = lane >> 3, cc = lane & 7;   // copy-out: plane jj, 16-byte chunk cc
  const bool copier = jj < nc && 16 * cc < TP;
  const bool aligned = (P % 16) == 0 && (reinterpret_cast<uintptr_t>(images) % 16) == 0;
  run_tiles<NKB, G2>(cube, B, P, tab, acc0, lds, [&](int64_t t, const f32x4 (&acc)[RB]) {
    const int64_t pb = t * TP;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const uint32_t mine = quant(acc[rb][0], sc, of) | (quant(acc[rb][1], sc, of) << 8) |
                            (quant(acc[rb][2], sc, of) << 16) | (quant(acc[rb][3], sc, of) << 24);
      if constexpr (G2 == 2) {
        // even pixels of rows 16 rb + 4 g + e here, odd ones in lane ^ 8
        const uint32_t other = __shfl_xor(mine, 8, 64);
        if (writer) {
          const uint32_t lo = __builtin_amdgcn_perm(other, mine, 0x05010400u);
          const uint32_t hi = __builtin_amdgcn_perm(other, mine, 0x07030602u);
          *reinterpret_cast<uint2*>(ow + TP * j + 2 * (16 * rb + 4 * g)) = make_uint2(lo, hi);
        }
      } else {
        if (writer) *reinterpret_cast<uint32_t*>(ow + TP * j + 16 * rb + 4 * g) = mine;
      }
    }
    wave_lds_sync();
    if (copier) {
      const int64_t px = pb + 16 * cc;
      const u32x4 v = *reinterpret_cast<const u32x4*>(ow + TP * jj + 16 * cc);
      uint8_t* dst = images + (int64_t)jj * P + px;
      if (aligned && px + 16 <= P) {
        *reinterpret_cast<u32x4*>(dst) = v;
      } else {
        for (int e = 0; e < 16; ++e)
          if (px + e < P) dst[e] = (uint8_t)(v[e >> 2] >> (8 * (e & 3)));
      }
    }
  });
}

template <int NKB, int G2>
__global__ __launch_bounds__(kBlock, NKB <= 5 ? 2 : 1) void k_stretch_u16(const void* __restrict__ cube, int B,
                                                                        int64_t P, int nc, ProjArgs a,
                                                                        const float* __restrict__ range_dev,
                                                                        uint8_t* __restrict__ images) {
  extern __shared__ __align__(16) uint32_t lds[];
  stretch_page<NKB, G2>(cube, B, P, nc, a, range_dev, images, lds);
}

// Pass 2 after a pass 1 that stored fp16 planes: from the planes, unless
// pass 1 found their error bound too large for some component (a flag
// uniform over the grid), then from the page as k_stretch_u16.
template <int NKB, int G2>
__global__ __launch_bounds__(kBlock, NKB <= 5 ? 2 : 1) void k_stretch_h16(const void* __restrict__ cube, int B,
                                                                        int64_t P, int nc, ProjArgs a,
                                                                        const float* __restrict__ range_dev,
                                                                        const _Float16* __restrict__ planes,
                                                                        int64_t Pp, uint8_t* __restrict__ images) {
  extern __shared__ __align__(16) uint32_t lds[];
  if (reinterpret_cast<const unsigned*>(range_dev)[32] != 0u) {
    stretch_page<NKB, G2>(cube, B, P, nc, a, range_dev, images, lds);
    return;
  }
  stretch_stored(planes, Pp, P, nc, range_dev, images);
}

// The FP32 component planes, scaled back by 2^-s_j (exact), so they hold
// the very values whose min/max and stretch the two passes above take.
// Lane (g, p, j) ends with 4 consecutive pixels of plane j per row block:
// for two-pixel rows the partner lane l ^ 8 holds the other pixel of each
// row, and the two lanes swap halves so that each writes a 16-byte run.
template <int NKB, int G2>
__global__ __launch_bounds__(kBlock, NKB <= 5 ? 2 : 1) void k_float_u16(const void* __restrict__ cube, int B,
                                                                      int64_t P, int nc, ProjArgs a,
                                                                      float* __restrict__ y) {
  extern __shared__ __align__(16) uint32_t lds[];
  constexpr int RB = row_blocks<NKB>();
  constexpr int TP = 16 * RB * G2;   // pixels per wave tile
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15, p = col >> 3, j = col & 7;
  const bool live = p < G2 && j < nc;
  ProjArgs& sa = *reinterpret_cast<ProjArgs*>(lds);   // set-up only: the tiles reuse it
  stage_args(a, sa);
  __shared__ OpsTab<NKB> tab;
  const float acc0 = build_ops<NKB, G2>(sa, B, nc, tab);
  const float inv = 1.f / sa.scale[j];   // a power of two: exact
  __syncthreads();
  float* plane = y + (int64_t)(live ? j : 0) * P;
  const bool aligned = (P & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0;
  run_tiles<NKB, G2>(cube, B, P, tab, acc0, lds, [&](int64_t t, const f32x4 (&acc)[RB]) {
    const int64_t pb = t * TP;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      f32x4 v;
      int64_t px;
      if constexpr (G2 == 2) {
        // this lane: pixel p of rows 4 g + e; send the partner the two rows it writes
        const float s0 = p == 0 ? acc[rb][2] : acc[rb][0];
        const float s1 = p == 0 ? acc[rb][3] : acc[rb][1];
        const float r0 = __shfl_xor(s0, 8, 64), r1 = __shfl_xor(s1, 8, 64);
        v = p == 0 ? f32x4{acc[rb][0], r0, acc[rb][1], r1} : f32x4{r0, acc[rb][2], r1, acc[rb][3]};
        px = pb + 2 * (16 * rb + 4 * g) + 4 * p;
      } else {
        v = acc[rb];
        px = pb + 16 * rb + 4 * g;
      }
      v *= inv;
      if (live) {
        if (aligned && px + 3 < P) {
          *reinterpret_cast<f32x4*>(plane + px) = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (px + e < P) plane[px + e] = v[e];
        }
      }
    }
  });
}

// LDS: the wave slices plus 8 dwords that the last row's reads may reach;
// at least one ProjArgs, which set-up stages there.
template <int NKB, int G2>
size_t smem(int B) {
  const int S = G2 == 2 ? B : B / 2;
  const size_t tiles = ((size_t)kWaves * slice_dwords<NKB>(S, G2) + 8) * 4;
  return std::max(tiles, sizeof(ProjArgs));
}

// Blocks of one resident round (at most max_per_cu per CU), at most
// nblocks, and no more than the page has wave tiles for.
int grid(const void* kernel, size_t sm, int nblocks, int64_t P, int B, int rows, int max_per_cu = 1 << 20) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, sm) != hipSuccess || per < 1)
    per = 1, ncu = 1;
  per = std::min(per, max_per_cu);
  const int64_t tp = (int64_t)rows * ((B & 1) ? 2 : 1);
  const int64_t waves = (P + tp - 1) / tp;
  int64_t n = std::min<int64_t>((int64_t)per * ncu, nblocks);
  n = std::min<int64_t>(n, (waves + kWaves - 1) / kWaves);
  return (int)std::max<int64_t>(n, 1);
}

template <int NKB, int G2, bool H16>
hipError_t range_k(const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks, float* part,
                   unsigned* ticket, float* range_dev, float* ab_dev, const H16Args& h, _Float16* planes,
                   int64_t Pp, hipStream_t s) {
  const size_t sm = smem<NKB, G2>(B);
  const void* k = reinterpret_cast<const void*>(&k_range_u16<NKB, G2, H16>);
  // the storing pass fits three blocks per CU but runs faster at two
  // (0.605 against 0.640 ms on the 7216 x 5412 x 33 page at 7 components)
  const int nb = grid(k, sm, nblocks, P, B, 16 * row_blocks<NKB>(), H16 ? 2 : 1 << 20);
  hipLaunchKernelGGL((k_range_u16<NKB, G2, H16>), dim3(nb), dim3(kBlock), sm, s, cube, B, P, nc, a, part, ticket,
                     range_dev, ab_dev, h, planes, Pp);
  return hipGetLastError();
}

template <int NKB, int G2>
hipError_t stretch_k(const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks,
                     const float* range_dev, uint8_t* images, hipStream_t s) {
  const size_t sm = smem<NKB, G2>(B);
  const void* k = reinterpret_cast<const void*>(&k_stretch_u16<NKB, G2>);
  const int nb = grid(k, sm, nblocks, P, B, 16 * row_blocks<NKB>());
  hipLaunchKernelGGL((k_stretch_u16<NKB, G2>), dim3(nb), dim3(kBlock), sm, s, cube, B, P, nc, a, range_dev,
                     images);
  return hipGetLastError();
}

template <int NKB, int G2>
hipError_t stretch_h16_k(const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks,
                         const float* range_dev, const _Float16* planes, int64_t Pp, uint8_t* images,
                         hipStream_t s) {
  const size_t sm = smem<NKB, G2>(B);
  const void* k = reinterpret_cast<const void*>(&k_stretch_h16<NKB, G2>);
  const int nb = grid(k, sm, nblocks, P, B, 16 * row_blocks<NKB>());
  hipLaunchKernelGGL((k_stretch_h16<NKB, G2>), dim3(nb), dim3(kBlock), sm, s, cube, B, P, nc, a, range_dev,
                     planes, Pp, images);
  return hipGetLastError();
}

template <int NKB, int G2>
hipError_t float_k(const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks, float* y,
                   hipStream_t s) {
  const size_t sm = smem<NKB, G2>(B);
  const void* k = reinterpret_cast<const void*>(&k_float_u16<NKB, G2>);
  const int nb = grid(k, sm, nblocks, P, B, 16 * row_blocks<NKB>());
  hipLaunchKernelGGL((k_float_u16<NKB, G2>), dim3(nb), dim3(kBlock), sm, s, cube, B, P, nc, a, y);
  return hipGetLastError();
}

}  // namespace

// NKB = ceil(S / 8) K-blocks for S dwords per row (S = B for odd B, else B / 2).
#define CVX_U16_SWITCH(CALL)                                  \
  const int S = (B & 1) ? B : B / 2;                          \
  const int nkb = (S + 7) / 8;                                \
  if (B & 1) {                                                \
    switch (nkb) {                                            \
      case 1: return CALL(1, 2); case 2: return CALL(2, 2);   \
      case 3: return CALL(3, 2); case 4: return CALL(4, 2);   \
      case 5: return CALL(5, 2); case 6: return CALL(6, 2);   \
      case 7: return CALL(7, 2); case 8: return CALL(8, 2);   \
    }                                                         \
  } else {                                                    \
    switch (nkb) {                                            \
      case 1: return CALL(1, 1); case 2: return CALL(2, 1);   \
      case 3: return CALL(3, 1); case 4: return CALL(4, 1);   \
    }                                                         \
  }                                                           \
  return hipErrorInvalidValue;

hipError_t launch_project_range_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks,
                                    float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                    hipStream_t s) {
  if (B < 1 || B > kMaxB || nc < 1 || nc > 8) return hipErrorInvalidValue;
  const H16Args h{};
#define CVX_R(N, G) range_k<N, G, false>(cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, h, nullptr, 0, s)
  CVX_U16_SWITCH(CVX_R)
#undef CVX_R
}

hipError_t launch_project_range_h16_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                        int nblocks, float* part, unsigned* ticket, float* range_dev,
                                        float* ab_dev, const H16Args& h, uint16_t* planes16, int64_t Pp,
                                        hipStream_t s) {
  if (B < 1 || B > kMaxB || nc < 1 || nc > 8 || Pp < P || Pp % 256 != 0) return hipErrorInvalidValue;
  _Float16* planes = reinterpret_cast<_Float16*>(planes16);
#define CVX_R(N, G) range_k<N, G, true>(cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, h, planes, Pp, s)
  CVX_U16_SWITCH(CVX_R)
#undef CVX_R
}

hipError_t launch_project_stretch_h16_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                          int nblocks, const float* range_dev, const uint16_t* planes16, int64_t Pp,
                                          uint8_t* images, hipStream_t s) {
  if (B < 1 || B > kMaxB || nc < 1 || nc > 8 || Pp < P || Pp % 256 != 0) return hipErrorInvalidValue;
  const _Float16* planes = reinterpret_cast<const _Float16*>(planes16);
#define CVX_S(N, G) stretch_h16_k<N, G>(cube, B, P, nc, a, nblocks, range_dev, planes, Pp, images, s)
  CVX_U16_SWITCH(CVX_S)
#undef CVX_S
}

hipError_t launch_project_stretch_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                      int nblocks, const float* range_dev, uint8_t* images, hipStream_t s) {
  if (B < 1 || B > kMaxB || nc < 1 || nc > 8) return hipErrorInvalidValue;
#define CVX_S(N, G) stretch_k<N, G>(cube, B, P, nc, a, nblocks, range_dev, images, s)
  CVX_U16_SWITCH(CVX_S)
#undef CVX_S
}

hipError_t launch_project_float_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks,
                                    float* y, hipStream_t s) {
  if (B < 1 || B > kMaxB || nc < 1 || nc > 8) return hipErrorInvalidValue;
#define CVX_F(N, G) float_k<N, G>(cube, B, P, nc, a, nblocks, y, s)
  CVX_U16_SWITCH(CVX_F)
#undef CVX_F
}

#undef CVX_U16_SWITCH

}  // namespace cvx

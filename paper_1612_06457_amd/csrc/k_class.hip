// Class moments of the training pixels (paper Section 2, canonical
// variates: within- and between-class scatter from per-class sums and
// products).  Per class k, the augmented Gram of [x - c_k, 1] over the
// class's pixels, either in FP32 register tiles flushed to FP64 after every
// chunk (plain path) or on the matrix cores with the compensated split of
// k_split.hpp.  Block partials use the packed upper-triangular 4 x 4 tile
// layout and are combined by the fixed-order FP64 reduction.
//
// Gather.  The pixels of class k are listed, in raster order, in
// idx[offsets[k] ..); block g of the class takes chunks g, g + G, ... of
// kChunk = 128 rows.  A row (B elements, `rowbytes` bytes) lies inside NQ
// aligned 8-byte words; the block loads all kChunk NQ words of a chunk in
// one branch-free round of 8-byte loads (a word that is not wholly inside
// the page is read from a dummy location instead and replaced by the page's
// trailing bytes or by zero), stores them in LDS and reads its elements
// from there.  The words of the next chunk and the row indices of the one
// after it are in flight while the current chunk is accumulated.
//
// Shift.  c_k is the mean of the class's first min(64, n) pixels, rounded to
// the element type for 16-bit pages (so x - c_k is exact), summed in a fixed
// order by every block of the class, so all blocks agree bit for bit.  The
// host removes the shift exactly from the augmented Gram.
#include "k_gram.hpp"
#include "k_split.hpp"
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {

namespace {

struct Gather {
  const unsigned char* base;    // page
  const unsigned char* dummy;   // any readable 8-byte location
  int64_t total;                // page bytes
  int64_t tail_at;              // start of the word that straddles the end (total rounded down to 8)
  uint64_t tail;                // the page's bytes from tail_at, zero padded
  int rowbytes, esize, NQ;
};

// Words of a row: from its byte offset rounded down to 8, to cover
// rowbytes + 6 bytes.
__host__ __device__ inline int words_per_row(int rowbytes) { return (rowbytes + 6 + 7) / 8; }

// Issue the loads of the chunk whose rows are the pixels rp[0 .. kChunk)
// (-1: no pixel).  Thread item u is word i = threadIdx.x + kBlock u of the
// chunk (row i / NQ, word i % NQ).  bad / strad flag the items not loaded
// from the page and the one that straddles its end.
template <int UM>
__device__ __forceinline__ void gather_issue(const Gather& g, const int* __restrict__ rp, u32x2 (&v)[UM],
                                             uint32_t& bad, uint32_t& strad) {
  bad = 0u;
  strad = 0u;
#pragma unroll
  for (int u = 0; u < UM; ++u) {
    const int i = threadIdx.x + kBlock * u;
    const int row = i / g.NQ, q = i - row * g.NQ;
    const int p = row < kChunk ? rp[row] : -1;
    const int64_t qa = p >= 0 ? (((int64_t)p * g.rowbytes) & ~7LL) + 8 * q : 0;
    const bool ok = p >= 0 && qa + 8 <= g.total;
    v[u] = *reinterpret_cast<const u32x2*>(ok ? g.base + qa : g.dummy);
    bad |= (ok ? 0u : 1u) << u;
    strad |= (p >= 0 && !ok && qa == g.tail_at) ? (1u << u) : 0u;
  }
}

template <int UM>
__device__ __forceinline__ void gather_store(const Gather& g, const u32x2 (&v)[UM], uint32_t bad, uint32_t strad,
                                             u32x2* __restrict__ stg) {
  const u32x2 tail = {(uint32_t)g.tail, (uint32_t)(g.tail >> 32)};
  const u32x2 zero = {0u, 0u};
#pragma unroll
  for (int u = 0; u < UM; ++u) {
    const int i = threadIdx.x + kBlock * u;
    if (i < kChunk * g.NQ) stg[i] = ((bad >> u) & 1u) ? (((strad >> u) & 1u) ? tail : zero) : v[u];
  }
}

// Element b of staged row r (byte offset of the row inside its first word: ro).
template <int DT>
__device__ __forceinline__ float staged(const u32x2* __restrict__ stg, int NQ, int r, int ro, int b) {
  const unsigned char* row = reinterpret_cast<const unsigned char*>(stg + r * NQ) + ro;
  if constexpr (DT == DT_F32) {
    return *reinterpret_cast<const float*>(row + 4 * b);
  } else {
    return to_float<DT>(*reinterpret_cast<const uint16_t*>(row + 2 * b));
  }
}

// The raw 16-bit element b of staged row r.
__device__ __forceinline__ uint32_t staged_u16(const u32x2* __restrict__ stg, int NQ, int r, int ro, int b) {
  const unsigned char* row = reinterpret_cast<const unsigned char*>(stg + r * NQ) + ro;
  return *reinterpret_cast<const uint16_t*>(row + 2 * b);
}

template <int DT>
__device__ __forceinline__ float round_elem(float c) {
  return round_shift<DT>(c);
}

// Row index of row `tid` of chunk ch (-1 beyond the class); the load is
// unconditional (index clamped into the class, n >= 1).
__device__ __forceinline__ int row_pixel(const int32_t* __restrict__ idx, int off, int n, int nch, int ch, int tid) {
  const int pos = ch * kChunk + tid;
  const int v = idx[off + min(max(pos, 0), n - 1)];
  return (tid < kChunk && ch < nch && pos < n) ? v : -1;
}

// The shared driver: shift, then the chunk pipeline; consume(rp, ro) runs
// on each staged chunk with rp = its row pixels and ro = their row offsets
// (both in LDS) after a block barrier, and must end with one.
template <int DT, int UM, typename Consume>
__device__ __forceinline__ void class_rows(const void* __restrict__ cube, int B, int64_t P,
                                           const int32_t* __restrict__ idx, int off, int n, int G,
                                           const void* dummy, u32x2* __restrict__ stg, float* __restrict__ cs,
                                           double* __restrict__ shift_out, Consume consume) {
  __shared__ int ridx[2][kChunk];
  __shared__ int roff[kChunk];
  __shared__ uint64_t tail_sh;
  const int tid = threadIdx.x;
  const int k = blockIdx.y, g = blockIdx.x;
  Gather gt;
  gt.base = reinterpret_cast<const unsigned char*>(cube);
  gt.dummy = reinterpret_cast<const unsigned char*>(dummy);
  gt.esize = DT == DT_F32 ? 4 : 2;
  gt.rowbytes = B * gt.esize;
  gt.total = P * gt.rowbytes;
  gt.tail_at = gt.total & ~7LL;
  gt.NQ = words_per_row(gt.rowbytes);
  if (tid == 0) {
    uint64_t t = 0;
    for (int64_t o = gt.tail_at; o < gt.total; o += 2)
      t |= (uint64_t)(*reinterpret_cast<const uint16_t*>(gt.base + o)) << (8 * (o - gt.tail_at));
    tail_sh = t;
  }
  const int ns = n < 64 ? n : 64;
  if (tid < kChunk) ridx[0][tid] = tid < ns ? idx[off + tid] : -1;
  __syncthreads();
  gt.tail = tail_sh;
  u32x2 v[UM];
  uint32_t bad, strad;
  gather_issue<UM>(gt, ridx[0], v, bad, strad);
  gather_store<UM>(gt, v, bad, strad, stg);
  if (tid < kChunk) roff[tid] = ridx[0][tid] >= 0 ? (int)(((int64_t)ridx[0][tid] * gt.rowbytes) & 7) : 0;
  __syncthreads();
  for (int b = tid; b < B; b += kBlock) {
    float s = 0.f;
    for (int r = 0; r < ns; ++r) s += staged<DT>(stg, gt.NQ, r, roff[r], b);
    const float c = round_elem<DT>(s / (float)ns);
    cs[b] = c;
    if (g == 0) shift_out[(int64_t)k * B + b] = (double)c;
  }
  const int nch = (n + kChunk - 1) / kChunk;
  int ch = g;
  const int first = row_pixel(idx, off, n, nch, ch, tid);
  __syncthreads();
  if (tid < kChunk) ridx[0][tid] = first;
  __syncthreads();
  gather_issue<UM>(gt, ridx[0], v, bad, strad);
  int iv = row_pixel(idx, off, n, nch, ch + G, tid);
  int cur = 0;
  for (; ch < nch; ch += G) {
    gather_store<UM>(gt, v, bad, strad, stg);
    if (tid < kChunk) {
      const int p = ridx[cur][tid];
      roff[tid] = p >= 0 ? (int)(((int64_t)p * gt.rowbytes) & 7) : 0;
      ridx[cur ^ 1][tid] = iv;
    }
    __syncthreads();
    gather_issue<UM>(gt, ridx[cur ^ 1], v, bad, strad);
    iv = row_pixel(idx, off, n, nch, ch + 2 * G, tid);
    __builtin_amdgcn_sched_barrier(0);   // keep the next chunk's loads ahead of the work
    consume(ridx[cur], roff);
    cur ^= 1;
  }
}

template <int DT, int UM>
__global__ __launch_bounds__(kBlock) void k_class_fp32(const void* __restrict__ cube, int B, int64_t P,
                                                       const int32_t* __restrict__ idx,
                                                       const int32_t* __restrict__ offsets, int G,
                                                       double* __restrict__ part, double* __restrict__ shift_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float cs[kMaxB];
  const int k = blockIdx.y, g = blockIdx.x;
  const int BP = (B + 1 + 3) & ~3;
  const int NQ = words_per_row(B * (DT == DT_F32 ? 4 : 2));
  u32x2* stg = reinterpret_cast<u32x2*>(smem);
  float* xs = reinterpret_cast<float*>(smem + (size_t)kChunk * NQ * 8);
  double* red = reinterpret_cast<double*>(smem);
  const int off = offsets[k];
  const int n = offsets[k + 1] - off;
  const TileAssign ta = assign_tiles(BP);
  float acc[16];
  double accd[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acc[e] = 0.f;
    accd[e] = 0.0;
  }
  if (n > 0) {
    const int rstep = kBlock / BP, bstep = kBlock % BP;
    class_rows<DT, UM>(cube, B, P, idx, off, n, G, part, stg, cs, shift_out,
                       [&](const int* __restrict__ rp, const int* __restrict__ ro) {
      int r = threadIdx.x / BP, b = threadIdx.x % BP;
      for (int e = threadIdx.x; e < kChunk * BP; e += kBlock) {
        float x = 0.f;
        const int p = rp[r];
        if (p >= 0) {
          if (b < B) x = staged<DT>(stg, NQ, r, ro[r], b) - cs[b];
          else if (b == B) x = 1.f;
        }
        xs[e] = x;
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
      __syncthreads();
    });
  }
  write_partial(ta, accd, red, part + ((int64_t)k * G + g) * ta.nblk * 16);
}

template <int DT, int SPLIT, int NRB, int UM>
__global__ __launch_bounds__(kBlock) void k_class_split(const void* __restrict__ cube, int B, int64_t P,
                                                        const int32_t* __restrict__ idx,
                                                        const int32_t* __restrict__ offsets, int G, float scale,
                                                        double* __restrict__ part, double* __restrict__ shift_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float cs[kMaxB];
  const int k = blockIdx.y, g = blockIdx.x;
  const int NQ = words_per_row(B * (DT == DT_F32 ? 4 : 2));
  u32x2* stg = reinterpret_cast<u32x2*>(smem);
  double* red = reinterpret_cast<double*>(smem);
  const int off = offsets[k];
  const int n = offsets[k + 1] - off;
  const int w = threadIdx.x >> 6;
  constexpr int NP = npairs(NRB);
  f32x4 acc[NP];
  double accd[NP][4];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[p][e] = 0.f;
      accd[p][e] = 0.0;
    }
  if (n > 0) {
    class_rows<DT, UM>(cube, B, P, idx, off, n, G, part, stg, cs, shift_out,
                       [&](const int* __restrict__ rp, const int* __restrict__ ro) {
      // wave w takes rows 32 w .. 32 w + 31 of the chunk
      auto get = [&](int r, int band) {
        float v = 0.f;
        if (rp[r] >= 0) {
          if (band < B) v = (staged<DT>(stg, NQ, r, ro[r], band) - cs[band]) * scale;
          else if (band == B) v = 1.f;
        }
        return v;
      };
      kstep<SPLIT, NRB>(get, 32 * w, acc);
      fold<NRB>(acc, accd);
      __syncthreads();
    });
  }
  __syncthreads();
  const int nb = (B + 4) / 4;
  block_combine<NRB>(accd, B, scale, red, part + ((int64_t)k * G + g) * (nb * (nb + 1) / 2 * 16));
}

// uint16 pages: the Gram of (x - c_k) / 1024 on the fp16 matrix units with
// operands built exactly by bit operations (U16Lane, k_split.hpp), summed as
// HH + HL + LH + LL and unscaled by 2^20 in FP64.  Same gather, shift and
// output layout as k_class_split; every product is exact.
// Three waves per SIMD where the registers allow it without spilling.
template <int NRB, int UM>
constexpr int class_u16_waves() { return ((NRB == 2 && UM <= 9) || (NRB == 3 && UM <= 5)) ? 3 : 1; }

template <int NRB, int UM>
__global__ __launch_bounds__(kBlock, (class_u16_waves<NRB, UM>())) void k_class_u16(const void* __restrict__ cube, int B, int64_t P,
                                                      const int32_t* __restrict__ idx,
                                                      const int32_t* __restrict__ offsets, int G,
                                                      double* __restrict__ part, double* __restrict__ shift_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float cs[kMaxB];
  const int k = blockIdx.y, g = blockIdx.x;
  const int NQ = words_per_row(B * 2);
  u32x2* stg = reinterpret_cast<u32x2*>(smem);
  double* red = reinterpret_cast<double*>(smem);
  const int off = offsets[k];
  const int n = offsets[k + 1] - off;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  constexpr int NP = npairs(NRB);
  f32x4 acc[NP];
  double accd[NP][4];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[p][e] = 0.f;
      accd[p][e] = 0.0;
    }
  if (n > 0) {
    const U16Masks mk = make_u16_masks();
    class_rows<DT_U16, UM>(cube, B, P, idx, off, n, G, part, stg, cs, shift_out,
                           [&](const int* __restrict__ rp, const int* __restrict__ ro) {
      U16Lane<NRB> ln;   // the class shift is in cs from the first chunk on
      ln.init(B, cs, col);
      // wave w takes rows 32 w .. 32 w + 31 of the chunk
      const int k0 = 32 * w;
      f16x8 Hv[NRB], Lv[NRB];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        u32x4 H, L;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = k0 + 8 * grp + 2 * u;
          const uint32_t d = staged_u16(stg, NQ, r, ro[r], ln.bcol[rb]) |
                             (staged_u16(stg, NQ, r + 1, ro[r + 1], ln.bcol[rb]) << 16);
          const uint32_t rm = (rp[r] >= 0 ? 0x0000ffffu : 0u) | (rp[r + 1] >= 0 ? 0xffff0000u : 0u);
          uint32_t h, l;
          ln.terms(d, rb, rm, mk, h, l);
          H[u] = h;
          L[u] = l;
        }
        Hv[rb] = __builtin_bit_cast(f16x8, H);
        Lv[rb] = __builtin_bit_cast(f16x8, L);
      }
      u16_tile_products<NRB>(Hv, Lv, acc);
      fold<NRB>(acc, accd);
      __syncthreads();
    });
  }
  __syncthreads();
  const int nb = (B + 4) / 4;
  block_combine<NRB>(accd, B, 1.f / 1024.f, red, part + ((int64_t)k * G + g) * (nb * (nb + 1) / 2 * 16));
}

// Loads per thread per chunk: ceil(kChunk NQ / kBlock), rounded up to an instantiated bound.
int um_for(int dtype, int B) {
  const int nq = words_per_row(B * (dtype == DT_F32 ? 4 : 2));
  const int u = (kChunk * nq + kBlock - 1) / kBlock;
  return u <= 3 ? 3 : u <= 5 ? 5 : u <= 9 ? 9 : 17;
}

size_t fp32_smem(int dtype, int B) {
  const int BP = (B + 1 + 3) & ~3, nb = BP / 4, nblk = nb * (nb + 1) / 2;
  const size_t nq = words_per_row(B * (dtype == DT_F32 ? 4 : 2));
  const size_t work = (size_t)kChunk * nq * 8 + (size_t)kChunk * BP * 4;
  const size_t red = (size_t)(kBlock / nblk) * nblk * 16 * 8;
  return std::max(work, red);
}

size_t split_smem(int dtype, int B) {
  const size_t nq = words_per_row(B * (dtype == DT_F32 ? 4 : 2));
  return std::max((size_t)kChunk * nq * 8, packed_doubles(B) * 8);
}

template <int DT>
hipError_t fp32_dt(int um, const void* cube, int B, int64_t P, const int32_t* idx, const int32_t* offsets, int K,
                   int G, double* part, double* shift_out, hipStream_t s) {
  const dim3 grid(G, K);
  const size_t sm = fp32_smem(DT, B);
#define CVX_C(U)                                                                                            \
  case U:                                                                                                   \
    hipLaunchKernelGGL((k_class_fp32<DT, U>), grid, dim3(kBlock), sm, s, cube, B, P, idx, offsets, G, part, \
                       shift_out);                                                                          \
    break;
  switch (um) { CVX_C(3) CVX_C(5) CVX_C(9) CVX_C(17) default: return hipErrorInvalidValue; }
#undef CVX_C
  return hipGetLastError();
}

template <int DT, int SPLIT, int NRB>
hipError_t split_nrb(int um, const void* cube, int B, int64_t P, const int32_t* idx, const int32_t* offsets,
                     int K, int G, double* part, double* shift_out, hipStream_t s) {
  const dim3 grid(G, K);
  const size_t sm = split_smem(DT, B);
  const float sc = prescale(DT, SPLIT);
#define CVX_C(U)                                                                                             \
  case U:                                                                                                    \
    hipLaunchKernelGGL((k_class_split<DT, SPLIT, NRB, U>), grid, dim3(kBlock), sm, s, cube, B, P, idx,       \
                       offsets, G, sc, part, shift_out);                                                     \
    break;
  switch (um) { CVX_C(3) CVX_C(5) CVX_C(9) CVX_C(17) default: return hipErrorInvalidValue; }
#undef CVX_C
  return hipGetLastError();
}

template <int DT, int SPLIT>
hipError_t split_dt(int um, const void* cube, int B, int64_t P, const int32_t* idx, const int32_t* offsets, int K,
                    int G, double* part, double* shift_out, hipStream_t s) {
  switch (nrb_for(B)) {
    case 2: return split_nrb<DT, SPLIT, 2>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case 3: return split_nrb<DT, SPLIT, 3>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    default: return split_nrb<DT, SPLIT, 5>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
  }
}

template <int NRB>
hipError_t u16_nrb(int um, const void* cube, int B, int64_t P, const int32_t* idx, const int32_t* offsets, int K,
                   int G, double* part, double* shift_out, hipStream_t s) {
  const dim3 grid(G, K);
  const size_t sm = split_smem(DT_U16, B);
#define CVX_C(U)                                                                                              \
  case U:                                                                                                     \
    hipLaunchKernelGGL((k_class_u16<NRB, U>), grid, dim3(kBlock), sm, s, cube, B, P, idx, offsets, G, part,   \
                       shift_out);                                                                            \
    break;
  switch (um) { CVX_C(3) CVX_C(5) CVX_C(9) CVX_C(17) default: return hipErrorInvalidValue; }
#undef CVX_C
  return hipGetLastError();
}

hipError_t u16_launch(const void* cube, int B, int64_t P, const int32_t* idx, const int32_t* offsets, int K, int G,
                      double* part, double* shift_out, hipStream_t s) {
  const int um = um_for(DT_U16, B);
  switch (nrb_for(B)) {
    case 2: return u16_nrb<2>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case 3: return u16_nrb<3>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    default: return u16_nrb<5>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
  }
}

template <int SPLIT>
hipError_t split_launch(int dtype, const void* cube, int B, int64_t P, const int32_t* idx, const int32_t* offsets,
                        int K, int G, double* part, double* shift_out, hipStream_t s) {
  const int um = um_for(dtype, B);
  switch (dtype) {
    // uint16 pages: the exact bit-built operands whatever split was asked
    case DT_U16: return u16_launch(cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case DT_F32: return split_dt<DT_F32, SPLIT>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case DT_BF16: return split_dt<DT_BF16, SPLIT>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case DT_F16: return split_dt<DT_F16, SPLIT>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_class_moments(int dtype, const void* cube, int B, int64_t P, const int32_t* idx,
                                const int32_t* offsets, int K, int G, double* part, double* shift_out,
                                hipStream_t s) {
  if (B < 1 || B > kMaxB || K < 1 || G < 1) return hipErrorInvalidValue;
  const int um = um_for(dtype, B);
  switch (dtype) {
    case DT_U16: return fp32_dt<DT_U16>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case DT_F32: return fp32_dt<DT_F32>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case DT_BF16: return fp32_dt<DT_BF16>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
    case DT_F16: return fp32_dt<DT_F16>(um, cube, B, P, idx, offsets, K, G, part, shift_out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_class_moments_mfma(int dtype, int split, const void* cube, int B, int64_t P, const int32_t* idx,
                                     const int32_t* offsets, int K, int G, double* part, double* shift_out,
                                     hipStream_t s) {
  if (B < 1 || B > kMaxB || K < 1 || G < 1) return hipErrorInvalidValue;
  if (split == 0) return split_launch<0>(dtype, cube, B, P, idx, offsets, K, G, part, shift_out, s);
  return split_launch<1>(dtype, cube, B, P, idx, offsets, K, G, part, shift_out, s);
}

}  // namespace cvx

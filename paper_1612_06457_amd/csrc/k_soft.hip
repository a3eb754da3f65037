// Soft-label CVA on the training pixels X (N x B float32) with real class
// weights w (N x K float32).  Not in the paper: with one-hot weights it is
// the paper's CVA (Section 2, canonical variates paragraph).
//
// Forward, two passes over X:
//   1. n_c = sum_p w_pc and t_c = sum_p w_pc x_p (w^T [X, 1] on the FP32 matrix instruction)
//      into block partials; the partials are combined by the fixed-order
//      reduction, and a one-block kernel stores the class means
//      m_c = t_c / n_c;
//   2. per class, the weighted augmented Gram of [x - m_c, 1]: sum w d d^T,
//      sum w d and sum w (d = x - float(m_c)) on the matrix cores (see
//      k_soft_scatter_mfma); the host removes the tiny offset between
//      float(m_c) and m_c exactly.
// Both passes stream chunks of kChunk rows of X and of w through a block-wide
// prefetching driver: the next chunk's 16-byte loads are in flight while the
// current chunk is accumulated.
// Backward: per pixel, u = x - m, z_j = w_j^T u for the C canonical
// vectors, and dJ/dw_pc = sum_j z_j^2 - sum_j (1 + lambda_j)(z_j - d_jc)^2
// with d_jc = w_j^T (m_c - m).
#include "k_gram.hpp"
#include "k_split.hpp"
#include "k_tile.hpp"
#include "launch.hpp"

namespace cvx {

typedef float f4v __attribute__((ext_vector_type(4)));

namespace {

// Chunks ch = first, first + stride, ... of X and w, staged raw in LDS
// (xr: kChunk B floats, wr: kChunk K floats), compute(ch, rows) per chunk
// after a block barrier; a barrier follows it.  QX, QW bound the 16-byte
// loads per thread of the two tiles.  With every > 1 only the chunks
// 0, every, 2 every, ... take part (chunk v of that sample is chunk
// v every of X and w); stride and first count sample chunks.
template <int QX, int QW, typename Compute>
__device__ __forceinline__ void for_each_chunk(const float* __restrict__ X, const float* __restrict__ W, int64_t N,
                                               int B, int K, int64_t first, int64_t stride,
                                               uint32_t* __restrict__ xr, uint32_t* __restrict__ wr,
                                               Compute compute, int64_t every = 1) {
  const int tid = threadIdx.x;
  const unsigned char* xb = reinterpret_cast<const unsigned char*>(X);
  const unsigned char* wb = reinterpret_cast<const unsigned char*>(W);
  const int xbytes = kChunk * B * 4, wbytes = kChunk * K * 4;
  const int64_t xtotal = N * B * 4, wtotal = N * K * 4;
  const int64_t nall = (N + kChunk - 1) / kChunk;
  const int64_t nch = (nall + every - 1) / every;   // sample chunks
  const int64_t nfull = N / kChunk;
  auto rows_of = [&](int64_t c) { return (int)(N - c * kChunk < kChunk ? N - c * kChunk : kChunk); };
  int64_t ch = first;
  if (nfull == 0) {
    for (; ch < nch; ch += stride) {
      copy_partial_tile<kBlock>(xb, xtotal, ch * every, xbytes, tid, xr);
      copy_partial_tile<kBlock>(wb, wtotal, ch * every, wbytes, tid, wr);
      __syncthreads();
      compute(ch * every, rows_of(ch * every));
      __syncthreads();
    }
    return;
  }
  // the chunk to prefetch for sample chunk x (a whole one: past the end the
  // current, or the last whole chunk, whose loads are then not stored)
  auto next = [&](int64_t x, int64_t cur) {
    const int64_t a = x * every, c = cur * every;
    return x < nch && a < nfull ? a : (c < nfull ? c : nfull - 1);
  };
  u32x4 rx[QX], rw[QW];
  load_tile<QX, kBlock, false>(xb, next(ch, ch), xbytes, tid, rx);
  load_tile<QW, kBlock, false>(wb, next(ch, ch), wbytes, tid, rw);
  for (; ch < nch; ch += stride) {
    const int64_t a = ch * every;
    if (a < nfull) {
      store_tile<QX, kBlock>(xr, xbytes, tid, rx);
      store_tile<QW, kBlock>(wr, wbytes, tid, rw);
    } else {
      copy_partial_tile<kBlock>(xb, xtotal, a, xbytes, tid, xr);
      copy_partial_tile<kBlock>(wb, wtotal, a, wbytes, tid, wr);
    }
    __syncthreads();
    load_tile<QX, kBlock, false>(xb, next(ch + stride, ch), xbytes, tid, rx);
    load_tile<QW, kBlock, false>(wb, next(ch + stride, ch), wbytes, tid, rw);
    __builtin_amdgcn_sched_barrier(0);   // keep the next chunk's loads ahead of the work
    compute(a, rows_of(a));
    __syncthreads();
  }
}

__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Pass 1 on the FP32 matrix instruction (v_mfma_f32_16x16x4_f32, FP32
// operands and products, as on the vector ALU): per 4 rows,
// C[c][j] += sum_r w[r][c] [x_r, 1][j] with A = w (lane: class 16 cb + l % 16,
// row l / 16) and B = [X, 1] (lane: column 16 rb + l % 16, same row).  Wave
// v takes rows 32 v .. 32 v + 31 of each chunk; its FP32 tiles fold into
// FP64 after every chunk, and the waves of a block combine in a fixed order
// into the block partial [c][j], c < KP, j < BP.  Rows past N have zero
// weights (the partial chunk is zero-filled), so they add nothing.
template <int NCB, int NRB, int QX, int QW>
__global__ __launch_bounds__(kBlock) void k_soft_first(const float* __restrict__ X, const float* __restrict__ W,
                                                       int64_t N, int B, int K, int64_t every,
                                                       double* __restrict__ part) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* xr = lds;                 // kChunk x B raw rows of X
  uint32_t* wr = lds + kChunk * B;    // kChunk x K raw rows of w
  double* red = reinterpret_cast<double*>(lds);
  const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int BP = (B + 1 + 3) & ~3, KP = (K + 3) & ~3;
  int bcol[NRB], kcol[NCB];
  bool real[NRB], kreal[NCB];
  float onev[NRB];
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    const int band = 16 * rb + col;
    real[rb] = band < B;
    bcol[rb] = band < B ? band : 0;
    onev[rb] = band == B ? 1.f : 0.f;
  }
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int cl = 16 * cb + col;
    kreal[cb] = cl < K;
    kcol[cb] = cl < K ? cl : 0;
  }
  f32x4 acc[NCB][NRB];
  double accd[NCB][NRB][4];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[cb][rb][e] = 0.f;
        accd[cb][rb][e] = 0.0;
      }
  const float* xf = reinterpret_cast<const float*>(xr);
  const float* wf = reinterpret_cast<const float*>(wr);
  auto body = [&](int64_t, int) {
#pragma unroll
    for (int s = 0; s < kChunk / (4 * kWaves); ++s) {
      const int r = (kChunk / kWaves) * v + 4 * s + grp;
      float a[NCB], x[NRB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) a[cb] = kreal[cb] ? wf[r * K + kcol[cb]] : 0.f;
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) x[rb] = real[rb] ? xf[r * B + bcol[rb]] : onev[rb];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) acc[cb][rb] = mma_f32(a[cb], x[rb], acc[cb][rb]);
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          accd[cb][rb][e] += (double)acc[cb][rb][e];
          acc[cb][rb][e] = 0.f;
        }
  };
  for_each_chunk<QX, QW>(X, W, N, B, K, blockIdx.x, gridDim.x, xr, wr, body, every);
  // waves in a fixed order into the block partial [c][j]
  const int L = KP * BP;
  for (int t = threadIdx.x; t < L; t += kBlock) red[t] = 0.0;
  __syncthreads();
  for (int ww = 0; ww < kWaves; ++ww) {
    if (v == ww) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = 16 * cb + 4 * grp + e, j = 16 * rb + col;
            if (c < KP && j < BP) red[c * BP + j] += accd[cb][rb][e];
          }
    }
    __syncthreads();
  }
  double* mine = part + (int64_t)blockIdx.x * L;
  for (int t = threadIdx.x; t < L; t += kBlock) mine[t] = red[t];
}

// One block: from the reduced first moments (KP x BP, packed by class), the
// moments n_c, t_c per class (first[c][0..B]) and the shifts the scatter
// centres each class on, in FP32: the class means of those moments.  When
// the moments come from a sample of the pixels, a class whose weight in the
// sample is not positive or below 10^-6 of the largest takes the weighted
// mean of all classes instead (0 if the total weight is not positive).  Any
// shift is exact for the scatter, which carries sum w (x - s) and sum w;
// a shift close to the class mean only keeps its FP32 sums small.
__global__ __launch_bounds__(kBlock) void k_soft_means(int B, int K, const double* __restrict__ fp,
                                                       double* __restrict__ first, float* __restrict__ mc_f) {
  __shared__ double tot[kMaxB + 1];
  __shared__ double nmax;
  const int BP = (B + 1 + 3) & ~3;
  for (int t = threadIdx.x; t < K * (B + 1); t += kBlock) first[t] = fp[(t / (B + 1)) * BP + t % (B + 1)];
  for (int b = threadIdx.x; b <= B; b += kBlock) {
    double v = 0.0;
    for (int c = 0; c < K; ++c) v += fp[c * BP + b];
    tot[b] = v;
  }
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int c = 0; c < K; ++c) m = fmax(m, fp[c * BP + B]);
    nmax = m;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < K * B; t += kBlock) {
    const int c = t / B, b = t % B;
    const double n = fp[c * BP + B];
    if (n > 0.0 && n >= 1e-6 * nmax) mc_f[t] = (float)(fp[c * BP + b] / n);
    else mc_f[t] = tot[B] > 0.0 ? (float)(tot[b] / tot[B]) : 0.f;
  }
}

// Pass 2 on the matrix cores, grid (G, ceil(K / (4 CPW))): block (g, q)
// takes chunks g, g + G, ... of X and w (through the prefetching driver) and
// its wave v the classes c = 4 CPW q + 4 u + v, u < CPW.  The weighted Gram of d = [x - m_c, 1] is
// sum_p a_p d_p^T with a = w_pc d, accumulated with the FP32 matrix
// instruction v_mfma_f32_16x16x4_f32: FP32 operands, FP32 products and
// accumulation, so the arithmetic is that of the plain FP32 path; the FP32
// tiles fold into FP64 after every chunk.  Operand layout: lane l holds
// pixel k0 + l / 16 and band 16 r + l % 16 of both operands (A[i][k] and
// B[k][j]); the output tile as for the other MFMA shapes (rows
// 4 (l / 16) + e, column l % 16).  Rows past N have zero weights (the partial
// chunk is zero-filled), so they add nothing.  Each wave writes its classes'
// partials in the packed layout of the fixed-order reduction.

// Tail columns.  When B + 1 = 16 NRB + T with T = 1 or 2, the matrix cores
// take the 16 NRB leading columns and the vector ALU the T trailing ones:
// the ones column (T = 1), or the last band and the ones column (T = 2).
// Each lane then also accumulates, for its band j and pixel row,
// sum w d_j (the ones column), for T = 2 sum w d_t d_j with t = B - 1, and
// the corner sums sum w, sum w d_t, sum w d_t^2.  At 33 bands this halves
// the matrix instructions (three tile pairs instead of six per 4 rows) for
// a few vector ones.  The tail sums fold into FP64 after every chunk like the
// tiles, and the four row groups of a wave combine at the end in a fixed
// order.  T = 0: the ones column is a column of the last row block.
//
// Classes per wave: CPW = 2 lets one pass over the chunk serve eight
// classes (two per wave) where the registers allow it, so the training
// pixels are read once for K <= 8 instead of once per group of four.
//
// Waves per SIMD: three where the registers allow it without spilling (at
// most 168 VGPRs), else two or one.
template <int NRB, int QX, int T, int CPW>
constexpr int scatter_waves() {
  if (CPW == 2) return 2;
  return (NRB <= 1 || (NRB == 2 && (QX == 5 || T < 2)) || (NRB == 3 && QX == 5 && T == 0)) ? 3
         : (NRB == 2 ? 2 : 1);
}

template <int NRB, int QX, int QW, int T, int CPW>
__global__ __launch_bounds__(kBlock, (scatter_waves<NRB, QX, T, CPW>())) void k_soft_scatter_mfma(
    const float* __restrict__ X, const float* __restrict__ W, int64_t N, int B, int K,
    const float* __restrict__ mc_f, double* __restrict__ part) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* xr = lds;                 // kChunk x B raw rows of X
  uint32_t* wr = lds + kChunk * B;    // kChunk x K raw rows of w
  const int G = gridDim.x, g = blockIdx.x;
  const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  // wave v takes classes c[u] = blockIdx.y kWaves CPW + kWaves u + v
  int cls[CPW];
  bool live[CPW];
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    cls[u] = blockIdx.y * kWaves * CPW + kWaves * u + v;
    live[u] = cls[u] < K;
  }
  int bcol[NRB];
  float mrb[CPW][NRB], onev[NRB], mt[CPW];
  bool real[NRB];
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    const int band = 16 * rb + col;
    real[rb] = band < B;
    bcol[rb] = band < B ? band : 0;
    onev[rb] = band == B ? 1.f : 0.f;
#pragma unroll
    for (int u = 0; u < CPW; ++u) mrb[u][rb] = (live[u] && band < B) ? mc_f[cls[u] * B + band] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < CPW; ++u) mt[u] = (T == 2 && live[u]) ? mc_f[cls[u] * B + B - 1] : 0.f;
  constexpr int NP = npairs(NRB);
  f32x4 acc[CPW][NP];
  double accd[CPW][NP][4];
  // tail sums: ts = sum w d_j, te = sum w d_t d_j, and the corner tw, tst, ttt
  float ts[CPW][NRB], te[CPW][NRB], tw[CPW], tst[CPW], ttt[CPW];
  double tsd[CPW][NRB], ted[CPW][NRB], twd[CPW], tstd[CPW], tttd[CPW];
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[u][p][e] = 0.f;
        accd[u][p][e] = 0.0;
      }
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      ts[u][rb] = te[u][rb] = 0.f;
      tsd[u][rb] = ted[u][rb] = 0.0;
    }
    tw[u] = tst[u] = ttt[u] = 0.f;
    twd[u] = tstd[u] = tttd[u] = 0.0;
  }
  const float* xf = reinterpret_cast<const float*>(xr);
  const float* wf = reinterpret_cast<const float*>(wr);
  auto body = [&](int64_t, int) {
    if (!live[0]) return;
    constexpr int kUnroll = 4 / CPW;
#pragma unroll kUnroll
    for (int k0 = 0; k0 < kChunk; k0 += 4) {
      const int r = k0 + grp;
      float xv[NRB];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        if constexpr (T > 0) xv[rb] = xf[r * B + 16 * rb + col];   // every band is real
        else xv[rb] = real[rb] ? xf[r * B + bcol[rb]] : 0.f;
      }
      const float xt = T == 2 ? xf[r * B + B - 1] : 0.f;
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        if (u > 0 && !live[u]) break;
        const float wv = wf[r * K + cls[u]];
        float a[NRB], d[NRB];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          if constexpr (T > 0) d[rb] = xv[rb] - mrb[u][rb];
          else d[rb] = real[rb] ? xv[rb] - mrb[u][rb] : onev[rb];
          a[rb] = wv * d[rb];
        }
        if constexpr (T > 0) {
#pragma unroll
          for (int rb = 0; rb < NRB; ++rb) ts[u][rb] += a[rb];
          tw[u] += wv;
          if constexpr (T == 2) {
            const float dt = xt - mt[u];
            const float at = wv * dt;
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) te[u][rb] = fmaf(at, d[rb], te[u][rb]);
            tst[u] += at;
            ttt[u] = fmaf(at, dt, ttt[u]);
          }
        }
        int p = 0;
#pragma unroll
        for (int ri = 0; ri < NRB; ++ri)
#pragma unroll
          for (int rj = ri; rj < NRB; ++rj, ++p) acc[u][p] = mma_f32(a[ri], d[rj], acc[u][p]);
      }
    }
#pragma unroll
    for (int u = 0; u < CPW; ++u) {
      fold<NRB>(acc[u], accd[u]);
      if constexpr (T > 0) {
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          tsd[u][rb] += (double)ts[u][rb];
          ted[u][rb] += (double)te[u][rb];
          ts[u][rb] = te[u][rb] = 0.f;
        }
        twd[u] += (double)tw[u];
        tstd[u] += (double)tst[u];
        tttd[u] += (double)ttt[u];
        tw[u] = tst[u] = ttt[u] = 0.f;
      }
    }
  };
  for_each_chunk<QX, QW>(X, W, N, B, K, g, G, xr, wr, body);
  const int BP = (B + 1 + 3) & ~3, nb = BP / 4, L = nb * (nb + 1) / 2 * 16;
  auto pos = [&](int I, int J) {   // packed index of (I, J), tile row <= tile column
    const int bi = I >> 2, bj = J >> 2;
    return (bi * nb - bi * (bi - 1) / 2 + (bj - bi)) * 16 + (I & 3) * 4 + (J & 3);
  };
#pragma unroll
  for (int u = 0; u < CPW; ++u) {
    if (!live[u]) break;
    double* out = part + ((int64_t)cls[u] * G + g) * L;
    int p = 0;
#pragma unroll
    for (int ri = 0; ri < NRB; ++ri) {
#pragma unroll
      for (int rj = ri; rj < NRB; ++rj, ++p) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int I = 16 * ri + 4 * grp + e, J = 16 * rj + col;
          // every packed entry (4 x 4 tiles bi <= bj of the padded matrix) once
          if ((I >> 2) <= (J >> 2) && I < BP && J < BP) out[pos(I, J)] = accd[u][p][e];
        }
      }
    }
    if constexpr (T > 0) {
      // the four row groups in a fixed order, then the last tile column
      // (columns 16 NRB .. 16 NRB + 3) and its diagonal tile
      double sd[NRB], ed[NRB];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        sd[rb] = tsd[u][rb] + __shfl_xor(tsd[u][rb], 16);
        sd[rb] += __shfl_xor(sd[rb], 32);
        ed[rb] = ted[u][rb] + __shfl_xor(ted[u][rb], 16);
        ed[rb] += __shfl_xor(ed[rb], 32);
      }
      double sw = twd[u] + __shfl_xor(twd[u], 16);
      sw += __shfl_xor(sw, 32);
      double st = tstd[u] + __shfl_xor(tstd[u], 16);
      st += __shfl_xor(st, 32);
      double tt = tttd[u] + __shfl_xor(tttd[u], 16);
      tt += __shfl_xor(tt, 32);
      const int jt = 16 * NRB;
      if (grp == 0) {
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          const int j = 16 * rb + col;
          out[pos(j, jt)] = T == 2 ? ed[rb] : sd[rb];
          out[pos(j, jt + 1)] = T == 2 ? sd[rb] : 0.0;
          out[pos(j, jt + 2)] = 0.0;
          out[pos(j, jt + 3)] = 0.0;
        }
      }
      if (lane < 16) {
        const int I = jt + (lane >> 2), J = jt + (lane & 3);
        double val = 0.0;
        if (T == 2) {
          if (I == jt && J == jt) val = tt;
          else if (I + J == 2 * jt + 1) val = st;
          else if (I == jt + 1 && J == jt + 1) val = sw;
        } else if (I == jt && J == jt) {
          val = sw;
        }
        out[pos(I, J)] = val;
      }
    }
  }
}

// The plain FP32 reference path of the forward passes, on the vector ALU.
//
// First moments: thread t owns the entries o = t, t + 256, ... of the KP x BP
// block partial ([c][j] = sum_r w[r][c] [x_r, 1][j], zero padding) and sums
// the chunk's rows for each in FP32, folding into FP64 after every chunk;
// every entry has one owner, so the partial is written without a combine.
template <int QX, int QW>
__global__ __launch_bounds__(kBlock) void k_soft_first_valu(const float* __restrict__ X, const float* __restrict__ W,
                                                            int64_t N, int B, int K, int64_t every,
                                                            double* __restrict__ part) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* xr = lds;
  uint32_t* wr = lds + kChunk * B;
  const int BP = (B + 1 + 3) & ~3, KP = (K + 3) & ~3, L = KP * BP;
  constexpr int U = 9;   // entries per thread: KP BP <= 32 x 68 < 9 x 256
  double accd[U];
#pragma unroll
  for (int u = 0; u < U; ++u) accd[u] = 0.0;
  const float* xf = reinterpret_cast<const float*>(xr);
  const float* wf = reinterpret_cast<const float*>(wr);
  auto body = [&](int64_t, int rows) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int o = threadIdx.x + kBlock * u;
      const int c = o / BP, j = o - c * BP;
      if (o >= L || c >= K || j > B) continue;
      float acc = 0.f;
      for (int r = 0; r < rows; ++r) {
        const float xv = j < B ? xf[r * B + j] : 1.f;
        acc = fmaf(wf[r * K + c], xv, acc);
      }
      accd[u] += (double)acc;
    }
  };
  for_each_chunk<QX, QW>(X, W, N, B, K, blockIdx.x, gridDim.x, xr, wr, body, every);
  double* mine = part + (int64_t)blockIdx.x * L;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int o = threadIdx.x + kBlock * u;
    if (o < L) mine[o] = accd[u];
  }
}

// Scatter: block (g, c) takes chunks g, g + G, ... of X and w for class c
// (the training pixels are read once per class), and thread (slice, tile)
// owns a 4 x 4 tile of the weighted augmented Gram of d = [x - m_c, 1]:
// sum over its rows of (w d_I) d_J in FP32, with d formed from the staged
// raw rows, folded into FP64 after every chunk; the slices combine in a
// fixed order into the packed block partial.
template <int QX, int QW>
__global__ __launch_bounds__(kBlock) void k_soft_scatter_valu(const float* __restrict__ X,
                                                              const float* __restrict__ W, int64_t N, int B, int K,
                                                              const float* __restrict__ mc_f,
                                                              double* __restrict__ part) {
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* xr = lds;
  uint32_t* wr = lds + kChunk * B;
  double* red = reinterpret_cast<double*>(lds);
  const int G = gridDim.x, g = blockIdx.x, c = blockIdx.y;
  const int BP = (B + 1 + 3) & ~3;
  const TileAssign ta = assign_tiles(BP);
  // this thread's eight columns: value = x - m (band < B), 1 (band B), 0
  float mi[4], mj[4];
  int ki[4], kj[4];   // 0: band, 1: the ones column, 2: padding
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int I = 4 * ta.bi + e, J = 4 * ta.bj + e;
    ki[e] = I < B ? 0 : (I == B ? 1 : 2);
    kj[e] = J < B ? 0 : (J == B ? 1 : 2);
    mi[e] = I < B ? mc_f[c * B + I] : 0.f;
    mj[e] = J < B ? mc_f[c * B + J] : 0.f;
  }
  float acc[16];
  double accd[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    acc[e] = 0.f;
    accd[e] = 0.0;
  }
  const float* xf = reinterpret_cast<const float*>(xr);
  const float* wf = reinterpret_cast<const float*>(wr);
  auto body = [&](int64_t, int rows) {
    if (ta.active) {
      for (int r = ta.slice; r < rows; r += ta.nslice) {
        const float wv = wf[r * K + c];
        float a[4], b[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float xi = ki[e] == 0 ? xf[r * B + 4 * ta.bi + e] - mi[e] : (ki[e] == 1 ? 1.f : 0.f);
          const float xj = kj[e] == 0 ? xf[r * B + 4 * ta.bj + e] - mj[e] : (kj[e] == 1 ? 1.f : 0.f);
          a[e] = wv * xi;
          b[e] = xj;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[4 * i + j] = fmaf(a[i], b[j], acc[4 * i + j]);
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      accd[e] += (double)acc[e];
      acc[e] = 0.f;
    }
  };
  for_each_chunk<QX, QW>(X, W, N, B, K, g, G, xr, wr, body);
  write_partial(ta, accd, red, part + ((int64_t)c * G + g) * ta.nblk * 16);
}

// The mixed-precision scatter: per class (one per wave, four per block) the
// same weighted Gram, sum_p a_p d_p^T with a = w d and d = [x - m_c, 1], on
// v_mfma_f32_16x16x32_{bf16,f16} with the compensated split: a = a_h + a_l,
// d = d_h + d_l (each the nearest 16-bit value to what is left), and every
// tile pair sums a_h d_h + a_h d_l + a_l d_h + a_l d_l over 32 rows per
// instruction with FP32 accumulation, folded into FP64 after every chunk of
// 128 rows.  All B + 1 columns run on the matrix cores (NRB row blocks of
// 16).  Per entry the error is at most (2 u^2 + 512 2^-24) sum_p |w_p|
// |d_pi| |d_pj| (u = 2^-8 for bf16, 2^-11 for fp16; 512 FP32 terms per
// fold), plus, for values whose tail falls below fp16's normal range, at
// most 2^-40 of the chunk's largest product per term.
// Operand layout as in k_split.hpp: lane l holds row k0 + 8 (l / 16) + t,
// band 16 rb + l % 16 of both operands.
template <int SPLIT, int NRB, int QX, int QW>
__global__ __launch_bounds__(kBlock) void k_soft_scatter_split(const float* __restrict__ X,
                                                               const float* __restrict__ W, int64_t N, int B,
                                                               int K, const float* __restrict__ mc_f,
                                                               double* __restrict__ part) {
  using ST = SplitT<SPLIT>;
  using V = typename ST::V;
  using S = typename ST::S;
  extern __shared__ __align__(16) uint32_t lds[];
  uint32_t* xr = lds;
  uint32_t* wr = lds + kChunk * B;
  const int G = gridDim.x, g = blockIdx.x;
  const int v = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int cls = blockIdx.y * kWaves + v;
  const bool live = cls < K;
  float mrb[NRB];
  int kind[NRB];   // 0: band, 1: the ones column, 2: padding
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    const int band = 16 * rb + col;
    kind[rb] = band < B ? 0 : (band == B ? 1 : 2);
    mrb[rb] = (live && band < B) ? mc_f[cls * B + band] : 0.f;
  }
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
  const float* xf = reinterpret_cast<const float*>(xr);
  const float* wf = reinterpret_cast<const float*>(wr);
  auto dval = [&](int r, int rb) {
    return kind[rb] == 0 ? xf[r * B + 16 * rb + col] - mrb[rb] : (kind[rb] == 1 ? 1.f : 0.f);
  };
  auto body = [&](int64_t, int) {
    if (!live) return;
    // a power of two per operand and chunk brings the chunk's largest |d|
    // and |w d| into [2^14, 2^15): the split values stay inside fp16's
    // range, far above its subnormals; the tiles are unscaled exactly when
    // they fold into FP64
    float md = 0.f, ma = 0.f;
    for (int r = grp; r < kChunk; r += 4) {
      const float wv = fabsf(wf[r * K + cls]);
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        const float d = fabsf(dval(r, rb));
        md = fmaxf(md, d);
        ma = fmaxf(ma, wv * d);
      }
    }
    md = wave_max(md);
    ma = wave_max(ma);
    int ed = 0, ea = 0;
    if (md > 0.f) frexpf(md, &ed);
    if (ma > 0.f) frexpf(ma, &ea);
    const float sd = md > 0.f ? ldexpf(1.f, 15 - ed) : 1.f;
    const float sa = ma > 0.f ? ldexpf(1.f, 15 - ea) : 1.f;
    for (int k0 = 0; k0 < kChunk; k0 += 32) {
      V ah[NRB], al[NRB], dh[NRB], dl[NRB];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int r = k0 + 8 * grp + t;
        const float wv = wf[r * K + cls];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
          const float d0 = dval(r, rb);
          const float a = (wv * d0) * sa;
          const float d = d0 * sd;
          const S h1 = (S)a, h2 = (S)d;
          ah[rb][t] = h1;
          al[rb][t] = (S)(a - (float)h1);
          dh[rb][t] = h2;
          dl[rb][t] = (S)(d - (float)h2);
        }
      }
      int p = 0;
#pragma unroll
      for (int ri = 0; ri < NRB; ++ri)
#pragma unroll
        for (int rj = ri; rj < NRB; ++rj, ++p) {
          acc[p] = ST::mma(al[ri], dl[rj], acc[p]);   // smallest terms first
          acc[p] = ST::mma(ah[ri], dl[rj], acc[p]);
          acc[p] = ST::mma(al[ri], dh[rj], acc[p]);
          acc[p] = ST::mma(ah[ri], dh[rj], acc[p]);
        }
    }
    const double inv = 1.0 / ((double)sa * (double)sd);   // powers of two: exact
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        accd[p][e] += (double)acc[p][e] * inv;
        acc[p][e] = 0.f;
      }
  };
  for_each_chunk<QX, QW>(X, W, N, B, K, g, G, xr, wr, body);
  if (!live) return;
  const int BP = (B + 1 + 3) & ~3, nb = BP / 4, L = nb * (nb + 1) / 2 * 16;
  double* out = part + ((int64_t)cls * G + g) * L;
  int p = 0;
#pragma unroll
  for (int ri = 0; ri < NRB; ++ri)
#pragma unroll
    for (int rj = ri; rj < NRB; ++rj, ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int I = 16 * ri + 4 * grp + e, J = 16 * rj + col;
        // every packed entry (4 x 4 tiles bi <= bj of the padded matrix) once
        if ((I >> 2) <= (J >> 2) && I < BP && J < BP) {
          const int bi = I >> 2, bj = J >> 2;
          out[(bi * nb - bi * (bi - 1) / 2 + (bj - bi)) * 16 + (I & 3) * 4 + (J & 3)] = accd[p][e];
        }
      }
}

__global__ __launch_bounds__(kBlock) void k_soft_backward(const float* __restrict__ X, int64_t N, int B,
                                                          int K, SoftBwdArgs a, int accumulate,
                                                          float* __restrict__ dw) {
  extern __shared__ __align__(16) uint32_t lds[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int S = B;                         // a lane group is one row of B dwords
  uint32_t* my = lds + w * 64 * (B > K ? B : K);   // a slice fits the tile and its gradients
  const int64_t nt = (N + 63) / 64;
  const unsigned char* base = reinterpret_cast<const unsigned char*>(X);
  for_each_tile<kMaxQ, false>(base, N * B * 4, nt, S, my, [&](int64_t t) {
    float z[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = 0.f;
    const uint32_t* d = my + lane * S;
    for (int b = 0; b < B; ++b) {
      const float u = __uint_as_float(d[b]) - a.m[b];
#pragma unroll
      for (int j = 0; j < 8; ++j) z[j] = fmaf(a.w[b * 8 + j], u, z[j]);
    }
    // the tile's 64 x K gradients go through the wave's LDS slice (its rows
    // have been read) and leave as 16-byte stores of the contiguous block
    float* gs = reinterpret_cast<float*>(my);
    float tz = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) tz = fmaf(z[j], z[j], tz);
    for (int c = 0; c < K; ++c) {
      float q = 0.f;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float e = z[j] - a.d[c * 8 + j];
        q = fmaf(a.lam1[j] * e, e, q);
      }
      gs[lane * K + c] = a.scale * (tz - q);
    }
    wave_lds_sync();
    const int64_t r0 = t * 64;
    const int nv = (int)((N - r0 < 64 ? N - r0 : 64) * K);   // values of the tile inside dw
    float* out = dw + r0 * K;
    for (int i = 4 * lane; i < nv; i += 4 * 64) {
      if (i + 4 <= nv) {
        f4v v = *reinterpret_cast<const f4v*>(gs + i);
        if (accumulate) v += *reinterpret_cast<const f4v*>(out + i);
        *reinterpret_cast<f4v*>(out + i) = v;
      } else {
        for (int e = i; e < nv; ++e) out[e] = accumulate ? out[e] + gs[e] : gs[e];
      }
    }
    wave_lds_sync();
  });
}

// One step of mask refinement by the gradient of J (paper Section 4 calls
// for an automatic choice of training points; the step itself is not in the
// paper): per pixel, the gradient minus its mean over the classes (its part
// within the plane of the simplex), scaled so that its largest entry is
// `step`, is added to the weights, and the sum is projected onto the
// probability simplex, w = max(v - theta, 0) with theta making the entries
// sum to one.  theta comes from Michelot's active-set iteration: start with
// every class, set theta = (sum of the active v - 1) / (their number), drop
// the classes with v <= theta, repeat until none drops (at most K rounds;
// exact).  A pixel whose gradient is the same for every class keeps its
// weights, projected.
__global__ __launch_bounds__(kBlock) void k_soft_update(const float* __restrict__ g, float* __restrict__ w,
                                                        int64_t N, int K, float step) {
  constexpr int KM = 32;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += (int64_t)gridDim.x * kBlock) {
    float gv[KM], v[KM];
    float mean = 0.f;
#pragma unroll
    for (int c = 0; c < KM; ++c) {
      gv[c] = c < K ? g[p * K + c] : 0.f;
      v[c] = c < K ? w[p * K + c] : 0.f;
      mean += gv[c];
    }
    mean /= (float)K;
    float smax = 0.f;
#pragma unroll
    for (int c = 0; c < KM; ++c)
      if (c < K) smax = fmaxf(smax, fabsf(gv[c] - mean));
    const float sc = smax > 0.f ? step / smax : 0.f;
#pragma unroll
    for (int c = 0; c < KM; ++c) v[c] = fmaf(gv[c] - mean, sc, v[c]);
    uint32_t active = K >= 32 ? 0xffffffffu : ((1u << K) - 1u);
    float theta = 0.f;
    for (int it = 0; it <= K; ++it) {
      float sum = 0.f;
      int cnt = 0;
#pragma unroll
      for (int c = 0; c < KM; ++c)
        if ((active >> c) & 1u) {
          sum += v[c];
          ++cnt;
        }
      theta = (sum - 1.f) / (float)cnt;
      uint32_t next = 0u;
#pragma unroll
      for (int c = 0; c < KM; ++c)
        if (((active >> c) & 1u) && v[c] > theta) next |= 1u << c;
      if (next == active || next == 0u) break;
      active = next;
    }
#pragma unroll
    for (int c = 0; c < KM; ++c)
      if (c < K) w[p * K + c] = fmaxf(v[c] - theta, 0.f);
  }
}

// LDS of the forward kernels: the raw chunk tiles, or the first pass's
// combine buffer, whichever is larger.
size_t first_smem(int B, int K) {
  const size_t a = (size_t)kChunk * (B + K) * sizeof(float);
  const size_t r = (size_t)((K + 3) & ~3) * ((B + 1 + 3) & ~3) * sizeof(double);
  return a > r ? a : r;
}

size_t scatter_smem(int B, int K) { return (size_t)kChunk * (B + K) * sizeof(float); }

// Two classes per wave for the narrow instances (up to two row blocks on
// the matrix cores) once there are more than four classes.
int scatter_cpw(int B, int K) {
  const bool narrow = nrb_for(B) == 2 || B == 16 || B == 17 || B == 32 || B == 33;
  return (narrow && K > kWaves) ? 2 : 1;
}

template <int NRB, int T, int CPW>
hipError_t scatter_launch(const float* X, const float* w, int64_t N, int B, int K, int G, const float* mc_f,
                          double* part, hipStream_t s) {
  const dim3 grid(G, (K + kWaves * CPW - 1) / (kWaves * CPW));
  if (B <= 40 && K <= 8)
    hipLaunchKernelGGL((k_soft_scatter_mfma<NRB, 5, 1, T, CPW>), grid, dim3(kBlock), scatter_smem(B, K), s, X,
                       w, N, B, K, mc_f, part);
  else
    hipLaunchKernelGGL((k_soft_scatter_mfma<NRB, 8, 4, T, CPW>), grid, dim3(kBlock), scatter_smem(B, K), s, X,
                       w, N, B, K, mc_f, part);
  return hipGetLastError();
}

template <int NRB, int T>
hipError_t scatter_nrb(const float* X, const float* w, int64_t N, int B, int K, int G, const float* mc_f,
                       double* part, hipStream_t s) {
  if constexpr (NRB <= 2) {
    if (scatter_cpw(B, K) == 2) return scatter_launch<NRB, T, 2>(X, w, N, B, K, G, mc_f, part, s);
  }
  return scatter_launch<NRB, T, 1>(X, w, N, B, K, G, mc_f, part, s);
}

}  // namespace

hipError_t launch_soft_first(const float* X, const float* w, int64_t N, int B, int K, int64_t every, int nblocks,
                             double* part, hipStream_t s) {
  if (B < 1 || B > kMaxB || K < 1 || K > 32 || nblocks < 1 || every < 1) return hipErrorInvalidValue;
  const int nrb = nrb_for(B);
  const bool small = B <= 40 && K <= 8;
  const size_t sm = first_smem(B, K);
  const dim3 grid(nblocks);
#define CVX_F(NCB, NRB)                                                                                      \
  if (small)                                                                                                 \
    hipLaunchKernelGGL((k_soft_first<NCB, NRB, 5, 1>), grid, dim3(kBlock), sm, s, X, w, N, B, K, every, part);  \
  else                                                                                                       \
    hipLaunchKernelGGL((k_soft_first<NCB, NRB, 8, 4>), grid, dim3(kBlock), sm, s, X, w, N, B, K, every, part);
  if (K <= 16) {
    if (nrb == 2) { CVX_F(1, 2) } else if (nrb == 3) { CVX_F(1, 3) } else { CVX_F(1, 5) }
  } else {
    if (nrb == 2) { CVX_F(2, 2) } else if (nrb == 3) { CVX_F(2, 3) } else { CVX_F(2, 5) }
  }
#undef CVX_F
  return hipGetLastError();
}

hipError_t launch_soft_means(int B, int K, const double* fp, double* first, float* mc_f, hipStream_t s) {
  hipLaunchKernelGGL(k_soft_means, dim3(1), dim3(kBlock), 0, s, B, K, fp, first, mc_f);
  return hipGetLastError();
}

int soft_scatter_classes_per_block(int B, int K) { return kWaves * scatter_cpw(B, K); }

int soft_scatter_blocks_per_cu(int B, int K) { return scatter_cpw(B, K) == 2 ? 2 : 3; }

hipError_t launch_soft_scatter(const float* X, const float* w, int64_t N, int B, int K, int G,
                               const float* mc_f, double* part, hipStream_t s) {
  if (B < 1 || B > kMaxB || K < 1 || K > 32 || G < 1) return hipErrorInvalidValue;
  // B + 1 = 16 m + 1 or 16 m + 2: m row blocks on the matrix cores and the
  // tail columns on the vector ALU
  switch (B) {
    case 16: return scatter_nrb<1, 1>(X, w, N, B, K, G, mc_f, part, s);
    case 17: return scatter_nrb<1, 2>(X, w, N, B, K, G, mc_f, part, s);
    case 32: return scatter_nrb<2, 1>(X, w, N, B, K, G, mc_f, part, s);
    case 33: return scatter_nrb<2, 2>(X, w, N, B, K, G, mc_f, part, s);
    case 48: return scatter_nrb<3, 1>(X, w, N, B, K, G, mc_f, part, s);
    case 49: return scatter_nrb<3, 2>(X, w, N, B, K, G, mc_f, part, s);
    case 64: return scatter_nrb<4, 1>(X, w, N, B, K, G, mc_f, part, s);
  }
  switch (nrb_for(B)) {
    case 2: return scatter_nrb<2, 0>(X, w, N, B, K, G, mc_f, part, s);
    case 3: return scatter_nrb<3, 0>(X, w, N, B, K, G, mc_f, part, s);
    default: return scatter_nrb<5, 0>(X, w, N, B, K, G, mc_f, part, s);
  }
}

hipError_t launch_soft_first_plain(const float* X, const float* w, int64_t N, int B, int K, int64_t every,
                                   int nblocks, double* part, hipStream_t s) {
  if (B < 1 || B > kMaxB || K < 1 || K > 32 || nblocks < 1 || every < 1) return hipErrorInvalidValue;
  const size_t sm = scatter_smem(B, K);
  if (B <= 40 && K <= 8)
    hipLaunchKernelGGL((k_soft_first_valu<5, 1>), dim3(nblocks), dim3(kBlock), sm, s, X, w, N, B, K, every, part);
  else
    hipLaunchKernelGGL((k_soft_first_valu<8, 4>), dim3(nblocks), dim3(kBlock), sm, s, X, w, N, B, K, every, part);
  return hipGetLastError();
}

hipError_t launch_soft_scatter_plain(const float* X, const float* w, int64_t N, int B, int K, int G,
                                     const float* mc_f, double* part, hipStream_t s) {
  if (B < 1 || B > kMaxB || K < 1 || K > 32 || G < 1) return hipErrorInvalidValue;
  const int BP = padded_bp(B), nb = BP / 4, nblk = nb * (nb + 1) / 2;
  const size_t red = (size_t)(kBlock / nblk) * nblk * 16 * sizeof(double);
  const size_t sm = std::max(scatter_smem(B, K), red);
  const dim3 grid(G, K);
  if (B <= 40 && K <= 8)
    hipLaunchKernelGGL((k_soft_scatter_valu<5, 1>), grid, dim3(kBlock), sm, s, X, w, N, B, K, mc_f, part);
  else
    hipLaunchKernelGGL((k_soft_scatter_valu<8, 4>), grid, dim3(kBlock), sm, s, X, w, N, B, K, mc_f, part);
  return hipGetLastError();
}

template <int SPLIT, int NRB>
hipError_t split_scatter_nrb(const float* X, const float* w, int64_t N, int B, int K, int G, const float* mc_f,
                             double* part, hipStream_t s) {
  const dim3 grid(G, (K + kWaves - 1) / kWaves);
  const size_t sm = scatter_smem(B, K);
  if (B <= 40 && K <= 8)
    hipLaunchKernelGGL((k_soft_scatter_split<SPLIT, NRB, 5, 1>), grid, dim3(kBlock), sm, s, X, w, N, B, K, mc_f,
                       part);
  else
    hipLaunchKernelGGL((k_soft_scatter_split<SPLIT, NRB, 8, 4>), grid, dim3(kBlock), sm, s, X, w, N, B, K, mc_f,
                       part);
  return hipGetLastError();
}

hipError_t launch_soft_scatter_split(int split, const float* X, const float* w, int64_t N, int B, int K, int G,
                                     const float* mc_f, double* part, hipStream_t s) {
  if (B < 1 || B > kMaxB || K < 1 || K > 32 || G < 1) return hipErrorInvalidValue;
  const int nrb = nrb_for(B);
#define CVX_S(SP)                                                                                 \
  switch (nrb) {                                                                                  \
    case 2: return split_scatter_nrb<SP, 2>(X, w, N, B, K, G, mc_f, part, s);                     \
    case 3: return split_scatter_nrb<SP, 3>(X, w, N, B, K, G, mc_f, part, s);                     \
    default: return split_scatter_nrb<SP, 5>(X, w, N, B, K, G, mc_f, part, s);                    \
  }
  if (split == 0) { CVX_S(0) }
  CVX_S(1)
#undef CVX_S
}

hipError_t launch_soft_update(const float* g, float* w, int64_t N, int K, float step, int num_cu, hipStream_t s) {
  if (K < 2 || K > 32 || N < 1) return hipErrorInvalidValue;
  const int64_t need = (N + kBlock - 1) / kBlock;
  const int nb = (int)std::min<int64_t>(need, (int64_t)num_cu * 8);
  hipLaunchKernelGGL(k_soft_update, dim3(nb), dim3(kBlock), 0, s, g, w, N, K, step);
  return hipGetLastError();
}

hipError_t launch_soft_backward(const float* X, int64_t N, int B, int K, const SoftBwdArgs& a,
                                bool accumulate, int nblocks, float* dw, hipStream_t s) {
  // each wave's slice holds its 64-row tile of X, then the tile's gradients
  const size_t sm = (size_t)kWaves * 64 * std::max(B, K) * 4;
  hipLaunchKernelGGL(k_soft_backward, dim3(nblocks), dim3(kBlock), sm, s, X, N, B, K, a,
                     accumulate ? 1 : 0, dw);
  return hipGetLastError();
}

}  // namespace cvx

// Host-side launchers for the gfx950 kernels (defined in the k_*.hip files).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cvx {

constexpr int kLabelWave = 4096;   // label entries per wave tile in the label kernels
constexpr int kBlock = 256;         // threads per block in every kernel
constexpr int kWaves = kBlock / 64; // waves per block
constexpr int kChunk = 128;         // rows staged per chunk in the scatter kernels
constexpr int kMaxB = 64;

// Parameters of one projection pass, passed by value in the kernel
// arguments (fits the 4 KiB argument limit).
struct ProjArgs {
  float w[64 * 8];   // W[b * nc + j] for this group of nc <= 8 components (row stride nc)
  float c[64];       // per-band centre (integer for uint16 pages)
  float off[8];      // sum_b W[b][j] (c_b - centre_b), added to each y_j
  float scale[8];    // power of two per component (uint16 matrix-core kernels)
};

// The fp16 intermediate of the one-read projection schedule: pass 1 stores
// each component value as fp16 of (scaled sum x f[j]), f[j] a power of two
// chosen on the host so that no stored value can overflow; pass 2 re-reads
// the page instead of the stored values when its computed error bound (in
// grey levels) exceeds `limit`.
struct H16Args {
  float f[8];
  float limit;
};

struct SoftBwdArgs {
  float w[64 * 8];   // W[b * 8 + j] for this group of 8 components (zero padded)
  float m[64];       // grand mean
  float d[32 * 8];   // d[c * 8 + j] = w_j^T (m_c - m)
  float lam1[8];     // 1 + lambda_j (zero for padded components)
  float scale;       // dJ
};

// label bookkeeping
// label bookkeeping over nW = ceil(P / kLabelWave) wave tiles:
// wave_counts is K + 1 rows of nW entries, each row label_row_stride(nW)
// entries apart (class-major; row K: a flag per wave tile for entries
// outside -1..K-1); the count kernel writes the counts and flags,
// the scan kernel turns each class row into exclusive offsets within the
// class (in place), writes the K class totals and sets err_flag[0] to 1 or
// 0 (err_flag[1] to 0), the index kernel writes the class-grouped list and
// the counts and offsets
__host__ __device__ inline int64_t label_row_stride(int nW) { return ((int64_t)nW + 3) & ~int64_t(3); }
hipError_t launch_label_count(const int8_t* labels, int64_t P, int K, int nW, int32_t* wave_counts,
                              hipStream_t s);
hipError_t launch_label_scan(int32_t* wave_counts, int nW, int K, int32_t* class_total, int32_t* err_flag,
                             hipStream_t s);
hipError_t launch_label_index(const int8_t* labels, int64_t P, int K, int nW, const int32_t* wave_off,
                              const int32_t* class_total, int32_t* idx, int64_t* counts_out, int32_t* offsets_out,
                              hipStream_t s);

// training points as a list: turn the class-grouped list positions in idx
// (offsets[K] of them) into pixels; ORs 2 into *err_flag for a pixel
// outside 0..P-1
hipError_t launch_points_to_pixels(const int64_t* pixels, int32_t* idx, const int32_t* offsets, int K, int64_t N,
                                   int64_t P, int32_t* err_flag, int num_cu, hipStream_t s);

// class moments: per-class augmented Gram of [x - c_k, 1] about a per-class
// shift c_k; partials part[(k * G + g) * L + t], L = nblk * 16.
hipError_t launch_class_moments(int dtype, const void* cube, int B, int64_t P, const int32_t* idx,
                                const int32_t* offsets, int K, int G, double* part,
                                double* shift_out, hipStream_t s);
// PCA: augmented Gram of [x - s, 1] over all (or masked) pixels.
hipError_t launch_pca_gram(int dtype, const void* cube, int B, int64_t P,
                           const uint8_t* mask, int nblocks, double* part,
                           double* shift_out, hipStream_t s);
// The same two Gram matrices on the matrix cores with a compensated
// 16-bit split (split 0 = bf16, 1 = fp16); identical output layout.
hipError_t launch_class_moments_mfma(int dtype, int split, const void* cube, int B, int64_t P,
                                     const int32_t* idx, const int32_t* offsets, int K, int G,
                                     double* part, double* shift_out, hipStream_t s);
hipError_t launch_pca_gram_mfma(int dtype, int split, const void* cube, int B, int64_t P,
                                const uint8_t* mask, int nblocks, double* part,
                                double* shift_out, hipStream_t s);
// Blocks per CU that the uint16 page-covariance kernel keeps resident at
// B bands (its waves per SIMD): the grid that fills the device in one round.
int pca_u16_blocks_per_cu(int B);
// out[s * L + t] = sum_g part[(s * G + g) * L + t]
hipError_t launch_reduce_part(const double* part, int nsets, int G, int L, double* out,
                              hipStream_t s);
// the same with out in page-locked host memory, and hdr_bytes (a multiple
// of 4) copied from hdr_src to hdr_dst in the same launch
hipError_t launch_reduce_part_out(const double* part, int nsets, int G, int L, double* out_host,
                                  const void* hdr_src, void* hdr_dst, int64_t hdr_bytes, hipStream_t s);

// projection, pass 1 (range) and pass 2 (stretch to uint8); vector = the
// FP32 vector-ALU kernels whatever the page type (else uint16 pages take the
// matrix cores); the ProjArgs must be made for the same choice
hipError_t launch_project_range(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                const ProjArgs& a, int nblocks, float* part,
                                unsigned* ticket, float* range_dev, float* ab_dev,
                                hipStream_t s);
hipError_t launch_project_stretch(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                  const ProjArgs& a, int nblocks, const float* range_dev, uint8_t* images,
                                  hipStream_t s);

// matrix-core projection of uint16 pages (same contract as above)
hipError_t launch_project_range_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                    int nblocks, float* part, unsigned* ticket, float* range_dev,
                                    float* ab_dev, hipStream_t s);
hipError_t launch_project_stretch_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                      int nblocks, const float* range_dev, uint8_t* images,
                                      hipStream_t s);

hipError_t launch_project_float_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a, int nblocks,
                                    float* y, hipStream_t s);

// the one-read schedule for any page type (dispatching as the two-pass
// launchers above): pass 1 also stores the fp16 planes, pass 2 maps them
hipError_t launch_project_range_h16(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                    const ProjArgs& a, int nblocks, float* part, unsigned* ticket,
                                    float* range_dev, float* ab_dev, const H16Args& h, uint16_t* planes,
                                    int64_t Pp, hipStream_t s);
hipError_t launch_project_stretch_h16(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                      const ProjArgs& a, int nblocks, const float* range_dev,
                                      const uint16_t* planes, int64_t Pp, uint8_t* images, hipStream_t s);
// the one-read schedule on uint16 pages: pass 1 as launch_project_range_u16
// and also the fp16 planes (nc planes of Pp >= P values, Pp a multiple of
// 256; range_dev[16..32) the map of the stored values, range_dev[32] the
// fallback flag, range_dev[40..48) the error bounds); pass 2 quantises the
// planes, or re-reads the page when the flag is set
hipError_t launch_project_range_h16_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                        int nblocks, float* part, unsigned* ticket, float* range_dev,
                                        float* ab_dev, const H16Args& h, uint16_t* planes, int64_t Pp,
                                        hipStream_t s);
hipError_t launch_project_stretch_h16_u16(const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                          int nblocks, const float* range_dev, const uint16_t* planes, int64_t Pp,
                                          uint8_t* images, hipStream_t s);

// rescaling from FP32 component planes y (nc planes of P floats, nc <= 64)
constexpr int kSelTargets = 4;   // order statistics wanted per plane by one select
constexpr int kSelPasses = 3;    // radix passes of 11, 11 and 10 bits over the 32-bit keys
constexpr int kSelBins = 2048;   // histogram bins per pass (the widest digit)
// low bit and width of the digit of pass p
__host__ __device__ constexpr int sel_shift(int p) { return p == 0 ? 21 : p == 1 ? 10 : 0; }
__host__ __device__ constexpr int sel_width(int p) { return p == 2 ? 10 : 11; }
// blocks per plane for the reductions over m values of each of nc planes
int stretch_reduce_blocks(int64_t m, int nc, int num_cu);
// part[(j * nb + blk) * 2 + {0, 1}]: block partial min/max of plane j over
// all pixels, or over idx[0..n) if idx is non-NULL (an index outside
// 0..P-1 ORs 2 into *err and is skipped)
hipError_t launch_plane_minmax(const float* y, int64_t P, int nc, const int64_t* idx, int64_t n, int nb,
                               float* part, int32_t* err, hipStream_t s);
// exact order statistics of ranks[t] (0-based) in every plane: sel
// (nc x kSelTargets) ends with their order-preserving keys; hist holds
// 2 x nc x kSelTargets x kSelBins counters
hipError_t launch_select(const float* y, int64_t P, int nc, const uint32_t (&ranks)[kSelTargets], int nb,
                         uint2* sel, uint32_t* hist, hipStream_t s);
// range ab[2 j + {0, 1}] = (a_j, b_j): mode 1 / 2 fold the nb partials per
// plane, mode 3 interpolates the order statistics in sel
hipError_t launch_stretch_finish(int mode, int nc, int nb, const float* part, const uint2* sel, double g_lo,
                                 double g_hi, double* ab, hipStream_t s);
hipError_t launch_stretch_planes(const float* y, int64_t P, int nc, const double* ab, int bits, void* out,
                                 int num_cu, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_compose_rgb(const uint8_t* r, const uint8_t* g, const uint8_t* b, int64_t P, uint8_t* rgb,
                              int num_cu, hipStream_t s);
// projection to FP32 planes (y[j][p] = w_j^T (x_p - c), n_comp x P)
hipError_t launch_project_float(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                const ProjArgs& a, int nblocks, float* y, hipStream_t s);

// cluster-separation indices: per class k of the class-grouped points,
// sums[k * L + f] = sum of feature f (L = cluster_sum_len(n)) and
// dsum[k] = sum of ||X - A_k||_p with A_k = sums[k] / counts[k]; part holds
// K x G x (L + 1) doubles
int cluster_sum_len(int n);
hipError_t launch_cluster_moments(int dtype, const void* img, int64_t P, int n, const int32_t* idx,
                                  const int32_t* offsets, const int64_t* counts, int K, int G, double p,
                                  double* part, double* sums, double* dsum, hipStream_t s);

// band-sequential stack (B planes of P; uint8, uint16 or float32) to the
// band-interleaved page (uint16 for 8/16-bit bands, float32 for float)
hipError_t launch_bands_to_cube(int in_dtype, const void* bands, int B, int64_t P, void* cube, hipStream_t s);

// Fixed device scratch of the allocation-free projection entry point, one
// copy per GPU (k_scratch.hip).  Layout in bytes: [0, 256) tickets,
// [256, 512) the stretch map of the current group, [512, 1024) the range
// (min, max) of up to 64 components, then the block partials of up to
// kScratchBlocks blocks (32 floats each).
constexpr int kScratchBlocks = 4096;
constexpr int kScratchPartOffset = 1024;
constexpr size_t kScratchBytes = (size_t)kScratchPartOffset + (size_t)kScratchBlocks * 32 * sizeof(float);
// looks up the scratch's device address on `device`, which must be current;
// once per device (later calls return at once)
hipError_t scratch_setup(int device);
// that address, or nullptr before scratch_setup succeeded on `device`
void* scratch_address(int device);

// the reference read stream: bytes (a multiple of 16) from src, once
hipError_t launch_stream_read(const void* src, int64_t bytes, uint32_t key, uint32_t* sink, int num_cu,
                              hipStream_t s);
hipError_t launch_stream_mix(const void* src, int64_t read_bytes, void* dst, int64_t write_bytes, uint32_t key,
                             uint32_t* sink, int num_cu, hipStream_t s);

// n bytes from device memory to page-locked host memory, by a kernel
hipError_t launch_copy_out(void* dst, const void* src, int64_t n, hipStream_t s);

// soft-label CVA
// pass 1: block partials of w^T [X, 1] (KP x BP each), over the chunks
// 0, every, 2 every, ... of kChunk rows (every = 1: all of them)
hipError_t launch_soft_first(const float* X, const float* w, int64_t N, int B, int K, int64_t every, int nblocks,
                             double* part, hipStream_t s);
// from the reduced first moments fp (KP x BP): first[c][0..B] and the class
// means in FP32
hipError_t launch_soft_means(int B, int K, const double* fp, double* first, float* mc_f, hipStream_t s);
// pass 2: per-class weighted Gram partials part[(c * G + g) * L + t]
// classes one scatter block takes, and the blocks per CU it keeps resident
int soft_scatter_classes_per_block(int B, int K);
int soft_scatter_blocks_per_cu(int B, int K);
hipError_t launch_soft_scatter(const float* X, const float* w, int64_t N, int B, int K, int G,
                               const float* mc_f, double* part, hipStream_t s);
// the plain FP32 reference path of the two forward passes (vector ALU;
// same outputs and layouts), and the split scatter on the bf16 (split 0) or
// fp16 (split 1) matrix units
hipError_t launch_soft_first_plain(const float* X, const float* w, int64_t N, int B, int K, int64_t every,
                                   int nblocks, double* part, hipStream_t s);
hipError_t launch_soft_scatter_plain(const float* X, const float* w, int64_t N, int B, int K, int G,
                                     const float* mc_f, double* part, hipStream_t s);
hipError_t launch_soft_scatter_split(int split, const float* X, const float* w, int64_t N, int B, int K, int G,
                                     const float* mc_f, double* part, hipStream_t s);
// one refinement step of the weights w (N x K) along the gradient g:
// mean-free, scaled to `step` at its largest entry, projected onto the simplex
hipError_t launch_soft_update(const float* g, float* w, int64_t N, int K, float step, int num_cu, hipStream_t s);
hipError_t launch_soft_backward(const float* X, int64_t N, int B, int K, const SoftBwdArgs& a,
                                bool accumulate, int nblocks, float* dw, hipStream_t s);

inline int padded_bp(int B) { return (B + 1 + 3) & ~3; }
inline int tri_blocks(int B) {
  const int nb = padded_bp(B) / 4;
  return nb * (nb + 1) / 2;
}

}  // namespace cvx

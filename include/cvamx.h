/*
 * cvamx: canonical variates analysis (CVA) and PCA enhancement of
 * multispectral page images on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every entry point takes plain pointers and sizes; "device" means
 * memory allocated on the context's GPU (hipMalloc, or a torch CUDA/HIP
 * tensor), "host" means ordinary CPU memory.  The caller owns every buffer;
 * the library never frees caller memory.  Scratch space lives in the
 * context.  All functions return CVAMX_OK (0) or a negative CVAMX_E_* code;
 * on error no host output is written and cvamx_last_error() describes the
 * failure.  A context is not thread safe; use one per host thread/stream.
 *
 * Method (paper: Section 2, canonical variates paragraph; Section 4, the
 * GSL implementation with a generalized symmetric-definite eigensolver;
 * Section 2, regression coefficients multiplied with every band of the
 * page and the rescale to 0..255):
 *   n_k = #{p : label_p = k},  m_k = mean of class k,  m = mean of all
 *   training pixels,  S_w = sum_k sum_{p in k} (x_p - m_k)(x_p - m_k)^T,
 *   S_b = sum_k n_k (m_k - m)(m_k - m)^T,
 *   S_b w = lambda (S_w + ridge I) w,  w^T (S_w + ridge I) w = 1,
 *   lambda descending, C = min(K-1, B) components, the largest-magnitude
 *   entry of each w positive (ties: lowest band),
 *   y_jp = w_j^T (x_p - m),  q_jp = clamp(floor(255 (y_jp - a_j) /
 *   (b_j - a_j) + 1/2), 0, 255) with a_j, b_j the page-wide min and max.
 * Scatter, not covariance: no division by degrees of freedom.
 *
 * Layouts.  A page ("cube") is band-interleaved by pixel (BIP): element
 * (y, x, b) sits at offset (y * width + x) * bands + b; its base address
 * must be 16-byte aligned.  Label maps are int8 height x width, -1 = not a
 * training pixel, 0..K-1 = class.  Matrices are row-major float64:
 * W is bands x n_comp (W[b * n_comp + j]), S_w and S_b are bands x bands,
 * class means K x bands.  Output images are planar uint8
 * n_comp x height x width.
 */
#ifndef CVAMX_H
#define CVAMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CVAMX_OK             0
#define CVAMX_E_INVALID_ARG (-1) /* null pointer, bad size, K < 2, n_comp out of range, label outside -1..K-1 */
#define CVAMX_E_UNSUPPORTED (-2) /* dtype/precision not supported, bands > CVAMX_MAX_BANDS, misaligned cube */
#define CVAMX_E_EMPTY_CLASS (-3) /* some class has no training pixel (or zero total weight) */
#define CVAMX_E_NOT_PD      (-4) /* S_w (+ ridge I) is not positive definite: Cholesky failed */
#define CVAMX_E_DEVICE      (-5) /* HIP runtime error, or a context without a device */
#define CVAMX_E_NO_MEMORY   (-6) /* device or pinned host allocation failed */
#define CVAMX_E_NUMERIC     (-7) /* eigensolver did not converge */

#define CVAMX_MAX_BANDS   64
#define CVAMX_MAX_CLASSES 127

/* ---- element types and precisions -------------------------------------- */
typedef enum {
  CVAMX_U16 = 0,   /* unsigned 16-bit detector counts */
  CVAMX_F32 = 1,
  CVAMX_BF16 = 2,
  CVAMX_F16 = 3,
  CVAMX_U8 = 4     /* 8-bit values: band images for cvamx_bands_to_cube and cvamx_run_pages, images for cvamx_cluster_indices */
} cvamx_dtype;

typedef enum {
  CVAMX_PREC_FP32 = 0,    /* FP32 accuracy: FP32 sums, FP64 combine; on uint16 pages the products run exactly on the matrix cores (bit-built fp16 terms), elsewhere plain FP32 on the vector ALUs (cvamx_set_plain_fp32: vector ALUs everywhere) */
  CVAMX_PREC_BF16X3 = 1,  /* MFMA, values split hi+lo in bf16, hi*hi + hi*lo + lo*hi (+ lo*lo for integer pages), FP32 accumulate, FP64 combine */
  CVAMX_PREC_F16X3 = 2    /* same with an fp16 split */
} cvamx_prec;

typedef struct cvamx_ctx cvamx_ctx;

/* A page resident in device memory. */
typedef struct {
  const void* data;   /* device, height*width*bands elements, BIP, 16-byte aligned */
  int64_t height;
  int64_t width;
  int64_t bands;      /* 1..CVAMX_MAX_BANDS */
  int32_t dtype;      /* cvamx_dtype */
} cvamx_cube;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` (>= 0).  device = -1 makes a
 * context without a GPU: argument checking and the host-only calls work,
 * every compute call returns CVAMX_E_DEVICE.  *out receives the context.
 * Launch shapes can be set for measurement from the environment when the
 * context is made: CVAMX_PROJ_BLOCKS (blocks of the page-streaming
 * projection passes; default 8 per compute unit) and CVAMX_GRAM_BLOCKS
 * (blocks of the PCA Gram pass; default one resident round for uint16
 * pages on the matrix cores, 4 per compute unit otherwise; for the exact
 * integer covariance of uint16 pages it is raised where needed so that no
 * block covers more than 2^21 pixels).  The images and ranges do not
 * depend on them; the PCA covariance may change in its last bits (another
 * summation order), except that of uint16 pages on the matrix cores, which
 * is exact. */
int cvamx_create(cvamx_ctx** out, int device);
void cvamx_destroy(cvamx_ctx* ctx);
const char* cvamx_status_str(int status);
const char* cvamx_last_error(const cvamx_ctx* ctx);   /* never NULL */

/* ---- CVA ---------------------------------------------------------------- */

/* Fit CVA on the training pixels of a page (paper Section 2, canonical
 * variates paragraph; Section 4, generalized symmetric-definite solve).
 *   labels   device, height*width int8 (-1 or 0..K-1), 16-byte aligned
 *   K        number of classes, 2..CVAMX_MAX_CLASSES
 *   prec     cvamx_prec for the scatter accumulation
 *   ridge    >= 0, added to the diagonal of S_w before the solve
 *   n_comp   1..min(K-1, bands)
 * Host outputs (row-major float64): W bands x n_comp, eigvals n_comp,
 * mean bands (the grand mean, used to centre projections), counts K
 * (int64, exact).  Optional (may be NULL): class_means K x bands,
 * Sw and Sb bands x bands.
 * Runs on `stream` (a hipStream_t, NULL = default stream) and synchronises
 * it before returning (the outputs are host memory). */
int cva_fit(cvamx_ctx* ctx, const cvamx_cube* cube, const int8_t* labels,
            int32_t K, int32_t prec, double ridge, int32_t n_comp,
            double* W, double* eigvals, double* mean, int64_t* counts,
            double* class_means, double* Sw, double* Sb, void* stream);

/* The same fit from a list of training points, as the analyst picks them
 * (paper Section 2: a set of points per class; Section 4: the points given
 * as (x, y) coordinates), instead of a label map.
 *   pixels   device, N int64 pixel indices y * width + x, each in
 *            0..height*width-1, 8-byte aligned; a pixel may repeat (each
 *            entry is one training sample)
 *   classes  device, N int8 (-1 = skip the entry, or 0..K-1), 16-byte
 *            aligned
 *   N        1..2^31-1
 * Other arguments and outputs as cva_fit; a pixel outside the page gives
 * CVAMX_E_INVALID_ARG.  Within a class the samples keep the list order. */
int cva_fit_points(cvamx_ctx* ctx, const cvamx_cube* cube, const int64_t* pixels,
                   const int8_t* classes, int64_t N, int32_t K, int32_t prec,
                   double ridge, int32_t n_comp, double* W, double* eigvals,
                   double* mean, int64_t* counts, double* class_means,
                   double* Sw, double* Sb, void* stream);

/* The training pixels of each class, as the fits gather them (paper
 * Section 2: the analyst's set of points per class): the positions of the
 * entries equal to k, in increasing order, for k = 0..K-1, one class after
 * the other.
 *   labels   device, n int8 (-1 = no class, or 0..K-1), 16-byte aligned
 *   n        1..2^31-1
 *   K        1..CVAMX_MAX_CLASSES
 *   idx      device, int32, room for n entries, 4-byte aligned: receives
 *            the positions of class k at idx[offsets[k] .. offsets[k+1])
 *   counts   host, K int64: entries per class
 *   offsets  host, K + 1 int32: offsets[0] = 0, offsets[K] = labelled total
 * A label outside -1..K-1 gives CVAMX_E_INVALID_ARG (idx then undefined).
 * Synchronises `stream`. */
int cvamx_label_index(cvamx_ctx* ctx, const int8_t* labels, int64_t n,
                      int32_t K, int32_t* idx, int64_t* counts,
                      int32_t* offsets, void* stream);

/* Project every pixel onto n_comp vectors and stretch each component to
 * 8 bits by its page-wide min and max (paper Section 2, regression
 * coefficients multiplied with the whole page; first rescale mode).
 *   W        host, bands x n_comp row-major float64 (from cva_fit / pca_fit)
 *   center   host, bands float64 (the mean returned by the fit)
 *   n_comp   1..CVAMX_MAX_BANDS
 *   images   device, n_comp x height x width uint8 (planar)
 *   range    host, 2*n_comp float (min_j, max_j pairs) or NULL
 * Asynchronous on `stream` unless `range` is non-NULL (then it
 * synchronises).  W and center are read before the call returns.  The
 * page is read once or twice (cvamx_set_schedule). */
int cva_project(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W,
                const double* center, int32_t n_comp, uint8_t* images,
                float* range, void* stream);

/* cva_project for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, images and range, with every piece of device scratch (block
 * partials, the last-block ticket, the stretch map and range slots) in a
 * fixed array of 513 KiB that each GPU holds from the first cvamx_create on
 * it until the process ends.  The call makes no hipMalloc, hipFree or other
 * allocating call; it launches a one-element fill kernel that clears the
 * ticket, then the same two passes as cva_project.  Limit: a projection grid
 * of at most 4096 blocks (the default grid is 8 blocks per compute unit;
 * CVAMX_PROJ_BLOCKS above that fails with CVAMX_E_UNSUPPORTED).  All calls
 * on one GPU share the array, which keeps the last call's contents: calls
 * that overlap on one GPU (other streams, other contexts, other threads)
 * race and must be serialised by the caller.  With range = NULL the call
 * is asynchronous on `stream` and records only kernel launches; a non-NULL
 * range is copied to the host with hipMemcpyAsync and synchronises. */
int cva_project_noalloc(cvamx_ctx* ctx, const cvamx_cube* cube,
                        const double* W, const double* center,
                        int32_t n_comp, uint8_t* images, float* range,
                        void* stream);

/* cva_fit followed by cva_project with the fitted (W, mean), in one call:
 * the projection is launched straight after the host's FP64 finish, with
 * no return to the caller in between.  Arguments as for the two calls
 * (W, eigvals, mean, counts required; images device n_comp x height x
 * width uint8; range host 2*n_comp float or NULL).  Synchronises `stream`
 * for the fit; the projection is asynchronous unless range is non-NULL. */
int cva_fit_project(cvamx_ctx* ctx, const cvamx_cube* cube,
                    const int8_t* labels, int32_t K, int32_t prec,
                    double ridge, int32_t n_comp, double* W,
                    double* eigvals, double* mean, int64_t* counts,
                    uint8_t* images, float* range, void* stream);

/* ---- PCA ---------------------------------------------------------------- */

/* Covariance PCA of the page (paper Section 2, PCA paragraph: centre,
 * covariance, eigenvectors; unsupervised whole-page variant).
 *   mask     device, height*width uint8 (non-zero = use pixel) or NULL for
 *            every pixel
 * Host outputs: V bands x n_comp, eigvals n_comp (covariance eigenvalues,
 * divisor P-1, descending), mean bands; cov bands x bands or NULL.
 * Synchronises `stream`. */
int pca_fit(cvamx_ctx* ctx, const cvamx_cube* cube, const uint8_t* mask,
            int32_t n_comp, int32_t prec, double* V, double* eigvals,
            double* mean, double* cov, void* stream);

/* With enable = 1, pca_fit on this context standardises every band to unit
 * variance over the selected pixels first (the methods the paper compares
 * with standardise their inputs, Section 2): eigvals are those of the
 * correlation matrix R = D^-1/2 C D^-1/2 (D = diag C, C the covariance, which
 * cov still returns), and V holds the projection vectors D^-1/2 u_j, so that
 * pca_project with (V, mean) maps the scores of the standardised bands
 * (C V = D V diag(eigvals), V^T D V = I).  A band of zero variance
 * then fails with CVAMX_E_INVALID_ARG.  0 (the default) restores covariance
 * PCA.  Host-only: never fails for a valid context. */
int cvamx_set_pca_standardize(cvamx_ctx* ctx, int enable);

/* Same as cva_project with (V, mean) from pca_fit. */
int pca_project(cvamx_ctx* ctx, const cvamx_cube* cube, const double* V,
                const double* mean, int32_t n_comp, uint8_t* images,
                float* range, void* stream);

/* CVA and PCA of one page in one call (paper Section 2: the canonical
 * variates and the principal components of the same page, each projected
 * and stretched to 8-bit images).  The result equals cva_fit_project (with
 * range = NULL) followed by pca_fit (cov = NULL) and pca_project with its
 * (V, mean), bit for bit; the call only orders the work so that each FP64
 * host finish overlaps GPU work: the class moments and then the PCA
 * covariance pass are queued, the CVA finish runs while the covariance pass
 * reads the page and queues the CVA projection, and the PCA finish runs
 * while that projection reads the page and queues the PCA projection.
 *   labels, K, prec, ridge, n_cva, W, eigvals, mean, counts, cva_images:
 *            as for cva_fit_project (cva_images device n_cva x height x
 *            width uint8)
 *   mask, n_pca, V, pca_eigvals, pca_mean: as for pca_fit with n_comp =
 *            n_pca; pca_images device n_pca x height x width uint8
 * The host outputs are set when the call returns; both projections are
 * asynchronous on `stream`.  Honours cvamx_set_pca_standardize.  Errors as
 * for the separate calls; a call that fails after queuing work returns once
 * `stream` has drained. */
int cvamx_cva_pca(cvamx_ctx* ctx, const cvamx_cube* cube, const int8_t* labels,
                  int32_t K, int32_t prec, double ridge, int32_t n_cva,
                  double* W, double* eigvals, double* mean, int64_t* counts,
                  uint8_t* cva_images, const uint8_t* mask, int32_t n_pca,
                  double* V, double* pca_eigvals, double* pca_mean,
                  uint8_t* pca_images, void* stream);

/* ---- float images, rescaling modes, 16-bit output, colour ---------------- */

/* The float images themselves: y_jp = w_j^T (x_p - center) for every pixel
 * (paper Section 2: the regression coefficients multiplied with every band
 * give one array of floating point numbers per component).  Works for the
 * (W, mean) of cva_fit and the (V, mean) of pca_fit alike; the values are
 * the very ones whose min/max and stretch cva_project takes.
 *   W, center, n_comp   as for cva_project
 *   y        device, n_comp x height x width float32 (planar), 4-byte
 *            aligned (16-byte aligned with height*width % 4 == 0 for
 *            full-width stores)
 * Asynchronous on `stream`; W and center are read before the call returns.
 * Misaligned y: CVAMX_E_UNSUPPORTED. */
int cvamx_project_float(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W,
                        const double* center, int32_t n_comp, float* y,
                        void* stream);

/* Rescaling modes (paper Section 2, the three ways of mapping the float
 * arrays onto 0..255): */
enum {
  CVAMX_STRETCH_MINMAX = 1,     /* a_j, b_j = min and max over the page */
  CVAMX_STRETCH_TRAINING = 2,   /* a_j, b_j = min and max over the training pixels */
  CVAMX_STRETCH_PERCENTILE = 3  /* a_j, b_j = the pct-th and (100 - pct)-th
                                   percentiles, linear interpolation between
                                   order statistics at (P - 1) q as NumPy's
                                   default; the values beyond are clamped */
};

/* Stretch planar float images to 8 or 16 bits:
 *   q_jp = clamp(floor(L (y_jp - a_j) / (b_j - a_j) + 1/2), 0, L),
 *   L = 255 or 65535, evaluated in FP64 operation by operation (exact for
 *   the FP32 input values; cva_project evaluates the same map in FP32 as
 *   floor(y s + o), so mode 1 here finds its range exactly and its bytes
 *   within one level); b_j = a_j gives q = 0.
 *   y        device, n_comp x P float32 (from cvamx_project_float),
 *            4-byte aligned
 *   mode     CVAMX_STRETCH_*
 *   pct      mode 3: percentage in [0, 50) (the paper names 0.01, 0.1, 1
 *            and 5); ignored otherwise
 *   train_pixels, n_train   mode 2: device int64 pixel indices
 *            (0..P-1, n_train >= 1, 8-byte aligned); ignored otherwise
 *   bits     8 (out is uint8) or 16 (out is uint16)
 *   out      device, n_comp x P planar, aligned to its element size
 *   range    host, 2*n_comp float64 (a_j, b_j pairs) or NULL
 * Order statistics are exact (radix select on the FP32 values); a_j, b_j
 * are interpolated in FP64.  Asynchronous on `stream` except that mode 2
 * synchronises to check the pixel list (a pixel outside 0..P-1:
 * CVAMX_E_INVALID_ARG, nothing written) and a non-NULL range
 * synchronises. */
int cvamx_stretch(cvamx_ctx* ctx, const float* y, int64_t P, int32_t n_comp,
                  int32_t mode, double pct, const int64_t* train_pixels,
                  int64_t n_train, int32_t bits, void* out, double* range,
                  void* stream);

/* Interleave three 8-bit planes into an RGB image (paper Section 2: three
 * grayscale images combined, the one with the clearest underwriting usually
 * in the green channel; Section 4: that image may fill two channels).
 *   r, g, b  device, P uint8 each, or NULL for an all-zero channel
 *   rgb      device, 3*P uint8: rgb[3p + c]
 * Asynchronous on `stream`. */
int cvamx_compose_rgb(cvamx_ctx* ctx, const uint8_t* r, const uint8_t* g,
                      const uint8_t* b, int64_t P, uint8_t* rgb, void* stream);

/* ---- pages as image stacks, many pages ------------------------------------ */

/* A page's band images as read from one image file per band (paper
 * Section 2: the multispectral images of a page, 8-bit), band-sequential
 * (B planes of P pixels), into the band-interleaved page the other calls
 * read.  uint8 and uint16 bands give a CVAMX_U16 page (values kept),
 * float32 bands a CVAMX_F32 page.
 *   bands    device, B x P, in_dtype (CVAMX_U8, CVAMX_U16, CVAMX_F32),
 *            aligned to its element size (16-byte aligned, P % 4 == 0 for
 *            full-width loads)
 *   cube     device, P x B (uint16, or float32 for float bands), 16-byte
 *            aligned
 * Asynchronous on `stream`. */
int cvamx_bands_to_cube(cvamx_ctx* ctx, const void* bands, int32_t in_dtype,
                        int32_t B, int64_t P, void* cube, void* stream);

/* One page of a batch for cvamx_run_pages.  All pointers are host memory;
 * page-locked memory (hipHostMalloc) lets its copies overlap the other
 * pages' work (ordinary memory works, without the overlap). */
typedef struct {
  const void* bands;        /* B x height x width band-sequential, in_dtype */
  const int64_t* pixels;    /* n_points training pixel indices (y * width + x) */
  const int8_t* classes;    /* n_points classes, -1 = skip */
  int64_t n_points;
  void* images;             /* out: n_comp x height x width, uint8 or uint16 */
  double* W;                /* out: bands x n_comp, or NULL */
  double* eigvals;          /* out: n_comp, or NULL */
  double* range;            /* out: 2 * n_comp (a_j, b_j) of the stretch, or NULL */
  int32_t status;           /* out: CVAMX_OK or this page's error code */
} cvamx_page;

/* CVA enhancement of many pages of one geometry (paper Section 4: a whole
 * manuscript, pages re-run with other training points): per page, the
 * band images to the page (cvamx_bands_to_cube), the fit from its points
 * (cva_fit_points), the float images (cvamx_project_float) and the
 * stretch (cvamx_stretch with mode, pct, bits; mode 2 takes the page's
 * points of any class).  The next page's host-to-device copy and the
 * previous page's image copy run on their own streams, overlapped with the
 * current page's kernels and its host eigensolve.  A page whose pointers
 * or sizes are bad, or whose fit fails (e.g. an empty class), gets that
 * status and the batch goes on; a device error stops the batch and is
 * returned.  Device memory: two staging slots of the band images and the
 * points, one page, its float images and two image slots, freed on return.
 * The batch runs on streams of its own after draining `stream`, and
 * returns when every page is done. */
int cvamx_run_pages(cvamx_ctx* ctx, int32_t in_dtype, int32_t bands,
                    int64_t height, int64_t width, int32_t K, int32_t n_comp,
                    int32_t prec, double ridge, int32_t mode, double pct,
                    int32_t bits, cvamx_page* pages, int32_t n_pages,
                    void* stream);

/* ---- numerical assessment ------------------------------------------------ */

/* Cluster-separation indices of labelled points on a set of images (paper
 * Section 3, Eqs. 1-5).  A point's feature vector X is the values of the
 * n_feat planes at its pixel; for each class k:
 *   A_k = mean of X over the class's points (centroid),
 *   S_k = mean of ||X - A_k||_p over the class's points (Eq. 1),
 * and for each pair M_ij = ||A_i - A_j||_p (Eq. 2),
 *   R_ij = (S_i + S_j) / M_ij (Eq. 3, Davies-Bouldin),
 *   D_ij = (M_ij - S_i - S_j) / max(S_i, S_j) (Eq. 5, Dunn),
 * with R_ii = D_ii = 0.  scores[0] = (1/K) sum_i max_{j != i} R_ij and
 * scores[1] = min_{i != j} (M_ij - S_i - S_j) / max_k S_k; with K = 2 they
 * are the paper's two-cluster values.
 *   images   device, n_feat x P planar, element type dtype (CVAMX_U8,
 *            CVAMX_U16, CVAMX_F32, CVAMX_BF16, CVAMX_F16), aligned to it
 *   pixels   device, N int64 pixel indices (0..P-1), 8-byte aligned
 *   classes  device, N int8 (-1 = skip, else 0..K-1), 16-byte aligned
 *   K        2..CVAMX_MAX_CLASSES; every class needs a point
 *   p        the norm's order, p >= 1 (the paper: usually 2)
 * Host outputs (each nullable except scores): centroids K x n_feat,
 * scatter K, dist K x K (M), dbi K x K (R), dunn K x K (D), scores 2.
 * Sums and distances in FP64 in a fixed order: repeatable bit for bit.
 * Synchronises `stream`.  A class outside -1..K-1 or a pixel outside the
 * page: CVAMX_E_INVALID_ARG; an empty class: CVAMX_E_EMPTY_CLASS. */
int cvamx_cluster_indices(cvamx_ctx* ctx, const void* images, int32_t dtype,
                          int64_t P, int32_t n_feat, const int64_t* pixels,
                          const int8_t* classes, int64_t N, int32_t K,
                          double p, double* centroids, double* scatter,
                          double* dist, double* dbi, double* dunn,
                          double* scores, void* stream);

/* ---- soft-label CVA ------------------------------------------------------ */

/* Fisher criterion J = sum of the C = min(K-1, B) generalized eigenvalues
 * of the weighted problem, with real per-pixel class weights w_pc
 * (n_c = sum_p w_pc, m_c, m and the scatters weighted accordingly).  Not in
 * the paper: it reduces to the paper's CVA for one-hot weights.
 *   X        device, N x B float32 (row-major), 16-byte aligned
 *   w        device, N x K float32 (row-major), 16-byte aligned
 *   prec     CVAMX_PREC_FP32: FP32 products and accumulation, on the FP32
 *            matrix instruction (or, with cvamx_set_plain_fp32, on the
 *            vector ALU); CVAMX_PREC_BF16X3 / F16X3: the weighted scatter
 *            on the 16-bit matrix units with each operand split into a
 *            16-bit head and tail (four products, FP32 accumulation, a
 *            power of two per chunk keeping the values in range); error
 *            per S_w entry at most (2 u^2 + 512 2^-24) sum_p |w_pc|
 *            |d_i| |d_j|, u = 2^-8 (bf16) or 2^-11 (fp16)
 * Host outputs: J; W B x C, eigvals C, mean B, class_means K x B (all
 * float64; keep them for cva_soft_backward).  Synchronises `stream`.
 * Misaligned X or w: CVAMX_E_UNSUPPORTED. */
int cva_soft_forward(cvamx_ctx* ctx, const float* X, const float* w,
                     int64_t N, int32_t B, int32_t K, int32_t prec,
                     double ridge, double* J, double* W, double* eigvals,
                     double* mean, double* class_means, void* stream);

/* Gradient of J with respect to the weights, scaled by dJ:
 *   dw_pc = dJ * sum_{k<C} [ (w_k^T (x_p - m))^2
 *                            - (1 + lambda_k) (w_k^T (x_p - m_c))^2 ]
 * (the terms for the null-space directions of S_b cancel).
 *   W, eigvals, mean, class_means   host, from cva_soft_forward
 *   X        device, N x B float32, 16-byte aligned
 *   dw       device, N x K float32
 * Asynchronous on `stream`. */
int cva_soft_backward(cvamx_ctx* ctx, const float* X, const double* W,
                      const double* eigvals, const double* mean,
                      const double* class_means, int64_t N, int32_t B,
                      int32_t K, double dJ, float* dw, void* stream);

/* One refinement step of the class weights along the gradient of J (paper
 * Section 4 calls for an automatic choice of training points; Section 3,
 * Eqs. 1-5, measures the result): for each pixel p,
 *   d = grad_p - mean_c(grad_pc)   (the part within the simplex's plane)
 *   v = w_p + step * d / max_c |d_c|   (v = w_p if d = 0)
 *   w_p = the Euclidean projection of v onto {w >= 0, sum_c w_c = 1}.
 * A pixel labelled with the wrong class has its weight moved towards the
 * class that raises the Fisher criterion most; a correctly labelled
 * one-hot pixel stays where it is.  grad: device N x K float32 (e.g. from
 * cva_soft_backward with dJ = 1); w: device N x K float32, updated in place;
 * both 4-byte aligned.  K in 2..32, step finite and >= 0.  Asynchronous on
 * `stream`. */
int cva_soft_update(cvamx_ctx* ctx, const float* grad, float* w, int64_t N,
                    int32_t K, double step, void* stream);

/* ---- plain FP32 reference path ------------------------------------------ */

/* With enable = 1, every FP32 request on this context runs the plain FP32
 * vector-ALU kernels whatever the page type: the class moments of the fits
 * and the PCA covariance (prec CVAMX_PREC_FP32), and all projections
 * (cva_project, pca_project, cva_fit_project, cvamx_project_float), and
 * the two forward passes of cva_soft_forward.  By
 * default uint16 pages take the matrix cores with exactly split operands
 * for the moments and the projections, and the soft-label passes take the
 * FP32 matrix instruction; the plain path is
 * the reference those paths are measured against (same FP32 accumulation,
 * so the same tolerances hold).  0 restores the default.  Host-only: never
 * fails for a valid context. */
int cvamx_set_plain_fp32(cvamx_ctx* ctx, int enable);

/* ---- projection schedule ------------------------------------------------ */

/* How cva_project, pca_project and cva_fit_project read the page (paper
 * Section 2: the float arrays are rescaled onto 0..255 by their page-wide
 * min and max, so every value is needed twice: once for the range, once
 * for the map).
 *   CVAMX_SCHEDULE_AUTO (default): the page is read once, for every page
 *     type and on the plain FP32 path too; pass 1 finds the range and
 *     stores every component value as fp16 (2 bytes per pixel and
 *     component, in scratch owned by the context: n_comp <= 8 planes of
 *     the page rounded up to 256 pixels), pass 2 maps the stored values.
 *     Pass 1 also bounds how far the fp16 rounding can move the argument
 *     of the map's floor: 255 (2^-11 max(|a_j|, |b_j|) + tiny terms) /
 *     (b_j - a_j) grey levels, at most 0.125 when the center lies inside
 *     the page's projected range (the fit's mean always does).  Beyond 0.5
 *     levels for some component, or when a stored value could have
 *     overflowed fp16, pass 2 re-reads the page instead (decided on the
 *     device), so every byte stays within one level of the two-read
 *     result.
 *   CVAMX_SCHEDULE_TWO_READS: the page is read twice (range, then map), as
 *     for the other page types.
 *   CVAMX_SCHEDULE_FORCE_REREAD: pass 1 of the one-read schedule, then the
 *     fallback of pass 2, whatever the bound (for testing the fallback).
 * The ranges are identical under all three. */
enum {
  CVAMX_SCHEDULE_AUTO = 0,
  CVAMX_SCHEDULE_TWO_READS = 1,
  CVAMX_SCHEDULE_FORCE_REREAD = 2
};
/* Host-only; unknown values: CVAMX_E_INVALID_ARG. */
int cvamx_set_schedule(cvamx_ctx* ctx, int schedule);

/* ---- measurement ----------------------------------------------------------- */

/* The read ceiling the page passes are measured against: reads `bytes` (a
 * positive multiple of 16) of device memory at src (16-byte aligned) once,
 * with non-temporal 16-byte loads, eight in flight per thread, as the page
 * passes stream the page, and no arithmetic beyond folding the words
 * together.  sink (device, 4-byte aligned) receives one word only if the
 * fold happens to equal a fixed key (a guard against the loads being
 * optimised away).  Asynchronous on `stream`. */
int cvamx_stream_read(cvamx_ctx* ctx, const void* src, int64_t bytes,
                      uint32_t* sink, void* stream);

/* The ceiling for a pass that writes as it reads: the stream above over
 * read_bytes of src, and, spread evenly over it, write_bytes of dst (device,
 * 16-byte aligned, write_bytes <= read_bytes, both positive multiples of
 * 16) written once with non-temporal 16-byte stores of the words just read.
 * dst's contents afterwards are unspecified.  Bad sizes:
 * CVAMX_E_INVALID_ARG; misaligned pointers: CVAMX_E_UNSUPPORTED.
 * Asynchronous on `stream`. */
int cvamx_stream_mix(cvamx_ctx* ctx, const void* src, int64_t read_bytes,
                     void* dst, int64_t write_bytes, uint32_t* sink,
                     void* stream);

/* ---- kernel timing ------------------------------------------------------ */

/* Per-kernel timing on this context: with enable = 1 every kernel the
 * library launches is bracketed by a pair of HIP events on its stream; with
 * 2 only the page-streaming projection passes are (their names begin with
 * "project_"), which keeps the event records out of the short kernels of
 * the fits; 0 (or any other value) disables it.  Enabling clears the
 * accumulated totals.  Costs two event records per timed launch. */
int cvamx_profile_enable(cvamx_ctx* ctx, int enable);

/* Wait for the timed kernels and write one text line per kernel name,
 * "name launches total_ms\n", into buf (NUL terminated, truncated to len).
 * Returns the length needed including the NUL, or a negative status. */
int64_t cvamx_profile_report(cvamx_ctx* ctx, char* buf, int64_t len);

/* ---- host-only FP64 finishers (no GPU needed) ---------------------------- */

/* The CVA solve from class moments: S_b from counts and class means,
 * Cholesky of S_w + ridge I, generalized symmetric-definite eigenproblem,
 * descending order, sign rule (paper Section 4, generalized
 * symmetric-definite eigensolver).  counts K, class_means K x B, Sw B x B
 * (host).  Outputs W B x n_comp, eigvals n_comp, mean B (may be NULL). */
int cva_solve_moments(const int64_t* counts, const double* class_means,
                      const double* Sw, int32_t K, int32_t B, double ridge,
                      int32_t n_comp, double* W, double* eigvals, double* mean);

/* Full symmetric eigendecomposition of an n x n row-major matrix A (host,
 * only its lower triangle is read): eigenvalues descending into w[n],
 * orthonormal eigenvectors as the columns of V (n x n row-major), sign rule
 * applied.  Householder tridiagonalisation then implicit QR steps with a
 * Wilkinson shift. */
int cvamx_sym_eig(int32_t n, const double* A, double* w, double* V);

/* The k leading eigenpairs of an n x n row-major symmetric matrix A (host,
 * lower triangle read), 1 <= k <= n: all n eigenvalues descending into w[n],
 * the eigenvectors of the k largest as the orthonormal columns of V (n x k
 * row-major), sign rule applied.  Eigenvalues by implicit QR steps on the
 * Householder tridiagonal form with no vector accumulation, the k vectors by
 * inverse iteration on it (kept orthogonal within clusters of eigenvalues
 * closer than 1e-3 of the matrix norm), then mapped back through the stored
 * reflectors; when k exceeds n / 4 it is cvamx_sym_eig's decomposition.
 * PCA needs only its leading axes (paper Section 2). */
int cvamx_sym_eig_top(int32_t n, const double* A, int32_t k, double* w, double* V);

#ifdef __cplusplus
}
#endif
#endif /* CVAMX_H */

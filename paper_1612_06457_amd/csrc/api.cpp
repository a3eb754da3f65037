// C ABI of the cvamx library: argument checking, scratch management,
// kernel orchestration on the caller's HIP stream, and the FP64 finish of
// every fit on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ctx_internal.hpp"
#include "cvamx.h"
#include "finisher.h"
#include "launch.hpp"

namespace {

enum Buf { B_TILECNT, B_IDX, B_PART, B_RES, B_PROJPART, B_FIRST, B_MCF, B_SPART, B_SHIST, B_SFIX, B_H16,
           B_PPART, B_PRES, B_COUNT };

}  // namespace

struct cvamx_ctx {
  int device = -1;
  int num_cu = 256;
  int proj_blocks = 0;   // 0 = automatic
  bool plain = false;    // FP32 requests on the plain vector-ALU kernels
  int schedule = CVAMX_SCHEDULE_AUTO;   // projection schedule (cvamx_set_schedule)
  bool pca_standardize = false;         // pca_fit on the correlation matrix (cvamx_set_pca_standardize)
  int gram_blocks = 0;
  std::string err;
  void* buf[B_COUNT] = {};
  size_t cap[B_COUNT] = {};
  void* pinned = nullptr;     // page-locked staging of small results
  size_t pinned_cap = 0;
  void* pinned2 = nullptr;    // a second one, for the PCA half of cvamx_cva_pca
  size_t pinned2_cap = 0;
  hipEvent_t ev_fit = nullptr, ev_pca = nullptr;   // cvamx_cva_pca's two hand-over points
  unsigned* tickets = nullptr;   // [0] projection range
  float* range_dev = nullptr;    // 16 floats: scale[8], offset[8] of the current group
  float* ab_dev = nullptr;       // 2 * CVAMX_MAX_BANDS floats: (min, max) per component
  // kernel timing (cvamx_profile_enable)
  int prof = 0;   // 0 off, 1 every kernel, 2 the page-streaming projection passes only
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  std::map<std::string, std::pair<long, double>> prof_acc;
  // state of the page batches (pipeline.cpp), freed through module_free
  void* module = nullptr;
  void (*module_free)(void*) = nullptr;
};

namespace {

int fail(cvamx_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_fail(cvamx_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, CVAMX_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, where)                         \
  do {                                               \
    hipError_t _e = (call);                          \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

int ensure(cvamx_ctx* ctx, Buf b, size_t bytes) {
  if (ctx->cap[b] >= bytes && ctx->buf[b]) return 0;
  if (ctx->buf[b]) {
    hipError_t e = hipFree(ctx->buf[b]);
    ctx->buf[b] = nullptr;
    ctx->cap[b] = 0;
    if (e != hipSuccess) return hip_fail(ctx, e, "hipFree");
  }
  size_t want = std::max<size_t>(bytes, 256);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) return fail(ctx, CVAMX_E_NO_MEMORY, "hipMalloc of scratch failed");
  ctx->buf[b] = p;
  ctx->cap[b] = want;
  return 0;
}

int ensure_pinned(cvamx_ctx* ctx, size_t bytes, int slot = 0) {
  void*& pin = slot == 0 ? ctx->pinned : ctx->pinned2;
  size_t& cap = slot == 0 ? ctx->pinned_cap : ctx->pinned2_cap;
  if (cap >= bytes && pin) return 0;
  if (pin) {
    (void)hipHostFree(pin);
    pin = nullptr;
    cap = 0;
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, std::max<size_t>(bytes, 4096), hipHostMallocDefault) != hipSuccess)
    return fail(ctx, CVAMX_E_NO_MEMORY, "hipHostMalloc of staging failed");
  pin = p;
  cap = std::max<size_t>(bytes, 4096);
  return 0;
}

// Small results into the context's page-locked staging buffer.  A kernel
// writes them, not the copy engines, so they never wait behind a large
// transfer queued on another stream.
hipError_t to_pinned(cvamx_ctx* ctx, const void* src, size_t bytes, hipStream_t s) {
  return cvx::launch_copy_out(ctx->pinned, src, (int64_t)bytes, s);
}

hipEvent_t get_event(cvamx_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Bracket one kernel launch with events when timing is enabled.
void prof_begin(cvamx_ctx* ctx, hipStream_t s, const char* name) {
  if (!ctx->prof) return;
  if (ctx->prof == 2 && std::strncmp(name, "project_", 8) != 0) return;
  hipEvent_t a = get_event(ctx);
  if (!a) return;
  (void)hipEventRecord(a, s);
  ctx->pending.push_back({name, a, nullptr});
}

void prof_end(cvamx_ctx* ctx, hipStream_t s) {
  if (!ctx->prof || ctx->pending.empty() || ctx->pending.back().b) return;
  hipEvent_t b = get_event(ctx);
  if (!b) return;
  (void)hipEventRecord(b, s);
  ctx->pending.back().b = b;
}

void prof_collect(cvamx_ctx* ctx) {
  for (auto& p : ctx->pending) {
    if (p.b) {
      float ms = 0.f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto& e = ctx->prof_acc[p.name];
        e.first += 1;
        e.second += ms;
      }
      ctx->ev_pool.push_back(p.b);
    }
    ctx->ev_pool.push_back(p.a);
  }
  ctx->pending.clear();
}

size_t esize(int dtype) { return dtype == CVAMX_F32 ? 4 : 2; }

// For uint16 pages the scatter kernels centre on an integer, so x - c is an
// integer below 2^17 in magnitude and its two-term bf16 (or fp16) split is
// exact: every matrix-core product is exact and only the FP32 accumulation
// rounds, as on the FP32 VALU path.  FP32 requests on such pages therefore
// take the matrix-core kernels (bf16 split).
bool split_is_exact(int dtype) { return dtype == CVAMX_U16; }

// Round to the nearest bf16 / fp16 value (ties to even), returned as double.
double bf16_round(double x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

double f16_round(double x) {
  // fp16 has 11 significant bits; values here lie well inside its normal range
  if (x == 0.0 || !std::isfinite(x)) return x;
  int e;
  std::frexp(x, &e);
  const double q = std::ldexp(1.0, e - 11);
  return std::nearbyint(x / q) * q;
}

int check_cube(cvamx_ctx* ctx, const cvamx_cube* c) {
  if (!c) return fail(ctx, CVAMX_E_INVALID_ARG, "cube is NULL");
  if (!c->data) return fail(ctx, CVAMX_E_INVALID_ARG, "cube data is NULL");
  if (c->height < 1 || c->width < 1 || c->bands < 1)
    return fail(ctx, CVAMX_E_INVALID_ARG, "cube dimensions must be positive");
  if (c->bands > CVAMX_MAX_BANDS)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "bands > CVAMX_MAX_BANDS");
  if (c->dtype < CVAMX_U16 || c->dtype > CVAMX_F16)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "unknown dtype");
  if (c->height > (int64_t(1) << 31) || c->width > (int64_t(1) << 31))
    return fail(ctx, CVAMX_E_INVALID_ARG, "cube dimensions overflow");
  const int64_t P = c->height * c->width;
  if (P >= (int64_t(1) << 31) - 1)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "pages with 2^31 or more pixels are not supported");
  if ((reinterpret_cast<uintptr_t>(c->data) & 15u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "cube data must be 16-byte aligned");
  return 0;
}

int check_device(cvamx_ctx* ctx) {
  if (ctx->device < 0) return fail(ctx, CVAMX_E_DEVICE, "context has no device");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  return 0;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

// Expand the packed upper-triangular 4x4 tiles of an (B+1) x (B+1)
// augmented Gram into a full symmetric matrix.
void unpack_gram(int B, const double* packed, std::vector<double>& G) {
  const int BP = cvx::padded_bp(B), nb = BP / 4, n1 = B + 1;
  G.assign((size_t)n1 * n1, 0.0);
  int blk = 0;
  for (int bi = 0; bi < nb; ++bi)
    for (int bj = bi; bj < nb; ++bj, ++blk)
      for (int e = 0; e < 16; ++e) {
        const int i = 4 * bi + e / 4, j = 4 * bj + e % 4;
        if (i < n1 && j < n1) {
          G[(size_t)i * n1 + j] = packed[blk * 16 + e];
          G[(size_t)j * n1 + i] = packed[blk * 16 + e];
        }
      }
}

// Layout of the fit result region (device, copied to host in one go).
struct FitLayout {
  size_t counts, offsets, err, shift, gram, total;
  FitLayout(int K, int B, int L) {
    counts = 0;
    offsets = counts + 8 * (size_t)K;
    err = offsets + ((4 * (size_t)(K + 1) + 7) & ~size_t(7));
    shift = err + 8;
    gram = shift + 8 * (size_t)K * B;
    total = gram + 8 * (size_t)K * L;
  }
};

// Wave tiles of the projection kernels, and their block count.
int proj_nblocks(cvamx_ctx* ctx, const cvamx_cube* cube) {
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  const int g2 = (cube->dtype != CVAMX_F32 && (B & 1)) ? 2 : 1;
  const int64_t nt = (P + 64 * g2 - 1) / (64 * g2);
  const int nblocks = ctx->proj_blocks > 0 ? ctx->proj_blocks : ctx->num_cu * 8;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nblocks, (nt + cvx::kWaves - 1) / cvx::kWaves));
}

// Whether a group of nc components projects on the vector-ALU passes: on
// the plain FP32 path, and for every page type but uint16 (uint16 pages take
// the matrix cores at any component count: at three components the two
// forms measured within 1 %, from four on the matrix cores win, by 13 % at
// seven).
bool proj_vector(const cvamx_ctx* ctx, const cvamx_cube* cube, int /*nc*/) {
  return ctx->plain || cube->dtype != CVAMX_U16;
}

// The kernel arguments of components g0 .. g0 + nc - 1.
void make_proj_args(const cvamx_cube* cube, const double* W, const double* center, int n_comp, int g0, int nc,
                    bool plain, cvx::ProjArgs& a) {
  const int B = (int)cube->bands;
  std::memset(&a, 0, sizeof(a));
  double c[CVAMX_MAX_BANDS];   // on the stack: the allocation-free entry point comes through here
  for (int b = 0; b < B; ++b) {
    // uint16 pages: an integer centre, passed as 2^23 + c (exact in FP32),
    // which the kernels subtract from the bit-built float 2^23 + x
    // bf16 / fp16 pages: a centre of the page's own type, so that x - c of
    // two such values is exact in FP32 whenever their exponents are within
    // 16 (bf16) or 13 (fp16) of each other; the FP64 offset below absorbs
    // the difference between c and the requested centre either way
    switch (cube->dtype) {
      case CVAMX_U16: c[b] = std::nearbyint(center[b]); break;
      case CVAMX_BF16: c[b] = bf16_round(center[b]); break;
      case CVAMX_F16: c[b] = f16_round(center[b]); break;
      default: c[b] = (double)(float)center[b]; break;
    }
    a.c[b] = (cube->dtype == CVAMX_U16) ? (float)(8388608.0 + c[b]) : (float)c[b];
  }
  for (int j = 0; j < nc; ++j) {
    double off = 0.0;
    for (int b = 0; b < B; ++b) {
      const double wv = W[(size_t)b * n_comp + g0 + j];
      a.w[b * nc + j] = (float)wv;
      off += wv * (c[b] - center[b]);
      // uint16 pages on the matrix cores: the kernels multiply 1024 + (x mod
      // 1024) rather than its centred value, so the constant 1024 + (c mod
      // 1024) comes off here (the plain kernels use x - c itself)
      if (cube->dtype == CVAMX_U16 && !plain)
        off -= (double)a.w[b * nc + j] * (1024.0 + std::fmod(c[b], 1024.0));
    }
    a.off[j] = (float)off;
    // a power of two that brings the largest |W[b][j]| into [16, 32)
    double wmax = 0.0;
    for (int b = 0; b < B; ++b) wmax = std::max(wmax, std::fabs((double)a.w[b * nc + j]));
    int ex = 0;
    if (wmax > 0.0) std::frexp(wmax, &ex);
    a.scale[j] = (float)std::ldexp(1.0, wmax > 0.0 ? 5 - ex : 0);
  }
}

// Device buffers of the two projection passes: block partials (at most 32
// floats per block), the last-block ticket (zero between calls), the
// stretch map of the current group and the range of every component.
struct ProjBufs {
  float* part;
  unsigned* ticket;
  float* range_dev;
  float* ab_dev;
};

int proj_groups_with(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center,
                     int n_comp, uint8_t* images, const ProjBufs& pb, bool timed, hipStream_t s) {
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  const int nblocks = proj_nblocks(ctx, cube);
  for (int g0 = 0; g0 < n_comp; g0 += 8) {
    const int nc = std::min(8, n_comp - g0);   // the kernels are instantiated for 1..8 components
    const bool pv = proj_vector(ctx, cube, nc);
    cvx::ProjArgs a;
    make_proj_args(cube, W, center, n_comp, g0, nc, pv, a);
    static const char* kRangeName[9] = {"", "project_range_nc1", "project_range_nc2", "project_range_nc3",
                                        "project_range_nc4", "project_range_nc5", "project_range_nc6",
                                        "project_range_nc7", "project_range_nc8"};
    static const char* kStretchName[9] = {"", "project_stretch_nc1", "project_stretch_nc2", "project_stretch_nc3",
                                          "project_stretch_nc4", "project_stretch_nc5", "project_stretch_nc6",
                                          "project_stretch_nc7", "project_stretch_nc8"};
    if (timed) prof_begin(ctx, s, kRangeName[nc]);
    hipError_t e = cvx::launch_project_range(cube->dtype, pv, cube->data, B, P, nc, a, nblocks, pb.part,
                                             pb.ticket, pb.range_dev, pb.ab_dev + 2 * g0, s);
    if (timed) prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "project range launch");
    if (timed) prof_begin(ctx, s, kStretchName[nc]);
    e = cvx::launch_project_stretch(cube->dtype, pv, cube->data, B, P, nc, a, nblocks, pb.range_dev,
                                    images + (int64_t)g0 * P, s);
    if (timed) prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "project stretch launch");
  }
  return 0;
}

// Storage factors of the fp16 intermediate for one group of components: the
// power of two f_j that keeps a bound on the values the kernels store at or
// below 2^15 (fp16's largest value is 65504), with a margin for the FP32
// rounding of the sums.  uint16 and fp16 pages bound every value:
// |y_j| <= sum_b |W[b][j]| max |x - c_b| over the element range; the
// matrix-core passes of uint16 pages store 2^s_j y_j.  bf16 and float32
// pages have no useful bound, so |x - c_b| <= 1024 (|c_b| + 1) is assumed:
// a page outside it makes pass 1 see a stored value beyond the limit and
// pass 2 re-read the page, so the images are right either way, and fp16's
// thirty binades leave that much headroom at no cost in precision.
void h16_args(const cvx::ProjArgs& a, const double* center, int B, int nc, int dtype, bool scaled, float limit,
              cvx::H16Args& h) {
  std::memset(&h, 0, sizeof(h));
  for (int j = 0; j < nc; ++j) {
    double bnd = 0.0;
    for (int b = 0; b < B; ++b) {
      const double c = std::fabs(center[b]);
      double dx;
      switch (dtype) {
        case CVAMX_U16: dx = std::max(c, std::fabs(65535.0 - center[b])); break;
        case CVAMX_F16: dx = 65504.0 + c; break;
        default: dx = 1024.0 * (c + 1.0); break;
      }
      bnd += std::fabs((double)a.w[b * nc + j]) * dx;
    }
    bnd *= (scaled ? (double)a.scale[j] : 1.0) * (1.0 + 1.0 / 1024.0);
    int ex = 0;
    if (bnd > 0.0) {
      std::frexp(32768.0 / bnd, &ex);   // 32768 / bnd in [2^(ex-1), 2^ex)
      ex -= 1;
    }
    ex = std::max(-60, std::min(60, ex));
    h.f[j] = (float)std::ldexp(1.0, ex);
  }
  h.limit = limit;
}

// The one-read schedule: pass 1 reads the page once for the range and
// stores every component value in fp16; pass 2 quantises the stored values
// (or re-reads the page, decided on the device, when their error bound
// exceeds the limit).
int proj_groups_h16(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center, int n_comp,
                    uint8_t* images, const ProjBufs& pb, hipStream_t s) {
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  const int64_t Pp = (P + 255) / 256 * 256;
  const int nblocks = proj_nblocks(ctx, cube);
  if (int st = ensure(ctx, B_H16, (size_t)std::min(n_comp, 8) * (size_t)Pp * 2)) return st;
  uint16_t* planes = static_cast<uint16_t*>(ctx->buf[B_H16]);
  const float limit = ctx->schedule == CVAMX_SCHEDULE_FORCE_REREAD ? -1.f : 0.5f;
  for (int g0 = 0; g0 < n_comp; g0 += 8) {
    const int nc = std::min(8, n_comp - g0);
    const bool pv = proj_vector(ctx, cube, nc);
    cvx::ProjArgs a;
    make_proj_args(cube, W, center, n_comp, g0, nc, pv, a);
    cvx::H16Args h;
    h16_args(a, center, B, nc, cube->dtype, cube->dtype == CVAMX_U16 && !pv, limit, h);
    static const char* kRangeName[9] = {"", "project_range_store_nc1", "project_range_store_nc2",
                                        "project_range_store_nc3", "project_range_store_nc4",
                                        "project_range_store_nc5", "project_range_store_nc6",
                                        "project_range_store_nc7", "project_range_store_nc8"};
    static const char* kStretchName[9] = {"", "project_stretch_stored_nc1", "project_stretch_stored_nc2",
                                          "project_stretch_stored_nc3", "project_stretch_stored_nc4",
                                          "project_stretch_stored_nc5", "project_stretch_stored_nc6",
                                          "project_stretch_stored_nc7", "project_stretch_stored_nc8"};
    prof_begin(ctx, s, kRangeName[nc]);
    hipError_t e = cvx::launch_project_range_h16(cube->dtype, pv, cube->data, B, P, nc, a, nblocks, pb.part,
                                                 pb.ticket, pb.range_dev, pb.ab_dev + 2 * g0, h, planes, Pp, s);
    prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "project range launch");
    prof_begin(ctx, s, kStretchName[nc]);
    e = cvx::launch_project_stretch_h16(cube->dtype, pv, cube->data, B, P, nc, a, nblocks, pb.range_dev,
                                        planes, Pp, images + (int64_t)g0 * P, s);
    prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "project stretch launch");
  }
  return 0;
}

int proj_groups(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center,
                int n_comp, uint8_t* images, hipStream_t s) {
  const int nblocks = proj_nblocks(ctx, cube);
  // block partials: 16 floats (VALU kernels) or 32 (matrix-core kernels)
  if (int st = ensure(ctx, B_PROJPART, (size_t)nblocks * 32 * sizeof(float))) return st;
  const ProjBufs pb{(float*)ctx->buf[B_PROJPART], ctx->tickets, ctx->range_dev, ctx->ab_dev};
  if (ctx->schedule != CVAMX_SCHEDULE_TWO_READS) return proj_groups_h16(ctx, cube, W, center, n_comp, images, pb, s);
  return proj_groups_with(ctx, cube, W, center, n_comp, images, pb, true, s);
}

// Checks shared by the projection entry points.
int check_proj_args(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center,
                    int32_t n_comp, const void* out) {
  if (int st = check_cube(ctx, cube)) return st;
  if (!W || !center || !out) return fail(ctx, CVAMX_E_INVALID_ARG, "W, center and the output must be non-NULL");
  if (n_comp < 1 || n_comp > CVAMX_MAX_BANDS)
    return fail(ctx, CVAMX_E_INVALID_ARG, "n_comp must lie in 1..CVAMX_MAX_BANDS");
  const int B = (int)cube->bands;
  for (int i = 0; i < B * n_comp; ++i)
    if (!std::isfinite(W[i])) return fail(ctx, CVAMX_E_INVALID_ARG, "W has a non-finite entry");
  for (int b = 0; b < B; ++b)
    if (!std::isfinite(center[b])) return fail(ctx, CVAMX_E_INVALID_ARG, "center has a non-finite entry");
  return 0;
}

int project_common(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center,
                   int32_t n_comp, uint8_t* images, float* range, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (int st = check_proj_args(ctx, cube, W, center, n_comp, images)) return st;
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  if (int st = proj_groups(ctx, cube, W, center, n_comp, images, s)) return st;
  if (range) {
    if (int st = ensure_pinned(ctx, 2 * sizeof(float) * n_comp)) return st;
    HIP_TRY(to_pinned(ctx, ctx->ab_dev, 2 * sizeof(float) * n_comp, s), "range copy");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    std::memcpy(range, ctx->pinned, 2 * sizeof(float) * n_comp);
  }
  return 0;
}

}  // namespace

namespace cvamx {
int set_error(cvamx_ctx* ctx, int code, const std::string& msg) { return fail(ctx, code, msg); }
int ctx_device(const cvamx_ctx* ctx) { return ctx ? ctx->device : -1; }
void** ctx_module_state(cvamx_ctx* ctx) { return &ctx->module; }
void ctx_set_module_free(cvamx_ctx* ctx, void (*fn)(void*)) { ctx->module_free = fn; }
}  // namespace cvamx

extern "C" {

const char* cvamx_status_str(int st) {
  switch (st) {
    case CVAMX_OK: return "ok";
    case CVAMX_E_INVALID_ARG: return "invalid argument";
    case CVAMX_E_UNSUPPORTED: return "unsupported";
    case CVAMX_E_EMPTY_CLASS: return "empty class";
    case CVAMX_E_NOT_PD: return "within-class scatter not positive definite";
    case CVAMX_E_DEVICE: return "device error";
    case CVAMX_E_NO_MEMORY: return "out of memory";
    case CVAMX_E_NUMERIC: return "eigensolver did not converge";
    default: return "unknown status";
  }
}

const char* cvamx_last_error(const cvamx_ctx* ctx) {
  if (!ctx) return "no context";
  return ctx->err.c_str();
}

int cvamx_create(cvamx_ctx** out, int device) {
  if (!out) return CVAMX_E_INVALID_ARG;
  *out = nullptr;
  cvamx_ctx* ctx = new (std::nothrow) cvamx_ctx();
  if (!ctx) return CVAMX_E_NO_MEMORY;
  if (device < -1) {
    delete ctx;
    return CVAMX_E_INVALID_ARG;
  }
  if (device >= 0) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
      delete ctx;
      return CVAMX_E_DEVICE;
    }
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
      delete ctx;
      return CVAMX_E_DEVICE;
    }
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
      ctx->num_cu = cu;
    if (const char* v = std::getenv("CVAMX_PROJ_BLOCKS")) ctx->proj_blocks = std::atoi(v);
    if (const char* v = std::getenv("CVAMX_GRAM_BLOCKS")) ctx->gram_blocks = std::atoi(v);
    void* p = nullptr;
    const size_t small = 256 + 256 + 2 * CVAMX_MAX_BANDS * sizeof(float);
    if (hipMalloc(&p, small) != hipSuccess) {
      delete ctx;
      return CVAMX_E_NO_MEMORY;
    }
    if (hipMemset(p, 0, small) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      (void)hipFree(p);
      delete ctx;
      return CVAMX_E_DEVICE;
    }
    if (cvx::scratch_setup(device) != hipSuccess) {
      (void)hipFree(p);
      delete ctx;
      return CVAMX_E_DEVICE;
    }
    ctx->tickets = static_cast<unsigned*>(p);
    ctx->range_dev = reinterpret_cast<float*>(static_cast<char*>(p) + 256);
    ctx->ab_dev = reinterpret_cast<float*>(static_cast<char*>(p) + 512);
  }
  *out = ctx;
  return CVAMX_OK;
}

void cvamx_destroy(cvamx_ctx* ctx) {
  if (!ctx) return;
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->module && ctx->module_free) ctx->module_free(ctx->module);
    for (int b = 0; b < B_COUNT; ++b)
      if (ctx->buf[b]) (void)hipFree(ctx->buf[b]);
    if (ctx->tickets) (void)hipFree(ctx->tickets);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->pinned2) (void)hipHostFree(ctx->pinned2);
    if (ctx->ev_fit) (void)hipEventDestroy(ctx->ev_fit);
    if (ctx->ev_pca) (void)hipEventDestroy(ctx->ev_pca);
    prof_collect(ctx);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  }
  delete ctx;
}

// Arguments shared by the two fit entry points.
static int check_fit_args(cvamx_ctx* ctx, const cvamx_cube* cube, int32_t K, int32_t prec, double ridge,
                   int32_t n_comp, const double* W, const double* eigvals, const double* mean,
                   const int64_t* counts) {
  if (int st = check_cube(ctx, cube)) return st;
  if (K < 2 || K > CVAMX_MAX_CLASSES) return fail(ctx, CVAMX_E_INVALID_ARG, "K must lie in 2..127");
  if (prec < CVAMX_PREC_FP32 || prec > CVAMX_PREC_F16X3)
    return fail(ctx, CVAMX_E_INVALID_ARG, "unknown precision");
  if (!finite_nonneg(ridge)) return fail(ctx, CVAMX_E_INVALID_ARG, "ridge must be finite and >= 0");
  const int C = std::min(K - 1, (int)cube->bands);
  if (n_comp < 1 || n_comp > C) return fail(ctx, CVAMX_E_INVALID_ARG, "n_comp must lie in 1..min(K-1, bands)");
  if (!W || !eigvals || !mean || !counts)
    return fail(ctx, CVAMX_E_INVALID_ARG, "W, eigvals, mean and counts must be non-NULL");
  return 0;
}

// The class-grouped index list of training pixels: from a label map of P
// entries (list = nullptr), or from a list of N (pixel, class) points, where
// the label kernels run over the N classes and their positions are then
// mapped to pixels.  Counts, offsets and the error flag land in the results
// region; returns the number of label entries scanned.
static int build_index(cvamx_ctx* ctx, const int8_t* labels, const int64_t* points, int64_t n, int64_t P, int K,
                const FitLayout& lay, char* res, hipStream_t s) {
  const int nW = (int)((n + cvx::kLabelWave - 1) / cvx::kLabelWave);
  const size_t ld = (size_t)cvx::label_row_stride(nW);
  if (int st = ensure(ctx, B_TILECNT, (ld * (K + 1) + K + 1) * 4)) return st;
  int32_t* wave_counts = (int32_t*)ctx->buf[B_TILECNT];
  int32_t* class_total = wave_counts + ld * (K + 1);
  if (int st = ensure(ctx, B_IDX, (size_t)n * 4)) return st;
  hipError_t e;
  prof_begin(ctx, s, "label_count");
  e = cvx::launch_label_count(labels, n, K, nW, wave_counts, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "label count launch");
  prof_begin(ctx, s, "label_scan");
  e = cvx::launch_label_scan(wave_counts, nW, K, class_total, (int32_t*)(res + lay.err), s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "label scan launch");
  prof_begin(ctx, s, "label_index");
  e = cvx::launch_label_index(labels, n, K, nW, wave_counts, class_total, (int32_t*)ctx->buf[B_IDX],
                              (int64_t*)(res + lay.counts), (int32_t*)(res + lay.offsets), s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "label index launch");
  if (points) {
    prof_begin(ctx, s, "points_to_pixels");
    e = cvx::launch_points_to_pixels(points, (int32_t*)ctx->buf[B_IDX], (const int32_t*)(res + lay.offsets), K, n,
                                     P, (int32_t*)(res + lay.err), ctx->num_cu, s);
    prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "point mapping launch");
  }
  return 0;
}

// Class moments and their reduction into the page-locked staging buffer
// (with the results header: counts, offsets, flags, shifts).
static int fit_moments_launch(cvamx_ctx* ctx, const cvamx_cube* cube, int32_t K, int32_t prec,
                              const FitLayout& lay, char* res, int G, int L, hipStream_t s) {
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  hipError_t e;
  if (prec == CVAMX_PREC_FP32 && (ctx->plain || !split_is_exact(cube->dtype))) {
    prof_begin(ctx, s, "class_moments");
    e = cvx::launch_class_moments(cube->dtype, cube->data, B, P, (const int32_t*)ctx->buf[B_IDX],
                                  (const int32_t*)(res + lay.offsets), K, G, (double*)ctx->buf[B_PART],
                                  (double*)(res + lay.shift), s);
  } else {
    prof_begin(ctx, s, "class_moments_mfma");
    e = cvx::launch_class_moments_mfma(cube->dtype, prec == CVAMX_PREC_F16X3 ? 1 : 0, cube->data, B, P,
                                       (const int32_t*)ctx->buf[B_IDX], (const int32_t*)(res + lay.offsets), K,
                                       G, (double*)ctx->buf[B_PART], (double*)(res + lay.shift), s);
  }
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "class moments launch");
  prof_begin(ctx, s, "reduce_partials");
  char* h = static_cast<char*>(ctx->pinned);
  e = cvx::launch_reduce_part_out((const double*)ctx->buf[B_PART], K, G, L, (double*)(h + lay.gram), res, h,
                                  (int64_t)lay.gram, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
  return 0;
}

// The FP64 finish on the host, once the reduction has landed in staging.
static int fit_host_finish(cvamx_ctx* ctx, int B, int32_t K, double ridge, int32_t n_comp, double* W,
                           double* eigvals, double* mean, int64_t* counts, double* class_means, double* Sw,
                           double* Sb, const FitLayout& lay, int L) {
  const char* h = static_cast<const char*>(ctx->pinned);
  int32_t errflag;
  std::memcpy(&errflag, h + lay.err, 4);
  if (errflag & 1) return fail(ctx, CVAMX_E_INVALID_ARG, "a label lies outside -1..K-1");
  if (errflag & 2) return fail(ctx, CVAMX_E_INVALID_ARG, "a training point lies outside the page");
  std::vector<int64_t> cnt(K);
  std::memcpy(cnt.data(), h + lay.counts, 8 * (size_t)K);
  for (int k = 0; k < K; ++k)
    if (cnt[k] < 1) return fail(ctx, CVAMX_E_EMPTY_CLASS, "class " + std::to_string(k) + " has no training pixel");
  const double* shift = reinterpret_cast<const double*>(h + lay.shift);
  const double* gram = reinterpret_cast<const double*>(h + lay.gram);
  std::vector<double> cm((size_t)K * B), Swv((size_t)B * B, 0.0), G1, cntd(K);
  for (int k = 0; k < K; ++k) {
    unpack_gram(B, gram + (size_t)k * L, G1);
    const double n = (double)cnt[k];
    cntd[k] = n;
    const int n1 = B + 1;
    for (int i = 0; i < B; ++i) cm[(size_t)k * B + i] = shift[(size_t)k * B + i] + G1[(size_t)i * n1 + B] / n;
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < B; ++j)
        Swv[(size_t)i * B + j] += G1[(size_t)i * n1 + j] - G1[(size_t)i * n1 + B] * G1[(size_t)j * n1 + B] / n;
  }
  std::vector<double> Wt((size_t)B * n_comp), lam(n_comp), m(B), Sbv((size_t)B * B);
  const int st = cvamx::cva_solve(K, B, cntd.data(), cm.data(), Swv.data(), ridge, n_comp, Wt.data(),
                                  lam.data(), m.data(), Sb ? Sbv.data() : nullptr, &ctx->err);
  if (st != 0) return st;
  std::copy(Wt.begin(), Wt.end(), W);
  std::copy(lam.begin(), lam.end(), eigvals);
  std::copy(m.begin(), m.end(), mean);
  std::copy(cnt.begin(), cnt.end(), counts);
  if (class_means) std::copy(cm.begin(), cm.end(), class_means);
  if (Sw) std::copy(Swv.begin(), Swv.end(), Sw);
  if (Sb) std::copy(Sbv.begin(), Sbv.end(), Sb);
  return CVAMX_OK;
}

// Class moments, reduction, the copy to the host and the FP64 finish.
static int fit_from_index(cvamx_ctx* ctx, const cvamx_cube* cube, int32_t K, int32_t prec, double ridge, int32_t n_comp,
                   double* W, double* eigvals, double* mean, int64_t* counts, double* class_means, double* Sw,
                   double* Sb, const FitLayout& lay, char* res, int G, int L, hipStream_t s) {
  if (int st = fit_moments_launch(ctx, cube, K, prec, lay, res, G, L, s)) return st;
  HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
  return fit_host_finish(ctx, (int)cube->bands, K, ridge, n_comp, W, eigvals, mean, counts, class_means, Sw, Sb,
                         lay, L);
}

static int fit_layout_and_buffers(cvamx_ctx* ctx, int K, int B, int& G, int& L, char*& res) {
  L = cvx::tri_blocks(B) * 16;
  // blocks per class: three per CU over all classes (one round at three resident blocks)
  G = std::max(1, std::min(256, 3 * ctx->num_cu / K));
  const FitLayout lay(K, B, L);
  if (int st = ensure(ctx, B_PART, (size_t)K * G * L * 8)) return st;
  if (int st = ensure(ctx, B_RES, lay.total)) return st;
  if (int st = ensure_pinned(ctx, lay.total)) return st;
  res = static_cast<char*>(ctx->buf[B_RES]);
  return 0;
}

int cva_fit(cvamx_ctx* ctx, const cvamx_cube* cube, const int8_t* labels, int32_t K, int32_t prec,
            double ridge, int32_t n_comp, double* W, double* eigvals, double* mean, int64_t* counts,
            double* class_means, double* Sw, double* Sb, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (int st = check_fit_args(ctx, cube, K, prec, ridge, n_comp, W, eigvals, mean, counts)) return st;
  if (!labels) return fail(ctx, CVAMX_E_INVALID_ARG, "labels is NULL");
  if ((reinterpret_cast<uintptr_t>(labels) & 15u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "labels must be 16-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  int G, L;
  char* res;
  if (int st = fit_layout_and_buffers(ctx, K, B, G, L, res)) return st;
  const FitLayout lay(K, B, L);
  if (int st = build_index(ctx, labels, nullptr, P, P, K, lay, res, s)) return st;
  return fit_from_index(ctx, cube, K, prec, ridge, n_comp, W, eigvals, mean, counts, class_means, Sw, Sb, lay, res,
                        G, L, s);
}

int cva_fit_project(cvamx_ctx* ctx, const cvamx_cube* cube, const int8_t* labels, int32_t K, int32_t prec,
                    double ridge, int32_t n_comp, double* W, double* eigvals, double* mean, int64_t* counts,
                    uint8_t* images, float* range, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!images) return fail(ctx, CVAMX_E_INVALID_ARG, "images must be non-NULL");
  if (int st = cva_fit(ctx, cube, labels, K, prec, ridge, n_comp, W, eigvals, mean, counts, nullptr, nullptr,
                       nullptr, stream))
    return st;
  return project_common(ctx, cube, W, mean, n_comp, images, range, stream);
}

static int pca_launch(cvamx_ctx* ctx, const cvamx_cube* cube, const uint8_t* mask, int32_t prec, Buf bpart,
                      Buf bres, int slot, hipStream_t s);
static int pca_host_finish(cvamx_ctx* ctx, int B, int32_t n_comp, int slot, double* V, double* eigvals,
                           double* mean, double* cov);

// CVA and PCA of one page in one call, scheduled so that each FP64 host
// finish runs while the GPU works: the class moments, then the PCA Gram
// (into buffers of its own) are queued; the CVA finish runs as the Gram
// streams the page, and queues the CVA projection; the PCA finish runs as
// that projection streams the page, and queues the PCA projection.  The
// kernels and their order of arithmetic are those of the separate calls.
int cvamx_cva_pca(cvamx_ctx* ctx, const cvamx_cube* cube, const int8_t* labels, int32_t K, int32_t prec,
                  double ridge, int32_t n_cva, double* W, double* eigvals, double* mean, int64_t* counts,
                  uint8_t* cva_images, const uint8_t* mask, int32_t n_pca, double* V, double* pca_eigvals,
                  double* pca_mean, uint8_t* pca_images, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (int st = check_fit_args(ctx, cube, K, prec, ridge, n_cva, W, eigvals, mean, counts)) return st;
  if (!labels) return fail(ctx, CVAMX_E_INVALID_ARG, "labels is NULL");
  if ((reinterpret_cast<uintptr_t>(labels) & 15u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "labels must be 16-byte aligned");
  const int B = (int)cube->bands;
  if (n_pca < 1 || n_pca > B) return fail(ctx, CVAMX_E_INVALID_ARG, "n_pca must lie in 1..bands");
  if (!V || !pca_eigvals || !pca_mean)
    return fail(ctx, CVAMX_E_INVALID_ARG, "V, pca_eigvals and pca_mean must be non-NULL");
  if (!cva_images || !pca_images) return fail(ctx, CVAMX_E_INVALID_ARG, "the image outputs must be non-NULL");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t P = cube->height * cube->width;
  // the projection buffers of the larger group first: nothing is reallocated
  // while queued kernels may still use it
  const int64_t Pp = (P + 255) / 256 * 256;
  if (int st = ensure(ctx, B_H16, (size_t)std::min(std::max(n_cva, n_pca), 8) * (size_t)Pp * 2)) return st;
  if (int st = ensure(ctx, B_PROJPART, (size_t)proj_nblocks(ctx, cube) * 32 * sizeof(float))) return st;
  if (!ctx->ev_fit) HIP_TRY(hipEventCreateWithFlags(&ctx->ev_fit, hipEventDisableTiming), "event create");
  if (!ctx->ev_pca) HIP_TRY(hipEventCreateWithFlags(&ctx->ev_pca, hipEventDisableTiming), "event create");
  int G, L;
  char* res;
  if (int st = fit_layout_and_buffers(ctx, K, B, G, L, res)) return st;
  const FitLayout lay(K, B, L);
  // once work is queued, an error returns only after the stream has
  // drained, so that no queued kernel outlives the caller's buffers
  auto drained = [&](int st) {
    (void)hipStreamSynchronize(s);
    return st;
  };
  if (int st = build_index(ctx, labels, nullptr, P, P, K, lay, res, s)) return drained(st);
  if (int st = fit_moments_launch(ctx, cube, K, prec, lay, res, G, L, s)) return drained(st);
  if (hipError_t e = hipEventRecord(ctx->ev_fit, s)) return drained(hip_fail(ctx, e, "event record"));
  if (int st = pca_launch(ctx, cube, mask, prec, B_PPART, B_PRES, 1, s)) return drained(st);
  if (hipError_t e = hipEventRecord(ctx->ev_pca, s)) return drained(hip_fail(ctx, e, "event record"));
  if (hipError_t e = hipEventSynchronize(ctx->ev_fit)) return drained(hip_fail(ctx, e, "event synchronise"));
  if (int st = fit_host_finish(ctx, B, K, ridge, n_cva, W, eigvals, mean, counts, nullptr, nullptr, nullptr, lay, L))
    return drained(st);
  if (int st = project_common(ctx, cube, W, mean, n_cva, cva_images, nullptr, stream)) return drained(st);
  if (hipError_t e = hipEventSynchronize(ctx->ev_pca)) return drained(hip_fail(ctx, e, "event synchronise"));
  if (int st = pca_host_finish(ctx, B, n_pca, 1, V, pca_eigvals, pca_mean, nullptr)) return drained(st);
  if (int st = project_common(ctx, cube, V, pca_mean, n_pca, pca_images, nullptr, stream)) return drained(st);
  return CVAMX_OK;
}

int cva_fit_points(cvamx_ctx* ctx, const cvamx_cube* cube, const int64_t* pixels, const int8_t* classes,
                   int64_t N, int32_t K, int32_t prec, double ridge, int32_t n_comp, double* W, double* eigvals,
                   double* mean, int64_t* counts, double* class_means, double* Sw, double* Sb, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (int st = check_fit_args(ctx, cube, K, prec, ridge, n_comp, W, eigvals, mean, counts)) return st;
  if (!pixels || !classes) return fail(ctx, CVAMX_E_INVALID_ARG, "pixels and classes must be non-NULL");
  if (N < 1 || N >= (int64_t(1) << 31)) return fail(ctx, CVAMX_E_INVALID_ARG, "N must lie in 1..2^31-1");
  if ((reinterpret_cast<uintptr_t>(classes) & 15u) != 0 || (reinterpret_cast<uintptr_t>(pixels) & 7u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "classes must be 16-byte aligned and pixels 8-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  int G, L;
  char* res;
  if (int st = fit_layout_and_buffers(ctx, K, B, G, L, res)) return st;
  const FitLayout lay(K, B, L);
  if (int st = build_index(ctx, classes, pixels, N, P, K, lay, res, s)) return st;
  return fit_from_index(ctx, cube, K, prec, ridge, n_comp, W, eigvals, mean, counts, class_means, Sw, Sb, lay, res,
                        G, L, s);
}

int cvamx_label_index(cvamx_ctx* ctx, const int8_t* labels, int64_t n, int32_t K, int32_t* idx, int64_t* counts,
                      int32_t* offsets, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!labels || !idx || !counts || !offsets)
    return fail(ctx, CVAMX_E_INVALID_ARG, "labels, idx, counts and offsets must be non-NULL");
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(ctx, CVAMX_E_INVALID_ARG, "n must lie in 1..2^31-1");
  if (K < 1 || K > CVAMX_MAX_CLASSES) return fail(ctx, CVAMX_E_INVALID_ARG, "K must lie in 1..127");
  if ((reinterpret_cast<uintptr_t>(labels) & 15u) != 0 || (reinterpret_cast<uintptr_t>(idx) & 3u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "labels must be 16-byte aligned and idx 4-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const FitLayout lay(K, 1, 0);
  if (int st = ensure(ctx, B_RES, lay.total)) return st;
  if (int st = ensure_pinned(ctx, lay.total)) return st;
  char* res = static_cast<char*>(ctx->buf[B_RES]);
  if (int st = build_index(ctx, labels, nullptr, n, n, K, lay, res, s)) return st;
  HIP_TRY(to_pinned(ctx, res, lay.total, s), "result copy");
  HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
  const char* h = static_cast<const char*>(ctx->pinned);
  int32_t errflag;
  std::memcpy(&errflag, h + lay.err, 4);
  if (errflag & 1) return fail(ctx, CVAMX_E_INVALID_ARG, "a label lies outside -1..K-1");
  std::memcpy(counts, h + lay.counts, 8 * (size_t)K);
  std::memcpy(offsets, h + lay.offsets, 4 * (size_t)(K + 1));
  const int64_t total = offsets[K];
  if (total > 0) {
    HIP_TRY(hipMemcpyAsync(idx, ctx->buf[B_IDX], (size_t)total * 4, hipMemcpyDeviceToDevice, s), "index copy");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
  }
  return CVAMX_OK;
}

int cva_project(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center,
                int32_t n_comp, uint8_t* images, float* range, void* stream) {
  return project_common(ctx, cube, W, center, n_comp, images, range, stream);
}

int cva_project_noalloc(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center,
                        int32_t n_comp, uint8_t* images, float* range, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (int st = check_proj_args(ctx, cube, W, center, n_comp, images)) return st;
  if (int st = check_device(ctx)) return st;
  char* base = static_cast<char*>(cvx::scratch_address(ctx->device));
  if (!base) return fail(ctx, CVAMX_E_DEVICE, "the fixed scratch has no address on this device");
  const int nblocks = proj_nblocks(ctx, cube);
  if (nblocks > cvx::kScratchBlocks)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "the projection grid (" + std::to_string(nblocks) +
                                              " blocks) exceeds the fixed scratch's " +
                                              std::to_string(cvx::kScratchBlocks));
  hipStream_t s = (hipStream_t)stream;
  const ProjBufs pb{reinterpret_cast<float*>(base + cvx::kScratchPartOffset), reinterpret_cast<unsigned*>(base),
                    reinterpret_cast<float*>(base + 256), reinterpret_cast<float*>(base + 512)};
  // the ticket must start at zero: a fill kernel, not a memset, so that the
  // call can be captured into a graph
  HIP_TRY(cvx::launch_zero_u32(pb.ticket, 1, s), "ticket clear");
  if (int st = proj_groups_with(ctx, cube, W, center, n_comp, images, pb, false, s)) return st;
  if (range) {
    HIP_TRY(hipMemcpyAsync(range, pb.ab_dev, 2 * sizeof(float) * n_comp, hipMemcpyDeviceToHost, s), "range copy");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
  }
  return 0;
}

int pca_project(cvamx_ctx* ctx, const cvamx_cube* cube, const double* V, const double* mean,
                int32_t n_comp, uint8_t* images, float* range, void* stream) {
  return project_common(ctx, cube, V, mean, n_comp, images, range, stream);
}

int cvamx_project_float(cvamx_ctx* ctx, const cvamx_cube* cube, const double* W, const double* center,
                        int32_t n_comp, float* y, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (int st = check_proj_args(ctx, cube, W, center, n_comp, y)) return st;
  if ((reinterpret_cast<uintptr_t>(y) & 3u) != 0) return fail(ctx, CVAMX_E_UNSUPPORTED, "y must be 4-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  const int nblocks = proj_nblocks(ctx, cube);
  for (int g0 = 0; g0 < n_comp; g0 += 8) {
    const int nc = std::min(8, n_comp - g0);
    const bool pv = proj_vector(ctx, cube, nc);
    cvx::ProjArgs a;
    make_proj_args(cube, W, center, n_comp, g0, nc, pv, a);
    prof_begin(ctx, s, "project_float");
    hipError_t e = cvx::launch_project_float(cube->dtype, pv, cube->data, B, P, nc, a, nblocks,
                                             y + (int64_t)g0 * P, s);
    prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "project float launch");
  }
  return 0;
}

int cvamx_stretch(cvamx_ctx* ctx, const float* y, int64_t P, int32_t n_comp, int32_t mode, double pct,
                  const int64_t* train_pixels, int64_t n_train, int32_t bits, void* out, double* range,
                  void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!y || !out) return fail(ctx, CVAMX_E_INVALID_ARG, "y and out must be non-NULL");
  if (P < 1 || P >= (int64_t(1) << 31) - 1) return fail(ctx, CVAMX_E_INVALID_ARG, "P must lie in 1..2^31-2");
  if (n_comp < 1 || n_comp > CVAMX_MAX_BANDS)
    return fail(ctx, CVAMX_E_INVALID_ARG, "n_comp must lie in 1..CVAMX_MAX_BANDS");
  if (bits != 8 && bits != 16) return fail(ctx, CVAMX_E_INVALID_ARG, "bits must be 8 or 16");
  if (mode < CVAMX_STRETCH_MINMAX || mode > CVAMX_STRETCH_PERCENTILE)
    return fail(ctx, CVAMX_E_INVALID_ARG, "unknown stretch mode");
  if (mode == CVAMX_STRETCH_TRAINING && (!train_pixels || n_train < 1))
    return fail(ctx, CVAMX_E_INVALID_ARG, "mode 2 needs a non-empty list of training pixels");
  if (mode == CVAMX_STRETCH_PERCENTILE && !(std::isfinite(pct) && pct >= 0.0 && pct < 50.0))
    return fail(ctx, CVAMX_E_INVALID_ARG, "pct must lie in [0, 50)");
  if ((reinterpret_cast<uintptr_t>(y) & 3u) != 0 || (reinterpret_cast<uintptr_t>(out) & (bits / 8 - 1)) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "y and out must be aligned to their element size");
  if (mode == CVAMX_STRETCH_TRAINING && (reinterpret_cast<uintptr_t>(train_pixels) & 7u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "train_pixels must be 8-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  // fixed state: range (2 x 64 doubles), selection (64 x kSelTargets uint2), error flag
  const size_t ab_off = 0, sel_off = ab_off + 1024, err_off = sel_off + 8 * 64 * cvx::kSelTargets;
  if (int st = ensure(ctx, B_SFIX, err_off + 16)) return st;
  char* fix = static_cast<char*>(ctx->buf[B_SFIX]);
  double* ab = reinterpret_cast<double*>(fix + ab_off);
  uint2* sel = reinterpret_cast<uint2*>(fix + sel_off);
  int32_t* err = reinterpret_cast<int32_t*>(fix + err_off);
  hipError_t e;
  int nb = 1;
  double g_lo = 0.0, g_hi = 0.0;
  if (mode != CVAMX_STRETCH_PERCENTILE) {
    const int64_t m = mode == CVAMX_STRETCH_TRAINING ? n_train : P;
    nb = cvx::stretch_reduce_blocks(m, n_comp, ctx->num_cu);
    if (int st = ensure(ctx, B_SPART, (size_t)n_comp * nb * 2 * sizeof(float))) return st;
    if (mode == CVAMX_STRETCH_TRAINING) {
      e = cvx::launch_zero_u32(reinterpret_cast<uint32_t*>(err), 1, s);
      if (e != hipSuccess) return hip_fail(ctx, e, "flag clear launch");
    }
    prof_begin(ctx, s, "plane_minmax");
    e = cvx::launch_plane_minmax(y, P, n_comp, mode == CVAMX_STRETCH_TRAINING ? train_pixels : nullptr, n_train, nb,
                                 (float*)ctx->buf[B_SPART], err, s);
    prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "min/max launch");
    if (mode == CVAMX_STRETCH_TRAINING) {
      if (int st = ensure_pinned(ctx, 16)) return st;
      HIP_TRY(to_pinned(ctx, err, 4, s), "flag copy");
      HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
      int32_t flag = 0;
      std::memcpy(&flag, ctx->pinned, 4);
      if (flag & 2) return fail(ctx, CVAMX_E_INVALID_ARG, "a training pixel lies outside 0..P-1");
    }
  } else {
    // linear interpolation between the order statistics around the virtual
    // index h = (P - 1) q, evaluated as NumPy does for its linear method
    auto vindex = [&](double q, uint32_t& r0, uint32_t& r1, double& g) {
      const double h = (double)P * q + (1.0 - q) - 1.0;
      double f = std::floor(h);
      if (h >= (double)(P - 1)) {
        r0 = r1 = (uint32_t)(P - 1);
        g = 0.0;
        return;
      }
      if (h < 0.0) f = 0.0;
      r0 = (uint32_t)f;
      r1 = (uint32_t)std::min<int64_t>((int64_t)f + 1, P - 1);
      g = h < 0.0 ? 0.0 : h - f;
    };
    uint32_t ranks[cvx::kSelTargets];
    vindex(pct / 100.0, ranks[0], ranks[1], g_lo);
    vindex((100.0 - pct) / 100.0, ranks[2], ranks[3], g_hi);
    nb = cvx::stretch_reduce_blocks(P, n_comp, ctx->num_cu);
    if (int st = ensure(ctx, B_SHIST, (size_t)2 * n_comp * cvx::kSelTargets * cvx::kSelBins * 4)) return st;
    prof_begin(ctx, s, "select");
    e = cvx::launch_select(y, P, n_comp, ranks, nb, sel, (uint32_t*)ctx->buf[B_SHIST], s);
    prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "select launch");
  }
  e = cvx::launch_stretch_finish(mode, n_comp, nb, (const float*)ctx->buf[B_SPART], sel, g_lo, g_hi, ab, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "stretch range launch");
  prof_begin(ctx, s, "stretch_planes");
  e = cvx::launch_stretch_planes(y, P, n_comp, ab, bits, out, ctx->num_cu, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "stretch launch");
  if (range) {
    if (int st = ensure_pinned(ctx, 2 * sizeof(double) * n_comp)) return st;
    HIP_TRY(to_pinned(ctx, ab, 2 * sizeof(double) * n_comp, s), "range copy");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
    std::memcpy(range, ctx->pinned, 2 * sizeof(double) * n_comp);
  }
  return 0;
}

int cvamx_compose_rgb(cvamx_ctx* ctx, const uint8_t* r, const uint8_t* g, const uint8_t* b, int64_t P,
                      uint8_t* rgb, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!rgb) return fail(ctx, CVAMX_E_INVALID_ARG, "rgb must be non-NULL");
  if (P < 1) return fail(ctx, CVAMX_E_INVALID_ARG, "P must be positive");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  prof_begin(ctx, s, "compose_rgb");
  hipError_t e = cvx::launch_compose_rgb(r, g, b, P, rgb, ctx->num_cu, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "compose launch");
  return 0;
}

int cvamx_bands_to_cube(cvamx_ctx* ctx, const void* bands, int32_t in_dtype, int32_t B, int64_t P, void* cube,
                        void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!bands || !cube) return fail(ctx, CVAMX_E_INVALID_ARG, "bands and cube must be non-NULL");
  if (in_dtype != CVAMX_U8 && in_dtype != CVAMX_U16 && in_dtype != CVAMX_F32)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "band images must be uint8, uint16 or float32");
  if (B < 1 || B > CVAMX_MAX_BANDS) return fail(ctx, CVAMX_E_INVALID_ARG, "B must lie in 1..CVAMX_MAX_BANDS");
  if (P < 1 || P >= (int64_t(1) << 31) - 1) return fail(ctx, CVAMX_E_INVALID_ARG, "P must lie in 1..2^31-2");
  const size_t ein = in_dtype == CVAMX_U8 ? 1 : (in_dtype == CVAMX_U16 ? 2 : 4);
  if ((reinterpret_cast<uintptr_t>(bands) & (ein - 1)) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "bands must be aligned to their element size");
  if ((reinterpret_cast<uintptr_t>(cube) & 15u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "cube must be 16-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  prof_begin(ctx, s, "bands_to_cube");
  hipError_t e = cvx::launch_bands_to_cube(in_dtype, bands, B, P, cube, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "bands launch");
  return 0;
}

int cvamx_cluster_indices(cvamx_ctx* ctx, const void* images, int32_t dtype, int64_t P, int32_t n_feat,
                          const int64_t* pixels, const int8_t* classes, int64_t N, int32_t K, double p,
                          double* centroids, double* scatter, double* dist, double* dbi, double* dunn,
                          double* scores, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!images || !pixels || !classes || !scores)
    return fail(ctx, CVAMX_E_INVALID_ARG, "images, pixels, classes and scores must be non-NULL");
  if (dtype < CVAMX_U16 || dtype > CVAMX_U8) return fail(ctx, CVAMX_E_UNSUPPORTED, "unknown dtype");
  if (P < 1 || P >= (int64_t(1) << 31) - 1) return fail(ctx, CVAMX_E_INVALID_ARG, "P must lie in 1..2^31-2");
  if (n_feat < 1 || n_feat > CVAMX_MAX_BANDS)
    return fail(ctx, CVAMX_E_INVALID_ARG, "n_feat must lie in 1..CVAMX_MAX_BANDS");
  if (N < 1 || N >= (int64_t(1) << 31)) return fail(ctx, CVAMX_E_INVALID_ARG, "N must lie in 1..2^31-1");
  if (K < 2 || K > CVAMX_MAX_CLASSES) return fail(ctx, CVAMX_E_INVALID_ARG, "K must lie in 2..127");
  if (!(std::isfinite(p) && p >= 1.0)) return fail(ctx, CVAMX_E_INVALID_ARG, "p must be finite and >= 1");
  const size_t el = dtype == CVAMX_U8 ? 1 : esize(dtype);
  if ((reinterpret_cast<uintptr_t>(images) & (el - 1)) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "images must be aligned to their element size");
  if ((reinterpret_cast<uintptr_t>(pixels) & 7u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "pixels must be 8-byte aligned");
  if ((reinterpret_cast<uintptr_t>(classes) & 15u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "classes must be 16-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int L = cvx::cluster_sum_len(n_feat);
  const int G = std::max(1, std::min(64, 2 * ctx->num_cu / K));
  // results: counts, offsets, error flag (FitLayout with one "band" for the
  // distance sums in the shift slot and the feature sums in the Gram slot)
  const FitLayout lay(K, 1, L);
  if (int st = ensure(ctx, B_PART, (size_t)K * G * (L + 1) * 8)) return st;
  if (int st = ensure(ctx, B_RES, lay.total)) return st;
  if (int st = ensure_pinned(ctx, lay.total)) return st;
  char* res = static_cast<char*>(ctx->buf[B_RES]);
  if (int st = build_index(ctx, classes, pixels, N, P, K, lay, res, s)) return st;
  prof_begin(ctx, s, "cluster_moments");
  hipError_t e = cvx::launch_cluster_moments(dtype, images, P, n_feat, (const int32_t*)ctx->buf[B_IDX],
                                             (const int32_t*)(res + lay.offsets), (const int64_t*)(res + lay.counts),
                                             K, G, p, (double*)ctx->buf[B_PART], (double*)(res + lay.gram),
                                             (double*)(res + lay.shift), s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "cluster moments launch");
  HIP_TRY(to_pinned(ctx, res, lay.total, s), "result copy");
  HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
  const char* h = static_cast<const char*>(ctx->pinned);
  int32_t errflag;
  std::memcpy(&errflag, h + lay.err, 4);
  if (errflag & 1) return fail(ctx, CVAMX_E_INVALID_ARG, "a class lies outside -1..K-1");
  if (errflag & 2) return fail(ctx, CVAMX_E_INVALID_ARG, "a point lies outside the page");
  std::vector<int64_t> cnt(K);
  std::memcpy(cnt.data(), h + lay.counts, 8 * (size_t)K);
  for (int k = 0; k < K; ++k)
    if (cnt[k] < 1) return fail(ctx, CVAMX_E_EMPTY_CLASS, "class " + std::to_string(k) + " has no point");
  const double* sums = reinterpret_cast<const double*>(h + lay.gram);
  const double* dsum = reinterpret_cast<const double*>(h + lay.shift);
  const int n = n_feat;
  std::vector<double> A((size_t)K * n), S(K), M((size_t)K * K, 0.0), R((size_t)K * K, 0.0), D((size_t)K * K, 0.0);
  for (int k = 0; k < K; ++k) {
    for (int f = 0; f < n; ++f) A[(size_t)k * n + f] = sums[(size_t)k * L + f] / (double)cnt[k];
    S[k] = dsum[k] / (double)cnt[k];
  }
  auto norm = [&](const double* a, const double* b) {
    double t = 0.0;
    for (int f = 0; f < n; ++f) {
      const double d = std::fabs(a[f] - b[f]);
      t += p == 2.0 ? d * d : (p == 1.0 ? d : std::pow(d, p));
    }
    return p == 2.0 ? std::sqrt(t) : (p == 1.0 ? t : std::pow(t, 1.0 / p));
  };
  double smax = 0.0, dmin = INFINITY, dbi_sum = 0.0;
  for (int k = 0; k < K; ++k) smax = std::max(smax, S[k]);
  for (int i = 0; i < K; ++i) {
    double rmax = -INFINITY;
    for (int j = 0; j < K; ++j) {
      if (i == j) continue;
      const double m = norm(&A[(size_t)i * n], &A[(size_t)j * n]);
      M[(size_t)i * K + j] = m;
      R[(size_t)i * K + j] = (S[i] + S[j]) / m;
      D[(size_t)i * K + j] = (m - S[i] - S[j]) / std::max(S[i], S[j]);
      rmax = std::max(rmax, R[(size_t)i * K + j]);
      dmin = std::min(dmin, m - S[i] - S[j]);
    }
    dbi_sum += rmax;
  }
  scores[0] = dbi_sum / K;
  scores[1] = dmin / smax;
  if (centroids) std::copy(A.begin(), A.end(), centroids);
  if (scatter) std::copy(S.begin(), S.end(), scatter);
  if (dist) std::copy(M.begin(), M.end(), dist);
  if (dbi) std::copy(R.begin(), R.end(), dbi);
  if (dunn) std::copy(D.begin(), D.end(), dunn);
  return CVAMX_OK;
}

// The PCA Gram and its reduction into page-locked staging slot `slot`
// (the shift, then the packed Gram), in device buffers bpart and bres.
static int pca_launch(cvamx_ctx* ctx, const cvamx_cube* cube, const uint8_t* mask, int32_t prec, Buf bpart,
                      Buf bres, int slot, hipStream_t s) {
  const int B = (int)cube->bands;
  const int64_t P = cube->height * cube->width;
  const int L = cvx::tri_blocks(B) * 16;
  const bool vector_path = prec == CVAMX_PREC_FP32 && (ctx->plain || !split_is_exact(cube->dtype));
  // uint16 pages on the matrix cores: one resident round of blocks (a
  // partial second round cost 4 % at 33 bands); else four blocks per CU
  const int per_cu = (!vector_path && cube->dtype == CVAMX_U16) ? cvx::pca_u16_blocks_per_cu(B) : 4;
  int nblocks = ctx->gram_blocks > 0 ? ctx->gram_blocks : ctx->num_cu * per_cu;
  nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(nblocks, (P + cvx::kChunk - 1) / cvx::kChunk));
  // the exact integer Gram of uint16 pages needs every block to cover fewer
  // than 2^22 pixels (its LDS sums stay integers below 2^53): a smaller grid,
  // asked for through CVAMX_GRAM_BLOCKS, is raised to keep at most 2^21
  if (!vector_path && cube->dtype == CVAMX_U16)
    nblocks = (int)std::max<int64_t>(nblocks, (P + (int64_t(1) << 21) - 1) >> 21);
  const size_t res_bytes = 8 * (size_t)B + 8 * (size_t)L;
  if (int st = ensure(ctx, bpart, (size_t)nblocks * L * 8)) return st;
  if (int st = ensure(ctx, bres, res_bytes)) return st;
  if (int st = ensure_pinned(ctx, res_bytes, slot)) return st;
  char* res = static_cast<char*>(ctx->buf[bres]);
  void* pin = slot == 0 ? ctx->pinned : ctx->pinned2;
  hipError_t e;
  if (vector_path) {
    prof_begin(ctx, s, "pca_gram");
    e = cvx::launch_pca_gram(cube->dtype, cube->data, B, P, mask, nblocks, (double*)ctx->buf[bpart],
                             (double*)res, s);
  } else {
    prof_begin(ctx, s, "pca_gram_mfma");
    e = cvx::launch_pca_gram_mfma(cube->dtype, prec == CVAMX_PREC_F16X3 ? 1 : 0, cube->data, B, P, mask,
                                  nblocks, (double*)ctx->buf[bpart], (double*)res, s);
  }
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "pca gram launch");
  prof_begin(ctx, s, "reduce_partials");
  e = cvx::launch_reduce_part_out((const double*)ctx->buf[bpart], 1, nblocks, L,
                                  (double*)(static_cast<char*>(pin) + 8 * B), res, pin,
                                  (int64_t)8 * B, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
  return 0;
}

// The covariance and its leading axes from staging slot `slot`.
static int pca_host_finish(cvamx_ctx* ctx, int B, int32_t n_comp, int slot, double* V, double* eigvals,
                           double* mean, double* cov) {
  const double* shift = static_cast<const double*>(slot == 0 ? ctx->pinned : ctx->pinned2);
  std::vector<double> G1;
  unpack_gram(B, shift + B, G1);
  const int n1 = B + 1;
  const double n = G1[(size_t)B * n1 + B];
  if (!(n >= 2.0)) return fail(ctx, CVAMX_E_INVALID_ARG, "PCA needs at least two selected pixels");
  std::vector<double> C((size_t)B * B), w(B), Vf((size_t)B * B), mu(B);
  for (int i = 0; i < B; ++i) mu[i] = shift[i] + G1[(size_t)i * n1 + B] / n;
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < B; ++j)
      C[(size_t)i * B + j] = (G1[(size_t)i * n1 + j] - G1[(size_t)i * n1 + B] * G1[(size_t)j * n1 + B] / n) / (n - 1.0);
  // standardised: the eigenproblem of R = D^-1/2 C D^-1/2 (D = diag C), and
  // the projection vectors D^-1/2 u
  std::vector<double> sd(B, 1.0), A = C;
  if (ctx->pca_standardize) {
    for (int i = 0; i < B; ++i) {
      sd[i] = std::sqrt(C[(size_t)i * B + i]);
      if (!(sd[i] > 0.0)) return fail(ctx, CVAMX_E_INVALID_ARG, "band " + std::to_string(i) + " has zero variance");
    }
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < B; ++j) A[(size_t)i * B + j] = C[(size_t)i * B + j] / (sd[i] * sd[j]);
  }
  // the leading n_comp axes only (inverse iteration on the tridiagonal form)
  const int st = cvamx::sym_eig_top(B, A.data(), n_comp, w.data(), Vf.data());
  if (st != 0) return fail(ctx, st, "PCA eigensolver did not converge");
  std::vector<double> Vo((size_t)B * n_comp);
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < n_comp; ++j) Vo[(size_t)i * n_comp + j] = Vf[(size_t)i * n_comp + j] / sd[i];
  cvamx::sign_rule(B, n_comp, Vo.data());
  std::copy(Vo.begin(), Vo.end(), V);
  std::copy(w.begin(), w.begin() + n_comp, eigvals);
  std::copy(mu.begin(), mu.end(), mean);
  if (cov) std::copy(C.begin(), C.end(), cov);
  return CVAMX_OK;
}

int pca_fit(cvamx_ctx* ctx, const cvamx_cube* cube, const uint8_t* mask, int32_t n_comp, int32_t prec,
            double* V, double* eigvals, double* mean, double* cov, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (int st = check_cube(ctx, cube)) return st;
  const int B = (int)cube->bands;
  if (n_comp < 1 || n_comp > B) return fail(ctx, CVAMX_E_INVALID_ARG, "n_comp must lie in 1..bands");
  if (prec < CVAMX_PREC_FP32 || prec > CVAMX_PREC_F16X3)
    return fail(ctx, CVAMX_E_INVALID_ARG, "unknown precision");
  if (!V || !eigvals || !mean) return fail(ctx, CVAMX_E_INVALID_ARG, "V, eigvals and mean must be non-NULL");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  if (int st = pca_launch(ctx, cube, mask, prec, B_PART, B_RES, 0, s)) return st;
  HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
  return pca_host_finish(ctx, B, n_comp, 0, V, eigvals, mean, cov);
}

int cva_soft_forward(cvamx_ctx* ctx, const float* X, const float* w, int64_t N, int32_t B, int32_t K,
                     int32_t prec, double ridge, double* J, double* W, double* eigvals, double* mean,
                     double* class_means, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!X || !w) return fail(ctx, CVAMX_E_INVALID_ARG, "X and w must be non-NULL");
  if (N < 2 || N >= (int64_t(1) << 31)) return fail(ctx, CVAMX_E_INVALID_ARG, "N must lie in 2..2^31-1");
  if (B < 1 || B > CVAMX_MAX_BANDS) return fail(ctx, CVAMX_E_INVALID_ARG, "B must lie in 1..64");
  if (K < 2 || K > 32) return fail(ctx, CVAMX_E_INVALID_ARG, "soft-label CVA supports K in 2..32");
  if (prec < CVAMX_PREC_FP32 || prec > CVAMX_PREC_F16X3)
    return fail(ctx, CVAMX_E_INVALID_ARG, "unknown precision");
  if (!finite_nonneg(ridge)) return fail(ctx, CVAMX_E_INVALID_ARG, "ridge must be finite and >= 0");
  if (!J || !W || !eigvals || !mean || !class_means)
    return fail(ctx, CVAMX_E_INVALID_ARG, "J, W, eigvals, mean and class_means must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(X) & 15u) != 0 || (reinterpret_cast<uintptr_t>(w) & 15u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "X and w must be 16-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int BP = cvx::padded_bp(B), KP = (K + 3) & ~3;
  const int L = cvx::tri_blocks(B) * 16;
  const int64_t nch = (N + cvx::kChunk - 1) / cvx::kChunk;
  // pass 1 finds the shift the scatter centres each class on: the class
  // means of a strided sample of about kSoftSampleChunks chunks (all of
  // them when there are fewer).  Any shift is exact, since the scatter also
  // sums w (x - s) and w and the host removes the shift in FP64; one near
  // the class mean keeps the FP32 sums as small as the centred ones.
  constexpr int64_t kSoftSampleChunks = 512;
  const int64_t every = std::max<int64_t>(1, nch / kSoftSampleChunks);
  const int64_t nsample = (nch + every - 1) / every;
  const int nb1 = (int)std::max<int64_t>(1, std::min<int64_t>(3 * ctx->num_cu, nsample));
  // the scatter's path: FP32 products on the FP32 matrix instruction (the
  // default), the plain FP32 vector-ALU reference (cvamx_set_plain_fp32),
  // or the compensated bf16 / fp16 split on the 16-bit matrix units
  const bool plain = prec == CVAMX_PREC_FP32 && ctx->plain;
  const bool split = prec != CVAMX_PREC_FP32;
  // pass 2: about one resident round of blocks over all class groups
  int G;
  if (plain) {
    G = (int)std::max<int64_t>(1, std::min<int64_t>(3 * ctx->num_cu / K, nch));
  } else if (split) {
    const int groups = (K + cvx::kWaves - 1) / cvx::kWaves;
    G = (int)std::max<int64_t>(1, std::min<int64_t>(2 * ctx->num_cu / groups, nch));
  } else {
    const int cpb = cvx::soft_scatter_classes_per_block(B, K);
    const int groups = (K + cpb - 1) / cpb;
    G = (int)std::max<int64_t>(1, std::min<int64_t>(cvx::soft_scatter_blocks_per_cu(B, K) * ctx->num_cu / groups, nch));
  }
  const size_t first_bytes = 8 * (size_t)K * (B + 1);
  const size_t mcf_off = first_bytes;
  const size_t gram_off = (mcf_off + 4 * (size_t)K * B + 7) & ~size_t(7);
  const size_t res_bytes = gram_off + 8 * (size_t)K * L;
  // pass-1 scratch: block partials, then their reduction
  const size_t fp_off = (size_t)nb1 * KP * BP * 8;
  if (int st = ensure(ctx, B_FIRST, fp_off + (size_t)KP * BP * 8)) return st;
  if (int st = ensure(ctx, B_PART, (size_t)K * G * L * 8)) return st;
  if (int st = ensure(ctx, B_RES, res_bytes)) return st;
  if (int st = ensure_pinned(ctx, res_bytes)) return st;
  char* res = static_cast<char*>(ctx->buf[B_RES]);
  char* f1 = static_cast<char*>(ctx->buf[B_FIRST]);
  prof_begin(ctx, s, plain ? "soft_first_plain" : "soft_first");
  hipError_t e = plain ? cvx::launch_soft_first_plain(X, w, N, B, K, every, nb1, (double*)f1, s)
                       : cvx::launch_soft_first(X, w, N, B, K, every, nb1, (double*)f1, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "soft first launch");
  e = cvx::launch_reduce_part((const double*)f1, 1, nb1, KP * BP, (double*)(f1 + fp_off), s);
  if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
  e = cvx::launch_soft_means(B, K, (const double*)(f1 + fp_off), (double*)res, (float*)(res + mcf_off), s);
  if (e != hipSuccess) return hip_fail(ctx, e, "class means launch");
  const float* mcf_d = (const float*)(res + mcf_off);
  double* part = (double*)ctx->buf[B_PART];
  if (plain) {
    prof_begin(ctx, s, "soft_scatter_plain");
    e = cvx::launch_soft_scatter_plain(X, w, N, B, K, G, mcf_d, part, s);
  } else if (split) {
    prof_begin(ctx, s, "soft_scatter_split");
    e = cvx::launch_soft_scatter_split(prec == CVAMX_PREC_F16X3 ? 1 : 0, X, w, N, B, K, G, mcf_d, part, s);
  } else {
    prof_begin(ctx, s, "soft_scatter");
    e = cvx::launch_soft_scatter(X, w, N, B, K, G, mcf_d, part, s);
  }
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "soft scatter launch");
  prof_begin(ctx, s, "reduce_partials");
  e = cvx::launch_reduce_part((const double*)ctx->buf[B_PART], K, G, L, (double*)(res + gram_off), s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
  HIP_TRY(to_pinned(ctx, res, res_bytes, s), "result copy");
  HIP_TRY(hipStreamSynchronize(s), "stream synchronise");
  const char* h = static_cast<const char*>(ctx->pinned);
  const float* mcf = reinterpret_cast<const float*>(h + mcf_off);
  const double* gram = reinterpret_cast<const double*>(h + gram_off);
  std::vector<double> cm((size_t)K * B), Swv((size_t)B * B, 0.0), G1, n(K);
  const int n1 = B + 1;
  for (int c = 0; c < K; ++c) {
    unpack_gram(B, gram + (size_t)c * L, G1);
    const double nc = G1[(size_t)B * n1 + B];
    if (!(nc > 0.0)) return fail(ctx, CVAMX_E_EMPTY_CLASS, "class " + std::to_string(c) + " has no positive weight");
    n[c] = nc;
    for (int i = 0; i < B; ++i) cm[(size_t)c * B + i] = (double)mcf[(size_t)c * B + i] + G1[(size_t)i * n1 + B] / nc;
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < B; ++j)
        Swv[(size_t)i * B + j] += G1[(size_t)i * n1 + j] - G1[(size_t)i * n1 + B] * G1[(size_t)j * n1 + B] / nc;
  }
  const int C = std::min(K - 1, B);
  std::vector<double> Wt((size_t)B * C), lam(C), m(B);
  const int st = cvamx::cva_solve(K, B, n.data(), cm.data(), Swv.data(), ridge, C, Wt.data(), lam.data(),
                                  m.data(), nullptr, &ctx->err);
  if (st != 0) return st;
  double Jv = 0.0;
  for (int j = 0; j < C; ++j) Jv += lam[j];
  *J = Jv;
  std::copy(Wt.begin(), Wt.end(), W);
  std::copy(lam.begin(), lam.end(), eigvals);
  std::copy(m.begin(), m.end(), mean);
  std::copy(cm.begin(), cm.end(), class_means);
  return CVAMX_OK;
}

int cva_soft_backward(cvamx_ctx* ctx, const float* X, const double* W, const double* eigvals,
                      const double* mean, const double* class_means, int64_t N, int32_t B, int32_t K,
                      double dJ, float* dw, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!X || !W || !eigvals || !mean || !class_means || !dw)
    return fail(ctx, CVAMX_E_INVALID_ARG, "pointer arguments must be non-NULL");
  if (N < 1 || N >= (int64_t(1) << 31)) return fail(ctx, CVAMX_E_INVALID_ARG, "N must lie in 1..2^31-1");
  if (B < 1 || B > CVAMX_MAX_BANDS) return fail(ctx, CVAMX_E_INVALID_ARG, "B must lie in 1..64");
  if (K < 2 || K > 32) return fail(ctx, CVAMX_E_INVALID_ARG, "soft-label CVA supports K in 2..32");
  if (!std::isfinite(dJ)) return fail(ctx, CVAMX_E_INVALID_ARG, "dJ must be finite");
  if ((reinterpret_cast<uintptr_t>(X) & 15u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "X must be 16-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int C = std::min(K - 1, B);
  const int64_t nt = (N + 63) / 64;
  const int nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(ctx->num_cu * 8, (nt + 3) / 4));
  for (int g0 = 0; g0 < C; g0 += 8) {
    const int nc = std::min(8, C - g0);
    cvx::SoftBwdArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int b = 0; b < B; ++b) a.m[b] = (float)mean[b];
    for (int j = 0; j < nc; ++j) {
      for (int b = 0; b < B; ++b) a.w[b * 8 + j] = (float)W[(size_t)b * C + g0 + j];
      a.lam1[j] = (float)(1.0 + eigvals[g0 + j]);
      for (int c = 0; c < K; ++c) {
        double d = 0.0;
        for (int b = 0; b < B; ++b) d += W[(size_t)b * C + g0 + j] * (class_means[(size_t)c * B + b] - mean[b]);
        a.d[c * 8 + j] = (float)d;
      }
    }
    a.scale = (float)dJ;
    prof_begin(ctx, s, "soft_backward");
    hipError_t e = cvx::launch_soft_backward(X, N, B, K, a, g0 > 0, nblocks, dw, s);
    prof_end(ctx, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "soft backward launch");
  }
  return CVAMX_OK;
}

int cva_soft_update(cvamx_ctx* ctx, const float* grad, float* w, int64_t N, int32_t K, double step, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!grad || !w) return fail(ctx, CVAMX_E_INVALID_ARG, "grad and w must be non-NULL");
  if (N < 1 || N >= (int64_t(1) << 31)) return fail(ctx, CVAMX_E_INVALID_ARG, "N must lie in 1..2^31-1");
  if (K < 2 || K > 32) return fail(ctx, CVAMX_E_INVALID_ARG, "soft-label CVA supports K in 2..32");
  if (!finite_nonneg(step)) return fail(ctx, CVAMX_E_INVALID_ARG, "step must be finite and >= 0");
  if ((reinterpret_cast<uintptr_t>(grad) & 3u) != 0 || (reinterpret_cast<uintptr_t>(w) & 3u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "grad and w must be 4-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  prof_begin(ctx, s, "soft_update");
  hipError_t e = cvx::launch_soft_update(grad, w, N, K, (float)step, ctx->num_cu, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "soft update launch");
  return CVAMX_OK;
}

int cvamx_set_plain_fp32(cvamx_ctx* ctx, int enable) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  ctx->plain = enable != 0;
  return CVAMX_OK;
}

int cvamx_stream_read(cvamx_ctx* ctx, const void* src, int64_t bytes, uint32_t* sink, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!src || !sink) return fail(ctx, CVAMX_E_INVALID_ARG, "src and sink must be non-NULL");
  if (bytes < 16 || bytes % 16 != 0) return fail(ctx, CVAMX_E_INVALID_ARG, "bytes must be a positive multiple of 16");
  if ((reinterpret_cast<uintptr_t>(src) & 15u) != 0 || (reinterpret_cast<uintptr_t>(sink) & 3u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "src must be 16-byte aligned and sink 4-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  prof_begin(ctx, s, "stream_read");
  hipError_t e = cvx::launch_stream_read(src, bytes, 0x9e3779b9u, sink, ctx->num_cu, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "stream read launch");
  return CVAMX_OK;
}

int cvamx_stream_mix(cvamx_ctx* ctx, const void* src, int64_t read_bytes, void* dst, int64_t write_bytes,
                     uint32_t* sink, void* stream) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!src || !dst || !sink) return fail(ctx, CVAMX_E_INVALID_ARG, "src, dst and sink must be non-NULL");
  if (read_bytes < 16 || read_bytes % 16 != 0 || write_bytes < 16 || write_bytes % 16 != 0)
    return fail(ctx, CVAMX_E_INVALID_ARG, "read_bytes and write_bytes must be positive multiples of 16");
  if (write_bytes > read_bytes) return fail(ctx, CVAMX_E_INVALID_ARG, "write_bytes must not exceed read_bytes");
  if ((reinterpret_cast<uintptr_t>(src) & 15u) != 0 || (reinterpret_cast<uintptr_t>(dst) & 15u) != 0 ||
      (reinterpret_cast<uintptr_t>(sink) & 3u) != 0)
    return fail(ctx, CVAMX_E_UNSUPPORTED, "src and dst must be 16-byte aligned and sink 4-byte aligned");
  if (int st = check_device(ctx)) return st;
  hipStream_t s = (hipStream_t)stream;
  prof_begin(ctx, s, "stream_mix");
  hipError_t e = cvx::launch_stream_mix(src, read_bytes, dst, write_bytes, 0x9e3779b9u, sink, ctx->num_cu, s);
  prof_end(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "stream mix launch");
  return CVAMX_OK;
}

int cvamx_set_pca_standardize(cvamx_ctx* ctx, int enable) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  ctx->pca_standardize = enable != 0;
  return CVAMX_OK;
}

int cvamx_set_schedule(cvamx_ctx* ctx, int schedule) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (schedule != CVAMX_SCHEDULE_AUTO && schedule != CVAMX_SCHEDULE_TWO_READS &&
      schedule != CVAMX_SCHEDULE_FORCE_REREAD)
    return fail(ctx, CVAMX_E_INVALID_ARG, "unknown projection schedule");
  ctx->schedule = schedule;
  return CVAMX_OK;
}

int cvamx_profile_enable(cvamx_ctx* ctx, int enable) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (ctx->device < 0) return fail(ctx, CVAMX_E_DEVICE, "context has no device");
  prof_collect(ctx);
  ctx->prof_acc.clear();
  ctx->prof = (enable == 1 || enable == 2) ? enable : 0;
  return CVAMX_OK;
}

int64_t cvamx_profile_report(cvamx_ctx* ctx, char* buf, int64_t len) {
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (ctx->device >= 0) {
    (void)hipSetDevice(ctx->device);
    prof_collect(ctx);
  }
  std::string out;
  char line[160];
  for (const auto& kv : ctx->prof_acc) {
    std::snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  const int64_t need = (int64_t)out.size() + 1;
  if (buf && len > 0) {
    const int64_t n = std::min<int64_t>(len - 1, (int64_t)out.size());
    std::memcpy(buf, out.data(), (size_t)n);
    buf[n] = 0;
  }
  return need;
}

}  // extern "C"

// Many pages through one context: the CVA enhancement of each page from its
// band images and training points, with the transfers of neighbouring pages
// overlapped with the work on the current one (paper Section 4: a whole
// palimpsest of about 240 pages was processed, and pages were re-run with
// other training points).
//
// Three streams: the caller's (every kernel, in page order), one for
// host-to-device and one for device-to-host copies.  Page t's band images
// and points travel into one of two staging slots while page t - 1 is
// computed; page t's images travel back from one of two output slots while
// page t + 1 is computed; the host's FP64 eigensolve of page t runs while
// the copy engines move its neighbours.  Events order the slots:
//   in[s]    the page in slot s has landed            (h2d -> compute)
//   done[s]  the page in slot s no longer needs it    (compute -> h2d)
//   img[s]   the images in output slot s are complete (compute -> d2h)
//   out[s]   the images in output slot s have left    (d2h -> compute)
// The device work per page is the library's own entry points
// (cvamx_bands_to_cube, cva_fit_points, cvamx_project_float, cvamx_stretch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "ctx_internal.hpp"
#include "cvamx.h"

namespace {

struct Slots {
  hipStream_t cs = nullptr, h2d = nullptr, d2h = nullptr;   // cs: the caller's stream (not owned)
  hipEvent_t in[2] = {}, done[2] = {}, img[2] = {}, out[2] = {};
  void* bands[2] = {};
  int64_t* pix[2] = {};
  int8_t* cls[2] = {};
  int64_t* train[2] = {};
  void* images[2] = {};
  void* cube = nullptr;
  float* y = nullptr;

  ~Slots() {
    // nothing may still use the slots when they are freed
    (void)hipStreamSynchronize(cs);
    if (h2d) (void)hipStreamSynchronize(h2d);
    if (d2h) (void)hipStreamSynchronize(d2h);
    for (int s = 0; s < 2; ++s) {
      for (hipEvent_t e : {in[s], done[s], img[s], out[s]})
        if (e) (void)hipEventDestroy(e);
      for (void* p : {bands[s], (void*)pix[s], (void*)cls[s], (void*)train[s], images[s]})
        if (p) (void)hipFree(p);
    }
    if (cube) (void)hipFree(cube);
    if (y) (void)hipFree(y);
    if (h2d) (void)hipStreamDestroy(h2d);
    if (d2h) (void)hipStreamDestroy(d2h);
  }
};

bool alloc(void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 256)) == hipSuccess; }

}  // namespace

extern "C" int cvamx_run_pages(cvamx_ctx* ctx, int32_t in_dtype, int32_t B, int64_t H, int64_t Wd, int32_t K,
                               int32_t n_comp, int32_t prec, double ridge, int32_t mode, double pct, int32_t bits,
                               cvamx_page* pages, int32_t n_pages, void* stream) {
  using cvamx::set_error;
  if (!ctx) return CVAMX_E_INVALID_ARG;
  if (!pages || n_pages < 1) return set_error(ctx, CVAMX_E_INVALID_ARG, "pages must be non-NULL and n_pages >= 1");
  if (in_dtype != CVAMX_U8 && in_dtype != CVAMX_U16 && in_dtype != CVAMX_F32)
    return set_error(ctx, CVAMX_E_UNSUPPORTED, "band images must be uint8, uint16 or float32");
  if (B < 1 || B > CVAMX_MAX_BANDS) return set_error(ctx, CVAMX_E_INVALID_ARG, "bands must lie in 1..64");
  if (H < 1 || Wd < 1 || H * Wd >= (int64_t(1) << 31) - 1)
    return set_error(ctx, CVAMX_E_INVALID_ARG, "page dimensions must be positive, below 2^31 - 1 pixels");
  if (K < 2 || K > CVAMX_MAX_CLASSES) return set_error(ctx, CVAMX_E_INVALID_ARG, "K must lie in 2..127");
  if (n_comp < 1 || n_comp > std::min<int>(K - 1, B))
    return set_error(ctx, CVAMX_E_INVALID_ARG, "n_comp must lie in 1..min(K-1, bands)");
  if (mode < CVAMX_STRETCH_MINMAX || mode > CVAMX_STRETCH_PERCENTILE)
    return set_error(ctx, CVAMX_E_INVALID_ARG, "unknown stretch mode");
  if (bits != 8 && bits != 16) return set_error(ctx, CVAMX_E_INVALID_ARG, "bits must be 8 or 16");
  const int dev = cvamx::ctx_device(ctx);
  if (dev < 0) return set_error(ctx, CVAMX_E_DEVICE, "context has no device");
  if (hipSetDevice(dev) != hipSuccess) return set_error(ctx, CVAMX_E_DEVICE, "hipSetDevice failed");
  hipStream_t cs = (hipStream_t)stream;
  const int64_t P = H * Wd;
  const size_t ein = in_dtype == CVAMX_U8 ? 1 : (in_dtype == CVAMX_U16 ? 2 : 4);
  const size_t eout = in_dtype == CVAMX_F32 ? 4 : 2;
  const size_t img_bytes = (size_t)n_comp * P * (bits / 8);

  // pages with bad pointers or sizes are marked and skipped
  std::vector<int> todo;
  int64_t max_n = 1;
  for (int i = 0; i < n_pages; ++i) {
    cvamx_page& pg = pages[i];
    pg.status = CVAMX_OK;
    if (!pg.bands || !pg.pixels || !pg.classes || !pg.images || pg.n_points < 1 ||
        pg.n_points >= (int64_t(1) << 31)) {
      pg.status = CVAMX_E_INVALID_ARG;
      continue;
    }
    todo.push_back(i);
    max_n = std::max(max_n, pg.n_points);
  }
  if (todo.empty()) return CVAMX_OK;
  // mode 2: the listed points of a class (not the skipped ones), per page
  std::vector<std::vector<int64_t>> train(todo.size());
  if (mode == CVAMX_STRETCH_TRAINING)
    for (size_t t = 0; t < todo.size(); ++t) {
      const cvamx_page& pg = pages[todo[t]];
      for (int64_t k = 0; k < pg.n_points; ++k)
        if (pg.classes[k] >= 0) train[t].push_back(pg.pixels[k]);
    }

  Slots sl;
  sl.cs = cs;
  bool ok = hipStreamCreateWithFlags(&sl.h2d, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&sl.d2h, hipStreamNonBlocking) == hipSuccess;
  for (int s = 0; s < 2 && ok; ++s)
    ok = hipEventCreateWithFlags(&sl.in[s], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done[s], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.img[s], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.out[s], hipEventDisableTiming) == hipSuccess;
  if (!ok) return set_error(ctx, CVAMX_E_DEVICE, "stream or event creation failed");
  for (int s = 0; s < 2 && ok; ++s)
    ok = alloc(&sl.bands[s], (size_t)B * P * ein) && alloc((void**)&sl.pix[s], (size_t)max_n * 8) &&
         alloc((void**)&sl.cls[s], (size_t)max_n + 16) && alloc((void**)&sl.train[s], (size_t)max_n * 8) &&
         alloc(&sl.images[s], img_bytes);
  ok = ok && alloc(&sl.cube, (size_t)B * P * eout) && alloc((void**)&sl.y, (size_t)n_comp * P * 4);
  if (!ok) return set_error(ctx, CVAMX_E_NO_MEMORY, "device memory for the page slots");

  bool in_used[2] = {false, false}, out_used[2] = {false, false};
  auto upload = [&](size_t t) -> bool {
    const cvamx_page& pg = pages[todo[t]];
    const int s = (int)(t & 1);
    if (in_used[s] && hipStreamWaitEvent(sl.h2d, sl.done[s], 0) != hipSuccess) return false;
    bool r = hipMemcpyAsync(sl.bands[s], pg.bands, (size_t)B * P * ein, hipMemcpyHostToDevice, sl.h2d) ==
                 hipSuccess &&
             hipMemcpyAsync(sl.pix[s], pg.pixels, (size_t)pg.n_points * 8, hipMemcpyHostToDevice, sl.h2d) ==
                 hipSuccess &&
             hipMemcpyAsync(sl.cls[s], pg.classes, (size_t)pg.n_points, hipMemcpyHostToDevice, sl.h2d) ==
                 hipSuccess;
    if (r && !train[t].empty())
      r = hipMemcpyAsync(sl.train[s], train[t].data(), train[t].size() * 8, hipMemcpyHostToDevice, sl.h2d) ==
          hipSuccess;
    return r && hipEventRecord(sl.in[s], sl.h2d) == hipSuccess;
  };
  auto fatal = [](int st) { return st == CVAMX_E_DEVICE || st == CVAMX_E_NO_MEMORY; };

  const cvamx_cube cube = {sl.cube, H, Wd, B, in_dtype == CVAMX_F32 ? CVAMX_F32 : CVAMX_U16};
  std::vector<double> Wb((size_t)B * n_comp), lam(n_comp), mean(B), rng(2 * (size_t)n_comp);
  std::vector<int64_t> counts(K);
  if (!upload(0)) return set_error(ctx, CVAMX_E_DEVICE, "page copy");
  for (size_t t = 0; t < todo.size(); ++t) {
    cvamx_page& pg = pages[todo[t]];
    const int s = (int)(t & 1);
    if (hipStreamWaitEvent(cs, sl.in[s], 0) != hipSuccess) return set_error(ctx, CVAMX_E_DEVICE, "stream wait");
    int st = cvamx_bands_to_cube(ctx, sl.bands[s], in_dtype, B, P, sl.cube, cs);
    if (fatal(st)) return st;
    // the next page's copy overlaps this page's fit, eigensolve and projection
    if (t + 1 < todo.size() && !upload(t + 1)) return set_error(ctx, CVAMX_E_DEVICE, "page copy");
    if (st == CVAMX_OK)
      st = cva_fit_points(ctx, &cube, sl.pix[s], sl.cls[s], pg.n_points, K, prec, ridge, n_comp, Wb.data(),
                          lam.data(), mean.data(), counts.data(), nullptr, nullptr, nullptr, cs);
    if (st == CVAMX_OK) st = cvamx_project_float(ctx, &cube, Wb.data(), mean.data(), n_comp, sl.y, cs);
    if (st == CVAMX_OK && mode == CVAMX_STRETCH_TRAINING && train[t].empty())
      st = set_error(ctx, CVAMX_E_INVALID_ARG, "mode 2 needs a point of some class");
    if (st == CVAMX_OK) {
      if (out_used[s] && hipStreamWaitEvent(cs, sl.out[s], 0) != hipSuccess)
        return set_error(ctx, CVAMX_E_DEVICE, "stream wait");
      st = cvamx_stretch(ctx, sl.y, P, n_comp, mode, pct, sl.train[s], (int64_t)train[t].size(), bits,
                         sl.images[s], rng.data(), cs);
    }
    if (st == CVAMX_OK) {
      if (hipEventRecord(sl.img[s], cs) != hipSuccess || hipStreamWaitEvent(sl.d2h, sl.img[s], 0) != hipSuccess ||
          hipMemcpyAsync(pg.images, sl.images[s], img_bytes, hipMemcpyDeviceToHost, sl.d2h) != hipSuccess ||
          hipEventRecord(sl.out[s], sl.d2h) != hipSuccess)
        return set_error(ctx, CVAMX_E_DEVICE, "image copy");
      out_used[s] = true;
      if (pg.W) std::copy(Wb.begin(), Wb.end(), pg.W);
      if (pg.eigvals) std::copy(lam.begin(), lam.end(), pg.eigvals);
      if (pg.range) std::copy(rng.begin(), rng.end(), pg.range);
    }
    pg.status = st;
    if (fatal(st)) return st;
    if (hipEventRecord(sl.done[s], cs) != hipSuccess) return set_error(ctx, CVAMX_E_DEVICE, "event record");
    in_used[s] = true;
  }
  if (hipStreamSynchronize(sl.d2h) != hipSuccess || hipStreamSynchronize(cs) != hipSuccess)
    return set_error(ctx, CVAMX_E_DEVICE, "stream synchronise");
  return CVAMX_OK;
}

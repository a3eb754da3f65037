// Many pages through one context: the CVA enhancement of each page from its
// band images and training points, with the transfers of neighbouring pages
// overlapped with the work on the current one (paper Section 4: a whole
// palimpsest of about 240 pages was processed, and pages were re-run with
// other training points).
//
// Three streams of the batch's own: one for every kernel, in page order, one
// for host-to-device and one for device-to-host copies.  Page t's band images
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
#include <new>
#include <string>
#include <vector>

#include "ctx_internal.hpp"
#include "cvamx.h"

namespace {

// Streams, events and slot buffers of the batches of one context.  They
// outlive a call (a batch of pages re-run with other points costs no
// allocation) and grow when a batch needs more; the context frees them.
struct PipeState {
  hipStream_t cs = nullptr, h2d = nullptr, d2h = nullptr;
  hipEvent_t in[2] = {}, done[2] = {}, img[2] = {}, out[2] = {};
  void* bands[2] = {};
  void* pts[2] = {};     // device: pixels (8 n), classes (n, padded), training pixels (8 n)
  void* host[2] = {};    // page-locked staging of the same (copies from ordinary memory block the host)
  void* images[2] = {};
  void* cube = nullptr;
  void* y = nullptr;
  size_t cap_bands[2] = {}, cap_pts[2] = {}, cap_host[2] = {}, cap_images[2] = {}, cap_cube = 0, cap_y = 0;

  void idle() const {
    for (hipStream_t st : {cs, h2d, d2h})
      if (st) (void)hipStreamSynchronize(st);
  }
  ~PipeState() {
    idle();
    for (int s = 0; s < 2; ++s) {
      for (hipEvent_t e : {in[s], done[s], img[s], out[s]})
        if (e) (void)hipEventDestroy(e);
      for (void* p : {bands[s], pts[s], images[s]})
        if (p) (void)hipFree(p);
      if (host[s]) (void)hipHostFree(host[s]);
    }
    if (cube) (void)hipFree(cube);
    if (y) (void)hipFree(y);
    for (hipStream_t st : {cs, h2d, d2h})
      if (st) (void)hipStreamDestroy(st);
  }
  bool init() {
    bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&h2d, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&d2h, hipStreamNonBlocking) == hipSuccess;
    for (int s = 0; s < 2 && ok; ++s)
      ok = hipEventCreateWithFlags(&in[s], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&done[s], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&img[s], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&out[s], hipEventDisableTiming) == hipSuccess;
    return ok;
  }
};

void free_state(void* p) { delete static_cast<PipeState*>(p); }

// Grow a device (or page-locked host) buffer to `want` bytes; called only
// while every stream of the state is idle.
bool grow(void*& p, size_t& cap, size_t want, bool host = false) {
  if (p && cap >= want) return true;
  if (p) (void)(host ? hipHostFree(p) : hipFree(p));
  p = nullptr;
  cap = 0;
  want = std::max<size_t>(want, 256);
  if ((host ? hipHostMalloc(&p, want, hipHostMallocDefault) : hipMalloc(&p, want)) != hipSuccess) {
    p = nullptr;
    return false;
  }
  cap = want;
  return true;
}

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

  // The kernels run on a stream of the batch's own: the caller's may be the
  // null stream, whose synchronisation (inside each fit) would also wait for
  // the copy streams.  The caller's stream is drained first.
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return set_error(ctx, CVAMX_E_DEVICE, "stream synchronise");
  void** slot = cvamx::ctx_module_state(ctx);
  if (!*slot) {
    PipeState* ps = new (std::nothrow) PipeState();
    if (!ps) return set_error(ctx, CVAMX_E_NO_MEMORY, "batch state");
    if (!ps->init()) {
      delete ps;
      return set_error(ctx, CVAMX_E_DEVICE, "stream or event creation failed");
    }
    *slot = ps;
    cvamx::ctx_set_module_free(ctx, free_state);
  }
  PipeState& sl = *static_cast<PipeState*>(*slot);
  const hipStream_t cs = sl.cs;
  // per slot: pixels (8 n), classes (n, padded), training pixels (8 n)
  // (16-byte aligned parts: the label kernels read the classes in 16-byte words)
  const size_t cls_off = ((size_t)max_n * 8 + 15) & ~size_t(15);
  const size_t tr_off = cls_off + (((size_t)max_n + 15) & ~size_t(15));
  const size_t pts_bytes = tr_off + (size_t)max_n * 8;
  bool ok = true;
  for (int s = 0; s < 2 && ok; ++s)
    ok = grow(sl.bands[s], sl.cap_bands[s], (size_t)B * P * ein) && grow(sl.pts[s], sl.cap_pts[s], pts_bytes) &&
         grow(sl.host[s], sl.cap_host[s], pts_bytes, true) && grow(sl.images[s], sl.cap_images[s], img_bytes);
  ok = ok && grow(sl.cube, sl.cap_cube, (size_t)B * P * eout) && grow(sl.y, sl.cap_y, (size_t)n_comp * P * 4);
  if (!ok) return set_error(ctx, CVAMX_E_NO_MEMORY, "memory for the page slots");
  auto dpix = [&](int s) { return static_cast<int64_t*>(sl.pts[s]); };
  auto dcls = [&](int s) { return static_cast<int8_t*>(sl.pts[s]) + cls_off; };
  auto dtrain = [&](int s) { return reinterpret_cast<int64_t*>(static_cast<char*>(sl.pts[s]) + tr_off); };
  // a fatal error leaves nothing in flight
  auto bail = [&](int code, const char* msg) {
    sl.idle();
    return set_error(ctx, code, msg);
  };

  bool in_used[2] = {false, false}, out_used[2] = {false, false};
  // The host staging of slot s is rewritten for page t once the copies of
  // page t - 2 out of it have completed (in practice long done: that page
  // has been fitted since).
  auto upload = [&](size_t t) -> bool {
    const cvamx_page& pg = pages[todo[t]];
    const int s = (int)(t & 1);
    if (in_used[s] && hipEventSynchronize(sl.in[s]) != hipSuccess) return false;
    char* hs = static_cast<char*>(sl.host[s]);
    std::memcpy(hs, pg.pixels, (size_t)pg.n_points * 8);
    std::memcpy(hs + cls_off, pg.classes, (size_t)pg.n_points);
    if (!train[t].empty()) std::memcpy(hs + tr_off, train[t].data(), train[t].size() * 8);
    if (in_used[s] && hipStreamWaitEvent(sl.h2d, sl.done[s], 0) != hipSuccess) return false;
    // the points first (small), then the band images
    const size_t nb = train[t].empty() ? cls_off + (size_t)pg.n_points : tr_off + train[t].size() * 8;
    bool r = hipMemcpyAsync(sl.pts[s], hs, nb, hipMemcpyHostToDevice, sl.h2d) == hipSuccess &&
             hipMemcpyAsync(sl.bands[s], pg.bands, (size_t)B * P * ein, hipMemcpyHostToDevice, sl.h2d) ==
                 hipSuccess;
    return r && hipEventRecord(sl.in[s], sl.h2d) == hipSuccess;
  };
  auto fatal = [](int st) { return st == CVAMX_E_DEVICE || st == CVAMX_E_NO_MEMORY; };

  const cvamx_cube cube = {sl.cube, H, Wd, B, in_dtype == CVAMX_F32 ? CVAMX_F32 : CVAMX_U16};
  float* y = static_cast<float*>(sl.y);
  std::vector<double> Wb((size_t)B * n_comp), lam(n_comp), mean(B), rng(2 * (size_t)n_comp);
  std::vector<int64_t> counts(K);
  if (!upload(0)) return bail(CVAMX_E_DEVICE, "page copy");
  for (size_t t = 0; t < todo.size(); ++t) {
    cvamx_page& pg = pages[todo[t]];
    const int s = (int)(t & 1);
    if (hipStreamWaitEvent(cs, sl.in[s], 0) != hipSuccess) return bail(CVAMX_E_DEVICE, "stream wait");
    int st = cvamx_bands_to_cube(ctx, sl.bands[s], in_dtype, B, P, sl.cube, cs);
    if (fatal(st)) {
      sl.idle();
      return st;
    }
    // the next page's copy overlaps this page's fit, eigensolve and projection
    if (t + 1 < todo.size() && !upload(t + 1)) return bail(CVAMX_E_DEVICE, "page copy");
    if (st == CVAMX_OK)
      st = cva_fit_points(ctx, &cube, dpix(s), dcls(s), pg.n_points, K, prec, ridge, n_comp, Wb.data(),
                          lam.data(), mean.data(), counts.data(), nullptr, nullptr, nullptr, cs);
    if (st == CVAMX_OK) st = cvamx_project_float(ctx, &cube, Wb.data(), mean.data(), n_comp, y, cs);
    if (st == CVAMX_OK && mode == CVAMX_STRETCH_TRAINING && train[t].empty())
      st = set_error(ctx, CVAMX_E_INVALID_ARG, "mode 2 needs a point of some class");
    if (st == CVAMX_OK) {
      if (out_used[s] && hipStreamWaitEvent(cs, sl.out[s], 0) != hipSuccess)
        return bail(CVAMX_E_DEVICE, "stream wait");
      st = cvamx_stretch(ctx, y, P, n_comp, mode, pct, dtrain(s), (int64_t)train[t].size(), bits,
                         sl.images[s], rng.data(), cs);
    }
    if (st == CVAMX_OK) {
      if (hipEventRecord(sl.img[s], cs) != hipSuccess || hipStreamWaitEvent(sl.d2h, sl.img[s], 0) != hipSuccess ||
          hipMemcpyAsync(pg.images, sl.images[s], img_bytes, hipMemcpyDeviceToHost, sl.d2h) != hipSuccess ||
          hipEventRecord(sl.out[s], sl.d2h) != hipSuccess)
        return bail(CVAMX_E_DEVICE, "image copy");
      out_used[s] = true;
      if (pg.W) std::copy(Wb.begin(), Wb.end(), pg.W);
      if (pg.eigvals) std::copy(lam.begin(), lam.end(), pg.eigvals);
      if (pg.range) std::copy(rng.begin(), rng.end(), pg.range);
    }
    pg.status = st;
    if (fatal(st)) {
      sl.idle();
      return st;
    }
    if (hipEventRecord(sl.done[s], cs) != hipSuccess) return bail(CVAMX_E_DEVICE, "event record");
    in_used[s] = true;
  }
  if (hipStreamSynchronize(sl.d2h) != hipSuccess || hipStreamSynchronize(cs) != hipSuccess)
    return bail(CVAMX_E_DEVICE, "stream synchronise");
  return CVAMX_OK;
}

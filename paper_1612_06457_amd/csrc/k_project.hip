// Projection passes on the VALU, and the dispatchers.  uint16 pages take the
// matrix-core passes of k_project_u16.hip unless the caller asks for the
// vector path (the plain FP32 reference path); float32, bf16 and fp16 pages
// take the VALU passes here.
// For 16-bit float pages the VALU measured faster than a matrix-core form
// with split operands at every band and component count tried (1.2-2.7x at
// 16 to 48 bands and 1 to 12 components): the products are few per byte.
#include "k_project.hpp"

namespace cvx {

// The VALU passes for any element type: the path of float32, bf16 and fp16
// pages, and the plain FP32 reference path of uint16 pages.
#define CVX_GENERIC(CALL)                       \
  switch (dtype) {                              \
    case DT_U16: return CALL(DT_U16);           \
    case DT_F32: return CALL(DT_F32);           \
    case DT_BF16: return CALL(DT_BF16);         \
    case DT_F16: return CALL(DT_F16);           \
    default: return hipErrorInvalidValue;       \
  }

hipError_t project_range_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                 int nblocks, float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                 hipStream_t s) {
#define CVX_C(D) proj::range_nc<D>(nc, cube, B, P, a, nblocks, part, ticket, range_dev, ab_dev, s)
  CVX_GENERIC(CVX_C)
#undef CVX_C
}

hipError_t project_stretch_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                   int nblocks, const float* range_dev, uint8_t* images, hipStream_t s) {
#define CVX_C(D) proj::stretch_nc<D>(nc, cube, B, P, a, nblocks, range_dev, images, s)
  CVX_GENERIC(CVX_C)
#undef CVX_C
}

hipError_t project_float_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                 int nblocks, float* y, hipStream_t s) {
#define CVX_C(D) proj::float_nc<D>(nc, cube, B, P, a, nblocks, y, s)
  CVX_GENERIC(CVX_C)
#undef CVX_C
}

hipError_t project_range_h16_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                     int nblocks, float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                     const H16Args& h, _Float16* planes, int64_t Pp, hipStream_t s) {
#define CVX_C(D) proj::range_nc<D, true>(nc, cube, B, P, a, nblocks, part, ticket, range_dev, ab_dev, s, h, planes, Pp)
  CVX_GENERIC(CVX_C)
#undef CVX_C
}

hipError_t project_stretch_h16_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                       int nblocks, const float* range_dev, const _Float16* planes, int64_t Pp,
                                       uint8_t* images, hipStream_t s) {
#define CVX_C(D) proj::stretch_h16_nc<D>(nc, cube, B, P, a, nblocks, range_dev, planes, Pp, images, s)
  CVX_GENERIC(CVX_C)
#undef CVX_C
}

#undef CVX_GENERIC

hipError_t launch_project_range_h16(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                    const ProjArgs& a, int nblocks, float* part, unsigned* ticket,
                                    float* range_dev, float* ab_dev, const H16Args& h, uint16_t* planes,
                                    int64_t Pp, hipStream_t s) {
  if (Pp < P || Pp % 256 != 0) return hipErrorInvalidValue;
  if (dtype == DT_U16 && !vector)
    return launch_project_range_h16_u16(cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, h, planes, Pp,
                                        s);
  return project_range_h16_generic(dtype, nc, cube, B, P, a, nblocks, part, ticket, range_dev, ab_dev, h,
                                   reinterpret_cast<_Float16*>(planes), Pp, s);
}

hipError_t launch_project_stretch_h16(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                      const ProjArgs& a, int nblocks, const float* range_dev,
                                      const uint16_t* planes, int64_t Pp, uint8_t* images, hipStream_t s) {
  if (Pp < P || Pp % 256 != 0) return hipErrorInvalidValue;
  if (dtype == DT_U16 && !vector)
    return launch_project_stretch_h16_u16(cube, B, P, nc, a, nblocks, range_dev, planes, Pp, images, s);
  return project_stretch_h16_generic(dtype, nc, cube, B, P, a, nblocks, range_dev,
                                     reinterpret_cast<const _Float16*>(planes), Pp, images, s);
}

hipError_t launch_project_range(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                const ProjArgs& a, int nblocks, float* part, unsigned* ticket,
                                float* range_dev, float* ab_dev, hipStream_t s) {
  if (dtype == DT_U16 && !vector)
    return launch_project_range_u16(cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, s);
  return project_range_generic(dtype, nc, cube, B, P, a, nblocks, part, ticket, range_dev, ab_dev, s);
}

hipError_t launch_project_stretch(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                  const ProjArgs& a, int nblocks, const float* range_dev, uint8_t* images,
                                  hipStream_t s) {
  if (dtype == DT_U16 && !vector)
    return launch_project_stretch_u16(cube, B, P, nc, a, nblocks, range_dev, images, s);
  return project_stretch_generic(dtype, nc, cube, B, P, a, nblocks, range_dev, images, s);
}

hipError_t launch_project_float(int dtype, bool vector, const void* cube, int B, int64_t P, int nc,
                                const ProjArgs& a, int nblocks, float* y, hipStream_t s) {
  if (dtype == DT_U16 && !vector) return launch_project_float_u16(cube, B, P, nc, a, nblocks, y, s);
  return project_float_generic(dtype, nc, cube, B, P, a, nblocks, y, s);
}

}  // namespace cvx

// Projection passes on the VALU (float32 pages), and the dispatchers: uint16
// pages go to k_project_u16.hip, bf16 / fp16 pages to k_project_mfma.hip.
#include "k_project.hpp"

namespace cvx {

hipError_t project_range_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                 int nblocks, float* part, unsigned* ticket, float* range_dev, float* ab_dev,
                                 hipStream_t s) {
  if (dtype != DT_F32) return hipErrorInvalidValue;
  return proj::range_nc<DT_F32>(nc, cube, B, P, a, nblocks, part, ticket, range_dev, ab_dev, s);
}

hipError_t project_stretch_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                   int nblocks, const float* range_dev, uint8_t* images, hipStream_t s) {
  if (dtype != DT_F32) return hipErrorInvalidValue;
  return proj::stretch_nc<DT_F32>(nc, cube, B, P, a, nblocks, range_dev, images, s);
}

hipError_t project_float_generic(int dtype, int nc, const void* cube, int B, int64_t P, const ProjArgs& a,
                                 int nblocks, float* y, hipStream_t s) {
  if (dtype != DT_F32) return hipErrorInvalidValue;
  return proj::float_nc<DT_F32>(nc, cube, B, P, a, nblocks, y, s);
}

hipError_t launch_project_range(int dtype, const void* cube, int B, int64_t P, int nc,
                                const ProjArgs& a, int nblocks, float* part, unsigned* ticket,
                                float* range_dev, float* ab_dev, hipStream_t s) {
  if (dtype == DT_U16)
    return launch_project_range_u16(cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, s);
  if (dtype != DT_F32)
    return launch_project_range_mfma(dtype, cube, B, P, nc, a, nblocks, part, ticket, range_dev, ab_dev, s);
  return project_range_generic(dtype, nc, cube, B, P, a, nblocks, part, ticket, range_dev, ab_dev, s);
}

hipError_t launch_project_stretch(int dtype, const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                  int nblocks, const float* range_dev, uint8_t* images, hipStream_t s) {
  if (dtype == DT_U16) return launch_project_stretch_u16(cube, B, P, nc, a, nblocks, range_dev, images, s);
  if (dtype != DT_F32)
    return launch_project_stretch_mfma(dtype, cube, B, P, nc, a, nblocks, range_dev, images, s);
  return project_stretch_generic(dtype, nc, cube, B, P, a, nblocks, range_dev, images, s);
}

hipError_t launch_project_float(int dtype, const void* cube, int B, int64_t P, int nc, const ProjArgs& a,
                                int nblocks, float* y, hipStream_t s) {
  if (dtype == DT_U16) return launch_project_float_u16(cube, B, P, nc, a, nblocks, y, s);
  if (dtype != DT_F32) return launch_project_float_mfma(dtype, cube, B, P, nc, a, nblocks, y, s);
  return project_float_generic(dtype, nc, cube, B, P, a, nblocks, y, s);
}

}  // namespace cvx

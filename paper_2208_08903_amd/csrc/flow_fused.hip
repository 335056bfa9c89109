// Fused flow kernels (placeholder: no shape is covered yet).
#include "lfs_common.hpp"
#include "lfs_internal.hpp"

namespace lfs {
bool fused_supported(const FlowGeom&, int) { return false; }
size_t fused_ws_bytes(const FlowGeom&, int, int) { return 0; }
int32_t fused_forward(const FlowGeom&, const float*, int, const float*, float*, double*, double*,
                      float*, char*, hipStream_t) {
  return LFS_EUNSUPPORTED;
}
int32_t fused_backward(const FlowGeom&, const float*, int, const float*, const float*, double,
                       float*, float*, char*, hipStream_t) {
  return LFS_EUNSUPPORTED;
}
}  // namespace lfs

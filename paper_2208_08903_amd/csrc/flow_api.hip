// C ABI of the flow: descriptor validation, parameter layout, workspace
// sizing and dispatch between the fused and the generic kernel families.
#include <hip/hip_runtime.h>

#include "lfs_common.hpp"
#include "lfs_internal.hpp"

namespace lfs {

int32_t make_geom(const lfs_flow_desc* d, FlowGeom* g) {
  if (!d || !g) return LFS_EINVAL;
  if (d->dim != 2 && d->dim != 3) return LFS_EINVAL;
  if (d->L < 2 || (d->L & 1)) return LFS_EINVAL;
  if (d->n_layers < 1) return LFS_EINVAL;
  if (d->final_tanh != 0 && d->final_tanh != 1) return LFS_EINVAL;
  if (d->parity0 != 0 && d->parity0 != 1) return LFS_EINVAL;
  if (d->precision != LFS_PLAIN_FP32 && d->precision != LFS_BF16_CONV) return LFS_EINVAL;
  if (d->algo < LFS_ALGO_AUTO || d->algo > LFS_ALGO_FUSED) return LFS_EINVAL;
  if (d->L > 256 || (d->dim == 3 && d->L > 64)) return LFS_EUNSUPPORTED;
  if (d->hidden != 8 && d->hidden != 16 && d->hidden != 32) return LFS_EUNSUPPORTED;
  g->dim = d->dim;
  g->L = d->L;
  g->V = d->dim == 2 ? d->L * d->L : d->L * d->L * d->L;
  g->T = d->dim == 2 ? 9 : 27;
  g->N = d->n_layers;
  g->C = d->hidden;
  g->final_tanh = d->final_tanh;
  g->parity0 = d->parity0;
  g->precision = d->precision;
  g->algo = d->algo;
  const size_t C = g->C, T = g->T;
  g->off_W1 = 0;
  g->off_b1 = g->off_W1 + C * T;
  g->off_W2 = g->off_b1 + C;
  g->off_b2 = g->off_W2 + C * C * T;
  g->off_W3 = g->off_b2 + C;
  g->off_b3 = g->off_W3 + 2 * C * T;
  g->P_layer = g->off_b3 + 2;
  g->P_total = g->P_layer * (size_t)g->N;
  return LFS_OK;
}

namespace {

bool use_fused(const FlowGeom& g, int bwd) {
  if (g.algo == LFS_ALGO_GENERIC) return false;
  return fused_supported(g, bwd);
}

}  // namespace
}  // namespace lfs

extern "C" const char* lfs_status_string(int32_t s) {
  switch (s) {
    case LFS_OK: return "LFS_OK";
    case LFS_EINVAL: return "LFS_EINVAL: invalid argument";
    case LFS_EUNSUPPORTED: return "LFS_EUNSUPPORTED: valid but unsupported configuration";
    case LFS_EWORKSPACE: return "LFS_EWORKSPACE: workspace too small";
    case LFS_EDEVICE: return "LFS_EDEVICE: HIP launch or device error";
  }
  return "unknown lfs status";
}

extern "C" const char* lfs_version(void) { return "lfs 0.1.0 (gfx950)"; }

extern "C" size_t lfs_param_count(const lfs_flow_desc* desc) {
  lfs::FlowGeom g;
  return lfs::make_geom(desc, &g) == LFS_OK ? g.P_total : 0;
}

extern "C" int32_t lfs_workspace_bytes(const lfs_flow_desc* desc, int32_t B, int32_t for_backward,
                                       size_t* bytes) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B <= 0 || !bytes) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED && !lfs::fused_supported(g, for_backward))
    return LFS_EUNSUPPORTED;
  *bytes = lfs::use_fused(g, for_backward) ? lfs::fused_ws_bytes(g, B, for_backward)
                                           : lfs::generic_ws_bytes(g, B, for_backward);
  return LFS_OK;
}

extern "C" int32_t lfs_flow_forward(const lfs_flow_desc* desc, const float* params, int32_t B,
                                    const float* z, float* phi, double* logq, double* logdet,
                                    float* saved_x, void* ws, size_t ws_bytes, void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B <= 0 || !params || !z || !phi || !logq) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED && !lfs::fused_supported(g, 0)) return LFS_EUNSUPPORTED;
  const bool fused = lfs::use_fused(g, 0);
  const size_t need = fused ? lfs::fused_ws_bytes(g, B, 0) : lfs::generic_ws_bytes(g, B, 0);
  if (need > 0 && (!ws || ws_bytes < need)) return LFS_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  return fused ? lfs::fused_forward(g, params, B, z, phi, logq, logdet, saved_x, (char*)ws, st)
               : lfs::generic_forward(g, params, B, z, phi, logq, logdet, saved_x, (char*)ws, st);
}

extern "C" int32_t lfs_flow_backward(const lfs_flow_desc* desc, const float* params, int32_t B,
                                     const float* saved_x, const float* g_phi, double g_logq,
                                     float* g_params, float* g_z, void* ws, size_t ws_bytes,
                                     void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B <= 0 || !params || !saved_x || !g_phi || !g_params) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED && !lfs::fused_supported(g, 1)) return LFS_EUNSUPPORTED;
  const bool fused = lfs::use_fused(g, 1);
  const size_t need = fused ? lfs::fused_ws_bytes(g, B, 1) : lfs::generic_ws_bytes(g, B, 1);
  if (need > 0 && (!ws || ws_bytes < need)) return LFS_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  return fused ? lfs::fused_backward(g, params, B, saved_x, g_phi, g_logq, g_params, g_z,
                                     (char*)ws, st)
               : lfs::generic_backward(g, params, B, saved_x, g_phi, g_logq, g_params, g_z,
                                       (char*)ws, st);
}

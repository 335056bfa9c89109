// C ABI of the flow: descriptor validation, parameter layout, workspace
// sizing and dispatch between the fused and the generic kernel families.
#include <hip/hip_runtime.h>

#include <mutex>

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
  const int K = d->kernel == 0 ? 3 : d->kernel;
  if (K < 1 || K > 7 || !(K & 1)) return LFS_EINVAL;
  if (d->n_hidden < 0 || d->n_hidden > LFS_MAX_HIDDEN) return LFS_EINVAL;
  if (d->batch_norm != 0 && d->batch_norm != 1) return LFS_EINVAL;
  int widths[LFS_MAX_HIDDEN], nh;
  if (d->n_hidden == 0) {
    if (d->hidden != 8 && d->hidden != 16 && d->hidden != 32) return LFS_EUNSUPPORTED;
    nh = 2;
    widths[0] = widths[1] = d->hidden;
  } else {
    nh = d->n_hidden;
    for (int i = 0; i < nh; ++i) {
      if (d->hidden_sizes[i] < 1) return LFS_EINVAL;
      if (d->hidden_sizes[i] > 64) return LFS_EUNSUPPORTED;
      widths[i] = d->hidden_sizes[i];
    }
  }
  g->dim = d->dim;
  g->L = d->L;
  g->V = d->dim == 2 ? d->L * d->L : d->L * d->L * d->L;
  g->K = K;
  g->T = d->dim == 2 ? K * K : K * K * K;
  g->N = d->n_layers;
  g->bn = d->batch_norm == 1;
  g->net_default = !g->bn && K == 3 && nh == 2 && widths[0] == widths[1] &&
                   (widths[0] == 8 || widths[0] == 16 || widths[0] == 32);
  g->C = g->net_default ? widths[0] : 0;
  g->n_conv = nh + 1;
  {
    size_t off = 0, soff = 0;
    for (int i = 0; i < g->n_conv; ++i) {
      g->cin[i] = i == 0 ? 1 : widths[i - 1];
      g->cout[i] = i == nh ? 2 : widths[i];
      g->offW[i] = off;
      off += (size_t)g->cout[i] * g->cin[i] * g->T;
      g->offb[i] = off;
      off += g->cout[i];
      if (g->bn && i < nh) {
        g->offg[i] = off;
        off += 2 * (size_t)g->cout[i];
        g->offS[i] = soff;
        soff += 2 * (size_t)g->cout[i];
      }
    }
    g->P_layer = off;
    g->S_layer = soff;
  }
  g->final_tanh = d->final_tanh;
  g->parity0 = d->parity0;
  g->precision = d->precision;
  g->algo = d->algo;
  // the default network's blocks (same offsets as offW/offb above)
  g->off_W1 = g->offW[0];
  g->off_b1 = g->offb[0];
  g->off_W2 = g->offW[1];
  g->off_b2 = g->offb[1];
  g->off_W3 = g->offW[g->n_conv - 1];
  g->off_b3 = g->offb[g->n_conv - 1];
  g->P_total = g->P_layer * (size_t)g->N;
  g->S_total = g->S_layer * (size_t)g->N;
  return LFS_OK;
}

namespace {

// Kernel family of a validated geometry: fused (default network, a fused kernel
// for the shape, algo not GENERIC), generic (default network) or general net.
enum class Family { Fused, Generic, Net };

bool fused_ok(const FlowGeom& g, int bwd) { return g.net_default && fused_supported(g, bwd); }

Family family(const FlowGeom& g, int bwd) {
  if (!g.net_default) return Family::Net;
  if (g.algo != LFS_ALGO_GENERIC && fused_supported(g, bwd)) return Family::Fused;
  return Family::Generic;
}

size_t ws_bytes_of(const FlowGeom& g, int B, int bwd) {
  switch (family(g, bwd)) {
    case Family::Fused: return fused_ws_bytes(g, B, bwd);
    case Family::Generic: return generic_ws_bytes(g, B, bwd);
    default: return net_ws_bytes(g, B, bwd);
  }
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

extern "C" size_t lfs_bn_stats_count(const lfs_flow_desc* desc) {
  lfs::FlowGeom g;
  return lfs::make_geom(desc, &g) == LFS_OK ? g.S_total : 0;
}

extern "C" int32_t lfs_workspace_bytes(const lfs_flow_desc* desc, int32_t B, int32_t for_backward,
                                       size_t* bytes) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B < 0 || !bytes) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED && !lfs::fused_ok(g, for_backward)) return LFS_EUNSUPPORTED;
  *bytes = B == 0 ? 0 : lfs::ws_bytes_of(g, B, for_backward);
  return LFS_OK;
}

extern "C" int32_t lfs_flow_forward(const lfs_flow_desc* desc, const float* params, int32_t B,
                                    const float* z, float* phi, double* logq, double* logdet,
                                    float* saved_x, void* ws, size_t ws_bytes, void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B < 0 || g.bn) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED && !lfs::fused_ok(g, 0)) return LFS_EUNSUPPORTED;
  if (B == 0) return LFS_OK;
  if (!params || !z || !phi || !logq) return LFS_EINVAL;
  const size_t need = lfs::ws_bytes_of(g, B, 0);
  if (need > 0 && (!ws || ws_bytes < need)) return LFS_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  switch (lfs::family(g, 0)) {
    case lfs::Family::Fused:
      return lfs::fused_forward(g, params, B, z, phi, logq, logdet, saved_x, nullptr, (char*)ws, st);
    case lfs::Family::Generic:
      return lfs::generic_forward(g, params, B, z, phi, logq, logdet, saved_x, (char*)ws, st);
    default:
      return lfs::net_forward(g, params, B, z, phi, logq, logdet, saved_x, (char*)ws, st);
  }
}

namespace lfs {
namespace {

// Backward of a validated flow without batch norm; g_logq_vec (nullable) gives
// each sample its own cotangent of log q.
int32_t backward_plain(const lfs_flow_desc* desc, const FlowGeom& g, const float* params, int32_t B,
                       const float* saved_x, const float* g_phi, double g_logq,
                       const double* g_logq_vec, float* g_params, float* g_z, void* ws,
                       size_t ws_bytes, void* stream, const float* saved_h = nullptr) {
  if (B <= 0 || !params || !saved_x || !g_phi || !g_params || g.bn) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED && !fused_ok(g, 1)) return LFS_EUNSUPPORTED;
  const size_t need = ws_bytes_of(g, B, 1);
  if (need > 0 && (!ws || ws_bytes < need)) return LFS_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  switch (family(g, 1)) {
    case Family::Fused:
      return fused_backward(g, params, B, saved_x, saved_h, g_phi, g_logq, g_logq_vec, g_params,
                            g_z, (char*)ws, st);
    case Family::Generic:
      return generic_backward(g, params, B, saved_x, g_phi, g_logq, g_logq_vec, g_params, g_z,
                              (char*)ws, st);
    default:
      return net_backward(g, params, B, saved_x, g_phi, g_logq, g_logq_vec, g_params, g_z,
                          (char*)ws, st);
  }
}

}  // namespace
}  // namespace lfs

extern "C" int32_t lfs_flow_backward(const lfs_flow_desc* desc, const float* params, int32_t B,
                                     const float* saved_x, const float* g_phi, double g_logq,
                                     float* g_params, float* g_z, void* ws, size_t ws_bytes,
                                     void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  return lfs::backward_plain(desc, g, params, B, saved_x, g_phi, g_logq, nullptr, g_params, g_z, ws,
                             ws_bytes, stream);
}

extern "C" int32_t lfs_flow_backward_vec(const lfs_flow_desc* desc, const float* params, int32_t B,
                                         const float* saved_x, const float* g_phi,
                                         const double* g_logq, float* g_params, float* g_z, void* ws,
                                         size_t ws_bytes, void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (!g_logq) return LFS_EINVAL;
  return lfs::backward_plain(desc, g, params, B, saved_x, g_phi, 0.0, g_logq, g_params, g_z, ws,
                             ws_bytes, stream);
}

namespace lfs {
namespace {
// bytes of the saved h2 of a validated flow at batch B (0: its backward recomputes)
size_t saved_h_bytes_of(const FlowGeom& g, int B) {
  if (B <= 0 || family(g, 0) != Family::Fused || family(g, 1) != Family::Fused) return 0;
  return fused_hsave_bytes(g, B);
}
}  // namespace
}  // namespace lfs

extern "C" int32_t lfs_saved_h_bytes(const lfs_flow_desc* desc, int32_t B, size_t* bytes) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B < 0 || !bytes) return LFS_EINVAL;
  *bytes = g.bn ? 0 : lfs::saved_h_bytes_of(g, B);
  return LFS_OK;
}

extern "C" int32_t lfs_flow_forward_train(const lfs_flow_desc* desc, const float* params, int32_t B,
                                          const float* z, float* phi, double* logq, double* logdet,
                                          float* saved_x, float* saved_h, void* ws, size_t ws_bytes,
                                          void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B < 0 || g.bn) return LFS_EINVAL;
  if (B > 0 && !saved_x) return LFS_EINVAL;
  const size_t hb = lfs::saved_h_bytes_of(g, B);
  if (hb == 0) return lfs_flow_forward(desc, params, B, z, phi, logq, logdet, saved_x, ws, ws_bytes, stream);
  if (desc->algo == LFS_ALGO_FUSED && !lfs::fused_ok(g, 0)) return LFS_EUNSUPPORTED;
  if (!params || !z || !phi || !logq || !saved_h) return LFS_EINVAL;
  const size_t need = lfs::ws_bytes_of(g, B, 0);
  if (need > 0 && (!ws || ws_bytes < need)) return LFS_EWORKSPACE;
  return lfs::fused_forward(g, params, B, z, phi, logq, logdet, saved_x, saved_h, (char*)ws,
                            (hipStream_t)stream);
}

extern "C" int32_t lfs_flow_backward_saved(const lfs_flow_desc* desc, const float* params, int32_t B,
                                           const float* saved_x, const float* saved_h,
                                           const float* g_phi, double g_logq, const double* g_logq_vec,
                                           float* g_params, float* g_z, void* ws, size_t ws_bytes,
                                           void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (g.bn) return LFS_EINVAL;
  const size_t hb = lfs::saved_h_bytes_of(g, B);
  if (hb > 0 && !saved_h) return LFS_EINVAL;
  return lfs::backward_plain(desc, g, params, B, saved_x, g_phi, g_logq, g_logq_vec, g_params, g_z, ws,
                             ws_bytes, stream, hb > 0 ? saved_h : nullptr);
}

extern "C" int32_t lfs_flow_forward_bn(const lfs_flow_desc* desc, const float* params, int32_t B,
                                       const float* z, float* phi, double* logq, double* logdet,
                                       float* saved_x, int32_t bn_mode, float* bn_stats,
                                       double momentum, void* ws, size_t ws_bytes, void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (!g.bn) return lfs_flow_forward(desc, params, B, z, phi, logq, logdet, saved_x, ws, ws_bytes, stream);
  if (B < 0 || (B == 0 && bn_mode == LFS_BN_BATCH)) return LFS_EINVAL;  // no statistics of nothing
  if (bn_mode != LFS_BN_BATCH && bn_mode != LFS_BN_RUNNING) return LFS_EINVAL;
  if (!(momentum >= 0.0 && momentum <= 1.0)) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED) return LFS_EUNSUPPORTED;
  if (B == 0) return LFS_OK;
  if (!params || !z || !phi || !logq) return LFS_EINVAL;
  if (bn_mode == LFS_BN_RUNNING && !bn_stats) return LFS_EINVAL;
  const size_t need = lfs::net_ws_bytes(g, B, 0);
  if (!ws || ws_bytes < need) return LFS_EWORKSPACE;
  return lfs::net_forward_bn(g, params, B, z, phi, logq, logdet, saved_x, bn_mode, bn_stats,
                             (float)momentum, (char*)ws, (hipStream_t)stream);
}

extern "C" int32_t lfs_flow_backward_bn(const lfs_flow_desc* desc, const float* params, int32_t B,
                                        const float* saved_x, const float* g_phi, double g_logq,
                                        const double* g_logq_vec, int32_t bn_mode,
                                        const float* bn_stats, float* g_params, float* g_z, void* ws,
                                        size_t ws_bytes, void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (!g.bn)
    return lfs::backward_plain(desc, g, params, B, saved_x, g_phi, g_logq, g_logq_vec, g_params, g_z,
                               ws, ws_bytes, stream);
  if (B <= 0 || !params || !saved_x || !g_phi || !g_params) return LFS_EINVAL;
  if (bn_mode != LFS_BN_BATCH && bn_mode != LFS_BN_RUNNING) return LFS_EINVAL;
  if (bn_mode == LFS_BN_RUNNING && !bn_stats) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED) return LFS_EUNSUPPORTED;
  const size_t need = lfs::net_ws_bytes(g, B, 1);
  if (!ws || ws_bytes < need) return LFS_EWORKSPACE;
  return lfs::net_backward_bn(g, params, B, saved_x, g_phi, g_logq, g_logq_vec, bn_mode, bn_stats,
                              g_params, g_z, (char*)ws, (hipStream_t)stream);
}

// ---- allocation-free forward ------------------------------------------------
// The forward's workspace (weight fragments, or the generic kernels' hidden
// activations) lives in one file-scope device array instead of caller memory.
// Its device address differs per GPU and is looked up once per device with
// that device current; host code never passes the array's name to a kernel.
namespace lfs {
namespace {

__device__ __align__(256) unsigned char scratch[LFS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LFS_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LFS_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LFS_OK;
}

}  // namespace
}  // namespace lfs

extern "C" int32_t lfs_flow_forward_noalloc(const lfs_flow_desc* desc, const float* params, int32_t B,
                                            const float* z, float* phi, double* logq, double* logdet,
                                            float* saved_x, void* stream) {
  lfs::FlowGeom g;
  const int32_t s = lfs::make_geom(desc, &g);
  if (s != LFS_OK) return s;
  if (B < 0 || g.bn) return LFS_EINVAL;
  if (desc->algo == LFS_ALGO_FUSED && !lfs::fused_ok(g, 0)) return LFS_EUNSUPPORTED;
  if (B == 0) return LFS_OK;
  if (lfs::ws_bytes_of(g, B, 0) > LFS_NOALLOC_SCRATCH_BYTES) return LFS_EWORKSPACE;
  void* ws = nullptr;
  const int32_t sp = lfs::scratch_of_current_device(&ws);
  if (sp != LFS_OK) return sp;
  return lfs_flow_forward(desc, params, B, z, phi, logq, logdet, saved_x, ws,
                          LFS_NOALLOC_SCRATCH_BYTES, stream);
}

// Host-side internal interface between the C ABI and the flow kernel families.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "lfs.h"

namespace lfs {

// Geometry of a validated flow descriptor and offsets into the packed
// parameter vector (per layer: W1[C][1][T] b1[C] W2[C][C][T] b2[C] W3[2][C][T] b3[2]).
struct FlowGeom {
  int dim, L, V, T, N, C;
  int final_tanh, parity0, precision, algo;
  size_t off_W1, off_b1, off_W2, off_b2, off_W3, off_b3;  // within a layer (default network)
  size_t P_layer, P_total;
  // every network: kernel size, convolutions with their channel counts and
  // offsets within a layer; net_default: the default network (kernel 3, two
  // hidden convolutions of C = 8, 16 or 32 channels)
  int K, n_conv;
  int cin[LFS_MAX_HIDDEN + 1], cout[LFS_MAX_HIDDEN + 1];
  size_t offW[LFS_MAX_HIDDEN + 1], offb[LFS_MAX_HIDDEN + 1];
  bool net_default;
  // batch norm: gamma (beta follows at + cout) of hidden convolution i within a
  // layer; its statistics (mean, then var at + cout) within a layer's block of
  // S_layer entries of the statistics vector
  bool bn;
  size_t offg[LFS_MAX_HIDDEN], offS[LFS_MAX_HIDDEN];
  size_t S_layer, S_total;

  int frozen_parity(int layer) const { return (layer + parity0) & 1; }
  bool bf16() const { return precision == LFS_BF16_CONV; }
};

// Validates desc; returns LFS_OK and fills g, or a negative status.
int32_t make_geom(const lfs_flow_desc* desc, FlowGeom* g);

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Generic kernels: any supported (dim, L, C), activations staged in HBM.
size_t generic_ws_bytes(const FlowGeom& g, int B, int for_backward);
int32_t generic_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                        double* logq, double* logdet, float* saved, char* ws, hipStream_t st);
int32_t generic_backward(const FlowGeom& g, const float* params, int B, const float* saved,
                         const float* g_phi, double g_logq, const double* g_logq_vec, float* g_params,
                         float* g_z, char* ws,
                         hipStream_t st);

// General-network kernels: any hidden_sizes / odd kernel, activations in HBM.
size_t net_ws_bytes(const FlowGeom& g, int B, int for_backward);
int32_t net_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                    double* logq, double* logdet, float* saved, char* ws, hipStream_t st);
int32_t net_backward(const FlowGeom& g, const float* params, int B, const float* saved,
                     const float* g_phi, double g_logq, const double* g_logq_vec, float* g_params,
                     float* g_z, char* ws,
                     hipStream_t st);
// Batch-norm variants (g.bn): bn_mode lfs_bn_mode; stats per the statistics
// layout (running statistics, updated in batch mode if not null).
int32_t net_forward_bn(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                       double* logq, double* logdet, float* saved, int bn_mode, float* stats,
                       float momentum, char* ws, hipStream_t st);
int32_t net_backward_bn(const FlowGeom& g, const float* params, int B, const float* saved,
                        const float* g_phi, double g_logq, const double* g_logq_vec, int bn_mode,
                        const float* stats,
                        float* g_params, float* g_z, char* ws, hipStream_t st);

// Fused kernels: LDS-resident per-sample lattices, matrix-core convolutions.
bool fused_supported(const FlowGeom& g, int for_backward);
size_t fused_ws_bytes(const FlowGeom& g, int B, int for_backward);
// hsave (nullable): the training forward's saved activations of every layer
// (the resident kernels' HSave images of h2, [N][B] samples, or the
// plane-streaming kernels' RingSave blocks); fused_hsave_bytes gives its size
// (0: the shape's backward recomputes them, and hsave is ignored)
int32_t fused_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                      double* logq, double* logdet, float* saved, float* hsave, char* ws,
                      hipStream_t st);
size_t fused_hsave_bytes(const FlowGeom& g, int B);
int32_t fused_backward(const FlowGeom& g, const float* params, int B, const float* saved,
                       const float* hsave, const float* g_phi, double g_logq,
                       const double* g_logq_vec, float* g_params, float* g_z, char* ws,
                       hipStream_t st);

namespace fused {
// Fused forward streaming planes through LDS rings (3D lattices too large to
// keep resident), implemented next to its kernel.
bool ring_supported(const FlowGeom& g);
size_t ring_ws_bytes(const FlowGeom& g);
// hsave (nullable): the activations saved for the plane-streaming backward
// (RingSave layout, ring_hsave_bytes of them; 0 bytes: not saved for this shape)
int32_t ring_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                     double* logq, double* logdet, float* saved, unsigned char* hsave, char* ws,
                     hipStream_t st);
size_t ring_hsave_bytes(const FlowGeom& g, int B);
// Fused backward (one launch per layer), implemented next to its kernels.
bool bwd_supported(const FlowGeom& g);
size_t bwd_ws_bytes(const FlowGeom& g, int B);
int32_t bwd_run(const FlowGeom& g, const float* params, int B, const float* saved,
                const float* hsave, const float* g_phi, double g_logq, const double* g_logq_vec,
                float* g_params, float* g_z, char* ws, hipStream_t st);
// Fused backward streaming planes (3D lattices too large to keep resident;
// three launches per layer), implemented next to its kernels.
bool ring_bwd_supported(const FlowGeom& g);
size_t ring_bwd_ws_bytes(const FlowGeom& g, int B);
int32_t ring_bwd_run(const FlowGeom& g, const float* params, int B, const float* saved,
                     const unsigned char* hsave, const float* g_phi, double g_logq,
                     const double* g_logq_vec, float* g_params, float* g_z, char* ws, hipStream_t st);
}  // namespace fused

}  // namespace lfs

// Pieces shared by the fused backward kernels: the fragment table of a
// layer's backward, the fixed-order reduction of the per-workgroup weight-
// gradient partials, and the prior term of the gradient with respect to z.
#pragma once

#include "fused_kernels.hpp"
#include "lfs_internal.hpp"

namespace lfs {
namespace fused {
namespace {  // each translation unit keeps its own copy of the kernels

// Sum of the G workgroup partials of P parameters: a block of 16 waves covers
// 64 parameters; wave s sums partials [G s / 16, G (s + 1) / 16) in index order
// (loads unrolled, so several are in flight), then the 16 slice sums are
// combined in index order.  The order depends on G and P only: deterministic.
constexpr int kRedCols = 64, kRedSlices = 16;
__global__ void __launch_bounds__(kRedCols * kRedSlices) kf_reduce(int G, int P,
                                                                  const float* __restrict__ partial,
                                                                  float* __restrict__ out) {
  __shared__ float sh[kRedSlices][kRedCols + 1];
  const int col = threadIdx.x % kRedCols, sl = threadIdx.x / kRedCols;
  const int i = blockIdx.x * kRedCols + col;
  float acc = 0.f;
  if (i < P) {
    const int g0 = (int)((long)G * sl / kRedSlices), g1 = (int)((long)G * (sl + 1) / kRedSlices);
#pragma unroll 8
    for (int g = g0; g < g1; ++g) acc += partial[(size_t)g * P + i];
  }
  sh[sl][col] = acc;
  __syncthreads();
  if (sl == 0 && i < P) {
    float r = sh[0][col];
#pragma unroll
    for (int q = 1; q < kRedSlices; ++q) r += sh[q][col];
    out[i] = r;
  }
}

// The same fixed-order sum done inside a backward launch by its whole grid (for
// the previous layer's partials): blocks of NT / 16 consecutive parameters (a
// whole cache line of each partial row at 512 threads) go to the workgroups in
// turn; slice s of a parameter sums partials [G s / 16, G (s + 1) / 16) in index
// order and the 16 slice sums are combined in index order -- the order of
// kf_reduce, so results are identical.
template <int NT>
__device__ __forceinline__ void grid_reduce(const float* __restrict__ partial, float* __restrict__ out,
                                            int G, int P) {
  constexpr int PW = NT / kRedSlices;  // parameters per pass
  __shared__ float sh[kRedSlices][PW + 1];
  const int q = threadIdx.x % PW, sl = threadIdx.x / PW;
  const int g0 = (int)((long)G * sl / kRedSlices), g1 = (int)((long)G * (sl + 1) / kRedSlices);
  for (int base = blockIdx.x * PW; base < P; base += gridDim.x * PW) {
    const int i = base + q;
    float acc = 0.f;
    if (i < P) {
#pragma unroll 8
      for (int g = g0; g < g1; ++g) acc += partial[(size_t)g * P + i];
    }
    sh[sl][q] = acc;
    __syncthreads();
    if (sl == 0 && i < P) {
      float r = sh[0][q];
#pragma unroll
      for (int k = 1; k < kRedSlices; ++k) r += sh[k][q];
      out[i] = r;
    }
    __syncthreads();
  }
}

// g_z = g_x - g_logq z (d log r / dz = -z); g_logq per sample if g_logq_vec is given.
__global__ void kf_gz(int64_t n, const float* __restrict__ gx, const float* __restrict__ z,
                      float g_logq, const double* __restrict__ g_logq_vec, int64_t V,
                      float* __restrict__ gz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gl = g_logq_vec ? (float)g_logq_vec[i / V] : g_logq;
  gz[i] = gx[i] - gl * z[i];
}

}  // namespace

// x4: the kernel shares conv3 accumulators between four tiles (extra placements)
// quad (FP32 fused backward): conv3 and conv1^T in the 4x4-block layout
inline FragTable bwd_table(const FlowGeom& g, bool bf16, bool x4, bool quad = false) {
  const int T = g.T, C = g.C;
  // FP32 2D: conv1 and conv3^T by site parity (one block per parity of the taps)
  const int ps = !bf16 && T == 9 ? 1 : 0;
  const LayerFrags lf = layer_frags(T, C, bf16, x4, quad, ps);
  const int kt3 = bf16 ? kchunks_bf16(2 * T) : kblocks_f32(2 * T);
  const int k1t = quad ? T * C / 4 : lf.k2;
  const int q = quad ? 1 : 0;
  FragTable t{};
  int n = 0;
  t.s[n++] = FragSpec{0, (int)g.off_W1, 1, C, C, lf.nct, lf.k1, lf.off1, ps ? 0 : 1, 0, 0, ps};
  t.s[n++] = FragSpec{0, (int)g.off_W2, C, C, C, lf.nct, lf.k2, lf.off2, 0, 0, 0};
  t.s[n++] = FragSpec{0, (int)g.off_W3, C, 2, 2, 1, lf.k3, lf.off3, 0, 0, q};
  if (lf.x4)
    for (int u = 1; u < 4; ++u)
      t.s[n++] = FragSpec{0, (int)g.off_W3, C, 2, 2, 1, lf.k2, lf.off3q + (u - 1) * lf.k2, 0, 4 * u, 0};
  t.s[n++] = FragSpec{1, (int)g.off_W3, C, 2, C, lf.nct, kt3, lf.total, 0, 0, 0, ps};
  t.s[n++] = FragSpec{1, (int)g.off_W2, C, C, C, lf.nct, lf.k2, lf.total + lf.nct * kt3, 0, 0, 0};
  t.s[n++] = FragSpec{1, (int)g.off_W1, 1, C, 1, 1, k1t, lf.total + lf.nct * kt3 + lf.nct * lf.k2, 0, 0, q};
  t.count = n;
  t.total = t.s[n - 1].off + k1t;
  return t;
}

}  // namespace fused
}  // namespace lfs

// Generic flow kernels: direct periodic convolutions, one thread per
// (sample, site), activations staged in HBM.  They cover every supported
// shape and serve as the fallback for shapes without a fused kernel.
//
// Coupling layer (paper Sec. 1, coupling-layer equation): the frozen
// sublattice, as one channel with the active sites zeroed, goes through
// conv(1->C)+LeakyReLU, conv(C->C)+LeakyReLU, conv(C->2); s = tanh(o_0) (or o_0),
// t = o_1; active sites become x exp(s) + t and log|det| grows by sum_A s.
// In BF16 mode every convolution operand (activation, gradient, weight) is
// rounded to BF16 and products are accumulated in FP32.
#include <algorithm>

#include "lfs_common.hpp"
#include "lfs_internal.hpp"

namespace lfs {
namespace {

template <int DIM>
constexpr int taps() {
  return DIM == 2 ? 9 : 27;
}

inline dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

// h1 = leaky(conv(mask_F x; W1, b1)), stored [B][V][C].
template <int DIM, int C, bool BF16>
__global__ void __launch_bounds__(256) kg_conv1(int L, int V, int B, int fpar,
                                                const float* __restrict__ x,
                                                const float* __restrict__ W1,
                                                const float* __restrict__ b1,
                                                float* __restrict__ h1) {
  constexpr int T = taps<DIM>();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * V) return;
  const int b = (int)(idx / V), n = (int)(idx % V);
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = b1[c];
  for (int t = 0; t < T; ++t) {
    const int m = neighbor<DIM>(n, t, L);
    const float v = opnd<BF16>(site_parity<DIM>(m, L) == fpar ? x[(size_t)b * V + m] : 0.f);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] += opnd<BF16>(W1[c * T + t]) * v;
  }
#pragma unroll
  for (int c = 0; c < C; ++c) h1[idx * C + c] = leaky(acc[c]);
}

// h2 = leaky(conv(h1; W2, b2)).
template <int DIM, int C, bool BF16>
__global__ void __launch_bounds__(256) kg_conv2(int L, int V, int B, const float* __restrict__ h1,
                                                const float* __restrict__ W2,
                                                const float* __restrict__ b2,
                                                float* __restrict__ h2) {
  constexpr int T = taps<DIM>();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * V) return;
  const int b = (int)(idx / V), n = (int)(idx % V);
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = b2[c];
  for (int t = 0; t < T; ++t) {
    const float* hin = h1 + ((size_t)b * V + neighbor<DIM>(n, t, L)) * C;
    for (int ci = 0; ci < C; ++ci) {
      const float v = opnd<BF16>(hin[ci]);
#pragma unroll
      for (int co = 0; co < C; ++co) acc[co] += opnd<BF16>(W2[(co * C + ci) * T + t]) * v;
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) h2[idx * C + c] = leaky(acc[c]);
}

// o = conv(h2; W3, b3) at one active site.
template <int DIM, int C, bool BF16>
__device__ __forceinline__ void conv3_at(int L, int V, int b, int n, const float* __restrict__ h2,
                                         const float* __restrict__ W3,
                                         const float* __restrict__ b3, float& o0, float& o1) {
  constexpr int T = taps<DIM>();
  o0 = b3[0];
  o1 = b3[1];
  for (int t = 0; t < T; ++t) {
    const float* hin = h2 + ((size_t)b * V + neighbor<DIM>(n, t, L)) * C;
#pragma unroll
    for (int ci = 0; ci < C; ++ci) {
      const float v = opnd<BF16>(hin[ci]);
      o0 += opnd<BF16>(W3[ci * T + t]) * v;
      o1 += opnd<BF16>(W3[(C + ci) * T + t]) * v;
    }
  }
}

// Affine update of the active sites and per-sample log-det (one block per sample).
template <int DIM, int C, bool BF16, typename R>
__global__ void __launch_bounds__(256) kg_couple(int L, int V, int fpar, int final_tanh,
                                                 const float* __restrict__ xin,
                                                 const float* __restrict__ h2,
                                                 const float* __restrict__ W3,
                                                 const float* __restrict__ b3,
                                                 float* __restrict__ xout,
                                                 double* __restrict__ logdet_acc) {
  __shared__ R sh[16];
  const int b = blockIdx.x;
  R ssum = 0;
  for (int n = threadIdx.x; n < V; n += blockDim.x) {
    const float x = xin[(size_t)b * V + n];
    if (site_parity<DIM>(n, L) == fpar) {
      xout[(size_t)b * V + n] = x;
      continue;
    }
    float o0, o1;
    conv3_at<DIM, C, BF16>(L, V, b, n, h2, W3, b3, o0, o1);
    const float s = final_tanh ? tanhf(o0) : o0;
    xout[(size_t)b * V + n] = x * expf(s) + o1;
    ssum += (R)s;
  }
  ssum = block_sum(ssum, sh);
  if (threadIdx.x == 0) logdet_acc[b] += (double)ssum;
}

// log r(z) = -1/2 sum z^2 - (V/2) ln 2pi (one block per sample); zeroes the log-det accumulator.
template <typename R>
__global__ void __launch_bounds__(256) kg_logr(int V, const float* __restrict__ z,
                                               double* __restrict__ logr,
                                               double* __restrict__ logdet_acc) {
  __shared__ R sh[16];
  const int b = blockIdx.x;
  R acc = 0;
  for (int n = threadIdx.x; n < V; n += blockDim.x) {
    const R v = (R)z[(size_t)b * V + n];
    acc += v * v;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    logr[b] = -0.5 * (double)acc - 0.5 * (double)V * 1.8378770664093454836;
    logdet_acc[b] = 0.0;
  }
}

// logq = log r - logdet.
__global__ void kg_finalize(int B, const double* __restrict__ logr,
                            const double* __restrict__ logdet_acc, double* __restrict__ logq,
                            double* __restrict__ logdet) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  logq[b] = logr[b] - logdet_acc[b];
  if (logdet) logdet[b] = logdet_acc[b];
}

// Backward of the affine update: cotangents of (o_0, o_1) at active sites and
// of x (active: g exp(s); frozen: g, the conv path is added by kg_conv1T).
template <int DIM, int C, bool BF16>
__global__ void __launch_bounds__(256) kg_couple_bwd(int L, int V, int B, int fpar, int final_tanh,
                                                     const float* __restrict__ x,
                                                     const float* __restrict__ h2,
                                                     const float* __restrict__ W3,
                                                     const float* __restrict__ b3,
                                                     const float* __restrict__ gy, float g_ld,
                                                     const double* __restrict__ g_ld_vec,
                                                     float* __restrict__ g_o,
                                                     float* __restrict__ gx) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * V) return;
  const int b = (int)(idx / V), n = (int)(idx % V);
  const float g = gy[idx];
  if (site_parity<DIM>(n, L) == fpar) {
    g_o[2 * idx] = 0.f;
    g_o[2 * idx + 1] = 0.f;
    gx[idx] = g;
    return;
  }
  float o0, o1;
  conv3_at<DIM, C, BF16>(L, V, b, n, h2, W3, b3, o0, o1);
  const float s = final_tanh ? tanhf(o0) : o0;
  const float es = expf(s);
  const float gs = g * x[idx] * es + (g_ld_vec ? (float)(-g_ld_vec[b]) : g_ld);
  g_o[2 * idx] = final_tanh ? gs * (1.f - s * s) : gs;
  g_o[2 * idx + 1] = g;
  gx[idx] = g * es;
}

// g_a2 = leaky'(h2) * conv3^T(g_o).
template <int DIM, int C, bool BF16>
__global__ void __launch_bounds__(256) kg_conv3T(int L, int V, int B, const float* __restrict__ g_o,
                                                 const float* __restrict__ W3,
                                                 const float* __restrict__ h2,
                                                 float* __restrict__ g_a2) {
  constexpr int T = taps<DIM>();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * V) return;
  const int b = (int)(idx / V), m = (int)(idx % V);
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.f;
  for (int t = 0; t < T; ++t) {
    const size_t n = (size_t)b * V + neighbor<DIM>(m, t, L, -1);
    const float g0 = opnd<BF16>(g_o[2 * n]), g1 = opnd<BF16>(g_o[2 * n + 1]);
#pragma unroll
    for (int ci = 0; ci < C; ++ci)
      acc[ci] += opnd<BF16>(W3[ci * T + t]) * g0 + opnd<BF16>(W3[(C + ci) * T + t]) * g1;
  }
#pragma unroll
  for (int c = 0; c < C; ++c) g_a2[idx * C + c] = acc[c] * leaky_grad_from_out(h2[idx * C + c]);
}

// g_a1 = leaky'(h1) * conv2^T(g_a2).
template <int DIM, int C, bool BF16>
__global__ void __launch_bounds__(256) kg_conv2T(int L, int V, int B, const float* __restrict__ g_a2,
                                                 const float* __restrict__ W2,
                                                 const float* __restrict__ h1,
                                                 float* __restrict__ g_a1) {
  constexpr int T = taps<DIM>();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * V) return;
  const int b = (int)(idx / V), m = (int)(idx % V);
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.f;
  for (int t = 0; t < T; ++t) {
    const float* gin = g_a2 + ((size_t)b * V + neighbor<DIM>(m, t, L, -1)) * C;
    for (int co = 0; co < C; ++co) {
      const float g = opnd<BF16>(gin[co]);
#pragma unroll
      for (int ci = 0; ci < C; ++ci) acc[ci] += opnd<BF16>(W2[(co * C + ci) * T + t]) * g;
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) g_a1[idx * C + c] = acc[c] * leaky_grad_from_out(h1[idx * C + c]);
}

// gx[frozen] += conv1^T(g_a1) (the masked input h0 only sees frozen sites).
template <int DIM, int C, bool BF16>
__global__ void __launch_bounds__(256) kg_conv1T(int L, int V, int B, int fpar,
                                                 const float* __restrict__ g_a1,
                                                 const float* __restrict__ W1,
                                                 float* __restrict__ gx) {
  constexpr int T = taps<DIM>();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * V) return;
  const int b = (int)(idx / V), m = (int)(idx % V);
  if (site_parity<DIM>(m, L) != fpar) return;
  float acc = 0.f;
  for (int t = 0; t < T; ++t) {
    const float* gin = g_a1 + ((size_t)b * V + neighbor<DIM>(m, t, L, -1)) * C;
#pragma unroll
    for (int c = 0; c < C; ++c) acc += opnd<BF16>(W1[c * T + t]) * opnd<BF16>(gin[c]);
  }
  gx[idx] += acc;
}

// Per-sample weight-gradient partials:
//   dW[co][ci][t] = sum_n g[n][co] u[n + delta_t][ci],  db[co] = sum_n g[n][co].
// When fpar >= 0, u is the masked field: u[m] = x[m] at frozen sites, else 0.
template <int DIM, bool BF16>
__global__ void __launch_bounds__(256) kg_wgrad(int L, int V, int Co, int Ci, int fpar,
                                                const float* __restrict__ g,
                                                const float* __restrict__ u,
                                                float* __restrict__ partial, int ldp, int woff,
                                                int boff) {
  constexpr int T = taps<DIM>();
  const int b = blockIdx.y;
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int nW = Co * Ci * T;
  if (w >= nW + Co) return;
  const float* gb = g + (size_t)b * V * Co;
  float acc = 0.f;
  if (w < nW) {
    const int co = w / (Ci * T), ci = (w / T) % Ci, t = w % T;
    for (int n = 0; n < V; ++n) {
      const int m = neighbor<DIM>(n, t, L);
      float uv;
      if (fpar >= 0)
        uv = site_parity<DIM>(m, L) == fpar ? u[(size_t)b * V + m] : 0.f;
      else
        uv = u[((size_t)b * V + m) * Ci + ci];
      acc += opnd<BF16>(gb[(size_t)n * Co + co]) * opnd<BF16>(uv);
    }
    partial[(size_t)b * ldp + woff + w] = acc;
  } else {
    const int co = w - nW;
    for (int n = 0; n < V; ++n) acc += gb[(size_t)n * Co + co];
    partial[(size_t)b * ldp + boff + co] = acc;
  }
}

// out[i] = sum_b partial[b][i] in sample order (FP64 accumulation).
__global__ void __launch_bounds__(256) kg_reduce(int B, int P, const float* __restrict__ partial,
                                                 float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  double acc = 0.0;
  for (int b = 0; b < B; ++b) acc += partial[(size_t)b * P + i];
  out[i] = (float)acc;
}

// g_z = g_x - g_logq z (d log r / dz = -z); g_logq per sample if g_logq_vec is given.
__global__ void kg_gz(int64_t n, const float* __restrict__ gx, const float* __restrict__ z,
                      float g_logq, const double* __restrict__ g_logq_vec, int64_t V,
                      float* __restrict__ gz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gl = g_logq_vec ? (float)g_logq_vec[i / V] : g_logq;
  gz[i] = gx[i] - gl * z[i];
}

struct GenericWs {
  double *logdet, *logr;
  float *h1, *h2, *g_o, *g_a2, *g_a1, *gA, *gB, *partial;
};

GenericWs carve(const FlowGeom& g, int B, char* base, size_t* total) {
  GenericWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const size_t BV = (size_t)B * g.V;
  w.logdet = (double*)take(sizeof(double) * B);
  w.logr = (double*)take(sizeof(double) * B);
  w.h1 = (float*)take(sizeof(float) * BV * g.C);
  w.h2 = (float*)take(sizeof(float) * BV * g.C);
  const size_t fwd = off;
  w.g_o = (float*)take(sizeof(float) * BV * 2);
  w.g_a2 = (float*)take(sizeof(float) * BV * g.C);
  w.g_a1 = (float*)take(sizeof(float) * BV * g.C);
  w.gA = (float*)take(sizeof(float) * BV);
  w.gB = (float*)take(sizeof(float) * BV);
  w.partial = (float*)take(sizeof(float) * (size_t)B * g.P_layer);
  total[0] = fwd;
  total[1] = off;
  return w;
}

template <int DIM, int C, bool BF16>
int32_t forward_impl(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                     double* logq, double* logdet, float* saved, char* ws, hipStream_t st) {
  size_t tot[2];
  GenericWs w = carve(g, B, ws, tot);
  const int V = g.V, L = g.L;
  const size_t BV = (size_t)B * V;
  // log r first: phi may alias z.
  if (BF16)
    hipLaunchKernelGGL(kg_logr<double>, dim3(B), dim3(256), 0, st, V, z, w.logr, w.logdet);
  else
    hipLaunchKernelGGL(kg_logr<float>, dim3(B), dim3(256), 0, st, V, z, w.logr, w.logdet);
  float* cur = saved ? saved : phi;
  if (cur != z) hipMemcpyAsync(cur, z, sizeof(float) * BV, hipMemcpyDeviceToDevice, st);
  for (int l = 0; l < g.N; ++l) {
    const float* p = params + (size_t)l * g.P_layer;
    const float* xin = saved ? saved + (size_t)l * BV : phi;
    float* xout = saved ? saved + (size_t)(l + 1) * BV : phi;
    const int fpar = g.frozen_parity(l);
    hipLaunchKernelGGL((kg_conv1<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, fpar, xin,
                       p + g.off_W1, p + g.off_b1, w.h1);
    hipLaunchKernelGGL((kg_conv2<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, w.h1,
                       p + g.off_W2, p + g.off_b2, w.h2);
    if (BF16)
      hipLaunchKernelGGL((kg_couple<DIM, C, BF16, double>), dim3(B), dim3(256), 0, st, L, V, fpar,
                         g.final_tanh, xin, w.h2, p + g.off_W3, p + g.off_b3, xout, w.logdet);
    else
      hipLaunchKernelGGL((kg_couple<DIM, C, BF16, float>), dim3(B), dim3(256), 0, st, L, V, fpar,
                         g.final_tanh, xin, w.h2, p + g.off_W3, p + g.off_b3, xout, w.logdet);
  }
  if (saved && phi) hipMemcpyAsync(phi, saved + (size_t)g.N * BV, sizeof(float) * BV,
                                   hipMemcpyDeviceToDevice, st);
  hipLaunchKernelGGL(kg_finalize, grid1(B), dim3(256), 0, st, B, w.logr, w.logdet, logq, logdet);
  return launch_status();
}

template <int DIM, int C, bool BF16>
int32_t backward_impl(const FlowGeom& g, const float* params, int B, const float* saved,
                      const float* g_phi, double g_logq, const double* g_logq_vec, float* g_params,
                      float* g_z, char* ws,
                      hipStream_t st) {
  constexpr int T = taps<DIM>();
  size_t tot[2];
  GenericWs w = carve(g, B, ws, tot);
  const int V = g.V, L = g.L;
  const size_t BV = (size_t)B * V;
  const float* gy = g_phi;
  float* bufs[2] = {w.gA, w.gB};
  int which = 0;
  const int ldp = (int)g.P_layer;
  for (int l = g.N - 1; l >= 0; --l) {
    const float* p = params + (size_t)l * g.P_layer;
    const float* x = saved + (size_t)l * BV;
    const int fpar = g.frozen_parity(l);
    float* gx = bufs[which];
    hipLaunchKernelGGL((kg_conv1<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, fpar, x,
                       p + g.off_W1, p + g.off_b1, w.h1);
    hipLaunchKernelGGL((kg_conv2<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, w.h1,
                       p + g.off_W2, p + g.off_b2, w.h2);
    hipLaunchKernelGGL((kg_couple_bwd<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, fpar,
                       g.final_tanh, x, w.h2, p + g.off_W3, p + g.off_b3, gy, (float)(-g_logq),
                       g_logq_vec, w.g_o, gx);
    hipLaunchKernelGGL((kg_conv3T<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, w.g_o,
                       p + g.off_W3, w.h2, w.g_a2);
    hipLaunchKernelGGL((kg_conv2T<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, w.g_a2,
                       p + g.off_W2, w.h1, w.g_a1);
    hipLaunchKernelGGL((kg_conv1T<DIM, C, BF16>), grid1(BV), dim3(256), 0, st, L, V, B, fpar,
                       w.g_a1, p + g.off_W1, gx);
    hipLaunchKernelGGL((kg_wgrad<DIM, BF16>), dim3((2 * C * T + 2 + 255) / 256, B), dim3(256), 0,
                       st, L, V, 2, C, -1, w.g_o, w.h2, w.partial, ldp, (int)g.off_W3,
                       (int)g.off_b3);
    hipLaunchKernelGGL((kg_wgrad<DIM, BF16>), dim3((C * C * T + C + 255) / 256, B), dim3(256), 0,
                       st, L, V, C, C, -1, w.g_a2, w.h1, w.partial, ldp, (int)g.off_W2,
                       (int)g.off_b2);
    hipLaunchKernelGGL((kg_wgrad<DIM, BF16>), dim3((C * T + C + 255) / 256, B), dim3(256), 0, st,
                       L, V, C, 1, fpar, w.g_a1, x, w.partial, ldp, (int)g.off_W1, (int)g.off_b1);
    hipLaunchKernelGGL(kg_reduce, grid1(g.P_layer), dim3(256), 0, st, B, ldp, w.partial,
                       g_params + (size_t)l * g.P_layer);
    gy = gx;
    which ^= 1;
  }
  if (g_z)
    hipLaunchKernelGGL(kg_gz, grid1(BV), dim3(256), 0, st, (int64_t)BV, gy, saved,
                       (float)g_logq, g_logq_vec, (int64_t)V, g_z);
  return launch_status();
}

template <int DIM, bool BF16>
int32_t fwd_c(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
              double* logq, double* logdet, float* saved, char* ws, hipStream_t st) {
  switch (g.C) {
    case 8: return forward_impl<DIM, 8, BF16>(g, params, B, z, phi, logq, logdet, saved, ws, st);
    case 16: return forward_impl<DIM, 16, BF16>(g, params, B, z, phi, logq, logdet, saved, ws, st);
    case 32: return forward_impl<DIM, 32, BF16>(g, params, B, z, phi, logq, logdet, saved, ws, st);
  }
  return LFS_EUNSUPPORTED;
}

template <int DIM, bool BF16>
int32_t bwd_c(const FlowGeom& g, const float* params, int B, const float* saved,
              const float* g_phi, double g_logq, const double* g_logq_vec, float* g_params, float* g_z,
              char* ws,
              hipStream_t st) {
  switch (g.C) {
    case 8:
      return backward_impl<DIM, 8, BF16>(g, params, B, saved, g_phi, g_logq, g_logq_vec, g_params, g_z, ws,
                                         st);
    case 16:
      return backward_impl<DIM, 16, BF16>(g, params, B, saved, g_phi, g_logq, g_logq_vec, g_params, g_z, ws,
                                          st);
    case 32:
      return backward_impl<DIM, 32, BF16>(g, params, B, saved, g_phi, g_logq, g_logq_vec, g_params, g_z, ws,
                                          st);
  }
  return LFS_EUNSUPPORTED;
}

}  // namespace

size_t generic_ws_bytes(const FlowGeom& g, int B, int for_backward) {
  size_t tot[2];
  carve(g, B, nullptr, tot);
  return tot[for_backward ? 1 : 0];
}

int32_t generic_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                        double* logq, double* logdet, float* saved, char* ws, hipStream_t st) {
  if (g.dim == 2)
    return g.bf16() ? fwd_c<2, true>(g, params, B, z, phi, logq, logdet, saved, ws, st)
                    : fwd_c<2, false>(g, params, B, z, phi, logq, logdet, saved, ws, st);
  return g.bf16() ? fwd_c<3, true>(g, params, B, z, phi, logq, logdet, saved, ws, st)
                  : fwd_c<3, false>(g, params, B, z, phi, logq, logdet, saved, ws, st);
}

int32_t generic_backward(const FlowGeom& g, const float* params, int B, const float* saved,
                         const float* g_phi, double g_logq, const double* g_logq_vec, float* g_params,
                         float* g_z, char* ws,
                         hipStream_t st) {
  if (g.dim == 2)
    return g.bf16() ? bwd_c<2, true>(g, params, B, saved, g_phi, g_logq, g_logq_vec, g_params, g_z, ws, st)
                    : bwd_c<2, false>(g, params, B, saved, g_phi, g_logq, g_logq_vec, g_params, g_z, ws, st);
  return g.bf16() ? bwd_c<3, true>(g, params, B, saved, g_phi, g_logq, g_logq_vec, g_params, g_z, ws, st)
                  : bwd_c<3, false>(g, params, B, saved, g_phi, g_logq, g_logq_vec, g_params, g_z, ws, st);
}

}  // namespace lfs

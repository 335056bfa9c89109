// General s/t networks: the example parameter file's hidden_sizes and
// kernel_size beyond the default two hidden convolutions of C channels with
// kernel 3.  Per layer the network is conv(1 -> w_1) + LeakyReLU, ...,
// conv(w_{n-1} -> w_n) + LeakyReLU, conv(w_n -> 2) with an odd kernel K per
// axis (paper Sec. 1, coupling-layer equation; taps row-major over
// {-K/2..K/2}^dim, axis 0 slowest).  Direct periodic convolutions with runtime
// channel counts and the kernel size as a template parameter, kSplit lanes per
// (sample, site, output channel), activations in HBM.  In BF16 mode every
// convolution operand is rounded to BF16 and products are accumulated in FP32,
// as in the other kernel families.
//
// Batch norm (the parameter file's use_bn): a hidden convolution's output a is
// kept, its per-channel statistics are reduced over the batch and all sites in
// FP64 with a fixed chunk order (two passes: the mean, then the squared
// deviations), and h = leaky(gamma (a - mean) r + beta), r = 1/sqrt(var + eps),
// is written next to it.  The backward turns g_y = g_h leaky'(y) into g_a with
// the per-channel sums of g_y xhat and g_y.
#include <type_traits>

#include "lfs_common.hpp"
#include "lfs_internal.hpp"

namespace lfs {
namespace {

inline dim3 grid_for(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

constexpr int ipow(int k, int d) { return d == 0 ? 1 : k * ipow(k, d - 1); }

constexpr int kWgChunk = 4096;  // (sample, site) terms per weight-gradient or batch-norm partial sum
// Lanes that share one convolution output: lane s of a group takes the (tap,
// channel) pairs q = t cin + ci with q = s mod kSplit, and the group's partial
// sums are combined by a fixed xor-shuffle tree (deterministic).
constexpr int kSplit = 8;

__device__ __forceinline__ float split_sum(float v) {
#pragma unroll
  for (int o = kSplit / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kSplit);
  return v;
}

// First channel c of the pairs (t, c), c = c0, c0 + kSplit, ..., that lane s takes.
__device__ __forceinline__ int split_first(int s, int t, int nc) { return (s - t * nc) & (kSplit - 1); }

constexpr double kBnEps = 1e-5;
constexpr int kMaxWidth = 64;   // hidden_sizes entries are at most 64

// Site arithmetic of the periodic L^DIM lattice (row-major, axis 0 slowest):
// coordinates by shift and mask when L is a power of two (lg = log2 L), by
// division otherwise, and (c + d) mod L for kernel offsets |d| <= 3 by two
// conditional corrections each way (L >= 2).
template <int DIM>
struct SiteMath {
  int L, lg;
  __device__ __forceinline__ void coords(int n, int (&c)[DIM]) const {
#pragma unroll
    for (int mu = DIM - 1; mu >= 0; --mu) {
      if (lg >= 0) {
        c[mu] = n & (L - 1);
        n >>= lg;
      } else {
        c[mu] = n % L;
        n /= L;
      }
    }
  }
  __device__ __forceinline__ int wrap(int v) const {
    v = v < 0 ? v + L : v;
    v = v < 0 ? v + L : v;
    v = v >= L ? v - L : v;
    return v >= L ? v - L : v;
  }
  // sample and site of the (sample, site) term bn
  __device__ __forceinline__ void split(int64_t bn, int V, int& b, int& n) const {
    if (lg >= 0) {
      b = (int)(bn >> (lg * DIM));
      n = (int)(bn & (V - 1));
    } else {
      b = (int)(bn / V);
      n = (int)(bn % V);
    }
  }
};

// f(t, m) for every tap t of an odd kernel K, m = the site at coordinates
// c + sign * delta_t; taps row-major over {-K/2..K/2}^DIM, axis 0 slowest.  K is
// a compile-time constant so that a row of taps unrolls and its loads overlap.
template <int DIM, int K, typename F>
__device__ __forceinline__ void for_taps(const SiteMath<DIM>& sm, const int (&c)[DIM], int sign, F&& f) {
  constexpr int r = K >> 1;
  int t = 0;
  if constexpr (DIM == 2) {
    for (int d0 = -r; d0 <= r; ++d0) {
      const int row = sm.wrap(c[0] + sign * d0) * sm.L;
#pragma unroll
      for (int d1 = -r; d1 <= r; ++d1, ++t) f(t, row + sm.wrap(c[1] + sign * d1));
    }
  } else {
    for (int d0 = -r; d0 <= r; ++d0) {
      const int pl = sm.wrap(c[0] + sign * d0) * sm.L;
      for (int d1 = -r; d1 <= r; ++d1) {
        const int row = (pl + sm.wrap(c[1] + sign * d1)) * sm.L;
#pragma unroll
        for (int d2 = -r; d2 <= r; ++d2, ++t) f(t, row + sm.wrap(c[2] + sign * d2));
      }
    }
  }
}

// out[b][n][co] = act(bias[co] + sum_t sum_ci W[co][ci][t] in[b][n + delta_t][ci]),
// kSplit lanes per output.  first: the input is the layer's field with the
// active sites zeroed (cin = 1).
template <int DIM, int K, bool BF16>
__global__ void __launch_bounds__(256) kn_conv(int L, int lg, int V, int B, int cin, int cout,
                                               int first, int fpar, int act,
                                               const float* __restrict__ in,
                                               const float* __restrict__ W,
                                               const float* __restrict__ bias,
                                               float* __restrict__ out) {
  constexpr int T = ipow(K, DIM);
  const int64_t gidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // groups of kSplit lanes never straddle the end (the grid is a multiple of kSplit)
  if (gidx >= (int64_t)B * V * cout * kSplit) return;
  const int s = (int)(gidx & (kSplit - 1));
  const int64_t idx = gidx / kSplit;
  const int co = (int)(idx % cout);
  const int64_t bn = idx / cout;
  const SiteMath<DIM> sm{L, lg};
  int b, n, c[DIM];
  sm.split(bn, V, b, n);
  sm.coords(n, c);
  const float* w = W + (size_t)co * cin * T;
  const float* ib = in + (size_t)b * V * (first ? 1 : cin);
  float acc = 0.f;
  for_taps<DIM, K>(sm, c, 1, [&](int t, int m) {
    if (first) {
      if (((t - s) & (kSplit - 1)) == 0) {
        const float v = site_parity<DIM>(m, L) == fpar ? ib[m] : 0.f;
        acc += opnd<BF16>(w[t]) * opnd<BF16>(v);
      }
    } else {
      const float* h = ib + (size_t)m * cin;
      for (int ci = split_first(s, t, cin); ci < cin; ci += kSplit)
        acc += opnd<BF16>(w[(size_t)ci * T + t]) * opnd<BF16>(h[ci]);
    }
  });
  acc = split_sum(acc) + bias[co];
  if (s == 0) out[idx] = act ? leaky(acc) : acc;
}

// Affine update of the active sites from o = (o_0, o_1) and per-sample log-det
// (one block per sample).
template <int DIM, typename R>
__global__ void __launch_bounds__(256) kn_couple(int L, int V, int fpar, int final_tanh,
                                                 const float* __restrict__ xin,
                                                 const float* __restrict__ o,
                                                 float* __restrict__ xout,
                                                 double* __restrict__ logdet_acc) {
  __shared__ R sh[16];
  const int b = blockIdx.x;
  R ssum = 0;
  for (int n = threadIdx.x; n < V; n += blockDim.x) {
    const size_t i = (size_t)b * V + n;
    const float x = xin[i];
    if (site_parity<DIM>(n, L) == fpar) {
      xout[i] = x;
      continue;
    }
    const float s = final_tanh ? tanhf(o[2 * i]) : o[2 * i];
    xout[i] = x * expf(s) + o[2 * i + 1];
    ssum += (R)s;
  }
  ssum = block_sum(ssum, sh);
  if (threadIdx.x == 0) logdet_acc[b] += (double)ssum;
}

// log r(z) per sample (one block per sample); zeroes the log-det accumulator.
template <typename R>
__global__ void __launch_bounds__(256) kn_logr(int V, const float* __restrict__ z,
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

__global__ void kn_finalize(int B, const double* __restrict__ logr, const double* __restrict__ ld,
                            double* __restrict__ logq, double* __restrict__ logdet) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  logq[b] = logr[b] - ld[b];
  if (logdet) logdet[b] = ld[b];
}

// Backward of the affine update: g_o at the active sites (zero at the frozen
// ones) and g_x (active: g e^s; frozen: g, the network's path is added later).
// The log-det's cotangent is g_ld, or -g_ld_vec[b] per sample when given.
template <int DIM>
__global__ void __launch_bounds__(256) kn_affine_bwd(int L, int V, int B, int fpar, int final_tanh,
                                                     const float* __restrict__ x,
                                                     const float* __restrict__ o,
                                                     const float* __restrict__ gy, float g_ld,
                                                     const double* __restrict__ g_ld_vec,
                                                     float* __restrict__ go,
                                                     float* __restrict__ gx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * V) return;
  const int n = (int)(i % V);
  const float g = gy[i];
  if (site_parity<DIM>(n, L) == fpar) {
    go[2 * i] = 0.f;
    go[2 * i + 1] = 0.f;
    gx[i] = g;
    return;
  }
  const float s = final_tanh ? tanhf(o[2 * i]) : o[2 * i];
  const float es = expf(s);
  const float gs = g * x[i] * es + (g_ld_vec ? (float)(-g_ld_vec[i / V]) : g_ld);
  go[2 * i] = final_tanh ? gs * (1.f - s * s) : gs;
  go[2 * i + 1] = g;
  gx[i] = g * es;
}

// Data gradient of a convolution: gin[b][m][ci] = sum_t sum_co W[co][ci][t]
// g[b][m - delta_t][co], times LeakyReLU' of the input h (from its sign), or,
// for the first convolution, added to gx at the frozen sites; kSplit lanes per
// output.
template <int DIM, int K, bool BF16>
__global__ void __launch_bounds__(256) kn_conv_t(int L, int lg, int V, int B, int cin, int cout,
                                                 int first, int fpar, const float* __restrict__ g,
                                                 const float* __restrict__ W,
                                                 const float* __restrict__ h,
                                                 float* __restrict__ gin) {
  constexpr int T = ipow(K, DIM);
  const int64_t gidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gidx >= (int64_t)B * V * cin * kSplit) return;   // whole groups of kSplit lanes
  const int s = (int)(gidx & (kSplit - 1));
  const int64_t idx = gidx / kSplit;
  const int ci = (int)(idx % cin);
  const int64_t bm = idx / cin;
  const SiteMath<DIM> sm{L, lg};
  int b, m, c[DIM];
  sm.split(bm, V, b, m);
  sm.coords(m, c);
  const float* gb = g + (size_t)b * V * cout;
  float acc = 0.f;
  for_taps<DIM, K>(sm, c, -1, [&](int t, int nb) {
    const float* gr = gb + (size_t)nb * cout;
    for (int co = split_first(s, t, cout); co < cout; co += kSplit)
      acc += opnd<BF16>(W[((size_t)co * cin + ci) * T + t]) * opnd<BF16>(gr[co]);
  });
  acc = split_sum(acc);
  if (s != 0) return;
  if (first) {
    if (site_parity<DIM>(m, L) == fpar) gin[bm] += acc;
  } else {
    gin[idx] = acc * leaky_grad_from_out(h[idx]);
  }
}

// Partial weight and bias gradients of one convolution over the (sample, site)
// terms [chunk * kWgChunk, +kWgChunk): parameter p < cout cin T is W[co][ci][t]
// (sum of g[.][n][co] u[.][n + delta_t][ci]), the rest b[co] (sum of g).  One
// workgroup per (parameter, chunk); fixed-order sums.  With a single chunk the
// sum is the gradient and goes straight to `direct`.
template <int DIM, bool BF16>
__global__ void __launch_bounds__(256) kn_wgrad(int L, int lg, int V, int B, int K, int T, int cin, int cout,
                                                int first, int fpar, const float* __restrict__ g,
                                                const float* __restrict__ u,
                                                double* __restrict__ partial, int P,
                                                float* __restrict__ direct) {
  __shared__ double sh[16];
  const int p = blockIdx.x, chunk = blockIdx.y;
  const int64_t BV = (int64_t)B * V;
  const int64_t t0 = (int64_t)chunk * kWgChunk, t1 = t0 + kWgChunk < BV ? t0 + kWgChunk : BV;
  const int nW = cout * cin * T;
  double acc = 0.0;
  if (p < nW) {
    const int co = p / (cin * T), ci = (p / T) % cin;
    // this parameter's tap offsets
    const SiteMath<DIM> sm{L, lg};
    int d[DIM];
    {
      int t = p % T;
#pragma unroll
      for (int mu = DIM - 1; mu >= 0; --mu) {
        d[mu] = t % K - (K >> 1);
        t /= K;
      }
    }
    // four terms' loads in flight at a time, summed in term order
    auto term = [&](int64_t bn) {
      int b, n, c[DIM];
      sm.split(bn, V, b, n);
      sm.coords(n, c);
      int m = 0;
#pragma unroll
      for (int mu = 0; mu < DIM; ++mu) m = m * L + sm.wrap(c[mu] + d[mu]);
      float uv;
      if (first)
        uv = site_parity<DIM>(m, L) == fpar ? u[(size_t)b * V + m] : 0.f;
      else
        uv = u[((size_t)b * V + m) * cin + ci];
      return opnd<BF16>(g[bn * cout + co]) * opnd<BF16>(uv);
    };
    const int64_t step = blockDim.x;
    int64_t bn = t0 + threadIdx.x;
    for (; bn + 3 * step < t1; bn += 4 * step) {
      const float q0 = term(bn), q1 = term(bn + step), q2 = term(bn + 2 * step), q3 = term(bn + 3 * step);
      acc += (double)q0;
      acc += (double)q1;
      acc += (double)q2;
      acc += (double)q3;
    }
    for (; bn < t1; bn += step) acc += (double)term(bn);
  } else {
    const int co = p - nW;
    for (int64_t bn = t0 + threadIdx.x; bn < t1; bn += blockDim.x) acc += (double)g[bn * cout + co];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (direct)
      direct[p] = (float)acc;
    else
      partial[(size_t)chunk * P + p] = acc;
  }
}

// out[p] = sum over chunks of partial[chunk][p], in chunk order.
__global__ void __launch_bounds__(256) kn_reduce(int G, int P, const double* __restrict__ partial,
                                                 float* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double acc = 0.0;
  for (int c = 0; c < G; ++c) acc += partial[(size_t)c * P + p];
  out[p] = (float)acc;
}

// g_z = g_x - g_logq z (d log r / dz = -z); g_logq per sample if g_logq_vec is given.
__global__ void kn_gz(int64_t n, const float* __restrict__ gx, const float* __restrict__ z,
                      float g_logq, const double* __restrict__ g_logq_vec, int64_t V,
                      float* __restrict__ gz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gl = g_logq_vec ? (float)g_logq_vec[i / V] : g_logq;
  gz[i] = gx[i] - gl * z[i];
}

// ---- batch norm ------------------------------------------------------------

__device__ __forceinline__ float bn_xhat(float a, double mean, double r) {
  return (float)(((double)a - mean) * r);
}

// Per-channel partial sums of a [B V][c] tensor over the (sample, site) terms of
// chunk blockIdx.y, channel blockIdx.x:
//   OP 0: sum a                      -> partial[chunk][ch]
//   OP 1: sum (a - mean)^2           -> partial[chunk][ch], mean = sums[ch] / n
//   OP 2: sum g xhat and sum g       -> partial[chunk][ch] and partial[chunk][c + ch]
template <int OP>
__global__ void __launch_bounds__(256) kn_bn_partial(int64_t BV, int c, const float* __restrict__ a,
                                                     const float* __restrict__ g,
                                                     const double* __restrict__ sums,
                                                     const double* __restrict__ mean,
                                                     const double* __restrict__ rstd,
                                                     double* __restrict__ partial, int P) {
  __shared__ double sh[16];
  const int ch = blockIdx.x, chunk = blockIdx.y;
  const int64_t t0 = (int64_t)chunk * kWgChunk, t1 = t0 + kWgChunk < BV ? t0 + kWgChunk : BV;
  double s0 = 0.0, s1 = 0.0;
  const double mu = OP == 1 ? sums[ch] / (double)BV : OP == 2 ? mean[ch] : 0.0;
  const double r = OP == 2 ? rstd[ch] : 0.0;
  for (int64_t bn = t0 + threadIdx.x; bn < t1; bn += blockDim.x) {
    const float v = a[bn * c + ch];
    if (OP == 0) {
      s0 += (double)v;
    } else if (OP == 1) {
      const double d = (double)v - mu;
      s0 += d * d;
    } else {
      const float gv = g[bn * c + ch];
      s0 += (double)gv * (double)bn_xhat(v, mu, r);
      s1 += (double)gv;
    }
  }
  s0 = block_sum(s0, sh);
  if (OP == 2) s1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    partial[(size_t)chunk * P + ch] = s0;
    if (OP == 2) partial[(size_t)chunk * P + c + ch] = s1;
  }
}

// out[p] = sum over chunks of partial[chunk][p], in chunk order (FP64).
__global__ void __launch_bounds__(256) kn_reduce_d(int G, int P, const double* __restrict__ partial,
                                                   double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double acc = 0.0;
  for (int k = 0; k < G; ++k) acc += partial[(size_t)k * P + p];
  out[p] = acc;
}

// Batch statistics of channel ch from sums[ch] = sum a and the partials of
// sum (a - mean)^2; optionally the running-statistics update.
__global__ void kn_bn_batch_stats(int c, int G, int64_t BV, const double* __restrict__ sums,
                                  const double* __restrict__ partial, double* __restrict__ mean,
                                  double* __restrict__ rstd, float* __restrict__ running,
                                  float momentum) {
  const int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= c) return;
  double sq = 0.0;
  for (int k = 0; k < G; ++k) sq += partial[(size_t)k * c + ch];
  const double n = (double)BV;
  const double mu = sums[ch] / n, var = sq / n;
  mean[ch] = mu;
  rstd[ch] = 1.0 / sqrt(var + kBnEps);
  if (running) {
    const double m = (double)momentum;
    running[ch] = (float)((1.0 - m) * (double)running[ch] + m * mu);
    running[c + ch] = (float)((1.0 - m) * (double)running[c + ch] + m * var * (n / (n - 1.0)));
  }
}

// Running statistics (mean[c] then var[c]) into mean and r.
__global__ void kn_bn_running_stats(int c, const float* __restrict__ stats, double* __restrict__ mean,
                                    double* __restrict__ rstd) {
  const int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= c) return;
  mean[ch] = (double)stats[ch];
  rstd[ch] = 1.0 / sqrt((double)stats[c + ch] + kBnEps);
}

// h = leaky(gamma xhat + beta) over [B V][c].
__global__ void __launch_bounds__(256) kn_bn_apply(int64_t n, int c, const float* __restrict__ a,
                                                   const double* __restrict__ mean,
                                                   const double* __restrict__ rstd,
                                                   const float* __restrict__ gamma,
                                                   const float* __restrict__ beta,
                                                   float* __restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ch = (int)(i % c);
  h[i] = leaky(gamma[ch] * bn_xhat(a[i], mean[ch], rstd[ch]) + beta[ch]);
}

// g_y -> g_a in place (batch statistics: gamma r (g_y - sg / n - xhat sgx / n);
// running: gamma r g_y), sums = (sgx[c], sg[c]); the first 2c threads also
// write the gamma and beta gradients (sgx, then sg; B V >= 4 so the grid of
// B V c threads covers them).
__global__ void __launch_bounds__(256) kn_bn_bwd(int64_t BV, int c, int batch, const float* __restrict__ a,
                                                 const double* __restrict__ mean,
                                                 const double* __restrict__ rstd,
                                                 const float* __restrict__ gamma,
                                                 const double* __restrict__ sums, float* __restrict__ g,
                                                 float* __restrict__ g_gamma_beta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * c) g_gamma_beta[i] = (float)sums[i];
  if (i >= BV * c) return;
  const int ch = (int)(i % c);
  const double k = (double)gamma[ch] * rstd[ch];
  double ga = (double)g[i];
  if (batch) {
    const double n = (double)BV;
    ga -= sums[c + ch] / n + (double)bn_xhat(a[i], mean[ch], rstd[ch]) * (sums[ch] / n);
  }
  g[i] = (float)(k * ga);
}

// ---------------------------------------------------------------------------

// log2 L for a power of two, else -1 (the kernels then divide)
int log2_or_neg(int L) { return (L & (L - 1)) == 0 ? __builtin_ctz((unsigned)L) : -1; }

// f(std::integral_constant<int, K>) for the odd kernel sizes 1..7 (validated by make_geom)
template <typename F>
void with_kernel_size(int K, F&& f) {
  switch (K) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    default: f(std::integral_constant<int, 7>{}); break;
  }
}

struct NetWs {
  double *logdet, *logr, *partial;
  float* h[LFS_MAX_HIDDEN];
  float *o, *go, *gA, *gB, *gxA, *gxB;
  // batch norm: pre-normalisation outputs, per-channel mean and r of every
  // hidden convolution, and per-channel sums
  float* a[LFS_MAX_HIDDEN];
  double *bn_mean, *bn_rstd, *bn_sum;
};

// How a layer's network normalises (batch norm only).
struct BnRun {
  int mode;              // LFS_BN_BATCH or LFS_BN_RUNNING
  const float* stats;    // running mode: the layer's statistics block
  float* running;        // batch mode: the layer's running statistics to update, or null
  float momentum;
};

int max_width(const FlowGeom& g) {
  int w = 2;
  for (int i = 0; i < g.n_conv; ++i) w = w > g.cout[i] ? w : g.cout[i];
  return w;
}

size_t max_conv_params(const FlowGeom& g) {
  size_t m = 2 * kMaxWidth;  // batch-norm partials: two sums per channel
  for (int i = 0; i < g.n_conv; ++i) {
    const size_t p = (size_t)g.cout[i] * g.cin[i] * g.T + g.cout[i];
    m = m > p ? m : p;
  }
  return m;
}

int wg_chunks(int B, int V) { return (int)(((int64_t)B * V + kWgChunk - 1) / kWgChunk); }

NetWs carve(const FlowGeom& g, int B, char* base, size_t* total) {
  NetWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const size_t BV = (size_t)B * g.V;
  w.logdet = (double*)take(sizeof(double) * B);
  w.logr = (double*)take(sizeof(double) * B);
  for (int i = 0; i + 1 < g.n_conv; ++i) w.h[i] = (float*)take(sizeof(float) * BV * g.cout[i]);
  w.o = (float*)take(sizeof(float) * BV * 2);
  const size_t partial_bytes = sizeof(double) * (size_t)wg_chunks(B, g.V) * max_conv_params(g);
  if (g.bn) {
    for (int i = 0; i + 1 < g.n_conv; ++i) w.a[i] = (float*)take(sizeof(float) * BV * g.cout[i]);
    w.bn_mean = (double*)take(sizeof(double) * LFS_MAX_HIDDEN * kMaxWidth);
    w.bn_rstd = (double*)take(sizeof(double) * LFS_MAX_HIDDEN * kMaxWidth);
    w.bn_sum = (double*)take(sizeof(double) * 2 * kMaxWidth);
    w.partial = (double*)take(partial_bytes);
  }
  const size_t fwd = off;
  const int mw = max_width(g);
  w.go = (float*)take(sizeof(float) * BV * 2);
  w.gA = (float*)take(sizeof(float) * BV * mw);
  w.gB = (float*)take(sizeof(float) * BV * mw);
  w.gxA = (float*)take(sizeof(float) * BV);
  w.gxB = (float*)take(sizeof(float) * BV);
  if (!g.bn) w.partial = (double*)take(partial_bytes);
  total[0] = fwd;
  total[1] = off;
  return w;
}

// Batch norm of hidden convolution i from w.a[i] into w.h[i] (statistics into
// w.bn_mean / w.bn_rstd + i * kMaxWidth).
void run_bn(const FlowGeom& g, const float* p, int B, int i, const BnRun& bn, const NetWs& w,
            hipStream_t st) {
  const int64_t BV = (int64_t)B * g.V;
  const int c = g.cout[i], G = wg_chunks(B, g.V);
  double* mean = w.bn_mean + i * kMaxWidth;
  double* rstd = w.bn_rstd + i * kMaxWidth;
  if (bn.mode == LFS_BN_BATCH) {
    hipLaunchKernelGGL(kn_bn_partial<0>, dim3(c, G), dim3(256), 0, st, BV, c, w.a[i], nullptr, nullptr,
                       nullptr, nullptr, w.partial, c);
    hipLaunchKernelGGL(kn_reduce_d, dim3(1), dim3(kMaxWidth), 0, st, G, c, w.partial, w.bn_sum);
    hipLaunchKernelGGL(kn_bn_partial<1>, dim3(c, G), dim3(256), 0, st, BV, c, w.a[i], nullptr, w.bn_sum,
                       nullptr, nullptr, w.partial, c);
    hipLaunchKernelGGL(kn_bn_batch_stats, dim3(1), dim3(kMaxWidth), 0, st, c, G, BV, w.bn_sum, w.partial,
                       mean, rstd, bn.running ? bn.running + g.offS[i] : nullptr, bn.momentum);
  } else {
    hipLaunchKernelGGL(kn_bn_running_stats, dim3(1), dim3(kMaxWidth), 0, st, c, bn.stats + g.offS[i],
                       mean, rstd);
  }
  hipLaunchKernelGGL(kn_bn_apply, grid_for(BV * c), dim3(256), 0, st, BV * c, c, w.a[i], mean, rstd,
                     p + g.offg[i], p + g.offg[i] + c, w.h[i]);
}

// The layer's network from its input field x: hidden activations into w.h, output into w.o.
template <int DIM, bool BF16>
void run_net(const FlowGeom& g, const float* p, int B, const float* x, int fpar, const NetWs& w,
             const BnRun& bn, hipStream_t st) {
  const int64_t BV = (int64_t)B * g.V;
  for (int i = 0; i < g.n_conv; ++i) {
    const bool last = i + 1 == g.n_conv;
    const bool norm = g.bn && !last;
    float* out = last ? w.o : norm ? w.a[i] : w.h[i];
    const float* in = i == 0 ? x : w.h[i - 1];
    with_kernel_size(g.K, [&](auto kc) {
      hipLaunchKernelGGL((kn_conv<DIM, decltype(kc)::value, BF16>), grid_for(BV * g.cout[i] * kSplit),
                         dim3(256), 0, st, g.L, log2_or_neg(g.L), g.V, B, g.cin[i], g.cout[i], i == 0, fpar,
                         !last && !norm, in, p + g.offW[i], p + g.offb[i], out);
    });
    if (norm) run_bn(g, p, B, i, bn, w, st);
  }
}

template <int DIM, bool BF16>
int32_t forward_impl(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                     double* logq, double* logdet, float* saved, int bn_mode, float* stats,
                     float momentum, char* ws, hipStream_t st) {
  size_t tot[2];
  NetWs w = carve(g, B, ws, tot);
  const size_t BV = (size_t)B * g.V;
  // log r first: phi may alias z
  if (BF16)
    hipLaunchKernelGGL(kn_logr<double>, dim3(B), dim3(256), 0, st, g.V, z, w.logr, w.logdet);
  else
    hipLaunchKernelGGL(kn_logr<float>, dim3(B), dim3(256), 0, st, g.V, z, w.logr, w.logdet);
  float* cur = saved ? saved : phi;
  if (cur != z && hipMemcpyAsync(cur, z, sizeof(float) * BV, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return LFS_EDEVICE;
  for (int l = 0; l < g.N; ++l) {
    const float* p = params + (size_t)l * g.P_layer;
    const float* xin = saved ? saved + (size_t)l * BV : phi;
    float* xout = saved ? saved + (size_t)(l + 1) * BV : phi;
    const int fpar = g.frozen_parity(l);
    BnRun bn{bn_mode, nullptr, nullptr, momentum};
    if (g.bn && stats) {
      if (bn_mode == LFS_BN_RUNNING)
        bn.stats = stats + (size_t)l * g.S_layer;
      else
        bn.running = stats + (size_t)l * g.S_layer;
    }
    run_net<DIM, BF16>(g, p, B, xin, fpar, w, bn, st);
    if (BF16)
      hipLaunchKernelGGL((kn_couple<DIM, double>), dim3(B), dim3(256), 0, st, g.L, g.V, fpar,
                         g.final_tanh, xin, w.o, xout, w.logdet);
    else
      hipLaunchKernelGGL((kn_couple<DIM, float>), dim3(B), dim3(256), 0, st, g.L, g.V, fpar,
                         g.final_tanh, xin, w.o, xout, w.logdet);
  }
  if (saved && phi &&
      hipMemcpyAsync(phi, saved + (size_t)g.N * BV, sizeof(float) * BV, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return LFS_EDEVICE;
  hipLaunchKernelGGL(kn_finalize, grid_for(B), dim3(256), 0, st, B, w.logr, w.logdet, logq, logdet);
  return launch_status();
}

template <int DIM, bool BF16>
int32_t backward_impl(const FlowGeom& g, const float* params, int B, const float* saved,
                      const float* g_phi, double g_logq, const double* g_logq_vec, int bn_mode,
                      const float* stats,
                      float* g_params, float* g_z, char* ws, hipStream_t st) {
  size_t tot[2];
  NetWs w = carve(g, B, ws, tot);
  const int64_t BV = (int64_t)B * g.V;
  const int G = wg_chunks(B, g.V);
  const float* gy = g_phi;
  float* gxs[2] = {w.gxA, w.gxB};
  float* gbuf[2] = {w.gA, w.gB};
  int which = 0;
  for (int l = g.N - 1; l >= 0; --l) {
    const float* p = params + (size_t)l * g.P_layer;
    float* gp = g_params + (size_t)l * g.P_layer;
    const float* x = saved + (size_t)l * BV;
    const int fpar = g.frozen_parity(l);
    float* gx = gxs[which];
    // batch statistics are recomputed (no running update); running ones are read
    const BnRun bn{bn_mode, g.bn && bn_mode == LFS_BN_RUNNING ? stats + (size_t)l * g.S_layer : nullptr,
                   nullptr, 0.f};
    run_net<DIM, BF16>(g, p, B, x, fpar, w, bn, st);
    hipLaunchKernelGGL((kn_affine_bwd<DIM>), grid_for(BV), dim3(256), 0, st, g.L, g.V, B, fpar,
                       g.final_tanh, x, w.o, gy, (float)(-g_logq), g_logq_vec, w.go, gx);
    // back through the convolutions, last to first; gcur is the gradient of
    // convolution i's output
    const float* gcur = w.go;
    for (int i = g.n_conv - 1; i >= 0; --i) {
      const int P = g.cout[i] * g.cin[i] * g.T + g.cout[i];
      const float* u = i == 0 ? x : w.h[i - 1];
      hipLaunchKernelGGL((kn_wgrad<DIM, BF16>), dim3(P, G), dim3(256), 0, st, g.L, log2_or_neg(g.L), g.V,
                         B, g.K, g.T, g.cin[i], g.cout[i], i == 0, fpar, gcur, u, w.partial, P,
                         G == 1 ? gp + g.offW[i] : nullptr);
      if (G > 1)
        hipLaunchKernelGGL(kn_reduce, grid_for(P), dim3(256), 0, st, G, P, w.partial, gp + g.offW[i]);
      float* gin = i == 0 ? gx : gbuf[i & 1];
      with_kernel_size(g.K, [&](auto kc) {
        hipLaunchKernelGGL((kn_conv_t<DIM, decltype(kc)::value, BF16>), grid_for(BV * g.cin[i] * kSplit),
                           dim3(256), 0, st, g.L, log2_or_neg(g.L), g.V, B, g.cin[i], g.cout[i], i == 0,
                           fpar, gcur, p + g.offW[i], i == 0 ? nullptr : w.h[i - 1], gin);
      });
      if (g.bn && i > 0) {
        // gin holds g_y of hidden convolution j = i - 1: back through its normalisation
        const int j = i - 1, c = g.cout[j];
        const double* mean = w.bn_mean + j * kMaxWidth;
        const double* rstd = w.bn_rstd + j * kMaxWidth;
        hipLaunchKernelGGL(kn_bn_partial<2>, dim3(c, G), dim3(256), 0, st, BV, c, w.a[j], gin, nullptr,
                           mean, rstd, w.partial, 2 * c);
        hipLaunchKernelGGL(kn_reduce_d, dim3(1), dim3(2 * kMaxWidth), 0, st, G, 2 * c, w.partial,
                           w.bn_sum);
        hipLaunchKernelGGL(kn_bn_bwd, grid_for(BV * c), dim3(256), 0, st, BV, c,
                           bn_mode == LFS_BN_BATCH, w.a[j], mean, rstd, p + g.offg[j], w.bn_sum, gin,
                           gp + g.offg[j]);
      }
      gcur = gin;
    }
    gy = gx;
    which ^= 1;
  }
  if (g_z)
    hipLaunchKernelGGL(kn_gz, grid_for(BV), dim3(256), 0, st, BV, gy, saved, (float)g_logq, g_logq_vec,
                       (int64_t)g.V, g_z);
  return launch_status();
}

}  // namespace

size_t net_ws_bytes(const FlowGeom& g, int B, int for_backward) {
  size_t tot[2];
  carve(g, B, nullptr, tot);
  return tot[for_backward ? 1 : 0];
}

int32_t net_forward_bn(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                       double* logq, double* logdet, float* saved, int bn_mode, float* stats,
                       float momentum, char* ws, hipStream_t st) {
  if (g.dim == 2)
    return g.bf16() ? forward_impl<2, true>(g, params, B, z, phi, logq, logdet, saved, bn_mode, stats,
                                            momentum, ws, st)
                    : forward_impl<2, false>(g, params, B, z, phi, logq, logdet, saved, bn_mode, stats,
                                             momentum, ws, st);
  return g.bf16() ? forward_impl<3, true>(g, params, B, z, phi, logq, logdet, saved, bn_mode, stats,
                                          momentum, ws, st)
                  : forward_impl<3, false>(g, params, B, z, phi, logq, logdet, saved, bn_mode, stats,
                                           momentum, ws, st);
}

int32_t net_backward_bn(const FlowGeom& g, const float* params, int B, const float* saved,
                        const float* g_phi, double g_logq, const double* g_logq_vec, int bn_mode,
                        const float* stats,
                        float* g_params, float* g_z, char* ws, hipStream_t st) {
  if (g.dim == 2)
    return g.bf16() ? backward_impl<2, true>(g, params, B, saved, g_phi, g_logq, g_logq_vec, bn_mode, stats,
                  g_params,
                                             g_z, ws, st)
                    : backward_impl<2, false>(g, params, B, saved, g_phi, g_logq, g_logq_vec, bn_mode, stats,
                                              g_params, g_z, ws, st);
  return g.bf16() ? backward_impl<3, true>(g, params, B, saved, g_phi, g_logq, g_logq_vec, bn_mode, stats,
                g_params,
                                           g_z, ws, st)
                  : backward_impl<3, false>(g, params, B, saved, g_phi, g_logq, g_logq_vec, bn_mode, stats,
                                            g_params,
                                            g_z, ws, st);
}

int32_t net_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                    double* logq, double* logdet, float* saved, char* ws, hipStream_t st) {
  return net_forward_bn(g, params, B, z, phi, logq, logdet, saved, LFS_BN_BATCH, nullptr, 0.f, ws, st);
}

int32_t net_backward(const FlowGeom& g, const float* params, int B, const float* saved,
                     const float* g_phi, double g_logq, const double* g_logq_vec, float* g_params,
                     float* g_z, char* ws,
                     hipStream_t st) {
  return net_backward_bn(g, params, B, saved, g_phi, g_logq, g_logq_vec, LFS_BN_BATCH, nullptr, g_params,
                         g_z, ws, st);
}

}  // namespace lfs

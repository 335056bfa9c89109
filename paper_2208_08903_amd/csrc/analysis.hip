// Chain-quality analysis (paper Sec. 1: the statistical error of a Monte Carlo
// average falls as 1/sqrt(N_indep), N_indep = N_conf / (2 tau_ac); Sec. 2.2 and
// the conclusions: the condensate, zero-momentum two-point functions, the
// autocorrelation time and the effective sample size as analysis quantities).
// All sums in FP64 and in a fixed order, so results are reproducible bit for bit.
#include <algorithm>
#include <cmath>

#include "lfs_common.hpp"

namespace lfs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kAcChunk = 2048;   // series elements per autocovariance workgroup
constexpr int kAcMaxLag = 8192;  // (chunk + lags) FP64 values staged in LDS: <= 80 KB

// Sum over the workgroup: lanes by butterfly, then the waves in index order.
// Every thread of the workgroup must call it; all receive the sum.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) s = fmax(s, red[w]);
  return s;
}

// One workgroup per configuration.  Time slice t (first coordinate t) is the
// contiguous block of `slice` = L^(d-1) sites at t * slice; wave w sums slices
// w, w + 4, ... with its lanes strided over the slice, 16 bytes per lane and
// load when every slice starts 16-byte aligned (vec).  Then M = sum_t Phi(t) / V
// (slices in order) and C(t) = (1/V) sum_t0 Phi(t0) Phi((t0 + t) mod L) by thread t.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_observables(int L, int slice, int vec, const T* __restrict__ phi,
                                                         double* __restrict__ M, double* __restrict__ C) {
  extern __shared__ double Phi[];  // [L]
  constexpr int E = 16 / sizeof(T);  // elements per 16 bytes
  struct alignas(16) Vec { T v[E]; };
  const int b = blockIdx.x, lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const T* f = phi + (size_t)b * L * slice;
  for (int t = w; t < L; t += kWaves) {
    const T* s = f + (size_t)t * slice;
    double acc = 0.0;
    if (vec) {
      for (int i = lane; i < slice / E; i += kWave) {
        const Vec x = reinterpret_cast<const Vec*>(s)[i];
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) part += (double)x.v[e];
        acc += part;
      }
    } else {
      for (int i = lane; i < slice; i += kWave) acc += (double)s[i];
    }
    acc = wave_sum(acc);
    if (lane == 0) Phi[t] = acc;
  }
  __syncthreads();
  const double V = (double)L * slice;
  if (M && threadIdx.x == 0) {
    double m = 0.0;
    for (int t = 0; t < L; ++t) m += Phi[t];
    M[b] = m / V;
  }
  if (C) {
    for (int t = threadIdx.x; t < L; t += kThreads) {
      double c = 0.0;
      for (int t0 = 0, t1 = t; t0 < L; ++t0, t1 = (t1 + 1 == L ? 0 : t1 + 1)) c += Phi[t0] * Phi[t1];
      C[(size_t)b * L + t] = c / V;
    }
  }
}

// Element k of series s: x[s * ldx + k], or x[s * ldx + index[s * n + k]].
__device__ __forceinline__ int64_t series_at(const int64_t* index, int64_t n, int s, int64_t k) {
  return index ? index[(size_t)s * n + k] : k;
}

// Series mean (strided per-thread sums, then block_sum), and whether any index
// falls outside [0, ldx).
__global__ void __launch_bounds__(kThreads) k_ac_mean(int64_t n, const double* __restrict__ x, int64_t ldx,
                                                     const int64_t* __restrict__ index,
                                                     double* __restrict__ mean, int32_t* __restrict__ bad) {
  __shared__ double red[kWaves];
  const int s = blockIdx.x;
  double acc = 0.0, nbad = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kThreads) {
    const int64_t j = series_at(index, n, s, k);
    if (j < 0 || j >= ldx) {
      nbad += 1.0;
    } else {
      acc += x[(size_t)s * ldx + j];
    }
  }
  acc = block_sum(acc, red);
  nbad = block_sum(nbad, red);
  if (threadIdx.x == 0) {
    mean[s] = acc / (double)n;
    bad[s] = nbad > 0.0;
  }
}

// Partial autocovariance sums of one chunk: elements i0 .. i0 + kAcChunk - 1
// against i + t for every lag t <= T (deviations from the mean staged in LDS).
__global__ void __launch_bounds__(kThreads) k_ac_partial(int64_t n, int T, const double* __restrict__ x,
                                                        int64_t ldx, const int64_t* __restrict__ index,
                                                        const double* __restrict__ mean,
                                                        const int32_t* __restrict__ bad,
                                                        double* __restrict__ partial) {
  extern __shared__ double d[];  // [kAcChunk + T]
  const int c = blockIdx.x, s = blockIdx.y, nchunk = gridDim.x;
  const int64_t i0 = (int64_t)c * kAcChunk;
  double* out = partial + ((size_t)s * nchunk + c) * (T + 1);
  if (bad[s]) {
    for (int t = threadIdx.x; t <= T; t += kThreads) out[t] = 0.0;
    return;
  }
  const int len = (int)std::min<int64_t>(kAcChunk + T, n - i0);
  const double mu = mean[s];
  for (int q = threadIdx.x; q < len; q += kThreads) d[q] = x[(size_t)s * ldx + series_at(index, n, s, i0 + q)] - mu;
  __syncthreads();
  const int iend = (int)std::min<int64_t>(kAcChunk, n - i0);
  for (int t = threadIdx.x; t <= T; t += kThreads) {
    // pairs (i, i + t) with i + t < n - i0
    const int lim = (int)std::min<int64_t>(iend, n - i0 - t);
    double acc = 0.0;
    for (int i = 0; i < lim; ++i) acc += d[i] * d[i + t];
    out[t] = acc;
  }
}

// Gamma(t) = (chunk partials summed in chunk order) / (n - t), then the
// Madras-Sokal window by one thread: tau = 1/2 + sum_{t=1}^{W} Gamma(t) / Gamma(0)
// for W = 1, 2, ... until W >= c tau.
__global__ void __launch_bounds__(kThreads) k_ac_final(int64_t n, int T, int nchunk, int w_max, double cwin,
                                                      const double* __restrict__ partial,
                                                      const int32_t* __restrict__ bad, double* __restrict__ gamma,
                                                      double* __restrict__ tau, int32_t* __restrict__ window,
                                                      uint8_t* __restrict__ found, double* __restrict__ n_indep) {
  extern __shared__ double g[];  // [T + 1]
  const int s = blockIdx.x;
  const bool isbad = bad[s] != 0;
  const double nan = __builtin_nan("");
  for (int t = threadIdx.x; t <= T; t += kThreads) {
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += partial[((size_t)s * nchunk + c) * (T + 1) + t];
    g[t] = isbad ? nan : acc / (double)(n - t);
  }
  __syncthreads();
  if (gamma)
    for (int t = threadIdx.x; t <= w_max; t += kThreads) gamma[(size_t)s * (w_max + 1) + t] = t <= T ? g[t] : nan;
  if (threadIdx.x != 0) return;
  double tv = nan, ni = 0.0;
  int W = 0;
  uint8_t fo = 0;
  if (isbad) {
    W = -1;
    ni = nan;
  } else if (g[0] != 0.0) {
    tv = 0.5;
    for (W = 1; W <= T; ++W) {
      tv += g[W] / g[0];
      if ((double)W >= cwin * tv) {
        fo = 1;
        break;
      }
    }
    if (!fo) W = T;
    ni = (double)n / (2.0 * tv);
  }
  tau[s] = tv;
  if (window) window[s] = W;
  if (found) found[s] = fo;
  if (n_indep) n_indep[s] = ni;
}

// Normalised ESS of series s: (sum e^{w - max})^2 / (n sum e^{2 (w - max)}).
__global__ void __launch_bounds__(kThreads) k_ess(int64_t n, const double* __restrict__ logw, int64_t ldw,
                                                 double* __restrict__ ess) {
  __shared__ double red[kWaves];
  const double* w = logw + (size_t)blockIdx.x * ldw;
  double mx = -HUGE_VAL;
  for (int64_t k = threadIdx.x; k < n; k += kThreads) mx = fmax(mx, w[k]);
  mx = block_max(mx, red);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kThreads) {
    const double e = exp(w[k] - mx);
    s1 += e;
    s2 += e * e;
  }
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) ess[blockIdx.x] = s1 * s1 / ((double)n * s2);
}

struct AcLayout {
  int T, nchunk;
  size_t off_bad, off_partial, total;
};

AcLayout ac_layout(int32_t n_series, int64_t n, int32_t w_max) {
  AcLayout a{};
  a.T = (int)std::min<int64_t>(w_max, n - 1);
  a.nchunk = (int)((n + kAcChunk - 1) / kAcChunk);
  const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  a.off_bad = up((size_t)n_series * sizeof(double));
  a.off_partial = a.off_bad + up((size_t)n_series * sizeof(int32_t));
  a.total = a.off_partial + up((size_t)n_series * a.nchunk * (a.T + 1) * sizeof(double));
  return a;
}

bool ac_args_ok(int32_t n_series, int64_t n, int32_t w_max) {
  return n_series >= 1 && n >= 1 && w_max >= 0;
}

}  // namespace
}  // namespace lfs

extern "C" int32_t lfs_observables(int32_t dim, int32_t L, int32_t B, const void* phi, int32_t fp64,
                                   double* M, double* C, void* stream) {
  LFS_RETURN_IF(dim != 2 && dim != 3, LFS_EINVAL);
  LFS_RETURN_IF(L < 2 || B < 0 || !phi || (!M && !C), LFS_EINVAL);
  LFS_RETURN_IF(L > 4096, LFS_EUNSUPPORTED);
  if (B == 0) return LFS_OK;
  const int slice = dim == 2 ? L : L * L;
  const size_t shm = (size_t)L * sizeof(double);
  const int vec = (slice * (fp64 ? 8 : 4)) % 16 == 0 && reinterpret_cast<uintptr_t>(phi) % 16 == 0;
  hipStream_t st = (hipStream_t)stream;
  if (fp64)
    hipLaunchKernelGGL(lfs::k_observables<double>, dim3(B), dim3(lfs::kThreads), shm, st, L, slice, vec,
                       (const double*)phi, M, C);
  else
    hipLaunchKernelGGL(lfs::k_observables<float>, dim3(B), dim3(lfs::kThreads), shm, st, L, slice, vec,
                       (const float*)phi, M, C);
  return lfs::launch_status();
}

extern "C" size_t lfs_autocorr_workspace_bytes(int32_t n_series, int64_t n, int32_t w_max) {
  if (!lfs::ac_args_ok(n_series, n, w_max)) return 0;
  return lfs::ac_layout(n_series, n, w_max).total;
}

extern "C" int32_t lfs_autocorr(int32_t n_series, int64_t n, const double* x, int64_t ldx,
                                const int64_t* index, int32_t w_max, double c, double* gamma,
                                double* tau, int32_t* window, uint8_t* found, double* n_indep,
                                void* ws, size_t ws_bytes, void* stream) {
  LFS_RETURN_IF(!lfs::ac_args_ok(n_series, n, w_max) || !x || !tau || !ws || !(c > 0.0), LFS_EINVAL);
  LFS_RETURN_IF(ldx < 1 || (!index && ldx < n), LFS_EINVAL);
  LFS_RETURN_IF(w_max > lfs::kAcMaxLag || n_series > 65535, LFS_EUNSUPPORTED);
  const lfs::AcLayout a = lfs::ac_layout(n_series, n, w_max);
  LFS_RETURN_IF(ws_bytes < a.total, LFS_EWORKSPACE);
  LFS_RETURN_IF(a.nchunk > (1 << 30), LFS_EUNSUPPORTED);
  char* base = static_cast<char*>(ws);
  double* mean = reinterpret_cast<double*>(base);
  int32_t* bad = reinterpret_cast<int32_t*>(base + a.off_bad);
  double* partial = reinterpret_cast<double*>(base + a.off_partial);
  const size_t shm_partial = (size_t)(lfs::kAcChunk + a.T) * sizeof(double);
  if (shm_partial > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(lfs::k_ac_partial),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_partial) != hipSuccess)
    return LFS_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(lfs::k_ac_mean, dim3(n_series), dim3(lfs::kThreads), 0, st, n, x, ldx, index, mean, bad);
  hipLaunchKernelGGL(lfs::k_ac_partial, dim3(a.nchunk, n_series), dim3(lfs::kThreads), shm_partial, st, n, a.T, x, ldx, index, mean, bad,
                     partial);
  hipLaunchKernelGGL(lfs::k_ac_final, dim3(n_series), dim3(lfs::kThreads), (size_t)(a.T + 1) * sizeof(double),
                     st, n, a.T, a.nchunk, w_max, c, partial, bad, gamma, tau, window, found, n_indep);
  return lfs::launch_status();
}

extern "C" int32_t lfs_ess(int32_t n_series, int64_t n, const double* logw, int64_t ldw, double* ess,
                           void* stream) {
  LFS_RETURN_IF(n_series < 1 || n < 1 || ldw < n || !logw || !ess, LFS_EINVAL);
  hipLaunchKernelGGL(lfs::k_ess, dim3(n_series), dim3(lfs::kThreads), 0, (hipStream_t)stream, n, logw, ldw,
                     ess);
  return lfs::launch_status();
}

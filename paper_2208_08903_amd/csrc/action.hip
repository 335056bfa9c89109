// Lattice phi^4 action and force (paper Sec. 1, action, Laplacian and
// potential equations), and the log-weights / reverse-KL loss.
#include "lfs_common.hpp"

namespace lfs {
namespace {

// Coordinate of site n along the axis with the given stride: shift and mask
// when L is a power of two (lg = log2 L), integer division otherwise (lg < 0).
__device__ __forceinline__ int coord(int n, int stride_lg, int stride, int L, int lg) {
  return lg >= 0 ? (n >> stride_lg) & (L - 1) : (n / stride) % L;
}

// Per-site action term (added to acc) and force of site value p with
// neighbour sum nb.
template <int DIM, typename R>
__device__ __forceinline__ float site_terms(R p, R nb, R m2, R lam, R scale, R& acc) {
  const R lap = nb - (R)(2 * DIM) * p;
  const R p2 = p * p;
  acc += -p * lap + m2 * p2 + lam * p2 * p2;
  return (float)(scale * ((R)-2 * lap + (R)2 * m2 * p + (R)4 * lam * p2 * p));
}

// One block per sample, four consecutive sites of a row per thread and step
// (L a multiple of 4, field and force 16-byte aligned): the field is staged in
// LDS (V <= 16384) with 16-byte loads; a quad reads its own 16 bytes, one
// value on each side along the fast axis and the 16-byte quads above and
// below along the others, so the coordinate arithmetic is paid once per four
// sites; the force leaves as one 16-byte store.  Neighbour sums are formed in
// the same order as the site-by-site kernel below, so the force is the same.
template <int DIM, typename R>
__global__ void __launch_bounds__(256) k_action_quad(int L, int lg, const float* __restrict__ phi,
                                                     const double* __restrict__ m2p,
                                                     const double* __restrict__ lamp, int per_sample,
                                                     double* __restrict__ S, float* __restrict__ force,
                                                     double force_scale) {
  extern __shared__ __align__(16) float f[];
  __shared__ R sh[16];
  const int b = blockIdx.x;
  int V = L;
  for (int i = 1; i < DIM; ++i) V *= L;
  const float4* pb = reinterpret_cast<const float4*>(phi + (size_t)b * V);
  float4* f4 = reinterpret_cast<float4*>(f);
  for (int q = threadIdx.x; q < V / 4; q += blockDim.x) f4[q] = pb[q];
  __syncthreads();
  const R m2 = (R)m2p[per_sample ? b : 0], lam = (R)lamp[per_sample ? b : 0];
  const R scale = (R)force_scale;
  float4* fb = force ? reinterpret_cast<float4*>(force + (size_t)b * V) : nullptr;
  R acc = 0;
  for (int q = threadIdx.x; q < V / 4; q += blockDim.x) {
    const int n = 4 * q;
    const int x0 = coord(n, 0, 1, L, lg);
    const int rs = n - x0;
    const float4 c = f4[q];
    const float xl = f[rs + (x0 == 0 ? L - 1 : x0 - 1)];
    const float xr = f[rs + (x0 + 4 == L ? 0 : x0 + 4)];
    // fast axis first (up + down), as in the site-by-site kernel
    R nb0 = (R)c.y + (R)xl, nb1 = (R)c.z + (R)c.x, nb2 = (R)c.w + (R)c.y, nb3 = (R)xr + (R)c.z;
    int stride = L, stride_lg = lg;
#pragma unroll
    for (int mu = DIM - 2; mu >= 0; --mu) {
      const int cm = coord(n, stride_lg, stride, L, lg);
      const int up = (cm == L - 1) ? n - (L - 1) * stride : n + stride;
      const int dn = (cm == 0) ? n + (L - 1) * stride : n - stride;
      const float4 u = f4[up >> 2], d = f4[dn >> 2];
      nb0 += (R)u.x + (R)d.x;
      nb1 += (R)u.y + (R)d.y;
      nb2 += (R)u.z + (R)d.z;
      nb3 += (R)u.w + (R)d.w;
      stride *= L;
      stride_lg += lg;
    }
    float4 o;
    o.x = site_terms<DIM, R>((R)c.x, nb0, m2, lam, scale, acc);
    o.y = site_terms<DIM, R>((R)c.y, nb1, m2, lam, scale, acc);
    o.z = site_terms<DIM, R>((R)c.z, nb2, m2, lam, scale, acc);
    o.w = site_terms<DIM, R>((R)c.w, nb3, m2, lam, scale, acc);
    if (fb) fb[q] = o;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) S[b] = (double)acc;
}

// One block per sample; the sample's field is staged in LDS (V <= 16384) with
// 16-byte loads when every sample starts 16-byte aligned (vec).
template <int DIM, typename R>
__global__ void __launch_bounds__(256) k_action(int L, int lg, int vec, const float* __restrict__ phi,
                                                const double* __restrict__ m2p,
                                                const double* __restrict__ lamp, int per_sample,
                                                double* __restrict__ S, float* __restrict__ force,
                                                double force_scale) {
  extern __shared__ __align__(16) float f[];
  __shared__ R sh[16];
  const int b = blockIdx.x;
  int V = L;
  for (int i = 1; i < DIM; ++i) V *= L;
  const float* pb = phi + (size_t)b * V;
  if (vec) {
    for (int q = threadIdx.x; q < V / 4; q += blockDim.x)
      reinterpret_cast<float4*>(f)[q] = reinterpret_cast<const float4*>(pb)[q];
  } else {
    for (int n = threadIdx.x; n < V; n += blockDim.x) f[n] = pb[n];
  }
  __syncthreads();
  const R m2 = (R)m2p[per_sample ? b : 0], lam = (R)lamp[per_sample ? b : 0];
  const R scale = (R)force_scale;
  R acc = 0;
  // Plus-direction neighbours are taps with exactly one +1 offset.
  for (int n = threadIdx.x; n < V; n += blockDim.x) {
    const R p = (R)f[n];
    R nb = 0;
    int stride = 1, stride_lg = 0;
#pragma unroll
    for (int mu = DIM - 1; mu >= 0; --mu) {
      const int c = coord(n, stride_lg, stride, L, lg);
      const int up = (c == L - 1) ? n - (L - 1) * stride : n + stride;
      const int dn = (c == 0) ? n + (L - 1) * stride : n - stride;
      nb += (R)f[up] + (R)f[dn];
      stride *= L;
      stride_lg += lg;
    }
    const float fo = site_terms<DIM, R>(p, nb, m2, lam, scale, acc);
    if (force) force[(size_t)b * V + n] = fo;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) S[b] = (double)acc;
}

// logw = -S - logq per sample; loss = mean(logq + S) in a fixed order (one block).
__global__ void __launch_bounds__(256) k_log_weights(int B, const double* __restrict__ S,
                                                     const double* __restrict__ logq,
                                                     double* __restrict__ logw,
                                                     double* __restrict__ loss) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    const double w = -S[b] - logq[b];
    logw[b] = w;
    acc += logq[b] + S[b];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0 && loss) *loss = acc / (double)B;
}

}  // namespace
}  // namespace lfs

extern "C" int32_t lfs_action(int32_t dim, int32_t L, int32_t B, const float* phi, const double* m2,
                              const double* lam, int32_t per_sample, int32_t precision, double* S,
                              float* force, double force_scale, void* stream) {
  LFS_RETURN_IF(dim != 2 && dim != 3, LFS_EINVAL);
  LFS_RETURN_IF(L < 2 || B < 0, LFS_EINVAL);
  LFS_RETURN_IF(precision != LFS_PLAIN_FP32 && precision != LFS_BF16_CONV, LFS_EINVAL);
  const long V = dim == 2 ? (long)L * L : (long)L * L * L;
  LFS_RETURN_IF(V > 16384, LFS_EUNSUPPORTED);
  if (B == 0) return LFS_OK;
  LFS_RETURN_IF(!phi || !m2 || !lam || !S, LFS_EINVAL);
  const size_t shm = (size_t)V * sizeof(float);
  hipStream_t st = (hipStream_t)stream;
  const bool f64 = precision == LFS_BF16_CONV;
  const int lg = (L & (L - 1)) == 0 ? __builtin_ctz((unsigned)L) : -1;
  const int vec = (V % 4 == 0) && (reinterpret_cast<uintptr_t>(phi) % 16 == 0);
  const bool quad = vec && L % 4 == 0 && (!force || reinterpret_cast<uintptr_t>(force) % 16 == 0);
  if (quad) {
    if (dim == 2) {
      if (f64)
        hipLaunchKernelGGL((lfs::k_action_quad<2, double>), dim3(B), dim3(256), shm, st, L, lg, phi, m2,
                           lam, per_sample, S, force, force_scale);
      else
        hipLaunchKernelGGL((lfs::k_action_quad<2, float>), dim3(B), dim3(256), shm, st, L, lg, phi, m2,
                           lam, per_sample, S, force, force_scale);
    } else {
      if (f64)
        hipLaunchKernelGGL((lfs::k_action_quad<3, double>), dim3(B), dim3(256), shm, st, L, lg, phi, m2,
                           lam, per_sample, S, force, force_scale);
      else
        hipLaunchKernelGGL((lfs::k_action_quad<3, float>), dim3(B), dim3(256), shm, st, L, lg, phi, m2,
                           lam, per_sample, S, force, force_scale);
    }
    return lfs::launch_status();
  }
  if (dim == 2) {
    if (f64)
      hipLaunchKernelGGL((lfs::k_action<2, double>), dim3(B), dim3(256), shm, st, L, lg, vec, phi, m2, lam,
                         per_sample, S, force, force_scale);
    else
      hipLaunchKernelGGL((lfs::k_action<2, float>), dim3(B), dim3(256), shm, st, L, lg, vec, phi, m2, lam,
                         per_sample, S, force, force_scale);
  } else {
    if (f64)
      hipLaunchKernelGGL((lfs::k_action<3, double>), dim3(B), dim3(256), shm, st, L, lg, vec, phi, m2, lam,
                         per_sample, S, force, force_scale);
    else
      hipLaunchKernelGGL((lfs::k_action<3, float>), dim3(B), dim3(256), shm, st, L, lg, vec, phi, m2, lam,
                         per_sample, S, force, force_scale);
  }
  return lfs::launch_status();
}

extern "C" int32_t lfs_log_weights(int32_t B, const double* S, const double* logq, double* logw,
                                   double* loss, void* stream) {
  LFS_RETURN_IF(B <= 0 || !S || !logq || !logw, LFS_EINVAL);
  hipLaunchKernelGGL(lfs::k_log_weights, dim3(1), dim3(256), 0, (hipStream_t)stream, B, S, logq,
                     logw, loss);
  return lfs::launch_status();
}

// Independence Metropolis-Hastings chains (paper Sec. 1, the MH test that
// corrects flow proposals to exp(-S)/Z) and the FP64 HMC baseline (paper
// Sec. 2.2, HMC for the same theory, "to compare results").
#include "lfs_common.hpp"

namespace lfs {
namespace {

// One 64-lane block per chain.  Chunks of 64 proposals are staged through LDS
// with coalesced loads; lane 0 makes the sequential decisions.
// Chain c reads proposals [offsets[c], offsets[c+1]) (rectangular calls pass
// offsets == NULL and use [c * n_prop, (c+1) * n_prop)); its state lives at
// state[state_index[c]] (or state[c]).
__global__ void __launch_bounds__(64) k_mh_chain(int n_prop_rect, const int64_t* __restrict__ offsets,
                                                 const double* __restrict__ logw,
                                                 const double* __restrict__ log_u,
                                                 lfs_chain_state* __restrict__ states,
                                                 const int32_t* __restrict__ state_index,
                                                 int64_t* __restrict__ cur_idx,
                                                 uint8_t* __restrict__ accepted) {
  __shared__ double sw[kWave], su[kWave];
  __shared__ int64_t sidx[kWave];
  __shared__ uint8_t sacc[kWave];
  const int c = blockIdx.x, lane = threadIdx.x;
  const size_t base = offsets ? (size_t)offsets[c] : (size_t)c * n_prop_rect;
  const int n_prop = offsets ? (int)(offsets[c + 1] - offsets[c]) : n_prop_rect;
  lfs_chain_state* state = states + (state_index ? state_index[c] : c);
  lfs_chain_state st = *state;
  const int64_t seen0 = st.n_seen;
  for (int k0 = 0; k0 < n_prop; k0 += kWave) {
    const int k = k0 + lane;
    if (k < n_prop) {
      sw[lane] = logw[base + k];
      su[lane] = log_u[base + k];
    }
    __syncthreads();
    if (lane == 0) {
      const int m = min(kWave, n_prop - k0);
      for (int i = 0; i < m; ++i) {
        const int64_t g = seen0 + k0 + i;
        uint8_t a = 0;
        if (!st.has_state) {
          st.has_state = 1;
          st.w_cur = sw[i];
          st.idx_cur = g;
          a = 1;
        } else {
          const double d = sw[i] - st.w_cur;  // one rounded FP64 subtraction
          if (su[i] < d) {
            st.w_cur = sw[i];
            st.idx_cur = g;
            st.n_acc += 1;
            a = 1;
          }
        }
        sidx[i] = st.idx_cur;
        sacc[i] = a;
      }
    }
    __syncthreads();
    if (k < n_prop) {
      cur_idx[base + k] = sidx[lane];
      if (accepted) accepted[base + k] = sacc[lane];
    }
    __syncthreads();
  }
  if (lane == 0) {
    st.n_seen = seen0 + n_prop;
    *state = st;
  }
}

// Per-site action density and force from an LDS-resident FP64 field.  L is the
// compile-time LT where LT > 0 (a power of two: the coordinate arithmetic is shifts
// and masks), else the runtime value.
template <int DIM, int LT>
__device__ __forceinline__ void site_terms(const double* f, int n, int Lrt, double m2, double lam,
                                           double& dens, double& frc) {
  const int L = LT > 0 ? LT : Lrt;
  const double p = f[n];
  double nb = 0.0;
  int stride = 1;
#pragma unroll
  for (int mu = DIM - 1; mu >= 0; --mu) {
    const int c = (n / stride) % L;
    const int up = (c == L - 1) ? n - (L - 1) * stride : n + stride;
    const int dn = (c == 0) ? n + (L - 1) * stride : n - stride;
    nb += f[up] + f[dn];
    stride *= L;
  }
  const double lap = nb - 2.0 * DIM * p;
  const double p2 = p * p;
  dens = -p * lap + m2 * p2 + lam * p2 * p2;
  frc = -2.0 * lap + 2.0 * m2 * p + 4.0 * lam * p2 * p;
}

// One block per chain; phi, pi and the force stay in LDS for the whole
// trajectory.  Kick-drift-kick: the closing half-kick of a step and the opening
// half-kick of the next use the force at the same field, so it is evaluated
// once per step (and once at the start); both half-kicks are still applied as
// two separate subtractions, as the definition has them.  The last force pass
// also sums the final Hamiltonian.  Every thread owns sites tid, tid + blockDim, ...
// in every pass, so its kicks read only its own force entries.
template <int DIM, int LT>
__global__ void __launch_bounds__(256) k_hmc(int Lrt, double* __restrict__ phi,
                                             const double* __restrict__ pi0,
                                             const double* __restrict__ log_u,
                                             const double* __restrict__ m2p,
                                             const double* __restrict__ lamp, int per_sample,
                                             int n_steps, double dt, double* __restrict__ dH,
                                             uint8_t* __restrict__ accepted) {
  extern __shared__ double smem[];
  __shared__ double sh[16];
  const int L = LT > 0 ? LT : Lrt;
  int V = L;
  for (int i = 1; i < DIM; ++i) V *= L;
  double* f = smem;
  double* p = smem + V;
  double* F = smem + 2 * V;
  const int b = blockIdx.x;
  const double m2 = m2p[per_sample ? b : 0], lam = lamp[per_sample ? b : 0];
  for (int n = threadIdx.x; n < V; n += blockDim.x) {
    f[n] = phi[(size_t)b * V + n];
    p[n] = pi0[(size_t)b * V + n];
  }
  __syncthreads();
  double h = 0.0, dens, frc;
  for (int n = threadIdx.x; n < V; n += blockDim.x) {
    site_terms<DIM, LT>(f, n, L, m2, lam, dens, frc);
    F[n] = frc;
    h += 0.5 * p[n] * p[n] + dens;
  }
  const double H0 = block_sum(h, sh);  // ends with a barrier
  const double hdt = 0.5 * dt;
  h = 0.0;
  for (int s = 0; s < n_steps; ++s) {
    for (int n = threadIdx.x; n < V; n += blockDim.x) {
      p[n] = p[n] - hdt * F[n];
      f[n] = f[n] + dt * p[n];
    }
    __syncthreads();
    const bool last = s == n_steps - 1;
    for (int n = threadIdx.x; n < V; n += blockDim.x) {
      site_terms<DIM, LT>(f, n, L, m2, lam, dens, frc);
      F[n] = frc;
      p[n] = p[n] - hdt * frc;
      if (last) h += 0.5 * p[n] * p[n] + dens;
    }
    __syncthreads();  // the next drift rewrites f, which this pass read at neighbours
  }
  const double H1 = n_steps > 0 ? block_sum(h, sh) : H0;
  const double d = H1 - H0;
  const bool acc = log_u[b] < -d;
  if (acc)
    for (int n = threadIdx.x; n < V; n += blockDim.x) phi[(size_t)b * V + n] = f[n];
  if (threadIdx.x == 0) {
    dH[b] = d;
    accepted[b] = acc ? 1 : 0;
  }
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float inv_bc1, float inv_bc2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi * inv_bc1) / (sqrtf(vi * inv_bc2) + eps);
  }
}

}  // namespace
}  // namespace lfs

extern "C" int32_t lfs_mh_chain(int32_t n_chains, int32_t n_prop, const double* logw,
                                const double* log_u, lfs_chain_state* state, int64_t* cur_idx,
                                uint8_t* accepted, void* stream) {
  LFS_RETURN_IF(n_chains < 0 || n_prop < 0, LFS_EINVAL);
  if (n_chains == 0 || n_prop == 0) return LFS_OK;
  LFS_RETURN_IF(!logw || !log_u || !state || !cur_idx, LFS_EINVAL);
  hipLaunchKernelGGL(lfs::k_mh_chain, dim3(n_chains), dim3(lfs::kWave), 0, (hipStream_t)stream,
                     n_prop, nullptr, logw, log_u, state, nullptr, cur_idx, accepted);
  return lfs::launch_status();
}

extern "C" int32_t lfs_mh_chain_ragged(int32_t n_chains, const int64_t* offsets, const double* logw,
                                       const double* log_u, lfs_chain_state* states,
                                       const int32_t* state_index, int64_t* cur_idx,
                                       uint8_t* accepted, void* stream) {
  LFS_RETURN_IF(n_chains < 0, LFS_EINVAL);
  if (n_chains == 0) return LFS_OK;
  LFS_RETURN_IF(!offsets || !logw || !log_u || !states || !state_index || !cur_idx, LFS_EINVAL);
  hipLaunchKernelGGL(lfs::k_mh_chain, dim3(n_chains), dim3(lfs::kWave), 0, (hipStream_t)stream, 0,
                     offsets, logw, log_u, states, state_index, cur_idx, accepted);
  return lfs::launch_status();
}

extern "C" int32_t lfs_hmc_step(int32_t dim, int32_t L, int32_t B, double* phi, const double* pi0,
                                const double* log_u, const double* m2, const double* lam,
                                int32_t per_sample, int32_t n_steps, double dt, double* dH,
                                uint8_t* accepted, void* stream) {
  LFS_RETURN_IF(dim != 2 && dim != 3, LFS_EINVAL);
  LFS_RETURN_IF(L < 2 || B < 0 || n_steps < 0, LFS_EINVAL);
  const long V = dim == 2 ? (long)L * L : (long)L * L * L;
  LFS_RETURN_IF(V > 4096, LFS_EUNSUPPORTED);  // phi, pi and the force in at most 96 KB of LDS
  if (B == 0) return LFS_OK;
  LFS_RETURN_IF(!phi || !pi0 || !log_u || !m2 || !lam || !dH || !accepted, LFS_EINVAL);
  const size_t shm = 3 * (size_t)V * sizeof(double);
  hipStream_t st = (hipStream_t)stream;
  // compile-time lattice sizes for the common powers of two, the runtime L otherwise
  using Kern = void (*)(int, double*, const double*, const double*, const double*, const double*, int, int,
                        double, double*, uint8_t*);
  const int li = L == 4 ? 1 : L == 8 ? 2 : L == 16 ? 3 : 0;
  static const Kern k2[4] = {lfs::k_hmc<2, 0>, lfs::k_hmc<2, 4>, lfs::k_hmc<2, 8>, lfs::k_hmc<2, 16>};
  static const Kern k3[4] = {lfs::k_hmc<3, 0>, lfs::k_hmc<3, 4>, lfs::k_hmc<3, 8>, lfs::k_hmc<3, 16>};
  const Kern k = dim == 2 ? k2[li] : k3[li];
  if (shm > 64 * 1024)
    LFS_RETURN_IF(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)shm) != hipSuccess,
                  LFS_EDEVICE);
  hipLaunchKernelGGL(k, dim3(B), dim3(256), shm, st, L, phi, pi0, log_u, m2, lam, per_sample, n_steps, dt, dH,
                     accepted);
  return lfs::launch_status();
}

extern "C" int32_t lfs_adam_step(int64_t n, float* p, const float* g, float* m, float* v, float lr,
                                 float b1, float b2, float eps, int64_t t, void* stream) {
  LFS_RETURN_IF(n <= 0 || t < 1 || !p || !g || !m || !v, LFS_EINVAL);
  const double bc1 = 1.0 - pow((double)b1, (double)t), bc2 = 1.0 - pow((double)b2, (double)t);
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(lfs::k_adam, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, n, p,
                     g, m, v, lr, b1, b2, eps, (float)(1.0 / bc1), (float)(1.0 / bc2));
  return lfs::launch_status();
}

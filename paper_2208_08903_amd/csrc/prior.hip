// Prior draw: Philox4x32-10 counter-based generator (Salmon et al., SC'11) and
// the Box-Muller transform, one FP32 standard normal per site (paper Sec. 1,
// point-wise independent prior; example parameter file Normal{Float32}(0,1)).
#include "lfs_common.hpp"

namespace lfs {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kWeyl0;
      k1 += kWeyl1;
    }
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c[0];
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// u = (floor(x / 2^9) + 1/2) 2^-23: exact in FP32, strictly inside (0, 1).
__device__ __forceinline__ float word_to_unit(uint32_t x) {
  return ((float)(x >> 9) + 0.5f) * 0x1p-23f;
}

// One block per sample; each thread produces 4 sites per Philox call.  The
// sample's key and counter come from (key, counter0 + b) or, if keys != NULL,
// from keys[b] and counters[b].
__global__ void __launch_bounds__(256) k_prior(uint32_t key0_, uint32_t key1_, uint64_t counter0,
                                               const uint64_t* __restrict__ keys,
                                               const uint64_t* __restrict__ counters, int V,
                                               float* __restrict__ z, double* __restrict__ logr) {
  __shared__ double sh[16];
  const int b = blockIdx.x;
  const uint64_t cb = keys ? counters[b] : counter0 + (uint64_t)b;
  const uint32_t key0 = keys ? (uint32_t)keys[b] : key0_;
  const uint32_t key1 = keys ? (uint32_t)(keys[b] >> 32) : key1_;
  float4* zb = reinterpret_cast<float4*>(z + (size_t)b * V);
  double acc = 0.0;
  for (int j = threadIdx.x; j < V / 4; j += blockDim.x) {
    uint32_t c[4] = {(uint32_t)j, (uint32_t)cb, (uint32_t)(cb >> 32), 0u};
    philox4x32_10(c, key0, key1);
    float4 out;
    float s, co;
    float r = sqrtf(-2.f * logf(word_to_unit(c[0])));
    sincospif(2.f * word_to_unit(c[1]), &s, &co);
    out.x = r * co;
    out.y = r * s;
    r = sqrtf(-2.f * logf(word_to_unit(c[2])));
    sincospif(2.f * word_to_unit(c[3]), &s, &co);
    out.z = r * co;
    out.w = r * s;
    zb[j] = out;
    acc += (double)out.x * out.x + (double)out.y * out.y + (double)out.z * out.z +
           (double)out.w * out.w;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0 && logr) logr[b] = -0.5 * acc - 0.5 * (double)V * 1.8378770664093454836;
}

}  // namespace
}  // namespace lfs

extern "C" int32_t lfs_prior_normal(uint64_t key, uint64_t counter0, int32_t B, int32_t V, float* z,
                                    double* logr, void* stream) {
  LFS_RETURN_IF(B < 0 || V <= 0 || (V % 4) != 0, LFS_EINVAL);
  if (B == 0) return LFS_OK;
  LFS_RETURN_IF(z == nullptr || ((uintptr_t)z & 15u) != 0, LFS_EINVAL);  // float4 stores
  hipLaunchKernelGGL(lfs::k_prior, dim3(B), dim3(256), 0, (hipStream_t)stream, (uint32_t)key,
                     (uint32_t)(key >> 32), counter0, nullptr, nullptr, V, z, logr);
  return lfs::launch_status();
}

extern "C" int32_t lfs_prior_normal_streams(int32_t B, int32_t V, const uint64_t* keys,
                                            const uint64_t* counters, float* z, double* logr,
                                            void* stream) {
  LFS_RETURN_IF(B < 0 || V <= 0 || (V % 4) != 0, LFS_EINVAL);
  if (B == 0) return LFS_OK;
  LFS_RETURN_IF(!z || !keys || !counters || ((uintptr_t)z & 15u) != 0, LFS_EINVAL);
  hipLaunchKernelGGL(lfs::k_prior, dim3(B), dim3(256), 0, (hipStream_t)stream, 0u, 0u, 0ull, keys,
                     counters, V, z, logr);
  return lfs::launch_status();
}

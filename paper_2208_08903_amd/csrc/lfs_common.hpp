// Device and host helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "lfs.h"

#define LFS_RETURN_IF(cond, code) \
  do {                            \
    if (cond) return (code);      \
  } while (0)

namespace lfs {

constexpr float kLeakySlope = 0.01f;
constexpr int kWave = 64;

inline int32_t launch_status() {
  return hipGetLastError() == hipSuccess ? LFS_OK : LFS_EDEVICE;
}

// Host-side facts cached per device (ordinals below kCachedDevices; others are
// looked up on every call).  Safe to call from several host threads.
constexpr int kCachedDevices = 64;

// Raises kernel KERN's dynamic LDS limit to `bytes` on the current device, once
// per device.
template <auto KERN>
inline bool set_lds_limit(size_t bytes) {
  static std::atomic<uint64_t> done{0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  const uint64_t bit = (dev >= 0 && dev < kCachedDevices) ? (1ull << dev) : 0;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return true;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(KERN), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes) != hipSuccess)
    return false;
  if (bit) done.fetch_or(bit, std::memory_order_acq_rel);
  return true;
}

// Compute units of the current device (256 if the query fails).
inline int num_cus() {
  static std::atomic<int> cache[kCachedDevices];
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  const bool cached = dev >= 0 && dev < kCachedDevices;
  if (cached && (n = cache[dev].load(std::memory_order_relaxed)) > 0) return n;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
  if (cached) cache[dev].store(n, std::memory_order_relaxed);
  return n;
}

inline int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Round an FP32 value to the nearest BF16 (ties to even) and widen it back.
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

template <bool BF16>
__device__ __forceinline__ float opnd(float x) {
  if constexpr (BF16) return bf16_round(x);
  return x;
}

// LeakyReLU with slope in (0, 1): max(a, slope * a).  One v_max_f32: fmaxf
// would first canonicalise an operand the compiler cannot prove canonical
// (an MFMA result), a third instruction for nothing, as a is never a
// signalling NaN here.
__device__ __forceinline__ float leaky(float a) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(kLeakySlope * a));
  return r;
}
// LeakyReLU'(a) from its output h = leaky(a): sign(h) == sign(a), h == 0 iff a == 0.
__device__ __forceinline__ float leaky_grad_from_out(float h) { return h >= 0.f ? 1.f : kLeakySlope; }

// Sum over the 64 lanes of a wavefront, fixed butterfly order (deterministic).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over a block (blockDim.x a multiple of 64, at most 1024).  `sh` holds 16 T.
// Waves are combined in index order by thread 0, so the result is deterministic.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T r = sh[0];
    for (int i = 1; i < nw; ++i) r += sh[i];
    sh[0] = r;
  }
  __syncthreads();
  T r = sh[0];
  __syncthreads();
  return r;
}

// Lattice helpers.  Sites are row-major with axis 0 slowest; taps are row-major
// over delta in {-1,0,1}^DIM with axis 0 slowest.
template <int DIM>
__device__ __forceinline__ int site_parity(int n, int L) {
  int p = 0;
#pragma unroll
  for (int mu = 0; mu < DIM; ++mu) {
    p += n % L;
    n /= L;
  }
  return p & 1;
}

__device__ __forceinline__ int wrap(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// Site n + delta_t (sign = +1) or n - delta_t (sign = -1), periodic.
template <int DIM>
__device__ __forceinline__ int neighbor(int n, int t, int L, int sign = 1) {
  int coord[DIM];
#pragma unroll
  for (int mu = DIM - 1; mu >= 0; --mu) {
    coord[mu] = n % L;
    n /= L;
  }
  int r = 0;
#pragma unroll
  for (int mu = 0; mu < DIM; ++mu) {
    int div = 1;
#pragma unroll
    for (int k = mu + 1; k < DIM; ++k) div *= 3;
    const int d = ((t / div) % 3) - 1;
    r = r * L + wrap(coord[mu] + sign * d, L);
  }
  return r;
}

}  // namespace lfs

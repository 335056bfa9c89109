// Shared pieces of the fused (LDS-resident, matrix-core) flow kernels:
// compile-time lattice geometry, MFMA operand types and the weight-fragment
// layout.
//
// Every convolution is an implicit GEMM  D^T[c_out][site] = sum_k A[c_out][k] B[k][site]
// with k = (tap, c_in), c_in fastest, tap-major.  A holds the weights
// (prepared once per call into "fragment order" so that each lane loads its
// operand with one 16-byte read), B is gathered from the LDS-resident
// activations of the sample at the periodic neighbours of the tile's sites.
//
// Lane layout of the 16x16 MFMA tiles (wave64, lane l, j = l / 16, m = l % 16):
//   A: lane holds A[m][k] for its K slice, B: lane holds B[k][m] for the same
//   K slice, D: lane holds D[4 j + i][m], i = 0..3.
//   BF16 (v_mfma_f32_16x16x32_bf16): K slice of a lane = k in [8 j, 8 j + 8)
//     of a 32-wide chunk: 8 consecutive input channels of one tap.
//   FP32 (v_mfma_f32_16x16x4_f32, 4 k per instruction, one per lane group):
//     four consecutive instructions r = 0..3 form a 16-wide block in which lane
//     group j holds k = 4 j + r, so a lane's four operands are 4 consecutive
//     input channels of one tap and arrive with one 16-byte read.
#pragma once

#include "lfs_common.hpp"

namespace lfs {
namespace fused {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(float a, float b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// FP32 -> BF16 bits, round to nearest even (same rounding as bf16_round).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return bf16_bits(lo) | (bf16_bits(hi) << 16);
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ bf16x8 as_bf16x8(const u32x4& v) { return __builtin_bit_cast(bf16x8, v); }

// Compile-time lattice: V sites, T taps, row-major, axis 0 slowest.
template <int DIM, int L>
struct Geo {
  static constexpr int V = DIM == 2 ? L * L : L * L * L;
  static constexpr int T = DIM == 2 ? 9 : 27;
  static constexpr int HALF = V / 2;

  __device__ static __forceinline__ int wrapc(int c) { return c < 0 ? c + L : (c >= L ? c - L : c); }

  // Offset component of tap t along axis mu (-1, 0, +1).
  __device__ static __forceinline__ int tap_d(int t, int mu) {
    if constexpr (DIM == 2) return (mu == 0 ? t / 3 : t % 3) - 1;
    return (mu == 0 ? t / 9 : (mu == 1 ? (t / 3) % 3 : t % 3)) - 1;
  }

  // Site n + sign * delta_t, periodic.
  __device__ static __forceinline__ int nbr(int n, int t, int sign = 1) {
    if constexpr (DIM == 2) {
      const int y = n / L, x = n - (n / L) * L;
      return wrapc(y + sign * tap_d(t, 0)) * L + wrapc(x + sign * tap_d(t, 1));
    } else {
      const int z = n / (L * L), y = (n / L) % L, x = n % L;
      return (wrapc(z + sign * tap_d(t, 0)) * L + wrapc(y + sign * tap_d(t, 1))) * L +
             wrapc(x + sign * tap_d(t, 2));
    }
  }

  __device__ static __forceinline__ int parity(int n) {
    if constexpr (DIM == 2) return (n / L + n % L) & 1;
    return (n / (L * L) + (n / L) % L + n % L) & 1;
  }

  // The a-th site (row-major order) among the V/2 sites of parity `par`.
  __device__ static __forceinline__ int half_site(int a, int par) {
    const int row = a / (L / 2), i = a - row * (L / 2);
    const int lead = DIM == 2 ? row : row / L + row % L;
    return row * L + 2 * i + ((par + lead) & 1);
  }
};

// Number of 32-wide BF16 K chunks / 16-wide FP32 K blocks of a convolution
// with K = taps * cin.
__host__ __device__ constexpr int kchunks_bf16(int K) { return (K + 31) / 32; }
__host__ __device__ constexpr int kblocks_f32(int K) { return (K + 15) / 16; }

// Fragment bookkeeping for one layer (counts of 1 KB fragments = 64 lanes x 16 B).
struct LayerFrags {
  int nct;           // output-channel tiles of conv1/conv2 (16 rows each)
  int k1, k2;        // K chunks (BF16) or blocks (FP32) of conv1 and of conv2/conv3
  int off1, off2, off3, total;  // fragment offsets within the layer
};

__host__ __device__ constexpr LayerFrags layer_frags(int T, int C, bool bf16) {
  LayerFrags f{};
  f.nct = C >= 16 ? C / 16 : 1;
  f.k1 = bf16 ? kchunks_bf16(T) : kblocks_f32(T);
  f.k2 = bf16 ? kchunks_bf16(T * C) : kblocks_f32(T * C);
  f.off1 = 0;
  f.off2 = f.nct * f.k1;
  f.off3 = f.off2 + f.nct * f.k2;
  f.total = f.off3 + f.k2;
  return f;
}

}  // namespace fused
}  // namespace lfs

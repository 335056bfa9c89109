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
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(float a, float b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even (v_cvt_pk_bf16_f32; same rounding as bf16_round).
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const bf16x2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ uint32_t bf16_bits(float x) { return pack_bf16(x, 0.f) & 0xFFFFu; }
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ bf16x8 as_bf16x8(const u32x4& v) { return __builtin_bit_cast(bf16x8, v); }

// e^x from the hardware base-2 exponential (v_exp_f32): e^x = 2^(x log2 e).
__device__ __forceinline__ float fast_exp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}
// tanh(x) = 1 - 2 / (e^{2x} + 1) with v_exp_f32 and v_rcp_f32 (saturates to +-1).
__device__ __forceinline__ float fast_tanh(float x) {
  return 1.f - 2.f * __builtin_amdgcn_rcpf(fast_exp(2.f * x) + 1.f);
}

// Wave index as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Compile-time lattice: V sites, T taps, row-major, axis 0 slowest.
template <int DIM, int L>
struct Geo {
  static constexpr int Dim = DIM;
  static constexpr int V = DIM == 2 ? L * L : L * L * L;
  static constexpr int T = DIM == 2 ? 9 : 27;
  static constexpr int HALF = V / 2;

  __device__ static __forceinline__ int wrapc(int c) { return c < 0 ? c + L : (c >= L ? c - L : c); }

  // Offset component of tap t along axis mu (-1, 0, +1).
  __device__ static __forceinline__ int tap_d(int t, int mu) {
    if constexpr (DIM == 2) return (mu == 0 ? t / 3 : t % 3) - 1;
    return (mu == 0 ? t / 9 : (mu == 1 ? (t / 3) % 3 : t % 3)) - 1;
  }

  // Site n + sign * delta_t, periodic (power-of-two L: coordinates by shift and
  // mask, the wrap by a mask, which also holds for the -1 offset).
  __device__ static __forceinline__ int nbr(int n, int t, int sign = 1) {
    if constexpr ((L & (L - 1)) == 0) {
      constexpr int LG = L <= 1 ? 0 : 31 - __builtin_clz(L), MK = L - 1;
      if constexpr (DIM == 2) {
        const int y = n >> LG, x = n & MK;
        return (((y + sign * tap_d(t, 0)) & MK) << LG) | ((x + sign * tap_d(t, 1)) & MK);
      } else {
        const int z = n >> (2 * LG), y = (n >> LG) & MK, x = n & MK;
        return (((((z + sign * tap_d(t, 0)) & MK) << LG) | ((y + sign * tap_d(t, 1)) & MK)) << LG) |
               ((x + sign * tap_d(t, 2)) & MK);
      }
    } else if constexpr (DIM == 2) {
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

// Storage of a site-major lattice tensor in LDS.  PAD: a one-site periodic halo
// on every side, so the neighbour of a site is its storage index plus a
// constant per tap, and producers also write the halo copies of boundary sites.
// Without PAD the storage index is the site index and neighbours come from
// periodic wrap arithmetic (for shapes whose padded lattice does not fit LDS).
// QM (FP32, unpadded): channels stored quad-major, [C / 4][site][4] with the quad
// planes QSZ elements apart (QSZ * 4 bytes = 64 mod 256), instead of site-major
// [site][C].  Sixteen lanes reading the same channel quad of sixteen consecutive
// sites then touch 256 contiguous bytes (site-major: 64 bytes apart, four lanes per
// bank group), and sixteen lanes reading the sixteen channels of one site still hit
// sixteen different banks.
template <int DIM, int L, bool PAD, bool QM = false>
struct Lay {
  using G = Geo<DIM, L>;
  static constexpr bool padded = PAD;
  static constexpr bool quad_major = QM;
  static constexpr int Ls = L;
  static constexpr int LP = PAD ? L + 2 : L;
  static constexpr int VS = DIM == 2 ? LP * LP : LP * LP * LP;  // storage sites
  // One extra all-zero site after the lattice: gathers of taps beyond the
  // convolution's K read it instead of branching.
  static constexpr int ZS = VS;
  static constexpr int VSZ = VS + 1;  // sites to allocate
  // quad-plane stride (QM, 4-byte elements): at least 4 VSZ, and 16 mod 64
  static constexpr int QSZ = (4 * VSZ + 47) / 64 * 64 + 16;
  // element offset of channel ch of storage site p in a tensor of C channels
  template <int C>
  __host__ __device__ static constexpr int off(int p, int ch) {
    if constexpr (QM)
      return (ch >> 2) * QSZ + p * 4 + (ch & 3);
    else
      return p * C + ch;
  }
  // elements to allocate for a tensor of C channels
  template <int C>
  __host__ __device__ static constexpr int elems() {
    return QM ? C / 4 * QSZ : VSZ * C;
  }

  __device__ static __forceinline__ int idx(int n) {
    if constexpr (!PAD) return n;
    if constexpr (DIM == 2) return (n / L + 1) * LP + n % L + 1;
    return ((n / (L * L) + 1) * LP + (n / L) % L + 1) * LP + n % L + 1;
  }
  // Parity of the site stored at index q (halo entries hold sites of the same
  // parity as their storage coordinates minus one, since L is even).
  __device__ static __forceinline__ int spar(int q) {
    if constexpr (!PAD) return G::parity(q);
    if constexpr (DIM == 2) return (q / LP + q % LP) & 1;
    return (q / (LP * LP) + (q / LP) % LP + q % LP + 1) & 1;
  }
  // Storage-index offset of tap t (padded layout).
  __device__ static __forceinline__ int toff(int t) {
    if constexpr (DIM == 2) return G::tap_d(t, 0) * LP + G::tap_d(t, 1);
    return (G::tap_d(t, 0) * LP + G::tap_d(t, 1)) * LP + G::tap_d(t, 2);
  }
  // Storage index of site n + sign * delta_t; p = idx(n).
  __device__ static __forceinline__ int nbr(int n, int p, int t, int sign) {
    if constexpr (PAD) return p + sign * toff(t);
    return G::nbr(n, t, sign);
  }
  // Interior site held at storage index p (PAD: halo entries map to their source).
  __device__ static __forceinline__ int site_of(int p) {
    if constexpr (!PAD) return p;
    if constexpr (DIM == 2) {
      const int py = p / LP, px = p % LP;
      return ((py + L - 1) % L) * L + (px + L - 1) % L;
    } else {
      const int pz = p / (LP * LP), py = (p / LP) % LP, px = p % LP;
      return (((pz + L - 1) % L) * L + (py + L - 1) % L) * L + (px + L - 1) % L;
    }
  }
  // Halo entries of the padded layout: every storage position with a coordinate
  // 0 or LP - 1.  halo_entry(h) gives the h-th one (h < NHALO) and the storage
  // index of the interior position it mirrors (coordinate 0 mirrors L, LP - 1
  // mirrors 1).  2D: rows 0 and LP - 1 whole, then columns 0 and LP - 1 of the
  // interior rows.  3D: planes 0 and LP - 1 whole, then each interior plane's
  // 2D halo.
  static constexpr int RING2 = 2 * LP + 2 * L;
  static constexpr int NHALO = DIM == 2 ? RING2 : 2 * LP * LP + L * RING2;
  __device__ static __forceinline__ int mirror(int c) { return c == 0 ? L : (c == LP - 1 ? 1 : c); }
  __device__ static __forceinline__ void ring2(int r, int& y, int& x) {
    if (r < 2 * LP) {
      y = r < LP ? 0 : LP - 1;
      x = r < LP ? r : r - LP;
    } else {
      y = 1 + ((r - 2 * LP) >> 1);
      x = (r & 1) ? LP - 1 : 0;
    }
  }
  __device__ static __forceinline__ void halo_entry(int h, int& dst, int& src) {
    int z = 0, y, x;
    if constexpr (DIM == 2) {
      ring2(h, y, x);
    } else if (h < 2 * LP * LP) {
      const int r = h < LP * LP ? h : h - LP * LP;
      z = h < LP * LP ? 0 : LP - 1;
      y = r / LP;
      x = r - y * LP;
    } else {
      const int r = h - 2 * LP * LP;
      z = 1 + r / RING2;
      ring2(r - (z - 1) * RING2, y, x);
    }
    if constexpr (DIM == 2) {
      dst = y * LP + x;
      src = mirror(y) * LP + mirror(x);
    } else {
      dst = (z * LP + y) * LP + x;
      src = (mirror(z) * LP + mirror(y)) * LP + mirror(x);
    }
  }
  // Calls f(storage index) for every stored copy of site n.  Lanes whose site
  // has a mirror run every mirror combination without branching: a combination
  // that needs a mirror the site lacks keeps its own coordinate there, so it
  // lands on a copy that is stored anyway (f must be an idempotent store).
  template <class F>
  __device__ static __forceinline__ void copies(int n, F&& f) {
    f(idx(n));
    if constexpr (PAD) {
      int c[DIM], a[DIM];
      int q = n;
#pragma unroll
      for (int mu = DIM - 1; mu >= 0; --mu) {
        c[mu] = q % L;
        q /= L;
      }
      bool any = false;
#pragma unroll
      for (int mu = 0; mu < DIM; ++mu) {
        a[mu] = c[mu] == 0 ? L + 1 : (c[mu] == L - 1 ? 0 : -1);
        any |= a[mu] >= 0;
      }
      if (any) {
#pragma unroll
        for (int msk = 1; msk < (1 << DIM); ++msk) {
          int p = 0;
#pragma unroll
          for (int mu = 0; mu < DIM; ++mu) {
            const bool alt = (msk >> (DIM - 1 - mu)) & 1;
            p = p * LP + (alt && a[mu] >= 0 ? a[mu] : c[mu] + 1);
          }
          f(p);
        }
      }
    }
  }
  // copies(16 tile + m, f) for lane m of a 16-site tile, without divergent
  // branches: every lane stores its x mirror, and a lane away from the x edges
  // stores its own site again instead (f must be an idempotent store).  A tile
  // lies in one plane and spans whole rows or part of one, so whether it meets
  // a y or z edge is decided once per tile; its lanes then store their y (or z)
  // mirror, again falling back to their own site.  A mirror of coordinate 0
  // sits L storage steps above it, one of coordinate L-1 L steps below.
  template <class F>
  __device__ static __forceinline__ void copies_tile(int tile, int m, F&& f) {
    if constexpr (PAD && (L % 16 == 0 || 16 % L == 0)) {
      constexpr int R = L >= 16 ? 1 : 16 / L;  // rows per tile
      const int n0 = tile * 16;                // wave-uniform
      const int x = L >= 16 ? n0 % L + m : m % L;
      const int p = L >= 16 ? idx(n0) + m : idx(n0 + m);
      const int ax = x == 0 ? L : (x == L - 1 ? -L : 0);
      f(p);
      f(p + ax);
      const int y0 = (n0 / L) % L;
      const int y = L >= 16 ? y0 : y0 + m / L;
      const int ay = y == 0 ? L * LP : (y == L - 1 ? -L * LP : 0);
      const bool yedge = y0 == 0 || y0 + R - 1 == L - 1;
      if (yedge) {
        f(p + ay);
        f(p + ay + ax);
      }
      if constexpr (DIM == 3) {
        const int z = n0 / (L * L);
        const int az = z == 0 ? L * LP * LP : (z == L - 1 ? -L * LP * LP : 0);
        if (az) {
          f(p + az);
          f(p + az + ax);
          if (yedge) {
            f(p + az + ay);
            f(p + az + ay + ax);
          }
        }
      }
    } else {
      copies(tile * 16 + m, f);
    }
  }
};

// Storage index of lane m's site in tile `tile` (16 consecutive sites): when a row
// holds whole tiles the row part is wave-uniform.
template <class LY>
__device__ __forceinline__ int tile_p(int tile, int m) {
  if constexpr (LY::padded && LY::Ls % 16 == 0) return LY::idx(tile * 16) + m;
  return LY::idx(tile * 16 + m);
}

// The second hidden activation h2 = leaky(W2 * h1 + b2) of every site, saved by
// the training forward so that the backward reads it instead of recomputing
// conv2: FP32 2D L = 32, C = 16, whose backward holds h2 unpadded and
// quad-major.  A sample's entry is the image of the backward's h2 slot
// restricted to the lattice sites: C / 4 contiguous segments (segment q holds
// channels 4q .. 4q + 3 of site n at 4 n), which the backward copies into LDS
// as 1 KB chunks (64 lanes x 16 bytes).  After the N B images: s at the active
// sites, [N][B][V / 2] FP32 in half-site order, so that the backward also skips
// conv3.  (The BF16 2D L = 32 step was slower this way: without conv2 its
// backward still waits on the copy, and its conv1 loses the row triples built
// in the h2 slot.)
template <int DIM, int L, int C, bool BF16>
struct HSave {
  static constexpr int V = DIM == 2 ? L * L : L * L * L;
  static constexpr bool ok = !BF16 && DIM == 2 && L == 32 && C == 16;
  static constexpr int SEGS = C / 4;
  static constexpr int SEG_BYTES = 16 * V;
  static constexpr int CHUNKS = SEGS * SEG_BYTES / 1024;
  static constexpr size_t sample_bytes = (size_t)SEGS * SEG_BYTES;
  static constexpr size_t s_bytes = (size_t)V / 2 * 4;  // per sample and layer
  static_assert(SEG_BYTES % 1024 == 0, "whole 1 KB chunks per segment");
  // float offset of the s block of (layer, sample b), N layers of B samples
  __host__ __device__ static constexpr size_t s_off(int N, int B, int layer, int b) {
    return ((size_t)N * B * sample_bytes + ((size_t)layer * B + b) * s_bytes) / 4;
  }
  // float offset of channels ch0 .. ch0 + 3 (ch0 % 4 == 0) of site n in a sample
  __host__ __device__ static constexpr int off4(int n, int ch0) { return ((ch0 >> 2) * V + n) * 4; }
};

// Activations the plane-streaming training forward (3D, BF16 convolutions) saves
// for the backward, which then skips recomputing them; one block per layer of a
// batch of B samples, V sites, C channels: h1 and h2 channel-major BF16
// [B][C][V], the LeakyReLU sign word of every site of h1 and of h2 [B][V] (bit c
// set iff channel c's output is >= 0), and s at the active sites [B][V] FP32
// (frozen entries not written).  Byte offsets within a layer's block.
struct RingSave {
  size_t h1, h2, m1, m2, s, layer;
  __host__ __device__ RingSave(size_t B, int C, int V) {
    const size_t hb = B * (size_t)C * V * 2, wb = B * (size_t)V * 4;
    h1 = 0;
    h2 = hb;
    m1 = 2 * hb;
    m2 = 2 * hb + wb;
    s = 2 * hb + 2 * wb;
    layer = 2 * hb + 3 * wb;
  }
};

// Parity of |delta_t|_1: a neighbour at tap t has parity p(n) ^ todd(t).
template <int DIM>
__device__ __forceinline__ int todd(int t) {
  if constexpr (DIM == 2) return (t / 3 + t % 3) & 1;  // (d0+1) + (d1+1) has the parity of d0 + d1
  return (t / 9 + (t / 3) % 3 + t % 3 + 1) & 1;
}

// Number of 32-wide BF16 K chunks / 16-wide FP32 K blocks of a convolution
// with K = taps * cin.
__host__ __device__ constexpr int kchunks_bf16(int K) { return (K + 31) / 32; }
// K of conv1 in row-triple order: one slot per (row offset, dx) with dx in
// {-1, 0, +1, pad}; T / 3 row offsets (the taps of all axes but the fastest).
__host__ __device__ constexpr int k_tri(int T) { return T / 3 * 4; }
__host__ __device__ constexpr int kblocks_f32(int K) { return (K + 15) / 16; }

// Fragment bookkeeping for one layer (counts of 1 KB fragments = 64 lanes x 16 B).
struct LayerFrags {
  int nct;           // output-channel tiles of conv1/conv2 (16 rows each)
  int k1, k2;        // K chunks (BF16) or blocks (FP32) of conv1 and of conv2
  int k3;            // fragments of conv3: k2, or T C / 4 in quad layout
  int off1, off2, off3, total;  // fragment offsets within the layer
  // x4: conv3's two output rows also placed at rows 4u, 4u+1 (u = 1, 2, 3; fragments
  // from off3q, k2 per placement), so four tiles can share one accumulator with
  // tile u's s and t landing in lane group u
  bool x4;
  // quad (FP32): conv3 on v_mfma_f32_4x4x1f32, 16 blocks of 4 output rows x 4 sites;
  // fragment q holds k = 4q .. 4q + 3 of row (lane & 3)
  bool quad;
  int off3q;
};

// ps1 (FP32 2D backward): conv1's fragments split by tap parity, one block each
__host__ __device__ constexpr LayerFrags layer_frags(int T, int C, bool bf16, bool x4 = false,
                                                     bool quad = false, bool ps1 = false) {
  LayerFrags f{};
  f.nct = C >= 16 ? C / 16 : 1;
  f.k1 = ps1 ? 2 : bf16 ? kchunks_bf16(k_tri(T)) : kblocks_f32(k_tri(T));
  f.k2 = bf16 ? kchunks_bf16(T * C) : kblocks_f32(T * C);
  f.quad = quad;
  f.k3 = quad ? T * C / 4 : f.k2;
  f.off1 = 0;
  f.off2 = f.nct * f.k1;
  f.off3 = f.off2 + f.nct * f.k2;
  f.x4 = x4;
  f.off3q = f.off3 + f.k3;
  f.total = f.off3q + (f.x4 ? 3 * f.k2 : 0);
  return f;
}

}  // namespace fused
}  // namespace lfs

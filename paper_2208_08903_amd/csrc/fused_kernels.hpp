// Device helpers shared by the fused forward and backward kernels: weight
// fragment preparation, operand gathers from LDS-resident activations, the MFMA
// step and the hidden-activation epilogue.
#pragma once

#include <type_traits>

#include "fused_common.hpp"

namespace lfs {
namespace fused {

// A convolution's weights as MFMA A-fragments.  kind: 0 = forward
// convolution (rows = output channels, k = tap * cin + ci), 1 = its transpose
// used by the data gradient (rows = input channels, k = tap * cout + co).
struct FragSpec {
  int transposed, woff, cin, cout, rows, nct, nk, off;
};
constexpr int kMaxSpecs = 6;
struct FragTable {
  FragSpec s[kMaxSpecs];
  int count, total;  // fragments per layer
};

// One thread per (layer, fragment, lane): writes that lane's 16-byte operand.
// Rows beyond `rows` and k beyond taps * (cin or cout) are zero.
template <bool BF16>
__global__ void kf_prep(const float* __restrict__ params, int N, int T, int P_layer, FragTable tab,
                        u32x4* __restrict__ frags) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per_layer = (long)tab.total * 64;
  if (gid >= per_layer * N) return;
  const int layer = (int)(gid / per_layer);
  const int rem = (int)(gid % per_layer), f = rem / 64, l = rem % 64;
  const int j = l >> 4, m = l & 15;
  int si = 0;
  while (si + 1 < tab.count && f >= tab.s[si + 1].off) ++si;
  const FragSpec sp = tab.s[si];
  const int fl = f - sp.off, ct = fl / sp.nk, c = fl % sp.nk, row = ct * 16 + m;
  const float* W = params + (size_t)layer * P_layer + sp.woff;
  const int kdiv = sp.transposed ? sp.cout : sp.cin;
  const int K = T * kdiv;
  auto w_at = [&](int k) -> float {
    if (row >= sp.rows || k >= K) return 0.f;
    const int tap = k / kdiv, ch = k % kdiv;
    return sp.transposed ? W[(ch * sp.cin + row) * T + tap] : W[(row * sp.cin + ch) * T + tap];
  };
  u32x4 out;
  if constexpr (BF16) {
    const int k0 = 32 * c + 8 * j;
    for (int q = 0; q < 4; ++q) out[q] = pack_bf16(w_at(k0 + 2 * q), w_at(k0 + 2 * q + 1));
  } else {
    const int k0 = 16 * c + 4 * j;
    for (int q = 0; q < 4; ++q) out[q] = __float_as_uint(w_at(k0 + q));
  }
  frags[gid] = out;
}

template <bool BF16>
using HElem = std::conditional_t<BF16, uint16_t, float>;

// B operand of a C-input convolution at output site n (storage index p) for K
// chunk (BF16) / block (FP32) c: the lane's 8 (4) consecutive input channels at
// one tap, site n + SIGN * delta_tap.
template <class LY, int C, bool BF16, int SIGN = 1>
__device__ __forceinline__ u32x4 gather_h(const HElem<BF16>* h, int n, int p, int c, int j) {
  constexpr int K = LY::G::T * C;
  const int k0 = BF16 ? 32 * c + 8 * j : 16 * c + 4 * j;
  const int tap = k0 / C, ci0 = k0 % C;
  const int e = k0 < K ? LY::nbr(n, p, tap < LY::G::T ? tap : 0, SIGN) * C + ci0 : LY::ZS * C;
  return *reinterpret_cast<const u32x4*>(h + e);
}

// B operand of conv1: the masked field (frozen sites only) at the taps of the
// lane's K slice; xs is stored with layout LY; pn = parity of site n.
template <class LY, bool BF16>
__device__ __forceinline__ u32x4 gather_x(const float* xs, int n, int p, int pn, int fpar, int c,
                                          int j) {
  constexpr int T = LY::G::T;
  constexpr int NV = BF16 ? 8 : 4;
  const int t0 = BF16 ? 32 * c + 8 * j : 16 * c + 4 * j;
  float v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    // taps past T read the site itself (always in range) and are masked to 0
    const int t = t0 + i;
    const float xv = xs[t < T ? LY::nbr(n, p, t, 1) : p];
    v[i] = t < T && (pn ^ todd<LY::G::T == 9 ? 2 : 3>(t)) == fpar ? xv : 0.f;
  }
  u32x4 r;
  if constexpr (BF16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = pack_bf16(v[2 * q], v[2 * q + 1]);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = __float_as_uint(v[q]);
  }
  return r;
}

// B operand of conv1 from the masked field h0 (zero at active sites), stored with
// layout LY in BF16 (BF16 mode) or FP32: the taps of the lane's K slice.
template <class LY, bool BF16>
__device__ __forceinline__ u32x4 gather_h0(const HElem<BF16>* h0, int n, int p, int c, int j) {
  constexpr int T = LY::G::T;
  u32x4 r;
  if constexpr (BF16) {
    const int t0 = 32 * c + 8 * j;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ta = t0 + 2 * q, tb = ta + 1;
      const int ia = ta < T ? LY::nbr(n, p, ta, 1) : LY::ZS;
      const int ib = tb < T ? LY::nbr(n, p, tb, 1) : LY::ZS;
      r[q] = (uint32_t)h0[ia] | ((uint32_t)h0[ib] << 16);
    }
  } else {
    const int t0 = 16 * c + 4 * j;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      r[q] = __float_as_uint(h0[t0 + q < T ? LY::nbr(n, p, t0 + q, 1) : LY::ZS]);
  }
  return r;
}

// h0 = the field at frozen sites, 0 at active sites, in every stored position.
template <class LY, bool BF16, int NT>
__device__ __forceinline__ void build_h0(HElem<BF16>* h0, const float* xs, int fpar) {
  for (int q = threadIdx.x; q < LY::VSZ; q += NT) {
    const float v = q < LY::VS && LY::G::parity(LY::site_of(q)) == fpar ? xs[q] : 0.f;
    if constexpr (BF16) h0[q] = (uint16_t)bf16_bits(v);
    else h0[q] = v;
  }
}

// acc += A (fragment) x B (gathered) for one chunk / block.
template <bool BF16>
__device__ __forceinline__ f32x4 mma(const u32x4& a, const u32x4& b, f32x4 acc) {
  if constexpr (BF16) {
    return mfma(as_bf16x8(a), as_bf16x8(b), acc);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc = mfma(__uint_as_float(a[r]), __uint_as_float(b[r]), acc);
    return acc;
  }
}

// Store 4 channel values v (rows 4j..4j+3 of output-channel tile ct) of site n
// in every stored copy of the site; returns the packed BF16 words (BF16 mode).
template <class LY, int C, bool BF16>
__device__ __forceinline__ u32x2 store4(HElem<BF16>* h, int n, int co0, const float (&v)[4]) {
  if constexpr (BF16) {
    const u32x2 wv{pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3])};
    LY::copies(n, [&](int p) { *reinterpret_cast<u32x2*>(h + p * C + co0) = wv; });
    return wv;
  } else {
    const f32x4 fv{v[0], v[1], v[2], v[3]};
    LY::copies(n, [&](int p) { *reinterpret_cast<f32x4*>(h + p * C + co0) = fv; });
    return u32x2{0u, 0u};
  }
}

// Store leaky(acc + bias) for rows 4j..4j+3 of output-channel tile ct at site n.
template <class LY, int C, bool BF16>
__device__ __forceinline__ u32x2 store_hidden(HElem<BF16>* h, int n, int ct, int j,
                                              const f32x4& acc, const f32x4& bias) {
  const int co0 = ct * 16 + 4 * j;
  if (co0 >= C) return u32x2{0u, 0u};
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = leaky(acc[i] + bias[i]);
  return store4<LY, C, BF16>(h, n, co0, v);
}

// store4 for lane m of a 16-site tile (all stored copies of its site).
template <class LY, int C, bool BF16>
__device__ __forceinline__ u32x2 store4_tile(HElem<BF16>* h, int tile, int m, int co0,
                                             const float (&v)[4]) {
  if constexpr (BF16) {
    const u32x2 wv{pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3])};
    LY::copies_tile(tile, m, [&](int p) { *reinterpret_cast<u32x2*>(h + p * C + co0) = wv; });
    return wv;
  } else {
    const f32x4 fv{v[0], v[1], v[2], v[3]};
    LY::copies_tile(tile, m, [&](int p) { *reinterpret_cast<f32x4*>(h + p * C + co0) = fv; });
    return u32x2{0u, 0u};
  }
}

// Store leaky(a) for rows 4j..4j+3 of output-channel tile ct at lane m of a
// tile; a already holds the bias (the MFMA accumulator starts from it).
template <class LY, int C, bool BF16>
__device__ __forceinline__ u32x2 store_act_tile(HElem<BF16>* h, int tile, int m, int ct, int j,
                                                const f32x4& a) {
  const int co0 = ct * 16 + 4 * j;
  if (co0 >= C) return u32x2{0u, 0u};
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = leaky(a[i]);
  return store4_tile<LY, C, BF16>(h, tile, m, co0, v);
}

template <int C>
__device__ __forceinline__ f32x4 load_bias4(const float* b, int ct, int j) {
  const int co0 = ct * 16 + 4 * j;
  f32x4 r{0.f, 0.f, 0.f, 0.f};
  if (co0 < C) {
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = b[co0 + i];
  }
  return r;
}

// One implicit-GEMM pass over ntiles output tiles of 16 sites.  Wave w owns
// tiles w, w + nw, w + 2 nw, ... and takes TU of them per iteration: per K
// chunk it gathers the B operands of all TU tiles, then issues their MFMAs, and
// only after the last chunk runs the epilogues.  The TU independent chains let
// one tile's LDS latency hide behind another's MFMAs, which the compiler cannot
// arrange by itself (it cannot prove the epilogue's stores miss the next
// tile's loads).  Accumulators start from init (a bias, or zeros).
// gather(tile, c) -> u32x4; epi(tile, f32x4 (&acc)[NCT]).
template <int TU, int NCT, int KC, bool BF16, class Gather, class Epi>
__device__ __forceinline__ void mma_tiles(int ntiles, int w, int nw, const u32x4 (&A)[NCT][KC],
                                          const f32x4 (&init)[NCT], Gather&& gather, Epi&& epi) {
  for (int t0 = w; t0 < ntiles; t0 += TU * nw) {
    int tt[TU];
#pragma unroll
    for (int u = 0; u < TU; ++u) tt[u] = t0 + u * nw < ntiles ? t0 + u * nw : t0;
    f32x4 acc[TU][NCT];
#pragma unroll
    for (int u = 0; u < TU; ++u)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[u][ct] = init[ct];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      u32x4 bop[TU];
#pragma unroll
      for (int u = 0; u < TU; ++u) bop[u] = gather(tt[u], c);
#pragma unroll
      for (int u = 0; u < TU; ++u)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[u][ct] = mma<BF16>(A[ct][c], bop[u], acc[u][ct]);
    }
#pragma unroll
    for (int u = 0; u < TU; ++u)
      if (t0 + u * nw < ntiles) epi(tt[u], acc[u]);
  }
}

template <int DIM, int L, int C, bool BF16>
struct FwdCfg {
  using G = Geo<DIM, L>;
  static constexpr int V = G::V, T = G::T;
  static constexpr LayerFrags LF = layer_frags(T, C, BF16);
  static constexpr size_t bytes_for(int vs) {
    return ((size_t)vs * 4 + 15) / 16 * 16 + 2 * (size_t)vs * C * sizeof(HElem<BF16>);
  }
  static constexpr bool PAD = bytes_for(Lay<DIM, L, true>::VSZ) <= 156 * 1024;
  using LY = Lay<DIM, L, PAD>;
  static constexpr size_t lds_bytes = bytes_for(LY::VSZ);
  static constexpr int NT = lds_bytes > 80 * 1024 ? 512 : 256;
  // tiles in flight per wave: conv1 (one K chunk in BF16) and conv2/conv3
  static constexpr int TU1 = BF16 ? 4 : 2;
  static constexpr int TU2 = (DIM == 3 && !BF16) ? 1 : 2;
};

}  // namespace fused
}  // namespace lfs

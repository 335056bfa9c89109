// Device helpers shared by the fused forward and backward kernels: weight
// fragment preparation, operand gathers from LDS-resident activations, the MFMA
// step and the hidden-activation epilogue.
#pragma once

#include <type_traits>

#include "fused_common.hpp"

namespace lfs {
namespace fused {

// A convolution's weights as MFMA A-fragments.  transposed = 0: forward
// convolution (rows = output channels, k = tap * cin + ci); 1: its transpose
// used by the data gradient (rows = input channels, k = tap * cout + co).
// tri = 1 (single-input-channel forward convolution only): k in row-triple
// order, k = 4 * (tap / 3) + tap % 3, the slots 4 r + 3 being zero.  shift:
// the convolution's output row r is placed at fragment row r + shift.  quad = 1
// (FP32, v_mfma_f32_4x4x1f32): fragment c holds, in every lane l, row (l & 3) at
// k = 4c .. 4c + 3 (each of the 16 blocks of 4 lanes has the same A).
struct FragSpec {
  int transposed, woff, cin, cout, rows, nct, nk, off, tri, shift, quad;
  // psplit (FP32, 2D): chunk c holds the taps t = 2 i + c (those of one parity of
  // |delta_t|_1) and MFMA r of the chunk takes k = 4 r + j (its k = i kdiv + ch)
  int psplit;
};
constexpr int kMaxSpecs = 9;
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
  const int fl = f - sp.off, ct = fl / sp.nk, c = fl % sp.nk;
  const int row = sp.quad ? (l & 3) - sp.shift : ct * 16 + m - sp.shift;
  const float* W = params + (size_t)layer * P_layer + sp.woff;
  const int kdiv = sp.transposed ? sp.cout : sp.cin;
  const int K = T * kdiv;
  auto w_at = [&](int k) -> float {
    if (row < 0) return 0.f;
    if (sp.tri) {
      const int r = k >> 2, dx = k & 3;
      if (row >= sp.rows || dx == 3 || r >= T / 3) return 0.f;
      return W[row * T + 3 * r + dx];
    }
    if (row >= sp.rows || k >= K) return 0.f;
    const int tap = k / kdiv, ch = k % kdiv;
    return sp.transposed ? W[(ch * sp.cin + row) * T + tap] : W[(row * sp.cin + ch) * T + tap];
  };
  u32x4 out;
  if constexpr (BF16) {
    const int k0 = 32 * c + 8 * j;
    for (int q = 0; q < 4; ++q) out[q] = pack_bf16(w_at(k0 + 2 * q), w_at(k0 + 2 * q + 1));
  } else if (sp.psplit) {
    for (int q = 0; q < 4; ++q) {
      const int kk = 4 * q + j, tap = 2 * (kk / kdiv) + c, ch = kk % kdiv;
      const bool ok = row >= 0 && row < sp.rows && tap < T;
      out[q] = __float_as_uint(!ok ? 0.f
                               : sp.transposed ? W[(ch * sp.cin + row) * T + tap]
                                               : W[(row * sp.cin + ch) * T + tap]);
    }
  } else {
    const int k0 = sp.quad ? 4 * c : 16 * c + 4 * j;
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
  const int e = k0 < K ? LY::template off<C>(LY::nbr(n, p, tap < LY::G::T ? tap : 0, SIGN), ci0)
                        : LY::template off<C>(LY::ZS, 0);
  return *reinterpret_cast<const u32x4*>(h + e);
}

// conv1 operands in row-triple order.  A row triple of storage index q holds
// the masked field (frozen parity fpar kept, the rest 0) at q's site and its
// two neighbours along the fastest axis, plus a zero: (x[q-1], x[q], x[q+1], 0)
// as 4 BF16 (8 bytes) or 4 FP32 (16 bytes).  The K slice of lane j in chunk c
// (BF16: 8 slots, row offsets 8c + 2j and 8c + 2j + 1) or block c (FP32: 4
// slots, row offset 4c + j) is then whole triples at fixed per-lane offsets.
// Row offsets past T / 3 meet zero weights and read the site's own triple.
template <class LY, bool BF16>
__device__ __forceinline__ u32x4 gather_tri(const HElem<BF16>* tri, int n, int p, int c, int j) {
  constexpr int NR = LY::G::T / 3;
  auto at = [&](int r) { return r < NR ? LY::nbr(n, p, 3 * r + 1, 1) : p; };
  if constexpr (BF16) {
    const int r0 = 8 * c + 2 * j;
    const u32x2 a = *reinterpret_cast<const u32x2*>(tri + 4 * at(r0));
    const u32x2 b = *reinterpret_cast<const u32x2*>(tri + 4 * at(r0 + 1));
    return u32x4{a[0], a[1], b[0], b[1]};
  } else {
    return *reinterpret_cast<const u32x4*>(tri + 4 * at(4 * c + j));
  }
}

// Row triples of every stored position from the field xs (layout LY).  Padded
// layouts skip the halo columns, which no gather reads.
template <class LY, bool BF16, int NT>
__device__ __forceinline__ void build_tri(HElem<BF16>* tri, const float* xs, int fpar) {
  constexpr int TC = (LY::G::T - 1) / 2;  // the centre tap; TC -+ 1 step along the fastest axis
  for (int q = threadIdx.x; q < LY::VS; q += NT) {
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    bool live = true;
    int qm, qp;
    if constexpr (LY::padded) {
      const int px = q % LY::LP;
      live = px != 0 && px != LY::LP - 1;
      qm = q - 1;
      qp = q + 1;
    } else {
      qm = LY::G::nbr(q, TC - 1, 1);
      qp = LY::G::nbr(q, TC + 1, 1);
    }
    if (live) {
      const bool frozen = LY::spar(q) == fpar;  // the x neighbours have the other parity
      v[0] = frozen ? 0.f : xs[qm];
      v[1] = frozen ? xs[q] : 0.f;
      v[2] = frozen ? 0.f : xs[qp];
    }
    if constexpr (BF16) {
      *reinterpret_cast<u32x2*>(tri + 4 * q) = u32x2{pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3])};
    } else {
      *reinterpret_cast<f32x4*>(tri + 4 * q) = f32x4{v[0], v[1], v[2], v[3]};
    }
  }
}

// conv1 operands in row-triple order straight from the field xs (layout LY)
// for the site n (storage index p, parity pn): the same values gather_tri
// reads from a built triple array.
template <class LY, bool BF16>
__device__ __forceinline__ u32x4 gather_tri_x(const float* xs, int n, int p, int pn, int fpar,
                                              int c, int j) {
  constexpr int NR = LY::G::T / 3;
  constexpr int DIM = LY::G::Dim;
  auto triple = [&](int r, float (&v)[3]) {
    const int rr = r < NR ? r : (NR - 1) / 2;
    const int t = 3 * rr + 1, q = LY::nbr(n, p, t, 1);
    const bool frozen = (pn ^ todd<DIM>(t)) == fpar;
    const float xm = xs[LY::nbr(n, p, t - 1, 1)], xc = xs[q], xp = xs[LY::nbr(n, p, t + 1, 1)];
    v[0] = frozen ? 0.f : xm;
    v[1] = frozen ? xc : 0.f;
    v[2] = frozen ? 0.f : xp;
  };
  if constexpr (BF16) {
    float a[3], b[3];
    triple(8 * c + 2 * j, a);
    triple(8 * c + 2 * j + 1, b);
    return u32x4{pack_bf16(a[0], a[1]), pack_bf16(a[2], 0.f), pack_bf16(b[0], b[1]), pack_bf16(b[2], 0.f)};
  } else {
    float a[3];
    triple(4 * c + j, a);
    return u32x4{__float_as_uint(a[0]), __float_as_uint(a[1]), __float_as_uint(a[2]), 0u};
  }
}

// MFMA operand whose K slots are 8 consecutive sites: lane (j, m) receives channel
// ch0 + m of sites s .. s + 7 (s = the lane group's first site), each displaced by
// SIGN * d_tap (tap < 0: not displaced), from a site-major BF16 tensor (layout LY,
// C channels).  Two transposing LDS reads (ds_read_b64_tr_b16): within a group of
// 16 lanes, lane r addresses four elements M[r] and lane i receives M[4k + i/4][i%4]
// in slot k; lane r = 4k + q addresses channels ch0 + 4q .. ch0 + 4q + 3 of site
// s + k, so lane i gets channel ch0 + i of sites s .. s + 3 (then s + 4 .. s + 7).
// Channels at or past C read the next stored site (finite values in rows or
// columns of the product that are discarded).
template <class LY, int C, int SIGN>
__device__ __forceinline__ u32x4 load_tr8(const uint16_t* hs, int s, int ch0, int tap, int m) {
  typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
  const int k = m >> 2, q = m & 3;
  const int n1 = s + k, n2 = s + 4 + k;
  int p1 = LY::idx(n1), p2 = LY::idx(n2);
  if (tap >= 0) {
    p1 = LY::nbr(n1, p1, tap, SIGN);
    p2 = LY::nbr(n2, p2, tap, SIGN);
  }
  const bf16x4 v1 = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
      (lds_bf16x4*)(const_cast<uint16_t*>(hs + p1 * C + ch0 + 4 * q)));
  const bf16x4 v2 = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
      (lds_bf16x4*)(const_cast<uint16_t*>(hs + p2 * C + ch0 + 4 * q)));
  const u32x2 a = __builtin_bit_cast(u32x2, v1), b = __builtin_bit_cast(u32x2, v2);
  return u32x4{a[0], a[1], b[0], b[1]};
}

// FP32 convolutions with one or two output channels (conv3, and conv1 transposed)
// on v_mfma_f32_4x4x1f32: 16 blocks of 4 lanes, block b = l / 4; lane l gives
// A[l & 3][k] (the block's output row l & 3) and B[k][l & 3] (the input at its own
// site), and receives D[r][l & 3] in register r: every lane ends with all output
// channels of its own site.  Against the 16 x 16 tile the padding to 16 output
// rows is gone (4 rows of which 2 or 1 are used).
__device__ __forceinline__ f32x4 mfma4(float a, float b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// The lane's 4 consecutive input channels of K chunk q (k = 4q .. 4q + 3, tap-major,
// channel fastest) at site n + SIGN delta_tap (storage index p of n), FP32 storage.
template <class LY, int C, int SIGN = 1>
__device__ __forceinline__ u32x4 gather_q(const float* h, int n, int p, int q) {
  const int k0 = 4 * q, tap = k0 / C, ci0 = k0 % C;
  return *reinterpret_cast<const u32x4*>(h + LY::template off<C>(LY::nbr(n, p, tap, SIGN), ci0));
}

// sum_k A[r][k] B[k] over KQ chunks of 4 k for the lane's site: fq points at the lane's
// A entry of the first chunk, chunks STRIDE entries apart (64 in the fragment layout,
// 4 in a compact table of 4 rows per chunk); two accumulator chains (even and odd
// chunks) summed at the end.  init: the first chain's start.
template <int KQ, int STRIDE = 64, class Gather>
__device__ __forceinline__ f32x4 quad_conv(const u32x4* fq, const f32x4& init, Gather&& gather) {
  static_assert(KQ % 2 == 0, "chunks come in pairs");
  f32x4 a0 = init, a1{0.f, 0.f, 0.f, 0.f};
  // fully unrolled where K is short (2D: 36 chunks), so every table read and gather
  // can be issued ahead of its MFMAs; the 3D shapes (108 chunks) have no registers
  // for that
#pragma unroll(KQ <= 36 ? KQ / 2 : 3)
  for (int q = 0; q < KQ; q += 2) {
    const u32x4 w0 = fq[q * STRIDE], w1 = fq[(q + 1) * STRIDE];
    const u32x4 b0 = gather(q), b1 = gather(q + 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a0 = mfma4(__uint_as_float(w0[r]), __uint_as_float(b0[r]), a0);
      a1 = mfma4(__uint_as_float(w1[r]), __uint_as_float(b1[r]), a1);
    }
  }
  return a0 + a1;
}

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
    LY::copies(n, [&](int p) { *reinterpret_cast<f32x4*>(h + LY::template off<C>(p, co0)) = fv; });
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

// conv1 on the vector ALUs (FP32, 2D, 3x3 taps): h1 = leaky(W1 * mask_F x + b1) at
// every site, each thread on one active and one frozen site per step.  The masked
// field is nonzero only at the frozen sites, so an active site sees just its four
// axis neighbours and a frozen site itself and its four diagonal neighbours: the
// other taps' zeros are skipped rather than multiplied.  Each output sums the bias,
// then the taps in increasing order.  Only the interior copy is written (a padded
// layout's halo is filled afterwards).  wt: the layer's weights and biases staged
// tap-major in LDS (stage_w1t), read by every lane at the same address (broadcast).
constexpr int w1t_floats(int C) { return 10 * C; }

// [9][C] weights (tap-major) then [C] biases of the first convolution, into LDS
template <int C, int NT>
__device__ __forceinline__ void stage_w1t(float* wt, const float* __restrict__ pl, int off_W1, int off_b1) {
  for (int i = threadIdx.x; i < 10 * C; i += NT) {
    const int t = i / C, co = i - t * C;
    wt[i] = t < 9 ? pl[off_W1 + co * 9 + t] : pl[off_b1 + co];
  }
}

template <class LY, int C, int NT>
__device__ __forceinline__ void conv1_valu(const float* xs, float* h1, const float* wt, int fpar) {
  using G = typename LY::G;
  static_assert(G::Dim == 2 && G::T == 9 && C % 4 == 0, "2D lattice, 3x3 taps, channel quads");
  constexpr int taps_f[5] = {0, 2, 4, 6, 8}, taps_a[4] = {1, 3, 5, 7};
  const f32x4* wt4 = reinterpret_cast<const f32x4*>(wt);
  for (int a = threadIdx.x; a < G::V / 2; a += NT) {
    const int na = G::half_site(a, fpar ^ 1), nf = G::half_site(a, fpar);
    const int pa = LY::idx(na), pf = LY::idx(nf);
    float va[4], vf[5];
#pragma unroll
    for (int i = 0; i < 4; ++i) va[i] = xs[LY::nbr(na, pa, taps_a[i], 1)];
#pragma unroll
    for (int i = 0; i < 5; ++i) vf[i] = xs[LY::nbr(nf, pf, taps_f[i], 1)];
#pragma unroll
    for (int q = 0; q < C / 4; ++q) {
      // the quad's nine tap weights and its biases, all read before the sums
      f32x4 w[10];
#pragma unroll
      for (int t = 0; t < 10; ++t) w[t] = wt4[t * (C / 4) + q];
      f32x4 sa = w[9], sf = w[9];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) sa[r] += w[taps_a[i]][r] * va[i];
#pragma unroll
      for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) sf[r] += w[taps_f[i]][r] * vf[i];
#pragma unroll
      for (int r = 0; r < 4; ++r) sa[r] = leaky(sa[r]), sf[r] = leaky(sf[r]);
      *reinterpret_cast<f32x4*>(h1 + LY::template off<C>(pa, 4 * q)) = sa;
      *reinterpret_cast<f32x4*>(h1 + LY::template off<C>(pf, 4 * q)) = sf;
    }
  }
}

// Four channels co0..co0+3 (BF16 pairs in hv) of site n of a channel-major tensor.
template <int C, int V>
__device__ __forceinline__ void store_cm_global(uint16_t* t, int n, int co0, const u32x2& hv) {
  if (co0 >= C) return;
  t[(size_t)(co0 + 0) * V + n] = (uint16_t)hv[0];
  t[(size_t)(co0 + 1) * V + n] = (uint16_t)(hv[0] >> 16);
  t[(size_t)(co0 + 2) * V + n] = (uint16_t)hv[1];
  t[(size_t)(co0 + 3) * V + n] = (uint16_t)(hv[1] >> 16);
}

// LeakyReLU' mask word of one 16-channel tile: bit k set iff channel k's output
// h >= 0 (then leaky' = 1, else the slope; -0 counts as >= 0, like the float
// comparison).  Lane j holds channels 4j..4j+3 (BF16 pairs in hv); the four
// lanes that share m combine their nibbles, so every lane returns the word.
__device__ __forceinline__ uint32_t sign_mask16(const u32x2& hv, int j) {
  const uint32_t nib = (uint32_t)(bf16_lo(hv[0]) >= 0.f) | (uint32_t)(bf16_hi(hv[0]) >= 0.f) << 1 |
                       (uint32_t)(bf16_lo(hv[1]) >= 0.f) << 2 | (uint32_t)(bf16_hi(hv[1]) >= 0.f) << 3;
  uint32_t w = nib << (4 * j);
  w |= __shfl_xor(w, 16, 64);
  w |= __shfl_xor(w, 32, 64);
  return w;
}

// store4 for lane m of a 16-site tile: all stored copies of its site (HALO), or
// only the interior one, the halo being filled afterwards by fill_halo.
template <class LY, int C, bool BF16, bool HALO = true>
__device__ __forceinline__ u32x2 store4_tile(HElem<BF16>* h, int tile, int m, int co0,
                                             const float (&v)[4]) {
  if constexpr (BF16) {
    const u32x2 wv{pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3])};
    if constexpr (HALO)
      LY::copies_tile(tile, m, [&](int p) { *reinterpret_cast<u32x2*>(h + p * C + co0) = wv; });
    else
      *reinterpret_cast<u32x2*>(h + tile_p<LY>(tile, m) * C + co0) = wv;
    return wv;
  } else {
    const f32x4 fv{v[0], v[1], v[2], v[3]};
    if constexpr (HALO)
      LY::copies_tile(tile, m, [&](int p) { *reinterpret_cast<f32x4*>(h + LY::template off<C>(p, co0)) = fv; });
    else
      *reinterpret_cast<f32x4*>(h + LY::template off<C>(tile_p<LY>(tile, m), co0)) = fv;
    return u32x2{0u, 0u};
  }
}

// Copies every halo entry of a site-major tensor (C channels, layout LY) from
// the interior position it mirrors, 16 bytes per item, all NT threads.  Runs
// between the barrier that ends the pass storing the interior and the barrier
// before the first periodic gather.  Unpadded layouts have no halo.
template <class LY, int C, bool BF16, int NT>
__device__ __forceinline__ void fill_halo(HElem<BF16>* h) {
  if constexpr (LY::padded) {
    constexpr int EL = BF16 ? 8 : 4;  // elements per 16 bytes
    static_assert(C % EL == 0, "fill_halo copies whole 16-byte chunks");
    constexpr int CH = C / EL;
    for (int i = threadIdx.x; i < LY::NHALO * CH; i += NT) {
      const int e = i / CH, k = i - e * CH;
      int dst, src;
      LY::halo_entry(e, dst, src);
      *reinterpret_cast<u32x4*>(h + LY::template off<C>(dst, k * EL)) =
          *reinterpret_cast<const u32x4*>(h + LY::template off<C>(src, k * EL));
    }
  }
}

// Store leaky(a) for rows 4j..4j+3 of output-channel tile ct at lane m of a
// tile; a already holds the bias (the MFMA accumulator starts from it).
template <class LY, int C, bool BF16, bool HALO = true>
__device__ __forceinline__ u32x2 store_act_tile(HElem<BF16>* h, int tile, int m, int ct, int j,
                                                const f32x4& a) {
  const int co0 = ct * 16 + 4 * j;
  if (co0 >= C) return u32x2{0u, 0u};
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = leaky(a[i]);
  return store4_tile<LY, C, BF16, HALO>(h, tile, m, co0, v);
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
//
// FP32: chunk c is four MFMAs, MFMA r taking k = 16 c + 4 j + r from lane group j;
// those whose k are all padding (k >= KLIM, or the zero slot 3 of every row
// triple when TRI) are not issued.
template <int TU, int NCT, int KC, bool BF16, int KLIM = (1 << 30), bool TRI = false, class Gather,
          class Epi>
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
        for (int ct = 0; ct < NCT; ++ct) {
          if constexpr (BF16) {
            acc[u][ct] = mma<true>(A[ct][c], bop[u], acc[u][ct]);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (16 * c + r < KLIM && !(TRI && r == 3))
                acc[u][ct] = mfma(__uint_as_float(A[ct][c][r]), __uint_as_float(bop[u][r]), acc[u][ct]);
          }
        }
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
  // FP32: conv3's quad A table, compact (4 rows of 16 bytes per chunk), after h2
  static constexpr size_t QT_BYTES = BF16 ? 0 : (size_t)(T * C / 4) * 4 * 16;
  // FP32 2D L = 32: activations quad-major (conflict-free gathers and stores) and
  // unpadded, periodic neighbours by shift and mask as in the backward (no halo
  // passes; forward 0.904 -> 0.898 ms per training step against the padded layout)
  static constexpr bool QM = !BF16 && DIM == 2 && L == 32;
  // FP32 2D L = 32: conv1 on the vector ALUs (conv1_valu: forward 0.948 -> 0.907 ms per
  // training step), its weights in an LDS table after conv3's (the next layer's staged
  // during conv3).  The backward keeps its matrix-core conv1, which was faster there.
  static constexpr bool C1V = !BF16 && DIM == 2 && L == 32;
  static constexpr size_t W1T_BYTES = C1V ? (size_t)w1t_floats(C) * 4 : 0;
  template <class LYX>
  static constexpr size_t bytes_of() {
    return ((size_t)LYX::VSZ * 4 + 15) / 16 * 16 + 2 * (size_t)LYX::template elems<C>() * sizeof(HElem<BF16>) +
           QT_BYTES + W1T_BYTES;
  }
  static constexpr bool PAD = !QM && bytes_of<Lay<DIM, L, true, QM>>() <= 156 * 1024;
  using LY = Lay<DIM, L, PAD, QM>;
  static constexpr size_t lds_bytes = bytes_of<LY>();
  static constexpr int NT = lds_bytes > 80 * 1024 ? 512 : 256;
  // tiles in flight per wave: conv1 (one K chunk in BF16) and conv2/conv3
  static constexpr int TU1 = BF16 ? 4 : 2;
  // (FP32 2D L = 32: all eight of a wave's conv2 tiles in flight at once, 222 registers:
  // four tiles were 1.8 % faster than two, eight another 1.5 %)
  static constexpr int TU2 = (DIM == 3 && !BF16) ? 1 : (!BF16 && DIM == 2 && L == 32 ? 8 : 2);
  // conv3 four tiles per accumulator (2D BF16: the FP32 and 3D fragments of four
  // placements do not fit the registers) when every wave has four active-site tiles
  static constexpr bool X4 = T == 9 && BF16 && V / 32 >= 4 * (NT / 64);
  // FP32 conv3 on the 4x4 matrix-core blocks (two of every four output rows used
  // instead of two of sixteen), every lane ending with its own site's s and t
  static constexpr bool Q3 = !BF16;
  static constexpr LayerFrags LF = layer_frags(T, C, BF16, X4, Q3);
  // each pass's weight fragments fetched during the previous pass (2D, C <= 16:
  // the extra live fragments fit the registers of two waves per SIMD)
  static constexpr bool PFA = DIM == 2 && C <= 16;
  // conv1 gathers its operands straight from the field instead of from row
  // triples built in a pass of their own: faster where the pass and its barrier
  // weigh more than the costlier gathers (2D FP32, and small 2D lattices whose
  // four tiles per sample leave the barrier exposed); the 2D L = 32 and 3D BF16
  // forwards are faster with the built triples
  static constexpr bool TRIX = DIM == 2 && (!BF16 || L <= 8);
};

}  // namespace fused
}  // namespace lfs

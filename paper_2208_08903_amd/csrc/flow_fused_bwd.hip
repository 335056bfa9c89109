// Fused backward of one coupling layer (the hand-written vector-Jacobian
// product of the layer; paper Sec. 1 defines the layer, its derivative is
// derived in the oracle's adjoint).  One launch per layer; persistent
// workgroups each take whole samples and keep the sample in LDS:
//
//   recompute  h1 = leaky(W1 * mask_F x + b1), h2 = leaky(W2 * h1 + b2),
//              (o0, o1) = W3 * h2 + b3 at the active sites, s = tanh(o0), t = o1
//              (FP32: conv3 and conv1^T on the 4x4 matrix-core blocks, quad_conv;
//              in training at 2D L = 32 h2 and s come from the forward's saved
//              copies instead, HS)
//   affine     g_t = g_y, g_s = g_y x e^s + g_logdet, g_o0 = g_s (1 - s^2),
//              g_x(active) = g_y e^s
//   conv3^T    g_a2 = leaky'(h2) (W3^T * g_o)        dW3 += g_o (x) h2
//   conv2^T    g_a1 = leaky'(h1) (W2^T * g_a2)       dW2 += g_a2 (x) h1
//   conv1^T    g_x(frozen) = g_y + W1^T * g_a1       dW1 += g_a1 (x) mask_F x
//
// Every convolution is an implicit GEMM on the matrix cores.  The weight
// gradients are GEMMs whose reduction runs over the sites; their operands are
// 8 (BF16) or 4 (FP32) consecutive sites of one channel.  In BF16 mode the
// activations stay site-major and those operands come from two transposing LDS
// reads (ds_read_b64_tr_b16); g_o, the masked field and, in 3D, g_a2 also keep
// channel-major rows, read 16 bytes at a time (a +-1 offset along the fast
// axis is a funnel shift with one extra element).  FP32 operands are single
// values read from the site-major tensors.  Halo copies of the site-major
// tensors are filled in one cooperative pass after each producing pass, and
// the layer's weight fragments are staged in LDS once per launch where they
// fit.  Weight-gradient tiles accumulate in registers over all of a
// workgroup's samples, are summed across waves in a fixed order, and written
// as one partial per workgroup; a fixed-order reduction over workgroups gives
// the gradient, so results are bitwise reproducible.
#include <algorithm>
#include <type_traits>

#include "fused_bwd_common.hpp"

namespace lfs {
namespace fused {
namespace {

constexpr size_t align16(size_t x) { return (x + 15) / 16 * 16; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr size_t cmaxz(size_t a, size_t b) { return a > b ? a : b; }

// SPLIT (2D BF16 at L = 32): the sample state of a 4-wave workgroup kept under
// half the LDS so that two workgroups share a CU: no g_y copy (read from L2),
// the masked field's channel-major row over g_o's (built after dW3), two slots.
template <int DIM, int L, int C, bool BF16, bool PAD, bool SPLIT = false, bool QM = false>
struct BwdLds {
  using LY = Lay<DIM, L, PAD, QM>;
  static constexpr int V = Geo<DIM, L>::V, VS = LY::VS;
  static constexpr int CSTR = V + 8;  // channel-major row stride in elements (BF16 mode)
  // site-major tensors and g_o carry the layout's extra all-zero site
  static constexpr size_t SA = (size_t)LY::template elems<C>() * (BF16 ? 2 : 4);  // activation tensor
  static constexpr size_t OFF_XS = 0;
  static constexpr size_t OFF_GY = align16((size_t)VS * 4);
  static constexpr size_t OFF_GOS = OFF_GY + (SPLIT ? 0 : align16((size_t)V * 4));
  static constexpr size_t GOS_BYTES = (size_t)LY::VSZ * (BF16 ? 4 : 8);
  static constexpr size_t OFF_GOC = OFF_GOS + align16(GOS_BYTES);
  static constexpr size_t GOC_BYTES = BF16 ? 2 * (size_t)CSTR * 2 : 0;
  static constexpr size_t OFF_H0C = SPLIT ? OFF_GOC : OFF_GOC + align16(GOC_BYTES);
  static constexpr size_t H0C_BYTES = BF16 ? (size_t)CSTR * 2 : 0;
  static constexpr size_t OFF_SLOT = SPLIT ? OFF_GOC + align16(GOC_BYTES) : OFF_H0C + align16(H0C_BYTES);
  // site-major slots: BF16 three (S0: h1; S1: conv1's row triples, then h2, then
  // g_a1; S2: g_a2), FP32 and SPLIT two (h1 then g_a1 in place; conv1's row
  // triples (BF16), then h2, then g_a2 in place).  The weight-gradient GEMMs read
  // their site-major operands with transposing LDS reads; g_o and the masked
  // field keep channel-major rows, and so does g_a2 in 3D (S3), whose 27 shifted
  // reads in dW2 would otherwise cost more registers in address arithmetic than
  // the lanes have.
  static constexpr bool CM2 = BF16 && DIM == 3;
  static constexpr size_t OFF_S0 = OFF_SLOT;
  static constexpr size_t OFF_S1 = OFF_S0 + SA;
  static constexpr size_t OFF_S2 = OFF_S1 + SA;
  static constexpr size_t OFF_S3 = OFF_S2 + SA;
  static constexpr size_t MAIN = (!BF16 || SPLIT) ? OFF_S2 : CM2 ? OFF_S3 + (size_t)C * CSTR * 2 : OFF_S3;
};

// Channel-major BF16 copy of four channels co0..co0+3 (packed pairs in hv) of
// site n: row co holds the V sites of channel co, CSTR elements apart.
template <int C, int CSTR>
__device__ __forceinline__ void store_cm4(uint16_t* hc, int n, int co0, const u32x2& hv) {
  if (co0 >= C) return;
  hc[(co0 + 0) * CSTR + n] = (uint16_t)hv[0];
  hc[(co0 + 1) * CSTR + n] = (uint16_t)(hv[0] >> 16);
  hc[(co0 + 2) * CSTR + n] = (uint16_t)hv[1];
  hc[(co0 + 3) * CSTR + n] = (uint16_t)(hv[1] >> 16);
}

template <int DIM, int L, int C, bool BF16>
struct BwdCfg {
  using G = Geo<DIM, L>;
  static constexpr int V = G::V, T = G::T;
  static constexpr int KT3 = BF16 ? kchunks_bf16(2 * T) : kblocks_f32(2 * T);
  static constexpr int P_LAYER = C * T + C + C * C * T + C + 2 * C * T + 2;
  // 2D BF16 at L = 32, C = 16: two 4-wave workgroups per CU, each on its own
  // sample, so that one workgroup's barriers and pass-start latencies overlap the
  // other's work (the passes are latency-bound: a few MFMAs per tile between LDS
  // round trips).  The sample state then has to fit half the LDS: unpadded layout
  // (periodic neighbours by shift and mask), g_a2 and g_a1 in place over h2 and h1
  // (dW3 runs before conv3^T overwrites h2), g_y read from L2 where it is used, and
  // the layer's weight fragments read from L2 instead of an LDS copy.
  static constexpr bool SPLIT = BF16 && DIM == 2 && L == 32 && C == 16;
  static constexpr bool PAD = !SPLIT && BwdLds<DIM, L, C, BF16, true>::MAIN <= 158 * 1024;
  // FP32 2D L = 32: activations quad-major (conflict-free gathers and stores)
  static constexpr bool QM = !BF16 && DIM == 2 && !PAD;
  using M = BwdLds<DIM, L, C, BF16, PAD, SPLIT, QM>;
  using LY = typename M::LY;
  static constexpr int CSTR = M::CSTR;
  // LDS of the sample state (and, after the sample loop, of the partial sums)
  // with saved activations: conv1's A fragments in LDS too (staged once per
  // launch), so that no global load waits behind the asynchronous h2 copy
  static constexpr bool A1L = HSave<DIM, L, C, BF16>::ok;
  static constexpr size_t A1_BYTES =
      A1L ? (size_t)((C + 15) / 16) * (!BF16 && DIM == 2 ? 2 : kblocks_f32(k_tri(T))) * 64 * 16 : 0;
  static constexpr size_t lds_main = cmaxz(M::MAIN + (BF16 ? 0 : 16 + (size_t)(T * C / 4) * 2 * 4 * 16) + A1_BYTES,
                                           (size_t)P_LAYER * 4);
  // 3D shapes need more than the 256 registers a lane gets at 2 waves per SIMD.
  static constexpr int NT = (lds_main > 80 * 1024 && DIM == 2) ? 512 : 256;
  // waves per SIMD the register allocation has to allow (SPLIT: two workgroups)
  static constexpr int MINW = SPLIT ? 2 : 1;
  static constexpr int NW = NT / 64;
  // Tiles in flight per wave in the tile passes: two where the registers allow
  // (3D shapes, and FP32 C=16 at two waves per SIMD, are already at the limit).
  static constexpr int TU = DIM == 2 && (BF16 || NT == 256 || C < 16) ? 2 : 1;
  // conv3 recompute: tiles whose affine backward share a pass -- four where the
  // extra fragments fit the registers, two (one shuffle) otherwise; BF16 with at
  // least that many active-site tiles per wave, else one (SPLIT: two, for registers)
  static constexpr int TPW3 = V / 32 / NW;
  static constexpr int QU3 = !(T == 9 && BF16) ? 1 : (NT == 256 && !SPLIT && TPW3 >= 4) ? 4 : (TPW3 >= 2 ? 2 : 1);
  // FP32: conv3 (recompute) and conv1^T (one output channel) on the 4x4 matrix-core
  // blocks (quad fragments), every lane with its own site's result
  // FP32 2D (PS1): conv1 by site parity -- a frozen site meets the masked field
  // only through the five taps of even |delta|_1, an active site only through the
  // four odd ones (K = 5 and 4 instead of the nine taps' row triples)
  static constexpr bool PS1 = !BF16 && DIM == 2 && T == 9;
  static constexpr LayerFrags LF = layer_frags(T, C, BF16, QU3 == 4, !BF16, PS1);
  static constexpr int K1T = BF16 ? LF.k2 : T * C / 4;  // conv1^T fragments
  static constexpr int OFF3T = LF.total;
  static constexpr int OFF2T = OFF3T + LF.nct * KT3;
  static constexpr int OFF1T = OFF2T + LF.nct * LF.k2;
  static constexpr int FRAGS = OFF1T + K1T;
  // The layer's weight fragments are the same for every sample of the launch:
  // where they fit next to the sample state without costing a workgroup per
  // CU, they are copied to LDS once per launch instead of being fetched from
  // L2 at the start of every pass of every sample.
  static constexpr size_t RED_STATIC = (size_t)kRedSlices * (NT / kRedSlices + 1) * 4;
  static constexpr size_t FRAG_BYTES = (size_t)FRAGS * 64 * 16;
  // FP32: the quad A tables of conv3 and conv1^T, compact (4 rows of 16 bytes per
  // chunk), staged in LDS once per launch after the sample state
  static constexpr size_t OFF_QT = align16(M::MAIN);
  static constexpr size_t QT_BYTES = BF16 ? 0 : (size_t)(LF.k3 + K1T) * 4 * 16;
  static constexpr size_t OFF_A1 = align16(OFF_QT + QT_BYTES);
  static constexpr size_t OFF_FRAG = align16(OFF_A1 + A1_BYTES);
  static constexpr int per_cu(size_t bytes) { return bytes > 160 * 1024 ? 0 : cmin(8, (int)(160 * 1024 / bytes)); }
  static constexpr bool FRAG_LDS = OFF_FRAG + FRAG_BYTES + RED_STATIC <= 158 * 1024 &&
                                   per_cu(OFF_FRAG + FRAG_BYTES + RED_STATIC) == per_cu(lds_main + RED_STATIC);
  static constexpr size_t lds_bytes = FRAG_LDS ? cmaxz(OFF_FRAG + FRAG_BYTES, (size_t)P_LAYER * 4) : lds_main;
  static constexpr int MT = (C + 15) / 16;
  static constexpr int NKC = BF16 ? V / 32 : V / 16;  // K chunks (sites) per sample
  // every wave's share of the K chunks, when it is the same for all waves (a
  // compile-time trip count lets the weight-gradient loops unroll)
  static constexpr bool KEXACT = NKC % NW == 0;
  static constexpr int KPW = NKC / NW;
  // unroll of the dW3 and dW1 chunk loops, 2D L=32 C=16 only (measured about
  // 1 % faster; elsewhere unrolling costs registers, spills in 3D): dW1 by 4
  // (by 2 in the FP32 kernel that recomputes h2, which would spill), dW3 by 4
  // in BF16 and not in FP32, where it would spill
  static constexpr bool DWX = DIM == 2 && L == 32 && C == 16;
  static constexpr int DWU3 = DWX && BF16 ? 4 : 1, DWU1 = DWX ? 4 : 1;
  // Weight-gradient output tiles; every wave accumulates all of them over its
  // contiguous range of K chunks, and the waves are summed in a fixed order.
  // FP32 2D (PS3): g_o is zero at the frozen sites, so in conv3^T and dW3 an active
  // site meets it only through the five taps of even |delta|_1 and a frozen site
  // only through the four odd ones: both passes run the two halves of the sites
  // apart, each with its own taps (dW3: one tile per half, columns (tap, co) of
  // that half's taps; conv3^T: K = 10 and 8 instead of 18).
  static constexpr bool PS3 = !BF16 && DIM == 2 && T == 9;
  static constexpr int NTL3 = PS3 ? 2 : (2 * T + 15) / 16, NTL1 = (T + 15) / 16;
  static constexpr int I3 = MT * NTL3;
  static constexpr int I2 = MT * T * MT;
  static constexpr int I1 = MT * NTL1;
};

// ---- weight-gradient operands ---------------------------------------------

// Row index (all axes but the last) of site s shifted by sign * delta_tap, and
// the shift along the last axis.
template <int DIM, int L>
__device__ __forceinline__ void shifted_row(int s, int tap, int sign, int& rowS, int& e) {
  using G = Geo<DIM, L>;
  const int row = s / L;
  if constexpr (DIM == 2) {
    rowS = G::wrapc(row + sign * G::tap_d(tap, 0));
    e = sign * G::tap_d(tap, 1);
  } else {
    const int z = row / L, y = row % L;
    rowS = G::wrapc(z + sign * G::tap_d(tap, 0)) * L + G::wrapc(y + sign * G::tap_d(tap, 1));
    e = sign * G::tap_d(tap, 2);
  }
}

// BF16, channel-major row `cr` (stride CSTR): the 8 sites s0..s0+7 (one row,
// s0 % 8 == 0) shifted by sign * delta_tap, as 4 packed BF16 pairs.
template <int DIM, int L>
__device__ __forceinline__ u32x4 load8_shift(const uint16_t* cr, int s0, int tap, int sign) {
  int rowS, e;
  shifted_row<DIM, L>(s0, tap, sign, rowS, e);
  const int x0 = s0 % L;
  const uint16_t* rp = cr + rowS * L;
  const u32x4 v = *reinterpret_cast<const u32x4*>(rp + x0);
  const uint32_t nxt = rp[(x0 + 8) & (L - 1)], prv = rp[(x0 + L - 1) & (L - 1)];
  const u32x4 up{__builtin_amdgcn_alignbit(v[1], v[0], 16), __builtin_amdgcn_alignbit(v[2], v[1], 16),
                 __builtin_amdgcn_alignbit(v[3], v[2], 16), __builtin_amdgcn_alignbit(nxt, v[3], 16)};
  const u32x4 dn{__builtin_amdgcn_alignbit(v[0], prv << 16, 16), __builtin_amdgcn_alignbit(v[1], v[0], 16),
                 __builtin_amdgcn_alignbit(v[2], v[1], 16), __builtin_amdgcn_alignbit(v[3], v[2], 16)};
  return e > 0 ? up : (e < 0 ? dn : v);
}

// FP32, site-major storage (layout LY, CH channels): channel ch of site s + sign * delta_tap.
template <class LY, int CH>
__device__ __forceinline__ float load1_shift(const float* h, int s, int ch, int tap, int sign) {
  return h[LY::nbr(s, LY::idx(s), tap, sign) * CH + ch];
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int DIM, int TAP, int MU>
constexpr int tap_dc() {
  return DIM == 2 ? (MU == 0 ? TAP / 3 : TAP % 3) - 1
                  : (MU == 0 ? TAP / 9 : (MU == 1 ? (TAP / 3) % 3 : TAP % 3)) - 1;
}

// Row (all axes but the last) of site s shifted by SIGN * delta_TAP.
template <int DIM, int L, int TAP, int SIGN>
__device__ __forceinline__ int shifted_row_c(int s) {
  using G = Geo<DIM, L>;
  const int row = s / L;
  if constexpr (DIM == 2) return G::wrapc(row + SIGN * tap_dc<DIM, TAP, 0>());
  const int z = row / L, y = row % L;
  return G::wrapc(z + SIGN * tap_dc<DIM, TAP, 0>()) * L + G::wrapc(y + SIGN * tap_dc<DIM, TAP, 1>());
}

// BF16: 8 sites x0 + E .. x0 + E + 7 (periodic) of row rp, x0 % 8 == 0, as 4 BF16 pairs.
template <int L, int E>
__device__ __forceinline__ u32x4 load8_e(const uint16_t* rp, int x0) {
  const u32x4 v = *reinterpret_cast<const u32x4*>(rp + x0);
  if constexpr (E == 0) {
    return v;
  } else if constexpr (E > 0) {
    const uint32_t nxt = rp[(x0 + 8) & (L - 1)];
    return u32x4{__builtin_amdgcn_alignbit(v[1], v[0], 16), __builtin_amdgcn_alignbit(v[2], v[1], 16),
                 __builtin_amdgcn_alignbit(v[3], v[2], 16), __builtin_amdgcn_alignbit(nxt, v[3], 16)};
  } else {
    const uint32_t prv = rp[(x0 + L - 1) & (L - 1)];
    return u32x4{__builtin_amdgcn_alignbit(v[0], prv << 16, 16), __builtin_amdgcn_alignbit(v[1], v[0], 16),
                 __builtin_amdgcn_alignbit(v[2], v[1], 16), __builtin_amdgcn_alignbit(v[3], v[2], 16)};
  }
}

// ---- saved h2 ----------------------------------------------------------------
// Asynchronous copy of one sample's saved h2 (HSave image at src) into the LDS
// slot dst, segment s at dst + s * seg_stride bytes: wave w copies chunks w,
// w + NW, ..., every lane 16 bytes (global_load_lds_dwordx4: lane i's bytes land
// at the chunk's LDS address + 16 i).  No registers hold the data; the copy
// counts as outstanding vector-memory loads until s_waitcnt vmcnt(0), after
// which a barrier publishes it to the workgroup.
template <class HS, int NW>
__device__ __forceinline__ void load_h2_async(const unsigned char* src, unsigned char* dst, int seg_stride,
                                              int w, int lane) {
  typedef __attribute__((address_space(1))) void* gptr;
  typedef __attribute__((address_space(3))) void* lptr;
  constexpr int CPS = HS::SEG_BYTES / 1024;
#pragma unroll
  for (int k = w; k < HS::CHUNKS; k += NW) {
    const int sg = k / CPS, o = (k - sg * CPS) * 1024;
    __builtin_amdgcn_global_load_lds((gptr)(src + (size_t)k * 1024 + lane * 16), (lptr)(dst + sg * seg_stride + o),
                                     16, 0, 0);
  }
}

// Workgroup barrier over LDS only: waits for the wave's LDS operations but not
// for its vector-memory ones, so that the asynchronous copy of the next sample's
// h2 stays in flight across it (a fenced barrier waits for it: the copy writes
// LDS).  Used only between passes that neither read the copy's destination nor
// exchange global memory.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ---- the kernel -------------------------------------------------------------

// HS: h2 and s are read from the training forward's saved copies (hsv, this
// layer's [B] HSave images; hss, its [B][V / 2] s at the active sites) instead
// of being recomputed.
template <int DIM, int L, int C, bool BF16, int NT, bool HS = false>
__global__ void __launch_bounds__(NT, (BwdCfg<DIM, L, C, BF16>::MINW)) kf_backward(
    const u32x4* frags, const float* __restrict__ pl, int off_b1, int off_b2,
    int off_b3, int off_W1, int off_W2, int off_W3, int fpar, int final_tanh, float g_ld,
    const double* __restrict__ g_ld_vec, int B,
    const float* __restrict__ xin, const float* __restrict__ gy, float* __restrict__ gx,
    float* __restrict__ partial, const float* __restrict__ prev_partial, float* __restrict__ prev_out,
    int n_parts, const unsigned char* __restrict__ hsv, const float* __restrict__ hss) {
  using Cfg = BwdCfg<DIM, L, C, BF16>;
  using G = Geo<DIM, L>;
  using HT = HElem<BF16>;
  constexpr int V = Cfg::V, T = Cfg::T, NW = Cfg::NW, MT = Cfg::MT, NKC = Cfg::NKC;
  constexpr int CSTR = Cfg::CSTR;
  constexpr LayerFrags LF = Cfg::LF;
  extern __shared__ __align__(16) unsigned char smem[];
  using M = typename Cfg::M;
  using LY = typename Cfg::LY;
  constexpr int VS = LY::VS;
  float* xs = reinterpret_cast<float*>(smem + M::OFF_XS);
  float* gys = reinterpret_cast<float*>(smem + M::OFF_GY);
  const int lane = threadIdx.x & 63, w = wave_id(), j = lane >> 4, m = lane & 15;
  const u32x4* fr;
  if constexpr (Cfg::FRAG_LDS) {
    u32x4* sfr = reinterpret_cast<u32x4*>(smem + Cfg::OFF_FRAG);
    for (int i = threadIdx.x; i < Cfg::FRAGS * 64; i += NT) sfr[i] = frags[i];
    fr = sfr + lane;  // visible after the first sample's staging barrier
  } else {
    fr = frags + lane;
  }
  const int apar = fpar ^ 1;
  const u32x4* qt = reinterpret_cast<const u32x4*>(smem + Cfg::OFF_QT);
  if constexpr (!BF16) {
    // quad A entries (rows 0..3 of every chunk) of conv3 and conv1^T; visible after
    // the first sample's staging barrier
    u32x4* q = reinterpret_cast<u32x4*>(smem + Cfg::OFF_QT);
    for (int i = threadIdx.x; i < (LF.k3 + Cfg::K1T) * 4; i += NT) {
      const int c = i >> 2;
      q[i] = frags[(c < LF.k3 ? LF.off3 + c : Cfg::OFF1T + c - LF.k3) * 64 + (i & 3)];
    }
  }
  const u32x4* a1s = reinterpret_cast<const u32x4*>(smem + Cfg::OFF_A1);
  if constexpr (Cfg::A1L) {
    static_assert(Cfg::A1_BYTES == (size_t)LF.nct * LF.k1 * 64 * 16, "conv1 fragments");
    u32x4* a1 = reinterpret_cast<u32x4*>(smem + Cfg::OFF_A1);
    for (int i = threadIdx.x; i < LF.nct * LF.k1 * 64; i += NT) a1[i] = frags[LF.off1 * 64 + i];
  }

  // The extra zero site of the site-major slots and of g_o: cleared once, never
  // written afterwards (every later store goes to a lattice site or its mirror).
  {
    HT* z0 = reinterpret_cast<HT*>(smem + M::OFF_S0);
    HT* z1 = reinterpret_cast<HT*>(smem + M::OFF_S1);
    HT* z2 = reinterpret_cast<HT*>(smem + (BF16 ? M::OFF_S2 : M::OFF_S1));
    for (int q = threadIdx.x; q < C; q += NT)
      z0[LY::template off<C>(LY::ZS, q)] = HT(0), z1[LY::template off<C>(LY::ZS, q)] = HT(0),
      z2[LY::template off<C>(LY::ZS, q)] = HT(0);
    if (threadIdx.x < (BF16 ? 1 : 2))
      reinterpret_cast<uint32_t*>(smem + M::OFF_GOS)[LY::ZS * (BF16 ? 1 : 2) + threadIdx.x] = 0u;
  }
  // site-major activations: h1 in S0, h2 in S1
  HT* h1s = reinterpret_cast<HT*>(smem + M::OFF_S0);
  HT* h2s = reinterpret_cast<HT*>(smem + M::OFF_S1);
  // HS: sample bb's saved h2 copied into S1 while the previous sample's tail
  // passes (dW1, conv1^T), the staging and conv1 run; S1 is free from the end of
  // conv2^T until conv1's barrier (conv1 gathers its operands from the field)
  using HSv = HSave<DIM, L, C, BF16>;
  static_assert(!HS || (HSv::ok && !LY::padded && LY::quad_major), "saved h2 image = LDS slot");
  auto load_h2 = [&](int bb) {
    if constexpr (HS) {
      if (bb < B) load_h2_async<HSv, NW>(hsv + (size_t)bb * HSv::sample_bytes, smem + M::OFF_S1, LY::QSZ * 4, w, lane);
    }
  };

  constexpr int NTL3 = Cfg::NTL3, NTL1 = Cfg::NTL1;
  f32x4 acc3[Cfg::I3], acc2[Cfg::I2], acc1[Cfg::I1];
#pragma unroll
  for (int i = 0; i < Cfg::I3; ++i) acc3[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < Cfg::I2; ++i) acc2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < Cfg::I1; ++i) acc1[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kc0 = w * NKC / NW, kc1 = (w + 1) * NKC / NW;  // this wave's K chunks
  float db3s = 0.f, db3t = 0.f;
  f32x4 db2[LF.nct], db1[LF.nct];
#pragma unroll
  for (int ct = 0; ct < LF.nct; ++ct) db2[ct] = db1[ct] = f32x4{0.f, 0.f, 0.f, 0.f};

  // 2D: a sample's x (in layout LY) and g_y are loaded into registers while the
  // previous sample is still being processed, so staging them is LDS writes
  // only.  3D shapes have no registers to spare and load them when staging.
  constexpr bool PF = DIM == 2;
  constexpr bool GYL = !Cfg::SPLIT;  // g_y staged in LDS (SPLIT: read from L2 where used)
  constexpr int NPX = PF ? (VS + NT - 1) / NT : 1, NPG = PF && GYL ? (V / 4 + NT - 1) / NT : 1;
  float pfx[NPX];
  f32x4 pfg[NPG];
  // HS: the wave's s values of the next sample (one active site per lane; one
  // 64-site group per wave)
  constexpr int NGS = (V / 2 + 63) / 64;
  static_assert(!HS || NGS == NW, "one group of active sites per wave");
  float pfs = 0.f;
  auto prefetch = [&](int bb) {
    if (bb >= B) return;
    if constexpr (HS) pfs = hss[(size_t)bb * (V / 2) + w * 64 + lane];
    const size_t s0 = (size_t)bb * V;
#pragma unroll
    for (int i = 0; i < NPX; ++i) {
      const int q = threadIdx.x + i * NT;
      pfx[i] = q < VS ? xin[s0 + LY::site_of(q)] : 0.f;
    }
    if constexpr (GYL) {
#pragma unroll
      for (int i = 0; i < NPG; ++i) {
        const int q = threadIdx.x + i * NT;
        pfg[i] = q < V / 4 ? reinterpret_cast<const f32x4*>(gy + s0)[q] : f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };
  if constexpr (PF) prefetch(blockIdx.x);
  // the hidden convolutions' biases, the same for every sample of the launch: held
  // in registers (2D; the 3D shapes have none to spare and reload them per pass)
  constexpr bool HB = DIM == 2;
  f32x4 hb1[LF.nct], hb2[LF.nct];
#pragma unroll
  for (int ct = 0; ct < LF.nct; ++ct) {
    hb1[ct] = HB ? load_bias4<C>(pl + off_b1, ct, j) : f32x4{};
    hb2[ct] = HB ? load_bias4<C>(pl + off_b2, ct, j) : f32x4{};
  }
  // the previous launch's (next layer's) weight gradient, while the prefetch is in flight
  if (prev_partial) grid_reduce<NT>(prev_partial, prev_out, n_parts, Cfg::P_LAYER);
  // the first sample's h2, issued once the prefetched values have landed (the
  // reduction above has waited for them already where it ran), so that staging
  // them does not wait for the copy
  if constexpr (HS) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  load_h2(blockIdx.x);

  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    // Weight fragments are reloaded per phase (from LDS, or L1/L2 hits) rather than
    // kept live across the whole sample loop, which would need every phase's
    // registers at once.
    asm volatile("" ::: "memory");
    const size_t sb = (size_t)b * V;
    // cotangent of the log-det: one for all samples, or this sample's
    const float gld = g_ld_vec ? (float)(-g_ld_vec[b]) : g_ld;
    // stage x and g_y; BF16: masked field channel-major for dW1
    if constexpr (PF) {
#pragma unroll
      for (int i = 0; i < NPX; ++i)
        if (threadIdx.x + i * NT < VS) xs[threadIdx.x + i * NT] = pfx[i];
      if constexpr (GYL) {
#pragma unroll
        for (int i = 0; i < NPG; ++i)
          if (threadIdx.x + i * NT < V / 4) reinterpret_cast<f32x4*>(gys)[threadIdx.x + i * NT] = pfg[i];
      }
    } else {
      for (int q = threadIdx.x; q < VS; q += NT) xs[q] = xin[sb + LY::site_of(q)];
      for (int q = threadIdx.x; q < V / 4; q += NT)
        reinterpret_cast<f32x4*>(gys)[q] = reinterpret_cast<const f32x4*>(gy + sb)[q];
    }
    if constexpr (HS)
      lds_barrier();
    else
      __syncthreads();
    // masked field, channel-major, for dW1 (SPLIT: built after dW3, over g_o's rows)
    auto build_h0c = [&]() {
      uint16_t* h0c = reinterpret_cast<uint16_t*>(smem + M::OFF_H0C);
      for (int n = threadIdx.x; n < V; n += NT)
        h0c[n] = (uint16_t)bf16_bits(G::parity(n) == fpar ? xs[LY::idx(n)] : 0.f);
    };
    if constexpr (BF16 && !Cfg::SPLIT) build_h0c();
    // conv1 operands (row triples of the masked field) in the (not yet written) h2
    // slot; HS: gathered from the field by every tile
    if constexpr (!HS && !Cfg::PS1) {
      build_tri<LY, BF16, NT>(h2s, xs, fpar);
      __syncthreads();
    }
    // ---- recompute conv1 -> h1 ----
    if constexpr (Cfg::PS1) {
      // the frozen half's tiles with the even taps, then the active half's with the
      // odd ones: fragment block c holds the taps 2 i + c, MFMA r takes k = 4 r + j
      // (tap 2 (4 r + j) + c), so K = 5 needs two MFMAs and K = 4 one
      static_for<0, 2>([&](auto CK) {
        constexpr int c = decltype(CK)::value;
        const int par = c == 0 ? fpar : apar;
        u32x4 A[LF.nct][1];
        f32x4 bias1[LF.nct];
#pragma unroll
        for (int ct = 0; ct < LF.nct; ++ct) {
          bias1[ct] = HB ? hb1[ct] : load_bias4<C>(pl + off_b1, ct, j);
          A[ct][0] = Cfg::A1L ? a1s[(ct * LF.k1 + c) * 64 + lane] : fr[(LF.off1 + ct * LF.k1 + c) * 64];
        }
        mma_tiles<Cfg::TU, LF.nct, 1, false, c == 0 ? 2 : 1>(
            V / 32, w, NW, A, bias1,
            [&](int tile, int) {
              const int n = G::half_site(tile * 16 + m, par), p = LY::idx(n);
              u32x4 bop;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int t = 2 * (4 * r + j) + c;
                const bool ok = t < T;
                bop[r] = __float_as_uint(xs[LY::nbr(n, p, ok ? t : c, 1)] * (ok ? 1.f : 0.f));
              }
              return bop;
            },
            [&](int tile, const f32x4(&acc)[LF.nct]) {
              const int p = LY::idx(G::half_site(tile * 16 + m, par));
#pragma unroll
              for (int ct = 0; ct < LF.nct; ++ct) {
                const int c0 = ct * 16 + 4 * j;
                if (c0 < C) {
                  f32x4 v;
#pragma unroll
                  for (int i = 0; i < 4; ++i) v[i] = leaky(acc[ct][i]);
                  *reinterpret_cast<f32x4*>(h1s + LY::template off<C>(p, c0)) = v;
                }
              }
            });
      });
    } else {
      u32x4 A[LF.nct][LF.k1];
      f32x4 bias1[LF.nct];
#pragma unroll
      for (int ct = 0; ct < LF.nct; ++ct) {
        bias1[ct] = HB ? hb1[ct] : load_bias4<C>(pl + off_b1, ct, j);
#pragma unroll
        for (int c = 0; c < LF.k1; ++c)
          A[ct][c] = Cfg::A1L ? a1s[(ct * LF.k1 + c) * 64 + lane] : fr[(LF.off1 + ct * LF.k1 + c) * 64];
      }
      mma_tiles<Cfg::TU, LF.nct, LF.k1, BF16, k_tri(T), true>(
          V / 16, w, NW, A, bias1,
          [&](int tile, int c) {
            if constexpr (HS) {
              const int n = tile * 16 + m;
              return gather_tri_x<LY, BF16>(xs, n, LY::idx(n), G::parity(n), fpar, c, j);
            } else {
              return gather_tri<LY, BF16>(h2s, tile * 16 + m, tile_p<LY>(tile, m), c, j);
            }
          },
          [&](int tile, const f32x4(&acc)[LF.nct]) {
#pragma unroll
            for (int ct = 0; ct < LF.nct; ++ct) store_act_tile<LY, C, BF16, false>(h1s, tile, m, ct, j, acc[ct]);
          });
    }
    // HS: the saved h2 has landed in S1 (the barrier publishes it)
    if constexpr (HS) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if constexpr (LY::padded) {
      fill_halo<LY, C, BF16, NT>(h1s);
      __syncthreads();
    }
    // ---- recompute conv2 -> h2 (HS: saved) ----
    if constexpr (!HS) {
      u32x4 A[LF.nct][LF.k2];
      f32x4 bias2[LF.nct];
#pragma unroll
      for (int ct = 0; ct < LF.nct; ++ct) {
        bias2[ct] = HB ? hb2[ct] : load_bias4<C>(pl + off_b2, ct, j);
#pragma unroll
        for (int c = 0; c < LF.k2; ++c) A[ct][c] = fr[(LF.off2 + ct * LF.k2 + c) * 64];
      }
      mma_tiles<Cfg::TU, LF.nct, LF.k2, BF16>(
          V / 16, w, NW, A, bias2,
          [&](int tile, int c) {
            return gather_h<LY, C, BF16>(h1s, tile * 16 + m, tile_p<LY>(tile, m), c, j);
          },
          [&](int tile, const f32x4(&acc)[LF.nct]) {
#pragma unroll
            for (int ct = 0; ct < LF.nct; ++ct) store_act_tile<LY, C, BF16, false>(h2s, tile, m, ct, j, acc[ct]);
          });
      __syncthreads();
    }
    fill_halo<LY, C, BF16, NT>(h2s);
    // ---- recompute conv3 at active sites; affine backward -> g_o, g_x(active) ----
    // g_o is zero at the frozen sites.
    uint32_t* gos_b = reinterpret_cast<uint32_t*>(smem + M::OFF_GOS);  // BF16 pairs, layout LY
    float* gos_f = reinterpret_cast<float*>(smem + M::OFF_GOS);        // FP32 pairs, layout LY
    uint16_t* goc = reinterpret_cast<uint16_t*>(smem + M::OFF_GOC);     // BF16 [2][CSTR]
    for (int q = threadIdx.x; q < V / 2; q += NT) {
      const int n = G::half_site(q, fpar);
      if constexpr (BF16) {
        LY::copies(n, [&](int pp) { gos_b[pp] = 0u; });
        goc[n] = 0;
        goc[CSTR + n] = 0;
      } else {
        LY::copies(n, [&](int pp) {
          gos_f[2 * pp] = 0.f;
          gos_f[2 * pp + 1] = 0.f;
        });
      }
    }
    // (the zeros go to frozen sites, the affine backward below writes active ones;
    // the barrier publishes h2's halo)
    if constexpr (LY::padded) __syncthreads();
    {
      // affine backward at active site n from conv3's s pre-activation o0
      // (is_s: o0 already is s)
      auto affine_bwd = [&](int n, float o0, bool is_s = false) {
        const int p = LY::idx(n);
        const float s = is_s ? o0 : final_tanh ? fast_tanh(o0) : o0;
        const float es = fast_exp(s);
        const float g = GYL ? gys[n] : gy[sb + n];
        const float gs = g * xs[p] * es + gld;
        const float go0 = final_tanh ? gs * (1.f - s * s) : gs;
        db3s += go0;
        db3t += g;
        gx[sb + n] = g * es;
        if constexpr (BF16) {
          const uint32_t pr = pack_bf16(go0, g);
          LY::copies(n, [&](int pp) { gos_b[pp] = pr; });
          goc[n] = (uint16_t)pr;
          goc[CSTR + n] = (uint16_t)(pr >> 16);
        } else {
          LY::copies(n, [&](int pp) {
            gos_f[2 * pp] = go0;
            gos_f[2 * pp + 1] = g;
          });
        }
      };
      const float bs = pl[off_b3];
      if constexpr (HS) {
        // s saved by the forward (prefetched), one active site per lane
        const int a = w * 64 + lane;
        const float s = pfs;
        if (a < V / 2) affine_bwd(G::half_site(a, apar), s, true);
      } else if constexpr (!BF16) {
        // 64 active sites per wave pass, one per lane (4x4 blocks: o0 in register 0)
        constexpr int NG = (V / 2 + 63) / 64;
        const f32x4 b3{bs, 0.f, 0.f, 0.f};
        for (int gi = w; gi < NG; gi += NW) {
          const int a = gi * 64 + lane;
          const bool valid = a < V / 2;
          const int n = G::half_site(valid ? a : 0, apar), p = LY::idx(n);
          const f32x4 o = quad_conv<LF.k3, 4>(qt + (lane & 3), b3,
                                              [&](int q) { return gather_q<LY, C>(h2s, n, p, q); });
          if (valid) affine_bwd(n, o[0]);
        }
      } else if constexpr (Cfg::QU3 == 2) {
        // two tiles with the plain fragments; tile 1's s moves from lane group 0 to
        // lane group 1, so the affine backward runs once on two lane groups
        u32x4 A[LF.k2];
#pragma unroll
        for (int c = 0; c < LF.k2; ++c) A[c] = fr[(LF.off3 + c) * 64];
        constexpr int NT3 = V / 32;
        for (int t0 = w; t0 < NT3; t0 += 2 * NW) {
          const int n0 = G::half_site(t0 * 16 + m, apar);
          const int n1 = G::half_site((t0 + NW < NT3 ? t0 + NW : t0) * 16 + m, apar);
          f32x4 a0{bs, 0.f, 0.f, 0.f}, a1{bs, 0.f, 0.f, 0.f};
#pragma unroll
          for (int c = 0; c < LF.k2; ++c) {
            const u32x4 g0 = gather_h<LY, C, BF16>(h2s, n0, LY::idx(n0), c, j);
            const u32x4 g1 = gather_h<LY, C, BF16>(h2s, n1, LY::idx(n1), c, j);
            a0 = mma<BF16>(A[c], g0, a0);
            a1 = mma<BF16>(A[c], g1, a1);
          }
          const float o1 = __shfl(a1[0], m, 64);  // row 0 of tile 1, from lane m
          const float o0 = j == 0 ? a0[0] : o1;
          if (j < 2 && t0 + j * NW < NT3) affine_bwd(j == 0 ? n0 : n1, o0);
        }
      } else if constexpr (Cfg::QU3 == 4) {
        // four tiles share an accumulator (outputs of tile u at rows 4u, 4u+1), so
        // the affine backward runs on all 64 lanes, group j for tile j; one chain
        // per pair of tiles
        constexpr int QU = 4;
        u32x4 A[QU][LF.k2];
#pragma unroll
        for (int c = 0; c < LF.k2; ++c) {
          A[0][c] = fr[(LF.off3 + c) * 64];
#pragma unroll
          for (int u = 1; u < QU; ++u) A[u][c] = fr[(LF.off3q + (u - 1) * LF.k2 + c) * 64];
        }
        constexpr int NT3 = V / 32;
        for (int t0 = w; t0 < NT3; t0 += QU * NW) {
          int nq[QU];
#pragma unroll
          for (int u = 0; u < QU; ++u) nq[u] = G::half_site((t0 + u * NW < NT3 ? t0 + u * NW : t0) * 16 + m, apar);
          f32x4 acc[QU / 2];
#pragma unroll
          for (int h = 0; h < QU / 2; ++h) acc[h] = f32x4{h == 0 ? bs : 0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int c = 0; c < LF.k2; ++c) {
            u32x4 gq[QU];
#pragma unroll
            for (int u = 0; u < QU; ++u) gq[u] = gather_h<LY, C, BF16>(h2s, nq[u], LY::idx(nq[u]), c, j);
#pragma unroll
            for (int u = 0; u < QU; ++u) acc[u / 2] = mma<BF16>(A[u][c], gq[u], acc[u / 2]);
          }
          float o0 = acc[0][0];
#pragma unroll
          for (int h = 1; h < QU / 2; ++h) o0 += acc[h][0];
          if (j < QU && t0 + j * NW < NT3) affine_bwd(G::half_site((t0 + j * NW) * 16 + m, apar), o0);
        }
      } else {
        u32x4 A[1][LF.k2];
#pragma unroll
        for (int c = 0; c < LF.k2; ++c) A[0][c] = fr[(LF.off3 + c) * 64];
        const f32x4 b3[1] = {f32x4{bs, 0.f, 0.f, 0.f}};
        mma_tiles<Cfg::TU, 1, LF.k2, BF16>(
            V / 32, w, NW, A, b3,
            [&](int tile, int c) {
              const int n = G::half_site(tile * 16 + m, apar);
              return gather_h<LY, C, BF16>(h2s, n, LY::idx(n), c, j);
            },
            [&](int tile, const f32x4(&acc3r)[1]) {
              if (j == 0) affine_bwd(G::half_site(tile * 16 + m, apar), acc3r[0][0]);
            });
      }
    }
    __syncthreads();
    // ---- dW3[co][ci][tap] += sum_m h2[m][ci] g_o[m - delta_tap][co] ----
    // tiles (mt, nt): rows ci = mt*16 + i, columns (tap, co) = nt*16 + m
    // FP32 and SPLIT write g_a2 over h2, which dW3 reads, so dW3 goes first; the
    // other BF16 layouts keep them apart and run dW3 after conv3^T, next to g_a2's
    // halo fill.
    // PS3: the two halves of the sites (kind 0: active, kind 1: frozen), 16-site
    // chunks of each split evenly over the waves; column m of tile (mt, kind) is
    // (tap, co) = (2 (m >> 1) + kind, m & 1)
    auto dw3_ps = [&]() {
      constexpr int KH = V / 32;
      static_for<0, 2>([&](auto KIND) {
        constexpr int kind = decltype(KIND)::value;
        const int par = apar ^ kind;
        const int tap = 2 * (m >> 1) + kind, co = m & 1;
        const bool tv = tap < T;
        const int tc = tv ? tap : kind;
        const float tm = tv ? 1.f : 0.f;
#pragma unroll 1
        for (int kc = w * KH / NW; kc < (w + 1) * KH / NW; ++kc) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int sx = G::half_site(kc * 16 + 4 * j + r, par), px = LY::idx(sx);
            const float bb = load1_shift<LY, 2>(gos_f, sx, co, tc, -1) * tm;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
              const int ci = mt * 16 + m;
              const float a = ci < C ? h2s[LY::template off<C>(px, ci)] : 0.f;
              acc3[mt * 2 + kind] = mfma(a, bb, acc3[mt * 2 + kind]);
            }
          }
        }
      });
    };
    auto dw3 = [&]() {
#pragma unroll(Cfg::DWU3)
      for (int kc = kc0, kk_ = 0; kk_ < (Cfg::KEXACT ? Cfg::KPW : kc1 - kc0); ++kk_, ++kc) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int ci = mt * 16 + m;
          if constexpr (BF16) {
            const int s0 = kc * 32 + 8 * j;
            const u32x4 a = load_tr8<LY, C, 1>(h2s, s0, mt * 16, -1, m);
#pragma unroll
            for (int nt = 0; nt < NTL3; ++nt) {
              const int col = nt * 16 + m, tap = col >> 1, co = col & 1;
              // branch-free: columns past the taps read tap 0 and select zero
              const u32x4 bv = load8_shift<DIM, L>(goc + co * CSTR, s0, tap < T ? tap : 0, -1);
              const u32x4 bb = tap < T ? bv : u32x4{0u, 0u, 0u, 0u};
              acc3[mt * NTL3 + nt] = mfma(as_bf16x8(a), as_bf16x8(bb), acc3[mt * NTL3 + nt]);
            }
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int sx = kc * 16 + 4 * j + r;
              const float a = ci < C ? h2s[LY::template off<C>(LY::idx(sx), ci)] : 0.f;
#pragma unroll
              for (int nt = 0; nt < NTL3; ++nt) {
                const int col = nt * 16 + m, tap = col >> 1, co = col & 1;
                const float bb = tap < T ? load1_shift<LY, 2>(gos_f, sx, co, tap, -1) : 0.f;
                acc3[mt * NTL3 + nt] = mfma(a, bb, acc3[mt * NTL3 + nt]);
              }
            }
          }
        }
      }
    };
    if constexpr (Cfg::PS3) {
      dw3_ps();
      __syncthreads();
    } else if constexpr (!BF16 || Cfg::SPLIT) {
      dw3();
      __syncthreads();
    }
    // ---- conv3^T: g_a2 = leaky'(h2) (W3^T * g_o) ----
    // BF16: into S2 (3D also channel-major into S3); FP32 and SPLIT: in place over h2.
    HT* ga2s = BF16 && !Cfg::SPLIT ? reinterpret_cast<HT*>(smem + M::OFF_S2) : h2s;
    uint16_t* ga2c = reinterpret_cast<uint16_t*>(smem + M::OFF_S3);
    if constexpr (Cfg::SPLIT) build_h0c();  // over g_o's channel-major rows, dead after dW3
    if constexpr (Cfg::PS3) {
      // the active half's tiles with the even taps (MFMA r: k = 4 r + j, (tap, co) =
      // (2 (2 r + (j >> 1)) + kind, j & 1); k < 10: three MFMAs), then the frozen
      // half's with the odd taps (k < 8: two)
      const f32x4 zero[LF.nct] = {};
      static_for<0, 2>([&](auto KIND) {
        constexpr int kind = decltype(KIND)::value;
        const int par = apar ^ kind;
        u32x4 A[LF.nct][1];
#pragma unroll
        for (int ct = 0; ct < LF.nct; ++ct) A[ct][0] = fr[(Cfg::OFF3T + ct * Cfg::KT3 + kind) * 64];
        mma_tiles<Cfg::TU, LF.nct, 1, false, kind ? 2 : 3>(
            V / 32, w, NW, A, zero,
            [&](int tile, int) {
              const int n = G::half_site(tile * 16 + m, par), p = LY::idx(n);
              u32x4 bop;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int t = 2 * (2 * r + (j >> 1)) + kind;
                const int nb = t < T ? LY::nbr(n, p, t, -1) : LY::ZS;
                bop[r] = __float_as_uint(gos_f[2 * nb + (j & 1)]);
              }
              return bop;
            },
            [&](int tile, const f32x4(&acc)[LF.nct]) {
              const int p = LY::idx(G::half_site(tile * 16 + m, par));
#pragma unroll
              for (int ct = 0; ct < LF.nct; ++ct) {
                const int c0 = ct * 16 + 4 * j;
                if (c0 < C) {
                  const f32x4 hh = *reinterpret_cast<const f32x4*>(h2s + LY::template off<C>(p, c0));
                  f32x4 v;
#pragma unroll
                  for (int i = 0; i < 4; ++i) v[i] = acc[ct][i] * leaky_grad_from_out(hh[i]);
                  *reinterpret_cast<f32x4*>(ga2s + LY::template off<C>(p, c0)) = v;
#pragma unroll
                  for (int i = 0; i < 4; ++i) db2[ct][i] += v[i];
                }
              }
            });
      });
    } else {
      u32x4 A[LF.nct][Cfg::KT3];
#pragma unroll
      for (int ct = 0; ct < LF.nct; ++ct)
#pragma unroll
        for (int c = 0; c < Cfg::KT3; ++c) A[ct][c] = fr[(Cfg::OFF3T + ct * Cfg::KT3 + c) * 64];
      const f32x4 zero[LF.nct] = {};
      mma_tiles<Cfg::TU, LF.nct, Cfg::KT3, BF16, 2 * T>(
          V / 16, w, NW, A, zero,
          [&](int tile, int c) {
            const int n = tile * 16 + m, p = tile_p<LY>(tile, m);
            u32x4 bop;
            if constexpr (BF16) {
              const int t0 = (32 * c + 8 * j) / 2;
#pragma unroll
              for (int q = 0; q < 4; ++q)
                bop[q] = gos_b[t0 + q < T ? LY::nbr(n, p, t0 + q, -1) : LY::ZS];
            } else {
              const int t0 = (16 * c + 4 * j) / 2;
#pragma unroll
              for (int q = 0; q < 2; ++q) {
                const int t = t0 + q;
                const int nb = t < T ? LY::nbr(n, p, t, -1) : LY::ZS;
                bop[2 * q] = __float_as_uint(gos_f[2 * nb]);
                bop[2 * q + 1] = __float_as_uint(gos_f[2 * nb + 1]);
              }
            }
            return bop;
          },
          [&](int tile, const f32x4(&acc)[LF.nct]) {
            const int n = tile * 16 + m, p = tile_p<LY>(tile, m);
#pragma unroll
            for (int ct = 0; ct < LF.nct; ++ct) {
              const int c0 = ct * 16 + 4 * j;
              if (c0 < C) {
                float v[4];
                if constexpr (BF16) {
                  const u32x2 hv = *reinterpret_cast<const u32x2*>(h2s + p * C + c0);
                  const float hh[4] = {bf16_lo(hv[0]), bf16_hi(hv[0]), bf16_lo(hv[1]), bf16_hi(hv[1])};
#pragma unroll
                  for (int i = 0; i < 4; ++i) v[i] = acc[ct][i] * leaky_grad_from_out(hh[i]);
                  const u32x2 gv = store4_tile<LY, C, BF16, false>(ga2s, tile, m, c0, v);
                  if constexpr (M::CM2) store_cm4<C, CSTR>(ga2c, n, c0, gv);
                } else {
                  const f32x4 hh = *reinterpret_cast<const f32x4*>(h2s + LY::template off<C>(p, c0));
#pragma unroll
                  for (int i = 0; i < 4; ++i) v[i] = acc[ct][i] * leaky_grad_from_out(hh[i]);
                  store4_tile<LY, C, BF16, false>(ga2s, tile, m, c0, v);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) db2[ct][i] += v[i];
              }
            }
          });
    }
    __syncthreads();
    // g_a2's halo, and BF16 (but SPLIT) dW3; nothing to do for unpadded FP32 and SPLIT
    if constexpr (LY::padded || (BF16 && !Cfg::SPLIT)) {
      fill_halo<LY, C, BF16, NT>(ga2s);
      if constexpr (BF16 && !Cfg::SPLIT) dw3();
      __syncthreads();
    }
    // ---- dW2[co][ci][tap] += sum_m h1[m][ci] g_a2[m - delta_tap][co] ----
    // tiles (mt, tap, nt): rows ci = mt*16 + i, columns co = nt*16 + m; the taps are
    // unrolled so each shift is known at compile time.
#pragma unroll 1
    for (int kc = kc0, kk_ = 0; kk_ < (Cfg::KEXACT ? Cfg::KPW : kc1 - kc0); ++kk_, ++kc) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int ci = mt * 16 + m;
        if constexpr (BF16) {
          const int s0 = kc * 32 + 8 * j;
          const u32x4 a = load_tr8<LY, C, 1>(h1s, s0, mt * 16, -1, m);
          const int x0 = s0 % L;
          static_for<0, T>([&](auto tc) {
            constexpr int TAP = decltype(tc)::value;
            constexpr int E = -tap_dc<DIM, TAP, DIM - 1>();
            const int rowS = shifted_row_c<DIM, L, TAP, -1>(s0);
#pragma unroll
            for (int nt = 0; nt < MT; ++nt) {
              u32x4 bb;
              if constexpr (M::CM2) {
                const int co = nt * 16 + m;
                bb = co < C ? load8_e<L, E>(ga2c + co * CSTR + rowS * L, x0) : u32x4{0u, 0u, 0u, 0u};
              } else {
                bb = load_tr8<LY, C, -1>(ga2s, s0, nt * 16, TAP, m);
              }
              acc2[(mt * T + TAP) * MT + nt] = mfma(as_bf16x8(a), as_bf16x8(bb), acc2[(mt * T + TAP) * MT + nt]);
            }
          });
        } else if constexpr (DIM == 2 && LY::quad_major && !LY::padded && L % 16 == 0 && C == 16) {
          // A 16-site chunk lies in one row: the lane's four sites x0 .. x0 + 3 and,
          // per tap row, the six columns x0 - 1 .. x0 + 4 they reach, read once each
          // (four sites of one channel are 16 bytes apart, so the middle four are two
          // paired reads; only the two edge columns wrap)
          const int y = (kc * 16) / L, x0 = (kc * 16) % L + 4 * j;
          const float* ap = h1s + LY::template off<C>(y * L + x0, m);
          const float av[4] = {ap[0], ap[4], ap[8], ap[12]};
          static_for<0, 3>([&](auto DY) {
            constexpr int dyi = decltype(DY)::value;  // taps 3 dyi .. 3 dyi + 2: row offset dyi - 1
            const int rs = ((y - (dyi - 1)) & (L - 1)) * L;
            const float* bp = ga2s + LY::template off<C>(rs + x0, m);
            const float bv[6] = {ga2s[LY::template off<C>(rs + ((x0 - 1) & (L - 1)), m)], bp[0], bp[4], bp[8], bp[12],
                                 ga2s[LY::template off<C>(rs + ((x0 + 4) & (L - 1)), m)]};
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int dxi = 0; dxi < 3; ++dxi) {
                // site x0 + r minus the tap's column offset dxi - 1: column index r - dxi + 2 of bv
                acc2[3 * dyi + dxi] = mfma(av[r], bv[r - dxi + 2], acc2[3 * dyi + dxi]);
              }
          });
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int sx = kc * 16 + 4 * j + r, px = LY::idx(sx);
            const float a = ci < C ? h1s[LY::template off<C>(px, ci)] : 0.f;
            static_for<0, T>([&](auto tc) {
              constexpr int TAP = decltype(tc)::value;
              const int nb = LY::nbr(sx, px, TAP, -1);
#pragma unroll
              for (int nt = 0; nt < MT; ++nt) {
                const int co = nt * 16 + m;
                const float bb = co < C ? ga2s[LY::template off<C>(nb, co)] : 0.f;
                acc2[(mt * T + TAP) * MT + nt] = mfma(a, bb, acc2[(mt * T + TAP) * MT + nt]);
              }
            });
          }
        }
      }
    }
    __syncthreads();
    // ---- conv2^T: g_a1 = leaky'(h1) (W2^T * g_a2) ----
    // BF16: into S1 (h2 is dead); FP32 and SPLIT: in place over h1.
    HT* ga1s = BF16 && !Cfg::SPLIT ? reinterpret_cast<HT*>(smem + M::OFF_S1) : h1s;
    {
      u32x4 A[LF.nct][LF.k2];
#pragma unroll
      for (int ct = 0; ct < LF.nct; ++ct)
#pragma unroll
        for (int c = 0; c < LF.k2; ++c) A[ct][c] = fr[(Cfg::OFF2T + ct * LF.k2 + c) * 64];
      // next sample's inputs: issued after this phase's fragment loads, so only
      // the next phase's fragment loads wait for them
      if constexpr (PF) prefetch(b + gridDim.x);
      const f32x4 zero[LF.nct] = {};
      mma_tiles<Cfg::TU, LF.nct, LF.k2, BF16>(
          V / 16, w, NW, A, zero,
          [&](int tile, int c) {
            return gather_h<LY, C, BF16, -1>(ga2s, tile * 16 + m, tile_p<LY>(tile, m), c, j);
          },
          [&](int tile, const f32x4(&acc)[LF.nct]) {
            const int n = tile * 16 + m, p = tile_p<LY>(tile, m);
#pragma unroll
            for (int ct = 0; ct < LF.nct; ++ct) {
              const int c0 = ct * 16 + 4 * j;
              if (c0 < C) {
                float v[4];
                if constexpr (BF16) {
                  const u32x2 hv = *reinterpret_cast<const u32x2*>(h1s + p * C + c0);
                  const float hh[4] = {bf16_lo(hv[0]), bf16_hi(hv[0]), bf16_lo(hv[1]), bf16_hi(hv[1])};
#pragma unroll
                  for (int i = 0; i < 4; ++i) v[i] = acc[ct][i] * leaky_grad_from_out(hh[i]);
                  store4_tile<LY, C, BF16, false>(ga1s, tile, m, c0, v);
                } else {
                  const f32x4 hh = *reinterpret_cast<const f32x4*>(h1s + LY::template off<C>(p, c0));
#pragma unroll
                  for (int i = 0; i < 4; ++i) v[i] = acc[ct][i] * leaky_grad_from_out(hh[i]);
                  store4_tile<LY, C, BF16, false>(ga1s, tile, m, c0, v);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) db1[ct][i] += v[i];
              }
            }
          });
    }
    __syncthreads();
    // S1 (g_a2) is dead from here on.  The vector-memory loads still in flight
    // (weight fragments) are waited for before the copy is issued: a later wait
    // for any of them would otherwise also wait for the whole copy.
    if constexpr (HS) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    load_h2(b + gridDim.x);
    // g_a1's halo (for conv1^T's gathers) is filled alongside dW1, which reads
    // interior sites only
    fill_halo<LY, C, BF16, NT>(ga1s);
    // ---- dW1[c][tap] += sum_n g_a1[n][c] h0[n + delta_tap] (h0 = mask_F x) ----
    // tiles (mt, nt): rows c = mt*16 + i, columns tap = nt*16 + m
    {
      const uint16_t* h0c = reinterpret_cast<const uint16_t*>(smem + M::OFF_H0C);
#pragma unroll(HS || BF16 ? Cfg::DWU1 : (Cfg::DWU1 > 2 ? 2 : Cfg::DWU1))
      for (int kc = kc0, kk_ = 0; kk_ < (Cfg::KEXACT ? Cfg::KPW : kc1 - kc0); ++kk_, ++kc) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int c = mt * 16 + m;
          if constexpr (BF16) {
            const int s0 = kc * 32 + 8 * j;
            const u32x4 a = load_tr8<LY, C, 1>(ga1s, s0, mt * 16, -1, m);
#pragma unroll
            for (int nt = 0; nt < NTL1; ++nt) {
              const int tap = nt * 16 + m;
              const u32x4 bv = load8_shift<DIM, L>(h0c, s0, tap < T ? tap : 0, 1);  // branch-free
              const u32x4 bb = tap < T ? bv : u32x4{0u, 0u, 0u, 0u};
              acc1[mt * NTL1 + nt] = mfma(as_bf16x8(a), as_bf16x8(bb), acc1[mt * NTL1 + nt]);
            }
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int sx = kc * 16 + 4 * j + r, px = LY::idx(sx);
              const float a = c < C ? ga1s[LY::template off<C>(px, c)] : 0.f;
#pragma unroll
              for (int nt = 0; nt < NTL1; ++nt) {
                // branch-free: columns past the T taps read a valid neighbour and
                // multiply it by 0 (the field is finite; a select would be turned back
                // into a branch around the read), so the reads of the unrolled chunks
                // stay in flight together
                const int tap = nt * 16 + m, tc = tap < T ? tap : 0;
                const float xv = xs[LY::nbr(sx, px, tc, 1)];
                const float bb = xv * (tap < T && (G::parity(sx) ^ todd<DIM>(tc)) == fpar ? 1.f : 0.f);
                acc1[mt * NTL1 + nt] = mfma(a, bb, acc1[mt * NTL1 + nt]);
              }
            }
          }
        }
      }
    }
    // dW1 and conv1^T only read LDS (conv1^T needs g_a1's halo where there is one)
    if constexpr (LY::padded) __syncthreads();
    // ---- conv1^T at the frozen sites: g_x = g_y + W1^T * g_a1 ----
    // (3D through the shared tile pass, which also frees registers there; 2D keeps
    // the plain loop, measured faster at the 2D shapes)
    if constexpr (!BF16) {
      // FP32: 64 frozen sites per wave pass on the 4x4 blocks (g_h0 in register 0)
      constexpr int NG = (V / 2 + 63) / 64;
      const f32x4 zero{0.f, 0.f, 0.f, 0.f};
      for (int gi = w; gi < NG; gi += NW) {
        const int a = gi * 64 + lane;
        const bool valid = a < V / 2;
        const int n = G::half_site(valid ? a : 0, fpar), p = LY::idx(n);
        const f32x4 o = quad_conv<Cfg::K1T, 4>(qt + LF.k3 * 4 + (lane & 3), zero,
                                               [&](int q) { return gather_q<LY, C, -1>(ga1s, n, p, q); });
        if (valid) gx[sb + n] = gys[n] + o[0];
      }
    } else if constexpr (DIM == 2) {
      u32x4 A[LF.k2];
#pragma unroll
      for (int c = 0; c < LF.k2; ++c) A[c] = fr[(Cfg::OFF1T + c) * 64];
      for (int tile = w; tile < V / 32; tile += NW) {
        const int n = G::half_site(tile * 16 + m, fpar), p = LY::idx(n);
        f32x4 acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < LF.k2; ++c)
          acc = mma<BF16>(A[c], gather_h<LY, C, BF16, -1>(ga1s, n, p, c, j), acc);
        if (j == 0) gx[sb + n] = (GYL ? gys[n] : gy[sb + n]) + acc[0];
      }
    } else {
      u32x4 A[1][LF.k2];
#pragma unroll
      for (int c = 0; c < LF.k2; ++c) A[0][c] = fr[(Cfg::OFF1T + c) * 64];
      const f32x4 zero[1] = {};
      mma_tiles<Cfg::TU, 1, LF.k2, BF16>(
          V / 32, w, NW, A, zero,
          [&](int tile, int c) {
            const int n = G::half_site(tile * 16 + m, fpar);
            return gather_h<LY, C, BF16, -1>(ga1s, n, LY::idx(n), c, j);
          },
          [&](int tile, const f32x4(&acc)[1]) {
            const int n = G::half_site(tile * 16 + m, fpar);
            if (j == 0) gx[sb + n] = gys[n] + acc[0][0];
          });
    }
    // SPLIT: the next sample's staging writes only the field, which the tail passes
    // (dW1, conv1^T) do not read; its first barrier comes before any other write
    if constexpr (HS)
      lds_barrier();
    else if constexpr (!Cfg::SPLIT)
      __syncthreads();
  }
  if constexpr (Cfg::SPLIT) __syncthreads();  // the partial sums below overwrite the sample state

  // ---- sum the waves' weight-gradient tiles in a fixed order, write the partial ----
  float* red = reinterpret_cast<float*>(smem);
  for (int i = threadIdx.x; i < Cfg::P_LAYER; i += NT) red[i] = 0.f;
  // bias partials: reduce over the 16 lanes that share j (and, for db3, over all lanes)
#pragma unroll
  for (int ct = 0; ct < LF.nct; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        db2[ct][i] += __shfl_xor(db2[ct][i], o, 64);
        db1[ct][i] += __shfl_xor(db1[ct][i], o, 64);
      }
  db3s = wave_sum(db3s);
  db3t = wave_sum(db3t);
  __syncthreads();
  for (int ww = 0; ww < NW; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTL3; ++nt) {
          const int col = nt * 16 + m, co = col & 1;
          const int tap = Cfg::PS3 ? 2 * (m >> 1) + nt : col >> 1;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int ci = mt * 16 + 4 * j + i;
            if (ci < C && tap < T) red[off_W3 + (co * C + ci) * T + tap] += acc3[mt * NTL3 + nt][i];
          }
        }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int tap = 0; tap < T; ++tap)
#pragma unroll
          for (int nt = 0; nt < MT; ++nt) {
            const int co = nt * 16 + m;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int ci = mt * 16 + 4 * j + i;
              if (ci < C && co < C)
                red[off_W2 + (co * C + ci) * T + tap] += acc2[(mt * T + tap) * MT + nt][i];
            }
          }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTL1; ++nt) {
          const int tap = nt * 16 + m;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = mt * 16 + 4 * j + i;
            if (c < C && tap < T) red[off_W1 + c * T + tap] += acc1[mt * NTL1 + nt][i];
          }
        }
      if (m == 0) {
#pragma unroll
        for (int ct = 0; ct < LF.nct; ++ct)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = ct * 16 + 4 * j + i;
            if (c < C) {
              red[off_b2 + c] += db2[ct][i];
              red[off_b1 + c] += db1[ct][i];
            }
          }
      }
      if (lane == 0) {
        red[off_b3] += db3s;
        red[off_b3 + 1] += db3t;
      }
    }
    __syncthreads();
  }
  float* out = partial + (size_t)blockIdx.x * Cfg::P_LAYER;
  for (int i = threadIdx.x; i < Cfg::P_LAYER; i += NT) out[i] = red[i];
}

// out[i] = sum over g of partial[g][i], fixed order: 32 parameters per block,
// ---- host -----------------------------------------------------------------

template <int DIM, int L, int C, bool BF16>
int bwd_grid(int B) {
  using Cfg = BwdCfg<DIM, L, C, BF16>;
  const int per_cu = std::max<int>(1, std::min<int>(8, (int)((160 * 1024) / Cfg::lds_bytes)));
  return std::min(B, num_cus() * per_cu);
}

template <int DIM, int L, int C, bool BF16>
size_t bwd_ws(const FlowGeom& g, int B) {
  using Cfg = BwdCfg<DIM, L, C, BF16>;
  const size_t frags = (size_t)Cfg::FRAGS * 64 * 16 * g.N;
  const size_t partial = (size_t)bwd_grid<DIM, L, C, BF16>(B) * Cfg::P_LAYER * 4;
  const size_t gbuf = (size_t)B * Cfg::V * 4;
  return align_up(frags) + 2 * align_up(partial) + 2 * align_up(gbuf);
}

template <int DIM, int L, int C, bool BF16>
int32_t launch_backward(const FlowGeom& g, const float* params, int B, const float* saved,
                        const float* hsave, const float* g_phi, double g_logq,
                        const double* g_logq_vec, float* g_params, float* g_z, char* ws,
                        hipStream_t st) {
  using Cfg = BwdCfg<DIM, L, C, BF16>;
  const int grid = bwd_grid<DIM, L, C, BF16>(B);
  const FragTable tab = bwd_table(g, BF16, Cfg::LF.x4, Cfg::LF.quad);
  if (tab.total != Cfg::FRAGS) return LFS_EDEVICE;  // the table and the kernel's offsets agree
  char* p = ws;
  u32x4* frags = reinterpret_cast<u32x4*>(p);
  p += align_up((size_t)Cfg::FRAGS * 64 * 16 * g.N);
  // two partial buffers: a launch reduces the previous launch's while writing its own
  float* partial[2] = {reinterpret_cast<float*>(p),
                       reinterpret_cast<float*>(p + align_up((size_t)grid * Cfg::P_LAYER * 4))};
  p += 2 * align_up((size_t)grid * Cfg::P_LAYER * 4);
  float* gbuf[2] = {reinterpret_cast<float*>(p),
                    reinterpret_cast<float*>(p + align_up((size_t)B * Cfg::V * 4))};
  const long nthreads = (long)tab.total * 64 * g.N;
  hipLaunchKernelGGL((kf_prep<BF16>), dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st,
                     params, g.N, g.T, (int)g.P_layer, tab, frags);
  using HSv = HSave<DIM, L, C, BF16>;
  if (!HSv::ok) hsave = nullptr;
  auto kern = kf_backward<DIM, L, C, BF16, Cfg::NT, false>;
  if constexpr (HSv::ok)
    if (hsave) kern = kf_backward<DIM, L, C, BF16, Cfg::NT, true>;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)Cfg::lds_bytes) !=
      hipSuccess)
    return LFS_EDEVICE;
  const size_t BV = (size_t)B * Cfg::V;
  const float* gy = g_phi;
  int which = 0;
  for (int l = g.N - 1; l >= 0; --l) {
    float* gx = gbuf[which];
    const bool first = l == g.N - 1;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(Cfg::NT), Cfg::lds_bytes, st,
                       frags + (size_t)l * tab.total * 64, params + (size_t)l * g.P_layer,
                       (int)g.off_b1, (int)g.off_b2, (int)g.off_b3, (int)g.off_W1, (int)g.off_W2,
                       (int)g.off_W3, g.frozen_parity(l), g.final_tanh, (float)(-g_logq), g_logq_vec, B,
                       saved + (size_t)l * BV, gy, gx, partial[l & 1],
                       first ? nullptr : (const float*)partial[(l + 1) & 1],
                       first ? nullptr : g_params + (size_t)(l + 1) * g.P_layer, grid,
                       hsave ? reinterpret_cast<const unsigned char*>(hsave) + (size_t)l * B * HSv::sample_bytes
                             : nullptr,
                       hsave ? hsave + HSv::s_off(g.N, B, l, 0) : nullptr);
    gy = gx;
    which ^= 1;
  }
  hipLaunchKernelGGL(kf_reduce, dim3((Cfg::P_LAYER + kRedCols - 1) / kRedCols),
                     dim3(kRedCols * kRedSlices), 0, st, grid, Cfg::P_LAYER,
                     (const float*)partial[0], g_params);
  if (g_z)
    hipLaunchKernelGGL(kf_gz, dim3((unsigned)((BV + 255) / 256)), dim3(256), 0, st, (int64_t)BV,
                       gy, saved, (float)g_logq, g_logq_vec, (int64_t)Cfg::V, g_z);
  return launch_status();
}

using BwdFn = int32_t (*)(const FlowGeom&, const float*, int, const float*, const float*,
                          const float*, double, const double*, float*, float*, char*, hipStream_t);
using BwdWsFn = size_t (*)(const FlowGeom&, int);

struct BwdEntry {
  int dim, L, C;
  bool bf16;
  BwdFn fn;
  BwdWsFn ws;
};

template <int DIM, int L, int C, bool BF16>
constexpr BwdEntry bwd_entry() {
  using Cfg = BwdCfg<DIM, L, C, BF16>;
  // dynamic LDS plus the static buffer of the in-kernel partial reduction
  static_assert(Cfg::lds_bytes + kRedSlices * (Cfg::NT / kRedSlices + 1) * 4 <= 160 * 1024,
                "LDS budget");
  return BwdEntry{DIM, L, C, BF16, &launch_backward<DIM, L, C, BF16>, &bwd_ws<DIM, L, C, BF16>};
}

// Training shapes with a fused backward (L a power of two, >= 8; the sample fits
// in LDS with both layouts in BF16 mode).
#define LFS_BWD_SHAPES(P) P(2, 8, 8) P(2, 8, 16) P(2, 16, 8) P(2, 16, 16) P(2, 32, 8) P(2, 32, 16) P(3, 8, 8) P(3, 8, 16)
#define LFS_B2(D, L, C) bwd_entry<D, L, C, false>(), bwd_entry<D, L, C, true>(),

const BwdEntry kBwdTable[] = {LFS_BWD_SHAPES(LFS_B2)};

const BwdEntry* find_bwd(const FlowGeom& g) {
  for (const auto& e : kBwdTable)
    if (e.dim == g.dim && e.L == g.L && e.C == g.C && e.bf16 == g.bf16()) return &e;
  return nullptr;
}

}  // namespace

bool bwd_supported(const FlowGeom& g) { return find_bwd(g) != nullptr; }
size_t bwd_ws_bytes(const FlowGeom& g, int B) {
  const BwdEntry* e = find_bwd(g);
  return e ? e->ws(g, B) : 0;
}
int32_t bwd_run(const FlowGeom& g, const float* params, int B, const float* saved,
                const float* hsave, const float* g_phi, double g_logq, const double* g_logq_vec,
                float* g_params, float* g_z, char* ws, hipStream_t st) {
  const BwdEntry* e = find_bwd(g);
  if (!e) return LFS_EUNSUPPORTED;
  return e->fn(g, params, B, saved, hsave, g_phi, g_logq, g_logq_vec, g_params, g_z, ws, st);
}

}  // namespace fused
}  // namespace lfs

// Fused backward of the coupling layers (paper Sec. 1: the gradient of the
// shifted reverse KL with respect to the network weights, z held fixed) for 3D
// lattices whose hidden activations do not fit LDS (L = 16, BF16 operands).
// Three kernels per layer, each streaming the planes of axis 0 through rings of
// three planes like the plane-streaming forward, with one workgroup per sample:
//
//   recompute  h1 = leaky(W1 * mask_F x), h2 = leaky(W2 * h1), s at the active
//              sites; affine backward: g_x(active) = g_y e^s,
//              g_o = (g_s (1 - s^2), g_t) (zero at the frozen sites), db3.
//              Writes h1, h2 channel-major and g_o as BF16 pairs.
//   transpose  g_a2 = leaky'(h2) (W3^T * g_o), g_a1 = leaky'(h1) (W2^T * g_a2),
//              g_x(frozen) = g_y + W1^T * g_a1; db2, db1.  Writes g_a2, g_a1
//              channel-major.  (The recompute also writes, per site, the sign
//              bits of h1 and h2 over the channels, which give leaky' here.)
//   weights    dW2[co][ci][t] = sum_m h1[m][ci] g_a2[m - d_t][co],
//              dW3[co][ci][t] = sum_m h2[m][ci] g_o[m - d_t][co],
//              dW1[c][t]      = sum_n g_a1[n][c] (mask_F x)[n + d_t]:
//              GEMMs over the sites of one plane at a time on the matrix cores,
//              the unshifted operand from the plane, the shifted one from a ring
//              of three planes (a +-1 shift along the 16-site rows is a funnel
//              shift of the row's two 8-site halves, periodic).
//
// In training the forward saves h1, h2, their sign words and s (RingSave), and a
// fourth kernel, the element-wise affine backward, takes the recompute's place.
//
// The three kernels run on the same grid, each workgroup looping over the same
// samples, and write disjoint slots of one partial per workgroup; the
// fixed-order reduction then sums the partials, so the gradient is bitwise
// reproducible.  Channel-major tensors are [B][C][V] BF16.
#include <algorithm>

#include "fused_bwd_common.hpp"

namespace lfs {
namespace fused {
namespace {

__device__ __forceinline__ int mod3(int v) { return ((v % 3) + 3) % 3; }

template <int L, int C>
struct RbCfg {
  using G = Geo<3, L>;
  using LX = Lay<3, L, true>;   // the layer's input field, whole sample
  using LP2 = Lay<2, L, true>;  // one plane of a ring, with its in-plane halo
  static constexpr int V = G::V, T = 27, PLANE = L * L, PS = LP2::VS, LP = L + 2;
  static constexpr int NCT = C / 16;
  static constexpr LayerFrags LF = layer_frags(T, C, true);
  static constexpr int KT3 = kchunks_bf16(2 * T);
  static constexpr int OFF3T = LF.total, OFF2T = OFF3T + LF.nct * KT3, OFF1T = OFF2T + LF.nct * LF.k2;
  static constexpr int FRAGS = OFF1T + LF.k2;
  static constexpr int P_LAYER = C * T + C + C * C * T + C + 2 * C * T + 2;
  static constexpr int ZS = 3 * PS;               // zero site after a ring's three planes
  static constexpr int RING = (3 * PS + 1) * C;   // BF16 elements of a hidden-tensor ring
  static constexpr size_t XS_BYTES = ((size_t)LX::VS * 4 + 15) / 16 * 16;
  static constexpr size_t GOR_BYTES = ((size_t)(3 * PS + 1) * 4 + 15) / 16 * 16;
  static constexpr bool NARROW_HELD = LF.nct == 1;
  // The narrow convolutions' A operands (conv3: rows s and t, lanes 16 j + m with
  // m < 2; conv1 transposed: row 0, lanes 16 j) in compact LDS tables copied once
  // per launch; every lane reads its row group's entry, so the other rows of the
  // product repeat the live ones and are never read.
  static constexpr size_t T3_BYTES = NARROW_HELD ? 0 : (size_t)LF.k2 * 8 * 16;
  static constexpr size_t T1_BYTES = NARROW_HELD ? 0 : (size_t)LF.k2 * 4 * 16;
  // recompute: conv1's operands as row triples of the masked field (x-1, x, x+1, 0
  // per site, 8 bytes) in a ring of four planes, built one step ahead of the conv1
  // passes that read them (three planes per pass)
  static constexpr size_t TRI_BYTES = 4 * (size_t)PLANE * 8;
  static constexpr size_t LDS_A = XS_BYTES + 2 * (size_t)RING * 2 + T3_BYTES + TRI_BYTES;
  // transpose: g_o ring, the LeakyReLU sign masks of one h2 and one h1 plane, two rings
  static constexpr size_t LDS_B = GOR_BYTES + 2 * (size_t)PLANE * 4 + 2 * (size_t)RING * 2 + T1_BYTES;
  // weights: three plane buffers [C][CS] (h1, h2, g_a1 of plane z) and rings of
  // three planes of g_a2 [C][CS], g_o [2][CS] and mask_F x [PLANE].  Channel rows
  // are CS = PLANE + 8 elements apart, so the 16 lanes reading 16 channels at the
  // same site hit different LDS banks.
  static constexpr int CS = PLANE + 8;
  static constexpr size_t LDS_C = (6 * (size_t)C * CS + 3 * 2 * (size_t)CS + 3 * (size_t)PLANE) * 2;
  // recompute and transpose with two output-channel tiles (C = 32): eight waves,
  // four per tile, each holding one tile's fragments of the C-output
  // convolutions; the narrow one (conv3, or conv1 transposed: 2 or 1 outputs)
  // reads its A operand from the compact LDS table instead of holding it, so that
  // two waves fit per SIMD
  static constexpr int NT_A = LF.nct == 2 ? 512 : 256, NT_B = NT_A, NT_C = 512;
  // weight-gradient GEMM tiles (16 x 16): rows are channels, columns (tap, channel)
  static constexpr int RT = C / 16;
  static constexpr int N2 = RT * (T * C / 16), N3 = RT * 4, N1 = RT * 2;
  static constexpr int NWC = NT_C / 64;
  static constexpr int S2 = (N2 + NWC - 1) / NWC, S3 = (N3 + NWC - 1) / NWC, S1 = (N1 + NWC - 1) / NWC;
  static_assert(C % 16 == 0 && L % 16 == 0, "ring backward shapes");
  // dynamic LDS plus the kernels' static buffers (partial reduction, bias sums)
  static_assert(LDS_A + kRedSlices * (NT_A / kRedSlices + 1) * 4 + 64 + 2 * PLANE * 4 <= 160 * 1024 &&
                    LDS_B + (NT_B / 64) * C * 4 + 2 * PLANE * 4 <= 160 * 1024 && LDS_C <= 160 * 1024,
                "LDS budget");
};

// B operand from a ring of three padded planes: the lane's 8 channels at tap
// k0 / C of the site at in-plane index pq of plane v, displaced by SIGN * d_tap;
// slots sm, s0, sp hold planes v-1, v, v+1.  K slots past T * C read the zero site.
template <int L, int C, int SIGN>
__device__ __forceinline__ u32x4 gather_rb(const uint16_t* ring, int pq, int sm, int s0, int sp,
                                           int c, int j) {
  using Cfg = RbCfg<L, C>;
  constexpr int K = 27 * C;
  const int k0 = 32 * c + 8 * j;
  const int tap = k0 / C, ci0 = k0 % C;
  const int dz = SIGN * (tap / 9 - 1), dy = SIGN * ((tap / 3) % 3 - 1), dx = SIGN * (tap % 3 - 1);
  const int slot = dz < 0 ? sm : (dz > 0 ? sp : s0);
  const int e = k0 < K ? (slot * Cfg::PS + pq + dy * Cfg::LP + dx) * C + ci0 : Cfg::ZS * C;
  return *reinterpret_cast<const u32x4*>(ring + e);
}

__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Sum over the 16 lanes of a wave that share j (lane bits 0-3), fixed order.
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-channel bias gradients db[ct][i] (channel ct*16 + 4j + i) of every wave,
// summed over lanes and then over waves in index order, into out[0..C).
template <int C, int NCT, int NW>
__device__ __forceinline__ void bias_partial(f32x4 (&db)[NCT], float* red, float* out) {
  const int lane = threadIdx.x & 63, w = wave_id(), j = lane >> 4, m = lane & 15;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) db[ct][i] = sum16(db[ct][i]);
  __syncthreads();
  if (m == 0) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[w * C + ct * 16 + 4 * j + i] = db[ct][i];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    float r = red[c];
    for (int ww = 1; ww < NW; ++ww) r += red[ww * C + c];
    out[c] = r;
  }
}

// ---------------------------------------------------------------------------
// recompute: h1, h2, s; affine backward
// ---------------------------------------------------------------------------
template <int L, int C, int NT>
__global__ void __launch_bounds__(NT) kr_recompute(
    const u32x4* frags, const float* __restrict__ pl, int off_b1, int off_b2, int off_b3,
    int fpar, int final_tanh, float g_ld, const double* __restrict__ g_ld_vec, int B,
    const float* __restrict__ xin,
    const float* __restrict__ gy, float* __restrict__ gx, uint16_t* __restrict__ h1c,
    uint16_t* __restrict__ h2c, uint32_t* __restrict__ m1, uint32_t* __restrict__ m2,
    uint32_t* __restrict__ go, float* __restrict__ partial, int P,
    const float* __restrict__ prev_partial, float* __restrict__ prev_out) {
  using Cfg = RbCfg<L, C>;
  using G = typename Cfg::G;
  using LX = typename Cfg::LX;
  using LP2 = typename Cfg::LP2;
  constexpr int V = Cfg::V, PLANE = Cfg::PLANE, PS = Cfg::PS;
  constexpr LayerFrags LF = Cfg::LF;
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float red[16];
  // g_y of the plane conv3 works on, two buffers: plane zr's is stored while conv3
  // of plane zr - 1 may still read the other
  static_assert(PLANE <= NT, "one g_y value per thread and plane");
  __shared__ float gys[2][PLANE];
  float* xs = reinterpret_cast<float*>(smem);
  uint16_t* r1 = reinterpret_cast<uint16_t*>(smem + Cfg::XS_BYTES);
  uint16_t* r2 = r1 + Cfg::RING;
  u32x4* t3 = reinterpret_cast<u32x4*>(r2 + Cfg::RING);  // visible after the sample loop's first barrier
  uint16_t* tr = reinterpret_cast<uint16_t*>(smem + Cfg::XS_BYTES + 2 * (size_t)Cfg::RING * 2 + Cfg::T3_BYTES);
  if constexpr (!Cfg::NARROW_HELD)
    for (int i = threadIdx.x; i < LF.k2 * 8; i += NT)
      t3[i] = frags[(LF.off3 + (i >> 3)) * 64 + 16 * ((i & 7) >> 1) + (i & 1)];
  for (int q = threadIdx.x; q < C; q += NT) r1[Cfg::ZS * C + q] = 0, r2[Cfg::ZS * C + q] = 0;
  const int lane = threadIdx.x & 63, w = wave_id(), j = lane >> 4, m = lane & 15;
  constexpr int WPC = NW / LF.nct;  // waves per output-channel tile
  static_assert(NW % LF.nct == 0, "waves split evenly over the channel tiles");
  // this wave's channel tile and its index among that tile's waves
  const int ct = LF.nct == 1 ? 0 : w / WPC, wc = LF.nct == 1 ? w : w % WPC;
  const int apar = fpar ^ 1;
  // the lane's four triple rows (chunk c, slot u: row r = 8 c + 2 j + u, past the nine
  // rows (dz, dy) = (r / 3 - 1, r % 3 - 1) the centre row, which meets zero weights)
  int tdz[4], tdy[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r0 = 8 * (i >> 1) + 2 * j + (i & 1), r = r0 < 9 ? r0 : 4;
    tdz[i] = r / 3 - 1;
    tdy[i] = r % 3 - 1;
  }
  const u32x4* fl = frags + lane;
  u32x4 A1[1][LF.k1], A2[1][LF.k2], A3[Cfg::NARROW_HELD ? LF.k2 : 1];
  const f32x4 bias1[1] = {load_bias4<C>(pl + off_b1, ct, j)}, bias2[1] = {load_bias4<C>(pl + off_b2, ct, j)};
#pragma unroll
  for (int c = 0; c < LF.k1; ++c) A1[0][c] = fl[(LF.off1 + ct * LF.k1 + c) * 64];
#pragma unroll
  for (int c = 0; c < LF.k2; ++c) A2[0][c] = fl[(LF.off2 + ct * LF.k2 + c) * 64];
  if constexpr (Cfg::NARROW_HELD) {
#pragma unroll
    for (int c = 0; c < LF.k2; ++c) A3[c] = fl[(LF.off3 + c) * 64];
  }
  // one channel tile's sign bits of a site: the whole mask word, or its half
  auto store_mask = [&](uint32_t* mk, size_t n, uint32_t mw) {
    if constexpr (LF.nct == 1)
      mk[n] = mw;
    else
      reinterpret_cast<uint16_t*>(mk)[2 * n + ct] = (uint16_t)mw;  // little-endian: tile ct's 16 bits
  };
  float db3s = 0.f, db3t = 0.f;
  // the previous launch's (next layer's) weight gradient; every kernel of a layer
  // runs on the same grid, so that is also the number of partials
  if (prev_partial) grid_reduce<NT>(prev_partial, prev_out, (int)gridDim.x, P);

  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const size_t sb = (size_t)b * V;
    // cotangent of the log-det: one for all samples, or this sample's
    const float gld = g_ld_vec ? (float)(-g_ld_vec[b]) : g_ld;
    uint16_t* h1b = h1c + (size_t)b * C * V;
    uint16_t* h2b = h2c + (size_t)b * C * V;
    __syncthreads();  // the previous sample's readers are done
    for (int q = threadIdx.x; q < LX::VS; q += NT) xs[q] = xin[sb + LX::site_of(q)];
    __syncthreads();

    // row triples of the masked field of virtual plane v into triple-ring slot v mod 4
    // (only frozen sites' values enter)
    auto build_tri_plane = [&](int v) {
      const int zr = ((v % L) + L) % L;
      uint16_t* dst = tr + (v & 3) * PLANE * 4;
      for (int q = threadIdx.x; q < PLANE; q += NT) {
        const int n = zr * PLANE + q, p = LX::idx(n);
        const bool frozen = G::parity(n) == fpar;  // the x neighbours have the other parity
        const float v0 = frozen ? 0.f : xs[p - 1], v1 = frozen ? xs[p] : 0.f, v2 = frozen ? 0.f : xs[p + 1];
        *reinterpret_cast<u32x2*>(dst + 4 * q) = u32x2{pack_bf16(v0, v1), pack_bf16(v2, 0.f)};
      }
    };
    // h1 of virtual plane v into ring slot v mod 3 (and, for a real plane, to h1c)
    auto conv1_plane = [&](int v) {
      const int zr = ((v % L) + L) % L;
      const bool real = v >= 0 && v < L;
      uint16_t* dst = r1 + mod3(v) * PS * C;
      int tbase[4];  // the lane's triple rows: ring slot of plane v + dz, as an element offset
#pragma unroll
      for (int i = 0; i < 4; ++i) tbase[i] = ((v + tdz[i]) & 3) * PLANE;
      mma_tiles<1, 1, LF.k1, true>(
          PLANE / 16, wc, WPC, A1, bias1,
          [&](int tile, int c) {  // tile = in-plane row y, m = x
            const int e0 = (tbase[2 * c] + ((tile + tdy[2 * c]) & (L - 1)) * L + m) * 4;
            const int e1 = (tbase[2 * c + 1] + ((tile + tdy[2 * c + 1]) & (L - 1)) * L + m) * 4;
            const u32x2 a = *reinterpret_cast<const u32x2*>(tr + e0), b = *reinterpret_cast<const u32x2*>(tr + e1);
            return u32x4{a[0], a[1], b[0], b[1]};
          },
          [&](int tile, const f32x4(&acc)[1]) {
            const u32x2 hv = store_act_tile<LP2, C, true>(dst, tile, m, ct, j, acc[0]);
            if (real) store_cm_global<C, V>(h1b, zr * PLANE + tile * 16 + m, ct * 16 + 4 * j, hv);
            const uint32_t mw = sign_mask16(hv, j);
            if (real && j == 0) store_mask(m1, sb + zr * PLANE + tile * 16 + m, mw);
          });
    };
    // h2 of virtual plane v from h1 planes v-1, v, v+1
    auto conv2_plane = [&](int v) {
      const int zr = ((v % L) + L) % L;
      const bool real = v >= 0 && v < L;
      uint16_t* dst = r2 + mod3(v) * PS * C;
      const int sm = mod3(v - 1), s0 = mod3(v), sp = mod3(v + 1);
      mma_tiles<1, 1, LF.k2, true>(
          PLANE / 16, wc, WPC, A2, bias2,
          [&](int tile, int c) { return gather_rb<L, C, 1>(r1, tile_p<LP2>(tile, m), sm, s0, sp, c, j); },
          [&](int tile, const f32x4(&acc)[1]) {
            const u32x2 hv = store_act_tile<LP2, C, true>(dst, tile, m, ct, j, acc[0]);
            if (real) store_cm_global<C, V>(h2b, zr * PLANE + tile * 16 + m, ct * 16 + 4 * j, hv);
            const uint32_t mw = sign_mask16(hv, j);
            if (real && j == 0) store_mask(m2, sb + zr * PLANE + tile * 16 + m, mw);
          });
    };
    // s at the active sites of plane zr; g_x there, g_o of the whole plane
    auto conv3_plane = [&](int zr) {
      const int sm = mod3(zr - 1), s0 = mod3(zr), sp = mod3(zr + 1);
      const int ppar = apar ^ (zr & 1);  // in-plane parity of the active sites
      for (int tile = w; tile < PLANE / 32; tile += NW) {
        const int q3 = LP2::idx(Geo<2, L>::half_site(tile * 16 + m, ppar));
        // two accumulator chains (even and odd chunks), summed at the end
        auto a3_of = [&](int c) -> u32x4 {
          if constexpr (Cfg::NARROW_HELD)
            return A3[c];
          else
            return t3[c * 8 + 2 * j + (m & 1)];
        };
        f32x4 ae{pl[off_b3], 0.f, 0.f, 0.f}, ao{0.f, 0.f, 0.f, 0.f};
#pragma unroll Cfg::NARROW_HELD ? LF.k2 / 2 : 2
        for (int c = 0; c + 1 < LF.k2; c += 2) {
          ae = mma<true>(a3_of(c), gather_rb<L, C, 1>(r2, q3, sm, s0, sp, c, j), ae);
          ao = mma<true>(a3_of(c + 1), gather_rb<L, C, 1>(r2, q3, sm, s0, sp, c + 1, j), ao);
        }
        if constexpr (LF.k2 % 2) ae = mma<true>(a3_of(LF.k2 - 1), gather_rb<L, C, 1>(r2, q3, sm, s0, sp, LF.k2 - 1, j), ae);
        const f32x4 acc[1] = {ae + ao};
        if (j == 0) {
          const int n = zr * PLANE + Geo<2, L>::half_site(tile * 16 + m, ppar);
          const float o0 = acc[0][0];
          const float s = final_tanh ? fast_tanh(o0) : o0;
          const float es = fast_exp(s);
          const float g = gys[zr & 1][n - zr * PLANE];
          const float gs = g * xs[LX::idx(n)] * es + gld;
          const float go0 = final_tanh ? gs * (1.f - s * s) : gs;
          db3s += go0;
          db3t += g;
          gx[sb + n] = g * es;
          go[sb + n] = pack_bf16(go0, g);
        }
      }
      for (int i = threadIdx.x; i < PLANE / 2; i += NT)
        go[sb + zr * PLANE + Geo<2, L>::half_site(i, ppar ^ 1)] = 0u;
    };

    // triple ring slot (v & 3): each plane's triples are built after the last conv1
    // pass that read the plane four back in the same slot
    for (int v = -3; v <= 0; ++v) build_tri_plane(v);
    __syncthreads();
    conv1_plane(-2);  // triples of planes -3 .. -1
    conv1_plane(-1);  // -2 .. 0
    __syncthreads();
    build_tri_plane(1);  // over plane -3's
    __syncthreads();
    conv1_plane(0);
    __syncthreads();
    conv2_plane(-1);
    build_tri_plane(2);  // over plane -2's, last read by conv1(-1)
    __syncthreads();
    conv1_plane(1);
    __syncthreads();
    conv2_plane(0);
    build_tri_plane(3);  // over plane -1's, last read by conv1(0)
    __syncthreads();
    for (int zr = 0; zr < L; ++zr) {
      // plane zr's g_y is read here and held in a register through conv1, so its
      // HBM latency hides behind that pass instead of stalling conv3's epilogue
      const float gpre = threadIdx.x < PLANE ? gy[sb + zr * PLANE + threadIdx.x] : 0.f;
      conv1_plane(zr + 2);  // triples of planes zr + 1 .. zr + 3
      if (threadIdx.x < PLANE) gys[zr & 1][threadIdx.x] = gpre;
      __syncthreads();
      conv2_plane(zr + 1);
      build_tri_plane(zr + 4);  // over plane zr's, last read by conv1(zr + 1)
      __syncthreads();
      conv3_plane(zr);
    }
  }
  db3s = block_sum(db3s, red);
  db3t = block_sum(db3t, red);
  if (threadIdx.x == 0) {
    partial[(size_t)blockIdx.x * P + off_b3] = db3s;
    partial[(size_t)blockIdx.x * P + off_b3 + 1] = db3t;
  }
}

// ---------------------------------------------------------------------------
// affine backward from the training forward's saved s (in place of recompute)
// ---------------------------------------------------------------------------
// At the active sites: g_x = g_y e^s, g_o = (g_s (1 - s^2), g_t) with g_s = g_y x e^s
// + g_ld (the log-det's cotangent) and g_t = g_y; zero g_o at the frozen sites; db3.
// (paper Sec. 1, coupling-layer equation).  Element-wise: four consecutive sites per
// thread and step.
template <int L, int NT>
__global__ void __launch_bounds__(NT) kr_affine(
    int fpar, int final_tanh, float g_ld, const double* __restrict__ g_ld_vec, int B,
    const float* __restrict__ xin, const float* __restrict__ gy, const float* __restrict__ ss,
    float* __restrict__ gx, uint32_t* __restrict__ go, float* __restrict__ partial, int P, int off_b3,
    const float* __restrict__ prev_partial, float* __restrict__ prev_out) {
  using G = Geo<3, L>;
  constexpr int V = G::V;
  static_assert(L % 4 == 0, "four sites of one row per thread");
  __shared__ float red[16];
  float db3s = 0.f, db3t = 0.f;
  // the previous launch's (next layer's) weight gradient (same grid as every kernel
  // of a layer, so also the number of partials)
  if (prev_partial) grid_reduce<NT>(prev_partial, prev_out, (int)gridDim.x, P);
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const size_t sb = (size_t)b * V;
    const float gld = g_ld_vec ? (float)(-g_ld_vec[b]) : g_ld;
    for (int q = threadIdx.x; q < V / 4; q += NT) {
      const int n0 = 4 * q;
      const f32x4 g = reinterpret_cast<const f32x4*>(gy + sb)[q];
      const f32x4 x = reinterpret_cast<const f32x4*>(xin + sb)[q];
      const f32x4 sv = reinterpret_cast<const f32x4*>(ss + sb)[q];
      f32x4 gxv;
      u32x4 gov;
      // sites n0 + i alternate in parity along the row; the frozen ones get g_o = 0
      // and a placeholder g_x, which the transpose kernel overwrites
      const int a0 = G::parity(n0) == fpar ? 1 : 0;  // first active offset
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if ((i & 1) == a0) {
          const float s = sv[i], es = fast_exp(s);
          const float gs = g[i] * x[i] * es + gld;
          const float go0 = final_tanh ? gs * (1.f - s * s) : gs;
          db3s += go0;
          db3t += g[i];
          gxv[i] = g[i] * es;
          gov[i] = pack_bf16(go0, g[i]);
        } else {
          gxv[i] = 0.f;
          gov[i] = 0u;
        }
      }
      reinterpret_cast<f32x4*>(gx + sb)[q] = gxv;
      reinterpret_cast<u32x4*>(go + sb)[q] = gov;
    }
  }
  db3s = block_sum(db3s, red);
  db3t = block_sum(db3t, red);
  if (threadIdx.x == 0) {
    partial[(size_t)blockIdx.x * P + off_b3] = db3s;
    partial[(size_t)blockIdx.x * P + off_b3 + 1] = db3t;
  }
}

// ---------------------------------------------------------------------------
// transpose: g_a2, g_a1, g_x(frozen)
// ---------------------------------------------------------------------------
template <int L, int C, int NT>
__global__ void __launch_bounds__(NT) kr_transpose(
    const u32x4* frags, int fpar, int B, const uint32_t* __restrict__ go,
    const uint32_t* __restrict__ m1, const uint32_t* __restrict__ m2,
    const float* __restrict__ gy, float* __restrict__ gx, uint16_t* __restrict__ ga2c,
    uint16_t* __restrict__ ga1c, float* __restrict__ partial, int P, int off_b1, int off_b2) {
  using Cfg = RbCfg<L, C>;
  using LP2 = typename Cfg::LP2;
  constexpr int V = Cfg::V, PLANE = Cfg::PLANE, PS = Cfg::PS, LP = Cfg::LP, NCT = Cfg::NCT;
  constexpr LayerFrags LF = Cfg::LF;
  constexpr int NW = NT / 64, KT3 = Cfg::KT3;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float red[NW * C];
  // g_y of the plane the g_x pass works on, two buffers (see the plane loop)
  static_assert(PLANE <= NT, "one g_y value per thread and plane");
  __shared__ float gys[2][PLANE];
  uint32_t* gor = reinterpret_cast<uint32_t*>(smem);
  uint32_t* sm2 = reinterpret_cast<uint32_t*>(smem + Cfg::GOR_BYTES);  // h2 signs of one plane
  uint32_t* sm1 = sm2 + PLANE;                                          // h1 signs of one plane
  uint16_t* ra2 = reinterpret_cast<uint16_t*>(smem + Cfg::GOR_BYTES + 2 * PLANE * 4);
  uint16_t* ra1 = ra2 + Cfg::RING;
  u32x4* t1 = reinterpret_cast<u32x4*>(ra1 + Cfg::RING);  // visible after the sample loop's first barrier
  if constexpr (!Cfg::NARROW_HELD)
    for (int i = threadIdx.x; i < LF.k2 * 4; i += NT) t1[i] = frags[(Cfg::OFF1T + (i >> 2)) * 64 + 16 * (i & 3)];
  if (threadIdx.x == 0) gor[Cfg::ZS] = 0u;
  for (int q = threadIdx.x; q < C; q += NT) ra2[Cfg::ZS * C + q] = 0, ra1[Cfg::ZS * C + q] = 0;
  const int lane = threadIdx.x & 63, w = wave_id(), j = lane >> 4, m = lane & 15;
  constexpr int WPC = NW / NCT;  // waves per output-channel tile
  static_assert(NW % NCT == 0, "waves split evenly over the channel tiles");
  // this wave's channel tile and its index among that tile's waves
  const int ct = NCT == 1 ? 0 : w / WPC, wc = NCT == 1 ? w : w % WPC;
  const u32x4* fl = frags + lane;
  u32x4 A3T[1][KT3], A2T[1][LF.k2], A1T[Cfg::NARROW_HELD ? LF.k2 : 1];
#pragma unroll
  for (int c = 0; c < KT3; ++c) A3T[0][c] = fl[(Cfg::OFF3T + ct * KT3 + c) * 64];
#pragma unroll
  for (int c = 0; c < LF.k2; ++c) A2T[0][c] = fl[(Cfg::OFF2T + ct * LF.k2 + c) * 64];
  if constexpr (Cfg::NARROW_HELD) {
#pragma unroll
    for (int c = 0; c < LF.k2; ++c) A1T[c] = fl[(Cfg::OFF1T + c) * 64];
  }
  const f32x4 zero1[1] = {};
  f32x4 db2{0.f, 0.f, 0.f, 0.f}, db1{0.f, 0.f, 0.f, 0.f};  // channels ct * 16 + 4 j + i

  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const size_t sb = (size_t)b * V;
    uint16_t* a2b = ga2c + (size_t)b * C * V;
    uint16_t* a1b = ga1c + (size_t)b * C * V;
    __syncthreads();

    // g_o of virtual plane v (BF16 pairs, padded plane) into its ring slot
    auto go_plane = [&](int v) {
      const int zr = ((v % L) + L) % L;
      uint32_t* dst = gor + mod3(v) * PS;
      for (int q = threadIdx.x; q < PS; q += NT) dst[q] = go[sb + zr * PLANE + LP2::site_of(q)];
    };
    // the sign words of virtual plane v of h (m2 or m1) into a one-plane buffer
    auto mask_plane = [&](const uint32_t* mk, uint32_t* dst, int v) {
      const int zr = ((v % L) + L) % L;
      for (int q = threadIdx.x; q < PLANE; q += NT) dst[q] = mk[sb + zr * PLANE + q];
    };
    // masked transposed-convolution output: leaky'(h) * acc, into a ring slot (and,
    // for a real plane, channel-major to global memory and the bias sums)
    auto epilogue = [&](const uint32_t* smk, uint16_t* dst, uint16_t* gout, f32x4& db, bool real,
                        int zr, int tile, const f32x4(&acc)[1]) {
      const int n = zr * PLANE + tile * 16 + m;
      const uint32_t mw = smk[tile * 16 + m];
      const int co0 = ct * 16 + 4 * j;
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (mw >> (co0 + i)) & 1u ? acc[0][i] : kLeakySlope * acc[0][i];
      const u32x2 pw = store4_tile<LP2, C, true>(dst, tile, m, co0, v);
      if (real) {
        store_cm_global<C, V>(gout, n, co0, pw);
#pragma unroll
        for (int i = 0; i < 4; ++i) db[i] += v[i];
      }
    };
    // g_a2 of virtual plane v from g_o planes v-1, v, v+1
    auto a2_plane = [&](int v) {
      const int zr = ((v % L) + L) % L;
      const bool real = v >= 0 && v < L;
      uint16_t* dst = ra2 + mod3(v) * PS * C;
      const int sm = mod3(v - 1), s0 = mod3(v), sp = mod3(v + 1);
      mma_tiles<1, 1, KT3, true>(
          PLANE / 16, wc, WPC, A3T, zero1,
          [&](int tile, int c) {
            const int pq = tile_p<LP2>(tile, m), t0 = 16 * c + 4 * j;  // K = tap * 2 + co
            u32x4 r;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int t = t0 + q;
              const int dz = 1 - t / 9, dy = 1 - (t / 3) % 3, dx = 1 - t % 3;  // -d_t
              const int slot = dz < 0 ? sm : (dz > 0 ? sp : s0);
              r[q] = gor[t < 27 ? slot * PS + pq + dy * LP + dx : Cfg::ZS];
            }
            return r;
          },
          [&](int tile, const f32x4(&acc)[1]) { epilogue(sm2, dst, a2b, db2, real, zr, tile, acc); });
    };
    // g_a1 of virtual plane v from g_a2 planes v-1, v, v+1
    auto a1_plane = [&](int v) {
      const int zr = ((v % L) + L) % L;
      const bool real = v >= 0 && v < L;
      uint16_t* dst = ra1 + mod3(v) * PS * C;
      const int sm = mod3(v - 1), s0 = mod3(v), sp = mod3(v + 1);
      mma_tiles<1, 1, LF.k2, true>(
          PLANE / 16, wc, WPC, A2T, zero1,
          [&](int tile, int c) { return gather_rb<L, C, -1>(ra2, tile_p<LP2>(tile, m), sm, s0, sp, c, j); },
          [&](int tile, const f32x4(&acc)[1]) { epilogue(sm1, dst, a1b, db1, real, zr, tile, acc); });
    };
    // g_x at the frozen sites of plane zr from g_a1 planes zr-1, zr, zr+1
    auto gx_plane = [&](int zr) {
      const int sm = mod3(zr - 1), s0 = mod3(zr), sp = mod3(zr + 1);
      const int fp = fpar ^ (zr & 1);  // in-plane parity of the frozen sites
      for (int tile = w; tile < PLANE / 32; tile += NW) {
        const int q = Geo<2, L>::half_site(tile * 16 + m, fp), pq = LP2::idx(q);
        // two accumulator chains (even and odd chunks), summed at the end
        auto a1_of = [&](int c) -> u32x4 {
          if constexpr (Cfg::NARROW_HELD)
            return A1T[c];
          else
            return t1[c * 4 + j];
        };
        f32x4 ae{0.f, 0.f, 0.f, 0.f}, ao{0.f, 0.f, 0.f, 0.f};
#pragma unroll Cfg::NARROW_HELD ? LF.k2 / 2 : 2
        for (int c = 0; c + 1 < LF.k2; c += 2) {
          ae = mma<true>(a1_of(c), gather_rb<L, C, -1>(ra1, pq, sm, s0, sp, c, j), ae);
          ao = mma<true>(a1_of(c + 1), gather_rb<L, C, -1>(ra1, pq, sm, s0, sp, c + 1, j), ao);
        }
        if constexpr (LF.k2 % 2) ae = mma<true>(a1_of(LF.k2 - 1), gather_rb<L, C, -1>(ra1, pq, sm, s0, sp, LF.k2 - 1, j), ae);
        const f32x4 acc = ae + ao;
        if (j == 0) gx[sb + zr * PLANE + q] = gys[zr & 1][q] + acc[0];
      }
    };

    // each mask buffer is refilled only after the pass that read it is behind a barrier
    go_plane(-3);
    go_plane(-2);
    go_plane(-1);
    mask_plane(m2, sm2, -2);
    __syncthreads();
    a2_plane(-2);
    __syncthreads();
    go_plane(0);
    mask_plane(m2, sm2, -1);
    __syncthreads();
    a2_plane(-1);
    __syncthreads();
    go_plane(1);
    mask_plane(m2, sm2, 0);
    mask_plane(m1, sm1, -1);
    __syncthreads();
    a2_plane(0);
    __syncthreads();
    a1_plane(-1);
    __syncthreads();
    go_plane(2);
    mask_plane(m2, sm2, 1);
    mask_plane(m1, sm1, 0);
    __syncthreads();
    a2_plane(1);
    __syncthreads();
    a1_plane(0);
    __syncthreads();
    // Software pipelining: the next step's g_o plane, sign words and g_y are read
    // into registers before the g_x pass and written to LDS at the top of the next
    // step (their previous readers, the a2 and a1 passes, are behind its barriers;
    // g_y alternates between two rows because the g_x pass may still read the
    // other), so the HBM latency hides behind the g_x pass.
    constexpr int GPT = (PS + NT - 1) / NT;
    uint32_t fgo[GPT], fm2 = 0u, fm1 = 0u;
    float fgy = 0.f;
    auto fetch = [&](int z) {
      const int zg = (((z + 3) % L) + L) % L, z2 = (((z + 2) % L) + L) % L, z1 = (((z + 1) % L) + L) % L;
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = threadIdx.x + r * NT;
        if (q < PS) fgo[r] = go[sb + zg * PLANE + LP2::site_of(q)];
      }
      if (threadIdx.x < PLANE) {
        fm2 = m2[sb + z2 * PLANE + threadIdx.x];
        fm1 = m1[sb + z1 * PLANE + threadIdx.x];
        fgy = gy[sb + z * PLANE + threadIdx.x];
      }
    };
    auto commit = [&](int z) {
      uint32_t* dst = gor + mod3(z + 3) * PS;
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = threadIdx.x + r * NT;
        if (q < PS) dst[q] = fgo[r];
      }
      if (threadIdx.x < PLANE) {
        sm2[threadIdx.x] = fm2;
        sm1[threadIdx.x] = fm1;
        gys[z & 1][threadIdx.x] = fgy;
      }
    };
    fetch(0);
    for (int z = 0; z < L; ++z) {
      commit(z);
      __syncthreads();
      a2_plane(z + 2);
      __syncthreads();
      a1_plane(z + 1);
      __syncthreads();
      if (z + 1 < L) fetch(z + 1);
      gx_plane(z);
    }
  }
  // every wave's sums for all channel tiles, zero for the tiles it did not compute
  f32x4 d2[NCT], d1[NCT];
#pragma unroll
  for (int t = 0; t < NCT; ++t) {
    d2[t] = t == ct ? db2 : f32x4{0.f, 0.f, 0.f, 0.f};
    d1[t] = t == ct ? db1 : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  bias_partial<C, NCT, NW>(d2, red, partial + (size_t)blockIdx.x * P + off_b2);
  bias_partial<C, NCT, NW>(d1, red, partial + (size_t)blockIdx.x * P + off_b1);
}

// ---------------------------------------------------------------------------
// weights: dW3, dW2, dW1 one plane at a time
// ---------------------------------------------------------------------------

// Eight consecutive sites of a 16-site row, periodic in x, from the lane's own
// half p of the row (x = 8h..8h+7) and the other half o: shifted by sx in
// {-1, 0, +1}, i.e. x = 8h + sx .. 8h + sx + 7.
__device__ __forceinline__ u32x4 shift_p1(const u32x4& p, const u32x4& o) {  // p[1..7], o[0]
  return u32x4{__builtin_amdgcn_alignbit(p[1], p[0], 16), __builtin_amdgcn_alignbit(p[2], p[1], 16),
               __builtin_amdgcn_alignbit(p[3], p[2], 16), __builtin_amdgcn_alignbit(o[0], p[3], 16)};
}
__device__ __forceinline__ u32x4 shift_m1(const u32x4& p, const u32x4& o) {  // o[7], p[0..6]
  return u32x4{__builtin_amdgcn_alignbit(p[0], o[3], 16), __builtin_amdgcn_alignbit(p[1], p[0], 16),
               __builtin_amdgcn_alignbit(p[2], p[1], 16), __builtin_amdgcn_alignbit(p[3], p[2], 16)};
}
__device__ __forceinline__ u32x4 shift_any(const u32x4& p, const u32x4& o, int sx) {
  const u32x4 a = shift_p1(p, o), b = shift_m1(p, o);
  u32x4 r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = sx > 0 ? a[q] : (sx < 0 ? b[q] : p[q]);
  return r;
}

template <int L, int C, int NT>
__global__ void __launch_bounds__(NT) kr_wgrad(
    int fpar, int B, const float* __restrict__ xin, const uint16_t* __restrict__ h1c,
    const uint16_t* __restrict__ h2c, const uint32_t* __restrict__ go,
    const uint16_t* __restrict__ ga2c, const uint16_t* __restrict__ ga1c,
    float* __restrict__ partial, int P, int off_W1, int off_W2, int off_W3) {
  using Cfg = RbCfg<L, C>;
  using G = typename Cfg::G;
  constexpr int V = Cfg::V, PLANE = Cfg::PLANE, T = Cfg::T, RT = Cfg::RT, NW = NT / 64;
  static_assert(L == 16, "rows of two 8-site halves");
  // dW2 jobs: (row offset (dz, dy), 16 channels co), each over every row tile of ci:
  // the three x offsets and the row tiles share the two loads of the source row (the
  // dW2 pass is bound by LDS reads: 4 KB per six MFMAs at C = 32, 6 KB when the row
  // tiles were separate jobs)
  constexpr int NCO = C / 16, J2 = 9 * NCO, JS2 = (J2 + NW - 1) / NW;
  // single tiles: dW3 (row tile, 16 (tap, co) columns), then dW1 (row tile, 16 taps)
  constexpr int N3 = Cfg::N3, J31 = Cfg::N3 + Cfg::N1, JS31 = (J31 + NW - 1) / NW;
  constexpr int CS = Cfg::CS;
  constexpr int PPT = (C * PLANE / 8 + NT - 1) / NT;  // 16-byte plane pieces per thread
  static_assert(PLANE <= NT, "one ring site per thread");
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* pa1 = reinterpret_cast<uint16_t*>(smem);  // h1 of plane z, [C][CS]
  uint16_t* pa2 = pa1 + C * CS;                        // h2 of plane z
  uint16_t* pa3 = pa2 + C * CS;                        // g_a1 of plane z
  uint16_t* rg2 = pa3 + C * CS;                        // g_a2 ring [3][C][CS]
  uint16_t* rgo = rg2 + 3 * C * CS;                    // g_o ring [3][2][CS]
  uint16_t* rh0 = rgo + 3 * 2 * CS;                    // mask_F x ring [3][PLANE]
  const int lane = threadIdx.x & 63, w = wave_id(), j = lane >> 4, m = lane & 15;
  const int h = j & 1, jr = j >> 1;  // the lane's half row and row within a K chunk
  f32x4 acc2[JS2][RT][3], acc31[JS31];
#pragma unroll
  for (int k = 0; k < JS2; ++k)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc2[k][rt][0] = acc2[k][rt][1] = acc2[k][rt][2] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < JS31; ++k) acc31[k] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const size_t sb = (size_t)b * V;
    auto load_ring = [&](int v) {
      const int zr = ((v % L) + L) % L, slot = mod3(v);
      for (int i = threadIdx.x; i < C * PLANE / 8; i += NT) {
        const int c = i / (PLANE / 8), k = i % (PLANE / 8);
        *reinterpret_cast<u32x4*>(rg2 + (slot * C + c) * CS + 8 * k) =
            *reinterpret_cast<const u32x4*>(ga2c + ((size_t)b * C + c) * V + zr * PLANE + 8 * k);
      }
      for (int i = threadIdx.x; i < PLANE; i += NT) {
        const uint32_t u = go[sb + zr * PLANE + i];
        rgo[(slot * 2 + 0) * CS + i] = (uint16_t)u;
        rgo[(slot * 2 + 1) * CS + i] = (uint16_t)(u >> 16);
        const int n = zr * PLANE + i;
        rh0[slot * PLANE + i] = G::parity(n) == fpar ? (uint16_t)bf16_bits(xin[sb + n]) : (uint16_t)0;
      }
    };
    // Software pipelining: the operands of the next step (plane z + 1 of h1, h2,
    // g_a1 and ring plane z + 2 of g_a2, g_o, mask_F x) are fetched into registers
    // while plane z is computed, and written to LDS after the step's closing
    // barrier, so the HBM latency hides behind the matrix work.
    u32x4 f1[PPT], f2[PPT], f3[PPT], fr[PPT];
    uint32_t fgo = 0u;
    float fx = 0.f;
    auto fetch = [&](int zp, int vr) {
      const int zr = ((vr % L) + L) % L;
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const int i = threadIdx.x + q * NT;
        if (i < C * PLANE / 8) {
          const int c = i / (PLANE / 8), k = i % (PLANE / 8);
          const size_t src = ((size_t)b * C + c) * V + zp * PLANE + 8 * k;
          f1[q] = *reinterpret_cast<const u32x4*>(h1c + src);
          f2[q] = *reinterpret_cast<const u32x4*>(h2c + src);
          f3[q] = *reinterpret_cast<const u32x4*>(ga1c + src);
          fr[q] = *reinterpret_cast<const u32x4*>(ga2c + ((size_t)b * C + c) * V + zr * PLANE + 8 * k);
        }
      }
      if (threadIdx.x < PLANE) {
        fgo = go[sb + zr * PLANE + threadIdx.x];
        fx = xin[sb + zr * PLANE + threadIdx.x];
      }
    };
    auto commit = [&](int vr) {
      const int zr = ((vr % L) + L) % L, slot = mod3(vr);
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const int i = threadIdx.x + q * NT;
        if (i < C * PLANE / 8) {
          const int c = i / (PLANE / 8), k = i % (PLANE / 8);
          const int dst = c * CS + 8 * k;
          *reinterpret_cast<u32x4*>(pa1 + dst) = f1[q];
          *reinterpret_cast<u32x4*>(pa2 + dst) = f2[q];
          *reinterpret_cast<u32x4*>(pa3 + dst) = f3[q];
          *reinterpret_cast<u32x4*>(rg2 + (slot * C + c) * CS + 8 * k) = fr[q];
        }
      }
      if (threadIdx.x < PLANE) {
        const int i = threadIdx.x, n = zr * PLANE + i;
        rgo[(slot * 2 + 0) * CS + i] = (uint16_t)fgo;
        rgo[(slot * 2 + 1) * CS + i] = (uint16_t)(fgo >> 16);
        rh0[slot * PLANE + i] = G::parity(n) == fpar ? (uint16_t)bf16_bits(fx) : (uint16_t)0;
      }
    };
    __syncthreads();
    load_ring(-1);
    load_ring(0);
    fetch(0, 1);
    for (int z = 0; z < L; ++z) {
      commit(z + 1);        // plane z and ring plane z + 1 (their previous readers passed the last barrier)
      __syncthreads();
      if (z + 1 < L) fetch(z + 1, z + 2);
      // dW2: D[ci][(tap, co)] += sum over the plane's sites m of h1[m][ci] g_a2[m - d][co]
#pragma unroll
      for (int k = 0; k < JS2; ++k) {
        const int id = k * NW + w;
        if (id < J2) {
          const int r9 = id % 9, cot = id / 9;
          const int dz = r9 / 3 - 1, dy = r9 % 3 - 1;
          const uint16_t* src = rg2 + (mod3(z - dz) * C + cot * 16 + m) * CS;
#pragma unroll 2
          for (int c = 0; c < PLANE / 32; ++c) {
            const uint16_t* row = src + ((2 * c + jr - dy) & (L - 1)) * L;
            const u32x4 p = *reinterpret_cast<const u32x4*>(row + 8 * h);
            const u32x4 o = *reinterpret_cast<const u32x4*>(row + 8 - 8 * h);
            const bf16x8 bp = as_bf16x8(shift_p1(p, o)), b0 = as_bf16x8(p), bm = as_bf16x8(shift_m1(p, o));
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
              const bf16x8 a = as_bf16x8(*reinterpret_cast<const u32x4*>(pa1 + (rt * 16 + m) * CS + 8 * j + 32 * c));
              acc2[k][rt][0] = mfma(a, bp, acc2[k][rt][0]);  // dx = -1: x + 1
              acc2[k][rt][1] = mfma(a, b0, acc2[k][rt][1]);
              acc2[k][rt][2] = mfma(a, bm, acc2[k][rt][2]);  // dx = +1: x - 1
            }
          }
        }
      }
      // dW3: D[ci][(tap, co)] += sum_m h2[m][ci] g_o[m - d][co];  dW1: D[c][tap] += sum_n g_a1[n][c] h0[n + d]
#pragma unroll
      for (int k = 0; k < JS31; ++k) {
        const int id = k * NW + w;
        if (id < J31) {
          const bool w3 = id < N3;
          const int id2 = w3 ? id : id - N3, rt = id2 % RT, ct = id2 / RT;
          const int col = ct * 16 + m;
          const int tap = std::min(w3 ? col >> 1 : col, T - 1), co = col & 1;
          const int dz = tap / 9 - 1, dy = tap / 3 % 3 - 1, dx = tap % 3 - 1;
          const int sgn = w3 ? -1 : 1;  // dW3 reads g_o at m - d, dW1 reads h0 at n + d
          const uint16_t* src = w3 ? rgo + (mod3(z - dz) * 2 + co) * CS : rh0 + mod3(z + dz) * PLANE;
          const uint16_t* ap = (w3 ? pa2 : pa3) + (rt * 16 + m) * CS + 8 * j;
#pragma unroll 2
          for (int c = 0; c < PLANE / 32; ++c) {
            const bf16x8 a = as_bf16x8(*reinterpret_cast<const u32x4*>(ap + 32 * c));
            const uint16_t* row = src + ((2 * c + jr + sgn * dy) & (L - 1)) * L;
            const u32x4 p = *reinterpret_cast<const u32x4*>(row + 8 * h);
            const u32x4 o = *reinterpret_cast<const u32x4*>(row + 8 - 8 * h);
            acc31[k] = mfma(a, as_bf16x8(shift_any(p, o, sgn * dx)), acc31[k]);
          }
        }
      }
      __syncthreads();
    }
  }
  // every weight-gradient slot belongs to exactly one lane of one wave
  float* out = partial + (size_t)blockIdx.x * P;
#pragma unroll
  for (int k = 0; k < JS2; ++k) {
    const int id = k * NW + w;
    if (id < J2) {
      const int r9 = id % 9, cot = id / 9, co = cot * 16 + m;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int dxi = 0; dxi < 3; ++dxi)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            out[off_W2 + (co * C + rt * 16 + 4 * j + i) * T + 3 * r9 + dxi] = acc2[k][rt][dxi][i];
    }
  }
#pragma unroll
  for (int k = 0; k < JS31; ++k) {
    const int id = k * NW + w;
    if (id < J31) {
      const bool w3 = id < N3;
      const int id2 = w3 ? id : id - N3, rt = id2 % RT, ct = id2 / RT, col = ct * 16 + m;
      const int tap = w3 ? col >> 1 : col, co = col & 1;
      if (tap < T)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = rt * 16 + 4 * j + i;
          out[w3 ? off_W3 + (co * C + c) * T + tap : off_W1 + c * T + tap] = acc31[k][i];
        }
    }
  }
}

// ---- host -----------------------------------------------------------------

template <int L, int C>
int rb_grid(int B) {
  return std::min(B, num_cus());
}

template <int L, int C>
size_t rb_ws(const FlowGeom& g, int B) {
  using Cfg = RbCfg<L, C>;
  const size_t BV = (size_t)B * Cfg::V;
  return align_up((size_t)Cfg::FRAGS * 64 * 16 * g.N) +
         2 * align_up((size_t)rb_grid<L, C>(B) * Cfg::P_LAYER * 4) + 2 * align_up(BV * 4) +
         4 * align_up(BV * C * 2) + 3 * align_up(BV * 4);
}

template <class K>
bool set_lds(K kern, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

template <int L, int C>
int32_t rb_run(const FlowGeom& g, const float* params, int B, const float* saved,
               const unsigned char* hsave, const float* g_phi, double g_logq, const double* g_logq_vec,
               float* g_params, float* g_z, char* ws, hipStream_t st) {
  using Cfg = RbCfg<L, C>;
  const int grid = rb_grid<L, C>(B);
  const FragTable tab = bwd_table(g, true, false);
  if (tab.total != Cfg::FRAGS || (int)g.P_layer != Cfg::P_LAYER) return LFS_EUNSUPPORTED;
  const size_t BV = (size_t)B * Cfg::V;
  char* p = ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += align_up(bytes);
    return r;
  };
  u32x4* frags = reinterpret_cast<u32x4*>(take((size_t)Cfg::FRAGS * 64 * 16 * g.N));
  // two partial buffers: a layer's first launch (recompute or affine backward)
  // reduces the previous layer's partials
  float* partials[2] = {reinterpret_cast<float*>(take((size_t)grid * Cfg::P_LAYER * 4)),
                        reinterpret_cast<float*>(take((size_t)grid * Cfg::P_LAYER * 4))};
  float* gbuf[2] = {reinterpret_cast<float*>(take(BV * 4)), reinterpret_cast<float*>(take(BV * 4))};
  uint16_t* h1c = reinterpret_cast<uint16_t*>(take(BV * C * 2));
  uint16_t* h2c = reinterpret_cast<uint16_t*>(take(BV * C * 2));
  uint16_t* ga2c = reinterpret_cast<uint16_t*>(take(BV * C * 2));
  uint16_t* ga1c = reinterpret_cast<uint16_t*>(take(BV * C * 2));
  uint32_t* go = reinterpret_cast<uint32_t*>(take(BV * 4));
  uint32_t* m1 = reinterpret_cast<uint32_t*>(take(BV * 4));
  uint32_t* m2 = reinterpret_cast<uint32_t*>(take(BV * 4));

  const long nthreads = (long)tab.total * 64 * g.N;
  hipLaunchKernelGGL((kf_prep<true>), dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st,
                     params, g.N, g.T, (int)g.P_layer, tab, frags);
  auto ka = kr_recompute<L, C, Cfg::NT_A>;
  // (512 threads: the fused reduction then reads whole 128-byte lines of every partial row)
  auto kaff = kr_affine<L, 512>;
  auto kb = kr_transpose<L, C, Cfg::NT_B>;
  auto kc = kr_wgrad<L, C, Cfg::NT_C>;
  if (!set_lds(ka, Cfg::LDS_A) || !set_lds(kb, Cfg::LDS_B) || !set_lds(kc, Cfg::LDS_C))
    return LFS_EDEVICE;
  const int P = Cfg::P_LAYER;
  const RingSave rs((size_t)B, C, Cfg::V);
  const float* gy = g_phi;
  int which = 0;
  for (int l = g.N - 1; l >= 0; --l) {
    float* gx = gbuf[which];
    const u32x4* fl = frags + (size_t)l * tab.total * 64;
    const float* pl = params + (size_t)l * g.P_layer;
    const float* xl = saved + (size_t)l * BV;
    const int fpar = g.frozen_parity(l);
    const bool first = l == g.N - 1;
    float* partial = partials[l & 1];
    const float* prev = first ? nullptr : (const float*)partials[(l + 1) & 1];
    float* prev_out = first ? nullptr : g_params + (size_t)(l + 1) * g.P_layer;
    const uint16_t *h1l = h1c, *h2l = h2c;
    const uint32_t *m1l = m1, *m2l = m2;
    if (hsave) {
      // the training forward's h1, h2, sign words and s: only the affine backward is left
      const unsigned char* hl = hsave + (size_t)l * rs.layer;
      h1l = reinterpret_cast<const uint16_t*>(hl + rs.h1);
      h2l = reinterpret_cast<const uint16_t*>(hl + rs.h2);
      m1l = reinterpret_cast<const uint32_t*>(hl + rs.m1);
      m2l = reinterpret_cast<const uint32_t*>(hl + rs.m2);
      hipLaunchKernelGGL(kaff, dim3(grid), dim3(512), 0, st, fpar, g.final_tanh, (float)(-g_logq), g_logq_vec,
                         B, xl, gy, reinterpret_cast<const float*>(hl + rs.s), gx, go, partial, P,
                         (int)g.off_b3, prev, prev_out);
    } else {
      hipLaunchKernelGGL(ka, dim3(grid), dim3(Cfg::NT_A), Cfg::LDS_A, st, fl, pl, (int)g.off_b1,
                         (int)g.off_b2, (int)g.off_b3, fpar, g.final_tanh, (float)(-g_logq), g_logq_vec, B,
                         xl, gy, gx, h1c, h2c, m1, m2, go, partial, P, prev, prev_out);
    }
    hipLaunchKernelGGL(kb, dim3(grid), dim3(Cfg::NT_B), Cfg::LDS_B, st, fl, fpar, B,
                       (const uint32_t*)go, m1l, m2l, gy, gx, ga2c, ga1c, partial, P, (int)g.off_b1,
                       (int)g.off_b2);
    hipLaunchKernelGGL(kc, dim3(grid), dim3(Cfg::NT_C), Cfg::LDS_C, st, fpar, B, xl, h1l, h2l,
                       (const uint32_t*)go, (const uint16_t*)ga2c, (const uint16_t*)ga1c, partial, P,
                       (int)g.off_W1, (int)g.off_W2, (int)g.off_W3);
    gy = gx;
    which ^= 1;
  }
  hipLaunchKernelGGL(kf_reduce, dim3((P + kRedCols - 1) / kRedCols), dim3(kRedCols * kRedSlices), 0,
                     st, grid, P, (const float*)partials[0], g_params);
  if (g_z)
    hipLaunchKernelGGL(kf_gz, dim3((unsigned)((BV + 255) / 256)), dim3(256), 0, st, (int64_t)BV,
                       gy, saved, (float)g_logq, g_logq_vec, (int64_t)g.V, g_z);
  return launch_status();
}

struct RbEntry {
  int L, C;
  int32_t (*fn)(const FlowGeom&, const float*, int, const float*, const unsigned char*, const float*,
                double, const double*, float*, float*, char*, hipStream_t);
  size_t (*ws)(const FlowGeom&, int);
};

const RbEntry kRbTable[] = {RbEntry{16, 16, &rb_run<16, 16>, &rb_ws<16, 16>},
                            RbEntry{16, 32, &rb_run<16, 32>, &rb_ws<16, 32>}};

const RbEntry* find_rb(const FlowGeom& g) {
  if (g.dim != 3 || !g.bf16()) return nullptr;
  for (const auto& e : kRbTable)
    if (e.L == g.L && e.C == g.C) return &e;
  return nullptr;
}

}  // namespace

bool ring_bwd_supported(const FlowGeom& g) { return find_rb(g) != nullptr; }
size_t ring_bwd_ws_bytes(const FlowGeom& g, int B) {
  const RbEntry* e = find_rb(g);
  return e ? e->ws(g, B) : 0;
}
int32_t ring_bwd_run(const FlowGeom& g, const float* params, int B, const float* saved,
                     const unsigned char* hsave, const float* g_phi, double g_logq,
                     const double* g_logq_vec, float* g_params, float* g_z, char* ws, hipStream_t st) {
  const RbEntry* e = find_rb(g);
  if (!e) return LFS_EUNSUPPORTED;
  return e->fn(g, params, B, saved, hsave, g_phi, g_logq, g_logq_vec, g_params, g_z, ws, st);
}

}  // namespace fused
}  // namespace lfs

// Fused flow forward for 3D lattices whose hidden activations do not fit LDS
// (L = 16: 128-256 KB per tensor per sample).  One workgroup still owns a whole
// sample and runs every coupling layer (paper Sec. 1, coupling-layer and
// composition equations), but the hidden activations stream along axis 0
// through rings of three planes:
//
//   for output plane z:  h1[z+2]  (conv1 of the masked field, planes z+1..z+3)
//                        h2[z+1]  (conv2 of h1 planes z..z+2)
//                        conv3 of h2 planes z-1..z+1 at the active sites of
//                        plane z, affine update, log-det
//
// Planes are indexed by a virtual plane number that runs from -2 to L+1, so the
// ring slot of virtual plane v is v mod 3 even across the periodic seam; the
// seam costs two extra conv1 planes and two extra conv2 planes per layer.  The
// field x is resident for the whole sample on a padded lattice; ring planes
// carry an in-plane periodic halo, so every gather is a base address plus a
// per-tap constant.  conv3 only changes active sites, and conv1 only reads
// frozen sites, so the update of plane z can overlap the next plane's conv1.
#include <type_traits>

#include "fused_kernels.hpp"
#include "lfs_internal.hpp"

namespace lfs {
namespace fused {
namespace {

constexpr double kHalfLog2PiR = 0.91893853320467274178;

template <int L, int C, bool BF16>
struct RingCfg {
  using G = Geo<3, L>;
  using LX = Lay<3, L, true>;   // the field
  using LP2 = Lay<2, L, true>;  // one plane of a ring
  static constexpr int V = G::V, T = 27, PS = LP2::VS, LP = L + 2;
  static constexpr LayerFrags LF = layer_frags(T, C, BF16);
  static constexpr size_t XS_BYTES = ((size_t)LX::VS * 4 + 15) / 16 * 16;
  static constexpr int ZS = 3 * PS;  // all-zero site after the three planes
  static constexpr size_t RING = (3 * (size_t)PS + 1) * C * sizeof(HElem<BF16>);
  // Two output-channel tiles (C = 32): eight waves, four per tile, so that a
  // wave holds one tile's conv1/conv2 fragments and conv3's come from LDS; the
  // registers then admit two waves per SIMD instead of one.
  static constexpr int NT = LF.nct == 2 ? 512 : 256;
  static constexpr bool A3_HELD = LF.nct == 1;
  // conv3's A operand has two live rows (s and t): lanes 16 j + m with m < 2.  A
  // compact LDS table holds those 8 lanes' entries per chunk (copied once per
  // layer), and every lane reads entry 2 j + (m & 1), so rows 2..15 repeat rows 0
  // and 1; those rows of the product are never read.
  static constexpr size_t T3_BYTES = A3_HELD ? 0 : (size_t)LF.k2 * 8 * 16;
  // BF16: conv1's operands as row triples of the masked field (x-1, x, x+1, 0 per
  // site, 8 bytes) in a ring of five planes, each built one step ahead of the
  // conv1 passes that read it (three planes per pass, five in the prologue)
  static constexpr bool TRIR = BF16;
  static constexpr size_t TRI_BYTES = TRIR ? 5 * (size_t)L * L * 8 : 0;
  static constexpr size_t lds_bytes = XS_BYTES + 2 * RING + T3_BYTES + TRI_BYTES;
};

__device__ __forceinline__ int mod3(int v) { return ((v % 3) + 3) % 3; }
__device__ __forceinline__ int mod5(int v) { return ((v % 5) + 5) % 5; }

// B operand of a C-input convolution on a ring: in-plane storage index pq of the
// output site, the ring slots of planes v-1, v, v+1.
template <int L, int C, bool BF16>
__device__ __forceinline__ u32x4 gather_ring(const HElem<BF16>* ring, int pq, int sm, int s0, int sp,
                                             int c, int j) {
  using Cfg = RingCfg<L, C, BF16>;
  constexpr int K = 27 * C;
  const int k0 = BF16 ? 32 * c + 8 * j : 16 * c + 4 * j;
  const int tap = k0 / C, ci0 = k0 % C;
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int slot = dz < 0 ? sm : (dz > 0 ? sp : s0);
  const int e = k0 < K ? (slot * Cfg::PS + pq + dy * Cfg::LP + dx) * C + ci0 : Cfg::ZS * C;
  return *reinterpret_cast<const u32x4*>(ring + e);
}

// shapes whose plane-streaming backward reads saved activations
template <int L, int C, bool BF16>
constexpr bool ring_saves() {
  return BF16 && L == 16 && (C == 16 || C == 32);
}

// SV (training, BF16): every layer's h1, h2, their sign words and s are also
// written to hsave (RingSave layout) for the backward.
template <int L, int C, bool BF16, int NT, bool SV = false>
__global__ void __launch_bounds__(NT) kf_forward_ring(
    const u32x4* __restrict__ frags, const float* __restrict__ params, int P_layer, int off_b1,
    int off_b2, int off_b3, int N, int parity0, int final_tanh, int B, const float* __restrict__ z,
    float* __restrict__ phi, float* __restrict__ saved, double* __restrict__ logq,
    double* __restrict__ logdet, unsigned char* __restrict__ hsave) {
  using Cfg = RingCfg<L, C, BF16>;
  using G = typename Cfg::G;
  using LX = typename Cfg::LX;
  using LP2 = typename Cfg::LP2;
  using HT = HElem<BF16>;
  using R = std::conditional_t<BF16, double, float>;
  constexpr int V = Cfg::V, PLANE = L * L, PS = Cfg::PS;
  constexpr LayerFrags LF = Cfg::LF;
  constexpr int NW = NT / 64;
  constexpr int WPC = NW / LF.nct;  // waves per output-channel tile
  static_assert(NW % LF.nct == 0, "waves split evenly over the channel tiles");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ R red[16];
  float* xs = reinterpret_cast<float*>(smem);
  HT* r1 = reinterpret_cast<HT*>(smem + Cfg::XS_BYTES);
  HT* r2 = r1 + (3 * PS + 1) * C;
  u32x4* t3 = reinterpret_cast<u32x4*>(smem + Cfg::XS_BYTES + 2 * Cfg::RING);
  uint16_t* tr = reinterpret_cast<uint16_t*>(smem + Cfg::XS_BYTES + 2 * Cfg::RING + Cfg::T3_BYTES);
  for (int q = threadIdx.x; q < C; q += NT) r1[Cfg::ZS * C + q] = HT(0), r2[Cfg::ZS * C + q] = HT(0);
  const int lane = threadIdx.x & 63, w = wave_id(), j = lane >> 4, m = lane & 15;
  // this wave's channel tile and its index among that tile's waves
  const int ct = LF.nct == 1 ? 0 : w / WPC, wc = LF.nct == 1 ? w : w % WPC;
  const size_t BV = (size_t)B * V;
  // the lane's four triple rows (chunk c, slot u: row r = 8 c + 2 j + u, past the nine
  // rows (dz, dy) = (r / 3 - 1, r % 3 - 1) the centre row, which meets zero weights)
  int tdz[4], tdy[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r0 = 8 * (i >> 1) + 2 * j + (i & 1), r = r0 < 9 ? r0 : 4;
    tdz[i] = r / 3 - 1;
    tdy[i] = r % 3 - 1;
  }

  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    R zz = 0;
    {
      const float* zb = z + (size_t)b * V;
      for (int q = threadIdx.x; q < LX::VS; q += NT) xs[q] = zb[LX::site_of(q)];
      for (int n = threadIdx.x; n < V; n += NT) {
        const float v = zb[n];
        if (saved) saved[(size_t)b * V + n] = v;
        zz += (R)v * v;
      }
    }
    R ld = 0;
    for (int layer = 0; layer < N; ++layer) {
      const int fpar = (layer + parity0) & 1, apar = fpar ^ 1;
      const u32x4* fl = frags + (size_t)layer * LF.total * 64 + lane;
      const float* pl = params + (size_t)layer * P_layer;
      u32x4 A1[LF.k1], A2[LF.k2], A3[Cfg::A3_HELD ? LF.k2 : 1];
      const f32x4 bias1 = load_bias4<C>(pl + off_b1, ct, j), bias2 = load_bias4<C>(pl + off_b2, ct, j);
#pragma unroll
      for (int c = 0; c < LF.k1; ++c) A1[c] = fl[(LF.off1 + ct * LF.k1 + c) * 64];
#pragma unroll
      for (int c = 0; c < LF.k2; ++c) A2[c] = fl[(LF.off2 + ct * LF.k2 + c) * 64];
      if constexpr (Cfg::A3_HELD) {
#pragma unroll
        for (int c = 0; c < LF.k2; ++c) A3[c] = fl[(LF.off3 + c) * 64];
      }
      const float bs = pl[off_b3], bt = pl[off_b3 + 1];
      // SV: this layer's and sample's saved tensors
      uint16_t *sh1 = nullptr, *sh2 = nullptr;
      uint32_t *sm1 = nullptr, *sm2 = nullptr;
      float* ssv = nullptr;
      if constexpr (SV) {
        const RingSave rs((size_t)B, C, V);
        unsigned char* hl = hsave + (size_t)layer * rs.layer;
        sh1 = reinterpret_cast<uint16_t*>(hl + rs.h1) + (size_t)b * C * V;
        sh2 = reinterpret_cast<uint16_t*>(hl + rs.h2) + (size_t)b * C * V;
        sm1 = reinterpret_cast<uint32_t*>(hl + rs.m1) + (size_t)b * V;
        sm2 = reinterpret_cast<uint32_t*>(hl + rs.m2) + (size_t)b * V;
        ssv = reinterpret_cast<float*>(hl + rs.s) + (size_t)b * V;
      }
      // SV: real plane zr of a ring (its slot) to the channel-major copy hc and the sign
      // words mk, by all threads while the plane is only read (between the barrier after
      // the pass that wrote it and the pass that overwrites its slot): item (g, q) takes
      // channels 8g .. 8g + 7 of in-plane site q, consecutive threads consecutive sites
      auto save_plane = [&](const HT* ring, int slot, int zr, uint16_t* hc, uint32_t* mk) {
        if constexpr (SV) {
          constexpr int NG = C / 8;
          // the thread index made opaque here, so that the items' offsets are computed
          // at each call instead of being hoisted out of the plane loop and held in
          // registers across the convolutions
          int t0 = threadIdx.x;
          asm volatile("" : "+v"(t0));
#pragma unroll 1
          for (int i = t0; i < NG * PLANE; i += NT) {
            const int g = i / PLANE, q = i - g * PLANE;
            const uint32_t* src = reinterpret_cast<const uint32_t*>(ring + (slot * PS + LP2::idx(q)) * C + 8 * g);
            const int n = zr * PLANE + q;  // 32-bit offsets from the uniform base hc
            uint32_t bits = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const uint32_t hw = src[k];
              hc[(8 * g + 2 * k) * V + n] = (uint16_t)hw;
              hc[(8 * g + 2 * k + 1) * V + n] = (uint16_t)(hw >> 16);
              bits |= (uint32_t)(bf16_lo(hw) >= 0.f) << (2 * k) | (uint32_t)(bf16_hi(hw) >= 0.f) << (2 * k + 1);
            }
            // byte g of site n's word holds channels 8g .. 8g + 7 (bit c: channel c)
            uint8_t* mb = reinterpret_cast<uint8_t*>(mk + n);
            mb[g] = (uint8_t)bits;
            if constexpr (C == 16) mb[g + 2] = 0;
          }
        }
      };

      // row triples of the masked field of virtual plane v into triple-ring slot v mod 5
      // (only frozen sites' values enter, which conv3 never changes)
      auto build_tri_plane = [&](int v) {
        const int zr = ((v % L) + L) % L;
        uint16_t* dst = tr + mod5(v) * PLANE * 4;
        for (int q = threadIdx.x; q < PLANE; q += NT) {
          const int n = zr * PLANE + q, p = LX::idx(n);
          const bool frozen = G::parity(n) == fpar;  // the x neighbours have the other parity
          const float v0 = frozen ? 0.f : xs[p - 1], v1 = frozen ? xs[p] : 0.f, v2 = frozen ? 0.f : xs[p + 1];
          *reinterpret_cast<u32x2*>(dst + 4 * q) = u32x2{pack_bf16(v0, v1), pack_bf16(v2, 0.f)};
        }
      };
      // h1 of virtual plane v into ring slot v mod 3
      auto conv1_plane = [&](int v) {
        const int zr = ((v % L) + L) % L;
        HT* dst = r1 + mod3(v) * PS * C;
        int tbase[4];  // the lane's triple rows: ring slot of plane v + dz, as an element offset
        if constexpr (Cfg::TRIR) {
          const int sm = mod5(v - 1) * PLANE, s0 = mod5(v) * PLANE, sp = mod5(v + 1) * PLANE;
#pragma unroll
          for (int i = 0; i < 4; ++i) tbase[i] = tdz[i] < 0 ? sm : (tdz[i] > 0 ? sp : s0);
        }
        for (int tile = wc; tile < PLANE / 16; tile += WPC) {
          const int q = tile * 16 + m, n = zr * PLANE + q;
          f32x4 acc{0.f, 0.f, 0.f, 0.f};
          if constexpr (Cfg::TRIR) {
            // tile = in-plane row y, m = x
#pragma unroll
            for (int c = 0; c < LF.k1; ++c) {
              const int e0 = (tbase[2 * c] + ((tile + tdy[2 * c]) & (L - 1)) * L + m) * 4;
              const int e1 = (tbase[2 * c + 1] + ((tile + tdy[2 * c + 1]) & (L - 1)) * L + m) * 4;
              const u32x2 a = *reinterpret_cast<const u32x2*>(tr + e0), b = *reinterpret_cast<const u32x2*>(tr + e1);
              acc = mma<BF16>(A1[c], u32x4{a[0], a[1], b[0], b[1]}, acc);
            }
          } else {
            const int p = LX::idx(n), pn = G::parity(n);
#pragma unroll
            for (int c = 0; c < LF.k1; ++c) acc = mma<BF16>(A1[c], gather_tri_x<LX, BF16>(xs, n, p, pn, fpar, c, j), acc);
          }
          store_hidden<LP2, C, BF16>(dst, q, ct, j, acc, bias1);
        }
      };
      // h2 of virtual plane v from h1 planes v-1, v, v+1
      auto conv2_plane = [&](int v) {
        HT* dst = r2 + mod3(v) * PS * C;
        const int sm = mod3(v - 1), s0 = mod3(v), sp = mod3(v + 1);
        for (int tile = wc; tile < PLANE / 16; tile += WPC) {
          const int q = tile * 16 + m, pq = tile_p<LP2>(tile, m);
          f32x4 acc{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int c = 0; c < LF.k2; ++c) acc = mma<BF16>(A2[c], gather_ring<L, C, BF16>(r1, pq, sm, s0, sp, c, j), acc);
          store_hidden<LP2, C, BF16>(dst, q, ct, j, acc, bias2);
        }
      };
      // conv3 of h2 planes z-1, z, z+1 at the active sites of plane z; affine update
      auto conv3_plane = [&](int zr) {
        const int sm = mod3(zr - 1), s0 = mod3(zr), sp = mod3(zr + 1);
        const int ppar = apar ^ (zr & 1);  // in-plane parity of the active sites
        for (int tile = w; tile < PLANE / 32; tile += NW) {
          const int q = Geo<2, L>::half_site(tile * 16 + m, ppar), pq = LP2::idx(q);
          // two accumulator chains (even and odd chunks), summed at the end
          auto a3_of = [&](int c) -> u32x4 {
            if constexpr (Cfg::A3_HELD)
              return A3[c];
            else
              return t3[c * 8 + 2 * j + (m & 1)];
          };
          f32x4 ae{0.f, 0.f, 0.f, 0.f}, ao{0.f, 0.f, 0.f, 0.f};
#pragma unroll Cfg::A3_HELD ? LF.k2 / 2 : 4
          for (int c = 0; c + 1 < LF.k2; c += 2) {
            ae = mma<BF16>(a3_of(c), gather_ring<L, C, BF16>(r2, pq, sm, s0, sp, c, j), ae);
            ao = mma<BF16>(a3_of(c + 1), gather_ring<L, C, BF16>(r2, pq, sm, s0, sp, c + 1, j), ao);
          }
          if constexpr (LF.k2 % 2) ae = mma<BF16>(a3_of(LF.k2 - 1), gather_ring<L, C, BF16>(r2, pq, sm, s0, sp, LF.k2 - 1, j), ae);
          const f32x4 acc = ae + ao;
          if (j == 0) {
            const int n = zr * PLANE + q;
            const float o0 = acc[0] + bs, t = acc[1] + bt;
            const float s = final_tanh ? fast_tanh(o0) : o0;
            const float xn = xs[LX::idx(n)] * fast_exp(s) + t;
            LX::copies(n, [&](int qq) { xs[qq] = xn; });
            ld += (R)s;
            if constexpr (SV) ssv[n] = s;
          }
        }
      };

      __syncthreads();  // field of the previous layer complete
      if constexpr (!Cfg::A3_HELD) {
        // conv3's live A rows into the compact table (read after the next barriers)
        const u32x4* f3 = frags + ((size_t)layer * LF.total + LF.off3) * 64;
        for (int i = threadIdx.x; i < LF.k2 * 8; i += NT) t3[i] = f3[(i >> 3) * 64 + 16 * ((i & 7) >> 1) + (i & 1)];
      }
      if constexpr (Cfg::TRIR) {
        for (int v = -3; v <= 1; ++v) build_tri_plane(v);
        __syncthreads();
      }
      conv1_plane(-2);
      conv1_plane(-1);
      conv1_plane(0);
      __syncthreads();
      conv2_plane(-1);
      save_plane(r1, mod3(0), 0, sh1, sm1);
      if constexpr (Cfg::TRIR) build_tri_plane(2);  // over plane -3's triples, last read by conv1(-2)
      __syncthreads();
      conv1_plane(1);
      __syncthreads();
      conv2_plane(0);
      save_plane(r1, mod3(1), 1, sh1, sm1);
      if constexpr (Cfg::TRIR) build_tri_plane(3);
      __syncthreads();
      save_plane(r2, mod3(0), 0, sh2, sm2);
      for (int zr = 0; zr < L; ++zr) {
        conv1_plane(zr + 2);  // triples of planes zr + 1 .. zr + 3
        __syncthreads();
        conv2_plane(zr + 1);
        if (zr + 2 < L) save_plane(r1, mod3(zr + 2), zr + 2, sh1, sm1);
        // plane zr + 4's triples (for the next conv1) over plane zr - 1's, last read by conv1(zr)
        if constexpr (Cfg::TRIR) build_tri_plane(zr + 4);
        __syncthreads();
        if (zr + 1 < L) save_plane(r2, mod3(zr + 1), zr + 1, sh2, sm2);
        conv3_plane(zr);
      }
      __syncthreads();
      if (saved) {
        float* sv = saved + (size_t)(layer + 1) * BV + (size_t)b * V;
        for (int n = threadIdx.x; n < V; n += NT) sv[n] = xs[LX::idx(n)];
      }
    }
    {
      float* pb = phi + (size_t)b * V;
      for (int n = threadIdx.x; n < V; n += NT) pb[n] = xs[LX::idx(n)];
    }
    ld = block_sum(ld, red);
    zz = block_sum(zz, red);
    if (threadIdx.x == 0) {
      const double logr = -0.5 * (double)zz - (double)V * kHalfLog2PiR;
      logq[b] = logr - (double)ld;
      if (logdet) logdet[b] = (double)ld;
    }
  }
}

template <int L, int C, bool BF16>
int32_t launch_ring(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                    double* logq, double* logdet, float* saved, unsigned char* hsave, char* ws,
                    hipStream_t st) {
  using Cfg = RingCfg<L, C, BF16>;
  constexpr LayerFrags LF = Cfg::LF;
  static_assert(Cfg::lds_bytes <= 160 * 1024, "LDS budget");
  u32x4* frags = reinterpret_cast<u32x4*>(ws);
  FragTable tab{};
  tab.count = 3;
  tab.s[0] = FragSpec{0, (int)g.off_W1, 1, C, C, LF.nct, LF.k1, LF.off1, 1};
  tab.s[1] = FragSpec{0, (int)g.off_W2, C, C, C, LF.nct, LF.k2, LF.off2};
  tab.s[2] = FragSpec{0, (int)g.off_W3, C, 2, 2, 1, LF.k2, LF.off3};
  tab.total = LF.total;
  const long nthreads = (long)LF.total * 64 * g.N;
  hipLaunchKernelGGL((kf_prep<BF16>), dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st,
                     params, g.N, g.T, (int)g.P_layer, tab, frags);
  auto kern = kf_forward_ring<L, C, BF16, Cfg::NT, false>;
  if constexpr (ring_saves<L, C, BF16>())
    if (hsave) kern = kf_forward_ring<L, C, BF16, Cfg::NT, true>;
  if (!ring_saves<L, C, BF16>()) hsave = nullptr;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)Cfg::lds_bytes) !=
      hipSuccess)
    return LFS_EDEVICE;
  hipLaunchKernelGGL(kern, dim3(B), dim3(Cfg::NT), Cfg::lds_bytes, st, frags, params,
                     (int)g.P_layer, (int)g.off_b1, (int)g.off_b2, (int)g.off_b3, g.N, g.parity0,
                     g.final_tanh, B, z, phi, saved, logq, logdet, hsave);
  return launch_status();
}

struct RingEntry {
  int L, C;
  bool bf16;
  int32_t (*fn)(const FlowGeom&, const float*, int, const float*, float*, double*, double*, float*,
                unsigned char*, char*, hipStream_t);
  size_t frag_bytes_per_layer;
  bool saves;  // the training forward saves the activations (RingSave) for the backward
};

template <int L, int C, bool BF16>
constexpr RingEntry ring_entry() {
  return RingEntry{L, C, BF16, &launch_ring<L, C, BF16>,
                   (size_t)RingCfg<L, C, BF16>::LF.total * 64 * 16, ring_saves<L, C, BF16>()};
}

const RingEntry kRingTable[] = {ring_entry<16, 8, false>(), ring_entry<16, 8, true>(),
                                ring_entry<16, 16, false>(), ring_entry<16, 16, true>(),
                                ring_entry<16, 32, true>()};

const RingEntry* find_ring(const FlowGeom& g) {
  if (g.dim != 3) return nullptr;
  for (const auto& e : kRingTable)
    if (e.L == g.L && e.C == g.C && e.bf16 == g.bf16()) return &e;
  return nullptr;
}

}  // namespace

bool ring_supported(const FlowGeom& g) { return find_ring(g) != nullptr; }
size_t ring_ws_bytes(const FlowGeom& g) {
  const RingEntry* e = find_ring(g);
  return e ? align_up(e->frag_bytes_per_layer * g.N) : 0;
}
int32_t ring_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                     double* logq, double* logdet, float* saved, unsigned char* hsave, char* ws,
                     hipStream_t st) {
  const RingEntry* e = find_ring(g);
  if (!e) return LFS_EUNSUPPORTED;
  return e->fn(g, params, B, z, phi, logq, logdet, saved, hsave, ws, st);
}
size_t ring_hsave_bytes(const FlowGeom& g, int B) {
  const RingEntry* e = find_ring(g);
  if (!e || !e->saves) return 0;
  return RingSave((size_t)B, g.C, g.V).layer * g.N;
}

}  // namespace fused
}  // namespace lfs

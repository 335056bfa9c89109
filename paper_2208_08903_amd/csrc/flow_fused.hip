// Fused flow forward: one workgroup per sample with the whole lattice and
// both hidden activations resident in LDS, all coupling layers in one launch,
// and every convolution on the matrix cores (implicit GEMM, see
// fused_common.hpp).  Paper Sec. 1, coupling-layer and composition equations.
//
// Per layer l (frozen parity f = (l + parity0) mod 2, active parity 1 - f):
//   conv1: h1 = leaky(W1 * mask_F x + b1)   over all V sites   (K = T taps; FP32 2D
//          L = 32 on the vector ALUs, see conv1_valu)
//   conv2: h2 = leaky(W2 * h1 + b2)         over all V sites   (K = T C)
//   conv3: (o0, o1) = W3 * h2 + b3          at the V/2 active sites only (FP32: on the
//          4x4 matrix-core blocks, see quad_conv)
//          x <- x exp(s) + t, s = tanh(o0) (or o0), t = o1; logdet += sum s
// Three workgroup barriers per layer separate the phases.  The training forward
// (FP32 2D L = 32) also writes h2 and s for the backward (HSave).
#include <type_traits>

#include "fused_kernels.hpp"
#include "lfs_internal.hpp"

namespace lfs {
namespace fused {
namespace {

constexpr double kHalfLog2Pi = 0.91893853320467274178;

template <int DIM, int L, int C, bool BF16, int NT>
__global__ void __launch_bounds__(NT) kf_forward(
    const u32x4* __restrict__ frags, const float* __restrict__ params, int P_layer, int off_b1,
    int off_b2, int off_b3, int N, int parity0, int final_tanh, int B, const float* __restrict__ z,
    float* __restrict__ phi, float* __restrict__ saved, double* __restrict__ logq,
    double* __restrict__ logdet, float* __restrict__ hsave, int off_W1) {
  using Cfg = FwdCfg<DIM, L, C, BF16>;
  using G = Geo<DIM, L>;
  using LY = typename Cfg::LY;
  using HT = HElem<BF16>;
  using R = std::conditional_t<BF16, double, float>;
  using HS = HSave<DIM, L, C, BF16>;
  constexpr int V = Cfg::V, VS = LY::VS;
  constexpr LayerFrags LF = Cfg::LF;
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ R red[16];
  float* xs = reinterpret_cast<float*>(smem);
  HT* h1 = reinterpret_cast<HT*>(smem + ((LY::VSZ * 4 + 15) / 16) * 16);
  HT* h2 = h1 + LY::template elems<C>();
  u32x4* qt = reinterpret_cast<u32x4*>(h2 + LY::template elems<C>());  // FP32: the layer's conv3 A table
  // C1V: conv1's weights and biases, tap-major (the first layer's staged here, the
  // next layer's during conv3; visible after the layer-start barrier)
  float* w1t = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(qt) + Cfg::QT_BYTES);
  if constexpr (Cfg::C1V) stage_w1t<C, NT>(w1t, params, off_W1, off_b1);
  for (int q = threadIdx.x; q < C; q += NT) h1[LY::template off<C>(LY::ZS, q)] = 0, h2[LY::template off<C>(LY::ZS, q)] = 0;
  const int lane = threadIdx.x & 63, w = wave_id(), j = lane >> 4, m = lane & 15;
  const size_t BV = (size_t)B * V;

  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    R zz = 0;
    {
      const float* zb = z + (size_t)b * V;
      for (int q = threadIdx.x; q < VS; q += NT) xs[q] = zb[LY::site_of(q)];
      for (int n = threadIdx.x; n < V; n += NT) {
        const float v = zb[n];
        if (saved) saved[(size_t)b * V + n] = v;
        zz += (R)v * v;
      }
    }
    R ld = 0;
    for (int layer = 0; layer < N; ++layer) {
      const int fpar = (layer + parity0) & 1;
      const u32x4* fl = frags + (size_t)layer * LF.total * 64 + lane;
      const float* pl = params + (size_t)layer * P_layer;
      __syncthreads();
      if constexpr (Cfg::Q3) {
        // conv3's quad A entries (rows 0..3 of every chunk) into LDS: read by every
        // conv3 chunk of every wave, visible after the next barrier
        const u32x4* f3 = frags + ((size_t)layer * LF.total + LF.off3) * 64;
        for (int i = threadIdx.x; i < LF.k3 * 4; i += NT) qt[i] = f3[(i >> 2) * 64 + (i & 3)];
      }
      // Weight fragments.  Where the registers allow (Cfg::PFA) each pass's are
      // fetched one pass ahead, so the L2 latency hides behind the previous
      // pass: conv1's and conv2's here, conv3's when conv2 starts; otherwise
      // each pass fetches its own.
      constexpr int NA3 = Cfg::X4 ? 4 : 1;
      constexpr int KA3 = Cfg::Q3 ? 1 : LF.k2;  // quad conv3 fetches its fragments per chunk
      u32x4 A1[LF.nct][LF.k1], A2[LF.nct][LF.k2], A3[NA3][KA3];
      auto load_a1 = [&]() {
#pragma unroll
        for (int ct = 0; ct < LF.nct; ++ct)
#pragma unroll
          for (int c = 0; c < LF.k1; ++c) A1[ct][c] = fl[(LF.off1 + ct * LF.k1 + c) * 64];
      };
      auto load_a2 = [&]() {
#pragma unroll
        for (int ct = 0; ct < LF.nct; ++ct)
#pragma unroll
          for (int c = 0; c < LF.k2; ++c) A2[ct][c] = fl[(LF.off2 + ct * LF.k2 + c) * 64];
      };
      auto load_a3 = [&]() {
        if constexpr (!Cfg::Q3) {
#pragma unroll
          for (int c = 0; c < LF.k2; ++c) {
            A3[0][c] = fl[(LF.off3 + c) * 64];
#pragma unroll
            for (int u = 1; u < NA3; ++u) A3[u][c] = fl[(LF.off3q + (u - 1) * LF.k2 + c) * 64];
          }
        }
      };
      if constexpr (Cfg::PFA) {
        if constexpr (!Cfg::C1V) load_a1();
        load_a2();
      }
      // conv1 operands: row triples of the masked field, built in the (dead) h2
      // buffer, or (Cfg::TRIX) gathered straight from the field by each tile
      if constexpr (!Cfg::TRIX) {
        build_tri<LY, BF16, NT>(h2, xs, fpar);
        __syncthreads();
      }
      // conv1 over all sites
      if constexpr (Cfg::C1V) {
        conv1_valu<LY, C, NT>(xs, h1, w1t, fpar);
      } else {
        if constexpr (!Cfg::PFA) load_a1();
        f32x4 bias[LF.nct];
#pragma unroll
        for (int ct = 0; ct < LF.nct; ++ct) bias[ct] = load_bias4<C>(pl + off_b1, ct, j);
        mma_tiles<Cfg::TU1, LF.nct, LF.k1, BF16, k_tri(Cfg::T), true>(
            V / 16, w, NW, A1, bias,
            [&](int tile, int c) {
              if constexpr (Cfg::TRIX) {
                const int n = tile * 16 + m;
                return gather_tri_x<LY, BF16>(xs, n, LY::idx(n), G::parity(n), fpar, c, j);
              } else {
                return gather_tri<LY, BF16>(h2, tile * 16 + m, tile_p<LY>(tile, m), c, j);
              }
            },
            [&](int tile, const f32x4(&acc)[LF.nct]) {
#pragma unroll
              for (int ct = 0; ct < LF.nct; ++ct) store_act_tile<LY, C, BF16, false>(h1, tile, m, ct, j, acc[ct]);
            });
      }
      __syncthreads();
      if constexpr (LY::padded) {
        fill_halo<LY, C, BF16, NT>(h1);
        __syncthreads();
      }
      // conv2 over all sites
      {
        if constexpr (Cfg::PFA)
          load_a3();
        else
          load_a2();
        f32x4 bias[LF.nct];
#pragma unroll
        for (int ct = 0; ct < LF.nct; ++ct) bias[ct] = load_bias4<C>(pl + off_b2, ct, j);
        mma_tiles<Cfg::TU2, LF.nct, LF.k2, BF16>(
            V / 16, w, NW, A2, bias,
            [&](int tile, int c) {
              return gather_h<LY, C, BF16>(h1, tile * 16 + m, tile_p<LY>(tile, m), c, j);
            },
            [&](int tile, const f32x4(&acc)[LF.nct]) {
#pragma unroll
              for (int ct = 0; ct < LF.nct; ++ct) store_act_tile<LY, C, BF16, false>(h2, tile, m, ct, j, acc[ct]);
              if constexpr (HS::ok) {
                // training: h2 saved for the backward (the same values as in LDS),
                // nontemporal: read back only by the backward, after every layer
                if (hsave) {
                  float* hb = hsave + ((size_t)layer * B + b) * (HS::sample_bytes / 4);
#pragma unroll
                  for (int ct = 0; ct < LF.nct; ++ct) {
                    const int co0 = ct * 16 + 4 * j;
                    if (co0 < C)
                      __builtin_nontemporal_store(
                          f32x4{leaky(acc[ct][0]), leaky(acc[ct][1]), leaky(acc[ct][2]), leaky(acc[ct][3])},
                          reinterpret_cast<f32x4*>(hb + HS::off4(tile * 16 + m, co0)));
                  }
                }
              }
            });
      }
      __syncthreads();
      if constexpr (LY::padded) {
        fill_halo<LY, C, BF16, NT>(h2);
        __syncthreads();
      }
      // conv3 at the active sites, affine update and log-det
      if constexpr (!Cfg::PFA) load_a3();
      if constexpr (Cfg::C1V)  // the next layer's (or next sample's first) conv1 weights
        stage_w1t<C, NT>(w1t, params + (size_t)(layer + 1 < N ? layer + 1 : 0) * P_layer, off_W1, off_b1);
      if constexpr (Cfg::Q3) {
        // FP32: 64 active sites per wave pass, one per lane, on the 4x4 blocks; every
        // lane updates its own site
        const int apar = fpar ^ 1;
        constexpr int NG = (V / 2 + 63) / 64;
        const f32x4 b3{pl[off_b3], pl[off_b3 + 1], 0.f, 0.f};
        for (int gi = w; gi < NG; gi += NW) {
          const int a = gi * 64 + lane;
          const bool valid = a < V / 2;
          const int n = G::half_site(valid ? a : 0, apar), p = LY::idx(n);
          const f32x4 o = quad_conv<LF.k3, 4>(qt + (lane & 3), b3,
                                              [&](int q) { return gather_q<LY, C>(h2, n, p, q); });
          if (valid) {
            const float s = final_tanh ? fast_tanh(o[0]) : o[0];
            const float xn = xs[p] * fast_exp(s) + o[1];
            LY::copies(n, [&](int q) { xs[q] = xn; });
            ld += (R)s;
            if constexpr (HS::ok)
              if (hsave) hsave[HS::s_off(N, B, layer, b) + a] = s;  // training: s for the backward
          }
        }
      } else if constexpr (Cfg::X4) {
        // four tiles share an accumulator: chunk c of tile u uses the fragments with
        // the outputs at rows 4u, 4u+1, so lane group j ends with tile j's s and t
        // and the epilogue runs on all 64 lanes (two chains: tiles 0-1 and 2-3)
        const auto& A = A3;
        const f32x4 b3{pl[off_b3], pl[off_b3 + 1], 0.f, 0.f};
        const int apar = fpar ^ 1;
        constexpr int NT3 = V / 32;
        for (int t0 = w; t0 < NT3; t0 += 4 * NW) {
          int n4[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) n4[u] = G::half_site((t0 + u * NW < NT3 ? t0 + u * NW : t0) * 16 + m, apar);
          f32x4 a01 = b3, a23{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int c = 0; c < LF.k2; ++c) {
            const u32x4 g0 = gather_h<LY, C, BF16>(h2, n4[0], LY::idx(n4[0]), c, j);
            const u32x4 g1 = gather_h<LY, C, BF16>(h2, n4[1], LY::idx(n4[1]), c, j);
            const u32x4 g2 = gather_h<LY, C, BF16>(h2, n4[2], LY::idx(n4[2]), c, j);
            const u32x4 g3 = gather_h<LY, C, BF16>(h2, n4[3], LY::idx(n4[3]), c, j);
            a01 = mma<BF16>(A[0][c], g0, a01);
            a23 = mma<BF16>(A[2][c], g2, a23);
            a01 = mma<BF16>(A[1][c], g1, a01);
            a23 = mma<BF16>(A[3][c], g3, a23);
          }
          if (t0 + j * NW < NT3) {
            const int n = G::half_site((t0 + j * NW) * 16 + m, apar), p = LY::idx(n);
            const float o0 = a01[0] + a23[0], t = a01[1] + a23[1];
            const float s = final_tanh ? fast_tanh(o0) : o0;
            const float xn = xs[p] * fast_exp(s) + t;
            LY::copies(n, [&](int q) { xs[q] = xn; });
            ld += (R)s;
          }
        }
      } else {
        const f32x4 b3[1] = {f32x4{pl[off_b3], pl[off_b3 + 1], 0.f, 0.f}};
        const int apar = fpar ^ 1;
        mma_tiles<Cfg::TU2, 1, LF.k2, BF16>(
            V / 32, w, NW, A3, b3,
            [&](int tile, int c) {
              const int n = G::half_site(tile * 16 + m, apar);
              return gather_h<LY, C, BF16>(h2, n, LY::idx(n), c, j);
            },
            [&](int tile, const f32x4(&acc)[1]) {
              if (j == 0) {
                const int n = G::half_site(tile * 16 + m, apar), p = LY::idx(n);
                const float o0 = acc[0][0], t = acc[0][1];
                const float s = final_tanh ? fast_tanh(o0) : o0;
                const float xn = xs[p] * fast_exp(s) + t;
                LY::copies(n, [&](int q) { xs[q] = xn; });
                ld += (R)s;
              }
            });
      }
      __syncthreads();
      if (saved) {
        float* sv = saved + (size_t)(layer + 1) * BV + (size_t)b * V;
        for (int n = threadIdx.x; n < V; n += NT) sv[n] = xs[LY::idx(n)];
      }
    }
    {
      float* pb = phi + (size_t)b * V;
      for (int n = threadIdx.x; n < V; n += NT) pb[n] = xs[LY::idx(n)];
    }
    ld = block_sum(ld, red);
    zz = block_sum(zz, red);
    if (threadIdx.x == 0) {
      const double logr = -0.5 * (double)zz - (double)V * kHalfLog2Pi;
      logq[b] = logr - (double)ld;
      if (logdet) logdet[b] = (double)ld;
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

template <int DIM, int L, int C, bool BF16>
int32_t launch_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                       double* logq, double* logdet, float* saved, float* hsave, char* ws,
                       hipStream_t st) {
  using Cfg = FwdCfg<DIM, L, C, BF16>;
  static_assert(Cfg::lds_bytes + 16 * 8 <= 160 * 1024, "LDS budget");
  constexpr LayerFrags LF = Cfg::LF;
  u32x4* frags = reinterpret_cast<u32x4*>(ws);
  FragTable tab{};
  tab.count = 3;
  tab.s[0] = FragSpec{0, (int)g.off_W1, 1, C, C, LF.nct, LF.k1, LF.off1, 1, 0};
  tab.s[1] = FragSpec{0, (int)g.off_W2, C, C, C, LF.nct, LF.k2, LF.off2, 0, 0};
  tab.s[2] = FragSpec{0, (int)g.off_W3, C, 2, 2, 1, LF.k3, LF.off3, 0, 0, LF.quad ? 1 : 0};
  if (LF.x4)
    for (int u = 1; u < 4; ++u)
      tab.s[tab.count++] = FragSpec{0, (int)g.off_W3, C, 2, 2, 1, LF.k2, LF.off3q + (u - 1) * LF.k2, 0, 4 * u};
  tab.total = LF.total;
  const long nthreads = (long)LF.total * 64 * g.N;
  hipLaunchKernelGGL((kf_prep<BF16>), dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st,
                     params, g.N, g.T, (int)g.P_layer, tab, frags);
  constexpr auto kern = kf_forward<DIM, L, C, BF16, Cfg::NT>;
  if (!set_lds_limit<kern>(Cfg::lds_bytes)) return LFS_EDEVICE;
  hipLaunchKernelGGL(kern, dim3(B), dim3(Cfg::NT), Cfg::lds_bytes, st, frags, params,
                     (int)g.P_layer, (int)g.off_b1, (int)g.off_b2, (int)g.off_b3, g.N, g.parity0,
                     g.final_tanh, B, z, phi, saved, logq, logdet,
                     HSave<DIM, L, C, BF16>::ok ? hsave : nullptr, (int)g.off_W1);
  return launch_status();
}

using FwdFn = int32_t (*)(const FlowGeom&, const float*, int, const float*, float*, double*,
                          double*, float*, float*, char*, hipStream_t);

struct FwdEntry {
  int dim, L, C;
  bool bf16;
  FwdFn fn;
  size_t frag_bytes_per_layer;
  size_t hsave_bytes_per_sample;  // 0: the backward recomputes h2
};

template <int DIM, int L, int C, bool BF16>
constexpr FwdEntry fwd_entry() {
  using HS = HSave<DIM, L, C, BF16>;
  return FwdEntry{DIM, L, C, BF16, &launch_forward<DIM, L, C, BF16>,
                  (size_t)FwdCfg<DIM, L, C, BF16>::LF.total * 64 * 16, HS::ok ? HS::sample_bytes + HS::s_bytes : 0};
}

// Shapes with a fused forward: the whole sample (field + two hidden tensors)
// fits in the 160 KB of LDS of one compute unit.
#define LFS_FWD_SHAPES(P)                                                                        \
  P(2, 8, 8) P(2, 8, 16) P(2, 8, 32) P(2, 16, 8) P(2, 16, 16) P(2, 16, 32) P(2, 32, 8)           \
  P(2, 32, 16) P(3, 4, 8) P(3, 4, 16) P(3, 8, 8) P(3, 8, 16) P(3, 12, 8)
#define LFS_FWD_BF16_ONLY(P) P(2, 32, 32) P(3, 12, 16)

#define LFS_E2(D, L, C) fwd_entry<D, L, C, false>(), fwd_entry<D, L, C, true>(),
#define LFS_E1(D, L, C) fwd_entry<D, L, C, true>(),

const FwdEntry kFwdTable[] = {LFS_FWD_SHAPES(LFS_E2) LFS_FWD_BF16_ONLY(LFS_E1)};

const FwdEntry* find_fwd(const FlowGeom& g) {
  for (const auto& e : kFwdTable)
    if (e.dim == g.dim && e.L == g.L && e.C == g.C && e.bf16 == g.bf16()) return &e;
  return nullptr;
}

}  // namespace
}  // namespace fused

bool fused_supported(const FlowGeom& g, int for_backward) {
  if (for_backward) return fused::bwd_supported(g) || fused::ring_bwd_supported(g);
  return fused::find_fwd(g) != nullptr || fused::ring_supported(g);
}

size_t fused_ws_bytes(const FlowGeom& g, int B, int for_backward) {
  if (for_backward)
    return fused::bwd_supported(g) ? fused::bwd_ws_bytes(g, B) : fused::ring_bwd_ws_bytes(g, B);
  if (!fused::find_fwd(g)) return fused::ring_ws_bytes(g);
  const fused::FwdEntry* e = fused::find_fwd(g);
  return e ? align_up(e->frag_bytes_per_layer * g.N) : 0;
}

int32_t fused_forward(const FlowGeom& g, const float* params, int B, const float* z, float* phi,
                      double* logq, double* logdet, float* saved, float* hsave, char* ws,
                      hipStream_t st) {
  const fused::FwdEntry* e = fused::find_fwd(g);
  if (!e)
    return fused::ring_forward(g, params, B, z, phi, logq, logdet, saved,
                               reinterpret_cast<unsigned char*>(hsave), ws, st);
  return e->fn(g, params, B, z, phi, logq, logdet, saved, hsave, ws, st);
}

size_t fused_hsave_bytes(const FlowGeom& g, int B) {
  const fused::FwdEntry* e = fused::find_fwd(g);
  if (!e) return fused::ring_bwd_supported(g) ? fused::ring_hsave_bytes(g, B) : 0;
  if (!e->hsave_bytes_per_sample || !fused::bwd_supported(g)) return 0;
  return e->hsave_bytes_per_sample * (size_t)B * g.N;
}

int32_t fused_backward(const FlowGeom& g, const float* params, int B, const float* saved,
                       const float* hsave, const float* g_phi, double g_logq,
                       const double* g_logq_vec, float* g_params, float* g_z, char* ws,
                       hipStream_t st) {
  if (fused::bwd_supported(g))
    return fused::bwd_run(g, params, B, saved, hsave, g_phi, g_logq, g_logq_vec, g_params, g_z, ws, st);
  return fused::ring_bwd_run(g, params, B, saved, reinterpret_cast<const unsigned char*>(hsave), g_phi,
                             g_logq, g_logq_vec, g_params, g_z, ws, st);
}

}  // namespace lfs

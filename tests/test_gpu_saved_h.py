"""The training pair that saves the second hidden activation (lfs_flow_forward_train,
lfs_flow_backward_saved) against the plain pair and the oracle.

The backward of a coupling layer needs h2 = LeakyReLU(W2 h1 + b2) at every site (paper
Sec. 1, the s/t networks of the coupling layers); the saved pair keeps it from the
forward instead of recomputing it.  Checked here, on 2D L = 32, hidden 16, plain FP32
(the shape the pair saves for), at batches that leave some workgroups two or three
samples:
  - the forward's outputs are bitwise those of lfs_flow_forward;
  - the saved h2 of every layer and sample equals the oracle's h2 of that layer's
    input field within 1e-5 (1 + |h2|) (FP32 sums of 9 and 144 terms);
  - the backward equals the recomputing backward within 1e-6 relative (measured:
    1e-7; the forward's conv1 runs on the vector ALUs and sums in another order than
    the recomputing backward's matrix-core conv1), and at a small batch the oracle
    within the FP32 bounds of the parity tests;
  - scalar and per-sample log q cotangents give the same bits;
  - on a shape without a saved layout the pair reports 0 bytes and falls back to
    the plain entry points' results.
"""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import flow as of
from paper_2208_08903_amd import lfs

from .gpu_util import DEV, dev, flow_buffers, host, rel_norm, run_backward, run_forward

pytestmark = pytest.mark.gpu


def _case(B, N=2, L=32, C=16, precision=lfs.LFS_PLAIN_FP32):
    desc = lfs.make_desc(2, L, N, C, precision=precision, algo=lfs.ALGO_FUSED)
    params = si.flow_params(2, N, C, seed=140 + L, w_std=0.1, b_std=0.05)
    z = si.normal_fields(240 + L, B, L * L)
    fs = of.FlowShape(2, L, N, C)
    return desc, params, z, fs


def _forward_train(desc, params_np, z_np):
    B = z_np.shape[0]
    b = flow_buffers(desc, B, True)
    hb = lfs.saved_h_bytes(desc, B)
    b["saved_h"] = torch.empty(max(hb, 1), device=DEV, dtype=torch.uint8) if hb else None
    b["params"], b["z"] = dev(params_np, torch.float32), dev(z_np, torch.float32)
    lfs.flow_forward_train(desc, b["params"], b["z"], b["phi"], b["logq"], b["saved"], b["saved_h"],
                           b["logdet"], b["ws"])
    torch.cuda.synchronize()
    return b


def _backward_saved(desc, fwd, g_phi_np, g_logq):
    B = g_phi_np.shape[0]
    ws = torch.empty(max(lfs.workspace_bytes(desc, B, True), 1), device=DEV, dtype=torch.uint8)
    gp = torch.empty_like(fwd["params"])
    gz = torch.empty(B, desc.L ** desc.dim, device=DEV, dtype=torch.float32)
    lfs.flow_backward_saved(desc, fwd["params"], fwd["saved"], fwd["saved_h"], dev(g_phi_np, torch.float32),
                            g_logq, gp, gz, ws)
    torch.cuda.synchronize()
    return host(gp), host(gz)


def test_saved_bytes():
    desc, *_ = _case(4, N=3)
    assert lfs.saved_h_bytes(desc, 5) == 3 * 5 * (16 * 1024 + 512) * 4
    assert lfs.saved_h_bytes(desc, 0) == 0
    for other in (lfs.make_desc(2, 8, 2, 16), lfs.make_desc(2, 32, 2, 8),
                  lfs.make_desc(2, 32, 2, 16, precision=lfs.LFS_BF16_CONV),
                  lfs.make_desc(3, 16, 2, 8, precision=lfs.LFS_BF16_CONV)):
        assert lfs.saved_h_bytes(other, 4) == 0


def test_forward_train_outputs_and_saved_h():
    """Outputs bitwise those of the plain forward; saved h2 = the oracle's h2 per layer."""
    B = 520
    print(f"forward_train 2D L=32 C=16 FP32 B={B}", flush=True)
    desc, params, z, fs = _case(B)
    a = run_forward(desc, params, z)
    t = _forward_train(desc, params, z)
    for k in ("phi", "logq", "logdet", "saved"):
        assert torch.equal(a[k], t[k]), k
    N, C, V = fs.n_layers, fs.hidden, 1024
    raw = host(t["saved_h"]).view(np.float32)
    # h2: [N][B][C/4][V][4] -> [N][B][C][V]; then s: [N][B][V/2] at the active sites
    hs = raw[:N * B * C * V].reshape(N, B, C // 4, V, 4).transpose(0, 1, 2, 4, 3)
    hs = hs.reshape(N, B, C, V).astype(np.float64)
    ss = raw[N * B * C * V:].reshape(N, B, V // 2).astype(np.float64)
    rows = [0, 1, 255, 256, 511, 519]
    saved = host(t["saved"]).reshape(N + 1, B, V).astype(np.float64)
    layers = of.unpack(params, fs)
    for l in range(N):
        # the oracle's network on the kernel's own layer input (FP32 values, exact in FP64)
        x = of.as_lattice(saved[l, rows], fs)
        mF = of.frozen_mask(fs, l)
        _, hl, _, s, _ = of.net(x, layers[l], mF, fs)
        h2 = hl[2].reshape(len(rows), C, V)
        got = hs[l, rows]
        # FP32 sums of 9 and 144 terms: well inside the forward's 1e-5 (1 + |phi|)
        err = np.max(np.abs(got - h2) / (1 + np.abs(h2)))
        # s at the active sites in half-site order (row-major among the active sites)
        s_act = s.reshape(len(rows), V)[:, mF.reshape(-1) == 0]
        err_s = np.max(np.abs(ss[l, rows] - s_act))
        print(f"  layer {l}: saved h2 vs oracle {err:.2e}, s {err_s:.2e}", flush=True)
        assert err <= 1e-5 and err_s <= 1e-5, (l, err, err_s)


@pytest.mark.parametrize("B", [520, 4])
def test_backward_saved_matches_recompute_and_oracle(B):
    """B = 520: the grid of 256 workgroups gives eight of them a third sample, whose
    saved h2 is copied in while the previous one's tail passes run."""
    print(f"backward_saved 2D L=32 C=16 FP32 B={B}", flush=True)
    desc, params, z, fs = _case(B)
    rng = np.random.default_rng(310)
    g_phi = rng.standard_normal(z.shape).astype(np.float32)
    t = _forward_train(desc, params, z)
    gs, gzs = _backward_saved(desc, t, g_phi, 0.37)
    gr, gzr = run_backward(desc, t, g_phi, 0.37)
    d = np.max(np.abs(gs - gr)) / np.max(np.abs(gr))
    dz = np.max(np.abs(gzs - gzr)) / np.max(np.abs(gzr))
    print(f"  saved vs recomputed: params {d:.2e}, g_z {dz:.2e}", flush=True)
    assert rel_norm(gs, gr) <= 1e-6 and d <= 1e-6
    assert rel_norm(gzs, gzr) <= 1e-6 and dz <= 1e-6
    if B <= 8:
        gpo, gzo = of.flow_vjp(params, z, fs, g_phi.astype(np.float64), 0.37)
        for lay_g, lay_o in zip(of.unpack(gs, fs), of.unpack(gpo, fs)):
            for a, b in zip(lay_g, lay_o):
                assert rel_norm(a, b) <= 1e-4, (rel_norm(a, b), a.shape)
                assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b)), a.shape
        assert rel_norm(gzs, gzo) <= 1e-4
        assert np.max(np.abs(gzs - gzo)) <= 1e-5 * np.max(np.abs(gzo))


def test_backward_saved_vector_cotangent_and_determinism():
    B = 600
    desc, params, z, fs = _case(B)
    g_phi = np.random.default_rng(311).standard_normal(z.shape).astype(np.float32)
    t = _forward_train(desc, params, z)
    g1, gz1 = _backward_saved(desc, t, g_phi, 0.25)
    g2, gz2 = _backward_saved(desc, t, g_phi, 0.25)
    np.testing.assert_array_equal(g1, g2)
    np.testing.assert_array_equal(gz1, gz2)
    ws = torch.empty(lfs.workspace_bytes(desc, B, True), device=DEV, dtype=torch.uint8)
    gp = torch.empty_like(t["params"])
    gz = torch.empty(B, 1024, device=DEV, dtype=torch.float32)
    vec = torch.full((B,), 0.25, device=DEV, dtype=torch.float64)
    lfs.flow_backward_saved(desc, t["params"], t["saved"], t["saved_h"], dev(g_phi, torch.float32), vec,
                            gp, gz, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(gp), g1)
    np.testing.assert_array_equal(host(gz), gz1)


def test_shapes_without_saved_layout_fall_back():
    """2D L = 8 (padded backward layout) and BF16: 0 saved bytes, the plain results."""
    for L, prec in ((8, lfs.LFS_PLAIN_FP32), (32, lfs.LFS_BF16_CONV)):
        desc, params, z, fs = _case(6, L=L, precision=prec)
        assert lfs.saved_h_bytes(desc, 6) == 0
        g_phi = np.random.default_rng(312).standard_normal(z.shape).astype(np.float32)
        a = run_forward(desc, params, z)
        t = _forward_train(desc, params, z)
        assert t["saved_h"] is None
        for k in ("phi", "logq", "saved"):
            assert torch.equal(a[k], t[k]), k
        gs, gzs = _backward_saved(desc, t, g_phi, 0.3)
        gr, gzr = run_backward(desc, a, g_phi, 0.3)
        np.testing.assert_array_equal(gs, gr)
        np.testing.assert_array_equal(gzs, gzr)


# ---- 3D L = 16 (BF16): the plane-streaming forward saves h1, h2, their sign words and s ----

def _bf16_round(a):
    """FP64 values rounded to BF16 (nearest even) through FP32, as the kernels store them."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ring_case(B, C, N=2):
    desc = lfs.make_desc(3, 16, N, C, precision=lfs.LFS_BF16_CONV, algo=lfs.ALGO_FUSED)
    params = si.flow_params(3, N, C, seed=160 + C, w_std=0.1, b_std=0.05)
    z = si.normal_fields(260 + C, B, 16 ** 3)
    fs = of.FlowShape(3, 16, N, C)
    return desc, params, z, fs


def _ring_blocks(raw, B, C, N, V=4096):
    """Split the saved bytes into per-layer (h1 [B][C][V], h2, m1 [B][V], m2, s [B][V])."""
    hb, wb = B * C * V * 2, B * V * 4
    lay = 2 * hb + 3 * wb
    assert raw.size == N * lay
    out = []
    for l in range(N):
        r = raw[l * lay:(l + 1) * lay]
        bf = lambda a: (a.view(np.uint16).astype(np.uint32) << 16).view(np.float32)
        out.append(dict(h1=bf(r[:hb]).reshape(B, C, V), h2=bf(r[hb:2 * hb]).reshape(B, C, V),
                        m1=r[2 * hb:2 * hb + wb].view(np.uint32).reshape(B, V),
                        m2=r[2 * hb + wb:2 * hb + 2 * wb].view(np.uint32).reshape(B, V),
                        s=r[2 * hb + 2 * wb:].view(np.float32).reshape(B, V)))
    return out


@pytest.mark.parametrize("C", [16, 32])
def test_ring_forward_train_saves(C):
    """Outputs bitwise those of the plain forward; the saved h1, h2 are the oracle's BF16
    emulation of them (within one BF16 ulp, rarely off), the sign words their signs, and
    s at the active sites the emulation's s."""
    B, N, V = 3, 2, 4096
    print(f"ring forward_train 3D L=16 C={C} B={B}", flush=True)
    desc, params, z, fs = _ring_case(B, C, N)
    assert lfs.saved_h_bytes(desc, B) == N * (2 * B * C * V * 2 + 3 * B * V * 4)
    a = run_forward(desc, params, z)
    t = _forward_train(desc, params, z)
    for k in ("phi", "logq", "logdet", "saved"):
        assert torch.equal(a[k], t[k]), k
    blocks = _ring_blocks(host(t["saved_h"]), B, C, N)
    saved = host(t["saved"]).reshape(N + 1, B, V).astype(np.float64)
    layers = of.unpack(params, fs)
    bits = np.arange(C, dtype=np.uint32)
    for l, blk in enumerate(blocks):
        mF = of.frozen_mask(fs, l)
        active = (mF.reshape(-1) == 0)
        _, hl, o, s, _ = of.net(of.as_lattice(saved[l], fs), layers[l], mF, fs, emulate="bf16")
        for name, ref in (("h1", hl[1]), ("h2", hl[2])):
            ref = _bf16_round(ref.reshape(B, C, V))
            got = blk[name].astype(np.float64)
            err = np.max(np.abs(got - ref) / (np.abs(ref) * 2.0 ** -7 + 1e-5))
            frac = np.mean(got != ref)
            print(f"  layer {l} {name}: worst {err:.2f} of one BF16 ulp, {frac:.1e} of entries differ", flush=True)
            assert err <= 1.0 and frac <= 1e-2, (l, name, err, frac)
            # sign words: bit c iff channel c >= 0 (upper bits zero below 32 channels)
            mk = blk["m1" if name == "h1" else "m2"]
            want = ((got >= 0).astype(np.uint32) << bits[None, :, None]).sum(axis=1).astype(np.uint32)
            np.testing.assert_array_equal(mk, want)
        # s: the oracle's conv3 (FP64 sums, BF16-rounded weights) of the kernel's own saved
        # h2, so that only the kernel's FP32 sums of 27 C terms and its tanh differ; against
        # the emulation itself one flipped h2 entry moves s by up to ~1e-3
        W3, b3 = of.split_convs(layers[l], fs)[-1][:2]
        o_k = of.conv(blk["h2"].astype(np.float64).reshape(B, C, 16, 16, 16), _bf16_round(W3), b3, 3)
        s_k = np.tanh(o_k[:, 0]).reshape(B, V)
        err_k = np.max(np.abs(blk["s"][:, active] - s_k[:, active]))
        err_e = np.max(np.abs(blk["s"][:, active] - s.reshape(B, V)[:, active]))
        print(f"  layer {l} s: vs the saved h2's conv3 {err_k:.2e}, vs the emulation {err_e:.2e}", flush=True)
        assert err_k <= 2e-5 and err_e <= 1e-2, (l, err_k, err_e)


@pytest.mark.parametrize("C", [16, 32])
def test_ring_backward_saved(C):
    """The plane-streaming backward from the saved activations against the oracle's BF16
    emulation with the bounds of the parity tests, bitwise reproducible, and close to the
    recomputing backward: the two sum h1 and h2 in different orders before rounding them to
    BF16, so a few stored entries differ by one BF16 ulp (measured: relative 2-norm 1e-3 of
    the parameter gradient, 2.6e-3 of g_z at C = 32), within the BF16 error itself."""
    from .test_gpu_parity import _check_backward_bf16
    B = 3
    print(f"ring backward_saved 3D L=16 C={C} B={B}", flush=True)
    desc, params, z, fs = _ring_case(B, C)
    g_phi = np.random.default_rng(320 + C).standard_normal(z.shape).astype(np.float32)
    t = _forward_train(desc, params, z)
    gs, gzs = _backward_saved(desc, t, g_phi, 0.3)
    gs2, gzs2 = _backward_saved(desc, t, g_phi, 0.3)
    np.testing.assert_array_equal(gs, gs2)
    np.testing.assert_array_equal(gzs, gzs2)
    gr, gzr = run_backward(desc, t, g_phi, 0.3)
    print(f"  saved vs recomputed: params {rel_norm(gs, gr):.2e}, g_z {rel_norm(gzs, gzr):.2e}", flush=True)
    gpo, gzo = of.flow_vjp(params, z, fs, g_phi.astype(np.float64), 0.3)
    _check_backward_bf16(params, z, fs, g_phi, 0.3, gs, gzs, gpo, gzo)
    assert rel_norm(gs, gr) <= 1e-2 and rel_norm(gzs, gzr) <= 1e-2

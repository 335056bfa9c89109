"""The HIP path at the workloads' full sizes, in the launch configuration the
benchmark times, against the FP64 oracle.

Training steps (2D L=32 C=16 at batch 1024, 3D L=8 C=16 at batch 512 with
N(0, 0.1^2) and with N(0, 0.05^2) weights, 3D L=16 C=32 at batch 256 with
N(0, 0.05^2) weights, BF16 only): one
trainer step's loss and gradient (the trainer's own prior draw, forward and
backward, i.e. the same kernels, grids and workspace as the timed step) against
the oracle's gradient of the same step, stored by tests/golden/make_full_size.py
as a stratified sample of entries, every parameter block's norm and 32 seeded
random projections R g.  For an error vector d, R d has N(0, |d|^2) entries, so
the projections bound the whole-vector error; block norms bound each block's.

Sampling (2D L=8 C=8 chain of 2000, 2D L=32 at batch 1024, 3D L=16 C=32 at
batch 4096): the flow outputs of sampled samples (all of them for the 2000-
proposal chain) against the oracle's forward of the same prior draw; a
sample's outputs depend only on its own input, so the oracle computes them one
sample at a time.

Tolerances are those of the small-size parity tests:
  FP32 gradient: per block and whole vector 1e-4 relative, or 12 times the
  error the oracle itself shows when it stores the conv operands and the field
  in FP32 and accumulates the weight gradients in FP32 (stored with the
  gradient), whichever is larger.  The 3D random-init flow amplifies rounding,
  and its first layers' bias gradients are sums of 262144 site terms of both
  signs; numpy's float32 sums are pairwise (about 18 additions deep), the
  kernels' chains (per-lane sums over a workgroup's tiles, lane and wave trees,
  the partials reduction) about 56, hence 3x, times a margin of 4.
  BF16 gradient: against the oracle's emulate="bf16" gradient of the same step
  (stored beside the FP64 one), per block 1e-2 relative (norms and sampled
  entries) and whole vector 5e-3 (for the 3D L=8 flow at N(0, 0.1^2) weights,
  whose loss is ~1e10: 2 % per block or the emulation's own relative distance
  from FP64 where that is larger, half of it whole; the same step at N(0, 0.05^2)
  has the tight bounds); against FP64, each block's norm within
  3 times the emulation's own relative distance.  Flow outputs: FP32 |dphi| <= 1e-5
  (T/9)(1+|phi|), |dlogq| <= 1e-4 V; BF16 as the small-size tests, against the
  emulation of the same samples.  Loss (a batch mean of log q + S): FP32 the
  log q bound plus the field bound propagated to S to first order, i.e. the phi
  tolerance times the oracle's batch mean of sum_n |dS/dphi_n| (1 + |phi_n|);
  BF16 against the emulation's loss: the element-wise field bound 1e-2 (T/9)
  (1+|phi|) propagated the same way, plus the emulation's own distance from FP64.
"""
import os

import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import flow as of
from oracle import prior as op
from paper_2208_08903_amd import flow as fl
from paper_2208_08903_amd import lfs

from .gpu_util import host
from .test_gpu_parity import _check_forward_bf16

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PRECISIONS = [lfs.LFS_BF16_CONV, lfs.LFS_PLAIN_FP32]


def _tol(T, V):
    """FP32 bounds (BF16 results are held to the emulation instead)."""
    return dict(phi=1e-5 * T / 9, logq=1e-4 * V, g_block=1e-4, g_whole=1e-4)


def _blocks(dim, N, C):
    out, off = [], 0
    for _ in range(N):
        for _, sz in si.layer_block_sizes(dim, C):
            out.append(slice(off, off + sz))
            off += sz
    return out


@pytest.mark.parametrize("name,precision", [
    ("2d_L32_C16_B1024", lfs.LFS_BF16_CONV), ("2d_L32_C16_B1024", lfs.LFS_PLAIN_FP32),
    ("3d_L8_C16_B512", lfs.LFS_BF16_CONV), ("3d_L8_C16_B512", lfs.LFS_PLAIN_FP32),
    ("3d_L8_C16_B512_w05", lfs.LFS_BF16_CONV), ("3d_L8_C16_B512_w05", lfs.LFS_PLAIN_FP32),
    ("3d_L16_C32_B256", lfs.LFS_BF16_CONV)])
def test_full_size_training_gradient(name, precision):
    g = np.load(os.path.join(GOLDEN, f"full_size_grad_{name}.npz"), allow_pickle=False)
    dim, L, N, C, B = (int(v) for v in g["config"])
    m2, lam = (float(v) for v in g["couplings"])
    key, c0, wseed, pseed = (int(v) for v in g["seeds"])
    assert c0 == 0  # the trainer's first step draws counters 0 .. B-1
    print(f"full-size training step {name} precision={precision}", flush=True)
    w_std = float(g["w_std"][0])
    f = fl.Flow(dim, L, N, C, precision, params=si.flow_params(dim, N, C, seed=wseed, w_std=w_std))
    tr = fl.Trainer(f, B, m2, lam, key=key)
    tr.draw()
    tr.forward()
    tr.backward()
    torch.cuda.synchronize()
    grad = host(tr.gparams).astype(np.float64)
    loss = float(tr.loss.item())
    if precision == lfs.LFS_BF16_CONV:
        _check_bf16_gradient(g, grad, loss, dim, N, C, ill_conditioned=w_std >= 0.1 and dim == 3)
        return
    tol = _tol(3 ** dim, L ** dim)
    blk_tol = np.full(len(g["block_norms"]), tol["g_block"])
    whole_tol = tol["g_whole"]
    # 12x the oracle's own error under FP32 storage and accumulation (see the header)
    blk_tol = np.maximum(blk_tol, 12 * g["fp32_block_err"])
    whole_tol = max(whole_tol, 12 * float(g["fp32_whole_err"][0]))

    # log q's bound plus S's first-order response to the field bound
    assert abs(loss - float(g["loss"][0])) <= tol["logq"] + tol["phi"] * float(g["loss_sensitivity"][0])
    _check_stored_gradient(grad, dim, N, C, g["idx"], g["vals"], g["block_norms"], blk_tol, g["proj"],
                           int(g["seeds"][3]), whole_tol, float(g["grad_norm"][0]))


def _check_stored_gradient(grad, dim, N, C, idx, vals, norms, blk_tol, proj, pseed, whole_tol, gnorm):
    """Every block's norm and its sampled entries against the stored ones, and the whole
    vector through the stored seeded projections."""
    for k, sl in enumerate(_blocks(dim, N, C)):
        ref = float(norms[k])
        got = np.linalg.norm(grad[sl])
        assert abs(got - ref) <= blk_tol[k] * ref + 1e-30, (k, got, ref)
        sel = (idx >= sl.start) & (idx < sl.stop)
        d = np.linalg.norm(grad[idx[sel]] - vals[sel])
        assert d <= blk_tol[k] * ref + 1e-30, (k, d, ref)
    # whole vector: R (grad - g_ref) = R grad - stored projections
    R = np.random.default_rng(pseed).standard_normal((proj.size, grad.size))
    dproj = R @ grad - proj
    assert np.max(np.abs(dproj)) <= 5 * whole_tol * gnorm


def _check_bf16_gradient(g, grad, loss, dim, N, C, ill_conditioned=False):
    """A BF16 step against the stored emulate="bf16" gradient and loss, and its block norms
    against FP64 within 3 times the emulation's own distance."""
    loss16, loss64 = float(g["bf16_loss"][0]), float(g["loss"][0])
    norms16 = g["bf16_block_norms"]
    print(f"  bf16 full-size step: loss {loss:.6f}, emulation {loss16:.6f}, FP64 {loss64:.6f}; "
          f"largest block error of the emulation vs FP64 {float(np.max(g['bf16_block_err'])):.3e}", flush=True)
    # the element-wise field bound against the emulation propagated to S to first order,
    # plus the log q bound (the emulation's own distance from FP64)
    T, V = 3 ** dim, g["config"][1] ** dim
    bound = 1e-2 * T / 9 * float(g["loss_sensitivity"][0]) + abs(loss16 - loss64) + 1e-6 * V * N
    assert abs(loss - loss16) <= bound, (loss, loss16, loss64, bound)
    # 1e-2 per block and 5e-3 whole.  The 3D L=8 flow at the workload's N(0, 0.1^2) weights
    # (loss ~1e10) amplifies rounding so much that the emulation itself is 1-25 % from FP64
    # per block and the BF16 roundings that FP32-versus-FP64 sums flip move the kernel by
    # 1-4 %: there a block must be within 2 % of the emulation or no further from it than
    # the emulation is from FP64, the whole vector within half the emulation's distance;
    # the same step at N(0, 0.05^2) weights is held to the tight bounds
    if ill_conditioned:
        blk = np.maximum(2e-2, g["bf16_block_err"])
        whole = max(5e-3, 0.5 * float(g["bf16_whole_err"][0]))
    else:
        blk, whole = np.full(len(norms16), 1e-2), 5e-3
    _check_stored_gradient(grad, dim, N, C, g["idx"], g["bf16_vals"], norms16, blk,
                           g["bf16_proj"], int(g["seeds"][3]), whole, float(g["bf16_grad_norm"][0]))
    for k, sl in enumerate(_blocks(dim, N, C)):
        ref = float(g["block_norms"][k])
        got = np.linalg.norm(grad[sl])
        assert abs(got - ref) <= (3 * float(g["bf16_block_err"][k]) + 1e-6) * ref, (k, got, ref)


def _sampled_forward_check(f, params, z_host_key, c0, phi, logq, samples, precision, rho=None):
    dim, L, N, C = f.dim, f.L, f.n_layers, f.hidden
    fs = of.FlowShape(dim, L, N, C)
    p = params.astype(np.float64)
    samples = list(samples)
    z = np.concatenate([op.prior_normal(z_host_key, c0 + int(b), 1, fs.V) for b in samples])
    if precision == lfs.LFS_BF16_CONV:
        ref = of.flow_forward(p, z, fs)
        _check_forward_bf16(p, z, fs, phi[samples].astype(np.float64), logq[samples], None, ref,
                            **({} if rho is None else {"rho": rho}))
        return
    tol = _tol(3 ** dim, fs.V)
    for k, b in enumerate(samples):
        o = of.flow_forward(p, z[k:k + 1], fs)
        po = o["phi"].reshape(-1)
        pg = phi[b].astype(np.float64)
        assert np.all(np.abs(pg - po) <= tol["phi"] * (1 + np.abs(po))), b
        assert abs(logq[b] - o["logq"][0]) <= tol["logq"], b


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_size_2d_L32_forward_sampled(precision):
    """The training step's forward at batch 1024: samples in the first, a middle and the
    last workgroup round."""
    print(f"full-size 2D L=32 forward precision={precision}", flush=True)
    params = si.flow_params(2, 16, 16)
    f = fl.Flow(2, 32, 16, 16, precision, params=params)
    tr = fl.Trainer(f, 1024, -4.0, 8.0, key=12345)
    tr.draw()
    tr.forward()
    torch.cuda.synchronize()
    _sampled_forward_check(f, params, 12345, 0, host(tr.phi), host(tr.logq), [0, 1, 255, 256, 511, 777, 1023],
                           precision)


def test_full_size_3d_L16_C32_sampling_sampled():
    """Sampling at batch 4096 with the 3D L=16 C=32 flow (BF16, the plane-streaming forward).

    With the workload's N(0, 0.1^2) weights this 16-layer map amplifies any rounding
    beyond use (the oracle's own FP32-operand emulation moves phi by up to 84% of
    1 + |phi|), so the comparison with the oracle uses N(0, 0.05^2) weights, under which
    the oracle's BF16 emulation stays within 1.3e-2 (1 + |phi|) of FP64 while the map
    still scales the field several-fold; same shapes, batch and launch."""
    print("full-size 3D L=16 C=32 sampling forward, batch 4096", flush=True)
    params = si.flow_params(3, 16, 32, w_std=0.05)
    f = fl.Flow(3, 16, 16, 32, lfs.LFS_BF16_CONV, params=params)
    B = 4096
    smp = fl.Sampler(f, B, -4.0, 5.0, key=4242)
    lu = torch.as_tensor(si.log_uniforms(5, (1, B)), device="cuda")
    smp.step(lu)
    torch.cuda.synchronize()
    # 16 layers of fan-in 864 spread the few BF16 roundings the FP32 sums flip over whole
    # samples: the share of the distance from FP64 not explained by the emulation is up to
    # ~0.8 here (the rounding points themselves are pinned exactly by the exact-operand tests)
    _sampled_forward_check(f, params, 4242, 0, host(smp.phi), host(smp.logq), [0, 2049, 4095],
                           lfs.LFS_BF16_CONV, rho=1.0)


def test_full_size_3d_L16_C32_batch_position_independent():
    """At the workload's own weights: a sample's outputs in the batch of 4096 are bitwise
    those of the same draw run alone (outputs depend only on the sample's input)."""
    print("full-size 3D L=16 C=32 batch-position independence, batch 4096", flush=True)
    f = fl.Flow(3, 16, 16, 32, lfs.LFS_BF16_CONV, params=si.flow_params(3, 16, 32))
    V = 16 ** 3
    z = torch.empty(4096, V, device="cuda", dtype=torch.float32)
    lfs.prior_normal(4242, 0, z)
    phi = torch.empty_like(z)
    logq = torch.empty(4096, device="cuda", dtype=torch.float64)
    lfs.flow_forward(f.desc, f.params, z, phi, logq, None, None, f.workspace(4096, False))
    for b in (0, 2049, 4095):
        z1 = torch.empty(1, V, device="cuda", dtype=torch.float32)
        lfs.prior_normal(4242, b, z1)
        p1 = torch.empty_like(z1)
        q1 = torch.empty(1, device="cuda", dtype=torch.float64)
        lfs.flow_forward(f.desc, f.params, z1, p1, q1, None, None, f.workspace(1, False))
        torch.cuda.synchronize()
        assert torch.equal(z1[0], z[b])
        assert torch.equal(p1[0], phi[b]) and torch.equal(q1[0], logq[b]), b


@pytest.mark.parametrize("precision", PRECISIONS)
def test_full_size_2d_L8_chain_batch(precision):
    """The 2D L=8 C=8 example shape: a batch of 2000 proposals, every sample checked."""
    print(f"full-size 2D L=8 chain batch 2000 precision={precision}", flush=True)
    params = si.flow_params(2, 16, 8)
    f = fl.Flow(2, 8, 16, 8, precision, params=params)
    B = 2000
    smp = fl.Sampler(f, B, -4.0, 8.0, key=12)
    lu = torch.as_tensor(si.log_uniforms(7, (1, B)), device="cuda")
    smp.step(lu)
    torch.cuda.synchronize()
    fs = of.FlowShape(2, 8, 16, 8)
    tol = _tol(9, 64)
    z = op.prior_normal(12, 0, B, fs.V)
    o = of.flow_forward(params.astype(np.float64), z, fs)
    pg = host(smp.phi).astype(np.float64)
    if precision == lfs.LFS_BF16_CONV:
        _check_forward_bf16(params.astype(np.float64), z, fs, pg, host(smp.logq), None, o)
        return
    po = o["phi"].reshape(B, -1)
    assert np.all(np.abs(pg - po) <= tol["phi"] * (1 + np.abs(po)))
    assert np.all(np.abs(host(smp.logq) - o["logq"]) <= tol["logq"])

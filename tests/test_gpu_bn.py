"""Batch-norm flows (lfs_flow_forward_bn / lfs_flow_backward_bn) on the GPU against
the FP64 oracle, under batch and running statistics.

Tolerances follow the general-network tests: FP32 forward |dphi| <= 1e-5 (T/9)
(1 + |phi|), log q within 1e-4 V, gradient blocks 1e-4 relative; BF16 against the
oracle's BF16-operand emulation (same rounded convolution operands, FP64 sums):
forward 1e-3 relative in norm (a field value on the other side of a BF16
rounding boundary than its emulated twin moves a few sites much more than the
rest), gradient blocks 5e-2, whole vectors 2e-2; and against plain FP64 with the
default BF16 bounds (forward 0.02 (T/9) (1 + |phi|) per site) or 3 times the
emulation's own deviation from FP64, whichever is larger: the normalisation
lifts the hidden activations to unit scale, so BF16 operand rounding moves s
and t more than in the default network (0.06 at some sites of the 2D L = 16
case).  Running statistics after the
update: 1e-5 (FP32) or 2e-3 (BF16, against the emulation) times (1 + |r|).  Under
batch statistics the hidden convolutions' bias gradients are zero in exact
arithmetic (the mean removes the bias); they are checked against 1e-4 (FP32) or
1e-2 (BF16) of the layer's largest gradient entry instead of relatively."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import flow as of

from paper_2208_08903_amd import lfs
from paper_2208_08903_amd.flow import Flow, Sampler, Trainer

from .gpu_util import dev, flow_buffers, host, rel_norm

pytestmark = pytest.mark.gpu

CASES = [
    # dim, L, N, kernel, hidden_sizes, B
    (2, 8, 2, 3, (4, 6), 5),
    (3, 4, 2, 3, (3,), 3),
    (2, 6, 3, 5, (3, 2, 4), 4),
    (2, 8, 2, 1, (5,), 2),
    (2, 16, 2, 3, (8, 8), 20),     # B V = 5120: two reduction chunks, the second ragged
]


def _case(dim, L, N, K, hs, B, precision, tanh=True):
    desc = lfs.make_desc(dim, L, N, 0, final_tanh=tanh, precision=precision, kernel=K, hidden_sizes=hs,
                         batch_norm=True)
    params = si.flow_params(dim, N, 0, seed=600 + L + K, w_std=0.2, b_std=0.1, kernel=K, hidden_sizes=hs,
                            batch_norm=True, gamma_std=0.2)
    z = si.normal_fields(700 + L, B, L ** dim)
    stats = si.bn_stats(800 + L, N, hs)
    fs = of.FlowShape(dim, L, N, 0, final_tanh=tanh, kernel=K, hidden_sizes=hs, batch_norm=True)
    return desc, params, z, stats, fs


def _forward(desc, params, z, mode, stats, momentum=0.1):
    b = flow_buffers(desc, z.shape[0])
    p, zt = dev(params, torch.float32), dev(z, torch.float32)
    st = dev(stats, torch.float32) if stats is not None else None
    lfs.flow_forward_bn(desc, p, zt, b["phi"], b["logq"], mode, st, momentum, b["logdet"], b["saved"], b["ws"])
    torch.cuda.synchronize()
    b.update(params=p, z=zt, stats=st)
    return b


def _backward(desc, fwd, g_phi, g_logq, mode):
    B, V = g_phi.shape
    ws = torch.empty(lfs.workspace_bytes(desc, B, True), device="cuda", dtype=torch.uint8)
    gp = torch.empty_like(fwd["params"])
    gz = torch.empty(B, V, device="cuda", dtype=torch.float32)
    lfs.flow_backward_bn(desc, fwd["params"], fwd["saved"], dev(g_phi, torch.float32), g_logq, gp, mode,
                         fwd["stats"], gz, ws)
    torch.cuda.synchronize()
    return host(gp), host(gz)


def _oracle_stats(stats, fs):
    return of.unpack_bn_stats(stats.astype(np.float64), fs)


def _check_forward(out, params, z, fs, precision, ref_stats):
    B, V = z.shape
    p64 = params.astype(np.float64)
    ref = of.flow_forward(p64, z, fs, bn_stats=ref_stats)
    phi, logq = host(out["phi"]).astype(np.float64), host(out["logq"])
    tf = fs.T / 9
    if precision == lfs.LFS_PLAIN_FP32:
        assert np.all(np.abs(phi - ref["phi"].reshape(B, V)) <= 1e-5 * tf * (1 + np.abs(ref["phi"].reshape(B, V))))
        assert np.all(np.abs(logq - ref["logq"]) <= 1e-4 * V)
        return ref
    emu = of.flow_forward(p64, z, fs, emulate="bf16", bn_stats=ref_stats)
    pe = emu["phi"].reshape(B, V)
    worst = np.max(np.abs(phi - pe) / (tf * (1 + np.abs(pe))))
    print(f"largest deviation from the BF16 emulation: {worst:.3g} (T/9)(1 + |phi|)", flush=True)
    assert rel_norm(phi, pe) <= 1e-3, rel_norm(phi, pe)
    # against FP64: the default BF16 bound, or 3 times the emulation's own deviation
    p64r = ref["phi"].reshape(B, V)
    bound = np.maximum(0.02 * tf * (1 + np.abs(p64r)), 3 * np.abs(pe - p64r))
    assert np.all(np.abs(phi - p64r) <= bound), np.max(np.abs(phi - p64r))
    lbound = np.maximum(0.05 * np.sqrt(V * fs.n_layers) + 1e-4 * V, 3 * np.abs(emu["logq"] - ref["logq"]))
    assert np.all(np.abs(logq - ref["logq"]) <= lbound)
    return emu


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", [lfs.LFS_PLAIN_FP32, lfs.LFS_BF16_CONV])
def test_bn_forward_batch_statistics(case, precision):
    print(f"batch norm forward, batch statistics {case} precision={precision}", flush=True)
    desc, params, z, stats, fs = _case(*case, precision)
    out = _forward(desc, params, z, lfs.BN_BATCH, stats)
    ref = _check_forward(out, params, z, fs, precision, None)
    # the running statistics moved towards this batch's (momentum 0.1, unbiased variance)
    want = of.pack_bn_stats(of.bn_running_update(_oracle_stats(stats, fs), ref["bn_used"], z.size))
    got = host(out["stats"]).astype(np.float64)
    tol = 1e-5 if precision == lfs.LFS_PLAIN_FP32 else 2e-3
    assert np.all(np.abs(got - want) <= tol * (1 + np.abs(want))), np.max(np.abs(got - want))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", [lfs.LFS_PLAIN_FP32, lfs.LFS_BF16_CONV])
def test_bn_forward_running_statistics(case, precision):
    print(f"batch norm forward, running statistics {case} precision={precision}", flush=True)
    desc, params, z, stats, fs = _case(*case, precision)
    out = _forward(desc, params, z, lfs.BN_RUNNING, stats)
    _check_forward(out, params, z, fs, precision, _oracle_stats(stats, fs))
    np.testing.assert_array_equal(host(out["stats"]), stats)       # read only


def _bn_bias_blocks(fs):
    """Indices, within a layer's block list, of the biases of normalised convolutions."""
    idx, k = [], 0
    for i in range(len(fs.conv_shapes)):
        if i < len(fs.conv_shapes) - 1:
            idx.append(k + 1)
            k += 4
        else:
            k += 2
    return idx


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", [lfs.LFS_PLAIN_FP32, lfs.LFS_BF16_CONV])
@pytest.mark.parametrize("mode", [lfs.BN_BATCH, lfs.BN_RUNNING])
def test_bn_backward(case, precision, mode):
    print(f"batch norm backward {case} precision={precision} mode={mode}", flush=True)
    desc, params, z, stats, fs = _case(*case, precision)
    out = _forward(desc, params, z, mode, stats, momentum=0.0)
    g_phi = np.random.default_rng(301).standard_normal(z.shape).astype(np.float32)
    gp, gz = _backward(desc, out, g_phi, 0.37, mode)
    ref_stats = None if mode == lfs.BN_BATCH else _oracle_stats(stats, fs)
    p64 = params.astype(np.float64)
    g64, z64 = of.flow_vjp(p64, z, fs, g_phi.astype(np.float64), 0.37, bn_stats=ref_stats)
    fp32 = precision == lfs.LFS_PLAIN_FP32
    if fp32:
        ge, ze = g64, z64
    else:
        ge, ze = of.flow_vjp(p64, z, fs, g_phi.astype(np.float64), 0.37, emulate="bf16", bn_stats=ref_stats)
    zero_bias = _bn_bias_blocks(fs) if mode == lfs.BN_BATCH else []
    for lay_g, lay_e, lay_64 in zip(of.unpack(gp, fs), of.unpack(ge, fs), of.unpack(g64, fs)):
        top = max(np.max(np.abs(a)) for a in lay_e)
        for k, (a, e, r) in enumerate(zip(lay_g, lay_e, lay_64)):
            if k in zero_bias:
                assert np.max(np.abs(a)) <= (1e-4 if fp32 else 1e-2) * top, (k, np.max(np.abs(a)), top)
                continue
            if fp32:
                assert rel_norm(a, e) <= 1e-4, (k, rel_norm(a, e), a.shape)
            else:
                assert rel_norm(a, e) <= 5e-2, (k, rel_norm(a, e), a.shape)
                assert rel_norm(a, r) <= max(0.4, 3 * rel_norm(e, r)), (k, rel_norm(a, r), a.shape)
    assert rel_norm(gz, ze) <= (1e-4 if fp32 else 2e-2)
    assert rel_norm(gp, ge) <= (1e-4 if fp32 else 2e-2)


def test_bn_momentum_and_statistics_buffer():
    """momentum 0 leaves the running statistics; momentum 1 replaces them by the batch's
    mean and unbiased variance; no buffer at all in batch mode gives the same outputs."""
    desc, params, z, stats, fs = _case(2, 8, 2, 3, (4, 6), 5, lfs.LFS_PLAIN_FP32)
    a = _forward(desc, params, z, lfs.BN_BATCH, stats, momentum=0.0)
    np.testing.assert_array_equal(host(a["stats"]), stats)
    b = _forward(desc, params, z, lfs.BN_BATCH, stats, momentum=1.0)
    c = _forward(desc, params, z, lfs.BN_BATCH, None)
    for k in ("phi", "logq"):
        assert torch.equal(a[k], b[k]) and torch.equal(a[k], c[k])
    ref = of.flow_forward(params.astype(np.float64), z, fs)
    n = z.size
    want = of.pack_bn_stats([[(m, v * n / (n - 1)) for m, v in lay] for lay in ref["bn_used"]])
    got = host(b["stats"]).astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-5 * (1 + np.abs(want)))


def test_bn_sample_coupling_and_independence():
    """Running statistics: a sample's outputs do not depend on its batch.  Batch
    statistics: they do (the batch is normalised together)."""
    desc, params, z, stats, fs = _case(2, 8, 2, 3, (4, 6), 6, lfs.LFS_BF16_CONV)
    full = _forward(desc, params, z, lfs.BN_RUNNING, stats)
    part = _forward(desc, params, z[2:4], lfs.BN_RUNNING, stats)
    np.testing.assert_array_equal(host(full["phi"])[2:4], host(part["phi"]))
    np.testing.assert_array_equal(host(full["logq"])[2:4], host(part["logq"]))
    fb = _forward(desc, params, z, lfs.BN_BATCH, stats)
    pb = _forward(desc, params, z[2:4], lfs.BN_BATCH, stats)
    assert np.max(np.abs(host(fb["phi"])[2:4] - host(pb["phi"]))) > 1e-4


def test_bn_deterministic():
    desc, params, z, stats, fs = _case(2, 16, 2, 3, (8, 8), 20, lfs.LFS_BF16_CONV)
    a = _forward(desc, params, z, lfs.BN_BATCH, stats)
    b = _forward(desc, params, z, lfs.BN_BATCH, stats)
    for k in ("phi", "logq", "stats"):
        assert torch.equal(a[k], b[k]), k
    g = np.random.default_rng(5).standard_normal(z.shape).astype(np.float32)
    ga, za = _backward(desc, a, g, 0.2, lfs.BN_BATCH)
    gb, zb = _backward(desc, b, g, 0.2, lfs.BN_BATCH)
    np.testing.assert_array_equal(ga, gb)
    np.testing.assert_array_equal(za, zb)


def test_bn_entry_points_without_batch_norm_match_plain():
    desc = lfs.make_desc(2, 8, 2, 0, precision=lfs.LFS_BF16_CONV, kernel=3, hidden_sizes=(4, 6))
    params = si.flow_params(2, 2, 0, seed=3, w_std=0.2, b_std=0.1, kernel=3, hidden_sizes=(4, 6))
    z = si.normal_fields(4, 3, 64)
    a = _forward(desc, params, z, lfs.BN_RUNNING, None)
    b = flow_buffers(desc, 3)
    lfs.flow_forward(desc, a["params"], a["z"], b["phi"], b["logq"], b["logdet"], b["saved"], b["ws"])
    torch.cuda.synchronize()
    assert torch.equal(a["phi"], b["phi"]) and torch.equal(a["logq"], b["logq"])


def test_bn_trainer_and_sampler():
    """A few training steps with batch statistics move the running statistics and
    lower nothing to NaN; sampling then uses the running statistics."""
    hs = (8, 8)
    params = si.flow_params(2, 4, 0, seed=9, w_std=0.1, kernel=3, hidden_sizes=hs, batch_norm=True)
    flow = Flow(2, 8, 4, 0, params=params, hidden_sizes=hs, kernel=3, batch_norm=True)
    s0 = flow.bn_stats.clone()
    tr = Trainer(flow, 32, -4.0, 8.0)
    for _ in range(5):
        tr.step()
    torch.cuda.synchronize()
    assert np.isfinite(tr.loss.item())
    assert not torch.equal(flow.bn_stats, s0) and torch.isfinite(flow.bn_stats).all()
    smp = Sampler(flow, 64, -4.0, 8.0)
    lu = torch.as_tensor(si.log_uniforms(3, (1, 64)), device="cuda")
    s1 = flow.bn_stats.clone()
    smp.step(lu)
    torch.cuda.synchronize()
    assert torch.equal(flow.bn_stats, s1)
    assert torch.isfinite(smp.logw).all()

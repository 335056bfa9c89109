"""General s/t networks (hidden_sizes, odd kernel size) on the GPU against the
FP64 oracle: forward outputs, log q, and the backward's parameter and z
gradients, with the tolerances of the default network's generic-path tests
(the field bound scales with the taps per convolution, T / 9).

BF16 forward: against the oracle's BF16 emulation as for the default network,
except the share of the distance from FP64 that the emulation must explain
(2-norms of phi and log q over the batch): 0.6 instead of 0.2.  A wide
kernel on a small lattice (5 x 5 taps on 8 x 8 sites) spreads one activation
whose BF16 rounding the FP32-versus-FP64 sums flip over the whole sample, and
such flips are the only difference left: on operands that make every sum exact
the general-network kernels match the emulation to FP32 rounding
(tests/test_gpu_rounding.py), so they round at the same points.

BF16 gradients: small networks with wide kernels (125 taps of 3 channels in
3D) amplify the BF16 rounding of the operands well past the default network's
0.4 per-block bound (one 3D case moves a bias block by 0.8 relative).  There the
kernels are checked against the oracle's own BF16-operand emulation (same
rounded operands, sums in FP64): 5e-2 per block, 2e-2 whole; and against FP64
with the default bounds or 3 times the emulation's own deviation, whichever is
larger."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import flow as of
from paper_2208_08903_amd import lfs

from .gpu_util import host, rel_norm, run_backward, run_forward
from .test_gpu_parity import _check_backward, _check_forward

pytestmark = pytest.mark.gpu

NET_CASES = [
    # dim, L, N, kernel, hidden_sizes, B
    (2, 8, 3, 5, (8, 8), 4),
    (2, 6, 2, 3, (3, 5, 4), 3),        # unequal widths, L not a power of two
    (3, 4, 2, 3, (4,), 2),             # one hidden convolution
    (2, 8, 2, 1, (6, 6), 3),           # pointwise network
    (2, 4, 2, 7, (2, 3), 2),           # kernel wider than the lattice: taps wrap
    (2, 8, 2, 3, (8, 8, 8, 8), 2),     # four hidden convolutions
    (3, 4, 2, 5, (3, 3), 2),
]


def _net_case(dim, L, N, K, hs, B, precision, tanh=True):
    desc = lfs.make_desc(dim, L, N, 0, final_tanh=tanh, precision=precision, kernel=K, hidden_sizes=hs)
    params = si.flow_params(dim, N, 0, seed=400 + L + K, w_std=0.1, b_std=0.05, kernel=K, hidden_sizes=hs)
    z = si.normal_fields(500 + L, B, L ** dim)
    fs = of.FlowShape(dim, L, N, 0, final_tanh=tanh, kernel=K, hidden_sizes=hs)
    return desc, params, z, fs


@pytest.mark.parametrize("case", NET_CASES)
@pytest.mark.parametrize("precision", [lfs.LFS_PLAIN_FP32, lfs.LFS_BF16_CONV])
def test_net_forward_backward(case, precision):
    print(f"general network {case} precision={precision}", flush=True)
    desc, params, z, fs = _net_case(*case, precision)
    out, _ = _check_forward(desc, params, z, fs, precision, rho=0.6)
    if precision == lfs.LFS_PLAIN_FP32:
        _check_backward(desc, params, z, fs, out, precision)
    else:
        _check_backward_bf16(params, z, fs, desc, out)


def _check_backward_bf16(params, z, fs, desc, out):
    B, V = z.shape
    g_phi = np.random.default_rng(300).standard_normal((B, V)).astype(np.float32)
    gp, gz = run_backward(desc, out, g_phi, 0.37)
    p64 = params.astype(np.float64)
    g64, z64 = of.flow_vjp(p64, z, fs, g_phi.astype(np.float64), 0.37)
    g16, z16 = of.flow_vjp(p64, z, fs, g_phi.astype(np.float64), 0.37, emulate="bf16")
    for lay_g, lay_16, lay_64 in zip(of.unpack(gp, fs), of.unpack(g16, fs), of.unpack(g64, fs)):
        for a, e, r in zip(lay_g, lay_16, lay_64):
            assert rel_norm(a, e) <= 5e-2, (rel_norm(a, e), a.shape)
            assert rel_norm(a, r) <= max(0.4, 3 * rel_norm(e, r)), (rel_norm(a, r), a.shape)
    assert rel_norm(gp, g16) <= 2e-2 and rel_norm(gz, z16) <= 2e-2
    assert rel_norm(gp, g64) <= max(0.1, 3 * rel_norm(g16, g64))


def test_net_without_tanh():
    desc, params, z, fs = _net_case(2, 6, 2, 5, (4, 3), 3, lfs.LFS_PLAIN_FP32, tanh=False)
    out, _ = _check_forward(desc, params, z, fs, lfs.LFS_PLAIN_FP32)
    _check_backward(desc, params, z, fs, out, lfs.LFS_PLAIN_FP32)


def test_net_deterministic_and_batch_position():
    desc, params, z, fs = _net_case(2, 8, 3, 5, (6, 4), 6, lfs.LFS_BF16_CONV)
    a = run_forward(desc, params, z)
    b = run_forward(desc, params, z)
    part = run_forward(desc, params, z[2:4])
    np.testing.assert_array_equal(host(a["phi"]), host(b["phi"]))
    np.testing.assert_array_equal(host(a["phi"])[2:4], host(part["phi"]))
    np.testing.assert_array_equal(host(a["logq"])[2:4], host(part["logq"]))
    g = np.random.default_rng(2).standard_normal(z.shape).astype(np.float32)
    ga, za = run_backward(desc, a, g, 0.2)
    gb, zb = run_backward(desc, b, g, 0.2)
    np.testing.assert_array_equal(ga, gb)
    np.testing.assert_array_equal(za, zb)


def test_explicit_default_network_matches_default():
    """hidden_sizes (C, C) with kernel 3 is the default network: same kernels, same bits."""
    params = si.flow_params(2, 4, 8, seed=7, w_std=0.1, b_std=0.05)
    z = si.normal_fields(8, 4, 64)
    d0 = lfs.make_desc(2, 8, 4, 8, precision=lfs.LFS_BF16_CONV)
    d1 = lfs.make_desc(2, 8, 4, 0, precision=lfs.LFS_BF16_CONV, kernel=3, hidden_sizes=(8, 8))
    a, b = run_forward(d0, params, z), run_forward(d1, params, z)
    np.testing.assert_array_equal(host(a["phi"]), host(b["phi"]))
    np.testing.assert_array_equal(host(a["logq"]), host(b["logq"]))

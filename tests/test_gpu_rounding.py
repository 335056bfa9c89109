"""Where the kernels round: one coupling layer on operands for which every
convolution sum is exact.

The prior field, weights and biases are chosen on coarse binary grids, with
positive inputs, weights and biases for the two hidden convolutions (so the
LeakyReLU is the identity there) and magnitudes small enough that every partial
sum of every convolution is a multiple of the product grid below 2^24 times it:
then FP32 accumulation in any order (the matrix cores' included) is exact, and
so is the oracle's FP64 sum.  Kernel and emulated oracle (emulate="bf16") then
round the same exact values at the same points, so the hidden
activations and s, t agree exactly; what is left is the FP32 tanh and exp of the
kernels against FP64, a few FP32 ulps.  A kernel that rounded an operand the
emulation keeps, or kept one it rounds, would move s by ~2^-9 relative and fail
by orders of magnitude.  One layer, each parity, every kernel family with BF16
convolutions.  (The plain FP32 path rounds nothing but the field between layers;
its hidden activations keep every bit, so no such grid keeps its sums exact, and
it is held to FP64 directly.)"""
import numpy as np
import pytest

from oracle import flow as of
from paper_2208_08903_amd import lfs

from .gpu_util import host, run_forward

pytestmark = pytest.mark.gpu


def _pow2_at_least(x):
    return 2.0 ** np.ceil(np.log2(x))


def exact_operands(fs: of.FlowShape, B, seed):
    """Prior field and one layer's parameters on grids that make every convolution exact.

    z = k/16 in [0, 2).  First convolution W = k/128 (k = 1..15), b = 1/2 + k/128; later
    hidden ones W = k s (k = 1..3), b = 1/2 + k/256 with s = 1/(4 T cin) rounded down to
    a power of two; the last W = k s (k = -3..3), b = k/256 with s = 1/(T cin) likewise
    (T = K^dim taps of the network's kernel K)."""
    rng = np.random.default_rng(seed)
    T = fs.T
    z = rng.integers(0, 32, size=(B, fs.V)) / 16.0
    lay = []
    convs = fs.conv_shapes
    for i, (co, ci) in enumerate(convs):
        if i == len(convs) - 1:
            sc = 1.0 / _pow2_at_least(T * ci)
            lay += [rng.integers(-3, 4, size=(co, ci, T)) * sc, rng.integers(-8, 9, size=co) / 256.0]
        elif i == 0:
            lay += [rng.integers(1, 16, size=(co, ci, T)) / 128.0, 0.5 + rng.integers(0, 16, size=co) / 128.0]
        else:
            sc = 1.0 / _pow2_at_least(4 * T * ci)
            lay += [rng.integers(1, 4, size=(co, ci, T)) * sc, 0.5 + rng.integers(0, 16, size=co) / 256.0]
    params = of.pack([tuple(lay)])
    return z.astype(np.float32), params.astype(np.float32)


def _grid(a):
    """Largest power of two dividing every nonzero entry of a (its exact binary grid)."""
    a = np.abs(np.asarray(a, np.float64).ravel())
    a = a[a > 0]
    if a.size == 0:
        return 1.0
    m, e = np.frexp(a)                       # a = m 2^e, m in [0.5, 1)
    bits = np.array([len(format(int(v), "b").rstrip("0")) for v in np.ldexp(m, 53).astype(np.int64)])
    return float(2.0 ** np.min(e - bits))


def assert_exact(params, z, fs):
    """Every partial sum of every convolution is exact in FP32: the product grid times
    2^24 exceeds the sum of the absolute terms plus the bias.  The hidden pre-activations
    are positive, so the LeakyReLU is the identity."""
    (lay,) = of.unpack(params, fs)
    convs = of.split_convs(lay, fs)
    R = of.ROUNDERS["bf16"]
    u = R((of.as_lattice(z, fs) * of.frozen_mask(fs, 0))[:, None])
    for i, (W, b, _, _) in enumerate(convs):
        grid = min(_grid(u) * _grid(W), _grid(b))
        bound = of.conv(np.abs(u), np.abs(W), np.abs(b), fs.dim)
        assert np.max(bound) < 2.0 ** 24 * grid, (i, np.max(bound), grid)
        if i < len(convs) - 1:
            a = of.conv(u, W, b, fs.dim)
            assert np.all(a > 0)
            u = R(a)


CASES = [
    # dim, L, C, B, algo
    (2, 8, 8, 3, lfs.ALGO_GENERIC),
    (3, 4, 16, 2, lfs.ALGO_GENERIC),
    (2, 8, 8, 3, lfs.ALGO_FUSED),
    (2, 32, 16, 2, lfs.ALGO_FUSED),
    (2, 16, 32, 2, lfs.ALGO_FUSED),
    (2, 32, 32, 2, lfs.ALGO_FUSED),
    (3, 8, 16, 2, lfs.ALGO_FUSED),
    (3, 12, 16, 2, lfs.ALGO_FUSED),
    (3, 16, 8, 2, lfs.ALGO_FUSED),     # plane-streaming forward
    (3, 16, 16, 2, lfs.ALGO_FUSED),
    (3, 16, 32, 2, lfs.ALGO_FUSED),
]
# general networks (their own kernels): dim, L, kernel, hidden_sizes, B
NET_CASES = [(2, 8, 5, (8, 8), 4), (2, 6, 3, (3, 5, 4), 3), (3, 4, 3, (4,), 2), (2, 8, 1, (6, 6), 3),
             (2, 4, 7, (2, 3), 2), (3, 4, 5, (3, 3), 2)]


def _run_exact(desc, fs, B, seed):
    z, params = exact_operands(fs, B, seed)
    assert_exact(params.astype(np.float64), z.astype(np.float64), fs)
    out = run_forward(desc, params, z)
    emu = of.flow_forward(params.astype(np.float64), z.astype(np.float64), fs, emulate="bf16")
    pe = emu["phi"].reshape(B, fs.V)
    phi = host(out["phi"]).astype(np.float64)
    # frozen sites are copied exactly
    frozen = of.frozen_mask(fs, 0).reshape(-1) > 0
    np.testing.assert_array_equal(phi[:, frozen], z[:, frozen])
    d = np.max(np.abs(phi - pe) / (1 + np.abs(pe)))
    dq = np.max(np.abs(host(out["logq"]) - emu["logq"]))
    print(f"  max |dphi|/(1+|phi|) {d:.2e}, max |dlogq| {dq:.2e}", flush=True)
    assert d <= 4e-6, d
    assert dq <= 2e-7 * fs.V, dq


@pytest.mark.parametrize("dim,L,C,B,algo", CASES)
@pytest.mark.parametrize("parity0", [0, 1])
def test_one_layer_exact_operands(dim, L, C, B, algo, parity0):
    print(f"exact-operand layer dim={dim} L={L} C={C} algo={algo} parity0={parity0}", flush=True)
    fs = of.FlowShape(dim, L, 1, C, parity0=parity0)
    desc = lfs.make_desc(dim, L, 1, C, parity0=parity0, precision=lfs.LFS_BF16_CONV, algo=algo)
    _run_exact(desc, fs, B, seed=31 * L + C + parity0)


@pytest.mark.parametrize("dim,L,K,hs,B", NET_CASES)
def test_one_layer_exact_operands_general_network(dim, L, K, hs, B):
    print(f"exact-operand layer, general network dim={dim} L={L} K={K} hidden={hs}", flush=True)
    fs = of.FlowShape(dim, L, 1, 0, kernel=K, hidden_sizes=hs)
    desc = lfs.make_desc(dim, L, 1, 0, precision=lfs.LFS_BF16_CONV, kernel=K, hidden_sizes=hs)
    _run_exact(desc, fs, B, seed=17 * L + K)

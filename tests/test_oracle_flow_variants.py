"""Pins for the oracle's general s/t networks (the example parameter file's
hidden_sizes and kernel_size): layout, tap order and orientation for other kernel
sizes, adjoints, invertibility, brute-force Jacobians, a hand-computed layer and
central finite differences of the loss."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.flow import (FlowShape, conv, conv_transpose, conv_weight_grad, coupling_forward,
                         flow_forward, flow_inverse, frozen_mask, kl_loss, loss_gradient, pack,
                         parity, tap_offsets, unpack)

from .test_oracle_flow import fd_jacobian


def test_variant_layout():
    # hidden (3, 5, 4), kernel 5 in 2D: convs 1->3, 3->5, 5->4, 4->2 with 25 taps
    fs = FlowShape(2, 6, 2, 0, kernel=5, hidden_sizes=(3, 5, 4))
    per_layer = (3 * 1 + 5 * 3 + 4 * 5 + 2 * 4) * 25 + (3 + 5 + 4 + 2)
    assert si.param_count(2, 2, 0, 5, (3, 5, 4)) == 2 * per_layer
    lay = unpack(np.arange(2 * per_layer, dtype=np.float64), fs)[1]
    shapes = [a.shape for a in lay]
    assert shapes == [(3, 1, 25), (3,), (5, 3, 25), (5,), (4, 5, 25), (4,), (2, 4, 25), (2,)]
    assert lay[0].ravel()[0] == per_layer          # layer 1 starts right after layer 0
    # the default network is hidden (C, C), kernel 3
    assert si.param_count(2, 16, 8, 3, (8, 8)) == si.param_count(2, 16, 8) == 12960


def test_variant_equal_to_default_is_identical():
    fs = FlowShape(2, 4, 3, 4)
    fv = FlowShape(2, 4, 3, 4, kernel=3, hidden_sizes=(4, 4))
    p = si.flow_params(2, 3, 4, seed=3, w_std=0.3, b_std=0.1)
    z = np.random.default_rng(4).standard_normal((2, 16))
    assert np.array_equal(flow_forward(p, z, fs)["phi"], flow_forward(p, z, fv)["phi"])
    assert np.array_equal(loss_gradient(p, z, fs, -1.0, 0.5), loss_gradient(p, z, fv, -1.0, 0.5))


@pytest.mark.parametrize("dim,K", [(2, 5), (3, 5), (2, 1), (2, 7)])
def test_tap_order_and_orientation(dim, K):
    """Taps are row-major over {-K//2..K//2}^dim (axis 0 slowest) and a one-hot kernel
    at offset d reads the site n + d."""
    r = K // 2
    offs = tap_offsets(dim, K)
    assert len(offs) == K ** dim and offs[0] == (-r,) * dim and offs[-1] == (r,) * dim
    if K > 1:
        assert offs[1] == (-r,) * (dim - 1) + (-r + 1,)
    L = 8
    u = np.random.default_rng(0).standard_normal((1, 1) + (L,) * dim)
    rng = np.random.default_rng(1)
    for _ in range(4):
        d = tuple(int(v) for v in rng.integers(-r, r + 1, dim))
        W = np.zeros((1, 1, K ** dim))
        W[0, 0, offs.index(d)] = 1.0
        out = conv(u, W, np.zeros(1), dim)
        np.testing.assert_array_equal(out, np.roll(u, tuple(-x for x in d), axis=tuple(range(2, 2 + dim))))


@pytest.mark.parametrize("dim,L,K", [(2, 4, 5), (2, 6, 5), (3, 4, 3), (2, 5, 7), (2, 4, 1)])
def test_variant_conv_adjoints(dim, L, K):
    rng = np.random.default_rng(2)
    u = rng.standard_normal((2, 3) + (L,) * dim)
    g = rng.standard_normal((2, 4) + (L,) * dim)
    W = rng.standard_normal((4, 3, K ** dim))
    lhs = np.sum(conv(u, W, np.zeros(4), dim) * g)
    np.testing.assert_allclose(lhs, np.sum(u * conv_transpose(g, W, dim)), rtol=1e-12)
    dW, _ = conv_weight_grad(g, u, dim, K)
    np.testing.assert_allclose(lhs, np.sum(dW * W), rtol=1e-12)


VARIANTS = [(2, 4, 3, 5, (3, 5, 4)), (2, 6, 2, 1, (4,)), (3, 4, 2, 3, (2, 3, 2)), (2, 4, 4, 7, (2, 2))]


@pytest.mark.parametrize("dim,L,N,K,hs", VARIANTS)
def test_variant_invertibility(dim, L, N, K, hs):
    fs = FlowShape(dim, L, N, 0, kernel=K, hidden_sizes=hs)
    p = si.flow_params(dim, N, 0, seed=6, w_std=0.2, b_std=0.2, kernel=K, hidden_sizes=hs)
    z = np.random.default_rng(7).standard_normal((3, L ** dim))
    f = flow_forward(p, z, fs)
    zi, ld = flow_inverse(p, f["phi"], fs)
    np.testing.assert_allclose(zi.reshape(3, -1), z, atol=1e-12)
    np.testing.assert_allclose(ld, f["logdet"], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,L,N,K,hs", [(2, 4, 3, 5, (3, 2)), (3, 2, 2, 3, (2, 3, 2)), (2, 4, 2, 1, (3,))])
def test_variant_bruteforce_jacobian(dim, L, N, K, hs):
    fs = FlowShape(dim, L, N, 0, kernel=K, hidden_sizes=hs)
    p = si.flow_params(dim, N, 0, seed=8, w_std=0.15, b_std=0.3, kernel=K, hidden_sizes=hs)
    z = np.random.default_rng(9).standard_normal(L ** dim)
    J = fd_jacobian(lambda v: flow_forward(p, v[None], fs)["phi"].ravel(), z)
    sign, logabs = np.linalg.slogdet(J)
    assert sign > 0
    assert abs(logabs - flow_forward(p, z[None], fs)["logdet"][0]) < 1e-6
    lay = unpack(p, fs)[0]
    Jl = fd_jacobian(lambda v: coupling_forward(v.reshape((1,) + fs.lattice), lay, 0, fs)[0].ravel(), z)
    F = frozen_mask(fs, 0).ravel() > 0
    assert np.max(np.abs(Jl[np.ix_(F, ~F)])) < 1e-9


def test_hand_computed_pointwise_layer():
    """Kernel 1, one hidden conv of 2 channels: W1 = 0, b1 = -1 -> h1 = -0.01 on both
    channels; W2_s = (1, 1), W2_t = (-1, -1), b2 = (0.5, 0) -> o_s = 0.48, t = 0.02."""
    fs = FlowShape(2, 4, 1, 0, kernel=1, hidden_sizes=(2,))
    W1, b1 = np.zeros((2, 1, 1)), np.full(2, -1.0)
    W2 = np.array([[[1.0], [1.0]], [[-1.0], [-1.0]]])
    b2 = np.array([0.5, 0.0])
    p = pack([(W1, b1, W2, b2)])
    z = np.random.default_rng(10).standard_normal((1, 16))
    f = flow_forward(p, z, fs)
    odd = parity(fs).ravel() == 1
    s = np.tanh(0.48)
    np.testing.assert_allclose(f["phi"].ravel()[odd], z.ravel()[odd] * np.exp(s) + 0.02, rtol=1e-12)
    np.testing.assert_array_equal(f["phi"].ravel()[~odd], z.ravel()[~odd])
    np.testing.assert_allclose(f["logdet"], 8 * s, rtol=1e-12)


@pytest.mark.parametrize("dim,L,N,K,hs,tanh", [(2, 4, 2, 5, (3, 2), True), (2, 2, 2, 1, (3, 2, 2), False),
                                                (3, 2, 2, 3, (2,), True), (2, 4, 2, 3, (2, 3, 2), True)])
def test_variant_loss_gradient_central_fd(dim, L, N, K, hs, tanh):
    fs = FlowShape(dim, L, N, 0, final_tanh=tanh, kernel=K, hidden_sizes=hs)
    p = si.flow_params(dim, N, 0, seed=11, w_std=0.4, b_std=0.2, kernel=K,
                       hidden_sizes=hs).astype(np.float64)
    z = np.random.default_rng(12).standard_normal((3, L ** dim))
    m2, lam = -1.5, 0.7
    g = loss_gradient(p, z, fs, m2, lam)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd[i] = (kl_loss(pp, z, fs, m2, lam) - kl_loss(pm, z, fs, m2, lam)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8 * np.max(np.abs(fd)))
    for lay in unpack(g, fs):
        for k, blk in enumerate(lay):
            if K == 1 and k == 0:
                # a pointwise first conv reads only the site itself, which is zeroed
                # wherever s and t are used: W1 cannot matter
                assert np.all(blk == 0)
            else:
                assert np.any(blk != 0)

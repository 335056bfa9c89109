"""Pins for oracle.flow: each one is fixed by something other than the oracle itself."""
import itertools

import numpy as np
import pytest
from scipy import stats

import seeded_inputs as si
from oracle.action import action
from oracle.flow import (FlowShape, conv, conv_transpose, conv_weight_grad, flow_forward,
                         flow_inverse, flow_vjp, frozen_mask, kl_loss, loss_gradient, pack,
                         parity, tap_offsets, unpack, coupling_forward)


def zero_layers(fs):
    return unpack(np.zeros(si.param_count(fs.dim, fs.n_layers, fs.hidden)), fs)


def with_bias(fs, bs=0.0, bt=0.0):
    lays = zero_layers(fs)
    for lay in lays:
        lay[5][0], lay[5][1] = bs, bt
    return pack(lays)


def test_param_count_matches_paper_example():
    # example parameter file: 2D, 16 layers, hidden [8, 8], kernel 3
    assert si.param_count(2, 16, 8) == 12960
    assert si.param_count(2, 16, 16) == 44320
    assert si.param_count(3, 12, 16) == 98904
    assert si.param_count(3, 16, 32) == 484896


@pytest.mark.parametrize("dim", [2, 3])
def test_conv_orientation_one_hot(dim):
    """One-hot kernel at offset +e_mu reads the neighbour at n + e_mu: out = roll(in, -1, mu)."""
    L = 4
    u = np.random.default_rng(0).standard_normal((2, 1) + (L,) * dim)
    offs = tap_offsets(dim)
    for mu in range(dim):
        for sgn in (1, -1):
            d = tuple(sgn if a == mu else 0 for a in range(dim))
            W = np.zeros((1, 1, 3 ** dim))
            W[0, 0, offs.index(d)] = 1.0
            out = conv(u, W, np.zeros(1), dim)
            np.testing.assert_array_equal(out, np.roll(u, -sgn, axis=2 + mu))
    # tap index is row-major over offsets with axis 0 slowest
    assert offs[0] == (-1,) * dim and offs[-1] == (1,) * dim and offs[1] == (-1,) * (dim - 1) + (0,)


@pytest.mark.parametrize("dim,L", [(2, 2), (2, 4), (3, 2), (3, 4)])
def test_conv_adjoints_dot_product(dim, L):
    rng = np.random.default_rng(1)
    u = rng.standard_normal((2, 3) + (L,) * dim)
    g = rng.standard_normal((2, 5) + (L,) * dim)
    W = rng.standard_normal((5, 3, 3 ** dim))
    lhs = np.sum((conv(u, W, np.zeros(5), dim)) * g)
    np.testing.assert_allclose(lhs, np.sum(u * conv_transpose(g, W, dim)), rtol=1e-12)
    dW, db = conv_weight_grad(g, u, dim)
    np.testing.assert_allclose(lhs, np.sum(dW * W), rtol=1e-12)
    np.testing.assert_allclose(db, g.sum(axis=(0,) + tuple(range(2, 2 + dim))), rtol=1e-12)


def test_checkerboard_parity_and_alternation():
    fs = FlowShape(2, 4, 4, 8)
    p = parity(fs)
    assert p[0, 0] == 0 and p[0, 1] == 1 and p[1, 1] == 0
    assert np.array_equal(frozen_mask(fs, 0), (p == 0)) and np.array_equal(frozen_mask(fs, 1), (p == 1))
    fs3 = FlowShape(3, 2, 2, 8)
    assert parity(fs3)[1, 1, 1] == 1


@pytest.mark.parametrize("dim,L,N", [(2, 4, 4), (3, 4, 2), (2, 8, 16)])
def test_identity_flow(dim, L, N):
    fs = FlowShape(dim, L, N, 8)
    z = np.random.default_rng(2).standard_normal((3, L ** dim))
    f = flow_forward(np.zeros(si.param_count(dim, N, 8)), z, fs)
    assert np.array_equal(f["phi"].reshape(3, -1), z) and np.all(f["logdet"] == 0)


def test_shift_flow_and_which_sites_move():
    fs = FlowShape(2, 4, 6, 8)
    z = np.random.default_rng(3).standard_normal((2, 16))
    f = flow_forward(with_bias(fs, bt=0.25), z, fs)
    np.testing.assert_allclose(f["phi"].reshape(2, -1), z + 3 * 0.25, rtol=0, atol=1e-15)
    assert np.all(f["logdet"] == 0)
    # a single layer (layer 0 freezes even sites) moves only the odd sites
    y, ld = coupling_forward(z.reshape(2, 4, 4), unpack(with_bias(fs, bt=1.0), fs)[0], 0, fs)
    d = (y - z.reshape(2, 4, 4))[0]
    assert d[0, 0] == 0 and d[1, 1] == 0 and d[0, 1] == 1 and d[1, 0] == 1


@pytest.mark.parametrize("dim,L,N,a", [(2, 4, 4, -0.9), (3, 2, 6, 0.3), (2, 8, 16, -1.2)])
def test_uniform_scale_flow_density(dim, L, N, a):
    """Zero weights and b_s = atanh(a / (N/2)): phi = e^a z, so q = N(0, e^{2a}) per site in closed form."""
    fs = FlowShape(dim, L, N, 4)
    z = np.random.default_rng(4).standard_normal((5, L ** dim))
    f = flow_forward(with_bias(fs, bs=np.arctanh(a / (N / 2))), z, fs)
    np.testing.assert_allclose(f["phi"].reshape(5, -1), np.exp(a) * z, rtol=1e-12)
    ref = stats.norm.logpdf(f["phi"].reshape(5, -1), scale=np.exp(a)).sum(axis=1)
    np.testing.assert_allclose(f["logq"], ref, rtol=1e-12)
    np.testing.assert_allclose(f["logdet"], L ** dim * a, rtol=1e-12)


def test_importance_sampling_free_field_lnZ():
    """The log q / log p chain end to end: ln mean(e^w) estimates the exact free-field ln Z."""
    dim, L, m2 = 2, 4, 4.0
    k = 2 * np.pi * np.arange(L) / L
    ev = m2 + np.array([np.sum(4 * np.sin(np.array(kk) / 2) ** 2) for kk in itertools.product(k, repeat=dim)])
    lnZ = 0.5 * L ** dim * np.log(np.pi) - 0.5 * np.sum(np.log(ev))
    N = 4
    a = 0.5 * np.log(1 / (2 * (m2 + 2 * dim)))
    fs = FlowShape(dim, L, N, 2)
    z = np.random.default_rng(5).standard_normal((40000, L ** dim))
    f = flow_forward(with_bias(fs, bs=np.arctanh(a / (N / 2))), z, fs)
    w = -action(f["phi"], m2, 0.0, dim) - f["logq"]
    est = np.log(np.mean(np.exp(w - w.max()))) + w.max()
    assert abs(est - lnZ) < 0.05, (est, lnZ)          # a flipped log-det sign moves it by 2 V a = -44


@pytest.mark.parametrize("dim,L,N,C,w", [(2, 4, 4, 8, 0.3), (3, 4, 3, 4, 0.3), (2, 8, 16, 8, 0.1)])
def test_invertibility(dim, L, N, C, w):
    # (deep flows with w = 0.3 grow fields to ~1e5 and the inverse loses digits to cancellation)
    fs = FlowShape(dim, L, N, C)
    p = si.flow_params(dim, N, C, seed=6, w_std=w, b_std=0.2)
    z = np.random.default_rng(7).standard_normal((3, L ** dim))
    f = flow_forward(p, z, fs)
    zi, ld = flow_inverse(p, f["phi"], fs)
    np.testing.assert_allclose(zi.reshape(3, -1), z, atol=1e-12)
    np.testing.assert_allclose(ld, f["logdet"], rtol=1e-12, atol=1e-12)


def fd_jacobian(fun, z, h=1e-5):
    V = z.size
    J = np.zeros((V, V))
    for i in range(V):
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        J[:, i] = (fun(zp) - fun(zm)) / (2 * h)
    return J


@pytest.mark.parametrize("dim,L,N", [(2, 2, 4), (2, 4, 4), (3, 2, 4), (3, 4, 2)])
def test_bruteforce_jacobian(dim, L, N):
    fs = FlowShape(dim, L, N, 4)
    # w = 0.15 keeps fields O(1): with saturated tanh the composed FD Jacobian loses digits
    p = si.flow_params(dim, N, 4, seed=8, w_std=0.15, b_std=0.3)
    z = np.random.default_rng(9).standard_normal(L ** dim)
    J = fd_jacobian(lambda v: flow_forward(p, v[None], fs)["phi"].ravel(), z)
    sign, logabs = np.linalg.slogdet(J)
    assert sign > 0
    assert abs(logabs - flow_forward(p, z[None], fs)["logdet"][0]) < 1e-6
    # each layer is triangular in the (frozen, active) ordering: d y_F / d x_A = 0
    lay = unpack(p, fs)[0]
    Jl = fd_jacobian(lambda v: coupling_forward(v.reshape((1,) + fs.lattice), lay, 0, fs)[0].ravel(), z)
    F = frozen_mask(fs, 0).ravel() > 0
    assert np.max(np.abs(Jl[np.ix_(F, ~F)])) < 1e-9
    np.testing.assert_allclose(Jl[np.ix_(F, F)], np.eye(F.sum()), atol=1e-9)


def test_hand_computed_single_layer():
    """W1 = 0, b1 = -1 -> h1 = -0.01 (LeakyReLU slope); W2 = 0.5 everywhere, b2 = 0 ->
    a2 = 0.5 * (2 ch * 9 taps) * (-0.01) = -0.09, h2 = -0.0009; W3_s = 1, b3_s = 0.5 ->
    o_s = 0.5 + 18 * (-0.0009) = 0.4838; W3_t = -1, b3_t = 0 -> t = 0.0162."""
    fs = FlowShape(2, 4, 1, 2)
    W1, b1 = np.zeros((2, 1, 9)), np.full(2, -1.0)
    W2, b2 = np.full((2, 2, 9), 0.5), np.zeros(2)
    W3 = np.stack([np.ones((2, 9)), -np.ones((2, 9))])
    b3 = np.array([0.5, 0.0])
    p = pack([(W1, b1, W2, b2, W3, b3)])
    z = np.random.default_rng(10).standard_normal((1, 16))
    f = flow_forward(p, z, fs)
    odd = parity(fs).ravel() == 1
    s = np.tanh(0.4838)
    np.testing.assert_allclose(f["phi"].ravel()[odd], z.ravel()[odd] * np.exp(s) + 0.0162, rtol=1e-12)
    np.testing.assert_array_equal(f["phi"].ravel()[~odd], z.ravel()[~odd])
    np.testing.assert_allclose(f["logdet"], 8 * s, rtol=1e-12)
    # without the final tanh, s is the raw 0.4838
    fs2 = FlowShape(2, 4, 1, 2, final_tanh=False)
    np.testing.assert_allclose(flow_forward(p, z, fs2)["logdet"], 8 * 0.4838, rtol=1e-12)


@pytest.mark.parametrize("dim,L,N,C,tanh", [(2, 4, 2, 3, True), (3, 2, 2, 2, True), (2, 2, 3, 2, False)])
def test_loss_gradient_central_fd(dim, L, N, C, tanh):
    fs = FlowShape(dim, L, N, C, final_tanh=tanh)
    p = si.flow_params(dim, N, C, seed=11, w_std=0.4, b_std=0.2).astype(np.float64)
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
    # every layer block receives a gradient
    for lay in unpack(g, fs):
        for blk in lay:
            assert np.any(blk != 0)


def test_vjp_wrt_z_central_fd():
    fs = FlowShape(2, 4, 3, 3)
    p = si.flow_params(2, 3, 3, seed=13, w_std=0.4, b_std=0.2)
    z = np.random.default_rng(14).standard_normal((2, 16))
    gphi = np.random.default_rng(15).standard_normal((2, 16))
    glq = np.array([0.3, -0.7])
    _, gz = flow_vjp(p, z, fs, gphi, glq)
    def scal(zz):
        f = flow_forward(p, zz, fs)
        return np.sum(f["phi"].reshape(2, -1) * gphi) + np.sum(glq * f["logq"])
    h = 1e-6
    fd = np.zeros_like(z)
    for b in range(2):
        for i in range(16):
            zp, zm = z.copy(), z.copy()
            zp[b, i] += h
            zm[b, i] -= h
            fd[b, i] = (scal(zp) - scal(zm)) / (2 * h)
    np.testing.assert_allclose(gz, fd, rtol=1e-6, atol=1e-8)

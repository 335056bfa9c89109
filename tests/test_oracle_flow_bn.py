"""Pins for the oracle's batch norm (the example parameter file's use_bn): layout,
the first hidden convolution against numpy's mean and variance, the bias dropping
out under batch statistics, running statistics equal to the batch's reproducing
batch mode, running mode equal to a plain network with the normalisation folded
into its convolutions, invertibility, the brute-force Jacobian of a whole batch,
the running average against numpy's unbiased variance, and central finite
differences of the loss under batch and running statistics."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle.flow import (BN_EPS, FlowShape, bn_running_update, flow_forward, flow_inverse, frozen_mask,
                         initial_bn_stats, kl_loss, loss_gradient, net, pack, pack_bn_stats, split_convs,
                         unpack, unpack_bn_stats)

from .test_oracle_flow import fd_jacobian


def _case(dim, L, N, K, hs, seed=5, w_std=0.3, b_std=0.2, tanh=True):
    fs = FlowShape(dim, L, N, 0, final_tanh=tanh, kernel=K, hidden_sizes=hs, batch_norm=True)
    p = si.flow_params(dim, N, 0, seed=seed, w_std=w_std, b_std=b_std, kernel=K, hidden_sizes=hs,
                       batch_norm=True, gamma_std=0.2).astype(np.float64)
    return fs, p


def test_bn_layout():
    assert BN_EPS == 1e-5
    fs, p = _case(2, 4, 2, 3, (3, 4))
    per_layer = (3 * 9 + 3 + 2 * 3) + (4 * 3 * 9 + 4 + 2 * 4) + (2 * 4 * 9 + 2)
    assert p.size == 2 * per_layer == si.param_count(2, 2, 0, 3, (3, 4), batch_norm=True)
    lay = unpack(np.arange(p.size, dtype=np.float64), fs)[0]
    assert [a.shape for a in lay] == [(3, 1, 9), (3,), (3,), (3,), (4, 3, 9), (4,), (4,), (4,), (2, 4, 9), (2,)]
    # gamma follows the bias and beta the gamma
    assert lay[2][0] == lay[1][-1] + 1 and lay[3][0] == lay[2][-1] + 1
    convs = split_convs(lay, fs)
    assert convs[-1][2] is None and convs[0][2] is lay[2]
    # the generator draws gamma around 1
    g = unpack(p, fs)[1][2]
    assert np.all(np.abs(g - 1.0) < 1.0) and np.any(g != 1.0)
    st = si.bn_stats(3, 2, (3, 4))
    assert st.size == 2 * 2 * (3 + 4)
    back = pack_bn_stats(unpack_bn_stats(st, fs))
    np.testing.assert_array_equal(back, st.astype(np.float64))
    init = pack_bn_stats(initial_bn_stats(fs))
    np.testing.assert_array_equal(init, np.tile(np.concatenate([np.zeros(3), np.ones(3), np.zeros(4), np.ones(4)]), 2))


def test_bn_first_hidden_conv_against_numpy():
    """y_1 = gamma (a_1 - mean) / sqrt(var + eps) + beta, a_1 from the plain network with
    the same W_1, b_1, mean and biased variance from numpy over batch and sites; the
    normalised activations have per-channel mean 0 and mean square var / (var + eps)."""
    fs, p = _case(2, 6, 1, 3, (4, 3))
    plain = FlowShape(2, 6, 1, 0, kernel=3, hidden_sizes=(4, 3))
    lay = unpack(p, fs)[0]
    W1, b1, g1, be1 = split_convs(lay, fs)[0]
    lay_plain = (W1, b1, np.zeros((3, 4, 9)), np.zeros(3), np.zeros((2, 3, 9)), np.zeros(2))
    x = np.random.default_rng(1).standard_normal((5, 6, 6))
    mF = frozen_mask(fs, 0)
    a1 = net(x, lay_plain, mF, plain)[0][0]
    mean = np.mean(a1, axis=(0, 2, 3))
    var = np.var(a1, axis=(0, 2, 3))
    cache = []
    y1 = net(x, lay, mF, fs, bn_cache=cache)[0][0]
    want = g1[None, :, None, None] * (a1 - mean[None, :, None, None]) / np.sqrt(var + BN_EPS)[None, :, None, None]
    np.testing.assert_allclose(y1, want + be1[None, :, None, None], rtol=1e-12, atol=1e-12)
    for xh, _, _, _ in cache:
        np.testing.assert_allclose(xh.mean(axis=(0, 2, 3)), 0.0, atol=1e-12)
        ms = (xh ** 2).mean(axis=(0, 2, 3))
        assert np.all(ms <= 1.0) and np.all(ms > 1.0 - 1e-3)


def test_bn_bias_drops_out_under_batch_statistics():
    fs, p = _case(2, 4, 2, 3, (3, 4))
    z = np.random.default_rng(2).standard_normal((3, 16))
    layers = unpack(p, fs)
    shifted = [list(lay) for lay in layers]
    rng = np.random.default_rng(3)
    for lay in shifted:
        lay[1] = lay[1] + rng.normal(0, 1.0, lay[1].shape)     # b_1
        lay[5] = lay[5] + rng.normal(0, 1.0, lay[5].shape)     # b_2
    q = pack([tuple(lay) for lay in shifted])
    f0, f1 = flow_forward(p, z, fs), flow_forward(q, z, fs)
    np.testing.assert_allclose(f1["phi"], f0["phi"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f1["logq"], f0["logq"], rtol=1e-12)
    # not under running statistics
    st = initial_bn_stats(fs)
    assert np.max(np.abs(flow_forward(q, z, fs, bn_stats=st)["phi"] - flow_forward(p, z, fs, bn_stats=st)["phi"])) > 1e-3
    g = loss_gradient(p, z, fs, -1.0, 0.5)
    for lay in unpack(g, fs):
        scale = max(np.max(np.abs(a)) for a in lay)
        assert np.max(np.abs(lay[1])) <= 1e-12 * scale and np.max(np.abs(lay[5])) <= 1e-12 * scale
        assert np.any(lay[2] != 0) and np.any(lay[3] != 0) and np.any(lay[9] != 0)


def test_bn_running_with_batch_statistics_reproduces_batch_mode():
    fs, p = _case(3, 4, 2, 3, (2, 3))
    z = np.random.default_rng(4).standard_normal((2, 64))
    fb = flow_forward(p, z, fs)
    fr = flow_forward(p, z, fs, bn_stats=fb["bn_used"])
    np.testing.assert_allclose(fr["phi"], fb["phi"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(fr["logq"], fb["logq"], rtol=1e-12)
    # the gradients differ: batch statistics are differentiated as functions of the batch
    gb = loss_gradient(p, z, fs, -1.0, 0.5)
    gr = loss_gradient(p, z, fs, -1.0, 0.5, bn_stats=fb["bn_used"])
    assert np.linalg.norm(gb - gr) > 1e-3 * np.linalg.norm(gb)


def test_bn_running_mode_is_folded_plain_network():
    fs, p = _case(2, 4, 3, 5, (3, 2), w_std=0.2)
    plain = FlowShape(2, 4, 3, 0, kernel=5, hidden_sizes=(3, 2))
    st = unpack_bn_stats(si.bn_stats(9, 3, (3, 2)), fs)
    folded = []
    for l, lay in enumerate(unpack(p, fs)):
        convs = split_convs(lay, fs)
        out = []
        for i, (W, b, g, be) in enumerate(convs):
            if g is not None:
                mean, var = st[l][i]
                k = g / np.sqrt(var + BN_EPS)
                W, b = W * k[:, None, None], (b - mean) * k + be
            out += [W, b]
        folded.append(tuple(out))
    q = pack(folded)
    z = np.random.default_rng(6).standard_normal((4, 16))
    fr, fp = flow_forward(p, z, fs, bn_stats=st), flow_forward(q, z, plain)
    np.testing.assert_allclose(fr["phi"], fp["phi"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(fr["logq"], fp["logq"], rtol=1e-12)


@pytest.mark.parametrize("running", [False, True])
def test_bn_invertibility(running):
    fs, p = _case(2, 6, 4, 3, (4, 4))
    st = unpack_bn_stats(si.bn_stats(10, 4, (4, 4)), fs) if running else None
    z = np.random.default_rng(7).standard_normal((3, 36))
    f = flow_forward(p, z, fs, bn_stats=st)
    zi, ld = flow_inverse(p, f["phi"], fs, bn_stats=st)
    np.testing.assert_allclose(zi.reshape(3, -1), z, atol=1e-11)
    np.testing.assert_allclose(ld, f["logdet"], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("running", [False, True])
def test_bn_batch_jacobian(running):
    """The batch map's Jacobian: its log-determinant is the sum of the samples' log-dets;
    its off-diagonal sample blocks are non-zero only under batch statistics."""
    fs, p = _case(2, 4, 2, 3, (3, 2), w_std=0.15)
    st = unpack_bn_stats(si.bn_stats(11, 2, (3, 2)), fs) if running else None
    B, V = 2, 16
    z = np.random.default_rng(8).standard_normal(B * V)
    J = fd_jacobian(lambda v: flow_forward(p, v.reshape(B, V), fs, bn_stats=st)["phi"].ravel(), z)
    sign, logabs = np.linalg.slogdet(J)
    f = flow_forward(p, z.reshape(B, V), fs, bn_stats=st)
    assert sign > 0 and abs(logabs - f["logdet"].sum()) < 1e-6
    cross = np.max(np.abs(J[:V, V:]))
    assert (cross < 1e-9) if running else (cross > 1e-4)


def test_bn_running_update_against_numpy():
    """Layer 0's first hidden convolution: after one batch, running = 0.9 running +
    0.1 (numpy mean, numpy unbiased variance) of its pre-normalisation output; the
    bn_used statistics are numpy's mean and biased variance."""
    fs, p = _case(2, 6, 2, 3, (3, 2))
    plain = FlowShape(2, 6, 2, 0, kernel=3, hidden_sizes=(3, 2))
    z = np.random.default_rng(12).standard_normal((4, 36))
    f = flow_forward(p, z, fs)
    W1, b1, _, _ = split_convs(unpack(p, fs)[0], fs)[0]
    lay_plain = (W1, b1, np.zeros((2, 3, 9)), np.zeros(2), np.zeros((2, 2, 9)), np.zeros(2))
    a1 = net(z.reshape(4, 6, 6), lay_plain, frozen_mask(fs, 0), plain)[0][0]
    mean, var = f["bn_used"][0][0]
    np.testing.assert_allclose(mean, np.mean(a1, axis=(0, 2, 3)), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(var, np.var(a1, axis=(0, 2, 3)), rtol=1e-12)
    r0 = unpack_bn_stats(si.bn_stats(13, 2, (3, 2)), fs)
    r1 = bn_running_update(r0, f["bn_used"], 4 * 36)
    np.testing.assert_allclose(r1[0][0][0], 0.9 * r0[0][0][0] + 0.1 * np.mean(a1, axis=(0, 2, 3)), rtol=1e-12)
    np.testing.assert_allclose(r1[0][0][1], 0.9 * r0[0][0][1] + 0.1 * np.var(a1, axis=(0, 2, 3), ddof=1),
                               rtol=1e-12)
    # k identical updates: r_k = 0.9^k r_0 + (1 - 0.9^k) s
    rk = r0
    for _ in range(5):
        rk = bn_running_update(rk, f["bn_used"], 4 * 36)
    s_var = np.var(a1, axis=(0, 2, 3), ddof=1)
    np.testing.assert_allclose(rk[0][0][1], 0.9 ** 5 * r0[0][0][1] + (1 - 0.9 ** 5) * s_var, rtol=1e-12)


@pytest.mark.parametrize("dim,L,N,K,hs,tanh,running", [
    (2, 4, 2, 3, (3, 2), True, False),
    (3, 2, 2, 3, (2,), True, False),
    (2, 4, 2, 1, (2, 3), False, False),
    (2, 4, 2, 3, (3,), True, True),
])
def test_bn_loss_gradient_central_fd(dim, L, N, K, hs, tanh, running):
    fs, p = _case(dim, L, N, K, hs, seed=14, w_std=0.4, tanh=tanh)
    st = unpack_bn_stats(si.bn_stats(15, N, hs), fs) if running else None
    z = np.random.default_rng(16).standard_normal((3, L ** dim))
    m2, lam = -1.5, 0.7
    g = loss_gradient(p, z, fs, m2, lam, bn_stats=st)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd[i] = (kl_loss(pp, z, fs, m2, lam, st) - kl_loss(pm, z, fs, m2, lam, st)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8 * np.max(np.abs(fd)))

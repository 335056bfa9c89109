"""Pins of oracle/analysis.py against closed forms, exact rational arithmetic,
known processes and brute force (CPU only)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import analysis as an


def test_autocovariance_alternating_exact():
    # x_i = (-1)^i, n even: mean 0 and Gamma(t) = (-1)^t for every lag
    n = 64
    x = np.array([(-1.0) ** i for i in range(n)])
    g = an.autocovariance(x, 20)
    assert np.array_equal(g, np.array([(-1.0) ** t for t in range(21)]))


def _ramp_gamma(n, t):
    # exact Gamma(t) of x_i = i (i = 0 .. n-1) with the 1/(n - t) normalisation
    m = Fraction(n - 1, 2)
    K = n - t
    s = sum((Fraction(i) - m) * (Fraction(i + t) - m) for i in range(K))
    return s / K


def test_autocovariance_linear_ramp_rational():
    n = 37
    g = an.autocovariance(np.arange(n, dtype=np.float64), 36)
    ref = np.array([float(_ramp_gamma(n, t)) for t in range(37)])
    assert np.allclose(g, ref, rtol=1e-13, atol=1e-12)
    assert g.shape == (37,)  # lags stop at n - 1 even when w_max is larger
    assert an.autocovariance(np.arange(5.0), 100).shape == (5,)


def test_gamma0_is_biased_variance():
    x = np.random.default_rng(3).standard_normal(1001)
    g0 = an.autocovariance(x, 0)[0]
    n = x.size
    assert np.isclose(g0, np.var(x, ddof=1) * (n - 1) / n, rtol=1e-13)


def test_window_hand_built():
    # rho(t) = 2^-t: tau(W) = 3/2 - 2^-W; with c = 4 the first W >= 4 tau(W) is W = 6
    g = [2.0 ** -t for t in range(20)]
    tau, W, found, nind = an.window(g, 4.0, 100)
    assert (W, found) == (6, True)
    assert tau == 1.5 - 2.0 ** -6
    assert nind == 100 / (2 * tau)
    # no window within the lags: W = last lag, not found
    tau, W, found, _ = an.window(g[:4], 4.0, 100)
    assert (W, found) == (3, False) and tau == 1.5 - 2.0 ** -3
    # zero variance: undefined
    tau, W, found, nind = an.window([0.0, 0.0], 4.0, 10)
    assert np.isnan(tau) and W == 0 and not found and nind == 0.0


def _ar1(a, n, seed):
    e = np.random.default_rng(seed).standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    s = np.sqrt(1 - a * a)
    for i in range(1, n):
        x[i] = a * x[i - 1] + s * e[i]
    return x


@pytest.mark.parametrize("a,n", [(0.5, 200_000), (0.9, 1_000_000)])
def test_tau_int_ar1(a, n):
    """AR(1) with coefficient a has rho(t) = a^t and tau_int = (1 + a) / (2 (1 - a)).
    The windowed estimator's standard error is about tau sqrt(2 (2W + 1) / n)
    (Madras-Sokal); the test allows five of them plus the truncated tail."""
    x = _ar1(a, n, seed=11)
    tau, W, found, nind, _ = an.tau_int(x, 400, 6.0)
    exact = (1 + a) / (2 * (1 - a))
    tail = a ** (W + 1) / (1 - a)
    assert found
    assert abs(tau - exact) <= 5 * exact * np.sqrt(2 * (2 * W + 1) / n) + tail
    assert np.isclose(nind, n / (2 * tau))


def test_tau_int_white_noise_and_constant():
    x = np.random.default_rng(5).standard_normal(100_000)
    tau, W, found, _, _ = an.tau_int(x, 100, 6.0)
    assert found and abs(tau - 0.5) < 0.03 and W <= 6
    tau, W, found, nind, _ = an.tau_int(np.full(50, 2.5), 10, 6.0)
    assert np.isnan(tau) and W == 0 and nind == 0.0
    tau, W, found, nind, _ = an.tau_int(np.array([1.0]), 10, 6.0)
    assert np.isnan(tau) and W == 0


def test_ess_closed_forms():
    N = 100
    assert an.ess(np.zeros(N)) == pytest.approx(1.0, rel=1e-15)
    assert an.ess(np.full(N, 123.0)) == pytest.approx(1.0, rel=1e-15)
    w = np.full(N, -np.inf)
    w[7] = 0.3
    assert an.ess(w) == pytest.approx(1.0 / N, rel=1e-15)
    # k weights 1 and N - k weights r: (k + (N-k) r)^2 / (N (k + (N-k) r^2))
    k, r = 30, 0.25
    w = np.concatenate([np.zeros(k), np.full(N - k, np.log(r))])
    assert an.ess(w) == pytest.approx((k + (N - k) * r) ** 2 / (N * (k + (N - k) * r * r)), rel=1e-14)
    # shift invariance, and no overflow far from zero
    assert an.ess(w + 700.0) == pytest.approx(an.ess(w), rel=1e-14)


@pytest.mark.parametrize("dim,L", [(2, 6), (3, 4)])
def test_observables_closed_forms(dim, L):
    V = L ** dim
    c = 0.75
    phi = np.full((1, V), c)
    assert an.condensate(phi, dim, L)[0] == pytest.approx(c, rel=1e-15)
    # constant field: Phi(t) = c L^(d-1), C(t) = c^2 L^(d-1)
    assert np.allclose(an.two_point_zero_momentum(phi, dim, L)[0], c * c * L ** (dim - 1), rtol=1e-14)
    # plane wave along time, k = 1: C(t) = (L^(d-1) / 2) cos(2 pi t / L), M = 0
    t = np.arange(L).reshape((L,) + (1,) * (dim - 1))
    pw = np.broadcast_to(np.cos(2 * np.pi * t / L), (L,) * dim).reshape(1, V)
    assert abs(an.condensate(pw, dim, L)[0]) < 1e-15
    ref = L ** (dim - 1) / 2 * np.cos(2 * np.pi * np.arange(L) / L)
    assert np.allclose(an.two_point_zero_momentum(pw, dim, L)[0], ref, atol=1e-13)


@pytest.mark.parametrize("dim,L", [(2, 4), (3, 3)])
def test_two_point_brute_force(dim, L):
    """C(t) = sum over spatial separations xs of (1/V) sum_y phi(y) phi(y + (t, xs)),
    written out over every pair of sites."""
    V = L ** dim
    phi = np.random.default_rng(9).standard_normal((2, V))
    coords = [tuple(int(v) for v in np.unravel_index(i, (L,) * dim)) for i in range(V)]
    index = {cc: i for i, cc in enumerate(coords)}
    for b in range(2):
        ref = np.zeros(L)
        for y in coords:
            for x in coords:  # separation x = (t, xs)
                z = tuple((y[mu] + x[mu]) % L for mu in range(dim))
                ref[x[0]] += phi[b, index[y]] * phi[b, index[z]] / V
        assert np.allclose(an.two_point_zero_momentum(phi[b:b + 1], dim, L)[0], ref, rtol=1e-12, atol=1e-13)
        assert an.condensate(phi[b:b + 1], dim, L)[0] == pytest.approx(sum(phi[b]) / V, rel=1e-13)

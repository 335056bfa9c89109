"""Pins for oracle.mh, oracle.hmc and oracle.adam."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle.action import action
from oracle.adam import adam_step
from oracle.hmc import hamiltonian, hmc_step, leapfrog
from oracle.mh import ChainState, acceptance_rate, mh_chain


def test_mh_log_u_minus_inf_accepts_all():
    w = np.random.default_rng(0).standard_normal(50) * 30
    cur, acc, st = mh_chain(w, np.full(50, -np.inf))
    assert np.all(acc == 1) and np.array_equal(cur, np.arange(50)) and st.n_acc == 49


def test_mh_constant_weight_accepts_all():
    u = np.random.default_rng(1).random(100)
    cur, acc, st = mh_chain(np.full(100, -3.25), np.log(u))
    assert np.all(acc == 1) and acceptance_rate(st) == 1.0


def test_mh_rejection_repeats_current_and_first_seeds():
    w = np.array([0.0, -10.0, -10.0, 5.0, 4.0])
    lu = np.log(np.array([0.5, 0.5, 0.5, 0.5, 0.5]))
    cur, acc, st = mh_chain(w, lu)
    # k=1: d=-10 < log .5 -> reject; k=3: d=5 -> accept; k=4: d=-1 < log .5 = -0.69 -> reject
    assert list(acc) == [1, 0, 0, 1, 0] and list(cur) == [0, 0, 0, 3, 3] and st.n_acc == 1


def test_mh_state_persists_across_calls():
    rng = np.random.default_rng(2)
    w, lu = rng.standard_normal(300), np.log(rng.random(300))
    c_all, a_all, s_all = mh_chain(w, lu)
    c1, a1, s1 = mh_chain(w[:120], lu[:120])
    c2, a2, s2 = mh_chain(w[120:], lu[120:], s1)
    assert np.array_equal(np.concatenate([c1, c2]), c_all) and np.array_equal(np.concatenate([a1, a2]), a_all)
    assert vars(s2) == vars(s_all)


def test_mh_independence_sampler_stationary_law():
    """Target N(0,1), proposals N(0, 2^2): w = log N(x;0,1) - log N(x;0,4); chain histogram -> N(0,1)."""
    rng = np.random.default_rng(3)
    K = 40000
    x = rng.normal(0, 2.0, K)
    w = stats.norm.logpdf(x) - stats.norm.logpdf(x, scale=2.0)
    cur, acc, st = mh_chain(w, np.log(rng.random(K)))
    chain = x[cur]
    thin = chain[::5]
    assert stats.kstest(thin, "norm").pvalue > 1e-3
    assert 0.5 < acceptance_rate(st) < 0.9


def free_field_sample(rng, L, dim, m2, n):
    """Exact draws from exp(-phi^T M phi), M = -Lap + m2 (covariance (2M)^-1)."""
    V = L ** dim
    A = np.zeros((V, V))
    idx = lambda c: int(np.ravel_multi_index(c, (L,) * dim))
    for c in itertools.product(range(L), repeat=dim):
        i = idx(c)
        A[i, i] += 2 * dim + m2
        for mu in range(dim):
            for s in (1, -1):
                nb = list(c)
                nb[mu] = (nb[mu] + s) % L
                A[i, idx(nb)] -= 1
    cov = np.linalg.inv(2 * A)
    return rng.multivariate_normal(np.zeros(V), cov, size=n).reshape((n,) + (L,) * dim)


@pytest.mark.parametrize("dim,L", [(2, 4), (3, 2)])
def test_leapfrog_reversible(dim, L):
    rng = np.random.default_rng(4)
    phi = rng.standard_normal((3,) + (L,) * dim)
    pi = rng.standard_normal(phi.shape)
    p1, q1 = leapfrog(phi, pi, -4.0, 5.0, dim, 10, 0.05)
    p2, q2 = leapfrog(p1, -q1, -4.0, 5.0, dim, 10, 0.05)
    np.testing.assert_allclose(p2, phi, atol=1e-11)
    np.testing.assert_allclose(-q2, pi, atol=1e-11)


def test_leapfrog_volume_preserving():
    dim, L = 2, 2
    rng = np.random.default_rng(5)
    x0 = rng.standard_normal(8) * 0.5
    def F(x):
        p, q = leapfrog(x[:4].reshape(1, 2, 2), x[4:].reshape(1, 2, 2), -1.0, 2.0, dim, 10, 0.1)
        return np.concatenate([p.ravel(), q.ravel()])
    J = np.zeros((8, 8))
    h = 1e-6
    for i in range(8):
        a, b = x0.copy(), x0.copy()
        a[i] += h
        b[i] -= h
        J[:, i] = (F(a) - F(b)) / (2 * h)
    assert abs(np.linalg.det(J) - 1) < 1e-7


def test_energy_error_scales_as_dt_squared():
    rng = np.random.default_rng(6)
    phi = free_field_sample(rng, 4, 2, 1.0, 1)
    pi = rng.standard_normal(phi.shape)
    H0 = hamiltonian(phi, pi, 1.0, 0.5, 2)
    errs = []
    for dt in (0.02, 0.01):
        n = int(round(0.4 / dt))
        p, q = leapfrog(phi, pi, 1.0, 0.5, 2, n, dt)
        errs.append(abs(hamiltonian(p, q, 1.0, 0.5, 2) - H0)[0])
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_creutz_identity_free_field():
    """Trajectories started from the exact free-field law: <exp(-dH)> = 1."""
    rng = np.random.default_rng(7)
    n = 4000
    phi = free_field_sample(rng, 4, 2, 1.0, n)
    pi = rng.standard_normal(phi.shape)
    _, dH, _ = hmc_step(phi, pi, np.zeros(n), 1.0, 0.0, 2, 10, 0.1)
    e = np.exp(-dH)
    assert abs(e.mean() - 1) < 5 * e.std() / np.sqrt(n)


@pytest.mark.slow
def test_hmc_free_field_phi2():
    """HMC chain on the free field (d=2, L=4, m2=1): <phi^2> = 0.1317460317.  Trajectory length 0.5:
    at length 1 the modes with m2 + p^2 = 5 rotate by ~pi per trajectory and barely mix."""
    rng = np.random.default_rng(8)
    phi = np.zeros((16, 4, 4))
    acc_phi2 = []
    for it in range(600):
        pi = rng.standard_normal(phi.shape)
        phi, dH, acc = hmc_step(phi, pi, np.log(rng.random(16)), 1.0, 0.0, 2, 10, 0.05)
        if it >= 100:
            acc_phi2.append(np.mean(phi ** 2, axis=(1, 2)))
    est = np.mean(acc_phi2)
    assert abs(est - 0.1317460317) < 0.005


def test_hmc_accept_rule_and_restore():
    rng = np.random.default_rng(9)
    phi = 0.5 * rng.standard_normal((4, 2, 2))
    pi = rng.standard_normal(phi.shape)
    out_acc, dH, acc = hmc_step(phi, pi, np.full(4, -np.inf), -4.0, 8.0, 2, 10, 0.02)
    assert np.all(np.isfinite(dH)) and np.all(acc == 1)
    out_rej, dH2, acc2 = hmc_step(phi, pi, np.full(4, np.inf), -4.0, 8.0, 2, 10, 0.02)
    assert np.all(acc2 == 0) and np.array_equal(out_rej, phi) and np.array_equal(dH, dH2)
    p1, _ = leapfrog(phi, pi, -4.0, 8.0, 2, 10, 0.02)
    np.testing.assert_array_equal(out_acc, p1)


def test_adam_second_step_pins_betas():
    """Two steps from zero state with different gradients.  After two updates
    m = (1 - b1)(b1 g1 + g2) and 1 - b1^2 = (1 - b1)(1 + b1), so the bias-corrected
    moments are weighted means, m_hat = (b1 g1 + g2)/(1 + b1) and
    v_hat = (b2 g1^2 + g2^2)/(1 + b2).  g = (1, -1) gives v_hat = 1 and
    m_hat = -(1 - b1)/(1 + b1) = -0.1/1.9, which fixes b1; g = (1, 0) gives
    m_hat = 0.9/1.9 and v_hat = 0.999/1.999, which then fixes b2 (the decimal values
    are those of b1 = 0.9, b2 = 0.999 written out)."""
    lr, eps = 1e-3, 1e-8
    for g1, g2, step in ((1.0, -1.0, lr * 0.052631578947368425 / (1 + eps)),
                         (1.0, 0.0, -lr * 0.4736842105263158 / (0.706929893933952 + eps)),
                         (-2.0, 0.5, -lr * (-1.8 + 0.5) / 1.9 / (np.sqrt((0.999 * 4 + 0.25) / 1.999) + eps))):
        p0 = np.array([0.25])
        p1, m, v = adam_step(p0, np.array([g1]), np.zeros(1), np.zeros(1), 1, lr=lr)
        p2, _, _ = adam_step(p1, np.array([g2]), m, v, 2, lr=lr)
        np.testing.assert_allclose(p2 - p1, [step], rtol=1e-12, atol=0)
    # a third step: m_hat = (b1^2 g1 + b1 g2 + g3)/(1 + b1 + b1^2), likewise v_hat with b2
    g = (0.5, -1.5, 3.0)
    p, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t, gt in enumerate(g, start=1):
        q, m, v = adam_step(p, np.array([gt]), m, v, t, lr=lr)
        last, p = q - p, q
    mh = (0.81 * 0.5 + 0.9 * -1.5 + 3.0) / (1 + 0.9 + 0.81)
    vh = (0.998001 * 0.25 + 0.999 * 2.25 + 9.0) / (1 + 0.999 + 0.998001)
    np.testing.assert_allclose(last, [-lr * mh / (np.sqrt(vh) + eps)], rtol=1e-12)


def test_adam_first_step_and_constant_gradient():
    rng = np.random.default_rng(10)
    g = rng.standard_normal(100)
    p = rng.standard_normal(100)
    p1, m, v = adam_step(p, g, np.zeros(100), np.zeros(100), 1, lr=1e-3)
    np.testing.assert_allclose(p1 - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    q, mm, vv = p1, m, v
    for t in range(2, 30):
        q2, mm, vv = adam_step(q, g, mm, vv, t, lr=1e-3)
        np.testing.assert_allclose(q2 - q, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        q = q2
    p0, _, _ = adam_step(p, np.zeros(100), np.zeros(100), np.zeros(100), 1)
    np.testing.assert_array_equal(p0, p)

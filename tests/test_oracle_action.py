"""Pins for oracle.action: closed forms, an independent site-loop rewriting, FD force, free field."""
import itertools

import numpy as np
import pytest

from oracle.action import action, force, laplacian


def action_by_links(phi, m2, lam, dim):
    """Independent rewriting with explicit site loops: sum over links of squared differences."""
    phi = np.asarray(phi, dtype=np.float64)
    L = phi.shape[1]
    out = np.zeros(phi.shape[0])
    for b in range(phi.shape[0]):
        s = 0.0
        for n in itertools.product(range(L), repeat=dim):
            v = phi[(b,) + n]
            s += m2 * v * v + lam * v ** 4
            for mu in range(dim):
                nb = list(n)
                nb[mu] = (nb[mu] + 1) % L
                s += (phi[(b,) + tuple(nb)] - v) ** 2
        out[b] = s
    return out


def lattice_laplacian_matrix(L, dim):
    V = L ** dim
    A = np.zeros((V, V))
    idx = lambda n: int(np.ravel_multi_index(n, (L,) * dim))
    for n in itertools.product(range(L), repeat=dim):
        i = idx(n)
        A[i, i] -= 2 * dim
        for mu in range(dim):
            for s in (1, -1):
                nb = list(n)
                nb[mu] = (nb[mu] + s) % L
                A[i, idx(nb)] += 1
    return A


@pytest.mark.parametrize("dim,m2,lam,c,per_site", [(2, -4.0, 8.0, 0.5, -0.5), (2, -4.0, 8.0, -0.5, -0.5),
                                                    (3, -4.0, 5.0, np.sqrt(0.4), -0.8)])
def test_constant_field(dim, m2, lam, c, per_site):
    L = 4
    phi = np.full((1,) + (L,) * dim, c)
    np.testing.assert_allclose(action(phi, m2, lam, dim), [per_site * L ** dim], rtol=1e-13)


@pytest.mark.parametrize("shape", [(2, 2), (2, 2, 2), (4, 4), (3, 5)[:0] or (8, 8), (4, 4, 4)])
def test_link_rewriting(shape):
    dim = len(shape)
    rng = np.random.default_rng(3)
    phi = rng.standard_normal((3,) + shape)
    np.testing.assert_allclose(action(phi, -1.3, 2.1, dim), action_by_links(phi, -1.3, 2.1, dim), rtol=1e-12)


@pytest.mark.parametrize("L,dim", [(2, 2), (4, 2), (2, 3), (4, 3)])
def test_quadratic_form_matrix(L, dim):
    """lambda = 0: S = phi^T (-Lap + m2) phi with the explicit periodic Laplacian matrix."""
    rng = np.random.default_rng(4)
    phi = rng.standard_normal((2,) + (L,) * dim)
    M = -lattice_laplacian_matrix(L, dim) + 0.7 * np.eye(L ** dim)
    f = phi.reshape(2, -1)
    np.testing.assert_allclose(action(phi, 0.7, 0.0, dim), np.einsum("bi,ij,bj->b", f, M, f), rtol=1e-12)
    np.testing.assert_allclose(laplacian(phi, dim).reshape(2, -1), f @ lattice_laplacian_matrix(L, dim).T,
                               atol=1e-12)


@pytest.mark.parametrize("shape", [(2, 2), (4, 4), (2, 2, 2), (4, 4, 4)])
def test_force_central_fd(shape):
    dim = len(shape)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((2,) + shape)
    m2 = np.array([-4.0, 1.5])
    lam = np.array([8.0, 0.3])
    F = force(phi, m2, lam, dim)
    h = 1e-6
    fd = np.zeros_like(phi)
    for n in itertools.product(*[range(s) for s in shape]):
        for b in range(2):
            p, q = phi.copy(), phi.copy()
            p[(b,) + n] += h
            q[(b,) + n] -= h
            fd[(b,) + n] = (action(p, m2, lam, dim)[b] - action(q, m2, lam, dim)[b]) / (2 * h)
    np.testing.assert_allclose(F, fd, rtol=1e-7, atol=1e-6)


def test_free_field_closed_forms():
    """d=2, L=4, m2=1, lambda=0: <phi^2> and ln Z from the momentum-space sum equal the matrix forms."""
    L, dim, m2 = 4, 2, 1.0
    k = 2 * np.pi * np.arange(L) / L
    ks = np.array(list(itertools.product(k, repeat=dim)))
    ev = m2 + np.sum(4 * np.sin(ks / 2) ** 2, axis=1)
    phi2 = np.mean(1 / (2 * ev))
    lnZ = 0.5 * L ** dim * np.log(np.pi) - 0.5 * np.sum(np.log(ev))
    M = -lattice_laplacian_matrix(L, dim) + m2 * np.eye(L ** dim)
    np.testing.assert_allclose(phi2, np.trace(np.linalg.inv(2 * M)) / L ** dim, rtol=1e-12)
    np.testing.assert_allclose(lnZ, 0.5 * L ** dim * np.log(np.pi) - 0.5 * np.linalg.slogdet(M)[1], rtol=1e-12)
    np.testing.assert_allclose(phi2, 0.1317460317, atol=1e-10)
    np.testing.assert_allclose(lnZ, -2.8581318146, atol=1e-9)

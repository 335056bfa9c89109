"""Statistical checks of the GPU HMC kernel on the free field (lambda = 0), whose
law exp(-phi^T M phi), M = -Lap + m^2, is known exactly:

* <phi^2> = (1/V) sum_p 1 / (2 (m^2 + phat^2)), phat^2 = sum_mu 4 sin^2(p_mu / 2),
  the momentum-space sum, against an HMC estimate within five standard errors of
  the chain means;
* the Creutz identity <exp(-dH)> = 1 for trajectories started from exact draws
  of the law (a dropped term in the force or the energy breaks it).

Seeded; the fixtures (momenta, uniforms, exact draws) are drawn on the host."""
import itertools

import numpy as np
import pytest
import torch

import seeded_inputs as si
from paper_2208_08903_amd import lfs

from .gpu_util import dev, host

pytestmark = pytest.mark.gpu


def exact_phi2(L, dim, m2):
    ks = 2 * np.pi * np.arange(L) / L
    tot = 0.0
    for p in itertools.product(ks, repeat=dim):
        tot += 1.0 / (2.0 * (m2 + sum(4 * np.sin(q / 2) ** 2 for q in p)))
    return tot / L ** dim


def exact_draws(rng, L, dim, m2, n):
    """Draws with covariance (2M)^-1 from the explicit lattice matrix."""
    V = L ** dim
    A = np.zeros((V, V))
    for c in itertools.product(range(L), repeat=dim):
        i = int(np.ravel_multi_index(c, (L,) * dim))
        A[i, i] += 2 * dim + m2
        for mu in range(dim):
            for s in (1, -1):
                nb = list(c)
                nb[mu] = (nb[mu] + s) % L
                A[i, int(np.ravel_multi_index(nb, (L,) * dim))] -= 1
    chol = np.linalg.cholesky(np.linalg.inv(2 * A))
    return rng.standard_normal((n, V)) @ chol.T


@pytest.mark.parametrize("dim,L,m2", [(2, 4, 1.0), (3, 4, 0.5)])
def test_hmc_free_field_phi2(dim, L, m2):
    print(f"HMC free field dim={dim} L={L} m2={m2}", flush=True)
    V, chains, n_traj, therm = L ** dim, 1024, 300, 60
    phi = torch.zeros(chains, V, dtype=torch.float64, device="cuda")
    m2t = torch.tensor([m2], dtype=torch.float64, device="cuda")
    lam = torch.zeros(1, dtype=torch.float64, device="cuda")
    dH = torch.empty(chains, dtype=torch.float64, device="cuda")
    acc = torch.empty(chains, dtype=torch.uint8, device="cuda")
    lu = dev(si.log_uniforms(11, (n_traj, chains)), torch.float64)
    sums = torch.zeros(chains, dtype=torch.float64, device="cuda")
    n_acc = 0
    for k in range(n_traj):
        pi = dev(si.momenta(1000 + k, chains, V), torch.float64)
        lfs.hmc_step(dim, L, phi, pi, lu[k], m2t, lam, 10, 0.05, dH, acc)
        if k >= therm:
            sums += (phi * phi).mean(dim=1)
            n_acc += int(acc.sum().item())
    torch.cuda.synchronize()
    per_chain = host(sums) / (n_traj - therm)
    est, se = per_chain.mean(), per_chain.std(ddof=1) / np.sqrt(chains)
    exact = exact_phi2(L, dim, m2)
    assert abs(est - exact) < 5 * se, (est, exact, se)
    assert n_acc / (chains * (n_traj - therm)) > 0.9


def test_hmc_creutz_identity():
    print("HMC Creutz identity", flush=True)
    dim, L, m2, n = 2, 4, 1.0, 8192
    rng = np.random.default_rng(12)
    phi = dev(exact_draws(rng, L, dim, m2, n), torch.float64)
    pi = dev(si.momenta(13, n, L ** dim), torch.float64)
    dH = torch.empty(n, dtype=torch.float64, device="cuda")
    acc = torch.empty(n, dtype=torch.uint8, device="cuda")
    lu = torch.full((n,), -np.inf, dtype=torch.float64, device="cuda")
    lfs.hmc_step(dim, L, phi, pi, lu, torch.tensor([m2], dtype=torch.float64, device="cuda"),
                 torch.zeros(1, dtype=torch.float64, device="cuda"), 10, 0.1, dH, acc)
    torch.cuda.synchronize()
    e = np.exp(-host(dH))
    assert abs(e.mean() - 1.0) < 5 * e.std() / np.sqrt(n), (e.mean(), e.std())
    assert np.all(host(acc) == 1)

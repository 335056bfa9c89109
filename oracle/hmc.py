"""HMC baseline for the same phi^4 theory, FP64.

Paper, Sec. 2.2: HMC for the 2D/3D scalar theory is provided "to compare
results"; no details are given.  Reading: Hamiltonian H = 1/2 sum pi^2 + S(phi),
momenta pi ~ N(0,1) per site (drawn on the host and passed in), leapfrog in
kick-drift-kick form with n_steps steps of size dt (10 steps of 0.1 in the
workloads), and accept iff log u < -(H_new - H_old); on rejection the field is
restored.

Pinned by: reversibility (flip the momenta and integrate back), unit Jacobian of
the leapfrog map (finite differences at L = 2), dt^2 scaling of the energy error,
the Creutz identity <exp(-dH)> = 1 and the free-field <phi^2>.
"""
from __future__ import annotations

import numpy as np

from .action import action, force


def leapfrog(phi, pi, m2, lam, dim: int, n_steps: int, dt: float):
    phi = np.array(phi, dtype=np.float64)
    pi = np.array(pi, dtype=np.float64)
    for _ in range(n_steps):
        pi = pi - 0.5 * dt * force(phi, m2, lam, dim)
        phi = phi + dt * pi
        pi = pi - 0.5 * dt * force(phi, m2, lam, dim)
    return phi, pi


def hamiltonian(phi, pi, m2, lam, dim: int):
    pi = np.asarray(pi, dtype=np.float64)
    ax = tuple(range(1, pi.ndim))
    return 0.5 * np.sum(pi * pi, axis=ax) + action(phi, m2, lam, dim)


def hmc_step(phi, pi0, log_u, m2, lam, dim: int, n_steps: int = 10, dt: float = 0.1):
    """One trajectory per sample.  phi, pi0: [B, *lattice].  Returns (phi_out, dH, accepted)."""
    phi = np.asarray(phi, dtype=np.float64)
    pi0 = np.asarray(pi0, dtype=np.float64).reshape(phi.shape)
    H0 = hamiltonian(phi, pi0, m2, lam, dim)
    phi1, pi1 = leapfrog(phi, pi0, m2, lam, dim, n_steps, dt)
    H1 = hamiltonian(phi1, pi1, m2, lam, dim)
    dH = H1 - H0
    acc = np.asarray(log_u, dtype=np.float64) < -dH
    shp = (-1,) + (1,) * dim
    out = np.where(acc.reshape(shp), phi1, phi)
    return out, dH, acc.astype(np.uint8)

"""Lattice phi^4 action and force, FP64.

Paper, Sec. 1, action, Laplacian and potential equations:

    S[phi] = - sum_n phi(n) d^2 phi(n) + sum_n V[phi](n),
    d^2 phi(n) = sum_mu [phi(n + mu) + phi(n - mu) - 2 phi(n)],
    V[phi](n) = m^2 phi(n)^2 + lambda phi(n)^4.

Readings: the kinetic term's site index is garbled in the paper; it is read as
phi(n) d^2 phi(n) summed over n.  The normalisation is taken literally (no 1/2,
no 1/4!).  The lattice is periodic in every direction.  At L = 2 the two
neighbours along an axis are the same site and both terms are kept.

Force (derivative of the quadratic form, which is symmetric):
    dS/dphi(n) = -2 d^2 phi(n) + 2 m^2 phi(n) + 4 lambda phi(n)^3.

Pinned by: the constant-field closed form, the difference-squared rewriting of
the kinetic term, central finite differences of S, and free-field Gaussian
integrals (lambda = 0).
"""
from __future__ import annotations

import numpy as np


def laplacian(phi, dim: int):
    """Periodic lattice Laplacian on the trailing `dim` axes."""
    phi = np.asarray(phi, dtype=np.float64)
    out = -2.0 * dim * phi
    for mu in range(dim):
        ax = phi.ndim - dim + mu
        out = out + np.roll(phi, -1, axis=ax) + np.roll(phi, 1, axis=ax)
    return out


def action(phi, m2, lam, dim: int) -> np.ndarray:
    """S per sample for phi of shape [B, L, ..., L] (dim lattice axes).  m2, lam: scalars or [B]."""
    phi = np.asarray(phi, dtype=np.float64)
    B = phi.shape[0]
    m2 = np.broadcast_to(np.asarray(m2, dtype=np.float64), (B,))
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (B,))
    ax = tuple(range(1, phi.ndim))
    kinetic = -np.sum(phi * laplacian(phi, dim), axis=ax)
    shp = (B,) + (1,) * dim
    pot = np.sum(m2.reshape(shp) * phi ** 2 + lam.reshape(shp) * phi ** 4, axis=ax)
    return kinetic + pot


def force(phi, m2, lam, dim: int) -> np.ndarray:
    """dS/dphi, same shape as phi."""
    phi = np.asarray(phi, dtype=np.float64)
    B = phi.shape[0]
    shp = (B,) + (1,) * dim
    m2 = np.broadcast_to(np.asarray(m2, dtype=np.float64), (B,)).reshape(shp)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (B,)).reshape(shp)
    return -2.0 * laplacian(phi, dim) + 2.0 * m2 * phi + 4.0 * lam * phi ** 3

"""Chain-quality analysis, FP64: observables, autocorrelation time, reweighting ESS.

TEST INFRASTRUCTURE ONLY (see the package header).

Paper, Sec. 1: a Monte Carlo average over N_conf configurations carries a
statistical error of order 1/sqrt(N_indep), with N_indep = N_conf / (2 tau_ac)
and tau_ac the autocorrelation time (after Luscher 2004); the point of the flow
sampler is a shorter tau_ac.  Sec. 2.2 and the conclusions name the analysis
quantities -- the condensate, zero-momentum two-point functions, the
autocorrelation time and the effective sample size (ESS) -- without formulas.
The readings used here (each a standard definition, named):

  condensate, per configuration:  M[phi] = (1/V) sum_n phi_n.

  zero-momentum two-point function, per configuration, with time along the
  first lattice axis: Phi(t) = sum of phi over the sites whose first
  coordinate is t, and
      C(t) = (1/V) sum_{t0} Phi(t0) Phi((t0 + t) mod L),   t = 0 .. L-1,
  i.e. the sum over spatial separations of (1/V) sum_y phi(y) phi(y + x) at
  time separation t.  Ensemble averages (and the connected part, which
  subtracts L^(d-1) <M>^2) are taken over configurations afterwards.

  autocorrelation of a series x_1 .. x_n (the standard windowed estimator):
      xbar = (1/n) sum_i x_i
      Gamma(t) = (1/(n - t)) sum_{i=1}^{n-t} (x_i - xbar)(x_{i+t} - xbar),
      rho(t) = Gamma(t) / Gamma(0),
      tau_int(W) = 1/2 + sum_{t=1}^{W} rho(t),
  with the automatic window of Madras and Sokal: W is the smallest W >= 1
  (W <= W_max, lags beyond n - 1 are not formed) with W >= c tau_int(W);
  if none qualifies W = W_max (or n - 1) and the window is reported as not
  found.  tau_ac = tau_int(W) and N_indep = n / (2 tau_ac).  A series with
  Gamma(0) = 0 (constant, or n = 1) has no defined tau: NaN, W = 0,
  N_indep = 0.

  reweighting ESS, normalised: for log-weights w_k = log p - log q (up to a
  constant), ESS = (sum_k e^{w_k})^2 / (N sum_k e^{2 w_k}), in [1/N, 1];
  evaluated with w_k - max_k w_k.

Pinned by tests/test_oracle_analysis.py: exact autocovariances of an
alternating series and of a linear ramp (rational arithmetic), Gamma(0) against
the textbook variance
with the n-1 .. n normalisation spelled out, the AR(1) process whose tau_int is
(1 + a) / (2 (1 - a)) within the estimator's statistical error, white noise,
a hand-built rho sequence whose window is known, the ESS of equal, one-hot and
two-valued weights, constant and plane-wave fields whose M and C(t) have
closed forms, and C(t) against a brute-force double sum over all site pairs.
"""
from __future__ import annotations

import numpy as np


def condensate(phi, dim: int, L: int):
    """M[phi] = (1/V) sum_n phi_n for each configuration of phi [B, V]."""
    phi = np.asarray(phi, dtype=np.float64).reshape(-1, L ** dim)
    return phi.sum(axis=1) / L ** dim


def slice_sums(phi, dim: int, L: int):
    """Phi(t): sums of phi over the sites with first coordinate t, [B, L]."""
    phi = np.asarray(phi, dtype=np.float64).reshape(-1, L, L ** (dim - 1))
    return phi.sum(axis=2)


def two_point_zero_momentum(phi, dim: int, L: int):
    """C(t) = (1/V) sum_{t0} Phi(t0) Phi((t0 + t) mod L) per configuration, [B, L]."""
    P = slice_sums(phi, dim, L)
    V = L ** dim
    out = np.zeros_like(P)
    for t in range(L):
        out[:, t] = np.sum(P * np.roll(P, -t, axis=1), axis=1) / V
    return out


def autocovariance(x, w_max: int):
    """Gamma(t) for t = 0 .. min(w_max, n - 1), the 1/(n - t) estimator."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    d = x - x.mean()
    T = min(w_max, n - 1)
    return np.array([np.dot(d[: n - t], d[t:]) / (n - t) for t in range(T + 1)])


def window(g, c: float, n: int):
    """Madras-Sokal window on autocovariances g = Gamma(0 .. T): (tau_ac, W, found, N_indep)."""
    g = np.asarray(g, dtype=np.float64)
    if g[0] == 0.0:
        return float("nan"), 0, False, 0.0
    tau = 0.5
    T = g.shape[0] - 1
    for W in range(1, T + 1):
        tau += g[W] / g[0]
        if W >= c * tau:
            return tau, W, True, n / (2.0 * tau)
    return tau, T, False, n / (2.0 * tau)


def tau_int(x, w_max: int, c: float):
    """(tau_ac, W, found, N_indep, Gamma) of the series x with the automatic window."""
    x = np.asarray(x, dtype=np.float64)
    g = autocovariance(x, w_max)
    return (*window(g, c, x.shape[0]), g)


def ess(logw):
    """Normalised reweighting ESS (sum e^w)^2 / (N sum e^{2w}) of log-weights [N]."""
    w = np.asarray(logw, dtype=np.float64)
    e = np.exp(w - w.max())
    return float(e.sum() ** 2 / (w.shape[0] * np.sum(e * e)))

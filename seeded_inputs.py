"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers and lays them out.  It holds none of the
method's arithmetic (no action, no coupling layer, no acceptance test), so the
oracle and the GPU path can both take their inputs from here without sharing any
computation.

Packed flow-parameter layout (a data contract, fixed here and restated
independently by the oracle and by the C library).  For every coupling layer, in
order, with C hidden channels and T = 3**dim stencil taps:

    W1[C][1][T]  b1[C]  W2[C][C][T]  b2[C]  W3[2][C][T]  b3[2]

Taps are row-major over the offset delta in {-1,0,1}**dim, axis 0 slowest.
Channel 0 of the last convolution is s, channel 1 is t.  With batch norm every
hidden convolution's bias is followed by its gamma[cout] and beta[cout]; the
normalisation statistics are a separate vector, per layer and hidden
convolution mean[cout] then var[cout].

The default initialisation follows the paper's example parameter file (model
seed 2021) with the weight law N(0, 0.1) read as standard deviation 0.1 and the
biases set to zero.  Tests use non-zero biases so that every bias path is
exercised.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def taps_per_conv(dim: int, kernel: int = 3) -> int:
    return kernel ** dim


def layer_block_sizes(dim: int, hidden: int, kernel: int = 3,
                      hidden_sizes=None, batch_norm: bool = False) -> list[tuple[str, int]]:
    """(name, size) of a layer's blocks: W_i[cout][cin][T], b_i[cout] for every
    convolution (then gamma_i[cout], beta_i[cout] for a hidden one with batch
    norm), with hidden widths hidden_sizes (default [hidden, hidden])."""
    T = taps_per_conv(dim, kernel)
    w = list(hidden_sizes) if hidden_sizes else [hidden, hidden]
    cin, cout = [1] + w, w + [2]
    out = []
    for i, (ci, co) in enumerate(zip(cin, cout), start=1):
        out += [(f"W{i}", co * ci * T), (f"b{i}", co)]
        if batch_norm and i <= len(w):
            out += [(f"gamma{i}", co), (f"beta{i}", co)]
    return out


def param_count(dim: int, n_layers: int, hidden: int, kernel: int = 3, hidden_sizes=None,
                batch_norm: bool = False) -> int:
    return n_layers * sum(n for _, n in layer_block_sizes(dim, hidden, kernel, hidden_sizes, batch_norm))


def flow_params(dim: int, n_layers: int, hidden: int, seed: int = 2021,
                w_std: float = 0.1, b_std: float = 0.0, kernel: int = 3,
                hidden_sizes=None, batch_norm: bool = False, gamma_std: float = 0.0) -> np.ndarray:
    """Packed FP32 flow parameters: weights N(0, w_std), biases and batch-norm betas
    N(0, b_std) (0 if b_std == 0), batch-norm gammas 1 + N(0, gamma_std)."""
    n = param_count(dim, n_layers, hidden, kernel, hidden_sizes, batch_norm)
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, w_std, size=n)
    brng = np.random.default_rng(seed + 7919)
    grng = np.random.default_rng(seed + 104729)
    off = 0
    for _ in range(n_layers):
        for name, sz in layer_block_sizes(dim, hidden, kernel, hidden_sizes, batch_norm):
            if name.startswith("gamma"):
                p[off:off + sz] = 1.0 + (grng.normal(0.0, gamma_std, size=sz) if gamma_std > 0 else 0.0)
            elif name.startswith("b"):
                p[off:off + sz] = brng.normal(0.0, b_std, size=sz) if b_std > 0 else 0.0
            off += sz
    return p.astype(np.float32)


def bn_stats(seed: int, n_layers: int, widths, mean_std: float = 0.3, var_range=(0.5, 2.0)) -> np.ndarray:
    """FP32 running statistics, per layer and hidden convolution of width w:
    mean[w] ~ N(0, mean_std) then var[w] ~ U(var_range)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_layers):
        for w in widths:
            out += [rng.normal(0.0, mean_std, size=w), rng.uniform(*var_range, size=w)]
    return np.concatenate(out).astype(np.float32)


def normal_fields(seed: int, B: int, V: int) -> np.ndarray:
    """FP32 N(0,1) fields [B, V] drawn on the host (used where the prior draw is not under test)."""
    return np.random.default_rng(seed).standard_normal((B, V)).astype(np.float32)


def log_uniforms(seed: int, shape) -> np.ndarray:
    """FP64 log u with u ~ U(0,1), for accept/reject decisions."""
    u = np.random.default_rng(seed).random(shape)
    u = np.where(u == 0.0, np.nextafter(0.0, 1.0), u)
    return np.log(u)


def momenta(seed: int, B: int, V: int) -> np.ndarray:
    """FP64 N(0,1) conjugate momenta [B, V] for the HMC baseline."""
    return np.random.default_rng(seed).standard_normal((B, V))


def couplings(seed: int, B: int, m2_range=(-4.5, -3.5), lam_range=(4.0, 9.0)):
    """Per-sample (m^2, lambda) pairs, FP64, uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(*m2_range, size=B), rng.uniform(*lam_range, size=B))


def logw_stream(seed: int, n: int, scale: float = 1.0) -> np.ndarray:
    """Synthetic FP64 log-weights for chain tests that do not involve a flow."""
    return scale * np.random.default_rng(seed).standard_normal(n)


def correlated_series(seed: int, n_series: int, n: int, a: float) -> np.ndarray:
    """FP64 [n_series, n] stationary AR(1) series x_k = a x_{k-1} + sqrt(1 - a^2) e_k,
    inputs with a known autocorrelation for the analysis tests."""
    e = np.random.default_rng(seed).standard_normal((n_series, n))
    x = np.empty_like(e)
    x[:, 0] = e[:, 0]
    s = math.sqrt(1.0 - a * a)
    for k in range(1, n):
        x[:, k] = a * x[:, k - 1] + s * e[:, k]
    return x


# ---------------------------------------------------------------------------
# Serving workload: Poisson arrivals of sampling requests.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Request:
    rid: int
    t_arrive: float      # seconds after the start of the run
    dim: int
    L: int
    m2: float
    lam: float
    n_samples: int
    seed: int            # per-request stream for prior draws and log u


L_CHOICES = {2: (8, 16, 32), 3: (8, 12, 16)}


def serving_requests(seed: int = 2208, rate: float = 200.0, duration: float = 60.0,
                     n_min: int = 64, n_max: int = 8192, max_requests: int | None = None):
    """Poisson(rate) arrivals over `duration` seconds; each request's shape and couplings
    are drawn from the same seeded stream: dim uniform in {2,3}, L uniform over the
    dim's set, m^2 ~ U[-4.5,-3.5], lambda ~ U[4,9], N log-uniform on [n_min, n_max]."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        dim = int(rng.integers(2, 4))
        L = int(rng.choice(L_CHOICES[dim]))
        m2 = float(rng.uniform(-4.5, -3.5))
        lam = float(rng.uniform(4.0, 9.0))
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        out.append(Request(rid, t, dim, L, m2, lam, n, int(rng.integers(0, 2**31 - 1))))
        rid += 1
        if max_requests is not None and rid >= max_requests:
            break
    return out

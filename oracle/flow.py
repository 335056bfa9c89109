"""RealNVP flow with checkerboard affine coupling layers, FP64.

Paper, Sec. 1: the untrivializing map phi = F^{-1}(z) is a composition of affine
coupling layers on the even/odd (checkerboard) decomposition of the lattice.  A
layer leaves one sublattice unchanged and updates the other one by a scale and a
shift, s and t, that a convolutional network computes from the unchanged
sublattice (coupling-layer equation); the Jacobian of a layer is triangular, so
its log-determinant is the sum of s over the updated sites (Sec. 1, the O(N)
Jacobian remark).  The model density is the prior density pushed through the map
(Sec. 1, P^(ML) equation), and training minimises the shifted reverse
Kullback-Leibler divergence E_q[ln q - ln p] - ln Z = E_q[ln q + S].

Readings of the paper used here (every one is listed with its reason in the
design notes):
  * Direction: a layer in the sampling direction is x_A <- x_A exp(s) + t on the
    active sites A; its log|det| is +sum_A s.  (The paper writes the layer in the
    trivializing direction; an affine coupling's inverse is again affine, so the
    family is the same.)
  * Density: log q(phi) = log r(z) - log|det dF^{-1}/dz| (change of variables;
    the paper's P^(ML) equation places the Jacobian on the other side).
  * Masks: site parity p(n) = (sum_mu n_mu) mod 2 with 0-based coordinates;
    layer l freezes the sites with p(n) = (l + parity0) mod 2; strict
    alternation.
  * Network: input is the full lattice as one channel with active sites zeroed;
    conv(1->C) + LeakyReLU(0.01), conv(C->C) + LeakyReLU(0.01), conv(C->2);
    channel 0 is s (tanh applied when final_tanh), channel 1 is t; kernel 3 per
    axis, periodic padding, cross-correlation with bias; s and t are read at the
    active sites only.  LeakyReLU'(0) is taken as 1.  The example parameter
    file's hidden_sizes and kernel_size generalise this: one conv + LeakyReLU
    per entry of hidden_sizes (default [C, C]), then conv(->2), all with an odd
    kernel K (default 3) per axis, offsets -K//2 .. K//2.
  * Loss: the batch mean of log q + S with z held fixed (path-wise gradient).

Parameter layout (shared data contract): per layer W1[C][1][T], b1[C],
W2[C][C][T], b2[C], W3[2][C][T], b3[2]; taps row-major over delta in
{-1,0,1}^dim, axis 0 slowest.  A general network stores, per layer and per
convolution i in order, W_i[cout_i][cin_i][T] then b_i[cout_i], with T = K^dim
and taps row-major over {-K//2..K//2}^dim.

Emulated storage precision (emulate = "fp32" or "bf16"; None is plain FP64):
every convolution's operands -- the input tensor and the weights, in the
forward and in the adjoint -- are rounded to that precision, the field (and its
gradient) is rounded to FP32 after each layer, and the weight and bias
gradients are accumulated in FP32; the convolutions' own sums, biases, tanh,
exp, s, t and log-det stay FP64.  Used only to size the parity tolerances of
implementations that store and accumulate so.

Pinned by: identity and pure-shift flows, a uniform-scale flow whose q is a known
Gaussian (importance-sampling estimate of a free-field ln Z), invertibility,
brute-force Jacobian determinants on L <= 4, one-hot convolution orientation,
hand-computed single-layer values, and central finite differences of the loss
for the adjoint gradient; for general networks (tests/test_oracle_flow_variants.py)
the layout, tap order and one-hot orientation for kernels 1, 5 and 7, conv
adjoints, invertibility, brute-force Jacobians, a hand-computed pointwise layer,
central finite differences of the loss, and bit-identity of the explicit
(C, C), kernel-3 network with the default one.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .action import action as _action, force as _force
from .prior import log_prior
from .rounding import ROUNDERS, to_fp32

LEAKY_SLOPE = 0.01


@dataclass(frozen=True)
class FlowShape:
    dim: int
    L: int
    n_layers: int
    hidden: int
    final_tanh: bool = True
    parity0: int = 0
    kernel: int = 3
    hidden_sizes: tuple = ()   # empty: (hidden, hidden)

    @property
    def V(self) -> int:
        return self.L ** self.dim

    @property
    def T(self) -> int:
        return self.kernel ** self.dim

    @property
    def widths(self) -> tuple:
        return tuple(self.hidden_sizes) if self.hidden_sizes else (self.hidden, self.hidden)

    @property
    def conv_shapes(self) -> list:
        """(cout, cin) of every convolution of a layer's network, in order."""
        w = self.widths
        return list(zip(w + (2,), (1,) + w))

    @property
    def lattice(self) -> tuple:
        return (self.L,) * self.dim


def tap_offsets(dim: int, kernel: int = 3):
    """Offsets delta in {-K//2..K//2}^dim, row-major (axis 0 slowest)."""
    r = kernel // 2
    return list(itertools.product(range(-r, r + 1), repeat=dim))


def _kernel_of(T: int, dim: int) -> int:
    K = int(round(T ** (1.0 / dim)))
    if K ** dim != T:
        raise ValueError(f"{T} taps is not a cube of an odd kernel in {dim} dimensions")
    return K


def unpack(params, fs: FlowShape):
    """Split the packed parameter vector into per-layer (W1, b1, ..., Wn, bn) in FP64
    (n = number of convolutions; (W1, b1, W2, b2, W3, b3) for the default network)."""
    p = np.asarray(params, dtype=np.float64).ravel()
    T = fs.T
    layers, off = [], 0

    def take(n, shape):
        nonlocal off
        a = p[off:off + n].reshape(shape)
        off += n
        return a

    for _ in range(fs.n_layers):
        lay = []
        for co, ci in fs.conv_shapes:
            lay.append(take(co * ci * T, (co, ci, T)))
            lay.append(take(co, (co,)))
        layers.append(tuple(lay))
    if off != p.size:
        raise ValueError(f"parameter vector has {p.size} entries, layout needs {off}")
    return layers


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([a.ravel() for a in lay]) for lay in layers])


def shifted(u, delta, dim: int):
    """v with v[..., n] = u[..., (n + delta) mod L] over the trailing dim axes."""
    axes = tuple(range(u.ndim - dim, u.ndim))
    return np.roll(u, shift=tuple(-d for d in delta), axis=axes)


def conv(u, W, b, dim: int):
    """Periodic cross-correlation with bias.

    u: [B, Cin, *lattice], W: [Cout, Cin, T], b: [Cout]
    out[b, co, n] = b[co] + sum_ci sum_t W[co, ci, t] u[b, ci, n + delta_t]
    """
    out = np.broadcast_to(b.reshape((1, -1) + (1,) * dim),
                          (u.shape[0], W.shape[0]) + u.shape[2:]).copy()
    for t, d in enumerate(tap_offsets(dim, _kernel_of(W.shape[2], dim))):
        out += np.einsum("oi,bi...->bo...", W[:, :, t], shifted(u, d, dim))
    return out


def conv_transpose(g, W, dim: int):
    """Adjoint of `conv` w.r.t. its input: g_u[b, ci, m] = sum_co sum_t W[co,ci,t] g[b, co, m - delta_t]."""
    out = np.zeros((g.shape[0], W.shape[1]) + g.shape[2:])
    for t, d in enumerate(tap_offsets(dim, _kernel_of(W.shape[2], dim))):
        out += np.einsum("oi,bo...->bi...", W[:, :, t], shifted(g, tuple(-x for x in d), dim))
    return out


def conv_weight_grad(g, u, dim: int, kernel: int = 3):
    """dW[co, ci, t] = sum_b sum_n g[b, co, n] u[b, ci, n + delta_t]; db[co] = sum g."""
    T = kernel ** dim
    dW = np.zeros((g.shape[1], u.shape[1], T))
    for t, d in enumerate(tap_offsets(dim, kernel)):
        us = shifted(u, d, dim)
        dW[:, :, t] = np.einsum("bon,bin->oi", g.reshape(g.shape[0], g.shape[1], -1),
                                us.reshape(us.shape[0], us.shape[1], -1))
    db = g.sum(axis=tuple(i for i in range(g.ndim) if i != 1))
    return dW, db


def leaky(a):
    return np.where(a >= 0, a, LEAKY_SLOPE * a)


def leaky_grad(a):
    return np.where(a >= 0, 1.0, LEAKY_SLOPE)


def parity(fs: FlowShape) -> np.ndarray:
    """p(n) = (sum_mu n_mu) mod 2 on the lattice, 0-based coordinates."""
    grids = np.meshgrid(*[np.arange(fs.L)] * fs.dim, indexing="ij")
    return (sum(grids) % 2).astype(np.int64)


def frozen_mask(fs: FlowShape, layer: int) -> np.ndarray:
    return (parity(fs) == (layer + fs.parity0) % 2).astype(np.float64)


def _identity(a):
    return a


def _rounders(emulate):
    """(operand rounding, field rounding) for an emulated storage precision."""
    if emulate is None:
        return _identity, _identity
    return ROUNDERS[emulate], to_fp32


def net(x, lay, mF, fs: FlowShape, emulate=None):
    """s/t network of one layer.  Returns (acts, hs, o, s, t): the hidden
    pre-activations a_1 .. a_n, the inputs h_0 = mask_F x, h_i = leaky(a_i) of
    every convolution, the output o and s, t."""
    R, _ = _rounders(emulate)
    h = (x * mF)[:, None]
    acts, hs = [], [h]
    nconv = len(lay) // 2
    for i in range(nconv - 1):
        a = conv(R(h), R(lay[2 * i]), lay[2 * i + 1], fs.dim)
        h = leaky(a)
        acts.append(a)
        hs.append(h)
    o = conv(R(h), R(lay[-2]), lay[-1], fs.dim)
    s = np.tanh(o[:, 0]) if fs.final_tanh else o[:, 0]
    t = o[:, 1]
    return acts, hs, o, s, t


def coupling_forward(x, lay, layer: int, fs: FlowShape, emulate=None):
    """One layer in the sampling direction.  Returns (y, sum_A s per sample)."""
    mF = frozen_mask(fs, layer)
    mA = 1.0 - mF
    *_, s, t = net(x, lay, mF, fs, emulate)
    y = _rounders(emulate)[1](np.where(mA > 0, x * np.exp(s) + t, x))
    ax = tuple(range(1, x.ndim))
    return y, np.sum(mA * s, axis=ax)


def coupling_inverse(y, lay, layer: int, fs: FlowShape):
    """Inverse of `coupling_forward`: s, t depend only on the frozen sites, which are unchanged."""
    mF = frozen_mask(fs, layer)
    mA = 1.0 - mF
    *_, s, t = net(y, lay, mF, fs)
    x = np.where(mA > 0, (y - t) * np.exp(-s), y)
    ax = tuple(range(1, y.ndim))
    return x, np.sum(mA * s, axis=ax)


def as_lattice(z, fs: FlowShape):
    z = np.asarray(z, dtype=np.float64)
    return z.reshape((z.shape[0],) + fs.lattice)


def flow_forward(params, z, fs: FlowShape, return_saved: bool = False, emulate=None):
    """phi = F^{-1}(z) with log q.  Returns dict(phi, logdet, logr, logq[, saved])."""
    layers = unpack(params, fs)
    x = as_lattice(z, fs)
    logdet = np.zeros(x.shape[0])
    saved = [x]
    for l, lay in enumerate(layers):
        x, ld = coupling_forward(x, lay, l, fs, emulate)
        logdet = logdet + ld
        saved.append(x)
    logr = log_prior(z)
    out = dict(phi=x, logdet=logdet, logr=logr, logq=logr - logdet)
    if return_saved:
        out["saved"] = saved
    return out


def flow_inverse(params, phi, fs: FlowShape):
    """z = F(phi) and the log-determinant of F^{-1} at z (for tests)."""
    layers = unpack(params, fs)
    x = as_lattice(phi, fs)
    logdet = np.zeros(x.shape[0])
    for l in reversed(range(fs.n_layers)):
        x, ld = coupling_inverse(x, layers[l], l, fs)
        logdet = logdet + ld
    return x, logdet


def log_weights(S, logq):
    """log w = log p - log q up to ln Z: w = -S - log q (FP64)."""
    return -np.asarray(S, dtype=np.float64) - np.asarray(logq, dtype=np.float64)


def kl_loss(params, z, fs: FlowShape, m2, lam) -> float:
    """Shifted reverse KL, batch mean of log q + S, with z fixed."""
    f = flow_forward(params, z, fs)
    S = _action(f["phi"], m2, lam, fs.dim)
    return float(np.mean(f["logq"] + S))


def flow_vjp(params, z, fs: FlowShape, g_phi, g_logq, emulate=None):
    """Vector-Jacobian product of (phi, log q) = flow_forward(params, z) w.r.t. (params, z).

    g_phi: [B, *lattice] or [B, V]; g_logq: [B] or scalar.  Returns (g_params packed, g_z [B, V]).
    Hand-derived adjoint, layer by layer in reverse, recomputing each layer's network
    from the layer's input field.
    """
    layers = unpack(params, fs)
    R, RF = _rounders(emulate)
    f = flow_forward(params, z, fs, return_saved=True, emulate=emulate)
    saved = f["saved"]
    B = saved[0].shape[0]
    g_logq = np.broadcast_to(np.asarray(g_logq, dtype=np.float64), (B,))
    g_ld = -g_logq                                   # log q = log r - logdet
    shp = (B,) + (1,) * fs.dim
    gx = np.asarray(g_phi, dtype=np.float64).reshape((B,) + fs.lattice)
    grads = [None] * fs.n_layers
    for l in reversed(range(fs.n_layers)):
        lay = layers[l]
        x = saved[l]
        mF = frozen_mask(fs, l)
        mA = 1.0 - mF
        acts, hs, o, s, t = net(x, lay, mF, fs, emulate)
        es = np.exp(s)
        g_y = gx
        g_t = mA * g_y
        g_s = mA * (g_y * x * es + g_ld.reshape(shp))
        g_o0 = g_s * (1.0 - s * s) if fs.final_tanh else g_s
        # back through the convolutions, last to first: g is the gradient of the
        # current convolution's output (g_o, then g_a_i = g_h_i leaky'(a_i))
        g = np.stack([g_o0, g_t], axis=1)
        nconv = len(lay) // 2
        lay_grads = [None] * (2 * nconv)
        for i in reversed(range(nconv)):
            lay_grads[2 * i], lay_grads[2 * i + 1] = _weight_grad(g, hs[i], fs.dim, R, fs.kernel)
            g_in = conv_transpose(R(g), R(lay[2 * i]), fs.dim)
            g = g_in * leaky_grad(acts[i - 1]) if i > 0 else g_in
        g_h0 = g[:, 0]
        gx = RF(np.where(mA > 0, g_y * es, g_y + mF * g_h0))
        grads[l] = tuple(lay_grads)
    g_z = gx.reshape(B, -1) - g_logq[:, None] * saved[0].reshape(B, -1)   # d log r / dz = -z
    return pack(grads), g_z


def _weight_grad(g, u, dim: int, R, kernel: int = 3):
    """conv_weight_grad; when emulating a storage precision, the weight gradient
    from rounded operands and, like the bias gradient (a plain sum of the
    unrounded g), accumulated in FP32 by numpy's float32 reductions."""
    if R is _identity:
        return conv_weight_grad(g, u, dim, kernel)
    f32 = np.float32
    dW, _ = conv_weight_grad(R(g).astype(f32), R(u).astype(f32), dim, kernel)
    db = np.asarray(g, f32).sum(axis=tuple(i for i in range(g.ndim) if i != 1))
    return dW, db.astype(np.float64)


def loss_gradient(params, z, fs: FlowShape, m2, lam, emulate=None):
    """Gradient of the batch-mean reverse-KL loss w.r.t. the packed parameters, z fixed."""
    f = flow_forward(params, z, fs, emulate=emulate)
    B = f["phi"].shape[0]
    g_phi = _force(f["phi"], m2, lam, fs.dim) / B
    g_params, _ = flow_vjp(params, z, fs, g_phi, 1.0 / B, emulate=emulate)
    return g_params

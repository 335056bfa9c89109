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
  * Batch norm (the example parameter file's use_bn, false there and otherwise
    undefined): with batch_norm, every hidden convolution's output a is
    normalised per channel before its LeakyReLU, y = gamma (a - mean) /
    sqrt(var + 1e-5) + beta, with learnable gamma, beta.  Training (batch
    statistics) takes the mean and the biased variance over the batch and all
    sites; sampling takes running statistics, updated after each training
    forward as r <- (1 - m) r + m s with momentum m (default 0.1) and the
    unbiased variance n/(n - 1) var, n = B V.  The network reads only the
    frozen sites, so the statistics do too and the log-det is still the sum of
    s over the active sites.

Parameter layout (shared data contract): per layer W1[C][1][T], b1[C],
W2[C][C][T], b2[C], W3[2][C][T], b3[2]; taps row-major over delta in
{-1,0,1}^dim, axis 0 slowest.  A general network stores, per layer and per
convolution i in order, W_i[cout_i][cin_i][T] then b_i[cout_i], with T = K^dim
and taps row-major over {-K//2..K//2}^dim.  With batch norm a hidden
convolution's b_i is followed by gamma_i[cout_i] then beta_i[cout_i]; the
statistics (not parameters) are stored per layer and hidden convolution as
mean[cout_i] then var[cout_i].

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
(C, C), kernel-3 network with the default one; for batch norm
(tests/test_oracle_flow_bn.py) the layout, unit statistics of the normalised
activations, the bias dropping out under batch statistics, running statistics
equal to the batch's reproducing batch mode, running mode equal to a plain
network with the normalisation folded into the convolutions, invertibility, the
brute-force Jacobian of a whole batch, the running average against numpy's
unbiased variance, and central finite differences of the loss in both modes.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .action import action as _action, force as _force
from .prior import log_prior
from .rounding import ROUNDERS, to_fp32

LEAKY_SLOPE = 0.01
BN_EPS = 1e-5
BN_MOMENTUM = 0.1


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
    batch_norm: bool = False

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

    n_conv = len(fs.conv_shapes)
    for _ in range(fs.n_layers):
        lay = []
        for i, (co, ci) in enumerate(fs.conv_shapes):
            lay.append(take(co * ci * T, (co, ci, T)))
            lay.append(take(co, (co,)))
            if fs.batch_norm and i < n_conv - 1:
                lay.append(take(co, (co,)))      # gamma
                lay.append(take(co, (co,)))      # beta
        layers.append(tuple(lay))
    if off != p.size:
        raise ValueError(f"parameter vector has {p.size} entries, layout needs {off}")
    return layers


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([a.ravel() for a in lay]) for lay in layers])


def split_convs(lay, fs: FlowShape):
    """Per convolution of a layer's tuple: (W, b, gamma, beta); gamma and beta are
    None without batch norm and for the last convolution."""
    out, k = [], 0
    n_conv = len(fs.conv_shapes)
    for i in range(n_conv):
        W, b = lay[k], lay[k + 1]
        k += 2
        g = be = None
        if fs.batch_norm and i < n_conv - 1:
            g, be = lay[k], lay[k + 1]
            k += 2
        out.append((W, b, g, be))
    return out


def initial_bn_stats(fs: FlowShape):
    """Running statistics before training: mean 0, variance 1, per layer and hidden convolution."""
    return [[(np.zeros(w), np.ones(w)) for w in fs.widths] for _ in range(fs.n_layers)]


def pack_bn_stats(stats) -> np.ndarray:
    return np.concatenate([np.concatenate([np.concatenate([m, v]) for m, v in lay]) for lay in stats])


def unpack_bn_stats(vec, fs: FlowShape):
    v = np.asarray(vec, dtype=np.float64).ravel()
    out, off = [], 0
    for _ in range(fs.n_layers):
        lay = []
        for w in fs.widths:
            lay.append((v[off:off + w], v[off + w:off + 2 * w]))
            off += 2 * w
        out.append(lay)
    if off != v.size:
        raise ValueError(f"statistics vector has {v.size} entries, layout needs {off}")
    return out


def _per_channel(v, ndim):
    return np.asarray(v).reshape((1, -1) + (1,) * (ndim - 2))


def batch_norm(a, gamma, beta, stats=None):
    """Per-channel normalisation of a [B, c, *lattice] over the batch and all sites.

    stats None: the batch's own mean and biased variance; else the given (mean, var).
    Returns y = gamma (a - mean) / sqrt(var + eps) + beta, the normalised xhat, the
    reciprocal deviation r = 1 / sqrt(var + eps), and the (mean, var) used."""
    ax = (0,) + tuple(range(2, a.ndim))
    if stats is None:
        mean = a.mean(axis=ax)
        var = ((a - _per_channel(mean, a.ndim)) ** 2).mean(axis=ax)
    else:
        mean, var = (np.asarray(x, dtype=np.float64) for x in stats)
    r = 1.0 / np.sqrt(var + BN_EPS)
    xh = (a - _per_channel(mean, a.ndim)) * _per_channel(r, a.ndim)
    y = _per_channel(gamma, a.ndim) * xh + _per_channel(beta, a.ndim)
    return y, xh, r, (mean, var)


def batch_norm_vjp(g_y, xh, r, gamma, batch_stats: bool):
    """Adjoint of `batch_norm`: (g_a, g_gamma, g_beta).  With batch statistics the
    mean and variance depend on every entry of a:
    g_a = gamma r (g_y - mean(g_y) - xhat mean(g_y xhat)), means per channel."""
    ax = (0,) + tuple(range(2, g_y.ndim))
    g_gamma = (g_y * xh).sum(axis=ax)
    g_beta = g_y.sum(axis=ax)
    scale = _per_channel(gamma * r, g_y.ndim)
    if not batch_stats:
        return scale * g_y, g_gamma, g_beta
    n = g_y.size // g_y.shape[1]
    return (scale * (g_y - _per_channel(g_beta / n, g_y.ndim) - xh * _per_channel(g_gamma / n, g_y.ndim)),
            g_gamma, g_beta)


def bn_running_update(running, batch, n: int, momentum: float = BN_MOMENTUM):
    """Running statistics after one training batch of n = B V terms per channel:
    r <- (1 - m) r + m s, with the unbiased variance n / (n - 1) var."""
    out = []
    for lay_r, lay_b in zip(running, batch):
        out.append([((1 - momentum) * rm + momentum * bm, (1 - momentum) * rv + momentum * bv * n / (n - 1))
                    for (rm, rv), (bm, bv) in zip(lay_r, lay_b)])
    return out


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


def net(x, lay, mF, fs: FlowShape, emulate=None, bn_stats=None, bn_cache=None):
    """s/t network of one layer.  Returns (acts, hs, o, s, t): the inputs of every
    LeakyReLU a_1 .. a_n (the normalised y_i with batch norm), the inputs h_0 =
    mask_F x, h_i = leaky(a_i) of every convolution, the output o and s, t.

    Batch norm: bn_stats is None for batch statistics or this layer's running
    (mean, var) per hidden convolution; bn_cache, a list, receives per hidden
    convolution (xhat, r, gamma, (mean, var) used)."""
    R, _ = _rounders(emulate)
    h = (x * mF)[:, None]
    acts, hs = [], [h]
    convs = split_convs(lay, fs)
    for i, (W, b, gamma, beta) in enumerate(convs[:-1]):
        a = conv(R(h), R(W), b, fs.dim)
        if gamma is not None:
            a, xh, r, st = batch_norm(a, gamma, beta, None if bn_stats is None else bn_stats[i])
            if bn_cache is not None:
                bn_cache.append((xh, r, gamma, st))
        h = leaky(a)
        acts.append(a)
        hs.append(h)
    o = conv(R(h), R(convs[-1][0]), convs[-1][1], fs.dim)
    s = np.tanh(o[:, 0]) if fs.final_tanh else o[:, 0]
    t = o[:, 1]
    return acts, hs, o, s, t


def coupling_forward(x, lay, layer: int, fs: FlowShape, emulate=None, bn_stats=None, bn_cache=None):
    """One layer in the sampling direction.  Returns (y, sum_A s per sample)."""
    mF = frozen_mask(fs, layer)
    mA = 1.0 - mF
    *_, s, t = net(x, lay, mF, fs, emulate, bn_stats, bn_cache)
    y = _rounders(emulate)[1](np.where(mA > 0, x * np.exp(s) + t, x))
    ax = tuple(range(1, x.ndim))
    return y, np.sum(mA * s, axis=ax)


def coupling_inverse(y, lay, layer: int, fs: FlowShape, bn_stats=None):
    """Inverse of `coupling_forward`: s, t depend only on the frozen sites, which are
    unchanged (and so are batch statistics over the same batch)."""
    mF = frozen_mask(fs, layer)
    mA = 1.0 - mF
    *_, s, t = net(y, lay, mF, fs, bn_stats=bn_stats)
    x = np.where(mA > 0, (y - t) * np.exp(-s), y)
    ax = tuple(range(1, y.ndim))
    return x, np.sum(mA * s, axis=ax)


def as_lattice(z, fs: FlowShape):
    z = np.asarray(z, dtype=np.float64)
    return z.reshape((z.shape[0],) + fs.lattice)


def _layer_stats(bn_stats, l):
    return None if bn_stats is None else bn_stats[l]


def flow_forward(params, z, fs: FlowShape, return_saved: bool = False, emulate=None, bn_stats=None):
    """phi = F^{-1}(z) with log q.  Returns dict(phi, logdet, logr, logq[, saved]).

    Batch norm: bn_stats None normalises with batch statistics, else with the given
    running statistics (per layer, per hidden convolution (mean, var)); the result
    then also holds bn_used, the (mean, var) each hidden convolution used (the
    batch's mean and biased variance under batch statistics)."""
    layers = unpack(params, fs)
    x = as_lattice(z, fs)
    logdet = np.zeros(x.shape[0])
    saved = [x]
    used = []
    for l, lay in enumerate(layers):
        cache = []
        x, ld = coupling_forward(x, lay, l, fs, emulate, _layer_stats(bn_stats, l), cache)
        used.append([c[3] for c in cache])
        logdet = logdet + ld
        saved.append(x)
    logr = log_prior(z)
    out = dict(phi=x, logdet=logdet, logr=logr, logq=logr - logdet)
    if fs.batch_norm:
        out["bn_used"] = used
    if return_saved:
        out["saved"] = saved
    return out


def flow_inverse(params, phi, fs: FlowShape, bn_stats=None):
    """z = F(phi) and the log-determinant of F^{-1} at z (for tests)."""
    layers = unpack(params, fs)
    x = as_lattice(phi, fs)
    logdet = np.zeros(x.shape[0])
    for l in reversed(range(fs.n_layers)):
        x, ld = coupling_inverse(x, layers[l], l, fs, _layer_stats(bn_stats, l))
        logdet = logdet + ld
    return x, logdet


def log_weights(S, logq):
    """log w = log p - log q up to ln Z: w = -S - log q (FP64)."""
    return -np.asarray(S, dtype=np.float64) - np.asarray(logq, dtype=np.float64)


def kl_loss(params, z, fs: FlowShape, m2, lam, bn_stats=None) -> float:
    """Shifted reverse KL, batch mean of log q + S, with z fixed."""
    f = flow_forward(params, z, fs, bn_stats=bn_stats)
    S = _action(f["phi"], m2, lam, fs.dim)
    return float(np.mean(f["logq"] + S))


def flow_vjp(params, z, fs: FlowShape, g_phi, g_logq, emulate=None, bn_stats=None):
    """Vector-Jacobian product of (phi, log q) = flow_forward(params, z) w.r.t. (params, z).

    g_phi: [B, *lattice] or [B, V]; g_logq: [B] or scalar.  Returns (g_params packed, g_z [B, V]).
    Hand-derived adjoint, layer by layer in reverse, recomputing each layer's network
    from the layer's input field.  bn_stats as in flow_forward; batch statistics are
    differentiated as functions of the whole batch.
    """
    layers = unpack(params, fs)
    R, RF = _rounders(emulate)
    f = flow_forward(params, z, fs, return_saved=True, emulate=emulate, bn_stats=bn_stats)
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
        cache = []
        acts, hs, o, s, t = net(x, lay, mF, fs, emulate, _layer_stats(bn_stats, l), cache)
        es = np.exp(s)
        g_y = gx
        g_t = mA * g_y
        g_s = mA * (g_y * x * es + g_ld.reshape(shp))
        g_o0 = g_s * (1.0 - s * s) if fs.final_tanh else g_s
        # back through the convolutions, last to first: g is the gradient of the
        # current convolution's output (g_o, then g_a_i = g_h_i leaky'(a_i), taken
        # back through the normalisation with batch norm)
        g = np.stack([g_o0, g_t], axis=1)
        convs = split_convs(lay, fs)
        conv_grads = [None] * len(convs)
        bn_grads = [()] * len(convs)
        for i in reversed(range(len(convs))):
            conv_grads[i] = _weight_grad(g, hs[i], fs.dim, R, fs.kernel)
            g = conv_transpose(R(g), R(convs[i][0]), fs.dim)
            if i == 0:
                break
            g = g * leaky_grad(acts[i - 1])
            if convs[i - 1][2] is not None:
                xh, r, gamma, _ = cache[i - 1]
                g, d_gamma, d_beta = batch_norm_vjp(g, xh, r, gamma, bn_stats is None)
                bn_grads[i - 1] = (d_gamma, d_beta)
        lay_grads = [a for cg, bg in zip(conv_grads, bn_grads) for a in (*cg, *bg)]
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


def loss_gradient(params, z, fs: FlowShape, m2, lam, emulate=None, bn_stats=None):
    """Gradient of the batch-mean reverse-KL loss w.r.t. the packed parameters, z fixed."""
    f = flow_forward(params, z, fs, emulate=emulate, bn_stats=bn_stats)
    B = f["phi"].shape[0]
    g_phi = _force(f["phi"], m2, lam, fs.dim) / B
    g_params, _ = flow_vjp(params, z, fs, g_phi, 1.0 / B, emulate=emulate, bn_stats=bn_stats)
    return g_params

"""Writes tests/golden/full_size_grad_<name>.npz: the FP64 oracle's reverse-KL
gradient for the full-size training steps, compressed to what the GPU test
compares (a stratified sample of entries, every parameter block's norm and 32
seeded random projections of the whole gradient), plus the batch-mean loss and
the batch mean of sum_n |dS/dphi_n| (1 + |phi_n|), the first-order sensitivity
of S to per-site field errors bounded by tol (1 + |phi_n|), and the relative
error of each block (and of the whole gradient) when the oracle stores the conv
operands and the field in FP32 (its emulate="fp32" mode): the error an FP32
implementation incurs from storage rounding alone.  For the BF16 path the
gradient of the oracle's emulate="bf16" mode (every convolution operand rounded
to BF16, the field kept in FP32, weight gradients accumulated in FP32) is stored
the same way (sampled entries, block norms, projections), with its loss and its
relative deviation from FP64 per block: an implementation that rounds at the
same points must match it far more closely than it matches FP64.

Only oracle/ and the seeded input generators are used: z is the oracle's own
Philox prior draw (key 12345, counter 0, as the trainer's first step draws it)
and the weights are the seeded N(0, 0.1) initialisation.

    python tests/golden/make_full_size.py [name ...]     (default: all)

The gradient of the batch mean is a sum over samples, so the batch is split
into chunks evaluated by a process pool and summed in chunk order.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

# name: (dim, L, n_layers, hidden, batch, m2, lambda, weight std, FP32 emulation)
# The 3D L=16 C=32 flow uses N(0, 0.05^2) weights: at the workload's N(0, 0.1^2)
# its 16 layers amplify rounding beyond any useful comparison (see the tests);
# it has a BF16 backward only, so no FP32 emulation is stored for it.
CONFIGS = {
    "2d_L32_C16_B1024": (2, 32, 16, 16, 1024, -4.0, 8.0, 0.1, True),
    "3d_L8_C16_B512": (3, 8, 12, 16, 512, -4.0, 5.0, 0.1, True),
    "3d_L16_C32_B256": (3, 16, 16, 32, 256, -4.0, 5.0, 0.05, False),
    # the 3D L=8 step again at N(0, 0.05^2) weights: at N(0, 0.1^2) the flow's loss is ~1e10
    # and BF16 rounding moves its gradient blocks by up to 25 %, too ill-conditioned for
    # tight bounds; here the same kernels are held to the tight ones
    "3d_L8_C16_B512_w05": (3, 8, 12, 16, 512, -4.0, 5.0, 0.05, True),
}
KEY, COUNTER0, WEIGHT_SEED = 12345, 0, 2021
PROJ_SEED, N_PROJ, PER_BLOCK = 4242, 32, 12
CHUNK = 32


def _chunk(args):
    import seeded_inputs as si
    from oracle import flow as of
    from oracle import prior as op
    from oracle import action as oa
    dim, L, N, C, B, m2, lam, w_std, emul32, start, n = args
    fs = of.FlowShape(dim, L, N, C)
    p = si.flow_params(dim, N, C, seed=WEIGHT_SEED, w_std=w_std).astype(np.float64)
    z = op.prior_normal(KEY, COUNTER0 + start, n, fs.V)
    g = of.loss_gradient(p, z, fs, m2, lam)
    g32 = of.loss_gradient(p, z, fs, m2, lam, emulate="fp32") if emul32 else g
    g16 = of.loss_gradient(p, z, fs, m2, lam, emulate="bf16")
    loss = of.kl_loss(p, z, fs, m2, lam)
    f16 = of.flow_forward(p, z, fs, emulate="bf16")
    loss16 = float(np.mean(f16["logq"] + oa.action(f16["phi"], m2, lam, dim)))
    # first-order sensitivity of S to per-site field errors e_n <= tol (1 + |phi_n|):
    # sum_n |dS/dphi_n| (1 + |phi_n|), per sample
    phi = of.flow_forward(p, z, fs)["phi"]
    F = oa.force(phi, m2, lam, dim).reshape(n, -1)
    sens = np.sum(np.abs(F) * (1.0 + np.abs(phi.reshape(n, -1))), axis=1)
    return (start, g * (n / B), g32 * (n / B), loss * (n / B), float(np.sum(sens)) / B,
            g16 * (n / B), loss16 * (n / B))


def block_slices(dim, N, C):
    """(layer, block name, slice) of every parameter block in the packed order."""
    import seeded_inputs as si
    out, off = [], 0
    for layer in range(N):
        for name, sz in si.layer_block_sizes(dim, C):
            out.append((layer, name, slice(off, off + sz)))
            off += sz
    return out


def sample_indices(dim, N, C):
    rng = np.random.default_rng(PROJ_SEED + 1)
    idx = []
    for _, _, sl in block_slices(dim, N, C):
        size = sl.stop - sl.start
        k = min(size, PER_BLOCK)
        idx.extend(sl.start + np.sort(rng.choice(size, size=k, replace=False)))
    return np.asarray(idx, np.int64)


def projections(g):
    R = np.random.default_rng(PROJ_SEED).standard_normal((N_PROJ, g.size))
    return R @ g


def make(name, pool):
    dim, L, N, C, B, m2, lam, w_std, emul32 = CONFIGS[name]
    t = time.time()
    jobs = [(dim, L, N, C, B, m2, lam, w_std, emul32, s, min(CHUNK, B - s)) for s in range(0, B, CHUNK)]
    res = sorted(pool.map(_chunk, jobs), key=lambda r: r[0])
    g = np.zeros_like(res[0][1])
    g32 = np.zeros_like(g)
    g16 = np.zeros_like(g)
    loss = sens = loss16 = 0.0
    for _, gc, g32c, lc, sc, g16c, l16c in res:
        g += gc
        g32 += g32c
        loss += lc
        sens += sc
        g16 += g16c
        loss16 += l16c
    idx = sample_indices(dim, N, C)
    norms = np.array([np.linalg.norm(g[sl]) for _, _, sl in block_slices(dim, N, C)])
    # how far FP32 storage of the conv operands and the field alone moves each block
    err32 = np.array([np.linalg.norm(g32[sl] - g[sl]) / max(np.linalg.norm(g[sl]), 1e-300)
                      for _, _, sl in block_slices(dim, N, C)])
    blocks = block_slices(dim, N, C)
    err16 = np.array([np.linalg.norm(g16[sl] - g[sl]) / max(np.linalg.norm(g[sl]), 1e-300) for _, _, sl in blocks])
    np.savez(os.path.join(HERE, f"full_size_grad_{name}.npz"),
             config=np.array([dim, L, N, C, B], np.int64), couplings=np.array([m2, lam]),
             w_std=np.array([w_std]),
             seeds=np.array([KEY, COUNTER0, WEIGHT_SEED, PROJ_SEED], np.int64),
             idx=idx, vals=g[idx], block_norms=norms, proj=projections(g),
             grad_norm=np.array([np.linalg.norm(g)]), loss=np.array([loss]),
             loss_sensitivity=np.array([sens]), fp32_block_err=err32,
             fp32_whole_err=np.array([np.linalg.norm(g32 - g) / np.linalg.norm(g)]),
             bf16_vals=g16[idx], bf16_block_norms=np.array([np.linalg.norm(g16[sl]) for _, _, sl in blocks]),
             bf16_proj=projections(g16), bf16_grad_norm=np.array([np.linalg.norm(g16)]),
             bf16_loss=np.array([loss16]), bf16_block_err=err16,
             bf16_whole_err=np.array([np.linalg.norm(g16 - g) / np.linalg.norm(g)]))
    print(f"{name}: {time.time() - t:.1f} s, |g| = {np.linalg.norm(g):.6g}, loss = {loss:.6f}, "
          f"FP32-operand error: max block {err32.max():.3g}, whole {np.linalg.norm(g32 - g) / np.linalg.norm(g):.3g}; "
          f"BF16-operand error: max block {err16.max():.3g}, whole {np.linalg.norm(g16 - g) / np.linalg.norm(g):.3g}", flush=True)


if __name__ == "__main__":
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"  # one BLAS thread per pool process
    names = sys.argv[1:] or list(CONFIGS)
    with mp.get_context("spawn").Pool(min(8, os.cpu_count() or 1)) as pool:
        for nm in names:
            make(nm, pool)

#!/usr/bin/env python3
"""Benchmark of the flow-based phi^4 sampler's hot path on one MI355X.

Workload (a "step"): one reverse-KL training iteration of the 2D phi^4 flow,
L = 32, m^2 = -4, lambda = 8, 16 affine coupling layers with hidden channels 16,
batch 1024, Adam lr 1e-3: prior draw -> flow forward with log q (saving the
layer inputs) -> action and force -> log-weights and loss -> hand-written flow
backward -> Adam.  Inputs are synthetic: seeded N(0, 0.1) weights (biases 0),
Philox prior draws.  `value` is plain-FP32 training steps per second (the
paper's arithmetic: FP32 convolutions, on FP32 matrix cores), with `roofline`
(the per-layer backward launch against the FP32 MFMA peak, and its HBM traffic
from the committed rocprofv3 summary) and `cpu_baseline` (the FP64 oracle on a
bounded sample of the batch, on all host cores, with the one-thread figure
beside it).  Beside it: the BF16-convolution form of the same step with its own
roofline, flow+MH sampling, the FP64 HMC baseline with its FP64 roofline, the
memory-side kernels against HBM (the prior also against the VALU issue peak),
the other workloads (2D L=8, 3D L=8 with its 10k-proposal chain, 3D L=16 C=32),
other s/t networks, the example schedule and the 3D L=8 flow trained with
acceptance over training and chain quality against HMC, serving in both
precisions, and the oracle on the other workloads.

Prints ONE JSON line (progress lines go to stderr).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # the headline workload (the default)
    "phi4-2d-L32-train": dict(workload="phi4-2d-L32-train", dim=2, L=32, m2=-4.0, lam=8.0,
                              n_layers=16, hidden=16, batch=1024, lr=1e-3),
    # the 3D L = 16 C = 32 training step (for its own profile; BF16 only)
    "phi4-3d-L16-C32-train": dict(workload="phi4-3d-L16-C32-train", dim=3, L=16, m2=-4.0, lam=5.0,
                                  n_layers=16, hidden=32, batch=256, lr=1e-3),
}
WORKLOAD = WORKLOADS["phi4-2d-L32-train"]
PEAK = {"bf16_mfma_tflops": 2500.0, "fp32_mfma_tflops": 157.3, "fp64_tflops": 78.6, "hbm_gbs": 8000.0}
KERNEL_SOURCES = ["paper_2208_08903_amd/csrc/flow_fused_bwd.hip",
                  "paper_2208_08903_amd/csrc/fused_kernels.hpp",
                  "paper_2208_08903_amd/csrc/fused_common.hpp",
                  "paper_2208_08903_amd/csrc/lfs_common.hpp",
                  "paper_2208_08903_amd/csrc/fused_bwd_common.hpp"]
# HBM bytes per backward launch (rocprofv3 FETCH_SIZE / WRITE_SIZE), per precision
TRAFFIC_FILES = {"fp32": "profiles/kf_backward_fp32_phi4-2d-L32-train_traffic.txt",
                 "bf16": "profiles/kf_backward_bf16_phi4-2d-L32-train_traffic.txt"}
# VALU instructions of the prior draw at the 4096 x 4096-site sampling shape
# (rocprofv3 SQ_INSTS_VALU); the prior is bound by its Philox and Box-Muller
# arithmetic, not by HBM
PRIOR_SOURCES = ["paper_2208_08903_amd/csrc/prior.hip", "paper_2208_08903_amd/csrc/lfs_common.hpp"]
PRIOR_VALU_FILE = "profiles/k_prior_phi4-3d-L16-sample_valu.txt"
# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD every 4 cycles
# (16 lanes per SIMD); reduced-rate instructions (64-bit integer multiply-add, transcendentals)
# take longer, so a fraction of this peak is a lower bound on the VALU's busy fraction
VALU_PEAK_G_WAVE_INSTR = 256 * 4 * 2.4 / 4


def _progress(msg):
    """One line per finished stage on stderr (the JSON result alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_source_sha(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _recorded(path, key, sources=None):
    """A figure from a committed rocprofv3 summary, if the kernel sources are unchanged
    since the counters were taken; else None."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != kernel_source_sha(sources):
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def recorded_traffic(prec_name):
    """HBM bytes per backward launch (rocprofv3 FETCH_SIZE / WRITE_SIZE summary)."""
    return _recorded(TRAFFIC_FILES[prec_name], "traffic_bytes_per_launch")


def recorded_prior_valu():
    """VALU wave instructions per prior launch at the sampling shape (SQ_INSTS_VALU summary)."""
    return _recorded(PRIOR_VALU_FILE, "valu_wave_instructions_per_launch", PRIOR_SOURCES)


def algorithmic_flops_per_sample_layer(dim, L, C):
    """2 T (C^2 + 1.5 C) flops per site: conv2 dense, conv1 on the non-zero (frozen) half of
    its taps, conv3 at the active half of the sites (forward pass)."""
    T = 3 ** dim
    return 2.0 * T * (C * C + 1.5 * C) * L ** dim


def time_phases(tr, steps, warmup):
    """Run warmup + timed steps; returns total seconds and per-phase event averages (ms)."""
    import torch
    for _ in range(warmup):
        tr.step()
    torch.cuda.synchronize()
    names = ["draw", "forward", "backward", "update"]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        e = ev[k]
        e[0].record()
        tr.draw()
        e[1].record()
        tr.forward()
        e[2].record()
        tr.backward()
        e[3].record()
        tr.update()
        e[4].record()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    phase = {n: sum(ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(steps)) / steps
             for i, n in enumerate(names)}
    return total, phase


def flow_forward_ms(flow, B, reps=20):
    """Average duration (ms) of one lfs_flow_forward call (fragment prep + the fused kernel)."""
    import torch
    from paper_2208_08903_amd import lfs
    z = torch.randn(B, flow.V, device="cuda")
    phi = torch.empty_like(z)
    lq = torch.empty(B, dtype=torch.float64, device="cuda")
    ws = flow.workspace(B, False)
    for _ in range(3):
        lfs.flow_forward(flow.desc, flow.params, z, phi, lq, None, None, ws)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        lfs.flow_forward(flow.desc, flow.params, z, phi, lq, None, None, ws)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def sampling_rate(flow, B, m2, lam, batches=10):
    import torch
    from paper_2208_08903_amd import flow as fl
    import seeded_inputs as si
    smp = fl.Sampler(flow, B, m2, lam, key=777)
    lu = torch.as_tensor(si.log_uniforms(5, (batches + 2, 1, B)), device="cuda")
    smp.step(lu[0])
    smp.step(lu[1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(batches):
        smp.step(lu[k + 2])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    acc, n_acc = smp.acceptance()
    return dict(proposals_per_s=B * batches / dt, acceptance=acc,
                accepted_per_s=acc * B * batches / dt, batch=B)


def hmc_flops_per_trajectory(dim, V, n_steps):
    """Algorithmic FP64 flops of one KDK trajectory of one chain: per site and leapfrog step
    the force -2 Lap phi + 2 m^2 phi + 4 lambda phi^3 (2 dim + 1 for the Laplacian, 5 for
    the rest: 2 dim + 6), two half-kicks and a drift (2 each: 6); the Hamiltonian at both
    ends (the action density and 1/2 pi^2: 2 dim + 8 each)."""
    return V * (n_steps * (2 * dim + 12) + 2 * (2 * dim + 8))


def hmc_rate(reps=5):
    """FP64 HMC baseline on the 3D L=8 theory: 512 chains x 10 leapfrog steps of 0.1, with
    its rate against the FP64 vector peak (a trajectory is latency-bound: 10 dependent
    steps, two barriers each, over 512 sites per chain)."""
    import torch
    from paper_2208_08903_amd import lfs
    import seeded_inputs as si
    B, L, dim, n_steps = 512, 8, 3, 10
    V = L ** dim
    phi = torch.as_tensor(0.5 * si.normal_fields(3, B, V).astype("float64"), device="cuda")
    pi = torch.as_tensor(si.momenta(4, B, V), device="cuda")
    lu = torch.as_tensor(si.log_uniforms(5, B), device="cuda")
    m2 = torch.tensor([-4.0], dtype=torch.float64, device="cuda")
    lam = torch.tensor([5.0], dtype=torch.float64, device="cuda")
    dH = torch.empty(B, dtype=torch.float64, device="cuda")
    acc = torch.empty(B, dtype=torch.uint8, device="cuda")
    lfs.hmc_step(dim, L, phi, pi, lu, m2, lam, n_steps, 0.1, dH, acc)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        lfs.hmc_step(dim, L, phi, pi, lu, m2, lam, n_steps, 0.1, dH, acc)
    e.record()
    torch.cuda.synchronize()
    dt = s.elapsed_time(e) * 1e-3 / reps
    flops = B * hmc_flops_per_trajectory(dim, V, n_steps)
    tf = flops / dt / 1e12
    return dict(trajectories_per_s=B / dt, chains=B, leapfrog_steps=n_steps, dt=0.1,
                acceptance=float(acc.float().mean().item()), us_per_call=round(dt * 1e6, 2),
                force_evaluations_per_trajectory=n_steps + 1,
                roofline={"bound": "fp64", "achieved": round(tf, 4), "peak": PEAK["fp64_tflops"],
                          "unit": "TFLOP/s", "frac": round(tf / PEAK["fp64_tflops"], 5),
                          "flops_per_call": flops})


def chain_3d_L8_10k():
    """The 3D L=8 workload's sampling chain: 10 000 flow proposals (12 layers, C=16, seeded
    N(0,0.1) weights) in one batch, their action and log-weights, and one independence-MH
    chain over them; proposals/s and acceptance, in both precisions."""
    import torch
    import seeded_inputs as si
    from paper_2208_08903_amd import flow as fl
    from paper_2208_08903_amd import lfs
    out = {}
    p3 = si.flow_params(3, 12, 16)
    n = 10_000
    lu = torch.as_tensor(si.log_uniforms(31, (3, 1, n)), device="cuda")
    for prec, name in ((lfs.LFS_BF16_CONV, "bf16"), (lfs.LFS_PLAIN_FP32, "fp32")):
        f = fl.Flow(3, 8, 12, 16, prec, params=p3)
        smp = fl.Sampler(f, n, -4.0, 5.0, key=2024)
        smp.step(lu[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smp.step(lu[1])
        smp.step(lu[2])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 2
        acc, n_acc = smp.acceptance()
        out[name] = {"proposals": n, "chain_ms": round(1e3 * dt, 3), "proposals_per_s": round(n / dt, 1),
                     "acceptance": acc, "accepted": n_acc}
    return out


def hbm_kernels(reps=20):
    """Achieved HBM bandwidth of the memory-bound kernels at a bandwidth-bound size: the 3D L=16
    sampling batch (4096 x 4096 sites) for the prior draw, the action with its force and the
    observables, and Adam over 16 M parameters.  Bytes are the algorithmic ones (each array read
    or written once); durations from HIP events on the library's stream."""
    import torch
    from paper_2208_08903_amd import lfs
    B, L, dim = 4096, 16, 3
    V = L ** dim
    dev = "cuda"
    z = torch.empty(B, V, dtype=torch.float32, device=dev)
    logr = torch.empty(B, dtype=torch.float64, device=dev)
    S = torch.empty(B, dtype=torch.float64, device=dev)
    force = torch.empty_like(z)
    M = torch.empty(B, dtype=torch.float64, device=dev)
    C = torch.empty(B, L, dtype=torch.float64, device=dev)
    m2 = torch.tensor([-4.0], dtype=torch.float64, device=dev)
    lam = torch.tensor([5.0], dtype=torch.float64, device=dev)
    n = 16 * 2 ** 20
    p, g = torch.zeros(n, device=dev), torch.full((n,), 1e-3, device=dev)
    mo, vo = torch.zeros(n, device=dev), torch.zeros(n, device=dev)
    lfs.prior_normal(5, 0, z, logr)
    cases = {
        "prior_normal": (lambda: lfs.prior_normal(5, 0, z, logr), B * V * 4 + B * 8),
        "action_force_fp64_sums": (lambda: lfs.action(dim, L, z, m2, lam, S, force, 1.0, lfs.LFS_BF16_CONV),
                                   2 * B * V * 4 + B * 8),
        "observables": (lambda: lfs.observables(dim, L, z, M, C), B * V * 4 + B * (L + 1) * 8),
        "adam": (lambda: lfs.adam_step(p, g, mo, vo, 1e-3, 0.9, 0.999, 1e-8, 1), 28 * n),
    }
    out = {}
    for name, (fn, nbytes) in cases.items():
        for _ in range(3):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        us = 1e3 * s.elapsed_time(e) / reps
        gbs = nbytes / us / 1e3
        out[name] = {"bytes": nbytes, "us": round(us, 2), "GB_s": round(gbs, 1), "frac_of_8TB_s": round(gbs / 8000, 3)}
    valu = recorded_prior_valu()
    if valu:
        g = valu / out["prior_normal"]["us"] / 1e3
        out["prior_normal"]["alu"] = {"bound": "alu", "achieved": round(g, 1), "peak": VALU_PEAK_G_WAVE_INSTR,
                                      "unit": "G VALU wave-instructions/s",
                                      "frac": round(g / VALU_PEAK_G_WAVE_INSTR, 3),
                                      "valu_wave_instructions_per_launch": valu}
    return out


def general_networks(steps=200):
    """Training steps/s of the example shape (2D L=8, 16 layers, batch 64, BF16) with other
    s/t networks from the parameter file's hidden_sizes / kernel_size / use_bn, on the
    general-network kernels, beside the default network (hidden [8, 8], kernel 3); each
    eagerly and with forward + backward replayed from a captured HIP graph."""
    import torch
    import seeded_inputs as si
    from paper_2208_08903_amd import flow as fl
    from paper_2208_08903_amd import lfs
    out = {}
    for name, K, hs, bn in (("default_8x8_k3", 0, None, False), ("hidden_8x8_k5", 5, (8, 8), False),
                            ("hidden_16x16x16_k3", 3, (16, 16, 16), False), ("hidden_8_k3", 3, (8,), False),
                            ("hidden_8x8_k3_batch_norm", 3, (8, 8), True)):
        row = {}
        for graph in (False, True):
            f = fl.Flow(2, 8, 16, 8, lfs.LFS_BF16_CONV, kernel=K, hidden_sizes=hs, batch_norm=bn,
                        params=si.flow_params(2, 16, 8, kernel=K or 3, hidden_sizes=hs, batch_norm=bn))
            tr = fl.Trainer(f, 64, -4.0, 8.0, graph=graph)
            for _ in range(5):
                tr.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                tr.step()
            torch.cuda.synchronize()
            row["params"] = f.P
            row["train_steps_per_s_graph" if graph else "train_steps_per_s"] = \
                round(steps / (time.perf_counter() - t0), 1)
        out[name] = row
    return out


def other_workloads(params_2d):
    """Side figures for the other workloads: the 2D L=8 example shape (latency of one batch of 64,
    a 2000-proposal chain), the 3D L=8 training step, and 3D L=16 C=32 training at batch 256
    (with its device-memory footprint) and sampling at batch 4096."""
    import numpy as np
    import torch
    import seeded_inputs as si
    from paper_2208_08903_amd import flow as fl
    from paper_2208_08903_amd import lfs
    out = {}
    # 2D L=8, 16 layers, C=8, m2=-4, lambda=8: one batch of 64, then a chain of 2000 proposals
    p8 = si.flow_params(2, 16, 8)
    f8 = fl.Flow(2, 8, 16, 8, lfs.LFS_BF16_CONV, params=p8)
    s64 = fl.Sampler(f8, 64, -4.0, 8.0, key=11)
    lu = torch.as_tensor(si.log_uniforms(6, (40, 1, 64)), device="cuda")
    for k in range(3):
        s64.step(lu[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(20):
        s64.step(lu[3 + k])
    torch.cuda.synchronize()
    out["2d_L8_batch64_us"] = round(1e6 * (time.perf_counter() - t0) / 20, 2)
    s2k = fl.Sampler(f8, 2000, -4.0, 8.0, key=12)
    lu2 = torch.as_tensor(si.log_uniforms(7, (3, 1, 2000)), device="cuda")
    s2k.step(lu2[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s2k.step(lu2[1])
    torch.cuda.synchronize()
    out["2d_L8_chain2000_ms"] = round(1e3 * (time.perf_counter() - t0), 4)
    # 3D L=8, 12 layers, C=16, batch 512 training (BF16 and FP32)
    p3 = si.flow_params(3, 12, 16)
    for prec, name in ((lfs.LFS_BF16_CONV, "bf16"), (lfs.LFS_PLAIN_FP32, "fp32")):
        f3 = fl.Flow(3, 8, 12, 16, prec, params=p3)
        tr = fl.Trainer(f3, 512, -4.0, 5.0)
        tt, ph = time_phases(tr, 5, 2)
        out[f"3d_L8_train_{name}_steps_per_s"] = round(5 / tt, 3)
    # 3D L=16, 16 layers, C=32, BF16: training at batch 256; the footprint is the peak of
    # every device allocation the trainer makes (weights, Adam state, saved fields,
    # workspaces)
    p16 = si.flow_params(3, 16, 32)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    f16t = fl.Flow(3, 16, 16, 32, lfs.LFS_BF16_CONV, params=p16)
    tr16 = fl.Trainer(f16t, 256, -4.0, 5.0)
    tt, ph = time_phases(tr16, 5, 2)
    out["3d_L16_C32_train_bf16_steps_per_s"] = round(5 / tt, 3)
    out["3d_L16_C32_train_bf16_phases_ms"] = {k: round(v, 3) for k, v in ph.items()}
    out["3d_L16_C32_train_hbm_bytes"] = int(torch.cuda.max_memory_allocated() - base)
    del tr16, f16t
    # 3D L=16, 16 layers, C=32, BF16: sampling at batch 4096
    f16 = fl.Flow(3, 16, 16, 32, lfs.LFS_BF16_CONV, params=p16)
    out["3d_L16_C32_sampling_bf16"] = sampling_rate(f16, 4096, -4.0, 5.0, batches=2)
    out["3d_L16_C32_forward_ms_b4096"] = round(flow_forward_ms(f16, 4096, reps=2), 3)
    return out


def trained_example(steps=20000):
    """The example parameter file's schedule (2D L=8, m2=-4, lambda=8, 16 layers, hidden 8,
    batch 64, Adam lr 1e-3, 200 x 100 iterations), trained once with the BF16 path and once
    with the plain FP32 path; MH acceptance and accepted configs/s of each trained flow,
    sampled in both precisions with the same weights."""
    import torch
    import seeded_inputs as si
    from paper_2208_08903_amd import flow as fl
    from paper_2208_08903_amd import lfs
    out = {"steps": steps, "batch": 64}
    for prec, name in ((lfs.LFS_BF16_CONV, "bf16"), (lfs.LFS_PLAIN_FP32, "fp32")):
        f = fl.Flow(2, 8, 16, 8, prec, params=si.flow_params(2, 16, 8))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr, hist = fl.train(f, steps, 64, -4.0, 8.0, lr=1e-3, record_every=steps // 4)
        torch.cuda.synchronize()
        tt = time.perf_counter() - t0
        row = {"train_s": round(tt, 3), "train_steps_per_s": round(steps / tt, 1),
               "loss": [(i, round(l, 4)) for i, l in hist]}
        for sp, sname in ((lfs.LFS_BF16_CONV, "bf16"), (lfs.LFS_PLAIN_FP32, "fp32")):
            acc, sec = fl.acceptance_rate(f.with_precision(sp), -4.0, 8.0, batches=16, B=4096)
            row[f"acceptance_sampled_{sname}"] = round(acc, 5)
            row[f"accepted_per_s_sampled_{sname}"] = round(acc * 16 * 4096 / sec, 1)
        if prec == lfs.LFS_BF16_CONV:
            # chain quality of the trained flow against HMC on the same theory (same GPU)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cq = fl.chain_quality(f, -4.0, 8.0, batches=16, B=4096)
            torch.cuda.synchronize()
            cq["seconds"] = round(time.perf_counter() - t0, 3)
            t0 = time.perf_counter()
            hq = fl.hmc_chain_quality(2, 8, -4.0, 8.0, n_chains=256, n_traj=2500)
            torch.cuda.synchronize()
            hq["seconds"] = round(time.perf_counter() - t0, 3)
            row["chain_quality"] = {"flow_mh": cq, "hmc": hq}
        out[f"trained_{name}"] = row
    return out


def trained_3d(steps=20000, B=256, w_std=0.02):
    """The 3D L=8 workload's flow (12 layers, C=16, m2=-4, lambda=5) trained to convergence
    at batch 256, Adam lr 1e-3, from N(0, 0.02^2) weights (at the workload's N(0, 0.1^2) the
    3D networks start deep in tanh saturation and the reverse-KL loss stays in the
    thousands with acceptance ~1e-3 after 60 000 steps), once with BF16 convolutions and
    once in plain FP32: loss and MH acceptance over training (4096-proposal batches), then
    for the BF16-trained flow the chain of 16 x 4096 proposals against FP64 HMC on the same
    theory: <M^2> and the zero-momentum two-point function C(t) with their errors."""
    import numpy as np
    import torch
    import seeded_inputs as si
    from paper_2208_08903_amd import flow as fl
    from paper_2208_08903_amd import lfs
    out = {"steps": steps, "batch": B, "lr": 1e-3, "w_std": w_std}
    marks = sorted({steps // 8, steps // 4, steps // 2, steps})
    for prec, name in ((lfs.LFS_BF16_CONV, "bf16"), (lfs.LFS_PLAIN_FP32, "fp32")):
        f = fl.Flow(3, 8, 12, 16, prec, params=si.flow_params(3, 12, 16, w_std=w_std))
        tr = fl.Trainer(f, B, -4.0, 5.0, lr=1e-3)
        hist, t_train, done = [], 0.0, 0
        for mk in marks:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while done < mk:
                tr.step()
                done += 1
            torch.cuda.synchronize()
            t_train += time.perf_counter() - t0
            acc, _ = fl.acceptance_rate(f, -4.0, 5.0, batches=2, B=4096)
            hist.append({"step": done, "loss": round(float(tr.loss.item()), 4), "acceptance": round(acc, 4)})
        row = {"train_s": round(t_train, 2), "train_steps_per_s": round(steps / t_train, 1), "history": hist}
        if prec == lfs.LFS_BF16_CONV:
            cq = fl.chain_quality(f, -4.0, 5.0, batches=16, B=4096)
            hq = fl.hmc_chain_quality(3, 8, -4.0, 5.0, n_chains=256, n_traj=1500)
            keep = ("acceptance", "tau_M", "n_indep_M", "ess", "M2_mean", "M2_err", "C_mean", "C_err")
            row["chain_quality"] = {"flow_mh": {k: cq[k] for k in keep},
                                    "hmc": {k: hq[k] for k in ("acceptance", "tau_M_mean", "M2_mean", "M2_err",
                                                                "C_mean", "C_err")}}
            d = np.abs(np.array(cq["C_mean"]) - np.array(hq["C_mean"]))
            sig = np.hypot(np.array(cq["C_err"]), np.array(hq["C_err"]))
            row["chain_quality"]["max_C_deviation_sigma"] = round(float(np.max(d / sig)), 3)
            row["chain_quality"]["M2_deviation_sigma"] = round(
                abs(cq["M2_mean"] - hq["M2_mean"]) / float(np.hypot(cq["M2_err"], hq["M2_err"])), 3)
        out[name] = row
        del tr, f
    return out


def serving(seconds=60.0, precision=None):
    """Poisson(200/s) sampling requests for `seconds` through the continuous-batching server
    (BF16 convolutions unless `precision` says otherwise), HBM budget 512 MB; peak admitted
    bytes (requests and group buffers) and peak device bytes of the run beside it."""
    import seeded_inputs as si
    from paper_2208_08903_amd import lfs
    from paper_2208_08903_amd.serve import DEFAULT_ARCH, Server, run_workload
    params = {d: si.flow_params(d, n, c, seed=2021 + d) for d, (n, c) in DEFAULT_ARCH.items()}
    reqs = si.serving_requests(seed=2208, rate=200.0, duration=seconds)
    prec = lfs.LFS_BF16_CONV if precision is None else precision
    srv = Server(params, precision=prec, hbm_budget=512 << 20)
    warm = si.serving_requests(seed=1, rate=200.0, duration=0.3)
    run_workload(srv, warm)
    srv.peak_used = 0
    srv.rounds = 0
    st = run_workload(srv, reqs)
    st["offered_rate_req_per_s"] = 200.0
    st["duration_s"] = seconds
    return st


def _oracle_gradient_seconds(args):
    """Process-pool worker: seconds the FP64 oracle (one BLAS thread) takes for the loss
    gradient of n samples of the workload."""
    dim, L, N, C, m2, lam, seed, n = args
    from threadpoolctl import threadpool_limits
    import seeded_inputs as si
    from oracle import flow as of
    fs = of.FlowShape(dim, L, N, C)
    p = si.flow_params(dim, N, C).astype("float64")
    z = si.normal_fields(seed, n, fs.V)
    with threadpool_limits(1):
        t = time.perf_counter()
        of.loss_gradient(p, z, fs, m2, lam)
        return time.perf_counter() - t


def cpu_baseline(w, target_s=10.0):
    """The FP64 oracle's training step (loss gradient + Adam) on a bounded sample of the
    batch, scaled to steps/s of the full batch (cost is linear in the batch: samples are
    independent): on all host cores (one oracle process per core, each on its own
    samples, one BLAS thread each), with the one-thread figure beside it."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    import seeded_inputs as si
    from oracle import adam as oadam
    key = (w["dim"], w["L"], w["n_layers"], w["hidden"], w["m2"], w["lam"])
    p = si.flow_params(w["dim"], w["n_layers"], w["hidden"]).astype(np.float64)
    with threadpool_limits(1):
        t = time.perf_counter()
        oadam.adam_step(p, np.ones_like(p), np.zeros_like(p), np.zeros_like(p), 1, lr=w["lr"])
        t_adam = time.perf_counter() - t
    t2 = _oracle_gradient_seconds((*key, 9, 2))
    b1 = int(max(2, min(128, round(2 * target_s / max(t2, 1e-3)))))
    tb = _oracle_gradient_seconds((*key, 9, b1))
    single = 1.0 / (tb / b1 * w["batch"] + t_adam)
    cores = len(os.sched_getaffinity(0))
    per = int(max(2, min(64, round(b1 * 0.8))))
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_gradient_seconds, [(*key, 9, 1)] * cores)       # imports done before timing
        t = time.perf_counter()
        pool.map(_oracle_gradient_seconds, [(*key, 100 + i, per) for i in range(cores)])
        wall = time.perf_counter() - t
    n = per * cores
    allc = 1.0 / (wall / n * w["batch"] + t_adam)
    return {"value": allc, "unit": "train steps/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle loss gradient on {n} of the {w['batch']} samples in {cores} processes "
                      f"({per} each, one BLAS thread each; {wall:.1f} s wall) plus one Adam step, "
                      "FP64 NumPy, scaled linearly to the full batch",
            "single_thread": {"value": single, "cores": 1,
                              "sample": f"{b1} samples in one thread ({tb:.1f} s) plus one Adam step"}}


def host_description():
    """CPU model, logical CPUs the process may use, and numpy's BLAS."""
    import numpy as np
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]["name"]
    except Exception:
        blas = "unknown"
    return {"cpu_model": model, "cpus_available": len(os.sched_getaffinity(0)), "numpy_blas": blas}


def oracle_timings():
    """The FP64 oracle, one thread, on the other workloads: the 2D L=8 example batch (forward,
    action, log-weights), a 2000-proposal MH chain, one HMC trajectory for 512 3D L=8 chains,
    and the 3D L=8 training step on a sample of its batch (scaled linearly)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import seeded_inputs as si
    from oracle import action as oa
    from oracle import flow as of
    from oracle import hmc as oh
    from oracle import mh as om
    out = {"host": host_description(), "threads": 1}
    with threadpool_limits(1):
        fs = of.FlowShape(2, 8, 16, 8)
        p = si.flow_params(2, 16, 8).astype(np.float64)
        z = si.normal_fields(3, 64, 64)
        t = time.perf_counter()
        f = of.flow_forward(p, z, fs)
        S = oa.action(f["phi"], -4.0, 8.0, 2)
        of.log_weights(S, f["logq"])
        out["2d_L8_batch64_forward_action_ms"] = round(1e3 * (time.perf_counter() - t), 2)
        lw, lu = si.logw_stream(4, 2000), si.log_uniforms(5, 2000)
        t = time.perf_counter()
        om.mh_chain(lw, lu)
        out["mh_chain_2000_ms"] = round(1e3 * (time.perf_counter() - t), 2)
        # the same start as the GPU figure (hmc_rate)
        phi = 0.5 * si.normal_fields(3, 512, 512).astype(np.float64).reshape(512, 8, 8, 8)
        pi = si.momenta(4, 512, 512)
        t = time.perf_counter()
        oh.hmc_step(phi, pi, si.log_uniforms(5, 512), -4.0, 5.0, 3, 10, 0.1)
        dt = time.perf_counter() - t
        out["hmc_3d_L8_512_chains_trajectories_per_s"] = round(512 / dt, 1)
        fs3 = of.FlowShape(3, 8, 12, 16)
        p3 = si.flow_params(3, 12, 16).astype(np.float64)
        b = 4
        z3 = si.normal_fields(9, b, 512)
        t = time.perf_counter()
        of.loss_gradient(p3, z3, fs3, -4.0, 5.0)
        dt = time.perf_counter() - t
        out["3d_L8_train_steps_per_s"] = round(b / (dt * 512), 5)
        out["3d_L8_train_sample"] = f"loss gradient on {b} of the 512 samples ({dt:.1f} s), scaled linearly"
    return out


def roofline_of(phase, fwd_ms, w, B, prec_name):
    """Dominant kernel of a training step and its rate against the matrix-core peak of its
    precision: the fused forward (one launch per call) or the per-layer backward launch
    (the backward phase's HIP-event time over its N launches; the fragment preparation,
    the last reduction and the tiny launches around them are in that time too, so this
    slightly understates the launch's own rate)."""
    fl_flops = algorithmic_flops_per_sample_layer(w["dim"], w["L"], w["hidden"])
    peak = PEAK["fp32_mfma_tflops"] if prec_name == "fp32" else PEAK["bf16_mfma_tflops"]
    if phase["backward"] > fwd_ms:
        name = ("flow_backward (per layer launch)" if w["dim"] == 2 else
                "flow_backward (per layer: kr_affine + kr_transpose + kr_wgrad)")
        ms = phase["backward"] / w["n_layers"]
        flops = 2 * fl_flops * B
        traffic = recorded_traffic(prec_name) if w is WORKLOAD else None
    else:
        name, ms, flops, traffic = "kf_forward (flow forward, all layers)", fwd_ms, fl_flops * w["n_layers"] * B, None
    achieved = flops / (ms * 1e-3) / 1e12
    return {"kernel": name, "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 5), "traffic": traffic,
            "flops_per_launch": flops, "ms_per_launch": round(ms, 5)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the side figures")
    ap.add_argument("--precision", choices=("both", "fp32", "bf16"), default="both",
                    help="which training steps to time (profiling runs time one)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default=WORKLOAD["workload"],
                    help="the training step to time (side figures run with the default only)")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="length of the Poisson arrival window of the BF16 serving figure")
    ap.add_argument("--serving-seconds-fp32", type=float, default=10.0,
                    help="the same for plain FP32 (which saturates at the offered load)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after the timed region, one device-to-device copy of this many MiB "
                         "(the known-size kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "every workload here is measured on a single GPU, and no multi-GPU figure is produced",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import seeded_inputs as si
    from paper_2208_08903_amd import flow as fl
    from paper_2208_08903_amd import lfs

    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    headline = w is WORKLOAD
    params = si.flow_params(w["dim"], w["n_layers"], w["hidden"])
    B = w["batch"]

    def make(prec):
        f = fl.Flow(w["dim"], w["L"], w["n_layers"], w["hidden"], prec, params=params)
        return f, fl.Trainer(f, B, w["m2"], w["lam"], lr=w["lr"])

    # the 3D L = 16 C = 32 workload has a BF16 backward only
    precs = [("fp32", lfs.LFS_PLAIN_FP32), ("bf16", lfs.LFS_BF16_CONV)]
    if args.precision != "both":
        precs = [p for p in precs if p[0] == args.precision]
    if w["dim"] == 3 and w["L"] == 16:
        precs = [p for p in precs if p[0] == "bf16"]
    runs = {}
    for name, prec in precs:
        flow, tr = make(prec)
        total, phase = time_phases(tr, args.steps, args.warmup)
        fwd_ms = flow_forward_ms(flow, B)
        runs[name] = {"steps_per_s": round(args.steps / total, 3), "ms_per_step": round(1000.0 * total / args.steps, 4),
                      "phases_ms": {k: round(v, 4) for k, v in phase.items()}, "forward_ms": round(fwd_ms, 4),
                      "loss_last": float(tr.loss.item()), "roofline": roofline_of(phase, fwd_ms, w, B, name)}
        del tr, flow
        _progress(f"{name} training steps timed")
    head_name = precs[0][0]
    head = runs[head_name]
    desc = "plain FP32" if head_name == "fp32" else "BF16 conv + FP64 sums"
    out = {
        "metric": f"train steps/s (reverse-KL, {desc})",
        "value": head["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": head_name, "data": "synthetic (seeded N(0,0.1) weights, Philox prior draws)",
        "config": {"workload": w["workload"], "dim": w["dim"], "L": w["L"], "m2": w["m2"],
                   "lambda": w["lam"], "n_layers": w["n_layers"], "hidden": w["hidden"],
                   "global_batch": B, "parallelism": "single GPU"},
        "phases_ms": head["phases_ms"],
        "loss_last": head["loss_last"],
        "roofline": head["roofline"],
    }
    for name, r in runs.items():
        if name != head_name:
            out[name] = r
    if "fp32" in runs and "bf16" in runs:
        out["bf16_speedup_vs_fp32"] = round(runs["bf16"]["steps_per_s"] / runs["fp32"]["steps_per_s"], 3)
    if headline and not args.no_extras:
        out["sampling_bf16"] = sampling_rate(fl.Flow(w["dim"], w["L"], w["n_layers"], w["hidden"],
                                                     lfs.LFS_BF16_CONV, params=params),
                                             B, w["m2"], w["lam"])
        out["sampling_fp32"] = sampling_rate(fl.Flow(w["dim"], w["L"], w["n_layers"], w["hidden"],
                                                     lfs.LFS_PLAIN_FP32, params=params),
                                             B, w["m2"], w["lam"], batches=4)
        _progress("sampling figures done")
        out["hmc_fp64_3d_L8"] = hmc_rate()
        out["hbm_kernels"] = hbm_kernels()
        out["other_workloads"] = other_workloads(params)
        out["chain_3d_L8_10k"] = chain_3d_L8_10k()
        _progress("other workloads done")
        out["general_networks_2d_L8"] = general_networks()
        out["trained_2d_L8_example"] = trained_example()
        _progress("trained example and chain quality done")
        out["trained_3d_L8"] = trained_3d()
        _progress("3D training and chain quality done")
        out["serving"] = serving(args.serving_seconds)
        _progress("serving (BF16) done")
        out["serving_fp32"] = serving(args.serving_seconds_fp32, lfs.LFS_PLAIN_FP32)
        _progress("serving (FP32) done")
    if args.copy_calibration_mb > 0:
        nb = args.copy_calibration_mb * 2 ** 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nb
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        _progress("oracle baseline done")
        if headline and not args.no_extras:
            out["oracle_timings"] = oracle_timings()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

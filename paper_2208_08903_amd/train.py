"""Training from a parameter file in the paper's layout (Sec. 2.1, example2d.toml):

    python -m paper_2208_08903_amd.train CONFIG.toml [--out DIR] [--device N] [--graph]

runs [training] epochs x iterations reverse-KL steps of the configured flow and
writes, after every epoch, one line of DIR/metrics.jsonl (epoch, step, loss of
the epoch's last batch, mean and standard deviation of its log-weights, the
independence-MH acceptance over that batch, steps/s) and DIR/checkpoint.npz.  A
[training] pretrained checkpoint resumes the run where it stopped (bit for bit:
the prior draws and the Adam step follow the step count).
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import config as cf
from . import lfs
from .flow import load_checkpoint, save_checkpoint


def _batch_metrics(tr, seed: int) -> dict:
    """log-weight statistics and the MH acceptance of one chain over the last batch."""
    w = tr.logw.cpu().numpy()
    u = np.random.default_rng(seed).random(tr.B)
    lu = torch.as_tensor(np.log(np.where(u == 0.0, np.nextafter(0.0, 1.0), u)).reshape(1, -1),
                         device=tr.logw.device)
    state = lfs.new_chain_state(1, tr.logw.device)
    cur = torch.empty(1, tr.B, dtype=torch.int64, device=tr.logw.device)
    lfs.mh_chain(tr.logw.view(1, -1), lu, state, cur)
    st = lfs.decode_chain_state(state)[0]
    return {"logw_mean": float(w.mean()), "logw_std": float(w.std()),
            "acceptance": st["n_acc"] / max(st["n_seen"] - 1, 1)}


def run(cfg: cf.RunConfig, out_dir: str, graph: bool = False, log=print) -> dict:
    os.makedirs(out_dir, exist_ok=True)
    torch.cuda.set_device(cfg.device.device_id)
    flow = cf.make_flow(cfg)
    tr = cf.make_trainer(cfg, flow, graph=graph)
    if cfg.training.pretrained:
        tr.load_state(load_checkpoint(cfg.training.pretrained))
    it = cfg.training.iterations
    first = tr.t // it
    if tr.t % it:
        raise cf.ConfigError(f"checkpoint at step {tr.t} is not at an epoch boundary of {it} iterations")
    metrics_path = os.path.join(out_dir, "metrics.jsonl")
    last = {}
    with open(metrics_path, "a") as mf:
        for epoch in range(first, cfg.training.epochs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(it):
                tr.step()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            last = {"epoch": epoch, "step": tr.t, "loss": float(tr.loss.item()),
                    **_batch_metrics(tr, cfg.training.seed + epoch), "steps_per_s": round(it / dt, 1)}
            mf.write(json.dumps(last) + "\n")
            mf.flush()
            save_checkpoint(os.path.join(out_dir, "checkpoint.npz"), tr)
            log(json.dumps(last))
    return last


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("config")
    ap.add_argument("--out", default="results")
    ap.add_argument("--device", type=int, default=None, help="override [device] device_id")
    ap.add_argument("--graph", action="store_true", help="replay each step's forward and backward from a HIP graph")
    args = ap.parse_args(argv)
    cfg = cf.load(args.config, device_id=args.device)
    run(cfg, args.out, graph=args.graph)


if __name__ == "__main__":
    main()

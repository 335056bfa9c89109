"""Training and sampling drivers over the HIP library.

PyTorch only provides device memory and the stream; every step of the path is
one of the library's entry points (see ``lfs``):

  train step (paper Sec. 1, reverse-KL training; example parameter file:
  Adam, lr 1e-3, fresh prior batch per iteration)
      prior_normal -> flow_forward (saving layer inputs; flow_forward_train also
      the second hidden activations) -> action (+force/B) -> log_weights (loss)
      -> flow_backward (flow_backward_saved) -> adam_step

  sampling (paper Sec. 1, flow proposals + Metropolis-Hastings test)
      prior_normal -> flow_forward -> action -> log_weights -> mh_chain

  chain quality (paper Sec. 1, N_indep = N / (2 tau_ac); Sec. 2.2, HMC "to
  compare results"): observables of every configuration, then autocorr over
  the chain (through the MH chain's current-configuration numbers) and ess.

A flow with batch norm (the example parameter file's use_bn) trains with batch
statistics, updating its running statistics (momentum 0.1) on every training
forward, and samples with the running statistics.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lfs


class Flow:
    """A flow architecture, its packed FP32 parameters on the device, and workspaces."""

    def __init__(self, dim, L, n_layers, hidden, precision=lfs.LFS_BF16_CONV, algo=lfs.ALGO_AUTO,
                 final_tanh=True, parity0=0, params=None, device="cuda", kernel=0, hidden_sizes=None,
                 batch_norm=False, bn_stats=None, bn_momentum=0.1):
        self.dim, self.L, self.n_layers, self.hidden = dim, L, n_layers, hidden
        self.kernel, self.hidden_sizes = kernel, hidden_sizes
        self.V = L ** dim
        self.precision = precision
        self.batch_norm, self.bn_momentum = bool(batch_norm), bn_momentum
        self.desc = lfs.make_desc(dim, L, n_layers, hidden, final_tanh, parity0, precision, algo,
                                  kernel, hidden_sizes, batch_norm)
        self.P = lfs.param_count(self.desc)
        if self.P == 0:
            raise lfs.LfsError("invalid flow description")
        self.bn_stats = None
        if self.batch_norm:
            # running statistics, per layer and hidden convolution mean[w] then var[w]
            widths = list(hidden_sizes) if hidden_sizes else [hidden, hidden]
            init = np.concatenate([np.concatenate([np.zeros(w), np.ones(w)]) for w in widths] * n_layers)
            if bn_stats is not None:
                init = np.asarray(bn_stats, np.float64).ravel()
            if init.size != lfs.bn_stats_count(self.desc):
                raise lfs.LfsError(f"expected {lfs.bn_stats_count(self.desc)} statistics, got {init.size}")
            self.bn_stats = torch.as_tensor(init.astype(np.float32)).to(device).contiguous()
        self.device = device
        if params is None:
            params = np.zeros(self.P, np.float32)
        params = torch.as_tensor(np.asarray(params, np.float32))
        if params.numel() != self.P:
            raise lfs.LfsError(f"expected {self.P} parameters, got {params.numel()}")
        self.params = params.to(device).contiguous()
        self._ws = {}

    def workspace(self, B, backward):
        key = (B, bool(backward))
        if key not in self._ws:
            n = max(lfs.workspace_bytes(self.desc, B, backward), 1)
            self._ws[key] = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def with_precision(self, precision):
        f = Flow(self.dim, self.L, self.n_layers, self.hidden, precision, self.desc.algo,
                 bool(self.desc.final_tanh), self.desc.parity0, device=self.device,
                 kernel=self.kernel, hidden_sizes=self.hidden_sizes, batch_norm=self.batch_norm,
                 bn_momentum=self.bn_momentum)
        f.params = self.params
        f.bn_stats = self.bn_stats
        return f

    def forward(self, z, phi, logq, logdet=None, saved_x=None, ws=None, train=False):
        """phi = F^{-1}(z) and log q.  Batch norm: train=True normalises with the batch's
        statistics and updates the running ones; otherwise the running ones are used."""
        if not self.batch_norm:
            lfs.flow_forward(self.desc, self.params, z, phi, logq, logdet, saved_x, ws)
        elif train:
            lfs.flow_forward_bn(self.desc, self.params, z, phi, logq, lfs.BN_BATCH, self.bn_stats,
                                self.bn_momentum, logdet, saved_x, ws)
        else:
            lfs.flow_forward_bn(self.desc, self.params, z, phi, logq, lfs.BN_RUNNING, self.bn_stats,
                                0.0, logdet, saved_x, ws)

    def backward(self, saved_x, g_phi, g_logq, g_params, g_z=None, ws=None, train=True):
        """Vector-Jacobian product of `forward` (batch statistics when train=True)."""
        if not self.batch_norm:
            lfs.flow_backward(self.desc, self.params, saved_x, g_phi, g_logq, g_params, g_z, ws)
        else:
            lfs.flow_backward_bn(self.desc, self.params, saved_x, g_phi, g_logq, g_params,
                                 lfs.BN_BATCH if train else lfs.BN_RUNNING, self.bn_stats, g_z, ws)


def step_lr(gamma: float, every: int):
    """Step-decay schedule: lr_t = lr gamma^floor((t - 1) / every) for Adam step t >= 1."""
    return lambda lr, t: lr * gamma ** ((t - 1) // every)


def exp_lr(gamma: float):
    """Exponential schedule: lr_t = lr gamma^(t - 1)."""
    return lambda lr, t: lr * gamma ** (t - 1)


class Trainer:
    """Reverse-KL training on fresh prior batches; all buffers allocated once.

    lr_schedule (the example parameter file's lr_scheduler, empty there: a constant
    rate): None, or a function (base_lr, t) -> learning rate of Adam step t >= 1,
    e.g. step_lr or exp_lr.  It runs on the host and only sets the rate passed to
    the Adam kernel.

    graph: replay forward + action + loss + backward (every launch but the prior
    draw and the Adam step, whose counters change each step) as one captured HIP
    graph.  The first step runs them eagerly and captures them; buffers are fixed,
    so later steps replay the same launches on fresh prior draws.  For small
    shapes, where a step is launch-bound.

    save_h: the forward keeps every layer's second hidden activation for the
    backward, which then skips recomputing it (lfs.flow_forward_train and
    lfs.flow_backward_saved), on the shapes where lfs.saved_h_bytes is not 0;
    elsewhere, and with save_h=False, the backward recomputes it."""

    def __init__(self, flow: Flow, B: int, m2: float, lam: float, lr=1e-3, key=12345,
                 betas=(0.9, 0.999), eps=1e-8, lr_schedule=None, graph=False, save_h=True):
        self.flow, self.B = flow, B
        dev, V, N = flow.device, flow.V, flow.n_layers
        self.m2 = torch.tensor([m2], dtype=torch.float64, device=dev)
        self.lam = torch.tensor([lam], dtype=torch.float64, device=dev)
        self.lr, self.betas, self.eps, self.key = lr, betas, eps, key
        self.lr_schedule = lr_schedule
        f32, f64 = torch.float32, torch.float64
        self.z = torch.empty(B, V, dtype=f32, device=dev)
        self.phi = torch.empty(B, V, dtype=f32, device=dev)
        self.logq = torch.empty(B, dtype=f64, device=dev)
        self.saved = torch.empty((N + 1) * B * V, dtype=f32, device=dev)
        self.S = torch.empty(B, dtype=f64, device=dev)
        self.gphi = torch.empty(B, V, dtype=f32, device=dev)
        self.logw = torch.empty(B, dtype=f64, device=dev)
        self.loss = torch.zeros(1, dtype=f64, device=dev)
        self.gparams = torch.empty(flow.P, dtype=f32, device=dev)
        self.m = torch.zeros(flow.P, dtype=f32, device=dev)
        self.v = torch.zeros(flow.P, dtype=f32, device=dev)
        self.ws_f = flow.workspace(B, False)
        self.ws_b = flow.workspace(B, True)
        hb = lfs.saved_h_bytes(flow.desc, B) if save_h and not flow.batch_norm else 0
        self.saved_h = torch.empty(hb, dtype=torch.uint8, device=dev) if hb else None
        self.t = 0
        self.graph = graph
        self._graph = None

    # The four phases, separately callable so a caller can time them.
    def draw(self):
        lfs.prior_normal(self.key, self.t * self.B, self.z)

    def forward(self):
        f = self.flow
        if self.saved_h is not None:
            lfs.flow_forward_train(f.desc, f.params, self.z, self.phi, self.logq, self.saved,
                                   self.saved_h, None, self.ws_f)
        else:
            f.forward(self.z, self.phi, self.logq, None, self.saved, self.ws_f, train=True)
        lfs.action(f.dim, f.L, self.phi, self.m2, self.lam, self.S, self.gphi, 1.0 / self.B,
                   f.precision)
        lfs.log_weights(self.S, self.logq, self.logw, self.loss)

    def backward(self):
        f = self.flow
        if self.saved_h is not None:
            lfs.flow_backward_saved(f.desc, f.params, self.saved, self.saved_h, self.gphi, 1.0 / self.B,
                                    self.gparams, None, self.ws_b)
        else:
            f.backward(self.saved, self.gphi, 1.0 / self.B, self.gparams, None, self.ws_b)

    def current_lr(self, t=None):
        t = self.t if t is None else t
        return self.lr if self.lr_schedule is None else float(self.lr_schedule(self.lr, t))

    def update(self):
        self.t += 1
        lfs.adam_step(self.flow.params, self.gparams, self.m, self.v, self.current_lr(),
                      self.betas[0], self.betas[1], self.eps, self.t)

    def _forward_backward(self):
        if not self.graph:
            self.forward()
            self.backward()
        elif self._graph is None:
            self.forward()
            self.backward()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self.forward()
                self.backward()
            self._graph = g
        else:
            self._graph.replay()

    def step(self):
        self.draw()
        self._forward_backward()
        self.update()

    # Checkpoints: with counter-based prior draws and the Adam step count in the
    # state, a resumed run continues bit for bit.
    def state(self) -> dict:
        """Host copies of everything a resume needs: parameters, Adam moments, the step
        count, the prior key (and batch-norm running statistics)."""
        st = {"params": self.flow.params.cpu().numpy(), "adam_m": self.m.cpu().numpy(),
              "adam_v": self.v.cpu().numpy(), "step": np.int64(self.t), "key": np.int64(self.key),
              "batch": np.int64(self.B)}
        if self.flow.batch_norm:
            st["bn_stats"] = self.flow.bn_stats.cpu().numpy()
        return st

    def load_state(self, st: dict):
        """Restore a state() into this trainer's buffers (in place, so a captured graph
        stays valid)."""
        for name, dst in (("params", self.flow.params), ("adam_m", self.m), ("adam_v", self.v)):
            a = np.asarray(st[name], np.float32)
            if a.size != dst.numel():
                raise lfs.LfsError(f"checkpoint {name} has {a.size} entries, the flow needs {dst.numel()}")
            dst.copy_(torch.as_tensor(a.reshape(dst.shape)))
        if self.flow.batch_norm:
            if "bn_stats" not in st:
                raise lfs.LfsError("checkpoint has no batch-norm statistics")
            self.flow.bn_stats.copy_(torch.as_tensor(np.asarray(st["bn_stats"], np.float32)))
        if int(st["key"]) != self.key or int(st["batch"]) != self.B:
            raise lfs.LfsError("checkpoint was written with another prior key or batch size")
        self.t = int(st["step"])


def save_checkpoint(path: str, trainer: Trainer):
    np.savez(path, **trainer.state())


def load_checkpoint(path: str) -> dict:
    with np.load(path, allow_pickle=False) as f:
        return {k: f[k] for k in f.files}


class Sampler:
    """Flow proposals and one persistent independence-MH chain per sampler."""

    def __init__(self, flow: Flow, B: int, m2: float, lam: float, key=12345, n_chains=1):
        self.flow, self.B = flow, B
        dev, V = flow.device, flow.V
        f32, f64 = torch.float32, torch.float64
        if B % n_chains:
            raise lfs.LfsError("B must be a multiple of n_chains")
        self.n_chains = n_chains
        self.m2 = torch.tensor([m2], dtype=f64, device=dev)
        self.lam = torch.tensor([lam], dtype=f64, device=dev)
        self.key = key
        self.z = torch.empty(B, V, dtype=f32, device=dev)
        self.phi = torch.empty(B, V, dtype=f32, device=dev)
        self.logq = torch.empty(B, dtype=f64, device=dev)
        self.S = torch.empty(B, dtype=f64, device=dev)
        self.logw = torch.empty(B, dtype=f64, device=dev)
        self.state = lfs.new_chain_state(n_chains, dev)
        self.cur = torch.empty(n_chains, B // n_chains, dtype=torch.int64, device=dev)
        self.acc = torch.empty(n_chains, B // n_chains, dtype=torch.uint8, device=dev)
        self.ws = flow.workspace(B, False)
        self.batch = 0

    def step(self, log_u):
        """One batch of B proposals; log_u is a [n_chains, B/n_chains] FP64 device tensor."""
        f = self.flow
        lfs.prior_normal(self.key, self.batch * self.B, self.z)
        f.forward(self.z, self.phi, self.logq, None, None, self.ws)
        lfs.action(f.dim, f.L, self.phi, self.m2, self.lam, self.S, None, 1.0, f.precision)
        lfs.log_weights(self.S, self.logq, self.logw)
        lfs.mh_chain(self.logw.view(self.n_chains, -1), log_u, self.state, self.cur, self.acc)
        self.batch += 1

    def acceptance(self):
        st = lfs.decode_chain_state(self.state)
        acc = sum(s["n_acc"] for s in st)
        dec = sum(max(s["n_seen"] - 1, 0) for s in st)
        return acc / max(dec, 1), acc


def train(flow: Flow, steps: int, B: int, m2: float, lam: float, lr=1e-3, key=12345,
          record_every: int = 0):
    """Reverse-KL training for `steps` iterations (the example parameter file runs
    200 epochs x 100 iterations at batch 64, lr 1e-3).  Returns the trainer and the
    recorded (step, loss) pairs."""
    tr = Trainer(flow, B, m2, lam, lr=lr, key=key)
    hist = []
    for i in range(steps):
        tr.step()
        if record_every and (i % record_every == 0 or i == steps - 1):
            hist.append((i, float(tr.loss.item())))
    return tr, hist


def acceptance_rate(flow: Flow, m2: float, lam: float, batches: int, B: int, key=4242, u_seed=77):
    """MH acceptance of `batches` x B proposals with one chain; returns (rate, seconds)."""
    import time
    rng = np.random.default_rng(u_seed)
    u = rng.random((batches, 1, B))
    lu = torch.as_tensor(np.log(np.where(u == 0, np.nextafter(0, 1), u)), device=flow.device)
    smp = Sampler(flow, B, m2, lam, key=key)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(batches):
        smp.step(lu[k])
    torch.cuda.synchronize()
    return smp.acceptance()[0], time.perf_counter() - t0


def _log_u(rng, shape, device):
    u = rng.random(shape)
    return torch.as_tensor(np.log(np.where(u == 0, np.nextafter(0, 1), u)), device=device)


def _tau(x, w_max, c, index=None):
    """tau_ac, window, found, N_indep of each row of x (through index if given)."""
    S = x.shape[0]
    o = [torch.empty(S, dtype=torch.float64, device=x.device), torch.empty(S, dtype=torch.int32, device=x.device),
         torch.empty(S, dtype=torch.uint8, device=x.device), torch.empty(S, dtype=torch.float64, device=x.device)]
    lfs.autocorr(x, w_max, c, o[0], o[1], o[2], o[3], index=index)
    return [t.cpu().numpy() for t in o]


def chain_quality(flow: Flow, m2: float, lam: float, batches: int, B: int, w_max=2000, c=6.0,
                  key=4242, u_seed=78):
    """One independence-MH chain over batches x B flow proposals.  Along the chain:
    the integrated autocorrelation time (automatic window, factor c) of the
    condensate M and of the action S, N_indep = N / (2 tau); the chain average of
    M^2 with its error sqrt(2 tau var / N) (tau of the M^2 series) and likewise of
    the zero-momentum two-point function C(t), t = 0 .. L-1 (tau of each C(t)
    series); plus the acceptance and the normalised reweighting ESS of all
    proposals."""
    dev, n, L = flow.device, batches * B, flow.L
    f64 = torch.float64
    M = torch.empty(1, n, dtype=f64, device=dev)
    Ct = torch.empty(n, L, dtype=f64, device=dev)
    S = torch.empty(1, n, dtype=f64, device=dev)
    logw = torch.empty(1, n, dtype=f64, device=dev)
    cur = torch.empty(1, n, dtype=torch.int64, device=dev)
    lu = _log_u(np.random.default_rng(u_seed), (batches, 1, B), dev)
    smp = Sampler(flow, B, m2, lam, key=key)
    for k in range(batches):
        sl = slice(k * B, (k + 1) * B)
        smp.step(lu[k])
        lfs.observables(flow.dim, flow.L, smp.phi, M[0, sl], Ct[sl])
        S[0, sl].copy_(smp.S)
        logw[0, sl].copy_(smp.logw)
        cur[0, sl].copy_(smp.cur[0])
    tm, wm, fm, nm = _tau(M, w_max, c, index=cur)
    ts, ws, fs, ns = _tau(S, w_max, c, index=cur)
    # M^2 and C(t) along the chain (the chain's configurations picked on the host)
    idx = cur.cpu().numpy()[0]
    m2_chain = M.cpu().numpy()[0][idx] ** 2
    t2, _, _, _ = _tau(torch.as_tensor(m2_chain.reshape(1, -1), device=dev), w_max, c)
    c_chain = Ct.cpu().numpy()[idx]                                     # [n, L]
    tc, _, _, _ = _tau(torch.as_tensor(np.ascontiguousarray(c_chain.T), device=dev), w_max, c)
    c_err = np.sqrt(2.0 * np.maximum(np.nan_to_num(tc, nan=0.5), 0.5) * c_chain.var(axis=0) / n)
    e = torch.empty(1, dtype=f64, device=dev)
    lfs.ess(logw, e)
    return {"proposals": n, "acceptance": round(smp.acceptance()[0], 5),
            "tau_M": float(tm[0]), "window_M": int(wm[0]), "window_found_M": bool(fm[0]),
            "n_indep_M": float(nm[0]), "tau_S": float(ts[0]), "window_S": int(ws[0]),
            "window_found_S": bool(fs[0]), "n_indep_S": float(ns[0]), "ess": float(e.item()),
            "M2_mean": float(m2_chain.mean()),
            "M2_err": float(np.sqrt(2.0 * max(float(t2[0]), 0.5) * m2_chain.var() / n)),
            "C_mean": [float(v) for v in c_chain.mean(axis=0)], "C_err": [float(v) for v in c_err]}


def hmc_chain_quality(dim: int, L: int, m2: float, lam: float, n_chains: int, n_traj: int,
                      n_steps=10, dt=0.1, w_max=2000, c=6.0, seed=91):
    """n_chains independent HMC chains (FP64, n_steps leapfrog steps of dt per
    trajectory, fresh momenta each trajectory) from a cold start phi = 0; the
    first n_traj // 5 trajectories are discarded.  Per chain, the integrated
    autocorrelation time of M over the remaining trajectories; returns the chain
    means, the acceptance, and the averages of M^2 and of the zero-momentum
    two-point function C(t) with their errors from the spread of the per-chain
    averages."""
    import seeded_inputs as si
    dev, V, f64 = "cuda", L ** dim, torch.float64
    phi = torch.zeros(n_chains, V, dtype=f64, device=dev)
    m2t = torch.tensor([m2], dtype=f64, device=dev)
    lamt = torch.tensor([lam], dtype=f64, device=dev)
    dH = torch.empty(n_chains, dtype=f64, device=dev)
    acc = torch.empty(n_chains, dtype=torch.uint8, device=dev)
    therm = n_traj // 5
    n = n_traj - therm
    Mt = torch.empty(n, n_chains, dtype=f64, device=dev)
    Ct = torch.empty(n, n_chains, L, dtype=f64, device=dev)
    lu = _log_u(np.random.default_rng(seed), (n_traj, n_chains), dev)
    n_acc = torch.zeros(n_chains, dtype=torch.int64, device=dev)
    for k in range(n_traj):
        pi = torch.as_tensor(si.momenta(seed * 100003 + k, n_chains, V), device=dev)
        lfs.hmc_step(dim, L, phi, pi, lu[k], m2t, lamt, n_steps, dt, dH, acc)
        if k >= therm:
            lfs.observables(dim, L, phi, Mt[k - therm], Ct[k - therm])
            n_acc += acc
    tm, wm, fm, _ = _tau(Mt.t().contiguous(), w_max, c)
    per_chain = (Mt.cpu().numpy() ** 2).mean(axis=0)
    c_chain = Ct.cpu().numpy().mean(axis=0)                             # [n_chains, L]
    return {"chains": n_chains, "trajectories": n, "leapfrog_steps": n_steps, "dt": dt,
            "acceptance": float(n_acc.sum().item()) / (n * n_chains),
            "tau_M_mean": float(np.nanmean(tm)), "window_found_M": int(fm.sum()),
            "n_indep_M_per_chain_mean": float(np.nanmean(n / (2 * tm))),
            "M2_mean": float(per_chain.mean()), "M2_err": float(per_chain.std(ddof=1) / np.sqrt(n_chains)),
            "C_mean": [float(v) for v in c_chain.mean(axis=0)],
            "C_err": [float(v) for v in c_chain.std(axis=0, ddof=1) / np.sqrt(n_chains)]}

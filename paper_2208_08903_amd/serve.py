"""Continuous-batching sampling server over the HIP library.

A request asks for N flow proposals of a 2D or 3D phi^4 theory with its own
lattice size and couplings, corrected by an independence Metropolis-Hastings
chain (paper Sec. 1: flow proposals plus the MH test that makes the ensemble
exact).  The server

  * admits waiting requests in arrival order while their device memory (the
    request's proposals, log-weights and chain record) fits an HBM budget and a
    chain-state slot is free; a request larger than the whole budget is
    rejected;
  * in every scheduling round groups the live requests by (dim, L) and gives
    each group one batch made of a chunk of every live request of that shape,
    so requests that arrived while others were running join the next round;
  * runs each group's batch on its own HIP stream (default priority), so the
    groups overlap on the device: prior draw with per-request Philox streams ->
    fused flow forward -> action with per-sample couplings -> log-weights ->
    ragged MH over the requests' persistent chain states;
  * returns a request and frees its memory as soon as its last chunk is done;
  * cancels a request on demand between scheduling rounds (nothing of it is on
    the device then): a waiting one is dropped, a live one retired early with
    its memory and chain-state slot freed;
  * refuses new requests while max_waiting are queued (overload).

A sample's computation never depends on which batch it is in (per-sample
kernels, per-request random streams, per-request chains whose state persists
across chunks), so a request's result is the same alone and in any mix.

One flow per lattice dimension serves every L (the convolutions do not depend
on L): by default the 2D stack has 16 layers of 16 hidden channels and the 3D
stack 12 layers of 16 hidden channels, seeded random-init weights.
"""
from __future__ import annotations

import math
import time
from collections import defaultdict, deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lfs
from .flow import Flow

DEFAULT_ARCH = {2: (16, 16), 3: (12, 16)}  # dim -> (n_layers, hidden)


@dataclass
class Result:
    rid: int
    dim: int
    L: int
    n: int
    t_arrive: float
    t_admit: float
    t_done: float
    n_acc: int
    acceptance: float
    proposals: torch.Tensor   # [n, V] FP32, the flow proposals in order
    logw: torch.Tensor        # [n] FP64
    cur_idx: torch.Tensor     # [n] int64: proposal index of the chain's state after each step
    accepted: torch.Tensor    # [n] uint8

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


@dataclass
class _Live:
    req: object
    slot: int
    t_admit: float
    nbytes: int
    proposals: torch.Tensor
    logw: torch.Tensor
    cur: torch.Tensor
    acc: torch.Tensor
    log_u: np.ndarray
    done: int = 0

    @property
    def remaining(self) -> int:
        return self.req.n_samples - self.done


def request_bytes(dim: int, L: int, n: int) -> int:
    """Device bytes a request holds while live: proposals (FP32), log-weights (FP64),
    chain indices (int64) and accept flags (uint8)."""
    return n * (L ** dim * 4 + 8 + 8 + 1)


def plan_admission(waiting, used: int, budget: int, free_slots: int):
    """Arrival-order admission: returns (admit, reject) lists of requests.  Stops at the
    first request that does not fit (no overtaking); rejects requests that can never fit."""
    admit, reject = [], []
    for r in waiting:
        need = request_bytes(r.dim, r.L, r.n_samples)
        if need > budget:
            reject.append(r)
            continue
        if free_slots <= len(admit) or used + need > budget:
            break
        admit.append(r)
        used += need
    return admit, reject


def plan_chunks(remaining, max_batch: int, quantum: int):
    """Chunk sizes for one round of a group: every live request (in order) gets up to
    `quantum` proposals while the batch has room; returns a list of (index, n)."""
    out, room = [], max_batch
    for i, rem in enumerate(remaining):
        if room <= 0:
            break
        n = min(rem, quantum, room)
        if n > 0:
            out.append((i, n))
            room -= n
    return out


class Server:
    def __init__(self, params_by_dim: dict, arch: dict | None = None,
                 precision=lfs.LFS_BF16_CONV, hbm_budget: int = 512 << 20, quantum: int = 2048,
                 max_batch: int = 8192, max_batch_sites: int = 8 << 20, max_live: int = 256,
                 max_waiting: int = 1 << 16, device="cuda", clock=time.perf_counter):
        self.arch = dict(DEFAULT_ARCH if arch is None else arch)
        self.precision = precision
        self.budget, self.quantum, self.max_batch, self.max_live = hbm_budget, quantum, max_batch, max_live
        self.max_waiting = max_waiting
        self.max_batch_sites = max_batch_sites
        self.device, self.clock = device, clock
        self.params = {d: torch.as_tensor(np.asarray(p, np.float32)).to(device)
                       for d, p in params_by_dim.items()}
        self.states = lfs.new_chain_state(max_live, device)
        self.free_slots = list(range(max_live))
        self.waiting: deque = deque()
        self.live: list[_Live] = []
        self.results: list[Result] = []
        self.rejected: list = []
        self.cancelled: list = []   # (rid, proposals decided before the cancellation)
        self.used = 0
        self.peak_used = 0
        self._groups = {}
        self.rounds = 0

    # -- per-shape resources -------------------------------------------------------
    def _group(self, dim, L):
        key = (dim, L)
        if key not in self._groups:
            n_layers, hidden = self.arch[dim]
            flow = Flow(dim, L, n_layers, hidden, self.precision, device=self.device)
            flow.params = self.params[dim]
            V = L ** dim
            Bm = max(1, min(self.max_batch, self.max_batch_sites // V))
            f32, f64, dev = torch.float32, torch.float64, self.device
            g = dict(flow=flow, stream=torch.cuda.Stream(device=dev), max_batch=Bm,
                     z=torch.empty(Bm, V, dtype=f32, device=dev),
                     phi=torch.empty(Bm, V, dtype=f32, device=dev),
                     logq=torch.empty(Bm, dtype=f64, device=dev),
                     S=torch.empty(Bm, dtype=f64, device=dev),
                     logw=torch.empty(Bm, dtype=f64, device=dev),
                     cur=torch.empty(Bm, dtype=torch.int64, device=dev),
                     acc=torch.empty(Bm, dtype=torch.uint8, device=dev),
                     ws=flow.workspace(Bm, False))
            self._groups[key] = g
        return self._groups[key]

    # -- request flow ---------------------------------------------------------------
    def submit(self, req) -> bool:
        """Queue a request; False (and the request is counted as rejected) when the
        waiting queue already holds max_waiting requests."""
        if len(self.waiting) >= self.max_waiting:
            self.rejected.append(req)
            return False
        self.waiting.append(req)
        return True

    def _admit(self):
        admit, reject = plan_admission(list(self.waiting), self.used, self.budget, len(self.free_slots))
        for r in reject:
            self.waiting.remove(r)
            self.rejected.append(r)
        now = self.clock()
        for r in admit:
            self.waiting.remove(r)
            slot = self.free_slots.pop(0)
            n, V = r.n_samples, r.L ** r.dim
            dev = self.device
            st = self.states[slot * lfs.CHAIN_STATE_BYTES:(slot + 1) * lfs.CHAIN_STATE_BYTES]
            st.zero_()
            rng = np.random.default_rng(r.seed)
            u = rng.random(n)
            log_u = np.log(np.where(u == 0.0, np.nextafter(0.0, 1.0), u))
            nbytes = request_bytes(r.dim, r.L, n)
            self.live.append(_Live(
                req=r, slot=slot, t_admit=now, nbytes=nbytes,
                proposals=torch.empty(n, V, dtype=torch.float32, device=dev),
                logw=torch.empty(n, dtype=torch.float64, device=dev),
                cur=torch.empty(n, dtype=torch.int64, device=dev),
                acc=torch.empty(n, dtype=torch.uint8, device=dev),
                log_u=log_u))
            self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)

    def _launch_group(self, key, members):
        dim, L = key
        g = self._group(dim, L)
        chunks = plan_chunks([lv.remaining for lv in members], g["max_batch"], self.quantum)
        if not chunks:
            return []
        B = sum(n for _, n in chunks)
        keys = np.empty(B, np.int64)
        ctrs = np.empty(B, np.int64)
        m2 = np.empty(B)
        lam = np.empty(B)
        lu = np.empty(B)
        offs = np.zeros(len(chunks) + 1, np.int64)
        sidx = np.empty(len(chunks), np.int32)
        o = 0
        for c, (i, n) in enumerate(chunks):
            lv = members[i]
            r = lv.req
            keys[o:o + n] = r.seed
            ctrs[o:o + n] = lv.done + np.arange(n)
            m2[o:o + n], lam[o:o + n] = r.m2, r.lam
            lu[o:o + n] = lv.log_u[lv.done:lv.done + n]
            sidx[c] = lv.slot
            o += n
            offs[c + 1] = o
        dev = self.device
        flow = g["flow"]
        with torch.cuda.stream(g["stream"]):
            t_keys = torch.from_numpy(keys).to(dev)
            t_ctrs = torch.from_numpy(ctrs).to(dev)
            t_m2 = torch.from_numpy(m2).to(dev)
            t_lam = torch.from_numpy(lam).to(dev)
            t_lu = torch.from_numpy(lu).to(dev)
            t_off = torch.from_numpy(offs).to(dev)
            t_sidx = torch.from_numpy(sidx).to(dev)
            z, phi, logq, S, logw = (g["z"][:B], g["phi"][:B], g["logq"][:B], g["S"][:B],
                                     g["logw"][:B])
            lfs.prior_normal_streams(t_keys, t_ctrs, z)
            flow.forward(z, phi, logq, None, None, g["ws"])
            lfs.action(dim, L, phi, t_m2, t_lam, S, None, 1.0, self.precision)
            lfs.log_weights(S, logq, logw)
            lfs.mh_chain_ragged(t_off, logw, t_lu, self.states, t_sidx, g["cur"][:B], g["acc"][:B])
            for c, (i, n) in enumerate(chunks):
                lv = members[i]
                a, b = int(offs[c]), int(offs[c + 1])
                lv.proposals[lv.done:lv.done + n].copy_(phi[a:b])
                lv.logw[lv.done:lv.done + n].copy_(logw[a:b])
                lv.cur[lv.done:lv.done + n].copy_(g["cur"][a:b])
                lv.acc[lv.done:lv.done + n].copy_(g["acc"][a:b])
        return [(members[i], n) for i, n in chunks]

    def step(self):
        """One scheduling round: admit, launch every group, wait, retire finished requests.
        Returns the number of proposals processed."""
        self._admit()
        groups = defaultdict(list)
        for lv in self.live:
            if lv.remaining > 0:
                groups[(lv.req.dim, lv.req.L)].append(lv)
        launched = []
        producer = torch.cuda.current_stream()   # chain-state slots were zeroed on this stream
        for key in sorted(groups):
            self._group(*key)["stream"].wait_stream(producer)
            launched += self._launch_group(key, groups[key])
        for g in self._groups.values():
            g["stream"].synchronize()
        done_n = 0
        for lv, n in launched:
            lv.done += n
            done_n += n
        now = self.clock()
        still = []
        finished = [lv for lv in self.live if lv.remaining == 0]
        if finished:
            st = lfs.decode_chain_state(self.states)
        for lv in self.live:
            if lv.remaining > 0:
                still.append(lv)
                continue
            s = st[lv.slot]
            r = lv.req
            self.results.append(Result(
                rid=r.rid, dim=r.dim, L=r.L, n=r.n_samples, t_arrive=r.t_arrive, t_admit=lv.t_admit,
                t_done=now, n_acc=s["n_acc"], acceptance=s["n_acc"] / max(s["n_seen"] - 1, 1),
                proposals=lv.proposals, logw=lv.logw, cur_idx=lv.cur, accepted=lv.acc))
            self.used -= lv.nbytes
            self.free_slots.append(lv.slot)
        self.live = still
        self.rounds += 1
        return done_n

    def cancel(self, rid) -> bool:
        """Withdraw request `rid` (call between steps; step() has finished all device
        work by the time it returns).  Returns False if it is not waiting or live."""
        for r in self.waiting:
            if r.rid == rid:
                self.waiting.remove(r)
                self.cancelled.append((rid, 0))
                return True
        for lv in self.live:
            if lv.req.rid == rid:
                self.live.remove(lv)
                self.used -= lv.nbytes
                self.free_slots.append(lv.slot)
                self.cancelled.append((rid, lv.done))
                return True
        return False

    def idle(self) -> bool:
        return not self.live and not self.waiting


def run_workload(server: Server, requests, time_scale: float = 1.0, keep_results: bool = False):
    """Feed requests at their arrival times (seconds after start, scaled by time_scale)
    into the server until all are done; returns summary statistics."""
    start = server.clock()
    pending = deque(sorted(requests, key=lambda r: r.t_arrive))
    t0 = time.perf_counter()
    n_prop = 0
    while pending or not server.idle():
        now = server.clock() - start
        while pending and pending[0].t_arrive * time_scale <= now:
            r = pending.popleft()
            server.submit(_shifted(r, start, time_scale))
        if server.idle():
            if pending:
                wait = pending[0].t_arrive * time_scale - (server.clock() - start)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
            continue
        n_prop += server.step()
    wall = time.perf_counter() - t0
    res = server.results
    lat = np.array([r.latency for r in res]) if res else np.zeros(1)
    n_acc = sum(r.n_acc for r in res)
    out = dict(requests=len(res), rejected=len(server.rejected), proposals=n_prop, wall_s=wall,
               proposals_per_s=n_prop / wall, accepted_per_s=n_acc / wall,
               acceptance=n_acc / max(sum(max(r.n - 1, 1) for r in res), 1),
               p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
               mean_latency_s=float(lat.mean()), rounds=server.rounds,
               peak_admitted_bytes=server.peak_used, hbm_budget_bytes=server.budget)
    if not keep_results:
        server.results = []
    return out


def _shifted(r, start, scale):
    """The request with its arrival time on the server clock."""
    from dataclasses import replace
    return replace(r, t_arrive=start + r.t_arrive * scale)

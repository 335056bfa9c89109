"""Continuous-batching sampling server over the HIP library.

A request asks for N flow proposals of a 2D or 3D phi^4 theory with its own
lattice size and couplings, corrected by an independence Metropolis-Hastings
chain (paper Sec. 1: flow proposals plus the MH test that makes the ensemble
exact).  The server

  * admits waiting requests in arrival order while their device memory fits an
    HBM budget and a chain-state slot is free; the budget counts the request's
    own buffers (its proposals, log-weights and chain record) and the buffers of
    the (dim, L) group it joins (batch fields, per-sample staging, the flow
    workspace), which are reserved when the group is created and given back
    when an idle group's room is needed; a request larger than the whole budget
    is rejected;
  * keeps at most one batch in flight per (dim, L) group, on the group's own HIP
    stream (default priority), so the groups overlap on the device: prior draw
    with per-request Philox streams -> fused flow forward -> action with
    per-sample couplings -> log-weights -> ragged MH over the requests' persistent
    chain states.  Each call of step() retires the groups whose batch has
    finished, admits, and launches the next batch of every idle group, made of a
    chunk of every live request of that shape -- so a request that arrives while
    other groups are busy starts as soon as its own group is free, not when the
    whole round ends;
  * stages a batch's per-sample keys, counters, couplings and log u in pinned
    host buffers and copies them asynchronously on the group's stream;
  * returns a request and frees its memory as soon as its last chunk is done;
  * cancels a request on demand (its group's batch in flight is finished first):
    a waiting one is dropped, a live one retired early with its memory and
    chain-state slot freed;
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


STAGE_BYTES_PER_SAMPLE = 5 * 8 + 8 + 4  # keys, counters, m2, lambda, log u; offsets; state index


def group_bytes(V: int, batch: int, ws_bytes: int) -> int:
    """Device bytes of a (dim, L) group: its batch's z and phi (FP32), log q, S and log w
    (FP64), chain indices and accept flags, the per-sample staging copies, and the flow
    workspace."""
    return batch * (2 * V * 4 + 3 * 8 + 8 + 1 + STAGE_BYTES_PER_SAMPLE) + 8 + ws_bytes


def plan_admission(waiting, used: int, budget: int, free_slots: int, extra=None):
    """Arrival-order admission: returns (admit, reject) lists of requests.  Stops at the
    first request that does not fit (no overtaking); rejects requests that can never fit.
    extra(r) gives further bytes a request brings with it (a group that must be created
    for it); it is charged once per shape."""
    admit, reject = [], []
    charged = set()
    for r in waiting:
        more = 0
        key = (r.dim, r.L)
        if extra is not None and key not in charged:
            more = extra(r)
        need = request_bytes(r.dim, r.L, r.n_samples) + more
        if need > budget:
            reject.append(r)
            continue
        if free_slots <= len(admit) or used + need > budget:
            break
        admit.append(r)
        used += need
        charged.add(key)
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
                 max_batch: int = 8192, max_batch_sites: int = 2 << 20, max_live: int = 256,
                 max_waiting: int = 1 << 16, group_share: float = 0.25, device="cuda",
                 clock=time.perf_counter):
        self.arch = dict(DEFAULT_ARCH if arch is None else arch)
        self.group_share = group_share
        self.precision = precision
        self.budget, self.quantum, self.max_batch, self.max_live = hbm_budget, quantum, max_batch, max_live
        self.max_waiting = max_waiting
        self.max_batch_sites = max_batch_sites
        self.device, self.clock = device, clock
        self.params = {d: torch.as_tensor(np.asarray(p, np.float32)).to(device)
                       for d, p in params_by_dim.items()}
        self._flows = {}
        self._gbatch = {}
        self.states = lfs.new_chain_state(max_live, device)
        self.free_slots = list(range(max_live))
        self.waiting: deque = deque()
        self.live: list[_Live] = []
        self.results: list[Result] = []
        self.rejected: list = []
        self.cancelled: list = []   # (rid, proposals decided before the cancellation)
        self.used = 0               # bytes of live requests
        self.reserved = 0           # bytes of the groups' buffers
        self.peak_used = 0          # largest used + reserved
        self._groups = {}
        self.rounds = 0             # batches launched (over all groups)

    # -- per-shape resources -------------------------------------------------------
    def _flow(self, dim, L):
        key = (dim, L)
        if key not in self._flows:
            n_layers, hidden = self.arch[dim]
            f = Flow(dim, L, n_layers, hidden, self.precision, device=self.device)
            f.params = self.params[dim]
            self._flows[key] = f
        return self._flows[key]

    def _group_bytes_at(self, dim, L, Bm):
        return group_bytes(L ** dim, Bm, lfs.workspace_bytes(self._flow(dim, L).desc, Bm, False))

    def _group_batch(self, dim, L):
        """A group's batch: max_batch samples or max_batch_sites sites, halved while the
        group's buffers would take more than group_share of the budget (shapes whose
        kernels keep hidden activations in the workspace)."""
        key = (dim, L)
        if key not in self._gbatch:
            Bm = max(1, min(self.max_batch, self.max_batch_sites // L ** dim))
            while Bm > 1 and self._group_bytes_at(dim, L, Bm) > self.group_share * self.budget:
                Bm //= 2
            self._gbatch[key] = Bm
        return self._gbatch[key]

    def _group_need(self, dim, L):
        return self._group_bytes_at(dim, L, self._group_batch(dim, L))

    def _group(self, dim, L):
        key = (dim, L)
        if key not in self._groups:
            flow = self._flow(dim, L)
            V = L ** dim
            Bm = self._group_batch(dim, L)
            f32, f64, i64, dev = torch.float32, torch.float64, torch.int64, self.device

            def pinned(n, dt):
                return torch.empty(n, dtype=dt, pin_memory=True)

            g = dict(flow=flow, stream=torch.cuda.Stream(device=dev), max_batch=Bm,
                     z=torch.empty(Bm, V, dtype=f32, device=dev),
                     phi=torch.empty(Bm, V, dtype=f32, device=dev),
                     logq=torch.empty(Bm, dtype=f64, device=dev),
                     S=torch.empty(Bm, dtype=f64, device=dev),
                     logw=torch.empty(Bm, dtype=f64, device=dev),
                     cur=torch.empty(Bm, dtype=i64, device=dev),
                     acc=torch.empty(Bm, dtype=torch.uint8, device=dev),
                     ws=flow.workspace(Bm, False),
                     # staging: pinned host buffers and their device copies
                     h_keys=pinned(Bm, i64), h_ctrs=pinned(Bm, i64), h_m2=pinned(Bm, f64),
                     h_lam=pinned(Bm, f64), h_lu=pinned(Bm, f64), h_off=pinned(Bm + 1, i64),
                     h_sidx=pinned(Bm, torch.int32),
                     keys=torch.empty(Bm, dtype=i64, device=dev), ctrs=torch.empty(Bm, dtype=i64, device=dev),
                     m2=torch.empty(Bm, dtype=f64, device=dev), lam=torch.empty(Bm, dtype=f64, device=dev),
                     lu=torch.empty(Bm, dtype=f64, device=dev), off=torch.empty(Bm + 1, dtype=i64, device=dev),
                     sidx=torch.empty(Bm, dtype=torch.int32, device=dev),
                     nbytes=self._group_need(dim, L), inflight=None, event=None)
            self.reserved += g["nbytes"]
            self._groups[key] = g
        return self._groups[key]

    def _release_idle_groups(self, keep=()):
        """Give back the buffers of groups with no live request and nothing in flight."""
        busy = {(lv.req.dim, lv.req.L) for lv in self.live}
        for key in [k for k, g in self._groups.items()
                    if k not in busy and k not in keep and g["inflight"] is None]:
            self.reserved -= self._groups.pop(key)["nbytes"]

    # -- request flow ---------------------------------------------------------------
    def submit(self, req) -> bool:
        """Queue a request; False (and the request is counted as rejected) when the
        waiting queue already holds max_waiting requests."""
        if len(self.waiting) >= self.max_waiting:
            self.rejected.append(req)
            return False
        self.waiting.append(req)
        return True

    def _plan(self):
        extra = lambda r: 0 if (r.dim, r.L) in self._groups else self._group_need(r.dim, r.L)  # noqa: E731
        return plan_admission(list(self.waiting), self.used + self.reserved, self.budget,
                              len(self.free_slots), extra)

    def _admit(self):
        admit, reject = self._plan()
        if not admit and self.waiting and self.waiting[0] not in reject and self._groups:
            # the head does not fit: give back the buffers of idle groups and try again
            self._release_idle_groups()
            admit, reject = self._plan()
        for r in reject:
            self.waiting.remove(r)
            self.rejected.append(r)
        now = self.clock()
        for r in admit:
            self.waiting.remove(r)
            self._group(r.dim, r.L)
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
        self.peak_used = max(self.peak_used, self.used + self.reserved)

    def _launch_group(self, key, members):
        dim, L = key
        g = self._group(dim, L)
        chunks = plan_chunks([lv.remaining for lv in members], g["max_batch"], self.quantum)
        if not chunks:
            return False
        B = sum(n for _, n in chunks)
        keys, ctrs = g["h_keys"].numpy(), g["h_ctrs"].numpy()
        m2, lam, lu = g["h_m2"].numpy(), g["h_lam"].numpy(), g["h_lu"].numpy()
        offs, sidx = g["h_off"].numpy(), g["h_sidx"].numpy()
        offs[0] = 0
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
        nc = len(chunks)
        flow = g["flow"]
        with torch.cuda.stream(g["stream"]):
            for name, n in (("keys", B), ("ctrs", B), ("m2", B), ("lam", B), ("lu", B), ("off", nc + 1),
                            ("sidx", nc)):
                g[name][:n].copy_(g["h_" + name][:n], non_blocking=True)
            z, phi, logq, S, logw = (g["z"][:B], g["phi"][:B], g["logq"][:B], g["S"][:B],
                                     g["logw"][:B])
            lfs.prior_normal_streams(g["keys"][:B], g["ctrs"][:B], z)
            flow.forward(z, phi, logq, None, None, g["ws"])
            lfs.action(dim, L, phi, g["m2"][:B], g["lam"][:B], S, None, 1.0, self.precision)
            lfs.log_weights(S, logq, logw)
            lfs.mh_chain_ragged(g["off"][:nc + 1], logw, g["lu"][:B], self.states, g["sidx"][:nc],
                                g["cur"][:B], g["acc"][:B])
            for c, (i, n) in enumerate(chunks):
                lv = members[i]
                a, b = int(offs[c]), int(offs[c + 1])
                lv.proposals[lv.done:lv.done + n].copy_(phi[a:b])
                lv.logw[lv.done:lv.done + n].copy_(logw[a:b])
                lv.cur[lv.done:lv.done + n].copy_(g["cur"][a:b])
                lv.acc[lv.done:lv.done + n].copy_(g["acc"][a:b])
            ev = torch.cuda.Event()
            ev.record()
        g["inflight"] = [(members[i], n) for i, n in chunks]
        g["event"] = ev
        g["seq"] = self.rounds
        self.rounds += 1
        return True

    def _complete(self, g):
        """Account a group's finished batch and retire the requests it completed."""
        done_n = 0
        for lv, n in g["inflight"]:
            lv.done += n
            done_n += n
        g["inflight"], g["event"] = None, None
        now = self.clock()
        still = []
        for lv in self.live:
            if lv.remaining > 0:
                still.append(lv)
                continue
            st = lfs.decode_chain_state(
                self.states[lv.slot * lfs.CHAIN_STATE_BYTES:(lv.slot + 1) * lfs.CHAIN_STATE_BYTES])[0]
            r = lv.req
            self.results.append(Result(
                rid=r.rid, dim=r.dim, L=r.L, n=r.n_samples, t_arrive=r.t_arrive, t_admit=lv.t_admit,
                t_done=now, n_acc=st["n_acc"], acceptance=st["n_acc"] / max(st["n_seen"] - 1, 1),
                proposals=lv.proposals, logw=lv.logw, cur_idx=lv.cur, accepted=lv.acc))
            self.used -= lv.nbytes
            self.free_slots.append(lv.slot)
        self.live = still
        return done_n

    def _members(self):
        groups = defaultdict(list)
        for lv in self.live:
            if lv.remaining > 0:
                groups[(lv.req.dim, lv.req.L)].append(lv)
        return groups

    def step(self):
        """One scheduling pass: retire the groups whose batch has finished, admit waiting
        requests, and launch the next batch of every idle group that has work.  When
        nothing could be retired or launched it waits for the oldest batch in flight.
        Returns the number of proposals whose batch finished during the call."""
        done_n = 0
        for g in self._groups.values():
            if g["inflight"] is not None and g["event"].query():
                done_n += self._complete(g)
        self._admit()
        launched = False
        producer = torch.cuda.current_stream()   # chain-state slots were zeroed on this stream
        members = self._members()
        for key in sorted(members):
            g = self._group(*key)
            if g["inflight"] is None:
                g["stream"].wait_stream(producer)
                launched |= self._launch_group(key, members[key])
        if not launched and done_n == 0:
            busy = [g for g in self._groups.values() if g["inflight"] is not None]
            if busy:
                g = min(busy, key=lambda x: x["seq"])
                g["event"].synchronize()
                done_n += self._complete(g)
        return done_n

    def cancel(self, rid) -> bool:
        """Withdraw request `rid`: a waiting one is dropped; a live one is retired early
        (its group's batch in flight, if any, is finished first, so nothing of it is on the
        device any more).  Returns False if it is not waiting or live."""
        for r in self.waiting:
            if r.rid == rid:
                self.waiting.remove(r)
                self.cancelled.append((rid, 0))
                return True
        for lv in self.live:
            if lv.req.rid == rid:
                g = self._groups.get((lv.req.dim, lv.req.L))
                if g is not None and g["inflight"] is not None:
                    g["event"].synchronize()
                    self._complete(g)
                if lv not in self.live:          # that batch completed it
                    return False
                self.live.remove(lv)
                self.used -= lv.nbytes
                self.free_slots.append(lv.slot)
                self.cancelled.append((rid, lv.done))
                return True
        return False

    def drain(self):
        """Finish every batch in flight (no new launches)."""
        for g in self._groups.values():
            if g["inflight"] is not None:
                g["event"].synchronize()
                self._complete(g)

    def idle(self) -> bool:
        return not self.live and not self.waiting


def run_workload(server: Server, requests, time_scale: float = 1.0, keep_results: bool = False):
    """Feed requests at their arrival times (seconds after start, scaled by time_scale)
    into the server until all are done; returns summary statistics.  Finished results
    are handed over (dropped) as they come unless keep_results, so the device memory
    of the run is the server's own working set; peak_device_bytes is torch's peak of
    allocated device memory during the run (everything the process holds, the server's
    flows, chain states, groups and live requests included), device_bytes_at_start what
    was allocated when it began."""
    start = server.clock()
    pending = deque(sorted(requests, key=lambda r: r.t_arrive))
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    n_prop = 0
    lat, n_acc, n_dec, kept = [], 0, 0, []

    def collect():
        nonlocal n_acc, n_dec
        for r in server.results:
            lat.append(r.latency)
            n_acc += r.n_acc
            n_dec += max(r.n - 1, 1)
        if keep_results:
            kept.extend(server.results)
        server.results = []

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
        collect()
    server.drain()
    collect()
    wall = time.perf_counter() - t0
    peak_device = torch.cuda.max_memory_allocated()
    server.results = kept
    lat = np.array(lat) if lat else np.zeros(1)
    out = dict(requests=len(lat), rejected=len(server.rejected), proposals=n_prop, wall_s=wall,
               proposals_per_s=n_prop / wall, accepted_per_s=n_acc / wall,
               acceptance=n_acc / max(n_dec, 1),
               p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
               mean_latency_s=float(lat.mean()), rounds=server.rounds,
               peak_admitted_bytes=server.peak_used, hbm_budget_bytes=server.budget,
               peak_device_bytes=int(peak_device), device_bytes_at_start=int(base))
    return out


def _shifted(r, start, scale):
    """The request with its arrival time on the server clock."""
    from dataclasses import replace
    return replace(r, t_arrive=start + r.t_arrive * scale)

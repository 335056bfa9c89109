"""Serving loop on the GPU: identity of a request's result alone and in a mix,
memory admission (request and group buffers within the budget), and oracle
checks of the served proposals and chain decisions in both precisions."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from oracle import action as oa
from oracle import flow as of
from oracle import mh as omh
from oracle import prior as op
from paper_2208_08903_amd import lfs
from paper_2208_08903_amd.serve import Server, request_bytes, run_workload

from .test_gpu_parity import _check_forward_bf16

pytestmark = pytest.mark.gpu

ARCH = {2: (4, 16), 3: (3, 16)}


def params():
    return {d: si.flow_params(d, n, c, seed=2021 + d, w_std=0.1) for d, (n, c) in ARCH.items()}


def req(rid, dim, L, n, seed, m2=-4.0, lam=6.0, t=0.0):
    return si.Request(rid, t, dim, L, m2, lam, n, seed)


def serve_all(reqs, **kw):
    srv = Server(params(), arch=ARCH, **kw)
    for r in reqs:
        srv.submit(r)
    while not srv.idle():
        srv.step()
    torch.cuda.synchronize()
    return srv, {r.rid: r for r in srv.results}


def test_result_same_alone_and_in_mix():
    target = req(0, 2, 16, 700, seed=99, m2=-4.2, lam=7.5)
    others = [req(1, 3, 8, 300, 5), req(2, 2, 16, 2500, 6, -3.7, 4.4), req(3, 2, 8, 90, 7),
              req(4, 3, 12, 64, 8), req(5, 2, 16, 1, 9)]
    _, alone = serve_all([target], quantum=256)
    _, mixed = serve_all(others[:2] + [target] + others[2:], quantum=100, max_batch=1000)
    a, b = alone[0], mixed[0]
    for f in ("proposals", "logw", "cur_idx", "accepted"):
        np.testing.assert_array_equal(getattr(a, f).cpu().numpy(), getattr(b, f).cpu().numpy())
    assert a.n_acc == b.n_acc
    assert len(mixed) == 6


def group_need(*shapes, max_batch=512):
    """Bytes the server reserves for the groups of these (dim, L) shapes (group_share 1: the
    group batch is max_batch whatever the budget)."""
    probe = Server(params(), arch=ARCH, max_batch=max_batch, hbm_budget=1 << 40, group_share=1.0)
    return sum(probe._group_need(d, L) for d, L in shapes)


def test_admission_waits_for_memory():
    big = request_bytes(2, 16, 3000)
    budget = int(1.5 * big) + group_need((2, 16), (2, 8))
    reqs = [req(0, 2, 16, 3000, 1), req(1, 2, 16, 3000, 2), req(2, 2, 8, 100, 3)]
    srv, res = serve_all(reqs, hbm_budget=budget, quantum=512, max_batch=512, group_share=1.0)
    assert res[1].t_admit >= res[0].t_done          # had to wait for the first to finish
    assert res[2].t_admit >= res[1].t_admit          # arrival order, no overtaking
    assert srv.peak_used <= budget and srv.used == 0
    assert srv.reserved == group_need(*srv._groups)  # the groups' buffers are counted


def test_group_buffers_count_against_the_budget():
    """A request whose group does not exist yet is admitted only with room for the group's
    buffers; idle groups give their room back when the head of the queue needs it."""
    g16, g8 = group_need((2, 16)), group_need((2, 8))
    r16 = request_bytes(2, 16, 300)
    srv = Server(params(), arch=ARCH, max_batch=512, quantum=128, hbm_budget=g16 + r16 + 1000, group_share=1.0)
    srv.submit(req(0, 2, 16, 300, 1))
    srv.submit(req(1, 2, 8, 300, 2))                 # its group does not fit next to the first
    srv.step()
    assert [lv.req.rid for lv in srv.live] == [0] and len(srv.waiting) == 1
    assert srv.used + srv.reserved <= srv.budget
    while not srv.idle():
        srv.step()
    torch.cuda.synchronize()
    assert sorted(r.rid for r in srv.results) == [0, 1]
    assert srv.peak_used <= srv.budget and g8 > 0


def test_oversized_request_rejected():
    srv, res = serve_all([req(0, 2, 8, 50, 1), req(1, 3, 16, 8192, 2)], hbm_budget=1 << 20, max_batch=256)
    assert list(res) == [0] and [r.rid for r in srv.rejected] == [1]


@pytest.mark.parametrize("precision", [lfs.LFS_BF16_CONV, lfs.LFS_PLAIN_FP32])
@pytest.mark.parametrize("dim,L", [(2, 16), (3, 8), (3, 16)])
def test_served_proposals_and_decisions_match_oracle(dim, L, precision):
    print(f"served proposals dim={dim} L={L} precision={precision}", flush=True)
    n = 40 if L < 16 or dim == 2 else 6
    r = req(0, dim, L, n, seed=1234, m2=-4.4, lam=5.5)
    _, res = serve_all([r], quantum=16, precision=precision)
    out = res[0]
    V = L ** dim
    z = op.prior_normal(1234, 0, n, V)                       # per-request Philox stream
    nl, c = ARCH[dim]
    fs = of.FlowShape(dim, L, nl, c)
    p64 = params()[dim].astype(np.float64)
    ref = of.flow_forward(p64, z, fs)
    phi = out.proposals.cpu().numpy().astype(np.float64)
    phio = ref["phi"].reshape(n, V)
    S = oa.action(phi.reshape((n,) + (L,) * dim), -4.4, 5.5, dim)
    w = out.logw.cpu().numpy()
    logq = -S - w                                            # the served log q, through log w
    if precision == lfs.LFS_BF16_CONV:
        # log q through the served log-weight and the FP64 action of the served proposal
        _check_forward_bf16(p64, z, fs, phi, logq, None, ref)
    else:
        assert np.all(np.abs(phi - phio) <= 1e-5 * (fs.T / 9) * (1 + np.abs(phio)))
        assert np.all(np.abs(logq - ref["logq"]) <= 1e-4 * V + 1e-4 * np.abs(S))
    u = np.random.default_rng(1234).random(n)
    co, ao, so = omh.mh_chain(w, np.log(u))
    np.testing.assert_array_equal(out.cur_idx.cpu().numpy(), co)
    np.testing.assert_array_equal(out.accepted.cpu().numpy(), ao)


def test_poisson_workload_runs():
    reqs = si.serving_requests(seed=2208, rate=200.0, duration=0.5, n_max=1024)
    assert {(r.dim, r.L) for r in reqs} == {(2, 8), (2, 16), (2, 32), (3, 8), (3, 12), (3, 16)}
    srv = Server(params(), arch=ARCH, hbm_budget=256 << 20)
    stats = run_workload(srv, reqs)
    assert stats["requests"] == len(reqs) and stats["rejected"] == 0
    assert stats["p99_latency_s"] >= stats["p50_latency_s"] > 0
    assert stats["peak_admitted_bytes"] <= 256 << 20


def test_cancellation_frees_memory_and_slot():
    """A waiting and a live request are cancelled between rounds: neither returns a
    result, their memory and chain slot come back, and a request that then takes the
    freed slot gives the same result as alone (its chain state starts from zero)."""
    late = req(9, 2, 16, 400, seed=31, m2=-3.9, lam=6.5)
    _, alone = serve_all([late], quantum=128)
    srv = Server(params(), arch=ARCH, quantum=128, max_live=2, max_batch=512, group_share=1.0,
                 hbm_budget=request_bytes(2, 16, 900) + request_bytes(2, 8, 600) + group_need((2, 16), (2, 8)))
    for r in (req(0, 2, 16, 900, 1), req(1, 2, 8, 600, 2), req(2, 3, 8, 50, 3)):
        srv.submit(r)
    srv.step()                                       # 0 and 1 live (two slots), 2 waiting; batches in flight
    assert [lv.req.rid for lv in srv.live] == [0, 1] and len(srv.waiting) == 1
    assert srv.cancel(2) and srv.cancel(0) and not srv.cancel(42)
    assert srv.used == request_bytes(2, 8, 600) and len(srv.free_slots) == 1
    srv.submit(late)                                 # takes the cancelled request's slot
    while not srv.idle():
        srv.step()
    torch.cuda.synchronize()
    res = {r.rid: r for r in srv.results}
    assert sorted(res) == [1, 9]
    assert [c[0] for c in srv.cancelled] == [2, 0] and srv.cancelled[1][1] == 128
    assert srv.used == 0 and sorted(srv.free_slots) == [0, 1]
    for f in ("proposals", "logw", "cur_idx", "accepted"):
        np.testing.assert_array_equal(getattr(res[9], f).cpu().numpy(), getattr(alone[9], f).cpu().numpy())


def test_queue_overflow_rejects():
    srv = Server(params(), arch=ARCH, max_waiting=2)
    assert srv.submit(req(0, 2, 8, 10, 1)) and srv.submit(req(1, 2, 8, 10, 2))
    assert not srv.submit(req(2, 2, 8, 10, 3))
    assert [r.rid for r in srv.rejected] == [2]
    while not srv.idle():
        srv.step()
    assert sorted(r.rid for r in srv.results) == [0, 1]
    assert srv.submit(req(3, 2, 8, 10, 4))           # room again once the queue drained

"""Host-side scheduling logic of the server (no GPU)."""
from dataclasses import dataclass

from paper_2208_08903_amd.serve import plan_admission, plan_chunks, request_bytes
import seeded_inputs as si


@dataclass
class R:
    dim: int
    L: int
    n_samples: int


def test_request_bytes():
    assert request_bytes(2, 8, 10) == 10 * (64 * 4 + 17)
    assert request_bytes(3, 16, 8192) == 8192 * (4096 * 4 + 17)


def test_admission_in_arrival_order_with_budget():
    w = [R(2, 32, 1000), R(2, 32, 1000), R(2, 8, 10)]
    one = request_bytes(2, 32, 1000)
    adm, rej = plan_admission(w, 0, int(1.5 * one), free_slots=8)
    assert adm == [w[0]] and rej == []            # second does not fit; the small third may not overtake
    adm, rej = plan_admission(w, 0, 3 * one, free_slots=8)
    assert adm == w
    adm, rej = plan_admission(w, 0, 3 * one, free_slots=1)
    assert adm == [w[0]]


def test_oversized_request_rejected():
    w = [R(3, 16, 8192), R(2, 8, 64)]
    adm, rej = plan_admission(w, 0, 1 << 20, free_slots=4)
    assert rej == [w[0]] and adm == [w[1]]


def test_chunk_plan_respects_quantum_and_batch():
    assert plan_chunks([5000, 100, 0, 3000], max_batch=4096, quantum=2048) == [(0, 2048), (1, 100), (3, 1948)]
    assert plan_chunks([10, 10], max_batch=15, quantum=100) == [(0, 10), (1, 5)]
    assert plan_chunks([], 10, 10) == []


def test_serving_workload_generator():
    reqs = si.serving_requests(seed=2208, rate=200.0, duration=5.0)
    assert 800 < len(reqs) < 1200
    assert all(r.dim in (2, 3) for r in reqs)
    assert all(r.L in si.L_CHOICES[r.dim] for r in reqs)
    assert all(64 <= r.n_samples <= 8192 for r in reqs)
    assert all(-4.5 <= r.m2 <= -3.5 and 4 <= r.lam <= 9 for r in reqs)
    ts = [r.t_arrive for r in reqs]
    assert ts == sorted(ts)
    assert reqs == si.serving_requests(seed=2208, rate=200.0, duration=5.0)

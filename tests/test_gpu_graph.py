"""Training steps replayed from a captured HIP graph (flow.Trainer(graph=True))
against eager steps on the same inputs: the kernels are deterministic, so every
replayed step must give the eager step's loss, gradient and parameters bit for bit.
Between replays the test does eager work of its own (a sampling batch) and
synchronises, and it checks every step, not only the last."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from paper_2208_08903_amd import lfs
from paper_2208_08903_amd.flow import Flow, Sampler, Trainer

pytestmark = pytest.mark.gpu

CASES = [
    # dim, L, N, hidden, precision, algo, kernel, hidden_sizes, batch_norm, B
    (2, 8, 4, 8, lfs.LFS_BF16_CONV, lfs.ALGO_AUTO, 0, None, False, 16),        # fused kernels
    (2, 8, 4, 8, lfs.LFS_PLAIN_FP32, lfs.ALGO_AUTO, 0, None, False, 16),
    (3, 4, 2, 8, lfs.LFS_BF16_CONV, lfs.ALGO_GENERIC, 0, None, False, 4),      # generic kernels
    (2, 8, 2, 0, lfs.LFS_BF16_CONV, lfs.ALGO_AUTO, 5, (4, 6), False, 8),       # general network
    (2, 8, 2, 0, lfs.LFS_PLAIN_FP32, lfs.ALGO_AUTO, 3, (4, 6), True, 8),       # batch norm
]


def _trainer(case, graph):
    dim, L, N, C, prec, algo, K, hs, bn, B = case
    params = si.flow_params(dim, N, C, seed=70, w_std=0.1, b_std=0.05, kernel=K or 3, hidden_sizes=hs,
                            batch_norm=bn, gamma_std=0.1 if bn else 0.0)
    f = Flow(dim, L, N, C, prec, algo, params=params, kernel=K, hidden_sizes=hs, batch_norm=bn)
    return Trainer(f, B, -4.0, 8.0, lr=1e-3, key=77, graph=graph)


@pytest.mark.parametrize("case", CASES)
def test_graph_replay_matches_eager(case):
    print(f"graph replay {case}", flush=True)
    eager, graphed = _trainer(case, False), _trainer(case, True)
    side = Sampler(eager.flow, 8, -4.0, 8.0, key=5)
    lu = torch.as_tensor(si.log_uniforms(6, (1, 8)), device="cuda")
    for step in range(5):
        eager.step()
        graphed.step()
        side.step(lu)                     # eager work of the program's own between replays
        torch.cuda.synchronize()
        assert torch.equal(eager.loss, graphed.loss), step
        assert torch.equal(eager.gparams, graphed.gparams), step
        assert torch.equal(eager.flow.params, graphed.flow.params), step
        if eager.flow.batch_norm:
            assert torch.equal(eager.flow.bn_stats, graphed.flow.bn_stats), step
    assert graphed._graph is not None and np.isfinite(float(graphed.loss.item()))

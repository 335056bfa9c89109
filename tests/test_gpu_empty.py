"""Empty batches through the Python binding: the per-sample entry points are
no-ops on zero-row tensors, the batch reductions raise."""
import pytest
import torch

import seeded_inputs as si
from paper_2208_08903_amd import lfs
from paper_2208_08903_amd.flow import Flow

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_empty_batch_per_sample_ops_are_noops():
    z = torch.empty(0, 1024, device=DEV, dtype=torch.float32)
    logr = torch.empty(0, device=DEV, dtype=torch.float64)
    lfs.prior_normal(5, 0, z, logr)
    f = Flow(2, 32, 2, 16, lfs.LFS_BF16_CONV, params=si.flow_params(2, 2, 16))
    assert f.workspace(0, False).numel() <= 1
    phi = torch.empty_like(z)
    logq = torch.empty(0, device=DEV, dtype=torch.float64)
    f.forward(z, phi, logq)
    S = torch.empty(0, device=DEV, dtype=torch.float64)
    m2 = torch.full((1,), -4.0, device=DEV, dtype=torch.float64)
    lam = torch.full((1,), 8.0, device=DEV, dtype=torch.float64)
    lfs.action(2, 32, phi, m2, lam, S, None, 1.0, lfs.LFS_BF16_CONV)
    torch.cuda.synchronize()
    # the loss is a mean over the batch: an empty one is an error
    with pytest.raises(lfs.LfsError):
        lfs.log_weights(S, logq, torch.empty(0, device=DEV, dtype=torch.float64),
                        torch.empty(1, device=DEV, dtype=torch.float64))
    # the batch still works afterwards
    z1 = torch.empty(3, 1024, device=DEV, dtype=torch.float32)
    lfs.prior_normal(5, 0, z1)
    phi1, logq1 = torch.empty_like(z1), torch.empty(3, device=DEV, dtype=torch.float64)
    f.forward(z1, phi1, logq1, ws=f.workspace(3, False))
    torch.cuda.synchronize()
    assert torch.isfinite(phi1).all() and torch.isfinite(logq1).all()

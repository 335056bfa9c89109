"""The allocation-free forward (lfs_flow_forward_noalloc, static device scratch)
against lfs_flow_forward with a caller workspace: same kernels, so the same bits,
on two calls in a row (the second with a smaller batch, so it reuses the scratch
the first left behind) for the fused, plane-streaming and generic families; no
device memory is allocated by the call; a flow whose workspace exceeds the
scratch is refused."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from paper_2208_08903_amd import lfs

from .gpu_util import DEV, dev, host, run_forward

pytestmark = pytest.mark.gpu

CASES = [
    # dim, L, N, C, precision, algo, batches (first, then smaller)
    (2, 32, 4, 16, lfs.LFS_BF16_CONV, lfs.ALGO_FUSED, (64, 7)),
    (2, 32, 3, 16, lfs.LFS_PLAIN_FP32, lfs.ALGO_FUSED, (33, 5)),
    (3, 16, 2, 32, lfs.LFS_BF16_CONV, lfs.ALGO_FUSED, (4, 2)),     # plane-streaming forward
    (2, 8, 3, 8, lfs.LFS_BF16_CONV, lfs.ALGO_GENERIC, (40, 3)),    # workspace grows with the batch
]


@pytest.mark.parametrize("dim,L,N,C,prec,algo,batches", CASES)
def test_noalloc_forward_matches_forward(dim, L, N, C, prec, algo, batches):
    print(f"noalloc forward dim={dim} L={L} N={N} C={C} precision={prec} algo={algo} batches={batches}",
          flush=True)
    desc = lfs.make_desc(dim, L, N, C, precision=prec, algo=algo)
    params = si.flow_params(dim, N, C, seed=50 + L, w_std=0.1, b_std=0.05)
    V = L ** dim
    for k, B in enumerate(batches):
        z = si.normal_fields(60 + k, B, V)
        ref = run_forward(desc, params, z)
        zt, pt = dev(z, torch.float32), dev(params, torch.float32)
        phi = torch.full((B, V), float("nan"), device=DEV)
        logq = torch.full((B,), float("nan"), device=DEV, dtype=torch.float64)
        logdet = torch.full((B,), float("nan"), device=DEV, dtype=torch.float64)
        saved = torch.full(((N + 1) * B * V,), float("nan"), device=DEV)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        lfs.flow_forward_noalloc(desc, pt, zt, phi, logq, logdet, saved)
        assert torch.cuda.memory_allocated() == before
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(phi), host(ref["phi"]))
        np.testing.assert_array_equal(host(logq), host(ref["logq"]))
        np.testing.assert_array_equal(host(logdet), host(ref["logdet"]))
        np.testing.assert_array_equal(host(saved), host(ref["saved"]))
        # phi may alias z, as in lfs_flow_forward
        lfs.flow_forward_noalloc(desc, pt, zt, zt, logq)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(zt), host(ref["phi"]))


def test_noalloc_forward_refuses_workspace_beyond_scratch():
    # the generic kernels keep the hidden activations in the workspace: 2 x B V C FP32
    desc = lfs.make_desc(2, 32, 2, 32, precision=lfs.LFS_BF16_CONV, algo=lfs.ALGO_GENERIC)
    B = 256
    assert lfs.workspace_bytes(desc, B, False) > lfs.NOALLOC_SCRATCH_BYTES
    V = 32 * 32
    params = torch.zeros(lfs.param_count(desc), device=DEV)
    z = torch.zeros(B, V, device=DEV)
    phi = torch.empty_like(z)
    logq = torch.empty(B, device=DEV, dtype=torch.float64)
    with pytest.raises(lfs.LfsError, match="static scratch"):
        lfs.flow_forward_noalloc(desc, params, z, phi, logq)


def test_noalloc_forward_empty_batch():
    desc = lfs.make_desc(2, 8, 2, 8, precision=lfs.LFS_BF16_CONV)
    params = torch.zeros(lfs.param_count(desc), device=DEV)
    z = torch.zeros(0, 64, device=DEV)
    lfs.flow_forward_noalloc(desc, params, z, z, torch.zeros(0, device=DEV, dtype=torch.float64))

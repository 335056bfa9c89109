"""End to end: a flow trained on the example theory (2D L = 8, m^2 = -4,
lambda = 8) and corrected by the independence MH chain reproduces HMC's <M^2>
on the same theory, within five combined standard errors (MH: from the chain's
integrated autocorrelation time; HMC: from 256 independent chains).  The MH
correction makes the flow ensemble exact whatever the training left, so a wrong
log-det sign, a Jacobian term, an action term or the accept rule would show up
here as a bias."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from paper_2208_08903_amd import lfs
from paper_2208_08903_amd.flow import Flow, chain_quality, hmc_chain_quality, train

pytestmark = pytest.mark.gpu


def test_flow_mh_matches_hmc():
    print("train the example flow (3000 steps), then MH and HMC", flush=True)
    flow = Flow(2, 8, 16, 8, lfs.LFS_BF16_CONV, params=si.flow_params(2, 16, 8))
    train(flow, 3000, 64, -4.0, 8.0, lr=1e-3)
    fq = chain_quality(flow, -4.0, 8.0, batches=16, B=4096)
    hq = hmc_chain_quality(2, 8, -4.0, 8.0, n_chains=256, n_traj=1500)
    torch.cuda.synchronize()
    print({k: fq[k] for k in ("acceptance", "M2_mean", "M2_err", "tau_M")},
          {k: hq[k] for k in ("acceptance", "M2_mean", "M2_err")}, flush=True)
    assert fq["acceptance"] > 0.1 and hq["acceptance"] > 0.5
    diff = abs(fq["M2_mean"] - hq["M2_mean"])
    assert diff < 5 * np.hypot(fq["M2_err"], hq["M2_err"]), (fq["M2_mean"], hq["M2_mean"], fq["M2_err"], hq["M2_err"])
    # the comparison has teeth: the errors are a few per cent of the value
    assert fq["M2_err"] < 0.05 * fq["M2_mean"] and hq["M2_err"] < 0.05 * hq["M2_mean"]

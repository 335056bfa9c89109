"""End to end: a flow trained on the example theory (2D L = 8, m^2 = -4,
lambda = 8), and one on the 3D L = 8 theory (m^2 = -4, lambda = 5, 12 layers of
16 channels), corrected by the independence MH chain, reproduce HMC's <M^2> and
zero-momentum two-point function C(t) on the same theory, within five combined
standard errors (MH: from the chain's integrated autocorrelation time of each
series; HMC: from 256 independent chains).  The MH correction makes the flow
ensemble exact whatever the training left, so a wrong log-det sign, a Jacobian
term, an action term or the accept rule would show up here as a bias."""
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
    _check_two_point(fq, hq)


def _check_two_point(fq, hq):
    cf, ef = np.array(fq["C_mean"]), np.array(fq["C_err"])
    ch, eh = np.array(hq["C_mean"]), np.array(hq["C_err"])
    print("C(t) flow+MH", np.round(cf, 4), "+-", np.round(ef, 4), flush=True)
    print("C(t) HMC    ", np.round(ch, 4), "+-", np.round(eh, 4), flush=True)
    assert np.all(np.abs(cf - ch) < 5 * np.hypot(ef, eh)), (cf, ch)
    # teeth: the errors are a few per cent of the function's scale C(0)
    assert np.all(ef < 0.05 * abs(cf[0])) and np.all(eh < 0.05 * abs(ch[0]))


def test_flow_mh_matches_hmc_3d():
    """3D L = 8: trained 5000 steps at batch 256 from N(0, 0.02^2) weights (the 3D networks
    at N(0, 0.1^2) start in tanh saturation and do not train at this length)."""
    print("train the 3D L=8 flow (5000 steps), then MH and HMC", flush=True)
    flow = Flow(3, 8, 12, 16, lfs.LFS_BF16_CONV, params=si.flow_params(3, 12, 16, w_std=0.02))
    train(flow, 5000, 256, -4.0, 5.0, lr=1e-3)
    fq = chain_quality(flow, -4.0, 5.0, batches=16, B=4096)
    hq = hmc_chain_quality(3, 8, -4.0, 5.0, n_chains=256, n_traj=1500)
    torch.cuda.synchronize()
    print({k: fq[k] for k in ("acceptance", "M2_mean", "M2_err", "tau_M")},
          {k: hq[k] for k in ("acceptance", "M2_mean", "M2_err")}, flush=True)
    assert fq["acceptance"] > 0.1 and hq["acceptance"] > 0.3
    diff = abs(fq["M2_mean"] - hq["M2_mean"])
    assert diff < 5 * np.hypot(fq["M2_err"], hq["M2_err"]), (fq["M2_mean"], hq["M2_mean"], fq["M2_err"], hq["M2_err"])
    assert fq["M2_err"] < 0.05 * fq["M2_mean"] and hq["M2_err"] < 0.05 * hq["M2_mean"]
    _check_two_point(fq, hq)

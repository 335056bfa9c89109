"""The C-ABI library loads, exports every symbol include/lfs.h declares, and its
host-side validation behaves as documented (no GPU call is made here)."""
import ctypes
import os
import re

import pytest

import seeded_inputs as si
from paper_2208_08903_amd import lfs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "lfs.h")).read()
    return sorted(set(re.findall(r"\b(lfs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_header_function():
    lib = lfs.load()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lfs.EXPORTED)


def test_struct_sizes_match_header():
    assert ctypes.sizeof(lfs.FlowDesc) == 60   # 10 int32 fields + hidden_sizes[4] + batch_norm
    assert lfs.CHAIN_STATE_BYTES == 40


@pytest.mark.parametrize("dim,N,K,hs", [(2, 16, 5, (8, 8)), (2, 3, 3, (3, 5, 4)), (3, 2, 5, (2,)),
                                        (2, 4, 1, (16, 16, 16, 16)), (3, 12, 3, (16, 16))])
def test_param_count_general_networks(dim, N, K, hs):
    d = lfs.make_desc(dim, 8, N, 0, kernel=K, hidden_sizes=hs)
    assert lfs.param_count(d) == si.param_count(dim, N, 0, K, hs)


def test_general_network_validation():
    lib = lfs.load()
    out = ctypes.c_size_t(0)
    for kw, code in [(dict(kernel=4), -1), (dict(kernel=9), -1), (dict(kernel=-1), -1),
                     (dict(hidden_sizes=(8, 0)), -1), (dict(hidden_sizes=(8, 65)), -2)]:
        d = lfs.make_desc(2, 8, 2, 8, **kw)
        assert lib.lfs_workspace_bytes(ctypes.byref(d), 4, 0, ctypes.byref(out)) == code, kw
    d = lfs.make_desc(2, 8, 2, 8)
    d.n_hidden = 5
    assert lib.lfs_workspace_bytes(ctypes.byref(d), 4, 0, ctypes.byref(out)) == -1
    # a non-default network has no fused kernel; the explicit default one does
    fused = lfs.make_desc(2, 8, 2, 8, kernel=5, algo=lfs.ALGO_FUSED)
    assert lib.lfs_workspace_bytes(ctypes.byref(fused), 4, 0, ctypes.byref(out)) == -2
    dflt = lfs.make_desc(2, 8, 2, 0, kernel=3, hidden_sizes=(8, 8), algo=lfs.ALGO_FUSED)
    assert lib.lfs_workspace_bytes(ctypes.byref(dflt), 4, 0, ctypes.byref(out)) == 0


@pytest.mark.parametrize("dim,N,K,hs", [(2, 3, 3, (3, 5, 4)), (3, 2, 5, (2,)), (2, 4, 3, (8, 8))])
def test_batch_norm_layout_and_validation(dim, N, K, hs):
    lib = lfs.load()
    d = lfs.make_desc(dim, 8, N, 0, kernel=K, hidden_sizes=hs, batch_norm=True)
    assert lfs.param_count(d) == si.param_count(dim, N, 0, K, hs, batch_norm=True)
    assert lfs.bn_stats_count(d) == N * 2 * sum(hs) == si.bn_stats(0, N, hs).size
    assert lfs.bn_stats_count(lfs.make_desc(dim, 8, N, 0, kernel=K, hidden_sizes=hs)) == 0
    out = ctypes.c_size_t(0)
    assert lib.lfs_workspace_bytes(ctypes.byref(d), 4, 0, ctypes.byref(out)) == 0 and out.value > 0
    need_f = out.value
    assert lib.lfs_workspace_bytes(ctypes.byref(d), 4, 1, ctypes.byref(out)) == 0 and out.value > need_f
    need_b = out.value
    # the plain entry points refuse a batch-norm flow; the _bn ones validate mode,
    # statistics, momentum and workspace before any launch (non-null dummies)
    assert lib.lfs_flow_forward(ctypes.byref(d), 1, 4, 1, 1, 1, None, None, 1, 1 << 40, None) == -1
    assert lib.lfs_flow_backward(ctypes.byref(d), 1, 4, 1, 1, 0.25, 1, None, 1, 1 << 40, None) == -1
    fwd = lib.lfs_flow_forward_bn
    assert fwd(ctypes.byref(d), 1, 4, 1, 1, 1, None, None, 2, 1, 0.1, 1, 1 << 40, None) == -1  # mode
    assert fwd(ctypes.byref(d), 1, 4, 1, 1, 1, None, None, 1, None, 0.1, 1, 1 << 40, None) == -1  # stats
    assert fwd(ctypes.byref(d), 1, 4, 1, 1, 1, None, None, 0, None, 1.5, 1, 1 << 40, None) == -1  # momentum
    assert fwd(ctypes.byref(d), 1, 4, 1, 1, 1, None, None, 0, None, float("nan"), 1, 1 << 40, None) == -1
    assert fwd(ctypes.byref(d), 1, 4, 1, 1, 1, None, None, 0, None, 0.1, 1, need_f - 1, None) == -3
    bwd = lib.lfs_flow_backward_bn
    assert bwd(ctypes.byref(d), 1, 4, 1, 1, 0.25, None, 1, None, 1, None, 1, 1 << 40, None) == -1  # stats
    assert bwd(ctypes.byref(d), 1, 4, 1, 1, 0.25, None, 3, 1, 1, None, 1, 1 << 40, None) == -1     # mode
    assert bwd(ctypes.byref(d), 1, 4, 1, 1, 0.25, 1, 0, None, 1, None, 1, need_b - 1, None) == -3
    # the per-sample entry point takes no batch-norm flow either
    assert lib.lfs_flow_backward_vec(ctypes.byref(d), 1, 4, 1, 1, 1, 1, None, 1, 1 << 40, None) == -1
    fused = lfs.make_desc(dim, 8, N, 0, kernel=K, hidden_sizes=hs, batch_norm=True, algo=lfs.ALGO_FUSED)
    assert lib.lfs_workspace_bytes(ctypes.byref(fused), 4, 0, ctypes.byref(out)) == -2
    assert fwd(ctypes.byref(fused), 1, 4, 1, 1, 1, None, None, 0, None, 0.1, 1, 1 << 40, None) == -2
    d.batch_norm = 2
    assert lib.lfs_workspace_bytes(ctypes.byref(d), 4, 0, ctypes.byref(out)) == -1
    assert lfs.param_count(d) == 0


@pytest.mark.parametrize("dim,N,C", [(2, 16, 8), (2, 16, 16), (3, 12, 16), (3, 16, 32)])
def test_param_count_matches_layout(dim, N, C):
    d = lfs.make_desc(dim, 8, N, C)
    assert lfs.param_count(d) == si.param_count(dim, N, C)


def test_status_strings_and_version():
    assert lfs.status_string(0) == "LFS_OK"
    for s in (-1, -2, -3, -4):
        assert lfs.status_string(s).startswith("LFS_E")
    assert "gfx950" in lfs.version()


@pytest.mark.parametrize("kw,code", [
    (dict(dim=4), -1), (dict(L=7), -1), (dict(L=0), -1), (dict(n_layers=0), -1),
    (dict(hidden=12), -2), (dict(precision=5), -1), (dict(parity0=2), -1), (dict(algo=9), -1),
])
def test_descriptor_validation(kw, code):
    base = dict(dim=2, L=8, n_layers=4, hidden=8)
    base.update({k: v for k, v in kw.items() if k in base})
    d = lfs.make_desc(**base)
    for k in ("precision", "parity0", "algo"):
        if k in kw:
            setattr(d, k, kw[k])
    out = ctypes.c_size_t(0)
    assert lfs.load().lfs_workspace_bytes(ctypes.byref(d), 4, 0, ctypes.byref(out)) == code
    assert lfs.param_count(d) == 0


def test_empty_batches():
    """B == 0 is a no-op (LFS_OK, no pointer read) for the per-sample entry points and an
    error for the reductions over the batch; negative sizes are errors everywhere."""
    lib = lfs.load()
    d = lfs.make_desc(2, 8, 4, 8)
    out = ctypes.c_size_t(7)
    assert lib.lfs_workspace_bytes(ctypes.byref(d), 0, 0, ctypes.byref(out)) == 0 and out.value == 0
    assert lib.lfs_workspace_bytes(ctypes.byref(d), -1, 0, ctypes.byref(out)) == -1
    assert lib.lfs_prior_normal(1, 0, 0, 64, None, None, None) == 0
    assert lib.lfs_prior_normal(1, 0, -1, 64, None, None, None) == -1
    assert lib.lfs_prior_normal(1, 0, 0, 6, None, None, None) == -1           # V % 4 still checked
    assert lib.lfs_prior_normal_streams(0, 64, None, None, None, None, None) == 0
    assert lib.lfs_flow_forward(ctypes.byref(d), None, 0, None, None, None, None, None, None, 0,
                                None) == 0
    assert lib.lfs_flow_forward(ctypes.byref(d), None, -1, None, None, None, None, None, None, 0,
                                None) == -1
    bad = lfs.make_desc(2, 8, 4, 8)
    bad.L = 7
    assert lib.lfs_flow_forward(ctypes.byref(bad), None, 0, None, None, None, None, None, None, 0,
                                None) == -1                                   # desc still checked
    assert lib.lfs_flow_backward(ctypes.byref(d), None, 0, None, None, 0.25, None, None, None, 0,
                                 None) == -1                                  # batch reduction
    bn = lfs.make_desc(2, 8, 2, 0, kernel=3, hidden_sizes=(8, 8), batch_norm=True)
    fwd = lib.lfs_flow_forward_bn
    assert fwd(ctypes.byref(bn), None, 0, None, None, None, None, None, lfs.BN_RUNNING, None, 0.0,
               None, 0, None) == 0
    assert fwd(ctypes.byref(bn), None, 0, None, None, None, None, None, lfs.BN_BATCH, None, 0.1,
               None, 0, None) == -1                                           # no statistics
    assert lib.lfs_action(2, 8, 0, None, None, None, 0, 1, None, None, 1.0, None) == 0
    assert lib.lfs_action(2, 8, -2, None, None, None, 0, 1, None, None, 1.0, None) == -1
    assert lib.lfs_action(2, 256, 0, None, None, None, 0, 1, None, None, 1.0, None) == -2  # V
    assert lib.lfs_log_weights(0, None, None, None, None, None) == -1
    assert lib.lfs_mh_chain(0, 10, None, None, None, None, None, None) == 0
    assert lib.lfs_mh_chain(3, 0, None, None, None, None, None, None) == 0
    assert lib.lfs_mh_chain(-1, 10, None, None, None, None, None, None) == -1
    assert lib.lfs_mh_chain_ragged(0, None, None, None, None, None, None, None, None) == 0
    assert lib.lfs_mh_chain_ragged(-1, None, None, None, None, None, None, None, None) == -1
    assert lib.lfs_hmc_step(2, 8, 0, None, None, None, None, None, 0, 10, 0.1, None, None,
                            None) == 0
    assert lib.lfs_hmc_step(3, 20, 0, None, None, None, None, None, 0, 10, 0.1, None, None,
                            None) == -2                                       # V > 4096


def test_null_and_shape_arguments_rejected_before_any_launch():
    lib = lfs.load()
    d = lfs.make_desc(2, 8, 4, 8)
    # null params / z / phi / logq
    assert lib.lfs_flow_forward(ctypes.byref(d), None, 4, None, None, None, None, None, None, 0,
                                None) == -1
    assert lib.lfs_flow_backward(ctypes.byref(d), None, 4, None, None, 0.25, None, None, None, 0,
                                 None) == -1
    assert lib.lfs_flow_backward_vec(ctypes.byref(d), 1, 4, 1, 1, None, 1, None, 1, 1 << 40,
                                     None) == -1                              # g_logq NULL
    need = lfs.workspace_bytes(d, 4, True)
    assert lib.lfs_flow_backward_vec(ctypes.byref(d), 1, 4, 1, 1, 1, 1, None, 1, need - 1,
                                     None) == -3
    assert lib.lfs_prior_normal(1, 0, 4, 6, None, None, None) == -1          # V % 4
    assert lib.lfs_action(4, 8, 4, None, None, None, 0, 1, None, None, 1.0, None) == -1
    assert lib.lfs_action(2, 256, 4, 1, 1, 1, 0, 1, 1, None, 1.0, None) == -2  # V too large
    assert lib.lfs_log_weights(0, None, None, None, None, None) == -1
    assert lib.lfs_mh_chain(1, 5, None, None, None, None, None, None) == -1   # nulls
    assert lib.lfs_hmc_step(2, 8, 4, None, None, None, None, None, 0, -1, 0.1, None, None,
                            None) == -1
    assert lib.lfs_hmc_step(3, 20, 1, 1, 1, 1, 1, 1, 0, 10, 0.1, 1, 1, None) == -2  # V > 4096
    assert lib.lfs_adam_step(0, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 1, None) == -1
    assert lib.lfs_adam_step(10, 1, 1, 1, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1  # t < 1
    assert lib.lfs_observables(4, 8, 2, 1, 0, 1, None, None) == -1           # dim
    assert lib.lfs_observables(2, 8, 2, 1, 0, None, None, None) == -1        # no output
    assert lib.lfs_observables(2, 4097, 2, 1, 0, 1, None, None) == -2        # L too large
    assert lib.lfs_observables(2, 8, 0, 1, 0, 1, None, None) == 0            # empty batch
    assert lib.lfs_autocorr_workspace_bytes(0, 100, 10) == 0
    big = 1 << 40
    assert lib.lfs_autocorr(0, 100, 1, 100, None, 10, 6.0, None, 1, None, None, None, 1, big,
                            None) == -1                                      # n_series
    assert lib.lfs_autocorr(1, 100, 1, 50, None, 10, 6.0, None, 1, None, None, None, 1, big,
                            None) == -1                                      # ldx < n
    assert lib.lfs_autocorr(1, 100, 1, 100, None, 10, 0.0, None, 1, None, None, None, 1, big,
                            None) == -1                                      # c <= 0
    assert lib.lfs_autocorr(1, 100, 1, 100, None, 9000, 6.0, None, 1, None, None, None, 1, big,
                            None) == -2                                      # w_max
    need = lib.lfs_autocorr_workspace_bytes(3, 5000, 300)
    assert need > 0
    assert lib.lfs_autocorr(3, 5000, 1, 5000, None, 300, 6.0, None, 1, None, None, None, 1,
                            need - 1, None) == -3                            # workspace
    assert lib.lfs_ess(1, 10, 1, 9, 1, None) == -1                           # ldw < n
    assert lib.lfs_ess(1, 0, 1, 9, 1, None) == -1                            # n < 1


def test_saved_h_bytes_and_validation():
    """The training pair's saved activations: h2 and s, N B (C V + V / 2) FP32 values, on
    2D L = 32, hidden 16, plain FP32; h1, h2, sign words and s on 3D L = 16 (BF16, hidden
    16 or 32); none elsewhere; missing buffers are rejected before any launch."""
    lib = lfs.load()
    d = lfs.make_desc(2, 32, 3, 16)
    assert lfs.saved_h_bytes(d, 5) == 3 * 5 * (16 * 1024 + 512) * 4
    assert lfs.saved_h_bytes(d, 0) == 0
    # 3D L = 16, BF16 (plane-streaming): h1, h2 BF16 channel-major, two sign words and s per site
    for C in (16, 32):
        d3 = lfs.make_desc(3, 16, 2, C, precision=lfs.LFS_BF16_CONV)
        assert lfs.saved_h_bytes(d3, 4) == 2 * (2 * 4 * C * 4096 * 2 + 3 * 4 * 4096 * 4)
    for other in (lfs.make_desc(2, 8, 2, 16), lfs.make_desc(2, 32, 2, 8),
                  lfs.make_desc(2, 32, 2, 16, precision=lfs.LFS_BF16_CONV),
                  lfs.make_desc(3, 16, 2, 8, precision=lfs.LFS_BF16_CONV),
                  lfs.make_desc(3, 16, 2, 16),
                  lfs.make_desc(2, 32, 2, 16, algo=lfs.ALGO_GENERIC)):
        assert lfs.saved_h_bytes(other, 4) == 0
    out = ctypes.c_size_t(0)
    assert lib.lfs_saved_h_bytes(ctypes.byref(d), -1, ctypes.byref(out)) == -1
    assert lib.lfs_saved_h_bytes(ctypes.byref(d), 4, None) == -1
    need = lfs.workspace_bytes(d, 4, False)
    # saved_x NULL, saved_h NULL
    assert lib.lfs_flow_forward_train(ctypes.byref(d), 1, 4, 1, 1, 1, None, None, 1, 1, need, None) == -1
    assert lib.lfs_flow_forward_train(ctypes.byref(d), 1, 4, 1, 1, 1, None, 1, None, 1, need, None) == -1
    assert lib.lfs_flow_forward_train(ctypes.byref(d), None, 0, None, None, None, None, None, None, None,
                                      0, None) == 0                                    # empty batch
    need_b = lfs.workspace_bytes(d, 4, True)
    assert lib.lfs_flow_backward_saved(ctypes.byref(d), 1, 4, 1, None, 1, 0.25, None, 1, None, 1, need_b,
                                       None) == -1                                     # saved_h NULL
    assert lib.lfs_flow_backward_saved(ctypes.byref(d), 1, 4, 1, 1, 1, 0.25, None, 1, None, 1, need_b - 1,
                                       None) == -3                                     # workspace
    bn = lfs.make_desc(2, 8, 2, 8, batch_norm=True)
    assert lib.lfs_flow_backward_saved(ctypes.byref(bn), 1, 4, 1, 1, 1, 0.25, None, 1, None, 1, 1 << 40,
                                       None) == -1                                     # batch norm


def test_workspace_too_small_is_reported():
    lib = lfs.load()
    d = lfs.make_desc(2, 8, 4, 8)
    need = lfs.workspace_bytes(d, 16, False)
    assert need > 0
    # non-null dummies: validation must fail on the workspace size before any launch
    assert lib.lfs_flow_forward(ctypes.byref(d), 1, 16, 1, 1, 1, None, None, 1, need - 1,
                                None) == -3

"""ctypes binding of liblfs.so: one Python function per C entry point, same names.

Argument marshalling only: tensors are checked for their sizes against the
shapes the call implies (batch B, sites V = L^dim, layers N from the flow
descriptor), then for device, dtype and contiguity; their data pointers and
torch's current HIP stream are passed through, and a negative status raises
LfsError.  A mis-sized buffer is an LfsError here, never an out-of-bounds
access in a kernel.  Every step of the computation
runs in the library's HIP kernels; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblfs.so")

LFS_PLAIN_FP32 = 0
LFS_BF16_CONV = 1
ALGO_AUTO, ALGO_GENERIC, ALGO_FUSED = 0, 1, 2
BN_BATCH, BN_RUNNING = 0, 1

c_i32, c_i64, c_u64, c_f32, c_f64, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                                 ctypes.c_float, ctypes.c_double, ctypes.c_void_p,
                                                 ctypes.c_size_t)


class LfsError(RuntimeError):
    pass


MAX_HIDDEN = 4


class FlowDesc(ctypes.Structure):
    _fields_ = [("dim", c_i32), ("L", c_i32), ("n_layers", c_i32), ("hidden", c_i32),
                ("final_tanh", c_i32), ("parity0", c_i32), ("precision", c_i32), ("algo", c_i32),
                ("kernel", c_i32), ("n_hidden", c_i32), ("hidden_sizes", c_i32 * MAX_HIDDEN),
                ("batch_norm", c_i32)]

    def key(self):
        return tuple(tuple(v) if f == "hidden_sizes" else getattr(self, f)
                     for f, _ in self._fields_ for v in [getattr(self, f)])


class ChainState(ctypes.Structure):
    _fields_ = [("w_cur", c_f64), ("idx_cur", c_i64), ("n_acc", c_i64), ("n_seen", c_i64),
                ("has_state", c_i32), ("reserved", c_i32)]


CHAIN_STATE_BYTES = ctypes.sizeof(ChainState)  # 40

_SIGS = {
    "lfs_status_string": (ctypes.c_char_p, [c_i32]),
    "lfs_version": (ctypes.c_char_p, []),
    "lfs_param_count": (c_sz, [ctypes.POINTER(FlowDesc)]),
    "lfs_workspace_bytes": (c_i32, [ctypes.POINTER(FlowDesc), c_i32, c_i32, ctypes.POINTER(c_sz)]),
    "lfs_prior_normal": (c_i32, [c_u64, c_u64, c_i32, c_i32, c_vp, c_vp, c_vp]),
    "lfs_prior_normal_streams": (c_i32, [c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lfs_mh_chain_ragged": (c_i32, [c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lfs_flow_forward": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_vp, c_vp,
                                 c_vp, c_vp, c_sz, c_vp]),
    "lfs_flow_backward": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_f64, c_vp,
                                  c_vp, c_vp, c_sz, c_vp]),
    "lfs_flow_forward_noalloc": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_vp, c_vp,
                                         c_vp, c_vp]),
    "lfs_bn_stats_count": (c_sz, [ctypes.POINTER(FlowDesc)]),
    "lfs_saved_h_bytes": (c_i32, [ctypes.POINTER(FlowDesc), c_i32, ctypes.POINTER(c_sz)]),
    "lfs_flow_forward_train": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_vp, c_vp,
                                       c_vp, c_vp, c_vp, c_sz, c_vp]),
    "lfs_flow_backward_saved": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_vp, c_f64,
                                        c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "lfs_flow_forward_bn": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_vp, c_vp,
                                    c_vp, c_i32, c_vp, c_f64, c_vp, c_sz, c_vp]),
    "lfs_flow_backward_bn": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_f64, c_vp,
                                     c_i32, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "lfs_flow_backward_vec": (c_i32, [ctypes.POINTER(FlowDesc), c_vp, c_i32, c_vp, c_vp, c_vp, c_vp,
                                      c_vp, c_vp, c_sz, c_vp]),
    "lfs_action": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp, c_f64,
                           c_vp]),
    "lfs_log_weights": (c_i32, [c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lfs_mh_chain": (c_i32, [c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lfs_hmc_step": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32,
                             c_f64, c_vp, c_vp, c_vp]),
    "lfs_adam_step": (c_i32, [c_i64, c_vp, c_vp, c_vp, c_vp, c_f32, c_f32, c_f32, c_f32, c_i64,
                              c_vp]),
    "lfs_observables": (c_i32, [c_i32, c_i32, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "lfs_autocorr_workspace_bytes": (c_sz, [c_i32, c_i64, c_i32]),
    "lfs_autocorr": (c_i32, [c_i32, c_i64, c_vp, c_i64, c_vp, c_i32, c_f64, c_vp, c_vp, c_vp, c_vp,
                             c_vp, c_vp, c_sz, c_vp]),
    "lfs_ess": (c_i32, [c_i32, c_i64, c_vp, c_i64, c_vp, c_vp]),
}
EXPORTED = tuple(_SIGS)

_lib = None


def load():
    """Load liblfs.so (built in-tree).  Raises LfsError if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LfsError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = res, args
        _lib = lib
    return _lib


def _check(status: int):
    if status != 0:
        raise LfsError(load().lfs_status_string(status).decode())


def status_string(status: int) -> str:
    return load().lfs_status_string(status).decode()


def version() -> str:
    return load().lfs_version().decode()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise LfsError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise LfsError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise LfsError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, n, name, exact=True):
    """t (if given) holds exactly n entries (at least n if not exact)."""
    if t is None:
        return
    k = t.numel()
    if (k != n) if exact else (k < n):
        raise LfsError(f"{name} has {k} entries, the call needs {'' if exact else 'at least '}{n}")


def _field(t, V, name):
    """A [B, V] field: returns B."""
    if t is None or t.dim() != 2 or t.shape[1] != V:
        shape = None if t is None else tuple(t.shape)
        raise LfsError(f"{name} must be a [B, {V}] tensor, got {shape}")
    return int(t.shape[0])


def _sites(desc) -> int:
    if desc.dim not in (2, 3) or desc.L < 2:
        raise LfsError(f"invalid lattice dim={desc.dim} L={desc.L}")
    return desc.L ** desc.dim


def _flow_sizes(desc, params, B, saved_x, bn_stats=None):
    V = _sites(desc)
    P = param_count(desc)
    if P == 0:
        raise LfsError("invalid flow descriptor")
    _need(params, P, "params")
    _need(saved_x, (desc.n_layers + 1) * B * V, "saved_x", exact=False)
    if bn_stats is not None:
        _need(bn_stats, bn_stats_count(desc), "bn_stats")
    return V, P


def make_desc(dim, L, n_layers, hidden, final_tanh=True, parity0=0,
              precision=LFS_PLAIN_FP32, algo=ALGO_AUTO, kernel=0, hidden_sizes=None,
              batch_norm=False) -> FlowDesc:
    """hidden_sizes: the widths of the hidden convolutions (None: two of `hidden`);
    kernel: odd kernel size per axis (0: 3); batch_norm: normalise every hidden
    convolution's output (the _bn entry points)."""
    hs = list(hidden_sizes or [])
    if len(hs) > MAX_HIDDEN:
        raise LfsError(f"at most {MAX_HIDDEN} hidden convolutions")
    arr = (c_i32 * MAX_HIDDEN)(*(hs + [0] * (MAX_HIDDEN - len(hs))))
    return FlowDesc(dim, L, n_layers, hidden, int(final_tanh), parity0, precision, algo, kernel,
                    len(hs), arr, int(batch_norm))


def param_count(desc: FlowDesc) -> int:
    return int(load().lfs_param_count(ctypes.byref(desc)))


def bn_stats_count(desc: FlowDesc) -> int:
    return int(load().lfs_bn_stats_count(ctypes.byref(desc)))


def workspace_bytes(desc: FlowDesc, B: int, for_backward: bool) -> int:
    out = c_sz(0)
    _check(load().lfs_workspace_bytes(ctypes.byref(desc), B, int(for_backward), ctypes.byref(out)))
    return int(out.value)


def prior_normal(key: int, counter0: int, z, logr=None):
    if z is None or z.dim() != 2:
        raise LfsError("z must be a [B, V] tensor")
    B, V = z.shape
    _need(logr, B, "logr")
    _check(load().lfs_prior_normal(key, counter0, B, V, _p(z, torch.float32, "z"),
                                   _p(logr, torch.float64, "logr"), _stream()))


def prior_normal_streams(keys, counters, z, logr=None):
    if z is None or z.dim() != 2:
        raise LfsError("z must be a [B, V] tensor")
    B, V = z.shape
    if keys.numel() != B or counters.numel() != B:
        raise LfsError("keys and counters need one entry per sample")
    _need(logr, B, "logr")
    _check(load().lfs_prior_normal_streams(B, V, _p(keys, torch.int64, "keys"),
                                           _p(counters, torch.int64, "counters"),
                                           _p(z, torch.float32, "z"),
                                           _p(logr, torch.float64, "logr"), _stream()))


def flow_forward(desc, params, z, phi, logq, logdet=None, saved_x=None, ws=None):
    B = _field(z, _sites(desc), "z")
    V, _ = _flow_sizes(desc, params, B, saved_x)
    _need(phi, B * V, "phi")
    _need(logq, B, "logq")
    _need(logdet, B, "logdet")
    nbytes = ws.numel() if ws is not None else 0
    _check(load().lfs_flow_forward(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                   _p(z, torch.float32, "z"), _p(phi, torch.float32, "phi"),
                                   _p(logq, torch.float64, "logq"),
                                   _p(logdet, torch.float64, "logdet"),
                                   _p(saved_x, torch.float32, "saved_x"),
                                   _p(ws, torch.uint8, "ws"), nbytes, _stream()))


NOALLOC_SCRATCH_BYTES = 8 << 20   # LFS_NOALLOC_SCRATCH_BYTES


def flow_forward_noalloc(desc, params, z, phi, logq, logdet=None, saved_x=None):
    """flow_forward with the library's static device scratch as workspace (no allocation
    anywhere in the call).  Calls that overlap on one GPU share the scratch and race."""
    B = _field(z, _sites(desc), "z")
    V, _ = _flow_sizes(desc, params, B, saved_x)
    _need(phi, B * V, "phi")
    _need(logq, B, "logq")
    _need(logdet, B, "logdet")
    st = load().lfs_flow_forward_noalloc(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                         _p(z, torch.float32, "z"), _p(phi, torch.float32, "phi"),
                                         _p(logq, torch.float64, "logq"),
                                         _p(logdet, torch.float64, "logdet"),
                                         _p(saved_x, torch.float32, "saved_x"), _stream())
    if st == -3:
        raise LfsError(f"flow_forward_noalloc: this flow at batch {B} needs more workspace than the "
                       f"{NOALLOC_SCRATCH_BYTES} bytes of static scratch (LFS_EWORKSPACE)")
    _check(st)


def flow_backward(desc, params, saved_x, g_phi, g_logq: float, g_params, g_z=None, ws=None):
    B = _field(g_phi, _sites(desc), "g_phi")
    V, P = _flow_sizes(desc, params, B, saved_x)
    _need(saved_x, (desc.n_layers + 1) * B * V, "saved_x", exact=False)
    _need(g_params, P, "g_params")
    _need(g_z, B * V, "g_z")
    nbytes = ws.numel() if ws is not None else 0
    _check(load().lfs_flow_backward(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                    _p(saved_x, torch.float32, "saved_x"),
                                    _p(g_phi, torch.float32, "g_phi"), float(g_logq),
                                    _p(g_params, torch.float32, "g_params"),
                                    _p(g_z, torch.float32, "g_z"), _p(ws, torch.uint8, "ws"),
                                    nbytes, _stream()))


def saved_h_bytes(desc: FlowDesc, B: int) -> int:
    """Bytes of the activations flow_forward_train saves (0: the backward recomputes them)."""
    out = c_sz(0)
    _check(load().lfs_saved_h_bytes(ctypes.byref(desc), B, ctypes.byref(out)))
    return int(out.value)


def flow_forward_train(desc, params, z, phi, logq, saved_x, saved_h, logdet=None, ws=None):
    """flow_forward that also saves the second hidden activation of every layer in saved_h
    (a uint8 device tensor of saved_h_bytes(desc, B) bytes, or None when that is 0)."""
    B = _field(z, _sites(desc), "z")
    if saved_x is None:
        raise LfsError("flow_forward_train needs saved_x")
    V, _ = _flow_sizes(desc, params, B, saved_x)
    _need(phi, B * V, "phi")
    _need(logq, B, "logq")
    _need(logdet, B, "logdet")
    hb = saved_h_bytes(desc, B)
    if hb and (saved_h is None or saved_h.numel() * saved_h.element_size() < hb):
        raise LfsError(f"saved_h needs {hb} bytes")
    nbytes = ws.numel() if ws is not None else 0
    _check(load().lfs_flow_forward_train(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                         _p(z, torch.float32, "z"), _p(phi, torch.float32, "phi"),
                                         _p(logq, torch.float64, "logq"),
                                         _p(logdet, torch.float64, "logdet"),
                                         _p(saved_x, torch.float32, "saved_x"),
                                         _p(saved_h if hb else None, None, "saved_h"),
                                         _p(ws, torch.uint8, "ws"), nbytes, _stream()))


def flow_backward_saved(desc, params, saved_x, saved_h, g_phi, g_logq, g_params, g_z=None, ws=None):
    """flow_backward (g_logq a float) or flow_backward_vec (g_logq a [B] FP64 device tensor)
    reading the activations flow_forward_train saved."""
    B = _field(g_phi, _sites(desc), "g_phi")
    V, P = _flow_sizes(desc, params, B, saved_x)
    _need(g_params, P, "g_params")
    _need(g_z, B * V, "g_z")
    hb = saved_h_bytes(desc, B)
    if hb and (saved_h is None or saved_h.numel() * saved_h.element_size() < hb):
        raise LfsError(f"saved_h needs {hb} bytes")
    vec = g_logq if isinstance(g_logq, torch.Tensor) else None
    if vec is not None and vec.numel() != B:
        raise LfsError("g_logq needs one entry per sample")
    scalar = 0.0 if vec is not None else float(g_logq)
    nbytes = ws.numel() if ws is not None else 0
    _check(load().lfs_flow_backward_saved(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                          _p(saved_x, torch.float32, "saved_x"),
                                          _p(saved_h if hb else None, None, "saved_h"),
                                          _p(g_phi, torch.float32, "g_phi"), scalar,
                                          _p(vec, torch.float64, "g_logq"),
                                          _p(g_params, torch.float32, "g_params"),
                                          _p(g_z, torch.float32, "g_z"), _p(ws, torch.uint8, "ws"),
                                          nbytes, _stream()))


def flow_forward_bn(desc, params, z, phi, logq, bn_mode, bn_stats=None, momentum=0.1, logdet=None,
                    saved_x=None, ws=None):
    """bn_mode BN_BATCH (bn_stats: running statistics updated in place, or None) or
    BN_RUNNING (bn_stats read)."""
    B = _field(z, _sites(desc), "z")
    V, _ = _flow_sizes(desc, params, B, saved_x, bn_stats)
    _need(phi, B * V, "phi")
    _need(logq, B, "logq")
    _need(logdet, B, "logdet")
    nbytes = ws.numel() if ws is not None else 0
    _check(load().lfs_flow_forward_bn(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                      _p(z, torch.float32, "z"), _p(phi, torch.float32, "phi"),
                                      _p(logq, torch.float64, "logq"),
                                      _p(logdet, torch.float64, "logdet"),
                                      _p(saved_x, torch.float32, "saved_x"), int(bn_mode),
                                      _p(bn_stats, torch.float32, "bn_stats"), float(momentum),
                                      _p(ws, torch.uint8, "ws"), nbytes, _stream()))


def flow_backward_vec(desc, params, saved_x, g_phi, g_logq, g_params, g_z=None, ws=None):
    """flow_backward with a per-sample cotangent of log q: g_logq is a [B] FP64 device tensor."""
    B = _field(g_phi, _sites(desc), "g_phi")
    if g_logq is None or g_logq.numel() != B:
        raise LfsError("g_logq needs one entry per sample")
    V, P = _flow_sizes(desc, params, B, saved_x)
    _need(saved_x, (desc.n_layers + 1) * B * V, "saved_x", exact=False)
    _need(g_params, P, "g_params")
    _need(g_z, B * V, "g_z")
    nbytes = ws.numel() if ws is not None else 0
    _check(load().lfs_flow_backward_vec(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                        _p(saved_x, torch.float32, "saved_x"),
                                        _p(g_phi, torch.float32, "g_phi"),
                                        _p(g_logq, torch.float64, "g_logq"),
                                        _p(g_params, torch.float32, "g_params"),
                                        _p(g_z, torch.float32, "g_z"), _p(ws, torch.uint8, "ws"),
                                        nbytes, _stream()))


def flow_backward_bn(desc, params, saved_x, g_phi, g_logq, g_params, bn_mode, bn_stats=None,
                     g_z=None, ws=None):
    """g_logq: a float (the same cotangent for every sample) or a [B] FP64 device tensor."""
    B = _field(g_phi, _sites(desc), "g_phi")
    V, P = _flow_sizes(desc, params, B, saved_x, bn_stats)
    _need(saved_x, (desc.n_layers + 1) * B * V, "saved_x", exact=False)
    _need(g_params, P, "g_params")
    _need(g_z, B * V, "g_z")
    nbytes = ws.numel() if ws is not None else 0
    vec = g_logq if isinstance(g_logq, torch.Tensor) else None
    if vec is not None and vec.numel() != B:
        raise LfsError("g_logq needs one entry per sample")
    scalar = 0.0 if vec is not None else float(g_logq)
    _check(load().lfs_flow_backward_bn(ctypes.byref(desc), _p(params, torch.float32, "params"), B,
                                       _p(saved_x, torch.float32, "saved_x"),
                                       _p(g_phi, torch.float32, "g_phi"), scalar,
                                       _p(vec, torch.float64, "g_logq"), int(bn_mode),
                                       _p(bn_stats, torch.float32, "bn_stats"),
                                       _p(g_params, torch.float32, "g_params"),
                                       _p(g_z, torch.float32, "g_z"), _p(ws, torch.uint8, "ws"),
                                       nbytes, _stream()))


def action(dim, L, phi, m2, lam, S, force=None, force_scale=1.0, precision=LFS_BF16_CONV):
    if dim not in (2, 3) or L < 2:
        raise LfsError(f"invalid lattice dim={dim} L={L}")
    B = _field(phi, L ** dim, "phi")
    _need(S, B, "S")
    _need(force, B * L ** dim, "force")
    per_sample = int(m2.numel() > 1)
    if m2.numel() not in (1, B) or lam.numel() != m2.numel():
        raise LfsError("m2 and lam must both have 1 or B entries")
    _check(load().lfs_action(dim, L, B, _p(phi, torch.float32, "phi"), _p(m2, torch.float64, "m2"),
                             _p(lam, torch.float64, "lam"), per_sample, precision,
                             _p(S, torch.float64, "S"), _p(force, torch.float32, "force"),
                             float(force_scale), _stream()))


def log_weights(S, logq, logw, loss=None):
    B = S.numel()
    _need(logq, B, "logq")
    _need(logw, B, "logw")
    _need(loss, 1, "loss")
    _check(load().lfs_log_weights(S.shape[0], _p(S, torch.float64, "S"),
                                  _p(logq, torch.float64, "logq"), _p(logw, torch.float64, "logw"),
                                  _p(loss, torch.float64, "loss"), _stream()))


def new_chain_state(n_chains: int, device="cuda"):
    """Zero-initialised lfs_chain_state array as raw bytes on the device."""
    return torch.zeros(n_chains * CHAIN_STATE_BYTES, dtype=torch.uint8, device=device)


def decode_chain_state(buf):
    """Host view of a chain-state byte tensor: list of dicts."""
    raw = buf.cpu().numpy().tobytes()
    out = []
    for i in range(len(raw) // CHAIN_STATE_BYTES):
        cs = ChainState.from_buffer_copy(raw[i * CHAIN_STATE_BYTES:(i + 1) * CHAIN_STATE_BYTES])
        out.append({f: getattr(cs, f) for f, _ in ChainState._fields_ if f != "reserved"})
    return out


def mh_chain(logw, log_u, state, cur_idx, accepted=None):
    if logw is None or logw.dim() != 2:
        raise LfsError("logw must be an [n_chains, n_prop] tensor")
    n_chains, n_prop = logw.shape
    _need(log_u, n_chains * n_prop, "log_u")
    _need(cur_idx, n_chains * n_prop, "cur_idx")
    _need(accepted, n_chains * n_prop, "accepted")
    if state.numel() < n_chains * CHAIN_STATE_BYTES:
        raise LfsError("chain state buffer too small")
    _check(load().lfs_mh_chain(n_chains, n_prop, _p(logw, torch.float64, "logw"),
                               _p(log_u, torch.float64, "log_u"), _p(state, torch.uint8, "state"),
                               _p(cur_idx, torch.int64, "cur_idx"),
                               _p(accepted, torch.uint8, "accepted"), _stream()))


def mh_chain_ragged(offsets, logw, log_u, states, state_index, cur_idx, accepted=None):
    """offsets: int64 [n_chains+1] device tensor; states: byte buffer of chain states.

    The offsets stay on the device, so what is checked here is that logw, log_u,
    cur_idx and accepted are equally long, that there is one state index per chain and
    room for that many states; the caller keeps offsets[-1] <= len(logw) and the state
    indices below the number of states."""
    n_chains = offsets.numel() - 1
    if n_chains < 0:
        raise LfsError("offsets needs n_chains + 1 entries")
    n = logw.numel()
    _need(log_u, n, "log_u")
    _need(cur_idx, n, "cur_idx")
    _need(accepted, n, "accepted")
    _need(state_index, n_chains, "state_index")
    _need(states, n_chains * CHAIN_STATE_BYTES, "states", exact=False)
    _check(load().lfs_mh_chain_ragged(n_chains, _p(offsets, torch.int64, "offsets"),
                                      _p(logw, torch.float64, "logw"),
                                      _p(log_u, torch.float64, "log_u"),
                                      _p(states, torch.uint8, "states"),
                                      _p(state_index, torch.int32, "state_index"),
                                      _p(cur_idx, torch.int64, "cur_idx"),
                                      _p(accepted, torch.uint8, "accepted"), _stream()))


def hmc_step(dim, L, phi, pi0, log_u, m2, lam, n_steps, dt, dH, accepted):
    if dim not in (2, 3) or L < 2:
        raise LfsError(f"invalid lattice dim={dim} L={L}")
    B = _field(phi, L ** dim, "phi")
    _need(pi0, B * L ** dim, "pi0")
    _need(log_u, B, "log_u")
    _need(dH, B, "dH")
    _need(accepted, B, "accepted")
    if m2.numel() not in (1, B) or lam.numel() != m2.numel():
        raise LfsError("m2 and lam must both have 1 or B entries")
    per_sample = int(m2.numel() > 1)
    _check(load().lfs_hmc_step(dim, L, B, _p(phi, torch.float64, "phi"),
                               _p(pi0, torch.float64, "pi0"), _p(log_u, torch.float64, "log_u"),
                               _p(m2, torch.float64, "m2"), _p(lam, torch.float64, "lam"),
                               per_sample, n_steps, float(dt), _p(dH, torch.float64, "dH"),
                               _p(accepted, torch.uint8, "accepted"), _stream()))


def adam_step(p, g, m, v, lr, b1, b2, eps, t):
    for t_, name in ((g, "g"), (m, "m"), (v, "v")):
        _need(t_, p.numel(), name)
    _check(load().lfs_adam_step(p.numel(), _p(p, torch.float32, "p"), _p(g, torch.float32, "g"),
                                _p(m, torch.float32, "m"), _p(v, torch.float32, "v"), lr, b1, b2,
                                eps, t, _stream()))


def observables(dim, L, phi, M=None, C=None):
    """Condensate M [B] and zero-momentum two-point function C [B, L] (FP64) of phi [B, V]."""
    if phi.dtype not in (torch.float32, torch.float64):
        raise LfsError("phi must be float32 or float64")
    if dim not in (2, 3) or L < 2:
        raise LfsError(f"invalid lattice dim={dim} L={L}")
    B = _field(phi, L ** dim, "phi")
    _need(M, B, "M")
    _need(C, B * L, "C")
    _check(load().lfs_observables(dim, L, B, _p(phi, None, "phi"), int(phi.dtype == torch.float64),
                                  _p(M, torch.float64, "M"), _p(C, torch.float64, "C"), _stream()))


def autocorr_workspace_bytes(n_series: int, n: int, w_max: int) -> int:
    return int(load().lfs_autocorr_workspace_bytes(n_series, n, w_max))


def autocorr(x, w_max: int, c: float, tau, window=None, found=None, n_indep=None, gamma=None,
             index=None, n=None, ws=None):
    """Windowed integrated autocorrelation time of the rows of x [n_series, ldx] (FP64).

    Without index the series are the first n (default: all) entries of each row;
    with index [n_series, n] (int64) entry k of series s is x[s, index[s, k]]."""
    n_series, ldx = x.shape
    if index is not None:
        n = index.shape[1]
    elif n is None:
        n = ldx
    if index is not None:
        _need(index, n_series * n, "index")
    elif n > ldx:
        raise LfsError(f"series of {n} entries do not fit rows of {ldx}")
    _need(gamma, n_series * (w_max + 1), "gamma")
    _need(tau, n_series, "tau")
    for t_, name in ((window, "window"), (found, "found"), (n_indep, "n_indep")):
        _need(t_, n_series, name)
    need = autocorr_workspace_bytes(n_series, n, w_max)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    _check(load().lfs_autocorr(n_series, n, _p(x, torch.float64, "x"), ldx,
                               _p(index, torch.int64, "index"), w_max, float(c),
                               _p(gamma, torch.float64, "gamma"), _p(tau, torch.float64, "tau"),
                               _p(window, torch.int32, "window"), _p(found, torch.uint8, "found"),
                               _p(n_indep, torch.float64, "n_indep"), _p(ws, torch.uint8, "ws"),
                               ws.numel(), _stream()))


def ess(logw, out):
    """Normalised reweighting ESS of each row of logw [n_series, n] (FP64) into out [n_series]."""
    if logw.dim() == 1:
        logw = logw.reshape(1, -1)
    n_series, n = logw.shape
    _need(out, n_series, "ess")
    _check(load().lfs_ess(n_series, n, _p(logw, torch.float64, "logw"), n,
                          _p(out, torch.float64, "ess"), _stream()))

"""Helpers shared by the GPU parity tests: device tensors and the oracle side by side."""
import numpy as np
import torch

from paper_2208_08903_amd import lfs

DEV = "cuda"


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def host(t):
    return t.detach().cpu().numpy()


def flow_buffers(desc, B, with_saved=True):
    V = desc.L ** desc.dim
    d = dict(
        phi=torch.empty(B, V, device=DEV, dtype=torch.float32),
        logq=torch.empty(B, device=DEV, dtype=torch.float64),
        logdet=torch.empty(B, device=DEV, dtype=torch.float64),
        saved=torch.empty((desc.n_layers + 1) * B * V, device=DEV, dtype=torch.float32)
        if with_saved else None,
        ws=torch.empty(max(lfs.workspace_bytes(desc, B, False), 1), device=DEV, dtype=torch.uint8),
    )
    return d


def run_forward(desc, params_np, z_np, with_saved=True):
    B = z_np.shape[0]
    b = flow_buffers(desc, B, with_saved)
    params = dev(params_np, torch.float32)
    z = dev(z_np, torch.float32)
    lfs.flow_forward(desc, params, z, b["phi"], b["logq"], b["logdet"], b["saved"], b["ws"])
    torch.cuda.synchronize()
    b["params"], b["z"] = params, z
    return b


def run_backward(desc, fwd, g_phi_np, g_logq, want_gz=True):
    B = g_phi_np.shape[0]
    V = desc.L ** desc.dim
    ws = torch.empty(max(lfs.workspace_bytes(desc, B, True), 1), device=DEV, dtype=torch.uint8)
    gp = torch.empty_like(fwd["params"])
    gz = torch.empty(B, V, device=DEV, dtype=torch.float32) if want_gz else None
    lfs.flow_backward(desc, fwd["params"], fwd["saved"], dev(g_phi_np, torch.float32), g_logq, gp,
                      gz, ws)
    torch.cuda.synchronize()
    return host(gp), (host(gz) if want_gz else None)


def rel_norm(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)

"""The flow as a torch.autograd.Function: the library's forward and its
hand-written backward kernels (paper Sec. 1, coupling-layer and composition
equations; reverse-KL training), so that (phi, log q) can enter any torch loss
and optimiser.

    phi, logq = flow_apply(flow, z)              # differentiable in flow.params and z

forward   lfs_flow_forward (lfs_flow_forward_bn for batch-norm flows), keeping
          the N + 1 layer inputs for the backward (each layer's hidden
          activations are recomputed from them there)
backward  lfs_flow_backward_vec (lfs_flow_backward_bn), with the per-sample
          cotangent of log q that autograd hands over

Both directions run entirely in the library's kernels; this module allocates
the outputs and passes pointers.  A cotangent autograd leaves out (an output
not used by the loss) is passed as zeros.
"""
from __future__ import annotations

import torch

from . import lfs


class FlowFunction(torch.autograd.Function):
    """apply(params, z, flow, train) -> (phi [B, V] FP32, logq [B] FP64)."""

    @staticmethod
    def forward(ctx, params, z, flow, train):
        if params.dtype != torch.float32 or z.dtype != torch.float32:
            raise lfs.LfsError("params and z must be float32")
        params, z = params.contiguous(), z.contiguous()
        B, dev = z.shape[0], z.device
        phi = torch.empty(B, flow.V, dtype=torch.float32, device=dev)
        logq = torch.empty(B, dtype=torch.float64, device=dev)
        saved = torch.empty((flow.n_layers + 1) * B * flow.V, dtype=torch.float32, device=dev)
        ws = flow.workspace(B, False)
        if flow.batch_norm:
            mode = lfs.BN_BATCH if train else lfs.BN_RUNNING
            lfs.flow_forward_bn(flow.desc, params, z, phi, logq, mode, flow.bn_stats,
                                flow.bn_momentum if train else 0.0, None, saved, ws)
        else:
            lfs.flow_forward(flow.desc, params, z, phi, logq, None, saved, ws)
        ctx.flow, ctx.train, ctx.saved_x = flow, train, saved
        ctx.save_for_backward(params)   # autograd then rejects a backward after params changed in place
        return phi, logq

    @staticmethod
    def backward(ctx, g_phi, g_logq):
        (params,) = ctx.saved_tensors
        flow, saved = ctx.flow, ctx.saved_x
        B = saved.numel() // ((flow.n_layers + 1) * flow.V)
        dev = saved.device
        if g_phi is None:
            g_phi = torch.zeros(B, flow.V, dtype=torch.float32, device=dev)
        g_phi = g_phi.to(torch.float32).contiguous()
        if g_logq is None:
            g_logq = torch.zeros(B, dtype=torch.float64, device=dev)
        g_logq = g_logq.to(torch.float64).contiguous()
        g_params = torch.empty_like(params)
        g_z = torch.empty(B, flow.V, dtype=torch.float32, device=dev) if ctx.needs_input_grad[1] else None
        ws = flow.workspace(B, True)
        if flow.batch_norm:
            mode = lfs.BN_BATCH if ctx.train else lfs.BN_RUNNING
            lfs.flow_backward_bn(flow.desc, params, saved, g_phi, g_logq, g_params, mode, flow.bn_stats,
                                 g_z, ws)
        else:
            lfs.flow_backward_vec(flow.desc, params, saved, g_phi, g_logq, g_params, g_z, ws)
        return (g_params if ctx.needs_input_grad[0] else None), g_z, None, None


def flow_apply(flow, z, train: bool = True, params=None):
    """(phi, log q) of the prior sample z [B, V] under `flow`, differentiable in the
    parameters (flow.params unless `params` is given; set requires_grad on it) and z.
    Batch-norm flows use batch statistics when train is True (updating the running
    ones) and the running statistics otherwise."""
    return FlowFunction.apply(flow.params if params is None else params, z, flow, train)

"""Weighted BP as a differentiable torch operation.

``WeightedBP.apply(llr, w, ctx_obj)`` runs ``wbp_forward`` (which checkpoints
the per-iteration R messages in a device workspace) and, on backward,
``wbp_backward`` (the hand-written adjoint kernel) for the weight gradient.
The channel LLRs are treated as data (no gradient).  ``WeightedBPDecoder``
holds the learnable weights w[T][n][2][N], initialised to 1 (plain min-sum
BP), and the workspace.
"""
from __future__ import annotations

import torch

from . import api


class _WbpState:
    """Code, schedule and a reusable workspace for one decoder."""

    def __init__(self, code: api.Code, T: int, pp: api.PPParams | None):
        self.code, self.T, self.pp = code, T, pp
        self.ws = None
        self.ws_frames = -1

    def workspace(self, F: int, device) -> torch.Tensor:
        need = api.wbp_workspace_bytes(self.code, F, self.T)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
        return self.ws


class WeightedBP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, llr, w, state: _WbpState):
        F = llr.shape[0]
        out = torch.empty((F, state.code.N), dtype=torch.float32, device=llr.device)
        ws = state.workspace(F, llr.device)
        api.wbp_forward(state.code, llr, w.detach(), state.pp, out, ws)
        ctx.save_for_backward(llr, w)
        ctx.state = state
        return out

    @staticmethod
    def backward(ctx, grad_out):
        llr, w = ctx.saved_tensors
        state = ctx.state
        gw = torch.empty_like(w)
        # the checkpoints of the forward call are still in the workspace
        api.wbp_backward(state.code, llr, w.detach(), state.pp, grad_out.contiguous(), gw,
                         state.ws)
        return None, gw, None


class WeightedBPDecoder(torch.nn.Module):
    """Unrolled weighted min-sum BP with weights per iteration, stage, sweep and row."""

    def __init__(self, code: api.Code, T: int, pp: api.PPParams | None = None, device="cuda"):
        super().__init__()
        self.code, self.T = code, T
        self.weight = torch.nn.Parameter(torch.ones((T, code.n, 2, code.N), dtype=torch.float32,
                                                    device=device))
        self._state = _WbpState(code, T, pp)

    def forward(self, llr):
        return WeightedBP.apply(llr, self.weight, self._state)


def bce_on_information_bits(out_llr, u_info_bits, info_idx):
    """Mean binary cross entropy of the output LLRs at the information rows.

    LLR > 0 favours bit 0, so P(bit = 1) = sigmoid(-LLR) and the loss of a row
    is u softplus(o) + (1 - u) softplus(-o).
    """
    o = out_llr[:, info_idx]
    u = u_info_bits.to(o.dtype)
    return (u * torch.nn.functional.softplus(o) + (1 - u) * torch.nn.functional.softplus(-o)).mean()

"""Weighted BP as a differentiable torch operation.

``WeightedBP.apply(llr, w, state, keep)`` runs ``wbp_forward`` (which checkpoints
the per-iteration R messages in a device workspace owned by that call's
autograd context) and, on backward, ``wbp_backward`` (the hand-written adjoint
kernel) for the weight gradient.  With keep=False (the decoder passes it under
torch.no_grad() or for frozen weights) the forward pass runs alone, without
checkpoints.  The channel LLRs are treated as
data (no gradient).  ``WeightedBPDecoder`` holds the learnable weights
w[T][n][2][N], initialised to 1 (plain min-sum BP).
"""
from __future__ import annotations

import torch

from . import api


class _WbpState:
    """Code and schedule of one decoder."""

    def __init__(self, code: api.Code, T: int, pp: api.PPParams | None):
        self.code, self.T, self.pp = code, T, pp

    def workspace(self, F: int, device) -> torch.Tensor:
        # one per forward call (from torch's caching allocator), so that a
        # second forward before the first backward cannot overwrite the
        # first call's checkpoints
        need = api.wbp_workspace_bytes(self.code, F, self.T)
        return torch.empty(max(need, 1), dtype=torch.uint8, device=device)


class WeightedBP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, llr, w, state: _WbpState, keep: bool = True):
        F = llr.shape[0]
        out = torch.empty((F, state.code.N), dtype=torch.float32, device=llr.device)
        ws = state.workspace(F, llr.device) if keep else None
        api.wbp_forward(state.code, llr, w.detach(), state.pp, out, ws)
        ctx.save_for_backward(llr, w)
        ctx.state = state
        ctx.ws = ws
        return out

    @staticmethod
    def backward(ctx, grad_out):
        llr, w = ctx.saved_tensors
        state = ctx.state
        if ctx.ws is None:
            raise RuntimeError("weighted BP forward ran without checkpoints (keep=False), or its "
                               "backward already ran: no backward")
        gw = torch.empty_like(w)
        api.wbp_backward(state.code, llr, w.detach(), state.pp, grad_out.contiguous(), gw, ctx.ws)
        # the checkpoints serve this one backward: release them now rather
        # than with the graph, which a caller holding the loss keeps alive
        ctx.ws = None
        return None, gw, None, None


class WeightedBPDecoder(torch.nn.Module):
    """Unrolled weighted min-sum BP with weights per iteration, stage, sweep and row."""

    def __init__(self, code: api.Code, T: int, pp: api.PPParams | None = None, device="cuda"):
        super().__init__()
        self.code, self.T = code, T
        self.weight = torch.nn.Parameter(torch.ones((T, code.n, 2, code.N), dtype=torch.float32,
                                                    device=device))
        self._state = _WbpState(code, T, pp)

    def forward(self, llr):
        keep = torch.is_grad_enabled() and self.weight.requires_grad
        return WeightedBP.apply(llr, self.weight, self._state, keep)


def bce_on_information_bits(out_llr, u_info_bits, info_idx):
    """Mean binary cross entropy of the output LLRs at the information rows.

    LLR > 0 favours bit 0, so P(bit = 1) = sigmoid(-LLR) and the loss of a row
    is u softplus(o) + (1 - u) softplus(-o): the binary cross entropy of
    logit o against the target 1 - u, which torch evaluates in one fused
    kernel each way.
    """
    # a gather, whose adjoint is a scatter-add; advanced indexing would
    # adjoin through index_put with accumulation, which sorts the indices
    idx = info_idx.view(1, -1).expand(out_llr.shape[0], -1)
    o = torch.gather(out_llr, 1, idx)
    target = 1 - u_info_bits.to(o.dtype)
    return torch.nn.functional.binary_cross_entropy_with_logits(o, target)

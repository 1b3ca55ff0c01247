"""Mixed-length batched decoding: round buffers and HIP-graph capture.

A ``BatchedDecoder`` owns the device buffers of one round (LLR pool, offsets,
code ids, decided-bit pool, iteration counts, verdicts, queue workspace).
``capture()`` records one call of ``pp_mt_bp_decode_batched`` -- the queue
preparation kernels and the persistent decoder -- into a torch CUDA graph
(a hipGraph on ROCm); ``replay()`` runs the round again on whatever frame
data the buffers hold.  No memset nodes are recorded: the library clears its
counters with a kernel.

The mixed workload that bench.py times lives beside it
(``bench_workloads.py``).
"""
from __future__ import annotations

from . import api


# the mixed stream: 4 block lengths x 5 rates, CRC-16, K counts the CRC
MIXED_N = (128, 256, 512, 1024)
MIXED_R = (1 / 4, 1 / 3, 1 / 2, 2 / 3, 3 / 4)


def mixed_codes(design_db: float = 2.5):
    codes = []
    for N in MIXED_N:
        for R in MIXED_R:
            codes.append(api.Code(N, int(round(R * N)), 16, 0x1021, design_db))
    return codes


class BatchedDecoder:
    """Fixed-size round of F frames over a list of codes."""

    def __init__(self, codes, F: int, bp: api.BPParams, pp: api.PPParams | None,
                 cfg: api.LaunchCfg | None = None, device="cuda"):
        import torch
        self.codes, self.F, self.bp, self.pp, self.cfg = codes, F, bp, pp, cfg
        self.N = torch.tensor([c.N for c in codes], dtype=torch.int64, device=device)
        self.Kmsg = torch.tensor([c.K_msg for c in codes], dtype=torch.int64, device=device)
        max_n = max(c.N for c in codes)
        max_k = max(c.K_msg for c in codes)
        self.code_id = torch.zeros(F, dtype=torch.int32, device=device)
        self.llr_off = torch.zeros(F, dtype=torch.int64, device=device)
        self.bits_off = torch.zeros(F, dtype=torch.int64, device=device)
        self.llr_pool = torch.zeros(F * max_n, dtype=torch.float32, device=device)
        self.bits_pool = torch.zeros(F * max_k, dtype=torch.uint8, device=device)
        self.iters = torch.zeros(F, dtype=torch.int32, device=device)
        self.ok = torch.zeros(F, dtype=torch.uint8, device=device)
        self.ws = torch.empty(api.batched_workspace_bytes(F), dtype=torch.uint8, device=device)
        self.graph = None

    def set_layout(self, code_id):
        """Assign each frame its code; offsets pack frames back to back."""
        import torch
        cid = code_id.to(torch.int64)
        n = self.N[cid]
        k = self.Kmsg[cid]
        self.code_id.copy_(code_id.to(torch.int32))
        self.llr_off.copy_(torch.cumsum(n, 0) - n)
        self.bits_off.copy_(torch.cumsum(k, 0) - k)

    def run(self):
        api.decode_batched(self.codes, self.code_id, self.llr_off, self.llr_pool, self.bp, self.pp,
                           self.bits_pool, self.bits_off, self.iters, self.ok, self.ws, self.cfg)

    def capture(self):
        import torch
        self.run()                      # warm-up outside capture (occupancy, tables)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

"""Mixed-length batched decoding: round buffers and HIP-graph capture.

A ``BatchedDecoder`` owns the device buffers of one round (LLR pool, offsets,
code ids, decided-bit pool, iteration counts, verdicts, queue workspace).
``capture()`` records one call of ``pp_mt_bp_decode_batched`` -- the queue
preparation kernels and the persistent decoder -- into a torch CUDA graph
(a hipGraph on ROCm); ``replay()`` runs the round again on whatever frame
data the buffers hold.  No memset nodes are recorded: the library clears its
counters with a kernel.

``make_mixed_stream`` draws the mixed workload (code per frame, Eb/N0 per
frame, message bits) and fills a round with encoded, AWGN-corrupted frames;
``bench_mixed`` times rounds of it for bench.py.
"""
from __future__ import annotations

import sys

from . import api


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def make_mixed_stream(torch, dec: BatchedDecoder, seed: int, lo_db=1.0, hi_db=4.0):
    """Fill a round: code uniform over dec.codes, Eb/N0 uniform on [lo, hi] dB
    per frame, uniform message bits; encoded on the GPU, BPSK over AWGN.
    Returns the messages per code group for error counting."""
    import synth
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    F = dec.F
    cid = torch.randint(0, len(dec.codes), (F,), generator=gen, device="cuda")
    dec.set_layout(cid)
    ebn0 = torch.rand(F, generator=gen, device="cuda", dtype=torch.float64) * (hi_db - lo_db) + lo_db
    groups = []
    for c_i, code in enumerate(dec.codes):
        idx = torch.nonzero(cid == c_i).flatten()
        if idx.numel() == 0:
            groups.append((idx, None))
            continue
        m = torch.randint(0, 2, (idx.numel(), code.K_msg), generator=gen, device="cuda",
                          dtype=torch.uint8)
        x = api.encode(code, m)
        llr = synth.awgn_llr_torch(x, ebn0[idx], code.K_msg, gen)
        # scatter the frames into the pool
        off = dec.llr_off[idx]
        cols = torch.arange(code.N, device="cuda")
        dec.llr_pool[(off[:, None] + cols[None, :]).flatten()] = llr.flatten()
        groups.append((idx, m))
    torch.cuda.synchronize()
    return groups


def frame_errors(torch, dec: BatchedDecoder, groups):
    errs = 0
    for c_i, (idx, m) in enumerate(groups):
        if m is None:
            continue
        code = dec.codes[c_i]
        off = dec.bits_off[idx]
        cols = torch.arange(code.K_msg, device="cuda")
        got = dec.bits_pool[(off[:, None] + cols[None, :])]
        errs += int((got != m).any(1).sum().item())
    return errs


def bench_mixed(torch, pbp, frames_total=4_000_000, rounds=4, cfg=None):
    """The mixed-length stream: frames_total frames in `rounds` graph-captured
    rounds.  Throughput counts decoded message bits of every frame."""
    bp = api.BPParams(max_iter=200, stop=api.STOP_CRC, it_min=3)
    pp = api.PPParams(mode=api.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=1)
    codes = mixed_codes()
    F = frames_total // rounds
    decs, groups = [], []
    for r in range(rounds):
        d = BatchedDecoder(codes, F, bp, pp, cfg)
        groups.append(make_mixed_stream(torch, d, seed=500 + r))
        if r == 0 and cfg is None:
            from .tune import tune_batched
            cfg, tuned = tune_batched(torch, d, path="/tmp/polarbp_tuned.json", force=True)
            _log(f"mixed stream tuned launch shape {tuned['all']}")
        d.cfg = cfg
        d.capture()
        decs.append(d)
    _log(f"mixed stream: {rounds} captured rounds of {F} frames")
    for d in decs:
        d.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for d in decs:
        d.replay()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    bits = sum(int(d.Kmsg[d.code_id.to(torch.int64)].sum().item()) for d in decs)
    errs = sum(frame_errors(torch, d, g) for d, g in zip(decs, groups))
    iters = torch.cat([d.iters for d in decs]).double()
    # algorithmic VALU lane-ops as for the single-length decoder: 6 per
    # processing element, N/2 per stage, n stages per L sweep and n-1 live
    # stages per R sweep (the deciding iteration runs no R sweep)
    ops = 0.0
    for d in decs:
        Nf = d.N[d.code_id.to(torch.int64)].double()
        nf = torch.log2(Nf)
        it = d.iters.double()
        ops += (3 * Nf * (nf * it + (nf - 1) * (it - 1))).sum().item()
    alu_peak = 256 * 64 * 2.4e9
    _log(f"mixed stream: {ms:.1f} ms")
    out = {"workload": f"{frames_total} frames, N ~ U{{128,256,512,1024}}, R ~ U{{1/4,1/3,1/2,2/3,3/4}}, "
                       "CRC-16, Eb/N0 ~ U[1,4] dB, PP-MT-BP k=4 T=10 Q=8, max 200 iterations, "
                       f"{rounds} hipGraph-captured rounds",
           "gbit_s": round(bits / (ms / 1e3) / 1e9, 3), "ms": round(ms, 2),
           "frames_s": round(frames_total / (ms / 1e3), 1),
           "avg_iters": round(iters.mean().item(), 3), "fer": errs / frames_total,
           "alu_frac": round(ops / (ms / 1e3) / alu_peak, 4),
           "launch": {"rho": cfg.rho, "slots": cfg.slots}}
    del decs
    torch.cuda.empty_cache()
    return out

"""Side workloads measured by bench.py beside the headline decode.

weighted_bp(): the weighted-BP training step (N = 256, K = 128 message bits +
CRC-16, 10 unrolled iterations, batch 16384, Eb/N0 uniform on [1, 4] dB per
frame, binary cross entropy of the output LLRs against the transmitted
information bits) timed forward + backward + SGD step, next to plain min-sum
BP decoding of the same frames.

batched_mixed(): the mixed-length stream through the persistent queue kernel
(see batched.py).
"""
from __future__ import annotations

import sys


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def polar_transform_torch(x, n):
    """u = x G_N on the device (G_N is an involution), for loss targets."""
    u = x.clone()
    F = u.shape[0]
    for b in range(n):
        v = u.view(F, -1, 2, 1 << b)
        v[:, :, 0, :] ^= v[:, :, 1, :]
    return u


def weighted_bp(torch, pbp, steps=5, warmup=2, F=16384, T=10):
    import synth
    from .wbp import WeightedBPDecoder, bce_on_information_bits
    code = pbp.Code(256, 144, 16, 0x1021, 2.5)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(77)
    m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
    x = pbp.encode(code, m)
    ebn0 = torch.rand(F, generator=gen, device="cuda", dtype=torch.float64) * 3.0 + 1.0
    llr = synth.awgn_llr_torch(x, ebn0, code.K_msg, gen)
    u = polar_transform_torch(x, code.n)
    info = torch.from_numpy(code.info_idx.astype("int64")).cuda()
    u_info = u[:, info]
    dec = WeightedBPDecoder(code, T)
    opt = torch.optim.SGD(dec.parameters(), lr=1e-2)

    def step():
        out = dec(llr)
        loss = bce_on_information_bits(out, u_info, info)
        opt.zero_grad(set_to_none=False)
        loss.backward()
        opt.step()
        return loss

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        loss = step()
    b.record()
    torch.cuda.synchronize()
    ms_train = a.elapsed_time(b) / steps
    # forward only
    with torch.no_grad():
        a.record()
        for _ in range(steps):
            out = dec(llr)
        b.record()
        torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b) / steps
    # plain BP, same frames, same iteration budget
    bp = pbp.BPParams(max_iter=T, stop=pbp.STOP_NONE)
    outs = pbp.bp_decode(code, llr, bp)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        pbp.bp_decode(code, llr, bp, out=outs)
    b.record()
    torch.cuda.synchronize()
    ms_plain = a.elapsed_time(b) / steps
    with torch.no_grad():
        fer_w = ((dec(llr)[:, info] < 0).to(torch.uint8) != u_info).any(1).double().mean().item()
    fer_p = (outs[0] != m).any(1).double().mean().item()
    _log(f"weighted BP: train step {ms_train:.2f} ms, forward {ms_fwd:.2f} ms, plain {ms_plain:.2f} ms")
    return {"workload": "weighted BP training, N=256 K=128+CRC16, 10 unrolled iterations, "
                        "batch 16384, Eb/N0 ~ U[1,4] dB, BCE on information bits, SGD",
            "fwd_bwd_frames_s": round(F / (ms_train / 1e3), 1),
            "fwd_frames_s": round(F / (ms_fwd / 1e3), 1),
            "plain_bp_frames_s": round(F / (ms_plain / 1e3), 1),
            "ms_train_step": round(ms_train, 3), "ms_forward": round(ms_fwd, 3),
            "ms_plain_decode": round(ms_plain, 3),
            "loss": round(float(loss.item()), 5),
            "fer_weighted_after_steps": fer_w, "fer_plain": fer_p}


def bench_extras(torch, pbp):
    from .batched import bench_mixed
    out = {}
    for name, fn in (("weighted_bp", weighted_bp), ("batched_mixed", bench_mixed)):
        try:
            out[name] = fn(torch, pbp)
        except Exception as e:  # report the failure in the JSON line, keep the rest
            out[name] = None
            out.setdefault("extras_errors", {})[name] = f"{type(e).__name__}: {e}"
            _log(f"{name} failed: {e}")
        torch.cuda.empty_cache()
    return out

"""Side workloads measured by bench.py beside the headline decode (benchmark
harness code: it drives the library through its Python binding and holds no
step of the decoder).

weighted_bp(): the weighted-BP training step (N = 256, K = 128 message bits +
CRC-16, 10 unrolled iterations, batch 16384, Eb/N0 uniform on [1, 4] dB per
frame, binary cross entropy of the output LLRs against the transmitted
information bits) timed forward + backward + SGD step, next to plain min-sum
BP decoding of the same frames.

weighted_bp_large(): the same at N=4096 with the last-5 trellis schedule and
20 unrolled iterations, beside unit-weight PP-MT-BP decoding.

batched_mixed(): the mixed-length stream through the persistent queue kernel
(rounds captured by paper_1911_08868_amd.batched.BatchedDecoder).

alg1_table1(): Algorithm 1 with random subgraphs (Table I parameters) beside
the fixed last-k schedule.
"""
from __future__ import annotations

import sys


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ALU peak of the processing element's instruction mix in lane-ops per second:
# 256 CUs x 2.4 GHz x 96 (2 v_add_f32 and 2 v_bitop3_b32 at 128 lanes per
# CU-clock, 2 v_med3_f32 at 64); bench.py replaces it by its calibrated value
# when that is larger.
ALU_PEAK = 256 * 96 * 2.4e9


def clopper_pearson(k: int, n: int, conf: float = 0.95):
    """Exact binomial (Clopper-Pearson) interval of k errors in n frames."""
    from scipy.stats import beta
    a = (1.0 - conf) / 2.0
    lo = float(beta.ppf(a, k, n - k + 1)) if k > 0 else 0.0
    hi = float(beta.ppf(1.0 - a, k + 1, n - k)) if k < n else 1.0
    return [lo, hi]


def _fresh_frames(torch, pbp, code, F, ebn0, gen):
    """F random messages, encoded by the library, over BPSK-AWGN at ebn0 (a
    scalar or a per-frame tensor) -> (messages, LLRs)."""
    import synth
    m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
    e = ebn0 if torch.is_tensor(ebn0) else torch.full((F,), float(ebn0), device="cuda", dtype=torch.float64)
    return m, synth.awgn_llr_torch(pbp.encode(code, m), e, code.K_msg, gen)


def _train_weighted(torch, pbp, code, dec, opt, steps, F, lo_db, hi_db, seed, clip=None):
    """SGD-type training on fresh frames every step (Eb/N0 ~ U[lo, hi] dB per
    frame): BCE of the output LLRs against u on the information rows (the
    message and its CRC, from polar_info_bits).  Returns the last losses."""
    from paper_1911_08868_amd.wbp import bce_on_information_bits
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    info = torch.from_numpy(code.info_idx.astype("int64")).cuda()
    losses = []
    for _ in range(steps):
        e = torch.rand(F, generator=gen, device="cuda", dtype=torch.float64) * (hi_db - lo_db) + lo_db
        m, llr = _fresh_frames(torch, pbp, code, F, e, gen)
        loss = bce_on_information_bits(dec(llr), pbp.info_bits(code, m), info)
        opt.zero_grad()
        loss.backward()
        if clip:
            torch.nn.utils.clip_grad_norm_(dec.parameters(), clip)
        opt.step()
        losses.append(loss.detach())
    return [round(float(x.item()), 5) for x in losses[-3:]]


def _fer_learned_vs_unit(torch, pbp, code, dec, pp, T, snrs, F, seed, chunk=65536):
    """Held-out frames (their own generator seed) at fixed Eb/N0 points: frame
    errors on the message bits of the learned weights, of unit weights through
    the same unrolled forward (no early stop), and of the library's
    PP-MT-BP / BP decoder with unit weights (CRC stop from iteration 3, at
    most T iterations), each with a 95% Clopper-Pearson interval (the frame
    error rate method of Sec. IV)."""
    from paper_1911_08868_amd.wbp import WeightedBPDecoder
    unit = WeightedBPDecoder(code, T, pp)
    msg_rows = torch.from_numpy(code.info_idx[:code.K_msg].astype("int64")).cuda()
    bp = pbp.BPParams(max_iter=T, stop=pbp.STOP_CRC, it_min=3)
    out = []
    for si, snr in enumerate(snrs):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed + 1000 * si)
        errs = {"learned": 0, "unit": 0, "decoder": 0}
        for c0 in range(0, F, chunk):
            f = min(chunk, F - c0)
            m, llr = _fresh_frames(torch, pbp, code, f, snr, gen)
            with torch.no_grad():
                for name, d in (("learned", dec), ("unit", unit)):
                    hat = (d(llr)[:, msg_rows] < 0).to(torch.uint8)
                    errs[name] += int((hat != m).any(1).sum().item())
            res = pbp.pp_mt_bp_decode(code, llr, bp, pp) if pp is not None else pbp.bp_decode(code, llr, bp)
            errs["decoder"] += int((res[0] != m).any(1).sum().item())
        row = {"ebn0_db": snr, "frames": F}
        for name, e in errs.items():
            row[name] = {"frame_errors": e, "fer": e / F, "ci95": clopper_pearson(e, F)}
        out.append(row)
        _log(f"learned vs unit weights N={code.N} at {snr} dB: fer {row['learned']['fer']:.4g} "
             f"vs {row['unit']['fer']:.4g} (decoder with CRC stop {row['decoder']['fer']:.4g})")
    return out


def _time_train_step(torch, pbp, code, dec, opt, llr, u_info, steps, warmup, clip=None):
    from paper_1911_08868_amd.wbp import bce_on_information_bits
    info = torch.from_numpy(code.info_idx.astype("int64")).cuda()

    def step():
        loss = bce_on_information_bits(dec(llr), u_info, info)
        opt.zero_grad()
        loss.backward()
        if clip:
            torch.nn.utils.clip_grad_norm_(dec.parameters(), clip)
        opt.step()
        return loss

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def weighted_bp(torch, pbp, steps=5, warmup=2, F=16384, T=10, epochs=10, epoch_frames=983_040,
                lr=1e-2, eval_frames=200_000, snrs=(1.5, 2.0, 2.5, 3.0, 3.5)):
    """Weighted BP at N = 256, K = 128 + CRC-16, 10 unrolled iterations, batch
    16384, Eb/N0 ~ U[1,4] dB per frame, BCE on the information rows.  Timed:
    the training step (forward with checkpoints, loss, adjoint, reduction,
    optimiser step), the forward alone and plain BP with the same 10
    iterations on the same frames.  Then whether the learned weights pay
    off: `epochs` epochs of `epoch_frames` fresh frames (Adam), and frame
    error rates of learned against unit weights on held-out frames."""
    from paper_1911_08868_amd.wbp import WeightedBPDecoder
    code = pbp.Code(256, 144, 16, 0x1021, 2.5)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(77)
    e = torch.rand(F, generator=gen, device="cuda", dtype=torch.float64) * 3.0 + 1.0
    m, llr = _fresh_frames(torch, pbp, code, F, e, gen)
    u_info = pbp.info_bits(code, m)
    tdec = WeightedBPDecoder(code, T)
    ms_train = _time_train_step(torch, pbp, code, tdec, torch.optim.SGD(tdec.parameters(), lr=1e-2),
                                llr, u_info, steps, warmup)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.no_grad():
        a.record()
        for _ in range(steps):
            tdec(llr)
        b.record()
        torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b) / steps
    bp = pbp.BPParams(max_iter=T, stop=pbp.STOP_NONE)
    outs = pbp.bp_decode(code, llr, bp)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        pbp.bp_decode(code, llr, bp, out=outs)
    b.record()
    torch.cuda.synchronize()
    ms_plain = a.elapsed_time(b) / steps
    _log(f"weighted BP: train step {ms_train:.2f} ms, forward {ms_fwd:.2f} ms, plain {ms_plain:.2f} ms")
    # payoff: train on fresh frames, evaluate on held-out ones
    dec = WeightedBPDecoder(code, T)
    opt = torch.optim.Adam(dec.parameters(), lr=lr)
    n_steps = epochs * (epoch_frames // F)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    losses = _train_weighted(torch, pbp, code, dec, opt, n_steps, F, 1.0, 4.0, seed=2001)
    t1.record()
    torch.cuda.synchronize()
    fer = _fer_learned_vs_unit(torch, pbp, code, dec, None, T, snrs, eval_frames, seed=9001)
    w = dec.weight.detach()
    return {"workload": f"weighted BP, N=256 K=128+CRC16, {T} unrolled iterations, batch {F}, "
                        f"Eb/N0 ~ U[1,4] dB, BCE on the information rows",
            "fwd_bwd_frames_s": round(F / (ms_train / 1e3), 1),
            "fwd_frames_s": round(F / (ms_fwd / 1e3), 1),
            "plain_bp_frames_s": round(F / (ms_plain / 1e3), 1),
            "ms_train_step": round(ms_train, 3), "ms_forward": round(ms_fwd, 3),
            "ms_plain_decode": round(ms_plain, 3),
            "payoff": {"training": f"{epochs} epochs x {epoch_frames} fresh frames ({n_steps} steps of {F}), "
                                   f"Adam lr {lr}, Eb/N0 ~ U[1,4] dB; held-out evaluation {eval_frames} "
                                   f"frames per point from another generator seed",
                       "train_s": round(t0.elapsed_time(t1) / 1e3, 2), "last_losses": losses,
                       "weights": {"min": round(float(w.min().item()), 4), "max": round(float(w.max().item()), 4),
                                   "mean": round(float(w.mean().item()), 4)},
                       "points": fer}}


def weighted_bp_large(torch, pbp, F_train=1024, F_dec=8192, T=20, steps=2, warmup=1, epochs=10,
                      epoch_frames=100_352, lr=3e-4, eval_frames=400_000, snrs=(1.0, 1.5, 2.0, 2.5, 3.0)):
    """Weighted PP-MT-BP at scale: N=4096, K=2048 + CRC-24 (K=2072), the last 5
    of 12 stages re-ordered every 10 iterations from 8 trellises, 20 unrolled
    iterations with weights tied across trellises, Eb/N0 ~ U[1,3] dB.  Timed:
    a training step (forward with checkpoints, adjoint, gradient-norm clip,
    optimiser step) on F_train frames, the weighted forward alone on F_dec
    frames, and unit-weight PP-MT-BP (CRC stop, same iteration budget) on the
    same frames.  Then the payoff: `epochs` epochs of fresh frames and frame
    error rates of learned against unit weights on held-out frames."""
    from paper_1911_08868_amd.wbp import WeightedBPDecoder
    code = pbp.Code(4096, 2072, 24, 0x1864CFB, 2.5)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=5, period_T=10, pool_Q=8, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(91)
    F = max(F_train, F_dec)
    e = torch.rand(F, generator=gen, device="cuda", dtype=torch.float64) * 2.0 + 1.0
    m, llr = _fresh_frames(torch, pbp, code, F, e, gen)
    u_info = pbp.info_bits(code, m)
    tdec = WeightedBPDecoder(code, T, pp)
    # Over 20 unrolled min-sum iterations the gradient of the earliest
    # iterations' weights can explode (every message fans out into later ones
    # while each check node routes its adjoint to one input; the FP64 oracle
    # gives entries up to ~1e15 on such frames), so the steps clip the
    # gradient norm.
    ms_train = _time_train_step(torch, pbp, code, tdec, torch.optim.SGD(tdec.parameters(), lr=1e-2),
                                llr[:F_train], u_info[:F_train], steps, warmup, clip=1.0)
    xd = llr[:F_dec]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.no_grad():
        tdec(xd)
        torch.cuda.synchronize()
        a.record()
        tdec(xd)
        b.record()
        torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b)
    bp = pbp.BPParams(max_iter=T, stop=pbp.STOP_CRC, it_min=3)
    outs = pbp.pp_mt_bp_decode(code, xd, bp, pp)
    torch.cuda.synchronize()
    a.record()
    outs = pbp.pp_mt_bp_decode(code, xd, bp, pp, out=outs[:3])
    b.record()
    torch.cuda.synchronize()
    ms_unit = a.elapsed_time(b)
    _log(f"weighted BP N=4096: train step {ms_train:.1f} ms ({F_train} frames), forward {ms_fwd:.1f} ms, "
         f"unit-weight PP-MT-BP {ms_unit:.1f} ms ({F_dec} frames)")
    dec = WeightedBPDecoder(code, T, pp)
    opt = torch.optim.Adam(dec.parameters(), lr=lr)
    n_steps = epochs * (epoch_frames // F_train)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    losses = _train_weighted(torch, pbp, code, dec, opt, n_steps, F_train, 1.0, 3.0, seed=3001, clip=1.0)
    t1.record()
    torch.cuda.synchronize()
    fer = _fer_learned_vs_unit(torch, pbp, code, dec, pp, T, snrs, eval_frames, seed=9101, chunk=32768)
    w = dec.weight.detach()
    return {"workload": f"weighted PP-MT-BP, N=4096 K=2048+CRC24, last 5 of 12 stages every 10 iterations "
                        f"(Q=8, weights tied across trellises), {T} unrolled iterations, Eb/N0 ~ U[1,3] dB; "
                        f"training batch {F_train}, decode {F_dec} frames",
            "train_frames_s": round(F_train / (ms_train / 1e3), 1), "ms_train_step": round(ms_train, 2),
            "fwd_frames_s": round(F_dec / (ms_fwd / 1e3), 1),
            "unit_pp_mt_bp_frames_s": round(F_dec / (ms_unit / 1e3), 1),
            "avg_iters_unit": round(outs[1].double().mean().item(), 3),
            "payoff": {"training": f"{epochs} epochs x {epoch_frames} fresh frames ({n_steps} steps of {F_train}), "
                                   f"Adam lr {lr}, gradient norm clipped to 1, Eb/N0 ~ U[1,3] dB; held-out "
                                   f"evaluation {eval_frames} frames per point ({eval_frames * len(snrs)} in all) "
                                   f"from another generator seed",
                       "train_s": round(t0.elapsed_time(t1) / 1e3, 2), "last_losses": losses,
                       "weights": {"min": round(float(w.min().item()), 4), "max": round(float(w.max().item()), 4),
                                   "mean": round(float(w.mean().item()), 4)},
                       "points": fer}}


def _alu_roof(ops, ms):
    achieved = ops / (ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK / 1e12, 2), "unit": "TOP/s",
            "frac": round(achieved * 1e12 / ALU_PEAK, 4)}


def alg1_table1(torch, pbp, F=65536, snrs=(1.5, 2.0, 2.5, 3.0)):
    """Algorithm 1 with random subgraphs (Table I, N_it,max = 200: P_range 2,
    P_level 6, D 8, N_min 4) at N=1024, R=1/2 (K=512 with CRC-24), under both
    readings of its subgraph (a component of the current graph; a block of the
    original graph), beside the fixed last-4 schedule on the same frames, and
    both with the exact boxplus.  Roofline entries count the processing
    elements' 6 lane-ops: 3 N (2n - 1) per frame-iteration."""
    import synth
    code = pbp.Code(1024, 512, 24, 0x1864CFB, 2.5)
    ops_fi = 3 * 1024 * (2 * 10 - 1)
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    bp_exact = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3, check=pbp.CHECK_EXACT)
    t = dict(P_range=2, P_level=6, D=8, N_min=4, seed=1)
    alg1 = pbp.PPParams(mode=pbp.PP_ALG1, **t)
    orig = pbp.PPParams(mode=pbp.PP_ALG1_ORIG, **t)
    lastk = pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=1)
    points = []
    for snr in snrs:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(snr * 100))
        m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
        x = pbp.encode(code, m)
        llr = synth.awgn_llr_torch(x, torch.full((F,), snr, device="cuda", dtype=torch.float64),
                                   code.K_msg, gen)
        row = {"ebn0_db": snr}
        for name, pp, bpx in (("alg1", alg1, bp), ("alg1_orig", orig, bp), ("lastk4", lastk, bp),
                              ("alg1_exact", alg1, bp_exact), ("alg1_orig_exact", orig, bp_exact)):
            out = pbp.pp_mt_bp_decode(code, llr, bpx, pp)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            out = pbp.pp_mt_bp_decode(code, llr, bpx, pp, out=out[:3])
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            fi = out[1].double().sum().item()
            row[name] = {"gbit_s": round(F * code.K_msg / (ms / 1e3) / 1e9, 3), "ms": round(ms, 2),
                         "avg_iters": round(fi / F, 3), "frame_it_s": round(fi / (ms / 1e3)),
                         "fer": (out[0] != m).any(1).double().mean().item()}
            if name != "lastk4" and not name.endswith("exact"):
                row[name]["roofline"] = _alu_roof(ops_fi * fi, ms)
        points.append(row)
        _log(f"Algorithm 1 at {snr} dB: current-graph {row['alg1']['ms']} ms "
             f"({row['alg1']['frame_it_s']:.3g} frame-it/s), original-graph {row['alg1_orig']['ms']} ms "
             f"({row['alg1_orig']['frame_it_s']:.3g}), last-4 {row['lastk4']['ms']} ms; fer "
             f"{row['alg1']['fer']:.4g} / {row['alg1_orig']['fer']:.4g} / {row['lastk4']['fer']:.4g}")
    return {"workload": f"Algorithm 1 (Table I, 200-iteration set: P_range 2, P_level 6, D 8, N_min 4), subgraph "
                        f"of the current graph (alg1) and of the original graph (alg1_orig), vs fixed last-4 "
                        f"schedule, and both with the exact boxplus, N=1024 K=512 incl. CRC-24, {F} frames per "
                        f"Eb/N0 point, max 200 iterations, CRC stop", "points": points}


def alg1_long(torch, pbp, F=8192, snrs=(2.0, 2.5, 3.0)):
    """Algorithm 1 with Table I's 2e4-iteration sets at their full budget:
    N=1024 R=1/2 (P_range 10, P_level 9, D 100, N_min 15) and N=512 R=0.65
    (K=333 with CRC-24; P_range 9, P_level 8, D 50, N_min 15), under both
    readings of its subgraph, beside plain BP with the same budget on the same
    frames."""
    import synth
    sets = (("N1024_R0.5", 1024, 512, dict(P_range=10, P_level=9, D=100, N_min=15)),
            ("N512_R0.65", 512, 333, dict(P_range=9, P_level=8, D=50, N_min=15)))
    bp = pbp.BPParams(max_iter=20000, stop=pbp.STOP_CRC, it_min=3)
    out = {}
    for name, N, K, t in sets:
        code = pbp.Code(N, K, 24, 0x1864CFB, 2.5)
        alg1 = pbp.PPParams(mode=pbp.PP_ALG1, seed=1, **t)
        orig = pbp.PPParams(mode=pbp.PP_ALG1_ORIG, seed=1, **t)
        # first launch of this length's kernels, outside the timed calls
        warm = torch.zeros((64, N), dtype=torch.float32, device="cuda")
        pbp.pp_mt_bp_decode(code, warm, pbp.BPParams(max_iter=5, stop=pbp.STOP_CRC), alg1)
        pbp.pp_mt_bp_decode(code, warm, pbp.BPParams(max_iter=5, stop=pbp.STOP_CRC), orig)
        pbp.bp_decode(code, warm, pbp.BPParams(max_iter=5, stop=pbp.STOP_CRC))
        points = []
        for snr in snrs:
            gen = torch.Generator(device="cuda")
            gen.manual_seed(int(snr * 100) + N)
            m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
            llr = synth.awgn_llr_torch(pbp.encode(code, m), torch.full((F,), snr, device="cuda",
                                                                       dtype=torch.float64), code.K_msg, gen)
            row = {"ebn0_db": snr}
            for dec, run in (("alg1", lambda: pbp.pp_mt_bp_decode(code, llr, bp, alg1)),
                             ("alg1_orig", lambda: pbp.pp_mt_bp_decode(code, llr, bp, orig)),
                             ("bp", lambda: pbp.bp_decode(code, llr, bp))):
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                res = run()
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                it = res[1].double()
                e = int((res[0] != m).any(1).sum().item())
                row[dec] = {"ms": round(ms, 2), "avg_iters": round(it.mean().item(), 2),
                            "max_iters": int(it.max().item()),
                            "frame_it_s": round(it.sum().item() / (ms / 1e3)),
                            "fer": e / F, "fer_ci95": [round(v, 6) for v in clopper_pearson(e, F)]}
            points.append(row)
            _log(f"Algorithm 1 {name} 2e4 set at {snr} dB: fer current-graph {row['alg1']['fer']:.4g} "
                 f"({row['alg1']['ms']} ms), original-graph {row['alg1_orig']['fer']:.4g} "
                 f"({row['alg1_orig']['ms']} ms), BP {row['bp']['fer']:.4g} ({row['bp']['ms']} ms)")
        out[name] = points
    return {"workload": f"Algorithm 1 with Table I's 2e4-iteration sets, subgraph of the current graph (alg1) "
                        f"and of the original graph (alg1_orig), vs plain BP, N_it,max = 20000, CRC-24, CRC stop "
                        f"from iteration 3, {F} frames per Eb/N0 point", "sets": out}


def error_classes(torch, pbp, F=65536, snrs=(1.5, 2.0, 2.5, 3.0), H=32):
    """Error classes of Sec. II-C (false converged / oscillation /
    unconverged) for plain BP, the fixed last-4 schedule and Algorithm 1 on
    the 1024-bit, rate-1/2 CRC-16 code, from the last H decision hashes of
    each frame; plus the time of the history-recording decode beside the
    plain one."""
    import synth
    code = pbp.Code(1024, 512, 16, 0x1021, 2.5)
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC)
    scheds = (("bp", None),
              ("lastk4", pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=1)),
              ("alg1", pbp.PPParams(mode=pbp.PP_ALG1, P_range=2, P_level=6, D=8, N_min=4, seed=1)),
              ("alg1_orig", pbp.PPParams(mode=pbp.PP_ALG1_ORIG, P_range=2, P_level=6, D=8, N_min=4, seed=1)))
    names = ("correct", "false_converged", "oscillation", "unconverged")
    points = []
    for snr in snrs:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(snr * 100) + 7)
        m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
        x = pbp.encode(code, m)
        llr = synth.awgn_llr_torch(x, torch.full((F,), snr, device="cuda", dtype=torch.float64),
                                   code.K_msg, gen)
        row = {"ebn0_db": snr}
        for name, pp in scheds:
            pbp.pp_mt_bp_decode_trace(code, llr, bp, pp, H)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            out = pbp.pp_mt_bp_decode_trace(code, llr, bp, pp, H)
            ev[1].record()
            ev[2].record()
            pbp.pp_mt_bp_decode(code, llr, bp, pp or pbp.PPParams())
            ev[3].record()
            cls, per = pbp.classify_errors(out[0], m, out[2], out[1], out[3])
            torch.cuda.synchronize()
            counts = torch.bincount(cls.long(), minlength=4).tolist()
            row[name] = {**{k: int(v) for k, v in zip(names, counts)},
                         "fer": round(1.0 - counts[0] / F, 6),
                         "oscillation_periods": {int(p): int(c) for p, c in
                                                 zip(*torch.unique(per[cls == 2], return_counts=True))},
                         "ms_trace": round(ev[0].elapsed_time(ev[1]), 2),
                         "ms_plain": round(ev[2].elapsed_time(ev[3]), 2)}
        points.append(row)
        _log(f"error classes at {snr} dB: " + ", ".join(
            f"{n}: fc {row[n]['false_converged']} osc {row[n]['oscillation']} unc {row[n]['unconverged']}"
            for n, _ in scheds))
    # the higher rate of Sec. IV's comparison (R = 0.65, CRC-24), where the
    # paper expects converged errors to dominate at high SNR
    code65 = pbp.Code(1024, 666, 24, 0x1864CFB, 2.5)
    bp65 = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    rate065 = []
    for snr in (3.5, 4.0):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(snr * 100) + 666)
        m = torch.randint(0, 2, (F, code65.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
        x = pbp.encode(code65, m)
        llr = synth.awgn_llr_torch(x, torch.full((F,), snr, device="cuda", dtype=torch.float64),
                                   code65.K_msg, gen)
        row = {"ebn0_db": snr}
        for name, pp in scheds[:2]:
            out = pbp.pp_mt_bp_decode_trace(code65, llr, bp65, pp, H)
            cls, per = pbp.classify_errors(out[0], m, out[2], out[1], out[3])
            counts = torch.bincount(cls.long(), minlength=4).tolist()
            row[name] = {k: int(v) for k, v in zip(names, counts)}
        rate065.append(row)
        _log(f"error classes R=0.65 at {snr} dB: " + ", ".join(
            f"{n}: fc {row[n]['false_converged']} osc {row[n]['oscillation']} unc {row[n]['unconverged']}"
            for n, _ in scheds[:2]))
    return {"workload": f"error classes (Sec. II-C) from the last {H} decision hashes, N=1024 K=496+CRC16, "
                        f"{F} frames per Eb/N0 point, max 200 iterations, CRC stop; plain BP, fixed last-4 "
                        f"(T=10, Q=8), Algorithm 1 (P_range 2, P_level 6, D 8, N_min 4) with subgraphs of "
                        f"the current graph (alg1) and of the original graph (alg1_orig); and N=1024 "
                        f"K=666 incl. CRC-24 (R=0.65), CRC stop from iteration 3, plain BP and last-4",
            "points": points, "rate_065": rate065}


def exact_boxplus(torch, pbp, F=262144, snrs=(1.5, 2.0, 2.5, 3.0, 3.5)):
    """The exact boxplus check function (Sec. II-B) beside min-sum on the
    1024-bit, rate-1/2 CRC-16 code with the fixed last-4 schedule (T=10, Q=8),
    at most 200 iterations, CRC stop, on the same frames."""
    import synth
    code = pbp.Code(1024, 512, 16, 0x1021, 2.5)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=1)
    pes = (2 * 10 - 1) * 512      # PEs per frame-iteration: L sweep 10 stages, R sweep 9
    points = []
    for snr in snrs:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(snr * 100) + 11)
        m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
        x = pbp.encode(code, m)
        llr = synth.awgn_llr_torch(x, torch.full((F,), snr, device="cuda", dtype=torch.float64),
                                   code.K_msg, gen)
        row = {"ebn0_db": snr}
        for name, chk in (("exact", pbp.CHECK_EXACT), ("minsum", pbp.CHECK_MINSUM)):
            bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, check=chk)
            out = pbp.pp_mt_bp_decode(code, llr, bp, pp)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            out = pbp.pp_mt_bp_decode(code, llr, bp, pp, out=out[:3])
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            its = out[1].double().sum().item()
            row[name] = {"gbit_s": round(F * code.K_msg / (ms / 1e3) / 1e9, 3), "ms": round(ms, 2),
                         "avg_iters": round(its / F, 3),
                         "fer": (out[0] != m).any(1).double().mean().item(),
                         "pe_per_s": round(its * pes / (ms / 1e3), 1)}
        points.append(row)
        _log(f"exact boxplus at {snr} dB: {row['exact']['gbit_s']} Gbit/s fer {row['exact']['fer']:.4g} "
             f"vs min-sum {row['minsum']['gbit_s']} Gbit/s fer {row['minsum']['fer']:.4g}")
    return {"workload": f"exact boxplus vs min-sum, N=1024 K=496+CRC16, fixed last-4 (T=10, Q=8), "
                        f"{F} frames per Eb/N0 point, max 200 iterations, CRC stop", "points": points}


def noise_aided(torch, pbp, F=65536, sigma=0.6):
    """Noise injected at the trellis events (sigma^2 = 0.36, the noise-aided BP
    setting of Table I) with and without the last-4 permutations, and at
    Algorithm 1's events (Table I 200-iteration set), beside the same
    schedules without noise and plain BP, on N=1024 codes of rate 1/2 and
    0.65 with CRC-24 (K includes the CRC), at most 200 iterations, CRC stop
    from iteration 3; fixed-schedule events every 10 iterations."""
    import synth
    out = []
    for rate, K, snrs in (("1/2", 512, (2.0, 3.0, 3.5)), ("0.65", 666, (2.5, 3.5, 4.0))):
        code = pbp.Code(1024, K, 24, 0x1864CFB, 2.5)
        bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
        lastk = dict(mode=pbp.PP_LASTK, k=4, period_T=10, seed=1)
        alg1 = dict(mode=pbp.PP_ALG1, P_range=2, P_level=6, D=8, N_min=4, seed=1)
        orig = dict(alg1, mode=pbp.PP_ALG1_ORIG)
        scheds = (("bp", pbp.PPParams()),
                  ("lastk4", pbp.PPParams(pool_Q=8, **lastk)),
                  ("lastk4_noise", pbp.PPParams(pool_Q=8, noise_sigma=sigma, **lastk)),
                  ("noise_only", pbp.PPParams(pool_Q=1, noise_sigma=sigma, **lastk)),
                  ("alg1", pbp.PPParams(**alg1)),
                  ("alg1_noise", pbp.PPParams(noise_sigma=sigma, **alg1)),
                  ("alg1_orig", pbp.PPParams(**orig)),
                  ("alg1_orig_noise", pbp.PPParams(noise_sigma=sigma, **orig)))
        for snr in snrs:
            gen = torch.Generator(device="cuda")
            gen.manual_seed(int(snr * 100) + K)
            m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
            x = pbp.encode(code, m)
            llr = synth.awgn_llr_torch(x, torch.full((F,), snr, device="cuda", dtype=torch.float64),
                                       code.K_msg, gen)
            row = {"rate": rate, "ebn0_db": snr}
            for name, pp in scheds:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                res = pbp.pp_mt_bp_decode(code, llr, bp, pp)
                b.record()
                torch.cuda.synchronize()
                row[name] = {"fer": (res[0] != m).any(1).double().mean().item(),
                             "avg_iters": round(res[1].double().mean().item(), 3),
                             "ms": round(a.elapsed_time(b), 2)}
            out.append(row)
            _log(f"noise-aided R={rate} {snr} dB: " + ", ".join(
                f"{n} fer {row[n]['fer']:.4g}" for n, _ in scheds))
    return {"workload": f"noise injected at the events (sigma^2 = {sigma * sigma:.2f}), N=1024, CRC-24, "
                        f"R = 1/2 (K=512) and 0.65 (K=666), {F} frames per point, max 200 iterations, "
                        f"CRC stop from iteration 3, fixed-schedule events every 10 iterations, "
                        f"Algorithm 1 with the Table I 200-iteration set, subgraphs of the current graph "
                        f"(alg1) and of the original graph (alg1_orig)", "points": out}


def n64_gtest(torch, pbp, F=2000, F_sustained=1 << 20, snrs=(1.0, 2.0, 3.0, 4.0)):
    """The 64-bit code: K = 32 without CRC, designed at 2 dB, scaled min-sum
    (alpha = 15/16), stop when u G_N equals the hard decision on the channel
    level (from iteration 1), at most 40 iterations; F frames per Eb/N0
    point, all-zero and random messages; plus the same decoder on F_sustained
    random frames per point for its sustained rate and ALU roofline fraction
    (a G-test iteration runs every stage of both sweeps: 6 lane-ops per
    processing element, N/2 per stage, 2n stages)."""
    import synth
    code = pbp.Code(64, 32, 0, 0, 2.0)
    bp = pbp.BPParams(max_iter=40, alpha=0.9375, stop=pbp.STOP_G, it_min=1)
    peak = ALU_PEAK
    points = []
    for si, snr in enumerate(snrs):
        row = {"ebn0_db": snr}
        for name, zero, nF in (("all_zero", True, F), ("random", False, F), ("sustained", False, F_sustained)):
            gen = torch.Generator(device="cuda")
            gen.manual_seed(640 + 10 * si + (1 if zero else 0) + (2 if nF != F else 0))
            if zero:
                m = torch.zeros((nF, code.K_msg), dtype=torch.uint8, device="cuda")
                llr = synth.awgn_llr_torch(pbp.encode(code, m), torch.full((nF,), snr, device="cuda",
                                                                           dtype=torch.float64), code.K_msg, gen)
            else:
                m, llr = _fresh_frames(torch, pbp, code, nF, snr, gen)
            out = pbp.bp_decode(code, llr, bp)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            out = pbp.bp_decode(code, llr, bp, out=out[:3])
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            it = out[1].double()
            e = int((out[0] != m).any(1).sum().item())
            ops = 3 * 64 * 2 * 6 * it.sum().item()
            row[name] = {"frames": nF, "ms": round(ms, 4), "fer": e / nF, "ci95": clopper_pearson(e, nF),
                         "avg_iters": round(it.mean().item(), 3),
                         "gbit_s": round(nF * code.K_msg / (ms / 1e3) / 1e9, 3),
                         "roofline": {"bound": "alu", "kernel": "k_decode<n=6,k=0,rho=2,G test,scaled>",
                                      "achieved": round(ops / (ms / 1e3) / 1e12, 3),
                                      "peak": round(peak / 1e12, 2), "unit": "TOP/s",
                                      "frac": round(ops / (ms / 1e3) / peak, 4)}}
        points.append(row)
        _log(f"N=64 G test at {snr} dB: fer {row['random']['fer']:.4g} (all-zero {row['all_zero']['fer']:.4g}), "
             f"sustained {row['sustained']['gbit_s']} Gbit/s ({row['sustained']['roofline']['frac']} of the ALU peak)")
    return {"workload": f"N=64 K=32 (no CRC) designed at 2 dB, min-sum scaled by 15/16, G-matrix stop from "
                        f"iteration 1, at most 40 iterations; {F} frames per Eb/N0 point of all-zero and of "
                        f"random messages, and {F_sustained} random frames per point for the sustained rate",
            "points": points}


def batched_mixed(torch, pbp, F=4_000_000):
    """The mixed-length stream of the batched decoder (F frames in 4 rounds)."""
    return bench_mixed(torch, pbp, frames_total=F)


def bench_extras(torch, pbp):
    out = {}
    for name, fn in (("n64_gtest", n64_gtest), ("weighted_bp", weighted_bp), ("weighted_bp_n4096", weighted_bp_large),
                     ("batched_mixed", batched_mixed), ("algorithm1", alg1_table1),
                     ("algorithm1_2e4", alg1_long),
                     ("error_classes", error_classes), ("exact_boxplus", exact_boxplus),
                     ("noise_aided", noise_aided)):
        try:
            out[name] = fn(torch, pbp)
        except Exception as e:  # report the failure in the JSON line, keep the rest
            out[name] = None
            out.setdefault("extras_errors", {})[name] = f"{type(e).__name__}: {e}"
            _log(f"{name} failed: {e}")
        torch.cuda.empty_cache()
    return out


def make_mixed_stream(torch, dec, seed: int, lo_db=1.0, hi_db=4.0):
    """Fill a round: code uniform over dec.codes, Eb/N0 uniform on [lo, hi] dB
    per frame, uniform message bits; encoded on the GPU, BPSK over AWGN.
    Returns the messages per code group for error counting."""
    import synth
    import paper_1911_08868_amd as pbp
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
        x = pbp.encode(code, m)
        llr = synth.awgn_llr_torch(x, ebn0[idx], code.K_msg, gen)
        # scatter the frames into the pool
        off = dec.llr_off[idx]
        cols = torch.arange(code.N, device="cuda")
        dec.llr_pool[(off[:, None] + cols[None, :]).flatten()] = llr.flatten()
        groups.append((idx, m))
    torch.cuda.synchronize()
    return groups


def frame_errors(torch, dec, groups):
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
    from paper_1911_08868_amd.batched import BatchedDecoder, mixed_codes
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=4, period_T=10, pool_Q=8, seed=1)
    codes = mixed_codes()
    F = frames_total // rounds
    decs, groups = [], []
    for r in range(rounds):
        d = BatchedDecoder(codes, F, bp, pp, cfg)
        groups.append(make_mixed_stream(torch, d, seed=500 + r))
        if r == 0 and cfg is None:
            from paper_1911_08868_amd.tune import tune_batched
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
    alu_peak = ALU_PEAK
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

"""Side workloads measured by bench.py beside the headline decode.

weighted_bp(): the weighted-BP training step (N = 256, K = 128 message bits +
CRC-16, 10 unrolled iterations, batch 16384, Eb/N0 uniform on [1, 4] dB per
frame, binary cross entropy of the output LLRs against the transmitted
information bits) timed forward + backward + SGD step, next to plain min-sum
BP decoding of the same frames.

weighted_bp_large(): the same at N=4096 with the last-5 trellis schedule and
20 unrolled iterations, beside unit-weight PP-MT-BP decoding.

batched_mixed(): the mixed-length stream through the persistent queue kernel
(see batched.py).

alg1_table1(): Algorithm 1 with random subgraphs (Table I parameters) beside
the fixed last-k schedule.
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
        opt.zero_grad()
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


def weighted_bp_large(torch, pbp, F_train=1024, F_dec=8192, T=20, steps=2, warmup=1):
    """Weighted PP-MT-BP at scale: N=4096, K=2048 + CRC-24 (K=2072), the last 5
    of 12 stages re-ordered every 10 iterations from 8 trellises, 20 unrolled
    iterations with weights tied across trellises, Eb/N0 ~ U[1,3] dB.  Timed:
    a training step (forward with checkpoints, adjoint, gradient-norm clip,
    SGD) on F_train frames,
    the weighted forward alone on F_dec frames, and unit-weight PP-MT-BP
    (CRC stop, same iteration budget) on the same frames."""
    import synth
    from .wbp import WeightedBPDecoder, bce_on_information_bits
    code = pbp.Code(4096, 2072, 24, 0x1864CFB, 2.5)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=5, period_T=10, pool_Q=8, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(91)
    F = max(F_train, F_dec)
    m = torch.randint(0, 2, (F, code.K_msg), generator=gen, device="cuda", dtype=torch.uint8)
    x = pbp.encode(code, m)
    ebn0 = torch.rand(F, generator=gen, device="cuda", dtype=torch.float64) * 2.0 + 1.0
    llr = synth.awgn_llr_torch(x, ebn0, code.K_msg, gen)
    u = polar_transform_torch(x, code.n)
    info = torch.from_numpy(code.info_idx.astype("int64")).cuda()
    u_info = u[:, info]
    dec = WeightedBPDecoder(code, T, pp)
    opt = torch.optim.SGD(dec.parameters(), lr=1e-2)
    xt, ut = llr[:F_train], u_info[:F_train]

    def step():
        out = dec(xt)
        loss = bce_on_information_bits(out, ut, info)
        opt.zero_grad()
        loss.backward()
        # Over 20 unrolled min-sum iterations the gradient of the earliest
        # iterations' weights can explode (every message fans out into later
        # ones while each check node routes its adjoint to one input; the
        # FP64 oracle gives entries up to ~1e15 on such frames), so the step
        # clips the gradient norm.
        torch.nn.utils.clip_grad_norm_(dec.parameters(), 1.0)
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
    xd = llr[:F_dec]
    with torch.no_grad():
        o = dec(xd)
        torch.cuda.synchronize()
        a.record()
        o = dec(xd)
        b.record()
        torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b)
    fer_w = ((o[:, info] < 0).to(torch.uint8) != u_info[:F_dec]).any(1).double().mean().item()
    bp = pbp.BPParams(max_iter=T, stop=pbp.STOP_CRC, it_min=3)
    outs = pbp.pp_mt_bp_decode(code, xd, bp, pp)
    torch.cuda.synchronize()
    a.record()
    outs = pbp.pp_mt_bp_decode(code, xd, bp, pp, out=outs[:3])
    b.record()
    torch.cuda.synchronize()
    ms_unit = a.elapsed_time(b)
    fer_u = (outs[0] != m[:F_dec]).any(1).double().mean().item()
    _log(f"weighted BP N=4096: train step {ms_train:.1f} ms ({F_train} frames), forward {ms_fwd:.1f} ms, "
         f"unit-weight PP-MT-BP {ms_unit:.1f} ms ({F_dec} frames)")
    return {"workload": f"weighted PP-MT-BP, N=4096 K=2048+CRC24, last 5 of 12 stages every 10 iterations "
                        f"(Q=8, weights tied across trellises), {T} unrolled iterations, Eb/N0 ~ U[1,3] dB; "
                        f"training batch {F_train}, decode {F_dec} frames",
            "train_frames_s": round(F_train / (ms_train / 1e3), 1), "ms_train_step": round(ms_train, 2),
            "fwd_frames_s": round(F_dec / (ms_fwd / 1e3), 1),
            "unit_pp_mt_bp_frames_s": round(F_dec / (ms_unit / 1e3), 1),
            "loss": round(float(loss.item()), 5),
            "fer_weighted_after_steps": fer_w, "fer_unit_pp_mt_bp": fer_u,
            "avg_iters_unit": round(outs[1].double().mean().item(), 3)}


def alg1_table1(torch, pbp, F=65536, snrs=(1.5, 2.0, 2.5, 3.0)):
    """Algorithm 1 with random subgraphs (Table I, N_it,max = 200: P_range 2,
    P_level 6, D 8, N_min 4) at N=1024, R=1/2 (K=512 with CRC-24), beside
    the fixed last-4 schedule on the same frames."""
    import synth
    code = pbp.Code(1024, 512, 24, 0x1864CFB, 2.5)
    bp = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3)
    bp_exact = pbp.BPParams(max_iter=200, stop=pbp.STOP_CRC, it_min=3, check=pbp.CHECK_EXACT)
    alg1 = pbp.PPParams(mode=pbp.PP_ALG1, P_range=2, P_level=6, D=8, N_min=4, seed=1)
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
        for name, pp, bpx in (("alg1", alg1, bp), ("lastk4", lastk, bp), ("alg1_exact", alg1, bp_exact)):
            out = pbp.pp_mt_bp_decode(code, llr, bpx, pp)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            out = pbp.pp_mt_bp_decode(code, llr, bpx, pp, out=out[:3])
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            row[name] = {"gbit_s": round(F * code.K_msg / (ms / 1e3) / 1e9, 3), "ms": round(ms, 2),
                         "avg_iters": round(out[1].double().mean().item(), 3),
                         "fer": (out[0] != m).any(1).double().mean().item()}
        points.append(row)
        _log(f"Algorithm 1 at {snr} dB: {row['alg1']['ms']} ms vs last-4 {row['lastk4']['ms']} ms; "
             f"with the exact boxplus {row['alg1_exact']['ms']} ms, fer {row['alg1_exact']['fer']:.4g} "
             f"(min-sum {row['alg1']['fer']:.4g})")
    return {"workload": f"Algorithm 1 (Table I, 200-iteration set: P_range 2, P_level 6, D 8, N_min 4) vs "
                        f"fixed last-4 schedule, and Algorithm 1 with the exact boxplus, N=1024 K=512 incl. "
                        f"CRC-24, {F} frames per Eb/N0 point, max 200 iterations, CRC stop", "points": points}


def alg1_long(torch, pbp, F=8192, snrs=(2.0, 2.5, 3.0)):
    """Algorithm 1 with Table I's 2e4-iteration sets at their full budget:
    N=1024 R=1/2 (P_range 10, P_level 9, D 100, N_min 15) and N=512 R=0.65
    (K=333 with CRC-24; P_range 9, P_level 8, D 50, N_min 15), beside plain
    BP with the same budget on the same frames."""
    import synth
    sets = (("N1024_R0.5", 1024, 512, dict(P_range=10, P_level=9, D=100, N_min=15)),
            ("N512_R0.65", 512, 333, dict(P_range=9, P_level=8, D=50, N_min=15)))
    bp = pbp.BPParams(max_iter=20000, stop=pbp.STOP_CRC, it_min=3)
    out = {}
    for name, N, K, t in sets:
        code = pbp.Code(N, K, 24, 0x1864CFB, 2.5)
        alg1 = pbp.PPParams(mode=pbp.PP_ALG1, seed=1, **t)
        # first launch of this length's kernels, outside the timed calls
        warm = torch.zeros((64, N), dtype=torch.float32, device="cuda")
        pbp.pp_mt_bp_decode(code, warm, pbp.BPParams(max_iter=5, stop=pbp.STOP_CRC), alg1)
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
                             ("bp", lambda: pbp.bp_decode(code, llr, bp))):
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                res = run()
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                it = res[1].double()
                row[dec] = {"ms": round(ms, 2), "avg_iters": round(it.mean().item(), 2),
                            "max_iters": int(it.max().item()),
                            "frame_it_s": round(it.sum().item() / (ms / 1e3)),
                            "fer": (res[0] != m).any(1).double().mean().item()}
            points.append(row)
            _log(f"Algorithm 1 {name} 2e4 set at {snr} dB: fer {row['alg1']['fer']:.4g} "
                 f"({row['alg1']['ms']} ms) vs BP fer {row['bp']['fer']:.4g} ({row['bp']['ms']} ms)")
        out[name] = points
    return {"workload": f"Algorithm 1 with Table I's 2e4-iteration sets vs plain BP, N_it,max = 20000, "
                        f"CRC-24, CRC stop from iteration 3, {F} frames per Eb/N0 point", "sets": out}


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
              ("alg1", pbp.PPParams(mode=pbp.PP_ALG1, P_range=2, P_level=6, D=8, N_min=4, seed=1)))
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
                        f"(T=10, Q=8), Algorithm 1 (P_range 2, P_level 6, D 8, N_min 4); and N=1024 "
                        f"K=666 incl. CRC-24 (R=0.65), CRC stop from iteration 3, plain BP and last-4",
            "points": points, "rate_065": rate065}


VALU_PEAK = 256 * 64 * 2.4e9          # non-packed 32-bit VALU lane-slots per second
EXACT_SLOTS_PER_PE = 2 * (11 + 4) + 2


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
            if name == "exact":
                # VALU instructions per PE of the exact form: per check node 11
                # plain ones and 4 transcendental ones (each at least one issue
                # slot), two check nodes and two additions per PE
                row[name]["alu_frac"] = round(row[name]["pe_per_s"] * EXACT_SLOTS_PER_PE / VALU_PEAK, 4)
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
        scheds = (("bp", pbp.PPParams()),
                  ("lastk4", pbp.PPParams(pool_Q=8, **lastk)),
                  ("lastk4_noise", pbp.PPParams(pool_Q=8, noise_sigma=sigma, **lastk)),
                  ("noise_only", pbp.PPParams(pool_Q=1, noise_sigma=sigma, **lastk)),
                  ("alg1", pbp.PPParams(**alg1)),
                  ("alg1_noise", pbp.PPParams(noise_sigma=sigma, **alg1)))
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
                        f"Algorithm 1 with the Table I 200-iteration set", "points": out}


def batched_mixed(torch, pbp, F=4_000_000):
    """The mixed-length stream of the batched decoder (F frames in 4 rounds)."""
    from .batched import bench_mixed
    return bench_mixed(torch, pbp, frames_total=F)


def bench_extras(torch, pbp):
    out = {}
    for name, fn in (("weighted_bp", weighted_bp), ("weighted_bp_n4096", weighted_bp_large),
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

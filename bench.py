#!/usr/bin/env python3
"""Throughput benchmark of PP-MT-BP polar decoding on one MI355X.

Workload (one step): N = 1024 polar code, K = 512 = 496 message bits + CRC-16
(0x1021), Bhattacharyya frozen set at design Eb/N0 = 2.5 dB, BPSK-AWGN frames
at Eb/N0 = 1.5, 1.75, ..., 3.5 dB (9 points) with --frames frames per point
(default 1e6), decoded by partially permuted multi-trellis BP in FP32: the
last k = 4 of the 10 stages re-ordered from a seeded pool of Q = 8 trellises
every T = 10 iterations, at most 200 iterations, CRC early stop from
iteration 3.  Inputs (channel LLRs) are generated in device memory before the
timed region.  value = decoded message bits per second over the whole step.

Prints one JSON line.  Extra fields: per-Eb/N0 breakdown, plain BP and full
permutation on the same frames, weighted-BP training throughput and the
mixed-length batched decode, a roofline entry for the decode kernel, and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, K, CRC_W, CRC_POLY, DESIGN_DB = 1024, 512, 16, 0x1021, 2.5
K_MSG = K - CRC_W
SNRS = [1.5 + 0.25 * i for i in range(9)]
MAX_ITER, IT_MIN = 200, 3
PP_K, PP_T, PP_Q, PP_SEED = 4, 10, 8, 1

# MI355X VALU issue rates per CU and clock (four SIMDs): FP32 add, mul, fma and
# 32-bit bitwise operations 128 lanes (the 157.3 TFLOP/s FP32 vector figure is
# 256 CUs x 2.4 GHz x 128 FMA lanes x 2 flops), v_med3_f32 64 lanes (half rate;
# both measured with per-instruction probes).  A processing element issues 2
# v_add_f32, 2 v_med3_f32 and 2 v_bitop3_b32: 2/64 + 4/128 = 1/16 CU-clock per
# lane, 96 of its lane-ops per CU-clock.  The roofline takes the larger of this
# figure and the calibration kernel's measured rate for the same mix.
PE_OPS_PER_CU_CLK = 6 / (2 / 64 + 4 / 128)
ALU_PEAK_TOPS = 256 * PE_OPS_PER_CU_CLK * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=1_000_000, help="frames per Eb/N0 point")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip side variants")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cfg", type=str, default="",
                    help="launch shape 'rho,slots' (skips the autotuner)")
    ap.add_argument("--calibrate", action="store_true",
                    help="only run the VALU and LDS calibration kernels and print their rates")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 4 times (HBM counter calibration)")
    ap.add_argument("--extra", type=str, default="",
                    help="only run one side workload of bench_workloads.py "
                         "(e.g. exact_boxplus, error_classes) and print its JSON")
    ap.add_argument("--extra-frames", type=int, default=0,
                    help="frames per point for --extra (0: the workload's default)")
    return ap.parse_args()


def calib_copy(torch):
    """A plain device-to-device copy of 2^30 bytes, four times: the reference
    for scaling FETCH_SIZE / WRITE_SIZE counters to bytes."""
    x = torch.empty(2 ** 28, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(4):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": 2 ** 30, "copies": 4}), flush=True)


def calibrate(torch, chains=False):
    """Measured roofline constants: the VALU issue rate of the decoder's
    instruction mix (add, v_med3_f32, v_bitop3_b32; 48 per loop trip) and the
    LDS read bandwidth (conflict-free 16-byte reads), from the kernels of
    libpbp_peak.so, each timed with HIP events on torch's stream.  chains:
    also the mix with the decoder's own dependencies (2, 4 or 8 rows per
    thread) at 1, 2, 4 and 8 waves per SIMD."""
    import ctypes
    path = os.path.join(ROOT, "paper_1911_08868_amd", "libpbp_peak.so")
    L = ctypes.CDLL(path)
    L.pbp_peak_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.pbp_peak_launch.restype = ctypes.c_int
    L.pbp_peak_launch_pe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p]
    L.pbp_peak_launch_pe.restype = ctypes.c_int
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {}
    if chains:
        tab = {}
        for rows in (2, 4, 8):
            for w in (1, 2, 4, 8):
                blocks, steps = 256 * w * 4, 4000
                out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
                ms = []
                for rep in range(3):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    rc = L.pbp_peak_launch_pe(rows, w, blocks, steps, ctypes.c_void_p(out.data_ptr()), stream)
                    b.record()
                    torch.cuda.synchronize()
                    if rc != 0:
                        raise RuntimeError(f"chain calibration rows {rows} waves {w}: HIP error {rc}")
                    ms.append(a.elapsed_time(b))
                ops = blocks * 256 * steps * 8 * (rows // 2) * 6
                tab[f"rows{rows}_waves{w}"] = round(ops / (min(ms) / 1e3) / 1e12, 2)
        res["pe_chain_TOPs"] = tab
    for which, blocks, threads, steps in ((0, 256 * 8, 256, 20000), (1, 256 * 2, 1024, 5000),
                                          (2, 256 * 8, 256, 15000), (3, 256 * 8, 256, 15000),
                                          (4, 256 * 8, 256, 15000)):
        out = torch.empty(blocks * threads, dtype=torch.int32, device="cuda")
        ms = []
        for rep in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            rc = L.pbp_peak_launch(which, blocks, steps, ctypes.c_void_p(out.data_ptr()), stream)
            b.record()
            torch.cuda.synchronize()
            if rc != 0:
                raise RuntimeError(f"calibration kernel {which}: HIP error {rc}")
            ms.append(a.elapsed_time(b))
        t = min(ms) / 1e3
        if which == 0:
            ops = blocks * 256 * 48 * steps
            res["valu_lane_ops_per_s"] = ops / t
            res["valu_frac_of_derived_peak"] = round(ops / t / (ALU_PEAK_TOPS * 1e12), 4)
        elif which == 1:
            byt = blocks * threads * 8 * 16 * steps
            res["lds_bytes_per_s"] = byt / t
            res["lds_bytes_per_clk_per_cu"] = round(byt / t / (256 * 2.4e9), 1)
        else:
            name = {2: "v_add_f32", 3: "v_med3_f32", 4: "v_xor_b32"}[which]
            ops = blocks * threads * 64 * steps
            res.setdefault("lanes_per_cu_clk", {})[name] = round(ops / t / (256 * 2.4e9), 1)
    return res


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("bp_core.h", "decode_kernel.h", "decode_inst.h"):
        with open(os.path.join(ROOT, "paper_1911_08868_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_inputs(pbp, code, frames, torch, seed=2024):
    """LLRs [len(SNRS)][frames, N] in device memory: random messages encoded on
    the GPU, BPSK over AWGN (synth's channel model)."""
    import synth
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    llrs, msgs = [], []
    for si, snr in enumerate(SNRS):
        m = torch.randint(0, 2, (frames, K_MSG), generator=gen, device="cuda", dtype=torch.uint8)
        x = pbp.encode(code, m)
        llrs.append(synth.awgn_llr_torch(x, snr, K_MSG, gen))
        del x
        msgs.append(m)
    torch.cuda.synchronize()
    return llrs, msgs


def alg_ops(iters):
    """Algorithmic VALU lane-ops of a decode launch: every processing element
    (N/2 per stage) costs 2 additions and 2 check-function evaluations of 2
    instructions each on gfx950 (clamp of one input by the magnitude of the
    other, then the other's sign applied), 6 ops, so a stage costs 3 N.  A
    frame needs `iters` L sweeps of n stages and iters - 1 R sweeps (the R
    sweep after the deciding L sweep cannot change the output) of n - 1
    stages (the R messages on the channel level are never read)."""
    n = 10
    it = iters.double().sum().item()
    return 3 * N * (n * it + (n - 1) * (it - iters.numel()))


def run_decode_set(pbp, code, llrs, outs, bp, pp, torch, events=None, cfg=None):
    for si in range(len(SNRS)):
        if events is not None:
            events[si][0].record()
        pbp.pp_mt_bp_decode(code, llrs[si], bp, pp, out=outs[si], cfg=cfg)
        if events is not None:
            events[si][1].record()


def cpu_cores():
    """(threads to use, cores visible): the cores this process may run on,
    capped at the 16 host cores an MI355X machine assigns to one GPU."""
    visible = os.cpu_count() or 1
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = visible
    return max(1, min(16, allowed)), visible, allowed


def cpu_baseline(args):
    """The oracle, as is, on a bounded sample of the same workload generated on
    the host (same code, decoder and parameters, FP32 mode), one thread per
    usable host core; also the oracle's frame error rate per Eb/N0 point with
    its 95% Clopper-Pearson interval, to set beside the GPU's."""
    import oracle
    import synth
    from bench_workloads import clopper_pearson
    threads, visible, allowed = cpu_cores()
    oc = oracle.construct(N, K, DESIGN_DB, CRC_W, CRC_POLY)
    p = oracle.DecodeParams(max_iter=MAX_ITER, stop=oracle.STOP_CRC, it_min=IT_MIN,
                            pp_mode=oracle.PP_LASTK, k=PP_K, T=PP_T, Q=PP_Q, seed=PP_SEED,
                            fp32=True)
    per = 16 * threads  # frames per Eb/N0 point in the first round; grown to fill the budget
    total_frames, total_time = 0, 0.0
    frames = [0] * len(SNRS)
    errors = [0] * len(SNRS)
    rounds = 0
    while total_time < args.cpu_seconds and rounds < 6:
        for si, snr in enumerate(SNRS):
            msg = synth.message_bits(1000 + rounds * 31 + si, per, K_MSG)
            _, x = oracle.encode(oc, msg)
            llr = synth.awgn_llr(x, snr, K_MSG, seed=2000 + rounds * 31 + si)
            t0 = time.perf_counter()
            r = oracle.decode(oc, llr, p, threads=threads)
            total_time += time.perf_counter() - t0
            total_frames += per
            frames[si] += per
            errors[si] += int((r.msg_hat != msg).any(1).sum())
        rounds += 1
        if total_time < args.cpu_seconds / 4:
            per *= 4
    gbps = total_frames * K_MSG / total_time / 1e9
    fer = [{"ebn0_db": snr, "frames": f, "frame_errors": e, "fer": e / f, "ci95": clopper_pearson(e, f)}
           for snr, f, e in zip(SNRS, frames, errors)]
    return {"value": gbps, "unit": "Gbit/s", "cores": threads, "kind": "oracle",
            "sample": f"{total_frames} frames spread evenly over the 9 Eb/N0 points "
                      f"(same code, decoder and parameters), FP32 mode, {total_time:.1f} s",
            "host_cores": {"visible": visible, "affinity": allowed, "used": threads},
            "fer": fer}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def lastk_variants(pbp, code, llrs, msgs, bp, cfg, torch, alu_peak):
    """PP-MT-BP with the last k in {3, 4, 5} of the 10 stages re-ordered
    every T in {5, 10} iterations (Q = 8 trellises), on the headline frames,
    each with its decoded Gbit/s and the decode kernel's ALU roofline
    fraction (same algorithmic count as the headline)."""
    F = llrs[0].shape[0]
    out = {}
    for k in (3, 4, 5):
        for T in (5, 10):
            pp = pbp.PPParams(mode=pbp.PP_LASTK, k=k, period_T=T, pool_Q=PP_Q, seed=PP_SEED)
            ox = [(torch.empty((F, K_MSG), dtype=torch.uint8, device="cuda"),
                   torch.empty(F, dtype=torch.int32, device="cuda"),
                   torch.empty(F, dtype=torch.uint8, device="cuda")) for _ in SNRS]
            run_decode_set(pbp, code, llrs, ox, bp, pp, torch, cfg=cfg)
            torch.cuda.synchronize()
            ev = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in SNRS]
            run_decode_set(pbp, code, llrs, ox, bp, pp, torch, events=ev, cfg=cfg)
            torch.cuda.synchronize()
            ms = sum(a.elapsed_time(b) for a, b in ev)
            ops = sum(alg_ops(o[1]) for o in ox)
            achieved = ops / (ms / 1e3) / 1e12
            out[f"k{k}_T{T}"] = {
                "gbit_s": round(len(SNRS) * F * K_MSG / (ms / 1e3) / 1e9, 3), "ms": round(ms, 2),
                "roofline": {"bound": "alu", "kernel": f"k_decode<n=10,k={k},rho={cfg.rho}>",
                             "achieved": round(achieved, 3), "peak": round(alu_peak, 2),
                             "unit": "TOP/s", "frac": round(achieved / alu_peak, 4)},
                "fer": [(o[0] != m).any(1).double().mean().item() for o, m in zip(ox, msgs)],
                "avg_iters": [round(o[1].double().mean().item(), 3) for o in ox]}
            log(f"last-{k} every {T}: {ms:.1f} ms, {out[f'k{k}_T{T}']['roofline']['frac']} of the ALU peak")
            del ox
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: only --gpus 1 is measured; decoding shards by frame ranges with no "
              "collective beyond a final count, so more GPUs would each run this same workload",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1911_08868_amd as pbp
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.calib_copy:
        calib_copy(torch)
        return
    if args.calibrate:
        print(json.dumps(calibrate(torch, chains=True)), flush=True)
        return
    if args.extra:
        import bench_workloads
        kw = {"F": args.extra_frames} if args.extra_frames else {}
        print(json.dumps(getattr(bench_workloads, args.extra)(torch, pbp, **kw)), flush=True)
        return
    code = pbp.Code(N, K, CRC_W, CRC_POLY, DESIGN_DB)
    F = args.frames
    llrs, msgs = make_inputs(pbp, code, F, torch)
    log(f"inputs ready: {len(SNRS)} x {F} frames")
    outs = [(torch.empty((F, K_MSG), dtype=torch.uint8, device="cuda"),
             torch.empty(F, dtype=torch.int32, device="cuda"),
             torch.empty(F, dtype=torch.uint8, device="cuda")) for _ in SNRS]
    bp = pbp.BPParams(max_iter=MAX_ITER, stop=pbp.STOP_CRC, it_min=IT_MIN)
    pp = pbp.PPParams(mode=pbp.PP_LASTK, k=PP_K, period_T=PP_T, pool_Q=PP_Q, seed=PP_SEED)
    # launch shape from the autotuner, timed on a sample of the 2.0 dB frames
    if args.cfg:
        rho, slots = (int(v) for v in args.cfg.split(","))
        cfg, tuned = pbp.LaunchCfg(rho, slots, 0), {"all": "fixed by --cfg"}
    else:
        cfg, tuned = pbp.tune.tune_decode(torch, code, llrs[2][: min(F, 200_000)], bp, pp,
                                          path=os.path.join("/tmp", "polarbp_tuned.json"),
                                          force=True)
    log(f"tuned launch shape rho={cfg.rho} slots={cfg.slots}: {tuned['all']}")
    cal = calibrate(torch)
    alu_peak = max(ALU_PEAK_TOPS, cal["valu_lane_ops_per_s"] / 1e12)
    log(f"calibration: the processing element's VALU mix at {cal['valu_lane_ops_per_s'] / 1e12:.2f} T lane-ops/s "
        f"({cal['valu_frac_of_derived_peak']} of the derived {ALU_PEAK_TOPS:.2f}), "
        f"LDS {cal['lds_bytes_per_clk_per_cu']} B/clk/CU; ALU peak taken {alu_peak:.2f} T lane-ops/s")
    lds_peak = cal["lds_bytes_per_s"] / 1e12

    for w in range(args.warmup):
        run_decode_set(pbp, code, llrs, outs, bp, pp, torch, cfg=cfg)
        torch.cuda.synchronize()
        log(f"warmup step {w + 1} done")
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in SNRS] for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for s in range(args.steps):
        run_decode_set(pbp, code, llrs, outs, bp, pp, torch, events=ev[s], cfg=cfg)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.2f} s")
    total_ms = start.elapsed_time(end)
    ms_per_step = total_ms / args.steps
    bits_per_step = len(SNRS) * F * K_MSG
    value = bits_per_step / (ms_per_step / 1e3) / 1e9

    # per-launch durations of the decode kernel and its algorithmic work
    per_snr = []
    launch_ms = 0.0
    ops_total = 0.0
    for si, snr in enumerate(SNRS):
        msg_hat, iters, ok = outs[si]
        d = sum(ev[s][si][0].elapsed_time(ev[s][si][1]) for s in range(args.steps)) / args.steps
        ops = alg_ops(iters)
        fer = (msg_hat != msgs[si]).any(1).double().mean().item()
        per_snr.append({"ebn0_db": snr, "ms": round(d, 3),
                        "gbit_s": round(F * K_MSG / (d / 1e3) / 1e9, 3),
                        "avg_iters": round(iters.double().mean().item(), 3),
                        "fer": fer})
        launch_ms += d
        ops_total += ops
    achieved = ops_total / (launch_ms / 1e3) / 1e12
    it_total = sum(o[1].double().sum().item() for o in outs)
    # group boundaries: the unpermuted 6 stages and the permuted 4 are each cut
    # into groups of at most rho stages
    boundaries = -(-(10 - PP_K) // cfg.rho) + -(-PP_K // cfg.rho) - 1
    lds_bytes_per_it = boundaries * 4 * 4 * N  # (L, R) x (written, read) x N x 4 B per boundary
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(alu_peak, 2),
            "unit": "TOP/s", "frac": round(achieved / alu_peak, 4), "traffic": None,
            "kernel": f"k_decode<n=10,k=4,rho={cfg.rho}>", "launch": {"rho": cfg.rho, "slots": cfg.slots,
                                                                   "tuned_ms": tuned["all"]},
            "ops_per_frame_iteration": 3 * N * (10 + 9),
            "launch_ms_avg": round(launch_ms / len(SNRS), 3),
            "lds": {"bytes_per_frame_iteration": lds_bytes_per_it,
                    "achieved_TBs": round(lds_bytes_per_it * it_total / (launch_ms / 1e3) / 1e12, 3),
                    "peak_TBs": round(lds_peak, 2), "peak_source": "measured (calibration)"},
            "peak_basis": f"max(derived {ALU_PEAK_TOPS:.2f}: 256 CUs x 2.4 GHz x 96 lane-ops of the processing "
                          f"element's mix per CU-clock, measured calibration)",
            "calibration": {"valu_TOPs": round(cal["valu_lane_ops_per_s"] / 1e12, 3),
                            "valu_frac_of_derived_peak": cal["valu_frac_of_derived_peak"],
                            "lds_TBs": round(lds_peak, 2),
                            "lds_bytes_per_clk_per_cu": cal["lds_bytes_per_clk_per_cu"],
                            "lanes_per_cu_clk": cal["lanes_per_cu_clk"]},
            "source_hash": kernel_source_hash()}
    prof = os.path.join(ROOT, "profiles", "k_decode_n1024_traffic.json")
    if os.path.exists(prof):
        try:
            t = json.load(open(prof))
            if t.get("source_hash") == roof["source_hash"]:
                roof["traffic"] = t.get("bytes_per_launch")
        except Exception:
            pass

    extras = {}
    if not args.no_extras:
        # plain BP and full permutation on the same frames (one pass each)
        for name, ppx in (("plain_bp", pbp.PPParams()),
                          ("full_permutation", pbp.PPParams(mode=pbp.PP_FULL, period_T=25,
                                                            pool_Q=8, seed=PP_SEED))):
            ox = [(torch.empty((F, K_MSG), dtype=torch.uint8, device="cuda"),
                   torch.empty(F, dtype=torch.int32, device="cuda"),
                   torch.empty(F, dtype=torch.uint8, device="cuda")) for _ in SNRS]
            run_decode_set(pbp, code, llrs, ox, bp, ppx, torch, cfg=cfg)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            run_decode_set(pbp, code, llrs, ox, bp, ppx, torch, cfg=cfg)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            log(f"{name}: {ms:.1f} ms")
            extras[name] = {"gbit_s": round(bits_per_step / (ms / 1e3) / 1e9, 3),
                            "ms": round(ms, 2),
                            "fer": [(o[0] != m).any(1).double().mean().item()
                                    for o, m in zip(ox, msgs)],
                            "avg_iters": [round(o[1].double().mean().item(), 3) for o in ox]}
            del ox
        # the other schedules of the same configuration: last k in {3, 4, 5}
        # stages every T in {5, 10} iterations (Q = 8), on the same frames
        extras["lastk_variants"] = lastk_variants(pbp, code, llrs, msgs, bp, cfg, torch, alu_peak)
        del llrs, outs
        torch.cuda.empty_cache()
        try:
            import bench_workloads
            bench_workloads.ALU_PEAK = alu_peak * 1e12
            extras.update(bench_workloads.bench_extras(torch, pbp))
        except ImportError as e:
            extras["weighted_bp"] = None
            extras["batched_mixed"] = None
            extras["extras_note"] = f"not available: {e}"

    out = {
        "metric": "decoded Gbit/s (N=1024 R=1/2 PP-MT-BP) + weighted-BP fwd+bwd frames/s vs plain",
        "value": round(value, 4), "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "PP-MT-BP N=1024 K=496+CRC16 R=1/2, Eb/N0 1.5:0.25:3.5 dB, "
                               f"{F} frames per point, last k=4 of 10 stages permuted every "
                               "T=10 iterations from Q=8 trellises, max 200 iterations, CRC stop",
                   "frames_per_step": len(SNRS) * F, "message_bits_per_frame": K_MSG},
        "roofline": roof,
        "per_ebn0": per_snr,
        "wall_s_timed": round(wall, 3),
    }
    out.update(extras)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args)
        # the oracle's frame error rate and interval beside the GPU's, per point
        for row, o in zip(per_snr, out["cpu_baseline"]["fer"]):
            row["oracle_fer"] = o["fer"]
            row["oracle_frames"] = o["frames"]
            row["oracle_ci95"] = [round(x, 6) for x in o["ci95"]]
            row["gpu_fer_in_oracle_ci95"] = bool(o["ci95"][0] <= row["fer"] <= o["ci95"][1])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Frame error rates of the two readings of Algorithm 1 (Sec. III), beside plain BP.

Test infrastructure, like the rest of this package: it calls only the oracle
and the seeded input generators, on the CPU.

Reading R1 (the one the library implements): each event draws its subgraph
from the CURRENT graph, permutes it, and leaves the rest of the graph as it
is, so permutations accumulate over events.
Reading R2: each event first restores the block it permuted last to the
original stage order (its inner levels reset), then permutes one aligned block
of the ORIGINAL graph, so the decoder is never more than one block away from
the original trellis.

Both use the Table I parameters for the 2e4-iteration budget, CRC early stop
from iteration 3, and the same frames (message bits and channel noise from the
same seeds).  Plain BP stops at 200 iterations: frames it has not decoded by
then are stuck in its fixed points, which is the case partial permutation is
meant for.

    python -m oracle.alg1_readings --frames 2000 --ebn0 2.0 2.5 3.0 --threads 8
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# Table I, N_it,max = 2e4, with the codes of Sec. IV
SETS = {
    "N1024_R0.5": dict(N=1024, K=512, crc=16, poly=0x1021, design=2.5,
                       P_range=10, P_level=9, D=100, N_min=15),
    "N512_R0.65": dict(N=512, K=333, crc=24, poly=0x1864CFB, design=2.5,
                       P_range=9, P_level=8, D=50, N_min=15),
}


def clopper_pearson(k: int, n: int, conf: float = 0.95):
    from scipy.stats import beta
    a = (1 - conf) / 2
    lo = 0.0 if k == 0 else float(beta.ppf(a, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - a, k + 1, n - k))
    return lo, hi


def run(name: str, ebn0: float, F: int, threads: int, max_iter: int, seed: int):
    s = SETS[name]
    code = oracle.construct(s["N"], s["K"], s["design"], s["crc"], s["poly"])
    msg = synth.message_bits(seed, F, code.K_msg)
    _, x = oracle.encode(code, msg)
    llr = synth.awgn_llr(x, ebn0, code.K_msg, seed=seed)
    out = {"set": name, "ebn0_db": ebn0, "frames": F}
    modes = (("plain", oracle.PP_NONE, 200), ("R1", oracle.PP_ALG1, max_iter),
             ("R2", oracle.PP_ALG1_R2, max_iter))
    for label, mode, mi in modes:
        p = oracle.DecodeParams(max_iter=mi, stop=oracle.STOP_CRC, it_min=3, pp_mode=mode,
                                P_range=s["P_range"], P_level=s["P_level"], D=s["D"],
                                N_min=s["N_min"], seed=seed + 17)
        t0 = time.time()
        r = oracle.decode(code, llr, p, threads=threads)
        err = int((r.msg_hat != msg).any(1).sum())
        out[label] = {"errors": err, "fer": err / F, "ci95": clopper_pearson(err, F),
                      "mean_iter": float(r.iters.mean()), "max_iter": mi,
                      "seconds": round(time.time() - t0, 1)}
        print(f"{name} {ebn0:.2f} dB {label:5s} FER {err}/{F} = {err / F:.4f} "
              f"CI [{out[label]['ci95'][0]:.4f}, {out[label]['ci95'][1]:.4f}] "
              f"mean it {r.iters.mean():.1f}  ({out[label]['seconds']} s)", flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", nargs="+", default=list(SETS))
    ap.add_argument("--ebn0", nargs="+", type=float, default=[2.0, 2.5, 3.0])
    ap.add_argument("--frames", type=int, default=2000)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--json", default="")
    a = ap.parse_args(argv)
    res = [run(s, e, a.frames, a.threads, a.max_iter, a.seed + int(round(e * 100)))
           for s in a.sets for e in a.ebn0]
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main()

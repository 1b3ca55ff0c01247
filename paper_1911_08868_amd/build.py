"""Build the HIP library ``libpolarbp.so`` for gfx950 with hipcc.

Every translation unit is compiled in parallel into ``_build/`` and linked
in-tree, so the library travels with the source tree.  The decode kernels are
instantiated once per block length (PBP_NLOG = 1..12) in separate objects,
and once more per length for each of the decision-history, exact-boxplus
and noise-injection kernel families.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpolarbp.so")
PEAK_LIB = os.path.join(HERE, "libpbp_peak.so")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PBP_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # IEEE arithmetic exactly as written: no fused multiply-add, no denormal flush
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-lambda-capture",
]


def _units():
    units = []
    for n in range(1, 13):
        units.append((os.path.join(CSRC, "decode_inst.hip"), f"decode_n{n:02d}.o", [f"-DPBP_NLOG={n}"]))
    for n in range(1, 13):
        units.append((os.path.join(CSRC, "decode_inst.hip"), f"decode_trace_n{n:02d}.o",
                      [f"-DPBP_NLOG={n}", "-DPBP_VARIANT=1"]))
        units.append((os.path.join(CSRC, "decode_inst.hip"), f"decode_exact_n{n:02d}.o",
                      [f"-DPBP_NLOG={n}", "-DPBP_VARIANT=2"]))
        units.append((os.path.join(CSRC, "decode_inst.hip"), f"decode_noise_n{n:02d}.o",
                      [f"-DPBP_NLOG={n}", "-DPBP_VARIANT=3"]))
    for n in range(4, 13):
        units.append((os.path.join(CSRC, "wbp_inst.hip"), f"wbp_n{n:02d}.o", [f"-DPBP_NLOG={n}"]))
    for src in ("host.cpp", "dispatch.cpp", "encode.hip", "wbp.hip", "batched.hip", "alg1.hip", "alg1_orig.hip", "diag.hip"):
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        units.append((os.path.join(CSRC, src), os.path.splitext(src)[0] + ".o", lang))
    return units


def _headers_mtime():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(os.path.dirname(HERE), "include", "polarbp.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(unit, extra, incremental=False, hdr_mtime=0.0):
    src, obj, defs = unit
    out = os.path.join(BUILD, obj)
    if incremental and os.path.exists(out) and \
            os.path.getmtime(out) > max(os.path.getmtime(src), hdr_mtime):
        return out
    cmd = [HIPCC, *FLAGS, *extra, *defs, "-c", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {defs}:\n{r.stdout}\n{r.stderr}")
    return out


def build(jobs: int | None = None, extra: list[str] | None = None, verbose: bool = False,
          incremental: bool = False) -> str:
    """Compile every unit and link.  incremental=True (development only)
    skips a unit whose object is newer than its source and every header."""
    os.makedirs(BUILD, exist_ok=True)
    extra = extra or []
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = _units()
    hm = _headers_mtime()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, extra, incremental, hm), units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # the roofline calibration kernels of bench.py, a library of their own
    peak_obj = _compile((os.path.join(CSRC, "peak.hip"), "peak.o", []), extra, incremental, hm)
    tmp = PEAK_LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, peak_obj],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PEAK_LIB)
    if verbose:
        print(f"built {LIB} and {PEAK_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)

"""Autotuner of launch shapes: rows per thread (rho, which sets the stage-group
tiling), frames per workgroup (slots) and grid size.

Each candidate is timed with HIP events on a sample of the real workload and
the fastest is kept.  Results are cached per device name and workload key in
``tuned.json`` next to this file (or a path given by the caller) so that a
tuning run on the GPU can be reused by later runs.
"""
from __future__ import annotations

import json
import os

from . import api

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def _device_key(torch) -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}:{getattr(p, 'gcnArchName', '')}:{p.multi_processor_count}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def decode_candidates(N: int):
    """Valid (rho, slots) shapes for one block length (workgroup <= 256 threads
    per frame set, or one frame when a frame needs more)."""
    out = []
    for rho in (2, 3):
        if (1 << rho) > N:
            continue
        tps = N >> rho
        max_slots = 1 if tps >= 256 else 256 // tps
        s = 1
        while s <= max_slots:
            out.append(api.LaunchCfg(rho, s, 0))
            s *= 2
    return out


def _pick(results, default=(2, 1, 0), margin=0.02):
    """Fastest shape, but the default unless another beats it by the margin:
    timing noise must not flip the choice between near-equal shapes."""
    best = min(results, key=lambda r: r[1])
    for cfg, ms in results:
        if cfg == default and best[1] * (1 + margin) >= ms:
            return (cfg, ms)
    return best


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_decode(torch, code: api.Code, llr, bp: api.BPParams, pp: api.PPParams | None,
                key: str | None = None, reps: int = 3, path: str = _CACHE, force=False):
    """Pick the fastest launch shape for decoding `llr` with this code and schedule."""
    key = key or f"decode:N{code.N}:K{code.K}:c{code.crc_width}:pp{pp.mode if pp else -1}:k{pp.k if pp else 0}"
    dk = _device_key(torch)
    cache = _load(path)
    if not force and dk in cache and key in cache[dk]:
        c = cache[dk][key]["cfg"]
        return api.LaunchCfg(*c), cache[dk][key]
    F = llr.shape[0]
    out = (torch.empty((F, code.K_msg), dtype=torch.uint8, device="cuda"),
           torch.empty(F, dtype=torch.int32, device="cuda"),
           torch.empty(F, dtype=torch.uint8, device="cuda"))
    results = []
    for cfg in decode_candidates(code.N):
        try:
            ms = _time(torch, lambda: api.pp_mt_bp_decode(code, llr, bp, pp, out=out, cfg=cfg), reps)
        except api.PolarError:
            continue
        results.append(((cfg.rho, cfg.slots, cfg.grid), ms))
    best = _pick(results)
    entry = {"cfg": list(best[0]), "ms": best[1], "all": [[list(c), m] for c, m in results],
             "frames": F}
    cache.setdefault(dk, {})[key] = entry
    try:
        _store(path, cache)
    except OSError:
        pass
    return api.LaunchCfg(*best[0]), entry


def tune_batched(torch, dec, reps: int = 2, path: str = _CACHE, force=False):
    """Pick rho, workgroup size and grid for the persistent mixed-length kernel."""
    key = "batched:" + ",".join(f"{c.N}/{c.K}" for c in dec.codes)
    dk = _device_key(torch)
    cache = _load(path)
    if not force and dk in cache and key in cache[dk]:
        c = cache[dk][key]["cfg"]
        return api.LaunchCfg(*c), cache[dk][key]
    results = []
    saved = dec.cfg
    for cfg in (api.LaunchCfg(0, 1, 0), api.LaunchCfg(0, 2, 0), api.LaunchCfg(2, 1, 0),
                api.LaunchCfg(2, 2, 0), api.LaunchCfg(3, 1, 0), api.LaunchCfg(3, 2, 0)):
        dec.cfg = cfg
        try:
            ms = _time(torch, dec.run, reps)
        except api.PolarError:
            continue
        results.append(((cfg.rho, cfg.slots, cfg.grid), ms))
    dec.cfg = saved
    best = _pick(results, default=(0, 1, 0))
    entry = {"cfg": list(best[0]), "ms": best[1], "all": [[list(c), m] for c, m in results],
             "frames": dec.F}
    cache.setdefault(dk, {})[key] = entry
    try:
        _store(path, cache)
    except OSError:
        pass
    return api.LaunchCfg(*best[0]), entry

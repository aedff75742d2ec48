"""Autotuner for choices that need a fresh context: kernel path (gather or
staged), list skin, staged tile length (cells per row tile).  Each candidate runs a short trial
from the caller's state in its own context (the caller's context is never
touched); inside each trial md_autotune picks the force-kernel variant
(lanes per particle, unroll).  The fastest candidate wins.

The skin only trades list length against rebuild frequency: the forces are
those of every pair within the cutoff whatever the skin, so tuning it changes
speed, not results.

Results are cached in a JSON file keyed by device name, particle-count
bucket, replica-count bucket, precision and largest cutoff.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import md

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                             "paper_1105_5613_amd", "tune.json")


def _key(params: md.Params, ntot: int, nrep: int) -> str:
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    rcmax = max(params.rc[a * md.MAXT + b] for a in range(params.ntypes)
                for b in range(params.ntypes))
    nb = 2 ** int(round(math.log2(max(ntot, 1))))
    rb = 2 ** int(round(math.log2(max(nrep, 1))))
    return f"{dev}|n{nb}|r{rb}|p{params.precision}|rc{rcmax:.4f}"


def _with(params: md.Params, **kw) -> md.Params:
    p = md.Params.from_buffer_copy(params)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _min_cells(L, params: md.Params, skin: float) -> int:
    rcmax = max(params.rc[a * md.MAXT + b] for a in range(params.ntypes)
                for b in range(params.ntypes))
    return min(int(math.floor(l / (rcmax + skin))) for l in L)


def autotune(params: md.Params, n, L, x, v, types, *, T0=None, steps: int = 60,
             warmup: int = 20, skins=None, paths=(md.MD_PATH_GATHER, md.MD_PATH_STAGED),
             tile_cells=(0,), cache_path: str | None = DEFAULT_CACHE,
             use_cache: bool = True):
    """Return (tuned Params, report).  n, L: per-replica sizes and box sides;
    x, v, types: the state to trial on (device or host arrays)."""
    import torch
    n = [int(t) for t in (n if hasattr(n, "__len__") else [n])]
    L = [float(t) for t in (L if hasattr(L, "__len__") else [L])]
    key = _key(params, sum(n), len(n))
    if use_cache and cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cached = json.load(f).get(key)
        if cached:
            return _with(params, **cached["choice"]), {"cached": True, **cached}
    skins = [params.skin] if skins is None else list(skins)
    cands = []
    for skin in skins:
        for path in paths:
            if path == md.MD_PATH_STAGED:
                if _min_cells(L, params, skin) < 3:
                    continue
                for tc in tile_cells:
                    cands.append(dict(path=path, skin=float(skin), tile_cells=int(tc)))
            else:
                cands.append(dict(path=path, skin=float(skin)))
    trials = []
    for cand in cands:
        p = _with(params, **cand)
        try:
            s = md.System(p, n, L)
        except md.MDError:
            continue
        s.set_state(x, v, types)
        s.step(warmup, T0=T0)
        t = s.autotune(reps=3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, T0=T0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        choice = dict(cand, tpp=t["tpp"], unroll=t["unroll"])
        trials.append({"choice": choice, "rate": sum(n) * steps / wall,
                       "force_ms": t["force_ms"]})
    if not trials:
        return params, {"cached": False, "trials": []}
    best = max(trials, key=lambda r: r["rate"])
    report = {"cached": False, "choice": best["choice"], "rate": best["rate"], "trials": trials}
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        data = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                data = json.load(f)
        data[key] = {"choice": best["choice"], "rate": best["rate"]}
        with open(cache_path, "w") as f:
            json.dump(data, f, indent=1)
    return _with(params, **best["choice"]), report

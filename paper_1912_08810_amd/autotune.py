"""Tile-shape autotuner for batched launches.

For every size bucket (energy count x frequency count) and precision, the tuner
times the persistent batched kernel on a representative instance for each
candidate pair (energies per tile ``sse_desc.tile_e``, frequencies per tap chunk
``sse_desc.chunk_taps``) and keeps the fastest.  The search is exhaustive over the
candidates -- the idea of choosing a decomposition by searching all feasible tile
sizes (the paper searches data-movement tilings exhaustively, Sec. 4.1) applied
to the on-chip tile.  Every bucket records the time of every candidate, the
library default's (0, 0) and the gain of the pick over it; a candidate replaces
the default only when it is at least 1% faster.  Results are cached
as JSON keyed by (arch, precision, Norb).
"""
from __future__ import annotations

import json
import os
import statistics

import numpy as np

from . import configs

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

# Buckets over (NE, Nw): upper bounds, inclusive.
NE_EDGES = (600, 1000, 1500)
NW_EDGES = (20, 30, 40)


def bucket_of(NE: int, Nw: int):
    bi = next((i for i, x in enumerate(NE_EDGES) if NE <= x), len(NE_EDGES) - 1)
    bj = next((j for j, x in enumerate(NW_EDGES) if Nw <= x), len(NW_EDGES) - 1)
    return bi, bj


def candidates(prec: int, Norb: int):
    """(tile_e, chunk_taps) pairs: the largest tile that fills a workgroup (the
    default), three quarters and half of it, each with the longest chunk the
    window holds (0, the default), 16 and 8 frequencies."""
    nn = Norb * Norb
    tmax = max(1, 1024 // nn)  # output positions per workgroup: 1024 on both paths
    tiles = sorted({tmax, max(1, tmax * 3 // 4), max(1, tmax // 2)}, reverse=True)
    return [(te, ct) for te in tiles for ct in (0, 16, 8)]


def _key(prec: int, Norb: int) -> str:
    return f"gfx950/prec={prec}/Norb={Norb}"


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def params_for(prec: int, Norb: int, NE: int, Nw: int, cache: dict | None = None):
    """Tuned (tile_e, chunk_taps) for an instance; (0, 0) (the library defaults)
    if the bucket is untuned."""
    cache = load_cache() if cache is None else cache
    tab = cache.get(_key(prec, Norb))
    if not tab:
        return 0, 0
    bi, bj = bucket_of(NE, Nw)
    ent = tab.get(f"{bi},{bj}", {})
    return int(ent.get("tile_e", 0)), int(ent.get("chunk_taps", 0))


def tile_for(prec: int, Norb: int, NE: int, Nw: int, cache: dict | None = None) -> int:
    """Tuned tile_e for an instance; 0 (library default) if the bucket is untuned."""
    return params_for(prec, Norb, NE, Nw, cache)[0]


def _time_instance(prob, prec, tile_e, chunk_taps, reps, seed):
    import torch
    from ssegen.device_problem import DeviceProblem
    from . import sse
    fp32 = prec in (1, 2, 3)
    dp = DeviceProblem(prob, seed, ncomp=1, fp32=fp32)
    desc = sse.make_desc(prob.NA, prob.NB, prob.Norb, prob.Nkz, prob.Nqz, prob.NE, prob.Nw,
                         prec=prec, tile_e=tile_e, chunk_taps=chunk_taps)
    plan = sse.sse_plan_batch([desc], [prob.shifts()])
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    item = [(dp.neigh, dp.dH, dp.G, dp.D, dp.Sigma)]
    sse.sse_wait(sse.sse_submit(plan, item, ws, stream))  # warm-up, builds tables
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        t = sse.sse_submit(plan, item, ws, stream)
        e1.record(stream)
        sse.sse_wait(t)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del dp, ws
    return statistics.median(ts)


def tune(prec: int, Norb: int = 10, NA: int = 192, reps: int = 3, seed: int = 7,
         path: str = CACHE, log=print) -> dict:
    """Exhaustive search over the candidates for every bucket; updates the cache."""
    tab = {}
    ne_lo = (200,) + tuple(x + 1 for x in NE_EDGES[:-1])
    nw_lo = (10,) + tuple(x + 1 for x in NW_EDGES[:-1])
    for bi, (lo, hi) in enumerate(zip(ne_lo, NE_EDGES)):
        for bj, (wl, wh) in enumerate(zip(nw_lo, NW_EDGES)):
            prob = configs.Problem(NA=NA, NB=4, Norb=Norb, Nkz=5, Nqz=5, NE=(lo + hi) // 2,
                                   Nw=(wl + wh) // 2)
            times = {(0, 0): _time_instance(prob, prec, 0, 0, reps, seed)}
            for te, ct in candidates(prec, Norb):
                times[(te, ct)] = _time_instance(prob, prec, te, ct, reps, seed)
            best = min(times, key=times.get)
            if times[(0, 0)] < 1.01 * times[best]:
                best = (0, 0)   # within timing noise of the default: keep it
            tab[f"{bi},{bj}"] = {
                "tile_e": best[0], "chunk_taps": best[1], "NE": prob.NE, "Nw": prob.Nw,
                "ms": {f"{te},{ct}": round(v * 1e3, 3) for (te, ct), v in times.items()},
                "default_ms": round(times[(0, 0)] * 1e3, 3),
                "gain_vs_default": round(times[(0, 0)] / times[best], 4)}
            log(f"tune prec={prec} bucket NE<={hi} Nw<={wh}: best tile_e={best[0]} "
                f"chunk_taps={best[1]}, {times[(0, 0)] / times[best]:.3f}x the default "
                f"({', '.join(f'{k[0]},{k[1]}:{v*1e3:.1f}ms' for k, v in times.items())})")
    cache = load_cache(path)
    cache[_key(prec, Norb)] = tab
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    return tab


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="tune (tile_e, chunk_taps) per size bucket")
    ap.add_argument("precs", nargs="*", type=int, default=[0, 1, 2])
    ap.add_argument("--out", default=CACHE, help="cache file to update")
    a = ap.parse_args()
    for p in a.precs:
        tune(p, path=a.out)

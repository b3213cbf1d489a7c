"""Tile autotuner: picks ligands-per-workgroup (LPW) and poses-per-lane (PPL).

For a workload (pockets + ligand sample + search settings) every admissible tile
is timed through the C ABI (device time of the dock launch, HIP events), the
fastest is kept, and the choice is cached in a JSON file keyed by device name,
search settings, texel storage, launch mode and a ligand-size bucket.
Marshalling and timing only: the docking itself runs in libexs.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np

from . import binding as B

PPL_CHOICES = (1, 2, 4)
LPW_CHOICES = (1, 2, 4, 8)


def candidate_tiles(n_orient: int) -> List[Tuple[int, int]]:
    """Every (poses per lane, ligands per workgroup) of {1, 2, 4} x {1, 2, 4, 8}: the library
    fits any of them in a workgroup (its waves take a tile's orientation chunks in turn when
    the tile has more chunks than the workgroup has waves) and refuses one only when a single
    wave's LDS does not fit, which tune() then skips."""
    return [(ppl, lpw) for ppl in PPL_CHOICES for lpw in LPW_CHOICES]


def cache_path() -> str:
    return os.environ.get("EXS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "exs", "tiles.json"))


def _device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:   # noqa: BLE001 - name only used as a cache key
        return "unknown"


def cache_key(search, storage: int, flags: int, mean_atoms: float) -> str:
    bucket = int(mean_atoms // 16) * 16
    return "|".join(str(x) for x in (_device_name(), search.n_orient, search.torsion_steps,
                                     search.passes, search.n_offsets, storage,
                                     flags & B.EXS_FLAG_PERSISTENT, bucket))


def load_cache() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: Dict[str, dict]):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def time_tile(batch_id: int, search, ppl: int, lpw: int, flags: int, reps: int = 2,
              stream=None) -> float:
    """Median device time (ms) of the dock launch(es) of one tile configuration."""
    prm = B.search_params(search.n_orient, search.torsion_steps, search.passes, search.n_offsets,
                          search.offset_step, search.clash_cutoff, search.clash_penalty,
                          top_k=search.top_k, poses_per_lane=ppl, ligands_per_wg=lpw, flags=flags)
    times = []
    for _ in range(reps + 1):
        job = B.exs_dock_batch(batch_id, prm, stream=stream)
        times.append(B.exs_job_elapsed_ms(job))
        B.exs_release_job(job)
    return float(np.median(times[1:]))


def tune(batch_id: int, search, storage: int, flags: int, mean_atoms: float,
         tiles: Optional[Iterable[Tuple[int, int]]] = None, use_cache: bool = True,
         stream=None, log=None) -> dict:
    """Time every admissible tile on an uploaded sample batch; returns
    {"ppl", "lpw", "ms", "timings"} and caches it."""
    key = cache_key(search, storage, flags, mean_atoms)
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key], cached=True)
    timings = {}
    for ppl, lpw in (tiles or candidate_tiles(search.n_orient)):
        try:
            ms = time_tile(batch_id, search, ppl, lpw, flags, stream=stream)
        except B.ExsError as e:      # a tile the settings do not admit
            if log:
                log("tile ppl=%d lpw=%d rejected: %s" % (ppl, lpw, e))
            continue
        timings["%d,%d" % (ppl, lpw)] = ms
        if log:
            log("tile ppl=%d lpw=%d: %.2f ms" % (ppl, lpw, ms))
    best = min(timings, key=timings.get)
    ppl, lpw = (int(x) for x in best.split(","))
    rec = {"ppl": ppl, "lpw": lpw, "ms": timings[best], "timings": timings}
    if use_cache:
        cache[key] = rec
        save_cache(cache)
    return dict(rec, cached=False)

"""Autotuner cache: launch choices found by ``ba_autotune`` stored as JSON,
keyed by the GPU architecture and a coarse class of the workload (windows,
clusters, largest voxel degree, storage precision), so that problems of the
same class skip the search."""
from __future__ import annotations

import json
import math
import os

import torch

from . import _lib

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2608_14266_amd", "tuning.json")


def _bucket(v: int) -> int:
    """Power-of-two bucket of a size (0 for 0)."""
    return 0 if v <= 0 else 1 << int(math.floor(math.log2(v)))


def workload_class(info: dict) -> str:
    return (f"w{_bucket(info['n_windows'])}-c{_bucket(info['n_clusters'])}-m{_bucket(info['max_m'])}"
            f"-p{info['precision']}")


def cache_key(info: dict, device=None) -> str:
    arch = torch.cuda.get_device_properties(device or torch.cuda.current_device()).gcnArchName.split(":")[0]
    return f"{arch}|{workload_class(info)}"


def tuned(problem, poses, cache_path: str | None = DEFAULT_CACHE, reps: int = 5, refresh: bool = False) -> dict:
    """Apply cached launch choices for this problem's class, or run the
    autotuner at `poses` and store its result.  Returns the choices and
    whether they came from the cache."""
    key = cache_key(problem.info())
    table = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if not refresh and key in table:
        _lib.problem_set_tuning(problem, table[key])
        return dict(table[key], cached=True, key=key)
    best = _lib.autotune(problem, poses, reps)
    if cache_path:
        table[key] = best
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return dict(best, cached=False, key=key)

"""Tuning cache of the Krylov step's launch parameters.

The library's autotuner (rann_dd_autotune) times CG iterations for every
candidate of the persistent grid of the FP64 local solves, the grid cap of the
CG vector kernels and graph replay of the check windows, and keeps the fastest
on the handle.  This module keeps its choices in a JSON file keyed by the GPU
architecture and the case (precision, preconditioner, stencil, right-hand
sides, and size buckets of the handle), so that later handles of the same
shape start from the stored parameters without timing again.

Cache file: $RANN_DD_TUNING_CACHE, else ~/.cache/rann_dd/tuning.json.
"""
from __future__ import annotations

import json
import math
import os

from . import binding


def cache_path() -> str:
    return os.environ.get("RANN_DD_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rann_dd", "tuning.json"))


def _arch(torch, dev) -> str:
    try:
        return str(torch.cuda.get_device_properties(dev).gcnArchName).split(":")[0]
    except Exception:  # a device without the property: the name stands in
        return torch.cuda.get_device_name(dev)


def _bucket(x: int) -> int:
    """Size bucket: the power of two at or above x."""
    return 1 << max(0, math.ceil(math.log2(max(int(x), 1))))


def case_key(solver, k: int) -> str:
    info = solver.info
    return "|".join([_arch(solver.torch, solver.dev), solver.precision, solver.precond, solver.stencil,
                     f"k{int(k)}", f"P{_bucket(info.P)}", f"F{_bucket(info.factor_elems)}",
                     f"N{_bucket(info.normal_elems)}"])


def _load(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def tune(solver, k: int, iters: int = 20, use_cache: bool = True) -> dict:
    """Set the solver's launch parameters for k right-hand sides and return
    them (with "source": "cache" or "timed" and the time per iteration)."""
    path = cache_path()
    key = case_key(solver, k)
    data = _load(path) if use_cache else {}
    rec = data.get(key)
    if rec is not None:
        solver.set_tuning(tile_grid=rec["tile_grid"], red_cap=rec["red_cap"], use_graph=rec["use_graph"])
        return dict(rec, source="cache")
    t, us = binding.rann_dd_autotune(solver.handle, k, iters)
    rec = dict(t.as_dict(), us_per_iteration=us)
    if use_cache:
        data = _load(path)
        data[key] = rec
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return dict(rec, source="timed")

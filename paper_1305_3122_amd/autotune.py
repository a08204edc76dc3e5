"""Autotuner of the row-owner launch shape (LDS tile size, persistent grid).

Times every candidate ``fem_tune`` on the actual pattern with HIP events and
keeps the fastest; results are cached in a JSON file keyed by device name and
problem size (``$FEM_TUNE_CACHE``, default ``~/.cache/fem_p1_tune.json``).
"""
from __future__ import annotations

import json
import os

from ._lib import fem_tune

LDS_ENTRIES = (448, 512, 640, 768)
GRID_PER_CU = (0, 8, 16, 32)      # 0: one workgroup per tile (non-persistent)


def _cache_path() -> str:
    return os.environ.get("FEM_TUNE_CACHE", os.path.expanduser("~/.cache/fem_p1_tune.json"))


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c: dict) -> None:
    try:
        os.makedirs(os.path.dirname(_cache_path()), exist_ok=True)
        with open(_cache_path(), "w") as f:
            json.dump(c, f, indent=1)
    except OSError:
        pass


def tune_batched(fem, torch, pat, q, nb: int, reps: int = 5, use_cache: bool = True):
    """Returns (best fem_tune, {candidate: microseconds})."""
    props = torch.cuda.get_device_properties(0)
    n_cu = props.multi_processor_count
    key = f"{props.name}|stiff_mass|nq={pat.nq}|nnz={pat.nnz}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        e = cache[key]
        return fem_tune(e["lds_entries"], e["grid_blocks"]), e.get("table", {})
    S = torch.empty(pat.nnz, dtype=torch.float64, device=q.device)
    M = torch.empty_like(S)
    table = {}
    best, best_us = None, float("inf")
    for eb in LDS_ENTRIES:
        for g in GRID_PER_CU:
            t = fem_tune(eb, g * n_cu)
            fem.fem_assemble_stiff_mass_batched(pat, q, nb, tune=t, out_S=S, out_M=M)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fem.fem_assemble_stiff_mass_batched(pat, q, nb, tune=t, out_S=S, out_M=M)
            b.record()
            torch.cuda.synchronize()
            us = a.elapsed_time(b) * 1e3 / reps
            table[f"{eb}/{g * n_cu}"] = round(us, 1)
            if us < best_us:
                best, best_us = t, us
    if use_cache:
        cache[key] = {"lds_entries": best.lds_entries, "grid_blocks": best.grid_blocks,
                      "table": table}
        _store_cache(cache)
    return best, table

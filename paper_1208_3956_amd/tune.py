"""On-disk cache of the strip solver's autotuned y-partition (rows per chunk).

One JSON object maps a problem-shape key to {"chunk_rows": m, "ms_per_apply": {...}}.
Writes go through a temporary file and a rename, so a reader never sees half a file.
"""
from __future__ import annotations

import json
import os
from typing import Optional, Sequence


def key(device: str, prec: str, mode: str, dims: Sequence[int], widths: Sequence[int], nrhs: int) -> str:
    return "|".join([device, prec, mode, "x".join(map(str, dims)),
                     ",".join(map(str, widths)), str(int(nrhs))])


def cache_path(cache: Optional[str]) -> Optional[str]:
    if cache is None:
        return None
    if cache != "default":
        return cache
    env = os.environ.get("HELM_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1208_3956_amd", "tune.json")


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def lookup(path: str, k: str) -> Optional[int]:
    ent = _load(path).get(k)
    if isinstance(ent, dict) and isinstance(ent.get("chunk_rows"), int) and ent["chunk_rows"] >= 2:
        return ent["chunk_rows"]
    return None


def store(path: str, k: str, best: int, times: dict) -> None:
    data = _load(path)
    data[k] = {"chunk_rows": int(best), "ms_per_apply": {str(c): float(t) for c, t in times.items()}}
    d = os.path.dirname(path)
    try:
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass            # a read-only home: the choice still applies to this handle

"""Autotuned (tile, pixels per lane) for batched fitting, remembered in a
JSON file.

`gs2d_autotune_batch` times every candidate on the device (a few graph-free
rounds of binning + persistent raster each) and returns the fastest.  The
choice depends on the GPU, the library build and the batch's frame sizes and
Gaussian counts, so that triple keys the cache: a later call with the same
key returns the stored choice without timing anything.  The file is written
atomically (temporary file + rename); a missing or unreadable file counts as
empty.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile

from . import _lib

CANDIDATES = ((8, 1), (16, 1), (16, 2), (32, 1), (32, 2), (32, 4))


def default_cache_path() -> str:
    """$GS2D_AUTOTUNE_CACHE, else ~/.cache/gs2d/autotune.json."""
    p = os.environ.get("GS2D_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "gs2d", "autotune.json")


def _library_digest() -> str:
    h = hashlib.sha256()
    with open(_lib.LIB_PATH, "rb") as f:
        for block in iter(lambda: f.read(1 << 20), b""):
            h.update(block)
    return h.hexdigest()[:16]


def cache_key(device_name: str, library: str, sizes, candidates) -> str:
    """Key of one tuning: device, library build, the batch's (W, H, N) list
    in order and the candidate list."""
    spec = json.dumps({"sizes": [list(map(int, s)) for s in sizes],
                       "candidates": [list(map(int, c)) for c in candidates]},
                      sort_keys=True)
    return f"{device_name}|{library}|{hashlib.sha256(spec.encode()).hexdigest()[:16]}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".autotune.", dir=d)
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise


def tuned_batch_config(sizes, targets, xy, chol, rgb, candidates=CANDIDATES, reps=3,
                       cache_path: str | None = None, device_name: str | None = None,
                       library: str | None = None):
    """(tile, px_per_lane) for this batch, the per-candidate ms per round
    ({} on a cache hit) and whether it came from the cache.  cache_path None
    disables the cache (always times)."""
    candidates = [tuple(c) for c in candidates]
    key = None
    if cache_path is not None:
        if device_name is None:
            import torch
            device_name = torch.cuda.get_device_name(xy.device)
        key = cache_key(device_name, library or _library_digest(), sizes, candidates)
        hit = _load(cache_path).get(key)
        if hit and tuple(hit.get("best", ())) in candidates:
            return tuple(hit["best"]), {}, True
    best, ms = _lib.autotune_batch(sizes, targets, xy, chol, rgb, candidates, reps=reps)
    timings = {f"{t}/{p}": m for (t, p), m in zip(candidates, ms)}
    if key is not None:
        data = _load(cache_path)
        data[key] = {"best": list(candidates[best]), "ms_per_round": timings}
        _store(cache_path, data)
    return candidates[best], timings, False

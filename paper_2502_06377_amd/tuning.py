"""Autotuner cache for the batched form.

``tuned(batch)`` looks up the tile configurations of a batch in a JSON cache keyed by GPU
architecture and the batch's sizes; on a miss it runs the library's autotuner
(``ibmi_batch_autotune``, which times sweeps of every candidate on the device) and stores the
winner.  The cache path is ``$IBMI_TUNE_CACHE`` or ``~/.cache/ibmi_tune.json``.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch


def cache_path() -> str:
    return os.environ.get("IBMI_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                          "ibmi_tune.json"))


def batch_key(batch) -> str:
    arch = torch.cuda.get_device_properties(batch.As[0].device).gcnArchName.split(":")[0]
    sig = hashlib.sha1(",".join(str(p) for p in sorted(batch.p)).encode()).hexdigest()[:16]
    o = batch.opts
    return f"{arch}/batch/n{batch.n}/b{o.block_rows}/o{o.overlap}/{sig}"


def tuned(batch, reps: int = 2, path: str | None = None) -> dict:
    """Apply cached or freshly autotuned tile configurations to ``batch``."""
    path = path or cache_path()
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    key = batch_key(batch)
    if key in cache:
        cfg = cache[key]["cfg"]
        batch.set_tuning(*cfg)
        return {"key": key, "cfg": tuple(cfg), "ms_per_sweep": cache[key]["ms_per_sweep"],
                "cached": True}
    cfg, ms = batch.autotune(reps)
    cache[key] = {"cfg": list(cfg), "ms_per_sweep": ms}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass
    return {"key": key, "cfg": tuple(cfg), "ms_per_sweep": ms, "cached": False}

"""Autotuner of the launch knobs (jpt_tuning) for a renderer's workload.

The knobs only change how work is spread over the GPU (workgroup counts of
the persistent decode kernels, tile strides of mark and resolve, the
XCD-contiguous tile order, the form of resolve's slot lookups), never what
is computed.  The tuner checks that:
every candidate frame must reproduce the default frame's work list,
counters, decoded texels and framebuffers byte for byte, or it is rejected.

Search: coordinate descent over one knob at a time (the phases a knob
touches are independent), each candidate timed as the median GPU time of
`reps` whole frames with HIP events on the current stream.  Results are
cached in a JSON file keyed by the workload's shape and the device name.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import jpt

CANDIDATES = {
    "flags": [0, jpt.TUNE_XCD_TILES, jpt.TUNE_RESOLVE_PAIRED, jpt.TUNE_RESOLVE_SINGLE,
              jpt.TUNE_XCD_TILES | jpt.TUNE_RESOLVE_PAIRED, jpt.TUNE_XCD_TILES | jpt.TUNE_RESOLVE_SINGLE],
    "mark_groups": [0, 512, 1024, 2048, 4096],
    "resolve_groups": [0, 512, 1024, 2048, 4096],
    "decode_groups": [0, 256, 512, 1024],
    "idct_groups": [0, 128, 256, 512, 1024],
    "wide_bits": [0, 384, 1024, 1 << 30],
}
ORDER = ["flags", "mark_groups", "resolve_groups", "decode_groups", "idct_groups", "wide_bits"]


def default_cache_path() -> str:
    base = os.environ.get("JPT_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "jpt")
    return base if base.endswith(".json") else os.path.join(base, "tune.json")


def workload_key(r: "jpt.Renderer") -> str:
    import torch
    dev = torch.cuda.get_device_name(r.scene.device)
    views = [tuple(v.shape[:2]) for v in r.views.gbufs]
    return json.dumps({"device": dev, "views": views, "filter": r.filter, "n_blocks": r.scene.n_blocks,
                       "n_levels": len(r.host.levels), "idct": r.idct_mode, "policy": r.cache.policy},
                      sort_keys=True)


def to_dict(t: "jpt.TuningC | None") -> dict:
    return {k: int(getattr(t, k)) if t is not None else 0 for k in ORDER}


def from_dict(d: dict) -> "jpt.TuningC":
    t = jpt.TuningC()
    for k in ORDER:
        setattr(t, k, int(d.get(k, 0)))
    return t


def frame_digest(r: "jpt.Renderer") -> str:
    """Everything a frame produced: counters, work list, new blocks' texels, framebuffers."""
    import torch
    torch.cuda.synchronize()
    h = hashlib.sha256()
    ctr = r.frame.counters_host()
    h.update(ctr[:7].tobytes())
    h.update(r.frame.work_items().tobytes())
    n_new = min(int(ctr[jpt.CTR_NEW]), r.cache.n_slots)
    h.update(r.cache.texels[: n_new * 256].cpu().numpy().tobytes())
    for i in range(r.views.n):
        h.update(r.views.frame_host(i).tobytes())
    return h.hexdigest()


def time_frames(r: "jpt.Renderer", reps: int) -> float:
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    r.render()
    ev[0].record()
    for i in range(reps):
        r.render()
        ev[i + 1].record()
    torch.cuda.synchronize()
    return float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]))


def tune(r: "jpt.Renderer", reps: int = 7, cache_path: str | None = None, use_cache: bool = True,
         log=None) -> "jpt.TuningC":
    """Tune r's launch knobs in place (r.tuning) and return them.  Only for a
    frame-local cache (the LRU state would change between candidate frames)."""
    if r.cache.policy != jpt.CACHE_NONE:
        raise ValueError("tune with a frame-local cache (JPT_CACHE_NONE)")
    path = cache_path or default_cache_path()
    key = workload_key(r)
    db = {}
    if use_cache and os.path.exists(path):
        with open(path) as f:
            db = json.load(f)
        if key in db:
            r.tuning = from_dict(db[key]["knobs"])
            return r.tuning
    r.tuning = None
    r.render()
    ref = frame_digest(r)
    best = to_dict(None)
    best_ms = time_frames(r, reps)
    base_ms = best_ms
    trials = []
    for knob in ORDER:
        for v in CANDIDATES[knob]:
            if v == best[knob]:
                continue
            cand = dict(best, **{knob: v})
            r.tuning = from_dict(cand)
            r.render()
            if frame_digest(r) != ref:
                raise RuntimeError("launch knobs %s changed the frame" % cand)
            ms = time_frames(r, reps)
            trials.append((cand, ms))
            if log:
                log("tune %s -> %.4f ms" % (cand, ms))
            if ms < best_ms:
                best, best_ms = cand, ms
    r.tuning = from_dict(best)
    db[key] = {"knobs": best, "ms": best_ms, "default_ms": base_ms, "trials": len(trials)}
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return r.tuning

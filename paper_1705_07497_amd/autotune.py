"""Autotuner for the launch parameters of a RadonOp.

It times the candidate launch shapes of the two products on the operator's own
geometry (HIP events on the current stream) and keeps the fastest:
  * waves per ray bundle in the forward product (2 or 4);
  * waves per 8x8 tile in the adjoint (1, 2 or 4);
  * images sharing each matrix load in a fused multi-image product, for each
    direction (1, 4, 8 or 16), timed at the batch size asked for.
Results are cached as JSON keyed by GPU architecture, geometry (n, angles,
bins, measured-angle mask) and operator kind, at $SPARSECT_AUTOTUNE_CACHE or
~/.cache/sparsect/autotune.json.  Tuning never changes what is computed; the
waves-per-item counts only change how each sum is split (rounding level).
"""
from __future__ import annotations

import hashlib
import json
import os

DEFAULT = {"fwd_waves": 2, "adj_waves": 0, "fwd_rhs": 4, "adj_rhs": 8}


def cache_path() -> str:
    return os.environ.get("SPARSECT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "sparsect", "autotune.json"))


def cache_key(arch: str, n: int, n_angles: int, n_bins: int, measured, kind: int) -> str:
    mh = hashlib.sha1(bytes(bytearray(int(v) != 0 for v in measured))).hexdigest()[:12]
    return f"{arch}|n{n}|a{n_angles}|b{n_bins}|m{mh}|k{kind}"


def _arch(op) -> str:
    import torch
    return getattr(torch.cuda.get_device_properties(op.device), "gcnArchName", "unknown")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def op_key(op) -> str:
    return cache_key(_arch(op), op.n, op.n_angles, op.n_bins, op.measured, op.kind)


def apply_cached(op, path: str | None = None) -> bool:
    """Set the cached tuning for this geometry if there is one."""
    entry = load_cache(path).get(op_key(op))
    if not entry:
        return False
    op.tuning = {k: entry["tuning"].get(k, DEFAULT[k]) for k in DEFAULT}
    return True


def _time(op, fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize(op.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize(op.device)
    return e0.elapsed_time(e1) / reps / 1e3


def autotune(op, batch: int = 16, reps: int = 10, path: str | None = None, save: bool = True) -> dict:
    """Time the candidates, set the best tuning on `op`, cache and return it."""
    import torch
    x1 = torch.randn((1, op.nn), dtype=op.dtype, device=op.device)
    y1 = torch.empty((1, op.rows), dtype=op.dtype, device=op.device)
    o1 = torch.empty_like(x1)
    best = dict(DEFAULT)
    timings = {}

    def trial(field, value, fn):
        op.tuning = {**best, field: value}
        t = _time(op, fn, reps)
        timings[f"{field}={value}"] = t
        return t

    fw = {v: trial("fwd_waves", v, lambda: op.fwd(x1, out=y1)) for v in (2, 4)}
    best["fwd_waves"] = min(fw, key=fw.get)
    op.fwd(x1, out=y1)
    aw = {v: trial("adj_waves", v, lambda: op.adj(y1, out=o1)) for v in (1, 2, 4)}
    best["adj_waves"] = min(aw, key=aw.get)
    if batch > 1:
        xb = torch.randn((batch, op.nn), dtype=op.dtype, device=op.device)
        yb = torch.empty((batch, op.rows), dtype=op.dtype, device=op.device)
        ob = torch.empty_like(xb)
        cands = [c for c in (1, 4, 8, 16) if c <= batch]
        fr = {c: trial("fwd_rhs", c, lambda: op.fwd(xb, out=yb)) for c in cands}
        best["fwd_rhs"] = min(fr, key=fr.get)
        op.fwd(xb, out=yb)
        ar = {c: trial("adj_rhs", c, lambda: op.adj(yb, out=ob)) for c in cands}
        best["adj_rhs"] = min(ar, key=ar.get)
    op.tuning = best
    entry = {"tuning": best, "batch": batch, "timings_s": timings}
    if save:
        store(op_key(op), entry, path)
    return entry

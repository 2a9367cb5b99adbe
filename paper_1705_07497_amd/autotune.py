"""Autotuner of a RadonOp: the forward bundle width (a layout chosen at build
time) and the launch settings (chosen by the library's radon_autotune).

* Launch settings: radon_autotune times, on the operator's own geometry, the
  waves per forward bundle (2, 4), the waves per adjoint tile (1, 2, 4) and,
  at the batch asked for, how many images share each matrix load (1, 4, 8,
  16) in each product, then the forward's gather layout (per image, or from
  a pixel-major copy of each chunk) and band height, and keeps the fastest.  Its cache is a text file with one
  ``sparsect-tune <key> ...`` line per (architecture, geometry, measured
  angles, kind, bundle width, batch).
* Bundle layout: rays per forward bundle (16, 32 or 64) and the consecutive
  measured angles they come from (1, 2 or 4, at least 16 adjacent bins of
  each).  One gather instruction covers a bundle's rays on one image line:
  more adjacent bins, or the same bins of neighbouring angles, which cross
  the line a few pixels apart, make it touch fewer cache lines, at the cost
  of more padded slots where the rays' line ranges differ.
  ``choose_bundle`` builds the operator once per candidate, tunes its launch
  settings and times the normal operator; the winner goes into the same file
  as a ``sparsect-bundle`` line.

The file is $SPARSECT_AUTOTUNE_CACHE, else ~/.cache/sparsect/autotune.txt.
Tuning never changes what is computed; the waves per item, the band height,
the gather layout and the bundle layout only change how each sum is split
(rounding level).
"""
from __future__ import annotations

import ctypes
import hashlib
import os

DEFAULT = {"fwd_waves": 2, "adj_waves": 0, "fwd_rhs": 4, "adj_rhs": 8, "fwd_layout": 0, "fwd_lines": 0,
           "adj_layout": 0, "reserved": 0}
BUNDLES = (16, 32, 64)
# (rays per bundle, angles per bundle) candidates of choose_bundle
LAYOUTS = ((16, 1), (32, 1), (64, 1), (32, 2), (64, 2), (64, 4))
SOURCES = {0: "unchanged", 1: "cache", 2: "timed"}


def cache_path() -> str:
    return os.environ.get("SPARSECT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "sparsect", "autotune.txt"))


def geometry_key(arch: str, n: int, n_angles: int, n_bins: int, measured, kind: int,
                 compact: bool = False, symmetric: bool = False) -> str:
    """Key of a geometry, operator kind and forward storage (compact, stored by
    symmetry; no bundle layout, no batch)."""
    mh = hashlib.sha1(bytes(bytearray(int(v) != 0 for v in measured))).hexdigest()[:12]
    return (f"{arch}|n{n}|a{n_angles}|b{n_bins}|m{mh}|k{kind}" + ("|c" if compact else "")
            + ("|s" if symmetric else ""))


def load_bundles(path: str | None = None) -> dict:
    """geometry key -> (rays, angles) per bundle from the cache file (the last
    line wins; a line without the angle count means one angle)."""
    out = {}
    try:
        with open(path or cache_path()) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) in (3, 4) and parts[0] == "sparsect-bundle" and all(
                        p.isdigit() for p in parts[2:]):
                    lay = (int(parts[2]), int(parts[3]) if len(parts) == 4 else 1)
                    if lay in LAYOUTS:
                        out[parts[1]] = lay
    except OSError:
        pass
    return out


def store_bundle(key: str, bw: int, angles: int = 1, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path, "a") as fh:
        fh.write(f"sparsect-bundle {key} {int(bw)} {int(angles)}\n")


def device_arch(device) -> str:
    import torch
    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "unknown")
    return name.split(":")[0]


def cached_bundle(n, n_angles, n_bins, measured, kind, device, path=None, compact=False,
                  symmetric=False) -> tuple | None:
    """(rays, angles) per bundle cached for this geometry, or None."""
    key = geometry_key(device_arch(device), n, n_angles, n_bins, measured, kind, compact, symmetric)
    return load_bundles(path).get(key)


def _path_arg(path):
    return None if path is None else os.fsencode(path)


def apply_cached(op, batch: int = 1, path: str | None = None) -> bool:
    """Apply the cached launch settings of this operator and batch, if any."""
    from . import _check, _vp, lib
    src = ctypes.c_int32(0)
    p = path or cache_path()
    if not os.path.exists(p):
        return False
    _check(lib().radon_autotune(op._h, int(batch), None, 0, _path_arg(p), 1, op._stream(),
                                ctypes.byref(src)))
    return src.value == 1


def autotune(op, batch: int = 16, path: str | None = None, save: bool = True) -> dict:
    """Time the launch candidates with radon_autotune and set the best on `op`
    (or apply a cached entry); returns {"tuning", "batch", "source"}."""
    import torch

    from . import WS_TUNE, _check, _vp, lib
    nbytes = lib().radon_workspace_bytes(op._h, WS_TUNE, int(batch))
    if nbytes < 0:
        _check(int(nbytes))
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=op.device)
    src = ctypes.c_int32(0)
    p = (path or cache_path()) if save else None
    if p is not None:
        os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    torch.cuda.synchronize(op.device)
    _check(lib().radon_autotune(op._h, int(batch), _vp(ws.data_ptr()), int(nbytes), _path_arg(p), 0,
                                op._stream(), ctypes.byref(src)))
    return {"tuning": op.tuning, "batch": int(batch), "source": SOURCES[src.value]}


def choose_bundle(n, n_angles, n_bins, measured=None, dtype=None, vec_dtype=None, device=None,
                  batch: int = 1, reps: int = 50, rounds: int = 3, path: str | None = None,
                  save: bool = True, layouts=LAYOUTS, compact: bool = False, symmetric: bool = False) -> dict:
    """Build the operator (forward storage compact and/or by symmetry, as
    asked) with each bundle
    layout (rays, angles), tune its launch settings, time its normal operator
    at `batch` (the best of `rounds` runs of `reps` calls, so that a layout is
    not ranked on one noisy run) and return the fastest {"bundle": rays,
    "angles": angles} (stored in the cache when save)."""
    import numpy as np
    import torch

    from . import RadonOp
    times = {}
    kind = None
    for bw, ang in layouts:
        op = RadonOp(n, n_angles, n_bins, measured, dtype=dtype, device=device, vec_dtype=vec_dtype,
                     tuning="default", bundle=bw, bundle_angles=ang, compact=compact, symmetric=symmetric)
        kind, dev = op.kind, op.device
        autotune(op, batch=batch, save=False)
        x = torch.randn((batch, op.nn), dtype=op.dtype, device=op.device)
        out = torch.empty_like(x)
        op.normal(x, 1.0, 1.0, out=out)
        torch.cuda.synchronize(op.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best_s = None
        for _ in range(rounds):
            e0.record()
            for _ in range(reps):
                op.normal(x, 1.0, 1.0, out=out)
            e1.record()
            torch.cuda.synchronize(op.device)
            s = e0.elapsed_time(e1) / reps / 1e3
            best_s = s if best_s is None else min(best_s, s)
        times[(bw, ang)] = best_s
        del op, x, out
    best = min(times, key=times.get)
    if save:
        m = np.ones(n_angles, np.uint8) if measured is None else measured
        store_bundle(geometry_key(device_arch(dev), n, n_angles, n_bins, m, kind, compact, symmetric), best[0],
                     best[1], path)
    return {"bundle": best[0], "angles": best[1],
            "normal_s": {f"{bw}x{ang}": t for (bw, ang), t in times.items()}}

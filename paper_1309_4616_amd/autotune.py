"""Tile-shape autotuner with a JSON cache.

`tune(op, dtype)` asks the library (expi_op_autotune) to time the fused
Newton product under every candidate tile setting on this operator, and,
where pair sweeps apply, a pair sweep against two single products; it keeps
the fastest on the operator and records it in a JSON cache keyed by operator
shape, boundary handling, coefficient kind, storage dtype and GPU, so later
processes reuse the choice without timing again (`load(op, dtype)`).

The cache lives at $EXPI_TUNE_CACHE, else ~/.cache/expi/tiles.json.
"""
from __future__ import annotations

import ctypes
import json
import os

from ._binding import check, lib


def cache_path() -> str:
    return os.environ.get("EXPI_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "expi", "tiles.json"))


def device_tag(device) -> str:
    import torch
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "") or ""
    return f"{arch.split(':')[0]}-{props.multi_processor_count}cu"


def op_key(op, dtype: str) -> str:
    """Cache key: what determines the best tile setting."""
    from . import CsrComplexOp, CsrOp, StencilOp
    if isinstance(op, StencilOp):
        kind = {0: "const", 1: "separable", 2: "field", 3: "dlap"}[op.coef_kind]
        body = f"stencil{len(op.shape)}d-{'x'.join(map(str, op.shape))}-{op.bc}-{kind}"
    elif isinstance(op, CsrOp):
        body = f"csr-n{op.size}-nnz{op.nnz}"
    elif isinstance(op, CsrComplexOp):
        body = f"csr-complex-n{op.size}-nnz{op.nnz}"
    else:
        raise TypeError("not an operator")
    return f"{body}-{dtype}-{device_tag(op.device)}"


def _read(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _write(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(op, dtype: str = "f64", path: str | None = None) -> bool:
    """Apply a cached setting if there is one; returns whether it did."""
    path = path or cache_path()
    entry = _read(path).get(op_key(op, dtype))
    if not entry:
        return False
    _apply(op, entry)
    return True


def _apply(op, entry: dict) -> None:
    op.set_tiles(*entry["tiles"])
    if "pairs" in entry and hasattr(op, "set_pairs"):
        rows = entry.get("pair_rows")
        op.set_pairs(int(rows) if (entry["pairs"] and rows) else bool(entry["pairs"]))


def tune(op, dtype: str = "f64", reps: int = 10, path: str | None = None,
         use_cache: bool = True, stream=None) -> dict:
    """Time every candidate, keep the fastest on `op`, record it; returns
    {'tiles': (vec, waves, march), 'us': best time, 'pairs': whether pair
    sweeps are kept (None where they do not apply), 'candidates': [...]}
    (the pair sweep is the candidate (0, 0, 2), its time per launch of two
    products; a 2D pair sweep is timed at several tile heights, (0, rows, 2),
    and 'pair_rows' records the one kept)."""
    import torch
    from . import _dtype_code, _stream_ptr
    path = path or cache_path()
    key = op_key(op, dtype)
    data = _read(path) if use_cache else {}
    if use_cache and key in data:
        _apply(op, data[key])
        return data[key]
    code = _dtype_code(dtype)
    ws = op.workspace(code)
    maxc = 64
    cand = (ctypes.c_int * (3 * maxc))()
    us = (ctypes.c_float * maxc)()
    nc = ctypes.c_int()
    check(lib().expi_op_autotune(op.handle, code, int(reps), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream_ptr(stream, op.device), cand, us, maxc,
                                 ctypes.byref(nc)))
    rows = [((cand[3 * i], cand[3 * i + 1], cand[3 * i + 2]), float(us[i]))
            for i in range(min(nc.value, maxc))]
    best = op.tiles()
    singles = [t for c, t in rows if c[0] != 0]
    paired = any(c[0] == 0 for c, _ in rows)
    entry = {"tiles": list(best), "us": min(singles) if singles else None,
             "pairs": (op.pairs() if paired else None),
             "candidates": [[list(c), t] for c, t in rows]}
    if paired and op.pair_setting() > 1:
        entry["pair_rows"] = op.pair_setting()   # the 2D pair sweep's tile height
    if use_cache:
        data = _read(path)
        data[key] = entry
        _write(path, data)
    torch.cuda.synchronize(op.device)
    return entry


def batch_key(batch) -> str:
    """Cache key of a batch: sizes, time steps, boundary, dtype and GPU."""
    import hashlib
    import numpy as np
    h = hashlib.sha1()
    for a in (batch._nx, batch._ny, batch._tau):
        h.update(np.ascontiguousarray(a).tobytes())
    return f"batch{batch.count}-{h.hexdigest()[:16]}-{batch.bc}-{batch.dtype}-{device_tag(batch.device)}"


def tune_batch(batch, v, y, reps: int = 1, path: str | None = None, use_cache: bool = True,
               stream=None) -> dict:
    """Solve the batch under every candidate tile setting (expi_batch_autotune),
    keep the fastest (prepared for the batch's workspace), record it; returns
    {'tiles': (waves, march), 'ms': best time, 'candidates': [...]}.  y is
    overwritten."""
    from . import _stream_ptr
    path = path or cache_path()
    key = batch_key(batch)
    data = _read(path) if use_cache else {}
    if use_cache and key in data:
        batch.set_tiles(*data[key]["tiles"])
        batch.prepare(stream)
        return data[key]
    ws = batch.workspace()
    maxc = 32
    cand = (ctypes.c_int * (2 * maxc))()
    ms = (ctypes.c_float * maxc)()
    nc = ctypes.c_int()
    check(lib().expi_batch_autotune(batch.handle, ctypes.c_void_p(v.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                    ws.numel(), int(reps), _stream_ptr(stream, batch.device), cand, ms,
                                    maxc, ctypes.byref(nc)))
    rows = [((cand[2 * i], cand[2 * i + 1]), float(ms[i])) for i in range(min(nc.value, maxc))]
    entry = {"tiles": list(batch.tiles()), "ms": min(t for _, t in rows) if rows else None,
             "candidates": [[list(c), t] for c, t in rows]}
    if use_cache:
        data = _read(path)
        data[key] = entry
        _write(path, data)
    return entry

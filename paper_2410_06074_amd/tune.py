"""Autotuning of the launch mapping (chunk lengths, workgroup size, persistent
grid) with an on-disk cache.  The search itself runs in the library
(smnn_autotune); this module marshals the arguments and keeps the cache.

Cache: JSON at $SMNN_TUNE_CACHE (default ~/.cache/smnn/autotune.json), keyed
by device architecture, block size, mode, and power-of-two buckets of the
instance count and mean sequence length (plus a ragged flag).
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np
import torch

from . import _lib


def _cache_path():
    return os.environ.get("SMNN_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "smnn", "autotune.json"))


def _key(order, mode, n_inst, steps, device):
    steps = np.atleast_1d(np.asarray(steps, dtype=np.int64))
    ragged = steps.size > 1 and not np.all(steps == steps[0])
    mean_t = float(steps.mean())
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    return "%s/R%d/%s/N%d/T%d/%s" % (arch, order, mode, int(math.log2(max(1, n_inst))),
                                     int(math.log2(max(1.0, mean_t))), "ragged" if ragged else "uniform")


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def autotune(order, n_init, n_inst, steps, mode, c, b, h, u0, w, gy, iters=3, use_cache=True, init_points=1):
    """Best {chunk, chunk_upper, block, max_blocks, ms} for this problem; the
    candidates timed are returned under 'candidates' when a search ran."""
    key = _key(order, mode, n_inst, steps, c.device)
    if use_cache:
        hit = _load().get(key)
        if hit:
            return dict(hit, cached=True)
    L = _lib.lib()
    d = _lib.PlanDesc()
    d.order, d.n_init, d.n_inst = int(order), int(n_init), int(n_inst)
    steps_arr = None
    if np.isscalar(steps):
        d.steps, d.steps_uniform = None, int(steps)
    else:
        steps_arr = np.ascontiguousarray(steps, dtype=np.int64)
        d.steps = steps_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.mode, d.refine_steps = _lib.MODES[mode], -1
    d.init_points = int(init_points)
    best = _lib.TuneResult()
    cap = 64
    all_ = (_lib.TuneResult * cap)()
    n = ctypes.c_int32(0)
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
    st = torch.cuda.current_stream(c.device).cuda_stream
    _lib.check(L.smnn_autotune(ctypes.byref(d), p(c), p(b), p(h), p(u0), p(w), p(gy), int(iters),
                               ctypes.c_void_p(st), ctypes.byref(best), all_, cap, ctypes.byref(n)),
               "smnn_autotune")
    res = {"chunk": best.chunk, "chunk_upper": best.chunk_upper, "block": best.block,
           "max_blocks": best.max_blocks, "ms": best.ms}
    if use_cache:
        cache = _load()
        cache[key] = res
        _store(cache)
    res["candidates"] = [{"chunk": r.chunk, "chunk_upper": r.chunk_upper, "block": r.block,
                          "max_blocks": r.max_blocks, "ms": r.ms} for r in all_[:n.value]]
    return res

"""Tile-shape autotuner: picks the stage kernels' workgroup size (256 or 512
threads, i.e. how many elements share a workgroup) per (degree, precision) by
timing a few RK steps of a droplet workload on the device.  Results do not
depend on the choice; only speed does.  The table is kept in a JSON file."""
from __future__ import annotations

import json
import os

from . import workloads as wl
from .nskr import NskrError, init_workload, solver_for

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "nskr_tiles.json")


def _key(N, precision):
    return f"N{N}_{precision}"


def tune_one(N, precision, n=(8, 8, 8), steps=3, candidates=(256, 512)):
    import torch
    w = wl.Workload(name=f"tune_N{N}", N=N, n=n, steps=steps)
    s = solver_for(w, precision)
    U = init_workload(s, w)
    R = s.new_state()
    dt = s.dt(U)
    stream = torch.cuda.current_stream()
    times = {}
    for bs in candidates:
        try:
            s.set_block(bs)
        except NskrError:
            continue
        s.rk_steps(U, R, dt, 1, stream)  # warm-up
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.rk_steps(U, R, dt, steps, stream)
        b.record(stream)
        torch.cuda.synchronize()
        times[bs] = a.elapsed_time(b) / steps
    best = min(times, key=times.get)
    return best, times


def load(path=DEFAULT_CACHE):
    if not path:
        return {}
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(pairs, path=DEFAULT_CACHE, n=(8, 8, 8), steps=3, force=False):
    """Tile table for the (N, precision) pairs, tuning the ones not cached."""
    table = {} if force else load(path)
    changed = False
    for N, prec in pairs:
        k = _key(N, prec)
        if k not in table:
            best, times = tune_one(N, prec, n, steps)
            table[k] = {"threads": best, "ms_per_step": times}
            changed = True
    if changed and path:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(table, f, indent=1)
        except OSError:
            pass
    return table


def threads_for(table, N, precision, default=256):
    return int(table.get(_key(N, precision), {}).get("threads", default))

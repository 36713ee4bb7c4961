"""Tile-shape autotuner: picks the stage kernels' workgroup size per (degree,
precision), i.e. how many elements share a workgroup and how tightly they fill
its waves, among the sizes the library builds for that degree (256, 512 and a
tight size: N = 2 192, N = 3 and 4 128, N = 5 448).  Each candidate runs a few
RK steps of a droplet workload at the mesh sizes the request stream draws,
from the same initial state; the fastest total wins.  The tuner also records
whether every candidate ended in bitwise the same state (an element's
arithmetic does not depend on its tile).  The table can be kept in a JSON
file."""
from __future__ import annotations

import json
import os

from . import workloads as wl
from .nskr import NskrError, init_workload, solver_for

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "nskr_tiles.json")

# the serving stream's smallest-but-one and largest element grids
DEFAULT_SIZES = ((8, 8, 8), (16, 16, 16))


def block_sizes(N):
    """Workgroup sizes the library builds for degree N."""
    tight = {2: 192, 3: 128, 4: 128, 5: 448}[N]
    return tuple(sorted({256, 512, tight}))


def _key(N, precision):
    return f"N{N}_{precision}"


def tune_one(N, precision, sizes=DEFAULT_SIZES, steps=3, candidates=None):
    """Time `steps` RK steps per candidate workgroup size on each mesh size;
    returns (best, {size: total ms per step}, bitwise_equal)."""
    import torch
    candidates = candidates or block_sizes(N)
    times = {}
    equal = True
    stream = torch.cuda.current_stream()
    for n in sizes:
        w = wl.Workload(name=f"tune_N{N}_{n[0]}x{n[1]}x{n[2]}", N=N, n=n, steps=steps)
        s = solver_for(w, precision)
        U0 = init_workload(s, w)
        dt = s.dt(U0)
        ref = None
        for bs in candidates:
            try:
                s.set_block(bs)
            except NskrError:
                continue
            U = U0.clone()
            R = s.new_state()
            s.rk_steps(U, R, dt, 1, stream)  # warm-up
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            s.rk_steps(U, R, dt, steps, stream)
            b.record(stream)
            torch.cuda.synchronize()
            times[bs] = times.get(bs, 0.0) + a.elapsed_time(b) / steps
            if ref is None:
                ref = U
            elif not torch.equal(ref, U):
                equal = False
        del s
    best = min(times, key=times.get)
    return best, times, equal


def load(path=DEFAULT_CACHE):
    if not path:
        return {}
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(pairs, path=DEFAULT_CACHE, sizes=DEFAULT_SIZES, steps=3, force=False):
    """Tile table for the (N, precision) pairs, tuning the ones not cached."""
    table = {} if force else load(path)
    changed = False
    for N, prec in pairs:
        k = _key(N, prec)
        if k not in table:
            best, times, equal = tune_one(N, prec, sizes, steps)
            table[k] = {"threads": best, "ms_per_step": times, "bitwise_equal": equal,
                        "sizes": [list(n) for n in sizes]}
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

"""Launch-shape autotuner for the dynamics kernels.

For one operation on one model/batch, times every candidate launch shape
(threads per workgroup, workgroup cap -- a cap below the work makes the launch
persistent), the kernel variant (one wavefront per 64 states, the role split
across wavefronts, or the segmented scans with 1 to 32 lanes, i.e. segments,
per chain -- at most 16 for forward dynamics) and, for one chain per state,
the chain order (natural, or longest first), with HIP events, and keeps the
fastest. Results are recorded in a
JSON table keyed by (operation, precision, model kind, links, states).
``apply`` installs the winner into libpdyn's own tuning table
(pdyn_load_tuning), which every later call of that operation on a model of
that kind and size consults when its batch leaves the launch fields at 0; the
chain order is a property of the model and is set on it.
"""

from __future__ import annotations

import itertools
import json
import os

import torch

from . import api

BLOCKS = (64, 128, 256)
CAPS = (0, 256, 512, 1024)
SEGMENTS = (1, 2, 4, 8, 16, 32)  # lanes per chain of the segmented-scan variant (4)


def key_of(op: int, model: api.Model, n_states: int) -> str:
    kind = "shared" if model.n_chains == 1 else "per_state"
    prec = "f64" if model.dtype == torch.float64 else "f32"
    return f"{op}:{prec}:{kind}:{model.n_links_max}:{n_states}"


def _time(fn, reps=20, warmup=3):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(op: int, model: api.Model, call, n_states: int, reps: int = 20):
    """Time `call()` (which issues `op` on `model`) for every candidate; return (best, timings)."""
    orders = (True, False) if model.n_chains > 1 else (True,)
    timings = []
    saved = api._launch_override.get(op)
    saved_order = model.use_order
    variants = (1, 2, 4) if op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD) else (1,)
    max_segments = 64 if op == api.OP_RNEA_ID else 16  # forward dynamics: at most 16 lanes per chain
    try:
        for bt, cap, use_order in itertools.product(BLOCKS, CAPS, orders):
            if cap and cap * bt >= n_states:
                continue  # not persistent: same as uncapped
            api.set_launch(op, bt, cap, 1)
            model.use_order = use_order
            timings.append({"block_threads": bt, "max_blocks": cap, "order": use_order, "variant": 1,
                            "ms": _time(call, reps)})
        if 2 in variants:
            for use_order in orders:
                api.set_launch(op, 0, 0, 2)
                model.use_order = use_order
                timings.append({"block_threads": 0, "max_blocks": 0, "order": use_order, "variant": 2,
                                "ms": _time(call, reps)})
        if 4 in variants:  # segmented scans: P lanes per chain, each folding about n / P links
            for P, use_order in itertools.product(SEGMENTS, orders):
                if P > max_segments or (P > 1 and model.n_links_max < 2 * P):
                    continue  # segments of fewer than two links
                api.set_launch(op, 0, 0, 4, P)
                model.use_order = use_order
                timings.append({"block_threads": 0, "max_blocks": 0, "order": use_order, "variant": 4,
                                "segments": P, "ms": _time(call, reps)})
    finally:
        model.use_order = saved_order
        if saved is None:
            api._launch_override.pop(op, None)
        else:
            api._launch_override[op] = saved
    best = min(timings, key=lambda r: r["ms"])
    return best, timings


def record(path: str, op: int, model: api.Model, n_states: int, best: dict):
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    table[key_of(op, model, n_states)] = best
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


# entries installed in the library, keyed like the JSON table
_installed = {}


def library_entry(op: int, model: api.Model, n_states: int, best: dict) -> dict:
    return {"op": int(op), "scalar": model.scalar_bytes, "shared": int(model.n_chains == 1),
            "n_max": int(model.n_links_max), "n_states": int(n_states), "block": int(best["block_threads"]),
            "max_blocks": int(best["max_blocks"]), "variant": int(best.get("variant", 0)),
            "segments": int(best.get("segments", 0))}


def install(entries) -> None:
    """Load tuning entries (dicts of library_entry's form) into libpdyn (pdyn_load_tuning)."""
    text = json.dumps({"entries": list(entries)}).encode()
    api._check(api.lib().pdyn_load_tuning(text), "pdyn_load_tuning")


def apply(best: dict, op: int, model: api.Model, n_states: int):
    """Make `best` the launch of `op` for models like `model` with about `n_states` states."""
    api._launch_override.pop(op, None)  # an explicit override would hide the table
    _installed[key_of(op, model, n_states)] = library_entry(op, model, n_states, best)
    install(_installed.values())
    model.use_order = bool(best.get("order", True))


def clear():
    _installed.clear()
    install(())

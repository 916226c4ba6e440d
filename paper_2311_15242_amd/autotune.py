"""Launch-shape autotuner of the solver.

The shapes it sweeps never change the results (each node's arithmetic and the
red-black order of the implicit solve are the same for every shape; the FP64
reductions keep a fixed shape):

* ``rows``: the step's node kernels (collision, macroscopic fields, geometry,
  FD right-hand sides, forces) run workgroups of 64 x rows nodes, a wavefront
  per row of 64 consecutive x; rows = 1, 2 or 4 trades LDS halo overhead of
  the staged kernels (66 x (rows + 2) cells per 64 x rows nodes) against
  workgroup count and occupancy;
* ``sor_wg_per_cu``: the persistent grid of the SOR half-sweeps, in workgroups
  of 256 per compute unit;
* ``sor_narrow``: the grid of sweeps past the third, which mostly find both
  systems converged and return (in a batch: which run over the instances
  still converging).

Each candidate is timed over whole steps with HIP events on the solver's
stream (median of several timed regions); the fastest is stored per workload
key (lattice, storage, size class, batch size) in ``tuning.json`` next to this
module, which ``Solver`` and ``Batch`` read at creation.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

from . import lbfd

ROWS = (1, 2, 4)
SOR_WG_PER_CU = (2, 4, 8, 16)
SOR_NARROW = (64, 256, 1024)


def _time(obj, steps: int, regions: int) -> float:
    """Median milliseconds per step over `regions` timed regions of `steps` steps."""
    import torch

    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(regions):
        torch.cuda.synchronize()
        a.record()
        obj.step(steps)
        b.record()
        torch.cuda.synchronize()
        runs.append(a.elapsed_time(b) / steps)
    return float(np.median(runs))


def tune_solver(params: dict, init: dict, steps: int = 20, warmup: int = 6, regions: int = 3) -> dict:
    """Sweep rows x SOR grid x narrow grid on one solver of the workload."""
    s = lbfd.Solver(params, tuning=None).init_fields(init).step(warmup)
    table = []
    for rows, wg, nar in itertools.product(ROWS, SOR_WG_PER_CU, SOR_NARROW):
        t = dict(rows=rows, sor_wg_per_cu=wg, sor_narrow=nar)
        s.set_tuning(t).step(4)            # captures the graphs of this shape
        table.append((_time(s, steps, regions), t))
    s.set_tuning(lbfd.DEFAULT_TUNING).step(4)
    default_ms = _time(s, steps, regions)
    if s.observables()["status"] != 0:
        raise RuntimeError("solver error while tuning")
    s.close()
    best_ms, best = min(table, key=lambda r: r[0])
    return dict(key=lbfd.tuning_key(params), tuning=best, ms_per_step=round(best_ms, 4),
                default_ms_per_step=round(default_ms, 4),
                candidates=[dict(t, ms_per_step=round(ms, 4)) for ms, t in table])


def tune_batch(params_list, inits, steps: int = 10, warmup: int = 4, regions: int = 3) -> dict:
    """Sweep rows x narrow grid on a batch (its first three SOR sweeps launch one
    workgroup per tile of every instance; the narrow grid runs the later sweeps
    over the instances still converging)."""
    b = lbfd.Batch(params_list, tuning=None)
    for m, q in zip(b.members, inits):
        m.init_fields(q)
    b.step(warmup)
    table = []
    for rows, nar in itertools.product(ROWS, SOR_NARROW):
        t = dict(lbfd.DEFAULT_TUNING, rows=rows, sor_narrow=nar)
        b.set_tuning(t).step(4)
        table.append((_time(b, steps, regions), t))
    b.set_tuning(lbfd.DEFAULT_TUNING).step(4)
    default_ms = _time(b, steps, regions)
    key = b.key
    b.close()
    best_ms, best = min(table, key=lambda r: r[0])
    return dict(key=key, tuning=best, ms_per_step=round(best_ms, 4), default_ms_per_step=round(default_ms, 4),
                candidates=[dict(t, ms_per_step=round(ms, 4)) for ms, t in table])


def write(results, path: str = lbfd.TUNING_FILE, device: str = "") -> dict:
    """Merge tuned entries into the table at `path`."""
    table = dict(entries={})
    if os.path.exists(path):
        with open(path) as fh:
            table = json.load(fh)
    for r in results:
        table["entries"][r["key"]] = dict(tuning=r["tuning"], ms_per_step=r["ms_per_step"],
                                          default_ms_per_step=r["default_ms_per_step"], device=device,
                                          candidates=r["candidates"])
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
        fh.write("\n")
    return table

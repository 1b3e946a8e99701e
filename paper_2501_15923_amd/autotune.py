"""Autotuner for the launch configuration of the stage kernels.

Single runs: tiles (lanes along r: 64 or 32) x phi planes per block, timed on
a throwaway solver of the same grid.  Ensembles: per-run planes policy and
persistent vs batched execution, timed on a throwaway ensemble of the same
grids.  Every candidate gives bit-identical results (the tile code is the
same), so tuning only changes speed.  Results are cached in a JSON file keyed
by device, precision and grid shapes.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import synth

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "icarus_mi355x", "tune.json")


def _device_name():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName


def _load(path):
    try:
        return json.load(open(path))
    except Exception:
        return {}


def _store(path, key, val):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    db = _load(path)
    db[key] = val
    tmp = path + ".tmp"
    json.dump(db, open(tmp, "w"), indent=1)
    os.replace(tmp, path)


def _uniform_inputs(g):
    """A static wind map for timing (the kernels' cost does not depend on it)."""
    return np.zeros(1), synth.static_map(g, 0)[None]


def _time(fn, reps):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    fn(reps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def solver_candidates(g, limiter=0):
    out = []
    # the WENO5 face-once tile exists in the 64-lane shape only; its 58-cell
    # rows make 11 tiles along r at n_r = 600, so chunks of 20-40 planes give
    # grids of about one or two rounds of the resident blocks
    plist = (2, 4, 5, 6, 8, 10, 12, 15, 16)
    if limiter == 2:
        plist += (20, 24, 30, 40)
    for tr in ((64,) if limiter == 2 else (64, 32)):
        for planes in plist:
            if planes <= g.np_:
                out.append((tr, planes))
    return out


def tune_solver(g, precision=64, flux=0, limiter=0, steps=32, cache=DEFAULT_CACHE):
    """Best (tile_r, planes) for one grid; cached."""
    key = f"solver|{_device_name()}|{precision}|{flux}{limiter}|{g.nr}x{g.nt}x{g.np_}"
    db = _load(cache) if cache else {}
    if key in db:
        return tuple(db[key]["best"])
    from .solver import Solver
    s = Solver(g, precision=precision, flux=flux, limiter=limiter)
    s.set_maps(*_uniform_inputs(g))
    s.init_radial()
    s.step(4 * steps)  # clocks up before the first candidate
    timings = {}
    for tr, planes in solver_candidates(g, limiter):
        s.set_launch(2, tr, planes, 1)
        s.step(16)
        timings[f"{tr}x{planes}"] = _time(s.step, steps)
    s.close()
    best = min(timings, key=timings.get)
    res = tuple(int(x) for x in best.split("x"))
    if cache:
        _store(cache, key, {"best": list(res), "ms_per_step": timings})
    return res


def _planes_policy(policy, g):
    if policy == "p4":
        return min(4, g.np_)
    if policy == "p8":
        return min(8, g.np_)
    if policy == "p12":
        return min(12, g.np_)
    # "even": split phi into equal chunks close to 8 planes
    chunks = max(1, round(g.np_ / 8))
    return -(-g.np_ // chunks)


def ensemble_candidates():
    return [(mode, pol) for mode in (1, 0) for pol in ("p4", "p8", "even", "p12")]


def tune_ensemble(grids, precision=64, flux=0, limiter=0, steps=2, cache=DEFAULT_CACHE):
    """Best (persistent, planes per run) for an ensemble of grids; cached."""
    shapes = ",".join(f"{g.nr}x{g.nt}x{g.np_}" for g in grids)
    digest = hashlib.sha1(shapes.encode()).hexdigest()[:16]
    key = f"ensemble|{_device_name()}|{precision}|{flux}{limiter}|{len(grids)}|{digest}"
    db = _load(cache) if cache else {}
    if key in db:
        v = db[key]["best"]
        return v["persistent"], v["planes"]
    from .ensemble import Ensemble
    e = Ensemble(grids, precision=precision, flux=flux, limiter=limiter)
    for g, run in zip(grids, e.runs):
        run.set_maps(*_uniform_inputs(g))
        run.init_radial()
    timings, choices = {}, {}
    for mode, pol in ensemble_candidates():
        planes = [_planes_policy(pol, g) for g in grids]
        for r, p in enumerate(planes):
            e.set_planes(r, p)
        e.set_mode(mode, 0, 1)
        e.step(1)
        name = f"{'persistent' if mode else 'batched'}-{pol}"
        timings[name] = _time(e.step, steps)
        choices[name] = {"persistent": mode, "planes": planes}
    e.close()
    best = min(timings, key=timings.get)
    if cache:
        _store(cache, key, {"best": choices[best], "ms_per_step": timings, "choice": best})
    return choices[best]["persistent"], choices[best]["planes"]

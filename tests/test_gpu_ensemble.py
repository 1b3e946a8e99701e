"""Batched ensemble on the GPU: every run is bit-identical to the same run
stepped alone through icr_step, in the persistent (one launch, device-wide
barriers) and the batched (one launch per phase) modes, also with the HLLD
flux, with the WENO5 reconstruction and with the passive CME tracer (state
and tracer bitwise), and one run is checked against the oracle."""
import sys

import numpy as np
import pytest

import parity
from paper_2501_15923_amd import synth

pytestmark = pytest.mark.gpu

GRIDS = [(70, 12, 20), (40, 8, 16), (64, 16, 32), (33, 10, 12), (150, 30, 9)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    import oracle
    from paper_2501_15923_amd import _abi, ensemble, solver
    _abi.lib()
    return oracle, solver, ensemble


def inputs(q, g):
    times, maps = synth.dynamic_maps(g, 500 + q, cadence=2400.0)
    earth = synth.orbit_table(synth.DAY, 600.0, synth.AU)
    cme = synth.cone_cme(600 + q, earth, t_start=300.0 * q, duration=3 * 3600.0,
                         half_width=(20 + 5 * q) * synth.DEG)
    return times, maps, cme


def build_ensemble(mods, planes, **phys):
    _, _, ensemble = mods
    grids = [synth.Grid(*s) for s in GRIDS]
    e = ensemble.Ensemble(grids, **phys)
    for q, (g, run) in enumerate(zip(grids, e.runs)):
        times, maps, cme = inputs(q, g)
        run.set_maps(times, maps)
        run.set_cmes(cme[None])
        run.init_radial()
        if planes:
            e.set_planes(q, min(planes[q % len(planes)], g.np_))
    return e, grids


@pytest.mark.parametrize("persistent,graphs", [(1, 1), (0, 1), (1, 0)])
def test_ensemble_runs_bitwise_equal_single_runs(mods, persistent, graphs):
    _, solver, _ = mods
    steps = 19  # two graph chunks of 8 plus an odd remainder
    e, grids = build_ensemble(mods, planes=[8, 5, 3])
    e.set_mode(persistent, 0, graphs)
    say(f"ensemble of {len(grids)} runs, persistent={persistent} graphs={graphs}")
    info = e.step(steps)
    assert all(i["steps"] == steps and i["status"] == 0 for i in info)
    for q, g in enumerate(grids):
        s = solver.Solver(g)
        times, maps, cme = inputs(q, g)
        s.set_maps(times, maps)
        s.set_cmes(cme[None])
        s.init_radial()
        s.step(steps)
        a = e.runs[q].get_state(kind=1)
        b = s.get_state(kind=1)
        assert np.array_equal(a, b), (q, parity.max_rel(a, b))
        assert e.runs[q].clock()["t"] == s.clock()["t"]
    e.close()


def test_ensemble_run_matches_oracle(mods):
    oracle = mods[0]
    e, grids = build_ensemble(mods, planes=None)
    e.step(12)
    q = 3
    g = grids[q]
    times, maps, cme = inputs(q, g)
    o = oracle.Oracle(g.nr, g.nt, g.np_)
    o.set_maps(times, maps)
    o.set_cmes(cme[None])
    o.init_radial()
    o.step(12)
    parity.assert_parity(e.runs[q].get_state(kind=1), o.get_state(kind=oracle.CONS_CODE),
                         what="ensemble run vs oracle")
    e.close()


def test_ensemble_grid_size_and_repeat_calls(mods):
    e, grids = build_ensemble(mods, planes=[4])
    e.set_mode(1, 64, 1)
    e.step(8)
    e.step(3)
    ref = [r.get_state(kind=1) for r in e.runs]
    e.close()
    e2, _ = build_ensemble(mods, planes=[4])
    e2.set_mode(0, 0, 0)
    e2.step(11)
    for a, r in zip(ref, e2.runs):
        assert np.array_equal(a, r.get_state(kind=1))
    e2.close()


@pytest.mark.parametrize("phys,persistent", [
    (dict(tracer=True), 1), (dict(tracer=True), 0), (dict(flux=2), 1),
    (dict(flux=2, limiter=1, tracer=True), 1), (dict(tracer=True, precision=32), 0),
    (dict(limiter=2), 1), (dict(limiter=2), 0), (dict(limiter=2, flux=2), 1),
    (dict(limiter=2, precision=32), 0)])
def test_ensemble_with_tracer_and_hlld_bitwise_equal_single_runs(mods, phys, persistent):
    """Every run carries a cone CME; with the tracer on, tau of every run is
    bit-identical to the single run's as well.  With WENO5 (limiter 2) the
    runs use the WENO5 face-once tile, as a single run does."""
    _, solver, _ = mods
    steps = 19
    e, grids = build_ensemble(mods, planes=[8, 5, 3], **phys)
    e.set_mode(persistent, 0, 1)
    say(f"ensemble {phys}, persistent={persistent}")
    info = e.step(steps)
    assert all(i["steps"] == steps and i["status"] == 0 for i in info)
    n_tau = 0
    for q, g in enumerate(grids):
        s = solver.Solver(g, **phys)
        times, maps, cme = inputs(q, g)
        s.set_maps(times, maps)
        s.set_cmes(cme[None])
        s.init_radial()
        s.step(steps)
        a, b = e.runs[q].get_state(kind=1), s.get_state(kind=1)
        assert np.array_equal(a, b), (q, parity.max_rel(a, b))
        if phys.get("tracer"):
            ta, tb = e.runs[q].get_tracer(), s.get_tracer()
            assert np.array_equal(ta, tb), (q, float(np.max(np.abs(ta - tb))))
            n_tau += int((ta > 1e-3).sum())
        s.close()
    if phys.get("tracer"):
        assert n_tau > 0  # CME material entered
    e.close()

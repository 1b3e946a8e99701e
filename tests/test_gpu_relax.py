"""GPU checks of the relaxation diagnostics and of the ensemble stop time.

  - icr_sample_shell against linear interpolation in r of the oracle's
    primitive state after the same steps (FP64 bar 1e-9);
  - an ensemble stepped towards a stop time ends exactly on it, bitwise equal
    to single runs stepped towards the same time;
  - the plain relaxation driver reports a consistent convergence record.
"""
import sys

import numpy as np
import pytest

import parity
from paper_2501_15923_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import oracle
    from paper_2501_15923_amd import _abi, relax, solver
    _abi.lib()
    return oracle, solver, relax


def shell_from_state(prim, edges_r, r):
    """prim [8][np][nt][nr] SI -> rho, v_r [2][nt][np] linear in r."""
    rc = 0.5 * (edges_r[1:] + edges_r[:-1])
    nr = len(rc)
    if r <= rc[0]:
        i, a = 0, 0.0
    elif r >= rc[-1]:
        i, a = nr - 2, 1.0
    else:
        i = int(np.searchsorted(rc, r, side="right")) - 1
        a = (r - rc[i]) / (rc[i + 1] - rc[i])
    out = (1 - a) * prim[:2, :, :, i] + a * prim[:2, :, :, i + 1]
    return np.transpose(out, (0, 2, 1))


@pytest.fixture(scope="module")
def stepped(mods):
    oracle, solver, _ = mods
    g = synth.Grid(150, 30, 60)
    m = synth.relax_map(g, 7)
    say("shell: grid 150x30x60, 30 steps")
    s = solver.Solver(g)
    o = oracle.Oracle(g.nr, g.nt, g.np_, r_in=g.r_in, r_out=g.r_out, th_min=g.th_min,
                      th_max=g.th_max)
    for x in (s, o):
        x.set_maps(np.zeros(1), m[None])
        x.init_radial()
    s.step(30)
    o.step(30)
    yield s, o.get_state(kind=oracle.PRIM_SI)
    s.close()


@pytest.mark.parametrize("r_au", [0.05, 0.5, 1.0, 1.999, 3.0])
def test_shell_matches_oracle_interpolation(stepped, r_au):
    s, prim = stepped
    say(f"shell r={r_au} AU")
    got = s.shell(r_au * synth.AU)
    want = shell_from_state(prim, s.edges()[0], r_au * synth.AU)
    rel = np.max(np.abs(got - want) / np.abs(want))
    say(f"  max rel {rel:.3e}")
    assert rel <= parity.TOL_F64


@pytest.mark.parametrize("precision", [64, 32])
def test_ensemble_stops_on_time_like_single_runs(mods, precision):
    _, solver, relax = mods
    from paper_2501_15923_amd.ensemble import Ensemble
    grids = [synth.Grid(64, 16, 32), synth.Grid(150, 30, 60), synth.Grid(97, 22, 40)]
    t_end = 2.0 * synth.HOUR
    say(f"ensemble t_end precision {precision}")
    e = Ensemble(grids, precision=precision)
    singles = []
    for q, (g, run) in enumerate(zip(grids, e.runs)):
        m = synth.relax_map(g, 40 + q)
        run.set_maps(np.zeros(1), m[None])
        run.init_radial()
        s = solver.Solver(g, precision=precision)
        s.set_maps(np.zeros(1), m[None])
        s.init_radial()
        singles.append(s)
    total = [0] * len(grids)
    for _ in range(100):
        info = e.step(64, t_end=t_end)
        for q, i in enumerate(info):
            total[q] += i["steps"]
        if max(i["steps"] for i in info) == 0:
            break
    for q, (run, s) in enumerate(zip(e.runs, singles)):
        n = 0
        while True:
            i = s.step(64, t_end=t_end)
            n += i["steps"]
            if i["steps"] < 64:
                break
        assert s.clock()["t"] == pytest.approx(t_end, rel=1e-12)
        assert run.clock()["t"] == pytest.approx(t_end, rel=1e-12)
        assert n == total[q], (q, n, total[q])
        assert np.array_equal(run.get_state(kind=1), s.get_state(kind=1)), q
        s.close()
    e.close()


def test_plain_relaxation_record(mods):
    _, solver, relax = mods
    g = synth.Grid(64, 16, 32)
    s = solver.Solver(g)
    s.set_maps(np.zeros(1), synth.relax_map(g, 3)[None])
    s.init_radial()
    t_ref = 1.5 * relax.slow_crossing_time(g)
    say("plain relaxation 64x16x32")
    out = relax.plain_with_reference(s, t_ref, chunk=200)
    say(f"  {out['total_steps']} steps, converged={out['converged']} at {out.get('steps')}")
    assert s.clock()["t"] == pytest.approx(t_ref, rel=1e-12)
    assert out["converged"]
    assert 0 < out["steps"] <= out["total_steps"]
    assert out["resid"] < 1e-4 and max(out["err_rho"], out["err_vr"]) <= 0.02
    # restarting from the relaxed state satisfies the criteria within one chunk
    res = relax.relax(s, out["ref"], 2 * t_ref, chunk=200)
    assert res["converged"] and res["steps"] <= 200
    s.close()


def test_committed_warm_start_relaxes_faster(mods):
    """The committed network on a held-out map: the warm start reaches the
    relaxed wind in well under half the plain steps (measured 650 vs 3350)."""
    import os

    import torch

    from paper_2501_15923_amd import warmstart
    from paper_2501_15923_amd.nn import WarmStartNet
    _, solver, relax = mods
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2501_15923_amd", "weights", "warmstart_150x30x60.npz")
    z = np.load(path)
    dims = tuple(int(v) for v in z["dims"])
    g = synth.Grid(dims[2], dims[0], dims[1])
    net = WarmStartNet.from_dims(dims, batch_max=1)
    net.set_params(z["params"])
    t_ref = 2.0 * relax.slow_crossing_time(g)
    say("warm start with committed weights, held-out seed 2031")
    rows = warmstart.evaluate(net, g, [2031], t_ref, {"warm": net.forward})
    plain, warm = rows[0]["plain"], rows[0]["warm"]
    say(f"  plain {plain['steps']} steps, warm {warm['steps']} steps")
    assert plain["converged"] and warm["converged"]
    assert warm["steps"] <= 0.5 * plain["steps"]
    # the network's state is physical and its 1 AU shell is already close
    assert warm["history"][0][3] < 0.1 and warm["history"][0][4] < 0.1
    net.close()
    torch.cuda.synchronize()


def test_committed_production_warm_start_relaxes_faster(mods):
    """The committed 600 x 60 x 120 network on held-out map 2031: the warm
    start relaxes in at most 0.45 of the plain steps (measured 3500 of 12100)
    and at most half of the plain wall time, network and upload included.
    The convergence criterion is the L2 error over the 1 AU shell; the
    largest pointwise errors at the relaxed check are recorded beside it
    (measured 11.8 % in rho, at a stream interface, and 1.0 % in v_r) and
    must stay below 15 %."""
    import os

    import torch

    from paper_2501_15923_amd import warmstart
    from paper_2501_15923_amd.nn import WarmStartNet
    _, solver, relax = mods
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2501_15923_amd", "weights", "warmstart_600x60x120.npz")
    z = np.load(path)
    dims = tuple(int(v) for v in z["dims"])
    g = synth.Grid(dims[2], dims[0], dims[1])
    assert (g.nr, g.nt, g.np_) == (600, 60, 120)
    net = WarmStartNet.from_dims(dims, batch_max=1)
    net.set_params(z["params"])
    t_ref = 2.0 * relax.slow_crossing_time(g)
    say("production-grid warm start with committed weights, held-out seed 2031")
    rows = warmstart.evaluate(net, g, [2031], t_ref, {"warm": net.forward})
    plain, warm = rows[0]["plain"], rows[0]["warm"]
    say(f"  plain {plain['steps']} steps {plain['wall']:.2f} s, warm {warm['steps']} steps "
        f"{warm['wall']:.2f} s, max shell errors {warm['err_rho_max']:.3f} {warm['err_vr_max']:.3f}")
    assert plain["converged"] and warm["converged"]
    assert warm["steps"] <= 0.45 * plain["steps"]
    assert warm["wall"] <= 0.5 * plain["wall"]
    assert max(warm["err_rho_max"], warm["err_vr_max"]) < 0.15
    net.close()
    torch.cuda.synchronize()

"""Parity of the block-refined HIP path (icr_amr_*) with the refined-grid
oracle (oracle/amr.py) through the C-ABI: one level against the uniform
oracle; three levels with a cone CME, the combined criterion and regrids
every 2 steps (same leaves, states within 1e-9 per conserved group); forced
refinement of a uniform static state."""
import numpy as np
import pytest

import parity
from paper_2501_15923_amd import synth

pytestmark = pytest.mark.gpu

G = synth.Grid(32, 8, 16)


def say(*a):
    print(*a, flush=True)


def _inputs(g=G):
    times, maps = synth.dynamic_maps(g, 3, cadence=1800.0)
    cme = np.array([0.0, 20000.0, 5 * synth.DEG, 1.2, 40 * synth.DEG, 1.5e6, 1e-18, 0.8e6])
    return times, maps, cme[None]


def _pair(max_level, criterion="combined", regrid_every=2, g=G, cme=True, **kw):
    import oracle
    from oracle.amr import AmrConfig, AmrOracle
    from paper_2501_15923_amd.amr import AmrSolver
    times, maps, cmes = _inputs(g)
    s = AmrSolver(g, block=(8, 4, 4), max_level=max_level, criterion=criterion,
                  regrid_every=regrid_every, max_blocks=2048, **kw)
    o = AmrOracle(AmrConfig(g.nr, g.nt, g.np_, g.r_in, g.r_out, g.th_min, g.th_max, br=8, bt=4,
                            bp=4, max_level=max_level, criterion=criterion,
                            regrid_every=regrid_every,
                            **{k: v for k, v in kw.items() if k in ("gravity",)}))
    for x in (s, o):
        x.set_maps(times, maps)
        if cme:
            x.set_cmes(cmes)
        x.init_radial()
    del oracle
    return s, o


def _compare(s, o, what):
    keys = s.leaves()
    assert keys == o.leaves(), what
    a = np.stack([s.block(k) for k in keys], axis=1)
    b = np.stack([o.blocks[k].U[:, 2:-2, 2:-2, 2:-2] for k in keys], axis=1)
    e = parity.rel_errors(a[:8], b[:8])
    e["tau"] = float(np.max(np.abs(a[8] / a[0] - b[8] / b[0])))
    say(what, len(keys), "leaves", e)
    assert max(e.values()) <= parity.TOL_F64, (what, e)
    return e


def test_amr_one_level_matches_the_uniform_oracle():
    import oracle
    s, o = _pair(1, cme=True)
    u = oracle.Oracle(G.nr, G.nt, G.np_, tracer=True)
    times, maps, cmes = _inputs()
    u.set_maps(times, maps)
    u.set_cmes(cmes)
    u.init_radial()
    s.step(20)
    u.step(20)
    U = u.get_state(kind=oracle.CONS_CODE)
    A = np.zeros((9,) + U.shape[1:])
    for k in s.leaves():
        _, bi, bj, bk = k
        A[:, bk * 4:(bk + 1) * 4, bj * 4:(bj + 1) * 4, bi * 8:(bi + 1) * 8] = s.block(k)
    e = parity.assert_parity(A[:8], U, what="amr one level")
    assert np.max(np.abs(A[8] / A[0] - u.get_tracer())) < 1e-9
    assert abs(s.clock()["t"] / u.clock()["t"] - 1) < 1e-11
    say("one level", e)


def test_amr_three_levels_cme_parity():
    s, o = _pair(3, "combined", 2)
    for n in range(4):
        s.step(2)
        o.step(2)
        _compare(s, o, f"after {2 * (n + 1)} steps")
    assert max(k[0] for k in s.leaves()) == 3
    assert abs(s.clock()["t"] / (o.t * __import__("oracle").units()["t"]) - 1) < 1e-11


def test_amr_tracing_and_shock_criteria_parity():
    """tracing with the CME; shock without it, at a lower compression
    threshold, so that the stream interfaces of the dynamic maps refine."""
    s, o = _pair(2, "tracing", 3)
    s.step(9)
    o.step(9)
    _compare(s, o, "tracing")
    assert len(s.leaves()) > 32
    from oracle.amr import AmrConfig, AmrOracle
    from paper_2501_15923_amd.amr import AmrSolver
    times, maps, _ = _inputs()
    s = AmrSolver(G, block=(8, 4, 4), max_level=2, criterion="shock", shock_threshold=0.05,
                  regrid_every=3, max_blocks=2048)
    o = AmrOracle(AmrConfig(G.nr, G.nt, G.np_, G.r_in, G.r_out, G.th_min, G.th_max, br=8, bt=4,
                            bp=4, max_level=2, criterion="shock", shock_thr=0.05,
                            regrid_every=3))
    for x in (s, o):
        x.set_maps(times, maps)
        x.init_radial()
    s.step(12)
    o.step(12)
    _compare(s, o, "shock")
    assert len(s.leaves()) > 32


def test_amr_forced_refinement_parity():
    """icr_amr_force_refine against the oracle's, including the coarser
    leaves the one-level rule adds, then steps with regrids."""
    s, o = _pair(3, "combined", 4)
    keys = [(1, 1, 0, 0), (1, 2, 1, 2)]
    s.force_refine(keys)
    o.force_refine(keys)
    _compare(s, o, "forced, before stepping")
    s.force_refine([(2, 3, 1, 0)])
    o.force_refine([(2, 3, 1, 0)])
    s.step(6)
    o.step(6)
    _compare(s, o, "forced, after 6 steps")

"""Pins of the refined-grid oracle (oracle/amr.py; Sect. 3.2 and Sect. 4:
block refinement with the tracing / shock / combined criteria):

- with one level it is the uniform oracle (same cells, same steps);
- mass, B_r and the CME tracer change over every step, regrids included,
  only by the flux through the domain's radial edges (to round-off): the
  coarse-fine flux correction and the conservative prolongation and
  restriction lose nothing;
- restriction of a prolongation returns the coarse cells;
- a uniform static state stays uniform across coarse-fine faces;
- face neighbours never differ by more than one level after a regrid;
- the tracing criterion flags exactly the blocks holding CME material;
- refining around the CME brings the solution there closer to a run on the
  uniformly refined grid than the coarse run is.
"""
import numpy as np
import pytest

from paper_2501_15923_amd import synth

G = synth.Grid(32, 8, 16)


def _inputs(g=G, cme_speed=1.5e6, hw=40):
    times, maps = synth.dynamic_maps(g, 3, cadence=1800.0)
    cme = np.array([0.0, 20000.0, 5 * synth.DEG, 1.2, hw * synth.DEG, cme_speed, 1e-18, 0.8e6])
    return times, maps, cme[None]


def _amr(orc, g=G, **kw):
    from oracle.amr import AmrConfig, AmrOracle
    cfg = AmrConfig(g.nr, g.nt, g.np_, g.r_in, g.r_out, g.th_min, g.th_max,
                    **{"br": 8, "bt": 4, "bp": 4, **kw})
    return AmrOracle(cfg)


def test_one_level_is_the_uniform_oracle(orc):
    times, maps, cme = _inputs()
    a = _amr(orc, max_level=1)
    a.set_maps(times, maps)
    a.set_cmes(cme)
    a.init_radial()
    o = orc.Oracle(G.nr, G.nt, G.np_, tracer=True)
    o.set_maps(times, maps)
    o.set_cmes(cme)
    o.init_radial()
    a.step(8)
    o.step(8)
    U, A = o.get_state(kind=orc.CONS_CODE), a.sample_level(1)
    for v in range(8):
        assert np.max(np.abs(A[v] - U[v])) <= 1e-13 * np.max(np.abs(U[v])), v
    assert np.max(np.abs(A[8] / A[0] - o.get_tracer())) < 1e-13
    assert a.t * orc.units()["t"] == pytest.approx(o.clock()["t"], rel=1e-14)


@pytest.fixture(scope="module")
def three_level_run(orc):
    """Three levels, combined criterion, regrid every 2 steps, a wide fast
    cone CME entering from t = 0: per step the conservation budget and the
    level balance."""
    times, maps, cme = _inputs()
    a = _amr(orc, max_level=3, criterion="combined", regrid_every=2)
    a.set_maps(times, maps)
    a.set_cmes(cme)
    a.init_radial()
    rows = []
    for _ in range(8):
        M0 = a.totals()
        S0 = sum((np.abs(a.blocks[k].U[:, 2:-2, 2:-2, 2:-2]) * a.cell_volumes(k)[None])
                 .sum(axis=(1, 2, 3)) for k in a.leaves())
        a.step(1)
        d = a.totals() - M0 - a.last_bflux
        scale = np.maximum(S0 + np.abs(a.last_bflux), 1e-300)
        rows.append((d / scale, dict(a.level_counts()), _balance_violations(a)))
    return a, rows


def _balance_violations(a):
    bad = 0
    for key in a.leaves():
        for dd in range(3):
            for side in (0, 1):
                nk = a.neighbour_key(key, dd, side)
                if nk is None:
                    continue
                # the neighbour region is covered by leaves of level l-1 .. l+1
                if nk not in a.blocks:
                    pk = a.parent(nk)
                    if not (pk in a.blocks and a.blocks[pk].leaf):
                        bad += 1
                elif not a.blocks[nk].leaf:
                    # its children that touch the shared face must be leaves
                    for ch in a.children(nk):
                        sub = (ch[1] - 2 * nk[1], ch[2] - 2 * nk[2], ch[3] - 2 * nk[3])
                        if sub[dd] == (0 if side else 1) and not a.blocks[ch].leaf:
                            bad += 1
    return bad


def test_budgets_to_round_off_across_levels_and_regrids(three_level_run):
    _, rows = three_level_run
    for rel, _, _ in rows:
        assert abs(rel[0]) < 1e-14, rel  # mass
        assert abs(rel[5]) < 1e-14, rel  # B_r
        assert abs(rel[8]) < 1e-13, rel  # CME material
    # the run did refine, to the top level
    assert max(max(c) for _, c, _ in rows) == 3


def test_level_balance_after_every_regrid(three_level_run):
    _, rows = three_level_run
    assert all(b == 0 for _, _, b in rows)


def test_tracing_flags_exactly_the_blocks_with_cme_material(three_level_run):
    a, _ = three_level_run
    a.fill_ghosts(a.t)
    n_flag = 0
    for key in a.leaves():
        U = a.blocks[key].U[:, 2:-2, 2:-2, 2:-2]
        has = bool((U[8] / U[0] >= a.cfg.tau_thr).any())
        a.cfg.criterion = "tracing"
        assert a.flagged(key) == has, key
        n_flag += has
    a.cfg.criterion = "combined"
    assert n_flag > 0


def test_prolongation_then_restriction_returns_the_coarse_cells(orc):
    a = _amr(orc, max_level=2)
    rng = np.random.default_rng(5)
    n = 20
    Uc = rng.uniform(0.5, 2.0, (9, n, 3, 3, 3))
    ic = rng.integers(0, G.nr, n)
    jc = rng.integers(0, G.nt, n)
    F = a.prolong(1, Uc, ic, jc)
    back = a.restrict(1, F, ic, jc)
    assert np.max(np.abs(back - Uc[..., 1, 1, 1])) < 1e-15 * 4


def test_uniform_static_state_across_coarse_fine_faces(orc):
    a = _amr(orc, max_level=2, gravity=False, corot=False, omega=0.0)
    m = np.zeros((1, 8, G.nt, G.np_))
    m[0, 0] = 5e-21
    m[0, 4] = 1e-9
    a.set_maps(np.zeros(1), m)
    a.init_radial()
    # a uniform state (the radial expansion of a uniform map is not uniform)
    for b in a.blocks.values():
        b.U[:] = 0.0
        b.U[0] = 5e-21 / orc.units()["rho"]
        b.U[4] = 1e-9 / orc.units()["p"] / 0.5
    a.force_refine([(1, 1, 0, 0), (1, 2, 1, 2), (1, 0, 1, 3)])
    assert a.level_counts().get(2, 0) >= 24
    a.step(10)
    for key in a.leaves():
        U = a.blocks[key].U[:, 2:-2, 2:-2, 2:-2]
        assert np.max(np.abs(U[0] * orc.units()["rho"] / 5e-21 - 1)) < 1e-13
        assert np.max(np.abs(U[1:4])) < 1e-12 * np.sqrt(U[4].max() * U[0].max())


def test_refinement_brings_the_cme_closer_to_the_fine_grid(orc):
    """A fast cone CME on 32 x 8 x 16 cells, refined to level 2 where it
    is (tracing): restricted to the coarse cells, the refined run is closer
    to the run on the uniform 64 x 16 x 32 grid than the coarse run, in the
    blocks that ended refined."""
    times, maps, cme = _inputs()
    t_end = 6000.0
    a = _amr(orc, max_level=2, criterion="tracing", regrid_every=1)
    a.set_maps(times, maps)
    a.set_cmes(cme)
    a.init_radial()
    a.force_refine([k for k in a.leaves() if k[1] == 0])  # the inner shell
    while a.t * orc.units()["t"] < t_end:
        a.step(1)
    t_amr = a.t * orc.units()["t"]

    def run(g):
        o = orc.Oracle(g.nr, g.nt, g.np_, tracer=True)
        f = g.nt // G.nt  # the map of the base column on every finer column
        o.set_maps(times, np.repeat(np.repeat(maps, f, axis=2), f, axis=3))
        o.set_cmes(cme)
        o.init_radial()
        o.step(100000, t_end=t_amr)
        return o.get_state(kind=orc.CONS_CODE)

    coarse = run(G)
    fine = run(synth.Grid(2 * G.nr, 2 * G.nt, 2 * G.np_))
    # the fine run restricted to the coarse cells (volume-weighted)
    from oracle.amr import NG  # noqa: F401
    f2 = fine.reshape(8, G.np_, 2, G.nt, 2, G.nr, 2).transpose(0, 1, 3, 5, 2, 4, 6)
    I, J = np.meshgrid(np.arange(G.nr), np.arange(G.nt), indexing="xy")
    I = np.broadcast_to(I, (G.np_, G.nt, G.nr))
    J = np.broadcast_to(J, (G.np_, G.nt, G.nr))
    ref = a.restrict(1, f2, I, J)
    amr = a.sample_level(1)[:8]
    refined = np.zeros((G.np_, G.nt, G.nr), bool)
    c = a.cfg
    for key in a.leaves(2):
        _, bi, bj, bk = key
        refined[bk * c.bp // 2:(bk + 1) * c.bp // 2, bj * c.bt // 2:(bj + 1) * c.bt // 2,
                bi * c.br // 2:(bi + 1) * c.br // 2] = True
    assert refined.sum() > 0.05 * refined.size
    e_amr = np.abs(amr[0] - ref[0])[refined].mean()
    e_coarse = np.abs(coarse[0] - ref[0])[refined].mean()
    assert e_amr < 0.7 * e_coarse, (e_amr, e_coarse)

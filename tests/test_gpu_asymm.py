"""Parity of the paper's 'asymm' transverse inner boundary (Sect. 2.1: the
quantities the coronal model does not provide vanish on the 0.1 AU
surface) between the HIP path and the oracle: both stage-kernel variants,
the tiny static grid and a ragged grid with a cone CME being inserted."""
import numpy as np
import pytest

import parity
from paper_2501_15923_amd import configs, synth
from test_gpu_parity import cons, mods, pair, say  # noqa: F401

pytestmark = pytest.mark.gpu

ASYMM = 1


@pytest.mark.parametrize("variant", [2, 1])
def test_asymm_tiny_static_parity(mods, variant):
    w = configs.tiny_static()
    s, o = pair(mods, w.grid, w.times, w.maps, bc_transverse=ASYMM)
    s.set_launch(variant=variant)
    say(f"asymm tiny static, variant {variant}, 100 steps")
    info = s.step(100)
    o.step(100)
    assert info["steps"] == 100
    e = parity.assert_parity(*cons(mods, s, o), what=f"asymm variant {variant}")
    say("errors", e)


def test_asymm_ragged_cme_parity(mods):
    g = synth.Grid(150, 30, 60)
    times, maps = synth.dynamic_maps(g, 4, cadence=1800.0)
    cme = np.array([600.0, 7200.0, 5 * synth.DEG, 1.2, 30 * synth.DEG, 1.2e6, 1e-18, 0.8e6])
    s, o = pair(mods, g, times, maps, cme[None], bc_transverse=ASYMM, limiter=1)
    s.set_clock(900.0)
    o.set_clock(900.0)
    say("asymm ragged 150x30x60 with a CME, 30 steps")
    s.step(30)
    o.step(30)
    e = parity.assert_parity(*cons(mods, s, o), what="asymm ragged cme")
    say("errors", e)


def test_asymm_changes_the_solution(mods):
    """The rule is exercised: the transverse boundary values differ from the
    map's (v_phi = -Omega r sin(theta), Parker B_phi), so the two boundary
    treatments give different states after a few steps."""
    w = configs.tiny_static()
    s1, _ = pair(mods, w.grid, w.times, w.maps, bc_transverse=0)
    s2, _ = pair(mods, w.grid, w.times, w.maps, bc_transverse=ASYMM)
    s1.step(20)
    s2.step(20)
    a, b = s1.get_state(kind=1), s2.get_state(kind=1)
    assert parity.max_rel(a, b) > 1e-4


def test_asymm_rejects_too_few_radial_cells(mods):
    _, solver, _abi = mods
    with pytest.raises(_abi.IcarusError):
        solver.Solver(synth.Grid(1, 8, 8), bc_transverse=ASYMM)

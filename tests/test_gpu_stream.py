"""Boundary-map streaming (icr_append_boundary_maps) on an extended domain
(outer boundary 5.5 AU): a run fed its maps a few at a time through a
4-map buffer is bitwise equal to the same run holding every map, and both
match the oracle (which holds every map) to the FP64 parity bar."""
import sys

import numpy as np
import pytest

import parity
from paper_2501_15923_amd import synth

pytestmark = pytest.mark.gpu
G = synth.Grid(120, 16, 32, r_out=5.5 * synth.AU)
CAD = 1800.0
N_MAPS = 12
STEPS = 150


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import oracle
    from paper_2501_15923_amd import _abi, solver
    _abi.lib()
    return oracle, solver, _abi


def maps():
    return synth.dynamic_maps(G, 8, n_maps=N_MAPS, cadence=CAD)


def test_streamed_maps_equal_all_maps_and_oracle(mods):
    oracle, solver, abi = mods
    times, mp = maps()
    say(f"streaming {N_MAPS} maps at {CAD:.0f} s through a buffer of 4, grid {G.nr}x{G.nt}x{G.np_}")
    full = solver.Solver(G, max_maps=16)
    full.set_maps(times, mp)
    full.init_radial()
    s = solver.Solver(G, max_maps=4)
    s.set_maps(times[:3], mp[:3])
    s.init_radial()
    nxt, held_max, refused = 3, 3, 0
    done = 0
    while done < STEPS:
        s.step(10)
        done += 10
        while nxt < N_MAPS:
            try:
                held_max = max(held_max, s.append_maps(times[nxt:nxt + 1], mp[nxt:nxt + 1]))
                nxt += 1
            except abi.IcarusError as e:
                assert e.code == abi.ICR_ERR_STATE
                refused += 1
                break
    full.step(STEPS)
    t = s.clock()["t"]
    say(f"  t = {t / 3600:.2f} h, appended up to map {nxt}, refused {refused} times")
    assert nxt == N_MAPS and refused > 0 and held_max <= 4
    assert t > times[-2], "the run must pass several map times"
    assert np.array_equal(s.get_state(kind=1), full.get_state(kind=1))
    o = oracle.Oracle(G.nr, G.nt, G.np_, r_in=G.r_in, r_out=G.r_out, th_min=G.th_min,
                      th_max=G.th_max)
    o.set_maps(times, mp)
    o.init_radial()
    o.step(STEPS)
    parity.assert_parity(s.get_state(kind=1), o.get_state(kind=oracle.CONS_CODE))
    s.close()
    full.close()


def test_append_rejects_bad_input(mods):
    _, solver, abi = mods
    times, mp = maps()
    s = solver.Solver(G, max_maps=4)
    with pytest.raises(abi.IcarusError) as e:  # nothing to append to
        s.append_maps(times[:1], mp[:1])
    assert e.value.code == abi.ICR_ERR_STATE
    s.set_maps(times[:3], mp[:3])
    s.init_radial()
    with pytest.raises(abi.IcarusError) as e:  # not after the last map
        s.append_maps(times[2:3], mp[2:3])
    assert e.value.code == abi.ICR_ERR_ARG
    assert s.append_maps(times[3:4], mp[3:4]) == 4
    with pytest.raises(abi.IcarusError) as e:  # buffer full, clock still at 0
        s.append_maps(times[4:5], mp[4:5])
    assert e.value.code == abi.ICR_ERR_STATE
    bad = mp[4:5].copy()
    bad[0, 0, 3, 5] = -1.0
    s.step(int(2.5 * CAD / 100))  # move on (dt ~ 100-250 s)
    with pytest.raises(abi.IcarusError) as e:  # rho <= 0
        s.append_maps(times[4:5], bad)
    assert e.value.code == abi.ICR_ERR_ARG
    s.close()

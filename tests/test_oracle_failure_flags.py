"""Failure handling of the oracle on the CPU: a run driven past the CFL
limit (Courant number 3 with the max-sum rule) blows up and is flagged as
non-physical with the index of its first invalid cell, instead of running on
with NaNs; the step that fails is the one reported."""
import numpy as np

from paper_2501_15923_amd import configs


def test_cfl_above_one_is_flagged_not_silent(orc):
    w = configs.tiny_static()
    g = w.grid
    o = orc.Oracle(g.nr, g.nt, g.np_, cfl=3.0)
    o.set_maps(w.times, w.maps)
    o.init_radial()
    status, steps = 0, 0
    for _ in range(400):
        info = o.step(1)
        if info["status"] != 0:
            status = info["status"]
            break
        steps += 1
    assert status == -3, "CFL 3 ran 400 steps without a non-physical cell"
    bad = info["bad_cell"]  # linear index k*nt*nr + j*nr + i
    assert 0 <= bad < g.cells
    k, rem = divmod(bad, g.nt * g.nr)
    j, i = divmod(rem, g.nr)
    W = o.get_state(kind=orc.PRIM_CODE)
    cell = W[:, k, j, i]
    assert not (np.all(np.isfinite(cell)) and cell[0] > 0 and cell[4] > 0), cell
    # every cell before it in the linear order is valid
    flat = W.reshape(8, -1)
    ok = np.isfinite(flat).all(axis=0) & (flat[0] > 0) & (flat[4] > 0)
    assert ok[:bad].all()
    # the same run at CFL 0.4 stays physical over the same number of steps
    o2 = orc.Oracle(g.nr, g.nt, g.np_, cfl=0.4)
    o2.set_maps(w.times, w.maps)
    o2.init_radial()
    assert o2.step(steps + 1)["status"] == 0

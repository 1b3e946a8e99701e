"""A solver whose workspace starts filled with NaN bit patterns (every byte
0xFF) gives bit-identical results to one created in fresh memory: no kernel
reads workspace memory that the library has not written first (ghost
layers, block partials, probe log, tracer fluxes, staging)."""
import ctypes

import numpy as np
import pytest

from paper_2501_15923_amd import synth

pytestmark = pytest.mark.gpu


def _poisoned_solver(g, **kw):
    import torch
    from paper_2501_15923_amd import _abi
    from paper_2501_15923_amd.solver import Solver, make_grid, make_phys
    gs = make_grid(g, 16, 4, 8, 1024, 64)
    ps = make_phys(tracer=kw.get("tracer", False))
    n = ctypes.c_size_t()
    _abi.check(_abi.lib().icr_workspace_bytes(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(n)))
    ws = torch.full((n.value + 256,), 255, dtype=torch.uint8, device="cuda")
    assert torch.isnan(ws[:8].view(torch.float64)).all()
    ptr = (ws.data_ptr() + 255) & ~255
    h = ctypes.c_void_p()
    _abi.check(_abi.lib().icr_create(ctypes.byref(gs), ctypes.byref(ps), ctypes.c_void_p(ptr),
                                     n.value, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                     ctypes.byref(h)))
    s = Solver.wrap(h, g, probe_log_rows=64)
    return s, ws


@pytest.mark.parametrize("tracer", [False, True])
def test_nan_poisoned_workspace_is_never_read(tracer):
    import torch
    from paper_2501_15923_amd import _abi
    from paper_2501_15923_amd.solver import Solver
    g = synth.Grid(150, 30, 60)
    times, maps = synth.dynamic_maps(g, 4, cadence=1800.0)
    cme = np.array([300.0, 7200.0, 5 * synth.DEG, 1.2, 30 * synth.DEG, 1.2e6, 1e-18, 0.8e6])
    tabs = synth.probe_tables(2 * synth.DAY, 1)
    ref = Solver(g, tracer=tracer, max_probes=8, max_traj_pts=1024, probe_log_rows=64)
    bad, ws = _poisoned_solver(g, tracer=tracer)
    for s in (ref, bad):
        s.set_maps(times, maps)
        s.set_cmes(cme[None])
        s.set_probes(tabs, cadence=600.0)
        s.init_radial()
        s.step(60)
    a, b = ref.get_state(kind=1), bad.get_state(kind=1)
    assert np.isfinite(b).all()
    assert np.array_equal(a, b)
    la, na = ref.read_probe_log()
    lb, nb = bad.read_probe_log()
    assert na == nb > 0 and np.array_equal(la, lb)
    assert np.array_equal(ref.divv(), bad.divv())
    assert np.array_equal(ref.shell(synth.AU), bad.shell(synth.AU))
    if tracer:
        assert np.array_equal(ref.get_tracer(), bad.get_tracer())
    _abi.lib().icr_destroy(bad.h)
    bad.h = None
    ref.close()
    del ws
    torch.cuda.synchronize()

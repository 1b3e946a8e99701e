"""CPU checks of the C-ABI library: it loads, exports every function that
include/icarus_hip.h declares, and validates arguments on the host (no GPU
call is made by icr_workspace_bytes)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("icarus_hip.h", "icarus_nn.h")]


def declared():
    names = set()
    for h in HEADERS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(icr_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2501_15923_amd import _abi
    return _abi


def test_header_declares_the_boundary():
    names = declared()
    for must in ("icr_create", "icr_set_boundary_maps", "icr_step", "icr_sample_probes",
                 "icr_workspace_bytes", "icr_grid_edges"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    L = lib.lib()
    for name in declared():
        assert hasattr(L, name), name
    assert set(declared()) == set(lib.SIGNATURES), "binding and header disagree"


def _grid(lib, **kw):
    from paper_2501_15923_amd import synth
    d = dict(n_r=600, n_theta=60, n_phi=120, r_in=0.1 * synth.AU, r_out=2 * synth.AU,
             th_min=30 * synth.DEG, th_max=150 * synth.DEG, max_maps=10, max_cmes=1,
             max_probes=4, max_traj_pts=500, probe_log_rows=100)
    d.update(kw)
    return lib.IcrGrid(**d)


def _phys(lib, **kw):
    d = dict(gamma=1.5, omega=2.87e-6, cfl=0.4, flux=0, limiter=0, precision=64, gravity=1,
             corotation=1)
    d.update(kw)
    return lib.IcrPhys(**d)


def test_workspace_size_and_validation(lib):
    L = lib.lib()
    n = ctypes.c_size_t()
    g, p = _grid(lib), _phys(lib)
    assert L.icr_workspace_bytes(ctypes.byref(g), ctypes.byref(p), ctypes.byref(n)) == 0
    state = 8 * 600 * 60 * 120 * 8
    assert 3 * state < n.value < 3 * state * 1.05
    p32 = _phys(lib, precision=32)
    n32 = ctypes.c_size_t()
    assert L.icr_workspace_bytes(ctypes.byref(g), ctypes.byref(p32), ctypes.byref(n32)) == 0
    assert n32.value < 0.6 * n.value
    bad = [
        (_grid(lib, n_r=0), p), (_grid(lib, r_out=0.05 * 1.5e11), p),
        (_grid(lib, th_min=0.0), p), (_grid(lib, th_max=3.5), p),
        (_grid(lib, n_r=2000, n_theta=2000, n_phi=1000), p),  # > 2^31 cells
        (_grid(lib, n_r=1024, n_theta=1024, n_phi=512), p),  # 2^29 cells: 4 GiB per variable
        (_grid(lib, max_maps=0), p), (_grid(lib, max_probes=2, max_traj_pts=1), p),
        (g, _phys(lib, gamma=1.0)), (g, _phys(lib, cfl=0.0)), (g, _phys(lib, cfl=1.5)),
        (g, _phys(lib, flux=7)), (g, _phys(lib, limiter=3)), (g, _phys(lib, limiter=4)), (g, _phys(lib, precision=16)),
        (g, _phys(lib, tracer=2)), (g, _phys(lib, bc_transverse=2)),
        # asymm mirrors active cells into the ghost layers: n_r >= ghost width
        (_grid(lib, n_r=1), _phys(lib, bc_transverse=1)),
        (_grid(lib, n_r=2), _phys(lib, bc_transverse=1, limiter=2)),
    ]
    for gg, pp in bad:
        rc = L.icr_workspace_bytes(ctypes.byref(gg), ctypes.byref(pp), ctypes.byref(n))
        assert rc == lib.ICR_ERR_ARG
        assert len(L.icr_last_error()) > 0
    # the largest grid the kernels address with 32-bit offsets is accepted
    big = _grid(lib, n_r=1024, n_theta=1024, n_phi=511)
    assert L.icr_workspace_bytes(ctypes.byref(big), ctypes.byref(p), ctypes.byref(n)) == 0


def test_units_match_the_oracle(lib):
    import numpy as np
    import oracle
    out = np.zeros(6)
    assert lib.lib().icr_units(out.ctypes.data_as(lib.D)) == 0
    u = oracle.units()
    assert np.allclose(out, [u["t"], u["L"], u["rho"], u["p"], u["B"], u["v"]], rtol=1e-15)


def test_network_shape_validation_and_parameter_count(lib):
    """icr_nn_param_count checks the shape on the host: the colatitude flag is
    0 or 1, and with it the first layer reads 10 features instead of 8 (the
    count grows by 3 * nk * 2 * c1); the other layers do not change."""
    L = lib.lib()
    n = ctypes.c_longlong()

    def count(**kw):
        d = dict(n_theta=60, n_phi=120, n_r=600, c1=64, c2=128, hidden=384, batch_max=8,
                 phi_lo=-2, phi_hi=46, coord=0)
        d.update(kw)
        rc = L.icr_nn_param_count(ctypes.byref(lib.NnShape(**d)), ctypes.byref(n))
        return rc, n.value

    rc0, p0 = count()
    assert rc0 == 0 and p0 == 2046720  # the network without the channels
    rc1, p1 = count(coord=1)
    assert rc1 == 0 and p1 - p0 == 3 * 49 * 2 * 64 and p1 == 2065536
    assert count(coord=2)[0] == -1  # ICR_NN_ERR_ARG
    assert count(phi_lo=1)[0] != 0 and count(c1=0)[0] != 0

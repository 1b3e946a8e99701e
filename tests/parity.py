"""Parity metric between the HIP path and the oracle.

Per conserved variable k: max|U_gpu - U_orc| / max|U_orc|, with the three
momentum components normalised together by max|m| and the three field
components by max|B|; the pass bar for the FP64 path is 1e-9.
"""
import numpy as np

TOL_F64 = 1e-9


def rel_errors(gpu, orc):
    groups = {"rho": slice(0, 1), "m": slice(1, 4), "e": slice(4, 5), "B": slice(5, 8)}
    out = {}
    for name, sl in groups.items():
        scale = np.max(np.abs(orc[sl]))
        out[name] = float(np.max(np.abs(gpu[sl] - orc[sl])) / scale)
    return out


def max_rel(gpu, orc):
    return max(rel_errors(gpu, orc).values())


def assert_parity(gpu, orc, tol=TOL_F64, what=""):
    e = rel_errors(gpu, orc)
    assert max(e.values()) <= tol, f"{what} parity {e} > {tol}"
    # pointwise relative error of the strictly positive rho and e as well
    for v in (0, 4):
        pr = np.max(np.abs(gpu[v] - orc[v]) / np.abs(orc[v]))
        assert pr <= 10 * tol, f"{what} pointwise rel err of var {v}: {pr}"
    return e

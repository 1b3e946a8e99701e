"""Pins for the oracle's HLLD flux (Miyoshi & Kusano 2005), the higher-order
flux option of the wider-stencil row.

What the method fixes, checked without retyping it:
  - consistency: equal face states give the physical flux (the TVDLF/HLL
    value of the same state);
  - an isolated stationary contact (density jump, equal p, v = 0, B_n != 0)
    and an isolated stationary rotational discontinuity (v_n = -|B_n| /
    sqrt(rho), B_t rotated at constant |B_t|, v_t jumping by -dB_t / sqrt(rho)
    (Walen relation of the + Alfven family)) are kept exactly, while TVDLF and
    HLL smear both; the discontinuity with the other Walen sign is not
    stationary and moves;
  - Sod's problem converges to the exact solution (B = 0: HLLD is HLLC) and
    with smaller error than HLL; the Brio-Wu problem self-converges; the
    circularly polarised Alfven wave converges at second order.
"""
import numpy as np
import pytest

import exact_solutions as ex
from test_oracle_pins import get_1d, prim_1d, run_to, slab

HLLD = 2


def _run(orc, W, flux, steps=60, gamma=5.0 / 3.0):
    o = slab(orc, W.shape[1], gamma=gamma, flux=flux)
    prim_1d(o, W)
    o.step(steps)
    return get_1d(o)


def test_consistency_equal_states(orc):
    o = slab(orc, 8, flux=HLLD)
    h = slab(orc, 8, flux=1)
    rng = np.random.default_rng(4)
    for _ in range(20):
        w = rng.normal(size=8)
        w[0], w[4] = abs(w[0]) + 0.3, abs(w[4]) + 0.3
        for n in (1, 2, 3):
            f, g = o.face_flux(w, w, n), h.face_flux(w, w, n)
            assert np.max(np.abs(f - g)) <= 1e-13 * (1 + np.max(np.abs(g)))


def test_stationary_contact_kept_exactly(orc):
    n = 64
    x = (np.arange(n) + 0.5) / n
    W = np.zeros((8, n))
    W[0] = np.where(x < 0.5, 1.0, 0.3)
    W[4], W[5], W[6], W[7] = 1.0, 0.75, 0.5, 0.2
    assert np.array_equal(_run(orc, W, HLLD), W)
    for f in (0, 1):
        assert np.max(np.abs(_run(orc, W, f)[0] - W[0])) > 0.05


def _rotational(n, sign):
    x = (np.arange(n) + 0.5) / n
    W = np.zeros((8, n))
    W[0], W[4], W[5], W[1] = 1.0, 1.0, 1.0, -1.0
    W[6] = np.where(x < 0.5, 1.0, 0.0)
    W[7] = np.where(x < 0.5, 0.0, 1.0)
    # v_t jumps by -sign * (B_tR - B_tL) / sqrt(rho); sign = +1 is the Walen
    # relation of the wave that the flow v_n = -c_A holds in place
    W[2] = np.where(x < 0.5, 0.0, sign * 1.0)
    W[3] = np.where(x < 0.5, 0.0, -sign * 1.0)
    return W


def test_stationary_rotational_discontinuity_kept_exactly(orc):
    W = _rotational(64, +1)
    assert np.array_equal(_run(orc, W, HLLD), W)
    for f in (0, 1):
        assert np.max(np.abs(_run(orc, W, f) - W)) > 0.1
    W2 = _rotational(64, -1)  # not a stationary wave
    assert np.max(np.abs(_run(orc, W2, HLLD) - W2)) > 0.1


def test_sod_converges_and_beats_hll(orc):
    errs = {}
    for flux in (1, HLLD):
        e = []
        for n in (100, 200, 400):
            o = slab(orc, n, gamma=1.4, flux=flux)
            x = (np.arange(n) + 0.5) / n
            W = np.zeros((8, n))
            W[0] = np.where(x < 0.5, 1.0, 0.125)
            W[4] = np.where(x < 0.5, 1.0, 0.1)
            prim_1d(o, W)
            run_to(o, 0.2)
            ref = ex.riemann_sample(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, (x - 0.5) / 0.2)
            e.append(np.mean(np.abs(get_1d(o)[0] - ref[0])))
        errs[flux] = e
    assert errs[HLLD][0] > errs[HLLD][1] > errs[HLLD][2]
    assert all(h < l for h, l in zip(errs[HLLD], errs[1])), errs


def test_brio_wu_self_convergence_hlld(orc):
    def run(n):
        o = slab(orc, n, gamma=2.0, limiter=1, flux=HLLD)
        x = (np.arange(n) + 0.5) / n
        W = np.zeros((8, n))
        W[0] = np.where(x < 0.5, 1.0, 0.125)
        W[4] = np.where(x < 0.5, 1.0, 0.1)
        W[5] = 0.75
        W[6] = np.where(x < 0.5, 1.0, -1.0)
        prim_1d(o, W)
        run_to(o, 0.1)
        return get_1d(o)[0]

    ref = run(2048)
    errs = []
    for n in (128, 256, 512):
        errs.append(np.mean(np.abs(run(n) - ref.reshape(n, -1).mean(axis=1))))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.01


def test_alfven_wave_second_order_hlld(orc):
    from test_oracle_pins import _cp_alfven
    errs = []
    for n in (16, 32, 64):
        o = slab(orc, n, gamma=5.0 / 3.0, periodic=True, limiter=1, flux=HLLD)
        W0, _ = _cp_alfven(o, n, 0)
        run_to(o, 1.0)
        got = get_1d(o)
        errs.append(np.mean(np.abs(got[6] - W0[6])) + np.mean(np.abs(got[7] - W0[7])))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[2] < 0.02 and order[-1] > 1.5, (errs, order)

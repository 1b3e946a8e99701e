"""CPU checks of host-side tools: the output-layer scaling that weights the
warm-start loss per variable, the ingest of rocprofv3 counter files into the
traffic record that bench.py reports, the relaxation criteria (first record
with residual < tol and both 1 AU shell errors within tol), the warm-start
longitude window and the evaluation summary."""
import csv
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_scale_output_round_trip_and_layout():
    from paper_2501_15923_amd.nn import init_params
    from paper_2501_15923_amd.warmstart import scale_output
    dims = (6, 8, 5, 4, 3, 7, -1, 2)
    p = init_params(*dims[:6], phi_lo=dims[6], phi_hi=dims[7], seed=1)
    p[-40:] += 0.25  # non-zero output biases
    s = np.ones(8)
    s[0], s[3] = 2.0, 0.5
    q = scale_output(p, dims, s)
    assert np.array_equal(scale_output(q, dims, 1.0 / s), p)  # powers of two: exact
    k1 = 3 * (dims[7] - dims[6] + 1) * 8
    c1, c2, h, no = dims[3], dims[4], dims[5], 8 * dims[2]
    off = k1 * c1 + c1 + 9 * c1 * c2 + c2 + c2 * h + h
    W, Wq = p[off:off + h * no].reshape(h, no), q[off:off + h * no].reshape(h, no)
    b, bq = p[off + h * no:], q[off + h * no:]
    for v in range(8):  # output index r * 8 + v
        assert np.allclose(Wq[:, v::8], s[v] * W[:, v::8])
        assert np.allclose(bq[v::8], s[v] * b[v::8])
    assert np.array_equal(q[:off], p[:off])  # encoder and first decoder layer untouched


def _write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_ingest_counters_scales_by_the_copy_and_adds_valu(tmp_path):
    import bench
    k2 = "void icr::k_stage_lds<double, 64, 4, 0, 0, 2, false>(icr::StageArgs<double>, int)"
    k1 = "void icr::k_stage_lds<double, 64, 4, 0, 0, 1, false>(icr::StageArgs<double>, int)"
    cp = "__amd_rocclr_copyBuffer"
    d = [str(tmp_path / n) for n in ("f", "w", "cf", "cw", "sq")]
    _write_counters(d[0], [dict(Kernel_Name=k2, Counter_Name="FETCH_SIZE", Counter_Value=v)
                           for v in (1000.0, 1200.0)] +
                    [dict(Kernel_Name=k1, Counter_Name="FETCH_SIZE", Counter_Value=9e9)])
    _write_counters(d[1], [dict(Kernel_Name=k2, Counter_Name="WRITE_SIZE", Counter_Value=500.0)])
    # the copy of 2 GiB reads 2^20 counted units for FETCH and 2^21 for WRITE
    _write_counters(d[2], [dict(Kernel_Name=cp, Counter_Name="FETCH_SIZE", Counter_Value=2**20)])
    _write_counters(d[3], [dict(Kernel_Name=cp, Counter_Name="WRITE_SIZE", Counter_Value=2**21)])
    _write_counters(d[4], [dict(Kernel_Name=k2, Counter_Name="SQ_INSTS_VALU", Counter_Value=64.0),
                           dict(Kernel_Name=k2, Counter_Name="SQ_WAVES", Counter_Value=1.0)])
    out = str(tmp_path / "t.json")
    bench.ingest_counters(d[:4], 64, out, "64,12")
    (rec,) = bench.traffic_records(out)
    assert rec["fetch_bytes"] == 1100.0 * 2048 and rec["write_bytes"] == 500.0 * 1024
    assert rec["bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"]
    assert rec["kernel_rev"] == bench.kernel_rev() and "valu_wave_instr_per_launch" not in rec
    assert rec["launch"] == [64, 12] and rec["flux"] == "tvdlf" and rec["limiter"] == "minmod"
    # the same launch shape again replaces its record; another one is kept beside it
    bench.ingest_counters(d, 64, out, "64,12")
    (rec,) = bench.traffic_records(out)
    assert rec["valu_wave_instr_per_launch"] == 64.0
    bench.ingest_counters(d[:4], 64, out, "64,15")
    recs = bench.traffic_records(out)
    assert [r["launch"] for r in recs] == [[64, 12], [64, 15]]
    # the bench picks the record of its own launch shape, scheme and precision
    assert bench.traffic_for(out, 64, "tvdlf", "minmod", [64, 15])["launch"] == [64, 15]
    assert bench.traffic_for(out, 64, "tvdlf", "minmod", [64, 8]) is None
    assert bench.traffic_for(out, 64, "hlld", "minmod", [64, 12]) is None
    assert bench.traffic_for(out, 32, "tvdlf", "minmod", [64, 12]) is None
    # a file holding one bare record still reads
    json.dump(rec, open(out, "w"))
    assert bench.traffic_records(out) == [rec]


def test_relaxation_criteria_pick_the_first_record_meeting_both():
    from paper_2501_15923_amd import relax
    # (steps, wall, residual, err_rho, err_vr)
    rec = [(50, 0.1, 3e-4, 0.50, 0.10), (100, 0.2, 9e-5, 0.030, 0.01),
           (150, 0.3, 2e-4, 0.015, 0.01), (200, 0.4, 8e-5, 0.019, 0.02),
           (250, 0.5, 5e-5, 0.010, 0.005)]
    out = relax.first_relaxed(rec, 1e-4, 0.02)
    assert out["converged"] and out["steps"] == 200 and out["wall"] == 0.4
    none = relax.first_relaxed(rec[:3], 1e-4, 0.02)
    assert not none["converged"] and none["steps"] == 150


def test_shell_errors_and_crossing_time():
    from paper_2501_15923_amd import relax, synth
    ref = np.stack([np.full((4, 5), 2.0), np.full((4, 5), 400e3)])
    sh = ref.copy()
    sh[0] *= 1.03
    sh[1, 0, 0] += 4e3  # one of 20 points off by 1 %
    er, ev = relax.shell_errors(sh, ref)
    assert abs(er - 0.03) < 1e-12
    assert abs(ev - 0.01 / np.sqrt(20)) < 1e-12
    g = synth.Grid(150, 30, 60)
    assert abs(relax.slow_crossing_time(g) - 1.9 * synth.AU / 350e3) < 1e-6 * 1.9 * synth.AU / 350e3


def test_default_window_reaches_the_slow_wind_footpoint():
    import math

    from paper_2501_15923_amd import synth
    from paper_2501_15923_amd.warmstart import default_window
    for g in (synth.Grid(150, 30, 60), synth.Grid(600, 60, 120)):
        lo, hi = default_window(g)
        dph = 2 * math.pi / g.np_
        lag = synth.OMEGA_SUN * (g.r_out - g.r_in) / 350e3  # longitude lag at r_out, rad
        assert lo == -2 and (hi - 1) * dph >= lag > (hi - 2) * dph
    assert default_window(synth.Grid(150, 30, 60)) == (-2, 24)
    assert default_window(synth.Grid(600, 60, 120)) == (-2, 46)


def test_summarise_ratios_over_converged_runs():
    from paper_2501_15923_amd.warmstart import summarise

    def row(ps, pw, ws, ww, conv=True):
        return dict(plain=dict(converged=True, steps=ps, wall=pw),
                    warm=dict(converged=conv, steps=ws, wall=ww, err_rho=0.019, err_vr=0.002))
    rows = [row(1000, 1.0, 300, 0.3), row(1200, 1.2, 600, 0.6), row(900, 0.9, 900, 0.9, False)]
    s = summarise(rows, ["warm"])["warm"]
    assert s["converged"] == 2 and s["of"] == 3
    assert abs(s["wall_ratio_median"] - 0.4) < 1e-12 and abs(s["wall_ratio_mean"] - 0.4) < 1e-12
    assert s["steps_median"] == 450.0 and s["plain_steps_median"] == 1100.0


def test_widened_network_keeps_its_function_and_trains_every_new_weight():
    """widen_params adds encoder channels and decoder units whose outgoing
    weights are zero: the oracle's forward pass gives the same outputs, and
    the oracle's gradient reaches the new weights (the first step can move
    them)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import nn_oracle as O
    from paper_2501_15923_amd.nn import init_params
    from paper_2501_15923_amd.warmstart import widen_params
    dims = (5, 8, 4, 3, 4, 6, -1, 2)
    p = init_params(*dims[:6], phi_lo=dims[6], phi_hi=dims[7], seed=3)
    rng = np.random.default_rng(0)
    p = (p + 0.05 * rng.standard_normal(p.size)).astype(np.float32)  # non-zero biases too
    q, d2 = widen_params(p, dims, 5, 7, 9, seed=1)
    assert d2 == (5, 8, 4, 5, 7, 9, -1, 2, 0)
    s1 = O.Shape(*dims[:6], phi_lo=dims[6], phi_hi=dims[7])
    s2 = O.Shape(*d2[:6], phi_lo=d2[6], phi_hi=d2[7])
    assert q.size == s2.nparam
    x = rng.standard_normal((2, dims[0], dims[1], 8))
    y1, _ = O.forward(s1, p.astype(np.float64), x, bf16=False)
    y2, _ = O.forward(s2, q.astype(np.float64), x, bf16=False)
    assert np.allclose(y1, y2, rtol=0, atol=1e-12)
    # old weights are carried over in place
    o1, o2 = s1.unpack(p), s2.unpack(q)
    assert np.array_equal(o2[0][:, :3], o1[0])
    assert np.array_equal(o2[2].reshape(9, 5, 7)[:, :3, :4], o1[2].reshape(9, 3, 4))
    assert np.array_equal(o2[6][:6], o1[6]) and not o2[6][6:].any()
    # every block of new weights receives a gradient
    t = rng.standard_normal(y2.shape)
    _, g = O.loss_grad(s2, q.astype(np.float64), x, t, bf16=False)
    G = s2.unpack(g)
    assert np.abs(G[6][6:]).max() > 0          # new decoder rows (outgoing)
    assert np.abs(G[4][4:]).max() > 0          # new second-layer channels (outgoing)
    assert np.abs(G[2].reshape(9, 5, 7)[:, 3:, :]).max() > 0  # new first-layer channels


def test_colatitude_channels_grown_into_a_trained_network():
    """Adding the two colatitude input channels with zero first-layer weights
    keeps the function: the oracle gives the same outputs on the features
    with and without them, the old first-layer rows keep their taps, and the
    new rows receive a gradient."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import nn_oracle as O
    from paper_2501_15923_amd.nn import init_params
    from paper_2501_15923_amd.warmstart import widen_params
    dims = (5, 8, 4, 3, 4, 6, -1, 2)
    p = init_params(*dims[:6], phi_lo=dims[6], phi_hi=dims[7], seed=4)
    rng = np.random.default_rng(1)
    p = (p + 0.05 * rng.standard_normal(p.size)).astype(np.float32)
    q, d2 = widen_params(p, dims, 3, 4, 6, coord=1)
    assert d2 == (5, 8, 4, 3, 4, 6, -1, 2, 1)
    s1 = O.Shape(*dims[:8])
    s2 = O.Shape(*d2)
    assert s2.cin == 10 and q.size == s2.nparam
    x8 = rng.standard_normal((2, 5, 8, 8))
    x10 = np.concatenate([x8, rng.standard_normal((2, 5, 8, 2))], axis=-1)
    y1, _ = O.forward(s1, p.astype(np.float64), x8, bf16=False)
    y2, _ = O.forward(s2, q.astype(np.float64), x10, bf16=False)
    assert np.allclose(y1, y2, rtol=0, atol=1e-12)
    W1o, W1n = s1.unpack(p)[0], s2.unpack(q)[0].reshape(-1, 10, 3)
    assert np.array_equal(W1n[:, :8, :].reshape(-1, 3), W1o) and not W1n[:, 8:, :].any()
    t = rng.standard_normal(y2.shape)
    _, g = O.loss_grad(s2, q.astype(np.float64), x10, t, bf16=False)
    assert np.abs(s2.unpack(g)[0].reshape(-1, 10, 3)[:, 8:, :]).max() > 0


def test_plain_cache_round_trip(tmp_path):
    from paper_2501_15923_amd.synth import Grid
    from paper_2501_15923_amd.warmstart import PlainCache
    g = Grid(12, 4, 6)
    path = str(tmp_path / "plain.npz")
    c = PlainCache(path, g, 1.5e6)
    assert c.get(7) is None
    ref = np.arange(48.0).reshape(2, 4, 6)
    c.put(7, dict(ref=ref, steps=350, wall=1.25, converged=True,
                  history=[(50, 0.1, 1e-3, 0.5, 0.2)]))
    c2 = PlainCache(path, g, 1.5e6)
    got = c2.get(7)
    assert got["steps"] == 350 and got["converged"] and np.array_equal(got["ref"], ref)
    assert got["history"][0][0] == 50
    assert PlainCache(path, g, 2.0e6).get(7) is None       # another reference time
    assert PlainCache(path, Grid(12, 4, 8), 1.5e6).get(7) is None  # another grid

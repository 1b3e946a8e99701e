"""Learned warm start of the relaxation phase.

Pipeline (all numerics on the GPU through libicarus_hip.so):
  1. dataset: static boundary maps (synth.relax_map, training and held-out
     seeds) relaxed plainly for two slow-wind crossing times by the batched
     ensemble; the relaxed states become network targets (icr_nn_encode_target);
  2. training: the network of include/icarus_nn.h with its own BF16-MFMA
     forward/backward kernels and Adam (FP32 masters);
  3. evaluation on held-out maps: steps and wall time to reach the relaxed
     wind (relax.py criteria) from the radial expansion (plain) and from the
     network's prediction (warm), plus the untrained network and the
     mean-target predictor as ablations.

    python -m paper_2501_15923_amd.warmstart --out WEIGHTS.npz --report REPORT.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import relax, synth
from .nn import full_dims, in_channels
from .synth import AU, Grid

TRAIN_SEED0, TEST_SEED0 = 1000, 2000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def grid_geometry(solver):
    """Cell-centre radii [m] and colatitudes of a solver (device tensors)."""
    import torch
    r, t, _ = solver.edges()
    rc = 0.5 * (r[1:] + r[:-1])
    thc = 0.5 * (t[1:] + t[:-1])
    return torch.from_numpy(rc).cuda(), torch.from_numpy(thc).cuda()


def relaxed_states(grid, seeds, t_ref, precision=64, batch=64, chunk=4000):
    """Relax each seed's map for t_ref; yields (seed, map, primitive SI state
    as a device tensor).  batch > 1: the batched ensemble, batch runs per
    launch (small grids); batch = 1: one solver per map, stepping in graphs
    (grids that fill the GPU on their own)."""
    if batch == 1:
        yield from _relaxed_single(grid, seeds, t_ref, precision, chunk)
        return
    from .ensemble import Ensemble
    for b0 in range(0, len(seeds), batch):
        sub = seeds[b0:b0 + batch]
        e = Ensemble([grid] * len(sub), precision=precision)
        maps = [synth.relax_map(grid, s) for s in sub]
        for m, run in zip(maps, e.runs):
            run.set_maps(np.zeros(1), m[None])
            run.init_radial()
        t0 = time.perf_counter()
        failed = set()
        while True:
            info = e.step(chunk, t_end=t_ref, raise_on_error=False)
            failed |= {q for q, i in enumerate(info) if i["status"] != 0}
            log(f"warmstart: batch at {b0}: t = {min(i['t'] for i in info) / 86400:.2f} d "
                f"after {time.perf_counter() - t0:.1f} s")
            if max(i["steps"] for i in info) < chunk:
                break
        log(f"warmstart: relaxed {len(sub)} maps to {t_ref / 86400:.1f} d in "
            f"{time.perf_counter() - t0:.1f} s" +
            (f"; dropped non-physical runs {sorted(sub[q] for q in failed)}" if failed else ""))
        for q, (s, m, run) in enumerate(zip(sub, maps, e.runs)):
            if q not in failed:
                yield s, m, run.get_state_device()
        e.close()


def _relaxed_single(grid, seeds, t_ref, precision, chunk):
    from .solver import Solver
    s = Solver(grid, precision=precision)
    t0 = time.perf_counter()
    for q, seed in enumerate(seeds):
        m = synth.relax_map(grid, seed)
        s.set_maps(np.zeros(1), m[None])
        s.init_radial()
        ok = True
        while True:
            info = s.step(chunk, t_end=t_ref, raise_on_error=False)
            if info["status"] != 0:
                ok = False
                break
            if info["steps"] < chunk:
                break
        log(f"warmstart: map {q + 1}/{len(seeds)} (seed {seed}) relaxed to "
            f"{t_ref / 86400:.1f} d, {time.perf_counter() - t0:.1f} s"
            + ("" if ok else "; non-physical, dropped"))
        if ok:
            yield seed, m, s.get_state_device()
    s.close()


def build_dataset(net, grid, seeds, t_ref, rc, thc, precision=64, batch=64):
    import torch
    n = len(seeds)
    X = torch.empty((n, grid.nt, grid.np_, net.cin), dtype=torch.float32, device="cuda")
    T = torch.empty((n, grid.nt * grid.np_, 8 * grid.nr), dtype=torch.float32, device="cuda")
    M = torch.empty((n, 8, grid.nt, grid.np_), dtype=torch.float64, device="cuda")
    q = 0
    for s, m, st in relaxed_states(grid, seeds, t_ref, precision, batch):
        dm = torch.from_numpy(m).cuda()
        M[q] = dm
        X[q] = net.encode_map(dm[None].contiguous(), thc, synth.OMEGA_SUN, grid.r_in)[0]
        net.encode_target(dm, st, rc, thc, synth.OMEGA_SUN, grid.r_in, out=T[q])
        q += 1
    return X[:q], T[:q], M[:q]


def scale_output(params, dims, s):
    """Scale the last layer's weights and biases of output r * 8 + v by s[v]
    (s of length 8) or by s[r * 8 + v] (length 8 n_r).  Training on targets
    scaled the same way weights the squared error of that output by s^2 (the
    last layer is linear); dividing by s afterwards returns the usual
    output."""
    nt, nph, nr, c1, c2, hidden, lo, hi, coord = full_dims(dims)
    k1 = 3 * (hi - lo + 1) * in_channels(coord)
    no = 8 * nr
    p = np.array(params, dtype=np.float32, copy=True)
    off = k1 * c1 + c1 + 9 * c1 * c2 + c2 + c2 * hidden + hidden
    W4 = p[off:off + hidden * no].reshape(hidden, no)
    b4 = p[off + hidden * no:off + hidden * no + no]
    s = np.asarray(s, dtype=np.float32)
    col = np.tile(s, nr) if s.size == 8 else s
    W4 *= col[None, :]
    b4 *= col
    assert off + hidden * no + no == p.size
    return p


def widen_params(params, dims, c1, c2, hidden, coord=None, seed=0):
    """Grow the encoder channels and the decoder width, and optionally add
    the colatitude input channels, without changing the network's function:
    the new units get random incoming weights (the spread of the existing
    ones, zero biases) and zero outgoing weights, and the new input channels
    zero first-layer weights, so every output is unchanged until training
    moves them.  Returns (params, dims) of the wider network."""
    nt, nph, nr, a1, a2, ah, lo, hi, acoord = full_dims(dims)
    coord = acoord if coord is None else int(coord)
    assert c1 >= a1 and c2 >= a2 and hidden >= ah and coord >= acoord
    rng = np.random.default_rng(seed)
    taps = 3 * (hi - lo + 1)
    ain, cin = in_channels(acoord), in_channels(coord)
    k1 = taps * ain
    no = 8 * nr
    p = np.asarray(params, dtype=np.float32)
    shapes = [(k1, a1), (a1,), (9, a1, a2), (a2,), (a2, ah), (ah,), (ah, no), (no,)]
    old, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        old.append(p[o:o + n].reshape(sh))
        o += n
    assert o == p.size, "parameter vector does not match dims"
    W1, b1, W2, b2, W3, b3, W4, b4 = old

    def grow(w, shape, fill_std):
        out = (rng.normal(0.0, fill_std, shape) if fill_std > 0 else np.zeros(shape))
        out = out.astype(np.float32)
        out[tuple(slice(0, s) for s in w.shape)] = w
        return out
    # first layer rows are tap * C + channel: the old channels keep their
    # taps, the new input channels start at zero
    W1 = W1.reshape(taps, ain, a1)
    nW1 = grow(W1, (taps, cin, c1), float(W1.std()))
    nW1[:, ain:, :] = 0.0
    nb1 = grow(b1, (c1,), 0.0)
    nW2 = grow(W2, (9, c1, c2), float(W2.std()))
    nW2[:, a1:, :] = 0.0          # new first-layer channels feed nothing yet
    nb2 = grow(b2, (c2,), 0.0)
    nW3 = grow(W3, (c2, hidden), float(W3.std()))
    nW3[a2:, :] = 0.0             # new second-layer channels feed nothing yet
    nb3 = grow(b3, (hidden,), 0.0)
    nW4 = grow(W4, (hidden, no), 0.0)  # new decoder units feed nothing yet
    q = np.concatenate([a.ravel() for a in (nW1, nb1, nW2, nb2, nW3, nb3, nW4, b4)])
    return q.astype(np.float32), (nt, nph, nr, c1, c2, hidden, lo, hi, coord)


class PlainCache:
    """Plain relaxations (reference shell, steps, wall time) of held-out maps
    kept in an .npz file, so that repeated evaluations of different weights
    on the same maps and grid step each plain run once."""

    def __init__(self, path, grid, t_ref):
        self.path, self.key = path, f"{grid.nr}x{grid.nt}x{grid.np_}_{t_ref:.6e}"
        self.ref, self.meta = {}, {}
        if path and os.path.exists(path):
            z = np.load(path)
            meta = json.loads(str(z["meta"]))
            if meta.get("key") == self.key:
                self.meta = {int(k): v for k, v in meta["runs"].items()}
                self.ref = {s: z[f"ref_{s}"] for s in self.meta}

    def get(self, seed):
        if seed not in self.meta:
            return None
        return dict(self.meta[seed], ref=self.ref[seed])

    def put(self, seed, plain):
        self.meta[seed] = {k: v for k, v in plain.items() if k != "ref"}
        self.ref[seed] = np.asarray(plain["ref"])
        if self.path:
            meta = json.dumps({"key": self.key, "runs": self.meta}, default=float)
            np.savez(self.path, meta=np.array(meta),
                     **{f"ref_{s}": r for s, r in self.ref.items()})


def default_window(grid, v_slow=350e3):
    """First-layer longitude offsets reaching the footpoint of slow wind at the
    outer radius: Omega (r_out - r_in) / v_slow, in cells, plus one; two
    cells downstream."""
    dph = 2.0 * math.pi / grid.np_
    hi = int(math.ceil(synth.OMEGA_SUN * (grid.r_out - grid.r_in) / v_slow / dph)) + 1
    return -2, min(hi, grid.np_ - 3)


def train(net, X, T, epochs=30, batch=8, lr=2e-3, seed=0):
    import torch
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * (n // batch)
    hist = []
    k = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot = 0.0
        for b in range(n // batch):
            idx = torch.from_numpy(perm[b * batch:(b + 1) * batch]).cuda()
            x = X[idx].contiguous()
            t = T[idx].reshape(batch * T.shape[1], T.shape[2]).contiguous()
            loss = net.loss_grad(x, t)
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * k / steps))
            net.adam_step(cur)
            tot += loss
            k += 1
        hist.append(tot / (n // batch))
        log(f"warmstart: epoch {ep} loss {hist[-1]:.3e}")
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def evaluate(net, grid, seeds, t_ref, predictors, chunk=50, precision=64, cache=None):
    """Plain vs warm relaxation on held-out maps.  predictors: name ->
    function(X [1][nt][np][8]) -> y [ncol][no] device tensor.  cache: a
    PlainCache whose stored plain runs are reused (and new ones added)."""
    import torch

    from .solver import Solver
    rows = []

    def ticker(label):
        last = [time.perf_counter()]

        def f(steps, wall):
            if time.perf_counter() - last[0] > 30.0:
                last[0] = time.perf_counter()
                log(f"warmstart: {label}: {steps} steps, {wall:.1f} s")
        return f

    for s in seeds:
        m = synth.relax_map(grid, s)
        solver = Solver(grid, precision=precision)
        solver.set_maps(np.zeros(1), m[None])
        solver.init_radial()
        rc, thc = grid_geometry(solver)
        plain = cache.get(s) if cache is not None else None
        if plain is None:
            plain = relax.plain_with_reference(solver, t_ref, chunk,
                                               progress=ticker(f"seed {s} plain"))
            if cache is not None:
                cache.put(s, plain)
        row = dict(seed=s, plain=dict((k, v) for k, v in plain.items() if k != "ref"))
        dm = torch.from_numpy(m).cuda()
        for name, pred in predictors.items():
            solver.set_clock(0.0, 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x = net.encode_map(dm[None].contiguous(), thc, synth.OMEGA_SUN, grid.r_in)
            y = pred(x)
            st = net.decode_state(dm, y, rc, thc, synth.OMEGA_SUN, grid.r_in)
            solver.set_state(st)
            torch.cuda.synchronize()
            w0 = time.perf_counter() - t0
            res = relax.relax(solver, plain["ref"], t_ref, chunk, wall0=w0,
                              progress=ticker(f"seed {s} {name}"))
            res["init_wall"] = w0
            row[name] = res
        solver.close()
        rows.append(row)
        log(f"warmstart: seed {s} plain {row['plain'].get('steps')} steps " +
            " ".join(f"{k} {row[k]['steps']}" for k in predictors))
    return rows


def summarise(rows, names):
    out = {}
    ok = [r for r in rows if r["plain"]["converged"]]
    for name in names:
        good = [r for r in ok if r[name]["converged"]]
        if not good:
            out[name] = dict(converged=0)
            continue
        ratio_w = [r[name]["wall"] / r["plain"]["wall"] for r in good]
        ratio_s = [r[name]["steps"] / r["plain"]["steps"] for r in good]
        out[name] = dict(converged=len(good), of=len(ok),
                         wall_ratio_median=float(np.median(ratio_w)),
                         wall_ratio_mean=float(np.mean(ratio_w)),
                         steps_ratio_median=float(np.median(ratio_s)),
                         plain_steps_median=float(np.median([r["plain"]["steps"] for r in good])),
                         steps_median=float(np.median([r[name]["steps"] for r in good])),
                         err_rho_median=float(np.median([r[name]["err_rho"] for r in good])),
                         err_vr_median=float(np.median([r[name]["err_vr"] for r in good])),
                         err_rho_max_median=float(np.median([r[name].get("err_rho_max", np.nan)
                                                             for r in good])),
                         err_vr_max_median=float(np.median([r[name].get("err_vr_max", np.nan)
                                                            for r in good])))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nr", type=int, default=150)
    ap.add_argument("--nt", type=int, default=30)
    ap.add_argument("--nph", type=int, default=60)
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--c1", type=int, default=64)
    ap.add_argument("--c2", type=int, default=128)
    ap.add_argument("--hidden", type=int, default=384)
    ap.add_argument("--coord", type=int, default=0,
                    help="1: two colatitude input channels (grown into --init-weights "
                         "with zero first-layer weights)")
    ap.add_argument("--phi-lo", type=int, default=None)
    ap.add_argument("--phi-hi", type=int, default=None)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--crossings", type=float, default=2.0,
                    help="reference relaxation length, slow-wind crossing times")
    ap.add_argument("--data-crossings", type=float, default=None,
                    help="relaxation length of the training targets (default: --crossings)")
    ap.add_argument("--ens-batch", type=int, default=64,
                    help="runs per ensemble launch; 1: one solver per map")
    ap.add_argument("--train-seed0", type=int, default=TRAIN_SEED0,
                    help="first training seed (disjoint chunks across calls)")
    ap.add_argument("--test-seed0", type=int, default=TEST_SEED0,
                    help="first held-out seed (evaluation split across calls)")
    ap.add_argument("--init-weights", default=None,
                    help="continue training from these weights")
    ap.add_argument("--data-precision", type=int, default=32)
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None, help="evaluate these weights (skip training)")
    ap.add_argument("--report", default=None)
    ap.add_argument("--outer-weight", type=float, default=1.0,
                    help="loss weight of every output beyond --outer-au (the 1 AU shell "
                         "criterion never sees them; they only feed the residual)")
    ap.add_argument("--outer-au", type=float, default=1.05)
    ap.add_argument("--rho-weight", type=float, default=1.0,
                    help="loss weight of the density output (targets and the output layer "
                         "scaled by its square root while training)")
    ap.add_argument("--widen", default=None, metavar="C1,C2,HIDDEN",
                    help="grow the --init-weights network to these widths first (same "
                         "function at the start, see widen_params)")
    ap.add_argument("--plain-cache", default=None,
                    help=".npz of plain runs of held-out maps: reused when present, "
                         "extended otherwise")
    ap.add_argument("--no-ablations", action="store_true",
                    help="evaluate the trained network only (no untrained / mean-state starts)")
    args = ap.parse_args(argv)
    import torch

    from .nn import WarmStartNet, init_params
    from .solver import Solver
    g = Grid(args.nr, args.nt, args.nph)
    t_ref = args.crossings * relax.slow_crossing_time(g)
    lo, hi = default_window(g)
    lo = lo if args.phi_lo is None else args.phi_lo
    hi = hi if args.phi_hi is None else args.phi_hi
    dims = (g.nt, g.np_, g.nr, args.c1, args.c2, args.hidden, lo, hi, args.coord)
    src = args.weights or args.init_weights
    p_widened = None
    if src:
        dims = full_dims(np.load(src)["dims"])
        assert dims[:3] == (g.nt, g.np_, g.nr), "weights for another grid"
        if (args.widen or args.coord > dims[8]) and not args.weights:
            w1, w2, wh = ((int(v) for v in args.widen.split(",")) if args.widen
                          else dims[3:6])
            p_widened, dims = widen_params(np.load(src)["params"], dims, w1, w2, wh,
                                           coord=max(args.coord, dims[8]))
    net = WarmStartNet.from_dims(dims, batch_max=8)
    p0 = init_params(*net.dims, seed=0)
    probe = Solver(g)
    rc, thc = grid_geometry(probe)
    probe.close()
    report = dict(grid=[g.nr, g.nt, g.np_], t_ref_days=t_ref / 86400, params=int(net.nparam),
                  dims=list(net.dims))
    mean_t = None
    if args.weights:
        w = np.load(args.weights)
        p = w["params"]
        if "mean_target" in w.files:
            mean_t = torch.from_numpy(w["mean_target"]).cuda()
    else:
        train_seeds = list(range(args.train_seed0, args.train_seed0 + args.train))
        t0 = time.perf_counter()
        t_data = t_ref if args.data_crossings is None else \
            args.data_crossings * relax.slow_crossing_time(g)
        report["data_t_days"] = t_data / 86400
        X, T, _ = build_dataset(net, g, train_seeds, t_data, rc, thc, args.data_precision,
                                args.ens_batch)
        report["dataset_seconds"] = time.perf_counter() - t0
        if not args.no_ablations:
            mean_t = T.mean(dim=0)
        p_init = np.load(args.init_weights)["params"] if args.init_weights else p0
        if p_widened is not None:
            p_init = p_widened
        report["widen"] = args.widen
        report["coord"] = net.dims[8]
        osc = np.ones(8 * g.nr)
        osc[0::8] = math.sqrt(args.rho_weight)
        rc_au = rc.cpu().numpy() / synth.AU
        osc.reshape(g.nr, 8)[rc_au > args.outer_au] *= math.sqrt(args.outer_weight)
        weighted = args.rho_weight != 1.0 or args.outer_weight != 1.0
        if weighted:
            T *= torch.from_numpy(osc.astype(np.float32)).cuda()
            p_init = scale_output(p_init, net.dims, osc)
        net.set_params(p_init)
        report["init_weights"] = args.init_weights
        report["rho_weight"] = args.rho_weight
        report["outer_weight"] = [args.outer_weight, args.outer_au]
        report["train_samples"] = int(X.shape[0])
        hist, tsec = train(net, X, T, args.epochs, lr=args.lr)
        report.update(train_loss=hist, train_seconds=tsec)
        p = net.get_params()
        if weighted:
            p = scale_output(p, net.dims, 1.0 / osc)
        if args.out:
            extra = {} if mean_t is None else {"mean_target": mean_t.cpu().numpy()}
            np.savez(args.out, params=p, dims=np.array(net.dims), **extra)
        del X, T
        torch.cuda.empty_cache()
    preds = {}

    def with_params(params):
        def f(x):
            net.set_params(params)
            return net.forward(x)
        return f
    preds["warm"] = with_params(p)
    if not args.no_ablations:
        preds["untrained"] = with_params(p0)
        if mean_t is not None:
            preds["mean_target"] = lambda x: mean_t
    if args.test == 0:
        if args.report:
            json.dump(report, open(args.report, "w"), indent=1, default=float)
        return report
    test_seeds = list(range(args.test_seed0, args.test_seed0 + args.test))
    cache = PlainCache(args.plain_cache, g, t_ref) if args.plain_cache else None
    rows = evaluate(net, g, test_seeds, t_ref, preds, cache=cache)
    report["summary"] = summarise(rows, list(preds))
    report["rows"] = rows
    log(json.dumps(report["summary"], indent=1))
    if args.report:
        json.dump(report, open(args.report, "w"), indent=1, default=float)
    return report


if __name__ == "__main__":
    main()

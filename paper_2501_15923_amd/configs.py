"""Workload presets (synthetic stand-ins for the paper's coronal-model driven
runs; see synth.py for how each input is drawn).

  tiny_static   64 x 16 x 32 cells, one static map, 200 RK2 steps, CFL 0.4
  prod_dynamic  600 x 60 x 120 cells, 10 maps 6 h apart, 3 simulated days,
                4 probe trajectories
  prod_cme      prod_dynamic plus one cone CME (1000 km/s, 30 deg, 8 h)
  jupiter_dynamic  outer boundary 5.5 AU (802 x 60 x 120), hourly maps to be
                streamed into a small map buffer
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import synth
from .synth import DAY, HOUR, Grid


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    times: np.ndarray      # [n_maps] s
    maps: np.ndarray       # [n_maps][8][nt][np] SI primitives
    cmes: np.ndarray       # [n_cme][8]
    probes: np.ndarray | None  # [n][npts][4]
    steps: int
    t_end: float           # s, <= 0: none
    gamma: float = 1.5
    omega: float = synth.OMEGA_SUN
    cfl: float = 0.4
    probe_cadence: float = 0.0  # s; 0: every step


def tiny_static(seed: int = 0) -> Workload:
    g = Grid(64, 16, 32)
    m = synth.static_map(g, seed)[None]
    return Workload("tiny_static_64x16x32", g, np.zeros(1), m,
                    np.zeros((0, 8)), None, 200, -1.0)


# The map variant the workloads use by default: rho v_r^2 constant with
# 300 cm^-3 in the 700 km/s fast wind (1200 cm^-3 at 350 km/s) and
# B_r = +-150 nT, plasma beta >= 0.36 at 0.1 AU.  CONFIGURED_MAPS is the
# thinner, stronger-field variant (300 cm^-3 at 350 km/s, 75 cm^-3 in the
# fast wind, +-250 nT, beta 0.085 in the fast wind).
DEFAULT_MAPS = "150 nT, 300 cm^-3 fast / 1200 cm^-3 slow wind, 1 MK"
CONFIGURED_MAPS = dict(b_r=250e-9, n_fast=75e6)
CONFIGURED_MAPS_NAME = "250 nT, 75 cm^-3 fast / 300 cm^-3 slow wind, 1 MK"


def prod_dynamic(seed: int = 1, nr: int = 600, nt: int = 60, nph: int = 120,
                 configured_maps: bool = False) -> Workload:
    g = Grid(nr, nt, nph)
    times, maps = synth.dynamic_maps(g, seed, **(CONFIGURED_MAPS if configured_maps else {}))
    probes = synth.probe_tables(3 * DAY, seed)
    return Workload(f"prod_dynamic_{nr}x{nt}x{nph}", g, times, maps,
                    np.zeros((0, 8)), probes, 0, 3 * DAY)


def prod_cme(seed: int = 2, nr: int = 600, nt: int = 60, nph: int = 120,
             configured_maps: bool = False) -> Workload:
    w = prod_dynamic(1, nr, nt, nph, configured_maps)
    cme = synth.cone_cme(seed, w.probes[1])
    w.name = f"prod_cme_{nr}x{nt}x{nph}"
    w.cmes = cme[None]
    w.probe_cadence = 600.0
    return w


JUPITER_AU = 5.5


def jupiter_dynamic(seed: int = 3, days: float = 2.0, cadence: float = HOUR, nt: int = 60,
                    nph: int = 120) -> Workload:
    """Domain extended to beyond Jupiter's orbit (outer boundary 5.5 AU), with
    the radial stretching of the production grid (803 cells from 0.1 to
    5.5 AU, the ratio of successive edges of 600 cells over 0.1-2 AU) and a
    map every `cadence` seconds over `days`, meant to be streamed into a
    small map buffer.  Probes: Venus-, Earth- and Mars-like circular orbits
    (0.72, 1.0, 1.52 AU) and Jupiter's (5.2 AU)."""
    import math
    nr = int(round(600 * math.log(JUPITER_AU / 0.1) / math.log(20.0)))
    g = Grid(nr, nt, nph, r_out=JUPITER_AU * synth.AU)
    n_maps = int(round(days * DAY / cadence)) + 1
    times, maps = synth.dynamic_maps(g, seed, n_maps=n_maps, cadence=cadence)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2 * math.pi, 4)
    t_end = days * DAY
    probes = np.ascontiguousarray(np.stack([
        synth.orbit_table(t_end, 600.0, a * synth.AU, 0.0, p)
        for a, p in zip((0.72, 1.0, 1.52, 5.2), ph)]))
    return Workload(f"jupiter_dynamic_{nr}x{nt}x{nph}", g, times, maps, np.zeros((0, 8)),
                    probes, 0, t_end, probe_cadence=600.0)

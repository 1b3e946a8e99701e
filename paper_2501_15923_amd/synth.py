"""Seeded synthetic inputs: 0.1 AU boundary maps, spacecraft trajectories and
cone-CME parameters, all in SI units.

These stand in for the coronal-model boundary files, trajectory files and CME
catalogue entries that drive the heliospheric model (Icarus 3.0, Sect. 2.1
boundary data, Sect. 2 trajectory files, Sect. 3.2 Table 2 cone CMEs).  The
module only *produces input data*; it holds no part of the MHD update, and
both the HIP library and the CPU oracle read its output.

Map channel order (primitive variables, as the lookup-table boundary uses,
Sect. 2.1): rho [kg/m^3], v_r, v_theta, v_phi (co-rotating frame) [m/s],
p [Pa], B_r, B_theta, B_phi [T].  Layout [8][n_theta][n_phi].
Angles: theta is colatitude, phi longitude in the co-rotating frame.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

AU = 1.495978707e11
M_PROTON = 1.67262192369e-27
K_BOLTZ = 1.380649e-23
GM_SUN = 1.32712440018e20
OMEGA_SUN = 2.87e-6  # equatorial rotation rate [rad/s] used for every preset
HOUR = 3600.0
DAY = 86400.0
DEG = math.pi / 180.0


@dataclasses.dataclass(frozen=True)
class Grid:
    """Solver grid: n_r x n_theta x n_phi active cells, radially stretched
    from r_in to r_out, colatitude th_min..th_max, full periodic longitude."""
    nr: int
    nt: int
    np_: int
    r_in: float = 0.1 * AU
    r_out: float = 2.0 * AU
    th_min: float = 30.0 * DEG
    th_max: float = 150.0 * DEG

    @property
    def cells(self) -> int:
        return self.nr * self.nt * self.np_


def angle_centres(g: Grid):
    """Uniform colatitude and longitude cell centres (radians)."""
    dth = (g.th_max - g.th_min) / g.nt
    th = g.th_min + (np.arange(g.nt) + 0.5) * dth
    dph = 2.0 * math.pi / g.np_
    ph = (np.arange(g.np_) + 0.5) * dph
    return th, ph


def wind_map(g: Grid, tilt: float, phi0: float, half_width: float = 15 * DEG,
             transition: float = 5 * DEG, v_slow: float = 350e3,
             v_fast: float = 700e3, n_fast: float = 300e6, temp: float = 1e6,
             b_r: float = 150e-9, omega: float = OMEGA_SUN) -> np.ndarray:
    """Bimodal wind around a tilted current sheet.

    The sheet is the great circle normal to n = (sin a cos p0, sin a sin p0,
    cos a); d = asin(x.n) is the signed angular distance to it.  Slow wind
    (v_slow) within +-half_width of the sheet, fast wind outside, joined by
    a tanh of the given width; density n_fast (v_fast / v_r)^2 (rho v_r^2
    constant: 300 cm^-3 in the fast and 1200 cm^-3 in the slow wind by
    default, the plasma beta at 0.1 AU staying above ~0.3);
    p = 2 n k_B T (fully ionised hydrogen); B_r = +b_r where d >= 0 and -b_r
    elsewhere; the transverse field and velocity follow the Parker relation
    at the inner radius (plasma not rotating in the inertial frame, field
    aligned with the co-rotating flow): v_phi' = -Omega r sin(theta),
    B_phi = B_r v_phi' / v_r, v_theta = B_theta = 0."""
    th, ph = angle_centres(g)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    nx = math.sin(tilt) * math.cos(phi0)
    ny = math.sin(tilt) * math.sin(phi0)
    nz = math.cos(tilt)
    dot = np.sin(TH) * np.cos(PH) * nx + np.sin(TH) * np.sin(PH) * ny + np.cos(TH) * nz
    d = np.arcsin(np.clip(dot, -1.0, 1.0))
    s = 0.5 * (1.0 + np.tanh((np.abs(d) - half_width) / transition))
    vr = v_slow + (v_fast - v_slow) * s
    n = n_fast * (v_fast / vr) ** 2
    out = np.zeros((8, g.nt, g.np_))
    out[0] = M_PROTON * n
    out[1] = vr
    out[3] = -omega * g.r_in * np.sin(TH)
    out[4] = 2.0 * n * K_BOLTZ * temp
    out[5] = np.where(d >= 0.0, b_r, -b_r)
    out[7] = out[5] * out[3] / vr
    return out


def monopole_map(g: Grid, v: float = 500e3, n: float = 100e6, temp: float = 1e6,
                 b_r: float = 100e-9, omega: float = OMEGA_SUN) -> np.ndarray:
    """Uniform, axisymmetric, single-polarity wind (Parker-spiral test)."""
    th, _ = angle_centres(g)
    out = np.zeros((8, g.nt, g.np_))
    out[0] = M_PROTON * n
    out[1] = v
    out[3] = (-omega * g.r_in * np.sin(th))[:, None]
    out[4] = 2.0 * n * K_BOLTZ * temp
    out[5] = b_r
    out[7] = out[5] * out[3] / v
    return out


def static_map(g: Grid, seed: int, tilt: float = 20 * DEG,
               omega: float = OMEGA_SUN) -> np.ndarray:
    """One static map: tilt 20 deg, current-sheet phase drawn U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    return wind_map(g, tilt, phi0, omega=omega)


def relax_map(g: Grid, seed: int, omega: float = OMEGA_SUN) -> np.ndarray:
    """Static map for relaxation studies: tilt ~ U[0, 40] deg, slow-band
    half-width 15 deg * U[0.8, 1.2], sheet phase ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    tilt = rng.uniform(0.0, 40.0) * DEG
    hw = 15.0 * DEG * rng.uniform(0.8, 1.2)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    return wind_map(g, tilt, phi0, half_width=hw, omega=omega)


def dynamic_maps(g: Grid, seed: int, n_maps: int = 10, cadence: float = 6 * HOUR,
                 tilt_max: float = 40 * DEG, width_var: float = 0.2,
                 omega: float = OMEGA_SUN, **wind):
    """Map sequence: tilt drifting linearly 0..tilt_max, slow-band half-width
    15 deg * (1 + width_var * u_k), u_k ~ U[-1, 1]; fixed sheet phase; extra
    keywords (b_r, n_fast, ...) go to wind_map.
    Returns (times [s], maps [n][8][nt][np])."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    u = rng.uniform(-1.0, 1.0, n_maps)
    times = np.arange(n_maps) * cadence
    maps = np.stack([
        wind_map(g, tilt_max * k / max(n_maps - 1, 1), phi0,
                 half_width=15 * DEG * (1.0 + width_var * u[k]), omega=omega, **wind)
        for k in range(n_maps)])
    return times, maps


def kepler_E(M: np.ndarray, e: float) -> np.ndarray:
    """Eccentric anomaly from E - e sin E = M by Newton iteration."""
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(60):
        f = E - e * np.sin(E) - M
        E = E - f / (1.0 - e * np.cos(E))
    return E


def orbit_table(t_end: float, cadence: float, a: float, e: float = 0.0,
                phase: float = 0.0, t0: float = 0.0) -> np.ndarray:
    """(t, r, theta, phi_inertial) rows of an in-ecliptic (theta = 90 deg)
    Keplerian orbit about the Sun, phi unwrapped.  Covers [t0, t_end]."""
    npts = int(math.ceil((t_end - t0) / cadence)) + 1
    t = t0 + np.arange(npts) * cadence
    n_mean = math.sqrt(GM_SUN / a ** 3)
    M = phase + n_mean * t
    if e == 0.0:
        r = np.full_like(t, a)
        phi = M
    else:
        E = kepler_E(np.mod(M, 2 * np.pi), e)
        r = a * (1.0 - e * np.cos(E))
        nu = 2.0 * np.arctan2(math.sqrt(1 + e) * np.sin(E / 2),
                              math.sqrt(1 - e) * np.cos(E / 2))
        phi = np.unwrap(nu)
        phi = phi + (M[0] - np.mod(M[0], 2 * np.pi))
    out = np.stack([t, r, np.full_like(t, math.pi / 2), phi], axis=1)
    return out


def probe_tables(t_end: float, seed: int, cadence: float = 600.0) -> np.ndarray:
    """Four trajectories: circular orbits at 0.72, 1.0 and 1.52 AU and an
    e = 0.3 orbit with a = 1 AU, seeded phases.  [4][npts][4]."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2 * math.pi, 4)
    rows = [orbit_table(t_end, cadence, 0.72 * AU, 0.0, ph[0]),
            orbit_table(t_end, cadence, 1.00 * AU, 0.0, ph[1]),
            orbit_table(t_end, cadence, 1.52 * AU, 0.0, ph[2]),
            orbit_table(t_end, cadence, 1.00 * AU, 0.3, ph[3])]
    return np.ascontiguousarray(np.stack(rows))


def cone_cme(seed: int, earth_table: np.ndarray, t_start: float = 12 * HOUR,
             duration: float = 8 * HOUR, speed: float = 1000e3,
             half_width: float = 30 * DEG, rho: float = 1e-18, temp: float = 0.8e6,
             omega: float = OMEGA_SUN, spread: float = 20 * DEG) -> np.ndarray:
    """One cone CME row (t_start, duration, latitude, co-rotating longitude,
    half-width, speed, density, temperature), SI.  Its axis is drawn within
    +-spread of the Earth probe's co-rotating longitude at t_start."""
    rng = np.random.default_rng(seed)
    lat = rng.uniform(-spread, spread)
    dlon = rng.uniform(-spread, spread)
    t = earth_table[:, 0]
    phi_e = np.interp(t_start, t, earth_table[:, 3])
    lon = math.fmod(phi_e - omega * t_start + dlon, 2 * math.pi)
    if lon < 0:
        lon += 2 * math.pi
    return np.array([t_start, duration, lat, lon, half_width, speed, rho, temp])


def ensemble_members(n_runs: int = 64, seed0: int = 100, grid: Grid | None = None):
    """Uneven ensemble: per run a grid with n_r ~ U{150..600},
    n_theta ~ U{30..60}, n_phi ~ U{60..120} (or the given grid for every
    run), a 10-map sequence and one cone CME with speed U[500, 2000] km/s
    and half-width U[15, 45] deg."""
    runs = []
    for q in range(n_runs):
        seed = seed0 + q
        rng = np.random.default_rng(seed)
        nr = int(rng.integers(150, 601))
        nt = int(rng.integers(30, 61))
        nph = int(rng.integers(60, 121))
        speed = rng.uniform(500e3, 2000e3)
        hw = rng.uniform(15 * DEG, 45 * DEG)
        g = Grid(nr, nt, nph) if grid is None else grid
        times, maps = dynamic_maps(g, seed)
        earth = orbit_table(3 * DAY, 600.0, AU, 0.0, rng.uniform(0, 2 * math.pi))
        cme = cone_cme(seed, earth, speed=speed, half_width=hw)
        runs.append(dict(seed=seed, grid=g, times=times, maps=maps, cme=cme))
    return runs

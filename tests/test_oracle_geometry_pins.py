"""Pins of the oracle's spherical source terms, fast speed, CFL rule and the
antisymmetric ('asymm') transverse inner boundary, each against something
the mathematics fixes:

- any uniform state written in Cartesian components (uniform rho, p, v, B,
  with v and B neither radial nor parallel) is an exact steady state of the
  ideal-MHD equations (Sect. 2, Eqs. 1-6 with Omega = g = 0).  In spherical
  components every geometric source term of the momentum and induction
  equations is non-zero for it, so the discrete drift must vanish at second
  order under refinement; a wrong sign or factor in any one term leaves an
  O(1) drift;
- the largest wave speed of the one-dimensional ideal-MHD system along a
  direction n is the spectral radius of its flux Jacobian dF_n/dU.  The
  Jacobian is differentiated numerically from the oracle's own (consistent)
  flux, so the check does not depend on how the oracle writes c_f.  The
  TVD-Lax-Friedrichs dissipation coefficient and the CFL rate must equal it;
- the 'asymm' boundary makes the transverse quantities vanish on the
  boundary surface: ghost values are the negated mirror images of the
  active cells about r_in, so every symmetric reconstruction gives opposite
  face states there.
"""
import math

import numpy as np
import pytest

from paper_2501_15923_amd import synth

AU = synth.AU


# ------------------------------------------------------------ uniform state --

V_CART = np.array([0.8, 0.3, -0.5])   # code units (100 km/s)
B_CART = np.array([0.2, 0.9, 0.4])    # code units, not parallel to V_CART
RHO, PRES = 4.0, 1.0


def _sph_components(vec, th, ph):
    """Spherical (r, theta, phi) components of a constant Cartesian vector."""
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    vr = vec[0] * st * cp + vec[1] * st * sp + vec[2] * ct
    vt = vec[0] * ct * cp + vec[1] * ct * sp - vec[2] * st
    vp = -vec[0] * sp + vec[1] * cp
    return vr, vt, vp


def _padded_centres(o, ng=2):
    re, te, pe = o.edges()
    q = re[1] / re[0]
    r_ext = np.concatenate([re[0] * q ** np.arange(-ng, 0), re,
                            re[-1] * q ** np.arange(1, ng + 1)])
    rc = 0.5 * (r_ext[1:] + r_ext[:-1])
    dth, dph = te[1] - te[0], pe[1] - pe[0]
    th = te[0] + (np.arange(-ng, len(te) - 1 + ng) + 0.5) * dth
    ph = (np.arange(-ng, len(pe) - 1 + ng) + 0.5) * dph
    return rc, th, ph


def _uniform_cartesian_padded(orc, o, gamma=1.5):
    rc, th, ph = _padded_centres(o)
    TH = th[None, :, None] * np.ones((len(ph), 1, len(rc)))
    PH = ph[:, None, None] * np.ones((1, len(th), len(rc)))
    v = _sph_components(V_CART, TH, PH)
    b = _sph_components(B_CART, TH, PH)
    U = np.zeros(o.padded_shape)
    U[0] = RHO
    for d in range(3):
        U[1 + d] = RHO * v[d]
        U[5 + d] = b[d]
    kin = 0.5 * RHO * float(V_CART @ V_CART)
    mag = 0.5 * float(B_CART @ B_CART)
    U[4] = PRES / (gamma - 1.0) + kin + mag
    return U


def _uniform_residual(orc, n):
    """Mean |dU/dt| over the active cells for the uniform Cartesian state,
    per group (rho, momentum, energy, field), ghosts frozen at the exact
    solution.  dU/dt is read from one step of length 1e-7 code units."""
    o = orc.Oracle(12 * n, 8 * n, 12 * n, gravity=False, corot=False, omega=0.0,
                   bc_mode=orc.BCM_FROZEN, limiter=orc.LIM_MC)
    U0 = _uniform_cartesian_padded(orc, o)
    o.set_state(U0, kind=orc.CONS_PADDED)
    delta = 1e-7
    info = o.step(1, t_end=delta * orc.units()["t"])
    assert info["status"] == 0
    U = o.get_state(kind=orc.CONS_PADDED)
    act = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    L = np.abs(U[act] - U0[act]) / delta
    return np.array([L[0].mean(), L[1:4].mean(), L[4].mean(), L[5:8].mean()])


def test_uniform_cartesian_state_is_steady_on_the_sphere(orc):
    """Uniform rho, p, v and B (v not parallel to B, both oblique to every
    grid direction) are a steady state: the curvature terms of rho v v - B B
    and of v B - B v cancel the metric part of the flux divergence.  The
    discrete rate of change is a truncation error that shrinks under
    refinement (second order in smooth cells; the limiter clips at the
    extrema of the spherical components, which leaves first order in the
    mean).  A wrong sign or factor in any one source term leaves a rate of
    order rho v^2 / r that does not shrink."""
    res = [_uniform_residual(orc, n) for n in (1, 2, 4)]
    groups = ("rho", "m", "e", "B")
    for g in range(4):
        assert res[0][g] / res[2][g] > 4.0, (groups[g], res)
        assert res[1][g] / res[2][g] > 2.0, (groups[g], res)


# ------------------------------------------------------- wave-speed pins --

def _cons(w, gamma):
    u = np.array(w, dtype=float)
    u[1:4] = w[0] * w[1:4]
    u[4] = w[4] / (gamma - 1.0) + 0.5 * w[0] * np.dot(w[1:4], w[1:4]) + \
        0.5 * np.dot(w[5:8], w[5:8])
    return u


def _prim(u, gamma):
    w = np.array(u, dtype=float)
    w[1:4] = u[1:4] / u[0]
    w[4] = (gamma - 1.0) * (u[4] - 0.5 * np.dot(u[1:4], u[1:4]) / u[0]
                            - 0.5 * np.dot(u[5:8], u[5:8]))
    return w


def _spectral_radius(o, w, n, gamma):
    """max |eigenvalue| of dF_n/dU at primitive state w, the Jacobian taken
    by central differences of the oracle's consistent flux F(w, w)."""
    u0 = _cons(w, gamma)
    J = np.zeros((8, 8))
    for q in range(8):
        h = 1e-6 * max(1.0, abs(u0[q]))
        up, um = u0.copy(), u0.copy()
        up[q] += h
        um[q] -= h
        wp, wm = _prim(up, gamma), _prim(um, gamma)
        J[:, q] = (o.face_flux(wp, wp, n) - o.face_flux(wm, wm, n)) / (2 * h)
    return float(np.max(np.abs(np.linalg.eigvals(J))))


def _oblique_state(rho, bmag, angle_deg, n, vn=0.3):
    """Primitive state with |B| = bmag at angle_deg to direction n (1..3)."""
    w = np.zeros(8)
    w[0] = rho
    w[4] = 0.7
    a = math.radians(angle_deg)
    t1, t2 = [d for d in (1, 2, 3) if d != n]
    w[n] = vn
    w[t1], w[t2] = -0.2, 0.15
    w[4 + n] = bmag * math.cos(a)
    w[4 + t1] = bmag * math.sin(a) * 0.8
    w[4 + t2] = bmag * math.sin(a) * 0.6
    return w


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("rho,angle", [(4.0, 40.0), (0.3, 65.0), (9.0, 10.0)])
def test_tvdlf_dissipation_is_the_flux_jacobian_spectral_radius(orc, n, rho, angle):
    gamma = 1.5
    o = orc.Oracle(4, 4, 4, gravity=False, corot=False, flux=orc.FLUX_TVDLF,
                   gamma=gamma)
    wl = _oblique_state(rho, 1.3, angle, n)
    wr = wl.copy()
    wr[0] *= 1.0 + 1e-7  # nudge the density only: alpha is read from F_rho
    fl, fr = o.face_flux(wl, wl, n), o.face_flux(wr, wr, n)
    fs = o.face_flux(wl, wr, n)
    du = _cons(wr, gamma)[0] - _cons(wl, gamma)[0]
    alpha = -2.0 * (fs[0] - 0.5 * (fl[0] + fr[0])) / du
    expect = max(_spectral_radius(o, wl, n, gamma), _spectral_radius(o, wr, n, gamma))
    assert abs(alpha / expect - 1.0) < 1e-5, (alpha, expect)


def test_cfl_rate_uses_the_spectral_radius_and_cell_widths(orc):
    """dt = CFL / max over cells of sum_d rho(J_d)/dx_d with dx = dr,
    r dtheta, r sin(theta) dphi, all recomputed here from the edges and the
    differentiated flux Jacobian.  The phi width binds at the colatitude
    edges, where sin(theta) = 1/2."""
    gamma, cfl = 1.5, 0.4
    nr, nt, nph = 5, 6, 8
    o = orc.Oracle(nr, nt, nph, gravity=False, corot=False, cfl=cfl, gamma=gamma)
    rng = np.random.default_rng(7)
    W = np.zeros(o.shape)
    W[0] = rng.uniform(0.5, 8.0, W[0].shape)
    W[1] = rng.uniform(2.0, 6.0, W[0].shape)
    W[2] = rng.uniform(-0.5, 0.5, W[0].shape)
    W[3] = rng.uniform(-3.0, 3.0, W[0].shape)
    W[4] = rng.uniform(0.2, 2.0, W[0].shape)
    for v in (5, 6, 7):
        W[v] = rng.uniform(-2.0, 2.0, W[0].shape)
    o.set_state(W, kind=3)
    re, te, pe = o.edges()
    rc = 0.5 * (re[1:] + re[:-1])
    thc = 0.5 * (te[1:] + te[:-1])
    dth, dph = te[1] - te[0], pe[1] - pe[0]
    rates = np.zeros((nph, nt, nr))
    phi_part = np.zeros_like(rates)
    for k in range(nph):
        for j in range(nt):
            for i in range(nr):
                w = W[:, k, j, i]
                dx = (re[i + 1] - re[i], rc[i] * dth, rc[i] * math.sin(thc[j]) * dph)
                terms = [_spectral_radius(o, w, d + 1, gamma) / dx[d] for d in range(3)]
                rates[k, j, i] = sum(terms)
                phi_part[k, j, i] = terms[2]
    dt_expect = cfl / rates.max() * orc.units()["t"]
    assert abs(o.dt() / dt_expect - 1.0) < 1e-6, (o.dt(), dt_expect)
    # the binding cell sits on a colatitude edge row and its phi term is a
    # large part of the rate, so dx_phi without sin(theta) would change dt
    kb, jb, ib = np.unravel_index(np.argmax(rates), rates.shape)
    assert jb in (0, nt - 1)
    assert phi_part[kb, jb, ib] > 0.3 * rates[kb, jb, ib]


# ------------------------------------------------------------ asymm pins --

def test_asymm_transverse_inner_boundary(orc):
    """Sect. 2.1: v_theta, v_phi, B_theta, B_phi get the 'asymm' rule at
    0.1 AU.  The ghost values mirror the active cells about r_in with the
    sign flipped, so the minmod face states on both sides of r_in are
    exact negatives (the transverse value on the face is zero), while rho,
    v_r, p and B_r keep the map value in every ghost layer."""
    g = synth.Grid(8, 6, 8)
    o = orc.Oracle(g.nr, g.nt, g.np_, bc_transverse=orc.BCT_ASYMM)
    m = synth.wind_map(g, 20 * synth.DEG, 0.7)
    o.set_maps(np.zeros(1), m[None])
    rng = np.random.default_rng(3)
    W = np.zeros(o.shape)
    W[0] = rng.uniform(1e-21, 5e-21, W[0].shape)
    W[1] = rng.uniform(3e5, 7e5, W[0].shape)
    W[2:4] = rng.uniform(-5e4, 5e4, W[2:4].shape)
    W[4] = rng.uniform(1e-10, 1e-9, W[0].shape)
    W[5:8] = rng.uniform(-1e-7, 1e-7, W[5:8].shape)
    o.set_state(W)
    U = o.fill_ghosts(0.0)
    u = orc.units()
    gam = 1.5
    rho = U[0]
    with np.errstate(invalid="ignore", divide="ignore"):  # unfilled corners
        v = U[1:4] / rho
        p = (gam - 1.0) * (U[4] - 0.5 * rho * np.sum(v * v, axis=0)
                           - 0.5 * np.sum(U[5:8] ** 2, axis=0))
    Wp = np.stack([rho, v[0], v[1], v[2], p, U[5], U[6], U[7]])
    act = (slice(2, -2), slice(2, -2))
    sc = [u["rho"], u["v"], u["v"], u["v"], u["p"], u["B"], u["B"], u["B"]]
    for var in (0, 1, 4, 5):
        want = m[var].T[:, :] / sc[var]  # map [nt][np] -> [np][nt]
        for gl in (0, 1):  # padded index of ghost layers 2 and 1
            got = Wp[var][act + (gl,)]
            assert np.allclose(got, want, rtol=1e-12, atol=0), var
    for var in (2, 3, 6, 7):
        col = Wp[var][act]  # [np][nt][nr + 4]
        g2, g1, c0, c1 = col[..., 0], col[..., 1], col[..., 2], col[..., 3]

        def mm(a, b):
            return np.where(a * b <= 0, 0.0, np.where(np.abs(a) < np.abs(b), a, b))
        wl = g1 + 0.5 * mm(g1 - g2, c0 - g1)
        wr = c0 - 0.5 * mm(c0 - g1, c1 - c0)
        scale = np.max(np.abs(col))
        assert np.max(np.abs(wl + wr)) <= 1e-14 * scale, var
        assert np.max(np.abs(g1 + c0)) <= 1e-14 * scale, var
        assert np.max(np.abs(c0)) > 0.1 * scale  # the check is not vacuous

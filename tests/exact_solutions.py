"""Closed-form and textbook reference solutions used to pin the CPU oracle.

- Exact Riemann solver for the 1D Euler equations (ideal gas), written from
  the standard two-wave pressure-function method (Toro, "Riemann Solvers and
  Numerical Methods for Fluid Dynamics", ch. 4): solve f_L(p*) + f_R(p*) +
  u_R - u_L = 0 by Newton iteration, then sample the self-similar solution.
- Rankine-Hugoniot jump for a fast MHD shock with B perpendicular to the
  normal: the jump reduces to gas dynamics with total pressure p + B^2/2 and
  B/rho conserved (Heaviside-Lorentz units, mu0 = 1).
- Circularly polarised Alfven wave: an exact nonlinear travelling solution.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, g):
    """Pressure function f_K and its derivative for one side."""
    ak = math.sqrt(g * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * ak / (g - 1.0) * (r - 1.0), 1.0 / (rho * ak) * (p / pk) ** (-(g + 1.0) / (2.0 * g))


def riemann_star(rl, ul, pl, rr, ur, pr, g):
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _fk(p, rl, pl, g)
        fr, dr = _fk(p, rr, pr, g)
        f = fl + fr + ur - ul
        pn = max(1e-12, p - f / (dl + dr))
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, g)
    fr, _ = _fk(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(rl, ul, pl, rr, ur, pr, g, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0) / t."""
    ps, us = riemann_star(rl, ul, pl, rr, ur, pr, g)
    out = np.zeros((3, len(xi)))
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:
                sl = ul - al * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    rs = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                    w = (rs, us, ps)
            else:
                shl = ul - al
                asl = al * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - asl
                if s <= shl:
                    w = (rl, ul, pl)
                elif s >= stl:
                    w = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (al + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (al + (g - 1) / 2 * (ul - s))
                    r = rl * (c / al) ** (2 / (g - 1))
                    w = (r, u, pl * (c / al) ** (2 * g / (g - 1)))
        else:
            if ps > pr:
                sr = ur + ar * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    rs = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                    w = (rs, us, ps)
            else:
                shr = ur + ar
                asr = ar * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + asr
                if s >= shr:
                    w = (rr, ur, pr)
                elif s <= str_:
                    w = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (ar - (g - 1) / 2 * (ur - s))
                    r = rr * (c / ar) ** (2 / (g - 1))
                    w = (r, u, pr * (c / ar) ** (2 * g / (g - 1)))
        out[:, n] = w
    return out


def perpendicular_shock(rho1, p1, b1, X, g):
    """Upstream (rho1, u=0, p1, B1 perpendicular) at rest; compression
    X = rho2/rho1.  Returns (shock speed s, rho2, u2, p2, B2).

    Shock-frame normal speeds w1 = -s, w2 = w1/X.  Mass and flux freezing
    give B2 = X B1.  Momentum gives p2 = p1 + rho1 w1^2 (1 - 1/X) +
    B1^2 (1 - X^2)/2.  Energy per unit mass flux:
    w^2/2 + g p / ((g-1) rho) + B^2/rho is the same on both sides, which is
    linear in w1^2 once p2 is substituted."""
    k = g / (g - 1.0)
    # w1^2 [1/2 - 1/(2X^2) - k (1 - 1/X)/X] = k (p1 + B1^2 (1-X^2)/2)/(X rho1)
    #        - k p1/rho1 + X B1^2/rho1 - B1^2/rho1
    lhs = 0.5 - 0.5 / X ** 2 - k * (1.0 - 1.0 / X) / X
    rhs = (k * (p1 + 0.5 * b1 ** 2 * (1.0 - X ** 2)) / (X * rho1)
           - k * p1 / rho1 + (X - 1.0) * b1 ** 2 / rho1)
    w1sq = rhs / lhs
    s = math.sqrt(w1sq)
    p2 = p1 + rho1 * w1sq * (1.0 - 1.0 / X) + 0.5 * b1 ** 2 * (1.0 - X ** 2)
    return s, X * rho1, s * (1.0 - 1.0 / X), p2, X * b1

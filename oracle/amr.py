"""Block-structured adaptive mesh refinement of the heliospheric update:
the CPU oracle of the refined-grid path.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): used by tests/ and the
bench's CPU leg; the product library never loads it.  Plain FP64 NumPy
around the C oracle: every block's stage right-hand side (fluxes, geometric
and co-rotation sources, Sect. 2 Eqs. 1-6) comes from orc_rhs on the block's
padded state, whose ghost layers are filled here.

What the paper fixes (Sect. 3.2 and Sect. 4): the 2015 run refines the
radially stretched grid up to five levels; the refinement criteria are
'tracing' (refine where CME material is, from the CME tracer), 'shock'
(refine around compression regions and shocks, from the velocity
divergence) and 'combined' (either); a block is refined when the CME or the
shock is present in it.  The paper runs MPI-AMRVAC; the reading of the
refined grid used here follows that family of codes:

  - blocks of br x bt x bp cells at every level; level 1 is the solver's
    base grid; a level-(l+1) block covers one octant of a level-l block with
    twice the resolution in r, theta and phi (radial edges split at the
    geometric mean, so every level is again a geometric radial grid);
  - one global time step for all levels (dt = CFL / max rate over the leaf
    cells of every level) and SSP-RK2 on the leaves;
  - two ghost layers per block: copies from a leaf of the same level,
    volume-weighted averages (restriction) of the finer leaves, or the
    conservative prolongation of a coarser leaf (minmod-limited linear in
    index space, then a constant correction that makes the 8 children's
    volume-weighted mean equal the coarse cell); physical edges as in the
    uniform solver (inner boundary from the maps, the value of the base
    column containing the cell, the CME tested at the cell's own centre;
    zero gradient at r_out; mirror rows at the colatitude edges; periodic
    phi);
  - flux correction: a coarse cell next to finer leaves takes, for that
    face, the area-weighted sum of the fine face fluxes instead of its own,
    so mass and B_r change only through the domain's outer faces;
  - the passive CME tracer rho*tau rides along as a ninth conserved variable
    (upwind tau times the mass flux, as in the uniform solver);
  - regridding every `regrid_every` steps: a leaf below the top level is
    refined when its criterion holds; the 8 children of a block are merged
    when all are leaves and none meets the criterion; refinement is spread
    so that face neighbours never differ by more than one level, and a merge
    that would break that is skipped; new children are prolongated
    conservatively, merged parents restricted.

Criteria on a leaf block (readings; the paper names them only):
  tracing:  max tau over the block's cells >= tau_thr (default 0.05);
  shock:    max over its cells of -div(V) r / (2 |v_r|) >= shock_thr
            (default 0.5): the flow converges at half the rate or more at
            which a steady radial wind diverges (div V = 2 v_r / r);
  combined: either.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import BCM_FROZEN, CONS_PADDED, Oracle, units

NG = 2  # ghost layers
NVAR = 9  # rho, m_r, m_t, m_p, e, B_r, B_t, B_p, rho*tau


@dataclass
class AmrConfig:
    nr: int
    nt: int
    nph: int
    r_in: float
    r_out: float
    th_min: float
    th_max: float
    br: int = 8
    bt: int = 4
    bp: int = 4
    max_level: int = 2
    criterion: str = "combined"      # tracing | shock | combined
    tau_thr: float = 0.05
    shock_thr: float = 0.5
    regrid_every: int = 5
    gamma: float = 1.5
    omega: float = 2.87e-6
    cfl: float = 0.4
    gravity: bool = True
    corot: bool = True
    flux: int = 0
    limiter: int = 0

    def check(self):
        assert self.nr % self.br == 0 and self.nt % self.bt == 0 and self.nph % self.bp == 0
        assert min(self.br, self.bt, self.bp) >= 4, "blocks of at least 4 cells per side"
        assert self.criterion in ("tracing", "shock", "combined")
        assert self.max_level >= 1


@dataclass
class Level:
    """Geometry of one refinement level (code units)."""
    nr: int
    nt: int
    nph: int
    re: np.ndarray
    te: np.ndarray
    pe: np.ndarray

    @property
    def rc(self):
        return 0.5 * (self.re[1:] + self.re[:-1])

    @property
    def tc(self):
        return 0.5 * (self.te[1:] + self.te[:-1])

    @property
    def pc(self):
        return 0.5 * (self.pe[1:] + self.pe[:-1])


@dataclass
class Block:
    U: np.ndarray                     # [9][bp+4][bt+4][br+4] conservative, code units
    leaf: bool = True
    L: np.ndarray | None = None       # stage right-hand side [9][bp][bt][br]
    faces: dict = field(default_factory=dict)


def minmod(a, b):
    return np.where(a * b <= 0.0, 0.0, np.where(np.abs(a) < np.abs(b), a, b))


class AmrOracle:
    """Refined-grid run.  Maps and CMEs in SI (as for Oracle); the state is
    kept in code units."""

    def __init__(self, cfg: AmrConfig):
        cfg.check()
        self.cfg = cfg
        u = units()
        self.u = u
        self.levels = {}
        for l in range(1, cfg.max_level + 1):
            f = 2 ** (l - 1)
            nr, nt, nph = cfg.nr * f, cfg.nt * f, cfg.nph * f
            r0, r1 = cfg.r_in / u["L"], cfg.r_out / u["L"]
            q = (r1 / r0) ** (1.0 / nr)
            re = r0 * q ** np.arange(nr + 1)
            re[-1] = r1
            te = cfg.th_min + (cfg.th_max - cfg.th_min) * np.arange(nt + 1) / nt
            pe = 2.0 * math.pi * np.arange(nph + 1) / nph
            self.levels[l] = Level(nr, nt, nph, re, te, pe)
        self.blocks: dict[tuple, Block] = {}
        self.oracles: dict[tuple, Oracle] = {}
        self.t = 0.0  # code time
        self.step_count = 0
        self.times = None
        self.maps = None
        self.cmes = np.zeros((0, 8))
        self._bnd = None  # a base-grid oracle for the inner-boundary values

    # ------------------------------------------------------------ set-up --
    def nblocks(self, l):
        lv, c = self.levels[l], self.cfg
        return lv.nr // c.br, lv.nt // c.bt, lv.nph // c.bp

    def set_maps(self, times, maps):
        self.times, self.maps = np.asarray(times, float), np.asarray(maps, float)
        self._boundary_oracle().set_maps(self.times, self.maps)

    def set_cmes(self, rows):
        self.cmes = np.atleast_2d(np.asarray(rows, float))
        self._boundary_oracle().set_cmes(self.cmes)

    def _boundary_oracle(self):
        if self._bnd is None:
            c = self.cfg
            self._bnd = Oracle(c.nr, c.nt, c.nph, r_in=c.r_in, r_out=c.r_out,
                               th_min=c.th_min, th_max=c.th_max, gamma=c.gamma,
                               omega=c.omega, gravity=c.gravity, corot=c.corot, tracer=True)
        return self._bnd

    def init_radial(self):
        """Level-1 leaves from the radial expansion of the first map
        (Sect. 2.1), tracer 0."""
        o = self._boundary_oracle()
        o.init_radial()
        U = o.get_state(kind=1)  # [8][np][nt][nr]
        c = self.cfg
        self.blocks = {}
        nbr, nbt, nbp = self.nblocks(1)
        for bk in range(nbp):
            for bj in range(nbt):
                for bi in range(nbr):
                    P = np.zeros((NVAR, c.bp + 2 * NG, c.bt + 2 * NG, c.br + 2 * NG))
                    P[:8, NG:-NG, NG:-NG, NG:-NG] = U[:, bk * c.bp:(bk + 1) * c.bp,
                                                       bj * c.bt:(bj + 1) * c.bt,
                                                       bi * c.br:(bi + 1) * c.br]
                    self.blocks[(1, bi, bj, bk)] = Block(P)
        self.t = 0.0
        self.step_count = 0

    # --------------------------------------------------------- geometry --
    def cell_volumes(self, key):
        l, bi, bj, bk = key
        lv, c = self.levels[l], self.cfg
        r = lv.re[bi * c.br:(bi + 1) * c.br + 1]
        t = lv.te[bj * c.bt:(bj + 1) * c.bt + 1]
        dph = lv.pe[1] - lv.pe[0]
        vr = (r[1:] ** 3 - r[:-1] ** 3) / 3.0
        vt = np.cos(t[:-1]) - np.cos(t[1:])
        return dph * vt[None, :, None] * vr[None, None, :] * np.ones((c.bp, 1, 1))

    def face_areas(self, key, d, side):
        """Areas of the block's faces on side (0 low, 1 high) along d."""
        l, bi, bj, bk = key
        lv, c = self.levels[l], self.cfg
        r = lv.re[bi * c.br:(bi + 1) * c.br + 1]
        t = lv.te[bj * c.bt:(bj + 1) * c.bt + 1]
        dph = lv.pe[1] - lv.pe[0]
        dth = lv.te[1] - lv.te[0]
        if d == 0:  # [bp][bt]
            rr = r[-1] if side else r[0]
            return np.ones((c.bp, 1)) * (rr * rr * (np.cos(t[:-1]) - np.cos(t[1:])) * dph)[None, :]
        if d == 1:  # [bp][br]
            tt = t[-1] if side else t[0]
            return np.ones((c.bp, 1)) * (math.sin(tt) * 0.5 * (r[1:] ** 2 - r[:-1] ** 2) * dph)[None, :]
        return np.ones((c.bt, 1)) * (0.5 * (r[1:] ** 2 - r[:-1] ** 2) * dth)[None, :]  # [bt][br]

    def block_oracle(self, key):
        if key not in self.oracles:
            l, bi, bj, bk = key
            lv, c = self.levels[l], self.cfg
            L = self.u["L"]
            self.oracles[key] = Oracle(
                c.br, c.bt, c.bp, r_in=lv.re[bi * c.br] * L, r_out=lv.re[(bi + 1) * c.br] * L,
                th_min=lv.te[bj * c.bt], th_max=lv.te[(bj + 1) * c.bt],
                ph_min=lv.pe[bk * c.bp], ph_max=lv.pe[(bk + 1) * c.bp],
                gamma=c.gamma, omega=c.omega, cfl=c.cfl, flux=c.flux, limiter=c.limiter,
                gravity=c.gravity, corot=c.corot, bc_mode=BCM_FROZEN, tracer=True)
        return self.oracles[key]

    # ------------------------------------------------------ tree queries --
    def leaves(self, l=None):
        return sorted(k for k, b in self.blocks.items() if b.leaf and (l is None or k[0] == l))

    def neighbour_key(self, key, d, side):
        """Same-level block key across face (d, side), phi wrapped; None
        beyond the r or theta edges."""
        l, *b = key
        n = list(self.nblocks(l))
        b = list(b)
        b[d] += 1 if side else -1
        if d == 2:
            b[2] %= n[2]
        elif b[d] < 0 or b[d] >= n[d]:
            return None
        return (l, *b)

    def parent(self, key):
        l, bi, bj, bk = key
        return (l - 1, bi // 2, bj // 2, bk // 2)

    def children(self, key):
        l, bi, bj, bk = key
        return [(l + 1, 2 * bi + a, 2 * bj + b, 2 * bk + e)
                for e in (0, 1) for b in (0, 1) for a in (0, 1)]

    # ------------------------------------------- prolongation / restriction --
    def _cell_vol_level(self, l, i, j):
        """Volumes (without dphi) of level-l cells at radial index array i and
        colatitude index array j."""
        lv = self.levels[l]
        vr = (lv.re[i + 1] ** 3 - lv.re[i] ** 3) / 3.0
        vt = np.cos(lv.te[j]) - np.cos(lv.te[j + 1])
        return vr * vt

    def prolong(self, l, Uc, ic, jc):
        """Children of coarse (level l) cells: Uc [9][...][3][3][3] holds each
        coarse cell (centre [1,1,1]) with its face neighbours along phi,
        theta, r; ic, jc the coarse cells' global r / theta indices at level
        l (same leading shape as Uc[0, ..., 0, 0, 0]).  Returns the children
        [9][...][2][2][2] (phi, theta, r sub-index), conservative."""
        c0 = Uc[..., 1, 1, 1]
        sr = minmod(c0 - Uc[..., 1, 1, 0], Uc[..., 1, 1, 2] - c0)
        st = minmod(c0 - Uc[..., 1, 0, 1], Uc[..., 1, 2, 1] - c0)
        sp = minmod(c0 - Uc[..., 0, 1, 1], Uc[..., 2, 1, 1] - c0)
        off = np.array([-0.25, 0.25])
        F = (c0[..., None, None, None] + sp[..., None, None, None] * off[:, None, None]
             + st[..., None, None, None] * off[None, :, None]
             + sr[..., None, None, None] * off[None, None, :])
        # conservative correction with the children's volumes (dphi cancels)
        vf = np.zeros(ic.shape + (2, 2, 2))
        for b in (0, 1):
            for a in (0, 1):
                vf[..., :, b, a] = self._cell_vol_level(l + 1, 2 * ic + a, 2 * jc + b)[..., None]
        vc = vf.sum(axis=(-1, -2, -3))
        mean = (F * vf).sum(axis=(-1, -2, -3)) / vc
        return F + (c0 - mean)[..., None, None, None]

    def restrict(self, l, Uf, i0c, j0c):
        """Coarse (level l) cells from their children Uf [9][...][2][2][2]
        (phi, theta, r sub-index) with the coarse cells' global r / theta
        indices i0c, j0c: volume-weighted mean."""
        vf = np.zeros(i0c.shape + (2, 2, 2))
        for b in (0, 1):
            for a in (0, 1):
                vf[..., :, b, a] = self._cell_vol_level(l + 1, 2 * i0c + a, 2 * j0c + b)[..., None]
        return (Uf * vf).sum(axis=(-1, -2, -3)) / vf.sum(axis=(-1, -2, -3))

    # ------------------------------------------------------------- ghosts --
    def level_value(self, l, i, j, k):
        """Conservative values of level-l cells (global indices, arrays of
        equal shape, all inside the domain) from the leaf that covers each:
        [9][...]."""
        out = np.zeros((NVAR,) + i.shape)
        for idx in np.ndindex(i.shape):
            out[(slice(None),) + idx] = self._value_at(l, int(i[idx]), int(j[idx]), int(k[idx]))
        return out

    def _key(self, l, i, j, k):
        c = self.cfg
        return (l, i // c.br, j // c.bt, k // c.bp)

    def _interior(self, key, i, j, k):
        c = self.cfg
        return self.blocks[key].U[:, NG + k - key[3] * c.bp, NG + j - key[2] * c.bt,
                                  NG + i - key[1] * c.br]

    def _value_at(self, l, i, j, k):
        """A level-l cell from the leaf of level l that holds it, the
        restriction of its 8 children in finer leaves, or the prolongation of
        the coarser leaf that covers it (slopes from that leaf's padded
        array, whose ghost layers are filled first)."""
        c = self.cfg
        key = self._key(l, i, j, k)
        b = self.blocks.get(key)
        if b is not None and b.leaf:
            return self._interior(key, i, j, k)
        if b is not None:
            ch = np.zeros((NVAR, 2, 2, 2))
            for e in (0, 1):
                for bb in (0, 1):
                    for a in (0, 1):
                        fi, fj, fk = 2 * i + a, 2 * j + bb, 2 * k + e
                        fkey = self._key(l + 1, fi, fj, fk)
                        assert self.blocks[fkey].leaf, "children of a face neighbour are leaves"
                        ch[:, e, bb, a] = self._interior(fkey, fi, fj, fk)
            return self.restrict(l, ch, np.array(i), np.array(j))
        ci, cj, ck = i // 2, j // 2, k // 2
        ckey = self._key(l - 1, ci, cj, ck)
        C = self.blocks[ckey]
        assert C.leaf, "a block's face neighbour region is at most one level coarser"
        pi = NG + ci - ckey[1] * c.br
        pj = NG + cj - ckey[2] * c.bt
        pk = NG + ck - ckey[3] * c.bp
        nb = np.zeros((NVAR, 3, 3, 3))
        for dp, dt, dr in ((0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
                           (0, 0, -1), (0, 0, 1)):
            nb[:, dp + 1, dt + 1, dr + 1] = C.U[:, pk + dp, pj + dt, pi + dr]
        F = self.prolong(l - 1, nb, np.array(ci), np.array(cj))
        return F[:, k - 2 * ck, j - 2 * cj, i - 2 * ci]

    def inner_ghost(self, l, j, k, t=None):
        """Conservative inner-ghost value at level l, column (j, k): the map
        (time-interpolated) of the base column that contains it, the cone CME
        tested at this column's centre; tracer 1 inside an inserted cone."""
        t = self.t if t is None else t
        f = 2 ** (l - 1)
        c = self.cfg
        w = self._map_prim(t, j // f, k // f).copy()
        lv = self.levels[l]
        th, ph = lv.tc[j], lv.pc[k]
        inside = 0.0
        for row in self._cme_code():
            t0, dur, colat, lon, cos_hw, v, rho, p = row
            if not (t >= t0 and t < t0 + dur):
                continue
            cosd = math.cos(th) * math.cos(colat) + math.sin(th) * math.sin(colat) * math.cos(ph - lon)
            if cosd >= cos_hw:
                inside = 1.0
                w[0], w[1], w[2] = rho, v, 0.0
                w[3] = -self._omega_code() * self.levels[1].re[0] * math.sin(th)
                w[4] = p
        out = np.zeros(NVAR)
        gam = c.gamma
        out[0] = w[0]
        out[1:4] = w[0] * w[1:4]
        out[4] = w[4] / (gam - 1.0) + 0.5 * w[0] * np.dot(w[1:4], w[1:4]) + 0.5 * np.dot(w[5:8], w[5:8])
        out[5:8] = w[5:8]
        out[8] = inside * w[0]
        return out

    def _omega_code(self):
        return self.cfg.omega * self.u["t"] if self.cfg.corot else 0.0

    def _cme_code(self):
        u = self.u
        rows = []
        for r in self.cmes:
            rows.append((r[0] / u["t"], r[1] / u["t"], 0.5 * math.pi - r[2], r[3],
                         math.cos(r[4]), r[5] / u["v"], r[6] / u["rho"],
                         2.0 * (r[6] / 1.67262192369e-27) * 1.380649e-23 * r[7] / u["p"]))
        return rows

    def _map_prim(self, t, j, k):
        """Time-interpolated map primitive (code units) at base column (j, k)."""
        u = self.u
        sc = np.array([u["rho"], u["v"], u["v"], u["v"], u["p"], u["B"], u["B"], u["B"]])
        tau = self.times / u["t"]
        m = self.maps[:, :, j, k] / sc[None, :]
        if len(tau) == 1 or t <= tau[0]:
            return m[0]
        if t >= tau[-1]:
            return m[-1]
        q = int(np.searchsorted(tau, t, side="right") - 1)
        q = min(q, len(tau) - 2)
        wgt = (t - tau[q]) / (tau[q + 1] - tau[q])
        return (1.0 - wgt) * m[q] + wgt * m[q + 1]

    def fill_ghosts(self, t):
        """Two ghost layers of every leaf, coarse levels first (a fine
        block's prolongated ghosts take slopes from the coarse leaf's
        ghosts)."""
        self.t_ghost = t
        saved = self.t
        self.t = t
        c = self.cfg
        for l in range(1, c.max_level + 1):
            for key in self.leaves(l):
                self._fill_block(key)
        self.t = saved

    def _fill_block(self, key):
        c = self.cfg
        l, bi, bj, bk = key
        lv = self.levels[l]
        b = self.blocks[key]
        P = b.U
        i0, j0, k0 = bi * c.br, bj * c.bt, bk * c.bp
        # faces along r
        for g in range(1, NG + 1):
            for side in (0, 1):
                i = i0 - g if side == 0 else i0 + c.br - 1 + g
                pi = NG - g if side == 0 else NG + c.br - 1 + g
                J, K = np.meshgrid(np.arange(j0, j0 + c.bt), np.arange(k0, k0 + c.bp), indexing="xy")
                if i < 0:
                    for kk in range(c.bp):
                        for jj in range(c.bt):
                            P[:, NG + kk, NG + jj, pi] = self.inner_ghost(l, j0 + jj, k0 + kk)
                elif i >= lv.nr:
                    P[:, NG:-NG, NG:-NG, pi] = P[:, NG:-NG, NG:-NG, NG + c.br - 1]
                else:
                    P[:, NG:-NG, NG:-NG, pi] = self.level_value(
                        l, np.full(J.shape, i), J, K)
        # faces along theta: mirror rows at the colatitude edges
        for g in range(1, NG + 1):
            for side in (0, 1):
                j = j0 - g if side == 0 else j0 + c.bt - 1 + g
                pj = NG - g if side == 0 else NG + c.bt - 1 + g
                if j < 0 or j >= lv.nt:
                    src = NG + g - 1 if side == 0 else NG + c.bt - g
                    row = P[:, NG:-NG, src, NG:-NG].copy()
                    row[2] = -row[2]
                    row[6] = -row[6]
                    P[:, NG:-NG, pj, NG:-NG] = row
                else:
                    I, K = np.meshgrid(np.arange(i0, i0 + c.br), np.arange(k0, k0 + c.bp), indexing="xy")
                    P[:, NG:-NG, pj, NG:-NG] = self.level_value(l, I, np.full(I.shape, j), K)
        # faces along phi: periodic
        for g in range(1, NG + 1):
            for side in (0, 1):
                k = (k0 - g) % lv.nph if side == 0 else (k0 + c.bp - 1 + g) % lv.nph
                pk = NG - g if side == 0 else NG + c.bp - 1 + g
                I, J = np.meshgrid(np.arange(i0, i0 + c.br), np.arange(j0, j0 + c.bt), indexing="xy")
                P[:, pk, NG:-NG, NG:-NG] = self.level_value(l, I, J, np.full(I.shape, k))

    # --------------------------------------------------------------- step --
    def dt(self):
        """Global CFL dt (code units) over the leaves of every level."""
        dts = []
        for key in self.leaves():
            o = self.block_oracle(key)
            o.set_state(self.blocks[key].U[:8], kind=CONS_PADDED)
            dts.append(o.dt() / self.u["t"])
        return min(dts)

    def _rhs_all(self, t):
        self.fill_ghosts(t)
        for key in self.leaves():
            b = self.blocks[key]
            o = self.block_oracle(key)
            L, LT, faces = o.rhs(b.U[:8], b.U[8])
            b.L = np.concatenate([L, LT[None]], axis=0)
            b.faces = faces
        self._reflux()

    def _reflux(self):
        """Replace a coarse leaf's flux on faces shared with finer leaves by
        the area-weighted sum of the fine fluxes."""
        c = self.cfg
        for key in self.leaves():
            l = key[0]
            if l == c.max_level:
                continue
            b = self.blocks[key]
            V = self.cell_volumes(key)
            for d in range(3):
                for side in (0, 1):
                    nk = self.neighbour_key(key, d, side)
                    if nk is None or nk not in self.blocks or self.blocks[nk].leaf:
                        continue
                    name = "rtp"[d] + ("+" if side else "-")
                    Ac = self.face_areas(key, d, side)
                    Fc = b.faces[name]  # [9][a][b]
                    fine = np.zeros_like(Fc)
                    for ch in self.children(nk):
                        # children touching the shared face (their opposite side)
                        sub = (ch[1] - 2 * nk[1], ch[2] - 2 * nk[2], ch[3] - 2 * nk[3])
                        if sub[d] != (0 if side else 1):
                            continue
                        fb = self.blocks[ch]
                        Af = self.face_areas(ch, d, 1 - side)
                        Ff = fb.faces["rtp"[d] + ("-" if side else "+")] * Af[None]
                        # fine face cells -> coarse face cells (2 x 2 sums)
                        if d == 0:
                            s = Ff.reshape(NVAR, c.bp // 2, 2, c.bt // 2, 2).sum(axis=(2, 4))
                            ob = (sub[2] * c.bp // 2, sub[1] * c.bt // 2)
                            fine[:, ob[0]:ob[0] + c.bp // 2, ob[1]:ob[1] + c.bt // 2] += s
                        elif d == 1:
                            s = Ff.reshape(NVAR, c.bp // 2, 2, c.br // 2, 2).sum(axis=(2, 4))
                            ob = (sub[2] * c.bp // 2, sub[0] * c.br // 2)
                            fine[:, ob[0]:ob[0] + c.bp // 2, ob[1]:ob[1] + c.br // 2] += s
                        else:
                            s = Ff.reshape(NVAR, c.bt // 2, 2, c.br // 2, 2).sum(axis=(2, 4))
                            ob = (sub[1] * c.bt // 2, sub[0] * c.br // 2)
                            fine[:, ob[0]:ob[0] + c.bt // 2, ob[1]:ob[1] + c.br // 2] += s
                    delta = fine - Ac[None] * Fc  # change of the face's A F
                    sgn = -1.0 if side else 1.0
                    if d == 0:
                        cell = (slice(None), slice(None), slice(None), -1 if side else 0)
                        b.L[cell] += sgn * delta / V[:, :, -1 if side else 0][None]
                    elif d == 1:
                        cell = (slice(None), slice(None), -1 if side else 0, slice(None))
                        b.L[cell] += sgn * delta / V[:, -1 if side else 0, :][None]
                    else:
                        cell = (slice(None), -1 if side else 0, slice(None), slice(None))
                        b.L[cell] += sgn * delta / V[-1 if side else 0, :, :][None]

    def step(self, n=1):
        for _ in range(n):
            dt = self.dt()
            inner = (slice(None), slice(NG, -NG), slice(NG, -NG), slice(NG, -NG))
            U0 = {k: self.blocks[k].U[inner].copy() for k in self.leaves()}
            self._rhs_all(self.t)
            b1 = self.boundary_flux()
            for k in self.leaves():
                b = self.blocks[k]
                b.U[inner] = U0[k] + dt * b.L
            self._rhs_all(self.t + dt)
            b2 = self.boundary_flux()
            for k in self.leaves():
                b = self.blocks[k]
                b.U[inner] = 0.5 * U0[k] + 0.5 * (b.U[inner] + dt * b.L)
            # net inflow of the step through the r edges (the colatitude
            # edges reflect and phi is periodic)
            self.last_bflux = 0.5 * dt * (b1 + b2)
            self.t += dt
            self.step_count += 1
            bad = self.first_bad()
            if bad is not None:
                raise FloatingPointError(f"non-physical cell in block {bad} after step "
                                         f"{self.step_count}")
            if self.cfg.max_level > 1 and self.step_count % self.cfg.regrid_every == 0:
                self.regrid()

    def first_bad(self):
        gam = self.cfg.gamma
        for key in self.leaves():
            U = self.blocks[key].U[:, NG:-NG, NG:-NG, NG:-NG]
            rho = U[0]
            p = (gam - 1.0) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho
                               - 0.5 * (U[5] ** 2 + U[6] ** 2 + U[7] ** 2))
            if not (np.isfinite(U).all() and (rho > 0).all() and (p > 0).all()):
                return key
        return None

    # ------------------------------------------------------------ regrid --
    def indicators(self, key):
        """(max tau, max compression) over the block's cells; ghosts must be
        filled."""
        b = self.blocks[key]
        o = self.block_oracle(key)
        o.set_state(b.U[:8], kind=CONS_PADDED)
        divv = o.divv() * self.u["t"]  # 1/code time
        U = b.U[:, NG:-NG, NG:-NG, NG:-NG]
        tau = U[8] / U[0]
        l, bi, bj, bk = key
        rc = self.levels[l].rc[bi * self.cfg.br:(bi + 1) * self.cfg.br]
        vr = U[1] / U[0]
        comp = -divv * rc[None, None, :] / (2.0 * np.abs(vr))
        return float(tau.max()), float(comp.max())

    def flagged(self, key):
        c = self.cfg
        tau, comp = self.indicators(key)
        tr = tau >= c.tau_thr
        sh = comp >= c.shock_thr
        return {"tracing": tr, "shock": sh, "combined": tr or sh}[c.criterion]

    def _balance(self, refine):
        """Add to `refine` the coarser leaves that must split first so that
        face neighbours never differ by more than one level."""
        changed = True
        while changed:
            changed = False
            for k in list(refine):
                for d in range(3):
                    for side in (0, 1):
                        nk = self.neighbour_key(k, d, side)
                        if nk is None or nk in self.blocks:
                            continue
                        pk = self.parent(nk)
                        if pk in self.blocks and self.blocks[pk].leaf and pk not in refine:
                            refine.add(pk)
                            changed = True
        return refine

    def force_refine(self, keys):
        """Split the given leaves (and what the level balance requires)."""
        self.fill_ghosts(self.t)
        refine = self._balance(set(keys))
        for k in sorted(refine, key=lambda x: x[0]):
            if k in self.blocks and self.blocks[k].leaf:
                self._split(k)

    def regrid(self):
        c = self.cfg
        self.fill_ghosts(self.t)
        flags = {k: self.flagged(k) for k in self.leaves()}
        refine = {k for k, f in flags.items() if f and k[0] < c.max_level}
        # 2:1 balance: a refined block's face neighbours must exist at its
        # level (a coarser leaf there is refined too)
        self._balance(refine)
        # merges: parents whose 8 children are unflagged leaves (and not
        # being refined), if no neighbour of the parent is refined twice
        coarsen = set()
        parents = {self.parent(k) for k in self.leaves() if k[0] > 1}
        for pk in sorted(parents):
            ch = self.children(pk)
            if not all(x in self.blocks and self.blocks[x].leaf and not flags.get(x, True)
                       and x not in refine for x in ch):
                continue
            ok = True
            for d in range(3):
                for side in (0, 1):
                    nk = self.neighbour_key(pk, d, side)
                    if nk is None:
                        continue
                    # a neighbour refined below the children's level (or about
                    # to be) forbids the merge
                    if nk in self.blocks and not self.blocks[nk].leaf:
                        if any(not self.blocks[g].leaf for g in self.children(nk)
                               if g in self.blocks):
                            ok = False
                    if nk in refine:
                        ok = False
                    for g in self.children(nk) if nk in self.blocks else []:
                        if g in refine:
                            ok = False
            if ok:
                coarsen.add(pk)
        for pk in sorted(coarsen):
            self._merge(pk)
        for k in sorted(refine, key=lambda x: x[0]):
            if k in self.blocks and self.blocks[k].leaf:
                self._split(k)

    def _split(self, key):
        c = self.cfg
        l, bi, bj, bk = key
        b = self.blocks[key]
        P = b.U
        for ch in self.children(key):
            sub = (ch[1] - 2 * bi, ch[2] - 2 * bj, ch[3] - 2 * bk)
            Q = np.zeros_like(P)
            # coarse cells of this octant with their face neighbours (ghosts
            # of the parent supply the outer ones)
            hr, ht, hp = c.br // 2, c.bt // 2, c.bp // 2
            for kk in range(hp):
                for jj in range(ht):
                    for ii in range(hr):
                        pk = NG + sub[2] * hp + kk
                        pj = NG + sub[1] * ht + jj
                        pi = NG + sub[0] * hr + ii
                        nb = np.zeros((NVAR, 3, 3, 3))
                        for dp in (-1, 0, 1):
                            for dt in (-1, 0, 1):
                                for dr in (-1, 0, 1):
                                    if abs(dp) + abs(dt) + abs(dr) > 1:
                                        continue
                                    nb[:, dp + 1, dt + 1, dr + 1] = P[:, pk + dp, pj + dt, pi + dr]
                        gi = bi * c.br + sub[0] * hr + ii
                        gj = bj * c.bt + sub[1] * ht + jj
                        F = self.prolong(l, nb, np.array(gi), np.array(gj))
                        Q[:, NG + 2 * kk:NG + 2 * kk + 2, NG + 2 * jj:NG + 2 * jj + 2,
                          NG + 2 * ii:NG + 2 * ii + 2] = F
            self.blocks[ch] = Block(Q)
        b.leaf = False

    def _merge(self, pk):
        c = self.cfg
        l = pk[0]
        P = self.blocks[pk].U
        hr, ht, hp = c.br // 2, c.bt // 2, c.bp // 2
        for ch in self.children(pk):
            sub = (ch[1] - 2 * pk[1], ch[2] - 2 * pk[2], ch[3] - 2 * pk[3])
            Q = self.blocks[ch].U[:, NG:-NG, NG:-NG, NG:-NG]
            Uf = Q.reshape(NVAR, hp, 2, ht, 2, hr, 2).transpose(0, 1, 3, 5, 2, 4, 6)
            gi = pk[1] * c.br + sub[0] * hr + np.arange(hr)
            gj = pk[2] * c.bt + sub[1] * ht + np.arange(ht)
            I, J = np.meshgrid(gi, gj, indexing="xy")
            I = np.broadcast_to(I, (hp, ht, hr))
            J = np.broadcast_to(J, (hp, ht, hr))
            P[:, NG + sub[2] * hp:NG + (sub[2] + 1) * hp, NG + sub[1] * ht:NG + (sub[1] + 1) * ht,
              NG + sub[0] * hr:NG + (sub[0] + 1) * hr] = self.restrict(l, Uf, I, J)
            del self.blocks[ch]
            self.oracles.pop(ch, None)
        self.blocks[pk].leaf = True

    # ------------------------------------------------------- diagnostics --
    def boundary_flux(self):
        """Inflow through r_in minus outflow through r_out of the current
        stage's fluxes, integrated over the faces (9 variables)."""
        out = np.zeros(NVAR)
        for key in self.leaves():
            l, bi = key[0], key[1]
            nbr = self.nblocks(l)[0]
            b = self.blocks[key]
            if bi == 0:
                out += (b.faces["r-"] * self.face_areas(key, 0, 0)[None]).sum(axis=(1, 2))
            if bi == nbr - 1:
                out -= (b.faces["r+"] * self.face_areas(key, 0, 1)[None]).sum(axis=(1, 2))
        return out

    def totals(self):
        """Volume integrals of the 9 conserved variables over the leaves."""
        s = np.zeros(NVAR)
        for key in self.leaves():
            V = self.cell_volumes(key)
            s += (self.blocks[key].U[:, NG:-NG, NG:-NG, NG:-NG] * V[None]).sum(axis=(1, 2, 3))
        return s

    def level_counts(self):
        out = {}
        for k in self.leaves():
            out[k[0]] = out.get(k[0], 0) + 1
        return out

    def sample_level(self, l):
        """The whole domain at level l's resolution (leaves prolongated or
        restricted to it): [9][nph][nt][nr] conservative, code units."""
        lv = self.levels[l]
        K, J, I = np.meshgrid(np.arange(lv.nph), np.arange(lv.nt), np.arange(lv.nr), indexing="ij")
        return self.level_value(l, I, J, K)

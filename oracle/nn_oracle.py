"""CPU oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

Plain NumPy FP64 forward and backward of the network described in
include/icarus_nn.h, written from its definition: 3x3 convolutions on the
(theta, phi) grid (periodic in phi, edge-clamped in theta) with SiLU, then a
per-column two-layer decoder, mean squared error.  With ``bf16=True`` the
operands of every product are rounded to bfloat16 (round to nearest even)
where the GPU rounds them, so GPU gradients can be compared with it; with
``bf16=False`` it is the exact FP64 function used for the finite-difference
check of its own backward.  Shares no code with the HIP library.
"""
from __future__ import annotations

import numpy as np


def to_bf16(x):
    """Round to bfloat16 (via float32, round-to-nearest-even), return float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def im2col(h, dk0=-1, nk=3):
    """h [B][nt][np][C] -> [B*nt*np][3*nk*C], column index tap*C + c with
    tap = (dj+1)*nk + (dk-dk0), dj in -1..1, dk in dk0..dk0+nk-1; theta
    clamped at the edges, phi periodic."""
    B, nt, nph, C = h.shape
    out = np.zeros((B, nt, nph, 3 * nk, C))
    for dj in (-1, 0, 1):
        jj = np.clip(np.arange(nt) + dj, 0, nt - 1)
        for dk in range(dk0, dk0 + nk):
            kk = (np.arange(nph) + dk) % nph
            out[:, :, :, (dj + 1) * nk + (dk - dk0), :] = h[:, jj][:, :, kk]
    return out.reshape(B * nt * nph, 3 * nk * C)


def col2im(da, B, nt, nph, C, dk0=-1, nk=3):
    """Adjoint of im2col."""
    da = da.reshape(B, nt, nph, 3 * nk, C)
    dh = np.zeros((B, nt, nph, C))
    for dj in (-1, 0, 1):
        jj = np.clip(np.arange(nt) + dj, 0, nt - 1)
        for dk in range(dk0, dk0 + nk):
            kk = (np.arange(nph) + dk) % nph
            tap = (dj + 1) * nk + (dk - dk0)
            for j in range(nt):
                for k in range(nph):
                    dh[:, jj[j], kk[k]] += da[:, j, k, tap, :]
    return dh


class Shape:
    def __init__(self, n_theta, n_phi, n_r, c1, c2, hidden, phi_lo=-1, phi_hi=1, coord=0):
        self.nt, self.np_, self.nr = n_theta, n_phi, n_r
        self.c1, self.c2, self.h = c1, c2, hidden
        self.phi_lo, self.nk = phi_lo, phi_hi - phi_lo + 1
        self.cin = 10 if coord else 8  # map features (+ two colatitude channels)
        self.k1 = 3 * self.nk * self.cin
        self.no = 8 * n_r
        self.sizes = [self.k1 * c1, c1, 9 * c1 * c2, c2, c2 * hidden, hidden, hidden * self.no,
                      self.no]

    @property
    def nparam(self):
        return int(sum(self.sizes))

    def unpack(self, p):
        out, o = [], 0
        shapes = [(self.k1, self.c1), (self.c1,), (9 * self.c1, self.c2), (self.c2,),
                  (self.c2, self.h), (self.h,), (self.h, self.no), (self.no,)]
        for sh in shapes:
            n = int(np.prod(sh))
            out.append(np.asarray(p[o:o + n], dtype=np.float64).reshape(sh))
            o += n
        return out


def forward(shape, params, x, bf16=True):
    """x [B][nt][np][8] -> y [B*nt*np][n_r*8] and the saved activations."""
    r = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3, W4, b4 = shape.unpack(params)
    B = x.shape[0]
    a1 = im2col(r(x), shape.phi_lo, shape.nk)
    z1 = a1 @ r(W1) + b1
    h1 = r(silu(z1))
    a2 = im2col(h1.reshape(B, shape.nt, shape.np_, shape.c1))
    z2 = a2 @ r(W2) + b2
    h2 = r(silu(z2))
    z3 = h2 @ r(W3) + b3
    h3 = r(silu(z3))
    y = h3 @ r(W4) + b4
    return y, dict(a1=a1, z1=z1, h1=h1, a2=a2, z2=z2, h2=h2, z3=z3, h3=h3)


def loss_grad(shape, params, x, t, bf16=True):
    """Mean squared error and its gradient with respect to the parameters."""
    r = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3, W4, b4 = shape.unpack(params)
    B = x.shape[0]
    y, s = forward(shape, params, x, bf16)
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / d.size
    dyr = r(dy)
    gW4 = s["h3"].T @ dyr
    gb4 = dy.sum(0)
    dz3 = (dyr @ r(W4).T) * silu_grad(s["z3"])
    gW3 = s["h2"].T @ r(dz3)
    gb3 = dz3.sum(0)
    dz2 = (r(dz3) @ r(W3).T) * silu_grad(s["z2"])
    gW2 = s["a2"].T @ r(dz2)
    gb2 = dz2.sum(0)
    da2 = r(dz2) @ r(W2).T
    dh1 = col2im(da2, B, shape.nt, shape.np_, shape.c1).reshape(-1, shape.c1)
    dz1 = dh1 * silu_grad(s["z1"])
    gW1 = s["a1"].T @ r(dz1)
    gb1 = dz1.sum(0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
    return loss, g


# ---- feature / target transforms (definitions of include/icarus_nn.h) ----
RHO0 = 1.67262192369e-27 * 1e8
P0 = 2.0 * 1e8 * 1.380649e-23 * 1e6
V0 = 1e5
B0 = 250e-9


def encode_map(maps, thc, omega, r_in, coord=0):
    """maps [B][8][nt][np] SI -> X [B][nt][np][C]; with coord the colatitude
    channels t (linear from -1 at the first to 1 at the last colatitude
    centre) and 2 t^2 - 1 follow the eight map features."""
    m = np.asarray(maps, dtype=np.float64)
    sth = np.sin(thc)[None, :, None]
    feats = [np.log(m[:, 0] / RHO0), m[:, 1] / V0 - 5.0, m[:, 2] / V0,
             (m[:, 3] + omega * r_in * sth) / V0, np.log(m[:, 4] / P0),
             m[:, 5] / B0, m[:, 6] / B0, m[:, 7] / B0]
    if coord:
        thc = np.asarray(thc, dtype=np.float64)
        t = ((2.0 * thc - thc[0] - thc[-1]) / (thc[-1] - thc[0]) if len(thc) > 1
             else np.zeros(1))
        tt = np.broadcast_to(t[None, :, None], m[:, 0].shape)
        feats += [tt, 2.0 * tt * tt - 1.0]
    return np.stack(feats, axis=-1)


def radial_base(m, rc, thc, omega, r_in, gamma):
    """Radial expansion of one map [8][nt][np] at radii rc: [8][np][nt][nr]."""
    x = (r_in / rc)[None, None, :]
    mt = np.transpose(m, (0, 2, 1))[..., None]  # [8][np][nt][1]
    sth = np.sin(thc)[None, :, None]
    w = np.zeros((8, m.shape[2], m.shape[1], len(rc)))
    w[0] = mt[0] * x ** 2
    w[1] = mt[1]
    w[3] = -omega * rc[None, None, :] * sth
    w[4] = mt[4] * x ** (2 * gamma)
    w[5] = mt[5] * x ** 2
    w[7] = mt[7] * x
    return w


def encode_target(m, state, rc, thc, omega, r_in, gamma):
    """Primitive SI state [8][np][nt][nr] -> T [nt*np][nr*8]."""
    w = radial_base(m, rc, thc, omega, r_in, gamma)
    bs = np.abs(w[5]) + np.abs(w[7]) + 1e-30
    t = np.stack([np.log(state[0] / w[0]), (state[1] - w[1]) / V0, state[2] / V0,
                  (state[3] - w[3]) / V0, np.log(state[4] / w[4]), (state[5] - w[5]) / bs,
                  state[6] / bs, (state[7] - w[7]) / bs], axis=-1)  # [np][nt][nr][8]
    return np.transpose(t, (1, 0, 2, 3)).reshape(m.shape[1] * m.shape[2], -1)


def decode_state(m, y, rc, thc, omega, r_in, gamma):
    nt, nph, nr = m.shape[1], m.shape[2], len(rc)
    w = radial_base(m, rc, thc, omega, r_in, gamma)
    bs = np.abs(w[5]) + np.abs(w[7]) + 1e-30
    o = np.transpose(np.asarray(y, dtype=np.float64).reshape(nt, nph, nr, 8), (3, 1, 0, 2))
    s = np.zeros_like(w)
    s[0] = w[0] * np.exp(o[0])
    s[1] = w[1] + V0 * o[1]
    s[2] = V0 * o[2]
    s[3] = w[3] + V0 * o[3]
    s[4] = w[4] * np.exp(o[4])
    s[5] = w[5] + bs * o[5]
    s[6] = bs * o[6]
    s[7] = w[7] + bs * o[7]
    return s

"""Pins for the NN oracle (CPU): its backward against central finite
differences of its own FP64 forward, the 3x3 gather against its adjoint,
bfloat16 rounding against exactly known values, and the feature / target
transforms against their inverses and the radial-expansion laws."""
import numpy as np
import pytest

from oracle import nn_oracle as no
from paper_2501_15923_amd import synth


def tiny(phi_lo=-1, phi_hi=1, coord=0):
    sh = no.Shape(4, 6, 3, 4, 5, 6, phi_lo, phi_hi, coord)
    rng = np.random.default_rng(1)
    p = rng.normal(0, 0.4, sh.nparam)
    x = rng.normal(0, 1, (2, 4, 6, sh.cin))
    t = rng.normal(0, 0.3, (2 * 4 * 6, sh.no))
    return sh, p, x, t


@pytest.mark.parametrize("window", [(-1, 1, 0), (-2, 3, 0), (-1, 2, 1)])
def test_backward_matches_finite_differences(window):
    sh, p, x, t = tiny(*window)
    loss, g = no.loss_grad(sh, p, x, t, bf16=False)
    rng = np.random.default_rng(2)
    idx = rng.choice(sh.nparam, 60, replace=False)
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (no.loss_grad(sh, pp, x, t, bf16=False)[0] -
              no.loss_grad(sh, pm, x, t, bf16=False)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_im2col_adjoint_and_boundaries():
    rng = np.random.default_rng(3)
    B, nt, nph, C = 2, 5, 7, 3
    h = rng.normal(size=(B, nt, nph, C))
    da = rng.normal(size=(B * nt * nph, 9 * C))
    lhs = np.sum(no.im2col(h) * da)
    rhs = np.sum(h * no.col2im(da, B, nt, nph, C))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    a = no.im2col(h).reshape(B, nt, nph, 9, C)
    # periodic in phi, clamped in theta
    assert np.array_equal(a[:, 2, 0, 1 * 3 + 0], h[:, 2, nph - 1])
    assert np.array_equal(a[:, 0, 3, 0 * 3 + 1], h[:, 0, 3])
    assert np.array_equal(a[:, nt - 1, 3, 2 * 3 + 1], h[:, nt - 1, 3])
    # a wide upstream window: dk in -2..4 wraps around the longitude period
    dk0, nk = -2, 7
    da = rng.normal(size=(B * nt * nph, 3 * nk * C))
    lhs = np.sum(no.im2col(h, dk0, nk) * da)
    rhs = np.sum(h * no.col2im(da, B, nt, nph, C, dk0, nk))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    a = no.im2col(h, dk0, nk).reshape(B, nt, nph, 3 * nk, C)
    assert np.array_equal(a[:, 1, 5, 1 * nk + (4 - dk0)], h[:, 1, (5 + 4) % nph])
    assert np.array_equal(a[:, 1, 0, 1 * nk + (-2 - dk0)], h[:, 1, nph - 2])
    assert np.array_equal(a[:, 0, 2, 0 * nk + (1 - dk0)], h[:, 0, 3])


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -9, -2.5, 3.0e38])
    exp = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -7, -2.5, 2.9999249e38])
    got = no.to_bf16(vals)
    assert np.allclose(got[:5], exp[:5], rtol=0, atol=0)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> 1
    assert got[1] == 1.0


def test_transforms_round_trip():
    g = synth.Grid(12, 6, 10)
    m = synth.static_map(g, 4)
    th, _ = synth.angle_centres(g)
    r = 0.1 * synth.AU * 20.0 ** (np.arange(g.nr + 1) / g.nr)
    rc = 0.5 * (r[1:] + r[:-1])
    om, rin = synth.OMEGA_SUN, g.r_in
    base = no.radial_base(m, rc, th, om, rin, 1.5)
    # the radial expansion itself has target zero
    t0 = no.encode_target(m, base, rc, th, om, rin, 1.5)
    assert np.max(np.abs(t0)) < 1e-12
    rng = np.random.default_rng(5)
    y = rng.normal(0, 0.2, t0.shape)
    s = no.decode_state(m, y, rc, th, om, rin, 1.5)
    assert np.allclose(no.encode_target(m, s, rc, th, om, rin, 1.5), y, atol=1e-10)
    x = no.encode_map(m[None], th, om, rin)
    # inertial v_phi of the map vanishes (plasma not rotating at r_in)
    assert np.max(np.abs(x[..., 3])) < 1e-9
    # the colatitude channels: -1 and 1 at the first and last row, 0 on the
    # mid row of an odd count, a parabola that is -1 there and 1 at the ends;
    # the map features are unchanged
    xc = no.encode_map(m[None], th, om, rin, coord=1)
    assert xc.shape[-1] == 10 and np.array_equal(xc[..., :8], x)
    t = xc[0, :, 0, 8]
    assert abs(t[0] + 1) < 1e-14 and abs(t[-1] - 1) < 1e-14
    assert np.allclose(t, t[::-1] * -1, atol=1e-14) and np.all(np.diff(t) > 0)
    assert np.allclose(xc[0, :, :, 9], 2 * xc[0, :, :, 8] ** 2 - 1, atol=1e-14)
    assert np.allclose(xc[0, :, 3, 8:], xc[0, :, 0, 8:])  # the same for every longitude
    assert np.allclose(np.exp(x[..., 0]) * no.RHO0, np.transpose(m[0])[None].transpose(0, 2, 1))

"""Pins for the radial cubic blob oracle (oracle/cubic.py): an independent
truncated-power form of the spline, its planar integral, smoothness at the
joins, the footprint and values of a single point evaluated pixel by pixel,
the projected world-space radius, finite differences of the adjoint (no edge
to skip: the blob is twice continuously differentiable), and the attribute
channel's linearity."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import cubic, splat

f32 = np.float32


def w_tp(q):
    """The cubic B-spline as truncated powers: 2 (1-q)_+^3 - 8 (1/2-q)_+^3."""
    return 2.0 * max(1.0 - q, 0.0) ** 3 - 8.0 * max(0.5 - q, 0.0) ** 3


def test_spline_equals_truncated_power_form():
    q = np.linspace(0.0, 1.3, 2001)
    want = np.array([w_tp(t) for t in q])
    assert np.allclose(cubic.w_profile(q), want, rtol=0, atol=1e-15)


def test_planar_integral_is_one():
    val = quad(lambda q: w_tp(q) * 2 * math.pi * q, 0.0, 1.0, points=[0.5])[0]
    assert abs(val * cubic.NORM - 1.0) < 1e-12
    # a wide blob sampled on the pixel grid sums to its mass
    cam = splat.Camera(0, 64, 64)
    img = cubic.render(cam, np.array([0.5 + 0.3 / 64], f32), np.array([0.5 - 0.2 / 64], f32),
                       np.zeros(1, f32), np.array([2.5], f32), h_px=12.0)
    assert abs(img.sum() - 2.5) < 2e-4 * 2.5


def test_spline_is_twice_differentiable_at_the_joins():
    for q0 in (0.5, 1.0):
        e = 1e-6
        for k, f in enumerate((cubic.w_profile, cubic.dw)):
            left, right = float(f(q0 - e)), float(f(q0 + e))
            assert abs(left - right) < 1e-4, (q0, k)
        # second derivative from both sides by differences of w'
        d2l = (float(cubic.dw(q0 - 1e-5)) - float(cubic.dw(q0 - 2e-5))) / 1e-5
        d2r = (float(cubic.dw(q0 + 2e-5)) - float(cubic.dw(q0 + 1e-5))) / 1e-5
        assert abs(d2l - d2r) < 1e-3, q0
    q = np.linspace(0.01, 0.99, 99)
    fd = (cubic.w_profile(q + 1e-7) - cubic.w_profile(q - 1e-7)) / 2e-7
    assert np.allclose(cubic.dw(q), fd, atol=1e-6)
    assert np.allclose(cubic.dw_over_q(q) * q, cubic.dw(q), atol=1e-12)


@pytest.mark.parametrize("h", [1.0, 2.3, 5.0])
def test_single_point_footprint_and_values(h):
    """Every pixel evaluated by hand: covered iff its centre lies strictly inside
    radius h, value m 40/(7 pi h^2) w(r/h) from the truncated-power form."""
    cam = splat.Camera(0, 32, 32)
    x = np.array([13.37 / 32], f32); y = np.array([17.81 / 32], f32)
    img = cubic.render(cam, x, y, np.zeros(1, f32), np.array([1.5], f32), h_px=h)
    h = float(f32(h))                                 # the radius is a float32 parameter
    u, v = float(x[0]) * 32, float(y[0]) * 32
    for j in range(32):
        for i in range(32):
            ox, oy = u - (i + 0.5), v - (j + 0.5)
            r = math.hypot(ox, oy)
            want = 1.5 * 40.0 / (7.0 * math.pi * h * h) * w_tp(r / h) if r < h else 0.0
            assert abs(img[j, i] - want) <= 1e-12 * (abs(want) + 1e-300), (i, j)
    assert img.max() == img[17, 13]


def test_world_radius_is_projected_and_clamped():
    cam = splat.Camera(1, 100, 100, pos=(0.5, 0.5, -1.0), F=80.0, near=0.01)
    zs = (-0.9, 0.0, 1.0, 3.0, 10.0)
    z = np.array(zs, f32)                                # zc = z + 1: radii 40, 4, 2, 1, 0.36 px
    x = np.full(5, f32(0.5)); y = np.full(5, f32(0.5))
    _, _, _, _, _, zc = splat.project(cam, x, y, z)
    h, clamped = cubic.pixel_radius(cam, zc, 0.0, 0.05)
    want = [min(max(80.0 * 0.05 / (float(f32(zz)) + 1.0), 1.0), 16.0) for zz in zs]
    assert np.allclose(h.astype(np.float64), want, rtol=1e-6)
    assert list(clamped) == [True, False, False, False, True]


@pytest.mark.parametrize("proj,h_world", [(0, 0.0), (1, 0.0), (1, 0.02)])
def test_adjoint_finite_differences_everywhere(proj, h_world):
    """No point is skipped: the blob has no truncation edge."""
    rng = np.random.default_rng(11)
    Np, W = 30, 32
    x = (0.3 + 0.4 * rng.random(Np)).astype(f32)
    y = (0.3 + 0.4 * rng.random(Np)).astype(f32)
    z = (0.3 + 0.4 * rng.random(Np)).astype(f32)
    m = rng.uniform(0.5, 1.5, Np).astype(f32)
    if proj == 0:
        cam = splat.Camera(0, W, W)
    else:
        cam = splat.Camera(1, W, W, pos=(0.5, 0.5, -1.0), right=(1, 0, 0), up=(0, 1, 0), fwd=(0, 0, 1),
                           F=32.0, near=0.01)
    g = rng.standard_normal((W, W))
    hp = float(f32(2.2))
    gm, gp = cubic.render_backward(cam, x, y, z, m, g, h_px=hp, h_world=h_world)
    m64 = m.astype(np.float64)

    def loss64(px, py, pz, mm):
        """independent float64 evaluation from the truncated-power form"""
        tot = 0.0
        for k in range(Np):
            if proj == 0:
                u, v, hk = px[k] * W, py[k] * W, hp
            else:
                zc = pz[k] + 1.0
                u = 32.0 * (px[k] - 0.5) / zc + W / 2; v = 32.0 * (py[k] - 0.5) / zc + W / 2
                hk = min(max(32.0 * float(f32(h_world)) / zc, 1.0), 16.0) if h_world else hp
            for j in range(W):
                for i in range(W):
                    r = math.hypot(u - (i + 0.5), v - (j + 0.5))
                    if r < hk:
                        tot += mm[k] * 40.0 / (7.0 * math.pi * hk * hk) * w_tp(r / hk) * g[j, i]
        return tot
    px, py, pz = (a.astype(np.float64) for a in (x, y, z))
    h = 1e-7
    for k in range(0, Np, 3):
        for ax, arr in enumerate((px, py, pz)):
            if proj == 0 and ax == 2:
                assert gp[k, 2] == 0.0
                continue
            old = arr[k]
            arr[k] = old + h; lp = loss64(px, py, pz, m64)
            arr[k] = old - h; lm = loss64(px, py, pz, m64)
            arr[k] = old
            fd = (lp - lm) / (2 * h)
            # the oracle's offsets come from the float32 projection (relative 1e-7)
            assert abs(fd - gp[k, ax]) < 2e-4 * (1 + abs(fd)), (k, ax, fd, gp[k, ax])
        mm = m64.copy(); mm[k] = 0.0
        base = loss64(px, py, pz, mm)
        mm[k] = 1.0
        # linear in m: exact up to rounding (orthographic), or up to the float32
        # projection's shift of u, v (perspective)
        tol = 1e-9 if proj == 0 else 1e-5
        assert abs((loss64(px, py, pz, mm) - base) - gm[k]) < tol * (1 + abs(gm[k]))


def test_attribute_channel_is_the_render_of_weighted_masses():
    s = synth.small_clustered(3000, 12)
    rng = np.random.default_rng(2)
    a = (rng.random(s.n) < 0.3).astype(f32)
    cam = splat.Camera(1, 64, 48, pos=(0.5, 0.5, -0.8), F=50.0, near=0.01)
    img, aimg = cubic.render(cam, s.x, s.y, s.z, s.m, h_px=2.0, aux=a)
    sel = a > 0
    want = cubic.render(cam, s.x[sel], s.y[sel], s.z[sel], s.m[sel], h_px=2.0)
    assert np.allclose(aimg, want, rtol=1e-12, atol=0)
    assert np.allclose(img, cubic.render(cam, s.x, s.y, s.z, s.m, h_px=2.0), rtol=0, atol=0)
    assert np.all(aimg <= img * (1 + 1e-12))

"""Pins for the time-interpolation oracle (oracle/interp.py): the end points
of the interpolation, the colour channel's linearity, and the motion codes
of stored points (static particles code zero; decode within the code's
quantum of the true position; saturation counted by brute force)."""
import numpy as np
import pytest

import synth
from oracle import cubic, interp, lod, splat

f32 = np.float32


def _pair(n=3000, seed=31, step=0.01):
    A = synth.small_clustered(n, seed)
    B, aa, ab = synth.evolve(A, seed + 1, step=step)
    return A, B, aa, ab


def test_lerp_end_points():
    rng = np.random.default_rng(1)
    a = rng.random(10000).astype(f32)
    b = rng.random(10000).astype(f32)
    assert np.array_equal(interp.lerp(a, b, 0.0), a)
    one = interp.lerp(a, b, 1.0)
    assert np.all(np.abs(one.astype(np.float64) - b) <= np.spacing(np.maximum(np.abs(b), np.abs(a))).astype(np.float64))
    mid = interp.lerp(a, b, 0.5).astype(np.float64)
    assert np.all(np.abs(mid - (a.astype(np.float64) + b) / 2) <= 2 * np.spacing(f32(1.0)))


def test_frame_at_zero_is_snapshot_a():
    A, B, aa, ab = _pair()
    cam = splat.Camera(1, 96, 72, pos=(0.5, 0.5, -0.8), F=80.0, near=0.01)
    img = interp.render(cam, (A.x, A.y, A.z, A.m), (B.x, B.y, B.z, B.m), 0.0)
    assert np.array_equal(img, splat.render(cam, A.x, A.y, A.z, A.m))
    img = interp.render(cam, (A.x, A.y, A.z, A.m), (B.x, B.y, B.z, B.m), 0.0, blob="cubic", hA=aa.h, hB=ab.h)
    assert np.array_equal(img, cubic.render(cam, A.x, A.y, A.z, A.m, h_world=aa.h))


def test_frame_at_one_is_snapshot_b_for_the_smooth_blob():
    """At t = 1 every interpolated value is within one float32 step of B's; the
    cubic blob is smooth, so the image matches B's within 1e-4 relative where
    it is well above zero."""
    A, B, aa, ab = _pair()
    cam = splat.Camera(1, 96, 72, pos=(0.5, 0.5, -0.8), F=80.0, near=0.01)
    img = interp.render(cam, (A.x, A.y, A.z, A.m), (B.x, B.y, B.z, B.m), 1.0, blob="cubic", hA=aa.h, hB=ab.h)
    ref = cubic.render(cam, B.x, B.y, B.z, B.m, h_world=ab.h)
    big = ref > 1e-3 * ref.max()
    assert big.sum() > 100
    assert np.max(np.abs(img[big] - ref[big]) / ref[big]) < 1e-4


def test_colour_channel_is_render_of_colour_weighted_masses():
    A, B, aa, ab = _pair()
    cam = splat.Camera(0, 64, 64)
    t = 0.37
    img, cimg = interp.render(cam, (A.x, A.y, A.z, A.m), (B.x, B.y, B.z, B.m), t, blob="cubic", h_px=2.0,
                              cA=aa.c, cB=ab.c)
    x, y, z, m = (interp.lerp(a, b, t) for a, b in ((A.x, B.x), (A.y, B.y), (A.z, B.z), (A.m, B.m)))
    c = interp.lerp(aa.c, ab.c, t)
    ref = cubic.render(cam, x, y, z, m, h_px=2.0)
    assert np.array_equal(img, ref)
    # sum m c W, against the plain render of masses m c (m c rounded to float32 there)
    refc = cubic.render(cam, x, y, z, (m.astype(np.float64) * c).astype(f32), h_px=2.0)
    assert np.allclose(cimg, refc, rtol=2e-7, atol=0)


@pytest.mark.parametrize("step,saturates", [(0.02, False), (0.4, True)])
def test_motion_codes_static_and_bounded(step, saturates):
    A, B, aa, ab = _pair(4000, 33, step=step)
    t = lod.lod_build(A.x, A.y, A.z, A.m, n=150, D=4, seed=3)
    # particles that do not move code zero motion
    z0 = interp.encode_motion(t, A.x, A.y, A.z)
    assert z0[3] == 0 and all(np.all(a == 0) for a in z0[:3])
    dqx, dqy, dqz, sat = interp.encode_motion(t, B.x, B.y, B.z)
    # brute force per stored point: decode within 2.5 quanta of B (or saturated)
    nodes = range(t.n_nodes)
    (xa, ya, za, _), (xb, yb, zb, _) = interp.decoded_motion_points(t, nodes, dqx, dqy, dqz)
    pid = t.pt_id.astype(np.int64)
    nsat = 0
    off = 0
    for v in nodes:
        d = int(t.depth[v]); k = int(t.pt_count[v])
        quantum = 2.0 ** -(d + 16)
        for got, true in ((xb, B.x), (yb, B.y), (zb, B.z)):
            err = np.abs(got[off:off + k].astype(np.float64) - true[pid[off:off + k]].astype(np.float64))
            far = err > 2.5 * quantum + np.spacing(f32(1.0))
            nsat += int(far.sum())
        off += k
    assert nsat == sat
    # a small flow stays within two block sides of depth-4 nodes; a large one does not
    assert (sat > 0) == saturates

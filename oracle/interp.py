"""Time interpolation between two snapshots -- plain definition (CPU oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The rendering paragraph: every point carries time information, so that the
graphics card can interpolate position, size and colour for each frame.
Readings used here:

* Two snapshots A and B of the same particles (matched by id), and a frame
  time t in [0, 1] between them.  Every interpolated quantity q is
  q(t) = fl(q_A + fl(t fl(q_B - q_A))) in float32, no fused multiply-add:
  positions x, y, z, mass m, world radius h (cubic blob), colour c.
* The image is the splat of the interpolated points; the colour image is
  the attribute channel sum m(t) c(t) W (colour = colour image / image).
* Stored LOD points carry their motion in the same 16-bit style as their
  positions: for a point stored at depth d with code Q0 = (c_d << 16) + q
  and its particle's B position with Q1 = floor(x_B 2^(d+16)), the motion
  code is dq = clamp(floor((Q1 - Q0 + 2) / 4), -32768, 32767) (the motion in
  units of four position quanta, rounded to nearest, a range of two block
  sides either way).  Decode: x_hat_B = the float32 nearest
  (2 (Q0 + 4 dq) + 1) 2^-(d+17).  A clamped code is counted as saturated.
"""
from __future__ import annotations

import numpy as np

from . import cubic, lod, splat

f32 = np.float32


def lerp(a, b, t):
    """fl(a + fl(t fl(b - a))) elementwise in float32."""
    a = np.asarray(a, dtype=f32)
    b = np.asarray(b, dtype=f32)
    return (a + (f32(t) * (b - a))).astype(f32)


def render(cam, A, B, t, blob="gauss", h_px=1.5, hA=None, hB=None, cA=None, cB=None, sigma=1.0,
           radius_sigmas=3.0):
    """float64 image (and colour image if colours are given) of the frame at t.

    A, B: (x, y, z, m) float32 arrays.  blob "gauss" or "cubic"; with hA, hB
    (world radii per point) the cubic radius is interpolated too.
    """
    x, y, z, m = (lerp(a, b, t) for a, b in zip(A, B))
    col = lerp(cA, cB, t) if cA is not None else None
    if blob == "cubic":
        hw = lerp(hA, hB, t) if hA is not None else 0.0
        return cubic.render(cam, x, y, z, m, h_px=h_px, h_world=hw, aux=col)
    if col is not None:
        img = splat.render(cam, x, y, z, m, sigma, radius_sigmas)
        cimg = splat.render(cam, x, y, z, (m.astype(np.float64) * col).astype(f32), sigma, radius_sigmas)
        return img, cimg
    return splat.render(cam, x, y, z, m, sigma, radius_sigmas)


def encode_motion(tree: lod.Tree, xB, yB, zB, snap_offsets=None):
    """Motion codes (dqx, dqy, dqz int16 per stored point) and the number of
    saturated components, for particle positions xB, yB, zB indexed like the
    build input (per snapshot by id)."""
    S = tree.n_points
    out = [np.zeros(S, dtype=np.int16) for _ in range(3)]
    sat = 0
    base = np.zeros(1, dtype=np.int64) if snap_offsets is None else np.asarray(snap_offsets, dtype=np.int64)
    D = tree.D
    for v in range(tree.n_nodes):
        (cx, cy, cz), d = lod.node_origin(tree, v)
        b, k = int(tree.pt_begin[v]), int(tree.pt_count[v])
        if k == 0:
            continue
        snap = int(tree.prefix[v]) >> (3 * d) if snap_offsets is not None else 0
        gid = base[snap] + tree.pt_id[b:b + k].astype(np.int64)
        for ax, (arr, c, q) in enumerate(((xB, cx, tree.qx), (yB, cy, tree.qy), (zB, cz, tree.qz))):
            Q1 = np.floor(np.asarray(arr, dtype=f32)[gid].astype(np.float64) * 2.0 ** (d + 16)).astype(np.int64)
            Q0 = (np.int64(c) << 16) + q[b:b + k].astype(np.int64)
            dq = np.floor_divide(Q1 - Q0 + 2, 4)
            sat += int(np.count_nonzero((dq < -32768) | (dq > 32767)))
            out[ax][b:b + k] = np.clip(dq, -32768, 32767).astype(np.int16)
    return out[0], out[1], out[2], sat


def decoded_motion_points(tree: lod.Tree, nodes, dqx, dqy, dqz):
    """(A, B) decoded positions (x, y, z, m) of the nodes' stored points: A from
    the position codes, B from position plus motion codes; masses unchanged."""
    xa, ya, za, ma, xb, yb, zb = [], [], [], [], [], [], []
    for v in nodes:
        (cx, cy, cz), d = lod.node_origin(tree, int(v))
        b, k = int(tree.pt_begin[v]), int(tree.pt_count[v])
        for c, q, dq, outa, outb in ((cx, tree.qx, dqx, xa, xb), (cy, tree.qy, dqy, ya, yb), (cz, tree.qz, dqz, za, zb)):
            Q0 = (np.int64(c) << 16) + q[b:b + k].astype(np.int64)
            outa.append(((2 * Q0 + 1).astype(np.float64) * 2.0 ** -(d + 17)).astype(f32))
            Q1 = Q0 + 4 * dq[b:b + k].astype(np.int64)
            outb.append(((2 * Q1 + 1).astype(np.float64) * 2.0 ** -(d + 17)).astype(f32))
        ma.append(tree.pt_mass[b:b + k])
    cat = lambda a: np.concatenate(a) if a else np.zeros(0, f32)   # noqa: E731
    m = cat(ma)
    return (cat(xa), cat(ya), cat(za), m), (cat(xb), cat(yb), cat(zb), m)

"""Additive point splat and its adjoint -- plain definition (CPU oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's rendering paragraph draws every point as a smeared blob whose
radial profile is evaluated for each pixel the point covers, and sums the
blobs.  The blob used here is a Gaussian of standard deviation sigma pixels,
truncated to a square of half-width R = radius_sigmas * sigma and normalised
by 1 / (2 pi sigma^2).

Screen position and the pixel offsets are fixed float32 operation sequences
(no fused multiply-add), replicated here with numpy float32 arithmetic so
that the set of pixels a point covers is decided identically on both sides:

* orthographic (looking down z):  u = fl(x W), v = fl(y H);
* perspective:  d = p - c;  xc = (d.x r.x + d.y r.y) + d.z r.z (each
  product and sum rounded), likewise yc with the up vector and zc with the
  forward vector; the point is culled unless zc > near;
  u = fl(F fl(xc / zc)) + fl(W / 2), v = fl(F fl(yc / zc)) + fl(H / 2);
* pixel (i, j): ox = fl(u - (i + 1/2)), oy = fl(v - (j + 1/2)); the pixel
  receives the point iff |ox| <= R, |oy| <= R and it lies in the image.

From the exponential onward everything is float64:
I[j, i] += m exp(-(ox^2 + oy^2) / (2 sigma^2)) / (2 pi sigma^2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

f32 = np.float32


@dataclass
class Camera:
    projection: int            # 0 orthographic along z, 1 perspective
    W: int
    H: int
    pos: tuple = (0.0, 0.0, 0.0)
    right: tuple = (1.0, 0.0, 0.0)
    up: tuple = (0.0, 1.0, 0.0)
    fwd: tuple = (0.0, 0.0, 1.0)
    F: float = 1.0
    near: float = 1e-3


def project(cam: Camera, x, y, z):
    """Return (u, v, keep, xc, yc, zc) with the pinned float32 sequence."""
    x = np.asarray(x, dtype=f32); y = np.asarray(y, dtype=f32); z = np.asarray(z, dtype=f32)
    if cam.projection == 0:
        u = x * f32(cam.W)
        v = y * f32(cam.H)
        keep = np.ones(x.shape, dtype=bool)
        return u, v, keep, None, None, None
    c = [f32(a) for a in cam.pos]
    r = [f32(a) for a in cam.right]
    up = [f32(a) for a in cam.up]
    fw = [f32(a) for a in cam.fwd]
    dx = x - c[0]; dy = y - c[1]; dz = z - c[2]
    xc = ((dx * r[0]) + (dy * r[1])) + (dz * r[2])
    yc = ((dx * up[0]) + (dy * up[1])) + (dz * up[2])
    zc = ((dx * fw[0]) + (dy * fw[1])) + (dz * fw[2])
    keep = zc > f32(cam.near)
    zs = np.where(keep, zc, f32(1.0))
    u = (f32(cam.F) * (xc / zs)) + f32(cam.W) * f32(0.5)
    v = (f32(cam.F) * (yc / zs)) + f32(cam.H) * f32(0.5)
    return u, v, keep, xc, yc, zc


def _window(R: float) -> int:
    return int(math.ceil(R)) + 2


def _covers(cam: Camera, u, v, keep, R32, di, dj):
    """Pixel indices and float32 offsets for window offset (di, dj)."""
    fu = np.floor(u.astype(np.float64)).astype(np.int64)
    fv = np.floor(v.astype(np.float64)).astype(np.int64)
    i = fu + di
    j = fv + dj
    ox = u - (i.astype(f32) + f32(0.5))
    oy = v - (j.astype(f32) + f32(0.5))
    ok = keep & (np.abs(ox) <= R32) & (np.abs(oy) <= R32)
    ok &= (i >= 0) & (i < cam.W) & (j >= 0) & (j < cam.H)
    return i, j, ox, oy, ok


def _visible(cam, u, v, keep, R):
    lim = R + 4.0
    u64 = u.astype(np.float64); v64 = v.astype(np.float64)
    return keep & np.isfinite(u64) & np.isfinite(v64) & (u64 > -lim) & (u64 < cam.W + lim) \
        & (v64 > -lim) & (v64 < cam.H + lim)


def render(cam: Camera, x, y, z, m, sigma: float = 1.0, radius_sigmas: float = 3.0) -> np.ndarray:
    """float64 image [H, W]."""
    img = np.zeros((cam.H, cam.W), dtype=np.float64)
    if len(np.asarray(x)) == 0:
        return img
    R32 = f32(radius_sigmas) * f32(sigma)
    u, v, keep, _, _, _ = project(cam, x, y, z)
    keep = _visible(cam, u, v, keep, float(R32))
    idx = np.nonzero(keep)[0]
    u, v = u[idx], v[idx]
    m64 = np.asarray(m, dtype=f32)[idx].astype(np.float64)
    s64 = float(f32(sigma))
    inv2s2 = 1.0 / (2.0 * s64 * s64)
    norm = 1.0 / (2.0 * math.pi * s64 * s64)
    win = _window(float(R32))
    ones = np.ones(len(idx), dtype=bool)
    for dj in range(-win, win + 1):
        for di in range(-win, win + 1):
            i, j, ox, oy, ok = _covers(cam, u, v, ones, R32, di, dj)
            if not ok.any():
                continue
            o64x = ox[ok].astype(np.float64)
            o64y = oy[ok].astype(np.float64)
            val = m64[ok] * np.exp(-(o64x * o64x + o64y * o64y) * inv2s2) * norm
            np.add.at(img, (j[ok], i[ok]), val)
    return img


def render_pixels(cam: Camera, x, y, z, m, pix_i, pix_j, sigma=1.0, radius_sigmas=3.0):
    """float64 values of individual pixels (pix_i, pix_j), summed over all points."""
    R32 = f32(radius_sigmas) * f32(sigma)
    u, v, keep, _, _, _ = project(cam, x, y, z)
    keep = _visible(cam, u, v, keep, float(R32))
    s64 = float(f32(sigma))
    inv2s2 = 1.0 / (2.0 * s64 * s64)
    norm = 1.0 / (2.0 * math.pi * s64 * s64)
    m32 = np.asarray(m, dtype=f32)
    out = np.zeros(len(pix_i), dtype=np.float64)
    u64 = u.astype(np.float64); v64 = v.astype(np.float64)
    for k, (pi, pj) in enumerate(zip(pix_i, pix_j)):
        near = keep & (np.abs(u64 - (pi + 0.5)) <= float(R32) + 1.0) \
            & (np.abs(v64 - (pj + 0.5)) <= float(R32) + 1.0)
        sel = np.nonzero(near)[0]
        ox = u[sel] - (f32(pi) + f32(0.5))
        oy = v[sel] - (f32(pj) + f32(0.5))
        ok = (np.abs(ox) <= R32) & (np.abs(oy) <= R32)
        o64x = ox[ok].astype(np.float64); o64y = oy[ok].astype(np.float64)
        out[k] = math.fsum((m32[sel][ok].astype(np.float64)
                            * np.exp(-(o64x * o64x + o64y * o64y) * inv2s2) * norm).tolist())
    return out


def render_backward(cam: Camera, x, y, z, m, grad_img, sigma=1.0, radius_sigmas=3.0):
    """Adjoint of `render` with respect to m and xyz (float64).

    dI/dm = G; dI/du = m G (-ox / sigma^2); the derivative of the truncation
    indicator is taken as zero.  Orthographic: du/dx = W, dv/dy = H.
    Perspective: du/dp = (F / zc) r - (F xc / zc^2) f, dv/dp likewise with
    the up vector.
    """
    x = np.asarray(x, dtype=f32); npt = len(x)
    gm = np.zeros(npt); gu = np.zeros(npt); gv = np.zeros(npt)
    gx = np.zeros(npt); gy = np.zeros(npt); gz = np.zeros(npt)
    if npt == 0:
        return gm, np.stack([gx, gy, gz], axis=1)
    g = np.asarray(grad_img, dtype=np.float64)
    R32 = f32(radius_sigmas) * f32(sigma)
    u, v, keep, xc, yc, zc = project(cam, x, y, z)
    keep = _visible(cam, u, v, keep, float(R32))
    s64 = float(f32(sigma))
    inv2s2 = 1.0 / (2.0 * s64 * s64)
    norm = 1.0 / (2.0 * math.pi * s64 * s64)
    m64 = np.asarray(m, dtype=f32).astype(np.float64)
    win = _window(float(R32))
    for dj in range(-win, win + 1):
        for di in range(-win, win + 1):
            i, j, ox, oy, ok = _covers(cam, u, v, keep, R32, di, dj)
            if not ok.any():
                continue
            k = np.nonzero(ok)[0]
            o64x = ox[k].astype(np.float64); o64y = oy[k].astype(np.float64)
            G = np.exp(-(o64x * o64x + o64y * o64y) * inv2s2) * norm
            gp = g[j[k], i[k]]
            np.add.at(gm, k, G * gp)
            np.add.at(gu, k, m64[k] * G * (-o64x / (s64 * s64)) * gp)
            np.add.at(gv, k, m64[k] * G * (-o64y / (s64 * s64)) * gp)
    if cam.projection == 0:
        gx = gu * float(cam.W)
        gy = gv * float(cam.H)
    else:
        F = float(f32(cam.F))
        zc64 = np.where(keep, zc.astype(np.float64), 1.0)
        xc64 = xc.astype(np.float64); yc64 = yc.astype(np.float64)
        r = np.array([float(f32(a)) for a in cam.right])
        up = np.array([float(f32(a)) for a in cam.up])
        fw = np.array([float(f32(a)) for a in cam.fwd])
        a = F / zc64
        bu = F * xc64 / (zc64 * zc64)
        bv = F * yc64 / (zc64 * zc64)
        for ax, out in enumerate((gx, gy, gz)):
            out[:] = gu * (a * r[ax] - bu * fw[ax]) + gv * (a * up[ax] - bv * fw[ax])
        gx[~keep] = 0.0; gy[~keep] = 0.0; gz[~keep] = 0.0
    return gm, np.stack([gx, gy, gz], axis=1)


def render_backward_bound(cam: Camera, x, y, z, m, weight_img, sigma=1.0, radius_sigmas=3.0):
    """Per-point sums of |dI_p/d(parameter)| * weight_img[p] (float64).

    Returns (bm, bxyz [N, 3]): the sums of absolute contributions that bound,
    element by element, how far a gradient sum_p dI_p/d(.) g_p can move when
    each g_p (or each term) carries an error of at most weight_img[p].  Same
    footprint and projection as `render_backward`.  The position bound adds
    the magnitudes of the projection Jacobian's terms separately (perspective:
    (|F/zc| |r| + |F xc/zc^2| |f|) for u, likewise for v), so it also covers
    rounding in an evaluation that cancels those terms.
    """
    x = np.asarray(x, dtype=f32); npt = len(x)
    bm = np.zeros(npt); bu = np.zeros(npt); bv = np.zeros(npt)
    if npt == 0:
        return bm, np.zeros((0, 3))
    wimg = np.abs(np.asarray(weight_img, dtype=np.float64))
    R32 = f32(radius_sigmas) * f32(sigma)
    u, v, keep, xc, yc, zc = project(cam, x, y, z)
    keep = _visible(cam, u, v, keep, float(R32))
    s64 = float(f32(sigma))
    inv2s2 = 1.0 / (2.0 * s64 * s64)
    norm = 1.0 / (2.0 * math.pi * s64 * s64)
    m64 = np.abs(np.asarray(m, dtype=f32).astype(np.float64))
    win = _window(float(R32))
    for dj in range(-win, win + 1):
        for di in range(-win, win + 1):
            i, j, ox, oy, ok = _covers(cam, u, v, keep, R32, di, dj)
            if not ok.any():
                continue
            k = np.nonzero(ok)[0]
            o64x = ox[k].astype(np.float64); o64y = oy[k].astype(np.float64)
            G = np.exp(-(o64x * o64x + o64y * o64y) * inv2s2) * norm
            wp = wimg[j[k], i[k]]
            np.add.at(bm, k, G * wp)
            np.add.at(bu, k, m64[k] * G * np.abs(o64x) / (s64 * s64) * wp)
            np.add.at(bv, k, m64[k] * G * np.abs(o64y) / (s64 * s64) * wp)
    out = np.zeros((npt, 3))
    if cam.projection == 0:
        out[:, 0] = bu * float(cam.W)
        out[:, 1] = bv * float(cam.H)
    else:
        F = float(f32(cam.F))
        zc64 = np.where(keep, zc.astype(np.float64), 1.0)
        xc64 = xc.astype(np.float64); yc64 = yc.astype(np.float64)
        r = np.array([float(f32(a)) for a in cam.right])
        up = np.array([float(f32(a)) for a in cam.up])
        fw = np.array([float(f32(a)) for a in cam.fwd])
        a = F / zc64
        cu = F * xc64 / (zc64 * zc64)
        cv = F * yc64 / (zc64 * zc64)
        for ax in range(3):
            out[:, ax] = (bu * (np.abs(a * r[ax]) + np.abs(cu * fw[ax]))
                          + bv * (np.abs(a * up[ax]) + np.abs(cv * fw[ax])))
        out[~keep] = 0.0
    return bm, out

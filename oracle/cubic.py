"""Radial cubic blob, its adjoint, and the second (attribute) channel --
plain definition (CPU oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The rendering paragraph of the paper evaluates a radial cubic function for
every pixel of every point.  The reading used here is the compact cubic
spline of smoothed-particle hydrodynamics (Monaghan and Lattanzio 1985, in
the form used by Springel's GADGET codes), normalised in two dimensions:

    W(r; h) = 40 / (7 pi h^2) w(r / h)
    w(q)    = 1 - 6 q^2 + 6 q^3      for 0 <= q <= 1/2
            = 2 (1 - q)^3             for 1/2 < q < 1
            = 0                       for q >= 1

w is twice continuously differentiable, so the blob has no truncation edge.

Pixel radius h (float32):
* fixed:        h = h_px;
* world size (perspective only): h = min(max(fl(fl(F h_world) / zc), 1), 16),
  the projected radius of a sphere of radius h_world, clamped to [1, 16]
  pixels (a point never shrinks below one pixel nor grows past 16).

Screen position and pixel offsets use the same pinned float32 sequence as the
Gaussian splat (`splat.project`; ox = fl(u - (i + 1/2)), oy likewise).  A
pixel receives the point iff fl64(ox^2) + fl64(oy^2), rounded once in float64,
is below fl64(h^2) (both squares are exact in float64), and it lies in the
image.  From there on everything is float64:

    I[j, i]     += m W(r; h)            r = sqrt(ox^2 + oy^2)
    A[j, i]     += m a W(r; h)          (optional second channel, attribute a)

The second channel carries a per-point attribute: 0/1 for ID highlighting
(the paper's highlighting paragraph), a colour value for interpolated
playback.
"""
from __future__ import annotations

import math

import numpy as np

from .splat import Camera, project

f32 = np.float32

H_MIN_PX = 1.0
H_MAX_PX = 16.0
NORM = 40.0 / (7.0 * math.pi)


def w_profile(q):
    """The dimensionless spline w(q) (float64)."""
    q = np.asarray(q, dtype=np.float64)
    return np.where(q <= 0.5, 1.0 - 6.0 * q * q + 6.0 * q ** 3,
                    np.where(q < 1.0, 2.0 * (1.0 - q) ** 3, 0.0))


def dw_over_q(q):
    """w'(q) / q (finite at q = 0)."""
    q = np.asarray(q, dtype=np.float64)
    qs = np.where(q > 0, q, 1.0)
    return np.where(q <= 0.5, -12.0 + 18.0 * q, np.where(q < 1.0, -6.0 * (1.0 - q) ** 2 / qs, 0.0))


def dw(q):
    """w'(q)."""
    q = np.asarray(q, dtype=np.float64)
    return np.where(q <= 0.5, -12.0 * q + 18.0 * q * q, np.where(q < 1.0, -6.0 * (1.0 - q) ** 2, 0.0))


def pixel_radius(cam: Camera, zc, h_px, h_world):
    """(h float32 per point, clamped mask) by the pinned sequence; h_world may
    be one radius or one per point."""
    if np.any(np.asarray(h_world) != 0):
        if cam.projection != 1:
            raise ValueError("a world-space size needs a perspective camera")
        zs = np.asarray(zc, dtype=f32)
        hw = f32(cam.F) * np.asarray(h_world, dtype=f32)
        hp = hw / np.where(zs > 0, zs, f32(1.0))
        h = np.minimum(np.maximum(hp, f32(H_MIN_PX)), f32(H_MAX_PX)).astype(f32)
        clamped = (hp < f32(H_MIN_PX)) | (hp > f32(H_MAX_PX))
        return h, clamped
    return f32(h_px), None


def _setup(cam, x, y, z, h_px, h_world):
    x = np.asarray(x, dtype=f32)
    u, v, keep, xc, yc, zc = project(cam, x, y, z)
    if np.any(np.asarray(h_world) != 0):
        h, clamped = pixel_radius(cam, zc, h_px, h_world)
    else:
        h = np.full(len(x), f32(h_px), dtype=f32)
        clamped = np.zeros(len(x), dtype=bool)
    u64 = u.astype(np.float64); v64 = v.astype(np.float64); h64 = h.astype(np.float64)
    lim = h64 + 4.0
    vis = keep & np.isfinite(u64) & np.isfinite(v64) & (u64 > -lim) & (u64 < cam.W + lim) \
        & (v64 > -lim) & (v64 < cam.H + lim)
    return u, v, h, vis, clamped, xc, yc, zc


def _pairs(cam, u, v, h, vis):
    """Yield (k, i, j, ox, oy, r2) for every covered (point, pixel), vectorised by window offset."""
    idx = np.nonzero(vis)[0]
    if len(idx) == 0:
        return
    hm = float(h[idx].max())
    win = int(math.ceil(hm)) + 2
    uu, vv, hh = u[idx], v[idx], h[idx].astype(np.float64)
    fu = np.floor(uu.astype(np.float64)).astype(np.int64)
    fv = np.floor(vv.astype(np.float64)).astype(np.int64)
    for dj in range(-win, win + 1):
        for di in range(-win, win + 1):
            i = fu + di
            j = fv + dj
            ox = uu - (i.astype(f32) + f32(0.5))
            oy = vv - (j.astype(f32) + f32(0.5))
            r2 = ox.astype(np.float64) ** 2 + oy.astype(np.float64) ** 2
            ok = (r2 < hh * hh) & (i >= 0) & (i < cam.W) & (j >= 0) & (j < cam.H)
            if ok.any():
                yield idx[ok], i[ok], j[ok], ox[ok], oy[ok], r2[ok]


def render(cam: Camera, x, y, z, m, h_px=1.5, h_world=0.0, aux=None):
    """float64 image [H, W] (and the attribute channel when aux is given)."""
    img = np.zeros((cam.H, cam.W))
    aimg = np.zeros((cam.H, cam.W)) if aux is not None else None
    if len(np.asarray(x)) == 0:
        return (img, aimg) if aux is not None else img
    u, v, h, vis, _, _, _, _ = _setup(cam, x, y, z, h_px, h_world)
    m64 = np.asarray(m, dtype=f32).astype(np.float64)
    a64 = np.asarray(aux, dtype=f32).astype(np.float64) if aux is not None else None
    h64 = h.astype(np.float64)
    for k, i, j, ox, oy, r2 in _pairs(cam, u, v, h, vis):
        q = np.sqrt(r2) / h64[k]
        val = m64[k] * NORM / (h64[k] * h64[k]) * w_profile(q)
        np.add.at(img, (j, i), val)
        if aux is not None:
            np.add.at(aimg, (j, i), val * a64[k])
    return (img, aimg) if aux is not None else img


def render_backward(cam: Camera, x, y, z, m, grad_img, h_px=1.5, h_world=0.0, bound_weights=None):
    """Adjoint of `render` with respect to m and xyz (float64).

    dI/dm = W; dI/dox = m NORM/h^2 w'(q) ox / (r h) = m NORM/h^4 (w'(q)/q) ox;
    with a world-space size and an unclamped radius h = F h_world / zc also
    dI/dh = m NORM/h^3 (-2 w(q) - q w'(q)), dh/dp = -(h / zc) f.
    Projection Jacobians as in `splat.render_backward`.

    With bound_weights (an image of non-negative weights), returns instead the
    per-point sums of |term| * weight for m and for x, y, z (the projection
    terms added in magnitude), an error scale for each gradient element.
    """
    x = np.asarray(x, dtype=f32); npt = len(x)
    gm = np.zeros(npt); gu = np.zeros(npt); gv = np.zeros(npt); gh = np.zeros(npt)
    if npt == 0:
        return gm, np.zeros((0, 3))
    absmode = bound_weights is not None
    g = np.abs(np.asarray(bound_weights, dtype=np.float64)) if absmode else np.asarray(grad_img, dtype=np.float64)
    u, v, h, vis, clamped, xc, yc, zc = _setup(cam, x, y, z, h_px, h_world)
    m64 = np.asarray(m, dtype=f32).astype(np.float64)
    h64 = h.astype(np.float64)
    A = np.abs if absmode else (lambda t: t)
    for k, i, j, ox, oy, r2 in _pairs(cam, u, v, h, vis):
        hk = h64[k]
        q = np.sqrt(r2) / hk
        gp = g[j, i]
        base = NORM / (hk * hk)
        np.add.at(gm, k, A(base * w_profile(q)) * gp)
        t = m64[k] * base / (hk * hk) * dw_over_q(q)
        np.add.at(gu, k, A(t * ox.astype(np.float64)) * gp)
        np.add.at(gv, k, A(t * oy.astype(np.float64)) * gp)
        if h_world:
            th = m64[k] * base / hk * (-2.0 * w_profile(q) - q * dw(q))
            np.add.at(gh, k, A(th) * gp)
    out = np.zeros((npt, 3))
    if cam.projection == 0:
        out[:, 0] = gu * float(cam.W)
        out[:, 1] = gv * float(cam.H)
        return gm, out
    F = float(f32(cam.F))
    keep = vis
    zc64 = np.where(keep, zc.astype(np.float64), 1.0)
    xc64 = xc.astype(np.float64); yc64 = yc.astype(np.float64)
    r = np.array([float(f32(a)) for a in cam.right])
    up = np.array([float(f32(a)) for a in cam.up])
    fw = np.array([float(f32(a)) for a in cam.fwd])
    a = F / zc64
    bu = F * xc64 / (zc64 * zc64)
    bv = F * yc64 / (zc64 * zc64)
    dh = np.where(clamped, 0.0, -h64 / zc64) if h_world else np.zeros(npt)
    for ax in range(3):
        if absmode:
            out[:, ax] = (gu * (np.abs(a * r[ax]) + np.abs(bu * fw[ax])) + gv * (np.abs(a * up[ax]) + np.abs(bv * fw[ax]))
                          + gh * np.abs(dh * fw[ax]))
        else:
            out[:, ax] = gu * (a * r[ax] - bu * fw[ax]) + gv * (a * up[ax] - bv * fw[ax]) + gh * dh * fw[ax]
    out[~keep] = 0.0
    return gm, out

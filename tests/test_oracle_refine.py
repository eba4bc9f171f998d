"""Pins for the refinement oracle (oracle/refine.py): finite differences of
the loss, Adam against torch's float64 Adam and its first-step closed form,
and the mass / cube projection.  CPU only."""
import math

import numpy as np
import pytest

from oracle import refine, splat


def _setup(seed=0):
    """Two orthographic views of different sizes (W, H powers of two, so the
    float32 projection u = x W is exact and positions can move by exact steps),
    30 stored points with masses of few mantissa bits, 400 full particles."""
    rng = np.random.default_rng(seed)
    cams = [splat.Camera(0, 64, 64), splat.Camera(0, 32, 32)]
    n, Nf = 30, 400
    x = (0.3 + 0.4 * rng.random(n)).astype(np.float32)
    y = (0.3 + 0.4 * rng.random(n)).astype(np.float32)
    z = np.zeros(n, np.float32)
    m = ((1 + rng.integers(0, 16, n)) / 16.0).astype(np.float32)
    fx = (0.3 + 0.4 * rng.random(Nf)).astype(np.float32)
    fy = (0.3 + 0.4 * rng.random(Nf)).astype(np.float32)
    fm = np.full(Nf, np.float32(n / Nf))
    targets = []
    for c in cams:
        F = splat.render(c, fx, fy, np.zeros(Nf, np.float32), fm)
        targets.append((F, float(F.mean())))
    return cams, targets, x, y, z, m


def _loss(cams, targets, x, y, z, m):
    return refine.loss_and_grad(cams, targets, x, y, z, m)[0]


def test_loss_gradient_finite_differences():
    """Central differences of the float64 loss along exact float32 steps: in
    mass (the image is linear in m; steps of m 2^-12 are exact for masses with
    five mantissa bits) and in x, y (steps of 2^-22 are exact for coordinates in
    [0.25, 1); u = x W is exact for W a power of two).  Points within 1e-3
    pixel of a truncation edge are skipped."""
    cams, targets, x, y, z, m = _setup(1)
    L, gm, gx = refine.loss_and_grad(cams, targets, x, y, z, m)
    assert L > 0
    checked = 0
    for k in range(len(x)):
        hm = np.float32(m[k] * 2.0 ** -12)
        mp = m.copy(); mp[k] = m[k] + hm
        mm = m.copy(); mm[k] = m[k] - hm
        fd = (_loss(cams, targets, x, y, z, mp) - _loss(cams, targets, x, y, z, mm)) / (2.0 * float(hm))
        assert abs(fd - gm[k]) <= 1e-6 * abs(fd) + 1e-12, (k, fd, gm[k])
        edge = False
        for c in cams:
            for a, S in ((x[k], c.W), (y[k], c.H)):
                f = (float(a) * S - 0.5) % 1.0
                edge |= min(f, 1.0 - f) < 1e-3
        if edge:
            continue
        h = 2.0 ** -22
        for ax, arr in ((0, x), (1, y)):
            ap = arr.copy(); ap[k] = arr[k] + np.float32(h)
            an = arr.copy(); an[k] = arr[k] - np.float32(h)
            args_p = (ap, y) if ax == 0 else (x, ap)
            args_n = (an, y) if ax == 0 else (x, an)
            fd = (_loss(cams, targets, *args_p, z, m) - _loss(cams, targets, *args_n, z, m)) / (2.0 * h)
            assert abs(fd - gx[k, ax]) <= 1e-5 * abs(fd) + 1e-9 * np.abs(gx).max(), (k, ax, fd, gx[k, ax])
        assert gx[k, 2] == 0.0       # orthographic along z: the image does not depend on z
        checked += 1
    assert checked >= 20


def test_grad_theta_chain_rule():
    """d/dtheta of the loss at m = exp(theta) by central differences in theta
    (float64 masses rounded to float32: the step is taken large enough that
    the rounding stays below the tolerance)."""
    cams, targets, x, y, z, m = _setup(2)
    L, gm, gx = refine.loss_and_grad(cams, targets, x, y, z, m)
    gth = refine.grad_theta(m, gm)
    th = np.log(m.astype(np.float64))
    for k in range(0, len(m), 5):
        h = 1e-3
        tp = th.copy(); tp[k] += h
        tn = th.copy(); tn[k] -= h
        fd = (_loss(cams, targets, x, y, z, np.exp(tp).astype(np.float32))
              - _loss(cams, targets, x, y, z, np.exp(tn).astype(np.float32))) / (2 * h)
        assert abs(fd - gth[k]) <= 2e-4 * abs(fd) + 1e-10, (k, fd, gth[k])


def test_adam_matches_torch_float64():
    """Three steps of the oracle's Adam equal torch.optim.Adam on float64 CPU tensors."""
    import torch
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 0, 50) for _ in range(3)]
    for lr in (1e-2, 3e-4):
        t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([t], lr=lr)
        p, ma, va = p0.copy(), np.zeros(50), np.zeros(50)
        for step, g in enumerate(grads, start=1):
            t.grad = torch.tensor(g, dtype=torch.float64)
            opt.step()
            p, ma, va = refine.adam_update(p, g, ma, va, step, lr)
            assert np.allclose(t.detach().numpy(), p, rtol=1e-14, atol=1e-15)
            st = opt.state[t]
            assert np.allclose(st["exp_avg"].numpy(), ma, rtol=1e-14, atol=0)
            assert np.allclose(st["exp_avg_sq"].numpy(), va, rtol=1e-14, atol=0)


def test_adam_first_step_closed_form():
    """From zero moments the first step moves every parameter by lr g / (|g| + eps)."""
    g = np.array([1e-3, -2.0, 5e-9, -1e-12, 0.0])
    p, _, _ = refine.adam_update(np.zeros(5), g, np.zeros(5), np.zeros(5), 1, 0.01)
    want = -0.01 * g / (np.abs(g) + refine.EPS)
    assert np.allclose(p, want, rtol=1e-12, atol=0)


def test_project_mass_and_cube():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(40) - 8.0
    xyz = rng.uniform(-0.1, 0.4, (40, 3))
    lo, side, M = (0.0, 0.125, 0.25), 0.125, 0.37
    th2, xyz2 = refine.project(th, xyz, lo, side, M)
    assert abs(math.fsum(np.exp(th2).tolist()) - M) <= 1e-14 * M
    # a uniform shift of theta changes nothing after the projection
    th3, _ = refine.project(th + 3.7, xyz, lo, side, M)
    assert np.allclose(th3, th2, rtol=0, atol=1e-13)
    # masses keep their ratios
    assert np.allclose(th2 - th2[0], th - th[0], rtol=0, atol=1e-13)
    for ax in range(3):
        a, b = lo[ax], lo[ax] + side
        assert np.all((xyz2[:, ax] >= a) & (xyz2[:, ax] <= b))
        inside = (xyz[:, ax] >= a) & (xyz[:, ax] <= b)
        assert np.array_equal(xyz2[inside, ax], xyz[inside, ax])
        assert np.all(xyz2[xyz[:, ax] < a, ax] == a) and np.all(xyz2[xyz[:, ax] > b, ax] == b)


def test_gradient_bounds_cover_perturbed_images():
    """The per-element bounds returned with image_rel_err = e cover the change
    of the gradient when every image pixel (stored points and full set) is
    scaled by a factor within 1 +- e."""
    cams, targets, x, y, z, m = _setup(5)
    e = 1e-5
    L, gm, gx, bL, bm, bx = refine.loss_and_grad(cams, targets, x, y, z, m, image_rel_err=e)
    rng = np.random.default_rng(6)
    # perturb the targets' images by relative errors within e, recompute
    pert = []
    for F, Fb in targets:
        F2 = F * (1.0 + e * rng.uniform(-1, 1, F.shape))
        pert.append((F2, float(F2.mean())))
    L2, gm2, gx2 = refine.loss_and_grad(cams, pert, x, y, z, m)
    assert abs(L2 - L) <= bL
    assert np.all(np.abs(gm2 - gm) <= bm + 1e-300)
    assert np.all(np.abs(gx2 - gx) <= bx + 1e-300)

"""Differentiable splat and node refinement on the GPU.

The adjoint goes through torch.autograd into the HIP backward kernel; it is
checked against the float64 oracle adjoint and against float64 central
finite differences of an independent float64 re-evaluation of the blobs.
"""
import math

import numpy as np
import pytest

import synth
from oracle import lod as olod
from oracle import splat as osplat
from paper_0811_2055_amd import lib

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def test_decode_matches_oracle():
    import torch
    s = synth.small_clustered(30000, 81)
    n = 200
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=n, D=5, seed=2)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=n, max_depth=5, seed=2))
    nodes = np.array([0, 3, 5, 17, ref.n_nodes - 1], dtype=np.int64)
    ids = torch.from_numpy(nodes.astype(np.int32)).cuda().view(torch.uint32)
    nid = torch.tensor([len(nodes)], dtype=torch.int64).cuda().view(torch.uint64)
    x, y, z, m, cnt = lib.decode_nodes(tree, ids, nid, 100000)
    k = int(lib._to_numpy(cnt)[0])
    rx, ry, rz, rm = olod.decoded_points(ref, nodes)
    assert k == len(rx)
    for got, want in ((x, rx), (y, ry), (z, rz), (m, rm)):
        got = got[:k].cpu().numpy()
        if want is rm:
            assert np.all(np.abs(got.view(np.int32).astype(np.int64) - want.view(np.int32)) <= 1)
        else:
            assert np.array_equal(got, want)


def _cam(proj, W, H):
    if proj == "ortho":
        return lib.Camera.ortho(W, H), osplat.Camera(0, W, H)
    c = lib.Camera.look_at((0.55, 0.45, -0.8), (0.5, 0.5, 0.5), W, H, fov_deg=50.0)
    return c, osplat.Camera(1, W, H, c.pos, c.right, c.up, c.fwd, c.F, c.near)


@pytest.mark.parametrize("proj", ["ortho", "persp"])
def test_autograd_matches_oracle_adjoint(proj):
    import torch
    from paper_0811_2055_amd.autograd import splat_render
    s = synth.small_clustered(4000, 82)
    cam, ocam = _cam(proj, 96, 80)
    g = np.random.default_rng(1).standard_normal((80, 96)).astype(np.float32)
    xs = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (s.x, s.y, s.z, s.m)]
    img = splat_render(*xs, cam)
    (img * torch.from_numpy(g).cuda()).sum().backward()
    rm, rp = osplat.render_backward(ocam, s.x, s.y, s.z, s.m, g.astype(np.float64))
    for t, want in zip(xs, (rp[:, 0], rp[:, 1], rp[:, 2], rm)):
        got = t.grad.cpu().numpy().astype(np.float64)
        scale = np.abs(want).max() + 1e-30
        assert np.max(np.abs(got - want)) <= 2e-5 * scale


def test_gradient_fp64_finite_differences():
    """Float64 central differences on a subset of points, away from truncation edges."""
    import torch
    from paper_0811_2055_amd.autograd import splat_render
    rng = np.random.default_rng(7)
    Np, W, H = 300, 64, 64
    x = (0.25 + 0.5 * rng.random(Np)).astype(np.float32)
    y = (0.25 + 0.5 * rng.random(Np)).astype(np.float32)
    z = (0.25 + 0.5 * rng.random(Np)).astype(np.float32)
    m = rng.uniform(0.5, 1.5, Np).astype(np.float32)
    cam = lib.Camera.look_at((0.5, 0.52, -0.7), (0.5, 0.5, 0.5), W, H, fov_deg=60.0)
    g = rng.standard_normal((H, W))
    xs = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (x, y, z, m)]
    img = splat_render(*xs, cam)
    (img * torch.from_numpy(g.astype(np.float32)).cuda()).sum().backward()
    grads = [t.grad.cpu().numpy().astype(np.float64) for t in xs]
    pos = np.array(cam.pos); r = np.array(cam.right); up = np.array(cam.up); fw = np.array(cam.fwd)

    def point_loss(k, p, mk):
        d = p - pos
        xc, yc, zc = d @ r, d @ up, d @ fw
        u = cam.F * xc / zc + W / 2
        v = cam.F * yc / zc + H / 2
        tot = 0.0
        for j in range(max(0, int(v) - 5), min(H, int(v) + 6)):
            for i in range(max(0, int(u) - 5), min(W, int(u) + 6)):
                ox, oy = u - (i + 0.5), v - (j + 0.5)
                if abs(ox) <= 3 and abs(oy) <= 3:
                    tot += mk * math.exp(-(ox * ox + oy * oy) / 2) / (2 * math.pi) * g[j, i]
        return tot, u, v

    checked = 0
    for k in rng.choice(Np, 40, replace=False):
        p0 = np.array([x[k], y[k], z[k]], dtype=np.float64)
        _, u, v = point_loss(k, p0, float(m[k]))
        fu, fv = (u - 0.5) % 1.0, (v - 0.5) % 1.0
        if min(fu, 1 - fu, fv, 1 - fv) < 1e-3:
            continue                     # within reach of a truncation edge
        h = 1e-6
        for ax in range(3):
            e = np.zeros(3); e[ax] = h
            fd = (point_loss(k, p0 + e, float(m[k]))[0] - point_loss(k, p0 - e, float(m[k]))[0]) / (2 * h)
            assert abs(fd - grads[ax][k]) <= 2e-3 * (abs(fd) + 1e-3 * np.abs(grads[ax]).max()), (k, ax)
        fdm = (point_loss(k, p0, float(m[k]) * (1 + 1e-6))[0] - point_loss(k, p0, float(m[k]) * (1 - 1e-6))[0]) \
            / (2e-6 * float(m[k]))
        assert abs(fdm - grads[3][k]) <= 1e-4 * (abs(fdm) + 1e-6)
        checked += 1
    assert checked >= 20


def test_refinement_lowers_heldout_error():
    import torch
    from paper_0811_2055_amd import refine
    s = synth.small_clustered(60000, 83)
    n = 1500
    d = to_dev(s)
    b = lib.Builder(s.n, lib.BuildParams(n=n, max_depth=3, seed=5))
    tree = b.build(*d)
    h = tree.host()
    v = next(i for i in range(h["n_nodes"]) if h["depth"][i] == 1 and h["first_child"][i] != lib.NONE)
    dd = int(h["depth"][v])
    cell = int(h["prefix"][v]) & ((1 << (3 * dd)) - 1)
    c = olod.deinterleave(cell, dd)
    side = 2.0 ** -dd
    lo = [ci * side for ci in c]
    ids = torch.tensor([v], dtype=torch.int32).cuda().view(torch.uint32)
    nid = torch.tensor([1], dtype=torch.int64).cuda().view(torch.uint64)
    px, py, pz, pm, cnt = lib.decode_nodes(tree, ids, nid, n)
    order = lib._to_numpy(b.view(1, torch.uint32)).astype(np.int64)
    pb, pc = int(h["part_begin"][v]), int(h["part_count"][v])
    members = torch.from_numpy(order[pb:pb + pc]).cuda()
    full = [a[members].contiguous() for a in d]
    centre = [l + side / 2 for l in lo]
    train = refine.node_views(centre, side, n, 4, seed=0, W=256, H=256)
    test = refine.node_views(centre, side, n, 4, seed=100, W=256, H=256)
    res, _ = refine.refine_node(px, py, pz, pm, full, lo, side, float(h["node_mass"][v]), train, test, steps=60)
    print(res, flush=True)
    assert res.loss_last < res.loss_first
    assert res.e_log_after < res.e_log_before

"""HIP splat, adjoint, cut and LOD render vs the CPU oracle, through the C ABI.

Images: every pixel the oracle leaves at zero is exactly zero, and every
positive pixel is within 1e-5 relative of the float64 oracle.
"""
import numpy as np
import pytest

import synth
from oracle import cut as ocut
from oracle import lod as olod
from oracle import splat as osplat
from paper_0811_2055_amd import lib

from gpu_util import image_rel_err, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _cams(W, H):
    out = [("ortho", lib.Camera.ortho(W, H), osplat.Camera(0, W, H))]
    for name, pos, tgt in (("outside", (0.5, 0.5, -0.9), (0.5, 0.5, 0.5)),
                           ("inside", (0.3, 0.6, 0.4), (0.7, 0.2, 0.9)),
                           ("oblique", (1.4, -0.3, 0.2), (0.5, 0.5, 0.5))):
        c = lib.Camera.look_at(pos, tgt, W, H, fov_deg=60.0)
        o = osplat.Camera(1, W, H, c.pos, c.right, c.up, c.fwd, c.F, c.near)
        out.append((name, c, o))
    return out


@pytest.mark.parametrize("sigma,radius", [(1.0, 3.0), (2.0, 2.5), (0.7, 3.0)])
def test_splat_matches_oracle(sigma, radius):
    s = synth.small_clustered(40000, 51)
    d = to_dev(s)
    for name, cam, ocam in _cams(200, 150):
        print(f"[splat parity] {name} sigma={sigma}", flush=True)
        img = lib.splat(*d, cam, sigma, radius).cpu().numpy()
        ref = osplat.render(ocam, s.x, s.y, s.z, s.m, sigma, radius)
        err, zeros_ok = image_rel_err(img, ref)
        assert zeros_ok, name
        assert err <= TOL, (name, err)


def test_splat_config1_ortho_full():
    s = synth.config1()
    img = lib.splat(*to_dev(s), lib.Camera.ortho(256, 256)).cpu().numpy()
    ref = osplat.render(osplat.Camera(0, 256, 256), s.x, s.y, s.z, s.m)
    err, zeros_ok = image_rel_err(img, ref)
    print(f"[splat parity] config1 256^2 max rel err {err:.3e}", flush=True)
    assert zeros_ok and err <= TOL


def test_splat_dense_pixel():
    """A single pixel receiving 300k contributions stays within tolerance."""
    rng = np.random.default_rng(3)
    N = 300000
    x = (0.5 + 0.5 / 64 * (rng.random(N) - 0.5)).astype(np.float32)
    y = (0.5 + 0.5 / 64 * (rng.random(N) - 0.5)).astype(np.float32)
    s = synth.Snapshot(x, y, np.zeros(N, np.float32), rng.uniform(0.5, 1.5, N).astype(np.float32))
    img = lib.splat(*to_dev(s), lib.Camera.ortho(64, 64)).cpu().numpy()
    ref = osplat.render(osplat.Camera(0, 64, 64), s.x, s.y, s.z, s.m)
    err, zeros_ok = image_rel_err(img, ref)
    assert zeros_ok and err <= TOL, err


def test_splat_empty_and_offscreen():
    import torch
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    img = lib.splat(e, e, e, e, lib.Camera.ortho(32, 48))
    assert img.shape == (48, 32) and float(img.abs().max()) == 0.0
    # everything behind the camera
    s = synth.small_clustered(1000, 2)
    cam = lib.Camera.look_at((0.5, 0.5, 2.0), (0.5, 0.5, 3.0), 32, 32)
    img = lib.splat(*to_dev(s), cam)
    assert float(img.abs().max()) == 0.0


@pytest.mark.parametrize("proj", ["ortho", "outside", "inside"])
def test_backward_matches_oracle(proj):
    """Every gradient element within 1e-5 of its own error scale: the sum of
    the absolute terms that make it up (oracle `render_backward_bound` with
    weights |g|), so points with small gradients are checked as tightly as
    large ones."""
    import torch
    s = synth.small_clustered(3000, 61)
    cam, ocam = {n: (c, o) for n, c, o in _cams(96, 80)}[proj]
    rng = np.random.default_rng(5)
    g = rng.standard_normal((80, 96)).astype(np.float32)
    gm, gx, gy, gz = lib.splat_backward(*to_dev(s), torch.from_numpy(g).cuda(), cam)
    rm, rp = osplat.render_backward(ocam, s.x, s.y, s.z, s.m, g.astype(np.float64))
    bm, bp = osplat.render_backward_bound(ocam, s.x, s.y, s.z, s.m, np.abs(g.astype(np.float64)))
    checked = 0
    for name, got, want, bound in (("m", gm, rm, bm), ("x", gx, rp[:, 0], bp[:, 0]),
                                   ("y", gy, rp[:, 1], bp[:, 1]), ("z", gz, rp[:, 2], bp[:, 2])):
        got = got.cpu().numpy().astype(np.float64)
        err = np.abs(got - want)
        tol = 1e-5 * bound
        bad = np.nonzero(err > tol)[0]
        assert bad.size == 0, (proj, name, bad[:5], got[bad[:5]], want[bad[:5]], bound[bad[:5]])
        # points the blob misses entirely have an exact zero gradient
        assert np.all(got[bound == 0] == 0.0), (proj, name)
        checked += int(np.count_nonzero(bound > 0))
    assert checked >= 1000


@pytest.mark.parametrize("proj", ["ortho", "outside"])
def test_adjoint_dot_product_mass(proj):
    """<J d, g> = <d, J^T g> through the HIP pair: the image is linear in the
    masses, so rendering the masses d gives J d exactly; both sides agree to
    the summed error scale of their terms."""
    import torch
    s = synth.small_clustered(5000, 62)
    cam, ocam = {n: (c, o) for n, c, o in _cams(96, 80)}[proj]
    rng = np.random.default_rng(6)
    g = rng.standard_normal((80, 96)).astype(np.float32)
    delta = rng.uniform(-1.0, 1.0, s.n).astype(np.float32)
    x, y, z, m = to_dev(s)
    Jd = lib.splat(x, y, z, torch.from_numpy(delta).cuda(), cam).cpu().numpy().astype(np.float64)
    gm, _, _, _ = lib.splat_backward(x, y, z, m, torch.from_numpy(g).cuda(), cam)
    lhs = float(np.sum(Jd * g.astype(np.float64)))
    rhs = float(np.sum(delta.astype(np.float64) * gm.cpu().numpy().astype(np.float64)))
    bm, _ = osplat.render_backward_bound(ocam, s.x, s.y, s.z, s.m, np.abs(g.astype(np.float64)))
    scale = float(np.sum(np.abs(delta) * bm))
    assert scale > 0
    assert abs(lhs - rhs) <= 2e-5 * scale, (lhs, rhs, scale)


def test_adjoint_dot_product_position():
    """<J d, g> = <d, J^T g> for a random direction d of all point positions:
    the left side by float64 central differences of an independent float64
    evaluation of the blobs (each point's own footprint), the right side from
    the HIP adjoint.  Points within 1e-3 pixel of a truncation edge get d = 0."""
    import math
    import torch
    rng = np.random.default_rng(9)
    Np, W, H = 400, 64, 64
    x = (0.3 + 0.4 * rng.random(Np)).astype(np.float32)
    y = (0.3 + 0.4 * rng.random(Np)).astype(np.float32)
    z = (0.3 + 0.4 * rng.random(Np)).astype(np.float32)
    m = rng.uniform(0.5, 1.5, Np).astype(np.float32)
    cam = lib.Camera.look_at((0.5, 0.52, -0.7), (0.5, 0.5, 0.5), W, H, fov_deg=60.0)
    g = rng.standard_normal((H, W))
    dev = [torch.from_numpy(a).cuda() for a in (x, y, z, m)]
    _, gx, gy, gz = lib.splat_backward(*dev, torch.from_numpy(g.astype(np.float32)).cuda(), cam)
    G = np.stack([t.cpu().numpy().astype(np.float64) for t in (gx, gy, gz)], axis=1)
    pos = np.array(cam.pos, dtype=np.float64); r = np.array(cam.right); up = np.array(cam.up)
    fw = np.array(cam.fwd)

    def uv(p):
        d = p - pos
        zc = d @ fw
        return cam.F * (d @ r) / zc + W / 2, cam.F * (d @ up) / zc + H / 2

    def contrib(p, mk):
        u, v = uv(p)
        tot, ab = 0.0, 0.0
        for j in range(max(0, int(v) - 5), min(H, int(v) + 6)):
            for i in range(max(0, int(u) - 5), min(W, int(u) + 6)):
                ox, oy = u - (i + 0.5), v - (j + 0.5)
                if abs(ox) <= 3 and abs(oy) <= 3:
                    t = mk * math.exp(-(ox * ox + oy * oy) / 2) / (2 * math.pi) * g[j, i]
                    tot += t
        return tot

    dirs = rng.standard_normal((Np, 3))
    h = 1e-7
    lhs, rhs, scale = 0.0, 0.0, 0.0
    used = 0
    for k in range(Np):
        p0 = np.array([x[k], y[k], z[k]], dtype=np.float64)
        u, v = uv(p0)
        fu, fv = (u - 0.5) % 1.0, (v - 0.5) % 1.0
        if min(fu, 1 - fu, fv, 1 - fv) < 1e-3:
            continue
        dk = dirs[k]
        fd = (contrib(p0 + h * dk, float(m[k])) - contrib(p0 - h * dk, float(m[k]))) / (2 * h)
        lhs += fd
        rhs += float(dk @ G[k])
        scale += float(np.abs(dk) @ np.abs(G[k]))
        used += 1
    assert used > 300
    assert abs(lhs - rhs) <= 1e-4 * scale, (lhs, rhs, scale)


def _tree(s, n, D, seed=0):
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=n, D=D, seed=seed)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=n, max_depth=D, seed=seed))
    return ref, tree


def test_cut_matches_oracle():
    s = synth.config1()
    n = 256
    ref, tree = _tree(s, n, 6)
    for name, cam, ocam in _cams(256, 256):
        for tau in (0.5, 1.0, 4.0):
            ids, nsel = lib.select_nodes(tree, cam, tau, n)
            k = int(lib._to_numpy(nsel)[0])
            got = lib._to_numpy(ids[:k]).astype(np.int64)
            want = ocut.select(ref, ocam, tau, n)
            assert np.array_equal(got, want), (name, tau, len(got), len(want))


def test_lod_render_matches_oracle():
    s = synth.small_clustered(60000, 71)
    n = 300
    ref, tree = _tree(s, n, 6)
    for name, cam, ocam in _cams(160, 160):
        ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
        want_ids = ocut.select(ref, ocam, 1.0, n)
        img = lib.splat_lod(tree, ids, nsel, tree.point_capacity, cam).cpu().numpy()
        px, py, pz, pm = olod.decoded_points(ref, want_ids)
        refimg = osplat.render(ocam, px, py, pz, pm)
        err, zeros_ok = image_rel_err(img, refimg)
        assert zeros_ok and err <= TOL, (name, err)


def test_splat_bit_reproducible():
    """Pair lists are built by a stable counting sort, so repeated renders
    (with different workspace contents) give identical bits."""
    import torch
    s = synth.small_clustered(600000, 72)
    d = to_dev(s)
    for cam in (lib.Camera.ortho(512, 384), lib.Camera.look_at((0.5, 0.45, -0.6), (0.5, 0.5, 0.5), 300, 200)):
        ws = lib.splat_workspace_bytes(s.n, cam)
        w1 = torch.zeros(ws, dtype=torch.uint8, device="cuda")
        w2 = torch.full((ws,), 0xA5, dtype=torch.uint8, device="cuda")
        a = lib.splat(*d, cam, workspace=w1).cpu().numpy()
        b = lib.splat(*d, cam, workspace=w2).cpu().numpy()
        c = lib.splat(*d, cam, workspace=w1).cpu().numpy()
        assert np.array_equal(a.view(np.int32), b.view(np.int32))
        assert np.array_equal(a.view(np.int32), c.view(np.int32))


@pytest.mark.parametrize("n", [16, 64, 700])
def test_lod_render_equals_render_of_decoded_points(n):
    """The LOD render decodes the stored points inside the binning; it must
    equal, bit for bit, the plain render of the decoded points (same point
    sequence, same units), also with invalid ids in the list and when
    max_points truncates the sequence."""
    import torch
    s = synth.small_clustered(120000, 73)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=n, max_depth=6, seed=1))
    h = tree.host()
    cam = lib.Camera.look_at((0.52, 0.47, -0.5), (0.5, 0.5, 0.5), 256, 192, fov_deg=55.0)
    ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
    k = int(lib._to_numpy(nsel)[0])
    chosen = lib._to_numpy(ids[:k]).astype(np.int64)
    # interleave invalid ids (beyond the node count)
    mixed = []
    for i, v in enumerate(chosen):
        mixed.append(v)
        if i % 5 == 0:
            mixed.append(h["n_nodes"] + 3 + i)
    mixed = np.array(mixed, dtype=np.int64)
    total = int(h["pt_count"][chosen].astype(np.int64).sum())
    for lst in (chosen, mixed):
        idt = torch.from_numpy(lst.astype(np.int32)).cuda().view(torch.uint32)
        nid = torch.tensor([len(lst)], dtype=torch.int64).cuda().view(torch.uint64)
        for cap in (total, total // 3 + 1):
            img = lib.splat_lod(tree, idt, nid, cap, cam).cpu().numpy()
            x, y, z, m, cnt = lib.decode_nodes(tree, idt, nid, cap)
            c = int(lib._to_numpy(cnt)[0])
            assert c == min(cap, total)
            ref = lib.splat(x[:c], y[:c], z[:c], m[:c], cam).cpu().numpy()
            assert np.array_equal(img.view(np.int32), ref.view(np.int32)), (n, len(lst), cap)


def test_splat_maximum_tile_count():
    """8,192 tiles of 16x16 (2040x1018, the limit; 13-bit tile
    ids in the wave matching) and a ragged last tile column and row; one more
    tile column is refused as unsupported."""
    s = synth.small_clustered(40000, 74)
    W, H = 2040, 1018
    for cam, ocam in ((lib.Camera.ortho(W, H), osplat.Camera(0, W, H)),):
        img = lib.splat(*to_dev(s), cam).cpu().numpy()
        ref = osplat.render(ocam, s.x, s.y, s.z, s.m)
        err, zeros_ok = image_rel_err(img, ref)
        assert zeros_ok and err <= TOL, err
    with pytest.raises(RuntimeError):
        lib.splat(*to_dev(s), lib.Camera.ortho(2064, 1024))

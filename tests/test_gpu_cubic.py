"""The radial cubic blob (fixed pixel radius and projected world radius),
the attribute channel and ID highlighting on the GPU, through the C ABI,
against the float64 oracle (oracle/cubic.py, oracle/splat.py, oracle/lod.py).

Images: exact zeros where the oracle is zero, every positive pixel within
1e-5 relative.  Gradients: every element within 1e-5 of its own error scale
(the sum of the absolute terms that make it up)."""
import math

import numpy as np
import pytest

import synth
from oracle import cubic as ocubic
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
                           ("near", (0.45, 0.5, 0.05), (0.5, 0.5, 0.5))):
        c = lib.Camera.look_at(pos, tgt, W, H, fov_deg=60.0)
        out.append((name, c, osplat.Camera(1, W, H, c.pos, c.right, c.up, c.fwd, c.F, c.near)))
    return out


# radii below 1.9 and 3.9 pixels take the windowed accumulation (4 and 8
# pixel windows), larger ones the gather form: both sides of each threshold
@pytest.mark.parametrize("h", [1.0, 1.5, 1.89, 1.95, 2.5, 3.89, 3.95, 6.0, 16.0])
def test_cubic_fixed_radius_matches_oracle(h):
    s = synth.small_clustered(30000, 401)
    d = to_dev(s)
    for name, cam, ocam in _cams(180, 136):
        print(f"[cubic parity] {name} h={h}", flush=True)
        img = lib.splat(*d, cam, blob=lib.Blob.cubic(h_px=h)).cpu().numpy()
        ref = ocubic.render(ocam, s.x, s.y, s.z, s.m, h_px=h)
        err, zeros_ok = image_rel_err(img, ref)
        assert zeros_ok, name
        assert err <= TOL, (name, err)


@pytest.mark.parametrize("hw", [0.002, 0.02])
def test_cubic_world_radius_matches_oracle(hw):
    """Projected world radii, including points clamped to 1 px (far) and to 16 px (near)."""
    s = synth.small_clustered(30000, 402)
    d = to_dev(s)
    for name, cam, ocam in _cams(200, 150)[1:]:
        img = lib.splat(*d, cam, blob=lib.Blob.cubic(h_world=hw)).cpu().numpy()
        ref = ocubic.render(ocam, s.x, s.y, s.z, s.m, h_world=hw)
        err, zeros_ok = image_rel_err(img, ref)
        print(f"[cubic world] {name} h_world={hw} max rel err {err:.2e}", flush=True)
        assert zeros_ok, name
        assert err <= TOL, (name, err)


def test_cubic_rejects_world_radius_in_orthographic_view():
    s = synth.small_clustered(100, 403)
    with pytest.raises(lib.LodError):
        lib.splat(*to_dev(s), lib.Camera.ortho(32, 32), blob=lib.Blob.cubic(h_world=0.01))
    with pytest.raises(lib.LodError):
        lib.splat(*to_dev(s), lib.Camera.ortho(32, 32), blob=lib.Blob.cubic(h_px=17.0))


@pytest.mark.parametrize("blob", ["gauss", "cubic", "cubic-1.5", "cubic-5"])
def test_attribute_channel_matches_oracle(blob):
    """The second channel sum m a W for a random colour attribute in [0, 1)
    (cubic radii 2, 1.5 and 5 pixels: both windowed forms and the gather)."""
    import torch
    s = synth.small_clustered(40000, 404)
    a = np.random.default_rng(3).random(s.n).astype(np.float32)
    d = to_dev(s)
    for name, cam, ocam in _cams(160, 120)[:2]:
        hpx = {"cubic": 2.0, "cubic-1.5": 1.5, "cubic-5": 5.0}.get(blob)
        b = lib.Blob.cubic(h_px=hpx) if hpx else None
        img, aimg = lib.splat_aux(*d, torch.from_numpy(a).cuda(), cam, blob=b)
        plain = lib.splat(*d, cam, blob=b)
        if hpx:
            ref, aref = ocubic.render(ocam, s.x, s.y, s.z, s.m, h_px=hpx, aux=a)
        else:
            ref = osplat.render(ocam, s.x, s.y, s.z, s.m)
            aref = osplat.render(ocam, s.x, s.y, s.z, (s.m.astype(np.float64) * a).astype(np.float32))
        for got, want in ((img, ref), (aimg, aref)):
            err, zeros_ok = image_rel_err(got.cpu().numpy(), want)
            assert zeros_ok and err <= TOL, (blob, name, err)
        # the first channel is the plain render, bit for bit
        assert torch.equal(img.view(torch.int32), plain.view(torch.int32)), (blob, name)


@pytest.mark.parametrize("hw", [0.0, 0.01])
def test_cubic_backward_matches_oracle(hw):
    import torch
    s = synth.small_clustered(3000, 405)
    for name, cam, ocam in _cams(96, 80)[(1 if hw else 0):3]:
        g = np.random.default_rng(5).standard_normal((80, 96)).astype(np.float32)
        b = lib.Blob.cubic(h_px=2.2, h_world=hw)
        gm, gx, gy, gz = lib.splat_backward(*to_dev(s), torch.from_numpy(g).cuda(), cam, blob=b)
        rm, rp = ocubic.render_backward(ocam, s.x, s.y, s.z, s.m, g.astype(np.float64), h_px=2.2, h_world=hw)
        bm, bp = ocubic.render_backward(ocam, s.x, s.y, s.z, s.m, None, h_px=2.2, h_world=hw,
                                        bound_weights=np.abs(g.astype(np.float64)))
        checked = 0
        for nm, got, want, bound in (("m", gm, rm, bm), ("x", gx, rp[:, 0], bp[:, 0]),
                                     ("y", gy, rp[:, 1], bp[:, 1]), ("z", gz, rp[:, 2], bp[:, 2])):
            got = got.cpu().numpy().astype(np.float64)
            bad = np.nonzero(np.abs(got - want) > 1e-5 * bound + 1e-30)[0]
            assert bad.size == 0, (name, nm, bad[:5], got[bad[:5]], want[bad[:5]], bound[bad[:5]])
            checked += int(np.count_nonzero(bound > 0))
        assert checked >= 1000, (name, checked)


def test_cubic_autograd_fp64_finite_differences_no_skipping():
    """Float64 central differences of an independent evaluation on every
    sampled point: the cubic blob has no edge, so none is skipped."""
    import torch
    from paper_0811_2055_amd.autograd import splat_render
    rng = np.random.default_rng(17)
    Np, W, H = 200, 64, 64
    x = (0.25 + 0.5 * rng.random(Np)).astype(np.float32)
    y = (0.25 + 0.5 * rng.random(Np)).astype(np.float32)
    z = (0.25 + 0.5 * rng.random(Np)).astype(np.float32)
    m = rng.uniform(0.5, 1.5, Np).astype(np.float32)
    cam = lib.Camera.look_at((0.5, 0.52, -0.7), (0.5, 0.5, 0.5), W, H, fov_deg=60.0)
    hw = 0.004
    b = lib.Blob.cubic(h_world=hw)
    g = rng.standard_normal((H, W))
    xs = [torch.from_numpy(a).cuda().requires_grad_(True) for a in (x, y, z, m)]
    img = splat_render(*xs, cam, blob=b)
    (img * torch.from_numpy(g.astype(np.float32)).cuda()).sum().backward()
    grads = [t.grad.cpu().numpy().astype(np.float64) for t in xs]
    pos = np.array(cam.pos, dtype=np.float64); r = np.array(cam.right); up = np.array(cam.up)
    fw = np.array(cam.fwd)
    Fhw = float(np.float32(cam.F) * np.float32(hw))

    def terms(p, mk):
        d = p - pos
        zc = d @ fw
        u = cam.F * (d @ r) / zc + W / 2
        v = cam.F * (d @ up) / zc + H / 2
        h = min(max(Fhw / zc, 1.0), 16.0)
        out = {}
        for j in range(max(0, int(v - h) - 1), min(H, int(v + h) + 2)):
            for i in range(max(0, int(u - h) - 1), min(W, int(u + h) + 2)):
                q = math.hypot(u - (i + 0.5), v - (j + 0.5)) / h
                if q < 1:
                    w = 1 - 6 * q * q + 6 * q ** 3 if q <= 0.5 else 2 * (1 - q) ** 3
                    out[(i, j)] = mk * 40 / (7 * math.pi * h * h) * w * g[j, i]
        return out

    checked = 0
    for k in rng.choice(Np, 40, replace=False):
        p0 = np.array([x[k], y[k], z[k]], dtype=np.float64)
        hstep = 1e-6
        for ax in range(3):
            e = np.zeros(3); e[ax] = hstep
            a, bb = terms(p0 + e, float(m[k])), terms(p0 - e, float(m[k]))
            dd = [(a.get(q, 0.0) - bb.get(q, 0.0)) / (2 * hstep) for q in set(a) | set(bb)]
            fd, scale = sum(dd), sum(abs(t) for t in dd)
            assert abs(fd - grads[ax][k]) <= 1e-4 * scale + 1e-6 * abs(fd), (k, ax, fd, grads[ax][k], scale)
        checked += 1
    assert checked == 40


def _tree(s, n, D, seed=0):
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=n, D=D, seed=seed)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=n, max_depth=D, seed=seed))
    return ref, tree


@pytest.mark.parametrize("blob", ["gauss", "cubic"])
def test_lod_highlight_matches_oracle(blob):
    """ID highlighting in the LOD render: the per-point flags are the
    membership of each stored point's id (ids past n_bits never are); the
    first image equals the plain LOD render bit for bit; the highlight image
    equals the oracle's render of the cut's decoded points whose id is in the
    set, twice in a row bit for bit; a cap below the selected count sets the
    capacity status bit."""
    import torch
    s = synth.small_clustered(60000, 406)
    n = 300
    ref, tree = _tree(s, n, 6)
    rng = np.random.default_rng(8)
    chosen = rng.choice(s.n, 6000, replace=False)
    n_bits = s.n - 5000                   # ids above n_bits are not highlighted even if listed
    bits = lib.highlight_bits(chosen, n_bits)
    member = np.zeros(s.n, dtype=bool)
    member[chosen[chosen < n_bits]] = True
    flags = lib.highlight_flags(tree, bits, n_bits)
    # the flags: bit s set iff stored point s has a selected id
    fl = lib._to_numpy(flags).astype(np.uint64)
    S = ref.n_points
    got_bits = ((fl[np.arange(S) >> 5] >> (np.arange(S) & 31).astype(np.uint64)) & np.uint64(1)).astype(bool)
    assert np.array_equal(got_bits, member[ref.pt_id.astype(np.int64)])
    # a reused output buffer holding garbage: every word is rewritten
    again = torch.full_like(flags.view(torch.int32), -1).view(torch.uint32)
    lib.highlight_flags(tree, bits, n_bits, out=again)
    assert torch.equal(again.view(torch.int32), flags.view(torch.int32))
    b = lib.Blob.cubic(h_px=1.7) if blob == "cubic" else None
    for name, cam, ocam in _cams(160, 160)[:3]:
        ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
        want_ids = ocut.select(ref, ocam, 1.0, n)
        img, hl = lib.splat_lod_highlight(tree, ids, nsel, tree.point_capacity, cam, flags, len(chosen), blob=b)
        plain = lib.splat_lod(tree, ids, nsel, tree.point_capacity, cam, blob=b)
        assert torch.equal(img.view(torch.int32), plain.view(torch.int32)), (blob, name)
        px, py, pz, pm = olod.decoded_points(ref, want_ids)
        pid = np.concatenate([ref.pt_id[int(ref.pt_begin[v]):int(ref.pt_begin[v]) + int(ref.pt_count[v])]
                              for v in want_ids]).astype(np.int64)
        on = member[pid]
        if blob == "cubic":
            want = ocubic.render(ocam, px[on], py[on], pz[on], pm[on], h_px=1.7)
        else:
            want = osplat.render(ocam, px[on], py[on], pz[on], pm[on])
        err, zeros_ok = image_rel_err(hl.cpu().numpy(), want)
        print(f"[highlight] {blob} {name}: {int(on.sum())} of {len(on)} drawn points highlighted, err {err:.2e}",
              flush=True)
        assert zeros_ok and err <= TOL, (blob, name, err)
        assert on.any()
        _, hl2 = lib.splat_lod_highlight(tree, ids, nsel, tree.point_capacity, cam, flags, len(chosen), blob=b)
        assert torch.equal(hl.view(torch.int32), hl2.view(torch.int32))
    # a cap below the number of highlighted drawn points: flagged, not overrun
    k = int(on.sum())
    assert k > 2
    lib.splat_lod_highlight(tree, ids, nsel, tree.point_capacity, cam, flags, k // 2, blob=b)
    st = int(lib._to_numpy(tree.counts)[2])
    assert st & lib.STATUS_CAPACITY
    tree.counts[2] = 0

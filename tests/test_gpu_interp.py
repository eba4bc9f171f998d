"""Time interpolation on the GPU against the oracle (oracle/interp.py):
frames between two ID-matched snapshots (position, mass, world radius and
colour), motion codes of stored points (bit-exact, with the saturation
count, single snapshot and batch), and the LOD render at a frame time."""
import numpy as np
import pytest

import synth
from oracle import cut as ocut
from oracle import interp as ointerp
from oracle import lod as olod
from oracle import splat as osplat
from paper_0811_2055_amd import lib

from gpu_util import image_rel_err, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _pair(n, seed, step=0.01):
    A = synth.small_clustered(n, seed)
    B, aa, ab = synth.evolve(A, seed + 1, step=step)
    return A, B, aa, ab


def _cams(W, H):
    c = lib.Camera.look_at((0.5, 0.45, -0.8), (0.5, 0.5, 0.5), W, H, fov_deg=60.0)
    return [("ortho", lib.Camera.ortho(W, H), osplat.Camera(0, W, H)),
            ("persp", c, osplat.Camera(1, W, H, c.pos, c.right, c.up, c.fwd, c.F, c.near))]


@pytest.mark.parametrize("t", [0.0, 0.3, 1.0])
def test_interpolated_frames_match_oracle(t):
    import torch
    A, B, aa, ab = _pair(30000, 501)
    dA, dB = to_dev(A), to_dev(B)
    hA, hB, cA, cB = (torch.from_numpy(a).cuda() for a in (aa.h, ab.h, aa.c, ab.c))
    for name, cam, ocam in _cams(160, 120):
        img = lib.splat_interp(dA, dB, t, cam).cpu().numpy()
        ref = ointerp.render(ocam, (A.x, A.y, A.z, A.m), (B.x, B.y, B.z, B.m), t)
        err, zeros_ok = image_rel_err(img, ref)
        assert zeros_ok and err <= TOL, ("gauss", name, t, err)
        if t == 0.0:
            plain = lib.splat(*dA, cam).cpu().numpy()
            assert np.array_equal(img.view(np.int32), plain.view(np.int32))
        if name == "persp":
            b = lib.Blob.cubic(h_world=0.004)
            img, cimg = lib.splat_interp(dA, dB, t, cam, blob=b, hA=hA, hB=hB, cA=cA, cB=cB)
            ref, cref = ointerp.render(ocam, (A.x, A.y, A.z, A.m), (B.x, B.y, B.z, B.m), t, blob="cubic",
                                       hA=aa.h, hB=ab.h, cA=aa.c, cB=ab.c)
        else:
            b = lib.Blob.cubic(h_px=2.0)
            img, cimg = lib.splat_interp(dA, dB, t, cam, blob=b, cA=cA, cB=cB)
            ref, cref = ointerp.render(ocam, (A.x, A.y, A.z, A.m), (B.x, B.y, B.z, B.m), t, blob="cubic",
                                       h_px=2.0, cA=aa.c, cB=ab.c)
        for got, want in ((img, ref), (cimg, cref)):
            err, zeros_ok = image_rel_err(got.cpu().numpy(), want)
            print(f"[interp] cubic {name} t={t} err {err:.2e}", flush=True)
            assert zeros_ok and err <= TOL, ("cubic", name, t, err)


def test_interp_rejects_bad_arguments():
    A, B, aa, ab = _pair(100, 502)
    dA, dB = to_dev(A), to_dev(B)
    cam = lib.Camera.ortho(32, 32)
    with pytest.raises(lib.LodError):
        lib.splat_interp(dA, dB, 1.5, cam)
    import torch
    h = torch.from_numpy(aa.h).cuda()
    with pytest.raises(lib.LodError):          # world radii need the cubic blob and a perspective camera
        lib.splat_interp(dA, dB, 0.5, cam, hA=h, hB=h)


@pytest.mark.parametrize("step", [0.02, 0.4])
def test_motion_codes_match_oracle(step):
    A, B, aa, ab = _pair(40000, 503, step=step)
    n, D = 200, 5
    ref = olod.lod_build(A.x, A.y, A.z, A.m, n=n, D=D, seed=4)
    tree = lib.build(*to_dev(A), lib.BuildParams(n=n, max_depth=D, seed=4))
    dB = to_dev(B)
    dqx, dqy, dqz, sat = lib.encode_motion(tree, dB[0], dB[1], dB[2])
    rx, ry, rz, rsat = ointerp.encode_motion(ref, B.x, B.y, B.z)
    S = ref.n_points
    for got, want in ((dqx, rx), (dqy, ry), (dqz, rz)):
        assert np.array_equal(got[:S].cpu().numpy(), want)
    assert int(lib._to_numpy(sat)[0]) == rsat
    assert (rsat > 0) == (step > 0.1)


def test_motion_codes_batch_matches_oracle():
    import torch
    snaps = [_pair(k, 510 + i, step=0.03) for i, k in enumerate((3000, 0, 5000))]
    n, D = 60, 4
    off = np.array([0, 3000, 3000, 8000], dtype=np.int64)
    cat = lambda idx, key: np.concatenate([getattr(p[idx], key) for p in snaps])   # noqa: E731
    XA = [cat(0, k) for k in "xyzm"]
    XB = [cat(1, k) for k in "xyz"]
    ref = olod.lod_build(*XA, n=n, D=D, seed=2, snap_offsets=off)
    offs = torch.from_numpy(off).cuda().view(torch.uint64)
    tree = lib.build(*[torch.from_numpy(a).cuda() for a in XA], lib.BuildParams(n=n, max_depth=D, seed=2),
                     snap_offsets=offs)
    dq = lib.encode_motion(tree, *[torch.from_numpy(a).cuda() for a in XB], snap_offsets=offs)
    want = ointerp.encode_motion(ref, *XB, snap_offsets=off)
    S = ref.n_points
    for got, w in zip(dq[:3], want[:3]):
        assert np.array_equal(got[:S].cpu().numpy(), w)
    assert int(lib._to_numpy(dq[3])[0]) == want[3]


@pytest.mark.parametrize("t", [0.0, 0.6])
def test_lod_motion_render_matches_oracle(t):
    """The LOD render at frame time t equals the oracle's render of the cut's
    points interpolated between their decoded positions and their decoded
    motion targets; at t = 0 it is the plain LOD render, bit for bit."""
    import torch
    A, B, aa, ab = _pair(60000, 504, step=0.02)
    n = 300
    ref = olod.lod_build(A.x, A.y, A.z, A.m, n=n, D=6, seed=0)
    tree = lib.build(*to_dev(A), lib.BuildParams(n=n, max_depth=6, seed=0))
    dB = to_dev(B)
    motion = lib.encode_motion(tree, dB[0], dB[1], dB[2])
    rx, ry, rz, _ = ointerp.encode_motion(ref, B.x, B.y, B.z)
    for name, cam, ocam in _cams(160, 160):
        ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
        want_ids = ocut.select(ref, ocam, 1.0, n)
        for blob, ob in ((None, "gauss"), (lib.Blob.cubic(h_px=1.8), "cubic")):
            img = lib.splat_lod_motion(tree, ids, nsel, tree.point_capacity, motion, t, cam, blob=blob)
            Aq, Bq = ointerp.decoded_motion_points(ref, want_ids, rx, ry, rz)
            want = ointerp.render(ocam, Aq, Bq, t, blob=ob, h_px=1.8)
            err, zeros_ok = image_rel_err(img.cpu().numpy(), want)
            print(f"[lod motion] {name} {ob} t={t}: err {err:.2e}", flush=True)
            assert zeros_ok and err <= TOL, (name, ob, t, err)
            if t == 0.0:
                plain = lib.splat_lod(tree, ids, nsel, tree.point_capacity, cam, blob=blob)
                assert torch.equal(img.view(torch.int32), plain.view(torch.int32))

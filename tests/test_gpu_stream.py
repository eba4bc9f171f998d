"""Block store and view-dependent streaming through the C ABI against the
oracle's policy (oracle/stream.py): per frame of a camera path, the loaded
and evicted nodes and the draw list are exactly the oracle's (its own tree,
built from the same particles), and the streamed render equals the oracle's
render of the decoded points of its draw list within 1e-5."""
import os

import numpy as np
import pytest

import synth
from oracle import lod as olod
from oracle import splat as osplat
from oracle import stream as ostream
from paper_0811_2055_amd import lib

from gpu_util import image_rel_err, to_dev

pytestmark = pytest.mark.gpu


def test_store_round_trip_and_streamed_frames(tmp_path):
    s = synth.small_clustered(50000, 701)
    n, D = 200, 6
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=n, D=D, seed=3)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=n, max_depth=D, seed=3))
    path = os.path.join(str(tmp_path), "c.lodstore")
    lib.store_save(tree, n, path)
    nn, npts, nstore = lib.store_info(path)
    assert (nn, npts, nstore) == (ref.n_nodes, ref.n_points, n)
    assert os.path.getsize(path) >= 14 * npts
    slots, budget = 60, 14 * n * 5
    st = lib.Streamer(path, slots)
    ost = ostream.Streamer(ref, slots)
    W = H = 128
    total_loaded = total_evicted = 0
    for f, a in enumerate(np.linspace(0.0, 1.0, 24)):
        p = 0.1 + 0.8 * a
        cam = lib.Camera.look_at((p, p, p), (0.5, 0.5, 0.55) if a < 0.5 else (0.9, 0.2, 0.4), W, H, fov_deg=60.0,
                                 near=1e-4)
        ocam = osplat.Camera(1, W, H, cam.pos, cam.right, cam.up, cam.fwd, cam.F, cam.near)
        ids, nd, stats, loaded, evicted = st.frame(cam, 4.0, budget, want_ids=True)
        odraw, oloaded, oevicted, obytes = ost.frame_step(ocam, 4.0, n, budget)
        k = int(lib._to_numpy(nd)[0])
        got = lib._to_numpy(ids[:k]).astype(np.int64)
        assert loaded == oloaded, (f, loaded[:8], oloaded[:8])
        assert evicted == oevicted, (f, evicted[:8], oevicted[:8])
        assert np.array_equal(got, np.array(odraw, dtype=np.int64)), f
        assert stats["bytes_loaded"] == obytes
        total_loaded += len(loaded)
        total_evicted += len(evicted)
        if f % 6 == 5:
            img = lib.splat_lod(st.view, ids, nd, slots * n, cam).cpu().numpy()
            px, py, pz, pm = olod.decoded_points(ref, odraw)
            want = osplat.render(ocam, px, py, pz, pm)
            err, zeros_ok = image_rel_err(img, want)
            print(f"[stream] frame {f}: drawn {k} nodes, loaded {len(loaded)}, evicted {len(evicted)}, "
                  f"bytes {stats['bytes_loaded']}, image err {err:.2e}", flush=True)
            assert zeros_ok and err <= 1e-5
    assert total_loaded > slots and total_evicted > 0
    st.close()


def test_streamer_rejects_a_pool_without_room_for_the_roots(tmp_path):
    s = synth.small_clustered(5000, 702)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=50, max_depth=4, seed=1))
    path = os.path.join(str(tmp_path), "d.lodstore")
    lib.store_save(tree, 50, path)
    with pytest.raises(lib.LodError):
        lib.Streamer(path, 0)


def test_tree_file_round_trip_on_device(tmp_path):
    """A GPU-built tree saved to a file and loaded into new device arrays
    holds the same bytes, and its cut and LOD render equal the original's bit
    for bit."""
    import torch
    s = synth.small_clustered(60000, 31)
    n = 300
    tree = lib.build(*to_dev(s), lib.BuildParams(n=n, max_depth=6, seed=4))
    path = str(tmp_path / "tree.npz")
    lib.save_tree(tree, path, n=n)
    t2, n2 = lib.load_tree(path)
    assert n2 == n
    h, h2 = tree.host(), t2.host()
    for k in ("n_nodes", "n_points", "status"):
        assert h[k] == h2[k], k
    for k in ("prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count", "pt_begin",
              "pt_count", "node_mass", "pt_id", "qx", "qy", "qz", "pt_mass"):
        assert np.array_equal(h[k], h2[k]), k
    cam = lib.Camera.look_at((0.5, 0.5, -0.8), (0.5, 0.5, 0.5), 128, 128, 60.0)
    ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
    ids2, nsel2 = lib.select_nodes(t2, cam, 1.0, n)
    k = int(lib._to_numpy(nsel)[0])
    assert k == int(lib._to_numpy(nsel2)[0]) and torch.equal(ids[:k], ids2[:k])
    img = lib.splat_lod(tree, ids, nsel, tree.point_capacity, cam)
    img2 = lib.splat_lod(t2, ids2, nsel2, t2.point_capacity, cam)
    assert torch.equal(img.view(torch.int32), img2.view(torch.int32))

"""Full-size checks of the two other workloads: 16.7 M NFW particles (n =
16000, D = 8, perspective 1024^2 render) and a batch of 128 Soneira-Peebles
snapshots of 0.5-8 M particles built in one graph-captured batched build
with a 512^2 render per snapshot.  Outputs are checked where the oracle can
compute them one by one: tree and sort properties, sampled nodes' stored
points from the definition, sampled pixels of the renders.
"""
import json
import time

import numpy as np
import pytest

import synth
from oracle import lod as olod
from oracle import splat as osplat
from paper_0811_2055_amd import lib

from gpu_util import check_node_against_definition, check_sort_and_tree, sample_nodes

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

TOL = 1e-5


def log(msg):
    print(f"[configs {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def pixels_match(img, ocam, x, y, z, m, rng, k=12):
    flat = np.argsort(-img.ravel())
    nz = np.nonzero(img.ravel() > 0)[0]
    pix = np.concatenate([flat[:4], rng.choice(nz, min(k - 4, len(nz)), replace=False)])
    W = img.shape[1]
    pi, pj = pix % W, pix // W
    want = osplat.render_pixels(ocam, x, y, z, m, pi, pj)
    got = img[pj, pi].astype(np.float64)
    err = np.abs(got - want) / np.maximum(want, 1e-300)
    assert np.all((want > 0) | (got == 0))
    return float(err[want > 0].max())


def test_nfw_16m_perspective():
    import torch
    log("generating 16.7M NFW particles")
    s = synth.config2()
    N, n, D = s.n, 16000, 8
    d = [torch.from_numpy(a).cuda() for a in (s.x, s.y, s.z, s.m)]
    b = lib.Builder(N, lib.BuildParams(n=n, max_depth=D, seed=0))
    tree = b.build(*d)
    h = tree.host()
    assert h["status"] == 0
    log(f"built: {h['n_nodes']} nodes {h['n_points']} points")
    keys_D = olod.interleave(*(olod.cell_coords(a, D) for a in (s.x, s.y, s.z)), D)
    check_sort_and_tree(b.view(0, torch.uint32).view(torch.int32), b.view(1, torch.uint32).view(torch.int32),
                        h, N, n, D, keys_D)
    dens = olod.density_counts(s.x, s.y, s.z, D)
    rng = np.random.default_rng(11)
    for v in sample_nodes(h, n, rng):
        check_node_against_definition(h, v, s.x, s.y, s.z, s.m, n, D, dens, keys_D)
    log("nodes ok")
    cam = lib.Camera.look_at((0.5, 0.5, -0.6), (0.5, 0.5, 0.5), 1024, 1024, fov_deg=60.0)
    ocam = osplat.Camera(1, 1024, 1024, cam.pos, cam.right, cam.up, cam.fwd, cam.F, cam.near)
    img = lib.splat(*d, cam).cpu().numpy()
    err = pixels_match(img, ocam, s.x, s.y, s.z, s.m, rng)
    log(f"perspective render: max relative error over sampled pixels {err:.2e}")
    assert err <= TOL


def _hash_tree(h):
    import hashlib
    hs = hashlib.sha1()
    for k in ("prefix", "depth", "part_count", "pt_begin", "pt_id", "qx", "qy", "qz", "pt_mass", "node_mass"):
        hs.update(np.ascontiguousarray(h[k]).tobytes())
    hs.update(np.array([h["n_nodes"], h["n_points"], h["status"]], dtype=np.int64).tobytes())
    return hs.hexdigest()


def test_batch_128_snapshots_graph_captured():
    import torch
    n, D = 16000, 8
    sizes = synth.config5_sizes()
    log(f"generating 128 Soneira-Peebles snapshots, {int(sizes.sum())} particles")
    snaps = [synth.config5_snapshot(i, int(sz)) for i, sz in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    N = int(off[-1])
    cat = [np.concatenate([getattr(p, k) for p in snaps]) for k in "xyzm"]
    d = [torch.from_numpy(a).cuda() for a in cat]
    offs = torch.from_numpy(off).cuda().view(torch.uint64)
    b = lib.Builder(N, lib.BuildParams(n=n, max_depth=D, seed=0), n_snapshots=len(sizes))
    tree = b.build(*d, snap_offsets=offs)
    h = tree.host()
    assert h["status"] == 0
    ref = _hash_tree(h)
    log(f"eager build: {h['n_nodes']} nodes {h['n_points']} points")
    # the same build captured in a HIP graph, replayed with eager work in between
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.build(*d, snap_offsets=offs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        b.build(*d, snap_offsets=offs)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        junk = torch.ones(1 << 20, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        assert _hash_tree(tree.host()) == ref, rep
        del junk
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    log(json.dumps({"batch": "128 snapshots", "particles": N, "graph_replay_ms": round(ms, 3),
                    "Mparticles_s": round(N / ms / 1e3, 1)}))
    # per snapshot: keys with the snapshot index above the Morton bits
    keys_D = np.concatenate([(olod.interleave(*(olod.cell_coords(a, D) for a in (p.x, p.y, p.z)), D)
                              | (np.uint64(i) << np.uint64(3 * D))) for i, p in enumerate(snaps)])
    check_sort_and_tree(b.view(0, torch.uint32).view(torch.int32), b.view(1, torch.uint32).view(torch.int32),
                        h, N, n, D, keys_D)
    log("sort and tree ok")
    depth = h["depth"].astype(np.int64)
    snap_of = (h["prefix"].astype(np.uint64) >> (np.uint64(3) * depth.astype(np.uint64))).astype(np.int64)
    rng = np.random.default_rng(12)
    order = np.argsort(sizes)
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        p = snaps[i]
        kd = olod.interleave(*(olod.cell_coords(a, D) for a in (p.x, p.y, p.z)), D)
        dens = olod.density_counts(p.x, p.y, p.z, D)
        mine = np.nonzero(snap_of == i)[0]
        picks = [int(mine[0])] + [int(v) for v in rng.choice(mine, min(4, len(mine)), replace=False)]
        for v in picks:
            check_node_against_definition(h, v, p.x, p.y, p.z, p.m, n, D, dens, kd, snap=i)
    log("sampled nodes ok")
    cam = lib.Camera.ortho(512, 512)
    ocam = osplat.Camera(0, 512, 512)
    ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
    cut = lib._to_numpy(ids[:int(lib._to_numpy(nsel)[0])]).astype(np.int64)
    errs, elog = [], []
    for i in np.linspace(0, len(sizes) - 1, 8).astype(int):
        a0, a1 = int(off[i]), int(off[i + 1])
        full = lib.splat(*(t[a0:a1] for t in d), cam)
        p = snaps[i]
        errs.append(pixels_match(full.cpu().numpy(), ocam, p.x, p.y, p.z, p.m, rng, k=8))
        mine = cut[snap_of[cut] == i]
        idt = torch.from_numpy(mine.astype(np.int32)).cuda().view(torch.uint32)
        nid = torch.tensor([len(mine)], dtype=torch.int64).cuda().view(torch.uint64)
        lod = lib.splat_lod(tree, idt, nid, a1 - a0, cam)
        mu = full.mean()
        elog.append(float(torch.sqrt(torch.mean((torch.log1p(lod / mu) - torch.log1p(full / mu)) ** 2))))
    log(json.dumps({"per_snapshot_max_rel_err": [f"{e:.2e}" for e in errs],
                    "per_snapshot_E_log_lod_vs_full": [round(e, 4) for e in elog]}))
    assert max(errs) <= TOL

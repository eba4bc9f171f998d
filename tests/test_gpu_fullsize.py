"""Full-size checks at the benchmark configuration (150 M Soneira-Peebles
particles, n = 16000, D = 8, the autotuned schedule), on outputs the oracle
computes one by one: sampled nodes' stored points straight from the
definition over the raw particles, properties of the sort and the tree that
hold at any size, and sampled pixels of the full render.
"""
import math
import time

import numpy as np
import pytest

import synth
from oracle import lod as olod
from oracle import splat as osplat
from paper_0811_2055_amd import autotune, lib

from gpu_util import kbin_of

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def log(msg):
    print(f"[fullsize {time.strftime('%H:%M:%S')}] {msg}", flush=True)


@pytest.fixture(scope="module")
def c3():
    import torch
    log("generating 150M Soneira-Peebles particles")
    s = synth.config3()
    d = [torch.from_numpy(a).cuda() for a in (s.x, s.y, s.z, s.m)]
    b = lib.Builder(s.n, lib.BuildParams(n=16000, max_depth=8, seed=0))
    rec = autotune.tune(b, *d, path="/tmp/lod_tune_test.json")
    log(f"schedule {b.params}")
    tree = b.build(*d)
    h = tree.host()
    log(f"built: {h['n_nodes']} nodes {h['n_points']} points status {h['status']}")
    keys_D = olod.interleave(*(olod.cell_coords(a, 8) for a in (s.x, s.y, s.z)), 8)
    log("oracle depth-8 keys")
    b.tune_record = rec
    return s, d, b, tree, h, keys_D


def test_sort_and_tree_properties(c3):
    import torch
    s, d, b, tree, h, keys_D = c3
    assert h["status"] == 0
    keys = b.view(0, torch.uint32).view(torch.int32).long() & 0xFFFFFFFF
    ids = b.view(1, torch.uint32).view(torch.int32).long()
    N = s.n
    # the sort: keys non-decreasing, ids ascending within equal keys, a permutation
    assert bool((keys[1:] >= keys[:-1]).all())
    eq = keys[1:] == keys[:-1]
    assert bool((ids[1:][eq] > ids[:-1][eq]).all())
    assert int(torch.bincount(ids, minlength=N).max()) == 1
    # keys of sampled particles from their raw coordinates (oracle key function)
    rng = np.random.default_rng(0)
    pos = rng.integers(0, N, 20000)
    gi = ids[torch.from_numpy(pos).cuda()].cpu().numpy()
    assert np.array_equal(keys[torch.from_numpy(pos).cuda()].cpu().numpy().astype(np.uint64), keys_D[gi])
    # density: the run length of equal keys at sampled positions
    w = b.view(2, torch.uint32).view(torch.int32).long()
    kn = keys.cpu().numpy()
    lo = np.searchsorted(kn, kn[pos], "left"); hi = np.searchsorted(kn, kn[pos], "right")
    assert np.array_equal(w[torch.from_numpy(pos).cuda()].cpu().numpy(), hi - lo)
    # key bins at the sampled positions: the bins of the oracle's keys K(U(id), w)
    kb = b.view(3, torch.uint16).view(torch.int16).long() & 0xFFFF
    U = olod.particle_uniform(gi.astype(np.uint64), 0, 0)
    K = olod.selection_keys(U, (hi - lo).astype(np.uint64), 1)
    assert np.array_equal(kb[torch.from_numpy(pos).cuda()].cpu().numpy(), kbin_of(K))
    # tree invariants
    n, D = 16000, 8
    internal = h["first_child"] != lib.NONE
    assert np.array_equal(internal, (h["part_count"] > n) & (h["depth"] < D))
    leaf = ~internal
    lb = h["part_begin"][leaf].astype(np.int64); lc = h["part_count"][leaf].astype(np.int64)
    o = np.argsort(lb)
    assert lb[o][0] == 0 and np.all(lb[o][1:] == (lb[o] + lc[o])[:-1]) and (lb[o] + lc[o])[-1] == N
    for v in np.nonzero(internal)[0]:
        fc = int(h["first_child"][v]); k = bin(int(h["child_mask"][v])).count("1")
        assert int(h["part_count"][fc:fc + k].sum()) == int(h["part_count"][v])
    sh = 3 * (D - h["depth"].astype(np.int64))
    assert np.array_equal(kn[h["part_begin"].astype(np.int64)] >> sh, h["prefix"].astype(np.int64))
    assert np.array_equal(h["pt_count"], np.minimum(h["part_count"], n))
    assert h["n_points"] == int(h["pt_count"].astype(np.int64).sum())


def test_sampled_nodes_match_direct_definition(c3):
    s, d, b, tree, h, keys_D = c3
    n, D = 16000, 8
    log("density counts")
    dens = olod.density_counts(s.x, s.y, s.z, D)
    counts = h["part_count"].astype(np.int64)
    depth = h["depth"].astype(np.int64)
    rng = np.random.default_rng(1)
    picks = []
    d1 = np.nonzero((depth == 1) & (counts > n))[0]
    picks.append(int(d1[np.argmin(counts[d1])]))       # the smallest depth-1 internal node
    for dd in (2, 3, 4, 5, 6, 7, 8):
        cand = np.nonzero((depth == dd) & (counts > n) & (counts < 4_000_000))[0]
        if len(cand):
            picks.append(int(rng.choice(cand)))
    small = np.nonzero(counts <= n)[0]
    picks += [int(v) for v in rng.choice(small, 3, replace=False)]
    for v in picks:
        dd = int(depth[v])
        cell = olod.deinterleave(int(h["prefix"][v]), dd)
        t0 = time.time()
        ids, qx, qy, qz, mass, M = olod.node_direct(s.x, s.y, s.z, s.m, cell, dd, n, D, dens_counts=dens,
                                                      keys_D=keys_D)
        pb, pc = int(h["pt_begin"][v]), int(h["pt_count"][v])
        log(f"node {v} depth {dd} count {counts[v]}: oracle {time.time() - t0:.1f} s")
        assert np.array_equal(h["pt_id"][pb:pb + pc], ids), v
        assert np.array_equal(h["qx"][pb:pb + pc], qx) and np.array_equal(h["qy"][pb:pb + pc], qy)
        assert np.array_equal(h["qz"][pb:pb + pc], qz)
        ulp = np.abs(h["pt_mass"][pb:pb + pc].view(np.int32).astype(np.int64) - mass.view(np.int32))
        assert ulp.max() <= 1, v
        assert abs(h["node_mass"][v] - M) <= 1e-12 * M


def test_sampled_pixels_of_full_render(c3):
    s, d, b, tree, h, keys_D = c3
    cam = lib.Camera.ortho(1024, 1024)
    img = lib.splat(*d, cam).cpu().numpy()
    rng = np.random.default_rng(2)
    flat = np.argsort(-img.ravel())
    pix = np.concatenate([flat[:4], rng.choice(np.nonzero(img.ravel() > 0)[0], 8, replace=False)])
    pi, pj = pix % 1024, pix // 1024
    log("oracle pixels")
    want = osplat.render_pixels(osplat.Camera(0, 1024, 1024), s.x, s.y, s.z, s.m, pi, pj)
    got = img[pj, pi].astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-5 * want), (got, want)


def test_every_schedule_byte_identical_at_full_size(c3):
    """The persistent schedule (mode 2, the tuner's fastest grid for it) and the
    per-level schedule with another block size give the same bytes as the tuned
    build, on every output array."""
    import torch
    s, d, b, tree, h, keys_D = c3
    mode2 = [(c, ms) for c, ms in b.tune_record["candidates"] if c["mode"] == 2]
    assert mode2
    best2 = min(mode2, key=lambda t: t[1])[0]
    nn, npt = h["n_nodes"], h["n_points"]
    for sched in (best2, {"mode": 1, "select_threads": 1024, "persistent_blocks": 0}):
        p = lib.BuildParams(n=16000, max_depth=8, seed=0, mode=sched["mode"],
                            select_threads=sched["select_threads"], persistent_blocks=sched["persistent_blocks"])
        b2 = lib.Builder(s.n, p)
        t2 = b2.build(*d)
        torch.cuda.synchronize()
        assert torch.equal(t2.counts, tree.counts), sched
        for k, a in tree.arrays.items():
            m = nn if k in ("prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count",
                            "pt_begin", "pt_count", "node_mass") else npt
            assert torch.equal(a[:m].view(torch.uint8), t2.arrays[k][:m].view(torch.uint8)), (sched, k)
        log(f"schedule {sched}: byte-identical")
        del b2, t2
        torch.cuda.empty_cache()


def test_thinned_cut_sampled_pixels(c3):
    """A cut that thins (orthographic 1024^2, tau = 4 px: depth-4 nodes of at
    most n points each, shallower leaves whole) drawn by the LOD render, on
    sampled pixels of one depth-4 (x, y) column, against the oracle: the
    column's part of the cut derived from the particles (ancestor counts), each
    of its nodes' stored points from the definition (`node_direct`), decoded,
    and the pixels summed in float64.  Pixels lie at least 4 px inside the
    column, so no point outside it reaches them."""
    import torch
    s, d, b, tree, h, keys_D = c3
    n, D, tau, W = 16000, 8, 4.0, 1024
    cam = lib.Camera.ortho(W, W)
    ids, nsel = lib.select_nodes(tree, cam, tau, n)
    k = int(lib._to_numpy(nsel)[0])
    cut = lib._to_numpy(ids[:k]).astype(np.int64)
    depth = h["depth"].astype(np.int64)
    leaf = h["first_child"] == lib.NONE
    # the orthographic cut stops at the first depth whose spacing is <= tau
    dstar = next(dd for dd in range(D + 1) if W * 2.0 ** -dd <= tau * np.cbrt(n))
    assert dstar == 4
    assert np.all((depth[cut] == dstar) | (leaf[cut] & (depth[cut] < dstar)))
    drawn = int(h["pt_count"][cut].astype(np.int64).sum())
    log(f"tau 4 cut: {k} nodes, {drawn} points drawn of {s.n}")
    assert drawn < s.n // 2
    img = lib.splat_lod(tree, ids, nsel, s.n, cam).cpu().numpy()
    # the heaviest depth-4 (x, y) column
    c4x = olod.cell_coords(s.x, 4); c4y = olod.cell_coords(s.y, 4)
    col = np.bincount(c4x + 16 * c4y, minlength=256)
    cx, cy = int(np.argmax(col) % 16), int(np.argmax(col) // 16)
    shift = [np.uint64(3 * (D - dd)) for dd in range(D + 1)]
    nodes = []
    for cz in range(16):
        for dd in range(0, dstar + 1):
            c = (cx >> (dstar - dd), cy >> (dstar - dd), cz >> (dstar - dd))
            pref = int(olod.interleave(np.array([c[0]]), np.array([c[1]]), np.array([c[2]]), dd)[0])
            cnt = int(np.count_nonzero((keys_D >> shift[dd]) == np.uint64(pref)))
            if cnt == 0:
                break
            if cnt <= n or dd == dstar:
                if (dd, c) not in nodes:
                    nodes.append((dd, c))
                break
    log(f"column ({cx}, {cy}): {len(nodes)} cut nodes from the definition")
    dens = olod.density_counts(s.x, s.y, s.z, D)
    X, Y, Z, M = [], [], [], []
    for dd, c in nodes:
        sel, qx, qy, qz, mass, _ = olod.node_direct(s.x, s.y, s.z, s.m, c, dd, n, D, dens_counts=dens, keys_D=keys_D)
        X.append(olod.decode(qx, c[0], dd)); Y.append(olod.decode(qy, c[1], dd)); Z.append(olod.decode(qz, c[2], dd))
        M.append(mass)
    X, Y, Z, M = (np.concatenate(a) for a in (X, Y, Z, M))
    rng = np.random.default_rng(3)
    lo_i, hi_i = cx * 64 + 4, cx * 64 + 59
    lo_j, hi_j = cy * 64 + 4, cy * 64 + 59
    sub = img[lo_j:hi_j + 1, lo_i:hi_i + 1]
    flat = np.argsort(-sub.ravel())[:4]
    rnd = rng.choice(sub.size, 8, replace=False)
    pix = np.concatenate([flat, rnd])
    pi = lo_i + pix % sub.shape[1]; pj = lo_j + pix // sub.shape[1]
    want = osplat.render_pixels(osplat.Camera(0, W, W), X, Y, Z, M, pi, pj)
    got = img[pj, pi].astype(np.float64)
    assert np.all((want > 0) | (got == 0))
    ok = want > 0
    err = np.abs(got[ok] - want[ok]) / want[ok]
    log(f"thinned cut pixels: max relative error {err.max():.2e} over {ok.sum()} pixels")
    assert err.max() <= 1e-5


def _leaf_points(s, keys_D, near, n, D):
    """Decoded positions of particles `near` as points of their leaves (the
    tau = 1 cut draws every leaf whole): each particle's leaf is the shallowest
    cell on its path holding at most n particles (depth D at the deepest), and
    its 16-bit codes are relative to that cell."""
    leaf_d = np.full(len(near), D, dtype=np.int64)
    kn = keys_D[near]
    for dd in range(D - 1, -1, -1):
        sh = np.uint64(3 * (D - dd))
        counts = np.bincount((keys_D >> sh).astype(np.int64), minlength=1 << (3 * dd))
        small = counts[(kn >> sh).astype(np.int64)] <= n
        leaf_d[small] = dd
    ld = leaf_d.astype(np.uint64)
    leaf_key = (ld << np.uint64(60)) | (kn >> (np.uint64(3) * (np.uint64(D) - ld)))
    uniq, inv = np.unique(leaf_key, return_inverse=True)
    X = np.empty(len(near), np.float32); Y = np.empty_like(X); Z = np.empty_like(X)
    order = np.argsort(inv, kind="stable")
    bounds = np.searchsorted(inv[order], np.arange(len(uniq) + 1))
    for u in range(len(uniq)):
        at = order[bounds[u]:bounds[u + 1]]
        dd = int(leaf_d[at[0]])
        for dst, a in zip((X, Y, Z), (s.x, s.y, s.z)):
            c = int(olod.cell_coords(a[near[at[:1]]], dd)[0])
            dst[at] = olod.decode(olod.quantise(a[near[at]], c, dd), c, dd)
    log(f"{len(near)} particles in {len(uniq)} leaves")
    return X, Y, Z


def test_cubic_lod_render_block_at_full_size(c3):
    """The cubic-blob LOD render that the benchmark times (orthographic
    1024^2, tau = 1 px: every leaf drawn whole, h = 1.5 px, the windowed
    accumulation) on a 16 x 16 pixel block of the heaviest depth-4 column,
    against the oracle: every particle near the block is a point of its leaf
    (the shallowest cell holding at most n particles, from the particle counts
    of each depth), quantised at the leaf's depth and decoded; the cubic
    oracle sums the block's pixels in float64.  The particles taken reach 3 px
    beyond the block, past any blob that touches it."""
    from oracle import cubic as ocubic
    s, d, b, tree, h, keys_D = c3
    n, D, W, hpx = 16000, 8, 1024, 1.5
    cam = lib.Camera.ortho(W, W)
    ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
    k = int(lib._to_numpy(nsel)[0])
    cut = lib._to_numpy(ids[:k]).astype(np.int64)
    assert np.all(h["first_child"][cut] == lib.NONE)      # tau 1 draws the leaves
    assert int(h["pt_count"][cut].astype(np.int64).sum()) == s.n
    img = lib.splat_lod(tree, ids, nsel, s.n, cam, blob=lib.Blob.cubic(h_px=hpx)).cpu().numpy()
    # the block: the centre of the heaviest depth-4 (x, y) column
    c4x = olod.cell_coords(s.x, 4); c4y = olod.cell_coords(s.y, 4)
    col = np.bincount(c4x + 16 * c4y, minlength=256)
    cx, cy = int(np.argmax(col) % 16), int(np.argmax(col) // 16)
    i0, j0 = cx * 64 + 24, cy * 64 + 24
    x64, y64 = s.x.astype(np.float64) * W, s.y.astype(np.float64) * W
    near = np.nonzero((x64 > i0 - 3) & (x64 < i0 + 19) & (y64 > j0 - 3) & (y64 < j0 + 19))[0]
    log(f"cubic block ({i0}, {j0}): {len(near)} particles nearby")
    X, Y, Z = _leaf_points(s, keys_D, near, n, D)
    want = ocubic.render(osplat.Camera(0, W, W), X, Y, Z, s.m[near], h_px=hpx)[j0:j0 + 16, i0:i0 + 16]
    got = img[j0:j0 + 16, i0:i0 + 16].astype(np.float64)
    assert np.all((want > 0) | (got == 0))
    ok = want > 0
    err = np.abs(got[ok] - want[ok]) / want[ok]
    log(f"cubic block: max relative error {err.max():.2e} over {ok.sum()} pixels")
    assert ok.sum() > 200 and err.max() <= 1e-5


def test_highlight_at_full_size(c3):
    """ID highlighting at the benchmark configuration (a million random ids,
    the tau = 1 cut): the flag of every one of the 229 M stored points equals
    the membership of its id (numpy over the stored ids), and on a 16 x 16
    block of the heaviest column the highlight image equals the oracle's
    Gaussian pixels over the highlighted particles' leaf points near it."""
    import torch
    s, d, b, tree, h, keys_D = c3
    n, D, W, N = 16000, 8, 1024, s.n
    sel = np.random.default_rng(7).choice(N, 1_000_000, replace=False)
    bits = lib.highlight_bits(sel, N, "cuda")
    flags = lib.highlight_flags(tree, bits, N)
    S = h["n_points"]
    got = np.unpackbits(lib._to_numpy(flags).view(np.uint8), bitorder="little")[:S].astype(bool)
    want = np.isin(h["pt_id"], sel)
    assert np.array_equal(got, want)
    log(f"flags: {int(want.sum())} of {S} stored points highlighted")
    cam = lib.Camera.ortho(W, W)
    ids, nsel = lib.select_nodes(tree, cam, 1.0, n)
    img = torch.empty((W, W), dtype=torch.float32, device="cuda")
    hl = torch.empty_like(img)
    ws = torch.empty(lib.splat_lod_highlight_workspace_bytes(tree.node_capacity, N, len(sel), cam),
                     dtype=torch.uint8, device="cuda")
    lib.splat_lod_highlight(tree, ids, nsel, N, cam, flags, len(sel), workspace=ws, out=img, out_hl=hl)
    hl = hl.cpu().numpy()
    c4x = olod.cell_coords(s.x, 4); c4y = olod.cell_coords(s.y, 4)
    col = np.bincount(c4x + 16 * c4y, minlength=256)
    cx, cy = int(np.argmax(col) % 16), int(np.argmax(col) // 16)
    i0, j0 = cx * 64 + 24, cy * 64 + 24
    x64, y64 = s.x.astype(np.float64) * W, s.y.astype(np.float64) * W
    near = np.nonzero((x64 > i0 - 5) & (x64 < i0 + 21) & (y64 > j0 - 5) & (y64 < j0 + 21))[0]
    on = np.isin(near, sel)
    X, Y, Z = _leaf_points(s, keys_D, near[on], n, D)
    pi, pj = np.meshgrid(np.arange(i0, i0 + 16), np.arange(j0, j0 + 16))
    pi, pj = pi.ravel(), pj.ravel()
    want_px = osplat.render_pixels(osplat.Camera(0, W, W), X, Y, Z, s.m[near[on]], pi, pj)
    got_px = hl[pj, pi].astype(np.float64)
    assert np.all((want_px > 0) | (got_px == 0))
    ok = want_px > 0
    err = np.abs(got_px[ok] - want_px[ok]) / want_px[ok]
    log(f"highlight block: {int(on.sum())} highlighted particles nearby, max relative error "
        f"{err.max():.2e} over {ok.sum()} pixels")
    assert ok.sum() > 50 and err.max() <= 1e-5

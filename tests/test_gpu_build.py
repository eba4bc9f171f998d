"""HIP LOD build vs the CPU oracle, through the C ABI.

Node tables, stored ids and 16-bit codes must be bit-exact; float64 node
masses within 1e-12 relative (summation order); float32 stored masses within
1 ulp (the float64 renormalisation sum is order dependent).
"""
import numpy as np
import pytest

import synth
from oracle import lod as olod
from paper_0811_2055_amd import lib

from gpu_util import compare_tree, kbin_of, to_dev

pytestmark = pytest.mark.gpu


def _face_set(N, seed):
    rng = np.random.default_rng(seed)
    x = rng.random(N).astype(np.float32)
    y = rng.random(N).astype(np.float32)
    z = rng.random(N).astype(np.float32)
    k = N // 8
    x[:k] = (rng.integers(0, 33, k) / 32.0).astype(np.float32)
    y[k:2 * k] = np.float32(1.0)
    z[2 * k:3 * k] = np.float32(0.0)
    m = rng.uniform(0.1, 5.0, N).astype(np.float32)
    return synth.Snapshot(x, y, z, m)


def _dup_set(N, seed):
    s = synth.small_clustered(N, seed)
    k = N // 3
    s.x[:k] = np.float32(0.3); s.y[:k] = np.float32(0.71); s.z[:k] = np.float32(0.123)
    return s


CASES = [
    # name, generator, n, D, alpha, seed, L_rho
    ("one", lambda: synth.uniform(1, 1), 4, 3, 1, 0, None),
    ("two_same", lambda: synth.Snapshot(np.full(2, 0.5, np.float32), np.full(2, 0.5, np.float32),
                                        np.full(2, 0.5, np.float32), np.ones(2, np.float32)), 1, 2, 1, 0, None),
    ("ragged", lambda: synth.small_clustered(5000, 1), 37, 5, 1, 3, None),
    ("faces", lambda: _face_set(9000, 2), 20, 4, 1, 4, None),
    ("dups_overfull", lambda: _dup_set(6000, 3), 50, 3, 1, 5, None),
    ("alpha0", lambda: synth.small_clustered(12000, 4), 64, 5, 0, 6, None),
    ("alpha_neg", lambda: synth.small_clustered(12000, 5), 64, 5, -1, 7, None),
    ("lrho", lambda: synth.small_clustered(12000, 6), 100, 6, 1, 8, 3),
    ("depth0", lambda: synth.small_clustered(3000, 7), 100, 0, 1, 9, None),
    ("n1", lambda: synth.small_clustered(2000, 8), 1, 4, 1, 10, None),
    ("nbig", lambda: synth.small_clustered(2000, 9), 5000, 4, 1, 11, None),
    ("deep", lambda: synth.small_clustered(100000, 10), 512, 7, 1, 12, None),
    ("d10", lambda: synth.small_clustered(30000, 11), 40, 10, 1, 13, None),
]


@pytest.mark.parametrize("mode", [2, 1])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_build_matches_oracle(case, mode):
    name, gen, n, D, alpha, seed, L = case
    s = gen()
    print(f"[build parity] {name} N={s.n} n={n} D={D} alpha={alpha} mode={mode}", flush=True)
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=n, D=D, L_rho=L, alpha=alpha, seed=seed)
    b = lib.Builder(s.n, lib.BuildParams(n=n, max_depth=D, density_level=L, alpha=alpha, seed=seed, mode=mode))
    tree = b.build(*to_dev(s))
    h = tree.host()
    compare_tree(h, ref, name)
    # intermediates
    import torch
    keys = lib._to_numpy(b.view(0, torch.uint32)).astype(np.uint64)
    ids = lib._to_numpy(b.view(1, torch.uint32)).astype(np.int64)
    w = lib._to_numpy(b.view(2, torch.uint32)).astype(np.uint64)
    kb = lib._to_numpy(b.view(3, torch.uint16)).astype(np.int64)
    wit = lib._to_numpy(b.view(4, torch.uint32)).astype(np.int64)[:ref.n_nodes]
    assert np.array_equal(keys, ref.skey)
    assert np.array_equal(ids, ref.order)
    assert np.array_equal(w, ref.w)
    # the bins are the bins of the oracle's keys (hence monotone in them)
    assert np.array_equal(kb, kbin_of(ref.K))
    sel = ref.witness >= 0
    assert np.array_equal(wit[sel], ref.witness[sel])


# Sizes around the sort's tile edges (4096 elements) and the digit-offset
# scan's block edges (4096 counts = 16 tiles): one tile short, exact and one
# over; a single scan block exactly full; two scan blocks, the second ragged;
# and D = 10 (four 8-bit passes).
SORT_EDGES = [(4095, 8), (4096, 8), (4097, 8), (12289, 8), (65536, 8), (69633, 8), (40961, 10)]


@pytest.mark.parametrize("N,D", SORT_EDGES, ids=[f"N{n}_D{d}" for n, d in SORT_EDGES])
def test_sort_at_tile_edges(N, D):
    """The sorted keys and ids equal a stable sort of the depth-D Morton keys
    (ids ascending within equal keys); a third of the particles share one
    cell, so equal keys span several tiles."""
    import torch
    s = _dup_set(N, 20 + N % 97)
    print(f"[sort edges] N={N} D={D}", flush=True)
    keys_D = olod.interleave(*(olod.cell_coords(a, D) for a in (s.x, s.y, s.z)), D)
    order = np.argsort(keys_D, kind="stable")
    b = lib.Builder(N, lib.BuildParams(n=64, max_depth=D, alpha=1, seed=1))
    b.build(*to_dev(s))
    keys = lib._to_numpy(b.view(0, torch.uint32)).astype(np.uint64)
    ids = lib._to_numpy(b.view(1, torch.uint32)).astype(np.int64)
    assert np.array_equal(ids, order)
    assert np.array_equal(keys, keys_D[order])


def test_empty_input():
    import torch
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    tree = lib.build(e, e, e, e, lib.BuildParams(n=4, max_depth=3))
    h = tree.host()
    assert h["n_nodes"] == 0 and h["n_points"] == 0 and h["status"] == 0


def test_config1_full_size():
    s = synth.config1()
    print(f"[build parity] config1 N={s.n}", flush=True)
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=4096, D=4, alpha=1, seed=0)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=4096, max_depth=4, alpha=1, seed=0))
    compare_tree(tree.host(), ref, "config1")


def test_schedules_identical():
    """Per-node launches, level launches and every block size give identical bytes."""
    s = synth.small_clustered(60000, 21)
    outs = []
    for mode, thr, grid in ((2, 0, 0), (1, 0, 0), (0, 0, 0), (1, 64, 0), (2, 256, 1), (2, 64, 7), (2, 512, 3000)):
        tree = lib.build(*to_dev(s), lib.BuildParams(n=300, max_depth=6, seed=2, mode=mode, select_threads=thr,
                                                     persistent_blocks=grid))
        outs.append(tree.host())
    for h in outs[1:]:
        for k, v in outs[0].items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, h[k]), k
            else:
                assert v == h[k], k


def test_persistent_handoffs_many_levels():
    """The persistent schedule hands a node from the block that finishes its
    last selecting child to whichever block reduces it, across XCDs: a deep
    tree with small nodes (thousands of climbs through ten levels) built in
    mode 2 with several grids equals the per-level build byte for byte, and
    the per-level build equals the oracle."""
    s = synth.small_clustered(200000, 23)
    p = dict(n=12, max_depth=10, seed=5)
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=12, D=10, alpha=1, seed=5)
    base = lib.build(*to_dev(s), lib.BuildParams(mode=1, **p)).host()
    compare_tree(base, ref)
    for thr, grid in ((256, 0), (1024, 0), (64, 4096), (512, 17)):
        h = lib.build(*to_dev(s), lib.BuildParams(mode=2, select_threads=thr, persistent_blocks=grid, **p)).host()
        for k, v in base.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, h[k]), (thr, grid, k)
            else:
                assert v == h[k], (thr, grid, k)


def test_repeat_runs_identical():
    s = synth.small_clustered(50000, 22)
    b = lib.Builder(s.n, lib.BuildParams(n=200, max_depth=6, seed=4))
    d = to_dev(s)
    h1 = b.build(*d).host()
    h2 = b.build(*d).host()
    for k, v in h1.items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, h2[k]), k


def test_builds_on_two_streams_match_builds_alone():
    """Two builders on two caller streams, launched alternately without
    waiting: the library's own second stream (the density kernel's), forked
    from and joined into each caller's stream, serves both.  Every tree equals
    the one built alone, in the per-level and the persistent schedule."""
    import torch
    sa, sb = synth.small_clustered(300000, 41), synth.small_clustered(220000, 42)
    da, db = to_dev(sa), to_dev(sb)
    for mode in (1, 2):
        p = lib.BuildParams(n=400, max_depth=7, seed=3, mode=mode)
        alone = []
        for s, d in ((sa, da), (sb, db)):
            b = lib.Builder(s.n, p)
            alone.append(b.build(*d).host())
        torch.cuda.synchronize()
        builders = [lib.Builder(sa.n, p), lib.Builder(sb.n, p)]
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        for _ in range(3):
            for b, d, st in zip(builders, (da, db), streams):
                with torch.cuda.stream(st):
                    b.build(*d)
        torch.cuda.synchronize()
        for b, ref in zip(builders, alone):
            h = b.tree.host()
            for k, v in ref.items():
                if isinstance(v, np.ndarray):
                    assert np.array_equal(v, h[k]), (mode, k)
                else:
                    assert v == h[k], (mode, k)


def test_builds_from_two_host_threads_match_builds_alone():
    """Two host threads, each building on its own stream (the library's fork
    onto its second stream is taken under a lock): every tree equals the one
    built alone."""
    import threading
    import torch
    sa, sb = synth.small_clustered(300000, 43), synth.small_clustered(260000, 44)
    da, db = to_dev(sa), to_dev(sb)
    p = lib.BuildParams(n=400, max_depth=7, seed=6, mode=1)
    alone = [lib.Builder(s.n, p).build(*d).host() for s, d in ((sa, da), (sb, db))]
    builders = [lib.Builder(sa.n, p), lib.Builder(sb.n, p)]
    torch.cuda.synchronize()
    errors = []

    def work(b, d):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for _ in range(4):
                    b.build(*d)
            st.synchronize()
        except Exception as e:          # reported by the main thread
            errors.append(e)
    threads = [threading.Thread(target=work, args=(b, d)) for b, d in zip(builders, (da, db))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    torch.cuda.synchronize()
    for b, ref in zip(builders, alone):
        h = b.tree.host()
        for k, v in ref.items():
            if isinstance(v, np.ndarray):
                assert np.array_equal(v, h[k]), k
            else:
                assert v == h[k], k


def test_batch_matches_oracle():
    import torch
    parts = [synth.small_clustered(3000, 31), synth.uniform(0, 1), synth.small_clustered(5000, 32),
             synth.uniform(700, 33)]
    x = np.concatenate([p.x for p in parts]); y = np.concatenate([p.y for p in parts])
    z = np.concatenate([p.z for p in parts]); m = np.concatenate([p.m for p in parts])
    off = np.concatenate([[0], np.cumsum([p.n for p in parts])]).astype(np.int64)
    ref = olod.lod_build(x, y, z, m, n=40, D=5, seed=9, snap_offsets=off)
    s = synth.Snapshot(x, y, z, m)
    offs = torch.from_numpy(off.astype(np.int64)).cuda().view(torch.uint64)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=40, max_depth=5, seed=9), snap_offsets=offs)
    compare_tree(tree.host(), ref, "batch")


def test_domain_error_is_flagged():
    s = synth.small_clustered(1000, 40)
    s.x[17] = np.float32(np.nan)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=16, max_depth=3))
    assert tree.host()["status"] & lib.STATUS_DOMAIN
    s = synth.small_clustered(1000, 41)
    s.m[3] = np.float32(-1.0)
    tree = lib.build(*to_dev(s), lib.BuildParams(n=16, max_depth=3))
    assert tree.host()["status"] & lib.STATUS_DOMAIN


def test_autotune_keeps_bytes_and_caches(tmp_path):
    from paper_0811_2055_amd import autotune
    s = synth.small_clustered(80000, 51)
    d = to_dev(s)
    b = lib.Builder(s.n, lib.BuildParams(n=400, max_depth=6, seed=3, mode=2))
    ref = b.build(*d).host()
    rec = autotune.tune(b, *d, path=str(tmp_path / "tune.json"), device_name="test")
    assert rec["mode"] in (1, 2) and len(rec["candidates"]) == 12
    got = b.build(*d).host()
    for k, v in ref.items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, got[k]), k
    b2 = lib.Builder(s.n, lib.BuildParams(n=400, max_depth=6, seed=3, mode=2))
    assert autotune.apply_cached(b2, "test", path=str(tmp_path / "tune.json"))
    assert (b2.params.mode, b2.params.select_threads) == (rec["mode"], rec["select_threads"])

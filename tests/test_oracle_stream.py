"""Pins for the streaming policy oracle (oracle/stream.py): every frame draws
a cut of the tree made of resident nodes (each leaf covered exactly once),
loads never exceed the byte budget nor the pool, a still camera converges to
the full view-dependent cut, and a fly-through under a tight budget and a
small pool keeps all of that while evicting."""
import numpy as np
import pytest

import synth
from oracle import cut, lod, splat, stream

NONE = 0xFFFFFFFF


def _leaf_cover(t, chosen):
    chosen = set(int(v) for v in chosen)
    for v in range(t.n_nodes):
        if int(t.first_child[v]) != NONE:
            continue
        hits, u = 0, v
        while True:
            hits += u in chosen
            p = int(t.parent[u])
            if p == NONE:
                break
            u = p
        assert hits == 1


@pytest.fixture(scope="module")
def tree():
    s = synth.small_clustered(40000, 601)
    return lod.lod_build(s.x, s.y, s.z, s.m, n=200, D=6, seed=1)


def test_still_camera_converges_to_the_cut(tree):
    cam = splat.Camera(1, 128, 128, pos=(0.45, 0.5, -0.3), F=110.0, near=1e-3)
    st = stream.Streamer(tree, slots=tree.n_nodes)
    want = cut.select(tree, cam, 1.0, 200)
    for f in range(tree.D + 2):
        draw, loaded, evicted, nbytes = st.frame_step(cam, 1.0, 200, budget=1 << 40)
        _leaf_cover(tree, draw)
        assert not evicted
    assert np.array_equal(np.array(draw), want)
    # nothing is left to load
    draw2, loaded2, _, nbytes2 = st.frame_step(cam, 1.0, 200, budget=1 << 40)
    assert loaded2 == [] and nbytes2 == 0 and draw2 == draw


def test_flythrough_under_budget_and_pool(tree):
    slots = 60
    budget = 14 * 200 * 5                  # about five full nodes per frame
    st = stream.Streamer(tree, slots=slots)
    rng_path = np.linspace(0.0, 1.0, 30)
    total_loaded = total_evicted = total_bytes = 0
    for a in rng_path:
        p = 0.1 + 0.8 * a                  # along the box diagonal, inside it
        cam = splat.Camera(1, 128, 128, pos=(p, p, p), F=110.0, near=1e-3)
        draw, loaded, evicted, nbytes = st.frame_step(cam, 4.0, 200, budget)
        _leaf_cover(tree, draw)
        assert nbytes <= budget + 8 * 200 * 14
        assert all(st.resident[v] for v in draw)
        assert int(st.resident.sum()) <= slots
        assert not set(evicted) & set(draw)
        total_loaded += len(loaded)
        total_evicted += len(evicted)
        total_bytes += nbytes
    assert total_loaded > slots and total_evicted > 0
    assert total_bytes <= len(rng_path) * budget          # the link's capacity over the path

"""Tree files (save_tree / load_tree): the round trip of every node and point
array, the counts and capacities, on CPU tensors holding a tree built by the
oracle; files that are not tree files are refused."""
import numpy as np
import pytest
import torch

import synth
from oracle import lod as olod
from paper_0811_2055_amd import lib

KEYS = ("prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count", "pt_begin",
        "pt_count", "node_mass", "pt_id", "qx", "qy", "qz", "pt_mass")


def _cpu_tree(ref, extra_nodes=5, extra_points=7):
    V, S = ref.n_nodes, ref.n_points
    t = lib.alloc_tree(V + extra_nodes, S + extra_points, "cpu")
    for k in KEYS:
        a = getattr(ref, k)
        dst = t.arrays[k]
        dst[:a.shape[0]].copy_(lib._from_numpy(a.astype(lib._to_numpy(dst[:1]).dtype), dst.dtype, "cpu"))
    t.arrays["pt_count"][V:].zero_()
    t.arrays["pt_begin"][V:].fill_(S)
    t.counts.copy_(lib._from_numpy(np.array([V, S, 0], dtype=np.uint64), torch.uint64, "cpu"))
    return t


def test_tree_file_round_trip(tmp_path):
    s = synth.small_clustered(8000, 5)
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=64, D=5, alpha=1, seed=2)
    t = _cpu_tree(ref)
    path = str(tmp_path / "tree.npz")
    lib.save_tree(t, path, n=64)
    t2, n = lib.load_tree(path, device="cpu")
    assert n == 64
    assert (t2.node_capacity, t2.point_capacity) == (t.node_capacity, t.point_capacity)
    h, h2 = t.host(), t2.host()
    assert (h2["n_nodes"], h2["n_points"], h2["status"]) == (ref.n_nodes, ref.n_points, 0)
    for k in KEYS:
        assert h2[k].dtype == getattr(ref, k).dtype or k == "pt_begin", k
        assert np.array_equal(h2[k], h[k]), k
        assert np.array_equal(h2[k].astype(np.float64), getattr(ref, k).astype(np.float64)), k
    V, S = ref.n_nodes, ref.n_points
    assert int(t2.arrays["pt_count"][V:].sum()) == 0
    assert np.all(lib._to_numpy(t2.arrays["pt_begin"][V:]) == S)
    # larger capacities on request
    t3, _ = lib.load_tree(path, device="cpu", node_capacity=V + 100, point_capacity=S + 1000)
    assert (t3.node_capacity, t3.point_capacity) == (V + 100, S + 1000)
    assert np.array_equal(t3.host()["pt_id"], h["pt_id"])


def test_tree_file_refusals(tmp_path):
    s = synth.small_clustered(3000, 6)
    ref = olod.lod_build(s.x, s.y, s.z, s.m, n=64, D=4, alpha=0, seed=1)
    t = _cpu_tree(ref)
    t.counts[2:3].fill_(2)                      # LOD_STATUS_CAPACITY: the build ran out of room
    with pytest.raises(ValueError):
        lib.save_tree(t, str(tmp_path / "bad.npz"))
    other = str(tmp_path / "other.npz")
    np.savez(other, a=np.zeros(3))
    with pytest.raises(ValueError):
        lib.load_tree(other, device="cpu")
    # a truncated array
    good = _cpu_tree(ref)
    path = str(tmp_path / "t.npz")
    lib.save_tree(good, path)
    with np.load(path, allow_pickle=False) as f:
        d = {k: f[k] for k in f.files}
    d["qx"] = d["qx"][:-1]
    np.savez(str(tmp_path / "short.npz"), **d)
    with pytest.raises(ValueError):
        lib.load_tree(str(tmp_path / "short.npz"), device="cpu")

"""Shared helpers for the GPU parity tests (no method arithmetic here)."""
import numpy as np

NODE_KEYS = ("prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count",
             "pt_begin", "pt_count")
POINT_KEYS = ("pt_id", "qx", "qy", "qz")


def to_dev(s, dev="cuda"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (s.x, s.y, s.z, s.m)]


def ulp_diff(a, b):
    a = np.ascontiguousarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    b = np.ascontiguousarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    return np.abs(a - b)


def compare_tree(h, ref, label=""):
    """Bit-exact node table and point ids/codes; masses to 1 ulp (float32) and 1e-12 (float64)."""
    assert h["status"] == 0, (label, "status", h["status"])
    assert h["n_nodes"] == ref.n_nodes, (label, h["n_nodes"], ref.n_nodes)
    assert h["n_points"] == ref.n_points, (label, h["n_points"], ref.n_points)
    for k in NODE_KEYS:
        got = h[k].astype(np.uint64)
        want = getattr(ref, k).astype(np.uint64)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (label, k, bad[:5], got[bad[:5]], want[bad[:5]])
    M, Mref = h["node_mass"], ref.node_mass
    assert np.all(np.abs(M - Mref) <= 1e-12 * np.abs(Mref)), (label, "node_mass")
    for k in POINT_KEYS:
        got, want = h[k], getattr(ref, k)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (label, k, bad[:5], got[bad[:5]], want[bad[:5]])
    u = ulp_diff(h["pt_mass"], ref.pt_mass)
    assert u.size == 0 or u.max() <= 1, (label, "pt_mass ulp", u.max())


def image_rel_err(img, ref):
    """Max relative error over pixels where the reference is positive, and whether zeros match."""
    img = np.asarray(img, dtype=np.float64)
    pos = ref > 0
    zeros_ok = bool(np.all(img[~pos] == 0.0))
    if not pos.any():
        return 0.0, zeros_ok
    rel = np.abs(img[pos] - ref[pos]) / ref[pos]
    return float(rel.max()), zeros_ok

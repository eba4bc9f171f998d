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


def check_sort_and_tree(keys, ids, h, N, n, D, keys_D, sample=20000, seed=0, snap_bits=0):
    """Properties of the sort and the tree that hold at any size.

    keys, ids: device tensors of the sorted keys and global ids; keys_D: the
    oracle's depth-D Morton keys (with the snapshot index above them when
    snap_bits > 0) of every particle, indexed by global id.
    """
    import torch
    keys = keys.long() & 0xFFFFFFFF
    ids = ids.long()
    assert bool((keys[1:] >= keys[:-1]).all()), "keys not sorted"
    eq = keys[1:] == keys[:-1]
    assert bool((ids[1:][eq] > ids[:-1][eq]).all()), "ids not ascending within equal keys"
    assert int(torch.bincount(ids, minlength=N).max()) == 1, "ids not a permutation"
    pos = np.random.default_rng(seed).integers(0, N, sample)
    pt = torch.from_numpy(pos).cuda()
    assert np.array_equal(keys[pt].cpu().numpy().astype(np.uint64), keys_D[ids[pt].cpu().numpy()])
    internal = h["first_child"] != 0xFFFFFFFF
    assert np.array_equal(internal, (h["part_count"] > n) & (h["depth"] < D))
    leaf = ~internal
    lb = h["part_begin"][leaf].astype(np.int64)
    lc = h["part_count"][leaf].astype(np.int64)
    o = np.argsort(lb)
    assert lb[o][0] == 0 and np.all(lb[o][1:] == (lb[o] + lc[o])[:-1]) and (lb[o] + lc[o])[-1] == N
    for v in np.nonzero(internal)[0]:
        fc = int(h["first_child"][v]); k = bin(int(h["child_mask"][v])).count("1")
        assert int(h["part_count"][fc:fc + k].sum()) == int(h["part_count"][v])
    kn = keys.cpu().numpy()
    sh = 3 * (D - h["depth"].astype(np.int64))
    assert np.array_equal(kn[h["part_begin"].astype(np.int64)] >> sh, h["prefix"].astype(np.int64))
    assert np.array_equal(h["pt_count"], np.minimum(h["part_count"], n))
    assert h["n_points"] == int(h["pt_count"].astype(np.int64).sum())


def sample_nodes(h, n, rng, depths=range(1, 9), cap=4_000_000, small=3):
    """The smallest depth-1 internal node, one random internal node per depth
    (at most `cap` particles) and a few small nodes."""
    counts = h["part_count"].astype(np.int64)
    depth = h["depth"].astype(np.int64)
    picks = []
    d1 = np.nonzero((depth == 1) & (counts > n))[0]
    if len(d1):
        picks.append(int(d1[np.argmin(counts[d1])]))
    for dd in depths:
        if dd == 1:
            continue
        cand = np.nonzero((depth == dd) & (counts > n) & (counts < cap))[0]
        if len(cand):
            picks.append(int(rng.choice(cand)))
    sm = np.nonzero(counts <= n)[0]
    picks += [int(v) for v in rng.choice(sm, min(small, len(sm)), replace=False)]
    return picks


def check_node_against_definition(h, v, x, y, z, m, n, D, dens, keys_D, snap=0):
    from oracle import lod as olod
    dd = int(h["depth"][v])
    cell = olod.deinterleave(int(h["prefix"][v]), dd)
    ids, qx, qy, qz, mass, M = olod.node_direct(x, y, z, m, cell, dd, n, D, dens_counts=dens, keys_D=keys_D,
                                                snap=snap)
    pb, pc = int(h["pt_begin"][v]), int(h["pt_count"][v])
    assert np.array_equal(h["pt_id"][pb:pb + pc], ids), v
    assert np.array_equal(h["qx"][pb:pb + pc], qx) and np.array_equal(h["qy"][pb:pb + pc], qy)
    assert np.array_equal(h["qz"][pb:pb + pc], qz)
    assert ulp_diff(h["pt_mass"][pb:pb + pc], mass).max(initial=0) <= 1, v
    assert abs(h["node_mass"][v] - M) <= 1e-12 * M


def kbin_of(K):
    """The 12-bit log-scale bin the selection keeps per particle: K < 128 maps
    to itself, larger K to 128 + 64 (e - 7) + the 6 bits after the leading one
    (e = its index)."""
    K = np.asarray(K, dtype=np.uint64)
    e = np.zeros(K.shape, dtype=np.int64)
    for b in range(1, 64):
        e[(K >> np.uint64(b)) != 0] = b
    out = np.where(K < 128, K, 0).astype(np.int64)
    big = K >= 128
    eb = e[big]
    out[big] = 128 + 64 * (eb - 7) + ((K[big] >> (eb - 6).astype(np.uint64)) & np.uint64(63)).astype(np.int64)
    return out

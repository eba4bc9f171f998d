"""Octree level-of-detail build -- plain definition (CPU oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (octree paragraph): a spatial octree whose every node
or leaf is represented by at most n points; surplus points are removed by
a density-weighted random subselection; a child covers the same space as
its part of the parent at eight times the detail.  Quantisation paragraph:
each stored coordinate is 2 bytes spanning the containing block.

Readings taken where the paper is silent (each a fixed choice):

* cells/keys: c = min(floor(a 2^D), 2^D - 1) per axis; the Morton key puts
  x in bit 0 of each 3-bit group; a batch prefixes the snapshot index above
  the 3D key bits.
* tree: root at depth 0 holds the snapshot; a node at depth d with more than
  n particles and d < D is internal and has its non-empty octants as
  children (ascending octant); all other nodes are leaves.  Node order is
  breadth first by level, Morton order within a level.
* density w_i: the number of particles in i's depth-L_rho cell.
* randomness: U_i = word 0 of Philox4x32-10 keyed by the seed, counter
  (id lo, id hi, snapshot, 0), plus one; u_i = U_i / 2^32.
* selection key (priority sampling with priority w^alpha / u, written as an
  unsigned integer so that every comparison is exact): alpha = +1:
  K = floor(U 2^31 / w); alpha = 0: K = U 2^31; alpha = -1: K = U w.
  Total order (K ascending, id ascending).
* selection: a node holding more than n particles stores the first n of its
  particles in that order; the (n+1)-th is the threshold witness t.  This is
  the direct definition; the bottom-up level-by-level construction gives
  the same set because top_k(A u B) = top_k(top_k(A) u top_k(B)).
* masses (float64): a_i = w_i^alpha, tau = a_t 2^32 / U_t,
  p_i = min(1, a_i / tau), mhat_i = m_i / p_i, s = M_node / sum(mhat),
  stored mass = fl32(s mhat_i).  Nodes holding at most n particles store
  their original masses.  M_node is the exactly rounded sum of the node's
  particle masses.
* quantisation: q = min(floor(a 2^(d+16)) - (c_d << 16), 65535) relative to
  the storing node at depth d; decode to the float32 nearest
  (c_d 2^16 + q + 1/2) 2^-(d+16).
* output: points grouped by node in node order, within a node ascending
  sorted position.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .philox import particle_uniform

NONE32 = 0xFFFFFFFF


class OracleError(ValueError):
    pass


@dataclass
class Tree:
    # node table (breadth-first order)
    prefix: np.ndarray        # uint64
    depth: np.ndarray         # uint8
    parent: np.ndarray        # uint32 (NONE32 for roots)
    first_child: np.ndarray   # uint32 (NONE32 for leaves)
    child_mask: np.ndarray    # uint8
    part_begin: np.ndarray    # uint64 (sorted position)
    part_count: np.ndarray    # uint64
    pt_begin: np.ndarray      # uint64
    pt_count: np.ndarray      # uint32
    node_mass: np.ndarray     # float64
    # stored points
    pt_id: np.ndarray         # uint32 (id within its snapshot)
    qx: np.ndarray            # uint16
    qy: np.ndarray
    qz: np.ndarray
    pt_mass: np.ndarray       # float32
    # intermediates, indexed by sorted position
    skey: np.ndarray = field(default=None)      # uint64 sorted keys
    order: np.ndarray = field(default=None)     # int64 global particle index
    w: np.ndarray = field(default=None)         # uint64 density
    U: np.ndarray = field(default=None)         # uint64
    K: np.ndarray = field(default=None)         # uint64
    witness: np.ndarray = field(default=None)   # int64 sorted position per node, -1 if none
    pt_pos: np.ndarray = field(default=None)    # int64 sorted position of each stored point
    pt_node: np.ndarray = field(default=None)   # int64 node of each stored point
    pt_mhat: np.ndarray = field(default=None)   # float64 m/p before the node rescale
    D: int = 0
    n: int = 0

    @property
    def n_nodes(self) -> int:
        return int(self.prefix.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.pt_id.shape[0])


# ---------------------------------------------------------------------------
# validation

def validate(x, y, z, m, n, D, L_rho, alpha, snap_offsets):
    if n < 1:
        raise OracleError("n must be >= 1")
    if not (0 <= D <= 10):
        raise OracleError("max depth must be in [0, 10]")
    if not (0 <= L_rho <= D):
        raise OracleError("density level must be in [0, D]")
    if alpha not in (-1, 0, 1):
        raise OracleError("alpha must be -1, 0 or +1")
    for a in (x, y, z):
        a64 = a.astype(np.float64)
        if not np.all(np.isfinite(a64)) or np.any(a64 < 0.0) or np.any(a64 > 1.0):
            raise OracleError("positions must be finite and inside [0, 1]")
    m64 = m.astype(np.float64)
    if not np.all(np.isfinite(m64)) or np.any(m64 < 0.0):
        raise OracleError("masses must be finite and non-negative")
    if np.any(np.diff(snap_offsets) < 0) or snap_offsets[0] != 0 or snap_offsets[-1] != len(x):
        raise OracleError("bad snapshot offsets")
    if np.any(np.diff(snap_offsets) >= 2 ** 31):
        raise OracleError("a snapshot must hold fewer than 2^31 particles")


# ---------------------------------------------------------------------------
# keys

def cell_coords(a: np.ndarray, d: int) -> np.ndarray:
    """c = min(floor(a 2^d), 2^d - 1); a*2^d is exact for float32 inputs."""
    c = np.floor(a.astype(np.float64) * (2.0 ** d)).astype(np.int64)
    return np.minimum(c, (1 << d) - 1)


def interleave(cx: np.ndarray, cy: np.ndarray, cz: np.ndarray, d: int) -> np.ndarray:
    """Morton code with x in bit 0 of each group of three."""
    key = np.zeros(cx.shape, dtype=np.uint64)
    for k in range(d):
        key |= (((cx >> k) & 1).astype(np.uint64) << np.uint64(3 * k))
        key |= (((cy >> k) & 1).astype(np.uint64) << np.uint64(3 * k + 1))
        key |= (((cz >> k) & 1).astype(np.uint64) << np.uint64(3 * k + 2))
    return key


def deinterleave(prefix: int, d: int):
    """Cell coordinates (cx, cy, cz) of a depth-d Morton prefix (snapshot bits ignored)."""
    cx = cy = cz = 0
    for k in range(d):
        cx |= ((prefix >> (3 * k)) & 1) << k
        cy |= ((prefix >> (3 * k + 1)) & 1) << k
        cz |= ((prefix >> (3 * k + 2)) & 1) << k
    return cx, cy, cz


def selection_keys(U: np.ndarray, w: np.ndarray, alpha: int) -> np.ndarray:
    U = U.astype(np.uint64)
    w = w.astype(np.uint64)
    if alpha == 1:
        return (U << np.uint64(31)) // w
    if alpha == 0:
        return U << np.uint64(31)
    return U * w


def weight_power(w: np.ndarray, alpha: int) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    if alpha == 1:
        return w
    if alpha == 0:
        return np.ones_like(w)
    return 1.0 / w


def exact_sum(v: np.ndarray) -> float:
    return math.fsum(np.asarray(v, dtype=np.float64).tolist())


def quantise(a: np.ndarray, c_node: int, d: int) -> np.ndarray:
    q = np.floor(a.astype(np.float64) * (2.0 ** (d + 16))).astype(np.int64) - (int(c_node) << 16)
    return np.minimum(q, 65535).astype(np.uint16)


def decode(q: np.ndarray, c_node, d: int) -> np.ndarray:
    """float32 nearest to (c 2^16 + q + 1/2) 2^-(d+16)."""
    num = (np.asarray(c_node, dtype=np.int64) << 16) + q.astype(np.int64)
    return ((2 * num + 1).astype(np.float64) * (2.0 ** -(d + 17))).astype(np.float32)


# ---------------------------------------------------------------------------
# the build

def lod_build(x, y, z, m, n: int, D: int, L_rho: int | None = None, alpha: int = 1,
              seed: int = 0, snap_offsets=None) -> Tree:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    m = np.ascontiguousarray(m, dtype=np.float32)
    N = int(x.shape[0])
    if L_rho is None:
        L_rho = D
    if snap_offsets is None:
        snap_offsets = np.array([0, N], dtype=np.int64)
    snap_offsets = np.asarray(snap_offsets, dtype=np.int64)
    validate(x, y, z, m, n, D, L_rho, alpha, snap_offsets)
    n_snap = len(snap_offsets) - 1

    snap = np.repeat(np.arange(n_snap, dtype=np.int64), np.diff(snap_offsets))
    pid = np.arange(N, dtype=np.int64) - snap_offsets[snap]

    # cells and Morton keys (snapshot index above the 3D key bits)
    key = interleave(cell_coords(x, D), cell_coords(y, D), cell_coords(z, D), D)
    key |= snap.astype(np.uint64) << np.uint64(3 * D)

    # stable sort: ties keep ascending particle index
    order = np.argsort(key, kind="stable")
    skey = key[order]

    # density: particles sharing the depth-L_rho cell
    cell = key >> np.uint64(3 * (D - L_rho))
    _, inv, cnt = np.unique(cell, return_inverse=True, return_counts=True)
    w_part = cnt[inv].astype(np.uint64)

    U_part = particle_uniform(pid, snap, seed)
    K_part = selection_keys(U_part, w_part, alpha)

    # breadth-first tree
    prefix, depth, parent, first_child, child_mask = [], [], [], [], []
    part_begin, part_count = [], []
    level = []
    for s in range(n_snap):
        lo = int(np.searchsorted(skey, np.uint64(s) << np.uint64(3 * D), "left"))
        hi = int(np.searchsorted(skey, np.uint64(s + 1) << np.uint64(3 * D), "left"))
        if hi > lo:
            level.append((s, 0, NONE32, lo, hi - lo))
    while level:
        nxt = []
        for (pfx, d, par, b, c) in level:
            idx = len(prefix)
            prefix.append(pfx); depth.append(d); parent.append(par)
            part_begin.append(b); part_count.append(c)
            first_child.append(NONE32); child_mask.append(0)
            if c > n and d < D:
                sh = 3 * (D - d - 1)
                mask = 0
                for o in range(8):
                    cp = pfx * 8 + o
                    lo = int(np.searchsorted(skey, np.uint64(cp << sh), "left"))
                    hi = int(np.searchsorted(skey, np.uint64((cp + 1) << sh), "left"))
                    if hi > lo:
                        mask |= 1 << o
                        nxt.append((cp, d + 1, idx, lo, hi - lo))
                child_mask[idx] = mask
        # children get indices after this level; fix first_child now
        base = len(prefix)
        for (cp, d1, par, b, c) in nxt:
            if first_child[par] == NONE32:
                first_child[par] = base
            base += 1
        level = nxt

    V = len(prefix)
    prefix = np.array(prefix, dtype=np.uint64)
    depth = np.array(depth, dtype=np.uint8)
    parent = np.array(parent, dtype=np.uint32)
    first_child = np.array(first_child, dtype=np.uint32)
    child_mask = np.array(child_mask, dtype=np.uint8)
    part_begin = np.array(part_begin, dtype=np.uint64)
    part_count = np.array(part_count, dtype=np.uint64)

    pt_count = np.minimum(part_count, np.uint64(n)).astype(np.uint32)
    pt_begin = np.zeros(V, dtype=np.uint64)
    if V:
        pt_begin[1:] = np.cumsum(pt_count.astype(np.uint64))[:-1]
    S = int(pt_count.astype(np.int64).sum())

    node_mass = np.zeros(V, dtype=np.float64)
    witness = np.full(V, -1, dtype=np.int64)
    pt_id = np.zeros(S, dtype=np.uint32)
    qx = np.zeros(S, dtype=np.uint16)
    qy = np.zeros(S, dtype=np.uint16)
    qz = np.zeros(S, dtype=np.uint16)
    pt_mass = np.zeros(S, dtype=np.float32)
    pt_pos = np.zeros(S, dtype=np.int64)
    pt_node = np.zeros(S, dtype=np.int64)
    pt_mhat = np.zeros(S, dtype=np.float64)

    for v in range(V):
        b, c, d = int(part_begin[v]), int(part_count[v]), int(depth[v])
        members = order[b:b + c]                       # global particle indices
        node_mass[v] = exact_sum(m[members])
        if c > n:
            # direct definition: the n+1 smallest (K, id) among the node's particles
            rank = np.lexsort((pid[members], K_part[members]))
            top = rank[:n + 1]
            chosen = np.sort(top[:n])                  # ascending sorted position
            t = members[top[n]]
            witness[v] = b + int(top[n])
            sel = members[chosen]
            a_sel = weight_power(w_part[sel], alpha)
            a_t = float(weight_power(np.array([w_part[t]]), alpha)[0])
            tau = a_t * 4294967296.0 / float(U_part[t])
            p = np.minimum(1.0, a_sel / tau)
            mhat = m[sel].astype(np.float64) / p
            s = node_mass[v] / exact_sum(mhat)
            mass_out = (s * mhat).astype(np.float32)
            pos = b + chosen
            est = mhat
        else:
            sel = members
            mass_out = m[sel].copy()
            pos = b + np.arange(c, dtype=np.int64)
            est = m[sel].astype(np.float64)
        o, k = int(pt_begin[v]), len(sel)
        pfx = int(prefix[v]) & ((1 << (3 * d)) - 1) if d else 0
        cx, cy, cz = deinterleave(pfx, d)
        pt_id[o:o + k] = pid[sel].astype(np.uint32)
        qx[o:o + k] = quantise(x[sel], cx, d)
        qy[o:o + k] = quantise(y[sel], cy, d)
        qz[o:o + k] = quantise(z[sel], cz, d)
        pt_mass[o:o + k] = mass_out
        pt_pos[o:o + k] = pos
        pt_node[o:o + k] = v
        pt_mhat[o:o + k] = est

    return Tree(prefix=prefix, depth=depth, parent=parent, first_child=first_child,
                child_mask=child_mask, part_begin=part_begin, part_count=part_count,
                pt_begin=pt_begin, pt_count=pt_count, node_mass=node_mass,
                pt_id=pt_id, qx=qx, qy=qy, qz=qz, pt_mass=pt_mass,
                skey=skey, order=order, w=w_part[order], U=U_part[order], K=K_part[order],
                witness=witness, pt_pos=pt_pos, pt_node=pt_node, pt_mhat=pt_mhat, D=D, n=n)


def node_origin(tree: Tree, v: int):
    d = int(tree.depth[v])
    pfx = int(tree.prefix[v]) & ((1 << (3 * d)) - 1) if d else 0
    return deinterleave(pfx, d), d


def decoded_points(tree: Tree, nodes=None):
    """Decode the stored points of `nodes` (all nodes if None) to float32 xyz and mass."""
    if nodes is None:
        nodes = range(tree.n_nodes)
    xs, ys, zs, ms = [], [], [], []
    for v in nodes:
        (cx, cy, cz), d = node_origin(tree, int(v))
        b, k = int(tree.pt_begin[v]), int(tree.pt_count[v])
        xs.append(decode(tree.qx[b:b + k], cx, d))
        ys.append(decode(tree.qy[b:b + k], cy, d))
        zs.append(decode(tree.qz[b:b + k], cz, d))
        ms.append(tree.pt_mass[b:b + k])
    if not xs:
        e = np.zeros(0, np.float32)
        return e, e, e, e
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(zs), np.concatenate(ms))


def node_direct(x, y, z, m, cell, d: int, n: int, D: int, L_rho: int | None = None, alpha: int = 1,
                seed: int = 0, dens_counts=None, keys_D=None, snap: int = 0):
    """Stored points of the single depth-d node with cell coordinates `cell`
    (cx, cy, cz), straight from the definition over the raw particles.

    Returns (ids ascending by (key, id), qx, qy, qz, masses, node mass), where the
    ids are the stored particles in the node's output order.  dens_counts may
    pass precomputed depth-L cell counts (see `density_counts`), keys_D the
    depth-D Morton keys of all particles (membership is then a key prefix test).
    For snapshot `snap` of a batch, x, y, z, m are that snapshot's particles
    (ids local to it) and snap enters the random stream.
    """
    if L_rho is None:
        L_rho = D
    if keys_D is not None:
        want = int(interleave(np.array([cell[0]]), np.array([cell[1]]), np.array([cell[2]]), d)[0])
        members = np.nonzero((keys_D >> np.uint64(3 * (D - d))) == np.uint64(want))[0]
    else:
        inside = np.ones(len(x), dtype=bool)
        for a, c in ((x, cell[0]), (y, cell[1]), (z, cell[2])):
            inside &= cell_coords(a, d) == c
        members = np.nonzero(inside)[0]
    mass_node = exact_sum(m[members])
    keys = interleave(cell_coords(x[members], D), cell_coords(y[members], D), cell_coords(z[members], D), D)
    order = np.lexsort((members, keys))            # sorted order: (key, id)
    members = members[order]
    if len(members) <= n:
        sel = members
        out_mass = m[sel].copy()
    else:
        if dens_counts is None:
            dens_counts = density_counts(x, y, z, L_rho)
        cl = (cell_coords(x[members], L_rho), cell_coords(y[members], L_rho), cell_coords(z[members], L_rho))
        w = dens_counts[cl[0] + (cl[1] << L_rho) + (cl[2] << (2 * L_rho))].astype(np.uint64)
        U = particle_uniform(members, snap, seed)
        K = selection_keys(U, w, alpha)
        rank = np.lexsort((members, K))
        top = rank[:n + 1]
        chosen = np.sort(top[:n])                   # ascending sorted position
        t = top[n]
        a_sel = weight_power(w[chosen], alpha)
        a_t = float(weight_power(np.array([w[t]]), alpha)[0])
        tau = a_t * 4294967296.0 / float(U[t])
        p = np.minimum(1.0, a_sel / tau)
        mhat = m[members[chosen]].astype(np.float64) / p
        s = mass_node / exact_sum(mhat)
        sel = members[chosen]
        out_mass = (s * mhat).astype(np.float32)
    q = [quantise(a[sel], c, d) for a, c in ((x, cell[0]), (y, cell[1]), (z, cell[2]))]
    return sel.astype(np.uint32), q[0], q[1], q[2], out_mass, mass_node


def density_counts(x, y, z, L: int) -> np.ndarray:
    """Particle count of every depth-L cell, indexed cx + cy 2^L + cz 2^(2L)."""
    idx = cell_coords(x, L) + (cell_coords(y, L) << L) + (cell_coords(z, L) << (2 * L))
    return np.bincount(idx, minlength=1 << (3 * L))

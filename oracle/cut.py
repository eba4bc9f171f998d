"""View-dependent node choice ("which blocks to draw") -- plain definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's block-choice paragraph: regions near the viewer are drawn from
deep in the tree, far regions from shallow nodes, and the CPU makes this
choice.  Reading used here: starting at the roots, descend into a node's
children while the node has children and either the camera is inside the
node's cube or the node's projected point spacing exceeds tau pixels.
Projected spacing of a depth-d node holding n points:
  orthographic  W 2^-d / n^(1/3)
  perspective   F 2^-d / (n^(1/3) dist),  dist = |node centre - camera|.
The cut lists, in node order, every node that is reached and not descended
into.  All arithmetic is float64 in the order written.
"""
from __future__ import annotations

import numpy as np

from .lod import Tree, node_origin
from .splat import Camera


def descends(tree: Tree, v: int, cam: Camera, tau_px: float, cbrt_n: float) -> bool:
    if int(tree.first_child[v]) == 0xFFFFFFFF:
        return False
    (cx, cy, cz), d = node_origin(tree, v)
    side = 2.0 ** -d
    if cam.projection == 0:
        return float(cam.W) * side > tau_px * cbrt_n
    ox, oy, oz = cx * side, cy * side, cz * side
    p = [float(np.float32(a)) for a in cam.pos]
    inside = (ox <= p[0] <= ox + side) and (oy <= p[1] <= oy + side) and (oz <= p[2] <= oz + side)
    if inside:
        return True
    h = side * 0.5
    dx = (ox + h) - p[0]
    dy = (oy + h) - p[1]
    dz = (oz + h) - p[2]
    dist = float(np.sqrt((dx * dx + dy * dy) + dz * dz))
    return float(np.float32(cam.F)) * side > (tau_px * cbrt_n) * dist


def select(tree: Tree, cam: Camera, tau_px: float, n: int) -> np.ndarray:
    cbrt_n = float(np.cbrt(np.float64(n)))
    V = tree.n_nodes
    reached = np.zeros(V, dtype=bool)
    desc = np.zeros(V, dtype=bool)
    out = []
    for v in range(V):                       # breadth-first order: parents come first
        par = int(tree.parent[v])
        reached[v] = (par == 0xFFFFFFFF) or (reached[par] and desc[par])
        if not reached[v]:
            continue
        desc[v] = descends(tree, v, cam, float(tau_px), cbrt_n)
        if not desc[v]:
            out.append(v)
    return np.array(out, dtype=np.int64)

"""Block store and view-dependent streaming -- plain definition (CPU oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's IO paragraphs: only the data a view needs is loaded, from a
spatially indexed store of blocks (octree nodes), at a rate an ordinary link
sustains (100 MB/s); the CPU decides which blocks to load and draw.  The
policy used here, per frame f, with a device pool of `slots` node slots and
a byte budget B (a node's block is 14 bytes per stored point):

1. desc(v): node v has children and the camera wants to descend into it (the
   view-dependent cut's test, `cut.descends`).
2. Visit from the roots over the resident tree: a visited node v is
   descended into when desc(v) and all its children are resident; every
   visited node is marked used at f.  Candidate groups: the children of each
   visited node with desc(v) whose children are not all resident.
3. The link carries B bytes per frame: a credit grows by B each frame and
   unused credit carries over, up to B plus one full group (8 n points of
   blocks) so that any group can eventually be loaded.  Groups are taken in
   order of priority: camera inside the parent's cube first, then larger
   projected point spacing of the parent, then smaller parent index.  A
   group costs the blocks of its non-resident children; loading stops at the
   first group that does not fit in the credit.
   Slots are freed first by evicting victims: resident non-root nodes with
   no resident children, not used at f, and not children of a node visited
   at f that the camera wants to descend into (the candidate groups), least
   recently used first (ties: larger node index first); loading stops when
   no victim is left.
4. The frame draws the visit of step 2 repeated over the new residency: the
   nodes visited and not descended into, in node order.
Roots are loaded when the store is opened and never evicted.
"""
from __future__ import annotations

import numpy as np

from . import cut, lod

NONE32 = 0xFFFFFFFF
BLOCK_BYTES_PER_POINT = 14


class Streamer:
    def __init__(self, tree: lod.Tree, slots: int):
        self.t = tree
        V = tree.n_nodes
        self.slots = slots
        self.resident = np.zeros(V, dtype=bool)
        self.used = np.full(V, -1, dtype=np.int64)
        self.wanted = np.full(V, -1, dtype=np.int64)   # frame at which v was visited with desc(v)
        self.frame = -1
        self.children = []
        for v in range(V):
            fc = int(tree.first_child[v])
            k = bin(int(tree.child_mask[v])).count("1")
            self.children.append(list(range(fc, fc + k)) if fc != NONE32 else [])
        self.roots = [v for v in range(V) if int(tree.parent[v]) == NONE32]
        if len(self.roots) > slots:
            raise ValueError("the pool cannot hold the roots")
        for r in self.roots:
            self.resident[r] = True
        self.free = slots - len(self.roots)
        self.credit = 0

    def _visit(self, desc):
        draw, visited = [], []
        stack = list(reversed(self.roots))
        while stack:
            v = stack.pop()
            visited.append(v)
            ch = self.children[v]
            if desc[v] and ch and all(self.resident[c] for c in ch):
                stack.extend(reversed(ch))
            else:
                draw.append(v)
        return sorted(draw), visited

    def frame_step(self, cam, tau_px: float, n: int, budget: int):
        """One frame; returns (draw list, loaded node ids, evicted node ids, bytes)."""
        self.frame += 1
        self.credit = min(self.credit + budget, budget + 8 * n * BLOCK_BYTES_PER_POINT)
        f = self.frame
        t = self.t
        V = t.n_nodes
        cbrt_n = float(np.cbrt(np.float64(n)))
        desc = np.array([cut.descends(t, v, cam, float(tau_px), cbrt_n) for v in range(V)], dtype=bool)
        _, visited = self._visit(desc)
        for v in visited:
            self.used[v] = f
            if desc[v]:
                self.wanted[v] = f
        groups = []
        for v in visited:
            ch = self.children[v]
            if desc[v] and ch and not all(self.resident[c] for c in ch):
                groups.append(v)

        def priority(v):
            (cx, cy, cz), d = lod.node_origin(t, v)
            side = 2.0 ** -d
            if cam.projection == 0:
                return (1, float(cam.W) * side / cbrt_n, -v)
            ox, oy, oz = cx * side, cy * side, cz * side
            p = [float(np.float32(a)) for a in cam.pos]
            inside = (ox <= p[0] <= ox + side) and (oy <= p[1] <= oy + side) and (oz <= p[2] <= oz + side)
            if inside:
                return (2, 0.0, -v)
            h = side * 0.5
            dx = (ox + h) - p[0]; dy = (oy + h) - p[1]; dz = (oz + h) - p[2]
            dist = float(np.sqrt((dx * dx + dy * dy) + dz * dz))
            return (1, float(np.float32(cam.F)) * side / (cbrt_n * dist), -v)
        groups.sort(key=priority, reverse=True)
        left = self.credit
        loaded, evicted = [], []
        for g in groups:
            need = [c for c in self.children[g] if not self.resident[c]]
            cost = BLOCK_BYTES_PER_POINT * sum(int(t.pt_count[c]) for c in need)
            if cost > left:
                break
            while self.free < len(need):
                vic = self._victim(f)
                if vic is None:
                    break
                self.resident[vic] = False
                self.free += 1
                evicted.append(vic)
            if self.free < len(need):
                break
            for c in need:
                self.resident[c] = True
                self.free -= 1
                loaded.append(c)
            left -= cost
        draw, _ = self._visit(desc)
        spent = self.credit - left
        self.credit = left
        return draw, loaded, evicted, spent

    def _victim(self, f):
        best = None
        for v in range(self.t.n_nodes):
            if not self.resident[v] or int(self.t.parent[v]) == NONE32:
                continue
            if self.used[v] >= f or self.wanted[int(self.t.parent[v])] >= f:
                continue
            if any(self.resident[c] for c in self.children[v]):
                continue
            key = (self.used[v], -v)
            if best is None or key < best[0]:
                best = (key, v)
        return None if best is None else best[1]

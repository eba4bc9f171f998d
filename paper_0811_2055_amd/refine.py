"""Gradient refinement of one octree node's stored points.

The paper asks that the reduced data be visually indistinguishable from the
full data.  The subselection alone only matches it in expectation; this loop
adjusts the float32 weights and positions of a node's n stored points so
that their splat matches the splat of every particle inside the node's cube,
over several views.

Loss: mean over training views and pixels of
    (log1p(I_lod / mean(I_full)) - log1p(I_full / mean(I_full)))^2.
Parameters: log-masses (Adam, lr 1e-2) and positions (Adam, lr 1e-3 x cube
side).  After every step the positions are clamped to the node's cube and the
masses rescaled so that they sum to the node mass.  Views: perspective, 60
degree field of view, camera on a seeded random direction around the node
centre at a distance where the node's projected point spacing lies in
[0.5, 1] pixel (where the view-dependent cut would draw this node).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import lib
from .autograd import splat_render


def node_views(centre, side: float, n: int, count: int, seed: int, W: int = 1024, H: int = 1024,
               fov_deg: float = 60.0):
    rng = np.random.default_rng(seed)
    F = (W / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    cams = []
    for _ in range(count):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        spacing = rng.uniform(0.5, 1.0)
        dist = F * side / (n ** (1.0 / 3.0) * spacing)
        pos = tuple(float(c + dist * e) for c, e in zip(centre, d))
        up = (0.0, 1.0, 0.0) if abs(d[1]) < 0.9 else (1.0, 0.0, 0.0)
        cams.append(lib.Camera.look_at(pos, tuple(centre), W, H, fov_deg, up_hint=up, near=1e-4))
    return cams


def log_image(img, mean):
    return torch.log1p(img / mean)


def e_log(lod_img, full_img):
    mean = full_img.mean()
    a, b = log_image(lod_img, mean), log_image(full_img, mean)
    return float(torch.sqrt(torch.mean((a - b) ** 2)))


@dataclass
class RefineResult:
    e_log_before: float
    e_log_after: float
    loss_first: float
    loss_last: float
    steps: int
    seconds: float


class NodeRefiner:
    """Adam over (log m, x, y, z) of one node's points against the renders of
    its full particle set.  One `step()` is: zero the gradients, render the
    points in every training view, loss and backward (the hand-written
    adjoint), Adam, then clamp the positions to the node's cube and shift the
    log-masses so that the masses sum to the node mass."""

    def __init__(self, px, py, pz, pm, full, lo, side: float, node_mass: float, train_cams,
                 lr_mass: float = 1e-2, lr_pos_frac: float = 1e-3, sigma: float = 1.0):
        dev = px.device
        self.sigma = sigma
        self.cams = list(train_cams)
        full_train = [lib.splat(*full, c, sigma) for c in self.cams]
        self.means = [f.mean() for f in full_train]
        self.targets = [log_image(f, mu) for f, mu in zip(full_train, self.means)]
        self.theta = torch.log(pm.clamp_min(1e-30)).clone().requires_grad_(True)
        self.xs = [a.clone().requires_grad_(True) for a in (px, py, pz)]
        self.lr_mass, self.lr_pos = lr_mass, lr_pos_frac * side
        self.opt = torch.optim.Adam([{"params": [self.theta], "lr": self.lr_mass},
                                     {"params": self.xs, "lr": self.lr_pos}])
        self.lo_t = [torch.tensor(float(v), device=dev) for v in lo]
        self.hi_t = [torch.tensor(float(v) + side, device=dev) for v in lo]
        self.logM = math.log(node_mass) if node_mass > 0 else 0.0

    def loss(self):
        m = torch.exp(self.theta)
        loss = 0.0
        for cam, tgt, mu in zip(self.cams, self.targets, self.means):
            img = splat_render(self.xs[0], self.xs[1], self.xs[2], m, cam, self.sigma)
            loss = loss + torch.mean((log_image(img, mu) - tgt) ** 2)
        return loss / len(self.cams)

    def step(self) -> float:
        self.opt.zero_grad(set_to_none=True)
        loss = self.loss()
        loss.backward()
        self.opt.step()
        with torch.no_grad():
            for a, l, h in zip(self.xs, self.lo_t, self.hi_t):
                a.clamp_(l, h)
            self.theta -= torch.logsumexp(self.theta, 0) - self.logM
        return float(loss.detach())

    def params(self):
        """(theta, x, y, z, masses) detached."""
        x, y, z = (a.detach() for a in self.xs)
        return self.theta.detach(), x, y, z, torch.exp(self.theta).detach()

    def grads(self):
        """Gradients of the last step: (dL/dtheta, dL/dx, dL/dy, dL/dz)."""
        return (self.theta.grad,) + tuple(a.grad for a in self.xs)

    def adam_state(self, t):
        """(exp_avg, exp_avg_sq, step) of parameter tensor t (zeros before the first step)."""
        st = self.opt.state.get(t, {})
        if not st:
            z = torch.zeros_like(t)
            return z, z, 0
        return st["exp_avg"], st["exp_avg_sq"], int(st["step"])

    # -- checkpoints ----------------------------------------------------------
    # The parameters (theta, x, y, z), each one's Adam moments and step count,
    # as numpy arrays; a refiner built on the same node and views continues
    # from them bit for bit.  Stored with numpy.savez (no pickled objects).
    CHECKPOINT_FORMAT = "lodrefine-npz-1"
    _NAMES = ("theta", "x", "y", "z")

    def state(self) -> dict:
        out = {"format": np.array(self.CHECKPOINT_FORMAT)}
        for name, t in zip(self._NAMES, [self.theta] + self.xs):
            ea, es, k = self.adam_state(t)
            out[name] = t.detach().cpu().numpy()
            out[name + "_exp_avg"] = ea.detach().cpu().numpy()
            out[name + "_exp_avg_sq"] = es.detach().cpu().numpy()
            out[name + "_step"] = np.array(k, dtype=np.int64)
        return out

    def load_state(self, st: dict):
        if str(st.get("format", "")) != self.CHECKPOINT_FORMAT:
            raise ValueError("not a node-refinement checkpoint")
        tensors = [self.theta] + self.xs
        for name, t in zip(self._NAMES, tensors):
            if tuple(st[name].shape) != tuple(t.shape):
                raise ValueError(f"checkpoint {name} has shape {st[name].shape}, the node {tuple(t.shape)}")
        with torch.no_grad():
            for name, t in zip(self._NAMES, tensors):
                t.copy_(torch.from_numpy(st[name]).to(t.device))
        sd = self.opt.state_dict()
        state = {}
        for i, (name, t) in enumerate(zip(self._NAMES, tensors)):
            k = int(st[name + "_step"])
            if k == 0:
                continue
            state[i] = {"step": torch.tensor(float(k), dtype=torch.float32),
                        "exp_avg": torch.from_numpy(st[name + "_exp_avg"]).to(t.device),
                        "exp_avg_sq": torch.from_numpy(st[name + "_exp_avg_sq"]).to(t.device)}
        self.opt.load_state_dict({"state": state, "param_groups": sd["param_groups"]})

    def save(self, path: str):
        np.savez(path, **self.state())

    def load(self, path: str):
        with np.load(path, allow_pickle=False) as f:
            self.load_state({k: f[k] for k in f.files})


def refine_node(px, py, pz, pm, full, lo, side: float, node_mass: float, train_cams, test_cams,
                steps: int = 200, lr_mass: float = 1e-2, lr_pos_frac: float = 1e-3, sigma: float = 1.0):
    """Refine one node's points (device float32 tensors) against its full particle set.

    full: (x, y, z, m) device tensors of every particle in the node's cube.
    lo: the cube's lower corner (3 floats); side: its edge length.
    """
    full_test = [lib.splat(*full, c, sigma) for c in test_cams]

    def evaluate(x, y, z, m):
        with torch.no_grad():
            errs = [e_log(lib.splat(x, y, z, m, c, sigma), f) for c, f in zip(test_cams, full_test)]
        return float(np.mean(errs))

    before = evaluate(px, py, pz, pm)
    r = NodeRefiner(px, py, pz, pm, full, lo, side, node_mass, train_cams, lr_mass, lr_pos_frac, sigma)
    first = last = None
    t0 = time.perf_counter()
    for _ in range(steps):
        v = r.step()
        first = v if first is None else first
        last = v
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    _, x, y, z, m = r.params()
    after = evaluate(x, y, z, m)
    return RefineResult(before, after, first, last, steps, secs), (x, y, z, m)


def exterior_views(side: float, n: int, count: int, seed: int, W: int = 1024, H: int = 1024, spacing: float = 0.75,
                   fov_deg: float = 60.0):
    """Cameras on seeded random directions around the box centre at the distance
    where a node of this side has the given projected point spacing, looking at
    the centre (the cut then draws nodes of that side there)."""
    rng = np.random.default_rng(seed)
    F = (W / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    dist = F * side / (n ** (1.0 / 3.0) * spacing)
    cams = []
    for _ in range(count):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        pos = tuple(float(0.5 + dist * e) for e in d)
        up = (0.0, 1.0, 0.0) if abs(d[1]) < 0.9 else (1.0, 0.0, 0.0)
        cams.append(lib.Camera.look_at(pos, (0.5, 0.5, 0.5), W, H, fov_deg, up_hint=up, near=1e-4))
    return cams


def main(argv=None):
    """Refine the depth-3 internal nodes of the NFW 16.7M-particle tree (n =
    16000, max depth 8) against their full particle sets, write the refined
    points back into the tree, and compare the plain and the refined tree's
    LOD renders with the full render in the same views; prints JSON lines."""
    import argparse
    import json
    import os
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--nodes", type=int, default=0, help="refine only the first K depth-3 nodes (0: all)")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--count", type=int, default=None, help="particles (default 16,777,216)")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    snap = synth.config2() if args.count is None else synth.nfw_mix(args.count, 2)
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(a).to(dev) for a in (snap.x, snap.y, snap.z, snap.m)]
    n = 16000
    # build throughput: one launch per node (plain) against one launch per level
    build_ms = {}
    for mode in (0, 1):
        bm = lib.Builder(snap.n, lib.BuildParams(n=n, max_depth=8, seed=0, mode=mode), dev)
        bm.build(*d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bm.build(*d)
        torch.cuda.synchronize()
        build_ms[mode] = (time.perf_counter() - t0) * 1e3
        del bm
    b = lib.Builder(snap.n, lib.BuildParams(n=n, max_depth=8, seed=0), dev)
    tree = b.build(*d)
    h = tree.host()
    order = b.view(1, torch.uint32).view(torch.int32).long()
    cand = [v for v in range(h["n_nodes"]) if h["depth"][v] == 3 and h["first_child"][v] != lib.NONE]
    if args.nodes:
        cand = cand[:args.nodes]
    # the plain tree's LOD renders against the full render, before any write-back
    side3 = 2.0 ** -3
    cams = exterior_views(side3, n, 8, seed=200, W=args.size, H=args.size)
    fulls = [lib.splat(*d, c) for c in cams]

    def lod_errors():
        errs = []
        for c, f in zip(cams, fulls):
            ids, nsel = lib.select_nodes(tree, c, 1.0, n)
            img = lib.splat_lod(tree, ids, nsel, snap.n, c)
            errs.append(e_log(img, f))
        return errs
    plain = lod_errors()
    print(json.dumps({"plain_tree_E_log": plain, "depth3_nodes": len(cand)}), flush=True)
    results = []
    t_all = time.perf_counter()
    for v in cand:
        cell = int(h["prefix"][v]) & ((1 << 9) - 1)
        cx = cy = cz = 0
        for k in range(3):
            cx |= ((cell >> (3 * k)) & 1) << k
            cy |= ((cell >> (3 * k + 1)) & 1) << k
            cz |= ((cell >> (3 * k + 2)) & 1) << k
        lo = [cx * side3, cy * side3, cz * side3]
        ids = torch.tensor([v], dtype=torch.int32, device=dev).view(torch.uint32)
        nid = torch.tensor([1], dtype=torch.int64, device=dev).view(torch.uint64)
        px, py, pz, pm, _ = lib.decode_nodes(tree, ids, nid, n)
        pb, pc = int(h["part_begin"][v]), int(h["part_count"][v])
        members = order[pb:pb + pc]
        full = [a[members].contiguous() for a in d]
        centre = [l + side3 / 2 for l in lo]
        train = node_views(centre, side3, n, args.views, seed=0, W=args.size, H=args.size)
        test = node_views(centre, side3, n, args.views, seed=100, W=args.size, H=args.size)
        res, (x, y, z, m) = refine_node(px, py, pz, pm, full, lo, side3, float(h["node_mass"][v]), train, test,
                                        steps=args.steps)
        lib.set_node_points(tree, v, x, y, z, m)
        rec = {"node": v, "particles": pc, "points": n, **res.__dict__}
        results.append(rec)
        print(json.dumps(rec), flush=True)
    secs_all = time.perf_counter() - t_all
    st = tree.host()["status"]
    refined = lod_errors()
    eb = float(np.mean([r["e_log_before"] for r in results])) if results else 0.0
    ea = float(np.mean([r["e_log_after"] for r in results])) if results else 0.0
    print(json.dumps({"summary": "depth-3 node refinement, NFW 16,777,216 particles, n=16000, D=8",
                      "nodes": len(results), "steps": args.steps, "views": args.views,
                      "image": f"{args.size}x{args.size}",
                      "E_log_heldout_node_views_before": eb, "E_log_heldout_node_views_after": ea,
                      "seconds_all_nodes": round(secs_all, 2),
                      "tree_views": "8 exterior perspective views, depth-3 spacing 0.75 px, cut tau 1 px",
                      "E_log_tree_views_plain": float(np.mean(plain)),
                      "E_log_tree_views_refined": float(np.mean(refined)),
                      "E_log_tree_views_plain_each": [round(e, 5) for e in plain],
                      "E_log_tree_views_refined_each": [round(e, 5) for e in refined],
                      "build_ms_per_node_schedule": round(build_ms[0], 2),
                      "build_ms_per_level_schedule": round(build_ms[1], 2),
                      "status_after_write_back": int(st)}), flush=True)


if __name__ == "__main__":
    main()

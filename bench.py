"""Benchmark: one step = LOD build of a particle snapshot + view-dependent cut
+ additive splat of the cut, all on one MI355X.

Default workload: 150,000,000 Soneira-Peebles particles (8 levels, eta 4,
lambda 1.9, seed 3), n = 16000, max depth 8, alpha = +1, orthographic
1024x1024 Gaussian splat (sigma 1 px, truncated at 3 sigma), cut at 1 px
point spacing.  Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line (rank 0) with throughput, the roofline of the
dominant kernel (HIP-event timed inside the run), the CPU oracle timed on a
bounded sample, and the LOD-vs-full image error.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "LOD build Mparticles/s + %HBM roofline; splat Mpts/s; LOD-vs-full image err"

# Algorithmic bytes per unit for each kernel (unit: particle for the build
# kernels, point for the splat binning, (point, tile) pair for accumulation).
KERNEL_BYTES = {
    "k_keygen": 12.0,            # read x,y,z (12); histogram only (masses checked in the first scatter)
    "k_scatter<true>": 36.0,     # read x,y,z,m (16) write key,id,fraction,mass (20)
    "k_scatter<false>": 40.0,    # read 20 write 20
    "k_upsweep": 4.0,            # read key
    "k_density": 14.0,           # read key, id (8) write w (4), kbin (2)
}


def selection_bytes(h, n):
    """Algorithmic bytes of one build's per-level selection launches, which
    also copy the leaves' particles to their stored points.

    Per selecting node: every candidate read once (6 B per entry of a
    selecting child's list: position and key bin; 2 B key bin per particle of
    a leaf child or of the node's own range), its n stored points gathered
    (id 4, codes 6, w 4, m 4) and written (14 B), its list of n+1 entries
    written (6 B each).  Per
    particle of a leaf holding at most n: 20 B read (key, id, fraction, mass)
    and 14 B written.
    """
    import numpy as np
    NONE = 0xFFFFFFFF
    cnt = h["part_count"].astype(np.int64)
    fc = h["first_child"].astype(np.int64)
    par = h["parent"].astype(np.int64)
    sel = cnt > n
    has_parent = par != NONE
    child_of_sel = np.zeros(cnt.size, dtype=bool)
    child_of_sel[has_parent] = sel[par[has_parent]]
    lists = int(np.count_nonzero(child_of_sel & sel))
    ranges = int(cnt[child_of_sel & ~sel].sum()) + int(cnt[sel & (fc == NONE)].sum())
    n_sel = int(np.count_nonzero(sel))
    leaf_particles = int(cnt[(fc == NONE) & ~sel].sum())
    return (6.0 * (n + 1) * lists + 2.0 * ranges + (18.0 + 14.0) * n * n_sel + 6.0 * (n + 1) * n_sel
            + 34.0 * leaf_particles)


KERNEL_SOURCES = ["paper_0811_2055_amd/csrc/lod_build.hip", "paper_0811_2055_amd/csrc/lod_splat.hip",
                  "paper_0811_2055_amd/csrc/lod_device.hpp", "paper_0811_2055_amd/csrc/lod_scan.hpp"]
TRAFFIC_TABLE = "profiles/hbm_traffic_sp150m_step.txt"


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed PMC table, or None when
    the table was measured on different kernel sources (or has no such kernel)."""
    import hashlib
    try:
        h = hashlib.sha1(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in KERNEL_SOURCES)).hexdigest()
        lines = open(os.path.join(ROOT, TRAFFIC_TABLE)).read().splitlines()
    except OSError:
        return None
    stamp = [l.split(":", 1)[1].strip() for l in lines if l.startswith("# kernel-source-sha1:")]
    if not stamp or stamp[0] != h:
        return None
    for l in lines:
        parts = l.split()
        if parts and parts[0] == kernel and len(parts) == 5:
            return float(parts[4]) * 1e9
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name: str, count: int | None):
    import synth
    if name == "c3":
        N = count or 150_000_000
        return synth.config3(N), dict(n=16000, D=8, W=1024, H=1024, label=(
            f"Soneira-Peebles {N} particles (8 levels, eta 4, lambda 1.9, seed 3), n=16000, D=8, "
            f"alpha=+1, ortho 1024x1024 splat sigma 1px, cut tau 1px"))
    if name == "c2":
        s = synth.config2()
        return s, dict(n=16000, D=8, W=1024, H=1024, label=(
            "NFW 16,777,216 particles (500 haloes + 20% uniform, seed 2), n=16000, D=8, alpha=+1, "
            "ortho 1024x1024 splat sigma 1px, cut tau 1px"))
    if name == "c1":
        s = synth.config1()
        return s, dict(n=4096, D=4, W=256, H=256, label=(
            "Plummer mix 262,144 particles (seed 0), n=4096, D=4, alpha=+1, ortho 256x256 splat, cut tau 1px"))
    raise SystemExit(f"unknown workload {name}")


def image_errors(lod_img, full_img):
    """E_log, E_tone, E_L1 between a LOD render and the full render (torch, on the GPU)."""
    import torch
    lod = lod_img.double(); full = full_img.double()
    mean = full.mean()
    if float(mean) <= 0:
        return dict(E_log=0.0, E_tone=0.0, E_L1=0.0)
    a = torch.log1p(lod / mean); b = torch.log1p(full / mean)
    e_log = float(torch.sqrt(torch.mean((a - b) ** 2)))
    top = torch.log1p(full.max() / mean)
    ta = torch.floor(255.0 * a / top); tb = torch.floor(255.0 * b / top)
    e_tone = float(((ta - tb).abs() > 1).double().mean())
    e_l1 = float((lod - full).abs().sum() / full.sum())
    return dict(E_log=e_log, E_tone=e_tone, E_L1=e_l1)


def cpu_baseline(snap, cfg, sample: int):
    """Time the CPU oracle (build + cut + LOD render) on the first `sample` particles."""
    from oracle import cut as ocut
    from oracle import lod as olod
    from oracle import splat as osplat
    sub = snap.subset(min(sample, snap.n))
    t0 = time.perf_counter()
    tr = olod.lod_build(sub.x, sub.y, sub.z, sub.m, n=cfg["n"], D=cfg["D"], alpha=1, seed=0)
    cam = osplat.Camera(0, cfg["W"], cfg["H"])
    c = ocut.select(tr, cam, 1.0, cfg["n"])
    px, py, pz, pm = olod.decoded_points(tr, c)
    osplat.render(cam, px, py, pz, pm)
    dt = time.perf_counter() - t0
    return {"value": sub.n / dt / 1e6, "unit": "Mparticles/s", "cores": 1, "kind": "oracle",
            "sample": (f"first {sub.n:,} particles of the same (shuffled) snapshot, same n and D; "
                       f"numpy oracle build + cut + LOD render, single thread, {dt:.1f} s")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--count", type=int, default=None, help="override the particle count (c3)")
    ap.add_argument("--cpu-sample", type=int, default=5_000_000)
    ap.add_argument("--mode", type=int, default=1, choices=[0, 1, 2],
                    help="selection schedule: 0 per-node launches, 1 per-level launches, 2 one persistent launch")
    ap.add_argument("--select-threads", type=int, default=512, help="threads per node block in the selection")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default selection schedule")
    ap.add_argument("--compare-modes", action="store_true",
                    help="also time one build in each selection schedule")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-render", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter calibration)")
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="only run this many plain steps (for profilers) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        sys.exit("bench.py runs on exactly one GPU: this build has no multi-GPU path "
                 "(the sharding design is described in DESIGN.md); use --gpus 1")

    import numpy as np
    import torch
    from paper_0811_2055_amd import lib

    torch.cuda.init()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    snap, cfg = workload(args.workload, args.count)
    log(f"[bench] workload generated: {snap.n} particles in {time.perf_counter() - t0:.1f} s")
    x, y, z, m = (torch.from_numpy(a).to(dev) for a in (snap.x, snap.y, snap.z, snap.m))
    N = snap.n
    params = lib.BuildParams(n=cfg["n"], max_depth=cfg["D"], alpha=1, seed=0, mode=args.mode,
                             select_threads=args.select_threads)
    builder = lib.Builder(N, params, dev)
    cam = lib.Camera.ortho(cfg["W"], cfg["H"])
    tree = builder.tree
    sel_ws_bytes = lib.C.c_size_t()
    lib.load().lod_select_plan(tree.node_capacity, lib.C.byref(sel_ws_bytes))
    sel_ws = torch.empty(max(sel_ws_bytes.value, 256), dtype=torch.uint8, device=dev)
    max_draw = N          # a cut never draws more points than particles
    lod_ws = torch.empty(lib.splat_lod_workspace_bytes(tree.node_capacity, max_draw, cam), dtype=torch.uint8,
                         device=dev)
    lod_img = torch.empty((cfg["H"], cfg["W"]), dtype=torch.float32, device=dev)
    log(f"[bench] workspace {builder.ws_bytes / 1e9:.2f} GB, tree caps {tree.node_capacity} nodes "
        f"{tree.point_capacity} points, splat ws {lod_ws.numel() / 1e9:.2f} GB")

    def step():
        builder.build(x, y, z, m)
        ids, nsel = lib.select_nodes(tree, cam, 1.0, cfg["n"], workspace=sel_ws)
        lib.splat_lod(tree, ids, nsel, max_draw, cam, workspace=lod_ws, out=lod_img)
        return ids, nsel

    if args.profile_steps is not None:
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        if args.copy_calibration:
            a = torch.empty(256 << 20, dtype=torch.float32, device=dev).fill_(1.0)
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            log(f"[bench] copy calibration: {a.numel() * 4} bytes read and written")
        log("[bench] profile steps done")
        return

    tuned = None
    if not args.no_autotune:
        from paper_0811_2055_amd import autotune
        rec = autotune.tune(builder, x, y, z, m, path=os.path.join(ROOT, "gpurun_out", "lod_tune.json"))
        tuned = {k: rec[k] for k in ("mode", "select_threads", "persistent_blocks", "ms")}
        log(f"[bench] autotuned schedule: {tuned}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h = tree.host()
    if h["status"]:
        raise SystemExit(f"build status word {h['status']}")
    log(f"[bench] warmup done: {h['n_nodes']} nodes, {h['n_points']} stored points")

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    log(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step")

    # per-kernel timing over a second timed region with every launch bracketed by events
    with lib.trace() as tr:
        for _ in range(args.steps):
            step()
    summ = tr.summary()
    per_step = {k: (c / args.steps, t / args.steps) for k, (c, t) in summ.items()}
    build_kernels = set()
    with lib.trace() as tb:
        builder.build(x, y, z, m)
    for name, _ in tb.records:
        build_kernels.add(name)
    # build wall time on the stream (the density kernel overlaps the tree
    # construction on a second stream, so kernel times do not add up to it)
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    b0.record(stream)
    for _ in range(args.steps):
        builder.build(x, y, z, m)
    b1.record(stream)
    torch.cuda.synchronize()
    build_ms = b0.elapsed_time(b1) / args.steps
    dom = max(per_step.items(), key=lambda kv: kv[1][1])
    dom_name, (dom_launches, dom_ms_step) = dom
    dom_avg = summ[dom_name][1] / summ[dom_name][0]
    per_unit = KERNEL_BYTES.get(dom_name)
    if dom_name == "k_select_level" and builder.params.mode == 1:
        # one launch per level: the per-launch figure is the build's total over its launches
        launch_bytes = selection_bytes(h, cfg["n"]) / dom_launches
        per_unit = launch_bytes / N
    if per_unit is not None:
        achieved = per_unit * N / (dom_avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom_name), "kernel": dom_name,
                "bytes_per_particle": round(per_unit, 3), "launches_per_step": dom_launches,
                "avg_launch_ms": round(dom_avg, 4)}
    else:
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": dom_name, "avg_launch_ms": round(dom_avg, 4)}
    # a plain device copy of 2 x 1 GiB, for the achievable-bandwidth context
    ca = torch.empty(256 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        cb.copy_(ca)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * ca.numel() * 4 * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del ca, cb
    roof["copy_measured_GBs"] = round(copy_gbs, 1)
    if roof.get("achieved") is not None:
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    S = h["n_points"]
    b_alg = 48.0 * N + 14.0 * S
    build_frac = b_alg / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS

    ids, nsel = lib.select_nodes(tree, cam, 1.0, cfg["n"], workspace=sel_ws)
    k = int(lib._to_numpy(nsel)[0])
    cut_nodes = lib._to_numpy(ids[:k]).astype(np.int64)
    drawn = int(h["pt_count"][cut_nodes].astype(np.int64).sum())

    extra = {}
    if not args.no_full_render:
        full_ws = torch.empty(lib.splat_workspace_bytes(N, cam), dtype=torch.uint8, device=dev)
        full = lib.splat(x, y, z, m, cam, workspace=full_ws)
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        reps = 3
        for _ in range(reps):
            lib.splat(x, y, z, m, cam, workspace=full_ws, out=full)
        f1.record(stream)
        torch.cuda.synchronize()
        full_ms = f0.elapsed_time(f1) / reps
        extra["splat_full_ms"] = round(full_ms, 3)
        extra["splat_full_Mpts_s"] = round(N / full_ms / 1e3, 1)
        step()
        torch.cuda.synchronize()
        extra.update({k: float(f"{v:.4g}") for k, v in image_errors(lod_img, full).items()})
        del full_ws

    if args.compare_modes:
        by_mode = {}
        for md in (0, 1, 2):
            bm = lib.Builder(N, lib.BuildParams(n=cfg["n"], max_depth=cfg["D"], alpha=1, seed=0, mode=md), dev)
            bm.build(x, y, z, m)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bm.build(x, y, z, m)
            torch.cuda.synchronize()
            by_mode[str(md)] = round((time.perf_counter() - t0) * 1e3, 3)
            if md == 1:
                with lib.trace() as tl:
                    bm.build(x, y, z, m)
                extra["select_ms_by_level_per_level_schedule"] = [
                    round(ms, 4) for name, ms in tl.records if name in ("k_select_level", "k_sel_output")]
            hm = bm.tree.host()
            for key in ("pt_id", "qx", "qy", "qz", "pt_mass", "prefix", "part_count"):
                if not np.array_equal(hm[key], h[key]):
                    raise SystemExit(f"schedule {md} differs from the timed schedule in {key}")
            del bm
            torch.cuda.empty_cache()
        extra["build_ms_by_schedule"] = by_mode
        log(f"[bench] build ms by schedule: {by_mode}")

    splat_ms = sum(t for k, (c, t) in per_step.items() if k not in build_kernels)
    out = {
        "metric": METRIC,
        "value": round(N / ms_step / 1e3, 2),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 keys, f64 masses, f32 splat",
        "data": "synthetic",
        "config": {"workload": cfg["label"], "particles": N, "n": cfg["n"], "max_depth": cfg["D"],
                   "image": f"{cfg['W']}x{cfg['H']}", "parallelism": "single GPU"},
        "roofline": roof,
        "schedule": tuned or {"mode": builder.params.mode, "select_threads": builder.params.select_threads,
                              "persistent_blocks": builder.params.persistent_blocks},
        "build_ms": round(build_ms, 4),
        "build_Mparticles_s": round(N / build_ms / 1e3, 1),
        "build_B_alg_GB": round(b_alg / 1e9, 3),
        "build_frac_hbm_B_alg": round(build_frac, 4),
        "stored_points": S,
        "nodes": h["n_nodes"],
        "lod_points_drawn": drawn,
        "splat_lod_ms": round(splat_ms, 4),
        "splat_lod_Mpts_s": round(drawn / max(splat_ms, 1e-9) / 1e3, 1),
        "kernels_ms_per_step": {k: round(t, 4) for k, (c, t) in sorted(per_step.items(), key=lambda kv: -kv[1][1])},
        "select_ms_by_level": [round(ms, 4) for name, ms in tb.records if name.startswith("k_select")],
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(snap, cfg, args.cpu_sample)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

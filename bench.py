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
    "k_scatter<true>": 34.0,     # read x,y,z,m (16) write key,id,fractions,mass (18)
    "k_scatter<false>": 36.0,    # read 18 write 18
    "k_upsweep": 4.0,            # read key
    "k_density": 14.0,           # read key, id (8) write w (4), kbin (2)
}


def selection_bytes(N, S):
    """The per-level selection launches' share of the build's compulsory bytes
    B_alg = 48 N + 14 S: the positions read again in Morton order for the
    node-relative quantisation (12 B per particle; the masses' 4 B are the
    leaf-mass pass's share) and every stored point written once (14 B:
    id 4, three 16-bit codes 6, mass 4).  Candidate re-reads, list traffic and
    gathers are the design's own and are not counted."""
    return 12.0 * N + 14.0 * S


KERNEL_SOURCES = ["paper_0811_2055_amd/csrc/lod_build.hip", "paper_0811_2055_amd/csrc/lod_splat.hip",
                  "paper_0811_2055_amd/csrc/lod_device.hpp", "paper_0811_2055_amd/csrc/lod_scan.hpp",
                  "paper_0811_2055_amd/csrc/lod_internal.hpp"]
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
            f"ortho 1024x1024 splat sigma 1px, cut tau 1px"))
    if name == "c2":
        s = synth.config2()
        return s, dict(n=16000, D=8, W=1024, H=1024, label=(
            "NFW 16,777,216 particles (500 haloes + 20% uniform, seed 2), n=16000, D=8, "
            "perspective 1024x1024 splat (FOV 60 deg, exterior camera) sigma 1px, cut tau 1px"))
    if name == "c1":
        s = synth.config1()
        return s, dict(n=4096, D=4, W=256, H=256, label=(
            "Plummer mix 262,144 particles (seed 0), n=4096, D=4, ortho 256x256 splat, cut tau 1px"))
    raise SystemExit(f"unknown workload {name}")


def views(name: str, cfg):
    """(label, camera) pairs: orthographic for c1 and c3; for c2 one exterior
    camera at (0.5, 0.5, -0.9) looking at the box centre and three seeded
    interior cameras (positions uniform in [0.2, 0.8]^3, looking at a seeded
    point), FOV 60 degrees."""
    import numpy as np
    from paper_0811_2055_amd import lib
    W, H = cfg["W"], cfg["H"]
    if name != "c2":
        return [("ortho", lib.Camera.ortho(W, H))]
    out = [("exterior", lib.Camera.look_at((0.5, 0.5, -0.9), (0.5, 0.5, 0.5), W, H, 60.0))]
    rng = np.random.default_rng(18)
    for i in range(3):
        pos = tuple(float(a) for a in rng.uniform(0.2, 0.8, 3))
        tgt = tuple(float(a) for a in rng.uniform(0.0, 1.0, 3))
        out.append((f"interior{i}", lib.Camera.look_at(pos, tgt, W, H, 60.0, near=1e-4)))
    return out


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


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def cpu_baseline(snap, cfg, sample: int, alpha: int, repeats: int):
    """Time the CPU oracle (build + cut + LOD render, numpy, one thread) on the
    first `sample` particles; median of `repeats` runs."""
    import statistics
    from threadpoolctl import threadpool_limits
    sub = snap.subset(min(sample, snap.n))
    # numpy's thread pools held to one thread: the oracle runs on one core
    with threadpool_limits(limits=1):
        times = _time_oracle(sub, cfg, alpha, repeats)
    dt = statistics.median(times)
    model, avail = host_cpu()
    whole = "all" if sub.n == snap.n else f"the first {sub.n:,} of {snap.n:,}"
    return {"value": sub.n / dt / 1e6, "unit": "Mparticles/s", "cores": 1, "kind": "oracle",
            "sample": (f"{whole} particles of the same (shuffled) snapshot, same n and D; numpy oracle build + "
                       f"cut + orthographic LOD render, single thread, median of {repeats}: {dt:.1f} s"),
            "cpu_model": model, "host_cpus_available": avail}


def _time_oracle(sub, cfg, alpha, repeats):
    from oracle import cut as ocut
    from oracle import lod as olod
    from oracle import splat as osplat
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        tr = olod.lod_build(sub.x, sub.y, sub.z, sub.m, n=cfg["n"], D=cfg["D"], alpha=alpha, seed=0)
        cam = osplat.Camera(0, cfg["W"], cfg["H"])
        c = ocut.select(tr, cam, 1.0, cfg["n"])
        px, py, pz, pm = olod.decoded_points(tr, c)
        osplat.render(cam, px, py, pz, pm)
        times.append(time.perf_counter() - t0)
    return times


def lod_sweep(tree, full_imgs, cams, taus, n, max_draw, sel_ws, lod_ws, N):
    """For every view and tau: the cut's points drawn and the LOD-vs-full errors."""
    import numpy as np
    import torch
    from paper_0811_2055_amd import lib
    rows = []
    pt_count = lib._to_numpy(tree.arrays["pt_count"]).astype(np.int64)
    for (label, cam), full in zip(cams, full_imgs):
        img = torch.empty((cam.H, cam.W), dtype=torch.float32, device=full.device)
        for tau in taus:
            ids, nsel = lib.select_nodes(tree, cam, tau, n, workspace=sel_ws)
            k = int(lib._to_numpy(nsel)[0])
            cut = lib._to_numpy(ids[:k]).astype(np.int64)
            lib.splat_lod(tree, ids, nsel, max_draw, cam, workspace=lod_ws, out=img)
            torch.cuda.synchronize()
            e = image_errors(img, full)
            rows.append({"view": label, "tau_px": tau, "nodes": k, "points_drawn": int(pt_count[cut].sum()),
                         "drawn_frac": round(int(pt_count[cut].sum()) / N, 4),
                         **{kk: float(f"{v:.4g}") for kk, v in e.items()}})
    return rows


def stream_leg(tree, N, cfg, dev, frames: int, fps: float, link_mb_s: float, slots: int):
    """View-dependent streaming of the built tree from a block store file: a
    camera flies from outside the box towards its densest depth-3 cell while
    the link carries link_mb_s MB/s at fps frames per second.  Per frame: the
    bytes loaded and the nodes drawn; every few frames the streamed render's
    E_log against the fully resident LOD render and against the full render."""
    import tempfile
    import numpy as np
    import torch
    from paper_0811_2055_amd import lib
    h = tree.host()
    path = os.path.join(tempfile.gettempdir(), f"lod_bench_{os.getpid()}.lodstore")
    t0 = time.perf_counter()
    lib.store_save(tree, cfg["n"], path)
    save_s = time.perf_counter() - t0
    file_mb = os.path.getsize(path) / 1e6
    budget = int(link_mb_s * 1e6 / fps)
    st = lib.Streamer(path, slots, dev)
    dense = np.nonzero(h["depth"] == 3)[0]
    target_v = int(dense[np.argmax(h["part_count"][dense])])
    cell = int(h["prefix"][target_v]) & 511
    c = [0, 0, 0]
    for k in range(3):
        for ax in range(3):
            c[ax] |= ((cell >> (3 * k + ax)) & 1) << k
    target = tuple((ci + 0.5) / 8 for ci in c)
    start = (0.5, 0.5, -1.5)
    W, H = cfg["W"], cfg["H"]
    full_ws = torch.empty(lib.splat_workspace_bytes(N, lib.Camera.ortho(W, H)), dtype=torch.uint8, device=dev)
    rows = []
    loaded_total = 0
    for f in range(frames):
        a = f / max(frames - 1, 1)
        pos = tuple(s0 + a * (t - s0) * 0.9 for s0, t in zip(start, target))
        cam = lib.Camera.look_at(pos, target, W, H, 60.0, near=1e-4)
        ids, nd, stats = st.frame(cam, 1.0, budget)
        loaded_total += stats["bytes_loaded"]
        row = {"frame": f, "MB": round(stats["bytes_loaded"] / 1e6, 3), "drawn": stats["nodes_drawn"],
               "waiting": stats["groups_waiting"], "resident": stats["resident_nodes"],
               "decide_ms": round(stats["decide_ms"], 3), "io_ms": round(stats["io_ms"], 3)}
        if f % 10 == 9 or f == frames - 1:
            img = lib.splat_lod(st.view, ids, nd, slots * cfg["n"], cam)
            rids, rn = lib.select_nodes(tree, cam, 1.0, cfg["n"])
            lod = lib.splat_lod(tree, rids, rn, N, cam)
            full = lib.splat(*tree._src, cam, workspace=full_ws)
            row["E_log_vs_resident_lod"] = round(image_errors(img, lod)["E_log"], 5)
            row["E_log_vs_full"] = round(image_errors(img, full)["E_log"], 5)
            row["E_log_resident_lod_vs_full"] = round(image_errors(lod, full)["E_log"], 5)
        rows.append(row)
        log(f"[bench] stream frame {f}: {row}")
    st.close()
    os.remove(path)
    return {"store_MB": round(file_mb, 1), "store_save_s": round(save_s, 2), "link_MB_s": link_mb_s, "fps": fps,
            "budget_MB_per_frame": round(budget / 1e6, 3), "pool_slots": slots, "frames": frames,
            "MB_loaded_total": round(loaded_total / 1e6, 2),
            "MB_per_frame_max": max(r["MB"] for r in rows),
            "decide_ms_mean": round(float(np.mean([r["decide_ms"] for r in rows])), 3),
            "io_ms_mean": round(float(np.mean([r["io_ms"] for r in rows])), 3),
            "checkpoints": [r for r in rows if "E_log_vs_resident_lod" in r]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--count", type=int, default=None, help="override the particle count (c3)")
    ap.add_argument("--alpha", type=int, default=1, choices=[-1, 0, 1], help="density exponent")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="particles the CPU oracle is timed on (default: all of c1 and c2, 5M of c3)")
    ap.add_argument("--mode", type=int, default=1, choices=[0, 1, 2],
                    help="selection schedule: 0 per-node launches, 1 per-level launches, 2 one persistent launch")
    ap.add_argument("--select-threads", type=int, default=512, help="threads per node block in the selection")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default selection schedule")
    ap.add_argument("--no-compare-modes", action="store_true",
                    help="skip timing one build in each selection schedule")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-render", action="store_true")
    ap.add_argument("--taus", default="1,2,4,8", help="cut thresholds (px) of the LOD-vs-full sweep")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter calibration)")
    ap.add_argument("--stream", action="store_true",
                    help="also stream the built tree from a block store file along a camera path")
    ap.add_argument("--stream-frames", type=int, default=60)
    ap.add_argument("--stream-slots", type=int, default=3000)
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="only run this many plain steps (for profilers) and exit")
    ap.add_argument("--pipelined", action="store_true",
                    help="also time steps alternating over two independent step pipelines on two streams")
    ap.add_argument("--profile-extras", action="store_true",
                    help="with --profile-steps: then build the highlight flags of a million ids once and draw "
                         "the highlighted and the cubic-blob LOD renders twice each")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        sys.exit("bench.py runs on exactly one GPU: this build has no multi-GPU path "
                 "(the sharding design is described in DESIGN.md); use --gpus 1")

    import statistics

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
    params = lib.BuildParams(n=cfg["n"], max_depth=cfg["D"], alpha=args.alpha, seed=0, mode=args.mode,
                             select_threads=args.select_threads)
    builder = lib.Builder(N, params, dev)
    cams = views(args.workload, cfg)
    cam = cams[0][1]
    tree = builder.tree
    sel_ws_bytes = lib.C.c_size_t()
    lib.load().lod_select_plan(tree.node_capacity, lib.C.byref(sel_ws_bytes))
    sel_ws = torch.empty(max(sel_ws_bytes.value, 256), dtype=torch.uint8, device=dev)
    max_draw = N          # a cut never draws more points than particles
    lod_ws = torch.empty(max(lib.splat_lod_workspace_bytes(tree.node_capacity, max_draw, c) for _, c in cams),
                         dtype=torch.uint8, device=dev)
    lod_img = torch.empty((cfg["H"], cfg["W"]), dtype=torch.float32, device=dev)
    log(f"[bench] workspace {builder.ws_bytes / 1e9:.2f} GB, tree caps {tree.node_capacity} nodes "
        f"{tree.point_capacity} points, splat ws {lod_ws.numel() / 1e9:.2f} GB")

    def step():
        builder.build(x, y, z, m)
        ids, nsel = lib.select_nodes(tree, cam, 1.0, cfg["n"], workspace=sel_ws)
        lib.splat_lod(tree, ids, nsel, max_draw, cam, workspace=lod_ws, out=lod_img)
        return ids, nsel

    def extras_setup():
        """The highlight (a million random ids) and cubic-blob inputs of the last step's cut."""
        ids1, nsel1 = lib.select_nodes(tree, cam, 1.0, cfg["n"], workspace=sel_ws)
        hl_ids = np.random.default_rng(7).choice(N, min(1_000_000, N), replace=False)
        bits = lib.highlight_bits(hl_ids, N, dev)
        flags = lib.highlight_flags(tree, bits, N)        # allocates once; later calls reuse the words
        hl_img = torch.empty_like(lod_img)
        hl_ws = torch.empty(lib.splat_lod_highlight_workspace_bytes(tree.node_capacity, max_draw, len(hl_ids), cam),
                            dtype=torch.uint8, device=dev)
        cub = lib.Blob.cubic(h_px=1.5)
        cub_ws = torch.empty(lib.splat_lod_workspace_bytes(tree.node_capacity, max_draw, cam, blob=cub),
                             dtype=torch.uint8, device=dev)

        def render_hl():
            lib.splat_lod_highlight(tree, ids1, nsel1, max_draw, cam, flags, len(hl_ids), workspace=hl_ws,
                                    out=lod_img, out_hl=hl_img)

        def render_cubic():
            lib.splat_lod(tree, ids1, nsel1, max_draw, cam, workspace=cub_ws, out=lod_img, blob=cub)

        return dict(ids=ids1, nsel=nsel1, hl_ids=hl_ids, bits=bits, flags=flags, hl_img=hl_img,
                    render_hl=render_hl, render_cubic=render_cubic)

    if args.profile_steps is not None:
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        if args.profile_extras:
            ex = extras_setup()
            for _ in range(2):
                ex["render_hl"]()
                ex["render_cubic"]()
            torch.cuda.synchronize()
            log("[bench] profile extras done")
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

    # the timed region: exactly K steps between two synchronisations, plus an
    # event pair around every step (all on the stream the library launches on)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    step_ms = [a.elapsed_time(b) for a, b in ev]
    log(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step (median {statistics.median(step_ms):.3f})")

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
    # build wall time on the stream, per build (the density kernel overlaps the
    # tree construction on a second stream, so kernel times do not add up to it)
    bev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(max(20, args.steps))]
    torch.cuda.synchronize()
    for a, b in bev:
        a.record(stream)
        builder.build(x, y, z, m)
        b.record(stream)
    torch.cuda.synchronize()
    build_runs = [a.elapsed_time(b) for a, b in bev]
    build_ms = statistics.median(build_runs)
    S = h["n_points"]
    dom = max(per_step.items(), key=lambda kv: kv[1][1])
    dom_name, (dom_launches, dom_ms_step) = dom
    dom_avg = summ[dom_name][1] / summ[dom_name][0]
    per_unit = KERNEL_BYTES.get(dom_name)
    if dom_name == "k_select_level" and builder.params.mode == 1:
        # one launch per level: the per-launch figure is the build's share over its launches
        per_unit = selection_bytes(N, S) / dom_launches / N
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
    b_alg = 48.0 * N + 14.0 * S
    build_frac = b_alg / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS

    ids, nsel = lib.select_nodes(tree, cam, 1.0, cfg["n"], workspace=sel_ws)
    k = int(lib._to_numpy(nsel)[0])
    cut_nodes = lib._to_numpy(ids[:k]).astype(np.int64)
    drawn = int(h["pt_count"][cut_nodes].astype(np.int64).sum())

    extra = {}
    if not args.no_full_render:
        full_ws = torch.empty(max(lib.splat_workspace_bytes(N, c) for _, c in cams), dtype=torch.uint8, device=dev)
        fulls = [lib.splat(x, y, z, m, c, workspace=full_ws) for _, c in cams]
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        reps = 3
        for _ in range(reps):
            lib.splat(x, y, z, m, cam, workspace=full_ws, out=fulls[0])
        f1.record(stream)
        torch.cuda.synchronize()
        full_ms = f0.elapsed_time(f1) / reps
        extra["splat_full_ms"] = round(full_ms, 3)
        extra["splat_full_Mpts_s"] = round(N / full_ms / 1e3, 1)
        del full_ws
        taus = [float(t) for t in args.taus.split(",")]
        sweep = lod_sweep(tree, fulls, cams, taus, cfg["n"], max_draw, sel_ws, lod_ws, N)
        first = next(r for r in sweep if r["view"] == cams[0][0] and r["tau_px"] == 1.0) \
            if 1.0 in taus else sweep[0]
        extra.update({kk: first[kk] for kk in ("E_log", "E_tone", "E_L1")})
        extra["lod_vs_full"] = sweep
        del fulls

    # ID highlighting (the paper claims no cost for testing each drawn point
    # against up to a million selected ids) and the radial cubic blob: the
    # timed step's LOD render, plain versus highlighted versus cubic
    def timed(fn, reps=5):
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return statistics.median(ts)
    ex = extras_setup()
    ids1, nsel1, hl_ids, hl_img = ex["ids"], ex["nsel"], ex["hl_ids"], ex["hl_img"]
    flags_ms = timed(lambda: lib.highlight_flags(tree, ex["bits"], N, out=ex["flags"]), reps=3)
    ex["render_hl"]()
    plain_ms = timed(lambda: lib.splat_lod(tree, ids1, nsel1, max_draw, cam, workspace=lod_ws, out=lod_img))
    hl_ms = timed(ex["render_hl"])
    extra["highlight"] = {"selected_ids": int(len(hl_ids)), "flags_ms_per_list": round(flags_ms, 4),
                          "lod_render_ms": round(plain_ms, 4),
                          "lod_render_highlight_ms": round(hl_ms, 4),
                          "penalty_frac": round(hl_ms / plain_ms - 1.0, 4),
                          "highlighted_mass_frac": round(float(hl_img.double().sum() / lod_img.double().sum()), 4)}
    cub_ms = timed(ex["render_cubic"])
    extra["cubic_blob"] = {"h_px": 1.5, "lod_render_ms": round(cub_ms, 4),
                           "Mpts_s": round(drawn / cub_ms / 1e3, 1)}
    del ex, hl_img
    log(f"[bench] highlight {extra['highlight']}, cubic {extra['cubic_blob']}")

    if not args.no_compare_modes:
        by_mode = {}
        for md in (0, 1, 2):
            bm = lib.Builder(N, lib.BuildParams(n=cfg["n"], max_depth=cfg["D"], alpha=args.alpha, seed=0,
                                                mode=md), dev)
            bm.build(x, y, z, m)
            torch.cuda.synchronize()
            runs = []
            for _ in range(1 if md == 0 else 5):
                t0 = time.perf_counter()
                bm.build(x, y, z, m)
                torch.cuda.synchronize()
                runs.append((time.perf_counter() - t0) * 1e3)
            by_mode[str(md)] = round(statistics.median(runs), 3)
            hm = bm.tree.host()
            for key in ("pt_id", "qx", "qy", "qz", "pt_mass", "prefix", "part_count"):
                if not np.array_equal(hm[key], h[key]):
                    raise SystemExit(f"schedule {md} differs from the timed schedule in {key}")
            del bm
            torch.cuda.empty_cache()
        extra["build_ms_by_schedule"] = by_mode
        extra["build_schedules"] = ("0: one selection launch per node (host-synchronised), 1: one launch per "
                                    "level, 2: one persistent launch; default grids, wall time with a "
                                    "synchronisation, median of 5 (mode 0: one run); outputs byte-identical")
        log(f"[bench] build ms by schedule: {by_mode}")

    if args.pipelined:
        # Two independent step pipelines (own tree, workspaces and image; two
        # streams of default priority), steps alternating between them: the
        # latency-bound top of one build's selection overlaps the other's work.
        # Each step is still a whole build + cut + LOD render of the snapshot.
        other = lib.Builder(N, builder.params, dev)
        o_sel = torch.empty_like(sel_ws)
        o_lod = torch.empty_like(lod_ws)
        o_img = torch.empty_like(lod_img)
        pipes = [(builder, sel_ws, lod_ws, lod_img, torch.cuda.Stream()),
                 (other, o_sel, o_lod, o_img, torch.cuda.Stream())]

        def pipe_step(i):
            bb, sw, lw, img, st = pipes[i % 2]
            with torch.cuda.stream(st):
                bb.build(x, y, z, m)
                ids_p, nsel_p = lib.select_nodes(bb.tree, cam, 1.0, cfg["n"], workspace=sw)
                lib.splat_lod(bb.tree, ids_p, nsel_p, max_draw, cam, workspace=lw, out=img)
        for i in range(4):
            pipe_step(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(2 * args.steps):
            pipe_step(i)
        torch.cuda.synchronize()
        p_ms = (time.perf_counter() - t0) * 1e3 / (2 * args.steps)
        same = bool(torch.equal(lod_img, o_img))
        extra["pipelined_two_streams"] = {"ms_per_step": round(p_ms, 4), "Mparticles_s": round(N / p_ms / 1e3, 1),
                                          "steps": 2 * args.steps, "images_equal": same}
        log(f"[bench] two pipelines: {p_ms:.3f} ms/step, images equal {same}")
        del other, o_sel, o_lod, o_img, pipes
        torch.cuda.empty_cache()

    if args.stream:
        tree._src = (x, y, z, m)
        extra["streaming"] = stream_leg(tree, N, cfg, dev, args.stream_frames, 10.0, 100.0, args.stream_slots)

    splat_ms = sum(t for k, (c, t) in per_step.items() if k not in build_kernels)
    out = {
        "metric": METRIC,
        "value": round(N / ms_step / 1e3, 2),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(statistics.median(step_ms), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 keys, f64 masses, f32 splat",
        "data": "synthetic",
        "config": {"workload": cfg["label"], "particles": N, "n": cfg["n"], "max_depth": cfg["D"],
                   "alpha": args.alpha, "image": f"{cfg['W']}x{cfg['H']}", "parallelism": "single GPU"},
        "roofline": roof,
        "schedule": tuned or {"mode": builder.params.mode, "select_threads": builder.params.select_threads,
                              "persistent_blocks": builder.params.persistent_blocks},
        "build_ms": round(build_ms, 4),
        "build_ms_runs": "median of %d event-timed builds" % len(build_runs),
        "build_Mparticles_s": round(N / build_ms / 1e3, 1),
        "build_B_alg_GB": round(b_alg / 1e9, 3),
        "build_frac_hbm_B_alg": round(build_frac, 4),
        "build_frac_copy_B_alg": round(b_alg / (build_ms * 1e-3) / 1e9 / copy_gbs, 4),
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
        sample = args.cpu_sample or (5_000_000 if args.workload == "c3" else N)
        log(f"[bench] timing the CPU oracle on {sample} particles")
        out["cpu_baseline"] = cpu_baseline(snap, cfg, sample, args.alpha, 3 if sample <= 1_000_000 else 1)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

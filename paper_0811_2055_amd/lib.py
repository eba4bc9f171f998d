"""ctypes binding of liblod.so (include/lod.h).  Argument marshalling only:
every step of the path runs in the library's HIP kernels.  PyTorch supplies
device memory and the current stream.

The library must have been built (``paper_0811_2055_amd/build.py`` or
``__graft_entry__.build()``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblod.so")

LOD_OK, LOD_EINVAL, LOD_EDOMAIN, LOD_ENOMEM, LOD_EDEVICE, LOD_ECAPACITY, LOD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_DOMAIN, STATUS_CAPACITY, STATUS_OFFSETS, STATUS_INTERNAL = 1, 2, 4, 8
NONE = 0xFFFFFFFF

EXPORTS = [
    "lod_build_plan", "lod_build", "lod_select_plan", "lod_select", "splat_plan",
    "splat_render", "splat_lod_plan", "splat_render_lod", "splat_render_backward",
    "lod_decode_plan", "lod_decode", "lod_autotune", "splat_render_noalloc",
    "splat_render_aux", "lod_highlight_flags", "splat_lod_highlight_plan", "splat_render_lod_highlight",
    "splat_render_interp", "lod_encode_motion", "splat_render_lod_motion",
    "lod_store_save", "lod_store_read_info", "lod_streamer_open", "lod_streamer_frame", "lod_streamer_close",
    "lod_set_node_points",
    "lod_workspace_view", "lod_trace_begin", "lod_trace_end", "lod_status_string", "lod_version",
]


class LodError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code})")


class Params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("max_depth", C.c_uint32), ("density_level", C.c_uint32),
                ("alpha", C.c_int32), ("seed", C.c_uint64), ("mode", C.c_uint32),
                ("select_threads", C.c_uint32), ("persistent_blocks", C.c_uint32), ("reserved", C.c_uint32)]


class Input(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("mass", C.c_void_p),
                ("n_particles", C.c_uint64), ("snap_offsets", C.c_void_p), ("n_snapshots", C.c_uint32)]


class TreeC(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in (
        "prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count",
        "pt_begin", "pt_count", "node_mass", "pt_id", "qx", "qy", "qz", "pt_mass")] + [
        ("node_capacity", C.c_uint64), ("point_capacity", C.c_uint64), ("counts", C.c_void_p)]


class CameraC(C.Structure):
    _fields_ = [("projection", C.c_uint32), ("W", C.c_uint32), ("H", C.c_uint32),
                ("pos", C.c_float * 3), ("right", C.c_float * 3), ("up", C.c_float * 3),
                ("fwd", C.c_float * 3), ("F", C.c_float), ("near_z", C.c_float)]


class FrameC(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "m", "h", "c")]


class StreamStats(C.Structure):
    _fields_ = [("bytes_loaded", C.c_uint64), ("nodes_loaded", C.c_uint32), ("nodes_evicted", C.c_uint32),
                ("nodes_drawn", C.c_uint32), ("groups_waiting", C.c_uint32), ("points_drawn", C.c_uint64),
                ("resident_nodes", C.c_uint64), ("decide_ms", C.c_double), ("io_ms", C.c_double),
                ("upload_ms", C.c_double)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char_p), ("ms", C.c_float)]


class SplatParamsC(C.Structure):
    _fields_ = [("sigma_px", C.c_float), ("radius_sigmas", C.c_float), ("blob", C.c_uint32),
                ("h_px", C.c_float), ("h_world", C.c_float)]


_lib = None


def load():
    """Load liblod.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0811_2055_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    st = C.c_int
    lib.lod_build_plan.argtypes = [C.POINTER(Input), C.POINTER(Params), C.POINTER(C.c_size_t),
                                   C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    lib.lod_build.argtypes = [C.POINTER(Input), C.POINTER(Params), P, C.c_size_t, C.POINTER(TreeC), P]
    lib.lod_select_plan.argtypes = [C.c_uint64, C.POINTER(C.c_size_t)]
    lib.lod_select.argtypes = [C.POINTER(TreeC), C.POINTER(CameraC), C.c_float, C.c_uint32, P,
                               C.c_uint64, P, P, C.c_size_t, P]
    lib.splat_plan.argtypes = [C.c_uint64, C.POINTER(CameraC), C.POINTER(SplatParamsC), C.POINTER(C.c_size_t)]
    lib.splat_render.argtypes = [P, P, P, P, C.c_uint64, C.POINTER(CameraC), C.POINTER(SplatParamsC),
                                 P, C.c_size_t, P, P]
    lib.splat_lod_plan.argtypes = [C.c_uint64, C.c_uint64, C.POINTER(CameraC), C.POINTER(SplatParamsC),
                                   C.POINTER(C.c_size_t)]
    lib.splat_render_lod.argtypes = [C.POINTER(TreeC), P, P, C.c_uint64, C.POINTER(CameraC),
                                     C.POINTER(SplatParamsC), P, C.c_size_t, P, P]
    lib.splat_render_backward.argtypes = [P, P, P, P, C.c_uint64, C.POINTER(CameraC),
                                          C.POINTER(SplatParamsC), P, P, P, P, P, P]
    lib.splat_render_noalloc.argtypes = [P, P, P, P, C.c_uint64, C.POINTER(CameraC), C.POINTER(SplatParamsC),
                                         P, P]
    lib.splat_render_aux.argtypes = [P, P, P, P, P, C.c_uint64, C.POINTER(CameraC), C.POINTER(SplatParamsC),
                                     P, C.c_size_t, P, P, P]
    lib.splat_lod_highlight_plan.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(CameraC),
                                             C.POINTER(SplatParamsC), C.POINTER(C.c_size_t)]
    lib.lod_highlight_flags.argtypes = [C.POINTER(TreeC), P, C.c_uint64, P, P]
    lib.splat_render_lod_highlight.argtypes = [C.POINTER(TreeC), P, P, C.c_uint64, C.POINTER(CameraC),
                                               C.POINTER(SplatParamsC), P, C.c_uint64, P, C.c_size_t, P, P, P]
    lib.splat_render_interp.argtypes = [C.POINTER(FrameC), C.POINTER(FrameC), C.c_uint64, C.c_float,
                                        C.POINTER(CameraC), C.POINTER(SplatParamsC), P, C.c_size_t, P, P, P]
    lib.lod_encode_motion.argtypes = [C.POINTER(TreeC), P, P, P, P, P, P, P, P, P]
    lib.splat_render_lod_motion.argtypes = [C.POINTER(TreeC), P, P, C.c_uint64, P, P, P, C.c_float,
                                            C.POINTER(CameraC), C.POINTER(SplatParamsC), P, C.c_size_t, P, P]
    lib.lod_set_node_points.argtypes = [C.POINTER(TreeC), C.c_uint32, P, P, P, P, C.c_uint32, P]
    lib.lod_store_save.argtypes = [C.POINTER(TreeC), C.c_uint32, C.c_char_p, P]
    lib.lod_store_read_info.argtypes = [C.c_char_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint32)]
    lib.lod_streamer_open.argtypes = [C.c_char_p, C.c_uint32, C.POINTER(TreeC), C.POINTER(C.c_void_p)]
    lib.lod_streamer_frame.argtypes = [P, C.POINTER(CameraC), C.c_float, C.c_uint64, P, P, C.POINTER(StreamStats),
                                       C.POINTER(C.c_uint32), C.c_uint32, C.POINTER(C.c_uint32), C.c_uint32, P]
    lib.lod_streamer_close.argtypes = [P]
    lib.lod_decode_plan.argtypes = [C.c_uint64, C.POINTER(C.c_size_t)]
    lib.lod_decode.argtypes = [C.POINTER(TreeC), P, P, C.c_uint64, P, P, P, P, P, P, C.c_size_t, P]
    lib.lod_autotune.argtypes = [C.POINTER(Input), C.POINTER(Params), P, C.c_size_t, C.POINTER(TreeC),
                                 C.POINTER(Params), C.POINTER(C.c_float), C.c_uint32, C.POINTER(C.c_uint32), P]
    lib.lod_workspace_view.argtypes = [C.POINTER(Input), C.POINTER(Params), P, C.c_uint32,
                                       C.POINTER(C.c_void_p), C.POINTER(C.c_uint64)]
    lib.lod_trace_begin.argtypes = []
    lib.lod_trace_end.argtypes = [C.POINTER(KernelTime), C.c_uint32, C.POINTER(C.c_uint32)]
    lib.lod_status_string.argtypes = [st]
    lib.lod_status_string.restype = C.c_char_p
    lib.lod_version.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("lod_status_string", "lod_version"):
            getattr(lib, name).restype = st
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().lod_status_string(int(code)).decode()


def _check(code, where):
    if code != LOD_OK:
        raise LodError(code, where)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# value types

@dataclass
class BuildParams:
    n: int
    max_depth: int
    density_level: int | None = None
    alpha: int = 1
    seed: int = 0
    mode: int = 1
    select_threads: int = 0
    persistent_blocks: int = 0

    def c(self) -> Params:
        L = self.max_depth if self.density_level is None else self.density_level
        return Params(self.n, self.max_depth, L, self.alpha, self.seed & ((1 << 64) - 1), self.mode,
                      self.select_threads, self.persistent_blocks, 0)


@dataclass
class Camera:
    projection: int
    W: int
    H: int
    pos: tuple = (0.0, 0.0, 0.0)
    right: tuple = (1.0, 0.0, 0.0)
    up: tuple = (0.0, 1.0, 0.0)
    fwd: tuple = (0.0, 0.0, 1.0)
    F: float = 1.0
    near: float = 1e-3

    def c(self) -> CameraC:
        f3 = C.c_float * 3
        return CameraC(self.projection, self.W, self.H, f3(*self.pos), f3(*self.right), f3(*self.up),
                       f3(*self.fwd), self.F, self.near)

    @staticmethod
    def ortho(W: int, H: int) -> "Camera":
        return Camera(0, W, H)

    @staticmethod
    def look_at(pos, target, W: int, H: int, fov_deg: float = 60.0, up_hint=(0.0, 1.0, 0.0),
                near: float = 1e-3) -> "Camera":
        """Perspective camera; the basis is computed in float64 and cast to float32."""
        f = [t - p for t, p in zip(target, pos)]
        fn = math.sqrt(sum(a * a for a in f))
        f = [a / fn for a in f]
        u0 = list(up_hint)
        r = [u0[1] * f[2] - u0[2] * f[1], u0[2] * f[0] - u0[0] * f[2], u0[0] * f[1] - u0[1] * f[0]]
        rn = math.sqrt(sum(a * a for a in r))
        if rn < 1e-12:
            u0 = [1.0, 0.0, 0.0]
            r = [u0[1] * f[2] - u0[2] * f[1], u0[2] * f[0] - u0[0] * f[2], u0[0] * f[1] - u0[1] * f[0]]
            rn = math.sqrt(sum(a * a for a in r))
        r = [a / rn for a in r]
        up = [f[1] * r[2] - f[2] * r[1], f[2] * r[0] - f[0] * r[2], f[0] * r[1] - f[1] * r[0]]
        F = (W / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
        return Camera(1, W, H, tuple(pos), tuple(r), tuple(up), tuple(f), F, near)


@dataclass
class Blob:
    """splat_params: kind 0 = truncated Gaussian (sigma, radius_sigmas), kind 1 =
    radial cubic spline of radius h_px pixels, or of world radius h_world
    (perspective cameras; projected radius clamped to [1, 16] pixels)."""
    kind: int = 0
    sigma: float = 1.0
    radius_sigmas: float = 3.0
    h_px: float = 0.0
    h_world: float = 0.0

    def c(self) -> SplatParamsC:
        return SplatParamsC(self.sigma, self.radius_sigmas, self.kind, self.h_px, self.h_world)

    @staticmethod
    def cubic(h_px: float = 0.0, h_world: float = 0.0) -> "Blob":
        return Blob(1, 1.0, 3.0, h_px, h_world)


def _sp(sigma, radius_sigmas, blob):
    return blob.c() if blob is not None else SplatParamsC(sigma, radius_sigmas, 0, 0.0, 0.0)


@dataclass
class Tree:
    """Device arrays of a built tree (capacity-sized) plus the counts word."""
    arrays: dict
    counts: object            # torch uint64 [3] on the device
    node_capacity: int
    point_capacity: int
    _c: TreeC = field(default=None, repr=False)

    def c(self) -> TreeC:
        if self._c is None:
            a = self.arrays
            self._c = TreeC(*[_ptr(a[k]) for k in (
                "prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count",
                "pt_begin", "pt_count", "node_mass", "pt_id", "qx", "qy", "qz", "pt_mass")],
                self.node_capacity, self.point_capacity, _ptr(self.counts))
        return self._c

    def host(self) -> dict:
        """Copy the used parts to host numpy arrays (synchronises)."""
        import numpy as np
        cnt = self.counts.cpu().numpy().view(np.uint64)
        nn, npt, status = int(cnt[0]), int(cnt[1]), int(cnt[2])
        out = {"n_nodes": nn, "n_points": npt, "status": status}
        for k in ("prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count",
                  "pt_begin", "pt_count", "node_mass"):
            out[k] = _to_numpy(self.arrays[k][:nn])
        for k in ("pt_id", "qx", "qy", "qz", "pt_mass"):
            out[k] = _to_numpy(self.arrays[k][:npt])
        return out


TREE_FILE_FORMAT = "lodtree-npz-1"
_NODE_KEYS = ("prefix", "depth", "parent", "first_child", "child_mask", "part_begin", "part_count", "pt_begin",
              "pt_count", "node_mass")
_POINT_KEYS = ("pt_id", "qx", "qy", "qz", "pt_mass")


def save_tree(tree: Tree, path: str, n: int = 0):
    """Write a built tree to a .npz file: the used part of every node and
    point array, the counts and the capacities (numpy.savez, no pickled
    objects).  n: the build's points per node, kept for the reader.  A tree
    whose status word is not 0 is refused (its outputs are undefined)."""
    import numpy as np
    h = tree.host()
    if h["status"] != 0:
        raise ValueError(f"tree status {h['status']:#x}: the build reported an error")
    np.savez(path, format=np.array(TREE_FILE_FORMAT), n_nodes=np.uint64(h["n_nodes"]),
             n_points=np.uint64(h["n_points"]), node_capacity=np.uint64(tree.node_capacity),
             point_capacity=np.uint64(tree.point_capacity), n=np.uint32(n),
             **{k: h[k] for k in _NODE_KEYS + _POINT_KEYS})


def _from_numpy(a, dtype, device):
    import numpy as np
    import torch
    signed = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32, np.dtype(np.uint16): np.int16}
    if a.dtype in signed:
        return torch.from_numpy(np.ascontiguousarray(a).view(signed[a.dtype])).to(device).view(dtype)
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def load_tree(path: str, device="cuda", node_capacity: int | None = None, point_capacity: int | None = None):
    """Read a tree written by save_tree into newly allocated arrays on
    `device` (capacities: the saved ones unless given larger).  Returns
    (tree, n).  Slots past the node count get pt_count 0 and pt_begin equal to
    the point count, as the build leaves them."""
    import numpy as np
    import torch
    with np.load(path, allow_pickle=False) as f:
        if "format" not in f.files or str(f["format"]) != TREE_FILE_FORMAT:
            raise ValueError(f"{path} is not a tree file")
        V, S = int(f["n_nodes"]), int(f["n_points"])
        nc = max(V, 1, int(node_capacity or f["node_capacity"]))
        pc = max(S, 1, int(point_capacity or f["point_capacity"]))
        tree = alloc_tree(nc, pc, device)
        for keys, count in ((_NODE_KEYS, V), (_POINT_KEYS, S)):
            for k in keys:
                a = f[k]
                dst = tree.arrays[k]
                if a.shape != (count,) or a.dtype.itemsize != dst.element_size():
                    raise ValueError(f"{path}: array {k} has shape {a.shape} and dtype {a.dtype}")
                if count:
                    dst[:count].copy_(_from_numpy(a, dst.dtype, device))
        n = int(f["n"])
    tree.arrays["pt_count"][V:].zero_()
    tree.arrays["pt_begin"][V:].fill_(S)
    tree.counts.copy_(_from_numpy(np.array([V, S, 0], dtype=np.uint64), torch.uint64, device))
    return tree, n


def _to_numpy(t):
    import numpy as np
    import torch
    conv = {torch.uint64: np.uint64, torch.uint32: np.uint32, torch.uint16: np.uint16}
    if t.dtype in conv:
        # torch lacks some unsigned ops; reinterpret through the signed type
        signed = {torch.uint64: torch.int64, torch.uint32: torch.int32, torch.uint16: torch.int16}[t.dtype]
        return t.view(signed).cpu().numpy().view(conv[t.dtype])
    return t.cpu().numpy()


def _empty(n, dtype, device):
    import torch
    return torch.empty(max(int(n), 1), dtype=dtype, device=device)


# ---------------------------------------------------------------------------
# build

def _input(x, y, z, m, snap_offsets):
    N = int(x.numel())
    if snap_offsets is None:
        return Input(_ptr(x), _ptr(y), _ptr(z), _ptr(m), N, C.c_void_p(0), 1)
    return Input(_ptr(x), _ptr(y), _ptr(z), _ptr(m), N, _ptr(snap_offsets), int(snap_offsets.numel()) - 1)


def build_plan(N: int, params: BuildParams, n_snapshots: int = 1):
    lib = load()
    inp = Input(None, None, None, None, N, C.c_void_p(1 if n_snapshots > 1 else 0), n_snapshots)
    ws, nc, pc = C.c_size_t(), C.c_uint64(), C.c_uint64()
    p = params.c()
    _check(lib.lod_build_plan(C.byref(inp), C.byref(p), C.byref(ws), C.byref(nc), C.byref(pc)), "lod_build_plan")
    return int(ws.value), int(nc.value), int(pc.value)


def alloc_tree(node_cap: int, point_cap: int, device) -> Tree:
    import torch
    a = {
        "prefix": _empty(node_cap, torch.uint64, device),
        "depth": _empty(node_cap, torch.uint8, device),
        "parent": _empty(node_cap, torch.uint32, device),
        "first_child": _empty(node_cap, torch.uint32, device),
        "child_mask": _empty(node_cap, torch.uint8, device),
        "part_begin": _empty(node_cap, torch.uint64, device),
        "part_count": _empty(node_cap, torch.uint64, device),
        "pt_begin": _empty(node_cap, torch.uint64, device),
        "pt_count": _empty(node_cap, torch.uint32, device),
        "node_mass": _empty(node_cap, torch.float64, device),
        "pt_id": _empty(point_cap, torch.uint32, device),
        "qx": _empty(point_cap, torch.uint16, device),
        "qy": _empty(point_cap, torch.uint16, device),
        "qz": _empty(point_cap, torch.uint16, device),
        "pt_mass": _empty(point_cap, torch.float32, device),
    }
    counts = torch.zeros(3, dtype=torch.uint64, device=device)
    return Tree(a, counts, max(int(node_cap), 1), max(int(point_cap), 1))


class Builder:
    """Plans once, keeps the workspace and output tree, rebuilds on demand."""

    def __init__(self, N: int, params: BuildParams, device="cuda", n_snapshots: int = 1):
        import torch
        self.N = N
        self.params = params
        self.n_snapshots = n_snapshots
        ws, nc, pc = build_plan(N, params, n_snapshots)
        self.ws_bytes = ws
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        self.tree = alloc_tree(nc, pc, device)

    def build(self, x, y, z, m, snap_offsets=None, stream=None):
        lib = load()
        if int(x.numel()) != self.N:
            raise ValueError("particle count differs from the plan")
        for t in (x, y, z, m):
            if t.dtype.itemsize != 4 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("x, y, z, mass must be contiguous float32 device tensors")
        inp = _input(x, y, z, m, snap_offsets)
        p = self.params.c()
        code = lib.lod_build(C.byref(inp), C.byref(p), _ptr(self.workspace), self.ws_bytes,
                             C.byref(self.tree.c()), stream if stream is not None else _stream())
        _check(code, "lod_build")
        self._inp = inp
        return self.tree

    def autotune(self, x, y, z, m, snap_offsets=None):
        """Time every candidate schedule on this input; adopt and return the fastest.

        Returns (best BuildParams, [(candidate BuildParams, ms), ...])."""
        lib = load()
        inp = _input(x, y, z, m, snap_offsets)
        p = self.params.c()
        cap = 64
        cands = (Params * cap)()
        ms = (C.c_float * cap)()
        n = C.c_uint32()
        _check(lib.lod_autotune(C.byref(inp), C.byref(p), _ptr(self.workspace), self.ws_bytes,
                                C.byref(self.tree.c()), cands, ms, cap, C.byref(n), _stream()), "lod_autotune")
        self.params.mode, self.params.select_threads, self.params.persistent_blocks = \
            p.mode, p.select_threads, p.persistent_blocks
        table = []
        for i in range(min(n.value, cap)):
            c = cands[i]
            table.append((dict(mode=c.mode, select_threads=c.select_threads,
                               persistent_blocks=c.persistent_blocks), float(ms[i])))
        return self.params, table

    def view(self, which: int, dtype):
        """Intermediate arrays (0 keys, 1 ids, 2 w, 3 key bins, 4 witness) as a torch view."""
        import torch
        lib = load()
        ptr, cnt = C.c_void_p(), C.c_uint64()
        p = self.params.c()
        _check(lib.lod_workspace_view(C.byref(self._inp), C.byref(p), _ptr(self.workspace), which,
                                      C.byref(ptr), C.byref(cnt)), "lod_workspace_view")
        base = self.workspace.data_ptr()
        off = ptr.value - base
        size = torch.tensor([], dtype=dtype).element_size()
        return self.workspace[off:off + int(cnt.value) * size].view(dtype)


def build(x, y, z, m, params: BuildParams, snap_offsets=None) -> Tree:
    nsnap = 1 if snap_offsets is None else int(snap_offsets.numel()) - 1
    b = Builder(int(x.numel()), params, x.device, nsnap)
    return b.build(x, y, z, m, snap_offsets)


class trace:
    """Context manager collecting (kernel name, ms) for every launch inside it."""

    def __enter__(self):
        _check(load().lod_trace_begin(), "lod_trace_begin")
        self.records = []
        return self

    def __exit__(self, *exc):
        lib = load()
        cap = 1 << 16
        buf = (KernelTime * cap)()
        n = C.c_uint32()
        _check(lib.lod_trace_end(buf, cap, C.byref(n)), "lod_trace_end")
        self.records = [(buf[i].name.decode(), float(buf[i].ms)) for i in range(min(n.value, cap))]
        return False

    def summary(self):
        """{kernel: (launches, total ms)}"""
        out = {}
        for name, ms in self.records:
            c, t = out.get(name, (0, 0.0))
            out[name] = (c + 1, t + ms)
        return out


# ---------------------------------------------------------------------------
# cut and splat

def select_nodes(tree: Tree, cam: Camera, tau_px: float, n: int, cap: int | None = None, workspace=None):
    """Returns (node_ids device uint32 [cap], n_selected device uint64 [1])."""
    import torch
    lib = load()
    dev = tree.counts.device
    cap = tree.node_capacity if cap is None else cap
    ws = C.c_size_t()
    _check(lib.lod_select_plan(tree.node_capacity, C.byref(ws)), "lod_select_plan")
    if workspace is None or workspace.numel() < ws.value:
        workspace = torch.empty(max(ws.value, 256), dtype=torch.uint8, device=dev)
    ids = torch.empty(max(cap, 1), dtype=torch.uint32, device=dev)
    nsel = torch.zeros(1, dtype=torch.uint64, device=dev)
    camc = cam.c()
    _check(lib.lod_select(C.byref(tree.c()), C.byref(camc), float(tau_px), int(n), _ptr(ids), cap,
                          _ptr(nsel), _ptr(workspace), ws.value, _stream()), "lod_select")
    return ids, nsel


def splat_workspace_bytes(max_points: int, cam: Camera, sigma=1.0, radius_sigmas=3.0, blob=None) -> int:
    lib = load()
    ws = C.c_size_t()
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_plan(int(max_points), C.byref(camc), C.byref(sp), C.byref(ws)), "splat_plan")
    return int(ws.value)


def splat(x, y, z, m, cam: Camera, sigma=1.0, radius_sigmas=3.0, workspace=None, out=None, blob=None):
    import torch
    lib = load()
    dev = x.device
    N = int(x.numel())
    ws = splat_workspace_bytes(N, cam, sigma, radius_sigmas, blob)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    img = out if out is not None else torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render(_ptr(x), _ptr(y), _ptr(z), _ptr(m), N, C.byref(camc), C.byref(sp),
                            _ptr(workspace), workspace.numel(), _ptr(img), _stream()), "splat_render")
    return img


def splat_aux(x, y, z, m, aux, cam: Camera, sigma=1.0, radius_sigmas=3.0, workspace=None, blob=None):
    """(image, attribute image) with the attribute image sum_k m_k a_k W_k."""
    import torch
    lib = load()
    dev = x.device
    N = int(x.numel())
    ws = splat_workspace_bytes(N, cam, sigma, radius_sigmas, blob)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    img = torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    aimg = torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render_aux(_ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(aux), N, C.byref(camc), C.byref(sp),
                                _ptr(workspace), workspace.numel(), _ptr(img), _ptr(aimg), _stream()),
           "splat_render_aux")
    return img, aimg


NOALLOC_SCRATCH_BYTES = 64 << 20


def splat_noalloc(x, y, z, m, cam: Camera, sigma=1.0, radius_sigmas=3.0, out=None, blob=None):
    """splat_render with the library's fixed device scratch array as workspace
    (no device allocation inside the call; `out` may be preallocated)."""
    import torch
    lib = load()
    N = int(x.numel())
    img = out if out is not None else torch.empty((cam.H, cam.W), dtype=torch.float32, device=x.device)
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render_noalloc(_ptr(x), _ptr(y), _ptr(z), _ptr(m), N, C.byref(camc), C.byref(sp), _ptr(img),
                                    _stream()), "splat_render_noalloc")
    return img


def splat_lod_workspace_bytes(node_capacity: int, max_points: int, cam: Camera, sigma=1.0, radius_sigmas=3.0,
                              blob=None):
    lib = load()
    ws = C.c_size_t()
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_lod_plan(int(node_capacity), int(max_points), C.byref(camc), C.byref(sp), C.byref(ws)),
           "splat_lod_plan")
    return int(ws.value)


def splat_lod(tree: Tree, node_ids, n_ids, max_points: int, cam: Camera, sigma=1.0, radius_sigmas=3.0,
              workspace=None, out=None, blob=None):
    import torch
    lib = load()
    dev = tree.counts.device
    ws = splat_lod_workspace_bytes(tree.node_capacity, max_points, cam, sigma, radius_sigmas, blob)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    img = out if out is not None else torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render_lod(C.byref(tree.c()), _ptr(node_ids), _ptr(n_ids), int(max_points), C.byref(camc),
                                C.byref(sp), _ptr(workspace), workspace.numel(), _ptr(img), _stream()),
           "splat_render_lod")
    return img


def highlight_bits(ids, n_bits: int, device="cuda"):
    """Device uint32 bitset over ids [0, n_bits) with the given ids set (host-side packing)."""
    import numpy as np
    import torch
    words = np.zeros(max(1, (int(n_bits) + 31) // 32), dtype=np.uint32)
    ids = np.asarray(ids, dtype=np.int64)
    ids = ids[(ids >= 0) & (ids < n_bits)]
    np.bitwise_or.at(words, ids >> 5, (np.uint32(1) << (ids & 31).astype(np.uint32)))
    return torch.from_numpy(words.view(np.int32)).to(device).view(torch.uint32)


def splat_lod_highlight_workspace_bytes(node_capacity: int, max_points: int, max_highlighted: int, cam: Camera,
                                        sigma=1.0, radius_sigmas=3.0, blob=None):
    lib = load()
    ws = C.c_size_t()
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_lod_highlight_plan(int(node_capacity), int(max_points), int(max_highlighted), C.byref(camc),
                                        C.byref(sp), C.byref(ws)), "splat_lod_highlight_plan")
    return int(ws.value)


def highlight_flags(tree: Tree, bits, n_bits: int, out=None):
    """One flag bit per stored point of the tree (device uint32 words): set when
    the point's id is in the id bitset `bits` of n_bits bits.  `out` (uint32,
    2 ceil(point_capacity / 64) words) is reused when given; every word is
    written."""
    import torch
    lib = load()
    words = 2 * ((tree.point_capacity + 63) // 64)
    if out is None:
        out = torch.empty(words, dtype=torch.int32, device=tree.counts.device).view(torch.uint32)
    elif out.numel() < words or out.element_size() != 4 or not out.is_contiguous():
        raise ValueError(f"flags need {words} contiguous 32-bit words")
    flags = out
    _check(lib.lod_highlight_flags(C.byref(tree.c()), _ptr(bits), int(n_bits), _ptr(flags), _stream()),
           "lod_highlight_flags")
    return flags


def splat_lod_highlight(tree: Tree, node_ids, n_ids, max_points: int, cam: Camera, flags, max_highlighted: int,
                        sigma=1.0, radius_sigmas=3.0, workspace=None, out=None, out_hl=None, blob=None):
    """(image, highlight image): the LOD render and the same render of the drawn
    points whose stored-point flag is set (`highlight_flags`), at most max_highlighted."""
    import torch
    lib = load()
    dev = tree.counts.device
    ws = splat_lod_highlight_workspace_bytes(tree.node_capacity, max_points, max_highlighted, cam, sigma,
                                             radius_sigmas, blob)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    img = out if out is not None else torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    hl = out_hl if out_hl is not None else torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render_lod_highlight(C.byref(tree.c()), _ptr(node_ids), _ptr(n_ids), int(max_points),
                                          C.byref(camc), C.byref(sp), _ptr(flags), int(max_highlighted),
                                          _ptr(workspace), workspace.numel(), _ptr(img), _ptr(hl), _stream()),
           "splat_render_lod_highlight")
    return img, hl


def splat_interp(A, B, t: float, cam: Camera, sigma=1.0, radius_sigmas=3.0, blob=None, hA=None, hB=None,
                 cA=None, cB=None, workspace=None):
    """The frame at time t between snapshots A and B (each (x, y, z, m) device
    float32 tensors of the same particles); optional per-particle world radii
    and colours.  Returns the image, or (image, colour image) with colours."""
    import torch
    lib = load()
    dev = A[0].device
    N = int(A[0].numel())
    ws = splat_workspace_bytes(N, cam, sigma, radius_sigmas, blob)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    fa = FrameC(*[_ptr(a) for a in (*A, hA, cA)])
    fb = FrameC(*[_ptr(b) for b in (*B, hB, cB)])
    img = torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    cimg = torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev) if cA is not None else None
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render_interp(C.byref(fa), C.byref(fb), N, float(t), C.byref(camc), C.byref(sp),
                                   _ptr(workspace), workspace.numel(), _ptr(img), _ptr(cimg), _stream()),
           "splat_render_interp")
    return (img, cimg) if cimg is not None else img


def encode_motion(tree: Tree, xB, yB, zB, snap_offsets=None):
    """Motion codes (dqx, dqy, dqz device int16 [point capacity]) and the
    saturated-component count (device uint64 [1])."""
    import torch
    lib = load()
    dev = tree.counts.device
    dq = [torch.zeros(tree.point_capacity, dtype=torch.int16, device=dev) for _ in range(3)]
    sat = torch.zeros(1, dtype=torch.uint64, device=dev)
    _check(lib.lod_encode_motion(C.byref(tree.c()), _ptr(xB), _ptr(yB), _ptr(zB), _ptr(snap_offsets),
                                 *[_ptr(a) for a in dq], _ptr(sat), _stream()), "lod_encode_motion")
    return (*dq, sat)


def splat_lod_motion(tree: Tree, node_ids, n_ids, max_points: int, motion, t: float, cam: Camera, sigma=1.0,
                     radius_sigmas=3.0, workspace=None, out=None, blob=None):
    """The LOD render at frame time t: stored points moved along their motion codes."""
    import torch
    lib = load()
    dev = tree.counts.device
    ws = splat_lod_workspace_bytes(tree.node_capacity, max_points, cam, sigma, radius_sigmas, blob)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
    img = out if out is not None else torch.empty((cam.H, cam.W), dtype=torch.float32, device=dev)
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render_lod_motion(C.byref(tree.c()), _ptr(node_ids), _ptr(n_ids), int(max_points),
                                       *[_ptr(a) for a in motion[:3]], float(t), C.byref(camc), C.byref(sp),
                                       _ptr(workspace), workspace.numel(), _ptr(img), _stream()),
           "splat_render_lod_motion")
    return img


def splat_backward(x, y, z, m, grad_image, cam: Camera, sigma=1.0, radius_sigmas=3.0, blob=None):
    import torch
    lib = load()
    N = int(x.numel())
    gm = torch.empty(N, dtype=torch.float32, device=x.device)
    gx = torch.empty(N, dtype=torch.float32, device=x.device)
    gy = torch.empty(N, dtype=torch.float32, device=x.device)
    gz = torch.empty(N, dtype=torch.float32, device=x.device)
    g = grad_image.contiguous()
    camc, sp = cam.c(), _sp(sigma, radius_sigmas, blob)
    _check(lib.splat_render_backward(_ptr(x), _ptr(y), _ptr(z), _ptr(m), N, C.byref(camc), C.byref(sp), _ptr(g),
                                     _ptr(gm), _ptr(gx), _ptr(gy), _ptr(gz), _stream()), "splat_render_backward")
    return gm, gx, gy, gz


def set_node_points(tree: Tree, node: int, x, y, z, m):
    """Write positions and masses (device float32) back as the node's stored points."""
    _check(load().lod_set_node_points(C.byref(tree.c()), int(node), _ptr(x), _ptr(y), _ptr(z), _ptr(m),
                                      int(x.numel()), _stream()), "lod_set_node_points")


def decode_nodes(tree: Tree, node_ids, n_ids, max_points: int):
    """Decode the stored points of the given nodes; returns (x, y, z, m, count tensor)."""
    import torch
    lib = load()
    dev = tree.counts.device
    ws = C.c_size_t()
    _check(lib.lod_decode_plan(tree.node_capacity, C.byref(ws)), "lod_decode_plan")
    work = torch.empty(max(ws.value, 256), dtype=torch.uint8, device=dev)
    out = [torch.empty(max(int(max_points), 1), dtype=torch.float32, device=dev) for _ in range(4)]
    cnt = torch.zeros(1, dtype=torch.uint64, device=dev)
    _check(lib.lod_decode(C.byref(tree.c()), _ptr(node_ids), _ptr(n_ids), int(max_points), *[_ptr(t) for t in out],
                          _ptr(cnt), _ptr(work), ws.value, _stream()), "lod_decode")
    return (*out, cnt)


# ---------------------------------------------------------------------------
# block store and streaming

def store_save(tree: Tree, n: int, path: str):
    """Write a built tree to a block store file (synchronises)."""
    _check(load().lod_store_save(C.byref(tree.c()), int(n), path.encode(), _stream()), "lod_store_save")


def store_info(path: str):
    """(node count, stored point count, n) of a store file."""
    nn, npts, n = C.c_uint64(), C.c_uint64(), C.c_uint32()
    _check(load().lod_store_read_info(path.encode(), C.byref(nn), C.byref(npts), C.byref(n)), "lod_store_read_info")
    return int(nn.value), int(npts.value), int(n.value)


class Streamer:
    """View-dependent streaming of a block store into a device pool of
    `slots` node slots; `frame()` returns the device draw list of the frame."""

    def __init__(self, path: str, slots: int, device="cuda"):
        import torch
        nn, npts, n = store_info(path)
        self.n = n
        self.view = alloc_tree(nn, slots * n, device)
        self.draw_ids = torch.empty(max(nn, 1), dtype=torch.uint32, device=device)
        self.n_draw = torch.zeros(1, dtype=torch.uint64, device=device)
        self._h = C.c_void_p()
        _check(load().lod_streamer_open(path.encode(), int(slots), C.byref(self.view.c()), C.byref(self._h)),
               "lod_streamer_open")
        self.n_nodes = nn

    def frame(self, cam: Camera, tau_px: float, budget_bytes: int, want_ids: bool = False):
        """One frame; returns (draw ids device tensor, count tensor, stats dict[, loaded, evicted])."""
        st = StreamStats()
        cap = self.n_nodes
        la = (C.c_uint32 * max(cap, 1))()
        ea = (C.c_uint32 * max(cap, 1))()
        camc = cam.c()
        _check(load().lod_streamer_frame(self._h, C.byref(camc), float(tau_px), int(budget_bytes), _ptr(self.draw_ids),
                                         _ptr(self.n_draw), C.byref(st), la, cap, ea, cap, _stream()),
               "lod_streamer_frame")
        stats = {k: getattr(st, k) for k, _ in StreamStats._fields_}
        if want_ids:
            return (self.draw_ids, self.n_draw, stats, [la[i] for i in range(min(st.nodes_loaded, cap))],
                    [ea[i] for i in range(min(st.nodes_evicted, cap))])
        return self.draw_ids, self.n_draw, stats

    def close(self):
        if self._h:
            _check(load().lod_streamer_close(self._h), "lod_streamer_close")
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

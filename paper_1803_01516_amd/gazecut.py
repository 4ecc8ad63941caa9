"""Thin ctypes binding of the gazecut C ABI (include/gazecut.h).

Argument marshalling only: every step of the path runs in the HIP library
``libgazecut.so`` built from ``csrc/gazecut.hip``.  Device buffers are torch
CUDA tensors (PyTorch is used for device memory and streams only).  There is
no CPU fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgazecut.so")

GC_OK = 0
GC_E_NOT_CONVERGED = -5


class GcProblem(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "width", "height", "labels", "cap", "penalty_h", "inhibit_h", "penalty_v", "inhibit_v")]


class GcGraph(ctypes.Structure):
    _fields_ = [("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t), ("p", GcProblem),
                ("window_block", ctypes.c_int32), ("compact", ctypes.c_int32)]


class GcSolveOpts(ctypes.Structure):
    _fields_ = [("relabel_period", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("tile_j", ctypes.c_int32), ("local_iters", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("relabel_passes", ctypes.c_int32)]


GC_OPT_TIME_KERNELS = 1
GC_OPT_SWEEP_GRAPH = 2
GC_OPT_WAVE_FIRST = 4
GC_OPT_FUSED_SWEEP = 16
GC_OPT_SPLIT_SWEEP = 64
GC_OPT_FIXED_PERIOD = 32
GC_OPT_BATCH_MERGED = 128
GC_OPT_LISTS = 256
GC_BATCH_LANES = 4
GC_BATCH_ENGINES = 3
GC_BATCH_MAX_GRAPHS = 256
GC_STATIC_SCRATCH_BYTES = 96 << 20
KERNEL_CLASSES = ("push", "relabel", "relax", "other")


class GcSolveStats(ctypes.Structure):
    _fields_ = [("pushes", ctypes.c_int64), ("sweeps", ctypes.c_int32),
                ("global_relabels", ctypes.c_int32), ("bfs_passes", ctypes.c_int32),
                ("active_last", ctypes.c_int32), ("kernel_launches", ctypes.c_int32 * 4),
                ("kernel_ms", ctypes.c_double * 4), ("done_ms", ctypes.c_double),
                ("active_visits", ctypes.c_int64)]

    def as_dict(self):
        d = {"pushes": int(self.pushes), "sweeps": int(self.sweeps),
             "global_relabels": int(self.global_relabels),
             "bfs_passes": int(self.bfs_passes), "active_last": int(self.active_last),
             "done_ms": float(self.done_ms), "active_visits": int(self.active_visits)}
        for i, k in enumerate(KERNEL_CLASSES):
            d[f"{k}_launches"] = int(self.kernel_launches[i])
            d[f"{k}_ms"] = float(self.kernel_ms[i])
        return d


EXPORTS = ("gc_status_str", "gc_last_hip_error", "gc_problem_check", "gc_graph_footprint_bytes",
           "stereo_cost_volume", "stereo_cost_volume_rgb", "graph_build", "maxflow_solve",
           "extract_labels", "gc_graph_state",
           "gc_coarse_problem", "coarse_cost_volume", "graph_build_window", "approx_level2_cut",
           "gc_batch_footprint_bytes", "gc_batch_create", "gc_batch_destroy", "gc_batch_members",
           "gc_batch_add", "gc_batch_round", "maxflow_solve_batch",
           "gc_solve_pair_static_bytes", "gc_solve_pair_static", "graph_warm_start",
           "graph_build_skin", "gc_skin_footprint_bytes")

_lib = None


class GazecutError(RuntimeError):
    def __init__(self, status: int, what: str):
        lib = _lib
        msg = lib.gc_status_str(status).decode() if lib is not None else str(status)
        extra = ""
        if lib is not None and status == -6:
            extra = f" (hipError {lib.gc_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{status}]{extra}")
        self.status = status


def load(path: str = LIB_PATH):
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"gazecut HIP library not found at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.gc_status_str.argtypes = [ctypes.c_int]
    lib.gc_status_str.restype = ctypes.c_char_p
    lib.gc_last_hip_error.argtypes = []
    lib.gc_last_hip_error.restype = ctypes.c_int
    lib.gc_problem_check.argtypes = [ctypes.POINTER(GcProblem)]
    lib.gc_problem_check.restype = ctypes.c_int
    lib.gc_graph_footprint_bytes.argtypes = [ctypes.POINTER(GcProblem)]
    lib.gc_graph_footprint_bytes.restype = ctypes.c_size_t
    lib.stereo_cost_volume.argtypes = [P, P, ctypes.POINTER(GcProblem), P, P]
    lib.stereo_cost_volume.restype = ctypes.c_int
    lib.stereo_cost_volume_rgb.argtypes = [P, P, ctypes.POINTER(GcProblem), P, P]
    lib.stereo_cost_volume_rgb.restype = ctypes.c_int
    lib.graph_build.argtypes = [ctypes.POINTER(GcProblem), P, P, ctypes.c_size_t,
                                ctypes.POINTER(GcGraph), P]
    lib.graph_build.restype = ctypes.c_int
    lib.maxflow_solve.argtypes = [ctypes.POINTER(GcGraph), ctypes.POINTER(GcSolveOpts),
                                  ctypes.POINTER(GcSolveStats), P]
    lib.maxflow_solve.restype = ctypes.c_int
    lib.extract_labels.argtypes = [ctypes.POINTER(GcGraph), P, P, P, P]
    lib.extract_labels.restype = ctypes.c_int
    lib.gc_graph_state.argtypes = [ctypes.POINTER(GcGraph), P, P, P]
    lib.gc_graph_state.restype = ctypes.c_int
    lib.gc_coarse_problem.argtypes = [ctypes.POINTER(GcProblem), ctypes.c_int32,
                                      ctypes.POINTER(GcProblem)]
    lib.gc_coarse_problem.restype = ctypes.c_int
    lib.coarse_cost_volume.argtypes = [ctypes.POINTER(GcProblem), P, ctypes.c_int32, P, P]
    lib.coarse_cost_volume.restype = ctypes.c_int
    lib.graph_build_window.argtypes = [ctypes.POINTER(GcProblem), P, P, ctypes.c_int32, P,
                                       ctypes.c_size_t, ctypes.POINTER(GcGraph), P]
    lib.graph_build_window.restype = ctypes.c_int
    lib.graph_build_skin.argtypes = [ctypes.POINTER(GcProblem), P, P, ctypes.c_int32, P,
                                     ctypes.c_size_t, ctypes.POINTER(GcGraph), P]
    lib.graph_build_skin.restype = ctypes.c_int
    lib.gc_skin_footprint_bytes.argtypes = [ctypes.POINTER(GcProblem), ctypes.c_int32]
    lib.gc_skin_footprint_bytes.restype = ctypes.c_size_t
    lib.approx_level2_cut.argtypes = [ctypes.POINTER(GcGraph), P, P, ctypes.c_int32, P, P, P]
    lib.approx_level2_cut.restype = ctypes.c_int
    lib.graph_warm_start.argtypes = [ctypes.POINTER(GcGraph), ctypes.POINTER(GcGraph), P, P]
    lib.graph_warm_start.restype = ctypes.c_int
    lib.gc_batch_footprint_bytes.argtypes = []
    lib.gc_batch_footprint_bytes.restype = ctypes.c_size_t
    lib.gc_batch_create.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(GcSolveOpts), ctypes.POINTER(P)]
    lib.gc_batch_create.restype = ctypes.c_int
    lib.gc_batch_destroy.argtypes = [P]
    lib.gc_batch_destroy.restype = ctypes.c_int
    lib.gc_batch_members.argtypes = [P]
    lib.gc_batch_members.restype = ctypes.c_int
    lib.gc_batch_add.argtypes = [P, ctypes.POINTER(GcGraph), ctypes.c_int64]
    lib.gc_batch_add.restype = ctypes.c_int
    lib.gc_batch_round.argtypes = [P, P, P, ctypes.POINTER(GcSolveStats), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.gc_batch_round.restype = ctypes.c_int
    lib.maxflow_solve_batch.argtypes = [ctypes.POINTER(ctypes.POINTER(GcGraph)), ctypes.c_int32, P,
                                        ctypes.c_size_t, ctypes.POINTER(GcSolveOpts),
                                        ctypes.POINTER(GcSolveStats), P]
    lib.maxflow_solve_batch.restype = ctypes.c_int
    lib.gc_solve_pair_static_bytes.argtypes = [ctypes.POINTER(GcProblem)]
    lib.gc_solve_pair_static_bytes.restype = ctypes.c_size_t
    lib.gc_solve_pair_static.argtypes = [P, P, ctypes.POINTER(GcProblem), ctypes.POINTER(GcSolveOpts),
                                         P, P, ctypes.POINTER(GcSolveStats), P]
    lib.gc_solve_pair_static.restype = ctypes.c_int
    _lib = lib
    return lib


def problem(width, height, labels, cap, penalty_h, inhibit_h, penalty_v=None, inhibit_v=None):
    return GcProblem(int(width), int(height), int(labels), int(cap), int(penalty_h),
                     int(inhibit_h), int(penalty_h if penalty_v is None else penalty_v),
                     int(inhibit_h if inhibit_v is None else inhibit_v))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(rc: int, what: str):
    if rc != GC_OK:
        raise GazecutError(rc, what)


def problem_check(p: GcProblem) -> int:
    return load().gc_problem_check(ctypes.byref(p))


def footprint_bytes(p: GcProblem) -> int:
    return int(load().gc_graph_footprint_bytes(ctypes.byref(p)))


def stereo_cost_volume(left, right, p: GcProblem, cost, stream=None):
    """left/right: uint8 [h][w] CUDA tensors; cost: int32 [m][h][w] CUDA tensor."""
    _check(load().stereo_cost_volume(ctypes.c_void_p(left.data_ptr()), ctypes.c_void_p(right.data_ptr()),
                                     ctypes.byref(p), ctypes.c_void_p(cost.data_ptr()),
                                     _stream_ptr(stream)), "stereo_cost_volume")


def stereo_cost_volume_rgb(left, right, p: GcProblem, cost, stream=None):
    """left/right: uint8 [h][w][3] CUDA tensors (channels interleaved);
    cost: int32 [m][h][w] CUDA tensor."""
    if left.dim() != 3 or left.shape[2] != 3 or tuple(right.shape) != tuple(left.shape):
        raise ValueError("colour images must be [h][w][3] and of equal shape")
    _check(load().stereo_cost_volume_rgb(ctypes.c_void_p(left.data_ptr()), ctypes.c_void_p(right.data_ptr()),
                                         ctypes.byref(p), ctypes.c_void_p(cost.data_ptr()),
                                         _stream_ptr(stream)), "stereo_cost_volume_rgb")


@dataclass
class Graph:
    handle: GcGraph
    ws: object          # the torch uint8 workspace tensor (kept alive here)


def graph_build(p: GcProblem, cost, ws, stream=None) -> Graph:
    """ws: uint8 CUDA tensor of at least footprint_bytes(p) bytes."""
    g = GcGraph()
    _check(load().graph_build(ctypes.byref(p), ctypes.c_void_p(cost.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                              ctypes.byref(g), _stream_ptr(stream)), "graph_build")
    return Graph(g, ws)


def maxflow_solve(graph: Graph, opts: GcSolveOpts | None = None, stream=None,
                  allow_not_converged: bool = False) -> GcSolveStats:
    st = GcSolveStats()
    rc = load().maxflow_solve(ctypes.byref(graph.handle),
                              ctypes.byref(opts) if opts is not None else None,
                              ctypes.byref(st), _stream_ptr(stream))
    if not (allow_not_converged and rc == GC_E_NOT_CONVERGED):
        _check(rc, "maxflow_solve")
    return st


def solve_pair_static_bytes(p: GcProblem) -> int:
    return int(load().gc_solve_pair_static_bytes(ctypes.byref(p)))


def solve_pair_static(left, right, p: GcProblem, labels, result, opts: GcSolveOpts | None = None,
                      stream=None) -> GcSolveStats:
    """The whole exact path on one pair with the cost volume and the graph in
    the library's static device array (no allocation by the library).
    labels: int32 [h][w], result: int64 [2] CUDA tensors (written)."""
    st = GcSolveStats()
    _check(load().gc_solve_pair_static(ctypes.c_void_p(left.data_ptr()),
                                       ctypes.c_void_p(right.data_ptr()), ctypes.byref(p),
                                       ctypes.byref(opts) if opts is not None else None,
                                       ctypes.c_void_p(labels.data_ptr()),
                                       ctypes.c_void_p(result.data_ptr()), ctypes.byref(st),
                                       _stream_ptr(stream)), "gc_solve_pair_static")
    return st


def extract_labels(graph: Graph, cost, labels, result, stream=None):
    """labels: int32 [h][w] CUDA tensor; result: int64 [2] CUDA tensor
    (energy, flow)."""
    _check(load().extract_labels(ctypes.byref(graph.handle), ctypes.c_void_p(cost.data_ptr()),
                                 ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(result.data_ptr()),
                                 _stream_ptr(stream)), "extract_labels")


def graph_state(graph: Graph, stream=None):
    """Exports the graph's state: (balances int32 [m-1][h][w], pair words int32
    [7][m-1][h][w]) as CUDA tensors (layout in gazecut.h)."""
    import torch
    p = graph.handle.p
    dev = graph.ws.device
    ex = torch.empty((max(p.labels - 1, 0), p.height, p.width), dtype=torch.int32, device=dev)
    words = torch.empty((7, max(p.labels - 1, 0), p.height, p.width), dtype=torch.int32, device=dev)
    _check(load().gc_graph_state(ctypes.byref(graph.handle), ctypes.c_void_p(ex.data_ptr()),
                                 ctypes.c_void_p(words.data_ptr()), _stream_ptr(stream)), "gc_graph_state")
    return ex, words


def alloc_workspace(p: GcProblem, device="cuda"):
    import torch
    nbytes = footprint_bytes(p)
    if nbytes == 0:
        _check(problem_check(p) or -1, "footprint")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def skin_footprint_bytes(p: GcProblem, block: int) -> int:
    return int(load().gc_skin_footprint_bytes(ctypes.byref(p), int(block)))


def alloc_skin_workspace(p: GcProblem, block: int, device="cuda"):
    """Workspace of a compact thin skin (graph_build_skin)."""
    import torch
    nbytes = skin_footprint_bytes(p, block)
    if nbytes == 0:
        _check(problem_check(p) or -1, "skin footprint")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def solve_pair(left, right, p: GcProblem, opts: GcSolveOpts | None = None, stream=None,
               ws=None):
    """Runs the whole path on one pair of uint8 CUDA tensors ([h][w] grey or
    [h][w][3] colour).  Returns (labels tensor, cost tensor, energy, flow,
    stats)."""
    import torch
    dev = left.device
    cost = torch.empty((p.labels, p.height, p.width), dtype=torch.int32, device=dev)
    labels = torch.empty((p.height, p.width), dtype=torch.int32, device=dev)
    result = torch.zeros(2, dtype=torch.int64, device=dev)
    if ws is None:
        ws = alloc_workspace(p, dev)
    if left.dim() == 3:
        stereo_cost_volume_rgb(left, right, p, cost, stream)
    else:
        stereo_cost_volume(left, right, p, cost, stream)
    g = graph_build(p, cost, ws, stream)
    st = maxflow_solve(g, opts, stream)
    extract_labels(g, cost, labels, result, stream)
    r = result.cpu()
    return labels, cost, int(r[0]), int(r[1]), st


# ---------------------------------------------------------------------------
# Hierarchical approximation, level 1 (Sec. 4.5)
# ---------------------------------------------------------------------------

def coarse_problem(p: GcProblem, block: int) -> GcProblem:
    c = GcProblem()
    _check(load().gc_coarse_problem(ctypes.byref(p), int(block), ctypes.byref(c)), "gc_coarse_problem")
    return c


def coarse_cost_volume(p: GcProblem, cost, block: int, coarse_cost, stream=None):
    _check(load().coarse_cost_volume(ctypes.byref(p), ctypes.c_void_p(cost.data_ptr()), int(block),
                                     ctypes.c_void_p(coarse_cost.data_ptr()), _stream_ptr(stream)),
           "coarse_cost_volume")


def graph_build_window(p: GcProblem, cost, coarse_labels, block: int, ws, stream=None) -> Graph:
    g = GcGraph()
    _check(load().graph_build_window(ctypes.byref(p), ctypes.c_void_p(cost.data_ptr()),
                                     ctypes.c_void_p(coarse_labels.data_ptr()), int(block),
                                     ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                     ctypes.byref(g), _stream_ptr(stream)), "graph_build_window")
    return Graph(g, ws)


def graph_build_skin(p: GcProblem, cost, coarse_labels, block: int, ws, stream=None) -> Graph:
    """The compact thin skin (only the windows' levels stored); ws of at
    least skin_footprint_bytes(p, block) bytes."""
    g = GcGraph()
    _check(load().graph_build_skin(ctypes.byref(p), ctypes.c_void_p(cost.data_ptr()),
                                   ctypes.c_void_p(coarse_labels.data_ptr()), int(block),
                                   ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                   ctypes.byref(g), _stream_ptr(stream)), "graph_build_skin")
    return Graph(g, ws)


# Wave steps (A - 1) of the level-2 cut when the caller gives none:
# max(32, labels).  Measured on MI355X: on the 384x288x16 pairs 32 steps
# reach the level-1 labels' quality (eq. (2) error 1195 against 1161 for
# level 1 b=3; 16 steps leave it at 137000) in 2.1 ms against 3.0 ms for 64;
# the 450x375x64 pairs with textureless regions need 64 (at 32 steps whole
# regions whose flow has not yet reached the cut are read out at the top of
# their windows: error 503000 against 49900).
def level2_wave_steps(labels: int) -> int:
    return max(32, int(labels))


def approx_level2_cut(skin: Graph, cost, coarse_labels, labels, result, stream=None,
                      wave_steps: int | None = None):
    if wave_steps is None:
        wave_steps = level2_wave_steps(skin.handle.p.labels)
    _check(load().approx_level2_cut(ctypes.byref(skin.handle), ctypes.c_void_p(cost.data_ptr()),
                                    ctypes.c_void_p(coarse_labels.data_ptr()), int(wave_steps),
                                    ctypes.c_void_p(labels.data_ptr()),
                                    ctypes.c_void_p(result.data_ptr()), _stream_ptr(stream)),
           "approx_level2_cut")


def approx_solve_opts(p: GcProblem) -> GcSolveOpts:
    """Options of the coarse and skin solves of the approximations when the
    caller gives none: the relabel period and early-stop pass count of the
    full problem's depth (32 sweeps and 16 passes from 32 levels on, else 24
    and 8).  The coarse graph of a deep problem has fewer levels but the same
    lateral structure and needs them too: with 8 passes, level 1 b = 2 on
    450x375x64 took 27.6 instead of 15.0 ms.  The cuts do not depend on them."""
    deep = p.labels - 1 >= 32
    return GcSolveOpts(relabel_period=32 if deep else 24, relabel_passes=16 if deep else 8)


def approx_level1(p: GcProblem, cost, block: int, opts: GcSolveOpts | None = None, stream=None,
                  ws=None, ws_coarse=None, level: int = 1, wave_steps: int | None = None):
    """Delegate-point cut, then the cut inside the thin skin (built compact,
    graph_build_skin; ws, if given, holds at least skin_footprint_bytes):
    exact (level 1) or block by block after a wave-front pass (level 2).  Returns (labels,
    energy, flow, coarse labels, (coarse stats, fine stats)); level 2 has
    flow -1 and no fine stats."""
    import torch
    dev = cost.device
    if opts is None:
        opts = approx_solve_opts(p)
    c = coarse_problem(p, block)
    ccost = torch.empty((c.labels, c.height, c.width), dtype=torch.int32, device=dev)
    clab = torch.empty((c.height, c.width), dtype=torch.int32, device=dev)
    cres = torch.zeros(2, dtype=torch.int64, device=dev)
    if ws_coarse is None:
        ws_coarse = alloc_workspace(c, dev)
    coarse_cost_volume(p, cost, block, ccost, stream)
    gcoarse = graph_build(c, ccost, ws_coarse, stream)
    st_c = maxflow_solve(gcoarse, opts, stream)
    extract_labels(gcoarse, ccost, clab, cres, stream)
    if ws is None:
        ws = alloc_skin_workspace(p, block, dev)
    labels = torch.empty((p.height, p.width), dtype=torch.int32, device=dev)
    res = torch.zeros(2, dtype=torch.int64, device=dev)
    gfine = graph_build_skin(p, cost, clab, block, ws, stream)
    if level == 1:
        st_f = maxflow_solve(gfine, opts, stream)
        extract_labels(gfine, cost, labels, res, stream)
    else:
        st_f = None
        approx_level2_cut(gfine, cost, clab, labels, res, stream, wave_steps)
    r = res.cpu()
    return labels, int(r[0]), int(r[1]), clab, (st_c, st_f)


def graph_warm_start(graph: Graph, skin: Graph, cost, stream=None):
    _check(load().graph_warm_start(ctypes.byref(graph.handle), ctypes.byref(skin.handle),
                                   ctypes.c_void_p(cost.data_ptr()), _stream_ptr(stream)),
           "graph_warm_start")


def solve_warm(p: GcProblem, cost, block: int, opts: GcSolveOpts | None = None, stream=None,
               ws=None, ws_skin=None, ws_coarse=None, approx_opts: GcSolveOpts | None = None,
               compact: bool = True):
    """Exact cut seeded from the level-1 approximation: delegate-point cut,
    thin-skin cut (a compact skin, or with compact=False one in the full
    layout), then the full graph warm-started from the skin's state and
    solved exactly.  Returns (labels, energy, flow, (coarse, skin, full
    stats), the solved full graph)."""
    import torch
    dev = cost.device
    if approx_opts is None:
        approx_opts = approx_solve_opts(p)
    c = coarse_problem(p, block)
    ccost = torch.empty((c.labels, c.height, c.width), dtype=torch.int32, device=dev)
    clab = torch.empty((c.height, c.width), dtype=torch.int32, device=dev)
    cres = torch.zeros(2, dtype=torch.int64, device=dev)
    if ws_coarse is None:
        ws_coarse = alloc_workspace(c, dev)
    if ws_skin is None:
        ws_skin = alloc_skin_workspace(p, block, dev) if compact else alloc_workspace(p, dev)
    if ws is None:
        ws = alloc_workspace(p, dev)
    coarse_cost_volume(p, cost, block, ccost, stream)
    gcoarse = graph_build(c, ccost, ws_coarse, stream)
    st_c = maxflow_solve(gcoarse, approx_opts, stream)
    extract_labels(gcoarse, ccost, clab, cres, stream)
    gskin = (graph_build_skin if compact else graph_build_window)(p, cost, clab, block, ws_skin, stream)
    st_s = maxflow_solve(gskin, approx_opts, stream)
    g = graph_build(p, cost, ws, stream)
    graph_warm_start(g, gskin, cost, stream)
    st_f = maxflow_solve(g, opts, stream)
    labels = torch.empty((p.height, p.width), dtype=torch.int32, device=dev)
    res = torch.zeros(2, dtype=torch.int64, device=dev)
    extract_labels(g, cost, labels, res, stream)
    r = res.cpu()
    return labels, int(r[0]), int(r[1]), (st_c, st_s, st_f), g


def approx_level2(p: GcProblem, cost, block: int, opts: GcSolveOpts | None = None, stream=None,
                  ws=None, ws_coarse=None, wave_steps: int | None = None):
    return approx_level1(p, cost, block, opts, stream, ws, ws_coarse, level=2,
                         wave_steps=wave_steps)


# ---------------------------------------------------------------------------
# Batched solve
# ---------------------------------------------------------------------------

def batch_footprint_bytes() -> int:
    return int(load().gc_batch_footprint_bytes())


class Batch:
    """Host handle of a gc_batch over a caller-owned device table."""

    def __init__(self, table_ptr: int, table_bytes: int, opts: GcSolveOpts | None = None,
                 table_owner=None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self._owner = table_owner            # keeps the device table alive
        self._graphs = {}                    # tag -> Graph (keeps workspaces alive)
        _check(self._lib.gc_batch_create(ctypes.c_void_p(table_ptr), ctypes.c_size_t(table_bytes),
                                         ctypes.byref(opts) if opts is not None else None,
                                         ctypes.byref(self._h)), "gc_batch_create")

    @classmethod
    def on_device(cls, opts: GcSolveOpts | None = None, device="cuda"):
        import torch
        t = torch.empty(batch_footprint_bytes(), dtype=torch.uint8, device=device)
        return cls(t.data_ptr(), t.numel(), opts, table_owner=t)

    def close(self):
        if self._h:
            self._lib.gc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:                    # interpreter shutdown: module globals gone
            pass

    def __len__(self):
        return int(self._lib.gc_batch_members(self._h))

    def add(self, graph: Graph, tag: int):
        _check(self._lib.gc_batch_add(self._h, ctypes.byref(graph.handle), int(tag)), "gc_batch_add")
        self._graphs[int(tag)] = graph

    def round(self, stream=None, max_done: int = GC_BATCH_MAX_GRAPHS):
        """One round; returns [(tag, GcSolveStats)] of the members that finished."""
        tags = (ctypes.c_int64 * max_done)()
        sts = (GcSolveStats * max_done)()
        nd = ctypes.c_int32()
        _check(self._lib.gc_batch_round(self._h, _stream_ptr(stream), tags, sts, max_done,
                                        ctypes.byref(nd)), "gc_batch_round")
        out = []
        for i in range(nd.value):
            self._graphs.pop(int(tags[i]), None)
            out.append((int(tags[i]), sts[i]))
        return out


def maxflow_solve_batch(graphs, opts: GcSolveOpts | None = None, stream=None, table=None):
    """Solves a list of built graphs together (concurrent lanes, or merged
    rounds with GC_OPT_BATCH_MERGED); returns their stats in order."""
    import torch
    n = len(graphs)
    arr = (ctypes.POINTER(GcGraph) * max(1, n))(*[ctypes.pointer(g.handle) for g in graphs])
    merged = opts is not None and bool(opts.flags & GC_OPT_BATCH_MERGED)
    if table is None and merged:                     # one table per engine
        table = torch.empty(GC_BATCH_ENGINES * batch_footprint_bytes(), dtype=torch.uint8, device="cuda")
    ptr, size = (table.data_ptr(), table.numel()) if table is not None else (None, 0)
    sts = (GcSolveStats * max(1, n))()
    _check(load().maxflow_solve_batch(arr, n, ctypes.c_void_p(ptr), ctypes.c_size_t(size),
                                      ctypes.byref(opts) if opts is not None else None, sts,
                                      _stream_ptr(stream)), "maxflow_solve_batch")
    return [sts[i] for i in range(n)]

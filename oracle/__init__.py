"""CPU oracle for the gaze-line stereo graph cut -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.  ``gazeoracle.c`` holds the arithmetic (plain C,
64-bit integers); this module only marshals numpy arrays through ctypes.

Functions follow the paper (Oguri & Shibata, arXiv 1803.01516):
  cost_volume      data term at every cross point          (Sec. 4.3, Sec. 3)
  energy           E(X) = sum g_v(X_v) + sum h~(X_u - X_v)  (Sec. 2, Sec. 3)
  solve            exact minimiser via max-flow on the layered graph, with the
                   canonical (minimal source side) labelling
  brute_force      every labelling of a tiny grid
  scanline_dp      exact dynamic programming for one-row images
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gazeoracle.c")
_LIB_PATH = os.path.join(_HERE, "libgazeoracle.so")
_lib = None

ORC_OK = 0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (host code only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    lib.orc_cost_volume.argtypes = [P, P, I, I, I, I, P]
    lib.orc_cost_volume.restype = I
    lib.orc_cost_volume_rgb.argtypes = [P, P, I, I, I, I, P]
    lib.orc_cost_volume_rgb.restype = I
    lib.orc_energy.argtypes = [P, P, I, I, I, I, I, I, I]
    lib.orc_energy.restype = I64
    lib.orc_graph_build.argtypes = [P, I, I, I, I, I, I, I]
    lib.orc_graph_build.restype = P
    lib.orc_graph_free.argtypes = [P]
    lib.orc_graph_free.restype = None
    lib.orc_graph_nodes.argtypes = [P]
    lib.orc_graph_nodes.restype = ctypes.c_int32
    lib.orc_graph_arcs.argtypes = [P]
    lib.orc_graph_arcs.restype = I64
    lib.orc_cut_capacity.argtypes = [P, P]
    lib.orc_cut_capacity.restype = I64
    lib.orc_maxflow_dinic.argtypes = [P, P]
    lib.orc_maxflow_dinic.restype = I
    lib.orc_maxflow_pushrelabel.argtypes = [P, P, P]
    lib.orc_maxflow_pushrelabel.restype = I
    lib.orc_labels_after_flow.argtypes = [P, P]
    lib.orc_labels_after_flow.restype = I
    lib.orc_labels_after_preflow.argtypes = [P, P, P]
    lib.orc_labels_after_preflow.restype = I
    lib.orc_labels_max_side.argtypes = [P, P]
    lib.orc_labels_max_side.restype = I
    lib.orc_check_flow.argtypes = [P, P]
    lib.orc_check_flow.restype = I
    lib.orc_solve.argtypes = [P, I, I, I, I, I, I, I, I, P, P, P]
    lib.orc_solve.restype = I
    lib.orc_brute_force.argtypes = [P, I, I, I, I, I, I, I, P, P, P, P]
    lib.orc_brute_force.restype = I
    lib.orc_scanline_dp.argtypes = [P, I, I, I, I, P, P]
    lib.orc_scanline_dp.restype = I
    lib.orc_solve_window.argtypes = [P, I, I, I, I, I, I, I, P, P, I, P, P, P]
    lib.orc_solve_window.restype = I
    lib.orc_coarse_cost.argtypes = [P, I, I, I, I, P]
    lib.orc_coarse_cost.restype = I
    lib.orc_skin_windows.argtypes = [P, I, I, I, I, P, P]
    lib.orc_skin_windows.restype = I
    lib.orc_approx_level1.argtypes = [P, I, I, I, I, I, I, I, I, P, P, P]
    lib.orc_approx_level1.restype = I
    lib.orc_brute_force_window.argtypes = [P, I, I, I, I, I, I, I, P, P, P, P]
    lib.orc_brute_force_window.restype = I
    lib.orc_approx_level2.argtypes = [P, I, I, I, I, I, I, I, I, I, P, P, P]
    lib.orc_approx_level2.restype = I
    lib.orc_level2_skin.argtypes = [P, I, I, I, I, I, I, I, P, P, I, I, I, P, P, P, P]
    lib.orc_level2_skin.restype = I
    lib.orc_solve_window_max_side.argtypes = [P, I, I, I, I, I, I, I, P, P, P, P]
    lib.orc_solve_window_max_side.restype = I
    lib.orc_graph_push.argtypes = [P, I64, I64]
    lib.orc_graph_push.restype = None
    lib.orc_graph_find_arc.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.orc_graph_find_arc.restype = I64
    lib.orc_certify_state.argtypes = [P, I, I, I, I, I, I, I, P, P, P, P, P]
    lib.orc_certify_state.restype = I
    lib.orc_graph_export_state.argtypes = [P, P, P, P]
    lib.orc_graph_export_state.restype = I
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != ORC_OK:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def cost_volume(left: np.ndarray, right: np.ndarray, m: int, cap: int) -> np.ndarray:
    """int32 [m][h][w]; truncated absolute difference per cross point."""
    left = np.ascontiguousarray(left, dtype=np.uint8)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    h, w = left.shape
    out = np.empty((m, h, w), dtype=np.int32)
    _check(_load().orc_cost_volume(_ptr(left), _ptr(right), w, h, m, cap, _ptr(out)),
           "cost_volume")
    return out


def cost_volume_rgb(left: np.ndarray, right: np.ndarray, m: int, cap: int) -> np.ndarray:
    """int32 [m][h][w]; colour sum of absolute differences per cross point
    (images uint8 [h][w][3])."""
    left = np.ascontiguousarray(left, dtype=np.uint8)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    if left.ndim != 3 or left.shape[2] != 3 or right.shape != left.shape:
        raise ValueError("colour images must be [h][w][3] and of equal shape")
    h, w = left.shape[:2]
    out = np.empty((m, h, w), dtype=np.int32)
    _check(_load().orc_cost_volume_rgb(_ptr(left), _ptr(right), w, h, m, cap, _ptr(out)),
           "cost_volume_rgb")
    return out


def _params(pen_h, inh_h, pen_v, inh_v):
    pv = pen_h if pen_v is None else pen_v
    iv = inh_h if inh_v is None else inh_v
    return int(pen_h), int(inh_h), int(pv), int(iv)


def energy(cost: np.ndarray, labels: np.ndarray, pen_h: int, inh_h: int,
           pen_v: int | None = None, inh_v: int | None = None) -> int:
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    m, h, w = cost.shape
    return int(_load().orc_energy(_ptr(cost), _ptr(labels), w, h, m,
                                  *_params(pen_h, inh_h, pen_v, inh_v)))


class Graph:
    """The explicit layered graph (arc pairs with residuals)."""

    def __init__(self, cost: np.ndarray, pen_h: int, inh_h: int,
                 pen_v: int | None = None, inh_v: int | None = None):
        self.cost = np.ascontiguousarray(cost, dtype=np.int32)
        self.m, self.h, self.w = self.cost.shape
        self._lib = _load()
        self._g = self._lib.orc_graph_build(_ptr(self.cost), self.w, self.h, self.m,
                                            *_params(pen_h, inh_h, pen_v, inh_v))
        if not self._g:
            raise MemoryError("oracle graph build failed")

    def close(self):
        if self._g:
            self._lib.orc_graph_free(self._g)
            self._g = None

    def __del__(self):
        self.close()

    @property
    def nodes(self) -> int:
        return int(self._lib.orc_graph_nodes(self._g))

    @property
    def arcs(self) -> int:
        return int(self._lib.orc_graph_arcs(self._g))

    def cut_capacity(self, labels: np.ndarray) -> int:
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        return int(self._lib.orc_cut_capacity(self._g, _ptr(labels)))

    def maxflow_dinic(self) -> int:
        f = np.zeros(1, dtype=np.int64)
        _check(self._lib.orc_maxflow_dinic(self._g, _ptr(f)), "dinic")
        return int(f[0])

    def maxflow_pushrelabel(self) -> tuple[int, np.ndarray]:
        f = np.zeros(1, dtype=np.int64)
        ex = np.zeros(self.nodes, dtype=np.int64)
        _check(self._lib.orc_maxflow_pushrelabel(self._g, _ptr(f), _ptr(ex)), "push-relabel")
        return int(f[0]), ex

    def labels_after_flow(self) -> np.ndarray:
        lab = np.empty((self.h, self.w), dtype=np.int32)
        _check(self._lib.orc_labels_after_flow(self._g, _ptr(lab)), "labels_after_flow")
        return lab

    def labels_after_preflow(self, excess: np.ndarray) -> np.ndarray:
        lab = np.empty((self.h, self.w), dtype=np.int32)
        excess = np.ascontiguousarray(excess, dtype=np.int64)
        _check(self._lib.orc_labels_after_preflow(self._g, _ptr(excess), _ptr(lab)),
               "labels_after_preflow")
        return lab

    def labels_max_side(self) -> np.ndarray:
        lab = np.empty((self.h, self.w), dtype=np.int32)
        _check(self._lib.orc_labels_max_side(self._g, _ptr(lab)), "labels_max_side")
        return lab

    def find_arc(self, u: int, v: int) -> int:
        return int(self._lib.orc_graph_find_arc(self._g, int(u), int(v)))

    def push(self, arc: int, delta: int):
        """Moves delta along an arc with no feasibility check (for checker tests)."""
        self._lib.orc_graph_push(self._g, int(arc), int(delta))

    def node(self, x: int, y: int, k: int) -> int:
        """Node id of level k (1..m-1) of site (x, y); 0 is s, 1 is t."""
        return 2 + ((k - 1) * self.h + y) * self.w + x

    def export_state(self, excess: np.ndarray | None = None):
        """(balances int32 [m-1][h][w], words int32 [7][m-1][h][w]) of the
        current flow or preflow in the overflow form (see certify_state)."""
        ex = np.zeros((self.m - 1, self.h, self.w), dtype=np.int32)
        words = np.zeros((7, self.m - 1, self.h, self.w), dtype=np.int32)
        exa = None if excess is None else np.ascontiguousarray(excess, dtype=np.int64)
        _check(self._lib.orc_graph_export_state(self._g, None if exa is None else _ptr(exa),
                                                _ptr(ex), _ptr(words)), "export_state")
        return ex, words

    def check_flow(self, excess: np.ndarray | None = None) -> int:
        if excess is None:
            return int(self._lib.orc_check_flow(self._g, None))
        excess = np.ascontiguousarray(excess, dtype=np.int64)
        return int(self._lib.orc_check_flow(self._g, _ptr(excess)))


def solve(cost: np.ndarray, pen_h: int, inh_h: int, pen_v: int | None = None,
          inh_v: int | None = None, algo: str = "pushrelabel"):
    """Exact minimiser.  Returns (labels int32 [h][w], flow, energy)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lab = np.empty((h, w), dtype=np.int32)
    f = np.zeros(1, dtype=np.int64)
    e = np.zeros(1, dtype=np.int64)
    a = {"dinic": 0, "pushrelabel": 1}[algo]
    _check(_load().orc_solve(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                             a, _ptr(lab), _ptr(f), _ptr(e)), "solve")
    return lab, int(f[0]), int(e[0])


def brute_force(cost: np.ndarray, pen_h: int, inh_h: int, pen_v: int | None = None,
                inh_v: int | None = None):
    """Returns (min energy, number of minimisers, pointwise-min, pointwise-max)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lo = np.empty((h, w), dtype=np.int32)
    hi = np.empty((h, w), dtype=np.int32)
    e = np.zeros(1, dtype=np.int64)
    n = np.zeros(1, dtype=np.int64)
    _check(_load().orc_brute_force(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                                   _ptr(e), _ptr(n), _ptr(lo), _ptr(hi)), "brute_force")
    return int(e[0]), int(n[0]), lo, hi


def scanline_dp(cost: np.ndarray, pen: int, inh: int):
    """One-row images only.  Returns (min energy, canonical labels [1][w])."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    if h != 1:
        raise ValueError("scanline_dp needs a one-row cost volume")
    lab = np.empty((1, w), dtype=np.int32)
    e = np.zeros(1, dtype=np.int64)
    _check(_load().orc_scanline_dp(_ptr(cost), w, m, int(pen), int(inh), _ptr(e), _ptr(lab)),
           "scanline_dp")
    return int(e[0]), lab


# ---------------------------------------------------------------------------
# Label windows and the hierarchical approximation (Sec. 4.5, level 1)
# ---------------------------------------------------------------------------

def solve_window(cost: np.ndarray, lo: np.ndarray, hi: np.ndarray, pen_h: int, inh_h: int,
                 pen_v: int | None = None, inh_v: int | None = None, algo: str = "pushrelabel"):
    """Exact minimiser of E with lo <= X <= hi per site.  Returns (labels, flow, energy)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    hi = np.ascontiguousarray(hi, dtype=np.int32)
    lab = np.empty((h, w), dtype=np.int32)
    f = np.zeros(1, dtype=np.int64)
    e = np.zeros(1, dtype=np.int64)
    a = {"dinic": 0, "pushrelabel": 1}[algo]
    _check(_load().orc_solve_window(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                                    _ptr(lo), _ptr(hi), a, _ptr(lab), _ptr(f), _ptr(e)),
           "solve_window")
    return lab, int(f[0]), int(e[0])


def coarse_cost(cost: np.ndarray, b: int) -> np.ndarray:
    """Delegate-point data term: int32 [ceil(m/b)][ceil(h/b)][ceil(w/b)]."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    out = np.empty((-(-m // b), -(-h // b), -(-w // b)), dtype=np.int32)
    _check(_load().orc_coarse_cost(_ptr(cost), w, h, m, int(b), _ptr(out)), "coarse_cost")
    return out


def skin_windows(coarse_labels: np.ndarray, w: int, h: int, m: int, b: int):
    cl = np.ascontiguousarray(coarse_labels, dtype=np.int32)
    lo = np.empty((h, w), dtype=np.int32)
    hi = np.empty((h, w), dtype=np.int32)
    _check(_load().orc_skin_windows(_ptr(cl), w, h, m, int(b), _ptr(lo), _ptr(hi)), "skin_windows")
    return lo, hi


def approx_level1(cost: np.ndarray, b: int, pen_h: int, inh_h: int, pen_v: int | None = None,
                  inh_v: int | None = None):
    """Returns (labels, energy, coarse labels)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lab = np.empty((h, w), dtype=np.int32)
    cl = np.empty((-(-h // b), -(-w // b)), dtype=np.int32)
    e = np.zeros(1, dtype=np.int64)
    _check(_load().orc_approx_level1(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                                     int(b), _ptr(lab), _ptr(e), _ptr(cl)), "approx_level1")
    return lab, int(e[0]), cl


def brute_force_window(cost: np.ndarray, lo: np.ndarray, hi: np.ndarray, pen_h: int, inh_h: int,
                       pen_v: int | None = None, inh_v: int | None = None):
    """Returns (min energy, pointwise-min minimiser) over windowed labellings."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    hi = np.ascontiguousarray(hi, dtype=np.int32)
    lab = np.empty((h, w), dtype=np.int32)
    e = np.zeros(1, dtype=np.int64)
    _check(_load().orc_brute_force_window(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                                          _ptr(lo), _ptr(hi), _ptr(e), _ptr(lab)),
           "brute_force_window")
    return int(e[0]), lab


def approx_level2(cost: np.ndarray, b: int, pen_h: int, inh_h: int, pen_v: int | None = None,
                  inh_v: int | None = None, wave_steps: int = 64):
    """Level-2 approximation (Sec. 4.5).  Returns (labels, energy, coarse labels)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lab = np.empty((h, w), dtype=np.int32)
    cl = np.empty((-(-h // b), -(-w // b)), dtype=np.int32)
    e = np.zeros(1, dtype=np.int64)
    _check(_load().orc_approx_level2(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                                     int(b), int(wave_steps), _ptr(lab), _ptr(e), _ptr(cl)),
           "approx_level2")
    return lab, int(e[0]), cl


def level2_skin(cost: np.ndarray, lo: np.ndarray, hi: np.ndarray, b: int, wave_steps: int,
                pen_h: int, inh_h: int, pen_v: int | None = None, inh_v: int | None = None,
                blocks: bool = True):
    """Level-2 cut inside given windows.  Returns (labels, excess, heights, block
    rounds); excess and heights are the state after the wave, before the blocks,
    as int64 [m-1][h][w] (heights >= 2**52 mean unreachable)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    hi = np.ascontiguousarray(hi, dtype=np.int32)
    lab = np.empty((h, w), dtype=np.int32)
    ex = np.zeros((max(m - 1, 0), h, w), dtype=np.int64)
    ht = np.zeros((max(m - 1, 0), h, w), dtype=np.int64)
    rounds = np.zeros(1, dtype=np.int64)
    _check(_load().orc_level2_skin(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                                   _ptr(lo), _ptr(hi), int(b), int(wave_steps), int(bool(blocks)),
                                   _ptr(lab), _ptr(ex), _ptr(ht), _ptr(rounds)), "level2_skin")
    return lab, ex, ht, int(rounds[0])


def solve_window_max_side(cost: np.ndarray, lo: np.ndarray, hi: np.ndarray, pen_h: int,
                          inh_h: int, pen_v: int | None = None, inh_v: int | None = None):
    """Back-most minimiser of E with lo <= X <= hi (maximal source side of a
    Dinic max flow).  Returns (labels, flow)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    hi = np.ascontiguousarray(hi, dtype=np.int32)
    lab = np.empty((h, w), dtype=np.int32)
    f = np.zeros(1, dtype=np.int64)
    _check(_load().orc_solve_window_max_side(_ptr(cost), w, h, m,
                                             *_params(pen_h, inh_h, pen_v, inh_v), _ptr(lo),
                                             _ptr(hi), _ptr(lab), _ptr(f)), "solve_window_max_side")
    return lab, int(f[0])


CERT_CODES = {0: "ok", 1: "residual out of bounds", 2: "conservation", 3: "not a maximum preflow",
              4: "labels differ from the minimal source side", 5: "flow value differs from E(labels)"}


def certify_state(cost: np.ndarray, ex: np.ndarray, words: np.ndarray, labels: np.ndarray,
                  pen_h: int, inh_h: int, pen_v: int | None = None, inh_v: int | None = None):
    """Independent certificate of a solved full graph given in the library's
    exported layout (balances [m-1][h][w], pair words [7][m-1][h][w]).
    Returns (code, flow, energy); code 0 means: capacity bounds and
    conservation hold, no excess reaches a deficit, the labels are the
    minimal source side and max-flow = E(labels)."""
    cost = np.ascontiguousarray(cost, dtype=np.int32)
    m, h, w = cost.shape
    ex = np.ascontiguousarray(ex, dtype=np.int32)
    words = np.ascontiguousarray(words, dtype=np.int32)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    if ex.size != (m - 1) * h * w or words.size != 7 * ex.size or labels.size != h * w:
        raise ValueError("state arrays do not match the cost volume's shape")
    f = np.zeros(1, dtype=np.int64)
    e = np.zeros(1, dtype=np.int64)
    rc = _load().orc_certify_state(_ptr(cost), w, h, m, *_params(pen_h, inh_h, pen_v, inh_v),
                                   _ptr(ex), _ptr(words), _ptr(labels), _ptr(f), _ptr(e))
    if rc < 0:
        raise RuntimeError(f"oracle certify_state failed with status {rc}")
    return rc, int(f[0]), int(e[0])

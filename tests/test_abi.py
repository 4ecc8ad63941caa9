"""CPU-side checks of the C ABI: the library loads, exports every function
include/gazecut.h declares, and its host-only validation behaves.  No
compute call runs here (there is no GPU)."""
import ctypes
import os
import re

import pytest

from paper_1803_01516_amd import gazecut as gc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "gazecut.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt)) - {"sizeof"})


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gc.LIB_PATH)
    names = _declared()
    assert {"stereo_cost_volume", "graph_build", "maxflow_solve", "extract_labels"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(gc.EXPORTS) | {"gc_status_str"}


def test_problem_validation_and_footprint():
    gc.load()
    ok = gc.problem(384, 288, 16, 30, 1, 1023)
    assert gc.problem_check(ok) == 0
    n = 384 * 288 * 15
    fp = gc.footprint_bytes(ok)
    assert fp >= 46 * n and fp < 46 * n + 96 * 1024
    assert gc.problem_check(gc.problem(4, 4, 0, 30, 1, 1023)) == -2      # labels < 1
    assert gc.problem_check(gc.problem(-1, 4, 4, 30, 1, 1023)) == -2
    assert gc.problem_check(gc.problem(4, 4, 4, 30, -1, 1023)) == -1     # eq. (1) needs >= 0
    assert gc.problem_check(gc.problem(4, 4, 4, 30, 1, 1023, 1, -3)) == -1
    big = gc.problem(1 << 14, 1 << 14, 2, 30, 1, 1023)                 # sites*cap >= 2^30
    assert gc.problem_check(big) == -4
    assert gc.footprint_bytes(big) == 0
    assert gc.problem_check(gc.problem(0, 0, 1, 30, 1, 1023)) == 0      # empty is valid
    assert gc.load().gc_status_str(-5).decode().startswith("iteration cap")


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError):
        gc._lib_backup = gc._lib
        gc._lib = None
        try:
            gc.load(str(tmp_path / "missing.so"))
        finally:
            gc._lib = gc._lib_backup

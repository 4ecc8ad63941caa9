import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def certify(orc):
    """certify(graph, cost_np, labels_np, params) reads a solved graph's state
    back (gc_graph_state) and runs the oracle's certificate on it: capacity
    bounds, conservation against the build, no residual path from an excess
    to a deficit, labels = minimal source side, flow value = E(labels).
    Returns the recomputed (flow, energy)."""
    def run(graph, cost_np, labels_np, params):
        import torch
        from paper_1803_01516_amd import gazecut as gc
        ex, words = gc.graph_state(graph)
        torch.cuda.synchronize()
        ex_np, words_np = ex.cpu().numpy(), words.cpu().numpy()
        del ex, words
        code, flow, energy = orc.certify_state(cost_np, ex_np, words_np, labels_np, *params)
        assert code == 0, orc.CERT_CODES[code]
        return flow, energy
    return run

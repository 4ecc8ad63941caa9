"""Writes stored oracle results for workloads too slow to solve inside a test.

Calls only the oracle and the seeded scene generator.  Run from the repo root:
    python tests/golden/make_golden.py [file name ...]
(no argument: every case; the 640x480x64 case takes a few minutes and about
12 GB of host memory in the oracle's explicit graph).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1803_01516_amd import scenegen as sg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [
    # (file, spec, seed, penalty, inhibit)
    ("large_450x375x64_seed3-0_lam1.npz", sg.LARGE, (3, 0), 1, 1023),
    ("mid_640x480x64_seed5-2-0_lam1.npz", sg.spec_like(sg.MID, 640, 480, 64), (5, 2, 0), 1, 1023),
]


def main(only=()):
    for fname, spec, seed, pen, inh in CASES:
        if only and fname not in only:
            continue
        p = sg.make_pair(spec, seed)
        cost = oracle.cost_volume(p.left, p.right, spec.m, spec.cap)
        labels, flow, energy = oracle.solve(cost, pen, inh, algo="pushrelabel")
        assert flow == energy
        np.savez_compressed(os.path.join(HERE, fname), labels=labels.astype(np.uint8),
                            flow=np.int64(flow), energy=np.int64(energy),
                            seed=np.array(seed), penalty=pen, inhibit=inh)
        print(fname, flow, energy, flush=True)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]))

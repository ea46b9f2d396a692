import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on cuda:0)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_tt32x5():
    """The oracle's whole sweep of the 32^5 rank-8 workload (500 MU iterations per stage,
    FP64): stage iterates at t = 1, 100, 500 and the objective of every 10th iterate.
    About half a minute on 16 host cores; computed once per test session."""
    import oracle as O
    import synth as S
    w = S.workload("tt32x5_r8")
    A = w.tensor()
    every = list(range(10, w.iters + 1, 10))
    ref = O.ntt_decompose(A, w.target_ranks, w.iters, eps=w.eps, seed=w.seed,
                          snapshots=(1, 100, w.iters), objective_at=every)
    return {"w": w, "A": A, "ref": ref, "every": every}

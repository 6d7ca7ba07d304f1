"""GPU tests of the autotuner: every candidate it times (engines, threads,
grids; batch engines, LDS residency, queue, planner constants) must give
bitwise the same state and duals, which the tuner asserts itself."""
import numpy as np
import pytest

from paper_2004_08227_amd import workloads as W

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2004_08227_amd")
from paper_2004_08227_amd import autotune as A  # noqa: E402


def _announce(*a):
    print("CASE", *a, flush=True)


@pytest.mark.parametrize("make", [lambda: W.pose(40, 20, seed=3), lambda: W.tiny(1, n=12, L=6)],
                         ids=["pose_fp32", "tiny_fp64"])
def test_solver_tuner_candidates_agree(make):
    _announce("solver tuner")
    model = make()
    opts, times = A.tune_solver(model, iters=4)
    assert len(times) >= 4
    assert json_key(opts) in times


def json_key(opts):
    import json
    return json.dumps(opts, sort_keys=True)


def test_batch_tuner_candidates_agree():
    _announce("batch tuner")
    rng = np.random.default_rng(0)
    models = [W.pose(int(rng.integers(8, 60)), int(rng.choice([5, 13, 16, 33, 64])), seed=10 + i) for i in range(10)]
    opts, ms, ms0 = A.tune_batch(models, iters=3, rounds=1)
    assert ms <= ms0
    assert set(opts) <= set(A.BATCH_CHOICES)

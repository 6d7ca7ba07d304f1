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


def test_solve_batch_tuned_and_untuned_agree():
    _announce("solve_batch")
    models = [W.pose(30, 13, seed=1), W.pose(18, 40, seed=2), W.potts_er(50, 9, 0.3, seed=3)]
    table = {A.batch_key(models): {"options": {"queue": 0, "wave_lat_mb_us": 4.0}, "workload": "test"}}
    d0, s0 = M.solve_batch(models, 5, tuned=False, states=True)
    with M.Batch(models) as b:
        assert A.apply_batch(b, models, table) == {"queue": 0, "wave_lat_mb_us": 4.0}
        b.iterate(5)
        d1 = b.dual_bounds()
        s1 = [b.get_state(i) for i in range(len(models))]
    d2 = M.solve_batch(models, 5)
    assert np.array_equal(d0, d1) and np.array_equal(d0, d2)
    for (a, b), (c, e) in zip(s0, s1):
        assert np.array_equal(a, c) and np.array_equal(b, e)

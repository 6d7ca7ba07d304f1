"""Host logic of the autotuner: table keys, the committed table's shape, and
that applying an entry sets exactly its options (no device work)."""
import json
import os

import numpy as np
import pytest

from paper_2004_08227_amd import autotune as A
from paper_2004_08227_amd import workloads as W


def test_keys_bucket_by_tile_and_size():
    assert A.next_tile(1) == 16 and A.next_tile(17) == 32 and A.next_tile(64) == 64 and A.next_tile(65) == 128
    with pytest.raises(ValueError):
        A.next_tile(129)
    k1 = A.solver_key(np.float32, 64, 200, 19900)
    k2 = A.solver_key(np.float32, 40, 255, 255 * 254 // 2)
    k3 = A.solver_key(np.float64, 64, 200, 19900)
    assert k1 == k2 != k3
    assert k1.startswith("solver/f32/lt64/n7/")
    a = [W.pose(20, 8, seed=i, dtype=np.float32, ) for i in range(3)]
    assert A.batch_key(a).startswith("batch/lt16/models1/")


def test_committed_table_entries_are_well_formed():
    table = A.load_table()
    if not table:
        pytest.skip("no tuned table committed")
    from paper_2004_08227_amd import BOPT
    import paper_2004_08227_amd as M
    for key, entry in table.items():
        assert set(entry) >= {"options", "workload"}, key
        if key.startswith("solver/"):
            for k in entry["options"]:
                assert hasattr(M, k) and k.startswith("OPT_"), (key, k)
        else:
            assert key.startswith("batch/")
            for k in entry["options"]:
                assert k in BOPT and k in A.BATCH_CHOICES, (key, k)


class _Fake:
    def __init__(self, dtype=np.float32):
        self.dtype = dtype
        self.set = []

    def set_option(self, k, v):
        self.set.append((k, v))


def test_apply_sets_exactly_the_entry():
    import paper_2004_08227_amd as M
    model = W.pose(30, 13, seed=1)
    key = A.solver_key(np.float32, model.L, model.n, model.m)
    table = {key: {"options": {"OPT_THREADS": 512, "OPT_GRID": 128}, "workload": "x"}}
    f = _Fake()
    assert A.apply_solver(f, model, table) == {"OPT_THREADS": 512, "OPT_GRID": 128}
    assert sorted(f.set) == sorted([(M.OPT_THREADS, 512), (M.OPT_GRID, 128)])
    assert A.apply_solver(_Fake(np.float64), model, table) == {}
    models = [model]
    bt = {A.batch_key(models): {"options": {"queue": 0}, "workload": "x"}}
    g = _Fake()
    assert A.apply_batch(g, models, bt) == {"queue": 0} and g.set == [("queue", 0)]

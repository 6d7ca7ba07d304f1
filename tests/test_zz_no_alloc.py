"""GPU test of mplpxx_solve_noalloc, the entry point that allocates no
device memory: through the C ABI it must give bitwise the state and dual
bound of the allocating calls (mplpxx_create_device + mplpxx_iterate +
mplpxx_get_state + mplpxx_dual_bound) on the same model, on two calls in a
row, the second with a smaller model (the shared working array still holds
the first call's contents), and reject a model too large for its array."""
import numpy as np
import pytest

import paper_2004_08227_amd as M
from paper_2004_08227_amd import workloads as W

pytestmark = pytest.mark.gpu


def _announce(*a):
    print("CASE", *a, flush=True)


def _allocating(model, iters):
    import torch
    un = torch.from_numpy(model.unaries).cuda()
    pw = torch.from_numpy(model.pairwise).cuda()
    with M.Solver.from_torch(model.n, model.L, model.edges, un, pw) as s:
        s.iterate(iters)
        U, phi = s.get_state()
        d = s.dual_bound()
    return U, phi, d


def _noalloc(model, iters):
    import torch
    un = torch.from_numpy(model.unaries).cuda()
    pw = torch.from_numpy(model.pairwise).cuda()
    U = torch.full((model.n, model.L), float("nan"), device="cuda")
    phi = torch.full((model.m, 2, model.L), float("nan"), device="cuda")
    torch.cuda.synchronize()
    d = M.solve_noalloc(model.edges, un, pw, iters, U, phi)
    return U.cpu().numpy(), phi.cpu().numpy(), d


def test_noalloc_equals_allocating_calls_on_two_calls_in_a_row():
    big = W.uniform(100, 32, seed=0)             # the differentiation workload's size
    small = W.pose(24, 13, seed=1)               # ragged label count
    flip = W.Model(small.n, small.L, small.edges[:, ::-1].copy(), small.unaries,
                   np.transpose(small.pairwise, (0, 2, 1)).copy())
    for model, iters in ((big, 10), (small, 7), (flip, 7)):
        _announce("noalloc", model.n, model.L, iters)
        got = _noalloc(model, iters)
        ref = _allocating(model, iters)
        assert np.array_equal(got[0], ref[0]), "U differs"
        assert np.array_equal(got[1], ref[1]), "phi differs"
        assert got[2] == ref[2], (got[2], ref[2])


def test_noalloc_rejects_a_model_larger_than_its_array():
    import torch
    _announce("noalloc too large")
    n, L = 60, 128                                # 116 MB of tables
    rng = np.random.default_rng(0)
    edges = W.complete_edges(n)
    un = torch.from_numpy(rng.random((n, L), dtype=np.float32)).cuda()
    pw = torch.from_numpy(rng.random((edges.shape[0], L, L), dtype=np.float32)).cuda()
    U = torch.empty((n, L), device="cuda")
    phi = torch.empty((edges.shape[0], 2, L), device="cuda")
    with pytest.raises(M.MplpError) as ei:
        M.solve_noalloc(edges, un, pw, 1, U, phi)
    assert ei.value.code == M.EINVAL and "working memory" in str(ei.value)

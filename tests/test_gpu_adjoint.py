"""GPU tests of the adjoint of K unrolled MPLP++ iterations.

D_K is piecewise linear in the costs.  The reference is the oracle's
forward-mode derivative of its own FP64 run (``oracle.dual_derivative``,
pinned against one-piece finite differences, closed forms and Euler's and
Danskin's theorems in test_oracle_derivative.py).  The FP64 adjoint must
match it coordinate by coordinate on a small model, with no misses.  On
the differentiation workload (n=100, L=32, K=50, checkpoints every 10) the
gradient of an FP32 handle (by default that of its exactly widened FP64
twin run) must match the stored oracle derivatives along 16 dense and 16
sparse seeded directions and 64 coordinates to 1e-4 relative, every one of
them; how far the FP32 run's own gradient sits is printed and bounded.
Checkpoint spacing must not change a bit."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2004_08227_amd import workloads as W

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2004_08227_amd")
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _announce(*a):
    print("CASE", *a, flush=True)


def _grad(model, K, every, adjoint_f64=1):
    with M.Solver.from_model(model) as s:
        s.set_option(M.OPT_ADJOINT_F64, adjoint_f64)
        loss = s.adjoint_forward(K, every)
        gu, gp = s.adjoint_backward()
    return loss, gu, gp


def _coord(model, idx, unary):
    du = np.zeros(model.unaries.shape)
    dp = np.zeros(model.pairwise.shape)
    (du if unary else dp)[idx] = 1.0
    return du, dp


def test_fp64_adjoint_matches_oracle_derivative_per_coordinate():
    _announce("fp64 adjoint all coordinates")
    model = W.uniform(9, 4, seed=21, dtype=np.float64)
    K, every = 6, 2
    loss, gu, gp = _grad(model, K, every)
    st, tr = oracle.run_model(model, K)
    assert abs(loss - st.dual()) <= 1e-12 * max(1, abs(loss))
    worst = 0.0
    for arr, g, unary in ((model.unaries, gu, True), (model.pairwise, gp, False)):
        for idx in np.ndindex(arr.shape):
            ref = oracle.dual_derivative(model, K, *_coord(model, idx, unary))
            worst = max(worst, abs(g[idx] - ref))
    print("fp64 adjoint vs oracle derivative, all", gu.size + gp.size, "coordinates: worst", worst, flush=True)
    assert worst <= 1e-10


def test_checkpoint_spacing_and_repeats_are_bitwise_identical():
    for dtype, f64 in ((np.float64, 1), (np.float32, 1), (np.float32, 0)):
        model = W.uniform(14, 6, seed=22, dtype=dtype)
        _announce("checkpoints", dtype.__name__, f64)
        ref = None
        for every in (1, 3, 7, 10):
            loss, gu, gp = _grad(model, 7, every, f64)
            if ref is None:
                ref = (loss, gu, gp)
            else:
                assert loss == ref[0] and np.array_equal(gu, ref[1]) and np.array_equal(gp, ref[2])


def _reference_errors(gu, gp, g, base):
    """Relative errors |<grad, v> - dD/dv| / max(1, |dD/dv|) against the
    stored oracle derivatives, per family of directions."""
    import sys
    sys.path.insert(0, GOLD)
    import make_golden as MG
    gu64, gp64 = gu.astype(np.float64), gp.astype(np.float64)
    out = {}
    for name, dirs in (("dense", MG.adjoint_directions(base, g["dense"]["count"], g["dense"]["seed"])),
                       ("sparse", MG.adjoint_sparse_directions(base, g["sparse"]["count"], g["sparse"]["seed"],
                                                               g["sparse"]["support"]))):
        out[name] = [abs(float((gu64 * du).sum() + (gp64 * dp).sum()) - ref) / max(1.0, abs(ref))
                     for (du, dp), ref in zip(dirs, g[name]["tangent"])]
    flat = np.concatenate([gu64.ravel(), gp64.ravel()])
    out["coords"] = [abs(float(flat[c]) - ref) / max(1.0, abs(ref))
                     for c, ref in zip(g["coords"]["index"], g["coords"]["tangent"])]
    return out


def test_fp32_adjoint_matches_oracle_derivatives_full_size():
    """The differentiation workload (n=100, L=32, K=50, checkpoints every 10)
    on an FP32 handle: loss and gradient (of the FP64 twin run, the default)
    against the oracle's derivatives of D_50 along 16 dense and 16 sparse
    seeded directions and 64 coordinates (three quarters of them on the
    gradient's support): every one within 1e-4 relative."""
    path = os.path.join(GOLD, "adjoint_uniform_k100_l32.json")
    g = json.load(open(path))
    _announce("fp32 adjoint n=100 L=32 K=50")
    model = W.uniform(100, 32, seed=0)
    loss, gu, gp = _grad(model, g["K"], g["every"])
    assert abs(loss - g["D"]) <= 1e-5 * abs(g["D"])
    base = model.astype(np.float64)
    errs = _reference_errors(gu, gp, g, base)
    nz = sum(1 for c, ref in zip(g["coords"]["index"], g["coords"]["tangent"]) if ref != 0.0)
    for name, e in errs.items():
        print(f"{name}: {len(e)} checks, worst relative error {max(e):.3e}", flush=True)
    print("coordinates with a nonzero reference:", nz, flush=True)
    bad = {name: [(k, x) for k, x in enumerate(e) if x > 1e-4] for name, e in errs.items()}
    assert not any(bad.values()), bad


def test_fp32_run_adjoint_is_close_to_the_fp64_twin():
    """The gradient of the FP32 run itself (OPT_ADJOINT_F64 = 0) picks a
    neighbouring linear piece for the minimizers that FP32 rounding flips;
    it stays within a few percent of the FP64 twin's gradient, and its loss
    within 1e-5 of the oracle's.  Its errors against the oracle's
    derivatives are printed."""
    path = os.path.join(GOLD, "adjoint_uniform_k100_l32.json")
    g = json.load(open(path))
    _announce("fp32-run adjoint vs fp64 twin")
    model = W.uniform(100, 32, seed=0)
    l32, gu32, gp32 = _grad(model, g["K"], g["every"], 0)
    l64, gu64, gp64 = _grad(model, g["K"], g["every"], 1)
    assert abs(l32 - g["D"]) <= 1e-5 * abs(g["D"])
    a = np.concatenate([gu32.ravel(), gp32.ravel()]).astype(np.float64)
    b = np.concatenate([gu64.ravel(), gp64.ravel()]).astype(np.float64)
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    print("fp32-run vs fp64-twin gradient: rel L2", rel, "entries equal", float(np.mean(a == b)), flush=True)
    for name, e in _reference_errors(gu32, gp32, g, model.astype(np.float64)).items():
        print(f"fp32-run gradient vs oracle, {name}: median {np.median(e):.2e}, worst {max(e):.2e}", flush=True)
    assert rel <= 3e-2


def test_orientation_and_degenerate_models():
    _announce("adjoint orientation/degenerate")
    model = W.uniform(7, 3, seed=23, dtype=np.float64)
    flip = W.Model(model.n, model.L, model.edges[:, ::-1].copy(), model.unaries,
                   np.transpose(model.pairwise, (0, 2, 1)).copy())
    la, gua, gpa = _grad(model, 4, 2)
    lb, gub, gpb = _grad(flip, 4, 2)
    assert la == lb and np.array_equal(gua, gub)
    assert np.array_equal(gpa, np.transpose(gpb, (0, 2, 1)))
    # no edges: D = sum_u min theta_u, gradient = one-hot at the smallest minimizer
    un = np.array([[0.5, 0.25, 0.25], [1.0, 2.0, 0.0]], np.float64)
    m0 = W.Model(2, 3, np.zeros((0, 2), np.int32), un, np.zeros((0, 3, 3)))
    loss, gu, gp = _grad(m0, 3, 2)
    assert loss == 0.25 and np.array_equal(gu, [[0, 1, 0], [0, 0, 1]])


def test_backward_requires_a_forward():
    _announce("adjoint state")
    model = W.uniform(6, 3, seed=24)
    with M.Solver.from_model(model) as s:
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_backward()
        assert ei.value.code == M.ESTATE
        s.adjoint_forward(3, 1)
        s.iterate(1)
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_backward()
        assert ei.value.code == M.ESTATE


@pytest.mark.parametrize("dtype,f64", [(np.float64, 1), (np.float32, 1), (np.float32, 0)])
def test_adjoint_allocation_failure_is_reported(dtype, f64):
    """Records for 2^31 - 1 iterations per segment need terabytes: the
    forward fails in hipMalloc before any kernel runs (MPLPXX_ENOMEM), the
    backward then refuses (no forward to differentiate), and a forward of a
    normal size afterwards gives the gradient of a fresh handle, bit for
    bit."""
    _announce("adjoint allocation failure", dtype.__name__, f64)
    model = W.tiny(5).astype(dtype)
    big = 2**31 - 1
    with M.Solver.from_model(model) as s:
        s.set_option(M.OPT_ADJOINT_F64, f64)
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_forward(big, big)
        assert ei.value.code == M.ENOMEM
        with pytest.raises(M.MplpError) as ei:
            s.adjoint_backward()
        assert ei.value.code == M.ESTATE
        loss = s.adjoint_forward(6, 2)
        gu, gp = s.adjoint_backward()
    with M.Solver.from_model(model) as s2:
        s2.set_option(M.OPT_ADJOINT_F64, f64)
        loss2 = s2.adjoint_forward(6, 2)
        gu2, gp2 = s2.adjoint_backward()
    assert loss == loss2 and np.array_equal(gu, gu2) and np.array_equal(gp, gp2)


def test_autograd_function():
    import torch
    from paper_2004_08227_amd.autograd import mplp_dual
    _announce("autograd")
    model = W.uniform(12, 5, seed=25)
    un = torch.tensor(model.unaries, device="cuda", requires_grad=True)
    pw = torch.tensor(model.pairwise, device="cuda", requires_grad=True)
    loss = mplp_dual(un, pw, model.edges, K=6, every=3)
    (2.0 * loss).backward()
    l2, gu, gp = _grad(model, 6, 3)
    assert float(loss.detach()) == np.float32(l2)
    assert np.array_equal(un.grad.cpu().numpy(), 2.0 * gu)
    assert np.array_equal(pw.grad.cpu().numpy(), 2.0 * gp)


def test_adjoint_memory_is_reported():
    """MPLPXX_INFO_ADJOINT_BYTES after a forward: checkpoints (K/every + 1
    copies of U and phi), one segment of argmin records (3 L bytes per edge
    and iteration), the adjoint buffers, and on the persistent path (FP64,
    L <= 64) a second segment of records, two sets of two-word mailboxes of
    the nodes (16 bytes per label each) and one segment of the reverse
    steps' scatter vectors (3 L doubles per edge and iteration); an FP32 handle differentiating its FP64 twin adds the twin's
    costs and state."""
    _announce("adjoint bytes")
    n, L, K, every = 12, 5, 9, 4
    m64 = W.uniform(n, L, seed=3, dtype=np.float64)
    m = m64.m
    nck = (K + every - 1) // every
    nL, mp = n * L, m * 2 * L
    per_matching = (nck + 1) * nL * 8 + (nck + 1) * mp * 8 + every * m * 3 * L + nL * 8 + mp * 8 + m * L * L * 8 + m * 8
    own64 = per_matching + every * m * 3 * L + 2 * nL * 16 + every * m * 3 * L * 8
    with M.Solver.from_model(m64) as s:
        assert s.info("adjoint_bytes") == 0
        s.adjoint_forward(K, every)
        assert s.info("adjoint_bytes") == own64
    with M.Solver.from_model(m64) as s:
        s.set_option(M.OPT_ENGINE, 1)
        s.adjoint_forward(K, every)
        assert s.info("adjoint_bytes") == per_matching
    m32 = W.uniform(n, L, seed=3, dtype=np.float32)
    with M.Solver.from_model(m32) as s:
        s.set_option(M.OPT_ADJOINT_F64, 1)
        s.adjoint_forward(K, every)
        twin = own64 + nL * 8 * 2 + m * L * L * 8 + mp * 8
        assert s.info("adjoint_bytes") == twin


@pytest.mark.parametrize("n,L,K", [(10, 64, 4), (8, 100, 3), (6, 128, 3)])
def test_fp64_adjoint_at_large_labels(n, L, K):
    """At L up to the library maximum (full and ragged tiles): adding c to
    every label of one node's unary, or to every entry of one edge's table,
    raises D_K by exactly c (the update (H) passes a uniform shift through
    and no argmin moves), so the gradient sums to 1 over each node's L
    entries and over each edge's L x L entries; and up to 32 coordinates, three
    quarters of them where the oracle's final state says the gradient is
    likely nonzero, plus 16 pairwise coordinates where the GPU gradient
    itself is nonzero (a gradient placed at a wrong (s, t) would meet an
    oracle derivative of 0 there), match the oracle's exact derivative with
    no misses, at least 16 of them nonzero."""
    import sys
    sys.path.insert(0, GOLD)
    import make_golden as MG
    _announce("fp64 adjoint large L", n, L, K)
    model = W.uniform(n, L, seed=40 + L, dtype=np.float64)
    loss, gu, gp = _grad(model, K, 1)
    st, _ = oracle.run_model(model, K)
    assert abs(loss - st.dual()) <= 1e-12 * max(1, abs(loss))
    assert np.max(np.abs(gu.sum(axis=1) - 1.0)) <= 1e-9
    assert np.max(np.abs(gp.sum(axis=(1, 2)) - 1.0)) <= 1e-9
    flat = np.concatenate([gu.ravel(), gp.ravel()])
    coords = list(MG.adjoint_coords(model, st.Tu, st.Te, 32, L))
    support = np.flatnonzero(gp.ravel()) + gu.size
    rng = np.random.default_rng(L)
    coords += [int(c) for c in rng.choice(support, size=min(16, support.size), replace=False)]
    worst, nonzero = 0.0, 0
    for c in coords:
        ref = oracle.dual_derivative(model, K, *MG.coord_direction(model, c))
        nonzero += ref != 0.0
        worst = max(worst, abs(float(flat[c]) - ref))
    print(f"L={L}: {len(coords)} coordinates, {nonzero} nonzero references, worst error {worst:.2e}", flush=True)
    assert worst <= 1e-10
    assert nonzero >= 16


@pytest.mark.parametrize("name,make,K,every", [
    ("uniform_n9_L4_fp64", lambda: W.uniform(9, 4, seed=41, dtype=np.float64), 6, 4),
    ("pose_n24_L13_ragged", lambda: W.pose(24, 13, seed=42), 7, 3),
    ("uniform_n30_L32", lambda: W.uniform(30, 32, seed=43), 9, 10),
    ("pose_n20_L33_ragged", lambda: W.pose(20, 33, seed=44), 5, 2),
    ("uniform_n16_L64", lambda: W.uniform(16, 64, seed=45), 4, 3),
    ("er_n40_L16_greedy", lambda: W.potts_er(40, 16, 0.3, seed=46), 6, 4),
    ("single_label_n6", lambda: W.uniform(6, 1, seed=47), 3, 2),
])
def test_persistent_adjoint_equals_per_matching_adjoint(name, make, K, every):
    """The persistent FP64 adjoint (forward, recorded recomputation and
    reverse in one launch per segment, values through tagged mailboxes,
    table adjoints added per slot) gives bitwise the loss and gradients of
    the per-matching kernels (MPLPXX_OPT_ENGINE = 1), for FP64 handles and
    for the FP64 twin of FP32 handles, with ragged tiles, a partial last
    segment, a greedy schedule and a single label."""
    _announce("persistent adjoint vs per-matching", name)
    model = make()
    out = {}
    for engine in (1, 0):
        with M.Solver.from_model(model) as s:
            s.set_option(M.OPT_ENGINE, engine)
            loss = s.adjoint_forward(K, every)
            gu, gp = s.adjoint_backward()
            U, phi = s.get_state()
        out[engine] = (loss, gu, gp, U, phi)
    a, b = out[1], out[0]
    assert a[0] == b[0], (a[0], b[0])
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    print(f"{name}: loss {b[0]:.12g}, |grad_u|_1 {np.abs(b[1]).sum():.6g}, bitwise equal", flush=True)

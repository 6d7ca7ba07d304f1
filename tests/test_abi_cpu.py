"""CPU-side checks of the C-ABI library: it loads without a GPU, exports
every function the header declares, rejects invalid models before any device
work, and its host-only schedule equals the oracle's independently computed
schedule bit for bit."""
import ctypes
import re

import numpy as np
import pytest

import oracle
import paper_2004_08227_amd as M
from paper_2004_08227_amd import workloads as W


def test_library_exports_every_header_symbol():
    lib = M.lib()
    syms = M.header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s


def test_header_constants_match_binding():
    text = open(M.HEADER).read()
    defs = dict(re.findall(r"#define (MPLPXX_\w+)\s+\(?(-?\d+)\)?", text))
    assert int(defs["MPLPXX_F32"]) == M.F32 and int(defs["MPLPXX_F64"]) == M.F64
    assert int(defs["MPLPXX_EINVAL"]) == M.EINVAL and int(defs["MPLPXX_ETIMEOUT"]) == M.ETIMEOUT
    assert int(defs["MPLPXX_ENOMEM"]) == M.ENOMEM and int(defs["MPLPXX_EDEVICE"]) == M.EDEVICE
    assert int(defs["MPLPXX_MAX_LABELS"]) == M.MAX_LABELS
    assert int(defs["MPLPXX_OPT_ENGINE"]) == M.OPT_ENGINE and int(defs["MPLPXX_OPT_SPIN_LIMIT"]) == M.OPT_SPIN_LIMIT
    for k, v in M.INFO.items():
        name = {"n": "N", "L": "L", "m": "M"}.get(k, k.upper())
        assert int(defs[f"MPLPXX_INFO_{name}"]) == v


def test_error_strings():
    lib = M.lib()
    for code in (M.OK, M.EINVAL, M.ENOMEM, M.EDEVICE, M.ETIMEOUT, M.ESTATE):
        assert lib.mplpxx_error_string(code)
    assert lib.mplpxx_error_string(12345) == b"unknown error"


def _create(n, L, edges, un, pw, dtype=M.F32):
    h = ctypes.c_void_p()
    e = None if edges is None else ctypes.c_void_p(edges.ctypes.data)
    u = None if un is None else ctypes.c_void_p(un.ctypes.data)
    p = None if pw is None else ctypes.c_void_p(pw.ctypes.data)
    m = 0 if edges is None else edges.shape[0]
    rc = M.lib().mplpxx_create(n, L, m, e, u, p, dtype, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["n0", "L0", "Lbig", "self", "range", "neg", "dup", "nan_u", "inf_p", "dtype",
                                  "null_u", "too_many"])
def test_invalid_models_rejected_without_device_work(case):
    n, L = 5, 3
    model = W.uniform(n, L, seed=0)
    edges, un, pw, dt = model.edges.copy(), model.unaries.copy(), model.pairwise.copy(), M.F32
    if case == "n0":
        n = 0
    elif case == "L0":
        L = 0
    elif case == "Lbig":
        L = M.MAX_LABELS + 1
    elif case == "self":
        edges[2] = [3, 3]
    elif case == "range":
        edges[2] = [3, 5]
    elif case == "neg":
        edges[0] = [-1, 2]
    elif case == "dup":
        edges[4] = edges[1][::-1]
    elif case == "nan_u":
        un[1, 1] = np.nan
    elif case == "inf_p":
        pw[3, 0, 2] = np.inf
    elif case == "dtype":
        dt = 7
    elif case == "null_u":
        un = None
    elif case == "too_many":
        n = 4                     # 10 edges > 4*3/2
    rc, h = _create(n, L, edges, un, pw, dt)
    assert rc == M.EINVAL and not h.value
    assert M.lib().mplpxx_last_error()


def test_null_out_and_null_handle():
    lib = M.lib()
    model = W.uniform(3, 2, seed=0)
    assert lib.mplpxx_create(3, 2, 3, ctypes.c_void_p(model.edges.ctypes.data), ctypes.c_void_p(model.unaries.ctypes.data),
                             ctypes.c_void_p(model.pairwise.ctypes.data), M.F32, None) == M.EINVAL
    assert lib.mplpxx_iterate(None, 1) == M.EINVAL
    d = ctypes.c_double()
    assert lib.mplpxx_dual_bound(None, ctypes.byref(d)) == M.EINVAL
    lib.mplpxx_destroy(None)


def test_stream_read_probe_rejects_bad_arguments_before_device_work():
    lib = M.lib()
    med, best = ctypes.c_double(), ctypes.c_double()
    for nbytes, reps, out in (((1 << 20) - 16, 3, ctypes.byref(med)), ((1 << 20) + 8, 3, ctypes.byref(med)),
                              (1 << 20, 0, ctypes.byref(med)), (1 << 20, 1001, ctypes.byref(med)), (1 << 20, 3, None)):
        assert lib.mplpxx_stream_read_probe(nbytes, reps, out, ctypes.byref(best)) == M.EINVAL
        assert M.lib().mplpxx_last_error()


@pytest.mark.parametrize("kind,args", [("complete", (2,)), ("complete", (3,)), ("complete", (8,)), ("complete", (57,)),
                                       ("complete", (200,)), ("er", (100, 0.05, 1)), ("er", (60, 0.5, 2)),
                                       ("er", (1000, 0.01, 3)), ("chain", (12,))])
def test_host_schedule_equals_oracle_schedule(kind, args):
    if kind == "complete":
        n = args[0]
        edges = W.complete_edges(n)
        # scramble the input order and orientation: the schedule must not care
        rng = np.random.default_rng(n)
        perm = rng.permutation(edges.shape[0])
        edges = edges[perm]
        flip = rng.random(edges.shape[0]) < 0.5
        edges[flip] = edges[flip][:, ::-1]
    elif kind == "er":
        n, p, seed = args
        edges = W.potts_er(n, 2, p, seed=seed).edges
    else:
        n = args[0]
        edges = W.chain(n, 2).edges
    sp, order = M.schedule(n, edges)
    canon = np.sort(edges, axis=1).astype(np.int32)
    sp_o, ord_o = oracle.schedule(n, canon)
    assert np.array_equal(sp, sp_o) and np.array_equal(order, ord_o)


@pytest.mark.parametrize("n,p,seed", [(12, 0.3, 0), (40, 0.1, 1), (60, 0.5, 2), (200, 0.05, 3), (1000, 0.01, 4),
                                      (1000, 0.05, 0), (9, 0.95, 5)])
def test_host_colour_schedule_equals_oracle_colour_schedule(n, p, seed):
    """The library's and the oracle's edge colourings are written
    separately; with every choice of the rule fixed they must agree exactly,
    whatever the input order and orientation of the edges."""
    edges = W.potts_er(n, 2, p, seed=seed).edges
    rng = np.random.default_rng(seed)
    edges = edges[rng.permutation(edges.shape[0])]
    flip = rng.random(edges.shape[0]) < 0.5
    edges[flip] = edges[flip][:, ::-1]
    sp, order = M.schedule(n, edges, M.SCHED_COLOR)
    sp_o, ord_o = oracle.schedule(n, np.sort(edges, axis=1).astype(np.int32), "color")
    assert np.array_equal(sp, sp_o) and np.array_equal(order, ord_o)
    deg = np.bincount(edges.ravel(), minlength=n)
    assert len(sp) - 1 <= deg.max() + 1


def test_host_schedule_rejects_bad_graphs():
    with pytest.raises(M.MplpError):
        M.schedule(3, np.array([[0, 1], [1, 0]], np.int32))
    with pytest.raises(M.MplpError):
        M.schedule(3, np.array([[0, 3]], np.int32))
    sp, order = M.schedule(4, np.zeros((0, 2), np.int32))
    assert list(sp) == [0] and order.size == 0


def test_pose_table_generator_c_and_numpy_agree_bitwise():
    W.build_generator()
    rng = np.random.default_rng(5)
    for n, L in [(7, 1), (12, 13), (25, 64)]:
        P = rng.random((n, L, 3))
        Q = P[np.arange(n), rng.integers(0, L, n)]
        e = W.complete_edges(n)
        a = W.pose_tables(e, P, Q, 0.04, use_c=True)
        b = W.pose_tables(e, P, Q, 0.04, use_c=False)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("case", ["nan_w", "inf_w", "big_w", "L65", "self", "nan_u", "dense_inf"])
def test_batch_inputs_rejected_without_device_work(case):
    """Batch creation validates every model before any device work: a
    non-finite or too large Potts weight, a Potts model with L > 64, a bad
    edge, a non-finite unary (Potts), and a non-finite dense table."""
    w, d = W.potts_pure(6, 5, 1.0, seed=1)
    weights, un, edges, L = w.pairwise.copy(), w.unaries.copy(), w.edges.copy(), w.L
    potts = case != "dense_inf"
    pw = weights if potts else d.pairwise.copy()
    if case == "nan_w":
        pw[3] = np.nan
    elif case == "inf_w":
        pw[0] = -np.inf
    elif case == "big_w":
        pw[1] = 1e30
    elif case == "L65":
        L = 65
        un = np.zeros((w.n, L), np.float32)
    elif case == "self":
        edges[2] = [4, 4]
    elif case == "nan_u":
        un[2, 1] = np.nan
    elif case == "dense_inf":
        pw[5, 1, 2] = np.inf
    good = W.potts_pure(4, 3, 1.0, seed=2)[0 if potts else 1]
    bad = W.Model(w.n, L, edges, un, pw, "bad")
    with pytest.raises(M.MplpError) as ei:
        M.Batch([good, bad], potts=potts)
    assert ei.value.code == M.EINVAL
    assert "model 1" in str(ei.value)


@pytest.mark.parametrize("case", ["nan_w", "big_w", "L65", "self", "count"])
def test_potts_solver_inputs_rejected_without_device_work(case):
    """mplpxx_create_potts validates before any device work: non-finite or
    oversized weights, L > 64, a bad edge, a weight array of the wrong size."""
    w, _ = W.potts_pure(6, 5, 1.0, seed=3)
    weights, un, edges, L = w.pairwise.copy(), w.unaries.copy(), w.edges.copy(), w.L
    if case == "nan_w":
        weights[2] = np.nan
    elif case == "big_w":
        weights[0] = -1e30
    elif case == "L65":
        L = 65
        un = np.zeros((w.n, L), np.float32)
    elif case == "self":
        edges[1] = [2, 2]
    elif case == "count":
        weights = weights[:-1]
    bad = W.Model(w.n, L, edges, un, weights, "bad")
    if case == "count":
        with pytest.raises(ValueError):
            M.Solver.from_potts(bad)
        return
    with pytest.raises(M.MplpError) as ei:
        M.Solver.from_potts(bad)
    assert ei.value.code == M.EINVAL


def test_from_torch_rejects_host_tensors_before_any_library_call(monkeypatch):
    """Solver.from_torch hands raw tensor pointers to the device copy, so it
    raises ValueError (not an assert) for tensors that are not CUDA tensors,
    and the library is never reached."""
    import torch
    called = []
    monkeypatch.setattr(M, "lib", lambda: called.append(1))
    model = W.uniform(4, 3, seed=0)
    un = torch.from_numpy(model.unaries)
    pw = torch.from_numpy(model.pairwise)
    with pytest.raises(ValueError):
        M.Solver.from_torch(model.n, model.L, model.edges, un, pw)
    with pytest.raises(ValueError):
        M.Solver.from_torch(model.n, model.L, model.edges, model.unaries, model.pairwise)
    assert not called


@pytest.mark.parametrize("case", ["neg_w", "neg_tau", "nan_tau", "inf_w", "kind", "null", "too_large"])
@pytest.mark.parametrize("cost", ["trunc_linear", "trunc_quad"])
def test_structured_costs_rejected_without_device_work(case, cost):
    """Truncated linear and quadratic parameters need finite w >= 0 and tau
    >= 0 and costs within the FP32 bound; an unknown cost kind or missing
    parameters are rejected before any device work (single model and
    batch)."""
    make = W.trunc_linear if cost == "trunc_linear" else W.trunc_quad
    params, _ = make(6, 5, 1.0, seed=0, tau=2.0)
    prm = params.pairwise.copy()
    kind = M.COST_TRUNC_LINEAR if cost == "trunc_linear" else M.COST_TRUNC_QUAD
    if case == "too_large":
        # fl(w tau) above 1e18 (for the quadratic kind also beyond (L_max - 1)^2)
        prm[2] = (1e15, 1e4)
    elif case == "neg_w":
        prm[3, 0] = -0.5
    elif case == "neg_tau":
        prm[2, 1] = -1.0
    elif case == "nan_tau":
        prm[1, 1] = np.nan
    elif case == "inf_w":
        prm[0, 0] = np.inf
    elif case == "kind":
        kind = 7
    edges = np.ascontiguousarray(params.edges)
    un = np.ascontiguousarray(params.unaries)
    h = ctypes.c_void_p()
    pp = None if case == "null" else ctypes.c_void_p(prm.ctypes.data)
    rc = M.lib().mplpxx_create_structured(params.n, params.L, params.m, ctypes.c_void_p(edges.ctypes.data),
                                          ctypes.c_void_p(un.ctypes.data), kind, pp, ctypes.byref(h))
    assert rc == M.EINVAL and not h.value
    n = np.array([params.n], np.int32)
    L = np.array([params.L], np.int32)
    m = np.array([params.m], np.int64)
    e_p = (ctypes.c_void_p * 1)(edges.ctypes.data)
    u_p = (ctypes.c_void_p * 1)(un.ctypes.data)
    p_p = (ctypes.c_void_p * 1)(None if case == "null" else prm.ctypes.data)
    rc = M.lib().mplpxx_batch_create_structured(1, ctypes.c_void_p(n.ctypes.data), ctypes.c_void_p(L.ctypes.data),
                                                ctypes.c_void_p(m.ctypes.data), e_p, u_p, kind, p_p, ctypes.byref(h))
    assert rc == M.EINVAL and not h.value


def test_trunc_linear_expansion_is_the_fp32_product():
    """The dense twin of a truncated linear model holds fl(w * min(|s - t|,
    tau)) in FP32, the same product the device forms for the dual bound."""
    params, dense = W.trunc_linear(5, 9, 1.0, seed=3, tau=3.5)
    for e in range(params.m):
        w, tau = params.pairwise[e]
        for s in range(9):
            for t in range(9):
                want = np.float32(w) * np.float32(min(abs(s - t), tau))
                assert dense.pairwise[e, s, t].view(np.uint32) == np.float32(want).view(np.uint32)


def test_trunc_quad_expansion_is_the_fp32_product():
    """The dense twin of a truncated quadratic model holds fl(w * min((s -
    t)^2, tau)) in FP32 (the square exact), the same product the device
    forms for the passes and the dual bound."""
    params, dense = W.trunc_quad(5, 11, 1.0, seed=3, tau=20.5)
    for e in range(params.m):
        w, tau = params.pairwise[e]
        for s in range(11):
            for t in range(11):
                want = np.float32(w) * np.float32(min((s - t) ** 2, tau))
                assert dense.pairwise[e, s, t].view(np.uint32) == np.float32(want).view(np.uint32)

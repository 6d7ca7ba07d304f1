"""Writes the stored expected values used by the full-size GPU parity tests.

Everything here is computed by the FP64 CPU oracle (``oracle/``) on inputs
from the seeded generators (``paper_2004_08227_amd/workloads.py``); nothing
comes from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py [all|pose|pose_rules|potts|potts_sched|batch|adjoint]

Outputs (JSON, one file per workload):
  pose_k200_l64.json        dual trace of 200 iterations, final node minima,
                            sampled entries of the final reparametrized
                            unaries and pairwise costs
  pose_k200_l64_rules.json  200-iteration dual traces of the (M) and (U) updates
  potts_er_n1000_l16.json   dual traces (30 iterations) at 5/25/50/100 % density
                            and sampled final state entries
  potts_er_n1000_l16_sched.json  the same workload under both schedules of
                            the oracle (greedy matchings, Delta + 1 edge
                            colouring) at 1/5/25/50 % density: schedule
                            sizes and 30-iteration dual traces
  batched_mix_samples.json  100-iteration traces and sampled final state
                            entries of 8 models of the 256-model mix
  adjoint_uniform_k100_l32.json  the oracle's derivative of D_50 along seeded
                            dense and sparse directions and coordinates,
                            and finite differences (four step sizes) along
                            the sparse directions and coordinates
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_08227_amd import workloads as W  # noqa: E402

THREADS = min(8, os.cpu_count() or 1)


def dump(name, obj):
    obj["_source"] = ("FP64 CPU oracle (oracle/mplp_oracle.c) on seeded inputs from workloads.py; "
                      "written by tests/golden/make_golden.py")
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, indent=1)
    print("wrote", name, flush=True)


def state_sample(st, seed, n_unary, n_pair):
    """Seeded entries of the oracle's state after its run: reparametrized
    unaries Tu[u][s] and reparametrized pairwise costs Te[e][s][t] (edges in
    the model's order, u < v), as index lists and values."""
    rng = np.random.default_rng(seed)
    iu = rng.choice(st.Tu.size, size=min(n_unary, st.Tu.size), replace=False)
    ie = rng.choice(st.Te.size, size=min(n_pair, st.Te.size), replace=False) if st.m else np.zeros(0, int)
    return {"seed": seed, "unary_index": [int(i) for i in iu], "unary": st.Tu.ravel()[iu].tolist(),
            "pair_index": [int(i) for i in ie], "pair": st.Te.ravel()[ie].tolist()}


def make_pose():
    model = W.pose(200, 64, seed=0)
    st = oracle.State(model)
    t = time.time()
    tr = st.run(200, trace=True, nthreads=THREADS)
    dump("pose_k200_l64.json", {"workload": "pose n=200 L=64 seed=0", "iters": 200, "trace": tr.tolist(),
                                "node_min": st.Tu.min(axis=1).tolist(), "seconds": time.time() - t,
                                "state": state_sample(st, 5, 4096, 8192)})


def make_pose_rules():
    model = W.pose(200, 64, seed=0)
    out = {"workload": "pose n=200 L=64 seed=0", "iters": 200, "traces": {}}
    for rule in ("M", "U"):
        st = oracle.State(model)
        out["traces"][rule] = st.run(200, rule=rule, trace=True, nthreads=THREADS).tolist()
        print("pose rule", rule, flush=True)
    dump("pose_k200_l64_rules.json", out)


def make_potts():
    out = {"workload": "potts_er n=1000 L=16 seed=0", "iters": 30, "traces": {}}
    for p in (0.05, 0.25, 0.5, 1.0):
        model = W.potts_er(1000, 16, p, seed=0)
        st = oracle.State(model)
        out["traces"][str(p)] = {"m": model.m, "steps": st.n_steps,
                                 "trace": st.run(30, trace=True, nthreads=THREADS).tolist(),
                                 "state": state_sample(st, 6, 2048, 4096)}
        print("potts", p, flush=True)
    dump("potts_er_n1000_l16.json", out)


def make_potts_sched():
    out = {"workload": "potts_er n=1000 L=16 seed=0", "iters": 30, "runs": {}}
    for kind in ("greedy", "color"):
        for p in (0.01, 0.05, 0.25, 0.5):
            if kind == "greedy" and p != 0.01:
                continue  # the greedy traces at 5/25/50 % are in potts_er_n1000_l16.json
            model = W.potts_er(1000, 16, p, seed=0)
            st = oracle.State(model, schedule_kind=kind)
            out["runs"][f"{kind}_{p}"] = {"m": model.m, "steps": st.n_steps,
                                          "trace": st.run(30, trace=True, nthreads=THREADS).tolist()}
            print("potts", kind, p, st.n_steps, flush=True)
    dump("potts_er_n1000_l16_sched.json", out)


def batch_samples():
    sizes = W.batched_mix(256, seed=0, models=False)
    cost = [n * (n - 1) // 2 * L * L for n, L in sizes]
    order = np.argsort(cost)
    rng = np.random.default_rng(123)
    picks = [int(order[0]), int(order[1]), int(order[-1]), int(order[-2])]
    rest = [i for i in range(256) if i not in picks]
    picks += [int(i) for i in rng.choice(rest, size=4, replace=False)]
    return sizes, picks


def make_batch():
    sizes, picks = batch_samples()
    out = {"workload": "batched_mix count=256 seed=0", "iters": 100, "models": {}}
    for i in picks:
        n, L = sizes[i]
        model = W.pose(n, L, seed=1_000_003 * 0 + i)
        st = oracle.State(model)
        tr = st.run(100, trace=True, nthreads=THREADS)
        out["models"][str(i)] = {"n": n, "L": L, "trace": tr.tolist(), "state": state_sample(st, 7, 512, 1024)}
        print("batch model", i, n, L, flush=True)
    dump("batched_mix_samples.json", out)


def adjoint_directions(model, count, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal(model.unaries.shape), rng.standard_normal(model.pairwise.shape))
            for _ in range(count)]


def adjoint_sparse_directions(model, count, seed, support=32):
    """Directions on `support` random coordinates (half unaries, half pairwise)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        du = np.zeros_like(model.unaries)
        dp = np.zeros_like(model.pairwise)
        du.flat[rng.choice(du.size, support // 2, replace=False)] = rng.standard_normal(support // 2)
        dp.flat[rng.choice(dp.size, support // 2, replace=False)] = rng.standard_normal(support // 2)
        out.append((du, dp))
    return out


def adjoint_coords(model, final_Tu, final_Te, count, seed):
    """Coordinates (flat indices into unaries then pairwise; edges u < v):
    the gradient of D_K is sparse, so three quarters sit where it is likely
    nonzero and one quarter anywhere.  Half unary: a node's final minimizing
    label s*_u.  Half pairwise: the zero of row s*_u of an edge's final
    reparametrized table, or the zero of its column s*_v (the entries the
    last passes through that table selected)."""
    rng = np.random.default_rng(seed)
    n, L = model.n, model.L
    nu = model.unaries.size
    best = np.argmin(final_Tu, axis=1)
    q = count // 4
    half = count // 2
    nodes = rng.choice(n, size=min(n, half - q // 2), replace=False)
    cu = [int(u * L + best[u]) for u in nodes] + [int(c) for c in rng.choice(nu, size=q // 2, replace=False)]
    cp = []
    for k, e in enumerate(rng.choice(model.m, size=min(model.m, half - q // 2), replace=False)):
        u, v = model.edges[e]
        if k % 2 == 0:
            s, t = best[u], int(np.argmin(final_Te[e, best[u], :]))
        else:
            s, t = int(np.argmin(final_Te[e, :, best[v]])), best[v]
        cp.append(int(nu + (e * L + s) * L + t))
    cp += [int(nu + c) for c in rng.choice(model.pairwise.size, size=q // 2, replace=False)]
    return cu + cp


def coord_direction(model, c):
    du = np.zeros_like(model.unaries)
    dp = np.zeros_like(model.pairwise)
    if c < model.unaries.size:
        du.flat[c] = 1.0
    else:
        dp.flat[c - model.unaries.size] = 1.0
    return du, dp


def make_adjoint():
    """Reference derivatives of D_50 on the differentiation workload: the
    oracle's forward-mode derivative along 16 dense and 16 sparse seeded
    directions and 64 coordinates.  For the sparse directions and the
    coordinates also central and one-sided differences of the oracle's D_50
    at four step sizes (D_K is piecewise linear: where the one-sided
    differences agree the step stayed inside one linear piece)."""
    K, every = 50, 10
    model = W.uniform(100, 32, seed=0)
    base = model.astype(np.float64)
    st = oracle.State(base)
    st.run(K, nthreads=THREADS)
    D0 = st.dual()

    def D(du, dp):
        mo = W.Model(base.n, base.L, base.edges, base.unaries + du, base.pairwise + dp)
        return oracle.dual_after(mo, K, nthreads=THREADS)

    def tangent(du, dp):
        return oracle.dual_derivative(base, K, du, dp, nthreads=THREADS)

    def diffs(du, dp, hs):
        rows = []
        for h in hs:
            p, m = D(h * du, h * dp), D(-h * du, -h * dp)
            rows.append({"h": h, "central": (p - m) / (2 * h), "right": (p - D0) / h, "left": (D0 - m) / h})
        return rows

    hs = (1e-5, 1e-6, 1e-7, 1e-8)
    out = {"workload": "uniform n=100 L=32 seed=0 (FP32 inputs promoted to FP64)", "K": K, "every": every, "D": D0,
           "dense": {"seed": 7, "count": 16, "tangent": []},
           "sparse": {"seed": 9, "count": 16, "support": 32, "tangent": [], "fd": []},
           "coords": {"seed": 11, "count": 64, "index": [], "tangent": [], "fd": []}}
    for du, dp in adjoint_directions(base, 16, 7):
        out["dense"]["tangent"].append(tangent(du, dp))
    print("dense directions", flush=True)
    for du, dp in adjoint_sparse_directions(base, 16, 9):
        out["sparse"]["tangent"].append(tangent(du, dp))
        out["sparse"]["fd"].append(diffs(du, dp, hs))
    print("sparse directions", flush=True)
    for c in adjoint_coords(base, st.Tu, st.Te, 64, 11):
        du, dp = coord_direction(base, c)
        out["coords"]["index"].append(c)
        out["coords"]["tangent"].append(tangent(du, dp))
        out["coords"]["fd"].append(diffs(du, dp, hs))
    print("coordinates", flush=True)
    dump("adjoint_uniform_k100_l32.json", out)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    W.build_generator()
    if what in ("all", "pose"):
        make_pose()
    if what in ("all", "pose_rules"):
        make_pose_rules()
    if what in ("all", "potts"):
        make_potts()
    if what in ("all", "potts_sched"):
        make_potts_sched()
    if what in ("all", "batch"):
        make_batch()
    if what in ("all", "adjoint"):
        make_adjoint()

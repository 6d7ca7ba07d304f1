"""Writes the stored expected values used by the full-size GPU parity tests.

Everything here is computed by the FP64 CPU oracle (``oracle/``) on inputs
from the seeded generators (``paper_2004_08227_amd/workloads.py``); nothing
comes from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py [all|pose|pose_rules|potts|potts_sched|batch|adjoint]

Outputs (JSON, one file per workload):
  pose_k200_l64.json        dual trace of 200 iterations, final node minima
  pose_k200_l64_rules.json  200-iteration dual traces of the (M) and (U) updates
  potts_er_n1000_l16.json   dual traces (30 iterations) at 5/25/50/100 % density
  potts_er_n1000_l16_sched.json  the same workload under both schedules of
                            the oracle (greedy matchings, Delta + 1 edge
                            colouring) at 1/5/25/50 % density: schedule
                            sizes and 30-iteration dual traces
  batched_mix_samples.json  100-iteration traces of 8 models of the 256-model mix
  adjoint_uniform_k100_l32.json  central and one-sided differences of D_50
                            along seeded dense and sparse directions and
                            coordinates, three step sizes each
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


def make_pose():
    model = W.pose(200, 64, seed=0)
    st = oracle.State(model)
    t = time.time()
    tr = st.run(200, trace=True, nthreads=THREADS)
    dump("pose_k200_l64.json", {"workload": "pose n=200 L=64 seed=0", "iters": 200, "trace": tr.tolist(),
                                "node_min": st.Tu.min(axis=1).tolist(), "seconds": time.time() - t})


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
                                 "trace": st.run(30, trace=True, nthreads=THREADS).tolist()}
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
        out["models"][str(i)] = {"n": n, "L": L, "trace": tr.tolist()}
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


def adjoint_coords(model, count, seed):
    """Coordinates: a third unary entries, the rest pairwise entries."""
    rng = np.random.default_rng(seed)
    nu = model.unaries.size
    cu = rng.choice(nu, size=count // 3, replace=False)
    cp = nu + rng.choice(model.pairwise.size, size=count - count // 3, replace=False)
    return [int(c) for c in np.concatenate([cu, cp])]


def make_adjoint():
    """D_K is piecewise linear in the costs with kinks at every scale along a
    generic direction, so each check stores, for several step sizes h, the
    central difference and both one-sided differences."""
    K, every = 50, 10
    model = W.uniform(100, 32, seed=0)
    base = model.astype(np.float64)
    nu = base.unaries.size

    def D(du, dp):
        mo = W.Model(base.n, base.L, base.edges, base.unaries + du, base.pairwise + dp)
        return oracle.dual_after(mo, K, nthreads=THREADS)

    D0 = D(0.0, 0.0)

    def diffs(du, dp, hs):
        rows = []
        for h in hs:
            p, m = D(h * du, h * dp), D(-h * du, -h * dp)
            rows.append({"h": h, "central": (p - m) / (2 * h), "right": (p - D0) / h, "left": (D0 - m) / h})
        return rows

    out = {"workload": "uniform n=100 L=32 seed=0 (FP32 inputs promoted to FP64)", "K": K, "every": every, "D": D0,
           "dense": {"seed": 7, "count": 8, "fd": []}, "sparse": {"seed": 9, "count": 8, "support": 32, "fd": []},
           "coords": {"seed": 11, "count": 24, "index": [], "fd": []}}
    for du, dp in adjoint_directions(base, 8, 7):
        out["dense"]["fd"].append(diffs(du, dp, (1e-7, 1e-8, 1e-9)))
    print("dense directions", flush=True)
    for du, dp in adjoint_sparse_directions(base, 8, 9):
        out["sparse"]["fd"].append(diffs(du, dp, (1e-6, 1e-7, 1e-8)))
    print("sparse directions", flush=True)
    for c in adjoint_coords(base, 24, 11):
        du = np.zeros_like(base.unaries)
        dp = np.zeros_like(base.pairwise)
        if c < nu:
            du.flat[c] = 1.0
        else:
            dp.flat[c - nu] = 1.0
        out["coords"]["index"].append(c)
        out["coords"]["fd"].append(diffs(du, dp, (1e-6, 1e-7, 1e-8)))
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

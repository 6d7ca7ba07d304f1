"""Benchmark of the MPLP++ hot path on one MI355X.

Workload: the fully connected 6D-pose-shaped model, n=200 nodes, L=64 labels
(19,900 edges, 326 MB of FP32 pairwise tables), synthetic and seeded.  One
"step" is one BCA-iteration: every edge receives one handshake update,
matching after matching (199 matchings of 100 edges).  The timed region runs
exactly --steps iterations with all inputs resident in HBM.

The JSON line reports edge-block updates/s (``value``), the HBM roofline of
the dominant kernel from its algorithmic bytes (4 L^2 table bytes + 16 L
message bytes per edge update), the oracle's CPU throughput on a bounded
sample, and time to reach the dual bound within epsilon of the best value
against the plain FP64 oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edge-block updates/s + HBM GB/s fraction; time-to-dual-bound vs plain, 1 MI355X"

# HBM traffic of the measured kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs (profiles/k_persistent_mb_pose_k200_l64.md): KiB per
# iteration of the pose n=200/L=64 launch, and the factors that map each
# counter to bytes, from the same counters on a 1 GiB copy.  Valid only for
# the kernel sources they were taken on (hash below); otherwise null.
TRAFFIC = {"src_sha": "8c57154f050dfbd2", "fetch_kib_per_iter": 3768204.6875 / 20, "fetch_scale": 2.0,
           "write_kib_per_iter": 457708.0 / 20, "write_scale": 1.0}
TRAFFIC_SRCS = ("paper_2004_08227_amd/csrc/common.h", "paper_2004_08227_amd/csrc/device_common.h",
                "paper_2004_08227_amd/csrc/step_common.h", "paper_2004_08227_amd/csrc/potts_passes.h",
                "paper_2004_08227_amd/csrc/potts_mb.h", "paper_2004_08227_amd/csrc/handshake.hip")


def kernel_src_sha():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SRCS:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(iters):
    """HBM bytes of one launch of `iters` iterations, or None if the kernel
    changed since the counters were taken."""
    try:
        if kernel_src_sha() != TRAFFIC["src_sha"]:
            return None
    except OSError:
        return None
    kib = TRAFFIC["fetch_kib_per_iter"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib_per_iter"] * TRAFFIC["write_scale"]
    return kib * 1024.0 * iters


def algorithmic_bytes_per_update(L, esz=4):
    # read-only L x L table + read and write the edge's 2L messages
    return esz * L * L + 4 * esz * L


def time_to_bound(trace, t_per_iter, d_star, eps):
    out = {}
    for e in eps:
        target = d_star - e * abs(d_star)
        idx = np.flatnonzero(trace >= target)
        out[f"{e:g}"] = None if idx.size == 0 else float((idx[0] + 1) * t_per_iter)
    return out


def cpu_baseline(model, iters_sample):
    import oracle
    threads = min(oracle.max_threads(), os.cpu_count() or 1)
    st = oracle.State(model)
    t0 = time.perf_counter()
    st.run(iters_sample, rule="H", nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": model.m * iters_sample / dt, "unit": "edge updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters_sample} of the iterations of {model.name} from phi=0 (FP64 oracle, OpenMP over the "
                      f"edges of each matching)", "seconds": dt, "s_per_iter": dt / iters_sample}


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": name, "logical_cpus": os.cpu_count()}


def oracle_one_thread(model, iters_sample=4):
    """Seconds per iteration of the oracle on one host thread (a short
    sample, for the single-thread time-to-bound)."""
    import oracle
    st = oracle.State(model)
    t0 = time.perf_counter()
    st.run(iters_sample, rule="H", nthreads=1)
    return (time.perf_counter() - t0) / iters_sample


def measured_stream_peak(gib=4, reps=5):
    """Device streaming rates measured with plain torch kernels on a
    `gib` GiB FP32 tensor (median of `reps`, torch events on torch's
    stream): a full read (sum) and a copy (read + write)."""
    import torch
    n = gib * (1 << 28)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("read_gbs", lambda: a.sum(), 4 * n), ("copy_gbs", lambda: b.copy_(a), 8 * n)):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        out[name] = nbytes / float(np.median(ts)) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def bench_batched(M, W, iters=100, per_problem=True):
    """The 256-model pose mix in one persistent launch vs the same models
    solved one after another with one launch per model: with the
    single-model engine (Solver), and as one-model batches on the batched
    engine; same iterations, device times from HIP events."""
    import torch
    models = W.batched_mix(256, seed=0)
    m_tot = sum(mo.m for mo in models)
    bytes_it = sum(mo.m * algorithmic_bytes_per_update(mo.L) for mo in models)
    with M.Batch(models) as b:
        b.iterate(2)                      # plan, capture the graph, warm up
        b.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.iterate(iters)
        wall_b = time.perf_counter() - t0
        ms_b = b.info("last_ms")
        info = {k: b.info(k) for k in ("engine", "waves", "grid", "tasks", "teams", "max_team", "lds_tasks",
                                       "lds_bytes", "plan_us")}
        info["wg_busy_max_ms"] = b.info("wg_max_us") / 1e3
        info["wg_busy_mean_ms"] = b.info("wg_mean_us") / 1e3
        d_b = b.dual_bounds()
        # the same launch with the autotuner's options for this batch (if the
        # committed table has an entry): the same duals, bit for bit
        from paper_2004_08227_amd import autotune as A
        tuned = A.apply_batch(b, models)
        if tuned:
            b.reset()
            b.iterate(2)
            b.reset()
            b.iterate(iters)
            info["tuned_options"] = tuned
            info["tuned_ms"] = b.info("last_ms")
            info["tuned_duals_bitwise_equal"] = bool(np.array_equal(b.dual_bounds(), d_b))
    out = {"workload": "batched_mix: 256 pose models, n ~ U{20..300}, L ~ U{8..64}, seed 0", "iterations": iters,
           "edges": m_tot, "batched_ms": ms_b, "batched_wall_s": wall_b,
           "updates_per_s": m_tot * iters / (ms_b / 1e3),
           "hbm_frac": bytes_it * iters / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS, "plan": info}
    if not per_problem:
        return out
    ms_p = 0.0
    t0 = time.perf_counter()
    d_p = []
    for mo in models:
        with M.Solver.from_model(mo) as s:
            s.iterate(iters)
            ms_p += s.last_iterate_ms()
            d_p.append(s.dual_bound())
    wall_p = time.perf_counter() - t0
    out.update({"per_problem_ms": ms_p, "per_problem_wall_s_incl_create": wall_p, "speedup": ms_p / ms_b,
                "max_dual_diff_vs_per_problem": float(np.max(np.abs(np.asarray(d_b) - np.asarray(d_p))))})
    # the same per-problem launches, each model as a batch of one (the
    # batched engine spreading a single model over the whole GPU)
    ms_q = 0.0
    d_q = []
    for mo in models:
        with M.Batch([mo]) as b1:
            b1.iterate(iters)
            ms_q += b1.info("last_ms")
            d_q.append(b1.dual_bounds()[0])
    out["per_problem_one_model_batches_ms"] = ms_q
    out["speedup_vs_one_model_batches"] = ms_q / ms_b
    out["max_dual_diff_vs_one_model_batches"] = float(np.max(np.abs(np.asarray(d_b) - np.asarray(d_q))))
    return out


def bench_c2(M, W, iters=30, with_cpu=True):
    """Sparsification study: Potts + noise on G(n = 1000, p), L = 16, at four
    densities; the single-model engine, `iters` iterations from phi = 0.
    Time-to-bound against the oracle's own stored traces (written by
    tests/golden/make_golden.py from the oracle alone) x its measured seconds
    per iteration on this host."""
    import torch
    gold = os.path.join(ROOT, "tests", "golden", "potts_er_n1000_l16.json")
    g = json.load(open(gold)) if os.path.exists(gold) else None
    gold2 = os.path.join(ROOT, "tests", "golden", "potts_er_n1000_l16_sched.json")
    g2 = json.load(open(gold2)) if os.path.exists(gold2) else None
    out = {"workload": "potts_er: n=1000, L=16, Potts w~U[0.1,1] + U[0,0.2) noise, unaries U[0,1), seed 0",
           "iterations": iters, "densities": {}, "colour_schedule": {}}
    runs = [(p, "greedy") for p in (0.01, 0.05, 0.25, 0.5, 1.0)] + [(p, "color") for p in (0.01, 0.05, 0.25, 0.5)]
    for p, kind in runs:
        model = W.potts_er(1000, 16, p, seed=0)
        B = algorithmic_bytes_per_update(model.L)
        sched = M.SCHED_COLOR if kind == "color" else M.SCHED_AUTO
        with M.Solver.from_model(model, schedule=sched) as s:
            U0, phi0 = s.get_state()
            s.iterate(1)
            s.set_state(U0, phi0)
            torch.cuda.synchronize()
            s.iterate(iters)
            ms = s.last_iterate_ms()
            s.set_state(U0, phi0)
            tr = s.iterate_trace(iters)
            steps = s.info("steps")
            eng = s.info("engine")
            nt = s.info("threads")
        t = ms / 1e3
        rec = {"m": model.m, "matchings": steps, "engine": eng, "threads": nt, "ms_per_iter": ms / iters,
               "updates_per_s": model.m * iters / t, "hbm_gbs": model.m * iters * B / t / 1e9,
               "hbm_frac": model.m * iters * B / t / 1e9 / HBM_PEAK_GBS, "dual": float(tr[-1])}
        ref = None
        if kind == "greedy" and g is not None and str(p) in g["traces"] and g["traces"][str(p)]["m"] == model.m:
            ref = np.asarray(g["traces"][str(p)]["trace"][:iters])
        elif g2 is not None and f"{kind}_{p}" in g2["runs"] and g2["runs"][f"{kind}_{p}"]["m"] == model.m:
            ref = np.asarray(g2["runs"][f"{kind}_{p}"]["trace"][:iters])
        if ref is not None:
            rec["max_rel_diff_vs_oracle_trace"] = float(np.max(np.abs(tr[:ref.size] - ref) / np.maximum(1.0, np.abs(ref))))
        if with_cpu:
            import oracle
            threads = min(oracle.max_threads(), os.cpu_count() or 1)
            st = oracle.State(model, schedule_kind=kind)
            t0 = time.perf_counter()
            st.run(1, rule="H", nthreads=threads)
            s_it = time.perf_counter() - t0
            d_star = float(max(tr.max(), ref.max() if ref is not None else -np.inf))
            eps = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5]
            rec["oracle_s_per_iter"] = s_it
            rec["oracle_cores"] = threads
            rec["time_to_dual_bound"] = {"d_star": d_star, "gpu_s": time_to_bound(tr, t / iters, d_star, eps),
                                         "plain_oracle_s": time_to_bound(ref if ref is not None else tr, s_it, d_star, eps)}
        (out["densities"] if kind == "greedy" else out["colour_schedule"])[str(p)] = rec
        del model
    return out


def bench_rules(M, W, iters=200):
    """MPLP (M) and uniform (U) against MPLP++ (H) from the same start (phi =
    0): dual traces of `iters` iterations, each rule on the per-matching
    engine (same kernel structure, one launch per matching), and every rule
    also on the persistent mailbox engine (timed there; the traces of (M) and
    (U) come from the per-matching engine, and the two engines' final states
    are compared bit for bit); seconds to reach D* - eps|D*|, D* the best final
    dual of all runs, from each run's own time per iteration."""
    out = {}
    for key, model in (("pose_k200_l64", W.pose(200, 64, seed=0)),
                       ("potts_er_n1000_l16_p0.25", W.potts_er(1000, 16, 0.25, seed=0))):
        runs = {}
        same = {}
        for name, rule, engine in (("H_persistent", M.RULE_H, M.ENGINE_PERSISTENT), ("H", M.RULE_H, M.ENGINE_STEP),
                                   ("M_persistent", M.RULE_M, M.ENGINE_PERSISTENT), ("M", M.RULE_M, M.ENGINE_STEP),
                                   ("U_persistent", M.RULE_U, M.ENGINE_PERSISTENT), ("U", M.RULE_U, M.ENGINE_STEP)):
            with M.Solver.from_model(model) as s:
                s.set_option(M.OPT_ENGINE, engine)
                s.set_option(M.OPT_RULE, rule)
                U0, phi0 = s.get_state()
                s.iterate(1)
                s.set_state(U0, phi0)
                s.iterate(iters)
                t_it = s.last_iterate_ms() / 1e3 / iters
                st_it = s.get_state(comp=True)
                s.set_state(U0, phi0)
                tr = s.iterate_trace(iters)
                st_tr = s.get_state(comp=True)
            if name in ("M_persistent", "U_persistent"):
                same[name] = all(np.array_equal(x, y) for x, y in zip(st_it, st_tr))
            runs[name] = (tr, t_it)
        d_star = float(max(tr.max() for tr, _ in runs.values()))
        eps = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5]
        rec = {"m": model.m, "iterations": iters, "d_star": d_star, "eps_rel": eps,
               "M_persistent_state_equals_per_matching": same.get("M_persistent"),
               "U_persistent_state_equals_per_matching": same.get("U_persistent")}
        for name, (tr, t_it) in runs.items():
            rec[name] = {"s_per_iter": t_it, "final_dual": float(tr[-1]), "time_to_bound_s": time_to_bound(tr, t_it, d_star, eps),
                         "iterations_to_bound": {f"{e:g}": (None if not np.any(tr >= d_star - e * abs(d_star))
                                                            else int(np.flatnonzero(tr >= d_star - e * abs(d_star))[0]) + 1)
                                                 for e in eps}}
        out[key] = rec
        del model
    return out


def bench_gap(M, W, iters=200):
    """Anytime primal-dual gap on the pose model: after each iteration the
    certified dual (Eq. 3) and the energy of the Eq. (5) rounding."""
    model = W.pose(200, 64, seed=0)
    with M.Solver.from_model(model) as s:
        s.iterate_gap(2)                       # warm up (compiles nothing; first-use allocations)
    with M.Solver.from_model(model) as s:
        t0 = time.perf_counter()
        d, e, _ = s.iterate_gap(iters)
        wall = time.perf_counter() - t0
    best_e = np.minimum.accumulate(e)
    best_d = np.maximum.accumulate(d)
    gap = (best_e - best_d) / np.abs(best_d)
    out = {"workload": "pose n=200 L=64 seed 0", "iterations": iters, "wall_s": wall,
           "final_dual": float(d[-1]), "best_energy": float(e.min()), "best_energy_iteration": int(np.argmin(e)) + 1,
           "final_rel_gap": float(gap[-1]),
           "iterations_to_rel_gap": {f"{g:g}": (None if not np.any(gap <= g) else int(np.flatnonzero(gap <= g)[0]) + 1)
                                     for g in (1e-1, 3e-2, 1e-2, 3e-3, 1e-3)},
           "energy_at": {str(i): float(e[i - 1]) for i in (1, 10, 50, 100, 200) if i <= iters},
           "dual_at": {str(i): float(d[i - 1]) for i in (1, 10, 50, 100, 200) if i <= iters}}
    return out


def bench_potts(M, W, iters=50, mix_count=64):
    """Structured Potts passes (one weight per edge, O(L) per pass) against
    the dense wave engine on the expanded tables w [s != t]: one complete
    pose-size model (n = 200, L = 64) as a batch of one, the first
    `mix_count` sizes of the batched mix (complete graphs), and the
    sparsification shape (n = 1000, L = 16, G(n, p)) as a batch of one;
    one-model cases also run on the single-model mailbox engine, dense and
    Potts (mplpxx_create_potts).  Same
    iterations from phi = 0; device times from HIP events; the duals of the
    two runs must be bitwise equal."""
    def run(models, potts):
        with M.Batch(models, potts=potts) as b:
            b.iterate(2)
            b.reset()
            b.iterate(iters)
            ms = b.info("last_ms")
            d = b.dual_bounds()
            tb = b.info("table_bytes")
        return ms, d, tb

    out = {"iterations": iters}
    sizes = W.batched_mix(mix_count, seed=0, models=False)
    cases = [("pose_size_complete_n200_l64", [(200, 64, 1.0)]),
             (f"mix_{mix_count}_complete", [(n, L, 1.0) for n, L in sizes])]
    cases += [(f"c2_shape_n1000_l16_p{p}", [(1000, 16, p)]) for p in (0.05, 0.25, 1.0)]
    for name, sz in cases:
        pairs = [W.potts_pure(n, L, p, seed=7 + i) for i, (n, L, p) in enumerate(sz)]
        m_tot = sum(p[0].m for p in pairs)
        bp = sum(p[0].m * (4 + 16 * p[0].L) for p in pairs)
        bd = sum(p[0].m * algorithmic_bytes_per_update(p[0].L) for p in pairs)
        weights, dense = [p[0] for p in pairs], [p[1] for p in pairs]
        del pairs
        ms_p, d_p, tb_p = run(weights, True)
        ms_d, d_d, tb_d = run(dense, False)
        ms_s = ms_sp = None
        if len(dense) == 1:
            # the same model on the single-model mailbox engine, dense and Potts
            def single(make):
                with make() as s1:
                    U0, phi0 = s1.get_state()
                    s1.iterate(2)
                    s1.set_state(U0, phi0)
                    s1.iterate(iters)
                    return s1.last_iterate_ms(), s1.dual_bound()
            ms_s, d_s = single(lambda: M.Solver.from_model(dense[0]))
            ms_sp, d_sp = single(lambda: M.Solver.from_potts(weights[0]))
        del weights, dense
        out[name] = {"models": len(sz), "edges": m_tot, "potts_ms_per_iter": ms_p / iters,
                     "dense_ms_per_iter": ms_d / iters, "speedup": ms_d / ms_p,
                     "potts_updates_per_s": m_tot * iters / (ms_p / 1e3),
                     "dense_updates_per_s": m_tot * iters / (ms_d / 1e3),
                     "potts_bytes_per_update": bp / m_tot, "dense_bytes_per_update": bd / m_tot,
                     "potts_hbm_frac": bp * iters / (ms_p / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "dense_hbm_frac": bd * iters / (ms_d / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "potts_table_bytes": tb_p, "dense_table_bytes": tb_d,
                     "duals_bitwise_equal": bool(np.array_equal(d_p, d_d))}
        if ms_s is not None:
            out[name]["dense_single_model_engine_ms_per_iter"] = ms_s / iters
            out[name]["speedup_vs_single_model_engine"] = ms_s / ms_p
            out[name]["potts_single_model_engine_ms_per_iter"] = ms_sp / iters
            out[name]["potts_single_vs_dense_single_speedup"] = ms_s / ms_sp
            out[name]["single_model_duals_bitwise_equal"] = bool(d_s == d_sp)
    return out


def bench_trunc_linear(M, W, iters=50, mix_count=64, tau=8.0, kind=None):
    """Truncated linear costs w min(|s - t|, tau) (mplpxx_*_create_structured,
    8 bytes of pairwise data per edge) against the dense engines on the
    expanded tables (4 L^2 bytes): one complete pose-size model (n = 200,
    L = 64) on the batched wave engine as a batch of one and on the
    single-model mailbox engine, and the first `mix_count` sizes of the
    batched mix (complete graphs) as one batch.  Same iterations from phi =
    0, device times from HIP events.  The wave engine runs the O(L)
    distance transform, whose sums round in another order than the dense
    passes: the largest relative difference of the final duals is reported
    (the parity tests hold both to the oracle at 1e-5).  The single-model
    engine forms each tile from (w, tau) by default (bitwise the dense
    engine) and is also timed in label order (the distance transform,
    threads 64).  kind = COST_TRUNC_QUAD: the same for truncated quadratic
    costs w min((s - t)^2, tau) (every candidate formed from the two
    parameters, bitwise the dense engines on either path: the differences
    are 0)."""
    kind = M.COST_TRUNC_LINEAR if kind is None else kind
    make = W.trunc_linear if kind == M.COST_TRUNC_LINEAR else W.trunc_quad
    def run_batch(models, kind):
        with M.Batch(models, kind=kind) as b:
            b.iterate(2)
            b.reset()
            b.iterate(iters)
            return b.info("last_ms"), np.asarray(b.dual_bounds())

    def run_single(make, threads=0):
        with make() as s1:
            if threads:
                s1.set_option(M.OPT_THREADS, threads)
            U0, phi0 = s1.get_state()
            s1.iterate(2)
            s1.set_state(U0, phi0)
            s1.iterate(iters)
            return s1.last_iterate_ms(), np.asarray([s1.dual_bound()])

    out = {"iterations": iters, "tau": tau}
    sizes = W.batched_mix(mix_count, seed=0, models=False)
    for name, sz in (("complete_n200_l64", [(200, 64)]), (f"mix_{mix_count}_complete", sizes)):
        pairs = [make(n, L, 1.0, seed=40 + i, tau=tau) for i, (n, L) in enumerate(sz)]
        m_tot = sum(p[0].m for p in pairs)
        b_tl = sum(p[0].m * (8 + 16 * p[0].L) for p in pairs)
        b_d = sum(p[0].m * algorithmic_bytes_per_update(p[0].L) for p in pairs)
        params, dense = [p[0] for p in pairs], [p[1] for p in pairs]
        del pairs
        ms_t, d_t = run_batch(params, kind)
        ms_d, d_d = run_batch(dense, 0)
        rec = {"models": len(sz), "edges": m_tot, "structured_ms_per_iter": ms_t / iters,
               "dense_ms_per_iter": ms_d / iters, "speedup": ms_d / ms_t,
               "structured_updates_per_s": m_tot * iters / (ms_t / 1e3),
               "structured_bytes_per_update": b_tl / m_tot, "dense_bytes_per_update": b_d / m_tot,
               "max_rel_dual_difference": float(np.max(np.abs(d_t - d_d) / np.maximum(1.0, np.abs(d_d))))}
        if len(sz) == 1:
            ms_s, d_s = run_single(lambda: M.Solver.from_model(dense[0]))
            ms_st, d_st = run_single(lambda: M.Solver.from_structured(params[0], kind))
            ms_lo, d_lo = run_single(lambda: M.Solver.from_structured(params[0], kind), threads=64)
            rec.update({"single_model_dense_ms_per_iter": ms_s / iters,
                        "single_model_structured_ms_per_iter": ms_st / iters,
                        "single_model_speedup": ms_s / ms_st,
                        "single_model_rel_dual_difference": float(abs(d_st[0] - d_s[0]) / max(1.0, abs(d_s[0]))),
                        "single_model_label_order_ms_per_iter": ms_lo / iters,
                        "single_model_label_order_rel_dual_difference":
                            float(abs(d_lo[0] - d_s[0]) / max(1.0, abs(d_s[0])))})
        out[name] = rec
        del params, dense
    return out


def summary(result):
    """The headline numbers of every section, short enough to survive the
    end of a long line."""
    sm = {"c1_ms_per_iter": result.get("ms_per_step"), "c1_hbm_frac": result.get("hbm_frac")}
    b = result.get("batched")
    if b:
        sm.update({"c3_batched_ms": b.get("batched_ms"), "c3_speedup_vs_per_problem": b.get("speedup"),
                   "c3_hbm_frac": b.get("hbm_frac")})
    ms = result.get("measured_stream")
    if ms:
        sm["measured_read_gbs"] = max(ms.get("read_gbs", 0.0), ms.get("hip_read_gbs", 0.0))
        sm["c1_frac_of_measured_read"] = ms.get("frac_of_measured_read")
        if b and b.get("hbm_frac") is not None:
            sm["c3_frac_of_measured_read"] = b["hbm_frac"] * HBM_PEAK_GBS / sm["measured_read_gbs"]
    c2 = result.get("c2")
    if c2 and isinstance(c2.get("densities"), dict):
        sm["c2_hbm_frac"] = {k: v.get("hbm_frac") for k, v in c2["densities"].items() if isinstance(v, dict)}
    a = result.get("adjoint")
    if a:
        tw = a.get("fp64_twin", {})
        sm["c4_forward_s"] = tw.get("forward_s")
        sm["c4_backward_s"] = tw.get("backward_s")
        sm["c4_fp32_forward_s"] = a.get("fp32_forward_s")
        sm["c4_backward_vs_fp32_forward"] = tw.get("backward_vs_fp32_forward")
    r = result.get("rules")
    if r and isinstance(r.get("pose_k200_l64"), dict):
        sm["c1_final_dual_by_rule"] = {k: v.get("final_dual") for k, v in r["pose_k200_l64"].items()
                                       if isinstance(v, dict) and "final_dual" in v}
        sm["c1_s_to_10pct_of_dstar_by_rule"] = {k: v["time_to_bound_s"].get("0.1")
                                                for k, v in r["pose_k200_l64"].items()
                                                if isinstance(v, dict) and "time_to_bound_s" in v}
    for sec in ("trunc_linear", "trunc_quad"):
        t = result.get(sec)
        if t:
            sm[sec + "_speedup"] = {k: v.get("speedup") for k, v in t.items() if isinstance(v, dict)}
            sm[sec + "_speedup"].update({k + "_single_model": v["single_model_speedup"] for k, v in t.items()
                                         if isinstance(v, dict) and "single_model_speedup" in v})
    return sm


def copy_calibration():
    """A plain 1 GiB device copy, three times: the reference for the HBM
    byte counters (run under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)."""
    import torch
    n = 256 * 1024 * 1024
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": "3 x 1 GiB device copy done"}))


def bench_adjoint(M, W, K=50, every=10):
    """Forward (K iterations with checkpoints) and backward of the
    differentiation workload on an FP32 handle: by default on its FP64 twin
    (persistent kernels: one launch per segment and direction), the same
    with one launch per matching (MPLPXX_OPT_ENGINE = 1, bitwise the same
    gradients), and the FP32 run's own adjoint; next to the plain FP32
    forward (K iterations from phi = 0 on the mailbox engine)."""
    import torch
    model = W.uniform(100, 32, seed=0)
    out = {"workload": "uniform n=100 L=32 seed 0, FP32 costs", "K": K, "every": every}
    with M.Solver.from_model(model) as s:
        U0, phi0 = s.get_state()
        s.iterate(K)
        s.set_state(U0, phi0)
        s.iterate(K)
        out["fp32_forward_s"] = s.last_iterate_ms() / 1e3
    grads = {}
    for key, f64, engine in (("fp64_twin", 1, 0), ("fp64_twin_per_matching", 1, 1), ("fp32_run", 0, 0)):
        with M.Solver.from_model(model) as s:
            s.set_option(M.OPT_ADJOINT_F64, f64)
            s.set_option(M.OPT_ENGINE, engine)
            s.adjoint_forward(K, every)
            s.adjoint_backward()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            loss = s.adjoint_forward(K, every)
            t1 = time.perf_counter()
            gu, gp = s.adjoint_backward()
            t2 = time.perf_counter()
            mem = s.info("adjoint_bytes")
        grads[key] = (gu, gp)
        out[key] = {"loss": loss, "forward_s": t1 - t0, "backward_s": t2 - t1,
                    "backward_vs_fp32_forward": (t2 - t1) / out["fp32_forward_s"], "adjoint_device_bytes": mem,
                    "model_device_bytes": model.m * (4 * model.L * model.L + 8 * model.L) + model.n * model.L * 12}
    a, b = grads["fp64_twin"], grads["fp64_twin_per_matching"]
    out["persistent_equals_per_matching"] = bool(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]))
    return out


def loaded_runtimes():
    """Paths of the HIP and HSA runtime libraries mapped into this process."""
    out = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1] if len(line.split()) >= 6 else ""
                if "libamdhip64" in path or "libhsa-runtime64" in path:
                    out.add(path)
    except OSError:
        pass
    return sorted(out)


def code_mappings():
    """Executable mappings of this process (address range, path), for
    reading addresses in a crash report."""
    out = []
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 6 and "x" in parts[1]:
                    out.append(f"{parts[0]} {parts[5]}")
    except OSError:
        pass
    return out


def kernel_only(steps, warmup):
    """The C1 launch alone, without PyTorch, on the library build linked
    against /opt/rocm's HIP runtime: the process for rocprofv3 runs (whose
    tool library loads /opt/rocm's HSA runtime; PyTorch's bundled HIP
    runtime next to it would add a second HSA runtime to the process)."""
    os.environ["MPLPXX_RUNTIME"] = "rocm"
    import paper_2004_08227_amd as M
    from paper_2004_08227_amd import workloads as W
    model = W.pose(200, 64, seed=0)
    with M.Solver.from_model(model) as s:
        U0, phi0 = s.get_state()
        if warmup:
            s.iterate(warmup)
        s.set_state(U0, phi0)
        s.iterate(steps)
        ms = s.last_iterate_ms()
        d = s.dual_bound()
        print(json.dumps({"kernel_only": "pose_k200_l64", "steps": steps, "ms_per_step": ms / steps, "dual_bound": d,
                          "hbm_frac": model.m * steps * algorithmic_bytes_per_update(64) / (ms / 1e3) / 1e9 /
                          HBM_PEAK_GBS, "runtimes": loaded_runtimes()}), flush=True)
    # (on stderr: the process's code mappings, to place the frames of a
    # report from exit handlers that run after this line)
    print("\n".join(code_mappings()), file=sys.stderr, flush=True)


def adjoint_only(steps, warmup):
    """The differentiation workload alone (uniform n=100, L=32, FP32 costs;
    50 iterations with a checkpoint every 10, then the backward on the FP64
    twin), without PyTorch, on the library build linked against /opt/rocm's
    HIP runtime: the process for rocprofv3 runs of the adjoint kernels.  The
    gradients stay on the device (the backward is called with no output)."""
    os.environ["MPLPXX_RUNTIME"] = "rocm"
    import paper_2004_08227_amd as M
    from paper_2004_08227_amd import workloads as W
    model = W.uniform(100, 32, seed=0)
    fwd, bwd = [], []
    with M.Solver.from_model(model) as s:
        for rep in range(warmup + steps):
            t0 = time.perf_counter()
            loss = s.adjoint_forward(50, 10)
            t1 = time.perf_counter()
            M._check(M.lib().mplpxx_adjoint_backward(s._h, None, None))
            t2 = time.perf_counter()
            if rep >= warmup:
                fwd.append(t1 - t0)
                bwd.append(t2 - t1)
            print(f"adjoint rep {rep}: forward {1e3 * (t1 - t0):.2f} ms, backward {1e3 * (t2 - t1):.2f} ms",
                  file=sys.stderr, flush=True)
    print(json.dumps({"adjoint_only": "uniform_n100_l32_k50_every10", "reps": steps, "loss": loss,
                      "forward_ms": 1e3 * float(np.median(fwd)), "backward_ms": 1e3 * float(np.median(bwd)),
                      "runtimes": loaded_runtimes()}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--engine", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the sparsification section (n=1000, L=16, 4 densities)")
    ap.add_argument("--no-rules", action="store_true", help="skip the MPLP / uniform vs MPLP++ comparison")
    ap.add_argument("--no-gap", action="store_true", help="skip the anytime primal-dual gap section")
    ap.add_argument("--no-potts", action="store_true", help="skip the structured Potts vs dense section")
    ap.add_argument("--no-stream", action="store_true", help="skip the measured streaming-rate reference")
    ap.add_argument("--only-potts", action="store_true", help="run only the structured Potts section")
    ap.add_argument("--only-batch", action="store_true", help="run only the batched-mix section")
    ap.add_argument("--no-trunc-linear", action="store_true", help="skip the truncated linear vs dense section")
    ap.add_argument("--only-adjoint", action="store_true", help="run only the adjoint (differentiation) section")
    ap.add_argument("--only-trunc-linear", action="store_true",
                    help="run only the truncated linear and truncated quadratic sections")
    ap.add_argument("--no-trunc-quad", action="store_true", help="skip the truncated quadratic vs dense section")
    ap.add_argument("--no-per-problem", action="store_true",
                    help="batched section without the per-problem comparison runs")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the timed pose n=200/L=64 launch, without PyTorch (for rocprofv3 runs)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="the differentiation workload alone, without PyTorch (for profiler runs)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only the library's streaming-read probe at 1, 2, 4 and 8 GiB, without PyTorch")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a 3 x 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "mplpxx runs on one GPU (the multi-GPU design is not implemented); --gpus must be 1"}))
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.kernel_only:
        kernel_only(args.steps, args.warmup)
        return
    if args.adjoint_only:
        adjoint_only(args.steps, args.warmup)
        return
    if args.stream_probe:
        os.environ["MPLPXX_RUNTIME"] = "rocm"
        import paper_2004_08227_amd as M
        out = {}
        for gib in (1, 2, 4, 8):
            med, best = M.stream_read_probe(gib << 30, 5)
            out[f"{gib}GiB"] = {"median_gbs": med, "best_gbs": best}
        print(json.dumps({"stream_read_probe": out}), flush=True)
        return

    import torch
    import paper_2004_08227_amd as M
    from paper_2004_08227_amd import workloads as W

    if args.only_potts:
        print(json.dumps({"potts": bench_potts(M, W)}))
        return
    if args.only_batch:
        print(json.dumps({"batched": bench_batched(M, W, per_problem=not args.no_per_problem)}))
        return
    if args.only_trunc_linear:
        print(json.dumps({"trunc_linear": bench_trunc_linear(M, W),
                          "trunc_quad": bench_trunc_linear(M, W, kind=M.COST_TRUNC_QUAD, tau=64.0)}))
        return
    if args.only_adjoint:
        print(json.dumps({"adjoint": bench_adjoint(M, W)}))
        return

    assert torch.cuda.is_available(), "bench needs a GPU"
    n, L, seed = 200, 64, 0
    model = W.pose(n, L, seed=seed)
    s = M.Solver.from_model(model)
    if args.engine:
        s.set_option(M.OPT_ENGINE, args.engine)
    if args.threads:
        s.set_option(M.OPT_THREADS, args.threads)
    U0, phi0 = s.get_state()

    # warmup, then restore the initial state so the timed run starts at phi=0
    if args.warmup:
        s.iterate(args.warmup)
    s.set_state(U0, phi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = s.last_iterate_ms()            # HIP events around the launch, on the library's stream
    d_final = s.dual_bound()

    m = model.m
    K = args.steps
    B = algorithmic_bytes_per_update(L)
    t = ev_ms / 1e3
    value = m * K / t
    gbs = m * K * B / t / 1e9

    # trace for time-to-dual-bound (separate, untimed run)
    s.set_state(U0, phi0)
    trace = s.iterate_trace(K)
    t_iter = t / K

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "edge updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ev_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "pose_k200_l64", "n": n, "L": L, "m": m, "seed": seed,
                   "matchings_per_iteration": s.info("steps"), "engine": s.info("engine"),
                   "threads_per_wg": s.info("threads"), "grid": s.info("grid")},
        "wall_s": wall,
        "hbm_gbs": gbs,
        "hbm_frac": gbs / HBM_PEAK_GBS,
        "dual_bound": d_final,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(K) if s.info("engine") == 2 else None,
                     "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, copy-calibrated)",
                     "kernel": (f"k_persistent_mb<{L},{s.info('threads')},...>" if s.info("engine") == 2
                                else f"k_step<float,{L},{s.info('threads')}>"),
                     "bytes_per_update": B, "updates_per_launch": m * K if s.info("engine") == 2 else m // s.info("steps")},
    }
    if not args.no_cpu:
        cb = cpu_baseline(model, args.cpu_iters)
        result["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        result["host_cpu"] = host_cpu()
        s1 = oracle_one_thread(model)
        result["oracle_one_thread"] = {"s_per_iter": s1, "value": m / s1, "unit": "edge updates/s",
                                       "sample": "4 iterations from phi=0, 1 host thread"}
        # the oracle's own trajectory: its stored 200-iteration trace on this
        # model (written by tests/golden/make_golden.py from the oracle alone)
        ref = None
        gold = os.path.join(ROOT, "tests", "golden", "pose_k200_l64.json")
        if os.path.exists(gold):
            g = json.load(open(gold))
            if g.get("workload") == "pose n=200 L=64 seed=0":
                ref = np.asarray(g["trace"][:K])
        d_star = float(max(trace.max(), ref.max() if ref is not None else -np.inf))
        eps = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5]
        gpu_tt = time_to_bound(trace, t_iter, d_star, eps)
        cpu_tt = time_to_bound(ref if ref is not None else trace, cb["s_per_iter"], d_star, eps)
        cpu1_tt = time_to_bound(ref if ref is not None else trace, s1, d_star, eps)
        result["time_to_dual_bound"] = {
            "d_star": d_star, "eps_rel": eps, "gpu_s": gpu_tt, "plain_oracle_s": cpu_tt,
            "plain_oracle_one_thread_s": cpu1_tt, "oracle_cores": cb["cores"],
            "note": "seconds until the dual bound reaches D* - eps|D*| (D* = best value of either run after "
                    f"{K} iterations): GPU = its trace's iterations x its measured time per iteration; plain "
                    "oracle = the iterations of its own stored trace x its measured seconds per iteration"}
    s.close()
    if not args.no_stream:
        sp = measured_stream_peak()
        med, best = M.stream_read_probe(4 << 30, 5)
        sp.update(hip_read_gbs=med, hip_read_best_gbs=best)
        ceiling = max(sp["read_gbs"], med)
        result["measured_stream"] = dict(sp, frac_of_measured_read=gbs / ceiling,
                                         note="torch sum (read) and copy_ (read + write) over 4 GiB, and the "
                                              "library's plain HIP read kernel over 4 GiB (median and best of 5); "
                                              "frac_of_measured_read uses the larger median read rate; the "
                                              "roofline peak stays the published 8 TB/s")
    if not args.no_batch:
        result["batched"] = bench_batched(M, W, per_problem=not args.no_per_problem)
    if not args.no_c2:
        result["c2"] = bench_c2(M, W, with_cpu=not args.no_cpu)
    if not args.no_adjoint:
        result["adjoint"] = bench_adjoint(M, W)
    if not args.no_rules:
        result["rules"] = bench_rules(M, W)
    if not args.no_gap:
        result["gap"] = bench_gap(M, W)
    if not args.no_potts:
        result["potts"] = bench_potts(M, W)
    if not args.no_trunc_linear:
        result["trunc_linear"] = bench_trunc_linear(M, W)
    if not args.no_trunc_quad:
        result["trunc_quad"] = bench_trunc_linear(M, W, kind=M.COST_TRUNC_QUAD, tau=64.0)
    result["summary"] = summary(result)
    print(json.dumps(result))


if __name__ == "__main__":
    main()

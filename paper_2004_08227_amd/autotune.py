"""Autotuner of the launch choices: the engine, threads per workgroup and
grid of a single model, and the engine, LDS residency, queue and planner
constants of a batch.

Every choice is a schedule and tiling decision only: each edge update is the
same IEEE operations in the same order whatever runs it, so every candidate
must give bitwise the same state and dual bounds.  The tuner checks that for
each candidate it times (a candidate that differs raises ``AssertionError``)
and keeps the fastest by the library's own device timing (HIP events on its
stream).  Results are kept in a JSON table keyed by the kind of run, dtype,
tile size and size bucket; ``apply_solver`` / ``apply_batch`` set a handle's
options from it.

    python -m paper_2004_08227_amd.autotune --out paper_2004_08227_amd/tuned.json

runs the tuner on the synthetic workloads of ``workloads.py`` (one GPU) and
writes the table that ``load_table()`` reads.
"""
import argparse
import json
import math
import os

import numpy as np

from . import workloads as W

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def _M():
    import paper_2004_08227_amd as M
    return M


def next_tile(L):
    for t in (16, 32, 64, 128):
        if L <= t:
            return t
    raise ValueError("L above the library maximum")


def solver_key(dtype, L, n, m):
    """Table key of a single model: dtype, tile size, and the log2 buckets of
    the node count and of the mean edges per node."""
    dens = 2.0 * m / max(1, n)
    return f"solver/{'f32' if np.dtype(dtype) == np.float32 else 'f64'}/lt{next_tile(L)}/" \
           f"n{int(math.log2(max(1, n)))}/d{int(math.log2(max(1.0, dens)))}"


def batch_key(models):
    """Table key of a batch: its size bucket and largest tile."""
    lt = max(next_tile(mo.L) for mo in models)
    edges = sum(mo.m for mo in models)
    return f"batch/lt{lt}/models{int(math.log2(max(1, len(models))))}/edges{int(math.log2(max(1, edges)))}"


def load_table(path=TABLE_PATH):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def apply_solver(solver, model, table=None):
    """Sets a solver's options from the table entry of its model (if any);
    returns the options applied."""
    M = _M()
    table = load_table() if table is None else table
    entry = table.get(solver_key(solver.dtype, model.L, model.n, model.m))
    if not entry:
        return {}
    opts = entry["options"]
    for k, v in opts.items():
        solver.set_option(getattr(M, k), v)
    return opts


def apply_batch(batch, models, table=None):
    """Sets a batch's options from the table entry of its models (if any)."""
    table = load_table() if table is None else table
    entry = table.get(batch_key(models))
    if not entry:
        return {}
    for k, v in entry["options"].items():
        batch.set_option(k, v)
    return entry["options"]


# ---------------------------------------------------------------------------
# single models
# ---------------------------------------------------------------------------
def solver_candidates(M, solver):
    """Options worth timing for this handle: the persistent engine at each
    valid thread count (FP32 up to 32 labels: also one compute wave, 64) and
    a few grids, and the per-matching engine; for
    FP32 handles also where a workgroup keeps its messages (LDS or global
    memory) and how far ahead the tables are prefetched (one step or two),
    at the default threads and grid and at the grid of one workgroup per
    edge of a matching when that differs."""
    L = solver.info("L")
    lt = next_tile(L)
    f32 = solver.info("dtype") == M.F32
    cands = [{}]
    threads = [nt for nt in (256, 512, 1024) if nt <= 16 * lt and (not f32 or nt <= 512)]
    if f32 and lt <= 32:
        threads = [64] + threads   # one compute wave (the mailbox engine)
    for nt in threads:
        for grid in (0, 128, 192):
            c = {"OPT_ENGINE": M.ENGINE_PERSISTENT, "OPT_THREADS": nt}
            if grid:
                c["OPT_GRID"] = grid
            cands.append(c)
    cands.append({"OPT_ENGINE": M.ENGINE_STEP})
    if f32:
        for phi, pre in ((2, 0), (0, 1), (2, 1)):
            c = {"OPT_ENGINE": M.ENGINE_PERSISTENT}
            if phi:
                c["OPT_PHI"] = phi
            if pre and lt <= 64:
                c["OPT_PREFETCH"] = pre
            if len(c) > 1:
                cands.append(c)
    return cands


def _time_solver(M, make, c, U0, phi0, iters):
    with make() as s:
        for k, v in c.items():
            s.set_option(getattr(M, k), v)
        s.iterate(2)
        s.set_state(U0, phi0)
        s.iterate(iters)
        return s.last_iterate_ms() / iters, s.get_state(comp=True), s.dual_bound()


def tune_solver(model, iters=20, make=None, log=None, gain=0.97, repeats=2):
    """Times every candidate on `model` from phi = 0 for `iters` iterations;
    returns (chosen options, {candidate: ms per iteration}).  Candidates the
    handle refuses (MPLPXX_EINVAL) are skipped.  The defaults are kept
    unless the fastest candidate beats them by more than 1 - `gain` and
    still does, on average, over `repeats` more interleaved runs of both
    (the spread between runs of one configuration is a few percent)."""
    M = _M()
    make = make or (lambda: M.Solver.from_model(model))
    with make() as s:
        U0, phi0 = s.get_state()
        cands = solver_candidates(M, s)
    ref = None
    times = {}
    for c in cands:
        try:
            ms, state, d = _time_solver(M, make, c, U0, phi0, iters)
        except M.MplpError:
            continue
        if ref is None:
            ref = (state, d)
        else:
            for a, b in zip(ref[0], state):
                assert np.array_equal(a, b), f"candidate {c} changed the state"
            assert d == ref[1], f"candidate {c} changed the dual bound"
        key = json.dumps(c, sort_keys=True)
        times[key] = ms
        if log:
            log(f"  {key}: {ms:.4f} ms/iter")
    default = json.dumps({}, sort_keys=True)
    best = min(times, key=times.get)
    if best == default or times[best] > gain * times[default]:
        return {}, times
    c_best = json.loads(best)
    tb = [_time_solver(M, make, c_best, U0, phi0, iters)[0] for _ in range(repeats)]
    td = [_time_solver(M, make, {}, U0, phi0, iters)[0] for _ in range(repeats)]
    if log:
        log(f"  confirm {best}: {np.mean(tb):.4f} vs defaults {np.mean(td):.4f} ms/iter")
    return (c_best if np.mean(tb) < 0.98 * np.mean(td) else {}), times


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------
BATCH_DEFAULTS = {"engine": 0, "lds": 1, "queue": 1, "one_per_model": 0, "wave_lat_mb_us": 2.0,
                  "wave_lat_lds_us": 2.4, "wave_edge16_us": 0.05, "wave_edge32_us": 0.08, "wave_edge64_us": 0.13}
BATCH_CHOICES = {"engine": [0, 1, 2], "lds": [1, 0], "queue": [1, 0], "one_per_model": [0, 1],
                 "wave_lat_mb_us": [1.0, 2.0, 4.0], "wave_lat_lds_us": [1.2, 2.4, 4.8],
                 "wave_edge16_us": [0.025, 0.05, 0.1], "wave_edge32_us": [0.04, 0.08, 0.16],
                 "wave_edge64_us": [0.08, 0.13, 0.2]}


PLAN_INFO = ("engine", "grid", "tasks", "teams", "max_team", "lds_tasks", "lds_bytes")


def _time_batch(b, opts, iters):
    """Sets every batch option (the defaults where `opts` has none), runs
    `iters` iterations from phi = 0 after a warm-up that plans and captures
    the launch, and returns (ms per iteration, duals, state of model 0, the
    plan's summary)."""
    for k, v in dict(BATCH_DEFAULTS, **opts).items():
        b.set_option(k, v)
    b.reset()
    b.iterate(2)
    b.reset()
    b.iterate(iters)
    # (the queue switch changes how the same tasks are taken, not the plan)
    plan = tuple(b.info(k) for k in PLAN_INFO) + (round(b.info("plan_us"), 3), dict(BATCH_DEFAULTS, **opts)["queue"])
    return b.info("last_ms") / iters, b.dual_bounds(), b.get_state(0, comp=True), plan


def tune_batch(models, iters=10, rounds=2, log=None, gain=0.97, repeats=2):
    """Coordinate descent over the batch options from the defaults, on one
    batch whose options change between runs: each round tries every value of
    every option with the others fixed.  A value whose plan is the current
    one is not timed; one that is faster by more than 1 - `gain` is kept if
    it still is, on average, over `repeats` more interleaved runs of both.
    Returns (options that differ from the defaults, best ms per iteration,
    default ms per iteration).  Values the batch refuses (an engine that
    cannot run these models) are skipped."""
    M = _M()
    best = dict(BATCH_DEFAULTS)
    with M.Batch(models) as b:
        best_ms, d_ref, s_ref, best_plan = _time_batch(b, best, iters)
        default_ms = best_ms
        if log:
            log(f"  defaults: {best_ms:.4f} ms/iter")
        for _ in range(rounds):
            improved = False
            for key, values in BATCH_CHOICES.items():
                for v in values:
                    if v == best[key]:
                        continue
                    cand = dict(best, **{key: v})
                    try:
                        ms, d, s0, plan = _time_batch(b, cand, iters)
                    except M.MplpError:
                        continue
                    assert np.array_equal(d, d_ref), f"{key}={v} changed the dual bounds"
                    for x, y in zip(s0, s_ref):
                        assert np.array_equal(x, y), f"{key}={v} changed the state"
                    if log:
                        log(f"  {key}={v}: {ms:.4f} ms/iter" + (" (same plan)" if plan == best_plan else ""))
                    if plan == best_plan or ms >= gain * best_ms:
                        continue
                    tc, tb = [], []
                    for _ in range(repeats):
                        tc.append(_time_batch(b, cand, iters)[0])
                        tb.append(_time_batch(b, best, iters)[0])
                    if log:
                        log(f"  confirm {key}={v}: {np.mean(tc):.4f} vs {np.mean(tb):.4f} ms/iter")
                    if np.mean(tc) < 0.98 * np.mean(tb):
                        best, best_ms, best_plan, improved = cand, float(np.mean(tc)), plan, True
            if not improved:
                break
    return {k: v for k, v in best.items() if v != BATCH_DEFAULTS[k]}, best_ms, default_ms


# ---------------------------------------------------------------------------
# the table for the workloads of workloads.py
# ---------------------------------------------------------------------------
def build_table(log=print, quick=False):
    table = {}
    solver_models = [W.pose(200, 64, seed=0), W.potts_er(1000, 16, 0.05, seed=0), W.potts_er(1000, 16, 0.25, seed=0),
                     W.potts_er(1000, 16, 1.0, seed=0), W.uniform(100, 32, seed=0).astype(np.float32)]
    if quick:
        solver_models = solver_models[:1]
    for mo in solver_models:
        key = solver_key(mo.unaries.dtype, mo.L, mo.n, mo.m)
        log(f"{key} ({mo.name})")
        opts, times = tune_solver(mo, log=log)
        table[key] = {"options": opts, "ms_per_iter": times, "workload": mo.name}
    models = W.batched_mix(64 if quick else 256, seed=0)
    key = batch_key(models)
    log(f"{key} (batched mix of {len(models)})")
    opts, ms, ms0 = tune_batch(models, log=log, rounds=1 if quick else 2)
    table[key] = {"options": opts, "ms_per_iter": ms, "default_ms_per_iter": ms0,
                  "workload": f"batched_mix({len(models)}, seed=0)"}
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--quick", action="store_true", help="one model and a 64-model batch")
    args = ap.parse_args()
    table = build_table(quick=args.quick)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps({"written": args.out, "keys": sorted(table)}))


if __name__ == "__main__":
    main()

"""FP64 CPU oracle for MPLP++ (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The solver library never imports it and it imports nothing
from the solver: the C source ``mplp_oracle.c`` is compiled with plain gcc
into ``liboracle.so`` and called through ctypes.

Every function follows a passage of the paper (Tourani et al., "MPLP++",
ECCV 2018):

* ``canonicalize``  edge orientation u < v (Sec. 3, "Notation");
* ``schedule``      Alg. 1 "Compute Edge Schedule" (Sec. 6);
* ``update``        one BCA update (U), (M) or (H) on one edge (Sec. 4);
* ``run``           BCA-iterations over the schedule (Sec. 5 definition,
                    Sec. 6 order), state = reparametrized costs (Eq. 2);
* ``dual``          the lower bound of Eq. (3);
* ``decode``        sequential primal rounding, Eq. (5);
* ``energy``        the energy of Eq. (1);
* ``bruteforce``    exhaustive MAP (the argmin of Eq. (1));
* ``dual_after``    D after K iterations as a function of the input costs,
                    for finite differences;
* ``dual_derivative`` the directional derivative of that function, by
                    forward-mode differentiation of the (H) iterations
                    (minima take the derivative of their lowest-index
                    minimizer).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mplp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# a different build of the oracle (the mutation tests load planted mistakes)
_LIB_OVERRIDE = os.environ.get("MPLP_ORACLE_LIB")
_lock = threading.Lock()
_lib = None

RULES = {"H": 0, "M": 1, "U": 2}

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (-O2, OpenMP, no fast-math, no FP
    contraction)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build()
            lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_canonicalize.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p, _f64p, _f64p,
                                         _i32p, _f64p]
        lib.orc_canonicalize.restype = ctypes.c_int
        lib.orc_schedule.argtypes = [ctypes.c_int, ctypes.c_int64, _i32p, _i32p, _i32p]
        lib.orc_schedule.restype = ctypes.c_int
        lib.orc_schedule_kind.argtypes = [ctypes.c_int, ctypes.c_int64, _i32p, ctypes.c_int, _i32p, _i32p]
        lib.orc_schedule_kind.restype = ctypes.c_int
        lib.orc_update.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, _f64p, _f64p]
        lib.orc_update.restype = ctypes.c_int
        lib.orc_dual.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _f64p, _f64p]
        lib.orc_dual.restype = ctypes.c_double
        lib.orc_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p, ctypes.c_int, _i32p, _i32p,
                                _f64p, _f64p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_run_tangent.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p, ctypes.c_int, _i32p,
                                        _i32p, _f64p, _f64p, _f64p, _f64p, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.orc_run_tangent.restype = ctypes.c_int
        lib.orc_decode.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p, _f64p, _f64p, _i32p]
        lib.orc_decode.restype = ctypes.c_int
        lib.orc_energy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p, _f64p, _f64p, _i32p]
        lib.orc_energy.restype = ctypes.c_double
        lib.orc_bruteforce.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p, _f64p, _f64p, _i32p]
        lib.orc_bruteforce.restype = ctypes.c_double
        lib.orc_openmp_max_threads.argtypes = []
        lib.orc_openmp_max_threads.restype = ctypes.c_int
        _lib = lib
        return lib


class OracleError(ValueError):
    pass


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def canonicalize(n, L, edges, unaries, pairwise):
    """Returns (edges with u < v, tables re-indexed [label u][label v]) as
    int32 / float64 arrays; raises OracleError on invalid input."""
    lib = _load()
    edges = _i32(edges).reshape(-1, 2)
    m = edges.shape[0]
    un = _f64(unaries).reshape(n, L)
    pw = _f64(pairwise).reshape(m, L, L) if m else np.zeros((0, L, L))
    e_out = np.empty_like(edges)
    pw_out = np.empty((m, L, L), dtype=np.float64)
    rc = lib.orc_canonicalize(n, L, m, edges, un, np.ascontiguousarray(pw), e_out, pw_out)
    if rc != 0:
        raise OracleError(f"invalid model (code {rc})")
    return e_out, pw_out


def schedule(n, edges, kind="greedy"):
    """Alg. 1 on canonical edges (u < v): returns (step_ptr int32 [S+1],
    order int32 [m]).  kind "greedy": round-robin for a complete graph,
    greedy maximal matchings otherwise; "color": round-robin for a complete
    graph, the colour classes of a Delta + 1 edge colouring otherwise."""
    lib = _load()
    edges = _i32(edges).reshape(-1, 2)
    m = edges.shape[0]
    step_ptr = np.zeros(m + 2, dtype=np.int32)
    order = np.zeros(max(m, 1), dtype=np.int32)
    if kind not in ("greedy", "color"):
        raise OracleError(f"unknown schedule kind {kind}")
    S = lib.orc_schedule_kind(n, m, edges, 0 if kind == "greedy" else 1, step_ptr, order)
    if S < 0:
        raise OracleError(f"schedule failed (code {S})")
    return step_ptr[:S + 1].copy(), order[:m].copy()


def update(rule, Te, Tu_u, Tu_v):
    """One BCA update (Sec. 4) on copies of one edge's state; returns the new
    (Te, Tu_u, Tu_v)."""
    lib = _load()
    Te = _f64(Te).copy()
    Tu_u = _f64(Tu_u).copy()
    Tu_v = _f64(Tu_v).copy()
    L = Tu_u.shape[0]
    assert Te.shape == (L, L) and Tu_v.shape == (L,)
    rc = lib.orc_update(RULES[rule], L, Te, Tu_u, Tu_v)
    if rc != 0:
        raise OracleError(f"update failed (code {rc})")
    return Te, Tu_u, Tu_v


def dual(Tu, Te):
    lib = _load()
    Tu = _f64(Tu)
    Te = _f64(Te)
    n, L = Tu.shape
    m = Te.shape[0]
    return float(lib.orc_dual(n, L, m, Tu, Te))


class State:
    """Reparametrized costs theta^phi (Eq. 2) of one model plus its schedule."""

    def __init__(self, model, step_ptr=None, order=None, schedule_kind="greedy"):
        self.n = int(model.n)
        self.L = int(model.L)
        self._edges_in = _i32(model.edges).reshape(-1, 2)
        self.edges, self.pairwise = canonicalize(self.n, self.L, model.edges, model.unaries, model.pairwise)
        self.unaries = _f64(model.unaries).reshape(self.n, self.L).copy()
        self.m = int(self.edges.shape[0])
        if step_ptr is None:
            step_ptr, order = schedule(self.n, self.edges, schedule_kind)
        self.step_ptr = _i32(step_ptr)
        self.order = _i32(order)
        self.Tu = self.unaries.copy()
        self.Te = self.pairwise.copy()
        self.iterations = 0

    @property
    def n_steps(self):
        return int(self.step_ptr.shape[0] - 1)

    def run(self, iters, rule="H", trace=False, nthreads=1):
        lib = _load()
        tr = np.zeros(max(iters, 1), dtype=np.float64) if trace else None
        rc = lib.orc_run(self.n, self.L, self.m, self.edges, self.n_steps, self.step_ptr, self.order, self.Tu,
                         self.Te, RULES[rule], int(iters), tr.ctypes.data if trace else None, int(nthreads))
        if rc != 0:
            raise OracleError(f"run failed (code {rc})")
        self.iterations += iters
        return tr[:iters].copy() if trace else None

    def dual(self):
        return dual(self.Tu, self.Te)

    def run_tangent(self, iters, du, dp, nthreads=1):
        """Runs ``iters`` (H) iterations (bitwise as ``run``) carrying the
        derivative of the state along the direction (du [n][L], dp [m][L][L]
        in the model's edge order and orientation); returns the derivative
        of D (Eq. 3) after them."""
        lib = _load()
        _, dTe = canonicalize(self.n, self.L, self._edges_in, _f64(du), _f64(dp))
        dTu = _f64(du).reshape(self.n, self.L).copy()
        out = ctypes.c_double(0.0)
        rc = lib.orc_run_tangent(self.n, self.L, self.m, self.edges, self.n_steps, self.step_ptr, self.order,
                                 self.Tu, self.Te, dTu, dTe, int(iters), ctypes.byref(out), int(nthreads))
        if rc != 0:
            raise OracleError(f"tangent run failed (code {rc})")
        self.iterations += iters
        return float(out.value)

    def decode(self):
        lib = _load()
        labels = np.zeros(self.n, dtype=np.int32)
        rc = lib.orc_decode(self.n, self.L, self.m, self.edges, self.Tu, self.Te, labels)
        if rc != 0:
            raise OracleError(f"decode failed (code {rc})")
        return labels

    def energy(self, labels, reparametrized=False):
        lib = _load()
        if reparametrized:
            return float(lib.orc_energy(self.n, self.L, self.m, self.edges, self.Tu, self.Te, _i32(labels)))
        return float(lib.orc_energy(self.n, self.L, self.m, self.edges, self.unaries, self.pairwise,
                                    _i32(labels)))


def energy(model, labels):
    st = State(model, step_ptr=np.zeros(1, np.int32), order=np.zeros(0, np.int32))
    return st.energy(labels)


def bruteforce(model):
    """Exhaustive MAP (argmin of Eq. (1)); returns (energy, labels)."""
    lib = _load()
    n, L = int(model.n), int(model.L)
    if float(L) ** n > 5e7:
        raise OracleError("brute force limited to L^n <= 5e7 labellings")
    edges, pw = canonicalize(n, L, model.edges, model.unaries, model.pairwise)
    un = _f64(model.unaries).reshape(n, L)
    best = np.zeros(n, dtype=np.int32)
    en = lib.orc_bruteforce(n, L, edges.shape[0], edges, un, pw, best)
    return float(en), best


def run_model(model, iters, rule="H", trace=True, nthreads=1, schedule_kind="greedy"):
    st = State(model, schedule_kind=schedule_kind)
    tr = st.run(iters, rule=rule, trace=trace, nthreads=nthreads)
    return st, tr


def dual_after(model, iters, rule="H", nthreads=1):
    """D of Eq. (3) after ``iters`` iterations from phi = 0, as a function of
    the model's costs."""
    st = State(model)
    st.run(iters, rule=rule, nthreads=nthreads)
    return st.dual()


def dual_derivative(model, iters, du, dp, nthreads=1):
    """Directional derivative of ``dual_after(model, iters)`` (rule (H))
    along (du, dp) (arrays shaped like the model's unaries and pairwise
    costs), exact for the linear piece that the run's minimizers select
    (lowest index on ties)."""
    st = State(model)
    return st.run_tangent(iters, du, dp, nthreads=nthreads)


def max_threads():
    return int(_load().orc_openmp_max_threads())

"""mplpxx — MPLP++ dual block-coordinate ascent on AMD MI355X (gfx950).

Thin ctypes binding of ``libmplpxx.so`` (C ABI in ``include/mplpxx.h``).  The
binding only marshals arguments: every step of the solver runs in the
library's HIP kernels.  PyTorch is used only to hand over device memory and
streams (``Solver.from_torch``).  There is no CPU fallback: if the library is
not built, every call raises.

Paper: Tourani et al., "MPLP++: Fast, Parallel Dual Block-Coordinate Ascent
for Dense Graphical Models", ECCV 2018.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MPLPXX_RUNTIME=rocm: the build linked against /opt/rocm's HIP runtime, and
# no PyTorch (for profiling under rocprofv3: one HIP/HSA runtime per process)
ROCM_ONLY = os.environ.get("MPLPXX_RUNTIME") == "rocm"
LIB_PATH = os.path.join(_HERE, "libmplpxx_rocm.so" if ROCM_ONLY else "libmplpxx.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mplpxx.h")

F32, F64 = 0, 1
OK, EINVAL, ENOMEM, EDEVICE, ETIMEOUT, ESTATE = 0, -1, -2, -3, -4, -5
MAX_LABELS = 128
OPT_ENGINE, OPT_THREADS, OPT_GRID, OPT_SPIN_LIMIT, OPT_PROFILE, OPT_ADJOINT_F64, OPT_RULE = 1, 2, 3, 4, 5, 6, 7
OPT_PHI, OPT_PREFETCH = 8, 9
RULE_H, RULE_M, RULE_U = 0, 1, 2
SCHED_AUTO, SCHED_GREEDY, SCHED_COLOR = 0, 1, 2
COST_POTTS, COST_TRUNC_LINEAR, COST_TRUNC_QUAD = 1, 2, 3
COST_PARAMS = {COST_POTTS: 1, COST_TRUNC_LINEAR: 2, COST_TRUNC_QUAD: 2}
ENGINE_AUTO, ENGINE_STEP, ENGINE_PERSISTENT = 0, 1, 2
BOPT = {"grid": 1, "graph": 2, "spin_limit": 3, "one_per_model": 4, "handoff_us": 5, "edge16_us": 6,
        "edge32_us": 7, "edge64_us": 8, "edge128_us": 9, "lds": 10, "engine": 11, "wave_edge16_us": 12,
        "wave_edge32_us": 13, "wave_edge64_us": 14, "wave_lat_lds_us": 15, "wave_lat_mb_us": 16,
        "queue": 17}
BINFO = {"count": 1, "grid": 2, "tasks": 3, "teams": 4, "max_team": 5, "plan_us": 6, "edges": 7, "last_ms": 8,
         "table_bytes": 9, "lds_tasks": 10, "lds_bytes": 11, "engine": 12, "waves": 13,
         "wg_max_us": 14, "wg_mean_us": 15}
INFO = {"n": 1, "L": 2, "m": 3, "steps": 4, "dtype": 5, "engine": 6, "grid": 7, "threads": 8, "iterations": 9,
        "wallclock_khz": 10, "adjoint_bytes": 11}

_lib = None
# open handles; closed by an exit hook before the interpreter shuts down, so
# that no handle is freed by a finalizer after the HIP runtime has begun its
# own teardown
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


class MplpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mplpxx error {code}: {msg}")
        self.code = code


def header_symbols():
    """Names of the functions declared in include/mplpxx.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mplpxx_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Loads libmplpxx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                           "or python paper_2004_08227_amd/build.py")
    if not ROCM_ONLY:
        try:
            # load PyTorch's HIP runtime first: the library then binds to the
            # same runtime (same soname), so device pointers and streams can
            # be shared
            import torch  # noqa: F401
        except ImportError:
            pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "mplpxx_create": (ctypes.c_int, [i32, i32, i64, vp, vp, vp, i32, pp]),
        "mplpxx_create_sched": (ctypes.c_int, [i32, i32, i64, vp, vp, vp, i32, i32, pp]),
        "mplpxx_create_device": (ctypes.c_int, [i32, i32, i64, vp, vp, vp, i32, vp, pp]),
        "mplpxx_iterate": (ctypes.c_int, [vp, i32]),
        "mplpxx_iterate_trace": (ctypes.c_int, [vp, i32, vp]),
        "mplpxx_dual_bound": (ctypes.c_int, [vp, ctypes.POINTER(dbl)]),
        "mplpxx_decode": (ctypes.c_int, [vp, vp, ctypes.POINTER(dbl)]),
        "mplpxx_destroy": (None, [vp]),
        "mplpxx_error_string": (ctypes.c_char_p, [ctypes.c_int]),
        "mplpxx_last_error": (ctypes.c_char_p, []),
        "mplpxx_set_stream": (ctypes.c_int, [vp, vp]),
        "mplpxx_get_schedule": (ctypes.c_int, [vp, vp, vp, vp]),
        "mplpxx_get_state": (ctypes.c_int, [vp, vp, vp, vp]),
        "mplpxx_schedule": (ctypes.c_int, [i32, i64, vp, vp, vp, vp]),
        "mplpxx_schedule_kind": (ctypes.c_int, [i32, i64, vp, i32, vp, vp, vp]),
        "mplpxx_set_state": (ctypes.c_int, [vp, vp, vp, vp]),
        "mplpxx_set_option": (ctypes.c_int, [vp, i32, i64]),
        "mplpxx_get_info": (ctypes.c_int, [vp, i32, ctypes.POINTER(i64)]),
        "mplpxx_last_iterate_ms": (ctypes.c_int, [vp, ctypes.POINTER(dbl)]),
        "mplpxx_get_step_profile": (ctypes.c_int, [vp, vp]),
        "mplpxx_adjoint_forward": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(dbl)]),
        "mplpxx_adjoint_backward": (ctypes.c_int, [vp, vp, vp]),
        "mplpxx_iterate_gap": (ctypes.c_int, [vp, i32, vp, vp, vp]),
        "mplpxx_batch_create": (ctypes.c_int, [i32, vp, vp, vp, vp, vp, vp, pp]),
        "mplpxx_batch_create_potts": (ctypes.c_int, [i32, vp, vp, vp, vp, vp, vp, pp]),
        "mplpxx_create_potts": (ctypes.c_int, [i32, i32, i64, vp, vp, vp, pp]),
        "mplpxx_create_structured": (ctypes.c_int, [i32, i32, i64, vp, vp, i32, vp, pp]),
        "mplpxx_batch_create_structured": (ctypes.c_int, [i32, vp, vp, vp, vp, vp, i32, vp, pp]),
        "mplpxx_batch_iterate": (ctypes.c_int, [vp, i32]),
        "mplpxx_batch_dual_bounds": (ctypes.c_int, [vp, vp]),
        "mplpxx_batch_get_state": (ctypes.c_int, [vp, i32, vp, vp, vp]),
        "mplpxx_batch_reset": (ctypes.c_int, [vp]),
        "mplpxx_batch_set_option": (ctypes.c_int, [vp, i32, dbl]),
        "mplpxx_batch_get_info": (ctypes.c_int, [vp, i32, ctypes.POINTER(dbl)]),
        "mplpxx_batch_wg_profile": (ctypes.c_int, [vp, vp, vp]),
        "mplpxx_batch_destroy": (None, [vp]),
        "mplpxx_solve_noalloc": (ctypes.c_int, [i32, i32, i64, vp, vp, vp, i32, vp, vp, ctypes.POINTER(dbl), vp]),
        "mplpxx_stream_read_probe": (ctypes.c_int, [i64, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise MplpError(rc, lib().mplpxx_last_error().decode())


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def stream_read_probe(nbytes=4 << 30, reps=5):
    """(median, best) streaming-read rate of the current device in GB/s
    from the library's plain read kernel over `nbytes` bytes (the measured
    ceiling beside the published HBM bandwidth)."""
    med, best = ctypes.c_double(), ctypes.c_double()
    _check(lib().mplpxx_stream_read_probe(int(nbytes), int(reps), ctypes.byref(med), ctypes.byref(best)))
    return med.value, best.value


def schedule(n, edges, kind=0):
    """Host-only schedule of Alg. 1 for a graph: (step_ptr [S+1], order [m]);
    kind: SCHED_AUTO, SCHED_GREEDY or SCHED_COLOR."""
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    m = edges.shape[0]
    S = ctypes.c_int32()
    sp = np.zeros(m + 1, dtype=np.int32)
    order = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().mplpxx_schedule_kind(int(n), int(m), _ptr(edges) if m else None, int(kind), ctypes.byref(S),
                                      _ptr(sp), _ptr(order)))
    return sp[:S.value + 1].copy(), order[:m].copy()


def _check_device_costs(torch, n, L, m, unaries, pairwise):
    """Argument checks of Solver.from_torch (ValueError, never assert)."""
    for name, t in (("unaries", unaries), ("pairwise", pairwise)):
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name} must be a torch tensor")
        if not t.is_cuda:
            raise ValueError(f"{name} must be on the GPU (got {t.device})")
        if t.dtype not in (torch.float32, torch.float64):
            raise ValueError(f"{name} must be float32 or float64 (got {t.dtype})")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if pairwise.dtype != unaries.dtype:
        raise ValueError(f"unaries and pairwise must share a dtype (got {unaries.dtype}, {pairwise.dtype})")
    if pairwise.device != unaries.device:
        raise ValueError(f"unaries and pairwise must be on one device (got {unaries.device}, {pairwise.device})")
    if unaries.device.index is not None and unaries.device.index != torch.cuda.current_device():
        raise ValueError(f"the tensors must be on the current device cuda:{torch.cuda.current_device()}")
    if tuple(unaries.shape) != (n, L):
        raise ValueError(f"unaries must have shape ({n}, {L}), got {tuple(unaries.shape)}")
    if tuple(pairwise.shape) != (m, L, L):
        raise ValueError(f"pairwise must have shape ({m}, {L}, {L}), got {tuple(pairwise.shape)}")


class Solver:
    """One model: ``Solver(n, L, edges, unaries, pairwise)`` with host numpy
    arrays (float32 or float64), or ``Solver.from_torch`` with device tensors."""

    def __init__(self, n, L, edges, unaries, pairwise, dtype=None, _handle=None, schedule=0):
        self._h = None
        if _handle is not None:
            self._h = _handle
        else:
            if dtype is None:
                dtype = np.asarray(unaries).dtype
            dt = np.dtype(dtype)
            if dt not in (np.float32, np.float64):
                raise ValueError("dtype must be float32 or float64")
            edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
            m = edges.shape[0]
            un = np.ascontiguousarray(unaries, dtype=dt)
            pw = np.ascontiguousarray(pairwise, dtype=dt)
            if un.size != n * L or pw.size != m * L * L:
                raise ValueError("unaries must hold n*L and pairwise m*L*L values")
            h = ctypes.c_void_p()
            _check(lib().mplpxx_create_sched(int(n), int(L), int(m), _ptr(edges) if m else None, _ptr(un),
                                             _ptr(pw) if m else None, F32 if dt == np.float32 else F64,
                                             int(schedule), ctypes.byref(h)))
            self._h = h
        _LIVE.add(self)
        self.n = self.info("n")
        self.L = self.info("L")
        self.m = self.info("m")
        self.dtype = np.float32 if self.info("dtype") == F32 else np.float64

    @classmethod
    def from_model(cls, model, schedule=0):
        return cls(model.n, model.L, model.edges, model.unaries, model.pairwise, schedule=schedule)

    @classmethod
    def from_potts(cls, model):
        """A Potts model (``mplpxx_create_potts``): ``model.pairwise`` holds
        one weight per edge [m] (pairwise term w_e [s != t]); FP32."""
        edges = np.ascontiguousarray(model.edges, dtype=np.int32).reshape(-1, 2)
        m = edges.shape[0]
        un = np.ascontiguousarray(model.unaries, dtype=np.float32)
        w = np.ascontiguousarray(model.pairwise, dtype=np.float32)
        if un.size != model.n * model.L or w.size != m:
            raise ValueError("unaries must hold n*L and weights m values")
        h = ctypes.c_void_p()
        _check(lib().mplpxx_create_potts(int(model.n), int(model.L), int(m), _ptr(edges) if m else None, _ptr(un),
                                         _ptr(w) if m else None, ctypes.byref(h)))
        return cls(model.n, model.L, None, None, None, _handle=h)

    @classmethod
    def from_structured(cls, model, kind):
        """A model with structured pairwise costs (``mplpxx_create_structured``):
        ``model.pairwise`` holds the parameters per edge [m, P] (Potts: w;
        truncated linear: w, tau); FP32."""
        edges = np.ascontiguousarray(model.edges, dtype=np.int32).reshape(-1, 2)
        m = edges.shape[0]
        un = np.ascontiguousarray(model.unaries, dtype=np.float32)
        prm = np.ascontiguousarray(model.pairwise, dtype=np.float32)
        if un.size != model.n * model.L or prm.size != m * COST_PARAMS.get(kind, 0):
            raise ValueError("unaries must hold n*L values and params m*P (P parameters of the cost kind)")
        h = ctypes.c_void_p()
        _check(lib().mplpxx_create_structured(int(model.n), int(model.L), int(m), _ptr(edges) if m else None, _ptr(un),
                                              int(kind), _ptr(prm) if m else None, ctypes.byref(h)))
        return cls(model.n, model.L, None, None, None, _handle=h)

    @classmethod
    def from_torch(cls, n, L, edges, unaries, pairwise, stream=None):
        """unaries [n, L] and pairwise [m, L, L]: contiguous float32/float64
        torch tensors of one dtype on the current GPU; edges: host int32
        [m, 2].  Raises ValueError before any library call otherwise (a
        host pointer handed to the device copy would fault the GPU)."""
        import torch  # (device memory and streams only)
        edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        m = edges.shape[0]
        _check_device_costs(torch, int(n), int(L), m, unaries, pairwise)
        dt = F32 if unaries.dtype == torch.float32 else F64
        h = ctypes.c_void_p()
        st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(lib().mplpxx_create_device(int(n), int(L), int(m), _ptr(edges) if m else None,
                                          ctypes.c_void_p(unaries.data_ptr()),
                                          ctypes.c_void_p(pairwise.data_ptr()) if m else None, dt, st,
                                          ctypes.byref(h)))
        return cls(n, L, None, None, None, _handle=h)

    # ------------------------------------------------------------------
    def close(self):
        if self._h is not None:
            lib().mplpxx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------
    def iterate(self, k=1):
        _check(lib().mplpxx_iterate(self._h, int(k)))

    def iterate_trace(self, k):
        tr = np.zeros(max(int(k), 1), dtype=np.float64)
        _check(lib().mplpxx_iterate_trace(self._h, int(k), _ptr(tr)))
        return tr[:k]

    def dual_bound(self):
        d = ctypes.c_double()
        _check(lib().mplpxx_dual_bound(self._h, ctypes.byref(d)))
        return d.value

    def decode(self):
        labels = np.zeros(self.n, dtype=np.int32)
        e = ctypes.c_double()
        _check(lib().mplpxx_decode(self._h, _ptr(labels), ctypes.byref(e)))
        return labels, e.value

    def schedule(self):
        S = ctypes.c_int32()
        _check(lib().mplpxx_get_schedule(self._h, ctypes.byref(S), None, None))
        sp = np.zeros(S.value + 1, dtype=np.int32)
        order = np.zeros(max(self.m, 1), dtype=np.int32)
        _check(lib().mplpxx_get_schedule(self._h, None, _ptr(sp), _ptr(order)))
        return sp, order[:self.m]

    def get_state(self, comp=False):
        """(U, phi), or (U, phi, U_comp) with comp=True: FP32 unaries are
        U + U_comp (a bf16 correction; zeros for FP64)."""
        U = np.zeros((self.n, self.L), dtype=self.dtype)
        phi = np.zeros((self.m, 2, self.L), dtype=self.dtype)
        c = np.zeros((self.n, self.L), dtype=np.float32) if comp else None
        _check(lib().mplpxx_get_state(self._h, _ptr(U), _ptr(phi) if self.m else None, _ptr(c)))
        return (U, phi, c) if comp else (U, phi)

    def set_state(self, U=None, phi=None, comp=None):
        U = None if U is None else np.ascontiguousarray(U, dtype=self.dtype).reshape(self.n, self.L)
        phi = None if phi is None else np.ascontiguousarray(phi, dtype=self.dtype).reshape(self.m, 2, self.L)
        comp = None if comp is None else np.ascontiguousarray(comp, dtype=np.float32).reshape(self.n, self.L)
        _check(lib().mplpxx_set_state(self._h, _ptr(U), _ptr(phi), _ptr(comp)))

    def set_option(self, key, value):
        _check(lib().mplpxx_set_option(self._h, int(key), int(value)))

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream (or None for the library default)."""
        _check(lib().mplpxx_set_stream(self._h, None if stream is None else ctypes.c_void_p(stream.cuda_stream)))

    def info(self, key):
        v = ctypes.c_int64()
        _check(lib().mplpxx_get_info(self._h, INFO[key], ctypes.byref(v)))
        return v.value

    def iterate_gap(self, k):
        """k iterations; after each the certified dual (Eq. 3) and the energy
        of the Eq. (5) rounding.  Returns (dual [k], energy [k], best labels)."""
        d = np.zeros(k, np.float64)
        e = np.zeros(k, np.float64)
        lab = np.zeros(self.n, np.int32)
        _check(lib().mplpxx_iterate_gap(self._h, int(k), d.ctypes.data, e.ctypes.data, lab.ctypes.data))
        return d, e, lab

    def adjoint_forward(self, K, every=10):
        """K iterations from phi = 0 with checkpoints every `every`; returns
        D_K = sum_u min_s U_u(s)."""
        d = ctypes.c_double()
        _check(lib().mplpxx_adjoint_forward(self._h, int(K), int(every), ctypes.byref(d)))
        return d.value

    def adjoint_backward_device(self, grad_unaries, grad_pairwise):
        """Writes dD_K/dunaries and dD_K/dpairwise into contiguous torch
        tensors on the GPU (the handle's dtype, the caller's layouts)."""
        _check(lib().mplpxx_adjoint_backward(self._h, ctypes.c_void_p(grad_unaries.data_ptr()),
                                             ctypes.c_void_p(grad_pairwise.data_ptr()) if self.m else None))

    def adjoint_backward(self):
        """Host copies (numpy) of the gradients of the last adjoint_forward."""
        import torch
        dt = torch.float32 if self.dtype == np.float32 else torch.float64
        gu = torch.empty((self.n, self.L), dtype=dt, device="cuda")
        gp = torch.empty((max(self.m, 1), self.L, self.L), dtype=dt, device="cuda")
        self.adjoint_backward_device(gu, gp)
        torch.cuda.synchronize()
        return gu.cpu().numpy(), gp[:self.m].cpu().numpy()

    def step_profile(self):
        """[m, 4] int64 timestamps (slot order) of the last iteration."""
        st = np.zeros((max(self.m, 1), 4), dtype=np.int64)
        _check(lib().mplpxx_get_step_profile(self._h, _ptr(st)))
        return st[:self.m]

    def last_iterate_ms(self):
        d = ctypes.c_double()
        _check(lib().mplpxx_last_iterate_ms(self._h, ctypes.byref(d)))
        return d.value


def solve_noalloc(edges, unaries, pairwise, iters, U_out, phi_out, stream=None):
    """``mplpxx_solve_noalloc``: `iters` iterations from phi = 0 of the FP32
    model (unaries [n, L], pairwise [m, L, L] float32 CUDA tensors; edges host
    int32 [m, 2]) with no device allocation; writes U [n, L] and phi
    [m, 2, L] into the float32 CUDA tensors U_out, phi_out and returns the
    dual bound of Eq. (3)."""
    import torch  # (device memory and streams only)
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    m = edges.shape[0]
    n, L = (int(x) for x in unaries.shape)
    _check_device_costs(torch, n, L, m, unaries, pairwise)
    for name, t, shape in (("U_out", U_out, (n, L)), ("phi_out", phi_out, (m, 2, L))):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and tuple(t.shape) == shape and t.device == unaries.device):
            raise ValueError(f"{name} must be a contiguous float32 tensor of shape {shape} on {unaries.device}")
    if unaries.dtype != torch.float32:
        raise ValueError("solve_noalloc takes float32 costs")
    d = ctypes.c_double()
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(lib().mplpxx_solve_noalloc(n, L, m, _ptr(edges) if m else None, ctypes.c_void_p(unaries.data_ptr()),
                                      ctypes.c_void_p(pairwise.data_ptr()) if m else None, int(iters),
                                      ctypes.c_void_p(U_out.data_ptr()), ctypes.c_void_p(phi_out.data_ptr()) if m else None,
                                      ctypes.byref(d), st))
    return d.value


class Batch:
    """Many independent FP32 models solved together (``mplpxx_batch_*``).
    ``kind`` (COST_POTTS, COST_TRUNC_LINEAR, COST_TRUNC_QUAD; ``potts=True`` means COST_POTTS):
    every model's ``pairwise`` holds the cost's parameters per edge [m, P]
    (``mplpxx_batch_create_structured``)."""

    def __init__(self, models, potts=False, kind=0):
        count = len(models)
        kind = COST_POTTS if potts and not kind else int(kind)
        self.models = models
        self.n = np.array([mo.n for mo in models], dtype=np.int32)
        self.L = np.array([mo.L for mo in models], dtype=np.int32)
        self.m = np.array([mo.m for mo in models], dtype=np.int64)
        keep = []
        e_ptrs = (ctypes.c_void_p * count)()
        u_ptrs = (ctypes.c_void_p * count)()
        p_ptrs = (ctypes.c_void_p * count)()
        for i, mo in enumerate(models):
            e = np.ascontiguousarray(mo.edges, dtype=np.int32)
            u = np.ascontiguousarray(mo.unaries, dtype=np.float32)
            pw = np.ascontiguousarray(mo.pairwise, dtype=np.float32)
            if kind and pw.size != mo.m * COST_PARAMS.get(kind, 0):
                raise ValueError("structured models take the cost's parameters per edge")
            keep += [e, u, pw]
            e_ptrs[i] = e.ctypes.data if mo.m else None
            u_ptrs[i] = u.ctypes.data
            p_ptrs[i] = pw.ctypes.data if mo.m else None
        h = ctypes.c_void_p()
        if kind:
            _check(lib().mplpxx_batch_create_structured(count, _ptr(self.n), _ptr(self.L), _ptr(self.m), e_ptrs, u_ptrs,
                                                        kind, p_ptrs, ctypes.byref(h)))
        else:
            _check(lib().mplpxx_batch_create(count, _ptr(self.n), _ptr(self.L), _ptr(self.m), e_ptrs, u_ptrs, p_ptrs,
                                             ctypes.byref(h)))
        self._h = h
        _LIVE.add(self)
        self.count = count

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().mplpxx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def iterate(self, k):
        _check(lib().mplpxx_batch_iterate(self._h, int(k)))

    def dual_bounds(self):
        out = np.zeros(self.count, dtype=np.float64)
        _check(lib().mplpxx_batch_dual_bounds(self._h, _ptr(out)))
        return out

    def get_state(self, i, comp=False):
        n, L, m = int(self.n[i]), int(self.L[i]), int(self.m[i])
        U = np.zeros((n, L), dtype=np.float32)
        phi = np.zeros((m, 2, L), dtype=np.float32)
        c = np.zeros((n, L), dtype=np.float32) if comp else None
        _check(lib().mplpxx_batch_get_state(self._h, int(i), _ptr(U), _ptr(phi) if m else None, _ptr(c)))
        return (U, phi, c) if comp else (U, phi)

    def reset(self):
        _check(lib().mplpxx_batch_reset(self._h))

    def set_option(self, key, value):
        _check(lib().mplpxx_batch_set_option(self._h, BOPT[key], float(value)))

    def info(self, key):
        v = ctypes.c_double()
        _check(lib().mplpxx_batch_get_info(self._h, BINFO[key], ctypes.byref(v)))
        return v.value

    def wg_profile(self):
        """(start_end_us [grid, 2], team_model [grid]) of the last launch:
        each logical workgroup's start and end (microseconds after the
        earliest start) and the model of its own team task (-1: queue only)."""
        g = int(self.info("grid"))
        se = np.zeros((g, 2), np.float64)
        tm = np.zeros(g, np.int32)
        _check(lib().mplpxx_batch_wg_profile(self._h, se.ctypes.data, tm.ctypes.data))
        return se, tm


def solve_batch(models, iters, potts=False, tuned=True, states=False):
    """Solves `models` together for `iters` iterations in one persistent
    launch (``Batch``), with the autotuner's options for such a batch when
    ``tuned`` (the committed table; results are the same bits either way).
    Returns the dual bounds [count] (FP64), and with ``states`` also the
    list of (U, phi) per model."""
    with Batch(models, potts=potts) as b:
        if tuned:
            from . import autotune
            autotune.apply_batch(b, models)
        b.iterate(iters)
        d = b.dual_bounds()
        if states:
            return d, [b.get_state(i) for i in range(len(models))]
        return d

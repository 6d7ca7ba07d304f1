"""Seeded synthetic pairwise MRF generators.

This module only draws inputs: it holds none of the solver's arithmetic and is
the single piece of code that both the HIP path and the CPU oracle are fed
from.  Every model is a triple (edges, unaries, pairwise) in the layout of the
energy of Eq. (1) in Sec. 3 of the paper:

* ``edges``    int32 [m, 2], each row (u, v) with u < v (the paper's edge
  orientation convention, Sec. 3 "Notation"), lexicographic order;
* ``unaries``  float [n, L], theta_u(s);
* ``pairwise`` float [m, L, L], theta_uv(s, t) with rows indexed by the label
  s of the lower node u and columns by the label t of v.

Draw order (numpy ``default_rng`` = PCG64): unaries first, then the graph (for
random graphs), then the pairwise potentials in edge order.  The workloads
stand in for the paper's datasets (Sec. 7), which are not available here:

* ``tiny``      K_8, L=4, i.i.d. uniform[0,1) costs (FP64 brute-force size);
* ``pose``      fully connected 6D-pose-shaped model (Sec. 7 "pose"): label s
  of node u is a 3D point p_us in the unit cube, node u has a model point
  q_u, and theta_uv(s,t) = min((| |p_us - p_vt| - |q_u - q_v| |)^2, tau).
  q_u is planted as p_{u, s*_u} for a random s*_u so that a zero-pairwise
  labelling exists, as for a real object under a correct pose;
* ``potts_er``  Erdos-Renyi graph of given density (the sparsification study
  of Sec. 7), Potts weight w_uv ~ U[0.1, 1] on s != t plus U[0, 0.2) noise;
* ``uniform``   fully connected, i.i.d. uniform[0,1) costs (the
  differentiation workload);
* ``batched_mix`` 256 pose-shaped models with n ~ U{20..300}, L ~ U{8..64}.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_GEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen")
_GEN_SRC = os.path.join(_GEN_DIR, "pose_tables.c")
_GEN_LIB = os.path.join(_GEN_DIR, "libpose_tables.so")
_gen = None


def build_generator() -> str:
    """Compiles the C helper that fills pose tables (OpenMP)."""
    tmp = _GEN_LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-o", tmp, _GEN_SRC, "-lm"], check=True)
    os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _gen_lib():
    global _gen
    if _gen is None and os.path.exists(_GEN_LIB) and os.path.getmtime(_GEN_LIB) >= os.path.getmtime(_GEN_SRC):
        g = ctypes.CDLL(_GEN_LIB)
        g.pose_tables.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.c_void_p]
        g.pose_tables.restype = None
        _gen = g
    return _gen


def pose_tables(edges, P, Q, tau, dtype=np.float32, use_c=True, chunk=4096):
    """table[e][s][t] = min((|P[u][s]-P[v][t]| - |Q[u]-Q[v]|)^2, tau) in FP64,
    rounded once; the C helper and the numpy path give the same bits."""
    m = edges.shape[0]
    L = P.shape[1]
    g = _gen_lib() if (use_c and dtype == np.float32) else None
    if g is not None:
        out = np.empty((m, L, L), dtype=np.float32)
        e = np.ascontiguousarray(edges, dtype=np.int32)
        Pc = np.ascontiguousarray(P, dtype=np.float64)
        Qc = np.ascontiguousarray(Q, dtype=np.float64)
        g.pose_tables(m, L, e.ctypes.data, Pc.ctypes.data, Qc.ctypes.data, float(tau), out.ctypes.data)
        return out
    out = np.empty((m, L, L), dtype=dtype)
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        u = edges[lo:hi, 0]
        v = edges[lo:hi, 1]
        q = Q[u] - Q[v]
        dq = np.sqrt((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2])[:, None, None]
        dif = P[u][:, :, None, :] - P[v][:, None, :, :]
        dp = np.sqrt((dif[..., 0] * dif[..., 0] + dif[..., 1] * dif[..., 1]) + dif[..., 2] * dif[..., 2])
        d = dp - dq
        out[lo:hi] = np.minimum(d * d, tau).astype(dtype)
    return out


@dataclass
class Model:
    n: int
    L: int
    edges: np.ndarray      # int32 [m, 2], u < v
    unaries: np.ndarray    # float [n, L]
    pairwise: np.ndarray   # float [m, L, L]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])

    def astype(self, dtype) -> "Model":
        return Model(self.n, self.L, self.edges,
                     np.ascontiguousarray(self.unaries, dtype=dtype),
                     np.ascontiguousarray(self.pairwise, dtype=dtype), self.name)


def complete_edges(n: int) -> np.ndarray:
    """All pairs u < v in lexicographic order, int32 [n(n-1)/2, 2]."""
    iu, iv = np.triu_indices(n, k=1)
    return np.ascontiguousarray(np.stack([iu, iv], axis=1).astype(np.int32))


def tiny(seed: int = 0, n: int = 8, L: int = 4, dtype=np.float64) -> Model:
    rng = np.random.default_rng(seed)
    unaries = rng.random((n, L))
    edges = complete_edges(n)
    pairwise = rng.random((edges.shape[0], L, L))
    return Model(n, L, edges, unaries.astype(dtype), pairwise.astype(dtype), f"tiny_n{n}_L{L}_s{seed}")


def uniform(n: int, L: int, seed: int = 0, dtype=np.float32) -> Model:
    rng = np.random.default_rng(seed)
    unaries = rng.random((n, L))
    edges = complete_edges(n)
    pairwise = rng.random((edges.shape[0], L, L))
    return Model(n, L, edges, unaries.astype(dtype), pairwise.astype(dtype), f"uniform_n{n}_L{L}_s{seed}")


def pose(n: int, L: int, seed: int = 0, tau: float = 0.04, dtype=np.float32,
         chunk: int = 4096) -> Model:
    """Fully connected pose-shaped model; pairwise is built in float64 and
    rounded once to ``dtype``."""
    rng = np.random.default_rng(seed)
    unaries = rng.random((n, L))
    P = rng.random((n, L, 3))
    star = rng.integers(0, L, size=n)
    Q = P[np.arange(n), star]                       # planted model points [n, 3]
    edges = complete_edges(n)
    pairwise = pose_tables(edges, P, Q, tau, dtype=dtype, chunk=chunk)
    return Model(n, L, edges, unaries.astype(dtype), pairwise, f"pose_n{n}_L{L}_s{seed}")


def potts_er(n: int, L: int, density: float, seed: int = 0, dtype=np.float32) -> Model:
    rng = np.random.default_rng(seed)
    unaries = rng.random((n, L))
    allpairs = complete_edges(n)
    if density >= 1.0:
        edges = allpairs
    else:
        keep = rng.random(allpairs.shape[0]) < density
        edges = np.ascontiguousarray(allpairs[keep])
    m = edges.shape[0]
    w = rng.uniform(0.1, 1.0, size=m)
    noise = rng.uniform(0.0, 0.2, size=(m, L, L))
    off = 1.0 - np.eye(L)
    pairwise = w[:, None, None] * off[None] + noise
    return Model(n, L, edges, unaries.astype(dtype), pairwise.astype(dtype),
                 f"potts_er_n{n}_L{L}_p{density}_s{seed}")


def potts_pure(n: int, L: int, density: float, seed: int = 0, w_range=(0.1, 1.0)):
    """Potts model w_uv [s != t] on G(n, density) (complete for density >= 1),
    w_uv ~ U[w_range], unaries U[0,1): (weights model, dense model) with the
    same edges and unaries; the dense model's tables are the expansion
    of the weights, w_uv off the diagonal and exactly +0 on it (FP32)."""
    rng = np.random.default_rng(seed)
    unaries = rng.random((n, L)).astype(np.float32)
    if density >= 1.0:
        edges = complete_edges(n)
    else:
        iu = np.triu_indices(n, 1)
        keep = rng.random(iu[0].shape[0]) < density
        edges = np.stack([iu[0][keep], iu[1][keep]], axis=1).astype(np.int32)
    w = rng.uniform(w_range[0], w_range[1], size=edges.shape[0]).astype(np.float32)
    name = f"potts_pure_n{n}_L{L}_p{density}_s{seed}"
    weights = Model(n, L, edges, unaries, w, name + "_weights")
    eye = np.eye(L, dtype=bool)[None, :, :]
    dense = Model(n, L, edges, unaries, np.where(eye, np.float32(0.0), w[:, None, None]).astype(np.float32), name)
    return weights, dense


def trunc_linear(n: int, L: int, density: float, seed: int = 0, tau=4.0, w_range=(0.05, 0.5), integer: bool = False):
    """Truncated linear model w_uv min(|s - t|, tau) on G(n, density)
    (complete for density >= 1), w_uv ~ U[w_range] (``integer``: w and the
    unaries small integers, so that many sums tie), unaries U[0,1): (params
    model with pairwise [m, 2] = (w, tau) per edge, dense model) with the same
    edges and unaries.  The dense tables are the expansion in FP32:
    th(s, t) = fl(w * min(|s - t|, tau)).  ``tau`` may be a number or an
    array of m values.  Stands in for the smoothness costs of the paper's
    stereo and segmentation datasets (Sec. 7)."""
    rng = np.random.default_rng(seed)
    if integer:
        unaries = rng.integers(0, 4, size=(n, L)).astype(np.float32)
    else:
        unaries = rng.random((n, L)).astype(np.float32)
    if density >= 1.0:
        edges = complete_edges(n)
    else:
        iu = np.triu_indices(n, 1)
        keep = rng.random(iu[0].shape[0]) < density
        edges = np.stack([iu[0][keep], iu[1][keep]], axis=1).astype(np.int32)
    m = edges.shape[0]
    if integer:
        w = rng.integers(0, 3, size=m).astype(np.float32)
    else:
        w = rng.uniform(w_range[0], w_range[1], size=m).astype(np.float32)
    t = np.broadcast_to(np.asarray(tau, dtype=np.float32), (m,)).astype(np.float32)
    name = f"trunc_linear_n{n}_L{L}_p{density}_s{seed}"
    params = Model(n, L, edges, unaries, np.stack([w, t], axis=1).astype(np.float32), name + "_params")
    d = np.abs(np.arange(L)[:, None] - np.arange(L)[None, :]).astype(np.float32)
    dense = Model(n, L, edges, unaries, (w[:, None, None] * np.minimum(d[None], t[:, None, None])).astype(np.float32),
                  name)
    return params, dense


def trunc_quad(n: int, L: int, density: float, seed: int = 0, tau=16.0, w_range=(0.005, 0.05),
               integer: bool = False):
    """Truncated quadratic model w_uv min((s - t)^2, tau) on G(n, density)
    (complete for density >= 1), w_uv ~ U[w_range] (``integer``: w and the
    unaries small integers, so that many sums tie), unaries U[0,1): (params
    model with pairwise [m, 2] = (w, tau) per edge, dense model) with the same
    edges and unaries.  The dense tables are the expansion in FP32:
    th(s, t) = fl(w * min((s - t)^2, tau)) ((s - t)^2 is exact).  ``tau`` may
    be a number or an array of m values; tau >= (L - 1)^2 gives the plain
    quadratic cost.  Stands in for the smoothness costs of the paper's
    stereo-type datasets (Sec. 7)."""
    rng = np.random.default_rng(seed)
    if integer:
        unaries = rng.integers(0, 4, size=(n, L)).astype(np.float32)
    else:
        unaries = rng.random((n, L)).astype(np.float32)
    if density >= 1.0:
        edges = complete_edges(n)
    else:
        iu = np.triu_indices(n, 1)
        keep = rng.random(iu[0].shape[0]) < density
        edges = np.stack([iu[0][keep], iu[1][keep]], axis=1).astype(np.int32)
    m = edges.shape[0]
    if integer:
        w = rng.integers(0, 3, size=m).astype(np.float32)
    else:
        w = rng.uniform(w_range[0], w_range[1], size=m).astype(np.float32)
    t = np.broadcast_to(np.asarray(tau, dtype=np.float32), (m,)).astype(np.float32)
    name = f"trunc_quad_n{n}_L{L}_p{density}_s{seed}"
    params = Model(n, L, edges, unaries, np.stack([w, t], axis=1).astype(np.float32), name + "_params")
    d = (np.arange(L)[:, None] - np.arange(L)[None, :]).astype(np.float32)
    d2 = d * d
    dense = Model(n, L, edges, unaries, (w[:, None, None] * np.minimum(d2[None], t[:, None, None])).astype(np.float32),
                  name)
    return params, dense


def batched_mix(count: int = 256, seed: int = 0, n_range=(20, 300), L_range=(8, 64),
                dtype=np.float32, models: bool = True):
    """Sizes (and, if ``models``, the models) of the batched pose-shaped mix.
    Model i is ``pose(n_i, L_i, seed=1_000_003 * seed + i)``."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=count)
    sizes = [(int(a), int(b)) for a, b in zip(ns, Ls)]
    if not models:
        return sizes
    return [pose(n, L, seed=1_000_003 * seed + i, dtype=dtype) for i, (n, L) in enumerate(sizes)]


def random_graph_model(n: int, L: int, density: float, seed: int = 0, dtype=np.float64,
                       lo: float = 0.0, hi: float = 1.0) -> Model:
    """Small random model on a G(n, p) graph with i.i.d. uniform costs (tests)."""
    rng = np.random.default_rng(seed)
    unaries = rng.uniform(lo, hi, size=(n, L))
    allpairs = complete_edges(n)
    keep = rng.random(allpairs.shape[0]) < density
    edges = np.ascontiguousarray(allpairs[keep])
    pairwise = rng.uniform(lo, hi, size=(edges.shape[0], L, L))
    return Model(n, L, edges, unaries.astype(dtype), pairwise.astype(dtype), f"rg_n{n}_L{L}_p{density}_s{seed}")


def chain(n: int, L: int, seed: int = 0, dtype=np.float64) -> Model:
    rng = np.random.default_rng(seed)
    unaries = rng.random((n, L))
    edges = np.ascontiguousarray(np.stack([np.arange(n - 1), np.arange(1, n)], axis=1).astype(np.int32))
    pairwise = rng.random((n - 1, L, L))
    return Model(n, L, edges, unaries.astype(dtype), pairwise.astype(dtype), f"chain_n{n}_L{L}_s{seed}")


# The five workloads the measurements and parity tests are quoted on.
CONFIGS = {
    "tiny_k8_l4_fp64": dict(kind="tiny", n=8, L=4, iters=200),
    "pose_k200_l64": dict(kind="pose", n=200, L=64, iters=200),
    "potts_er_n1000_l16": dict(kind="potts_er", n=1000, L=16, densities=(0.05, 0.25, 0.5, 1.0)),
    "batched_pose_mix_256": dict(kind="batched_mix", count=256, iters=100),
    "uniform_k100_l32_adjoint": dict(kind="uniform", n=100, L=32, K=50, every=10),
}

"""Element-wise comparison of an FP32 GPU state with the FP64 oracle's.

The GPU keeps each reparametrized unary as U + U_comp (FP32 plus a bf16
correction) and each edge's messages phi; the oracle keeps the
reparametrized costs themselves (Eq. 2): Tu[u][s] and
Te[e][s][t] = theta_e(s, t) - phi[e][0][s] - phi[e][1][t].  Both are compared
in FP64 at the same bar as the dual bound: |gpu - oracle| <= TOL *
max(1, |oracle|) for every entry checked."""
import numpy as np

TOL = 1e-5


def gpu_unaries(U, U_comp):
    return U.astype(np.float64) + U_comp.astype(np.float64)


def gpu_pairwise(pairwise, phi):
    """Reparametrized pairwise costs of every edge (edges given u < v)."""
    ph = phi.astype(np.float64)
    return pairwise.astype(np.float64) - ph[:, 0, :, None] - ph[:, 1, None, :]


def worst(gpu, ref):
    gpu = np.asarray(gpu, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    if gpu.size == 0:
        return 0.0
    return float(np.max(np.abs(gpu - ref) / np.maximum(1.0, np.abs(ref))))


def sampled_errors(model, U, U_comp, phi, sample):
    """Worst relative errors (unaries, pairwise) at the stored sample of the
    oracle's state (indices into Tu [n][L] and Te [m][L][L])."""
    assert np.all(model.edges[:, 0] < model.edges[:, 1])
    Ug = gpu_unaries(U, U_comp).ravel()
    iu = np.asarray(sample["unary_index"], np.int64)
    eu = worst(Ug[iu], sample["unary"])
    ip = np.asarray(sample["pair_index"], np.int64)
    L = model.L
    e, rest = np.divmod(ip, L * L)
    s, t = np.divmod(rest, L)
    ph = phi.astype(np.float64)
    te = model.pairwise[e, s, t].astype(np.float64) - ph[e, 0, s] - ph[e, 1, t]
    ep = worst(te, sample["pair"])
    return eu, ep

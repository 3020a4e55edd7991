"""Shared helpers of the GPU parity tests (imported only by tests)."""
import sys

import numpy as np

import oracle


def say(*a):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_03180_amd import md
    md.lib()


def force_error(gpu_f, ref):
    """e_F = max_i |F_i^gpu - F_i^ref| / A_i with A_i = sum_j |f_ij| r_ij (atoms with
    A_i == 0 must have exactly zero force on both sides)."""
    d = np.sqrt((gpu_f[0] - ref["fx"]) ** 2 + (gpu_f[1] - ref["fy"]) ** 2 +
                (gpu_f[2] - ref["fz"]) ** 2)
    A = ref["a_atom"]
    zero = A == 0.0
    assert np.all(d[zero] == 0.0), "force on an atom without interacting pairs"
    if np.all(zero):
        return 0.0
    return float(np.max(d[~zero] / A[~zero]))


def random_charges(sys, seed, hi=3):
    rng = np.random.default_rng(seed)
    qm = sys.qmax[sys.elem]
    return np.minimum(rng.integers(0, hi, sys.n_atoms), qm).astype(np.int8)


def sorted_pairs(p):
    p = np.asarray(p, dtype=np.int64)
    if p.size == 0:
        return p.reshape(0, 2)
    a = np.minimum(p[:, 0], p[:, 1])
    b = np.maximum(p[:, 0], p[:, 1])
    o = np.lexsort((b, a))
    return np.stack([a[o], b[o]], axis=1)


def oracle_kappa(sys, k):
    return oracle.kappa_from_lambda(sys.lambda_d[:, k])

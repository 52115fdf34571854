"""Helpers shared by the GPU tests (device placement, oracle comparisons)."""
import numpy as np

DEV = "cuda:0"


def torch():
    import torch as t

    return t


def to_dev(a: np.ndarray, dtype=None):
    t = torch()
    x = t.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return x if dtype is None else x.to(dtype)


def empty_like_padded(n, p, dtype, pad=0, offset=0):
    """(storage, view): an n x (p) view inside an n x (p + pad) tensor at column `offset`."""
    t = torch()
    base = t.zeros((n, p + pad), dtype=dtype, device=DEV)
    return base, base[:, offset: offset + p]


def rel_fro(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def max_rel(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))

"""Shared helpers of the GPU tests (no arithmetic of the method)."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def soft_mask(n, rng):
    return rng.uniform(0.0, 1.0, size=(n, n)).astype(np.float32)


def rand_c(shape, rng, scale=1.0):
    return (scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex64)

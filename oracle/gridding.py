"""FP64 CPU oracle of the gridding of radial k-space samples (test
infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product path never does.  It shares no
code with the HIP library.

What it computes.  The paper interpolates the measured non-Cartesian data
onto the Cartesian grid once, before the reconstruction (Sec. 3.1), and
doubles the grid so that this interpolation is accurate (Sec. 3.2).  Here
that step is convolution gridding with a Kaiser-Bessel window:

  samples   spoke s (angle theta_s) carries R samples at radii
            r_i = i - R/2 (grid units), position k_si = (n/2, n/2) + r_i (cos theta_s, sin theta_s);
  window    phi(u) = kb(u_0) kb(u_1),  kb(u) = I0(beta sqrt(1 - (2u/W)^2)) / I0(beta) for |u| <= W/2, else 0;
  gridding  G d [kappa] = sum_{s,i} w_i d_si phi(kappa - k_si)     (w: density compensation per radius);
  adjoint   (G^H g)_si = w_i sum_kappa phi(kappa - k_si) g[kappa],
with kappa - k_si taken on the periodic grid: a window that crosses the grid
edge wraps around (the DFT of the reconstruction is periodic in k).

G applied to all-ones data gives the gridded sampling density (the point
spread function's k-space weights that the reconstruction uses as P).

Readings where the paper is silent (also listed in the design notes): the
window (Kaiser-Bessel, width W, shape beta; W = 4 and the beta of Beatty et
al. for 2x oversampling by default), the radii (unit spacing on the doubled
grid, i.e. two samples per Nyquist interval of the base matrix), the
density compensation (an optional per-radius weight, |r| for a ramp), and no
deapodisation inside the reconstruction (the image is not divided by the
window's transform; the pins below do so only to compare with a direct
non-uniform Fourier sum).
"""
from __future__ import annotations

import math

import numpy as np


def default_beta(width: float, oversampling: float = 2.0) -> float:
    """Beatty et al. (2005) shape for a Kaiser-Bessel window of `width` grid
    cells at the given grid oversampling."""
    return math.pi * math.sqrt((width / oversampling) ** 2 * (oversampling - 0.5) ** 2 - 0.8)


def kb(u, width: float, beta: float):
    """1-D Kaiser-Bessel window, 1 at u = 0, 0 for |u| > width/2."""
    u = np.asarray(u, np.float64)
    t = 1.0 - (2.0 * u / width) ** 2
    out = np.zeros_like(u)
    inside = t >= 0.0
    out[inside] = np.i0(beta * np.sqrt(t[inside])) / np.i0(beta)
    return out


def radial_positions(n: int, angles, R: int):
    """k positions [S, R, 2] (grid index units, DC at n/2) of R samples per spoke."""
    r = np.arange(R, dtype=np.float64) - R // 2
    th = np.asarray(angles, np.float64)
    k0 = n / 2 + r[None, :] * np.cos(th)[:, None]
    k1 = n / 2 + r[None, :] * np.sin(th)[:, None]
    return np.stack([k0, k1], axis=-1)


def _window(k, h, width, beta):
    """Grid indices within h of position k (not yet reduced mod n) and the
    window's weights there."""
    idx = np.arange(math.ceil(k - h), math.floor(k + h) + 1)
    return idx, kb(idx - k, width, beta)


def grid(data, angles, n: int, width: float, beta: float, dcf=None) -> np.ndarray:
    """G d: data [J, S, R] -> grid [J, n, n], visiting every sample and every
    grid point inside its window."""
    data = np.asarray(data, np.complex128)
    J, S, R = data.shape
    pos = radial_positions(n, angles, R)
    w = np.ones(R) if dcf is None else np.asarray(dcf, np.float64)
    out = np.zeros((J, n, n), np.complex128)
    h = width / 2.0
    for s in range(S):
        for i in range(R):
            i0, a = _window(pos[s, i, 0], h, width, beta)
            i1, b = _window(pos[s, i, 1], h, width, beta)
            for u, au in zip(i0, a):
                for v, bv in zip(i1, b):
                    out[:, u % n, v % n] += w[i] * data[:, s, i] * au * bv
    return out


def grid_ones(angles, R: int, n: int, width: float, beta: float, dcf=None) -> np.ndarray:
    """G 1: the gridded sampling density [n, n] (real)."""
    ones = np.ones((1, len(angles), R), np.complex128)
    return np.real(grid(ones, angles, n, width, beta, dcf)[0])


def degrid(g, angles, R: int, width: float, beta: float, dcf=None) -> np.ndarray:
    """G^H g: grid [J, n, n] -> samples [J, S, R]."""
    g = np.asarray(g, np.complex128)
    J, n = g.shape[0], g.shape[-1]
    pos = radial_positions(n, angles, R)
    w = np.ones(R) if dcf is None else np.asarray(dcf, np.float64)
    out = np.zeros((J, len(angles), R), np.complex128)
    h = width / 2.0
    for s in range(len(angles)):
        for i in range(R):
            i0, a = _window(pos[s, i, 0], h, width, beta)
            i1, b = _window(pos[s, i, 1], h, width, beta)
            acc = np.zeros(J, np.complex128)
            for u, au in zip(i0, a):
                for v, bv in zip(i1, b):
                    acc += g[:, u % n, v % n] * au * bv
            out[:, s, i] = w[i] * acc
    return out

"""FP64 CPU oracle of the NLINV reconstruction (test infrastructure only).

This module is the plain, slow reference the GPU library is checked against.
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it; the product path never does.  It shares no code with the HIP
library and imports nothing from it.

What it computes (Schaetz & Uecker, Sec. 3.1):
  * the forward operator F = P_k . DTFT . M_Omega . C . W^{-1}   (Eq. 2),
  * its Frechet derivative DF and the adjoint DF^H,
  * one iteratively regularised Gauss-Newton (IRGNM) step (Eq. 3):
        (DF^H DF + alpha_n I)(x_{n+1} - x_n) = DF^H (y - F x_n) - alpha_n (x_n - x_ref),
    solved with plain conjugate gradients (CG),
  * the Newton loop around it, the combined image, a temporal series with the
    previous frame as x_ref (Sec. 3.2), and the gradient of F with respect to
    a real k-space weighting P.

Readings of the paper where it is silent (each is listed in the design notes):
  * DTFT: centred (DC at index n/2) and unitary in both directions.
  * W = diag(w) . DTFT on the coil sensitivities, w(k) = (1 + a|k|^2)^(l/2)
    with k_d = (kappa_d - n/2)/n, a = 220, l = 32, so W^{-1} chat = DTFT^{-1}(chat / w).
  * M_Omega restricts the image to a centred n_om x n_om rectangle; the image
    unknown rho lives on that rectangle (E = zero padding, E^H = crop).
  * P_k is a real array P on the grid; the normal operator therefore holds P^2.
  * alpha_n = max(alpha0 * q^n, alpha_min); CG starts from 0, runs a fixed
    number of iterations and stops early only on breakdown.
  * data are scaled to ||y|| = scale_norm before the solve (exact, F is bilinear);
    the default start is rho = 1 on Omega and chat = 0 in the scaled problem.

Every array is complex128 / float64 here; inputs arriving as complex64 /
float32 are promoted.  Pins of each function against values fixed by the
mathematics live in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

# FFT worker threads handed to scipy.fft (a library primitive; 1 = serial).
WORKERS = 1


def set_workers(k: int) -> None:
    global WORKERS
    WORKERS = max(1, int(k))


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Dims:
    n: int                 # grid size (square n x n)
    n_om: int              # side of the image region Omega
    ncoils: int
    sob_a: float = 220.0
    sob_l: float = 32.0

    @property
    def lo(self) -> int:   # first grid index of Omega along each axis
        return self.n // 2 - self.n_om // 2


def embed(img: np.ndarray, d: Dims) -> np.ndarray:
    """E: zero-pad an Omega-sized image (..., n_om, n_om) into the grid."""
    out = np.zeros(img.shape[:-2] + (d.n, d.n), dtype=np.complex128)
    out[..., d.lo:d.lo + d.n_om, d.lo:d.lo + d.n_om] = img
    return out


def crop(x: np.ndarray, d: Dims) -> np.ndarray:
    """E^H: restrict a grid array to Omega."""
    return x[..., d.lo:d.lo + d.n_om, d.lo:d.lo + d.n_om].copy()


# ---------------------------------------------------------------------------
# centred unitary DFT (the DTFT of Eq. 2 on the grid)
# ---------------------------------------------------------------------------

def dft2c(x: np.ndarray) -> np.ndarray:
    """(Fx)[kappa] = N^-1/2 sum_r x[r] exp(-2 pi i sum_d (kappa_d - n/2)(r_d - n/2)/n),
    over the last two axes.  The sign follows exp(-i k.x) of Eq. 1."""
    x = np.asarray(x, dtype=np.complex128)
    return np.fft.fftshift(sfft.fft2(np.fft.ifftshift(x, axes=(-2, -1)), norm="ortho",
                                     workers=WORKERS), axes=(-2, -1))


def idft2c(X: np.ndarray) -> np.ndarray:
    """Inverse (= adjoint) of dft2c."""
    X = np.asarray(X, dtype=np.complex128)
    return np.fft.fftshift(sfft.ifft2(np.fft.ifftshift(X, axes=(-2, -1)), norm="ortho",
                                      workers=WORKERS), axes=(-2, -1))


# ---------------------------------------------------------------------------
# Sobolev weight of W (Eq. 2, the smoothness prior on the sensitivities)
# ---------------------------------------------------------------------------

def sobolev_weight(d: Dims) -> np.ndarray:
    """w[kappa] = (1 + a |k|^2)^(l/2), k_d = (kappa_d - n/2)/n."""
    k = (np.arange(d.n, dtype=np.float64) - d.n // 2) / d.n
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    return (1.0 + d.sob_a * k2) ** (d.sob_l / 2.0)


def w_inverse(chat: np.ndarray, d: Dims) -> np.ndarray:
    """W^{-1} chat = DTFT^{-1}(chat / w): coil sensitivities on the grid."""
    return idft2c(np.asarray(chat, dtype=np.complex128) / sobolev_weight(d))


def w_inverse_adjoint(v: np.ndarray, d: Dims) -> np.ndarray:
    """W^{-H} v = DTFT(v) / w."""
    return dft2c(v) / sobolev_weight(d)


def coil_maps(chat: np.ndarray, d: Dims) -> np.ndarray:
    """c_j = E^H W^{-1} chat_j, the sensitivities restricted to Omega."""
    return crop(w_inverse(chat, d), d)


# ---------------------------------------------------------------------------
# operators of Eqs. 2 and 3
# ---------------------------------------------------------------------------

def forward(rho, chat, P, d: Dims, c=None) -> np.ndarray:
    """F(x)_j = P . DTFT(E(rho . c_j))  with c_j = E^H W^{-1} chat_j.
    Operators below take an optional c: the sensitivities at the current
    linearisation point, which the method computes once per Newton step."""
    c = coil_maps(chat, d) if c is None else c
    return np.asarray(P, np.float64) * dft2c(embed(np.asarray(rho, np.complex128) * c, d))


def deriv(rho, chat, P, drho, dchat, d: Dims, c=None) -> np.ndarray:
    """DF_x(drho, dchat)_j = P . DTFT(E(drho . c_j + rho . dc_j)),  dc_j = E^H W^{-1} dchat_j."""
    c = coil_maps(chat, d) if c is None else c
    dc = coil_maps(dchat, d)
    z = np.asarray(drho, np.complex128) * c + np.asarray(rho, np.complex128) * dc
    return np.asarray(P, np.float64) * dft2c(embed(z, d))


def adjoint(rho, chat, P, dy, d: Dims, c=None):
    """DF_x^H z:  u_j = E^H DTFT^{-1}(P . z_j);
    drho = sum_j conj(c_j) . u_j;  dchat_j = W^{-H} E(conj(rho) . u_j)."""
    c = coil_maps(chat, d) if c is None else c
    u = crop(idft2c(np.asarray(P, np.float64) * np.asarray(dy, np.complex128)), d)
    drho = np.sum(np.conj(c) * u, axis=0)
    dchat = w_inverse_adjoint(embed(np.conj(np.asarray(rho, np.complex128)) * u, d), d)
    return drho, dchat


def normal(rho, chat, P, alpha, drho, dchat, d: Dims, c=None):
    """(DF^H DF + alpha I) h, the left-hand side of Eq. 3."""
    c = coil_maps(chat, d) if c is None else c
    g_rho, g_chat = adjoint(rho, chat, P, deriv(rho, chat, P, drho, dchat, d, c=c), d, c=c)
    return g_rho + alpha * np.asarray(drho, np.complex128), \
        g_chat + alpha * np.asarray(dchat, np.complex128)


def mask_gradient(rho, chat, P, g, d: Dims) -> np.ndarray:
    """dL/dP for L depending on y = F(x; P), given g = dL/dRe(y) + i dL/dIm(y):
    Re sum_j conj(g_j) . S_j  with  S_j = DTFT(E(rho . c_j))."""
    c = coil_maps(chat, d)
    S = dft2c(embed(np.asarray(rho, np.complex128) * c, d))
    return np.real(np.sum(np.conj(np.asarray(g, np.complex128)) * S, axis=0))


def inner(a_rho, a_chat, b_rho, b_chat) -> complex:
    """<a, b> = sum conj(a) b over the image part and all sensitivity entries."""
    return complex(np.vdot(a_rho, b_rho) + np.vdot(a_chat, b_chat))


def combined_image(rho, chat, d: Dims) -> np.ndarray:
    """m = rho . sqrt(sum_j |c_j|^2) on Omega."""
    c = coil_maps(chat, d)
    return np.asarray(rho, np.complex128) * np.sqrt(np.sum(np.abs(c) ** 2, axis=0))


# ---------------------------------------------------------------------------
# conjugate gradients and the Gauss-Newton loop
# ---------------------------------------------------------------------------

@dataclass
class CGResult:
    x_rho: np.ndarray
    x_chat: np.ndarray
    rr: list = field(default_factory=list)   # <r,r> after each completed iteration
    breakdown: bool = False
    iters: int = 0


def cg(apply, b_rho, b_chat, iters: int) -> CGResult:
    """Plain Hestenes-Stiefel CG for a Hermitian positive definite operator,
    started from 0, `iters` iterations; stops when <r,r> = 0 or Re<p,Ap> <= 0."""
    x_rho = np.zeros_like(b_rho, dtype=np.complex128)
    x_chat = np.zeros_like(b_chat, dtype=np.complex128)
    r_rho, r_chat = np.array(b_rho, np.complex128), np.array(b_chat, np.complex128)
    p_rho, p_chat = r_rho.copy(), r_chat.copy()
    rr = inner(r_rho, r_chat, r_rho, r_chat).real
    out = CGResult(x_rho, x_chat)
    for _ in range(iters):
        q_rho, q_chat = apply(p_rho, p_chat)
        gamma = inner(p_rho, p_chat, q_rho, q_chat).real
        if rr == 0.0 or gamma <= 0.0:
            out.breakdown = True
            break
        a = rr / gamma
        x_rho += a * p_rho
        x_chat += a * p_chat
        r_rho -= a * q_rho
        r_chat -= a * q_chat
        rr_new = inner(r_rho, r_chat, r_rho, r_chat).real
        beta = rr_new / rr
        p_rho = r_rho + beta * p_rho
        p_chat = r_chat + beta * p_chat
        rr = rr_new
        out.rr.append(rr)
        out.iters += 1
    out.x_rho, out.x_chat = x_rho, x_chat
    return out


@dataclass
class IRGNMParams:
    newton_steps: int = 7
    cg_iters: int = 10
    alpha0: float = 1.0
    alpha_q: float = 0.5
    alpha_min: float = 0.0
    scale_norm: float = 100.0      # 0 disables data scaling


@dataclass
class IRGNMResult:
    rho: np.ndarray                # on Omega, in the units of the input data
    chat: np.ndarray
    image: np.ndarray
    scale: float
    r0_norms: list = field(default_factory=list)
    cg_rr: list = field(default_factory=list)
    breakdown: bool = False


def irgnm(y, P, d: Dims, prm: IRGNMParams, rho0=None, chat0=None,
          rho_ref=None, chat_ref=None) -> IRGNMResult:
    """Newton loop of Eq. 3.  With rho0 = chat0 = None the start is rho = 1 on
    Omega and chat = 0 in the scaled problem; otherwise x0 is given in data
    units and rho0 is scaled with the data.  x_ref defaults to x0."""
    y = np.asarray(y, np.complex128)
    P = np.asarray(P, np.float64)
    ynorm = float(np.linalg.norm(y))
    s = prm.scale_norm / ynorm if (prm.scale_norm > 0 and ynorm > 0) else 1.0
    y = s * y
    if rho0 is None:
        rho = np.ones((d.n_om, d.n_om), np.complex128)
        chat = np.zeros((d.ncoils, d.n, d.n), np.complex128)
    else:
        rho = s * np.asarray(rho0, np.complex128)
        chat = np.array(chat0, np.complex128)
    if rho_ref is None:
        xr_rho, xr_chat = rho.copy(), chat.copy()
    else:
        xr_rho = s * np.asarray(rho_ref, np.complex128)
        xr_chat = np.array(chat_ref, np.complex128)
    out = IRGNMResult(rho, chat, None, s)
    for step in range(prm.newton_steps):
        alpha = max(prm.alpha0 * prm.alpha_q ** step, prm.alpha_min)
        c = coil_maps(chat, d)
        r0 = y - forward(rho, chat, P, d, c=c)
        out.r0_norms.append(float(np.linalg.norm(r0)))
        g_rho, g_chat = adjoint(rho, chat, P, r0, d, c=c)
        b_rho = g_rho - alpha * (rho - xr_rho)
        b_chat = g_chat - alpha * (chat - xr_chat)
        res = cg(lambda hr, hc: normal(rho, chat, P, alpha, hr, hc, d, c=c), b_rho, b_chat,
                 prm.cg_iters)
        out.cg_rr.append(res.rr)
        out.breakdown |= res.breakdown
        rho = rho + res.x_rho
        chat = chat + res.x_chat
    out.rho = rho / s
    out.chat = chat
    out.image = combined_image(out.rho, chat, d)
    return out


def irgnm_series(frames_y, frames_P, d: Dims, prm: IRGNMParams):
    """Temporal series: frame 0 starts from the default guess; frame t > 0
    starts from, and is regularised towards, the result of frame t-1."""
    out = []
    prev = None
    for y, P in zip(frames_y, frames_P):
        if prev is None:
            res = irgnm(y, P, d, prm)
        else:
            res = irgnm(y, P, d, prm, rho0=prev.rho, chat0=prev.chat,
                        rho_ref=prev.rho, chat_ref=prev.chat)
        out.append(res)
        prev = res
    return out

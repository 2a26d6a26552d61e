"""Seeded synthetic MRI inputs for the NLINV reconstruction.

This module only *makes inputs*: a phantom, coil sensitivity profiles,
k-space sampling patterns, measurement noise and random probe vectors.  It
holds none of the reconstruction's arithmetic (no Sobolev weighting, no
Gauss-Newton, no derivative or adjoint).  Its one use of a Fourier transform
simulates the acquisition itself: the signal equation (Eq. 1) of the paper
evaluated on the Cartesian grid, i.e. each coil image rho*c_j is sampled in
k-space at the grid frequencies.

The paper's data are in-vivo radial cardiac scans that are not available;
these phantoms stand in for them at the paper's shapes (matrix 192-384,
grid doubled, 8-12 coils, complex single precision; Sec. 3.2).

Every random draw comes from ``numpy.random.default_rng([cfg, frame, stream])``
with streams 0 = phantom, 1 = sampling pattern, 2 = noise, 3 = logits/probes.
All arrays handed out are float32 / complex64, C-contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN_ANGLE = math.pi * (math.sqrt(5.0) - 1.0) / 2.0   # 111.246 degrees, in radians

STREAM_PHANTOM, STREAM_MASK, STREAM_NOISE, STREAM_PROBE = 0, 1, 2, 3


def rng_for(cfg: int, frame: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([cfg, frame, stream])


# ---------------------------------------------------------------------------
# phantom and coils, both sampled on the image region Omega (n_om x n_om)
# ---------------------------------------------------------------------------

def fov_coords(n_om: int):
    """FOV coordinates x in [-1/2, 1/2) along both axes of Omega."""
    t = (np.arange(n_om, dtype=np.float64) - n_om // 2) / n_om
    return np.meshgrid(t, t, indexing="ij")


@dataclass
class EllipsePhantom:
    """Outer ellipse plus 9 seeded inner ellipses; later ellipses overwrite."""
    centres: np.ndarray          # [10, 2]
    axes: np.ndarray             # [10, 2] semi-axes
    angles: np.ndarray           # [10]
    values: np.ndarray           # [10] intensities in [0, 1]
    motion_dir: np.ndarray = field(default=None)     # [10, 2] unit vectors
    motion_phase: np.ndarray = field(default=None)   # [10]

    @staticmethod
    def draw(rng: np.random.Generator, n_inner: int = 9) -> "EllipsePhantom":
        centres = [np.zeros(2)]
        axes = [np.array([0.45, 0.35])]
        angles = [0.0]
        for _ in range(n_inner):
            r = 0.6 * math.sqrt(rng.uniform())
            phi = rng.uniform(0.0, 2.0 * math.pi)
            centres.append(np.array([0.45 * r * math.cos(phi), 0.35 * r * math.sin(phi)]))
            axes.append(rng.uniform(0.03, 0.15, size=2))
            angles.append(rng.uniform(0.0, math.pi))
        values = rng.uniform(0.0, 1.0, size=n_inner + 1)
        mdir = rng.uniform(0.0, 2.0 * math.pi, size=n_inner + 1)
        motion_dir = np.stack([np.cos(mdir), np.sin(mdir)], axis=1)
        motion_dir[0] = 0.0                                  # outer ellipse stays put
        motion_phase = rng.uniform(0.0, 2.0 * math.pi, size=n_inner + 1)
        return EllipsePhantom(np.array(centres), np.array(axes), np.array(angles),
                              values, motion_dir, motion_phase)

    def render(self, n_om: int, t: float | None = None, period: float = 40.0,
               amplitude: float = 0.05) -> np.ndarray:
        x0, x1 = fov_coords(n_om)
        img = np.zeros((n_om, n_om))
        for e in range(len(self.values)):
            c = self.centres[e].copy()
            if t is not None:
                c = c + amplitude * math.sin(2.0 * math.pi * t / period + self.motion_phase[e]) \
                    * self.motion_dir[e]
            ca, sa = math.cos(self.angles[e]), math.sin(self.angles[e])
            u = (x0 - c[0]) * ca + (x1 - c[1]) * sa
            v = -(x0 - c[0]) * sa + (x1 - c[1]) * ca
            inside = (u / self.axes[e, 0]) ** 2 + (v / self.axes[e, 1]) ** 2 <= 1.0
            img[inside] = self.values[e]
        return img


def coil_profiles(n_om: int, ncoils: int, sigma: float = 0.4, ring: float = 0.5) -> np.ndarray:
    """Gaussian-bump magnitudes centred on a ring, times a linear phase."""
    x0, x1 = fov_coords(n_om)
    out = np.empty((ncoils, n_om, n_om), dtype=np.complex128)
    for j in range(ncoils):
        th = 2.0 * math.pi * j / ncoils
        d0, d1 = math.cos(th), math.sin(th)
        mag = np.exp(-((x0 - ring * d0) ** 2 + (x1 - ring * d1) ** 2) / (2.0 * sigma ** 2))
        out[j] = mag * np.exp(1j * (th + math.pi * (x0 * d0 + x1 * d1)))
    return out


# ---------------------------------------------------------------------------
# sampling patterns on the n x n grid (DC at index n/2)
# ---------------------------------------------------------------------------

def cartesian_mask(n: int, rng: np.random.Generator, centre: int = 16, frac_outer: float = 0.25):
    """Rows along axis 0; `centre` central rows plus a seeded share of the rest."""
    P = np.zeros((n, n), dtype=np.float32)
    lo = n // 2 - centre // 2
    rows_c = np.arange(lo, lo + centre)
    outer = np.setdiff1d(np.arange(n), rows_c)
    pick = rng.choice(outer, size=int(round(frac_outer * len(outer))), replace=False)
    P[rows_c, :] = 1.0
    P[np.sort(pick), :] = 1.0
    return P


def radial_mask(n: int, spokes: int, frame: int = 1):
    """Rasterised radial spokes: uniform angles within a frame, rotated by the
    golden angle per frame; n samples per spoke at radii -n/2..n/2-1; each
    sample rounds to the nearest grid point, off-grid samples are dropped."""
    P = np.zeros((n, n), dtype=np.float32)
    r = np.arange(-(n // 2), n - n // 2, dtype=np.float64)
    off = frame * GOLDEN_ANGLE
    for s in range(spokes):
        th = s * math.pi / spokes + off
        k0 = np.floor(n / 2 + r * math.cos(th) + 0.5).astype(np.int64)
        k1 = np.floor(n / 2 + r * math.sin(th) + 0.5).astype(np.int64)
        ok = (k0 >= 0) & (k0 < n) & (k1 >= 0) & (k1 < n)
        P[k0[ok], k1[ok]] = 1.0
    return P


# ---------------------------------------------------------------------------
# acquisition: grid samples of the signal equation plus complex noise
# ---------------------------------------------------------------------------

def acquire(coil_images: np.ndarray, n: int, P: np.ndarray, sigma: float,
            rng: np.random.Generator) -> np.ndarray:
    """k-space data of each coil image (given on the centred n_om x n_om region),
    at grid frequencies k = (kappa - n/2)/n with the orthonormal scaling,
    multiplied by P; complex Gaussian noise of std `sigma` where P > 0."""
    J, n_om, _ = coil_images.shape
    lo = n // 2 - n_om // 2
    full = np.zeros((J, n, n), dtype=np.complex128)
    full[:, lo:lo + n_om, lo:lo + n_om] = coil_images
    ksp = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(full, axes=(-2, -1)), norm="ortho"),
                          axes=(-2, -1))
    noise = (sigma / math.sqrt(2.0)) * (rng.standard_normal((J, n, n))
                                        + 1j * rng.standard_normal((J, n, n)))
    P64 = P.astype(np.float64)
    return (P64 * (ksp + np.where(P64 > 0, noise, 0.0))).astype(np.complex64)


def random_complex(shape, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    return (scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
            / math.sqrt(2.0)).astype(np.complex64)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

@dataclass
class Frame:
    n: int
    n_om: int
    ncoils: int
    P: np.ndarray              # float32 [n][n]
    y: np.ndarray              # complex64 [J][n][n]
    rho_true: np.ndarray       # complex64 [n_om][n_om]
    coils_true: np.ndarray     # complex64 [J][n_om][n_om]
    newton: int = 7
    cg: int = 10
    alpha0: float = 1.0
    alpha_q: float = 0.5
    spokes: int = 0


def make_frame(cfg: int, frame: int, n: int, n_om: int, ncoils: int, mask: str,
               spokes: int = 0, sigma: float = 1e-3, newton: int = 7, cg: int = 10,
               phantom: EllipsePhantom | None = None, t: float | None = None,
               mask_frame: int | None = None) -> Frame:
    if phantom is None:
        phantom = EllipsePhantom.draw(rng_for(cfg, frame, STREAM_PHANTOM))
    rho = phantom.render(n_om, t=t)
    coils = coil_profiles(n_om, ncoils)
    if mask == "cartesian":
        P = cartesian_mask(n, rng_for(cfg, frame, STREAM_MASK))
    elif mask == "radial":
        P = radial_mask(n, spokes, frame=1 if mask_frame is None else mask_frame)
    elif mask == "full":
        P = np.ones((n, n), dtype=np.float32)
    else:
        raise ValueError(mask)
    y = acquire(rho[None] * coils, n, P, sigma, rng_for(cfg, frame, STREAM_NOISE))
    return Frame(n=n, n_om=n_om, ncoils=ncoils, P=P, y=y,
                 rho_true=rho.astype(np.complex64), coils_true=coils.astype(np.complex64),
                 newton=newton, cg=cg, spokes=spokes)


def single_frame_64(sigma: float = 1e-3, mask: str = "cartesian") -> Frame:
    """64x64 grid, Omega = grid, 8 coils, Cartesian 16 central + 25% outer rows,
    6 Newton steps x 10 CG iterations."""
    return make_frame(1, 0, 64, 64, 8, mask, sigma=sigma, newton=6, cg=10)


def realtime_384(sigma: float = 1e-3) -> Frame:
    """384x384 grid (2x oversampled 192x192 FOV), 12 coils, 15 radial spokes
    with a golden-angle offset, 7 Newton steps x 10 CG iterations."""
    return make_frame(2, 0, 384, 192, 12, "radial", spokes=15, sigma=sigma, newton=7, cg=10)


def soft_mask_frame(n: int, ncoils: int, sigma: float = 1e-3):
    """Differentiation workload: Omega = grid, P = sigmoid(logits),
    logits ~ N(0, 1) from the probe stream. Returns (frame, logits)."""
    logits = rng_for(3, n, STREAM_PROBE).standard_normal((n, n)).astype(np.float32)
    P = (1.0 / (1.0 + np.exp(-logits.astype(np.float64)))).astype(np.float32)
    ph = EllipsePhantom.draw(rng_for(3, n, STREAM_PHANTOM))
    rho = ph.render(n)
    coils = coil_profiles(n, ncoils)
    y = acquire(rho[None] * coils, n, P, sigma, rng_for(3, n, STREAM_NOISE))
    fr = Frame(n=n, n_om=n, ncoils=ncoils, P=P, y=y, rho_true=rho.astype(np.complex64),
               coils_true=coils.astype(np.complex64), newton=0, cg=0)
    return fr, logits


BATCH_SIZES = (128, 192, 256, 384)
BATCH_COILS = (8, 12, 16, 32)
BATCH_SPOKES = (11, 15, 21)


def ragged_batch_shapes(nframes: int = 64):
    """(n, J, spokes) per frame for the uneven batch, from rng([4, 999])."""
    rng = np.random.default_rng([4, 999])
    ns = rng.choice(BATCH_SIZES, size=nframes)
    js = rng.choice(BATCH_COILS, size=nframes)
    ss = rng.choice(BATCH_SPOKES, size=nframes)
    return [(int(a), int(b), int(c)) for a, b, c in zip(ns, js, ss)]


def ragged_batch(nframes: int = 64, sigma: float = 1e-3):
    """Independent frames of uneven grid size (Omega = half grid), coils and spokes."""
    out = []
    for f, (n, J, S) in enumerate(ragged_batch_shapes(nframes)):
        out.append(make_frame(4, f, n, n // 2, J, "radial", spokes=S, sigma=sigma,
                              newton=7, cg=10, mask_frame=f))
    return out


def temporal_phantom() -> EllipsePhantom:
    return EllipsePhantom.draw(rng_for(5, 0, STREAM_PHANTOM))


def temporal_frame(t: int, phantom: EllipsePhantom | None = None, n: int = 512,
                   ncoils: int = 32, spokes: int = 13, sigma: float = 1e-3) -> Frame:
    """Frame t of a moving phantom (inner ellipses oscillate with period 40
    frames); the spokes rotate by the golden angle from frame to frame."""
    ph = temporal_phantom() if phantom is None else phantom
    return make_frame(5, t, n, n // 2, ncoils, "radial", spokes=spokes, sigma=sigma,
                      newton=7, cg=10, phantom=ph, t=float(t), mask_frame=t)


def temporal_series(nframes: int = 100, **kw):
    """Frames 0..nframes-1 of the temporal series, generated lazily."""
    ph = temporal_phantom()
    for t in range(nframes):
        yield temporal_frame(t, ph, **kw)

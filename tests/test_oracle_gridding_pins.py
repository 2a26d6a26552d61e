"""Pins of the gridding oracle (oracle/gridding.py) against what the
mathematics fixes: the Kaiser-Bessel window from the power series of I0,
the adjoint identity of gridding and degridding, and the direct non-uniform
Fourier sum that gridding approximates (to the window's aliasing error,
which must fall as the window widens)."""
import math

import numpy as np
import pytest

from oracle import gridding as GR

RNG = np.random.default_rng([99, 11, 3])


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def i0_series(x):
    """I0(x) = sum_k (x^2/4)^k / (k!)^2, summed until the terms vanish."""
    s, term, k = 1.0, 1.0, 0
    while term > 1e-18 * s:
        k += 1
        term *= (x * x / 4.0) / (k * k)
        s += term
    return s


@pytest.mark.parametrize("W", [3.0, 4.0, 6.0])
def test_window_from_the_bessel_series(W):
    beta = GR.default_beta(W)
    u = np.linspace(-W / 2 - 0.5, W / 2 + 0.5, 41)
    got = GR.kb(u, W, beta)
    for ui, g in zip(u, got):
        t = 1.0 - (2.0 * ui / W) ** 2
        ref = i0_series(beta * math.sqrt(t)) / i0_series(beta) if t >= 0 else 0.0
        assert abs(g - ref) < 1e-13
    assert GR.kb(np.array([0.0]), W, beta)[0] == 1.0


def test_beatty_shape_for_two_times_oversampling():
    # beta = pi sqrt((W/a)^2 (a - 1/2)^2 - 0.8): W = 4, a = 2 gives pi sqrt(8.2)
    assert math.isclose(GR.default_beta(4.0, 2.0), math.pi * math.sqrt(8.2), rel_tol=1e-15)


@pytest.mark.parametrize("n,S,R", [(16, 3, 16), (24, 5, 20), (32, 4, 33)])
def test_gridding_adjoint_identity(n, S, R):
    angles = RNG.uniform(0, math.pi, S)
    W = 4.0
    beta = GR.default_beta(W)
    dcf = np.abs(np.arange(R) - R // 2) + 0.5
    d = crand(2, S, R)
    g = crand(2, n, n)
    lhs = np.vdot(GR.grid(d, angles, n, W, beta, dcf), g)
    rhs = np.vdot(d, GR.degrid(g, angles, R, W, beta, dcf))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_ones_grid_to_the_sampling_density():
    angles = np.array([0.3, 1.4, 2.2])
    n, R, W = 20, 20, 4.0
    beta = GR.default_beta(W)
    P = GR.grid_ones(angles, R, n, W, beta)
    d = np.ones((1, 3, R))
    assert relerr(P, GR.grid(d, angles, n, W, beta)[0].real) < 1e-15
    assert np.all(P >= 0)


def _nudft_vs_gridding(n, S, W):
    """Image of gridded samples (centred IDFT, divided by the image of one
    unit sample at k = 0, i.e. the window's transform) against the direct sum
    f[r] = sum_s d_s exp(+2 pi i (k_s - n/2).(r - n/2) / n) on the central n/2 x n/2."""
    R = n
    angles = np.arange(S) * math.pi / S + 0.37
    beta = GR.default_beta(W)
    d = crand(1, S, R)
    g = GR.grid(d, angles, n, W, beta)[0]

    def idft2c(X):
        return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(X), norm="ortho"))

    x = idft2c(g)
    x0 = idft2c(_unit_at_centre(n, W, beta))    # placed by hand: a position offset in grid() shows
    est = x / x0
    pos = GR.radial_positions(n, angles, R).reshape(-1, 2) - n / 2
    lo, m = n // 4, n // 2
    r = np.arange(lo, lo + m) - n / 2
    ph = np.exp(2j * math.pi * (pos[:, 0][:, None, None] * r[None, :, None]
                                + pos[:, 1][:, None, None] * r[None, None, :]) / n)
    f = np.tensordot(d.reshape(-1), ph, axes=1)
    return relerr(est[lo:lo + m, lo:lo + m], f)


def _unit_at_centre(n, W, beta):
    """The grid of one unit sample at k = (n/2, n/2)."""
    g = np.zeros((n, n))
    h = int(W // 2)
    a = GR.kb(np.arange(-h, h + 1), W, beta)
    g[n // 2 - h:n // 2 + h + 1, n // 2 - h:n // 2 + h + 1] = np.outer(a, a)
    return g


def test_gridding_approximates_the_direct_fourier_sum():
    """Kaiser-Bessel aliasing falls about tenfold per added cell of width at 2x
    oversampling (measured: W = 4 -> 8e-4, W = 6 -> 8e-6); a wrong sign,
    scale or position in the gridding gives an error of order one."""
    e4 = _nudft_vs_gridding(32, 6, 4.0)
    e6 = _nudft_vs_gridding(32, 6, 6.0)
    assert e4 < 2e-3
    assert e6 < 2e-5
    assert e6 < e4 / 50


@pytest.mark.parametrize("n,S,frame", [(32, 5, 1), (48, 7, 3), (64, 13, 0)])
def test_sample_positions_round_to_the_rasterised_spokes(n, S, frame):
    """A window of width 1 weights only the nearest grid point of each sample,
    so the gridded density's support is exactly the rasterised radial mask of
    the same spokes (nearest-point rounding of the same radii and angles),
    an independent statement of the sampling geometry."""
    from paper_1301_1215_amd import synth
    angles = np.arange(S) * math.pi / S + frame * synth.GOLDEN_ANGLE
    P1 = GR.grid_ones(angles, n, n, 1.0, 0.0)
    mask = synth.radial_mask(n, S, frame=frame)
    assert np.array_equal(P1[1:, 1:] > 0, mask[1:, 1:] > 0)


def test_axis_spokes_land_on_grid_lines():
    """theta = 0 puts sample i at (n/2 + i - R/2, n/2), theta = pi/2 at
    (n/2, n/2 + i - R/2): a unit sample there grids to a window centred on
    that grid point."""
    n, R, W = 16, 16, 4.0
    beta = GR.default_beta(W)
    for th, axis in ((0.0, 0), (math.pi / 2, 1)):
        d = np.zeros((1, 1, R), np.complex128)
        d[0, 0, 11] = 1.0
        g = np.abs(GR.grid(d, np.array([th]), n, W, beta)[0])
        peak = np.unravel_index(np.argmax(g), g.shape)
        expect = [n // 2, n // 2]
        expect[axis] = n // 2 + 11 - R // 2
        assert tuple(peak) == tuple(expect) and abs(g[peak] - 1.0) < 1e-12

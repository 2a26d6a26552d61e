"""Seeded generator: determinism, shapes and the sampling fractions of the workloads."""
import numpy as np
import pytest

from paper_1301_1215_amd import synth


def test_deterministic():
    a, b = synth.single_frame_64(), synth.single_frame_64()
    assert np.array_equal(a.y, b.y) and np.array_equal(a.P, b.P)
    assert a.y.dtype == np.complex64 and a.P.dtype == np.float32


def test_cartesian_rows():
    fr = synth.single_frame_64()
    rows = fr.P[:, 0]
    assert rows.sum() == 28 and np.all(fr.P == rows[:, None])
    assert np.all(rows[24:40] == 1)


@pytest.mark.parametrize("n,S,frac", [(384, 15, 0.037), (512, 13, 0.024), (128, 11, 0.079), (256, 21, 0.076)])
def test_radial_fractions(n, S, frac):
    assert abs(synth.radial_mask(n, S).mean() - frac) < 0.0015


def test_noise_only_where_sampled():
    fr = synth.make_frame(2, 0, 64, 32, 4, "radial", spokes=7)
    assert np.all(fr.y[:, fr.P == 0] == 0)


def test_phantom_range_and_coils():
    ph = synth.EllipsePhantom.draw(synth.rng_for(1, 0, 0))
    img = ph.render(64)
    assert img.min() >= 0 and img.max() <= 1 and (img > 0).mean() > 0.3
    c = synth.coil_profiles(32, 8)
    assert c.shape == (8, 32, 32) and np.abs(c).max() <= 1.0


def test_ragged_batch_shapes():
    sh = synth.ragged_batch_shapes(64)
    assert len(sh) == 64
    assert {s[0] for s in sh} <= set(synth.BATCH_SIZES)
    assert {s[1] for s in sh} <= set(synth.BATCH_COILS)
    assert {s[2] for s in sh} <= set(synth.BATCH_SPOKES)


def test_temporal_motion():
    ph = synth.temporal_phantom()
    assert not np.array_equal(ph.render(64, t=0.0), ph.render(64, t=10.0))
    assert np.abs(ph.render(64, t=0.0) - ph.render(64, t=40.0)).mean() < 1e-3

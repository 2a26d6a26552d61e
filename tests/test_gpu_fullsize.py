"""Parity at the workloads' full sizes, in the launch configurations the
benchmark uses: sampled frames against the FP64 oracle (image NRMSE <= 1e-3)."""
import os

import numpy as np
import pytest

from oracle import nlinv_oracle as O
from paper_1301_1215_amd import Plan, synth
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu

NRMSE = 1e-3


def _workers():
    O.set_workers(min(16, os.cpu_count() or 1))


def _oracle(fr, newton=7, cg=10):
    _workers()
    return O.irgnm(fr.y, fr.P, O.Dims(fr.n, fr.n_om, fr.ncoils), O.IRGNMParams(newton, cg))


@pytest.mark.timeout(600)
def test_batched_realtime_384_as_benchmarked():
    """4 frames of 384x384, 12 coils, 15 spokes in one batched, graph-replayed
    solve (the benchmark's step); frames 0 and 3 against the oracle."""
    frames = [synth.make_frame(2, t, 384, 192, 12, "radial", spokes=15, mask_frame=t + 1) for t in range(4)]
    with Plan(frames=[(384, 192, 12)] * 4) as pl:
        pl.autotune()
        outs = pl.solve_batch([(dev(f.y), dev(f.P)) for f in frames], Plan.params(7, 10, use_graph=True))
        imgs = [host(o["image"]) for o in outs]
    for t in (0, 3):
        assert rel(imgs[t], _oracle(frames[t]).image) < NRMSE


@pytest.mark.timeout(900)
def test_ragged_batch_64_frames_sampled():
    """All 64 uneven frames in one batched, graph-replayed solve; sampled
    frames (the smallest grid, a 32-coil frame, a 384 grid and a 192 grid, the
    radix-3 size whose passes split 12 x 16) against the oracle, every frame
    finite and converging."""
    frames = synth.ragged_batch(64)
    with Plan(frames=[(f.n, f.n_om, f.ncoils) for f in frames]) as pl:
        pl.autotune()
        outs = pl.solve_batch([(dev(f.y), dev(f.P)) for f in frames], Plan.params(7, 10, use_graph=True))
        res = [{k: host(v) for k, v in o.items() if k in ("image", "stats")} for o in outs]
    for r in res:
        st = r["stats"]
        assert np.isfinite(r["image"]).all() and int(st[1]) == 0
        assert st[2 + 6] < st[2]        # residual falls over the Newton steps
    picks = {min(range(64), key=lambda i: frames[i].n),
             next(i for i in range(64) if frames[i].ncoils == 32),
             next(i for i in range(64) if frames[i].n == 384),
             next(i for i in range(64) if frames[i].n == 192)}
    for i in sorted(picks):
        assert rel(res[i]["image"], _oracle(frames[i]).image) < NRMSE, i


SERIES_FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "series_512_oracle.npz")


@pytest.mark.timeout(300)
def test_temporal_series_512_first_frames():
    """512x512, 32 coils, 13 golden-angle spokes: frames 0..7 of the series
    (the benchmark's step), each warm-started from the previous, against the
    oracle's series, so that FP32 drift along the chain of references is
    measured frame by frame.  The oracle's series takes minutes on the host,
    so its images (every second pixel of Omega) come from a file written by
    tests/golden/make_series_512.py, which calls only the oracle; the inputs
    are checked to be the ones that file was made from."""
    from tests.golden.make_series_512 import input_digest
    ref = np.load(SERIES_FIXTURE, allow_pickle=False)
    st = int(ref["stride"])
    F = ref["image_sampled"].shape[0]
    ph = synth.temporal_phantom()
    frames = [synth.temporal_frame(t, ph) for t in range(F)]
    for t, f in enumerate(frames):
        assert input_digest(f.y, f.P) == str(ref["input_sha256"][t]), \
            f"frame {t}: inputs differ from the fixture's; rerun tests/golden/make_series_512.py"
    prm = Plan.params(int(ref["newton"]), int(ref["cg"]), use_graph=True)
    with Plan(512, 256, 32) as pl:
        outs = pl.solve_series([(dev(f.y), dev(f.P)) for f in frames], prm)
        imgs = [host(o["image"]) for o in outs]
        stats = [host(o["stats"]) for o in outs]
    errs = [rel(img[::st, ::st], r) for img, r in zip(imgs, ref["image_sampled"])]
    print("series_512 image NRMSE per frame:", " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) < NRMSE, errs
    # the residual norms per Newton step follow the oracle's along the chain
    for t in range(F):
        r0 = stats[t][2:2 + int(ref["newton"])]
        np.testing.assert_allclose(r0, ref["r0_norms"][t], rtol=1e-3)

"""GPU PCA channel compression (Sec. 3.2) against the FP64 oracle
(oracle/coil_compression.py): eigenvalues, the kept subspace's projector
(unique when lambda_K > lambda_K+1), the compressed data element-wise (same
phase convention), data that span K channels reproduced exactly, odd and
trivial channel counts, the series workload's 32 coils compressed to 12, and
bitwise determinism."""
import numpy as np
import pytest

from oracle import coil_compression as CC
from paper_1301_1215_amd import _native as N
from paper_1301_1215_amd import synth
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def _rand(J, shape, seed):
    rng = np.random.default_rng([53, J, seed])
    return (rng.standard_normal((J,) + shape) + 1j * rng.standard_normal((J,) + shape)).astype(np.complex64)


def _check(y, K, tol_y=1e-5):
    got, lam, V = (host(t) for t in N.nlinv_coil_compress(dev(y), K))
    yk, VK, w = CC.compress(y, K)
    assert rel(lam, w) <= 1e-10
    assert rel(CC.projector(V), CC.projector(VK)) <= 1e-5
    assert rel(got, yk) <= tol_y
    return got, lam, V


@pytest.mark.parametrize("J,K,shape", [(8, 3, (64, 64)), (5, 2, (40, 40)), (12, 8, (33, 31)), (16, 16, (32, 32))])
def test_compression_matches_the_oracle(J, K, shape):
    _check(_rand(J, shape, 0), K)


def test_one_channel():
    y = _rand(1, (16, 16), 1)
    got, lam, V = _check(y, 1)
    assert np.allclose(V, 1.0) and rel(got, y) <= 1e-6


def test_rank_k_data_are_kept_exactly():
    rng = np.random.default_rng([54, 1])
    J, K = 10, 3
    s = rng.standard_normal((K, 48, 48)) + 1j * rng.standard_normal((K, 48, 48))
    M = rng.standard_normal((J, K)) + 1j * rng.standard_normal((J, K))
    y = np.tensordot(M, s, axes=1).astype(np.complex64)
    got, lam, V = (host(t) for t in N.nlinv_coil_compress(dev(y), K))
    assert rel(np.tensordot(V, got, axes=1), y) <= 1e-5
    assert np.all(np.abs(lam[K:]) <= 1e-6 * lam[0])


def test_series_coils_32_to_12_and_determinism():
    import torch
    fr = synth.temporal_frame(0, synth.temporal_phantom())
    got, lam, V = _check(fr.y, 12)
    a = N.nlinv_coil_compress(dev(fr.y), 12)[0]
    b = N.nlinv_coil_compress(dev(fr.y), 12)[0]
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # the kept channels hold the bulk of the energy
    assert lam[:12].sum() / lam.sum() > 0.99

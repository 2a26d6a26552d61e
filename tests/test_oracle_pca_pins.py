"""Pins of the PCA channel-compression oracle (oracle/coil_compression.py)
against what linear algebra fixes: data that span K channels survive a
compression to K channels exactly, the 2 x 2 eigenproblem's closed form,
the trace and energy identities, orthonormality, and equivariance under a
unitary mixing of the channels."""
import math

import numpy as np
import pytest

from oracle import coil_compression as CC

RNG = np.random.default_rng([99, 7, 3])


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


@pytest.mark.parametrize("J,K", [(8, 3), (32, 12), (12, 8)])
def test_rank_k_data_survive_compression_exactly(J, K):
    """y_j = sum_{k<K} M[j,k] s_k: the data span K channels, so the K kept
    virtual channels reproduce them, V_K y' = y, and the other eigenvalues vanish."""
    s = crand(K, 16, 16)
    M = crand(J, K)
    y = np.tensordot(M, s, axes=1)
    yk, VK, w = CC.compress(y, K)
    assert relerr(np.tensordot(VK, yk, axes=1), y) < 1e-12
    assert np.all(np.abs(w[K:]) < 1e-10 * w[0])
    assert np.all(w[:K] > 1e-6 * w[0])


def test_two_channel_closed_form():
    """A = [[a, c], [conj c, b]]: lambda = (a+b)/2 +- sqrt(((a-b)/2)^2 + |c|^2)."""
    y = crand(2, 40)
    a = float(np.sum(np.abs(y[0]) ** 2))
    b = float(np.sum(np.abs(y[1]) ** 2))
    c = complex(np.sum(y[0] * np.conj(y[1])))
    A = CC.channel_covariance(y)
    assert abs(A[0, 1] - c) < 1e-12 * abs(c) and abs(A[0, 0] - a) < 1e-12 * a
    w, V = CC.pca_basis(A)
    r = math.sqrt(((a - b) / 2) ** 2 + abs(c) ** 2)
    assert math.isclose(w[0], (a + b) / 2 + r, rel_tol=1e-12)
    assert math.isclose(w[1], (a + b) / 2 - r, rel_tol=1e-12, abs_tol=1e-12 * w[0])
    # eigenvector of the larger eigenvalue: (c, lambda - a) up to scale and phase
    v = np.array([c, w[0] - a])
    v /= np.linalg.norm(v)
    assert abs(abs(np.vdot(v, V[:, 0])) - 1.0) < 1e-12


def test_eigenpairs_orthonormal_descending_and_trace():
    y = crand(10, 24, 24)
    A = CC.channel_covariance(y)
    w, V = CC.pca_basis(A)
    assert np.all(np.diff(w) <= 0)
    assert relerr(V.conj().T @ V, np.eye(10)) < 1e-13
    assert relerr(A @ V, V * w[None, :]) < 1e-13
    assert math.isclose(float(np.sum(w)), float(np.sum(np.abs(y) ** 2)), rel_tol=1e-12)
    for k in range(10):   # the phase convention: largest entry real and positive
        i = int(np.argmax(np.abs(V[:, k])))
        assert V[i, k].real > 0 and abs(V[i, k].imag) < 1e-15


@pytest.mark.parametrize("K", [1, 4, 9])
def test_kept_energy_is_the_sum_of_the_kept_eigenvalues(K):
    y = crand(9, 20, 20)
    yk, VK, w = CC.compress(y, K)
    assert math.isclose(float(np.sum(np.abs(yk) ** 2)), float(np.sum(w[:K])), rel_tol=1e-12)


def test_unitary_mixing_rotates_the_projector():
    """Compressing U y (U unitary on the channels) keeps the eigenvalues and
    gives the projector U P U^H."""
    J, K = 8, 3
    y = crand(J, 12, 12)
    U, _ = np.linalg.qr(crand(J, J))
    _, VK, w = CC.compress(y, K)
    _, VK2, w2 = CC.compress(np.tensordot(U, y, axes=1), K)
    assert relerr(w2, w) < 1e-12
    assert relerr(CC.projector(VK2), U @ CC.projector(VK) @ U.conj().T) < 1e-11


def test_unsampled_points_add_nothing():
    """Zeros (points where P = 0) change neither the covariance nor the basis."""
    y = crand(6, 30)
    pad = np.concatenate([y, np.zeros((6, 50))], axis=1)
    assert relerr(CC.channel_covariance(pad), CC.channel_covariance(y)) < 1e-15

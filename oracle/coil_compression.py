"""FP64 CPU oracle of the PCA channel compression (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product path never does.  It shares no
code with the HIP library.

What it computes (Schaetz & Uecker, Sec. 3.2: before reconstruction the 32
receive channels are compressed to 8-12 by a principal component analysis,
after Huang et al. 2007):
  * the channel covariance A = Y Y^H of the J channels, Y = the J x M matrix
    of every channel's samples (all grid points of y; unsampled points hold
    zeros and add nothing),
  * its eigen-decomposition A = V diag(lambda) V^H with the eigenvalues in
    descending order,
  * the compressed data y'_k = sum_j conj(V[j, k]) y_j for the first K
    eigenvectors (the K virtual channels that keep the most energy).

Readings where the paper is silent (also listed in the design notes):
  * the covariance is taken over all grid samples of the data handed to the
    reconstruction (no separate calibration region);
  * each eigenvector is fixed up to its unit phase by making its
    largest-magnitude entry real and positive (the first such entry on a
    tie).  The reconstruction does not depend on this choice: the Newton
    iteration is equivariant under a unitary mixing of the channels, so the
    combined image is the same.
"""
from __future__ import annotations

import numpy as np


def channel_covariance(y) -> np.ndarray:
    """A[i, k] = sum over samples of y_i conj(y_k)   (J x J, Hermitian)."""
    y = np.asarray(y, np.complex128)
    Y = y.reshape(y.shape[0], -1)
    return Y @ Y.conj().T


def pca_basis(A):
    """Eigenvalues (descending) and eigenvectors (columns) of the Hermitian A,
    each eigenvector's largest-magnitude entry made real and positive."""
    w, V = np.linalg.eigh(np.asarray(A, np.complex128))
    order = np.argsort(-w, kind="stable")
    w, V = w[order], V[:, order].copy()
    for k in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, k])))
        V[:, k] *= np.conj(V[i, k]) / abs(V[i, k])
    return w, V


def compress(y, K: int):
    """(y' [K, ...], V_K [J, K], eigenvalues [J]) with y'_k = sum_j conj(V[j,k]) y_j."""
    y = np.asarray(y, np.complex128)
    w, V = pca_basis(channel_covariance(y))
    VK = V[:, :K]
    yk = np.tensordot(VK.conj().T, y, axes=1)
    return yk, VK, w


def projector(VK) -> np.ndarray:
    """V_K V_K^H: the orthogonal projector onto the kept channel subspace, which
    is unique (independent of the eigenvectors' phases) when lambda_K > lambda_{K+1}."""
    VK = np.asarray(VK, np.complex128)
    return VK @ VK.conj().T

"""Coil compression, FP64 (test infrastructure; oracle only).

Methods, Coil compression: a compression matrix built as in Huang et al.
(software channel compression by principal components) is applied to the coil
data and to the coil sensitivity maps; the least dominant virtual coils are
dropped.

Reading used here: the coil covariance is C = sum over k-space samples of
y y^H (y = the slice's acquired samples of all coils; zero-filled entries add
nothing).  By Parseval this equals the covariance of the zero-filled coil
images.  Its eigenvectors, ordered by descending eigenvalue, form U; the
virtual coils are y_v = U[:, :nv]^H y and S_v = U[:, :nv]^H S (per sample /
per pixel).  Eigenvectors are defined up to a unit phase each: everything
compared with another implementation must be invariant to it (the projector
U U^H, the system operator and its spectrum built from S_v).
"""
from __future__ import annotations

import numpy as np


def covariance(kspace: np.ndarray) -> np.ndarray:
    """C[i, j] = sum_k y_i(k) conj(y_j(k)) over all samples."""
    Y = kspace.reshape(kspace.shape[0], -1)
    return Y @ Y.conj().T


def compression_matrix(kspace: np.ndarray):
    """Eigenvalues (descending) and eigenvectors (columns) of the covariance."""
    w, U = np.linalg.eigh(covariance(kspace))
    order = np.argsort(w)[::-1]
    return w[order], U[:, order]


def compress(kspace: np.ndarray, sens: np.ndarray, nvirt: int):
    """(virtual k-space [nv][m][n], virtual maps [nv][m][n], eigenvalues, U)."""
    w, U = compression_matrix(kspace)
    Uv = U[:, :nvirt]
    mix = lambda a: np.tensordot(Uv.conj().T, a, axes=(1, 0))
    return mix(kspace), mix(sens), w, U

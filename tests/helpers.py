"""Small shared test utilities: dense matrices built straight from the
definitions (used to pin the oracle) and instance helpers."""
from __future__ import annotations

import numpy as np


def dense_dft(m: int) -> np.ndarray:
    """Unitary DFT matrix from its definition F[u, i] = exp(-2 pi i u i / m) / sqrt(m)."""
    u = np.arange(m)[:, None]
    i = np.arange(m)[None, :]
    return np.exp(-2j * np.pi * u * i / m) / np.sqrt(m)


def dense_dft2(m: int, n: int) -> np.ndarray:
    """2D DFT acting on row-major vec(x) (n contiguous): kron(F_m, F_n)."""
    return np.kron(dense_dft(m), dense_dft(n))


def dense_Dx(m: int, n: int) -> np.ndarray:
    """D_x from the finite-difference scheme: x[i,j] - x[i-1,j], periodic."""
    N = m * n
    D = np.zeros((N, N))
    for i in range(m):
        for j in range(n):
            D[i * n + j, i * n + j] += 1.0
            D[i * n + j, ((i - 1) % m) * n + j] -= 1.0
    return D


def dense_Dy(m: int, n: int) -> np.ndarray:
    N = m * n
    D = np.zeros((N, N))
    for i in range(m):
        for j in range(n):
            D[i * n + j, i * n + j] += 1.0
            D[i * n + j, i * n + (j - 1) % n] -= 1.0
    return D


def dense_of(op, m: int, n: int, dtype=np.complex128) -> np.ndarray:
    """Matrix of a linear map on m x n images, column by column."""
    N = m * n
    M = np.zeros((N, N), dtype)
    for c in range(N):
        e = np.zeros(N, dtype)
        e[c] = 1.0
        M[:, c] = op(e.reshape(m, n)).ravel()
    return M


def rand_complex(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def smooth_sens(rng, nc, m, n, normalise=True, asym=True):
    """Random smooth complex maps with asymmetric phase ramps (not
    centro-symmetric), optionally normalised to sum |S|^2 = 1."""
    Y, X = np.meshgrid(np.linspace(-1, 1, m), np.linspace(-1, 1, n), indexing="ij")
    S = np.empty((nc, m, n), np.complex128)
    for c in range(nc):
        cy, cx = rng.uniform(-1.2, 1.2, 2)
        w = rng.uniform(0.4, 0.9)
        ph = rng.uniform(0, 2 * np.pi) + (rng.uniform(-2, 2) * Y + rng.uniform(-2, 2) * X if asym else 0)
        S[c] = np.exp(-((Y - cy) ** 2 + (X - cx) ** 2) / (2 * w * w)) * np.exp(1j * ph)
    if normalise:
        S /= np.sqrt(np.sum(np.abs(S) ** 2, axis=0))[None]
    return S


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))

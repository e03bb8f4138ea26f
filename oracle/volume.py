"""3D extension of the system operator and the circulant preconditioner, FP64
(test infrastructure; oracle only).

The paper's Discussion names the 3D case as the natural extension: with a 3D
unitary DFT F, a 3D sampling mask R and periodic differences along all three
axes,
    A = mu sum_c S_c^H F^H R F S_c + lam (D_z^H D_z + D_y^H D_y + D_x^H D_x) + gam I
is again approximated by F^H diag(k) F with the same construction as Eqs. K,
Kdiag, d and diagonalelements, one dimension up:
    k = mu k_c + lam k_d + gam,
    k_c(j) = (1/N^2) sum_l r(l) P(l - j),  P = sum_c |DFT(s_c)|^2,
    k_d(w, u, v) = 6 - 2 cos(2 pi w / p) - 2 cos(2 pi u / m) - 2 cos(2 pi v / n).
Volumes are [p][m][n] (axis 0 = z).  Regularisers beyond W^H W = I (3D
wavelets, 3D shrinks) are not part of this extension.
"""
from __future__ import annotations

import numpy as np


def fft3u(x):
    return np.fft.fftn(x, axes=(-3, -2, -1), norm="ortho")


def ifft3u(x):
    return np.fft.ifftn(x, axes=(-3, -2, -1), norm="ortho")


def laplacian3(v):
    """(D_z^H D_z + D_y^H D_y + D_x^H D_x) v with periodic backward differences."""
    out = 6.0 * v
    for ax in range(3):
        out = out - np.roll(v, 1, axis=ax) - np.roll(v, -1, axis=ax)
    return out


def apply_A3(v, S, r3, mu, lam, gam):
    data = np.sum(np.conj(S) * ifft3u(r3[None] * fft3u(S * v[None])), axis=0)
    return mu * data + lam * laplacian3(v) + gam * v


def k_coil3(S, r3):
    """k_c(j) = (1/N^2) sum_l r(l) P(l - j), through the DFT (cross-correlation)."""
    N = r3.size
    P = np.sum(np.abs(np.fft.fftn(S, axes=(-3, -2, -1))) ** 2, axis=0)
    corr = np.fft.ifftn(np.fft.fftn(r3) * np.conj(np.fft.fftn(P))).real
    return corr / N**2


def k_laplacian3(p, m, n):
    w = np.arange(p)[:, None, None]
    u = np.arange(m)[None, :, None]
    v = np.arange(n)[None, None, :]
    return (6.0 - 2.0 * np.cos(2 * np.pi * w / p) - 2.0 * np.cos(2 * np.pi * u / m)
            - 2.0 * np.cos(2 * np.pi * v / n))


def circulant_k3(S, r3, mu, lam, gam):
    p, m, n = r3.shape
    return mu * k_coil3(S, r3) + lam * k_laplacian3(p, m, n) + gam


def apply_minv3(r, k):
    return ifft3u(fft3u(r) / k)


def brute_force_k3(S, r3, mu, lam, gam):
    """k_j = f_j^H A f_j over the 3D Fourier modes f_j = F^H e_j (tiny sizes)."""
    p, m, n = r3.shape
    k = np.empty((p, m, n))
    for idx in np.ndindex(p, m, n):
        e = np.zeros((p, m, n), complex)
        e[idx] = 1.0
        f = ifft3u(e)
        k[idx] = np.vdot(f, apply_A3(f, S, r3, mu, lam, gam)).real
    return k

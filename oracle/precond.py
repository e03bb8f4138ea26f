"""The circulant (BCCB) preconditioner, FP64 (test infrastructure; oracle only).

Theory, Preconditioning: M^{-1} = F^H diag(k)^{-1} F (Eq. precon) with k the
diagonal of K = F A F^H (Eq. K), k = mu k_c + lam k_d + gam k_w (Eq. Kdiag).

Efficient Implementation of the Preconditioner derives k_c from the BCCB
matrices C_i = F S_i F^H (Eqs. d and diagonalelements).  Written out with the
unnormalised DFT s^_i of the coil map s_i, (C_i)_{lj} = s^_i(l - j) / N, so
    k_c(j) = (1/N^2) sum_l r(l) P(l - j),   P = sum_i |s^_i|^2,
a circular cross-correlation of the mask with the k-space coil power (reading
of the paper's convolution notation, decided by the brute-force definition
below).  k_d is the symbol of the periodic Laplacian D_x^H D_x + D_y^H D_y
and k_w = 1 because W is unitary.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops


def coil_power(S: np.ndarray) -> np.ndarray:
    """P = sum_i |DFT(s_i)|^2 with the unnormalised 2D DFT."""
    return np.sum(np.abs(np.fft.fft2(S)) ** 2, axis=0)


def k_coil(S: np.ndarray, r2d: np.ndarray) -> np.ndarray:
    """k_c(j) = (1/N^2) sum_l r(l) P(l - j) via the DFT:
    the cross-correlation has DFT  DFT(r) conj(DFT(P))."""
    m, n = r2d.shape
    N = m * n
    P = coil_power(S)
    corr = np.fft.ifft2(np.fft.fft2(r2d) * np.conj(np.fft.fft2(P)))
    return corr.real / (N * N)


def k_coil_direct(S: np.ndarray, r2d: np.ndarray) -> np.ndarray:
    """The same sum evaluated term by term (small sizes only)."""
    m, n = r2d.shape
    N = m * n
    P = coil_power(S)
    out = np.zeros((m, n))
    for ju in range(m):
        for jv in range(n):
            # np.roll by +j gives sh[l] = P[(l - j) mod (m, n)]
            sh = np.roll(np.roll(P, ju, axis=0), jv, axis=1)
            out[ju, jv] = np.sum(r2d * sh) / (N * N)
    return out


def k_laplacian(m: int, n: int) -> np.ndarray:
    """k_d(p, q) = 4 - 2 cos(2 pi p / m) - 2 cos(2 pi q / n): the DFT of the
    first row of the periodic D_x^H D_x + D_y^H D_y."""
    p = np.arange(m)[:, None]
    q = np.arange(n)[None, :]
    return 4.0 - 2.0 * np.cos(2.0 * np.pi * p / m) - 2.0 * np.cos(2.0 * np.pi * q / n)


def circulant_k(S, r2d, mu, lam, gam):
    """k = mu k_c + lam k_d + gam (Eq. Kdiag)."""
    m, n = r2d.shape
    return mu * k_coil(S, r2d) + lam * k_laplacian(m, n) + gam


def brute_force_k(S, r2d, mu, lam, gam, wavelet=None):
    """k_j = f_j^H A f_j with f_j = F^H e_j: the definition k = diag(F A F^H).
    Costs N applications of A; small sizes only."""
    m, n = r2d.shape
    k = np.zeros((m, n))
    for ju in range(m):
        for jv in range(n):
            e = np.zeros((m, n), np.complex128)
            e[ju, jv] = 1.0
            f = ops.ifft2u(e)
            k[ju, jv] = np.vdot(f, ops.apply_A(f, S, r2d, mu, lam, gam, wavelet)).real
    return k


def apply_minv(r: np.ndarray, k: np.ndarray) -> np.ndarray:
    """M^{-1} r = F^H diag(k)^{-1} F r (Eq. precon)."""
    return ops.ifft2u(ops.fft2u(r) / k)


def jacobi_diag(S, r2d, mu, lam, gam):
    """diag(A): e_i^H A e_i = mu (|Omega| / N) sum_c |S_c,i|^2 + 4 lam + gam,
    since every diagonal entry of F^H R F is the sampled fraction."""
    m, n = r2d.shape
    frac = r2d.sum() / (m * n)
    return mu * frac * np.sum(np.abs(S) ** 2, axis=0) + 4.0 * lam + gam


def dense_K(S, r2d, mu, lam, gam):
    """The full K = F A F^H as a dense N x N matrix (small sizes only)."""
    m, n = r2d.shape
    N = m * n
    K = np.zeros((N, N), np.complex128)
    for j in range(N):
        e = np.zeros(N, np.complex128)
        e[j] = 1.0
        f = ops.ifft2u(e.reshape(m, n))
        K[:, j] = ops.fft2u(ops.apply_A(f, S, r2d, mu, lam, gam)).ravel()
    return K


def superoptimal_d(S, r2d, mu, lam, gam):
    """Per-frequency minimiser of ||diag(d) K - I||_F: d_j = K_jj / (K^2)_jj,
    with (K^2)_jj = ||A f_j||^2 for Hermitian A.  Small sizes only."""
    m, n = r2d.shape
    d = np.zeros((m, n))
    for ju in range(m):
        for jv in range(n):
            e = np.zeros((m, n), np.complex128)
            e[ju, jv] = 1.0
            f = ops.ifft2u(e)
            Af = ops.apply_A(f, S, r2d, mu, lam, gam)
            d[ju, jv] = np.vdot(f, Af).real / np.vdot(Af, Af).real
    return d

"""System operator and its parts, FP64 (test infrastructure; oracle only).

Notation follows the paper's Theory section: x is an m x n image (axis 0 = i,
length m; axis 1 = j, length n), S_c are diagonal coil sensitivities, F is the
unitary 2D DFT, R = diag(r) the binary sampling mask.
"""
from __future__ import annotations

import numpy as np


def fft2u(x: np.ndarray) -> np.ndarray:
    """Unitary 2D DFT F over the last two axes (F^H F = I, Theory, Structure of
    the System Matrix)."""
    return np.fft.fft2(x, norm="ortho")


def ifft2u(X: np.ndarray) -> np.ndarray:
    """F^H, the inverse of fft2u."""
    return np.fft.ifft2(X, norm="ortho")


def as_mask2d(mask: np.ndarray, m: int, n: int) -> np.ndarray:
    """Binary diagonal of R as a float64 [m][n] array.  A line mask r[u] samples
    every k-space location of row u."""
    mask = np.asarray(mask)
    if mask.ndim == 1:
        return np.repeat(mask.astype(np.float64)[:, None], n, axis=1)
    return mask.astype(np.float64)


def forward(x: np.ndarray, S: np.ndarray, r2d: np.ndarray) -> np.ndarray:
    """E_c x = R F S_c x for every coil (Eq. ill0).  Returns [nc][m][n]."""
    return r2d[None] * fft2u(S * x[None])


def adjoint(y: np.ndarray, S: np.ndarray, r2d: np.ndarray) -> np.ndarray:
    """sum_c (R F S_c)^H y_c = sum_c S_c^H F^H R^H y_c."""
    return np.sum(np.conj(S) * ifft2u(r2d[None] * y), axis=0)


def Dx(v: np.ndarray) -> np.ndarray:
    """(D_x v)[i,j] = v[i,j] - v[i-1,j], periodic in i (Theory, finite-difference
    scheme with periodic boundary conditions)."""
    return v - np.roll(v, 1, axis=0)


def Dy(v: np.ndarray) -> np.ndarray:
    """(D_y v)[i,j] = v[i,j] - v[i,j-1], periodic in j."""
    return v - np.roll(v, 1, axis=1)


def DxH(w: np.ndarray) -> np.ndarray:
    """Adjoint of D_x: (D_x^H w)[i,j] = w[i,j] - w[i+1,j]."""
    return w - np.roll(w, -1, axis=0)


def DyH(w: np.ndarray) -> np.ndarray:
    """Adjoint of D_y: (D_y^H w)[i,j] = w[i,j] - w[i,j+1]."""
    return w - np.roll(w, -1, axis=1)


def tv_normal(v: np.ndarray) -> np.ndarray:
    """(D_x^H D_x + D_y^H D_y) v."""
    return DxH(Dx(v)) + DyH(Dy(v))


def apply_data(v, S, r2d, mu):
    """The data-fidelity part mu sum_c (R F S_c)^H R F S_c v of A."""
    return mu * adjoint(forward(v, S, r2d), S, r2d)


def apply_A(v, S, r2d, mu, lam, gam, wavelet=None):
    """A v with A = mu sum_c (R F S_c)^H R F S_c + lam (D_x^H D_x + D_y^H D_y)
    + gam W^H W  (Eq. system).  With `wavelet=None` the last term is gam v,
    since the orthogonal wavelet transform is unitary; with a
    ``(analysis, synthesis)`` pair it is evaluated explicitly."""
    out = apply_data(v, S, r2d, mu) + lam * tv_normal(v)
    if wavelet is None:
        out = out + gam * v
    else:
        ana, syn = wavelet
        out = out + gam * syn(ana(v))
    return out


def shrink(v: np.ndarray, t: float) -> np.ndarray:
    """Complex soft threshold v * max(1 - t/|v|, 0), zero where |v| <= t.  It is
    the minimiser of t|d| + |d - v|^2 / 2 (the l1 subproblem of Algorithm 1)."""
    a = np.abs(v)
    scale = np.where(a > t, 1.0 - t / np.where(a > 0, a, 1.0), 0.0)
    return v * scale


def objective(x, S, r2d, y, mu, lam, gam, ana):
    """Eq. original with l1 weights 1 (the thresholds of Algorithm 1):
    mu/2 sum_c ||R F S_c x - y_c||^2 + ||D_x x||_1 + ||D_y x||_1 + ||W x||_1."""
    res = forward(x, S, r2d) - y
    return (0.5 * mu * np.sum(np.abs(res) ** 2) + np.sum(np.abs(Dx(x))) + np.sum(np.abs(Dy(x)))
            + np.sum(np.abs(ana(x))))

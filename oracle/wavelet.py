"""Periodised orthonormal 2D wavelet transforms, FP64 (test infrastructure;
oracle only).

The paper uses a unitary wavelet transform W (Theory, after the difference
operators; W^H W = I in Structure of the System Matrix) and names the
Daubechies-4 wavelet (Methods, Reconstruction).  Reading: db4 = the 8-tap
extremal-phase Daubechies filter with 4 vanishing moments, periodised so that W
stays unitary.

1D analysis of a length-L signal v (L even):
    a[k] = sum_t h[t] v[(2k + t) mod L],  d[k] = sum_t g[t] v[(2k + t) mod L],
    g[t] = (-1)^t h[K-1-t].
Synthesis is the transpose (scatter of the same products).
2D: filter along axis 1 (rows) then axis 0 (columns); the approximation band
occupies [0, m/2) x [0, n/2), the band high along axis 1 sits at
[0, m/2) x [n/2, n), high along axis 0 at [m/2, m) x [0, n/2), both high at
[m/2, m) x [n/2, n) (Mallat layout); the next level recurses on the
approximation band.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def daubechies_lowpass(p: int) -> tuple:
    """Daubechies' extremal-phase lowpass filter with p vanishing moments
    (2p taps), by spectral factorisation (Daubechies, Ten Lectures on
    Wavelets, ch. 6.1): |m0|^2 = cos^{2p}(w/2) P(sin^2(w/2)) with
    P(y) = sum_{k<p} C(p-1+k, k) y^k.  Each root y_k of P gives the pair
    z + 1/z = 2 - 4 y_k; the roots z inside the unit circle are kept.
    Normalised to sum sqrt(2)."""
    if p == 1:
        return (1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0))
    coeffs = [math.comb(p - 1 + k, k) for k in range(p)]  # ascending powers of y
    yroots = np.roots(coeffs[::-1])
    zroots = []
    for y in yroots:
        # z^2 - (2 - 4y) z + 1 = 0
        b = 2.0 - 4.0 * y
        disc = np.sqrt(b * b - 4.0 + 0j)
        z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
        zroots.append(z1 if abs(z1) < 1.0 else z2)
    poly = np.array([1.0 + 0j])
    for _ in range(p):
        poly = np.convolve(poly, [1.0, 1.0])
    for z in zroots:
        poly = np.convolve(poly, [1.0, -z])
    # np.convolve lists coefficients from the highest power of z down; that is
    # the order of Daubechies' tables (h_0 = (1 + sqrt 3) / (4 sqrt 2) for p = 2).
    h = np.real(poly)
    h = h * (math.sqrt(2.0) / h.sum())
    return tuple(float(v) for v in h)


def filters(name: str):
    if name == "haar":
        h = np.array(daubechies_lowpass(1))
    elif name == "db4":
        h = np.array(daubechies_lowpass(4))
    else:
        raise ValueError(name)
    K = len(h)
    g = np.array([(-1) ** t * h[K - 1 - t] for t in range(K)])
    return h, g


def analysis_1d(v: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    L = v.shape[axis]
    half = L // 2
    k = np.arange(half)
    a = np.zeros(v.shape[:axis] + (half,) + v.shape[axis + 1:], np.result_type(v, np.float64))
    d = np.zeros_like(a)
    for t in range(len(h)):
        idx = (2 * k + t) % L
        vt = np.take(v, idx, axis=axis)
        a = a + h[t] * vt
        d = d + g[t] * vt
    return a, d


def synthesis_1d(a: np.ndarray, d: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    half = a.shape[axis]
    L = 2 * half
    out_shape = list(a.shape)
    out_shape[axis] = L
    v = np.zeros(out_shape, np.result_type(a, np.float64))
    vm = np.moveaxis(v, axis, 0)
    am = np.moveaxis(a, axis, 0)
    dm = np.moveaxis(d, axis, 0)
    k = np.arange(half)
    for t in range(len(h)):
        idx = (2 * k + t) % L
        np.add.at(vm, idx, h[t] * am + g[t] * dm)
    return v


def analysis_2d(x: np.ndarray, name: str, levels: int) -> np.ndarray:
    """W x in the Mallat layout, same shape as x."""
    h, g = filters(name)
    c = np.array(x, dtype=np.result_type(x, np.float64), copy=True)
    m, n = x.shape
    for _ in range(levels):
        blk = c[:m, :n]
        lo, hi = analysis_1d(blk, h, g, axis=1)
        rows = np.concatenate([lo, hi], axis=1)
        lo2, hi2 = analysis_1d(rows, h, g, axis=0)
        c[:m, :n] = np.concatenate([lo2, hi2], axis=0)
        m, n = m // 2, n // 2
    return c


def synthesis_2d(c: np.ndarray, name: str, levels: int) -> np.ndarray:
    """W^H c, the inverse (and adjoint) of analysis_2d."""
    h, g = filters(name)
    x = np.array(c, dtype=np.result_type(c, np.float64), copy=True)
    M, N = c.shape
    sizes = [(M >> l, N >> l) for l in range(levels)]
    for m, n in reversed(sizes):
        blk = x[:m, :n]
        rows = synthesis_1d(blk[: m // 2], blk[m // 2:], h, g, axis=0)
        x[:m, :n] = synthesis_1d(rows[:, : n // 2], rows[:, n // 2:], h, g, axis=1)
    return x


def check_levels(m: int, n: int, levels: int) -> bool:
    """Every level must act on even extents."""
    for _ in range(levels):
        if m % 2 or n % 2 or m < 2 or n < 2:
            return False
        m, n = m // 2, n // 2
    return True


def make(name: str, levels: int):
    """(analysis, synthesis) callables, or None for no wavelet term."""
    if name == "none" or levels == 0:
        return (lambda v: np.array(v, copy=True), lambda c: np.array(c, copy=True))
    return (lambda v: analysis_2d(v, name, levels), lambda c: synthesis_2d(c, name, levels))

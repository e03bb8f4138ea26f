"""Split Bregman, Algorithm 1, FP64 (test infrastructure; oracle only).

Readings of the paper that this follows:
  * shrink(v, t) = v max(1 - t/|v|, 0), elementwise on the complex modulus;
    thresholds 1/lambda and 1/gamma as written in Algorithm 1 (l1 weight 1).
  * x^[1] = root-sum-of-squares of the zero-filled coil images
    sqrt(sum_i |F^H y_i|^2), as a complex image with zero imaginary part.
  * d and b persist across outer iterations; each solve starts from the latest
    x; the whole wavelet coefficient array (approximation band included) is
    shrunk.
  * PCG stops at relative residual eps (Methods, Reconstruction).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import operators as ops
from . import pcg as pcg_mod
from . import precond as pre
from . import wavelet as wav


@dataclasses.dataclass
class SbResult:
    x: np.ndarray
    pcg_iters: List[int]
    objective: List[float]
    x_first: np.ndarray          # x after the first solve


def sos_init(y: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum(np.abs(ops.ifft2u(y)) ** 2, axis=0)).astype(np.complex128)


def make_minv(kind: str, S, r2d, mu, lam, gam, correction=None):
    if kind == "none":
        return None
    if kind == "jacobi":
        dA = pre.jacobi_diag(S, r2d, mu, lam, gam)
        return lambda r: r / dA
    if kind in ("circulant", "learned"):
        k = pre.circulant_k(S, r2d, mu, lam, gam)
        if kind == "learned":
            k = k * correction
        return lambda r: pre.apply_minv(r, k)
    raise ValueError(kind)


def split_bregman(y, S, mask, mu, lam, gam, wavelet="db4", levels=3, n_outer=20, n_inner=1,
                  tol=1e-3, maxit=1000, precond="circulant", correction=None,
                  lock: Optional[Sequence[int]] = None, x0: Optional[np.ndarray] = None,
                  track_objective=False) -> SbResult:
    """Algorithm 1 with the k-space outer update (steps 13-15) as written.

    `lock`, if given, forces the PCG iteration count of each solve (tol 0 and
    maxit = lock[s] for solve s)."""
    nc, m, n = S.shape
    r2d = ops.as_mask2d(mask, m, n)
    ana, syn = wav.make(wavelet, levels)
    A = lambda v: ops.apply_A(v, S, r2d, mu, lam, gam)
    minv = make_minv(precond, S, r2d, mu, lam, gam, correction)

    y1 = np.array(y, dtype=np.complex128)
    yj = y1.copy()
    x = sos_init(y1) if x0 is None else np.array(x0, np.complex128)
    z = np.zeros((m, n), np.complex128)
    bx, by, bw, dx, dy, dw = (z.copy() for _ in range(6))
    iters, objs = [], []
    x_first = None
    solve = 0
    for _ in range(n_outer):
        for _ in range(n_inner):
            rhs = (mu * ops.adjoint(yj, S, r2d)
                   + lam * (ops.DxH(dx - bx) + ops.DyH(dy - by)) + gam * syn(dw - bw))
            if lock is not None:
                res = pcg_mod.pcg(A, rhs, x, minv, 0.0, int(lock[solve]))
            else:
                res = pcg_mod.pcg(A, rhs, x, minv, tol, maxit)
            x = res.x
            iters.append(res.iters)
            if x_first is None:
                x_first = x.copy()
            solve += 1
            Dxx, Dyx, Wx = ops.Dx(x), ops.Dy(x), ana(x)
            dx = ops.shrink(Dxx + bx, 1.0 / lam)
            dy = ops.shrink(Dyx + by, 1.0 / lam)
            dw = ops.shrink(Wx + bw, 1.0 / gam)
            bx = bx + Dxx - dx
            by = by + Dyx - dy
            bw = bw + Wx - dw
        yj = yj + y1 - ops.forward(x, S, r2d)
        if track_objective:
            objs.append(float(ops.objective(x, S, r2d, y1, mu, lam, gam, ana)))
    return SbResult(x, iters, objs, x_first)


def split_bregman_image_domain(y, S, mask, mu, lam, gam, wavelet="db4", levels=3, n_outer=20,
                               n_inner=1, tol=1e-3, maxit=1000, precond="circulant",
                               lock=None) -> SbResult:
    """The same iteration with the outer update carried in the image domain:
    g_j = mu sum_i S_i^H F^H R^H y_i^[j] obeys g_{j+1} = g_j + g_1 - A_data x,
    where A_data is the data-fidelity part of A (R^H R = R for a binary mask).
    Equal to `split_bregman` in exact arithmetic."""
    nc, m, n = S.shape
    r2d = ops.as_mask2d(mask, m, n)
    ana, syn = wav.make(wavelet, levels)
    A = lambda v: ops.apply_A(v, S, r2d, mu, lam, gam)
    minv = make_minv(precond, S, r2d, mu, lam, gam)
    y1 = np.array(y, dtype=np.complex128)
    g1 = mu * ops.adjoint(y1, S, r2d)
    g = g1.copy()
    x = sos_init(y1)
    z = np.zeros((m, n), np.complex128)
    bx, by, bw, dx, dy, dw = (z.copy() for _ in range(6))
    iters = []
    solve = 0
    for _ in range(n_outer):
        for _ in range(n_inner):
            rhs = g + lam * (ops.DxH(dx - bx) + ops.DyH(dy - by)) + gam * syn(dw - bw)
            if lock is not None:
                res = pcg_mod.pcg(A, rhs, x, minv, 0.0, int(lock[solve]))
            else:
                res = pcg_mod.pcg(A, rhs, x, minv, tol, maxit)
            x = res.x
            iters.append(res.iters)
            solve += 1
            Dxx, Dyx, Wx = ops.Dx(x), ops.Dy(x), ana(x)
            dx = ops.shrink(Dxx + bx, 1.0 / lam)
            dy = ops.shrink(Dyx + by, 1.0 / lam)
            dw = ops.shrink(Wx + bw, 1.0 / gam)
            bx, by, bw = bx + Dxx - dx, by + Dyx - dy, bw + Wx - dw
        g = g + g1 - ops.apply_data(x, S, r2d, mu)
    return SbResult(x, iters, [], None)

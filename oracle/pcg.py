"""Preconditioned conjugate gradients, FP64 (test infrastructure; oracle only).

The paper solves A x = b (Eq. system) by CG with the circulant preconditioner
used as a left preconditioner (Complexity section: M^{-1} A x = M^{-1} b, the
preconditioner applied once per iteration to the residual).  For Hermitian
positive definite A and M this is the standard PCG recurrence (Saad, Iterative
Methods for Sparse Linear Systems, Alg. 9.1), written here with the residual
r = b - A x:

    r = b - A x0;  stop if ||r|| <= eps ||b||   (0 iterations)
    z = M^{-1} r;  p = z;  rho = Re(r^H z)
    repeat:  q = A p;  sigma = Re(p^H q);  alpha = rho / sigma
             x += alpha p;  r -= alpha q;  iterations += 1
             stop if ||r|| <= eps ||b||
             z = M^{-1} r;  rho' = Re(r^H z);  p = z + (rho'/rho) p

The tolerance is the relative residual norm (Methods, Reconstruction:
eps = 1e-3).  The iteration count is the number of products q = A p.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class PcgResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float            # recursive ||r|| / ||b|| at exit
    history: List[float]     # relres before the first and after each iteration
    breakdown: bool = False


def pcg(apply_A: Callable, b: np.ndarray, x0: np.ndarray, minv: Optional[Callable],
        tol: float, maxit: int) -> PcgResult:
    """PCG as above.  `minv=None` is the unpreconditioned method.  With tol = 0
    exactly `maxit` iterations run (iteration-locked mode)."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return PcgResult(np.zeros_like(x), 0, True, 0.0, [0.0])
    r = b - apply_A(x)
    rr = float(np.vdot(r, r).real)
    hist = [np.sqrt(rr) / bnorm]
    if rr <= (tol * bnorm) ** 2:
        return PcgResult(x, 0, True, hist[-1], hist)
    z = minv(r) if minv is not None else r.copy()
    p = z.copy()
    rho = float(np.vdot(r, z).real)
    it = 0
    while it < maxit:
        q = apply_A(p)
        sigma = float(np.vdot(p, q).real)
        if not sigma > 0.0:
            return PcgResult(x, it, False, hist[-1], hist, breakdown=True)
        alpha = rho / sigma
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        rr = float(np.vdot(r, r).real)
        hist.append(np.sqrt(rr) / bnorm)
        if rr <= (tol * bnorm) ** 2:
            return PcgResult(x, it, True, hist[-1], hist)
        z = minv(r) if minv is not None else r.copy()
        rho_new = float(np.vdot(r, z).real)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return PcgResult(x, it, False, hist[-1], hist)

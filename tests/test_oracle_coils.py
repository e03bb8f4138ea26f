"""Pins of the coil-compression oracle (Methods, Coil compression): the
covariance is Hermitian positive semidefinite with trace equal to the data
energy; keeping every virtual coil is a unitary change of coils, which leaves
the system operator, its circulant spectrum and the right-hand side exactly
unchanged; data whose coils span an r-dimensional space compress without
loss to r virtual coils; dropping coils keeps the dominant energy."""
import numpy as np

from oracle import coils as oc
from oracle import operators as ops
from oracle import precond as opre
from paper_1710_01758_amd import inputs as gen
from tests import helpers as H


def _inst(nc=6, m=32, n=32, seed=5):
    spec = gen.SliceSpec(m, n, nc, 4.0, 8, wavelet="haar", levels=1)
    return gen.make_instance(spec, seed)


def test_covariance_hermitian_psd_and_trace():
    it = _inst()
    C = oc.covariance(it.kspace)
    assert np.allclose(C, C.conj().T, atol=1e-12 * np.abs(C).max())
    w = np.linalg.eigvalsh(C)
    assert w.min() > -1e-9 * w.max()
    assert np.isclose(np.trace(C).real, np.sum(np.abs(it.kspace) ** 2))
    # Parseval: the same covariance from the zero-filled coil images
    imgs = ops.ifft2u(it.kspace)
    assert H.rel_err(oc.covariance(imgs), C) < 1e-12


def test_full_rank_compression_leaves_operator_spectrum_and_rhs_unchanged():
    it = _inst()
    s = it.spec
    yv, Sv, w, U = oc.compress(it.kspace, it.sens, s.ncoils)
    assert np.allclose(U.conj().T @ U, np.eye(s.ncoils), atol=1e-12)
    assert np.all(np.diff(w) <= 1e-9 * w[0])
    r2d = it.mask2d.astype(np.float64)
    x = gen.random_image(3, s.m, s.n)
    a0 = ops.apply_A(x, it.sens, r2d, s.mu, s.lam, s.gam)
    a1 = ops.apply_A(x, Sv, r2d, s.mu, s.lam, s.gam)
    assert H.rel_err(a1, a0) < 1e-12
    k0 = opre.circulant_k(it.sens, r2d, s.mu, s.lam, s.gam)
    k1 = opre.circulant_k(Sv, r2d, s.mu, s.lam, s.gam)
    assert H.rel_err(k1, k0) < 1e-12
    b0 = ops.adjoint(it.kspace, it.sens, r2d)
    b1 = ops.adjoint(yv, Sv, r2d)
    assert H.rel_err(b1, b0) < 1e-12


def test_low_rank_coils_compress_without_loss():
    """Six coils that are mixtures of two: two virtual coils hold every sample
    and reproduce the data term exactly."""
    it = _inst(nc=2)
    rng = np.random.default_rng(9)
    Mx = rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2))
    S6 = np.tensordot(Mx, it.sens, axes=(1, 0))
    y6 = np.tensordot(Mx, it.kspace, axes=(1, 0))
    yv, Sv, w, U = oc.compress(y6, S6, 2)
    assert w[2:].max() < 1e-10 * w[0]
    r2d = it.mask2d.astype(np.float64)
    x = gen.random_image(4, it.spec.m, it.spec.n)
    s = it.spec
    assert H.rel_err(ops.apply_A(x, Sv, r2d, s.mu, 0, 0), ops.apply_A(x, S6, r2d, s.mu, 0, 0)) < 1e-10
    assert H.rel_err(ops.adjoint(yv, Sv, r2d), ops.adjoint(y6, S6, r2d)) < 1e-10


def test_dropped_coils_hold_the_least_energy():
    it = _inst(nc=8)
    for nv in (2, 4, 6):
        yv, Sv, w, U = oc.compress(it.kspace, it.sens, nv)
        kept = np.sum(np.abs(yv) ** 2)
        assert np.isclose(kept, w[:nv].sum(), rtol=1e-10)
        # any other nv orthonormal combinations keep no more energy
        rng = np.random.default_rng(nv)
        Q, _ = np.linalg.qr(rng.standard_normal((8, nv)) + 1j * rng.standard_normal((8, nv)))
        other = np.tensordot(Q.conj().T, it.kspace, axes=(1, 0))
        assert np.sum(np.abs(other) ** 2) <= kept * (1 + 1e-12)

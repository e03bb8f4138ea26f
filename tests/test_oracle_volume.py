"""Pins of the 3D oracle (the extension of Eqs. system, K, Kdiag, d and
diagonalelements to three dimensions): dense matrices from the definitions at
a tiny size, Hermitian positivity, the closed-form spectrum against
diag(F A F^H) by brute force, the exact BCCB case (constant maps, any mask:
one PCG iteration), and p = 1 reducing to the 2D operator and spectrum."""
import numpy as np

from oracle import operators as ops
from oracle import pcg as opcg
from oracle import precond as opre
from oracle import volume as ov
from paper_1710_01758_amd import inputs as gen
from tests import helpers as H


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _dense_dft(L):
    return np.exp(-2j * np.pi * np.outer(np.arange(L), np.arange(L)) / L) / np.sqrt(L)


def _dense_diff(L):
    return np.eye(L) - np.roll(np.eye(L), 1, axis=0)


def test_apply_A3_matches_dense_matrices():
    p, m, n, nc = 3, 4, 2, 2
    S = _rand((nc, p, m, n), 1)
    r3 = (np.random.default_rng(2).random((p, m, n)) < 0.5).astype(float)
    mu, lam, gam = 0.7, 0.3, 0.2
    F = np.kron(np.kron(_dense_dft(p), _dense_dft(m)), _dense_dft(n))
    I = lambda L: np.eye(L)
    Dz = np.kron(np.kron(_dense_diff(p), I(m)), I(n))
    Dy = np.kron(np.kron(I(p), _dense_diff(m)), I(n))
    Dx = np.kron(np.kron(I(p), I(m)), _dense_diff(n))
    R = np.diag(r3.ravel())
    A = sum(np.diag(S[c].ravel()).conj().T @ F.conj().T @ R @ F @ np.diag(S[c].ravel()) for c in range(nc))
    A = mu * A + lam * (Dz.T @ Dz + Dy.T @ Dy + Dx.T @ Dx) + gam * np.eye(p * m * n)
    v = _rand((p, m, n), 3)
    assert H.rel_err(ov.apply_A3(v, S, r3, mu, lam, gam).ravel(), A @ v.ravel()) < 1e-12
    assert np.allclose(A, A.conj().T, atol=1e-12)
    assert np.linalg.eigvalsh(A).min() >= gam * (1 - 1e-10)


def test_k3_closed_form_equals_brute_force():
    p, m, n, nc = 4, 6, 4, 3
    S = _rand((nc, p, m, n), 4) * np.exp(1j * np.random.default_rng(5).uniform(0, 6, (nc, p, m, n)))
    r3 = (np.random.default_rng(6).random((p, m, n)) < 0.4).astype(float)
    k = ov.circulant_k3(S, r3, 1e-1, 4e-2, 4e-2)
    kb = ov.brute_force_k3(S, r3, 1e-1, 4e-2, 4e-2)
    assert np.max(np.abs(k - kb)) < 1e-12 * np.max(kb)


def test_constant_maps_make_A_exactly_circulant():
    p, m, n, nc = 4, 8, 8, 2
    S = np.ones((nc, p, m, n)) * (np.array([0.6, 0.8])[:, None, None, None]) + 0j
    r3 = (np.random.default_rng(7).random((p, m, n)) < 0.3).astype(float)
    mu, lam, gam = 1e-1, 4e-2, 1e-2
    k = ov.circulant_k3(S, r3, mu, lam, gam)
    v = _rand((p, m, n), 8)
    assert H.rel_err(ov.apply_A3(v, S, r3, mu, lam, gam), ov.ifft3u(k * ov.fft3u(v))) < 1e-12
    A = lambda x: ov.apply_A3(x, S, r3, mu, lam, gam)
    b = _rand((p, m, n), 9)
    res = opcg.pcg(A, b, np.zeros_like(b), lambda r: ov.apply_minv3(r, k), 1e-10, 50)
    assert res.iters == 1


def test_single_plane_reduces_to_the_2d_operator():
    spec = gen.SliceSpec(16, 16, 3, 4.0, 4, wavelet="haar", levels=1)
    it = gen.make_instance(spec, 11)
    r2 = it.mask2d.astype(float)
    v = _rand((16, 16), 12)
    a3 = ov.apply_A3(v[None], it.sens[:, None], r2[None], spec.mu, spec.lam, spec.gam)[0]
    assert H.rel_err(a3, ops.apply_A(v, it.sens, r2, spec.mu, spec.lam, spec.gam)) < 1e-12
    k3 = ov.circulant_k3(it.sens[:, None], r2[None], spec.mu, spec.lam, spec.gam)[0]
    assert H.rel_err(k3, opre.circulant_k(it.sens, r2, spec.mu, spec.lam, spec.gam)) < 1e-12


def test_volume_generator():
    spec = gen.VolumeSpec(16, 32, 32, 4, 4.0, 6)
    a = gen.make_volume_instance(spec, 3)
    b = gen.make_volume_instance(spec, 3)
    assert np.array_equal(a.kspace, b.kspace)
    assert np.allclose(np.sum(np.abs(a.sens) ** 2, axis=0), 1.0)
    assert np.all(a.mask == a.mask[:, :, :1])  # fully sampled along x
    assert abs(a.mask[:, :, 0].mean() - 0.25) < 0.02
    assert np.all(a.kspace[:, a.mask == 0] == 0)

"""Pins of the oracle's circulant spectrum k against its definition
diag(F A F^H), invariants and exact special cases (no GPU)."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import pcg as pcg_mod
from oracle import precond as pre
from tests import helpers as H

CASES = [
    # (m, n, nc, mask kind, asymmetric phase)
    (16, 16, 2, "2d", True),
    (8, 6, 3, "2d", True),
    (32, 24, 5, "2d", True),
    (16, 12, 4, "lines", True),
]


def _case(m, n, nc, kind, asym, seed=11):
    rng = np.random.default_rng(seed + m + 7 * n + nc)
    S = H.smooth_sens(rng, nc, m, n, normalise=False, asym=asym)
    if kind == "lines":
        r = (rng.random(m) < 0.4).astype(np.uint8)
        r[0] = 1
        r2d = ops.as_mask2d(r, m, n)
    else:
        r2d = (rng.random((m, n)) < 0.35).astype(np.float64)
    return S, r2d


@pytest.mark.parametrize("m,n,nc,kind,asym", CASES)
def test_closed_form_k_equals_brute_force_definition(m, n, nc, kind, asym):
    S, r2d = _case(m, n, nc, kind, asym)
    mu, lam, gam = 1e-3, 4e-3, 4e-3
    k = pre.circulant_k(S, r2d, mu, lam, gam)
    kb = pre.brute_force_k(S, r2d, mu, lam, gam)
    assert np.max(np.abs(k - kb)) <= 1e-12 * np.max(np.abs(kb))
    # the literal convolution reading is measurably wrong for asymmetric maps
    P = pre.coil_power(S)
    conv = np.fft.ifft2(np.fft.fft2(r2d) * np.fft.fft2(P)).real / (m * n) ** 2
    kconv = mu * conv + lam * pre.k_laplacian(m, n) + gam
    if kind == "2d":
        assert np.max(np.abs(kconv - kb)) > 1e-3 * np.max(np.abs(mu * pre.k_coil(S, r2d)))


def test_direct_sum_matches_dft_form():
    S, r2d = _case(8, 6, 3, "2d", True)
    assert np.allclose(pre.k_coil(S, r2d), pre.k_coil_direct(S, r2d), atol=1e-15)


def test_trace_and_mean_identities():
    S, r2d = _case(16, 12, 3, "2d", True)
    m, n = r2d.shape
    N = m * n
    mu, lam, gam = 2e-3, 3e-3, 5e-3
    k = pre.circulant_k(S, r2d, mu, lam, gam)
    trA = np.sum(pre.jacobi_diag(S, r2d, mu, lam, gam))
    assert abs(k.sum() - trA) < 1e-12 * trA
    kc = pre.k_coil(S, r2d)
    assert abs(kc.mean() - r2d.sum() / N * np.mean(np.sum(np.abs(S) ** 2, axis=0))) < 1e-14
    # jacobi_diag closed form equals brute-force e_i^H A e_i
    dA = np.array([[ops.apply_A(np.eye(1, N, i * n + j).reshape(m, n), S, r2d, mu, lam, gam)[i, j].real
                    for j in range(n)] for i in range(m)])
    assert np.allclose(dA, pre.jacobi_diag(S, r2d, mu, lam, gam), atol=1e-15)


def test_line_mask_k_coil_constant_along_v():
    S, r2d = _case(16, 12, 4, "lines", True)
    kc = pre.k_coil(S, r2d)
    assert np.max(np.abs(kc - kc[:, :1])) < 1e-16 * 10


def test_k_is_frobenius_optimal_circulant():
    """diag(F A F^H) minimises ||F^H diag(d) F - A||_F over d (unitary
    invariance: the distance equals ||diag(d) - K||_F)."""
    S, r2d = _case(8, 6, 3, "2d", True)
    mu, lam, gam = 1e-3, 4e-3, 4e-3
    K = pre.dense_K(S, r2d, mu, lam, gam)
    k = pre.circulant_k(S, r2d, mu, lam, gam).ravel()
    base = np.linalg.norm(np.diag(k) - K)
    rng = np.random.default_rng(0)
    for _ in range(5):
        d = k + 1e-4 * rng.standard_normal(k.size)
        assert np.linalg.norm(np.diag(d) - K) > base
    assert np.all(k > 0)


@pytest.mark.parametrize("case", ["const_sens_any_mask", "full_sampling", "single_identity_coil"])
def test_exact_bccb_cases(case):
    """A is exactly BCCB, so M = A: A = F^H diag(k) F, PCG converges in one
    iteration and F^H diag(k)^{-1} F b is the exact solution."""
    rng = np.random.default_rng(5)
    m, n = 16, 12
    if case == "const_sens_any_mask":
        S = (rng.standard_normal((3, 1, 1)) + 1j * rng.standard_normal((3, 1, 1))) * np.ones((3, m, n))
        r2d = (rng.random((m, n)) < 0.3).astype(np.float64)
    elif case == "full_sampling":
        S = H.smooth_sens(rng, 4, m, n, normalise=True)
        r2d = np.ones((m, n))
    else:
        S = np.ones((1, m, n), np.complex128)
        r2d = (rng.random((m, n)) < 0.3).astype(np.float64)
    mu, lam, gam = 1e-3, 4e-3, 0.0 if case == "full_sampling" else 4e-3
    if case == "full_sampling":
        lam = 4e-3  # fully sampled, TV-only (gamma = 0): still positive definite via mu
    k = pre.circulant_k(S, r2d, mu, lam, gam)
    A = lambda v: ops.apply_A(v, S, r2d, mu, lam, gam)
    v = H.rand_complex(rng, m, n)
    assert np.allclose(A(v), ops.ifft2u(k * ops.fft2u(v)), atol=1e-14)
    b = H.rand_complex(rng, m, n)
    xs = pre.apply_minv(b, k)
    assert np.allclose(A(xs), b, atol=1e-12)
    res = pcg_mod.pcg(A, b, np.zeros_like(b), lambda r: pre.apply_minv(r, k), 1e-10, 50)
    assert res.iters == 1 and res.converged


def test_superoptimal_minimises_rowwise_frobenius():
    S, r2d = _case(8, 6, 2, "2d", True)
    mu, lam, gam = 1e-3, 4e-3, 4e-3
    K = pre.dense_K(S, r2d, mu, lam, gam)
    d = pre.superoptimal_d(S, r2d, mu, lam, gam).ravel()
    I = np.eye(K.shape[0])
    base = np.linalg.norm(np.diag(d) @ K - I)
    rng = np.random.default_rng(1)
    for _ in range(5):
        dd = d * (1 + 1e-3 * rng.standard_normal(d.size))
        assert np.linalg.norm(np.diag(dd) @ K - I) > base
    # circulant inverse is close but not better
    k = pre.circulant_k(S, r2d, mu, lam, gam).ravel()
    assert np.linalg.norm(np.diag(1 / k) @ K - I) >= base

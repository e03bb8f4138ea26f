"""Pins of the oracle's operators against dense matrices built from the
definitions, closed forms and invariants (no GPU)."""
import math

import numpy as np
import pytest

from oracle import operators as ops
from oracle import wavelet as wav
from tests import helpers as H


def test_unitary_fft_matches_dense_dft():
    rng = np.random.default_rng(0)
    m, n = 8, 6
    x = H.rand_complex(rng, m, n)
    F = H.dense_dft2(m, n)
    assert np.allclose(ops.fft2u(x).ravel(), F @ x.ravel(), atol=1e-13)
    assert np.allclose(ops.ifft2u(ops.fft2u(x)), x, atol=1e-13)
    assert np.allclose(F.conj().T @ F, np.eye(m * n), atol=1e-13)


def test_differences_match_definition_and_adjoints():
    rng = np.random.default_rng(1)
    m, n = 7, 5
    x = H.rand_complex(rng, m, n)
    w = H.rand_complex(rng, m, n)
    Dx, Dy = H.dense_Dx(m, n), H.dense_Dy(m, n)
    assert np.allclose(ops.Dx(x).ravel(), Dx @ x.ravel())
    assert np.allclose(ops.Dy(x).ravel(), Dy @ x.ravel())
    assert np.allclose(ops.DxH(w).ravel(), Dx.T @ w.ravel())
    assert np.allclose(ops.DyH(w).ravel(), Dy.T @ w.ravel())
    # spot values of the backward difference with wrap
    assert ops.Dx(x)[0, 2] == x[0, 2] - x[m - 1, 2]
    assert ops.Dy(x)[3, 0] == x[3, 0] - x[3, n - 1]


def test_laplacian_symbol_is_eigenvalues_of_dense_tv():
    m, n = 6, 8
    Lmat = H.dense_Dx(m, n).T @ H.dense_Dx(m, n) + H.dense_Dy(m, n).T @ H.dense_Dy(m, n)
    F = H.dense_dft2(m, n)
    K = F @ Lmat @ F.conj().T
    from oracle import precond as pre
    assert np.allclose(K, np.diag(pre.k_laplacian(m, n).ravel()), atol=1e-12)


def test_shrink_is_prox_by_grid_search():
    for v, t in [(0.3 + 0.4j, 0.2), (-1.0 + 0.1j, 0.5), (0.05 - 0.02j, 0.1), (2 - 2j, 1.0)]:
        g = np.linspace(-3, 3, 1201)
        D = g[:, None] + 1j * g[None, :]
        obj = t * np.abs(D) + 0.5 * np.abs(D - v) ** 2
        k = np.unravel_index(np.argmin(obj), obj.shape)
        best = D[k]
        assert abs(best - ops.shrink(np.array([v]), t)[0]) <= 0.01
    assert ops.shrink(np.array([0j]), 0.5)[0] == 0
    assert ops.shrink(np.array([0.5 + 0j]), 0.5)[0] == 0  # tie at |v| = t gives 0


# ---------------------------------------------------------------- wavelets


def test_haar_closed_form_one_level():
    x = np.array([[1.0, 2.0], [3.0, 5.0]])
    c = wav.analysis_2d(x, "haar", 1)
    a, b, cc, d = 1.0, 2.0, 3.0, 5.0
    assert np.allclose(c, [[(a + b + cc + d) / 2, (a - b + cc - d) / 2],
                           [(a + b - cc - d) / 2, (a - b - cc + d) / 2]])


def test_daubechies_filters_closed_form_and_invariants():
    h2 = np.array(wav.daubechies_lowpass(2))
    s3 = math.sqrt(3.0)
    ref = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * math.sqrt(2.0))
    assert np.allclose(h2, ref, atol=1e-14)
    for p in (2, 3, 4):
        h = np.array(wav.daubechies_lowpass(p))
        K = len(h)
        assert K == 2 * p
        assert abs(h.sum() - math.sqrt(2)) < 1e-13
        for s in range(p):  # orthonormal to even shifts
            assert abs(np.dot(h[: K - 2 * s], h[2 * s:]) - (1.0 if s == 0 else 0.0)) < 1e-13
        g = np.array([(-1) ** t * h[K - 1 - t] for t in range(K)])
        for q in range(p):  # p vanishing moments of the highpass
            assert abs(np.sum(g * np.arange(K) ** q)) < 1e-9 * max(1, K ** q)
    # extremal (minimum) phase: the partial energy builds up fastest among
    # orderings of the same |H|; here simply: the largest taps come first
    h4 = np.array(wav.daubechies_lowpass(4))
    assert np.argmax(np.abs(h4)) == 1


@pytest.mark.parametrize("name,levels,m,n", [("haar", 1, 8, 8), ("db4", 1, 16, 12), ("db4", 2, 16, 16),
                                             ("db4", 3, 32, 24), ("haar", 3, 16, 8)])
def test_wavelet_unitary(name, levels, m, n):
    Wm = H.dense_of(lambda v: wav.analysis_2d(v, name, levels), m, n)
    assert np.allclose(Wm.conj().T @ Wm, np.eye(m * n), atol=1e-12)
    assert np.allclose(Wm @ Wm.conj().T, np.eye(m * n), atol=1e-12)
    Sm = H.dense_of(lambda c: wav.synthesis_2d(c, name, levels), m, n)
    assert np.allclose(Sm, Wm.conj().T, atol=1e-12)


def test_wavelet_detail_bands_vanish_on_low_order_polynomials():
    m, n = 32, 32
    i = np.arange(m)[:, None] * np.ones((1, n))
    # a cubic along axis 0, constant along axis 1: db4 has 4 vanishing moments,
    # so every high-pass-along-axis-0 coefficient away from the wrap is zero
    x = (i / m) ** 3 - 0.5 * (i / m)
    c = wav.analysis_2d(x, "db4", 1)
    hi0 = c[m // 2:, :]
    assert np.max(np.abs(hi0[: m // 2 - 4])) < 1e-12
    assert np.max(np.abs(c[:, n // 2:])) < 1e-12  # constant along axis 1


# ------------------------------------------------------------ system matrix


def _dense_A(S, r2d, mu, lam, gam, wave=None):
    nc, m, n = S.shape
    F = H.dense_dft2(m, n)
    R = np.diag(r2d.ravel())
    A = np.zeros((m * n, m * n), np.complex128)
    for c in range(nc):
        E = R @ F @ np.diag(S[c].ravel())
        A += mu * E.conj().T @ E
    Dx, Dy = H.dense_Dx(m, n), H.dense_Dy(m, n)
    A += lam * (Dx.T @ Dx + Dy.T @ Dy)
    if wave is None:
        A += gam * np.eye(m * n)
    else:
        Wm = H.dense_of(lambda v: wav.analysis_2d(v, *wave), m, n)
        A += gam * Wm.conj().T @ Wm
    return A


@pytest.mark.parametrize("masktype", ["lines", "2d"])
def test_apply_A_matches_dense_A_16x16_2coils(masktype):
    rng = np.random.default_rng(2)
    m = n = 16
    S = H.smooth_sens(rng, 2, m, n)
    if masktype == "lines":
        r = (rng.random(m) < 0.4).astype(np.uint8)
        r[0] = 1
        r2d = ops.as_mask2d(r, m, n)
    else:
        r2d = (rng.random((m, n)) < 0.35).astype(np.float64)
    mu, lam, gam = 1e-3, 4e-3, 4e-3
    A = _dense_A(S, r2d, mu, lam, gam)
    v = H.rand_complex(rng, m, n)
    assert np.allclose(ops.apply_A(v, S, r2d, mu, lam, gam).ravel(), A @ v.ravel(), atol=1e-15, rtol=1e-12)
    # explicit W^H W term equals gam * I
    ana, syn = wav.make("db4", 2)
    A2 = _dense_A(S, r2d, mu, lam, gam, wave=("db4", 2))
    assert np.allclose(A2, A, atol=1e-14)
    assert np.allclose(ops.apply_A(v, S, r2d, mu, lam, gam, (ana, syn)), ops.apply_A(v, S, r2d, mu, lam, gam),
                       atol=1e-14)


def test_A_hermitian_positive_definite_and_rayleigh_bounds():
    rng = np.random.default_rng(3)
    m, n, nc = 24, 20, 3
    S = H.smooth_sens(rng, nc, m, n)
    r2d = (rng.random((m, n)) < 0.3).astype(np.float64)
    mu, lam, gam = 1e-2, 4e-3, 1e-3
    upper = mu * np.max(np.sum(np.abs(S) ** 2, axis=0)) + 8 * lam + gam
    for _ in range(8):
        u, v = H.rand_complex(rng, m, n), H.rand_complex(rng, m, n)
        Au, Av = ops.apply_A(u, S, r2d, mu, lam, gam), ops.apply_A(v, S, r2d, mu, lam, gam)
        assert abs(np.vdot(u, Av) - np.conj(np.vdot(v, Au))) < 1e-12 * np.linalg.norm(u) * np.linalg.norm(v)
        q = np.vdot(v, Av).real / np.vdot(v, v).real
        assert gam * (1 - 1e-12) <= q <= upper * (1 + 1e-12)


def test_line_mask_data_term_is_one_dimensional():
    """F^H R F for a line mask acts as a 1D transform along axis 0 only."""
    rng = np.random.default_rng(4)
    m, n = 16, 12
    r = (rng.random(m) < 0.5).astype(np.float64)
    v = H.rand_complex(rng, m, n)
    full = ops.ifft2u(ops.as_mask2d(r, m, n) * ops.fft2u(v))
    oned = np.fft.ifft(r[:, None] * np.fft.fft(v, axis=0), axis=0)
    assert np.allclose(full, oned, atol=1e-14)


def test_daubechies_4_matches_the_published_table():
    """The oracle derives db4 by spectral factorisation; the published values
    (tests/golden, Daubechies' Table 6.1) pin it from outside."""
    import pathlib
    path = pathlib.Path(__file__).parent / "golden" / "db4_lowpass_table_6_1.txt"
    ref = np.array([float(l) for l in path.read_text().splitlines() if l.strip() and not l.startswith("#")])
    h4 = np.array(wav.daubechies_lowpass(4))
    assert np.max(np.abs(h4 - ref)) < 1e-15 * 10

"""Pins of the oracle's learned-correction pieces (no GPU)."""
import math

import numpy as np
import pytest

from oracle import learned as L
from oracle import operators as ops
from oracle import precond as pre
from paper_1710_01758_amd import inputs as gen
from tests import helpers as H


def _small_problem(seed=0, m=16, n=12, nc=3):
    rng = np.random.default_rng(seed)
    S = H.smooth_sens(rng, nc, m, n)
    r = (rng.random(m) < 0.4).astype(np.uint8)
    r[0] = 1
    r2d = ops.as_mask2d(r, m, n)
    return rng, S, r2d


def test_param_layout_and_initial_correction_is_one():
    assert L.param_count() == gen.net_param_count()
    theta = gen.net_init(1)
    assert theta.size == L.param_count()
    feats = np.random.default_rng(0).standard_normal((2, 6, 16, 16))
    o, _ = L.forward(theta, feats)
    assert np.allclose(L.correction(o), 1.0, atol=1e-15)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = gen.net_init(7)
    theta[-17:-1] = 0.05 * rng.standard_normal(16)  # non-zero 1x1 weights so every layer matters
    B, Hh, W = 2, 10, 10
    feats = rng.standard_normal((B, 6, Hh, W))
    k = rng.uniform(0.5, 2.0, (B, Hh, W))
    G = rng.uniform(0.5, 2.0, (B, Hh, W))
    Hs = rng.uniform(0.2, 1.0, (B, Hh, W))
    Z = rng.uniform(0.5, 1.5, (B, Hh, W))
    f = lambda th: L.loss_and_grad_o(L.forward(th, feats)[0], k, G, Hs, Z)[0]
    _, g = L.loss_and_grad(theta, feats, k, G, Hs, Z)
    idx = np.concatenate([rng.choice(theta.size - 17, 40, replace=False), np.arange(theta.size - 17, theta.size)])
    for i in idx:
        e = np.zeros_like(theta)
        h = 1e-6 * max(1.0, abs(theta[i]))
        e[i] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def test_sufficient_statistics_loss_equals_direct_probe_loss():
    rng, S, r2d = _small_problem(4)
    m, n = r2d.shape
    mu, lam, gam = 1e-3, 4e-3, 4e-3
    A = lambda v: ops.apply_A(v, S, r2d, mu, lam, gam)
    k = pre.circulant_k(S, r2d, mu, lam, gam)
    probes = [H.rand_complex(rng, m, n) / math.sqrt(2) for _ in range(6)]
    G, Hs, Z = L.probe_stats(A, probes)
    c = rng.uniform(0.5, 2.0, (m, n))
    o = np.log(np.expm1(c))  # softplus^{-1}
    loss, _ = L.loss_and_grad_o(o[None], k[None], G[None], Hs[None], Z[None])
    assert abs(loss - L.direct_probe_loss(A, probes, k, c)) < 1e-12


def test_loss_floor_is_per_frequency_optimum_and_superoptimal_with_exact_statistics():
    rng, S, r2d = _small_problem(5, 8, 6, 2)
    m, n = r2d.shape
    mu, lam, gam = 1e-3, 4e-3, 4e-3
    A = lambda v: ops.apply_A(v, S, r2d, mu, lam, gam)
    # exact expectations for z ~ CN(0, I): G_j = ||A f_j||^2, H_j = k_j, Z_j = 1
    G = np.zeros((m, n))
    for ju in range(m):
        for jv in range(n):
            e = np.zeros((m, n), complex)
            e[ju, jv] = 1
            G[ju, jv] = np.linalg.norm(A(ops.ifft2u(e))) ** 2
    k = pre.circulant_k(S, r2d, mu, lam, gam)
    Z = np.ones((m, n))
    dstar = k / G
    assert np.allclose(dstar, pre.superoptimal_d(S, r2d, mu, lam, gam), rtol=1e-12)
    cstar = 1.0 / (k * dstar)
    assert np.all(cstar >= 1 - 1e-12)  # (K^2)_jj >= K_jj^2
    best, _ = L.loss_and_grad_o(np.log(np.expm1(cstar))[None], k[None], G[None], k[None], Z[None])
    for trial in range(5):
        c = cstar * np.exp(0.05 * rng.standard_normal((m, n)))
        other, _ = L.loss_and_grad_o(np.log(np.expm1(c))[None], k[None], G[None], k[None], Z[None])
        assert other > best
    circ, _ = L.loss_and_grad_o(np.full((1, m, n), math.log(math.e - 1)), k[None], G[None], k[None], Z[None])
    assert circ >= best


def test_upsample_constant_and_identity():
    c = np.full((64, 64), 1.7)
    assert np.allclose(L.upsample_correction(c, 256, 192), 1.7)
    rng = np.random.default_rng(0)
    c = rng.uniform(0.5, 2, (64, 64))
    up = L.upsample_correction(c, 64, 64)
    sh = L.shift_index(64)
    assert np.allclose(up[np.ix_(sh, sh)], c)


def test_adam_first_step_is_signed_learning_rate():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = L.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(t1, theta - 0.01 * np.sign(g), atol=1e-7)


def test_features_ranges():
    inst = gen.make_instance(gen.SLICE_64, gen.eval_seed(1))
    s = inst.spec
    k = pre.circulant_k(inst.sens, inst.mask2d.astype(float), s.mu, s.lam, s.gam)
    f = L.features(inst.mask2d, inst.sens, k, s.mu, s.lam, s.gam)
    assert f.shape == (6, 64, 64)
    assert np.all((f[0] >= 0) & (f[0] <= 1))
    assert f[0][32, 32] == 1.0  # DC line sampled
    assert np.allclose(f[3:], 0.0)

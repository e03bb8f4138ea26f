"""Pins of four oracle functions against definitions that do not go through the
oracle's own arithmetic (no GPU):

* the Split Bregman start x^[1] (Algorithm 1, step 1: root sum of squares of
  the zero-filled coil images) against coil images built with the dense DFT
  matrix written from its definition;
* the 3x3 circular convolution of the learned correction against SciPy's
  periodic correlation and against the convolution theorem;
* the cell-centred periodic bilinear upsampling against weights worked out by
  hand for a factor of 4;
* Adam's bias correction at t = 2, 3 against the closed form for a constant
  gradient.

Each test names the mistake it is meant to catch.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import learned as L
from oracle import sb
from tests import helpers as H


# ------------------------------------------------------------------ x^[1]

def _coil_kspace(images):
    """y_c = F x_c with F the unitary 2D DFT as a dense matrix (row-major
    vec, kron(F_m, F_n)), built from the definition in tests/helpers.py."""
    nc, m, n = images.shape
    F = H.dense_dft2(m, n)
    return np.stack([(F @ img.ravel()).reshape(m, n) for img in images])


def test_sos_init_single_coil_is_magnitude_of_image():
    """One coil, full sampling: x^[1] = |F^H y| = |x| pixel by pixel.
    Catches a non-unitary inverse transform (a factor sqrt(mn) or mn) and a
    transposed axis (the image is 6 x 10, not square)."""
    rng = np.random.default_rng(11)
    x = H.rand_complex(rng, 1, 6, 10)
    got = sb.sos_init(_coil_kspace(x))
    assert got.shape == (6, 10)
    assert np.all(got.imag == 0)
    assert np.allclose(got.real, np.abs(x[0]), rtol=1e-12, atol=1e-14)


def test_sos_init_two_coils_hand_case():
    """Coil images 3 and 4i at one pixel, 5 and 12 at another, zero elsewhere:
    the root sum of squares is 5 and 13 there (a sum of magnitudes would give
    7 and 17, a sum over the wrong axis a wrong shape)."""
    m, n = 4, 6
    imgs = np.zeros((2, m, n), complex)
    imgs[0, 1, 2], imgs[1, 1, 2] = 3.0, 4.0j
    imgs[0, 3, 5], imgs[1, 3, 5] = -5.0, 12.0
    want = np.zeros((m, n))
    want[1, 2], want[3, 5] = 5.0, 13.0
    got = sb.sos_init(_coil_kspace(imgs))
    assert np.allclose(got, want, atol=1e-13)


def test_sos_init_unsampled_kspace_contributes_nothing():
    """Zero-filled data: a coil whose k-space is all zero adds nothing."""
    rng = np.random.default_rng(12)
    x = H.rand_complex(rng, 1, 8, 8)
    y = np.concatenate([_coil_kspace(x), np.zeros((1, 8, 8), complex)])
    assert np.allclose(sb.sos_init(y).real, np.abs(x[0]), rtol=1e-12)


# ----------------------------------------------------------- conv3x3

def _scipy_conv3x3(x, W, b, dil):
    """The same operation through scipy.ndimage.correlate (periodic): the 3x3
    taps are embedded, dilated, in a (2 dil + 1)^2 kernel whose centre is tap
    (1, 1)."""
    nb, ci, h, w = x.shape
    co = W.shape[0]
    y = np.zeros((nb, co, h, w))
    for o in range(co):
        for c in range(ci):
            K = np.zeros((2 * dil + 1, 2 * dil + 1))
            K[::dil, ::dil] = W[o, c]
            for s in range(nb):
                y[s, o] += ndi.correlate(x[s, c], K, mode="wrap")
        y[:, o] += b[o]
    return y


def _fft_conv3x3(x, W, b, dil):
    """Convolution theorem: a periodic correlation with kernel k is
    IDFT(DFT(x) * conj(DFT(k))) with k placed at its offsets mod the grid."""
    nb, ci, h, w = x.shape
    co = W.shape[0]
    y = np.zeros((nb, co, h, w))
    for o in range(co):
        for c in range(ci):
            k = np.zeros((h, w))
            for ky in range(3):
                for kx in range(3):
                    k[(dil * (ky - 1)) % h, (dil * (kx - 1)) % w] += W[o, c, ky, kx]
            Kf = np.conj(np.fft.fft2(k))
            y[:, o] += np.fft.ifft2(np.fft.fft2(x[:, c]) * Kf).real
        y[:, o] += b[o]
    return y


@pytest.mark.parametrize("dil", [1, 2, 4])
def test_conv3x3_matches_periodic_correlation(dil):
    """6 x 5 grid (non-square, smaller than a dilation-4 footprint, so the wrap
    is exercised on both axes).  Catches an ignored dilation, a flipped tap
    (convolution instead of correlation), swapped axes and a dropped bias."""
    rng = np.random.default_rng(20 + dil)
    x = rng.standard_normal((2, 3, 6, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    got = L.conv3x3(x, W, b, dil)
    assert np.allclose(got, _scipy_conv3x3(x, W, b, dil), rtol=1e-12, atol=1e-12)
    assert np.allclose(got, _fft_conv3x3(x, W, b, dil), rtol=1e-10, atol=1e-10)


def test_conv3x3_single_tap_is_a_shift():
    """Only tap (ky, kx) = (0, 2) set, dilation 2: y[i, j] = x[i - 2, j + 2]."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 1, 6, 5))
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 0, 2] = 1.0
    got = L.conv3x3(x, W, np.zeros(1), 2)[0, 0]
    for i in range(6):
        for j in range(5):
            assert got[i, j] == x[0, 0, (i - 2) % 6, (j + 2) % 5]


# ------------------------------------------------------- upsampling

# Cell-centred bilinear interpolation at factor 4: output sample p = 4a + q of
# an axis sits at input coordinate a + (2q - 3)/8, so a one-hot input cell a0
# reaches the eight outputs 4a0 - 2 ... 4a0 + 5 with weights 1/8, 3/8, 5/8,
# 7/8, 7/8, 5/8, 3/8, 1/8 (one minus the distance to the cell centre).
_PROFILE4 = np.array([1, 3, 5, 7, 7, 5, 3, 1]) / 8.0


def _hand_profile(L_out, a0):
    p = np.zeros(L_out)
    for t, wgt in enumerate(_PROFILE4):
        p[(4 * a0 - 2 + t) % L_out] += wgt
    return p


@pytest.mark.parametrize("cell", [(0, 0), (17, 40), (63, 5)])
def test_upsample_one_hot_matches_hand_weights(cell):
    """64 x 64 one-hot map on the shifted grid upsampled to 256 x 256: the
    shifted output is the outer product of two hand-worked profiles, and the
    returned map is that, moved back to unshifted order (np.fft.ifftshift).
    Cells 0 and 63 wrap around the grid.  Catches a half-cell offset
    (sampling at a + q/4), a missing wrap and a wrong shift direction."""
    c = np.zeros((64, 64))
    c[cell] = 1.0
    want_shifted = np.outer(_hand_profile(256, cell[0]), _hand_profile(256, cell[1]))
    got = L.upsample_correction(c, 256, 256)
    assert np.allclose(got, np.fft.ifftshift(want_shifted), atol=1e-15)


def test_upsample_mixed_factors_row_and_column():
    """m = 256 (factor 4) and n = 64 (factor 1): along axis 1 the map is copied,
    along axis 0 it follows the factor-4 profile."""
    c = np.zeros((64, 64))
    c[10, 20] = 1.0
    want_shifted = np.outer(_hand_profile(256, 10), np.eye(64)[20])
    got = L.upsample_correction(c, 256, 64)
    assert np.allclose(got, np.fft.ifftshift(want_shifted), atol=1e-15)


# ---------------------------------------------------------------- Adam

def test_adam_bias_correction_constant_gradient():
    """With the same gradient g at every step, m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected step is lr g / (|g| + eps) at
    every t.  Without the correction, step 2 would be lr (1 - b1^2)/sqrt(1 - b2^2)
    ~ 4.25 lr.  Checked at t = 1, 2, 3."""
    lr, eps = 0.01, 1e-8
    g = np.array([0.3, -4.0, 2e-2])
    theta = np.array([1.0, -2.0, 0.5])
    m = np.zeros(3)
    v = np.zeros(3)
    for t in (1, 2, 3):
        new, m, v = L.adam_step(theta, g, m, v, t, lr, eps=eps)
        assert np.allclose(new - theta, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15), t
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
        theta = new


def test_adam_two_steps_hand_case():
    """g1 = 1, g2 = 3 (scalar): m2 = 0.09 + 0.3 = 0.39, v2 = 0.000999 + 0.009
    = 0.009999; corrected m2 / 0.19 = 2.052632, v2 / 0.001999 = 5.002001;
    step 2 = -lr * 2.052632 / (2.236515 + eps) = -0.917781 lr."""
    lr = 1.0
    th, m, v = L.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, lr)
    th2, m2, v2 = L.adam_step(th, np.array([3.0]), m, v, 2, lr)
    assert abs(m2[0] - 0.39) < 1e-15 and abs(v2[0] - 0.009999) < 1e-15
    mh = 0.39 / 0.19
    vh = 0.009999 / (1 - 0.999 ** 2)
    assert abs((th2 - th)[0] + mh / (np.sqrt(vh) + 1e-8)) < 1e-12
    assert abs((th2 - th)[0] + 0.917781) < 1e-6

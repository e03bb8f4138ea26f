"""Seeded input generators: determinism, normalisation, mask structure."""
import hashlib

import numpy as np
import pytest

from paper_1710_01758_amd import inputs as gen


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_seeded_determinism():
    a = gen.make_instance(gen.SLICE_64, gen.eval_seed(1))
    b = gen.make_instance(gen.SLICE_64, gen.eval_seed(1))
    for f in ("x_true", "sens", "mask", "kspace"):
        assert _h(getattr(a, f)) == _h(getattr(b, f))
    c = gen.make_instance(gen.SLICE_64, gen.eval_seed(1, 1))
    assert _h(a.kspace) != _h(c.kspace)


def test_coil_normalisation():
    inst = gen.make_instance(gen.SLICE_64, 123)
    s = np.sum(np.abs(inst.sens) ** 2, axis=0)
    assert np.allclose(s, 1.0, atol=1e-12)


@pytest.mark.parametrize("m,R,C", [(64, 4, 12), (256, 4, 24), (64, 8, 12), (512, 6, 32)])
def test_line_mask_counts_and_centre(m, R, C):
    rng = np.random.Generator(np.random.PCG64(5))
    mask = gen.line_mask(m, R, C, rng, vd=(m == 512))
    L = int(round(m / R))
    assert mask.sum() == L
    f = gen.signed_freq(m)
    ceff = min(C, L)
    # the centre rows: smallest |f|, ties towards negative f
    order = sorted(range(m), key=lambda u: (abs(int(f[u])), int(f[u])))
    assert all(mask[u] == 1 for u in order[:ceff])
    assert mask[0] == 1  # DC always sampled


def test_kspace_zero_filled_and_noise_level():
    spec = gen.SliceSpec(64, 64, 4, 4.0, 12, wavelet="haar", levels=1, noise_sigma=1e-3)
    inst = gen.make_instance(spec, 77)
    m2 = inst.mask2d
    assert np.all(inst.kspace[:, m2 == 0] == 0)
    # residual to the noiseless model has the requested per-sample variance
    clean = np.fft.fft2(inst.sens * inst.x_true[None], norm="ortho") * m2[None]
    res = (inst.kspace - clean)[:, m2 == 1]
    var = np.mean(np.abs(res) ** 2)
    assert 0.8e-6 < var < 1.2e-6


def test_ragged_batch_recipe():
    specs = gen.ragged_specs()
    assert len(specs) == 64
    assert {(s.m, s.n) for s in specs} <= set(gen.RAGGED_SHAPES)
    assert all(8 <= s.ncoils <= 32 for s in specs)
    assert {s.accel for s in specs} <= set(gen.RAGGED_ACCELS)
    assert all(s.centre == 2 * round(6 * s.m / 128) for s in specs)


@pytest.mark.parametrize("m,n,C", [(256, 256, 24), (64, 64, 12), (128, 192, 7), (64, 64, 1)])
def test_random_2d_mask_centre_block_is_exactly_centre_square(m, n, C):
    """The fully sampled centre of a 2D mask (Methods, Undersampling, second
    scheme) is a C x C block of the lowest frequencies, DC included: its rows
    are the C signed frequencies -C//2 .. C - C//2 - 1, likewise its columns."""
    rng = np.random.Generator(np.random.PCG64(9))
    mask = gen.random_2d_mask(m, n, 4.0, C, rng)
    fu, fv = gen.signed_freq(m), gen.signed_freq(n)
    rows = (fu >= -(C // 2)) & (fu < C - C // 2)
    cols = (fv >= -(C // 2)) & (fv < C - C // 2)
    assert rows.sum() == C and cols.sum() == C
    assert np.all(mask[np.ix_(rows, cols)] == 1)
    assert mask[0, 0] == 1
    assert mask.sum() == int(round(m * n / 4.0))

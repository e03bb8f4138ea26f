"""Every launch shape the autotuner can choose for the line-mask operator, at
every transform length: the default column-tile width and the two
alternatives (PICS_OPT_COL_TILE), each against the FP64 oracle -- apply_A
(Eq. system) within 1e-5 and three iteration-locked circulant PCG iterations
within 1e-4 (the PCG run also checks that the sigma partials follow the tile
count) -- plus the autotuner's own choice on a mixed batch."""
import sys

import numpy as np
import pytest

from oracle import operators as ops
from oracle import pcg as opcg
from oracle import sb as osb
from paper_1710_01758_amd import inputs as gen
from tests import helpers as H

pytestmark = pytest.mark.gpu

# (m, n, coils): every column-transform length, n at least 64
SHAPES = [(64, 64, 4), (128, 128, 8), (192, 192, 6), (224, 256, 5), (256, 256, 12), (320, 320, 6), (512, 512, 4),
          (1024, 512, 2)]
DEFAULT = {64: 16, 128: 16, 192: 16, 224: 16, 256: 16, 320: 16, 512: 4, 1024: 8}
ALTS = {64: (8, 32), 128: (8, 32), 224: (8, 32), 192: (8, 4), 256: (8, 4), 320: (8, 4), 512: (8, 2), 1024: (4, 2)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a ROCm device"
    return _t


@pytest.fixture(scope="module")
def B():
    from paper_1710_01758_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{m}x{n}x{c}" for m, n, c in SHAPES])
def test_every_tile_width_matches_oracle(torch, B, shape):
    m, n, nc = shape
    spec = gen.SliceSpec(m, n, nc, 4.0, max(4, m // 16), wavelet="haar", levels=1)
    it = gen.make_instance(spec, gen.eval_seed(9, m + n))
    r2d = it.mask2d.astype(np.float64)
    x = gen.random_image(31, m, n)
    ref_y = ops.apply_A(x, it.sens, r2d, spec.mu, spec.lam, spec.gam)
    A = lambda v: ops.apply_A(v, it.sens, r2d, spec.mu, spec.lam, spec.gam)
    b = spec.mu * ops.adjoint(it.kspace, it.sens, r2d)
    ref_x = opcg.pcg(A, b, np.zeros_like(b), osb.make_minv("circulant", it.sens, r2d, spec.mu, spec.lam, spec.gam),
                     0.0, 3).x
    ctx, _ = B.context_for([it])
    ctx.build_preconditioner("circulant")
    xd = B.to_device(x.astype(np.complex64).ravel())
    yd = torch.empty_like(xd)
    bd = B.to_device(b.astype(np.complex64).ravel())
    for tile in (0,) + ALTS[m]:
        ctx.set_option(B.OPT_COL_TILE, tile)
        assert ctx.tuning_tiles() == [tile or DEFAULT[m]]
        ctx.apply_A(xd, yd)
        e_apply = H.rel_err(yd.cpu().numpy().reshape(m, n), ref_y)
        sol = torch.zeros_like(bd)
        iters, _, _, _ = ctx.pcg_solve(bd, sol, 0.0, 0, maxit_per_slice=[3])
        e_pcg = H.rel_err(sol.cpu().numpy().reshape(m, n), ref_x)
        _say(f"  {m}x{n}x{nc} tile {tile or DEFAULT[m]}: apply {e_apply:.2e}, PCG x3 {e_pcg:.2e}")
        assert e_apply < 1e-5, (tile, e_apply)
        assert iters[0] == 3 and e_pcg < 1e-4, (tile, e_pcg)
    ctx.close()


def test_tile_option_rejects_unavailable_widths(torch, B):
    it = gen.make_instance(gen.SliceSpec(256, 256, 4, 4.0, 16, wavelet="haar", levels=1), 5)
    ctx, _ = B.context_for([it])
    for bad in (3, 32, 2, -1, 128):
        with pytest.raises(B.PicsError):
            ctx.set_option(B.OPT_COL_TILE, bad)
    ctx.set_option(B.OPT_COL_TILE, 8)
    ctx.set_option(B.OPT_COIL_GROUPS, 3)   # a split returns the group to the default tiles
    assert ctx.tuning_tiles() == [16] and ctx.tuning() == [3]
    ctx.close()


def test_autotuner_choice_is_valid_and_matches_oracle(torch, B, tmp_path, monkeypatch):
    monkeypatch.setenv("PICS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    specs = [gen.SliceSpec(128, 128, 8, 4.0, 12, wavelet="haar", levels=1),
             gen.SliceSpec(320, 320, 6, 4.0, 30, wavelet="haar", levels=1)]
    insts = [gen.make_instance(s, 6100 + i) for i, s in enumerate(specs)]
    ctx, _ = B.context_for(insts)
    split = ctx.autotune(B.TUNE_FORCE)
    tiles = ctx.tuning_tiles()
    _say(f"  autotuner: splits {split}, tiles {tiles}")
    for s, g, t in zip(specs, split, tiles):
        assert t == DEFAULT[s.m] or (t in ALTS[s.m] and g == 1)
    xs = [gen.random_image(40 + i, s.m, s.n) for i, s in enumerate(specs)]
    xd = B.to_device(B.pack_images(xs))
    yd = torch.empty_like(xd)
    ctx.apply_A(xd, yd)
    got = B.unpack_images(yd.cpu().numpy(), [(s.m, s.n) for s in specs])
    for it, x, g in zip(insts, xs, got):
        s = it.spec
        assert H.rel_err(g, ops.apply_A(x, it.sens, it.mask2d.astype(np.float64), s.mu, s.lam, s.gam)) < 1e-5
    text = (tmp_path / "tune.txt").read_text()
    assert text.count("=") == 2
    ctx.close()

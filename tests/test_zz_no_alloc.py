"""apply_A_noalloc (the operator for callers that cannot allocate) against
apply_A on the same inputs, through the C ABI: two calls in a row, the second
on a smaller input, so that the second reads a scratch array that still holds
the first call's partial sums.  Same kernels and the same coil split as
apply_A with that split set, so the outputs agree bit for bit; the operator
itself is also held to the oracle (Eq. system) at 1e-5 relative."""
import sys

import numpy as np
import pytest

from oracle import operators as ops
from paper_1710_01758_amd import inputs as gen
from tests import helpers as H

pytestmark = pytest.mark.gpu


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


def _case(torch, B, specs, seed0):
    insts = [gen.make_instance(sp, gen.eval_seed(8, seed0 + i)) for i, sp in enumerate(specs)]
    ctx, _ = B.context_for(insts)
    xs = [gen.random_image(700 + seed0 + i, it.spec.m, it.spec.n) for i, it in enumerate(insts)]
    xd = B.to_device(B.pack_images(xs))
    return insts, ctx, xs, xd


def _reference(torch, B, ctx, xd, split):
    """apply_A with the same coil split set on the context (its own table)."""
    y = torch.empty_like(xd)
    ctx.set_option(B.OPT_COIL_GROUPS, split)
    ctx.apply_A(xd, y, B.TERM_ALL)
    ctx.set_option(B.OPT_COIL_GROUPS, 1)
    return y


def test_apply_A_noalloc_equals_apply_A_on_two_calls(torch, B):
    big = [gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3)] * 3
    small = [gen.SliceSpec(128, 128, 8, 3.0, 12, wavelet="db4", levels=3)]
    _say("noalloc: call 1, 3 x 256x256x12, coil split 6; call 2, 1 x 128x128x8, coil split 3")
    ib, cb, xb, xdb = _case(torch, B, big, 0)
    is_, cs, xs, xds = _case(torch, B, small, 10)
    yb = torch.full_like(xdb, float("nan"))
    ys = torch.full_like(xds, float("nan"))
    cb.apply_A_noalloc(xdb, yb, B.TERM_ALL, 6)
    cs.apply_A_noalloc(xds, ys, B.TERM_ALL, 3)   # right after, on the smaller input
    torch.cuda.synchronize()
    got_b, got_s = yb.cpu().numpy(), ys.cpu().numpy()
    ref_b = _reference(torch, B, cb, xdb, 6).cpu().numpy()
    ref_s = _reference(torch, B, cs, xds, 3).cpu().numpy()
    assert np.isfinite(got_b).all() and np.isfinite(got_s).all()
    assert np.array_equal(got_b, ref_b), float(np.abs(got_b - ref_b).max())
    assert np.array_equal(got_s, ref_s), float(np.abs(got_s - ref_s).max())
    # the split only reorders the FP32 coil sum: within 1e-5 of the fused pass
    fused = torch.empty_like(xdb)
    cb.apply_A_noalloc(xdb, fused, B.TERM_ALL, 1)
    assert H.rel_err(got_b, fused.cpu().numpy()) < 1e-5
    # and the operator itself against the oracle
    for insts, got, xs_ in ((ib, got_b, xb), (is_, got_s, xs)):
        for it, g, x in zip(insts, B.unpack_images(got, [(i.spec.m, i.spec.n) for i in insts]), xs_):
            s = it.spec
            ref = ops.apply_A(x, it.sens, it.mask2d.astype(np.float64), s.mu, s.lam, s.gam)
            err = H.rel_err(g, ref)
            _say(f"  {s.m}x{s.n}x{s.ncoils}: relative error vs oracle {err:.2e}")
            assert err < 1e-5, err
    # a repeat of the first call after the second gives the same bits
    yb2 = torch.empty_like(xdb)
    cb.apply_A_noalloc(xdb, yb2, B.TERM_ALL, 6)
    assert np.array_equal(yb2.cpu().numpy(), got_b)
    cb.close()
    cs.close()


def test_apply_A_noalloc_rejects_a_split_beyond_the_scratch(torch, B):
    specs = [gen.SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3)] * 8
    _say("noalloc: 8 x 256x256x12 with a split of 12 needs 48 MiB > 32 MiB: rejected on the host")
    _, ctx, _, xd = _case(torch, B, specs, 20)
    y = torch.zeros_like(xd)
    with pytest.raises(B.PicsError) as e:
        ctx.apply_A_noalloc(xd, y, B.TERM_ALL, 12)
    assert e.value.code == B.PICS_ERR_INVALID
    assert "maximum" in str(e.value)
    with pytest.raises(B.PicsError):
        ctx.apply_A_noalloc(xd, y, B.TERM_ALL, 0)
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0   # nothing was launched
    # a split that fits still runs on the same context
    ctx.apply_A_noalloc(xd, y, B.TERM_ALL, 4)
    torch.cuda.synchronize()
    assert np.isfinite(y.cpu().numpy()).all()
    ctx.close()

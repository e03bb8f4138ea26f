"""GPU coil compression against the FP64 oracle (Methods, Coil compression):
eigenvalues of the coil covariance, and, because eigenvectors carry an
arbitrary phase each, quantities invariant to it: the system operator and
spectrum rebuilt from the virtual coil maps, and the data term of the
compressed k-space.  Keeping every virtual coil must reproduce the original
problem."""
import sys

import numpy as np
import pytest

from oracle import coils as oc
from oracle import operators as ops
from oracle import precond as opre
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


def _compressed(torch, B, insts, nvirt):
    ctx, ksp = B.context_for(insts)
    tot = sum(nvirt * it.spec.m * it.spec.n for it in insts)
    kout = torch.empty(tot, dtype=torch.complex64, device="cuda")
    sout = torch.empty(tot, dtype=torch.complex64, device="cuda")
    eig = ctx.coil_compress(ksp, nvirt, kout, sout)
    descs = [dict(B.spec_desc(it.spec), ncoils=nvirt) for it in insts]
    masks = B.to_device(B.pack_masks([it.mask for it in insts]))
    cv = B.Context(descs, sout, masks)
    return ctx, cv, kout, sout, eig


def _split(flat, insts, nvirt):
    out, o = [], 0
    for it in insts:
        k = nvirt * it.spec.m * it.spec.n
        out.append(flat[o:o + k].reshape(nvirt, it.spec.m, it.spec.n))
        o += k
    return out


def test_eigenvalues_and_compressed_operator_match_oracle(torch, B):
    _say("coil compression: eigenvalues, operator, spectrum")
    insts = [gen.make_instance(gen.SLICE_256, gen.eval_seed(2)),
             gen.make_instance(gen.SliceSpec(128, 128, 9, 3.0, 12, mask_kind="2d", wavelet="db4", levels=2), 31)]
    nvirt = 6
    ctx, cv, kout, sout, eig = _compressed(torch, B, insts, nvirt)
    o = 0  # offset of the slice's eigenvalues
    kg = _split(kout.cpu().numpy(), insts, nvirt)
    sg = _split(sout.cpu().numpy(), insts, nvirt)
    khat = torch.empty(cv.image_elems, dtype=torch.float32, device="cuda")
    cv.build_preconditioner("circulant", khat=khat)
    kk = B.unpack_images(khat.cpu().numpy(), [(it.spec.m, it.spec.n) for it in insts])
    xs = [gen.random_image(1100 + i, it.spec.m, it.spec.n) for i, it in enumerate(insts)]
    yd = torch.empty(cv.image_elems, dtype=torch.complex64, device="cuda")
    cv.apply_A(B.to_device(B.pack_images(xs)), yd)
    ys = B.unpack_images(yd.cpu().numpy(), [(it.spec.m, it.spec.n) for it in insts])
    for i, it in enumerate(insts):
        s = it.spec
        yv, Sv, w, U = oc.compress(it.kspace, it.sens, nvirt)
        e = eig[o:o + s.ncoils]
        o += s.ncoils
        assert np.max(np.abs(e - w)) < 1e-5 * w[0], (e, w)
        r2d = it.mask2d.astype(np.float64)
        ref = ops.apply_A(xs[i], Sv, r2d, s.mu, s.lam, s.gam)
        _say(f"  slice {i}: operator rel err {H.rel_err(ys[i], ref):.2e}")
        assert H.rel_err(ys[i], ref) < 1e-5
        kref = opre.circulant_k(Sv, r2d, s.mu, s.lam, s.gam)
        assert np.max(np.abs(kk[i] - kref)) / np.max(kref) < 1e-5
        bref = ops.adjoint(yv, Sv, r2d)
        bgot = ops.adjoint(kg[i].astype(np.complex128), sg[i].astype(np.complex128), r2d)
        assert H.rel_err(bgot, bref) < 1e-5
        # retained coil energy per pixel (phase-invariant)
        assert H.rel_err(np.sum(np.abs(sg[i]) ** 2, axis=0), np.sum(np.abs(Sv) ** 2, axis=0)) < 1e-5


def test_full_rank_compression_reproduces_the_problem(torch, B):
    _say("coil compression: all coils kept")
    insts = [gen.make_instance(gen.SLICE_64, gen.eval_seed(1))]
    nc = insts[0].spec.ncoils
    ctx, cv, kout, sout, eig = _compressed(torch, B, insts, nc)
    x = B.to_device(B.pack_images([gen.random_image(1200, 64, 64)]))
    y0 = torch.empty_like(x)
    y1 = torch.empty_like(x)
    ctx.apply_A(x, y0)
    cv.apply_A(x, y1)
    assert H.rel_err(y1.cpu().numpy(), y0.cpu().numpy()) < 1e-5
    k0 = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    k1 = torch.empty_like(k0)
    ctx.build_preconditioner("circulant", khat=k0)
    cv.build_preconditioner("circulant", khat=k1)
    assert H.rel_err(k1.cpu().numpy(), k0.cpu().numpy()) < 1e-5

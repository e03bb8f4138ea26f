"""Training and evaluation driver of the learned spectrum correction.

Host orchestration only: datasets are built, the network is trained and the
learned preconditioner is evaluated through libpics calls (features, probe
statistics, forward/backward/Adam kernels, spectrum build, PCG).  Random draws
(instances, probes, initial parameters, minibatch order) come from the seeded
generators in ``inputs``.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import binding as B
from . import inputs as gen

GRID = 64
NFEAT = 6


@dataclasses.dataclass
class Dataset:
    ctx: "B.Context"
    khat: object       # float [image-packed]
    features: object   # float [n][6][64][64]
    G: object
    H: object
    Z: object
    n: int
    instances: list


def build_dataset(instances, nprobes: int = 8, probe_seed: int = 90_000) -> Dataset:
    """Circulant spectra, features and probe statistics of 64 x 64 instances."""
    import torch
    ctx, _ = B.context_for(instances)
    khat = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    ctx.build_preconditioner("circulant", khat=khat)
    feats = torch.empty(len(instances) * NFEAT * GRID * GRID, dtype=torch.float32, device="cuda")
    ctx.features(khat, feats)
    probes = np.stack([B.pack_images([gen.probe_vectors(probe_seed + 7919 * i + p, 1, it.spec.m, it.spec.n)[0]
                                      for i, it in enumerate(instances)]) for p in range(nprobes)])
    pd = B.to_device(probes.astype(np.complex64).ravel())
    G = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    H = torch.empty_like(G)
    Z = torch.empty_like(G)
    ctx.probe_stats(pd, nprobes, G, H, Z)
    torch.cuda.synchronize()
    return Dataset(ctx, khat, feats, G, H, Z, len(instances), list(instances))


def dataset_loss(net: "B.Net", data: Dataset, batch: int = 16) -> float:
    """Mean loss of the network over every instance of the dataset."""
    import torch
    total = 0.0
    for s0 in range(0, data.n, batch):
        b = min(batch, data.n - s0)
        idx = torch.arange(s0, s0 + b, dtype=torch.int32, device="cuda")
        total += net.loss_grad(b, idx, data.features, data.khat, data.G, data.H, data.Z) * b
    return total / data.n


def train(net: "B.Net", data: Dataset, steps: int, batch: int = 16, lr: float = 1e-3, seed: int = 1234,
          log_every: int = 0, log=print) -> List[float]:
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = []
    order = rng.permutation(data.n)
    pos = 0
    for step in range(steps):
        if pos + batch > data.n:
            order = rng.permutation(data.n)
            pos = 0
        idx = torch.from_numpy(order[pos:pos + batch].astype(np.int32)).cuda()
        pos += batch
        losses.append(net.loss_grad(batch, idx, data.features, data.khat, data.G, data.H, data.Z))
        net.adam_step(lr)
        if log_every and (step + 1) % log_every == 0:
            log(f"learned: step {step + 1}/{steps} loss {np.mean(losses[-log_every:]):.6f}")
    return losses


def correction_for(net: "B.Net", ctx: "B.Context", khat) -> object:
    """Correction map (image-packed float) for every slice of ctx."""
    import torch
    feats = torch.empty(ctx.n * NFEAT * GRID * GRID, dtype=torch.float32, device="cuda")
    ctx.features(khat, feats)
    corr = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    net.correction(ctx, feats, corr)
    return corr


def relres_curve(ctx: "B.Context", b, x0, iters: int) -> List[float]:
    """Recursive relative residual after 0 .. iters PCG iterations (one
    iteration-locked solve per count, from the same start)."""
    import torch
    out = []
    for k in range(iters + 1):
        x = x0.clone()
        _, rel, _, _ = ctx.pcg_solve(b, x, 0.0, 0, maxit_per_slice=[k] * ctx.n)
        out.append(float(rel[0]))
    return out


def evaluate_on(instance, net: Optional["B.Net"], n_outer: int = 20, curve: int = 3) -> dict:
    """PCG and Split Bregman iteration counts of one slice with the circulant
    preconditioner and (if a network is given) the learned one."""
    import torch
    ctx, ksp = B.context_for([instance])
    s = instance.spec
    khat = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    ctx.build_preconditioner("circulant", khat=khat)
    corr = correction_for(net, ctx, khat) if net is not None else None
    res = {}
    kinds = ["circulant"] + (["learned"] if net is not None else [])
    for kind in kinds:
        rc = ctx.build_preconditioner(kind, correction=corr if kind == "learned" else None)
        x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")
        it, _ = ctx.split_bregman_recon(ksp, x, n_outer=n_outer, tol=1e-3, maxit=1000)
        r = {"sb_pcg_iters": it[:, 0].tolist(), "sb_total": int(it[:, 0].sum()), "build_rc": int(rc)}
        res[kind] = r
    if corr is not None:
        c = corr.cpu().numpy()
        res["correction_range"] = [float(c.min()), float(c.max())]
    ctx.close()
    return res


def pcg_first_solve(instance, net: Optional["B.Net"], curve: int = 3) -> dict:
    """PCG on A x = b with b = A x_true from x0 = 0: iterations to 1e-3 and
    the relative residual after 0..curve iterations, per preconditioner."""
    import torch
    ctx, ksp = B.context_for([instance])
    khat = torch.empty(ctx.image_elems, dtype=torch.float32, device="cuda")
    ctx.build_preconditioner("circulant", khat=khat)
    corr = correction_for(net, ctx, khat) if net is not None else None
    # right-hand side b = A x_true (x_true: the phantom)
    xt = B.to_device(instance.x_true.astype(np.complex64).ravel())
    b = torch.empty_like(xt)
    ctx.apply_A(xt, b, B.TERM_ALL)
    out = {}
    for kind in ["none", "circulant"] + (["learned"] if net is not None else []):
        ctx.build_preconditioner(kind, correction=corr if kind == "learned" else None)
        x0 = torch.zeros_like(b)
        x = x0.clone()
        it, rel, st, _ = ctx.pcg_solve(b, x, 1e-3, 1000)
        out[kind] = {"iters_to_1e-3": int(it[0]), "relres_curve": relres_curve(ctx, b, x0, curve)}
    ctx.close()
    return out


def evaluate_correction(instance, corr, n_outer: int = 20, curve: int = 3) -> dict:
    """Split Bregman counts and a PCG residual curve with a given correction."""
    import torch
    ctx, ksp = B.context_for([instance])
    rc = ctx.build_preconditioner("learned", correction=corr)
    x = torch.zeros(ctx.image_elems, dtype=torch.complex64, device="cuda")
    it, _ = ctx.split_bregman_recon(ksp, x, n_outer=n_outer, tol=1e-3, maxit=1000)
    xt = B.to_device(instance.x_true.astype(np.complex64).ravel())
    b = torch.empty_like(xt)
    ctx.apply_A(xt, b, B.TERM_ALL)
    x0 = torch.zeros_like(b)
    xx = x0.clone()
    itp, _, _, _ = ctx.pcg_solve(b, xx, 1e-3, 1000)
    out = {"sb_pcg_iters": it[:, 0].tolist(), "sb_total": int(it[:, 0].sum()), "build_rc": int(rc),
           "pcg_iters_to_1e-3": int(itp[0]), "relres_curve": relres_curve(ctx, b, x0, curve),
           "correction_range": [float(corr.min()), float(corr.max())]}
    ctx.close()
    return out

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


def superoptimal_loss(data: Dataset) -> float:
    """Loss floor of a per-instance diagonal d = H / G (reporting only)."""
    G = data.G.cpu().numpy().reshape(data.n, -1).astype(np.float64)
    H = data.H.cpu().numpy().reshape(data.n, -1).astype(np.float64)
    Z = data.Z.cpu().numpy().reshape(data.n, -1).astype(np.float64)
    per = (Z - H * H / G).sum(axis=1) / Z.sum(axis=1)
    return float(per.mean())


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

"""Seeded synthetic inputs for the PI-CS reconstruction workloads.

This module only draws random numbers and lays them out: a phantom image, smooth
complex coil sensitivities, a Cartesian random-line k-space mask and complex
Gaussian noise.  It also simulates the acquisition y_i = R (F S_i x + noise) of
the data model (paper, Theory, Eq. ill0) with ``numpy.fft`` so that a caller has
measured k-space to hand to a reconstruction.  It contains none of the
reconstruction method itself (no system operator, preconditioner, solver or
Split Bregman step) and imports neither the native library nor the oracle.

The in-vivo spine/brain data the paper measures on (Methods, MR Data
Acquisition) are not available; these generators stand in for them with the
paper's matrix sizes (128^2 .. 512^2), coil counts (12, 15) and sampling
patterns (random lines with a fully sampled centre, R = 4 / 8; Methods,
Undersampling).

Layouts (shared with the native library):
  image       complex [m][n], row-major, n contiguous; axis 0 is the
              phase-encode (line) axis
  sens        complex [nc][m][n]
  line mask   uint8  [m]        (k-space row u sampled or not; DC at u = 0)
  2D mask     uint8  [m][n]
  k-space     complex [nc][m][n], unshifted (DC at [0][0]), unitary DFT scale,
              zero at unsampled locations
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# ----------------------------------------------------------------------------
# workload descriptions
# ----------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class SliceSpec:
    """One reconstruction problem: sizes, sampling and regularisation."""

    m: int
    n: int
    ncoils: int
    accel: float            # undersampling factor R (lines kept = round(m / R))
    centre: int             # fully sampled centre lines requested
    vd: bool = False        # variable-density weights for the random lines
    mask_kind: str = "lines"  # "lines" or "2d"
    wavelet: str = "db4"    # "haar" | "db4" | "none"
    levels: int = 3
    mu: float = 1e-3
    lam: float = 4e-3
    gam: float = 4e-3
    noise_sigma: float = 1e-3
    data_scale: float = 1.0
    n_ellipses: int = 8


# Five workloads: small single slice, the headline 256^2 x 12 slice, a large
# 512^2 x 32 slice, a ragged 64-slice batch and the learned-correction case.
# Regularisation parameter sets (mu, lambda, gamma) of the paper's Methods
# section, used for the per-Bregman-iteration comparison of preconditioners.
PARAM_SETS = {1: (1e-3, 4e-3, 1e-3), 2: (1e-2, 4e-3, 1e-3), 3: (1e-3, 4e-3, 4e-3)}


SLICE_64 = SliceSpec(64, 64, 4, 4.0, 12, wavelet="haar", levels=1)
SLICE_256 = SliceSpec(256, 256, 12, 4.0, 24, wavelet="db4", levels=3)
SLICE_512 = SliceSpec(512, 512, 32, 6.0, 32, vd=True, wavelet="db4", levels=4)
LEARNED_SLICE = SLICE_256  # learned correction is evaluated on the 256^2 x 12 slice

RAGGED_SHAPES = ((128, 128), (192, 192), (256, 224), (320, 320))
RAGGED_ACCELS = (3.0, 4.0, 6.0)

EVAL_SEED_BASE = 17_100_000
TRAIN_SEED_BASE = 20_000
HELDOUT_SEED_BASE = 30_000


def eval_seed(family: int, slice_index: int = 0) -> int:
    """Seed of evaluation instance `slice_index` of a seed family (families
    keep the instances of different workloads and tests apart: 1 the 64²
    slice, 2 the 256² slice, 3 the 512² slice, 4 the ragged batch, 5 the
    learned-correction slice, others for individual tests)."""
    return EVAL_SEED_BASE + 1000 * family + slice_index


# ----------------------------------------------------------------------------
# generators
# ----------------------------------------------------------------------------


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]


def _grid(m: int, n: int):
    yi = -1.0 + (2.0 * np.arange(m) + 1.0) / m
    xj = -1.0 + (2.0 * np.arange(n) + 1.0) / n
    return np.meshgrid(yi, xj, indexing="ij")  # Y [m][n], X [m][n]


def phantom(m: int, n: int, rng: np.random.Generator, n_ellipses: int = 8) -> np.ndarray:
    """Sum of random complex ellipses on the pixel-centre grid of [-1, 1]^2."""
    Y, X = _grid(m, n)
    img = np.zeros((m, n), np.complex128)
    for _ in range(n_ellipses):
        cy, cx = rng.uniform(-0.6, 0.6, size=2)
        ay, ax = rng.uniform(0.1, 0.5, size=2)
        ang = rng.uniform(0.0, math.pi)
        inten = rng.uniform(0.1, 1.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        c, s = math.cos(ang), math.sin(ang)
        u = c * (X - cx) + s * (Y - cy)
        v = -s * (X - cx) + c * (Y - cy)
        inside = (u / ax) ** 2 + (v / ay) ** 2 <= 1.0
        img[inside] += inten * complex(math.cos(ph), math.sin(ph))
    return img


def coil_maps(m: int, n: int, nc: int, rng: np.random.Generator) -> np.ndarray:
    """Gaussian bumps on a ring of radius 1.2 with linear phase, normalised so
    that the sum over coils of |S_c|^2 is one at every pixel (the paper's
    sensitivity normalisation, Methods, Coil sensitivity maps)."""
    Y, X = _grid(m, n)
    S = np.empty((nc, m, n), np.complex128)
    for c in range(nc):
        a = 2.0 * math.pi * c / nc + rng.uniform(-math.pi / (2 * nc), math.pi / (2 * nc))
        width = rng.uniform(0.5, 0.8)
        phi0 = rng.uniform(0.0, 2.0 * math.pi)
        ay, bx = rng.uniform(-math.pi / 2, math.pi / 2, size=2)
        cy, cx = 1.2 * math.sin(a), 1.2 * math.cos(a)
        mag = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * width**2))
        S[c] = mag * np.exp(1j * (phi0 + ay * Y + bx * X))
    S /= np.sqrt(np.sum(np.abs(S) ** 2, axis=0))[None]
    return S


def signed_freq(m: int) -> np.ndarray:
    u = np.arange(m)
    return ((u + m // 2) % m) - m // 2


def line_mask(m: int, accel: float, centre: int, rng: np.random.Generator, vd: bool = False) -> np.ndarray:
    """Random k-space rows with a fully sampled centre (uint8 [m]).

    L = round(m / R) rows are kept.  The min(C, L) rows of smallest |f| form the
    centre (ties broken towards negative f); the rest are drawn without
    replacement, uniformly or with weights (1 - |f| / (m/2))^2 when vd.
    """
    L = int(round(m / accel))
    L = max(1, min(m, L))
    f = signed_freq(m)
    order = sorted(range(m), key=lambda u: (abs(int(f[u])), int(f[u])))
    c_eff = min(centre, L)
    centre_rows = order[:c_eff]
    rest = np.array(sorted(set(range(m)) - set(centre_rows)), dtype=np.int64)
    k = L - c_eff
    mask = np.zeros(m, np.uint8)
    mask[centre_rows] = 1
    if k > 0:
        if vd:
            w = (1.0 - np.abs(f[rest]) / (m / 2.0)) ** 2
            w = w / w.sum()
            pick = rng.choice(rest, size=k, replace=False, p=w)
        else:
            pick = rng.choice(rest, size=k, replace=False)
        mask[pick] = 1
    return mask


def random_2d_mask(m: int, n: int, accel: float, centre: int, rng: np.random.Generator) -> np.ndarray:
    """Fully random variable-density 2D mask (uint8 [m][n]) with a sampled
    centre square of side `centre` (Methods, Undersampling, second scheme)."""
    fu = signed_freq(m)[:, None] / (m / 2.0)
    fv = signed_freq(n)[None, :] / (n / 2.0)
    rad = np.sqrt(fu**2 + fv**2) / math.sqrt(2.0)
    w = (1.0 - rad) ** 2
    total = int(round(m * n / accel))
    mask = np.zeros((m, n), np.uint8)
    half = centre // 2
    fu_s, fv_s = signed_freq(m), signed_freq(n)
    cu = (fu_s >= -half) & (fu_s < centre - half)    # exactly `centre` rows, DC included
    cv = (fv_s >= -half) & (fv_s < centre - half)
    mask[np.ix_(cu, cv)] = 1
    k = total - int(mask.sum())
    if k > 0:
        cand = np.flatnonzero(mask.ravel() == 0)
        p = w.ravel()[cand]
        p = p / p.sum()
        pick = rng.choice(cand, size=k, replace=False, p=p)
        mask.ravel()[pick] = 1
    return mask


def expand_mask(mask: np.ndarray, m: int, n: int) -> np.ndarray:
    """A line mask uint8[m] as the equivalent 2D uint8[m][n] mask."""
    if mask.ndim == 1:
        return np.repeat(mask[:, None], n, axis=1)
    return mask


@dataclasses.dataclass
class Instance:
    spec: SliceSpec
    seed: int
    x_true: np.ndarray      # complex128 [m][n]
    sens: np.ndarray        # complex128 [nc][m][n]
    mask: np.ndarray        # uint8 [m] or [m][n]
    kspace: np.ndarray      # complex128 [nc][m][n]

    @property
    def mask2d(self) -> np.ndarray:
        return expand_mask(self.mask, self.spec.m, self.spec.n)


def simulate_kspace(x: np.ndarray, sens: np.ndarray, mask2d: np.ndarray, noise: np.ndarray) -> np.ndarray:
    """Acquisition simulation y_i = R (F S_i x + noise_i) with the unitary 2D DFT."""
    full = np.fft.fft2(sens * x[None], norm="ortho") + noise
    return full * mask2d[None].astype(np.float64)


def make_instance(spec: SliceSpec, seed: int) -> Instance:
    rp, rc, rm, rn = _streams(seed)
    x = phantom(spec.m, spec.n, rp, spec.n_ellipses) * spec.data_scale
    S = coil_maps(spec.m, spec.n, spec.ncoils, rc)
    if spec.mask_kind == "lines":
        mask = line_mask(spec.m, spec.accel, spec.centre, rm, spec.vd)
    else:
        mask = random_2d_mask(spec.m, spec.n, spec.accel, spec.centre, rm)
    sig = spec.noise_sigma * spec.data_scale / math.sqrt(2.0)
    noise = rn.normal(0.0, sig, size=(spec.ncoils, spec.m, spec.n)) + 1j * rn.normal(
        0.0, sig, size=(spec.ncoils, spec.m, spec.n))
    y = simulate_kspace(x, S, expand_mask(mask, spec.m, spec.n), noise)
    return Instance(spec, seed, x, S, mask, y)


def ragged_specs(seed: int = None, nslices: int = 64) -> List[SliceSpec]:
    """The ragged batch: per slice a size from RAGGED_SHAPES, 8..32 coils and
    R in {3, 4, 6}; centre = 2 round(6 m / 128); db4 with 3 levels."""
    if seed is None:
        seed = eval_seed(4, 999)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(nslices):
        m, n = RAGGED_SHAPES[int(rng.integers(0, len(RAGGED_SHAPES)))]
        nc = int(rng.integers(8, 33))
        accel = float(RAGGED_ACCELS[int(rng.integers(0, len(RAGGED_ACCELS)))])
        out.append(SliceSpec(m, n, nc, accel, 2 * int(round(6 * m / 128)), wavelet="db4", levels=3))
    return out


def training_spec(rng: np.random.Generator, m: int = 64, n: int = 64, nc: int = 4) -> SliceSpec:
    """One draw of the learned-correction training distribution: the small
    slice's generators with R ~ U[2, 8] and mu, lambda, gamma log-uniform over
    one decade either side of (1e-3, 4e-3, 4e-3)."""
    accel = float(rng.uniform(2.0, 8.0))
    mu, lam, gam = (b * 10.0 ** rng.uniform(-1.0, 1.0) for b in (1e-3, 4e-3, 4e-3))
    return SliceSpec(m, n, nc, accel, 12 if m == 64 else 24, wavelet="haar" if m == 64 else "db4",
                     levels=1 if m == 64 else 3, mu=mu, lam=lam, gam=gam)


def probe_vectors(seed: int, count: int, m: int, n: int) -> np.ndarray:
    """Complex Gaussian probes z ~ CN(0, I), complex128 [count][m][n]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = 1.0 / math.sqrt(2.0)
    return rng.normal(0.0, s, size=(count, m, n)) + 1j * rng.normal(0.0, s, size=(count, m, n))


def random_image(seed: int, m: int, n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))


def to_c64(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex64)


# ----------------------------------------------------------------------------
# learned spectrum correction: parameter draw and training instances
# ----------------------------------------------------------------------------

# Layer list of the correction network (cin, cout, dilation); the flat
# parameter order is W[cout][cin][3][3] then bias[cout] per layer, then the
# 1x1 layer's w[16] and bias[1] (the layout of include/pics.h).
NET_LAYERS = ((6, 32, 1), (32, 32, 1), (32, 32, 2), (32, 32, 4), (32, 32, 8), (32, 16, 1))
NET_FINAL_IN = 16


def net_param_count() -> int:
    return sum(co * ci * 9 + co for ci, co, _ in NET_LAYERS) + NET_FINAL_IN + 1


def net_init(seed: int) -> np.ndarray:
    """He-normal 3x3 weights (std sqrt(2 / (9 cin))), zero biases, zero 1x1
    weights and a 1x1 bias of ln(e - 1), so the initial correction is 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for ci, co, _ in NET_LAYERS:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), size=co * ci * 9))
        parts.append(np.zeros(co))
    parts.append(np.zeros(NET_FINAL_IN))
    parts.append(np.array([math.log(math.e - 1.0)]))
    return np.concatenate(parts)


def training_instances(count: int, base: int = TRAIN_SEED_BASE, m: int = 64, n: int = 64, nc: int = 4):
    """Instances of the learned-correction training distribution (seed base
    20000 for training, 30000 for held-out)."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(base + i))
        spec = training_spec(rng, m, n, nc)
        out.append(make_instance(spec, base + i))
    return out


# ------------------------------------------------------------------ volumes
@dataclasses.dataclass
class VolumeSpec:
    """A 3D problem [p][m][n] (axis 0 = z): ncoils, a 2D random
    variable-density pattern over the two phase-encode axes (z, y) with a
    sampled centre, fully sampled along x, and the regularisation weights."""

    p: int
    m: int
    n: int
    ncoils: int
    accel: float
    centre: int
    mu: float = 1e-3
    lam: float = 4e-3
    gam: float = 4e-3
    noise_sigma: float = 1e-3
    data_scale: float = 1.0


@dataclasses.dataclass
class VolumeInstance:
    spec: VolumeSpec
    seed: int
    x_true: np.ndarray      # complex128 [p][m][n]
    sens: np.ndarray        # complex128 [nc][p][m][n]
    mask: np.ndarray        # uint8 [p][m][n]
    kspace: np.ndarray      # complex128 [nc][p][m][n]


def volume_phantom(p: int, m: int, n: int, rng: np.random.Generator, count: int = 8) -> np.ndarray:
    """Sum of random complex ellipsoids on the voxel-centre grid of [-1, 1]^3."""
    z = -1.0 + (2.0 * np.arange(p) + 1.0) / p
    Y, X = _grid(m, n)
    out = np.zeros((p, m, n), np.complex128)
    for _ in range(count):
        cz, cy, cx = rng.uniform(-0.5, 0.5, size=3)
        az, ay, ax = rng.uniform(0.15, 0.5, size=3)
        inten = rng.uniform(0.1, 1.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        inside = (((z[:, None, None] - cz) / az) ** 2 + ((Y[None] - cy) / ay) ** 2
                  + ((X[None] - cx) / ax) ** 2) <= 1.0
        out[inside] += inten * complex(math.cos(ph), math.sin(ph))
    return out


def volume_coil_maps(p: int, m: int, n: int, nc: int, rng: np.random.Generator) -> np.ndarray:
    """Gaussian bumps on a ring around the z axis at alternating heights, with
    linear phase, normalised to sum_c |S_c|^2 = 1 at every voxel."""
    z = -1.0 + (2.0 * np.arange(p) + 1.0) / p
    Y, X = _grid(m, n)
    S = np.empty((nc, p, m, n), np.complex128)
    for c in range(nc):
        a = 2.0 * math.pi * c / nc + rng.uniform(-math.pi / (2 * nc), math.pi / (2 * nc))
        zc = 0.5 if c % 2 else -0.5
        width = rng.uniform(0.6, 0.9)
        phi0 = rng.uniform(0.0, 2.0 * math.pi)
        gz, gy, gx = rng.uniform(-math.pi / 2, math.pi / 2, size=3)
        cy, cx = 1.2 * math.sin(a), 1.2 * math.cos(a)
        d2 = (X[None] - cx) ** 2 + (Y[None] - cy) ** 2 + (z[:, None, None] - zc) ** 2
        S[c] = np.exp(-d2 / (2.0 * width**2)) * np.exp(1j * (phi0 + gz * z[:, None, None] + gy * Y[None]
                                                             + gx * X[None]))
    S /= np.sqrt(np.sum(np.abs(S) ** 2, axis=0))[None]
    return S


def make_volume_instance(spec: VolumeSpec, seed: int) -> VolumeInstance:
    rp, rc, rm, rn = _streams(seed)
    x = volume_phantom(spec.p, spec.m, spec.n, rp) * spec.data_scale
    S = volume_coil_maps(spec.p, spec.m, spec.n, spec.ncoils, rc)
    pe = random_2d_mask(spec.p, spec.m, spec.accel, spec.centre, rm)  # over (z, y)
    mask = np.repeat(pe[:, :, None], spec.n, axis=2)
    sig = spec.noise_sigma * spec.data_scale / math.sqrt(2.0)
    shape = (spec.ncoils, spec.p, spec.m, spec.n)
    noise = rn.normal(0.0, sig, size=shape) + 1j * rn.normal(0.0, sig, size=shape)
    full = np.fft.fftn(S * x[None], axes=(-3, -2, -1), norm="ortho") + noise
    return VolumeInstance(spec, seed, x, S, mask, full * mask[None].astype(np.float64))

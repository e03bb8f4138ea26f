"""Learned correction of the circulant spectrum, FP64 (test infrastructure;
oracle only).

Not in the paper: a small CNN predicts a positive multiplicative correction c
of the circulant spectrum k (Eq. Kdiag), giving M_c^{-1} = F^H diag(1/(k c)) F.
It is trained to minimise the expected preconditioned-residual energy

    L = E_z || M_c^{-1} A z - z ||^2 / E_z ||z||^2,   z ~ CN(0, I).

With a = F A z and zh = F z, F M_c^{-1} A z - F z = d a - zh (d = 1/(k c)), so
per frequency j the loss is d_j^2 G_j - 2 d_j H_j + Z_j with the probe
statistics G = E|a|^2, H = E Re(conj(a) zh), Z = E|zh|^2.  Its per-instance
minimiser d_j = H_j / G_j tends to k_j / (K^2)_jj, the row-wise Frobenius
minimiser of ||diag(d) K - I|| (the "superoptimal" diagonal).

Network (parameters in one flat float vector, order below):
  six 3x3 convolutions with circular padding, ReLU after each:
    (cin, cout, dilation) = (6,32,1) (32,32,1) (32,32,2) (32,32,4) (32,32,8) (32,16,1)
  each stored as W[cout][cin][3][3] then bias[cout];
  then a 1x1 convolution 16 -> 1: w[16] then bias[1];  c = max(softplus(o), 1e-3).
Features (6 x 64 x 64, frequency axes fft-shifted so DC sits at (32, 32)):
  0: sampled fraction of each block of k-space rows/columns (area pooling)
  1: log of the pooled unitary k-space coil energy sum_c |F s_c|^2 over its mean
  2: log of the pooled circulant spectrum k over its mean
  3-5: log10(mu / 1e-3), log10(lambda / 4e-3), log10(gamma / 4e-3)
"""
from __future__ import annotations

import math

import numpy as np

from . import operators as ops

LAYERS = [(6, 32, 1), (32, 32, 1), (32, 32, 2), (32, 32, 4), (32, 32, 8), (32, 16, 1)]
FINAL_IN = 16
GRID = 64
C_FLOOR = 1e-3
NFEAT = 6


def param_count() -> int:
    n = sum(co * ci * 9 + co for ci, co, _ in LAYERS)
    return n + FINAL_IN + 1


def unpack(theta: np.ndarray):
    """Flat vector -> list of (W, b) conv layers and (w, b) of the 1x1 layer."""
    out, o = [], 0
    for ci, co, _ in LAYERS:
        W = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    w = theta[o:o + FINAL_IN]
    o += FINAL_IN
    bf = theta[o:o + 1]
    return out, (w, bf)


def pack(convs, final) -> np.ndarray:
    parts = []
    for W, b in convs:
        parts += [np.asarray(W).ravel(), np.asarray(b).ravel()]
    parts += [np.asarray(final[0]).ravel(), np.asarray(final[1]).ravel()]
    return np.concatenate(parts)


# ------------------------------------------------------------------ layers

def conv3x3(x, W, b, dil):
    """y[n, o, i, j] = b[o] + sum_{c, ky, kx} x[n, c, (i + dil(ky-1)) mod H, (j + dil(kx-1)) mod W] W[o, c, ky, kx]."""
    y = np.zeros((x.shape[0], W.shape[0], x.shape[2], x.shape[3]))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(-dil * (ky - 1), -dil * (kx - 1)), axis=(2, 3))
            y += np.einsum("nchw,oc->nohw", xs, W[:, :, ky, kx])
    return y + b[None, :, None, None]


def conv3x3_backward(x, W, dil, gy):
    """Gradients of conv3x3 with respect to x, W and b given dL/dy."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            sh = (-dil * (ky - 1), -dil * (kx - 1))
            xs = np.roll(x, shift=sh, axis=(2, 3))
            gW[:, :, ky, kx] = np.einsum("nohw,nchw->oc", gy, xs)
            gxs = np.einsum("nohw,oc->nchw", gy, W[:, :, ky, kx])
            gx += np.roll(gxs, shift=(-sh[0], -sh[1]), axis=(2, 3))
    gb = gy.sum(axis=(0, 2, 3))
    return gx, gW, gb


def softplus(o):
    return np.where(o > 30, o, np.log1p(np.exp(np.minimum(o, 30))))


def sigmoid(o):
    return 1.0 / (1.0 + np.exp(-o))


def forward(theta, feats):
    """feats [B, 6, 64, 64] -> (o [B, 64, 64], cache)."""
    convs, (w, bf) = unpack(theta)
    acts = [feats]
    h = feats
    for (W, b), (_, _, dil) in zip(convs, LAYERS):
        h = np.maximum(conv3x3(h, W, b, dil), 0.0)
        acts.append(h)
    o = np.einsum("nchw,c->nhw", h, w) + bf[0]
    return o, acts


def correction(o):
    return np.maximum(softplus(o), C_FLOOR)


def loss_and_grad_o(o, k, G, H, Z):
    """Mean over the batch of sum_j (d^2 G - 2 d H + Z) / sum_j Z with
    d = 1 / (k c), c = max(softplus(o), floor); returns (loss, dL/do)."""
    c = correction(o)
    d = 1.0 / (k * c)
    Zs = Z.sum(axis=(1, 2))
    per = (d * d * G - 2.0 * d * H + Z).sum(axis=(1, 2)) / Zs
    B = o.shape[0]
    dLdd = (2.0 * d * G - 2.0 * H) / Zs[:, None, None] / B
    dddc = -d / c
    dcdo = np.where(softplus(o) > C_FLOOR, sigmoid(o), 0.0)
    return per.mean(), dLdd * dddc * dcdo


def backward(theta, acts, go):
    """dL/dtheta from dL/do."""
    convs, (w, bf) = unpack(theta)
    h = acts[-1]
    gw = np.einsum("nhw,nchw->c", go, h)
    gbf = np.array([go.sum()])
    gh = go[:, None, :, :] * w[None, :, None, None]
    grads = []
    for li in range(len(LAYERS) - 1, -1, -1):
        W, b = convs[li]
        dil = LAYERS[li][2]
        gh = gh * (acts[li + 1] > 0)
        gx, gW, gb = conv3x3_backward(acts[li], W, dil, gh)
        grads.append((gW, gb))
        gh = gx
    grads.reverse()
    return pack(grads, (gw, gbf))


def loss_and_grad(theta, feats, k, G, H, Z):
    o, acts = forward(theta, feats)
    L, go = loss_and_grad_o(o, k, G, H, Z)
    return L, backward(theta, acts, go)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba); t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------- features and data

def shift_index(m: int) -> np.ndarray:
    """Frequency row of shifted position a: (a - m/2) mod m (DC at m/2)."""
    return (np.arange(m) - m // 2) % m


def pool_shifted(img: np.ndarray) -> np.ndarray:
    """fft-shift an [m][n] frequency map and area-pool it to 64 x 64."""
    m, n = img.shape
    sh = img[np.ix_(shift_index(m), shift_index(n))]
    return sh.reshape(GRID, m // GRID, GRID, n // GRID).mean(axis=(1, 3))


def features(mask2d, S, k, mu, lam, gam) -> np.ndarray:
    m, n = mask2d.shape
    f0 = pool_shifted(mask2d.astype(np.float64))
    energy = np.sum(np.abs(ops.fft2u(S)) ** 2, axis=0)
    pe = pool_shifted(energy)
    f1 = np.log(pe / pe.mean() + 1e-6)
    pk = pool_shifted(k)
    f2 = np.log(pk / pk.mean())
    out = np.empty((NFEAT, GRID, GRID))
    out[0], out[1], out[2] = f0, f1, f2
    out[3] = math.log10(mu / 1e-3)
    out[4] = math.log10(lam / 4e-3)
    out[5] = math.log10(gam / 4e-3)
    return out


def upsample_correction(c64: np.ndarray, m: int, n: int) -> np.ndarray:
    """Periodic bilinear interpolation of a 64 x 64 shifted map to m x n
    (shifted, cell-centred sampling), then back to unshifted order."""
    def axis_weights(L):
        f = L // GRID
        pos = (np.arange(L) + 0.5) / f - 0.5
        i0 = np.floor(pos).astype(int)
        t = pos - i0
        return i0 % GRID, (i0 + 1) % GRID, t
    a0, a1, ta = axis_weights(m)
    b0, b1, tb = axis_weights(n)
    up = ((1 - ta)[:, None] * ((1 - tb)[None, :] * c64[np.ix_(a0, b0)] + tb[None, :] * c64[np.ix_(a0, b1)])
          + ta[:, None] * ((1 - tb)[None, :] * c64[np.ix_(a1, b0)] + tb[None, :] * c64[np.ix_(a1, b1)]))
    out = np.empty((m, n))
    out[np.ix_(shift_index(m), shift_index(n))] = up
    return out


def probe_stats(apply_A, probes):
    """G, H, Z over the probes (unitary DFT)."""
    G = H = Z = 0.0
    for z in probes:
        a = ops.fft2u(apply_A(z))
        zh = ops.fft2u(z)
        G = G + np.abs(a) ** 2
        H = H + (np.conj(a) * zh).real
        Z = Z + np.abs(zh) ** 2
    P = len(probes)
    return G / P, H / P, Z / P


def direct_probe_loss(apply_A, probes, k, c):
    """The loss evaluated straight from its definition on the probes."""
    num = den = 0.0
    for z in probes:
        rz = ops.ifft2u(ops.fft2u(apply_A(z)) / (k * c)) - z
        num += np.vdot(rz, rz).real
        den += np.vdot(z, z).real
    return num / den

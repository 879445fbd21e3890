"""FP64 reference of the peel-off optical-depth surrogate (test infrastructure only).

Only tests/ and the benchmark's checks use this module; the GPU library never
imports it.

The surrogate is not part of the paper.  It stands in for the exact mesh
traversal of a peel-off ray (Sec. 3.4, 3.6), which the paper reports as the
bulk of the run time (Sec. 3.1).  Network: 5 inputs (position x, y, z and
observer theta, phi, each mapped to [-1, 1] inside the domain) -> 4 hidden
layers of 64 ReLU units -> 1 linear output, the optical depth to the observer.  The position
enters in the coordinates of the surrogate's cylindrical domain (centre c,
outer radius r_out, scale height h(R) = h0 R^beta, half-thickness zmax h):
x = (p_x - c_x) / r_out, y = (p_y - c_y) / r_out, z = (p_z - c_z) / (zmax h(R)),
so that the steep vertical profile of a flared disk becomes a smooth function.

Flat parameter vector (12,929 values), layer by layer, each layer its weight
matrix W[in][out] row-major followed by its bias b[out]:
    W0 5x64, b0 64, W1 64x64, b1 64, W2 64x64, b2 64, W3 64x64, b3 64, W4 64x1, b4 1.
Layer l computes z_l = a_l W_l + b_l; a_{l+1} = max(z_l, 0) for l < 4; y = z_4.

`emulate_bf16` reproduces the rounding points of the BF16 matrix-core
kernels: inputs, weights, hidden activations and back-propagated errors are
rounded to bfloat16 (round to nearest, ties to even, from FP32), all sums are
exact (FP64) and biases stay unrounded.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

SIZES = (5, 64, 64, 64, 64, 1)
N_LAYERS = len(SIZES) - 1


def _offsets():
    offs, o = [], 0
    for l in range(N_LAYERS):
        w = o
        o += SIZES[l] * SIZES[l + 1]
        b = o
        o += SIZES[l + 1]
        offs.append((w, b))
    return offs, o


OFFSETS, N_PARAMS = _offsets()


def unpack(theta: np.ndarray) -> List[Tuple[np.ndarray, np.ndarray]]:
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out = []
    for l, (w, b) in enumerate(OFFSETS):
        W = theta[w:w + SIZES[l] * SIZES[l + 1]].reshape(SIZES[l], SIZES[l + 1])
        out.append((W, theta[b:b + SIZES[l + 1]]))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) after rounding to FP32; returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def forward(theta, X, emulate_bf16: bool = False):
    """Network output y[n] for inputs X[n][5]; also the activations a_0..a_4."""
    layers = unpack(theta)
    a = np.asarray(X, dtype=np.float64)
    if emulate_bf16:
        a = bf16(a)
    acts = [a]
    z = None
    for l, (W, b) in enumerate(layers):
        if emulate_bf16:
            W = bf16(W)
        z = a @ W + b
        if l < N_LAYERS - 1:
            a = np.maximum(z, 0.0)
            if emulate_bf16:
                a = bf16(a)
            acts.append(a)
    return z[:, 0], acts


def backward(theta, X, dy, emulate_bf16: bool = False) -> np.ndarray:
    """Gradient of sum_b dy[b] * y[b] with respect to the flat parameters
    (reverse-mode chain rule through the layers of `forward`)."""
    layers = unpack(theta)
    _, acts = forward(theta, X, emulate_bf16)
    delta = np.asarray(dy, dtype=np.float64)[:, None]        # dL/dz_4
    if emulate_bf16:
        delta = bf16(delta)
    grads = [None] * N_LAYERS
    for l in range(N_LAYERS - 1, -1, -1):
        W, _ = layers[l]
        if emulate_bf16:
            W = bf16(W)
        grads[l] = (acts[l].T @ delta, delta.sum(axis=0))
        if l > 0:
            g = delta @ W.T                                    # dL/da_l
            delta = g * (acts[l] > 0.0)                       # dL/dz_{l-1}
            if emulate_bf16:
                delta = bf16(delta)
    return pack(grads)


def weighted_mse(theta, X, t, w, emulate_bf16: bool = False):
    """Loss (1/n) sum w (y - t)^2 and the output error it back-propagates."""
    y, _ = forward(theta, X, emulate_bf16)
    n = len(t)
    r = y - t
    return float(np.sum(w * r * r) / n), 2.0 * w * r / n


def adam_step(theta, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, with bias correction); step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def he_uniform(seed: int) -> np.ndarray:
    """Random parameters: U(-sqrt(6/fan_in), sqrt(6/fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(N_LAYERS):
        lim = math.sqrt(6.0 / SIZES[l])
        layers.append((rng.uniform(-lim, lim, (SIZES[l], SIZES[l + 1])), np.zeros(SIZES[l + 1])))
    return pack(layers)


# ----------------------------------------------------------------------------
# validity mask of the surrogate domain

def disk_cell(p, center, r_in, r_out, h0, beta, zmax_over_h, n_r, n_z):
    """Cell (iR, iz) of positions p[n][3] in the cylindrical domain around
    `center`: R in [r_in, r_out) in n_r equal bins, z/h(R) in [-zmax, zmax) in
    n_z equal bins with h(R) = h0 R^beta; -1 where outside."""
    p = np.asarray(p, dtype=np.float64)
    d = p - np.asarray(center, dtype=np.float64)
    R = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    inside_r = (R >= r_in) & (R < r_out)
    h = h0 * np.power(np.where(R > 0, R, 1.0), beta)
    zh = d[:, 2] / h
    inside = inside_r & (np.abs(zh) < zmax_over_h)
    ir = np.floor((R - r_in) / (r_out - r_in) * n_r).astype(np.int64)
    iz = np.floor((zh + zmax_over_h) / (2 * zmax_over_h) * n_z).astype(np.int64)
    ok = inside & (ir >= 0) & (ir < n_r) & (iz >= 0) & (iz < n_z)
    return np.where(ok, ir, -1), np.where(ok, iz, -1)


def validity_mask(obs, ir, iz, tau, tau_hat, n_obs, n_r, n_z, max_err: float, min_count: int,
                  floor_frac: float = 0.0):
    """Per (observer, R bin, z bin): transmission error
    sum |exp(-tau_hat) - exp(-tau)| / sum max(exp(-tau), T_floor) over the
    validation samples in the cell, T_floor = floor_frac x the mean
    transmission of the observer's samples in the domain; valid where at least
    min_count samples fall in it and the error is at most max_err.
    Returns (valid uint8, error, count) of shape [n_obs][n_r][n_z]."""
    err_num = np.zeros((n_obs, n_r, n_z))
    den = np.zeros((n_obs, n_r, n_z))
    cnt = np.zeros((n_obs, n_r, n_z), dtype=np.int64)
    sel = ir >= 0
    o, r, z = np.asarray(obs)[sel], ir[sel], iz[sel]
    T = np.exp(-np.asarray(tau, dtype=np.float64)[sel])
    Th = np.exp(-np.maximum(np.asarray(tau_hat, dtype=np.float64)[sel], 0.0))
    t_mean = np.array([T[o == k].mean() if np.any(o == k) else 0.0 for k in range(n_obs)])
    np.add.at(err_num, (o, r, z), np.abs(Th - T))
    np.add.at(den, (o, r, z), np.maximum(T, floor_frac * t_mean[o]))
    np.add.at(cnt, (o, r, z), 1)
    err = np.where(den > 0, err_num / np.where(den > 0, den, 1.0), np.inf)
    valid = ((cnt >= min_count) & (err <= max_err)).astype(np.uint8)
    return valid, err, cnt

"""Pins of the FP64 surrogate-network oracle: gradients against central
differences, the layer wiring against a network built to compute a known
function, bfloat16 rounding against torch's conversion, Adam against its
closed-form first steps, and the validity mask against a hand-counted case."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    th = M.he_uniform(seed) * scale
    # non-zero biases so that their gradients are exercised too
    layers = M.unpack(th)
    layers = [(W.copy(), rng.uniform(-0.2, 0.2, b.shape)) for W, b in layers]
    return M.pack(layers)


def _inputs(seed, n):
    return np.random.default_rng(seed).uniform(-1, 1, (n, 5))


def test_parameter_count():
    assert M.N_PARAMS == 5 * 64 + 64 + 3 * (64 * 64 + 64) + 64 + 1 == 12929


def test_backward_matches_central_differences():
    th = _params(3)
    X = _inputs(4, 24)
    dy = np.random.default_rng(5).normal(size=24)
    # keep samples whose pre-activations are all well away from the ReLU kink
    layers = M.unpack(th)
    a, keep = X, np.ones(len(X), bool)
    for l, (W, b) in enumerate(layers[:-1]):
        z = a @ W + b
        keep &= np.min(np.abs(z), axis=1) > 1e-3
        a = np.maximum(z, 0)
    X, dy = X[keep], dy[keep]
    assert len(X) >= 8
    grad = M.backward(th, X, dy)

    def f(t):
        return float(np.dot(dy, M.forward(t, X)[0]))

    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.choice(M.N_PARAMS, 300, replace=False),
                          [b for _, b in M.OFFSETS], [M.N_PARAMS - 1]])
    h = 1e-6
    scale = np.abs(grad).max()
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (f(th + e) - f(th - e)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * scale, (i, fd, grad[i])


def test_wiring_computes_a_known_function():
    """Layer 0 splits each input into its positive and negative part, layers
    1-3 route units through different permutations, the output layer sums
    c_j |x_j| plus a constant carried by a bias unit.  A transposed weight, a
    wrong layer order or a misplaced bias changes the result."""
    rng = np.random.default_rng(11)
    perms = [rng.permutation(64) for _ in range(3)]
    W0 = np.zeros((5, 64)); b0 = np.zeros(64)
    for j in range(5):
        W0[j, 2 * j] = 1.0
        W0[j, 2 * j + 1] = -1.0
    b0[10] = 1.0                       # constant unit
    layers = [(W0, b0)]
    pos = np.arange(64)                # where each original unit sits now
    for P in perms:
        W = np.zeros((64, 64))
        W[pos, P[pos]] = 1.0           # unit at `pos` moves to P[pos]
        layers.append((W, np.zeros(64)))
        pos = P[pos]
    c = np.array([0.5, -1.25, 2.0, 0.75, -0.5])
    W4 = np.zeros((64, 1))
    for j in range(5):
        W4[pos[2 * j], 0] = c[j]
        W4[pos[2 * j + 1], 0] = c[j]
    W4[pos[10], 0] = 3.0               # 3 x the constant 1
    layers.append((W4, np.array([-0.25])))
    th = M.pack(layers)
    X = _inputs(12, 200)
    y, _ = M.forward(th, X)
    expect = np.abs(X) @ c + 3.0 - 0.25
    assert np.max(np.abs(y - expect)) < 1e-13


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 1.005859375, 1.001953125, 65504.0, 1e-30]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert M.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert M.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_bf16_emulation_stays_close_to_fp64():
    th = _params(7)
    X = _inputs(8, 500)
    y64, _ = M.forward(th, X)
    y16, _ = M.forward(th, X, emulate_bf16=True)
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 2e-2
    g64 = M.backward(th, X, np.ones(500))
    g16 = M.backward(th, X, np.ones(500), emulate_bf16=True)
    assert np.linalg.norm(g16 - g64) / np.linalg.norm(g64) < 5e-2


def test_adam_closed_form_first_steps():
    rng = np.random.default_rng(9)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50); v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = M.adam_step(th, m, v, g, 1, lr, eps=eps)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(th1, th - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps both corrected moments at g and g^2
    th2, m, v = M.adam_step(th1, m, v, g, 2, lr, eps=eps)
    assert np.allclose(th2, th1 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)


def test_weighted_mse_gradient_is_the_output_error():
    th = _params(13)
    X = _inputs(14, 40)
    t = np.random.default_rng(15).uniform(0, 3, 40)
    w = np.random.default_rng(16).uniform(0.1, 1, 40)
    L, dy = M.weighted_mse(th, X, t, w)
    h = 1e-6
    i = M.OFFSETS[4][1]        # output bias: dL/db4 = sum dy
    e = np.zeros(M.N_PARAMS); e[i] = h
    Lp, _ = M.weighted_mse(th + e, X, t, w)
    Lm, _ = M.weighted_mse(th - e, X, t, w)
    assert (Lp - Lm) / (2 * h) == pytest.approx(dy.sum(), rel=1e-8)


def test_training_fits_a_closed_form_optical_depth():
    """Homogeneous sphere: tau to the observer from p along o is
    k (-p.o + sqrt(R^2 - |p|^2 + (p.o)^2)); a short Adam run on it must cut the
    loss by two orders of magnitude."""
    rng = np.random.default_rng(21)
    n = 4096
    R, kr = 0.9, 2.0
    p = rng.uniform(-1, 1, (4 * n, 3))
    p = p[np.linalg.norm(p, axis=1) < R][:n]
    th_o = rng.uniform(0, math.pi, len(p))
    ph_o = rng.uniform(0, 2 * math.pi, len(p))
    o = np.stack([np.sin(th_o) * np.cos(ph_o), np.sin(th_o) * np.sin(ph_o), np.cos(th_o)], 1)
    po = np.sum(p * o, 1)
    tau = kr * (-po + np.sqrt(R * R - np.sum(p * p, 1) + po * po))
    X = np.column_stack([p, 2 * th_o / math.pi - 1, ph_o / math.pi - 1])
    w = np.ones(len(p))
    th = M.he_uniform(22)
    m = np.zeros_like(th); v = np.zeros_like(th)
    L0, _ = M.weighted_mse(th, X, tau, w)
    for step in range(1, 601):
        sel = rng.choice(len(p), 256, replace=False)
        _, dy = M.weighted_mse(th, X[sel], tau[sel], w[sel])
        g = M.backward(th, X[sel], dy)
        th, m, v = M.adam_step(th, m, v, g, step, 3e-3)
    L1, _ = M.weighted_mse(th, X, tau, w)
    assert L1 < 1e-2 * L0


def test_validity_mask_counts():
    # four samples in cell (obs 0, R bin 1, z bin 2), errors chosen by hand
    center = (0.0, 0.0, 0.0)
    n_r, n_z = 4, 6
    R = 0.05 + (1 + 0.5) * (0.95 / 4)          # middle of R bin 1
    h = 0.1 * R ** 1.125
    zh = -3 + (2 + 0.5) * 1.0                  # middle of z bin 2
    p = np.array([[R, 0, zh * h]] * 4 + [[0.01, 0, 0], [R, 0, 4 * h]])
    ir, iz = M.disk_cell(p, center, 0.05, 1.0, 0.1, 1.125, 3.0, n_r, n_z)
    assert list(ir) == [1, 1, 1, 1, -1, -1] and list(iz[:4]) == [2, 2, 2, 2]
    tau = np.array([1.0, 1.0, 2.0, 2.0, 1.0, 1.0])
    tau_hat = tau + np.array([0.01, -0.01, 0.0, 0.0, 5.0, 5.0])
    obs = np.zeros(6, dtype=np.int64)
    valid, err, cnt = M.validity_mask(obs, ir, iz, tau, tau_hat, 1, n_r, n_z, 0.02, 4)
    T = np.exp(-tau[:4]); Th = np.exp(-tau_hat[:4])
    assert cnt[0, 1, 2] == 4 and cnt.sum() == 4
    assert err[0, 1, 2] == pytest.approx(np.abs(Th - T).sum() / T.sum(), rel=1e-14)
    assert valid[0, 1, 2] == 1 and valid.sum() == 1
    valid, _, _ = M.validity_mask(obs, ir, iz, tau, tau_hat, 1, n_r, n_z, 0.002, 4)
    assert valid.sum() == 0
    valid, _, _ = M.validity_mask(obs, ir, iz, tau, tau_hat, 1, n_r, n_z, 0.02, 5)
    assert valid.sum() == 0


def test_validity_mask_floor():
    # one cell with faint light: relative error 50 %, but far below a floor of
    # 0.5 x the observer's mean transmission, which a bright cell sets
    center = (0.0, 0.0, 0.0)
    R = 0.05 + 0.5 * 0.95
    h = 0.1 * R ** 1.125
    p = np.array([[R, 0, -2.5 * h]] * 4 + [[R, 0, 2.5 * h]] * 4)
    ir, iz = M.disk_cell(p, center, 0.05, 1.0, 0.1, 1.125, 3.0, 1, 2)
    assert list(iz) == [0] * 4 + [1] * 4
    tau = np.array([8.0] * 4 + [0.1] * 4)
    tau_hat = tau + np.array([0.5] * 4 + [0.0] * 4)
    obs = np.zeros(8, dtype=np.int64)
    v0, e0, _ = M.validity_mask(obs, ir, iz, tau, tau_hat, 1, 1, 2, 0.02, 4)
    assert v0[0, 0, 0] == 0 and v0[0, 0, 1] == 1
    T = np.exp(-tau)
    floor = 0.5 * T.mean()
    v1, e1, _ = M.validity_mask(obs, ir, iz, tau, tau_hat, 1, 1, 2, 0.02, 4, floor_frac=0.5)
    expect = np.sum(np.abs(np.exp(-tau_hat[:4]) - T[:4])) / (4 * floor)
    assert e1[0, 0, 0] == pytest.approx(expect, rel=1e-12)
    assert v1[0, 0, 0] == 1 and v1[0, 0, 1] == 1

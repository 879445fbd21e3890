"""The oracle's surrogate peel-off: its C network against the numpy network,
its domain cells against the numpy definition, and its transport against the
exact transport event by event (the surrogate changes attenuation only)."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle import oracle as O
from synth import scenes


def _disk(n=32, orders=3, npix=32):
    return scenes.disk128(n_packets=1 << 10, n=n).replace(max_orders=orders, npix=npix, fp64=True)


def _sur(params, valid):
    return O.Surrogate(params, (0.0, 0.0, 0.0), 0.05, 1.0, 0.1, 1.125, 3.0, valid)


def test_c_network_matches_numpy_network():
    th = M.he_uniform(31).astype(np.float32)
    rng = np.random.default_rng(32)
    layers = M.unpack(th.astype(np.float64))
    layers = [(W, rng.uniform(-0.3, 0.3, b.shape)) for W, b in layers]
    th = M.pack(layers).astype(np.float32)
    X = rng.uniform(-1, 1, (2000, 5)).astype(np.float32).astype(np.float64)
    yc = O.mlp_batch(th, X)
    yn, _ = M.forward(th.astype(np.float64), X, emulate_bf16=True)
    # identical rounding points; sums differ only in FP64 order, which can flip a
    # bfloat16 tie in rare cases
    close = np.abs(yc - yn) <= 1e-12 * np.abs(yn).max()
    assert close.mean() > 0.99
    assert np.max(np.abs(yc - yn)) < 2e-2 * np.abs(yn).max()


def test_domain_cells_match_numpy_definition():
    sc = _disk()
    valid = np.ones((3, 16, 12), np.uint8)
    sg = _sur(np.zeros(M.N_PARAMS), valid)
    rng = np.random.default_rng(5)
    p = rng.uniform(-1, 1, (20000, 3))
    p[:, 2] *= 0.2
    c = O.dom_cells(sc, sg, p)
    ir, iz = M.disk_cell(p, (0, 0, 0), 0.05, 1.0, 0.1, 1.125, 3.0, 16, 12)
    expect = np.where(ir >= 0, ir * 12 + iz, -1)
    assert np.array_equal(c, expect)
    assert (c >= 0).sum() > 1000


def test_all_invalid_mask_is_the_exact_transport():
    sc = _disk()
    img0, c0, _ = O.run(sc, O.SOBOL, 1, 512)
    sg = _sur(M.he_uniform(3), np.zeros((3, 16, 12), np.uint8))
    img1, c1, _ = O.run(sc, O.SOBOL, 1, 512, surrogate=sg)
    assert np.array_equal(img0, img1)
    assert c1["surrogate"] == 0 and c1["fallbacks"] == c1["peel_rays"] == c0["peel_rays"]


def test_constant_network_changes_attenuation_only():
    """A network with zero weights and output bias c predicts tau = c.  Every
    event inside the domain must then carry exp(-c)/exp(-tau_exact) times the
    exact contribution; events outside must be unchanged."""
    sc = _disk()
    c = 0.7
    layers = [(np.zeros((M.SIZES[l], M.SIZES[l + 1])), np.zeros(M.SIZES[l + 1])) for l in range(5)]
    layers[4] = (layers[4][0], np.array([c]))
    sg = _sur(M.pack(layers), np.ones((3, 16, 12), np.uint8))
    n = 256
    _, c0, e0 = O.run(sc, O.SOBOL, 1, n, max_events=100000)
    _, c1, e1 = O.run(sc, O.SOBOL, 1, n, max_events=100000, surrogate=sg)
    assert e0.shape == e1.shape and len(e0) > 100
    assert np.array_equal(e0[:, :5], e1[:, :5])       # same positions and pixels
    cells = O.dom_cells(sc, sg, e0[:, :3])
    inside = cells >= 0
    assert inside.sum() == c1["surrogate"] > 0
    assert (~inside).sum() == c1["fallbacks"]
    osc = O.OracleScene(sc)
    for j in np.flatnonzero(inside)[:200]:
        ob = int(e0[j, 10])
        th, ph = sc.observers[ob]
        o = (math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th))
        tau, _ = O.tau_ray(osc, e0[j, :3], o)
        ratio = math.exp(-float(np.float32(c))) / math.exp(-tau)   # parameters are FP32
        assert e1[j, 5] == pytest.approx(e0[j, 5] * ratio, rel=1e-9, abs=1e-300)
    assert np.array_equal(e0[~inside, 5:8], e1[~inside, 5:8])


def test_mlp_tau_uses_domain_coordinates():
    sc = _disk()
    rng = np.random.default_rng(8)
    layers = [(rng.normal(size=(M.SIZES[l], M.SIZES[l + 1])) * 0.3, rng.normal(size=M.SIZES[l + 1]) * 0.1)
              for l in range(5)]
    th = M.pack(layers).astype(np.float32)
    sg = _sur(th, np.ones((3, 16, 12), np.uint8))
    p = np.array([0.3, -0.2, 0.01])
    for ob in range(3):
        thv, phv = sc.observers[ob]
        R = math.hypot(p[0], p[1])
        zn = p[2] / (3.0 * 0.1 * R ** 1.125)          # z over zmax h(R) of the disk domain
        x = np.array([[float(np.float32(p[0])), float(np.float32(p[1])), float(np.float32(zn)),
                       float(np.float32(2 * thv / math.pi - 1)), float(np.float32(phv / math.pi - 1))]])
        y, _ = M.forward(th.astype(np.float64), x, emulate_bf16=True)
        assert O.mlp_tau(sc, sg, p, ob) == pytest.approx(max(y[0], 0.0), rel=1e-6, abs=1e-9)

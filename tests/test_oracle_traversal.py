"""Pins of the oracle's mesh traversal (Sec. 3.4) against a brute-force integral:
collect every plane crossing along the ray, sort them, and sum kappa*rho*dt over
the pieces, each piece's cell found from its midpoint."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import scenes


def _grid_scene(shape=(7, 5, 6), seed=3, lo=(-1.0, -0.5, -0.75), hi=(1.0, 0.5, 0.75)):
    nz, ny, nx = shape
    kr = scenes.random_grid(shape, seed)
    sc = scenes.Scene(name="g", n=(nx, ny, nz), lo=lo, hi=hi, kappa_rho=kr, observers=[(0.0, 0.0)])
    return sc


def _brute_tau(sc, p, k, t_end=None):
    p = np.asarray(p, float)
    k = np.asarray(k, float)
    lo, hi, n = np.array(sc.lo), np.array(sc.hi), np.array(sc.n)
    h = (hi - lo) / n
    # exit distance of the box (the ray starts inside)
    t_exit = math.inf
    for a in range(3):
        if k[a] > 0:
            t_exit = min(t_exit, (hi[a] - p[a]) / k[a])
        elif k[a] < 0:
            t_exit = min(t_exit, (lo[a] - p[a]) / k[a])
    if t_end is not None:
        t_exit = min(t_exit, t_end)
    ts = [0.0, t_exit]
    for a in range(3):
        if k[a] == 0:
            continue
        planes = lo[a] + h[a] * np.arange(n[a] + 1)
        t = (planes - p[a]) / k[a]
        ts.extend(t[(t > 0) & (t < t_exit)].tolist())
    ts = np.unique(np.array(ts))
    tau = 0.0
    cells = set()
    for t0, t1 in zip(ts[:-1], ts[1:]):
        if t1 <= t0:
            continue
        mid = p + 0.5 * (t0 + t1) * k
        c = np.clip(np.floor((mid - lo) / h).astype(int), 0, n - 1)
        tau += float(sc.kappa_rho[c[2], c[1], c[0]]) * (t1 - t0)
        cells.add(tuple(c))
    return tau, len(cells)


def _rand_unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def test_tau_random_rays():
    sc = _grid_scene()
    osc = O.OracleScene(sc)
    rng = np.random.default_rng(11)
    for _ in range(400):
        p = rng.uniform(np.array(sc.lo) * 0.999, np.array(sc.hi) * 0.999)
        k = _rand_unit(rng)
        t, vis = O.tau_ray(osc, p, k)
        ref, ncell = _brute_tau(sc, p, k)
        assert t == pytest.approx(ref, rel=1e-12, abs=1e-13)
        assert vis == ncell


def _special_rays(sc):
    lo, hi, n = np.array(sc.lo), np.array(sc.hi), np.array(sc.n)
    h = (hi - lo) / n
    corner = lo + h * np.array([2, 1, 3])
    face_x = lo + h * np.array([3, 0.4, 2.7])
    rays = [
        (lo + h * np.array([1.3, 2.2, 0.7]), [1, 0, 0]),
        (lo + h * np.array([1.3, 2.2, 0.7]), [0, -1, 0]),
        (lo + h * np.array([1.3, 2.2, 0.7]), [0, 0, 1]),
        (corner, [1 / math.sqrt(2), 1 / math.sqrt(2), 0]),
        (corner, [-1 / math.sqrt(2), 0, 1 / math.sqrt(2)]),
        (corner, [1 / math.sqrt(3)] * 3),
        (corner, [-1 / math.sqrt(3)] * 3),
        (face_x, [1, 0, 0]),
        (face_x, [-1, 0, 0]),
        (face_x, [-0.6, 0.0, 0.8]),
        (lo + h * np.array([1.0, 2.0, 0.5]), [0, 0.6, -0.8]),
    ]
    return rays


def test_tau_special_rays():
    sc = _grid_scene(shape=(8, 8, 8), lo=(-1, -1, -1), hi=(1, 1, 1))
    osc = O.OracleScene(sc)
    for p, k in _special_rays(sc):
        k = np.array(k, float)
        k /= np.linalg.norm(k)
        t, vis = O.tau_ray(osc, p, k)
        ref, ncell = _brute_tau(sc, p, k)
        assert t == pytest.approx(ref, rel=1e-12, abs=1e-13)
        assert vis >= ncell   # zero-length pieces at edges and corners count as visits


def test_move_then_tau_back():
    sc = _grid_scene()
    osc = O.OracleScene(sc)
    rng = np.random.default_rng(5)
    n_stop = 0
    for _ in range(300):
        p = rng.uniform(np.array(sc.lo) * 0.99, np.array(sc.hi) * 0.99)
        k = _rand_unit(rng)
        edge, _ = _brute_tau(sc, p, k)
        target = rng.uniform(0.0, 1.3) * edge
        q, stopped, _ = O.move(osc, p, k, target)
        assert stopped == (target < edge) or abs(target - edge) < 1e-12
        if stopped:
            n_stop += 1
            dist = float(np.linalg.norm(q - p))
            back, _ = _brute_tau(sc, p, k, t_end=dist)
            assert back == pytest.approx(target, rel=1e-11, abs=1e-12)
    assert n_stop > 100


def test_move_zero_target_stays_put():
    sc = _grid_scene()
    osc = O.OracleScene(sc)
    p = np.array([0.1, 0.05, -0.2])
    q, stopped, vis = O.move(osc, p, [0.0, 0.6, 0.8], 0.0)
    assert stopped and vis == 1 and np.allclose(q, p, atol=0)


def test_homogeneous_chord_closed_form():
    # uniform kappa*rho: tau equals kappa*rho times the geometric chord to the box face
    n = 16
    sc = scenes.Scene(name="u", n=(n, n, n), lo=(-1,) * 3, hi=(1,) * 3,
                      kappa_rho=scenes.uniform_cube(n, 0.75), observers=[(0, 0)])
    osc = O.OracleScene(sc)
    rng = np.random.default_rng(2)
    for _ in range(200):
        p = rng.uniform(-0.9, 0.9, 3)
        k = _rand_unit(rng)
        tex = min(((1.0 if k[a] > 0 else -1.0) - p[a]) / k[a] for a in range(3) if k[a] != 0)
        t, _ = O.tau_ray(osc, p, k)
        assert t == pytest.approx(0.75 * tex, rel=1e-6)   # cells are float32 0.75 exactly

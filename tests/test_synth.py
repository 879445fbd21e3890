"""The seeded scene generators (input data only): reproducible per seed and
inside their stated ranges."""
import math

import numpy as np

from synth import scenes


def test_uneven_batch_is_reproducible():
    a = scenes.uneven_batch(7, 6, sizes=(16, 48, 16), log2_packets=(8.0, 10.0), npix=16)
    b = scenes.uneven_batch(7, 6, sizes=(16, 48, 16), log2_packets=(8.0, 10.0), npix=16)
    c = scenes.uneven_batch(8, 6, sizes=(16, 48, 16), log2_packets=(8.0, 10.0), npix=16)
    for x, y in zip(a, b):
        assert x.n == y.n and x.n_packets == y.n_packets and x.observers == y.observers
        assert np.array_equal(x.kappa_rho, y.kappa_rho)
    assert any(x.n_packets != z.n_packets or x.n != z.n for x, z in zip(a, c))


def test_uneven_batch_ranges():
    bs = scenes.uneven_batch(2406, 64)
    assert len(bs) == 64
    for sc in bs:
        n = sc.n[0]
        assert sc.n == (n, n, n) and 32 <= n <= 192 and n % 16 == 0
        assert sc.kappa_rho.shape == (n, n, n) and sc.kappa_rho.dtype == np.float32
        assert np.all(np.isfinite(sc.kappa_rho)) and np.all(sc.kappa_rho >= 0)
        assert 2 ** 16 <= sc.n_packets <= 2 ** 24
        assert 0.0 <= sc.g <= 0.8 and 0.3 <= sc.albedo <= 0.9 and sc.p_lin == 0.5
        assert 1 <= len(sc.observers) <= 4
        for th, ph in sc.observers:
            assert 0.0 <= th <= math.pi / 2 and 0.0 <= ph < 2 * math.pi
        assert 1 <= sc.max_orders <= 20 and sc.npix == 128 and not sc.fp64
        if sc.source_kind == scenes.SPHERE_SOURCE:
            assert sc.r_star == 0.02 and sc.emit_order in (0, 1)
        # optical depth along +x from the centre (the row the normalisation uses)
        row = sc.kappa_rho[n // 2, n // 2, n // 2:].astype(np.float64).sum() * (2.0 / n)
        assert 0.1 * (1 - 1e-5) <= row <= 20.0 * (1 + 1e-5)
    kinds = {sc.source_kind for sc in bs}
    assert kinds == {scenes.POINT_SOURCE, scenes.SPHERE_SOURCE}

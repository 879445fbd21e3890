"""The late-order launch (qrt_set_tail): orders from a given one on carried
through in one kernel, the peel-offs of their scatterings computed in one
launch afterwards and the peel-off rays walked in one more.

It changes how the work is launched, not what is computed, so against the
per-order launches of the same run the images agree up to the order of the
FP64 sums (per pixel |d| <= 1e-10 (I + 1e-12 max I)) and the event counters
are equal; against the oracle the FP64 gates of the parity tests hold.  The
region-full path (peel-offs computed and walked by the lane that reached the
scattering) is forced with a small limit of deferred scatterings.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from synth import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Q():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2406_15632_amd import qrt
    qrt.load()
    return qrt


@pytest.fixture()
def ctx(Q):
    c = Q.Context(0)
    yield c
    c.close()


def run(ctx, sc, kind, count, tail, max_deferred=0, precision=None, seed=0):
    ctx.set_scene(sc, kind=kind, seed=seed, precision=precision)
    ctx.set_tail(tail, max_deferred)
    ctx.reset_images()
    ctx.run(1, count)
    return ctx.read_images(normalized=False), ctx.counters()


def assert_sum_order_equal(a, b, what):
    mx = b[:, 0].max()
    assert mx > 0, what
    for ob in range(b.shape[0]):
        scale = b[ob, 0] + 1e-12 * mx
        for k in range(3):
            d = np.abs(a[ob, k] - b[ob, k])
            assert np.all(d <= 1e-10 * scale), f"{what} obs {ob} stokes {k}: max {np.max(d / scale):.3e}"


def assert_fp64_parity(g, o, what):
    for ob in range(o.shape[0]):
        Ig, Io = g[ob, 0], o[ob, 0]
        mx = Io.max()
        assert mx > 0, what
        big = Io > 1e-6 * mx
        dI = np.abs(Ig - Io)
        assert np.all(dI[big] <= 1e-5 * Io[big]), f"{what} obs {ob}: max rel {np.max(dI[big] / Io[big]):.3e}"
        assert np.all(dI[~big] <= 1e-11 * mx), what
        for s in (1, 2):
            assert np.all(np.abs(g[ob, s] - o[ob, s]) <= 1e-5 * Io + 1e-11 * mx), f"{what} obs {ob} stokes {s}"
        assert np.all(Ig[Io == 0] == 0), what


def assert_counters_close(cg, co, what):
    # the device's exp/log may differ from glibc's in the last place, which can
    # move a rare flight across a cell face or a packet across the cut-off
    for k in ("packets", "tau_cuts", "scatterings", "escapes", "visits", "peels", "occluded"):
        assert abs(cg[k] - co[k]) <= 4 + 1e-5 * co[k], f"{what} {k}: {cg[k]} vs {co[k]}"


@pytest.mark.parametrize("precision", [0, 1])
def test_tail_equals_per_order_launches(ctx, Q, precision):
    """disk at 64^3, 20 orders, three observers, 2^18 packets: the late-order
    launch from order 2, 7 and 15, and with at most 256 deferred scatterings
    (most peel-offs taken by the lanes that reached them), against every order launched on its
    own."""
    sc = scenes.disk128(n=64).replace(npix=64)
    n = 1 << 18
    _say(f"tail: per-order reference, precision {precision}")
    ref, cref = run(ctx, sc, Q.SOBOL, n, 0, precision=precision)
    assert cref["scatterings"] > 1.2 * cref["packets"]
    for tail, limit in ((2, 0), (7, 0), (15, 0), (2, 256)):
        _say(f"tail from {tail}, deferred limit {limit}, precision {precision}")
        img, cnt = run(ctx, sc, Q.SOBOL, n, tail, limit, precision=precision)
        assert cnt == cref, f"tail {tail} limit {limit}"
        assert_sum_order_equal(img, ref, f"tail {tail} limit {limit}")


@pytest.mark.parametrize("kind,limit", [(O.SOBOL, 0), (O.HALTON, 0), (O.PHILOX, 64)])
def test_tail_fp64_parity(ctx, Q, kind, limit):
    """FP64 transport with the late-order launch from order 2 (all but the
    first order in it) against the oracle: disk at 32^3, 20 orders."""
    sc = scenes.disk128(n=32).replace(npix=64, fp64=True, n_packets=1 << 14)
    _say(f"tail FP64 parity kind={kind} limit={limit}")
    g, cg = run(ctx, sc, kind, sc.n_packets, 2, limit, seed=12345)
    o, co, _ = O.run(sc, kind, count=sc.n_packets, seed=12345, nthreads=8)
    assert_fp64_parity(g / sc.n_packets, o, f"kind {kind}")
    assert_counters_close(cg, co, f"kind {kind}")


def test_tail_sphere_star_and_off_cases(ctx, Q):
    """A sphere star (direct order, occlusion) with the late-order launch from
    order 3 equals the per-order launches; a first order above max_orders
    leaves the run as it was; first orders 1 and -1 are refused."""
    sc = scenes.clumpy256(n=64).replace(max_orders=6, npix=64)
    n = 1 << 16
    _say("tail: sphere star")
    ref, cref = run(ctx, sc, Q.SOBOL, n, 0)
    img, cnt = run(ctx, sc, Q.SOBOL, n, 3)
    assert cnt == cref
    assert_sum_order_equal(img, ref, "sphere star tail 3")
    img, cnt = run(ctx, sc, Q.SOBOL, n, 7)   # beyond max_orders 6: per-order launches only
    assert cnt == cref
    assert_sum_order_equal(img, ref, "sphere star tail 7")
    for bad in (1, -1):
        with pytest.raises(Q.QRTError):
            ctx.set_tail(bad)


def test_batch_tail_equals_per_order_launches(ctx, Q):
    """Twelve uneven scenes (1 to 12 orders, 1 to 4 observers, envelopes and
    disks, point sources and stars) in one batch, FP32: the late-order launch
    from order 2 and from order 5, and from order 2 with at most 128 deferred
    scatterings, against every order launched on its own; per scene images up to the
    order of the sums, counters equal."""
    bs = scenes.uneven_batch(31, 12, sizes=(32, 64, 16), log2_packets=(14.0, 16.0), npix=64, orders=(1, 12))
    assert max(sc.max_orders for sc in bs) >= 5

    def batch(tail, limit=0):
        ctx.set_tail(tail, limit)
        ctx.batch_set(bs)
        ctx.batch_reset()
        ctx.batch_run(Q.SOBOL, 0, Q.FP32)
        return [ctx.batch_read_images(i, normalized=False) for i in range(len(bs))], ctx.counters()
    _say("batch tail: per-order reference")
    ref, cref = batch(0)
    for tail, limit in ((2, 0), (5, 0), (2, 128)):
        _say(f"batch tail from {tail}, deferred limit {limit}")
        img, cnt = batch(tail, limit)
        assert cnt == cref, f"tail {tail} limit {limit}"
        for i in range(len(bs)):
            assert_sum_order_equal(img[i], ref[i], f"scene {i} tail {tail} limit {limit}")


def test_tail_ragged_runs_fp64_parity(ctx, Q):
    """Runs of 1, 257 and 1000 packets (the deferred list and its sort nearly
    empty, a ragged last block) with the late-order launch from order 2,
    FP64, disk at 32^3, 20 orders, against the oracle."""
    sc = scenes.disk128(n=32).replace(npix=64, fp64=True)
    for first, count in ((1, 1), (2, 257), (7777, 1000)):
        _say(f"tail ragged run first={first} count={count}")
        ctx.set_scene(sc, kind=Q.HALTON, precision=None)
        ctx.set_tail(2)
        ctx.reset_images()
        ctx.run(first, count)
        g, cg = ctx.read_images(normalized=False), ctx.counters()
        o, co, _ = O.run(sc, O.HALTON, first=first, count=count, nthreads=8)
        if o[0, 0].max() > 0:
            assert_fp64_parity(g / count, o, f"first {first} count {count}")
        else:
            assert np.all(g == 0)
        assert_counters_close(cg, co, f"first {first} count {count}")


def test_tail_across_chunks(ctx, Q):
    """One run of 2^22 + 12345 packets, which the library splits into two
    chunks (each with its own late-order launch and deferred sort), against
    the same packets in two runs split elsewhere: disk at 32^3, 20 orders,
    FP32; images up to the order of the sums, counters equal."""
    sc = scenes.disk128(n=32).replace(npix=64)
    n = (1 << 22) + 12345
    _say("tail across chunks: one run")
    one, c1 = run(ctx, sc, Q.SOBOL, n, 2)
    _say("tail across chunks: two runs")
    ctx.set_scene(sc, kind=Q.SOBOL)
    ctx.set_tail(2)
    ctx.reset_images()
    ctx.run(1, 3000001)
    ctx.run(3000002, n - 3000001)
    two, c2 = ctx.read_images(normalized=False), ctx.counters()
    assert c1 == c2
    assert_sum_order_equal(two, one, "chunks")

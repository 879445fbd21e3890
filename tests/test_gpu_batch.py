"""Batches of uneven scenes on the GPU (qrt_batch_*), against the oracle and
against single-scene runs.

Gates:
  * FP64 batch, every scene against an oracle run of that scene alone (same
    point set, indices and seed): the per-pixel FP64 gate of the single-scene
    parity tests; event counters summed over the scenes.
  * FP32 batch against single-scene GPU runs of the same scenes: every packet
    takes the same FP32 steps in both, so images differ only by the order of
    the FP64 image sums (|d| <= 1e-10 (I + 1e-12 max I) per pixel) and the
    event counters are equal.
  * the full-size workload of 64 scenes (grids 32^3 to 192^3, up to 20
    orders): FP64 with 2^10 packets per scene against the oracle, and FP32 at
    the full packet counts against single-scene runs.
  * the workload of 256 small scenes (grids 32^3 to 96^3, 2^10 to 2^14
    packets, so that a chunk spans many scenes and the sort keys spend eight
    bits on the scene): FP32 against single-scene runs, FP64 of every eighth
    scene against the oracle.
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


def small_batch(seed=11, n_scenes=7):
    """Uneven scenes the oracle runs in seconds: grids 8^3 .. 24^3, 2^8 .. 2^11
    packets, 1 .. 6 orders, 16^2 images."""
    return [sc.replace(fp64=True) for sc in
            scenes.uneven_batch(seed, n_scenes, sizes=(8, 24, 8), log2_packets=(8.0, 11.0), npix=16, orders=(1, 6))]


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
            d = np.abs(g[ob, s] - o[ob, s])
            assert np.all(d <= 1e-5 * Io + 1e-11 * mx), f"{what} obs {ob} stokes {s}"
        assert np.all(Ig[Io == 0] == 0), what


def assert_sum_order_equal(b, s, what):
    """Per pixel |d| <= 1e-10 (I + 1e-12 max I): both runs compute every
    packet with the same FP32 steps (the library fuses multiply-adds only where
    the source asks), so only the order of the FP64 image sums differs."""
    mx = s[:, 0].max()
    for ob in range(s.shape[0]):
        scale = s[ob, 0] + 1e-12 * mx
        for k in range(3):
            d = np.abs(b[ob, k] - s[ob, k])
            assert np.all(d <= 1e-10 * scale), f"{what} obs {ob} stokes {k}: max {np.max(d / scale):.3e}"


def counters_close(cg, co):
    assert cg["packets"] == co["packets"]
    for k in ("visits", "peels", "peel_rays", "escapes", "tau_cuts", "scatterings", "occluded"):
        assert abs(cg[k] - co[k]) <= 4 * 8 + 1e-5 * co[k], f"{k}: gpu {cg[k]} oracle {co[k]}"


def sum_counters(cs):
    out = {}
    for c in cs:
        for k, v in c.items():
            out[k] = out.get(k, 0) + v
    return out


KINDS = [O.SOBOL, O.HALTON, O.NIEDERREITER2, O.HAMMERSLEY, O.PHILOX, O.SOBOL_OWEN]


@pytest.mark.parametrize("kind", KINDS)
def test_batch_fp64_matches_oracle_per_scene(ctx, Q, kind):
    bs = small_batch()
    seed = 977
    _say(f"batch fp64 kind={kind} scenes={len(bs)} packets={[s.n_packets for s in bs]}")
    ctx.batch_set(bs)
    ctx.batch_reset()
    ctx.batch_run(kind, seed, Q.FP64)
    cg = ctx.counters()
    cos = []
    for i, sc in enumerate(bs):
        g = ctx.batch_read_images(i)
        o, co, _ = O.run(sc, kind, 1, sc.n_packets, seed=seed, n_total=sc.n_packets)
        cos.append(co)
        assert_fp64_parity(g, o, f"scene {i}")
    counters_close(cg, sum_counters(cos))


def test_batch_index_ranges_and_empty_scene(ctx, Q):
    """first > 1, a scene with no packets, the same scene twice over
    consecutive index ranges (together they equal one run over both)."""
    bs = small_batch(seed=5, n_scenes=4)
    a = bs[0]
    n = a.n_packets
    scene_list = [a, bs[1], bs[2], a, bs[3]]
    firsts = [1, 1, 1, n + 1, 40]
    counts = [n, bs[1].n_packets, 0, n, bs[3].n_packets]
    _say(f"batch ranges counts={counts}")
    ctx.batch_set(scene_list, firsts=firsts, counts=counts, n_totals=[2 * n, 1, 1, 2 * n, bs[3].n_packets + 40])
    ctx.batch_reset()
    ctx.batch_run(Q.SOBOL, 0, Q.FP64)
    both = ctx.batch_read_images(0, normalized=False) + ctx.batch_read_images(3, normalized=False)
    o, _, _ = O.run(a, O.SOBOL, 1, 2 * n, normalize=False)
    assert_fp64_parity(both / (2 * n), o / (2 * n), "two ranges")
    assert np.all(ctx.batch_read_images(2, normalized=False) == 0)
    g = ctx.batch_read_images(4)
    o, _, _ = O.run(bs[3], O.SOBOL, 40, bs[3].n_packets)
    assert_fp64_parity(g, o, "first=40")


def test_batch_hammersley_uses_each_scenes_n(ctx, Q):
    bs = small_batch(seed=8, n_scenes=3)
    n_totals = [sc.n_packets + 17 * i for i, sc in enumerate(bs)]
    _say(f"batch hammersley n_totals={n_totals}")
    ctx.batch_set(bs, n_totals=n_totals)
    ctx.batch_reset()
    ctx.batch_run(Q.HAMMERSLEY, 0, Q.FP64)
    for i, sc in enumerate(bs):
        o, _, _ = O.run(sc, O.HAMMERSLEY, 1, sc.n_packets, n_total=n_totals[i])
        assert_fp64_parity(ctx.batch_read_images(i), o, f"scene {i}")


def single_runs(ctx, Q, scs, kind, seed, precision):
    out, cs = [], []
    for sc in scs:
        ctx.set_scene(sc, kind=kind, seed=seed, precision=precision)
        ctx.reset_images()
        ctx.run(1, sc.n_packets)
        out.append(ctx.read_images(normalized=False))
        cs.append(ctx.counters())
    return out, cs


@pytest.mark.parametrize("kind", [O.SOBOL, O.PHILOX])
def test_batch_fp32_equals_single_runs(ctx, Q, kind):
    bs = scenes.uneven_batch(21, 6, sizes=(32, 64, 16), log2_packets=(14.0, 17.0), npix=64, orders=(1, 12))
    _say(f"batch fp32 vs single kind={kind} packets={[s.n_packets for s in bs]}")
    single, cs = single_runs(ctx, Q, bs, kind, 31, Q.FP32)
    ctx.batch_set(bs)
    ctx.batch_reset()
    ctx.batch_run(kind, 31, Q.FP32)
    cb = ctx.counters()
    for i in range(len(bs)):
        assert_sum_order_equal(ctx.batch_read_images(i, normalized=False), single[i], f"scene {i}")
    assert cb == sum_counters(cs)


def test_batch_after_a_larger_single_scene_run(ctx, Q):
    """Queues grown by a larger single-scene run with one observer (packet
    lists for 2^22 packets, one peel slot each) and then a small batch with up
    to four observers per scene: the batch's peel regions are sized from the
    peel buffer it actually has, and every scene still equals its oracle run."""
    big = scenes.disk128(n_packets=1 << 22, n=32).replace(observers=[(0.4, 0.0)], max_orders=2, npix=16)
    _say("single-scene run of 2^22 packets, one observer")
    ctx.set_scene(big, precision=Q.FP32)
    ctx.run(1, 1 << 22)
    bs = small_batch(seed=12, n_scenes=5)
    _say(f"then a small fp64 batch, packets={[sc.n_packets for sc in bs]}")
    ctx.batch_set(bs)
    ctx.batch_reset()
    ctx.batch_run(Q.SOBOL, 0, Q.FP64)
    for i, sc in enumerate(bs):
        o, _, _ = O.run(sc, O.SOBOL, 1, sc.n_packets)
        assert_fp64_parity(ctx.batch_read_images(i), o, f"scene {i}")


def test_batch_runs_add_and_reset(ctx, Q):
    bs = small_batch(seed=3, n_scenes=3)
    ctx.batch_set(bs)
    ctx.batch_reset()
    ctx.batch_run(Q.SOBOL, 0, Q.FP64)
    one = [ctx.batch_read_images(i, normalized=False) for i in range(3)]
    ctx.batch_run(Q.SOBOL, 0, Q.FP64)
    for i in range(3):
        two = ctx.batch_read_images(i, normalized=False)
        assert np.allclose(two, 2 * one[i], rtol=1e-12, atol=1e-300)
        assert np.allclose(ctx.batch_read_images(i), one[i] / bs[i].n_packets, rtol=1e-12, atol=1e-300)
    ctx.batch_reset()
    for i in range(3):
        assert np.all(ctx.batch_read_images(i, normalized=False) == 0)
    assert ctx.counters()["packets"] == 0


def test_batch_refusals(ctx, Q):
    with pytest.raises(Q.QRTError):
        ctx.batch_run(Q.SOBOL, 0, Q.FP32)          # no batch set
    bs = small_batch(seed=3, n_scenes=2)
    ctx.batch_set(bs)
    with pytest.raises(Q.QRTError):
        ctx.batch_run(Q.FAURE, 0, Q.FP32)
    with pytest.raises(Q.QRTError):
        ctx.batch_run(Q.SOBOL, 0, 7)
    with pytest.raises(Q.QRTError):
        ctx.batch_read_images(2)
    bad = bs[0].replace(observers=[(0.1, 0.0)] * 4, source=(5.0, 0.0, 0.0))
    with pytest.raises(Q.QRTError):
        ctx.batch_set([bad])
    deep = bs[0].replace(max_orders=43)
    with pytest.raises(Q.QRTError):
        ctx.batch_set([deep])
    # Hammersley index beyond the scene's N
    ctx.batch_set(bs, n_totals=[bs[0].n_packets - 1, bs[1].n_packets])
    with pytest.raises(Q.QRTError):
        ctx.batch_run(Q.HAMMERSLEY, 0, Q.FP32)


# ------------------------------------------------------------------ the full-size workload
@pytest.fixture(scope="module")
def full_batch():
    return scenes.uneven_batch(2406, 64)


def test_full_batch_fp64_sampled_against_oracle(ctx, Q, full_batch):
    """All 64 full-size scenes (meshes, orders, observers, 128^2 images) in one
    FP64 batch with 2^10 packets each, every scene against the oracle."""
    n = 1 << 10
    _say("full batch fp64, 2^10 packets per scene")
    ctx.batch_set(full_batch, counts=[n] * len(full_batch))
    ctx.batch_reset()
    ctx.batch_run(Q.SOBOL, 0, Q.FP64)
    for i, sc in enumerate(full_batch):
        o, _, _ = O.run(sc, O.SOBOL, 1, n, nthreads=8)
        assert_fp64_parity(ctx.batch_read_images(i), o, f"scene {i} n={sc.n[0]} orders={sc.max_orders}")


@pytest.mark.parametrize("overlap", [False, True])
def test_full_batch_fp32_equals_single_runs(ctx, Q, full_batch, overlap):
    """The workload as timed (FP32, full packet counts, 2^23 to 2^31 batch
    numbers in chunks) against single-scene runs of every scene; with the
    overlap mode on, the batch's chunks go round the internal streams after
    the pending runs."""
    _say(f"full batch fp32 overlap={overlap}, {sum(s.n_packets for s in full_batch)} packets")
    single, cs = single_runs(ctx, Q, full_batch, Q.SOBOL, 0, Q.FP32)
    ctx.batch_set(full_batch)
    ctx.set_overlap(overlap)
    try:
        ctx.batch_reset()
        ctx.batch_run(Q.SOBOL, 0, Q.FP32)
        cb = ctx.counters()
    finally:
        ctx.set_overlap(False)
    for i in range(len(full_batch)):
        assert_sum_order_equal(ctx.batch_read_images(i, normalized=False), single[i], f"scene {i}")
    assert cb == sum_counters(cs)


# ------------------------------------------------------------------ many small scenes
@pytest.fixture(scope="module")
def small_scenes():
    return scenes.uneven_batch(2406, 256, sizes=(32, 96, 16), log2_packets=(10.0, 14.0))


def test_small_scenes_fp32_equals_single_runs(ctx, Q, small_scenes):
    """256 scenes in one chunk (the timed small-scene workload) against one
    single-scene run each."""
    _say(f"256 small scenes fp32, {sum(s.n_packets for s in small_scenes)} packets")
    single, cs = single_runs(ctx, Q, small_scenes, Q.SOBOL, 0, Q.FP32)
    ctx.batch_set(small_scenes)
    ctx.batch_reset()
    ctx.batch_run(Q.SOBOL, 0, Q.FP32)
    cb = ctx.counters()
    for i in range(len(small_scenes)):
        assert_sum_order_equal(ctx.batch_read_images(i, normalized=False), single[i], f"scene {i}")
    assert cb == sum_counters(cs)


def test_small_scenes_fp64_sampled_against_oracle(ctx, Q, small_scenes):
    """The same batch in FP64 with 2^9 packets per scene; every eighth scene
    against the oracle."""
    n = 1 << 9
    _say("256 small scenes fp64, 2^9 packets per scene")
    ctx.batch_set(small_scenes, counts=[n] * len(small_scenes))
    ctx.batch_reset()
    ctx.batch_run(Q.SOBOL, 0, Q.FP64)
    for i in range(0, len(small_scenes), 8):
        sc = small_scenes[i]
        o, _, _ = O.run(sc, O.SOBOL, 1, n, nthreads=8)
        assert_fp64_parity(ctx.batch_read_images(i), o, f"scene {i} n={sc.n[0]} orders={sc.max_orders}")

"""The allocation-free transport entry point (qrt_run_static) against qrt_run,
through the C ABI: two calls in a row on the device's static scratch, the
second with fewer packets than the first, each equal to qrt_run on the same
packets (FP64 transport: per pixel within 1e-12, far inside the 1e-5 parity
gate, since the two differ only in the order of the FP64 image sums; FP32
transport likewise, every packet taking the same arithmetic in both), with
equal event counts; and the size limit of the scratch."""
import sys

import numpy as np
import pytest

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


def _images(ctx, first, count, static):
    ctx.reset_images()
    if static:
        ctx.run_static(first, count)
    else:
        ctx.run(first, count)
    return ctx.read_images(normalized=False), ctx.counters()


def _assert_same(a, b):
    for ob in range(a.shape[0]):
        mx = np.abs(a[ob]).max()
        assert mx > 0
        assert np.all(np.abs(a[ob] - b[ob]) <= 1e-12 * np.abs(b[ob]) + 1e-15 * mx), f"obs {ob}"
        assert np.all(a[ob][b[ob] == 0] == 0)


@pytest.mark.parametrize("case", ["disk32_fp64", "disk128_fp32", "star_fp64"])
def test_static_run_equals_run(Q, case):
    if case == "disk32_fp64":
        sc = scenes.disk128(n_packets=1 << 12, n=32).replace(max_orders=5, npix=32, fp64=True)
        calls = [(1, 3 * (1 << 16) + 123), (77, 1000)]
    elif case == "disk128_fp32":
        sc = scenes.disk128()
        calls = [(1, (1 << 17) + 5), (1 << 20, 3000)]
    else:
        sc = scenes.clumpy256(n_packets=1 << 12, n=64).replace(fp64=True, npix=64)
        calls = [(1, (1 << 16) + 1), (9, 4097)]
    with Q.Context(0) as ref, Q.Context(0) as st:
        ref.set_scene(sc, kind=Q.SOBOL)
        st.set_scene(sc, kind=Q.SOBOL)
        for first, count in calls:
            _say(f"static run {case} first={first} count={count}")
            g, cg = _images(st, first, count, static=True)
            _say(f"reference run {case} first={first} count={count}")
            r, cr = _images(ref, first, count, static=False)
            _assert_same(g, r)
            assert cg == cr
            assert cg["packets"] == count


def test_static_run_limits(Q):
    from paper_2406_15632_amd.qrt import QRTError
    sc = scenes.envelope32(n_packets=1 << 10)
    with Q.Context(0) as ctx:
        ctx.set_scene(sc, kind=Q.SOBOL)
        _say("static run limits: 5 observers in FP64")
        ctx.set_observers([(0.3 * i, 0.1) for i in range(5)], sc.npix, sc.half_width)
        with pytest.raises(QRTError) as e:
            ctx.run_static(1, 100)
        assert e.value.code == Q.QRT_UNSUPPORTED
        ctx.set_transport(sc.max_orders, sc.tau_min, Q.FP32)
        ctx.set_observers([(0.3 * i, 0.1) for i in range(13)], sc.npix, sc.half_width)
        with pytest.raises(QRTError) as e:
            ctx.run_static(1, 100)
        assert e.value.code == Q.QRT_UNSUPPORTED
        # at the limits: 4 observers in FP64, 12 in FP32
        ctx.set_observers([(0.3 * i, 0.1) for i in range(12)], sc.npix, sc.half_width)
        ctx.run_static(1, 100)
        ctx.set_transport(sc.max_orders, sc.tau_min, Q.FP64)
        ctx.set_observers([(0.3 * i, 0.1) for i in range(4)], sc.npix, sc.half_width)
        ctx.run_static(1, 100)
        assert ctx.counters()["packets"] == 100
        # Faure tables are built by the allocating calls only
        ctx.set_sequence(Q.FAURE)
        with pytest.raises(QRTError) as e:
            ctx.run_static(1, 100)
        assert e.value.code == Q.QRT_BAD_STATE
        ctx.run(1, 10)
        ctx.run_static(11, 100)

"""Pins of the oracle's point sets (Sec. 3.1) against definitions outside the oracle:
scipy's unscrambled Sobol and Halton generators, exact rational radical inverses,
numpy's Philox4x64-10, and brute-force (t,m,s)-net counts."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from oracle import tables


def _scipy_sobol(dims, first, count):
    from scipy.stats import qmc
    eng = qmc.Sobol(dims, scramble=False, bits=32)
    eng.fast_forward(first)
    x = eng.random(count)
    return np.round(x * 2.0 ** 32).astype(np.uint64).astype(np.uint32)


@pytest.mark.parametrize("first,count", [(1, 4096), ((1 << 16) - 5, 16), ((1 << 20) - 3, 8)])
def test_sobol_matches_scipy(first, count):
    dims = 60
    ours = O.points(O.SOBOL, dims, first, count)
    ref = _scipy_sobol(dims, first, count)
    assert np.array_equal(ours, ref)


def test_sobol_high_columns_follow_scipy():
    # columns beyond the ones read from scipy come from the recurrence; check one
    # of them against scipy directly (point with Gray code 2^24 sits at index 2^25-1)
    V = tables.sobol_columns(60)
    ref = _scipy_sobol(60, (1 << 25) - 1, 1)[0]
    assert np.array_equal(V[:, 24], ref)


@pytest.mark.parametrize("kind", [O.SOBOL, O.NIEDERREITER2])
def test_generator_matrix_is_unit_upper_triangular(kind):
    # column b has its lowest set bit at 31-b: the 1-D projections are (0,m,1)-nets
    mat, _ = O.seq_tables(kind, 60)
    for d in range(60):
        for b in range(32):
            v = int(mat[d, b])
            assert (v >> (31 - b)) & 1 == 1
            assert v & ((1 << (31 - b)) - 1) == 0


def _net_counts_ok(pts, m, t, dims):
    """Every elementary box of volume 2^(t-m) holds exactly 2^t of the 2^m points."""
    s = len(dims)
    for comp in itertools.product(range(m - t + 1), repeat=s):
        if sum(comp) != m - t:
            continue
        key = np.zeros(len(pts), dtype=np.int64)
        for dd, di in zip(dims, comp):
            key = (key << di) | (pts[:, dd].astype(np.int64) >> (32 - di) if di else 0)
        counts = np.bincount(key, minlength=1 << (m - t))
        if not np.all(counts == (1 << t)):
            return False
    return True


def _first_pts(kind, dims, m, seed=0):
    # index 0 (the origin) plus indices 1 .. 2^m-1
    body = O.points(kind, dims, 1, (1 << m) - 1, seed=seed)
    origin = np.zeros((1, dims), dtype=np.uint32)
    return np.vstack([origin, body])


def _net_counts_one_short(pts, m, dims):
    """The 2^m - 1 points of indices 1 .. 2^m-1 of a (0,m,s)-net whose point of
    index 0 is left out: every elementary box of volume 2^-m holds one point,
    except exactly one box, which is empty."""
    s = len(dims)
    for comp in itertools.product(range(m + 1), repeat=s):
        if sum(comp) != m:
            continue
        key = np.zeros(len(pts), dtype=np.int64)
        for dd, di in zip(dims, comp):
            key = (key << di) | (pts[:, dd].astype(np.int64) >> (32 - di) if di else 0)
        counts = np.bincount(key, minlength=1 << m)
        if not (np.count_nonzero(counts == 1) == (1 << m) - 1 and np.count_nonzero(counts == 0) == 1):
            return False
    return True


@pytest.mark.parametrize("m", [4, 8, 12, 16])
def test_sobol_nets(m):
    pts = _first_pts(O.SOBOL, 8, m)
    for d in range(8):
        assert _net_counts_ok(pts, m, 0, [d])
    assert _net_counts_ok(pts, m, 0, [0, 1])


@pytest.mark.parametrize("m", [6, 9, 12])
def test_niederreiter_nets(m):
    polys = tables.irreducible_polys(4)
    degs = [p.bit_length() - 1 for p in polys]
    assert degs == [1, 1, 2, 3]
    pts = _first_pts(O.NIEDERREITER2, 4, m)
    for d in range(4):
        assert _net_counts_ok(pts, m, 0, [d])
    for s in range(2, 5):
        t = sum(e - 1 for e in degs[:s])
        assert _net_counts_ok(pts, m, t, list(range(s)))


def test_niederreiter_first_two_dims_equal_sobol():
    a = O.points(O.NIEDERREITER2, 2, 1, 5000)
    b = O.points(O.SOBOL, 2, 1, 5000)
    assert np.array_equal(a, b)


def test_niederreiter_planted_mistake_breaks_net():
    # a transposed matrix (a plausible bug) must fail the (t,m,s) check
    cols = tables.niederreiter_columns(4).copy()
    bits = np.array([[(int(cols[d, r]) >> (31 - j)) & 1 for r in range(32)] for d in range(4) for j in range(32)])
    bits = bits.reshape(4, 32, 32).transpose(0, 2, 1)
    bad = np.array([[sum(int(bits[d, j, r]) << (31 - j) for j in range(32)) for r in range(32)] for d in range(4)],
                   dtype=np.uint32)
    m = 10
    idx = np.arange(1 << m, dtype=np.uint64)
    gray = idx ^ (idx >> np.uint64(1))
    pts = np.zeros((1 << m, 4), dtype=np.uint32)
    for d in range(4):
        for r in range(m):
            sel = ((gray >> np.uint64(r)) & np.uint64(1)).astype(bool)
            pts[sel, d] ^= bad[d, r]
    assert not _net_counts_ok(pts, m, 3, [0, 1, 2, 3])


def _radical_inverse_exact(i, b):
    f, w = Fraction(0), Fraction(1, b)
    while i:
        f += (i % b) * w
        i //= b
        w /= b
    return f


@pytest.mark.parametrize("first", [1, 1000, (1 << 24) - 3, (1 << 32) - 6])
def test_halton_exact_rationals(first):
    dims = 60
    ours = O.points(O.HALTON, dims, first, 5)
    pr = tables.primes(dims)
    for j in range(5):
        for d in range(dims):
            ref = int(_radical_inverse_exact(first + j, int(pr[d])) * (1 << 32))
            assert int(ours[j, d]) == ref


def test_halton_close_to_scipy():
    from scipy.stats import qmc
    dims = 20
    x = qmc.Halton(dims, scramble=False).random(2001)[1:]
    ours = O.points(O.HALTON, dims, 1, 2000).astype(np.float64) / 2.0 ** 32
    assert np.max(np.abs(ours - x)) <= 2.0 ** -32 + 1e-15


def test_hammersley_definition():
    N = 3000
    pts = O.points(O.HAMMERSLEY, 4, 1, N, n_total=N)
    i = np.arange(1, N + 1, dtype=np.uint64)
    dim0 = ((i << np.uint64(32)) // np.uint64(N)) & np.uint64(0xFFFFFFFF)
    assert np.array_equal(pts[:, 0].astype(np.uint64), dim0)
    # i/N exactly for a power-of-two N
    N2 = 1 << 12
    p2 = O.points(O.HAMMERSLEY, 2, 1, N2, n_total=N2)
    assert np.array_equal(p2[:-1, 0].astype(np.uint64), np.arange(1, N2, dtype=np.uint64) << np.uint64(20))
    assert p2[-1, 0] == 0
    hal = O.points(O.HALTON, 3, 1, N)
    assert np.array_equal(pts[:, 1:], hal)


@pytest.mark.parametrize("seed", [0, 12345, 2 ** 63 + 7])
def test_philox_matches_numpy(seed):
    dims = 20
    first = 7
    ours = O.points(O.PHILOX, dims, first, 6, seed=seed)
    for j in range(6):
        i = first + j
        for blk in range((dims + 7) // 8):
            ctr = i | (blk << 64)
            words = np.random.Philox(key=seed, counter=ctr - 1).random_raw(4)
            w32 = []
            for w in words:
                w32 += [int(w) & 0xFFFFFFFF, int(w) >> 32]
            for d in range(blk * 8, min(dims, blk * 8 + 8)):
                assert int(ours[j, d]) == w32[d & 7]


# ---------------------------------------------------------------- Faure
def _faure_exact(i, d, b, m):
    """Faure coordinate from its definition with exact integers and fractions:
    digits of i, Pascal-matrix power P^d modulo b, radical inverse."""
    import math
    from fractions import Fraction
    a = []
    n = i
    for _ in range(m):
        a.append(n % b)
        n //= b
    x = Fraction(0)
    for r in range(m):
        y = sum(math.comb(k, r) * d ** (k - r) * a[k] for k in range(r, m)) % b
        x += Fraction(y, b ** (r + 1))
    return math.floor(x * 2 ** 32)


def test_faure_matches_its_definition():
    from oracle import tables
    for dims in (3, 7, 60):
        b, m, _ = tables.faure_matrices(dims)
        assert b == {3: 3, 7: 7, 60: 61}[dims]
        idx = [1, 2, b - 1, b, b * b + 3, 12345, 2 ** 31 + 7, 2 ** 32 - 1]
        pts = np.concatenate([O.points(O.FAURE, dims, i, 1) for i in idx])
        for row, i in zip(pts, idx):
            for d in (0, 1, dims // 2, dims - 1):
                assert int(row[d]) == _faure_exact(i, d, b, m), (dims, i, d)


def test_faure_first_coordinate_is_van_der_corput():
    from fractions import Fraction
    b = 5
    pts = O.points(O.FAURE, 5, 1, 400)
    for i in range(1, 401):
        x, n, f = Fraction(0), i, Fraction(1, b)
        while n:
            x += (n % b) * f
            n //= b
            f /= b
        assert int(pts[i - 1, 0]) == int(x * 2 ** 32)


def _is_net_base(pts01, b, m):
    """Every elementary interval of volume b^-m (exponents summing to m) holds
    exactly one of the b^m points."""
    s = pts01.shape[1]
    import itertools
    for ks in itertools.product(range(m + 1), repeat=s):
        if sum(ks) != m:
            continue
        cells = np.zeros(len(pts01), dtype=np.int64)
        for j, k in enumerate(ks):
            cells = cells * (b ** k) + np.floor(pts01[:, j] * b ** k).astype(np.int64)
        if len(np.unique(cells)) != len(pts01):
            return False
    return True


@pytest.mark.parametrize("b,s,m", [(5, 5, 3), (5, 4, 2), (7, 7, 2), (3, 3, 4)])
def test_faure_points_form_zero_nets(b, s, m):
    """The first b^m points (index 0, the all-zero point, included) of the
    s-dimensional Faure sequence, whose base b is the smallest prime >= s, form
    a (0, m, s)-net in base b."""
    from oracle import tables
    assert tables.faure_base(s) == b
    pts = O.points(O.FAURE, s, 1, b ** m - 1).astype(np.float64) / 2 ** 32
    pts = np.vstack([np.zeros((1, s)), pts])
    # x is stored as floor(x 2^32): move it back up by one unit before binning
    assert _is_net_base(pts + 2.0 ** -32, b, m)


def test_faure_planted_mistake_breaks_net():
    """Using the transposed Pascal matrices (a plausible slip) destroys the net."""
    from oracle import tables
    b, m, C = tables.faure_matrices(5)
    Ct = np.ascontiguousarray(np.transpose(C, (0, 2, 1)))
    out = np.zeros((124, 5), dtype=np.uint32)
    lib = O.lib()
    bases = np.array([b, m], dtype=np.uint32)
    lib.oracle_points(O.FAURE, 5, Ct.ctypes.data, bases.ctypes.data, 0, 0, 1, 124, out.ctypes.data)
    pts = np.vstack([np.zeros((1, 5)), out.astype(np.float64) / 2 ** 32])
    assert not _is_net_base(pts + 2.0 ** -32, 5, 3)


# ---------------------------------------------------------------- Owen scrambling
def _splitmix64(z):
    """splitmix64 output function (Steele, Lea and Flood 2014), 64-bit wrap-around."""
    M = (1 << 64) - 1
    z = (z + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_splitmix64_known_values():
    # published first outputs of the splitmix64 generator from state 0 (state
    # advanced by the increment before mixing): 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4
    assert _splitmix64(0) == 0xE220A8397B1DCDAF
    assert _splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


@pytest.mark.parametrize("m", [6, 10])
def test_owen_scrambling_keeps_sobol_nets(m):
    """Owen's scrambling permutes every elementary interval as a whole, so the
    first 2^m scrambled Sobol points are still (0,m,1)-nets per dimension and a
    (0,m,2)-net in dims 0-1.  Index 0 is not generated (Sec. 3.7), so the
    points of indices 1 .. 2^m-1 fill every elementary box but one."""
    for seed in (1, 99):
        pts = O.points(O.SOBOL_OWEN, 4, 1, (1 << m) - 1, seed=seed)
        for d in range(4):
            assert _net_counts_one_short(pts, m, [d])
        assert _net_counts_one_short(pts, m, [0, 1])


def _divergence_pairs(raw, d, depths):
    """Pairs (i, j) of points whose coordinate d agrees in its top t bits and
    differs in bit t (depth t, counted from the most significant bit), for each t
    in depths: the first such pair found in the list."""
    x = raw[:, d].astype(np.uint64)
    pairs = {}
    for t in depths:
        top = x >> np.uint64(31 - t)          # the top t+1 bits
        seen = {}
        for i, v in enumerate(top.tolist()):
            mate = seen.get(v ^ 1)            # same top t bits, other bit t
            if mate is not None:
                pairs[t] = (mate, i)
                break
            seen.setdefault(v, i)
    return pairs


def test_owen_scrambling_is_nested():
    """The defining property of nested uniform scrambling (Owen 1995), checked on
    the scrambled points alone.  Two coordinates that first differ at depth t keep
    their common top t bits after scrambling and still differ at depth t (the flips
    of those bits depend only on the common prefix); the flips of their lower bits
    depend on the bit where they part, so the XOR of their scrambled lower bits
    changes with the seed, and it is uniformly distributed.  A plain random digital
    shift (flips independent of the prefix) keeps that XOR equal to the XOR of the
    unscrambled bits for every seed, and fails here."""
    n = 1 << 12
    raw = O.points(O.SOBOL, 4, 1, n)
    seeds = list(range(1, 25))
    scr = [O.points(O.SOBOL_OWEN, 4, 1, n, seed=s) for s in seeds]
    depths = list(range(0, 12))
    low_bits_same = 0
    trials = 0
    bit_below = []
    for d in range(4):
        for t, (i, j) in _divergence_pairs(raw, d, depths).items():
            hi_mask = ((1 << t) - 1) << (32 - t) if t else 0
            bit_t = 1 << (31 - t)
            low_mask = bit_t - 1
            xr = int(raw[i, d]) ^ int(raw[j, d])
            assert xr & hi_mask == 0 and xr & bit_t
            lows = set()
            for sp in scr:
                a, b = int(sp[i, d]), int(sp[j, d])
                assert (a ^ b) & hi_mask == 0, (d, t)      # common prefix kept
                assert (a ^ b) & bit_t, (d, t)             # still part at depth t
                lows.add((a ^ b) & low_mask)
                low_bits_same += ((a ^ b) & low_mask) == (xr & low_mask)
                trials += 1
                bit_below.append(((a ^ b) >> (30 - t)) & 1)
            assert len(lows) > len(seeds) // 2, (d, t)     # the lower flips follow the parting bit
    # for a nested scrambling the scrambled lower bits of a pair match the raw ones
    # with probability 2^-(31-t) <= 2^-20 per seed; a digital shift matches always
    assert low_bits_same == 0
    # the first bit below the parting one is a fair coin over pairs and seeds
    frac = float(np.mean(bit_below))
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(len(bit_below)), frac


def test_owen_scrambling_top_flip_is_shared():
    """The flip of the top bit has no prefix to depend on: for one seed and
    dimension it is the same for every point, so the scrambled top bit is the raw
    top bit XOR a constant; over seeds that constant is a fair coin."""
    raw = O.points(O.SOBOL, 3, 1, 512)
    flips = []
    for seed in range(1, 41):
        scr = O.points(O.SOBOL_OWEN, 3, 1, 512, seed=seed)
        for d in range(3):
            f = (scr[:, d] >> 31) ^ (raw[:, d] >> 31)
            assert np.all(f == f[0])
            flips.append(int(f[0]))
    assert 0.25 < np.mean(flips) < 0.75
    # different seeds give different points
    assert not np.array_equal(O.points(O.SOBOL_OWEN, 3, 1, 64, seed=1), O.points(O.SOBOL_OWEN, 3, 1, 64, seed=2))

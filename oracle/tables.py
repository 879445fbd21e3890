"""Oracle-side generator tables (test infrastructure only).

Nothing here is imported by the GPU library; it builds its own tables from the
same public definitions.

* Sobol (paper Sec. 3.1, after Bratley & Fox 1988 and Joe & Kuo 2008): the
  direction numbers are read from scipy's public unscrambled Sobol generator.
  In Gray-code order the point with index 2^(b+1)-1 has Gray code 2^b, so it
  equals direction number b of every dimension.
* Niederreiter base 2 (Sec. 3.1, Niederreiter 1988 as implemented by
  Bratley, Fox & Niederreiter 1992): for the irreducible polynomial p of
  degree e attached to a dimension, output digit j (j>=1, weight 2^-j) is the
  GF(2) dot product of the index digits with row j of C, where
  C[j][r] is the coefficient of x^(-r-1) in the Laurent expansion of
  x^(e-u-1) / p(x)^(Q+1), with j-1 = Q*e + u, 0 <= u < e.
  Polynomials are taken in increasing degree and, within a degree, in
  increasing integer value of their coefficient bits, starting with p(x)=x.
* Halton / Hammersley: the first primes as bases.
"""
from __future__ import annotations

import functools
from typing import List

import math

import numpy as np


SOBOL_READ_BITS = 22   # columns read from scipy; the rest follow from the Sobol recurrence


def _sobol_recurrence_fit(v: List[int]):
    """Find (s, a) such that, for b >= s,
    v[b] = XOR_{i=1..s-1} a_i v[b-i]  ^  v[b-s]  ^  (v[b-s] >> s)
    (Bratley & Fox 1988), a_i being bit (s-1-i) of a.  Returns None if no fit."""
    n = len(v)
    for s in range(1, 13):
        if n - s < 6:
            break
        for a in range(1 << (s - 1)):
            ok = True
            for b in range(s, n):
                x = v[b - s] ^ (v[b - s] >> s)
                for i in range(1, s):
                    if (a >> (s - 1 - i)) & 1:
                        x ^= v[b - i]
                if x != v[b]:
                    ok = False
                    break
            if ok:
                return s, a
    return None


@functools.lru_cache(maxsize=None)
def sobol_columns(dims: int) -> np.ndarray:
    """uint32 [dims][32]: column b of dimension d (the value of bit b of the Gray code).

    Columns 0..SOBOL_READ_BITS-1 are read from scipy's public generator (the point
    at index 2^(b+1)-1); higher columns continue each dimension's direction-number
    recurrence, whose primitive polynomial is solved from the columns read.  The
    first dimension is the identity matrix (van der Corput)."""
    from scipy.stats import qmc
    nb = SOBOL_READ_BITS
    V = np.zeros((dims, 32), dtype=np.uint64)
    for b in range(nb):
        eng = qmc.Sobol(dims, scramble=False, bits=32)
        eng.fast_forward((1 << (b + 1)) - 1)
        pt = eng.random(1)[0]
        V[:, b] = [int(round(x * 2.0 ** 32)) for x in pt]
    for d in range(dims):
        known = [int(x) for x in V[d, :nb]]
        if all(known[b] == 1 << (31 - b) for b in range(nb)):
            full = [1 << (31 - b) for b in range(32)]
        else:
            fit = _sobol_recurrence_fit(known)
            if fit is None:
                raise RuntimeError(f"no Sobol recurrence fits dimension {d}")
            s, a = fit
            full = list(known)
            for b in range(nb, 32):
                x = full[b - s] ^ (full[b - s] >> s)
                for i in range(1, s):
                    if (a >> (s - 1 - i)) & 1:
                        x ^= full[b - i]
                full.append(x)
        V[d] = full
    return V.astype(np.uint32)


def _gf2_mul(a: int, b: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        b >>= 1
    return r


def _gf2_mod(a: int, m: int) -> int:
    dm = m.bit_length() - 1
    while a and a.bit_length() - 1 >= dm:
        a ^= m << (a.bit_length() - 1 - dm)
    return a


def _is_irreducible(p: int) -> bool:
    deg = p.bit_length() - 1
    if deg < 1:
        return False
    for q in range(2, 1 << (deg // 2 + 1)):
        if q.bit_length() - 1 > deg // 2:
            break
        if _gf2_mod(p, q) == 0:
            return False
    return True


@functools.lru_cache(maxsize=None)
def irreducible_polys(count: int) -> List[int]:
    out: List[int] = []
    deg = 1
    while len(out) < count:
        for p in range(1 << deg, 1 << (deg + 1)):
            if _is_irreducible(p):
                out.append(p)
                if len(out) == count:
                    break
        deg += 1
    return out


def _laurent_inverse_series(P: int, nterms: int) -> List[int]:
    """Coefficients b_k of 1/P(x) = x^-D * sum_k b_k x^-k for monic P of degree D over GF(2)."""
    D = P.bit_length() - 1
    rev = [(P >> (D - i)) & 1 for i in range(D + 1)]   # rev[i] = coefficient of x^(D-i)
    b = [0] * nterms
    b[0] = 1
    for kk in range(1, nterms):
        s = 0
        for i in range(1, min(kk, D) + 1):
            s ^= rev[i] & b[kk - i]
        b[kk] = s
    return b


def niederreiter_matrix(p: int, nbits: int = 32) -> np.ndarray:
    """0/1 matrix C[j-1][r] (j = 1..nbits output digit, r = 0..nbits-1 input digit)."""
    e = p.bit_length() - 1
    C = np.zeros((nbits, nbits), dtype=np.uint8)
    for j in range(1, nbits + 1):
        Q, u = divmod(j - 1, e)
        P = 1
        for _ in range(Q + 1):
            P = _gf2_mul(P, p)
        D = P.bit_length() - 1
        b = _laurent_inverse_series(P, nbits + e + D + 1)
        # x^(e-u-1)/P = sum_k b_k x^(e-u-1-D-k); the x^(-r-1) term has k = r + e - u - D
        for r in range(nbits):
            kk = r + e - u - D
            if kk >= 0:
                C[j - 1, r] = b[kk]
    return C


@functools.lru_cache(maxsize=None)
def niederreiter_columns(dims: int) -> np.ndarray:
    """uint32 [dims][32]: column r packed with digit j at bit 32-j."""
    out = np.zeros((dims, 32), dtype=np.uint32)
    for d, p in enumerate(irreducible_polys(dims)):
        C = niederreiter_matrix(p)
        for r in range(32):
            v = 0
            for j in range(1, 33):
                if C[j - 1, r]:
                    v |= 1 << (32 - j)
            out[d, r] = v
    return out


@functools.lru_cache(maxsize=None)
def primes(count: int) -> np.ndarray:
    out: List[int] = []
    c = 2
    while len(out) < count:
        if all(c % q for q in out if q * q <= c):
            out.append(c)
        c += 1
    return np.array(out, dtype=np.uint32)


# ----------------------------------------------------------------------------
# Faure (1982): digital sequence in the prime base b >= s; coordinate d of
# point i applies the d-th power of the Pascal matrix modulo b to the base-b
# digits of i, then takes the radical inverse of the resulting digits.

def faure_base(dims: int) -> int:
    """Smallest prime >= dims (at least 2)."""
    b = max(2, dims)
    while any(b % q == 0 for q in range(2, int(b ** 0.5) + 1)):
        b += 1
    return b


def faure_digits(b: int) -> int:
    """Base-b digits that every index below 2^32 needs: smallest m with b^m >= 2^32."""
    m, p = 0, 1
    while p < (1 << 32):
        p *= b
        m += 1
    return m


def faure_matrices(dims: int):
    """(b, m, C[dims][m][m]) with C_d[r][k] = binom(k, r) d^(k-r) mod b for k >= r
    (the d-th power of the upper-triangular Pascal matrix; d = 0 is the identity)."""
    b = faure_base(dims)
    m = faure_digits(b)
    C = np.zeros((dims, m, m), dtype=np.uint32)
    for d in range(dims):
        for r in range(m):
            for k in range(r, m):
                C[d, r, k] = (math.comb(k, r) * pow(d, k - r, b)) % b
    return b, m, C

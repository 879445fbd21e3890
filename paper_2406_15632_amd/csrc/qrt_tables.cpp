// Generator tables of the point sets (Sec. 3.1 of Shulman, "Quasi-Monte Carlo
// Radiative Transfer"), built on the host and uploaded once per context.
//
//  * Sobol: direction numbers of Bratley & Fox / Joe & Kuo, written into
//    qrt_sobol_table.h at build time from scipy's public unscrambled Sobol
//    generator (see gen_sobol_table.py).
//  * Niederreiter base 2 (Niederreiter 1988, as implemented by Bratley, Fox &
//    Niederreiter 1992): dimension d uses the d-th irreducible polynomial p over
//    GF(2) (increasing degree, then increasing coefficient bits; p = x first).
//    With e = deg p and output digit j >= 1 written as j-1 = Q e + u, row j of
//    the generator matrix holds the coefficients of x^(-r-1), r = 0, 1, ..., in
//    the Laurent expansion of x^(e-u-1) / p(x)^(Q+1).  Writing
//    1/p^(Q+1) = x^-D sum_k b_k x^-k (D = e (Q+1)), that coefficient is
//    b_(r-j+1) (zero for r < j-1): the matrix is unit upper triangular.
//  * Halton / Hammersley bases: the first primes.
#include <stdint.h>
#include <string.h>

#include "qrt_sobol_table.h"   // generated: QRT_SOBOL_DIMS, qrt_sobol_v[QRT_SOBOL_DIMS][32]

namespace qrt {

static int gf2_degree(uint64_t p)
{
    int d = -1;
    while (p) { ++d; p >>= 1; }
    return d;
}

static uint64_t gf2_mulmod_free(uint64_t a, uint64_t b)
{
    uint64_t r = 0;
    while (b) {
        if (b & 1) r ^= a;
        a <<= 1;
        b >>= 1;
    }
    return r;
}

static uint64_t gf2_rem(uint64_t a, uint64_t m)
{
    int dm = gf2_degree(m);
    for (int da = gf2_degree(a); da >= dm && a; da = gf2_degree(a)) a ^= m << (da - dm);
    return a;
}

static bool gf2_irreducible(uint64_t p)
{
    int d = gf2_degree(p);
    if (d < 1) return false;
    for (uint64_t q = 2; gf2_degree(q) <= d / 2; ++q)
        if (gf2_rem(p, q) == 0) return false;
    return true;
}

void niederreiter2_columns(int dims, uint32_t *out /* [dims][32] */)
{
    int found = 0;
    for (uint64_t p = 2; found < dims; ++p) {
        if (!gf2_irreducible(p)) continue;
        const int e = gf2_degree(p);
        uint32_t col[32];
        memset(col, 0, sizeof(col));
        for (int j = 1; j <= 32; ++j) {
            const int Q = (j - 1) / e;
            uint64_t P = 1;
            for (int t = 0; t <= Q; ++t) P = gf2_mulmod_free(P, p);
            const int D = gf2_degree(P);
            // b_0 = 1, b_k = sum_{i=1..min(k,D)} [coef of x^(D-i) in P] b_(k-i)
            uint8_t b[64];
            b[0] = 1;
            for (int kk = 1; kk < 64; ++kk) {
                uint8_t s = 0;
                for (int i = 1; i <= kk && i <= D; ++i) s ^= (uint8_t)(((P >> (D - i)) & 1u) & b[kk - i]);
                b[kk] = s;
            }
            for (int r = j - 1; r < 32; ++r)
                if (b[r - j + 1]) col[r] |= 1u << (32 - j);
        }
        memcpy(out + 32 * found, col, sizeof(col));
        ++found;
    }
}

void first_primes(int count, uint32_t *out)
{
    int n = 0;
    for (uint32_t c = 2; n < count; ++c) {
        bool prime = true;
        for (int i = 0; i < n && out[i] * out[i] <= c; ++i)
            if (c % out[i] == 0) { prime = false; break; }
        if (prime) out[n++] = c;
    }
}

int sobol_table_dims() { return QRT_SOBOL_DIMS; }

void sobol_columns(int dims, uint32_t *out)
{
    for (int d = 0; d < dims && d < QRT_SOBOL_DIMS; ++d)
        for (int b = 0; b < 32; ++b) out[32 * d + b] = qrt_sobol_v[d][b];
}

}  // namespace qrt

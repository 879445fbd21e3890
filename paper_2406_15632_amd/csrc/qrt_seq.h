// Device-side point sets (Sec. 3.1 of Shulman, "Quasi-Monte Carlo Radiative Transfer").
//
// Every lane computes coordinate d of point i directly from the index, so there
// is no generator state to share between lanes (the paper notes that threads
// cannot simply use independent seeds of a QMC generator; computing points by
// index removes that problem).  Values are unsigned 0.32 fixed point.
//
//  - Sobol and Niederreiter base 2: digital sequences in Gray-code order,
//    x = XOR of the generator-matrix columns picked by the set bits of i^(i>>1).
//  - Halton: floor(phi_b(i) * 2^32) for the radical inverse phi_b in base b,
//    exact: base 2 is a bit reversal; other bases form A/b^K from the reversed
//    digits and take the floor of A*2^32/b^K with a double quotient corrected
//    by an exact integer remainder.
//  - Hammersley: first coordinate i/N (mod 1, in 0.32 fixed point), the others
//    Halton in the first primes.
//  - Philox4x64-10 (Salmon et al., SC'11) for the Monte Carlo baseline:
//    counter (i, d/8, 0, 0), key (seed, 0), 32-bit word d%8, low half first.
//  - Sobol with Owen's nested uniform scrambling (randomised QMC): from the most
//    significant bit down, bit j of a coordinate is flipped by the top bit of
//    splitmix64 (Steele, Lea and Flood 2014) of a key made from the seed, the
//    dimension, the depth and the original bits above j.
//  - Faure (1982): base b = the smallest prime >= the number of coordinates;
//    coordinate d takes the base-b digits a of i, y = P^d a (mod b) with the
//    Pascal matrix power P^d[r][k] = binom(k, r) d^(k-r), and returns
//    floor(0.y_0 y_1 ... (base b) * 2^32), exact as for Halton.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrt {

enum SeqKind {
    SEQ_SOBOL = 0, SEQ_HALTON = 1, SEQ_NIED2 = 2, SEQ_HAMMERSLEY = 3, SEQ_PHILOX = 4, SEQ_FAURE = 5, SEQ_SOBOL_OWEN = 6
};

struct SeqParams {
    const uint32_t *mat;    // generator-matrix byte tables [dims][4][256] (Sobol or Niederreiter): entry
                            // [d][q][v] is the XOR of the columns 8q .. 8q+7 of d that the bits of v select
    const uint32_t *bases;  // Halton bases [dims]
    uint64_t seed;
    uint64_t n_total;       // Hammersley N
    const uint32_t *faure;  // Faure: [dims][m][m] matrices P^d mod b, then b^0 .. b^(m-1) at faure + fpow
    uint32_t fb, fm, fpow;  // Faure base, digits per index (b^m >= 2^32), offset of the powers
    uint64_t fbm;           // b^m
};

// The XOR of the generator columns that the bits of the Gray-code index
// select, one index byte at a time: four independent lookups in the
// dimension's byte tables t[4][256].
__device__ __forceinline__ uint32_t digital_point(const uint32_t *__restrict__ t, uint64_t i)
{
    const uint32_t g = (uint32_t)(i ^ (i >> 1));   // indices are < 2^32 for the 32-bit digital sequences
    return t[g & 255u] ^ t[256 + ((g >> 8) & 255u)] ^ t[512 + ((g >> 16) & 255u)] ^ t[768 + (g >> 24)];
}

// floor(num * 2^32 / den) for num < den < 2^53: double quotient, exact integer fix-up
__device__ __forceinline__ uint32_t frac_to_u32(uint64_t num, uint64_t den)
{
    double q = floor(((double)num * 4294967296.0) / (double)den);
    uint64_t qi = (uint64_t)q;
    // remainder num*2^32 - qi*den, exact modulo 2^64 and small in magnitude
    int64_t r = (int64_t)((num << 32) - qi * den);
    if (r < 0) qi -= 1;
    else if ((uint64_t)r >= den) qi += 1;
    return (uint32_t)qi;
}

__device__ __forceinline__ uint32_t radical_inverse(uint64_t i, uint32_t b)
{
    if (b == 2u) return __builtin_bitreverse32((uint32_t)i);
    uint64_t A = 0, B = 1;
    uint32_t n = (uint32_t)i;
    const double inv_b = 1.0 / (double)b;
    while (n) {
        uint32_t q = (uint32_t)((double)n * inv_b);
        int32_t r = (int32_t)(n - q * b);
        if (r < 0) { q -= 1; r += (int32_t)b; }
        else if (r >= (int32_t)b) { q += 1; r -= (int32_t)b; }
        A = A * b + (uint32_t)r;
        B *= b;
        n = q;
    }
    return frac_to_u32(A, B);
}

__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
{
    lo = a * b;
    hi = __umul64hi(a, b);
}

__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t h0, l0, h1, l1;
        mulhilo64(M0, c0, h0, l0);
        mulhilo64(M1, c2, h1, l1);
        uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0; c1 = l1; c2 = n2; c3 = l0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ uint32_t philox_word(uint64_t seed, uint64_t i, int d)
{
    uint64_t o[4];
    philox4x64_10(i, (uint64_t)(d >> 3), 0, 0, seed, 0, o);
    uint64_t w = o[(d & 7) >> 1];
    return (d & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
}

__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t owen_scramble(uint32_t x, uint64_t seed, int d)
{
    uint32_t out = x;
    for (int t = 0; t < 32; ++t) {
        const uint64_t prefix = t == 0 ? 0ull : (uint64_t)(x >> (32 - t));
        const uint64_t key = splitmix64_mix(seed ^ splitmix64_mix(((uint64_t)(uint32_t)d << 8) | (uint64_t)t)) ^ prefix;
        out ^= (uint32_t)(splitmix64_mix(key) >> 63) << (31 - t);
    }
    return out;
}

// Faure coordinate d of point i (< 2^32): digit k of i is (i / b^k) mod b,
// taken up to the highest nonzero one
__device__ __forceinline__ uint32_t faure_point(const SeqParams &S, uint64_t i, int d)
{
    const uint32_t b = S.fb, m = S.fm;
    const uint32_t *__restrict__ C = S.faure + (size_t)d * m * m;
    const uint32_t *__restrict__ pw = S.faure + S.fpow;
    const uint32_t n = (uint32_t)i;
    uint32_t top = 0;
    while (top + 1 < m && pw[top + 1] <= n) ++top;
    uint64_t Y = 0;
    for (uint32_t r = 0; r < m; ++r) {
        uint32_t y = 0;   // at most m (b-1)^2 < 2^20
        for (uint32_t k = r; k <= top; ++k) y += C[r * m + k] * ((n / pw[k]) % b);
        Y = Y * b + (y % b);
    }
    return frac_to_u32(Y, S.fbm);
}

template <int KIND>
__device__ __forceinline__ uint32_t seq_point(const SeqParams &S, uint64_t i, int d)
{
    if constexpr (KIND == SEQ_SOBOL || KIND == SEQ_NIED2) {
        return digital_point(S.mat + 1024 * d, i);
    } else if constexpr (KIND == SEQ_SOBOL_OWEN) {
        return owen_scramble(digital_point(S.mat + 1024 * d, i), S.seed, d);
    } else if constexpr (KIND == SEQ_HALTON) {
        return radical_inverse(i, S.bases[d]);
    } else if constexpr (KIND == SEQ_HAMMERSLEY) {
        if (d == 0) {
            // floor(i * 2^32 / N) modulo 2^32 (i = N maps to 0)
            double q = floor(((double)i * 4294967296.0) / (double)S.n_total);
            uint64_t qi = (uint64_t)q;
            int64_t r = (int64_t)((i << 32) - qi * S.n_total);
            if (r < 0) qi -= 1;
            else if ((uint64_t)r >= S.n_total) qi += 1;
            return (uint32_t)qi;
        }
        return radical_inverse(i, S.bases[d - 1]);
    } else if constexpr (KIND == SEQ_FAURE) {
        return faure_point(S, i, d);
    } else {
        return philox_word(S.seed, i, d);
    }
}

// Three consecutive coordinates d, d+1, d+2 (one flight); Philox shares its block.
template <int KIND>
__device__ __forceinline__ void seq_triple(const SeqParams &S, uint64_t i, int d, uint32_t x[3])
{
    if constexpr (KIND == SEQ_PHILOX) {
        uint64_t o[4];
        int blk = d >> 3;
        philox4x64_10(i, (uint64_t)blk, 0, 0, S.seed, 0, o);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            int dj = d + j;
            if ((dj >> 3) != blk) {
                blk = dj >> 3;
                philox4x64_10(i, (uint64_t)blk, 0, 0, S.seed, 0, o);
            }
            uint64_t w = o[(dj & 7) >> 1];
            x[j] = (dj & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) x[j] = seq_point<KIND>(S, i, d + j);
    }
}

// 0.32 fixed point to a uniform number in [0, 1): exact in both precisions.
template <typename R> __device__ __forceinline__ R to_unit(uint32_t x);
template <> __device__ __forceinline__ double to_unit<double>(uint32_t x) { return (double)x * 0x1p-32; }
template <> __device__ __forceinline__ float to_unit<float>(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

}  // namespace qrt

// Device-side scattering physics (Shulman, "Quasi-Monte Carlo Radiative
// Transfer", Sec. 2.2 and 3.5): Henyey-Greenstein sampling, White's Mueller
// matrix elements, Stokes reference-frame rotations.
//
// Stokes frames: a packet carries its direction k and a unit reference axis m
// perpendicular to k (n = k x m); Q > 0 means polarisation along m.  Rotating
// the reference axis by psi (m' = cos psi m + sin psi n) maps (Q, U) to
// (Q cos 2psi + U sin 2psi, -Q sin 2psi + U cos 2psi).
#pragma once

#include <hip/hip_runtime.h>

namespace qrt {

template <typename R> __device__ __forceinline__ void sincos_2pi(R u, R &s, R &c);
template <> __device__ __forceinline__ void sincos_2pi<float>(float u, float &s, float &c) { sincospif(2.0f * u, &s, &c); }
template <> __device__ __forceinline__ void sincos_2pi<double>(double u, double &s, double &c) { sincospi(2.0 * u, &s, &c); }

template <typename R> __device__ __forceinline__ R dot3(const R a[3], const R b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <typename R> __device__ __forceinline__ void cross3(const R a[3], const R b[3], R o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Henyey-Greenstein inverse CDF of cos(Theta); |g| < 1e-6 reads as isotropic
template <typename R>
__device__ __forceinline__ R hg_cos(R g, R v)
{
    R c;
    if (fabs(g) < (R)1e-6) {
        c = (R)2 * v - (R)1;
    } else {
        R f = ((R)1 - g * g) / ((R)1 - g + (R)2 * g * v);
        c = ((R)1 + g * g - f * f) / ((R)2 * g);
    }
    return c > (R)1 ? (R)1 : (c < (R)-1 ? (R)-1 : c);
}

// White's approximation with p_c = 0: P11 (Henyey-Greenstein), P12/P11, P33/P11
template <typename R>
__device__ __forceinline__ void mueller(R g, R p_lin, R c, R &p11, R &r12, R &r33)
{
    R den = (R)1 + g * g - (R)2 * g * c;
    p11 = ((R)1 - g * g) / (den * sqrt(den));
    R c2 = c * c;
    R inv = (R)1 / ((R)1 + c2);
    r12 = -p_lin * ((R)1 - c2) * inv;
    r33 = (R)2 * c * inv;
}

template <typename R>
__device__ __forceinline__ void rotate_stokes(R S[3], R cpsi, R spsi)
{
    R c2 = cpsi * cpsi - spsi * spsi, s2 = (R)2 * spsi * cpsi;
    R q = S[1] * c2 + S[2] * s2;
    R u = -S[1] * s2 + S[2] * c2;
    S[1] = q;
    S[2] = u;
}

// orthonormal completion of a unit vector (Duff et al. 2017): m with k x m = n
template <typename R>
__device__ __forceinline__ void basis_of(const R k[3], R m[3])
{
    R sg = k[2] >= (R)0 ? (R)1 : (R)-1;
    R a = (R)-1 / (sg + k[2]);
    R b = k[0] * k[1] * a;
    m[0] = (R)1 + sg * k[0] * k[0] * a;
    m[1] = sg * b;
    m[2] = -sg * k[0];
}

// Wave-level helpers (wave64)
__device__ __forceinline__ uint64_t lanes_below_mask()
{
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Slot of this lane in an append to *counter by every lane with flag set;
// call from code that all lanes of the wave execute.
__device__ __forceinline__ uint32_t wave_append(bool flag, uint32_t *counter)
{
    const uint64_t mask = __ballot(flag);
    if (mask == 0) return 0;
    uint32_t base = 0;
    if ((threadIdx.x & 63) == 0) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, 0, 64);
    return base + (uint32_t)__popcll(mask & lanes_below_mask());
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace qrt

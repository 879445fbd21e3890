// Per-packet physics shared by the single-scene and the batched launch
// sequences (Shulman, "Quasi-Monte Carlo Radiative Transfer"): emission of a
// point source or a spherical star (Sec. 3.2, 3.3), the state after the forced
// first flight, the peel-off contribution toward one observer (Sec. 2.2, 3.6)
// and the scattering into a new direction (Sec. 2.1, 2.2, 3.5).  Both launch
// sequences call these functions, so a packet takes the same arithmetic in
// either of them.
//
// Coordinates by purpose (Sec. 3.7): a point source takes its direction from
// coordinates 0 and 1 and the forced optical depth from coordinate 2; a star
// in the direct order takes the point on its surface from 0, 1, the local
// direction from 2, 3 (cos theta_l = sqrt(v): a uniform-brightness surface)
// and the forced depth from 4; in the inverse order the direction comes from
// 0, 1, the forced depth from 2 and the point from 3, 4 (cosine-weighted on
// the hemisphere facing the direction).  Scattering k >= 1 takes coordinates
// first_scatter_dim + 3 (k - 1) .. + 2: azimuth i1, cos(Theta), free-flight
// depth.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qrt_internal.h"
#include "qrt_physics.h"

namespace qrt {

__host__ __device__ __forceinline__ int first_scatter_dim(int src_kind) { return src_kind >= 1 ? 5 : 3; }
__host__ __device__ __forceinline__ int forced_tau_dim(int src_kind) { return src_kind == 1 ? 4 : 2; }

// Emission of packet idx.  src_kind: 0 point source, 1 sphere star in the
// direct order, 2 sphere star in the inverse order (a compile-time constant
// in the single-scene kernels, so their other branches fold away).  Each
// branch computes into local arrays and p, k are assigned once at the end:
// assignments to them on several paths would keep them in private memory.
template <typename R, int KIND>
__device__ __forceinline__ void emit_packet(int src_kind, const double src[3], double r_star, const SeqParams &q,
                                            uint64_t idx, R p_out[3], R k_out[3])
{
    uint32_t xa[3], xb[3];
    R p[3], k[3];
    seq_triple<KIND>(q, idx, 0, xa);
    if (src_kind == 0) {
        R sp, cp;
        sincos_2pi<R>(to_unit<R>(xa[0]), sp, cp);
        const R ct = (R)2 * to_unit<R>(xa[1]) - (R)1;
        const R st = sqrt(fmax((R)0, (R)1 - ct * ct));
        for (int a = 0; a < 3; ++a) p[a] = (R)src[a];
        k[0] = st * cp; k[1] = st * sp; k[2] = ct;
    } else {
        seq_triple<KIND>(q, idx, 2, xb);
        if (src_kind == 1) {
            // direct order: point on the star (v1, v2), local direction (v3, v4)
            R spe, cpe, spl, cpl;
            sincos_2pi<R>(to_unit<R>(xa[0]), spe, cpe);
            const R cte = (R)2 * to_unit<R>(xa[1]) - (R)1;
            const R ste = sqrt(fmax((R)0, (R)1 - cte * cte));
            sincos_2pi<R>(to_unit<R>(xb[0]), spl, cpl);
            const R ctl = sqrt(to_unit<R>(xb[1]));
            const R stl = sqrt(fmax((R)0, (R)1 - ctl * ctl));
            const R ne[3] = {ste * cpe, ste * spe, cte};
            const R t1[3] = {cte * cpe, cte * spe, -ste};
            const R t2[3] = {-spe, cpe, (R)0};
            for (int a = 0; a < 3; ++a) {
                p[a] = (R)src[a] + (R)r_star * ne[a];
                k[a] = ctl * ne[a] + stl * (cpl * t1[a] + spl * t2[a]);
            }
        } else {
            // inverse order: direction (v1, v2), emission point about it (v4, v5):
            // azimuth 2 pi v4 about k, cos(alpha) = sqrt(v5)
            R sp, cp, spr, cpr;
            sincos_2pi<R>(to_unit<R>(xa[0]), sp, cp);
            const R ct = (R)2 * to_unit<R>(xa[1]) - (R)1;
            const R st = sqrt(fmax((R)0, (R)1 - ct * ct));
            k[0] = st * cp; k[1] = st * sp; k[2] = ct;
            sincos_2pi<R>(to_unit<R>(xb[1]), spr, cpr);
            const R ca = sqrt(to_unit<R>(xb[2]));
            const R sa = sqrt(fmax((R)0, (R)1 - ca * ca));
            const R t1[3] = {ct * cp, ct * sp, -st};
            const R t2[3] = {-sp, cp, (R)0};
            for (int a = 0; a < 3; ++a)
                p[a] = (R)src[a] + (R)r_star * (ca * k[a] + sa * (cpr * t1[a] + spr * t2[a]));
        }
    }
    for (int a = 0; a < 3; ++a) {
        p_out[a] = p[a];
        k_out[a] = k[a];
    }
}

// The state of a packet at its first scattering: position p + t k (the stop
// of the forced flight; if rounding let the walk reach the edge first, the
// exit point), direction k, reference axis the orthonormal completion of k,
// Stokes weight (W1, 0, 0) with W1 = 1 - e^-tau1.  `tag` is 0 in the
// single-scene path and the scene number in a batch (below 1024); the point
// index idx is below 2^48.
template <typename R>
__device__ __forceinline__ void first_state(const R p[3], const R k[3], R t, R W1, uint64_t idx, uint32_t tag,
                                            PacketState<R> &s)
{
    for (int a = 0; a < 3; ++a) {
        s.p[a] = p[a] + t * k[a];
        s.k[a] = k[a];
    }
    basis_of(k, s.m);
    s.S[0] = W1; s.S[1] = (R)0; s.S[2] = (R)0;
    s.target = 0.0;
    s.word = state_word(idx, tag, 1);
}

// Dust and image geometry of one scene as the physics below needs them.
template <typename R>
struct SceneView {
    R g, p_lin, albedo;
    R half_width;
    int npix;
    int src_kind;
    R src[3], r_star2;
};

// Peel-off toward observer o (image axes ex, ey) of a packet at s.p with
// direction s.k, axis s.m, n_ax = k x m and albedo-weighted Stokes s.S:
// pixel (nearest, no splatting), visibility (inside the image and not behind
// the star) and the contribution before attenuation,
// R_img M(Theta_obs) R_in S / (4 pi).  occluded is set when the star blocks a
// ray that would be on the image.
template <typename R>
__device__ __forceinline__ void peel_contribution(const SceneView<R> &V, const PacketState<R> &s, const R n_ax[3],
                                                  const R o[3], const R ex[3], const R ey[3], bool &vis,
                                                  bool &occluded, R c3[3], uint32_t &pix)
{
    const R Rw = V.half_width;
    const R X = dot3(s.p, ex), Y = dot3(s.p, ey);
    const R fx = floor((X + Rw) / ((R)2 * Rw) * (R)V.npix);
    const R fy = floor((Y + Rw) / ((R)2 * Rw) * (R)V.npix);
    vis = fx >= (R)0 && fy >= (R)0 && fx < (R)V.npix && fy < (R)V.npix;
    occluded = false;
    c3[0] = c3[1] = c3[2] = (R)0;
    pix = 0;
    if (V.src_kind >= 1 && vis) {
        const R d[3] = {s.p[0] - V.src[0], s.p[1] - V.src[1], s.p[2] - V.src[2]};
        const R b = dot3(d, o), cc = dot3(d, d) - V.r_star2;
        if (b < (R)0 && b * b > cc) {   // the star blocks the ray
            occluded = true;
            vis = false;
        }
    }
    if (!vis) return;
    R c = dot3(s.k, o);
    c = c > (R)1 ? (R)1 : (c < (R)-1 ? (R)-1 : c);
    const R sn = sqrt(fmax((R)0, (R)1 - c * c));
    R St[3] = {s.S[0], s.S[1], s.S[2]};
    R mi[3];
    if (sn < (R)1e-12) {
        mi[0] = s.m[0]; mi[1] = s.m[1]; mi[2] = s.m[2];
    } else {
        const R inv_s = (R)1 / sn;
        for (int a = 0; a < 3; ++a) mi[a] = (o[a] - c * s.k[a]) * inv_s;
        rotate_stokes(St, dot3(s.m, mi), dot3(n_ax, mi));
    }
    R p11, r12, r33;
    mueller(V.g, V.p_lin, c, p11, r12, r33);
    const R w = p11 * (R)(0.25 / 3.14159265358979323846);
    c3[0] = w * (St[0] + r12 * St[1]);
    c3[1] = w * (r12 * St[0] + St[1]);
    c3[2] = w * (r33 * St[2]);
    R mo[3], no[3];
    for (int a = 0; a < 3; ++a) mo[a] = c * mi[a] - sn * s.k[a];
    cross3(o, mo, no);
    rotate_stokes(c3, dot3(mo, ex), dot3(no, ex));
    pix = (uint32_t)((int)fy * V.npix + (int)fx);
}

// Scattering into a new direction from coordinates x[0] (azimuth i1 = 2 pi x),
// x[1] (cos Theta from the Henyey-Greenstein inverse CDF) and x[2] (free-flight
// depth -ln w, all 32 bits in FP64): Stokes vector rotated into the scattering
// plane and multiplied by M(Theta) / P11(Theta), then the new direction and
// reference axis k' = cos Theta k + sin Theta m_in, m' = cos Theta m_in -
// sin Theta k with m_in = cos i1 m + sin i1 n.
template <typename R>
__device__ __forceinline__ void scatter_packet(const SceneView<R> &V, PacketState<R> &s, const R n_ax[3],
                                               const uint32_t x[3])
{
    R si, ci;
    sincos_2pi<R>(to_unit<R>(x[0]), si, ci);
    const R ct = hg_cos<R>(V.g, to_unit<R>(x[1]));
    const R st = sqrt(fmax((R)0, (R)1 - ct * ct));
    R mi[3];
    for (int a = 0; a < 3; ++a) mi[a] = ci * s.m[a] + si * n_ax[a];
    rotate_stokes(s.S, ci, si);
    R p11, r12, r33;
    mueller(V.g, V.p_lin, ct, p11, r12, r33);
    const R I1 = s.S[0] + r12 * s.S[1], Q1 = r12 * s.S[0] + s.S[1], U1 = r33 * s.S[2];
    s.S[0] = I1; s.S[1] = Q1; s.S[2] = U1;
    for (int a = 0; a < 3; ++a) {
        const R kn = ct * s.k[a] + st * mi[a];
        const R mn = ct * mi[a] - st * s.k[a];
        s.k[a] = kn;
        s.m[a] = mn;
    }
    s.target = -log((double)x[2] * 0x1p-32);
}

}  // namespace qrt

// Photon-packet transport kernels (Shulman, "Quasi-Monte Carlo Radiative
// Transfer", Sec. 3.2-3.7).
//
// One packet per lane in a persistent grid-stride loop over packet indices.
// A packet: emission (Sec. 3.2 point source, Sec. 3.3 sphere star in direct
// order) -> optical depth tau1 to the mesh edge; end if tau1 < tau_min ->
// forced first scattering, tau = -ln[1 - w (1 - e^-tau1)], move -> for each
// scattering: albedo weight (Sec. 2.1), peel-off to every observer with
// W = W0 e^-tau_obs P(Theta)/(4 pi) (Sec. 3.6), then unless it was the last,
// Henyey-Greenstein direction (Sec. 3.5), Stokes update with White's Mueller
// matrix (Sec. 2.2) divided by the sampled P11, free flight tau2 = -ln w,
// end when the packet leaves the mesh.
//
// Point coordinates are generated per lane on demand: flight k uses
// coordinates 3(k-1) .. 3(k-1)+2 (sphere star: 0..4 for the first flight,
// then 5 + 3(k-2) ..), and a packet that ends early never computes the rest
// (Sec. 3.7).
//
// Stokes frames: the packet carries its direction k and a unit reference axis
// m perpendicular to k (n = k x m); Q > 0 means polarisation along m.  A
// rotation of the reference axis by psi (m' = cos psi m + sin psi n) maps
// (Q, U) to (Q cos 2psi + U sin 2psi, -Q sin 2psi + U cos 2psi).  The
// scattering plane axis of a scattering by (Theta, i1) is m_in = cos i1 m +
// sin i1 n; after it, k' = cos Theta k + sin Theta m_in and
// m' = cos Theta m_in - sin Theta k.  The initial axis is the orthonormal
// completion of k of Duff et al. (2017).  Images use e_x = (-sin phi, cos phi, 0)
// and e_y = o x e_x.
//
// Precision R: float (FP32 positions, directions, Stokes; FP64 optical-depth
// sums, exp/log of per-flight scalars and image sums) or double throughout.
#include <hip/hip_runtime.h>

#include "qrt_internal.h"

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

// White's approximation: P11 (Henyey-Greenstein), P12/P11, P33/P11
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

struct LocalCounters {
    uint64_t visits;
    uint32_t packets, peels, peel_rays, escapes, tau_cuts, scatterings, occluded;
};

template <typename R, int SRC>
__device__ __forceinline__ void peel_all(const TransportParams &P, const RayGrid<R> &G, const R p[3], const R k[3],
                                         const R m[3], const R Sv[3], LocalCounters &L)
{
    const R Rw = (R)P.half_width;
    const size_t plane = (size_t)P.npix * (size_t)P.npix;
    R n[3];
    cross3(k, m, n);
    for (int ob = 0; ob < P.n_obs; ++ob) {
        const DevObserver &O = P.obs[ob];
        R o[3] = {(R)O.o[0], (R)O.o[1], (R)O.o[2]};
        R ex[3] = {(R)O.ex[0], (R)O.ex[1], (R)O.ex[2]};
        R ey[3] = {(R)O.ey[0], (R)O.ey[1], (R)O.ey[2]};
        R X = dot3(p, ex), Y = dot3(p, ey);
        R fx = floor((X + Rw) / ((R)2 * Rw) * (R)P.npix);
        R fy = floor((Y + Rw) / ((R)2 * Rw) * (R)P.npix);
        if (!(fx >= (R)0 && fy >= (R)0 && fx < (R)P.npix && fy < (R)P.npix)) continue;
        if constexpr (SRC == 1) {
            R d[3] = {p[0] - (R)P.src[0], p[1] - (R)P.src[1], p[2] - (R)P.src[2]};
            R b = dot3(d, o), cc = dot3(d, d) - (R)(P.r_star * P.r_star);
            if (b < (R)0 && b * b > cc) { L.occluded++; continue; }
        }
        R c = dot3(k, o);
        c = c > (R)1 ? (R)1 : (c < (R)-1 ? (R)-1 : c);
        R s = sqrt(fmax((R)0, (R)1 - c * c));
        R St[3] = {Sv[0], Sv[1], Sv[2]};
        R mi[3];
        if (s < (R)1e-12) {
            mi[0] = m[0]; mi[1] = m[1]; mi[2] = m[2];
        } else {
            R inv_s = (R)1 / s;
            for (int a = 0; a < 3; ++a) mi[a] = (o[a] - c * k[a]) * inv_s;
            rotate_stokes(St, dot3(m, mi), dot3(n, mi));
        }
        R p11, r12, r33;
        mueller((R)P.g, (R)P.p_lin, c, p11, r12, r33);
        R w = p11 * (R)(0.25 / 3.14159265358979323846);
        R Sp[3] = {w * (St[0] + r12 * St[1]), w * (r12 * St[0] + St[1]), w * (r33 * St[2])};
        R mo[3], no[3];
        for (int a = 0; a < 3; ++a) mo[a] = c * mi[a] - s * k[a];
        cross3(o, mo, no);
        rotate_stokes(Sp, dot3(mo, ex), dot3(no, ex));
        R tdummy;
        WalkResult wr = walk<R, WALK_EDGE>(G, p, o, 0.0, tdummy);
        L.visits += wr.visits;
        L.peel_rays++;
        double att = exp(-wr.tau);
        size_t base = (size_t)ob * 3 * plane + (size_t)(int)fy * (size_t)P.npix + (size_t)(int)fx;
        unsafeAtomicAdd(P.img + base, att * (double)Sp[0]);
        unsafeAtomicAdd(P.img + base + plane, att * (double)Sp[1]);
        unsafeAtomicAdd(P.img + base + 2 * plane, att * (double)Sp[2]);
        L.peels++;
    }
}

template <typename R, int KIND, int SRC>
__device__ __forceinline__ void transport_packet(const TransportParams &P, const RayGrid<R> &G, uint64_t idx,
                                                 LocalCounters &L)
{
    R p[3], k[3];
    int dim_tau, next_dim;
    L.packets++;
    if constexpr (SRC == 1) {
        // direct order: v1,v2 -> point on the star; v3,v4 -> local direction
        // (cos theta_l = sqrt(v4): uniform-brightness surface); v5 -> tau
        uint32_t xa[3], xb[3];
        seq_triple<KIND>(P.seq, idx, 0, xa);
        seq_triple<KIND>(P.seq, idx, 2, xb);   // coordinates 2, 3, 4
        R spe, cpe, spl, cpl;
        sincos_2pi<R>(to_unit<R>(xa[0]), spe, cpe);
        R cte = (R)2 * to_unit<R>(xa[1]) - (R)1;
        R ste = sqrt(fmax((R)0, (R)1 - cte * cte));
        sincos_2pi<R>(to_unit<R>(xb[0]), spl, cpl);
        R ctl = sqrt(to_unit<R>(xb[1]));
        R stl = sqrt(fmax((R)0, (R)1 - ctl * ctl));
        R ne[3] = {ste * cpe, ste * spe, cte};
        R t1[3] = {cte * cpe, cte * spe, -ste};
        R t2[3] = {-spe, cpe, (R)0};
        for (int a = 0; a < 3; ++a) {
            p[a] = (R)P.src[a] + (R)P.r_star * ne[a];
            k[a] = ctl * ne[a] + stl * (cpl * t1[a] + spl * t2[a]);
        }
        dim_tau = 4;
        next_dim = 5;
    } else {
        uint32_t x[3];
        seq_triple<KIND>(P.seq, idx, 0, x);
        R sp, cp;
        sincos_2pi<R>(to_unit<R>(x[0]), sp, cp);
        R ct = (R)2 * to_unit<R>(x[1]) - (R)1;
        R st = sqrt(fmax((R)0, (R)1 - ct * ct));
        p[0] = (R)P.src[0]; p[1] = (R)P.src[1]; p[2] = (R)P.src[2];
        k[0] = st * cp; k[1] = st * sp; k[2] = ct;
        dim_tau = 2;
        next_dim = 3;
    }
    R tx;
    WalkResult w1 = walk<R, WALK_EDGE>(G, p, k, 0.0, tx);
    L.visits += w1.visits;
    const double tau1 = w1.tau;
    if (tau1 < P.tau_min) {
        L.tau_cuts++;
        return;
    }
    const double W1 = -expm1(-tau1);
    // optical-depth targets use all 32 bits of the coordinate in FP64, in both precisions
    const double u_tau = (double)seq_point<KIND>(P.seq, idx, dim_tau) * 0x1p-32;
    const double tau_f = -log1p(-u_tau * W1);
    {
        R t;
        WalkResult wm = walk<R, WALK_MOVE>(G, p, k, tau_f, t);
        L.visits += wm.visits;
        // if rounding lets the walk reach the edge first, scatter at the exit point
        for (int a = 0; a < 3; ++a) p[a] += t * k[a];
    }
    R Sv[3] = {(R)W1, (R)0, (R)0};
    R m[3];
    basis_of(k, m);
    const R albedo = (R)P.albedo;
    for (int order = 1; order <= P.max_orders; ++order) {
        L.scatterings++;
        Sv[0] *= albedo; Sv[1] *= albedo; Sv[2] *= albedo;
        peel_all<R, SRC>(P, G, p, k, m, Sv, L);
        if (order == P.max_orders) return;
        uint32_t x[3];
        seq_triple<KIND>(P.seq, idx, next_dim, x);
        next_dim += 3;
        R si, ci;
        sincos_2pi<R>(to_unit<R>(x[0]), si, ci);
        R ct = hg_cos<R>((R)P.g, to_unit<R>(x[1]));
        R st = sqrt(fmax((R)0, (R)1 - ct * ct));
        R n[3], mi[3];
        cross3(k, m, n);
        for (int a = 0; a < 3; ++a) mi[a] = ci * m[a] + si * n[a];
        rotate_stokes(Sv, ci, si);
        R p11, r12, r33;
        mueller((R)P.g, (R)P.p_lin, ct, p11, r12, r33);
        R I1 = Sv[0] + r12 * Sv[1], Q1 = r12 * Sv[0] + Sv[1], U1 = r33 * Sv[2];
        Sv[0] = I1; Sv[1] = Q1; Sv[2] = U1;
        for (int a = 0; a < 3; ++a) {
            R kn = ct * k[a] + st * mi[a];
            R mn = ct * mi[a] - st * k[a];
            k[a] = kn;
            m[a] = mn;
        }
        const double tau2 = -log((double)x[2] * 0x1p-32);
        R t;
        WalkResult wm = walk<R, WALK_MOVE>(G, p, k, tau2, t);
        L.visits += wm.visits;
        if (!wm.stopped) {
            L.escapes++;
            return;
        }
        for (int a = 0; a < 3; ++a) p[a] += t * k[a];
    }
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void flush_counters(const LocalCounters &L, unsigned long long *cnt)
{
    uint64_t vals[CNT_COUNT] = {L.packets, L.visits, L.peels, L.peel_rays, L.escapes, L.tau_cuts,
                                L.scatterings, L.occluded, 0, 0};
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int i = 0; i < CNT_SCATTERINGS + 2; ++i) {
        uint64_t s = wave_sum_u64(vals[i]);
        if (lead && s) atomicAdd(cnt + i, (unsigned long long)s);
    }
}

template <typename R, int KIND, int SRC>
__global__ void __launch_bounds__(256) k_transport(const TransportParams P, uint64_t first, uint64_t count)
{
    const RayGrid<R> G = ray_grid<R>(P.grid);
    LocalCounters L = {};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride)
        transport_packet<R, KIND, SRC>(P, G, first + j, L);
    flush_counters(L, P.counters);
}

template <typename R, int KIND>
static hipError_t launch_src(const TransportParams &P, uint64_t first, uint64_t count, int blocks, hipStream_t st)
{
    if (P.src_kind == 1)
        hipLaunchKernelGGL((k_transport<R, KIND, 1>), dim3(blocks), dim3(256), 0, st, P, first, count);
    else
        hipLaunchKernelGGL((k_transport<R, KIND, 0>), dim3(blocks), dim3(256), 0, st, P, first, count);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_kind(const TransportParams &P, int kind, uint64_t first, uint64_t count, int blocks,
                              hipStream_t st)
{
    switch (kind) {
    case SEQ_SOBOL: return launch_src<R, SEQ_SOBOL>(P, first, count, blocks, st);
    case SEQ_HALTON: return launch_src<R, SEQ_HALTON>(P, first, count, blocks, st);
    case SEQ_NIED2: return launch_src<R, SEQ_NIED2>(P, first, count, blocks, st);
    case SEQ_HAMMERSLEY: return launch_src<R, SEQ_HAMMERSLEY>(P, first, count, blocks, st);
    case SEQ_PHILOX: return launch_src<R, SEQ_PHILOX>(P, first, count, blocks, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_transport(const TransportParams &P, int precision, int kind, uint64_t first, uint64_t count,
                            int grid_blocks, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    uint64_t need = (count + 255) / 256;
    int blocks = (int)(need < (uint64_t)grid_blocks ? need : (uint64_t)grid_blocks);
    if (precision == 1) return launch_kind<double>(P, kind, first, count, blocks, stream);
    return launch_kind<float>(P, kind, first, count, blocks, stream);
}

// ---------------------------------------------------------------- optical depth of given rays
template <typename R>
__global__ void __launch_bounds__(256) k_trace_tau(const DevGrid g, int64_t n, const double *__restrict__ p,
                                                   const double *__restrict__ k, double *__restrict__ tau,
                                                   int64_t *__restrict__ visits)
{
    const RayGrid<R> G = ray_grid<R>(g);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        R pp[3] = {(R)p[3 * i], (R)p[3 * i + 1], (R)p[3 * i + 2]};
        R kk[3] = {(R)k[3 * i], (R)k[3 * i + 1], (R)k[3 * i + 2]};
        // rays must start in the box (one cell of slack) with a unit direction
        bool ok = fabs(kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2] - (R)1) < (R)1e-3;
        for (int a = 0; a < 3; ++a)
            ok = ok && pp[a] >= (R)(g.lo[a] - g.h[a]) && pp[a] <= (R)(g.hi[a] + g.h[a]);
        if (!ok) {
            tau[i] = __builtin_nan("");
            if (visits) visits[i] = 0;
            continue;
        }
        R t;
        WalkResult w = walk<R, WALK_EDGE>(G, pp, kk, 0.0, t);
        tau[i] = w.tau;
        if (visits) visits[i] = (int64_t)w.visits;
    }
}

hipError_t launch_trace_tau(const DevGrid &g, int precision, int64_t n, const double *p, const double *k,
                            double *tau, int64_t *visits, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    int64_t need = (n + 255) / 256;
    int blocks = (int)(need < 4096 ? need : 4096);
    if (precision == 1)
        hipLaunchKernelGGL(k_trace_tau<double>, dim3(blocks), dim3(256), 0, stream, g, n, p, k, tau, visits);
    else
        hipLaunchKernelGGL(k_trace_tau<float>, dim3(blocks), dim3(256), 0, stream, g, n, p, k, tau, visits);
    return hipGetLastError();
}

}  // namespace qrt

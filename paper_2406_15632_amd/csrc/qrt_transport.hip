// Photon-packet transport kernel (Shulman, "Quasi-Monte Carlo Radiative
// Transfer", Sec. 3.2-3.7).
//
// What one packet does: emission (Sec. 3.2 point source, Sec. 3.3 sphere star
// in direct order) -> optical depth tau1 to the mesh edge; end if
// tau1 < tau_min -> forced first scattering, tau = -ln[1 - w (1 - e^-tau1)],
// move -> at each scattering: albedo weight (Sec. 2.1), peel-off to every
// observer with W = W0 e^-tau_obs P(Theta)/(4 pi) (Sec. 3.6), then unless it
// was the last scattering, Henyey-Greenstein direction (Sec. 3.5), Stokes
// update with White's Mueller matrix (Sec. 2.2) divided by the sampled P11,
// free flight tau2 = -ln w; end when the packet leaves the mesh.
//
// How the GPU runs it: a persistent kernel in which every lane owns one packet
// and one mesh walk at a time.  A packet is a small state machine whose states
// start walks (tau1, the forced move, each peel-off ray, each free flight); all
// walks of all lanes share one batched walk loop (qrt_walk.h), so lanes stay in
// the memory-bound inner loop while their packets are at different stages.
// Packet events (emission, scattering, peel-off bookkeeping) run only when at
// least a quarter of the wave's walks have finished.  Waves take packet
// indices from a global counter 64 at a time.
//
// Point coordinates are generated on demand from the packet index: flight k
// uses coordinates 3(k-1) .. 3(k-1)+2 (sphere star: 0..4 for the first
// flight, then 5 + 3(k-2) ..); a packet that ends early never computes the
// rest (Sec. 3.7).
//
// Stokes frames: the packet carries its direction k and a unit reference axis
// m perpendicular to k (n = k x m); Q > 0 means polarisation along m.  A
// rotation of the reference axis by psi (m' = cos psi m + sin psi n) maps
// (Q, U) to (Q cos 2psi + U sin 2psi, -Q sin 2psi + U cos 2psi).  A scattering
// by (Theta, i1) uses the scattering-plane axis m_in = cos i1 m + sin i1 n;
// then k' = cos Theta k + sin Theta m_in and m' = cos Theta m_in - sin Theta k.
// The initial axis is the orthonormal completion of k of Duff et al. (2017).
// Images use e_x = (-sin phi, cos phi, 0) and e_y = o x e_x.
//
// Precision R: float (FP32 positions, directions, Stokes; FP64 optical-depth
// sums, optical-depth targets and image sums) or double throughout.
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

enum Phase : int {
    PH_NEED = 0,    // wants a packet index
    PH_EMIT = 1,    // has a fresh index
    PH_T1 = 2,      // walking to the mesh edge from the source
    PH_FORCED = 3,  // walking the forced first flight
    PH_PEEL = 4,    // walking a peel-off ray
    PH_FLIGHT = 5,  // walking a free flight
    PH_DONE = 6     // no packets left
};

template <typename R>
struct Packet {
    uint64_t idx;
    R p[3], k[3], m[3], S[3];
    R c[3];        // pending peel-off contribution before attenuation
    int pix;       // its pixel offset within the observer's I plane
    int phase, order, next_dim, obs;
};

template <typename R>
struct SharedObs {
    R o[kMaxObs][3], ex[kMaxObs][3], ey[kMaxObs][3];
};

// Set up the next peel-off ray of the current scattering, or move on.  Returns
// true when a walk was started.
template <typename R, int SRC>
__device__ __forceinline__ bool next_peel(const TransportParams &P, const RayGrid<R> &G, const SharedObs<R> &SO,
                                          Packet<R> &pk, Walk<R> &W, LocalCounters &L)
{
    const R Rw = (R)P.half_width;
    while (pk.obs < P.n_obs) {
        const int ob = pk.obs;
        R o[3] = {SO.o[ob][0], SO.o[ob][1], SO.o[ob][2]};
        R ex[3] = {SO.ex[ob][0], SO.ex[ob][1], SO.ex[ob][2]};
        R ey[3] = {SO.ey[ob][0], SO.ey[ob][1], SO.ey[ob][2]};
        const R X = dot3(pk.p, ex), Y = dot3(pk.p, ey);
        const R fx = floor((X + Rw) / ((R)2 * Rw) * (R)P.npix);
        const R fy = floor((Y + Rw) / ((R)2 * Rw) * (R)P.npix);
        if (!(fx >= (R)0 && fy >= (R)0 && fx < (R)P.npix && fy < (R)P.npix)) { pk.obs++; continue; }
        if constexpr (SRC == 1) {
            R d[3] = {pk.p[0] - (R)P.src[0], pk.p[1] - (R)P.src[1], pk.p[2] - (R)P.src[2]};
            const R b = dot3(d, o), cc = dot3(d, d) - (R)(P.r_star * P.r_star);
            if (b < (R)0 && b * b > cc) { L.occluded++; pk.obs++; continue; }
        }
        R n[3];
        cross3(pk.k, pk.m, n);
        R c = dot3(pk.k, o);
        c = c > (R)1 ? (R)1 : (c < (R)-1 ? (R)-1 : c);
        const R s = sqrt(fmax((R)0, (R)1 - c * c));
        R St[3] = {pk.S[0], pk.S[1], pk.S[2]};
        R mi[3];
        if (s < (R)1e-12) {
            mi[0] = pk.m[0]; mi[1] = pk.m[1]; mi[2] = pk.m[2];
        } else {
            const R inv_s = (R)1 / s;
            for (int a = 0; a < 3; ++a) mi[a] = (o[a] - c * pk.k[a]) * inv_s;
            rotate_stokes(St, dot3(pk.m, mi), dot3(n, mi));
        }
        R p11, r12, r33;
        mueller((R)P.g, (R)P.p_lin, c, p11, r12, r33);
        const R w = p11 * (R)(0.25 / 3.14159265358979323846);
        R Sp[3] = {w * (St[0] + r12 * St[1]), w * (r12 * St[0] + St[1]), w * (r33 * St[2])};
        R mo[3], no[3];
        for (int a = 0; a < 3; ++a) mo[a] = c * mi[a] - s * pk.k[a];
        cross3(o, mo, no);
        rotate_stokes(Sp, dot3(mo, ex), dot3(no, ex));
        pk.c[0] = Sp[0]; pk.c[1] = Sp[1]; pk.c[2] = Sp[2];
        pk.pix = (int)fy * P.npix + (int)fx;
        walk_begin(W, G, pk.p, o, WALK_EDGE, 0.0);
        pk.phase = PH_PEEL;
        return true;
    }
    return false;
}

// Advance a lane's packet from a finished walk (or a fresh index) to its next
// walk; leaves the lane in PH_NEED when the packet is over.
template <typename R, int KIND, int SRC>
__device__ __forceinline__ void advance(const TransportParams &P, const RayGrid<R> &G, const SharedObs<R> &SO,
                                        Packet<R> &pk, Walk<R> &W, LocalCounters &L)
{
    bool scatter = false;
    if (pk.phase == PH_EMIT) {
        L.packets++;
        const uint64_t idx = pk.idx;
        if constexpr (SRC == 1) {
            // direct order: v1,v2 -> point on the star; v3,v4 -> local direction
            // (cos theta_l = sqrt(v4): uniform-brightness surface); v5 -> tau
            uint32_t xa[3], xb[3];
            seq_triple<KIND>(P.seq, idx, 0, xa);
            seq_triple<KIND>(P.seq, idx, 2, xb);
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
                pk.p[a] = (R)P.src[a] + (R)P.r_star * ne[a];
                pk.k[a] = ctl * ne[a] + stl * (cpl * t1[a] + spl * t2[a]);
            }
            pk.next_dim = 5;
        } else {
            uint32_t x[3];
            seq_triple<KIND>(P.seq, idx, 0, x);
            R sp, cp;
            sincos_2pi<R>(to_unit<R>(x[0]), sp, cp);
            const R ct = (R)2 * to_unit<R>(x[1]) - (R)1;
            const R st = sqrt(fmax((R)0, (R)1 - ct * ct));
            pk.p[0] = (R)P.src[0]; pk.p[1] = (R)P.src[1]; pk.p[2] = (R)P.src[2];
            pk.k[0] = st * cp; pk.k[1] = st * sp; pk.k[2] = ct;
            pk.next_dim = 3;
        }
        walk_begin(W, G, pk.p, pk.k, WALK_EDGE, 0.0);
        pk.phase = PH_T1;
        return;
    } else if (pk.phase == PH_T1) {
        L.visits += W.visits;
        const double tau1 = W.tau;
        if (tau1 < P.tau_min) {
            L.tau_cuts++;
            pk.phase = PH_NEED;
            return;
        }
        const double W1 = -expm1(-tau1);
        const int dim_tau = SRC == 1 ? 4 : 2;
        // optical-depth targets use all 32 bits of the coordinate in FP64, in both precisions
        const double u_tau = (double)seq_point<KIND>(P.seq, pk.idx, dim_tau) * 0x1p-32;
        const double tau_f = -log1p(-u_tau * W1);
        pk.S[0] = (R)W1; pk.S[1] = (R)0; pk.S[2] = (R)0;
        walk_begin(W, G, pk.p, pk.k, WALK_MOVE, tau_f);
        pk.phase = PH_FORCED;
        return;
    } else if (pk.phase == PH_FORCED) {
        L.visits += W.visits;
        // if rounding lets the walk reach the edge first, scatter at the exit point
        for (int a = 0; a < 3; ++a) pk.p[a] += W.t_out * pk.k[a];
        basis_of(pk.k, pk.m);
        pk.order = 1;
        scatter = true;
    } else if (pk.phase == PH_FLIGHT) {
        L.visits += W.visits;
        if (!W.stopped) {
            L.escapes++;
            pk.phase = PH_NEED;
            return;
        }
        for (int a = 0; a < 3; ++a) pk.p[a] += W.t_out * pk.k[a];
        pk.order++;
        scatter = true;
    } else if (pk.phase == PH_PEEL) {
        L.visits += W.visits;
        L.peel_rays++;
        L.peels++;
        const double att = exp(-W.tau);
        const size_t plane = (size_t)P.npix * (size_t)P.npix;
        double *base = P.img + (size_t)pk.obs * 3 * plane + (size_t)pk.pix;
        unsafeAtomicAdd(base, att * (double)pk.c[0]);
        unsafeAtomicAdd(base + plane, att * (double)pk.c[1]);
        unsafeAtomicAdd(base + 2 * plane, att * (double)pk.c[2]);
        pk.obs++;
    } else {
        return;   // PH_NEED / PH_DONE: nothing to advance
    }
    if (scatter) {
        L.scatterings++;
        const R albedo = (R)P.albedo;
        pk.S[0] *= albedo; pk.S[1] *= albedo; pk.S[2] *= albedo;
        pk.obs = 0;
    }
    // peel-off toward the remaining observers of this scattering
    if (next_peel<R, SRC>(P, G, SO, pk, W, L)) return;
    if (pk.order == P.max_orders) {
        pk.phase = PH_NEED;
        return;
    }
    // new direction: i1 from the first number of the triple, cos(Theta) from the second
    uint32_t x[3];
    seq_triple<KIND>(P.seq, pk.idx, pk.next_dim, x);
    pk.next_dim += 3;
    R si, ci;
    sincos_2pi<R>(to_unit<R>(x[0]), si, ci);
    const R ct = hg_cos<R>((R)P.g, to_unit<R>(x[1]));
    const R st = sqrt(fmax((R)0, (R)1 - ct * ct));
    R n[3], mi[3];
    cross3(pk.k, pk.m, n);
    for (int a = 0; a < 3; ++a) mi[a] = ci * pk.m[a] + si * n[a];
    rotate_stokes(pk.S, ci, si);
    R p11, r12, r33;
    mueller((R)P.g, (R)P.p_lin, ct, p11, r12, r33);
    const R I1 = pk.S[0] + r12 * pk.S[1], Q1 = r12 * pk.S[0] + pk.S[1], U1 = r33 * pk.S[2];
    pk.S[0] = I1; pk.S[1] = Q1; pk.S[2] = U1;
    for (int a = 0; a < 3; ++a) {
        const R kn = ct * pk.k[a] + st * mi[a];
        const R mn = ct * mi[a] - st * pk.k[a];
        pk.k[a] = kn;
        pk.m[a] = mn;
    }
    const double tau2 = -log((double)x[2] * 0x1p-32);
    walk_begin(W, G, pk.p, pk.k, WALK_MOVE, tau2);
    pk.phase = PH_FLIGHT;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void flush_counters(const LocalCounters &L, unsigned long long *cnt)
{
    uint64_t vals[CNT_SCATTERINGS + 2] = {L.packets, L.visits, L.peels, L.peel_rays, L.escapes, L.tau_cuts,
                                          L.scatterings, L.occluded};
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int i = 0; i < CNT_SCATTERINGS + 2; ++i) {
        uint64_t s = wave_sum_u64(vals[i]);
        if (lead && s) atomicAdd(cnt + i, (unsigned long long)s);
    }
}

constexpr int kWalkBatch = 4;
constexpr int kWaveRefill = 16;   // handle packet events once this many lanes of a wave are idle

template <typename R, int KIND, int SRC>
__global__ void __launch_bounds__(256) k_transport(const TransportParams P, uint64_t first, uint64_t count,
                                                   unsigned long long *__restrict__ work)
{
    __shared__ SharedObs<R> SO;
    for (int i = threadIdx.x; i < P.n_obs; i += blockDim.x) {
        for (int a = 0; a < 3; ++a) {
            SO.o[i][a] = (R)P.obs[i].o[a];
            SO.ex[i][a] = (R)P.obs[i].ex[a];
            SO.ey[i][a] = (R)P.obs[i].ey[a];
        }
    }
    __syncthreads();
    const RayGrid<R> G = ray_grid<R>(P.grid);
    LocalCounters L = {};
    Packet<R> pk;
    pk.phase = PH_NEED;
    pk.idx = 0;
    Walk<R> W;
    W.done = true;
    W.visits = 0;
    const int lane = threadIdx.x & 63;
    const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // wave-uniform pool of packet offsets [pool_next, pool_end)
    uint64_t pool_next = 0, pool_end = 0;
    bool pool_dry = false;
    for (;;) {
        // give packets to lanes that need one, then advance every lane whose walk
        // ended; twice, because a packet can end during its events
        for (int pass = 0; pass < 2; ++pass) {
            uint64_t need = __ballot(pk.phase == PH_NEED);
            while (need && !pool_dry) {
                if (pool_next >= pool_end) {
                    unsigned long long base = 0;
                    if (lane == 0) base = atomicAdd(work, 64ull);
                    base = __shfl(base, 0, 64);
                    pool_next = base;
                    pool_end = base + 64 < count ? base + 64 : count;
                    if (pool_next >= count) {
                        pool_dry = true;
                        break;
                    }
                }
                const uint64_t avail = pool_end - pool_next;
                const uint64_t take = (uint64_t)__popcll(need) < avail ? (uint64_t)__popcll(need) : avail;
                const uint64_t rank = (uint64_t)__popcll(need & lanes_below);
                if (pk.phase == PH_NEED && rank < take) {
                    pk.idx = first + pool_next + rank;
                    pk.phase = PH_EMIT;
                }
                pool_next += take;
                need = __ballot(pk.phase == PH_NEED);
            }
            if (pool_dry && pk.phase == PH_NEED) pk.phase = PH_DONE;
            if (pk.phase == PH_EMIT || (W.done && pk.phase != PH_NEED && pk.phase != PH_DONE))
                advance<R, KIND, SRC>(P, G, SO, pk, W, L);
        }
        if (__ballot(pk.phase != PH_DONE) == 0) break;
        // walk until enough lanes need events
        for (;;) {
            walk_batch<R, kWalkBatch>(W, G);
            const uint64_t idle = __ballot(W.done || pk.phase == PH_DONE || pk.phase == PH_NEED);
            if (__popcll(idle) >= kWaveRefill) break;
        }
    }
    flush_counters(L, P.counters);
}

// blocks of 256 that fit on the device at once (the kernel is persistent)
template <typename R, int KIND, int SRC>
static int resident_blocks()
{
    static int cached = 0;
    if (cached == 0) {
        int per_cu = 0, dev = 0;
        hipDeviceProp_t prop;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_transport<R, KIND, SRC>, 256, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        (void)hipGetDevice(&dev);
        int cus = 256;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
        cached = per_cu * cus;
    }
    return cached;
}

template <typename R, int KIND, int SRC>
static hipError_t launch_one(const TransportParams &P, uint64_t first, uint64_t count, int cap,
                             unsigned long long *work, hipStream_t st)
{
    const uint64_t need = (count + 255) / 256;
    int blocks = resident_blocks<R, KIND, SRC>();
    if (cap > 0 && blocks > cap) blocks = cap;
    if ((uint64_t)blocks > need) blocks = (int)need;
    hipLaunchKernelGGL((k_transport<R, KIND, SRC>), dim3(blocks), dim3(256), 0, st, P, first, count, work);
    return hipGetLastError();
}

template <typename R, int KIND>
static hipError_t launch_src(const TransportParams &P, uint64_t first, uint64_t count, int cap,
                             unsigned long long *work, hipStream_t st)
{
    if (P.src_kind == 1) return launch_one<R, KIND, 1>(P, first, count, cap, work, st);
    return launch_one<R, KIND, 0>(P, first, count, cap, work, st);
}

template <typename R>
static hipError_t launch_kind(const TransportParams &P, int kind, uint64_t first, uint64_t count, int blocks,
                              unsigned long long *work, hipStream_t st)
{
    switch (kind) {
    case SEQ_SOBOL: return launch_src<R, SEQ_SOBOL>(P, first, count, blocks, work, st);
    case SEQ_HALTON: return launch_src<R, SEQ_HALTON>(P, first, count, blocks, work, st);
    case SEQ_NIED2: return launch_src<R, SEQ_NIED2>(P, first, count, blocks, work, st);
    case SEQ_HAMMERSLEY: return launch_src<R, SEQ_HAMMERSLEY>(P, first, count, blocks, work, st);
    case SEQ_PHILOX: return launch_src<R, SEQ_PHILOX>(P, first, count, blocks, work, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_transport(const TransportParams &P, int precision, int kind, uint64_t first, uint64_t count,
                            int grid_blocks, unsigned long long *work, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(work, 0, sizeof(unsigned long long), stream);
    if (e != hipSuccess) return e;
    // grid_blocks > 0 caps the persistent grid (otherwise: every block that fits)
    if (precision == 1) return launch_kind<double>(P, kind, first, count, grid_blocks, work, stream);
    return launch_kind<float>(P, kind, first, count, grid_blocks, work, stream);
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
        Walk<R> W;
        walk_begin(W, G, pp, kk, WALK_EDGE, 0.0);
        walk_run<R, kWalkBatch>(W, G);
        tau[i] = W.tau;
        if (visits) visits[i] = (int64_t)W.visits;
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

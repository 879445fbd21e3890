// Photon-packet transport (Shulman, "Quasi-Monte Carlo Radiative Transfer",
// Sec. 3.2-3.7) as a wavefront of kernels over packet queues in HBM.
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
// How the GPU runs a chunk of packets:
//   k_key_emit and the radix sort: the packets in emission-direction order.
//   k_first    persistent; per packet: emission, walk to the edge (tau1), the
//              forced-flight walk; the states of the packets that scatter are
//              appended to the first live list (dense, ping-pong by order).
//   per scattering order:
//   k_scatter  one lane per live packet, in place: albedo, the peel-off
//              contribution and pixel for every observer (written as peel
//              rays in fixed slots), then the new direction, Stokes vector and
//              flight depth.
//   k_walk     persistent; walks every peel ray (adding e^-tau times its
//              contribution to the image) and every flight (the states of the
//              packets that stop inside the mesh go to the other live list).
//   from the first order of the late-order launch (qrt_set_tail) on:
//   k_tail     persistent; a lane carries a live packet through its remaining
//              orders (new direction, flight), keeping the state of every
//              scattering it reaches in the other list (a region per XCD);
//   k_def_keys and the radix sort: those scatterings in the order of their
//              positions; then k_scatter (peel-offs only) and k_walk over them.
// Only the persistent kernels walk the mesh; the per-ray events of the walks
// are a few loads and stores, so they keep a small register footprint.  The
// physics runs in k_first's events, in k_scatter, which is convergent, and in
// k_tail's scattering events.  Waves of
// the persistent kernels take work in blocks of 64 to 512 items from counters
// of their XCD (WorkPool) and refill once every lane of the wave is idle, which
// keeps a wave's rays together; the per-order walks hand out their items in
// 512-item blocks in a strided order (scatter_block), so that concurrent waves
// do not all walk rays of one part of the mesh.  The per-order walks run at three blocks per CU
// (kWalkBlocksPerCu): their flights are incoherent gathers, and fewer waves
// leave more of each lane's lines in the L1 cache.
//
// Point coordinates are generated from the packet index: flight k uses
// coordinates 3(k-1) .. 3(k-1)+2 (sphere star: 0..4 for the first flight, then
// 5 + 3(k-2) ..); a packet that ends early never computes the rest (Sec. 3.7).
//
// Stokes frames and the scattering geometry are described in qrt_physics.h: a
// scattering by (Theta, i1) uses the scattering-plane axis
// m_in = cos i1 m + sin i1 n; then k' = cos Theta k + sin Theta m_in and
// m' = cos Theta m_in - sin Theta k.  The initial axis is the orthonormal
// completion of k of Duff et al. (2017).  Images use e_x = (-sin phi, cos phi, 0)
// and e_y = o x e_x.
//
// Precision R: float (FP32 positions, directions, Stokes; FP64 optical-depth
// sums, optical-depth targets and image sums) or double throughout.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qrt_internal.h"
#include "qrt_mlp.h"
#include "qrt_packet.h"
#include <cstddef>

#include "qrt_physics.h"
#include "qrt_wave.h"

static_assert(sizeof(((qrt::Queues *)nullptr)->work[0]) ==
                  sizeof(unsigned long long) * qrt::kPoolParts * qrt::kPoolStride,
              "a pool's counters: kPoolParts lines of kPoolStride counters");

namespace qrt {

size_t packet_state_bytes(int precision)
{
    return precision == 1 ? sizeof(PacketState<double>) : sizeof(PacketState<float>);
}
size_t peel_ray_bytes(int precision) { return precision == 1 ? sizeof(PeelRay<double>) : sizeof(PeelRay<float>); }

// --------------------------------------------------------------------------
// coherence sorts
// --------------------------------------------------------------------------
// Mesh walks are bound by the rate of distinct cache lines that a wave's
// loads touch.  Lanes of a wave that walk nearly the same cells share lines,
// so the packets of a chunk are sorted by emission direction
// (octahedral map, 2 x 8 bits) before their first flights: a wave then walks
// 64 nearly parallel rays from the source.  The order only changes which lanes
// run which packets; every packet is computed as before.

template <typename R, int KIND, int SRC>
__device__ __forceinline__ void emit(const TransportParams &P, uint64_t idx, R p[3], R k[3]);

template <typename R, int KIND, int SRC>
__global__ void __launch_bounds__(256) k_key_emit(const TransportParams P, uint64_t first, uint32_t count,
                                                  uint32_t *__restrict__ keys)
{
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < count; j += gridDim.x * blockDim.x) {
        R p[3], k[3];
        emit<R, KIND, SRC>(P, first + j, p, k);
        keys[j] = direction_key(k);
    }
}

// The sort: a stable least-significant-digit radix sort of the packets by
// their 16-bit keys, in two passes of 8 bits.  Each pass splits the items into
// blocks of kSortItems, counts the digits per block (k_digit_hist), turns the
// counts into each block's start inside each digit (k_digit_scan), and places
// every item at the start of its digit, plus the items of that digit in
// earlier blocks, plus the earlier items of that digit in its own block
// (k_digit_scatter).  No device-wide atomics: every position is computed.

// hist[d * nb + b] = items of block b whose digit (key >> shift) & 255 is d
__global__ void __launch_bounds__(kSortDigit) k_digit_hist(const uint32_t *__restrict__ keys, uint32_t count, int shift,
                                                           uint32_t *__restrict__ hist,
                                                           const uint32_t *__restrict__ count_dev)
{
    __shared__ uint32_t h[kSortDigit];
    if (count_dev) count = min(count, *count_dev);
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t b0 = blockIdx.x * (uint32_t)kSortItems;
    for (int r = 0; r < kSortItems / kSortDigit; ++r) {
        const uint32_t i = b0 + (uint32_t)(r * kSortDigit) + threadIdx.x;
        if (i < count) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// exclusive prefix of an LDS array of kSortDigit entries (the block has kSortDigit threads)
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t *a)
{
    const int t = threadIdx.x;
    const uint32_t own = a[t];
    for (int off = 1; off < kSortDigit; off <<= 1) {
        const uint32_t v = t >= off ? a[t - off] : 0u;
        __syncthreads();
        a[t] += v;
        __syncthreads();
    }
    return a[t] - own;
}

// One block per digit d: hist[d * nb + b] becomes the sum over the blocks
// before b (nb <= 4 kSortDigit), and tot[d] the digit's total.
__global__ void __launch_bounds__(kSortDigit) k_digit_scan(uint32_t *__restrict__ hist, int nb,
                                                           uint32_t *__restrict__ tot)
{
    __shared__ uint32_t part[kSortDigit];
    uint32_t *row = hist + (size_t)blockIdx.x * nb;
    const int per = (nb + kSortDigit - 1) / kSortDigit;
    uint32_t v[4];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = (int)threadIdx.x * per + k;
        v[k] = (k < per && i < nb) ? row[i] : 0u;
        sum += v[k];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    uint32_t run = block_exclusive_scan(part);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = (int)threadIdx.x * per + k;
        if (k < per && i < nb) row[i] = run;
        run += v[k];
    }
    if (threadIdx.x == kSortDigit - 1) tot[blockIdx.x] = run;
}

// Stable placement of the items of one block by digit.  The block takes its
// items in rounds of kSortDigit, in order; inside a round, the lanes of a wave
// with the same digit are found with one ballot per digit bit, and the waves'
// counts per digit give each item its place in an LDS tile that holds the
// block's items ordered by digit (stably).  The tile is then written out in
// order: its entries of one digit go to consecutive places, so the stores of a
// wave coalesce instead of scattering over up to 64 digits.  keys_out may be
// null (last pass); vals_in null stands for the item numbers.
__global__ void __launch_bounds__(kSortDigit) k_digit_scatter(const uint32_t *__restrict__ keys_in,
                                                              const uint32_t *__restrict__ vals_in, uint32_t count,
                                                              int shift, const uint32_t *__restrict__ hist,
                                                              const uint32_t *__restrict__ tot,
                                                              uint32_t *__restrict__ keys_out,
                                                              uint32_t *__restrict__ vals_out,
                                                              const uint32_t *__restrict__ count_dev)
{
    constexpr int kWaves = kSortDigit / 64;
    if (count_dev) count = min(count, *count_dev);
    const uint32_t b0 = blockIdx.x * (uint32_t)kSortItems;
    if (b0 >= count) return;   // past the items (device count)
    __shared__ uint32_t base[kSortDigit];    // output place of the block's first item of each digit
    __shared__ uint32_t next[kSortDigit];    // tile place of each digit's next item
    __shared__ uint32_t first[kSortDigit];   // tile place of each digit's first item
    __shared__ uint32_t wc[kWaves][kSortDigit];
    __shared__ uint32_t tile_key[kSortItems], tile_val[kSortItems];
    const int t = threadIdx.x, w = t >> 6;
    const uint32_t n = count - b0 < (uint32_t)kSortItems ? count - b0 : (uint32_t)kSortItems;
    base[t] = tot[t];
    __syncthreads();
    const uint32_t start = block_exclusive_scan(base);
    // this block's items of digit t: the blocks' starts inside the digit are scanned
    const uint32_t off = hist[t * gridDim.x + blockIdx.x];
    const uint32_t mine = (blockIdx.x + 1 < gridDim.x ? hist[t * gridDim.x + blockIdx.x + 1] : tot[t]) - off;
    __syncthreads();
    base[t] = start + off;
    next[t] = mine;
    for (int v = 0; v < kWaves; ++v) wc[v][t] = 0;
    __syncthreads();
    const uint32_t tile_start = block_exclusive_scan(next);
    __syncthreads();
    next[t] = tile_start;
    first[t] = tile_start;
    __syncthreads();
    for (int r = 0; r < kSortItems / kSortDigit; ++r) {
        const uint32_t i = b0 + (uint32_t)(r * kSortDigit) + (uint32_t)t;
        const bool valid = i < count;
        const uint32_t key = valid ? keys_in[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool one = (d >> bit) & 1u;
            const uint64_t m = __ballot(valid && one);
            peers &= one ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanes_below_mask());
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = next[d] + rank;
            for (int v = 0; v < w; ++v) pos += wc[v][d];
            tile_key[pos] = key;
            tile_val[pos] = vals_in ? vals_in[i] : i;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int v = 0; v < kWaves; ++v) {
            add += wc[v][t];
            wc[v][t] = 0;
        }
        next[t] += add;
        __syncthreads();
    }
    for (uint32_t j = (uint32_t)t; j < n; j += kSortDigit) {
        const uint32_t key = tile_key[j];
        const uint32_t d = (key >> shift) & 255u;
        const uint32_t pos = base[d] + (j - first[d]);
        if (keys_out) keys_out[pos] = key;
        vals_out[pos] = tile_val[j];
    }
}

hipError_t launch_sort_keys(const TransportBuffers &B, uint32_t count, hipStream_t st, KernelTimer *timer,
                            const uint32_t *count_dev)
{
    if (count == 0) return hipSuccess;
    if (count > kChunk) return hipErrorInvalidValue;
    TimedLaunch tl(timer, st, TC_SORT);
    const int nb = (int)((count + kSortItems - 1) / kSortItems);
    uint32_t *tot = B.hist + (size_t)kSortDigit * (kChunk / kSortItems);
    uint32_t *tmp_keys = B.sort_tmp, *tmp_vals = B.sort_tmp + B.cap;
    // low digit: keys and packet numbers into the scratch lists
    hipLaunchKernelGGL(k_digit_hist, dim3(nb), dim3(kSortDigit), 0, st, (const uint32_t *)B.keys, count, 0, B.hist,
                       count_dev);
    hipLaunchKernelGGL(k_digit_scan, dim3(kSortDigit), dim3(kSortDigit), 0, st, B.hist, nb, tot);
    hipLaunchKernelGGL(k_digit_scatter, dim3(nb), dim3(kSortDigit), 0, st, (const uint32_t *)B.keys,
                       (const uint32_t *)nullptr, count, 0, (const uint32_t *)B.hist, (const uint32_t *)tot,
                       tmp_keys, tmp_vals, count_dev);
    // high digit: the packet numbers into order
    hipLaunchKernelGGL(k_digit_hist, dim3(nb), dim3(kSortDigit), 0, st, (const uint32_t *)tmp_keys, count, 8, B.hist,
                       count_dev);
    hipLaunchKernelGGL(k_digit_scan, dim3(kSortDigit), dim3(kSortDigit), 0, st, B.hist, nb, tot);
    hipLaunchKernelGGL(k_digit_scatter, dim3(nb), dim3(kSortDigit), 0, st, (const uint32_t *)tmp_keys,
                       (const uint32_t *)tmp_vals, count, 8, (const uint32_t *)B.hist, (const uint32_t *)tot,
                       (uint32_t *)nullptr, B.order, count_dev);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// first flight
// --------------------------------------------------------------------------
// SRC: 0 point source, 1 sphere star in direct order, 2 sphere star in inverse order
template <typename R, int KIND, int SRC>
__device__ __forceinline__ void emit(const TransportParams &P, uint64_t idx, R p[3], R k[3])
{
    emit_packet<R, KIND>(SRC, P.src, P.r_star, P.seq, idx, p, k);
}

enum FirstPhase : int { FF_IDLE = 0, FF_EDGE = 1, FF_FORCED = 2 };

template <typename R, int KIND, int SRC>
__global__ void __launch_bounds__(256) k_first(const TransportParams P, uint64_t first, uint32_t count,
                                               const uint32_t *__restrict__ order,
                                               PacketState<R> *__restrict__ out, Queues *__restrict__ Q)
{
    const RayGrid<R> G = ray_grid<R>(P.grid);
    uint64_t n_visits = 0;
    uint32_t n_packets = 0, n_cuts = 0;
    int phase = FF_IDLE;
    uint32_t j = 0;
    R p[3] = {(R)0, (R)0, (R)0}, k[3] = {(R)0, (R)0, (R)1};
    R S0 = (R)0;
    Walk<R> W;
    W.done = true;
    WorkPool pool;
    for (;;) {
        // packets whose forced flight ended go to the first live list, in place pos
        const bool append = W.done && phase == FF_FORCED;
        const uint32_t pos = wave_append(append, &Q->n_live[0]);
        if (W.done && phase == FF_EDGE) {
            n_visits += W.visits;
            const double tau1 = W.tau;
            if (tau1 < P.tau_min) {
                n_cuts++;
                phase = FF_IDLE;
            } else {
                const double W1 = -expm1(-tau1);
                // optical-depth targets use all 32 bits of the coordinate in FP64, in both precisions
                const double u = (double)seq_point<KIND>(P.seq, first + j, forced_tau_dim(SRC)) * 0x1p-32;
                S0 = (R)W1;
                walk_begin(W, G, p, k, WALK_MOVE, -log1p(-u * W1));
                phase = FF_FORCED;
            }
        } else if (append) {
            n_visits += W.visits;
            // if rounding lets the walk reach the edge first, scatter at the exit point
            PacketState<R> s;
            first_state<R>(p, k, W.t_out, S0, first + j, 0u, s);
            out[pos] = s;
            phase = FF_IDLE;
        }
        uint64_t item = 0;
        if (pool.take(phase == FF_IDLE, count, &Q->work[0][0][0], item)) {
            j = order[item];
            n_packets++;
            emit<R, KIND, SRC>(P, first + j, p, k);
            walk_begin(W, G, p, k, WALK_EDGE, 0.0);
            phase = FF_EDGE;
        }
        if (__ballot(phase != FF_IDLE) == 0 && pool.dry) break;
        if (__ballot(phase == FF_FORCED) == 0) {
            // no lane moves to a target: walks to the edge only
            for (;;) {
                walk_batch_edge<R, kWalkBatch>(W, G);
                if (__popcll(__ballot(W.done || phase == FF_IDLE)) >= kWaveRefill) break;
            }
        } else {
            for (;;) {
                walk_batch<R, kWalkBatch>(W, G);
                if (__popcll(__ballot(W.done || phase == FF_IDLE)) >= kWaveRefill) break;
            }
        }
    }
    flush_counters<4>(P.counters, {CNT_PACKETS, CNT_TAU_CUTS, CNT_VISITS, CNT_VISITS_FIRST},
                      {n_packets, n_cuts, n_visits, n_visits});
}

// --------------------------------------------------------------------------
// scattering: albedo, peel-off contributions, new direction
// --------------------------------------------------------------------------
template <typename R>
struct ObsTable {
    R o[kMaxObs][3], ex[kMaxObs][3], ey[kMaxObs][3];
};

template <typename R>
__device__ __forceinline__ void load_obs(const TransportParams &P, ObsTable<R> &T)
{
    for (int i = threadIdx.x; i < P.n_obs; i += blockDim.x)
        for (int a = 0; a < 3; ++a) {
            T.o[i][a] = (R)P.obs[i].o[a];
            T.ex[i][a] = (R)P.obs[i].ex[a];
            T.ey[i][a] = (R)P.obs[i].ey[a];
        }
    __syncthreads();
}

// The image copy of this block (blocks go round-robin to the XCDs), in the set
// of the scattering order when orders are kept apart.
__device__ __forceinline__ double *image_copy(const TransportParams &P, int order, size_t plane)
{
    const size_t set = (size_t)P.n_obs * 3 * plane;
    const size_t s = P.order_images > 0 ? (size_t)(order - 1) : 0;
    return P.img + (s * kImageCopies + (size_t)(blockIdx.x % kImageCopies)) * set;
}

// --------------------------------------------------------------------------
// surrogate peel-off (an addition to the method): inside the validated domain
// the network gives the optical depth to the observer
// --------------------------------------------------------------------------

// Surrogate peel-off of one order.  The scattering kernel queues the visible
// peel rays that start in a valid cell of the surrogate's domain, with their
// network inputs, pixel and contribution (one reservation per wave), and
// leaves them out of the walk; this kernel takes the queue in batches of 64
// rays per wave, so every batch but the last is full, runs the network on the
// matrix cores with the forward weight tiles in LDS, and adds the
// contributions attenuated by e^-max(tau_hat, 0) to the image, merged by
// pixel.  Its loads are coalesced reads of the queue.
struct __align__(16) PeelNetLds {
    bf16x8 Wt[kFwdTiles * 64];
    float bias[260];
    double merge[4][64][3];
};

__global__ void __launch_bounds__(256) k_peel_net(const TransportParams P, int order, int in,
                                                  const SurQuery *__restrict__ sur_q, const uint32_t *__restrict__ sur_n,
                                                  const Queues *__restrict__ Q)
{
    __shared__ PeelNetLds L;
    const int lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_blocks = (Q->n_live[in] + 63) / 64;
    // a wave takes `span` consecutive blocks at a time (at most 64, so that the
    // launch spreads over all waves): their counts, scanned over the wave, give
    // each queued ray its position in the wave's batches
    const uint32_t span = n_blocks > waves * 64 ? 64u : (n_blocks + waves - 1) / waves;
    // a block whose first wave has no blocks has no work at all (the late
    // orders): it leaves before loading the weights
    if ((uint64_t)blockIdx.x * (blockDim.x >> 6) * span >= n_blocks) return;
    mlp_tiles_to_lds(L.Wt, (const bf16x8 *)P.sur.tiles);
    mlp_bias_to_lds(L.bias, P.sur.params);
    __syncthreads();
    const size_t plane = (size_t)P.npix * (size_t)P.npix;
    double *img_copy = image_copy(P, order, plane);
    const int key_bits = bits_for((uint64_t)P.n_obs * 3 * plane);
    const size_t region = (size_t)64 * P.n_obs;
    for (uint32_t b0 = wave * span; b0 < n_blocks; b0 += waves * span) {
        const uint32_t b = b0 + (uint32_t)lane;
        const uint32_t cnt = ((uint32_t)lane < span && b < n_blocks) ? sur_n[b] : 0u;
        uint32_t incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(incl, off, 64);
            incl += lane >= off ? v : 0u;
        }
        const uint32_t excl = incl - cnt;
        const uint32_t total = __shfl(incl, 63, 64);
        for (uint32_t j = 0; j < total; j += 64) {
            const uint32_t qi = j + (uint32_t)lane;
            const bool on = qi < total;
            // the block holding ray qi: the last lane whose exclusive sum is <= qi
            int k = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const uint32_t e = __shfl(excl, k + step, 64);
                k = (k + step < 64 && e <= qi) ? k + step : k;
            }
            const uint32_t ek = __shfl(excl, k, 64);
            SurQuery q = {};
            if (on) q = sur_q[(size_t)(b0 + (uint32_t)k) * region + (qi - ek)];
            const float t = mlp_wave_lds(L.Wt, L.bias, q.x, lane);
            const double att = exp(-(double)fmaxf(t, 0.0f));
            wave_merge_add(on, q.key, att * q.c[0], att * q.c[1], att * q.c[2], img_copy, plane, key_bits,
                           L.merge[threadIdx.x >> 6]);
        }
    }
}

template <typename R>
__device__ __forceinline__ SceneView<R> scene_view(const TransportParams &P, int src_kind)
{
    SceneView<R> V;
    V.g = (R)P.g;
    V.p_lin = (R)P.p_lin;
    V.albedo = (R)P.albedo;
    V.half_width = (R)P.half_width;
    V.npix = P.npix;
    V.src_kind = src_kind;
    for (int a = 0; a < 3; ++a) V.src[a] = (R)P.src[a];
    V.r_star2 = (R)(P.r_star * P.r_star);
    return V;
}

// Scattering of the live packets of one order, one lane per packet: albedo,
// the peel-off contribution toward every observer (written as a peel ray for
// the walk), then the new direction and flight depth.  SUR: surrogate mode,
// in which the visible rays that start in a valid cell of the surrogate's
// domain are also queued for k_peel_net.
// def_cap > 0: the list holds the scatterings deferred by the late-order
// launch, in kPoolParts regions of def_cap states, some marked kNoState
// (reserved when a region was full, never scattered here: their order field
// holds kNoState); item i is state deferred_slot(perm[i]), perm being their
// order by position (k_def_keys), and their count goes to n_live[in] for the
// walks.
template <typename R, int KIND, int SRC, bool SUR>
__global__ void __launch_bounds__(256) k_scatter(const TransportParams P, int order, PacketState<R> *__restrict__ pks,
                                                 int in, PeelRay<R> *__restrict__ peels, SurQuery *__restrict__ sur_q,
                                                 uint32_t *__restrict__ sur_n, Queues *__restrict__ Q,
                                                 uint32_t def_cap, const uint32_t *__restrict__ perm)
{
    __shared__ ObsTable<R> T;
    load_obs(P, T);
    if (blockIdx.x == 0 && threadIdx.x < kPoolParts) {
        // counters of the walk that follows
        if (threadIdx.x == 0) Q->n_live[in ^ 1] = 0;
        Q->work[1][threadIdx.x][0] = 0;
    }
    const DeferredList D = deferred_list(Q, def_cap);
    const uint32_t n = def_cap ? (uint32_t)D.end[kPoolParts - 1] : Q->n_live[in];
    if (def_cap && blockIdx.x == 0 && threadIdx.x == 0) Q->n_live[in] = n;
    const int lane = threadIdx.x & 63;
    const uint32_t wave0 = (blockIdx.x * blockDim.x + threadIdx.x) - (uint32_t)lane;
    const uint32_t stride = gridDim.x * blockDim.x;
    const SceneView<R> V = scene_view<R>(P, SRC);
    const size_t cells = (size_t)P.sur.n_r * (size_t)P.sur.n_z;
    uint32_t n_scat = 0, n_occ = 0, n_sur = 0, n_fb = 0;
    for (uint32_t base = wave0; base < n; base += stride) {
        const uint32_t i = base + (uint32_t)lane;
        bool valid = i < n;
        PacketState<R> s = {};
        if (valid) {
            s = pks[def_cap ? deferred_slot(D, perm[i]) : i];
            valid = !def_cap || state_order(s.word) != kNoState;
        }
        if (valid) {
            n_scat++;
            s.S[0] *= V.albedo; s.S[1] *= V.albedo; s.S[2] *= V.albedo;
        }
        R n_ax[3];
        cross3(s.k, s.m, n_ax);
        uint32_t queued = 0;   // rays of this wave's 64-packet block queued for the network (wave-uniform)
        // the scattering point's cell of the surrogate's domain and its network inputs, which do not
        // depend on the observer
        int cell = -1;
        float x_pos[3] = {0.0f, 0.0f, 0.0f};
        if constexpr (SUR) {
            if (valid) {
                cell = dom_cell(P.sur, (double)s.p[0], (double)s.p[1], (double)s.p[2]);
                if (cell >= 0) {
                    float x[5];
                    mlp_inputs(P.sur.in, (double)s.p[0], (double)s.p[1], (double)s.p[2], 0, x);
                    x_pos[0] = x[0]; x_pos[1] = x[1]; x_pos[2] = x[2];
                }
            }
        }
        for (int ob = 0; ob < P.n_obs; ++ob) {
            bool vis = false, occ = false;
            R c3[3] = {(R)0, (R)0, (R)0};
            uint32_t pix = 0;
            if (valid) {
                const R o[3] = {T.o[ob][0], T.o[ob][1], T.o[ob][2]};
                const R ex[3] = {T.ex[ob][0], T.ex[ob][1], T.ex[ob][2]};
                const R ey[3] = {T.ey[ob][0], T.ey[ob][1], T.ey[ob][2]};
                peel_contribution<R>(V, s, n_ax, o, ex, ey, vis, occ, c3, pix);
                n_occ += occ ? 1u : 0u;
            }
            bool use = false;
            if constexpr (SUR) {
                if (vis) use = cell >= 0 && P.sur.valid[(size_t)ob * cells + (size_t)cell] != 0;
                n_fb += (vis && !use) ? 1u : 0u;
                n_sur += use ? 1u : 0u;
                // the block's queue region: its queued rays, observer after observer
                const uint64_t m = __ballot(use);
                if (use) {
                    SurQuery q;
                    q.x[0] = x_pos[0]; q.x[1] = x_pos[1]; q.x[2] = x_pos[2];
                    q.x[3] = P.sur.in.obs_in[ob][0];
                    q.x[4] = P.sur.in.obs_in[ob][1];
                    q.key = (uint32_t)ob * 3u * (uint32_t)((size_t)P.npix * (size_t)P.npix) + pix;
                    q.c[0] = (double)c3[0];
                    q.c[1] = (double)c3[1];
                    q.c[2] = (double)c3[2];
                    sur_q[(size_t)(i >> 6) * 64 * (size_t)P.n_obs + queued + (uint32_t)__popcll(m & lanes_below_mask())] = q;
                }
                queued += (uint32_t)__popcll(m);
            }
            {
                // slot layout: blocks of 64 rays, one observer per block, observers
                // cycling between blocks: a wave walks 64 neighbouring packets'
                // rays toward one observer while concurrent waves spread their
                // image writes over all observers.  Invisible rays and the lanes
                // past the end of the list are marked.
                PeelRay<R> r;
                r.p[0] = s.p[0]; r.p[1] = s.p[1]; r.p[2] = s.p[2];
                r.c[0] = c3[0]; r.c[1] = c3[1]; r.c[2] = c3[2];
                r.pix = (valid && vis && !use) ? pix : kNoPixel;   // a queued ray is not walked
                r.obs = (uint32_t)ob;
                peels[peel_slot(i, ob, P.n_obs)] = r;
            }
        }
        if constexpr (SUR) {
            if (lane == 0) sur_n[i >> 6] = queued;
        }
        if (valid && order < P.max_orders) {   // never for the deferred scatterings (order = max_orders)
            uint32_t x[3];
            seq_triple<KIND>(P.seq, state_idx(s.word), first_scatter_dim(SRC) + 3 * (order - 1), x);
            scatter_packet<R>(V, s, n_ax, x);
            pks[i] = s;
        }
    }
    if constexpr (SUR)
        flush_counters<5>(P.counters, {CNT_SCATTERINGS, CNT_OCCLUDED, CNT_SURROGATE, CNT_FALLBACKS, CNT_PEELS},
                          {n_scat, n_occ, n_sur, n_fb, n_sur});
    else
        flush_counters<2>(P.counters, {CNT_SCATTERINGS, CNT_OCCLUDED}, {n_scat, n_occ});
}

__device__ __forceinline__ KeyFrame box_key_frame(const DevGrid &g)
{
    KeyFrame f;
    for (int a = 0; a < 3; ++a) {
        f.lo[a] = (float)g.lo[a];
        f.scale[a] = (float)(32.0 / (g.hi[a] - g.lo[a]));
    }
    return f;
}

// The keys that k_tail stored beside its deferred scatterings (region layout,
// 0xFFFF for entries reserved but not deferred), gathered in list order for the
// sort; the scatterings' count goes to n_def_all.
__global__ void __launch_bounds__(256) k_def_keys(const uint32_t *__restrict__ region_keys, Queues *__restrict__ Q,
                                                  uint32_t def_cap, uint32_t *__restrict__ keys)
{
    const DeferredList D = deferred_list(Q, def_cap);
    const uint32_t n = (uint32_t)D.end[kPoolParts - 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) Q->n_def_all[0] = n;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        keys[i] = region_keys[deferred_slot(D, i)];
}

// --------------------------------------------------------------------------
// walks of one order: peel-off rays and flights
// --------------------------------------------------------------------------
enum WalkItem : int { WI_NONE = 0, WI_PEEL = 1, WI_MOVE = 2 };

// FLIGHTS = false builds the walk of peel rays alone (the deferred scatterings'
// peel rays): without the stop test and the appends it needs 114 VGPRs in FP32
// instead of 152, so four waves per SIMD are resident instead of three.  Those
// rays come sorted by position and gain from the extra waves; the per-order
// walks, whose flights gather incoherently, keep the full kernel at three.
template <typename R, bool FLIGHTS>
__global__ void __launch_bounds__(256) k_walk(const TransportParams P, int order,
                                              const PacketState<R> *__restrict__ pks, int in,
                                              PacketState<R> *__restrict__ out, const PeelRay<R> *__restrict__ peels,
                                              Queues *__restrict__ Q)
{
    __shared__ R s_o[kMaxObs][3];
    __shared__ double s_merge[4][64][3];   // per wave: pixel merge of the image contributions
    for (int i = threadIdx.x; i < P.n_obs; i += blockDim.x)
        for (int a = 0; a < 3; ++a) s_o[i][a] = (R)P.obs[i].o[a];
    __syncthreads();
    const RayGrid<R> G = ray_grid<R>(P.grid);
    const uint64_t n_live = Q->n_live[in];
    const uint64_t n_peel = (uint64_t)P.n_obs * 64 * ((n_live + 63) / 64);
    const uint64_t n_move = FLIGHTS && order < P.max_orders ? n_live : 0;
    const uint64_t total = n_peel + n_move;
    const uint64_t stride = block_stride(total >> kOrderBlockLog2);
    const size_t plane = (size_t)P.npix * (size_t)P.npix;
    // image copy of this block (blocks go round-robin to the XCDs), in the
    // set of this scattering order when orders are kept apart
    double *img_copy = image_copy(P, order, plane);
    const int key_bits = bits_for((uint64_t)P.n_obs * 3 * plane);
    uint64_t n_visits = 0;
    uint32_t n_peels = 0, n_esc = 0;
    int kind = WI_NONE;
    uint32_t slot = 0, pix = 0, obs = 0;
    R c3[3] = {(R)0, (R)0, (R)0};
    Walk<R> W;
    W.done = true;
    WorkPool pool;
    for (;;) {
        // packets whose flight stopped inside the mesh go to the next live list, in place pos
        const bool append = FLIGHTS && W.done && kind == WI_MOVE && W.stopped;
        const uint32_t pos = FLIGHTS ? wave_append(append, &Q->n_live[in ^ 1]) : 0u;
        const bool peel_done = W.done && kind == WI_PEEL;
        if (__ballot(peel_done) != 0) {
            double v[3] = {0.0, 0.0, 0.0};
            if (peel_done) {
                n_visits += W.visits;
                n_peels++;
                const double att = exp(-W.tau);
                v[0] = att * (double)c3[0];
                v[1] = att * (double)c3[1];
                v[2] = att * (double)c3[2];
                kind = WI_NONE;
            }
            // the key is the offset of the pixel's I value in the image set [obs][3][plane]
            const uint32_t key = peel_done ? obs * 3u * (uint32_t)plane + pix : 0u;
            wave_merge_add(peel_done, key, v[0], v[1], v[2], img_copy, plane, key_bits, s_merge[threadIdx.x >> 6]);
        }
        if (FLIGHTS && W.done && kind == WI_MOVE) {
            n_visits += W.visits;
            if (append) {
                PacketState<R> s = pks[slot];
                for (int a = 0; a < 3; ++a) s.p[a] = s.p[a] + W.t_out * s.k[a];
                out[pos] = s;
            } else {
                n_esc++;
            }
            kind = WI_NONE;
        }
        uint64_t item = 0;
        if (pool.take(kind == WI_NONE, total, &Q->work[1][0][0], item)) {
            item = scatter_block(item, total, stride);
            if (item < n_peel) {
                const PeelRay<R> r = peels[item];
                if (r.pix != kNoPixel) {
                    const R o[3] = {s_o[r.obs][0], s_o[r.obs][1], s_o[r.obs][2]};
                    c3[0] = r.c[0]; c3[1] = r.c[1]; c3[2] = r.c[2];
                    pix = r.pix;
                    obs = r.obs;
                    walk_begin(W, G, r.p, o, WALK_EDGE, 0.0);
                    kind = WI_PEEL;
                }
            } else if constexpr (FLIGHTS) {
                slot = (uint32_t)(item - n_peel);
                const PacketState<R> *ps = pks + slot;
                const R p0[3] = {ps->p[0], ps->p[1], ps->p[2]};
                const R k0[3] = {ps->k[0], ps->k[1], ps->k[2]};
                walk_begin(W, G, p0, k0, WALK_MOVE, ps->target);
                kind = WI_MOVE;
            }
        }
        if (__ballot(kind != WI_NONE) == 0) {
            if (pool.dry) break;
            continue;   // every item just taken was an invisible peel ray
        }
        if (!FLIGHTS || __ballot(kind == WI_MOVE) == 0) {
            // no lane moves to a target: walks to the edge only
            for (;;) {
                walk_batch_edge<R, kFlightBatch>(W, G);
                if (__popcll(__ballot(W.done || kind == WI_NONE)) >= kWaveRefill) break;
            }
        } else if constexpr (FLIGHTS) {
            for (;;) {
                walk_batch<R, kFlightBatch>(W, G);
                if (__popcll(__ballot(W.done || kind == WI_NONE)) >= kWaveRefill) break;
            }
        }
    }
    flush_counters<4>(P.counters, {CNT_VISITS, CNT_PEELS, CNT_PEEL_RAYS, CNT_ESCAPES}, {n_visits, n_peels, n_peels, n_esc});
}

// Peel-off rays of a walk launch without flights (the last scattering order),
// when the image set of the order fits in LDS: each block accumulates its rays'
// contributions into an FP64 image tile in LDS (LDS atomics), then adds the
// tile into its image copy once, with coalesced atomics.  Every contribution
// that k_walk would add to the global image is added to the tile instead, so
// the images differ only in the order of the FP64 sums.  Global atomics per
// launch fall from three per visible ray to three per pixel and block; for a
// 64^2 image these scattered atomics were most of the walk's time.  One block
// per CU (the tile takes most of the LDS) of 16 waves; peel rays walk to the
// edge only, so the kernel needs no stop test and few registers.
constexpr int kPeelLdsThreads = 1024;

template <typename R>
__global__ void __launch_bounds__(kPeelLdsThreads) k_walk_peel_lds(const TransportParams P, int order, int in,
                                                                  const PeelRay<R> *__restrict__ peels,
                                                                  Queues *__restrict__ Q)
{
    extern __shared__ double tile[];   // [n_obs][3][npix][npix]
    __shared__ R s_o[kMaxObs][3];
    const size_t plane = (size_t)P.npix * (size_t)P.npix;
    const size_t n_tile = (size_t)P.n_obs * 3 * plane;
    for (size_t i = threadIdx.x; i < n_tile; i += blockDim.x) tile[i] = 0.0;
    for (int i = threadIdx.x; i < P.n_obs; i += blockDim.x)
        for (int a = 0; a < 3; ++a) s_o[i][a] = (R)P.obs[i].o[a];
    __syncthreads();
    const RayGrid<R> G = ray_grid<R>(P.grid);
    const uint64_t n_live = Q->n_live[in];
    const uint64_t total = (uint64_t)P.n_obs * 64 * ((n_live + 63) / 64);
    const uint64_t stride = block_stride(total >> kOrderBlockLog2);
    uint64_t n_visits = 0;
    uint32_t n_peels = 0;
    bool busy = false;
    uint32_t pix = 0, obs = 0;
    R c3[3] = {(R)0, (R)0, (R)0};
    Walk<R> W;
    W.done = true;
    WorkPool pool;
    for (;;) {
        if (W.done && busy) {
            n_visits += W.visits;
            n_peels++;
            const double att = exp(-W.tau);
            double *dst = tile + (size_t)obs * 3 * plane + (size_t)pix;
            atomicAdd(dst, att * (double)c3[0]);
            atomicAdd(dst + plane, att * (double)c3[1]);
            atomicAdd(dst + 2 * plane, att * (double)c3[2]);
            busy = false;
        }
        uint64_t item = 0;
        if (pool.take(!busy, total, &Q->work[1][0][0], item)) {
            item = scatter_block(item, total, stride);
            const PeelRay<R> r = peels[item];
            if (r.pix != kNoPixel) {
                const R o[3] = {s_o[r.obs][0], s_o[r.obs][1], s_o[r.obs][2]};
                c3[0] = r.c[0]; c3[1] = r.c[1]; c3[2] = r.c[2];
                pix = r.pix;
                obs = r.obs;
                walk_begin(W, G, r.p, o, WALK_EDGE, 0.0);
                busy = true;
            }
        }
        if (__ballot(busy) == 0) {
            if (pool.dry) break;
            continue;   // every item just taken was an invisible peel ray
        }
        for (;;) {
            // FP64 steps take twice the registers: four steps per load batch keep 16 waves per CU
            // within 128 registers without spilling
            walk_batch_edge<R, sizeof(R) == 8 ? 4 : kFlightBatch>(W, G);
            if (__popcll(__ballot(W.done || !busy)) >= kWaveRefill) break;
        }
    }
    __syncthreads();
    double *img_copy = image_copy(P, order, plane);
    for (size_t i = threadIdx.x; i < n_tile; i += blockDim.x) {
        const double v = tile[i];
        if (v != 0.0) unsafeAtomicAdd(img_copy + i, v);
    }
    flush_counters<3>(P.counters, {CNT_VISITS, CNT_PEELS, CNT_PEEL_RAYS}, {n_visits, n_peels, n_peels});
}

// --------------------------------------------------------------------------
// late orders in one launch
// --------------------------------------------------------------------------
// Scattering orders order0 .. max_orders of the packets live after order
// order0 - 1, in one launch.  A lane takes a packet and carries it through its
// remaining orders: at each scattering the packet's state is appended to the
// list of deferred scatterings (one atomic per wave; the list is split into
// one region per XCD, and the sort key of the scattering's position goes to
// region_keys at the same place), the albedo and the new
// direction and flight depth are applied as k_scatter applies them, and the
// flight is walked as k_walk walks it, up to the next scattering where it
// stopped inside the mesh.  The peel-offs of the deferred scatterings are left
// to one k_scatter launch over the list after this kernel (converged, with the
// peel rays in fixed slots), then one walk launch; per-order launches would
// run these orders at low occupancy, each ended by its longest walk.  A wave
// whose reservation does not fit the list computes its scatterings' peel-offs
// itself and walks their rays to the edge at once (the reserved slots that fit
// are marked kNoState); in the surrogate mode those rays all walk exactly and
// count as fall-backs.  Lanes go back to the pool as their packets end
// (coherence among the few late packets is low anyway): a wave stops walking
// once kTailDoneEighths eighths of its flights have ended.  Every packet gets
// the arithmetic of the per-order launches, so images differ only in the order
// of the FP64 sums.
template <typename R, int KIND, int SRC, bool SUR>
// three waves per SIMD in FP32 (168 VGPRs, no spills; the compiler's own choice
// of 173 left two)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 1))) k_tail(const TransportParams P, int order0,
                                              const PacketState<R> *__restrict__ pks, int in,
                                              PacketState<R> *__restrict__ states, uint32_t state_cap,
                                              uint32_t *__restrict__ region_keys, Queues *__restrict__ Q)
{
    const KeyFrame kf = box_key_frame(P.grid);
    __shared__ ObsTable<R> T;
    load_obs(P, T);
    const RayGrid<R> G = ray_grid<R>(P.grid);
    const SceneView<R> V = scene_view<R>(P, SRC);
    const uint64_t n = Q->n_live[in];
    const size_t plane = (size_t)P.npix * (size_t)P.npix;
    double *img_copy = image_copy(P, order0, plane);
    const int lane = (int)(threadIdx.x & 63);
    // the deferred scatterings of this block: the region of its work-pool part (XCD)
    const int region = (int)(blockIdx.x % kPoolParts);
    PacketState<R> *sreg = states + (size_t)region * state_cap;
    uint32_t *sreg_n = &Q->n_def[region][0];
    uint64_t n_visits = 0;
    uint32_t n_scat = 0, n_occ = 0, n_esc = 0, n_peels = 0, n_fb = 0;
    PacketState<R> s = {};
    int order = 0;
    bool has = false, moving = false, at_scatter = false;
    Walk<R> W = {};
    W.done = true;
    WorkPool pool;
    for (;;) {
        // flights that ended: scatter where they stopped, or the packet left
        if (moving && W.done) {
            n_visits += W.visits;
            if (W.stopped) {
                for (int a = 0; a < 3; ++a) s.p[a] = s.p[a] + W.t_out * s.k[a];
                ++order;
                at_scatter = true;
            } else {
                n_esc++;
                has = false;
            }
            moving = false;
        }
        uint64_t item = 0;
        if (pool.take(!has, n, &Q->work[2][0][0], item)) {
            s = pks[item];
            order = order0;
            has = true;
            at_scatter = true;
        }
        if (__ballot(has) == 0 && pool.dry) break;
        const uint64_t ms = __ballot(at_scatter);
        if (ms != 0) {
            // the scattering's state (before the albedo) to the deferred list
            const uint32_t cnt = (uint32_t)__popcll(ms);
            uint32_t sbase = 0;
            if (lane == 0) sbase = atomicAdd(sreg_n, cnt);
            sbase = __shfl(sbase, 0, 64);
            const bool fits = (uint64_t)sbase + cnt <= (uint64_t)state_cap;
            if (at_scatter) {
                const uint32_t slot = sbase + (uint32_t)__popcll(ms & lanes_below_mask());
                if (slot < state_cap) {
                    PacketState<R> d = s;
                    d.word = with_order(d.word, fits ? (uint32_t)order : kNoState);
                    sreg[slot] = d;
                    region_keys[(size_t)region * state_cap + slot] = fits ? cell_key(kf, s.p) : 0xFFFFu;
                }
            }
            R n_ax[3] = {(R)0, (R)0, (R)0};
            if (at_scatter) {
                s.S[0] *= V.albedo; s.S[1] *= V.albedo; s.S[2] *= V.albedo;
                cross3(s.k, s.m, n_ax);
            }
            if (!fits) {
                // the list is full: this wave's scatterings peel off here
                if (at_scatter) n_scat++;
                for (int ob = 0; ob < P.n_obs; ++ob) {
                    bool vis = false, occ = false;
                    R c3[3] = {(R)0, (R)0, (R)0};
                    uint32_t pix = 0;
                    const R o[3] = {T.o[ob][0], T.o[ob][1], T.o[ob][2]};
                    if (at_scatter) {
                        const R ex[3] = {T.ex[ob][0], T.ex[ob][1], T.ex[ob][2]};
                        const R ey[3] = {T.ey[ob][0], T.ey[ob][1], T.ey[ob][2]};
                        peel_contribution<R>(V, s, n_ax, o, ex, ey, vis, occ, c3, pix);
                        n_occ += occ ? 1u : 0u;
                    }
                    if (vis) {
                        if constexpr (SUR) n_fb++;
                        // W is free: this lane's flight has ended
                        walk_begin(W, G, s.p, o, WALK_EDGE, 0.0);
                        walk_run<R, kFlightBatch>(W, G);
                        n_visits += W.visits;
                        n_peels++;
                        const double att = exp(-W.tau);
                        double *dst = img_copy + (size_t)ob * 3 * plane + pix;
                        unsafeAtomicAdd(dst, att * (double)c3[0]);
                        unsafeAtomicAdd(dst + plane, att * (double)c3[1]);
                        unsafeAtomicAdd(dst + 2 * plane, att * (double)c3[2]);
                    }
                }
            }
            if (at_scatter) {
                if (order < P.max_orders) {
                    uint32_t x[3];
                    seq_triple<KIND>(P.seq, state_idx(s.word), first_scatter_dim(SRC) + 3 * (order - 1), x);
                    scatter_packet<R>(V, s, n_ax, x);
                    walk_begin(W, G, s.p, s.k, WALK_MOVE, s.target);
                    moving = true;
                } else {
                    has = false;   // the last order scatters without a flight
                }
                at_scatter = false;
            }
        }
        const int movers = __popcll(__ballot(moving));
        if (movers == 0) continue;
        for (;;) {
            // only lanes with a flight under way step (the call's own test of W.done
            // alone gave visit counts that varied from run to run in this kernel)
            if (moving && !W.done) walk_batch<R, kTailBatch>(W, G);
            if (8 * __popcll(__ballot(moving && W.done)) >= kTailDoneEighths * movers) break;
        }
    }
    if constexpr (SUR)
        flush_counters<7>(P.counters,
                          {CNT_VISITS, CNT_SCATTERINGS, CNT_OCCLUDED, CNT_ESCAPES, CNT_PEELS, CNT_PEEL_RAYS,
                           CNT_FALLBACKS},
                          {n_visits, n_scat, n_occ, n_esc, n_peels, n_peels, n_fb});
    else
        flush_counters<6>(P.counters,
                          {CNT_VISITS, CNT_SCATTERINGS, CNT_OCCLUDED, CNT_ESCAPES, CNT_PEELS, CNT_PEEL_RAYS},
                          {n_visits, n_scat, n_occ, n_esc, n_peels, n_peels});
}

// Blocks and dynamic LDS bytes of k_walk_peel_lds for an image set of `bytes`,
// or 0 blocks when the set does not fit one block's LDS on this device.
template <typename R>
static int peel_lds_blocks(size_t bytes)
{
    static int max_lds = -1, attr_set = 0;
    if (max_lds < 0) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        max_lds = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess ? v : 0;
    }
    // static LDS of the kernel: observer directions and the counter sums
    const size_t reserve = 1024;
    if (bytes + reserve > (size_t)max_lds) return 0;
    if (!attr_set) {
        attr_set = hipFuncSetAttribute((const void *)k_walk_peel_lds<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds - (int)reserve) == hipSuccess ? 1 : -1;
    }
    if (attr_set < 0) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_walk_peel_lds<R>, kPeelLdsThreads, bytes) !=
            hipSuccess || per_cu < 1)
        return 0;
    return per_cu * device_cu_count();
}

// Pilot capture: (position, observer) of every visible peel ray inside the
// surrogate domain, appended while the buffer has room (the count goes on).
template <typename R>
__global__ void __launch_bounds__(256) k_capture(const TransportParams P, const PeelRay<R> *__restrict__ peels,
                                                 const Queues *__restrict__ Q, int in)
{
    const uint64_t n_live = Q->n_live[in];
    const uint64_t n_slots = (uint64_t)P.n_obs * 64 * ((n_live + 63) / 64);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t base = t0 - (threadIdx.x & 63); base < n_slots; base += stride) {
        const uint64_t i = base + (threadIdx.x & 63);
        bool take = false;
        PeelRay<R> r = {};
        if (i < n_slots) {
            r = peels[i];
            take = r.pix != kNoPixel && dom_cell(P.sur, (double)r.p[0], (double)r.p[1], (double)r.p[2]) >= 0;
        }
        const uint32_t pos = wave_append(take, P.sur.cap_count);
        if (take && pos < P.sur.cap_capacity) {
            float *c = P.sur.cap + (size_t)pos * 4;
            c[0] = (float)r.p[0];
            c[1] = (float)r.p[1];
            c[2] = (float)r.p[2];
            c[3] = (float)r.obs;
        }
    }
}

// --------------------------------------------------------------------------
// launch sequence
// --------------------------------------------------------------------------
template <typename F>
static int resident_blocks_of(F kernel)
{
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    (void)hipGetDevice(&dev);
    int cus = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
    return per_cu * cus;
}

template <typename R, int KIND, int SRC>
static hipError_t run_chunk(const TransportParams &P, uint64_t first, uint32_t count, const TransportBuffers &B,
                            hipStream_t st, KernelTimer *T)
{
    static int nb_first = 0, nb_scatter = 0, nb_walk = 0, nb_walk_peels = 0, nb_net = 0, nb_tail = 0, nb_tail_sur = 0;
    if (!nb_first) {
        nb_first = resident_blocks_of(k_first<R, KIND, SRC>);
        nb_scatter = resident_blocks_of(k_scatter<R, KIND, SRC, false>);
        nb_walk = resident_blocks_of(k_walk<R, true>);
        nb_walk_peels = resident_blocks_of(k_walk<R, false>);
        nb_net = resident_blocks_of(k_peel_net);
        nb_tail = resident_blocks_of(k_tail<R, KIND, SRC, false>);
        nb_tail_sur = resident_blocks_of(k_tail<R, KIND, SRC, true>);
    }
    PeelRay<R> *peels = (PeelRay<R> *)B.peels;
    const int walk_blocks = std::min(nb_walk, kWalkBlocksPerCu * device_cu_count());
    const uint32_t cblocks = (count + 255) / 256;
    const int b_elem = (int)(cblocks < 2048u ? cblocks : 2048u);
    hipError_t e = launch_clear_queues(B.q, st, T);
    if (e != hipSuccess) return e;
    // first flights in emission-direction order
    {
        TimedLaunch tl(T, st, TC_SORT);
        hipLaunchKernelGGL((k_key_emit<R, KIND, SRC>), dim3(b_elem), dim3(256), 0, st, P, first, count, B.keys);
    }
    if ((e = launch_sort_keys(B, count, st, T)) != hipSuccess) return e;
    const int bf = (int)(cblocks < (uint32_t)nb_first ? cblocks : (uint32_t)nb_first);
    {
        TimedLaunch tl(T, st, TC_FIRST);
        hipLaunchKernelGGL((k_first<R, KIND, SRC>), dim3(bf), dim3(256), 0, st, P, first, count,
                           (const uint32_t *)B.order, state_list<R>(B, 0), B.q);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int bs = (int)(cblocks < (uint32_t)nb_scatter ? cblocks : (uint32_t)nb_scatter);
    const size_t tile_bytes = (size_t)P.n_obs * 3 * (size_t)P.npix * (size_t)P.npix * sizeof(double);
    // orders from `tail` on run in one launch, their peel rays deferred to one walk
    // (exact peel-offs with one image set only)
    const bool tail_on = P.tail_from >= 2 && P.tail_from <= P.max_orders && !P.sur.cap && P.order_images == 0;
    const int last = tail_on ? P.tail_from - 1 : P.max_orders;
    for (int order = 1; order <= last; ++order) {
        const int in = (order - 1) & 1;
        {
            TimedLaunch tl(T, st, TC_SCATTER);
            if (P.peel_mode == 1)
                hipLaunchKernelGGL((k_scatter<R, KIND, SRC, true>), dim3(bs), dim3(256), 0, st, P, order,
                                   state_list<R>(B, in), in, peels, B.sur_q, B.sur_n, B.q, 0u,
                                   (const uint32_t *)nullptr);
            else
                hipLaunchKernelGGL((k_scatter<R, KIND, SRC, false>), dim3(bs), dim3(256), 0, st, P, order,
                                   state_list<R>(B, in), in, peels, B.sur_q, B.sur_n, B.q, 0u,
                                   (const uint32_t *)nullptr);
        }
        if (P.peel_mode == 1) {
            TimedLaunch tl(T, st, TC_PEEL_MLP);
            hipLaunchKernelGGL(k_peel_net, dim3(nb_net), dim3(256), 0, st, P, order, in, (const SurQuery *)B.sur_q,
                               (const uint32_t *)B.sur_n, (const Queues *)B.q);
        }
        if (P.sur.cap) {
            TimedLaunch tl(T, st, TC_OTHER);
            hipLaunchKernelGGL((k_capture<R>), dim3(bs), dim3(256), 0, st, P, (const PeelRay<R> *)peels,
                               (const Queues *)B.q, in);
        }
        // the last order walks peel rays only (no flights): those want every resident
        // wave, and an image set that fits in LDS is summed there first
        const int wb = order < P.max_orders ? walk_blocks : nb_walk;
        const int lds_blocks = order == P.max_orders ? peel_lds_blocks<R>(tile_bytes) : 0;
        {
            TimedLaunch tl(T, st, TC_WALK);
            if (lds_blocks > 0)
                hipLaunchKernelGGL((k_walk_peel_lds<R>), dim3(lds_blocks), dim3(kPeelLdsThreads), tile_bytes, st, P,
                                   order, in, (const PeelRay<R> *)peels, B.q);
            else
                hipLaunchKernelGGL((k_walk<R, true>), dim3(wb), dim3(256), 0, st, P, order,
                                   (const PacketState<R> *)state_list<R>(B, in), in, state_list<R>(B, in ^ 1),
                                   (const PeelRay<R> *)peels, B.q);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (tail_on) {
        const int in = last & 1;   // the live list of order `tail`; the other list takes the deferred scatterings
        // as many as the list, the peel slots (64 n_obs per 64 scatterings) and, in the
        // surrogate mode, the query queue hold
        uint64_t cap = B.cap;
        const uint64_t slot_groups = B.peel_bytes / sizeof(PeelRay<R>) / (64 * (uint64_t)P.n_obs);
        cap = std::min<uint64_t>(cap, 64 * slot_groups);
        if (P.peel_mode == 1) cap = std::min<uint64_t>(cap, 64 * (B.sur_entries / (64 * (uint64_t)P.n_obs)));
        if (P.def_limit) cap = std::min<uint64_t>(cap, P.def_limit);
        // in kPoolParts regions, one per work-pool part
        const uint32_t state_cap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap / kPoolParts, 0x1FFFFFFFull));
        const bool sur = P.peel_mode == 1;
        {
            TimedLaunch tl(T, st, TC_WALK);
            if (sur)
                hipLaunchKernelGGL((k_tail<R, KIND, SRC, true>), dim3(nb_tail_sur), dim3(256), 0, st, P, P.tail_from,
                                   (const PacketState<R> *)state_list<R>(B, in), in, state_list<R>(B, in ^ 1),
                                   state_cap, B.sort_tmp, B.q);
            else
                hipLaunchKernelGGL((k_tail<R, KIND, SRC, false>), dim3(nb_tail), dim3(256), 0, st, P, P.tail_from,
                                   (const PacketState<R> *)state_list<R>(B, in), in, state_list<R>(B, in ^ 1),
                                   state_cap, B.sort_tmp, B.q);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // the deferred scatterings in the order of their positions (the sort's count is
        // read on the device), then their peel-offs, as the last order's: scatter (no
        // new direction), the network in the surrogate mode, the walk of the peel rays
        const int din = in ^ 1;
        const uint32_t def_bound = (uint32_t)std::min<uint64_t>((uint64_t)kPoolParts * state_cap, B.cap);
        {
            TimedLaunch tl(T, st, TC_SORT);
            const int kb = (int)std::min<uint32_t>((def_bound + 255) / 256, 512u);
            hipLaunchKernelGGL(k_def_keys, dim3(kb), dim3(256), 0, st, (const uint32_t *)B.sort_tmp, B.q, state_cap,
                               B.keys);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const uint32_t *def_count = (const uint32_t *)((const char *)B.q + offsetof(Queues, n_def_all));
        if ((e = launch_sort_keys(B, def_bound, st, T, def_count)) != hipSuccess) return e;
        {
            TimedLaunch tl(T, st, TC_SCATTER);
            if (sur)
                hipLaunchKernelGGL((k_scatter<R, KIND, SRC, true>), dim3(nb_scatter), dim3(256), 0, st, P,
                                   P.max_orders, state_list<R>(B, din), din, peels, B.sur_q, B.sur_n, B.q,
                                   state_cap, (const uint32_t *)B.order);
            else
                hipLaunchKernelGGL((k_scatter<R, KIND, SRC, false>), dim3(nb_scatter), dim3(256), 0, st, P,
                                   P.max_orders, state_list<R>(B, din), din, peels, B.sur_q, B.sur_n, B.q,
                                   state_cap, (const uint32_t *)B.order);
        }
        if (sur) {
            TimedLaunch tl(T, st, TC_PEEL_MLP);
            hipLaunchKernelGGL(k_peel_net, dim3(nb_net), dim3(256), 0, st, P, P.max_orders, din,
                               (const SurQuery *)B.sur_q, (const uint32_t *)B.sur_n, (const Queues *)B.q);
        }
        const int lds_blocks = peel_lds_blocks<R>(tile_bytes);
        {
            TimedLaunch tl(T, st, TC_WALK);
            if (lds_blocks > 0)
                hipLaunchKernelGGL((k_walk_peel_lds<R>), dim3(lds_blocks), dim3(kPeelLdsThreads), tile_bytes, st, P,
                                   P.max_orders, din, (const PeelRay<R> *)peels, B.q);
            else
                hipLaunchKernelGGL((k_walk<R, false>), dim3(nb_walk_peels), dim3(256), 0, st, P, P.max_orders,
                                   (const PacketState<R> *)state_list<R>(B, din), din, state_list<R>(B, in),
                                   (const PeelRay<R> *)peels, B.q);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R, int KIND>
static hipError_t run_src(const TransportParams &P, uint64_t first, uint32_t count, const TransportBuffers &B,
                          hipStream_t st, KernelTimer *T)
{
    if (P.src_kind == 1) return run_chunk<R, KIND, 1>(P, first, count, B, st, T);
    if (P.src_kind == 2) return run_chunk<R, KIND, 2>(P, first, count, B, st, T);
    return run_chunk<R, KIND, 0>(P, first, count, B, st, T);
}

template <typename R>
static hipError_t run_kind(const TransportParams &P, int kind, uint64_t first, uint32_t count,
                           const TransportBuffers &B, hipStream_t st, KernelTimer *T)
{
    switch (kind) {
    case SEQ_SOBOL: return run_src<R, SEQ_SOBOL>(P, first, count, B, st, T);
    case SEQ_HALTON: return run_src<R, SEQ_HALTON>(P, first, count, B, st, T);
    case SEQ_NIED2: return run_src<R, SEQ_NIED2>(P, first, count, B, st, T);
    case SEQ_HAMMERSLEY: return run_src<R, SEQ_HAMMERSLEY>(P, first, count, B, st, T);
    case SEQ_PHILOX: return run_src<R, SEQ_PHILOX>(P, first, count, B, st, T);
    case SEQ_FAURE: return run_src<R, SEQ_FAURE>(P, first, count, B, st, T);
    case SEQ_SOBOL_OWEN: return run_src<R, SEQ_SOBOL_OWEN>(P, first, count, B, st, T);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_transport(const TransportParams &P, int precision, int kind, uint64_t first, uint64_t count,
                            const TransportBuffers &B, hipStream_t stream, KernelTimer *timer)
{
    for (uint64_t done = 0; done < count;) {
        const uint32_t n = (uint32_t)(count - done < kChunk ? count - done : kChunk);
        hipError_t e = precision == 1 ? run_kind<double>(P, kind, first + done, n, B, stream, timer)
                                      : run_kind<float>(P, kind, first + done, n, B, stream, timer);
        if (e != hipSuccess) return e;
        done += n;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- queue counters
// The queue counters of a chunk start at zero.  A kernel clears them rather
// than a memset node, so that a launch sequence captured into a graph replays
// the clear like its other kernels.
static_assert(sizeof(Queues) % 4 == 0, "the queue counters are whole words");

__global__ void __launch_bounds__(256) k_clear_words(uint32_t *__restrict__ p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

hipError_t launch_clear_queues(Queues *q, hipStream_t stream, KernelTimer *timer)
{
    TimedLaunch tl(timer, stream, TC_OTHER);
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(256), 0, stream, (uint32_t *)q, (uint32_t)(sizeof(Queues) / 4));
    return hipGetLastError();
}

// ---------------------------------------------------------------- image copies
// add copies 1.. into copy 0 and clear them
__global__ void __launch_bounds__(256) k_fold_images(double *__restrict__ img, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double s = img[i];
        for (int c = 1; c < kImageCopies; ++c) {
            s += img[c * n + i];
            img[c * n + i] = 0.0;
        }
        img[i] = s;
    }
}

hipError_t launch_fold_images(double *img, size_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    size_t need = (n + 255) / 256;
    int blocks = (int)(need < 4096 ? need : 4096);
    hipLaunchKernelGGL(k_fold_images, dim3(blocks), dim3(256), 0, stream, img, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- mesh layout
// x-fastest cells [nz][ny][nx] into 4x4x4 bricks (the destination is cleared
// beforehand: cells past the mesh edge stay 0)
__global__ void __launch_bounds__(256) k_to_bricks(const float *__restrict__ src, float *__restrict__ dst, int nx,
                                                   int ny, int nz, int nbx, int nby)
{
    const size_t n = (size_t)nx * ny * nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % (size_t)nx);
        const size_t r = i / (size_t)nx;
        const int y = (int)(r % (size_t)ny);
        const int z = (int)(r / (size_t)ny);
        dst[brick_index(x, y, z, nbx, nby)] = src[i];
    }
}

hipError_t launch_to_bricks(const float *src, float *dst, int nx, int ny, int nz, hipStream_t stream)
{
    const size_t n = (size_t)nx * ny * nz;
    if (n == 0) return hipSuccess;
    const size_t need = (n + 255) / 256;
    const int blocks = (int)(need < 8192 ? need : 8192);
    int nb[3];
    mesh_bricks(nx, ny, nz, nb);
    hipLaunchKernelGGL(k_to_bricks, dim3(blocks), dim3(256), 0, stream, src, dst, nx, ny, nz, nb[0], nb[1]);
    return hipGetLastError();
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

// Batched transport: many uneven scenes in one launch sequence.
//
// Every scene of a batch has its own mesh, source, dust, observers (up to 4),
// image and packet range; the packets of all scenes share one numbering and
// run through the same kernels as one work queue.  Each lane looks up the
// scene of its packet (a binary search over the scenes' first batch numbers)
// and walks that scene's mesh through a plain pointer.  The per-packet
// physics is that of the single-scene transport (qrt_transport.hip): emission
// (Sec. 3.2, 3.3), tau1 and the forced first scattering (Sec. 3.2), moves and
// peel-off walks (Sec. 3.4, 3.6), Henyey-Greenstein scattering with White's
// Mueller matrix (Sec. 2.2, 3.5), coordinates by purpose (Sec. 3.7).
//
// Launch sequence of a chunk of batch numbers: emission keys (scene and
// coarse emission direction) -> radix sort -> persistent first flight
// -> per order up to the largest order of the batch: scatter, then walk.  A
// packet whose scene has fewer orders stops at its own last order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstddef>

#include "qrt_internal.h"
#include "qrt_packet.h"
#include "qrt_physics.h"
#include "qrt_wave.h"

namespace qrt {

// scene of batch number b: the last scene whose first batch number is <= b
__device__ __forceinline__ int batch_scene(const BatchParams &P, uint64_t b)
{
    int lo = 0, hi = P.n_scenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.scenes[mid].begin <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename R>
__device__ __forceinline__ LaneGrid<R> lane_grid(const BScene &S)
{
    LaneGrid<R> G;
    G.kr = S.kr;
    G.nbx = S.nb[0];
    G.nby = S.nb[1];
    axis_masks(S.nb[0], S.nb[1], G.m);
    for (int a = 0; a < 3; ++a) {
        G.n[a] = S.n[a];
        G.lo[a] = (R)S.lo[a];
        G.h[a] = (R)S.h[a];
    }
    return G;
}

__device__ __forceinline__ SeqParams scene_seq(const BatchParams &P, const BScene &S)
{
    SeqParams q = P.seq;
    q.n_total = S.n_total;
    return q;
}

// Emission of a packet of scene S: the single-scene emission with the scene's source.
template <typename R, int KIND>
__device__ __forceinline__ void batch_emit(const BScene &S, const SeqParams &q, uint64_t idx, R p[3], R k[3])
{
    emit_packet<R, KIND>(S.src_kind, S.src, S.r_star, q, idx, p, k);
}

template <typename R>
__device__ __forceinline__ SceneView<R> scene_view(const BScene &S)
{
    SceneView<R> V;
    V.g = (R)S.g;
    V.p_lin = (R)S.p_lin;
    V.albedo = (R)S.albedo;
    V.half_width = (R)S.half_width;
    V.npix = S.npix;
    V.src_kind = S.src_kind;
    for (int a = 0; a < 3; ++a) V.src[a] = (R)S.src[a];
    V.r_star2 = (R)(S.r_star * S.r_star);
    return V;
}

// ---------------------------------------------------------------- emission sort
template <typename R, int KIND>
__global__ void __launch_bounds__(256) k_bkey(const BatchParams P, uint64_t b0, uint32_t count,
                                              uint32_t *__restrict__ keys)
{
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < count; j += gridDim.x * blockDim.x) {
        const uint64_t b = b0 + j;
        const int s = batch_scene(P, b);
        const BScene &S = P.scenes[s];
        R p[3], k[3];
        batch_emit<R, KIND>(S, scene_seq(P, S), S.first + (b - S.begin), p, k);
        const uint32_t key = ((uint32_t)(s - P.scene_base) << (kSortBits - P.scene_bits)) |
                             (direction_key(k) >> P.scene_bits);
        keys[j] = key;
    }
}

// ---------------------------------------------------------------- first flight
enum BatchFirstPhase : int { BF_IDLE = 0, BF_EDGE = 1, BF_FORCED = 2 };

template <typename R, int KIND>
__global__ void __launch_bounds__(256) k_bfirst(const BatchParams P, uint64_t b0, uint32_t count,
                                                const uint32_t *__restrict__ order, const uint32_t *__restrict__ keys,
                                                PacketState<R> *__restrict__ out, Queues *__restrict__ Q)
{
    uint64_t n_visits = 0;
    uint32_t n_packets = 0, n_cuts = 0;
    int phase = BF_IDLE;
    uint32_t j = 0;
    int s = 0;
    R p[3] = {(R)0, (R)0, (R)0}, k[3] = {(R)0, (R)0, (R)1};
    R S0 = (R)0;
    LaneGrid<R> G = {};
    Walk<R> W;
    W.done = true;
    WorkPool pool;
    for (;;) {
        // packets whose forced flight ended go to the first live list, in place pos
        const bool append = W.done && phase == BF_FORCED;
        const uint32_t pos = wave_append(append, &Q->n_live[0]);
        if (W.done && phase == BF_EDGE) {
            n_visits += W.visits;
            const BScene &S = P.scenes[s];
            const double tau1 = W.tau;
            if (tau1 < S.tau_min) {
                n_cuts++;
                phase = BF_IDLE;
            } else {
                const double W1 = -expm1(-tau1);
                const uint64_t idx = S.first + (b0 + j - S.begin);
                const double u = (double)seq_point<KIND>(scene_seq(P, S), idx, forced_tau_dim(S.src_kind)) * 0x1p-32;
                S0 = (R)W1;
                walk_begin(W, G, p, k, WALK_MOVE, -log1p(-u * W1));
                phase = BF_FORCED;
            }
        } else if (append) {
            n_visits += W.visits;
            const BScene &S = P.scenes[s];
            PacketState<R> st;
            // the batch keeps the scene in the tag
            first_state<R>(p, k, W.t_out, S0, S.first + (b0 + j - S.begin), (uint32_t)s, st);
            out[pos] = st;
            phase = BF_IDLE;
        }
        uint64_t item = 0;
        if (pool.take(phase == BF_IDLE, count, &Q->work[0][0][0], item)) {
            j = order[item];
            // the sort key holds the scene relative to the chunk's first
            s = P.scene_base + (int)(keys[j] >> (kSortBits - P.scene_bits));
            const BScene &S = P.scenes[s];
            n_packets++;
            batch_emit<R, KIND>(S, scene_seq(P, S), S.first + (b0 + j - S.begin), p, k);
            G = lane_grid<R>(S);
            walk_begin(W, G, p, k, WALK_EDGE, 0.0);
            phase = BF_EDGE;
        }
        if (__ballot(phase != BF_IDLE) == 0 && pool.dry) break;
        if (__ballot(phase == BF_FORCED) == 0) {
            // no lane moves to a target: walks to the edge only
            for (;;) {
                walk_batch_edge<R, kBatchWalkBatch>(W, G);
                if (__popcll(__ballot(W.done || phase == BF_IDLE)) >= kWaveRefill) break;
            }
        } else {
            for (;;) {
                walk_batch<R, kBatchWalkBatch>(W, G);
                if (__popcll(__ballot(W.done || phase == BF_IDLE)) >= kWaveRefill) break;
            }
        }
    }
    flush_counters<4>(P.counters, {CNT_PACKETS, CNT_TAU_CUTS, CNT_VISITS, CNT_VISITS_FIRST},
                      {n_packets, n_cuts, n_visits, n_visits});
}

// ---------------------------------------------------------------- scattering
// Albedo, peel-off contributions toward the scene's observers and, unless it
// was the scene's last order, the new direction and flight.  A packet at its
// scene's last order gets target -1 and does not move.  Scenes have 1 to
// kBatchObs observers, so instead of fixed slots the visible peel rays are
// appended: each wave reserves room for all its rays with one atomic and lays
// them out observer by observer, so a wave's rays toward one observer stay
// contiguous and no slot is empty.  The 64-packet block b of the live list
// appends to group b % kPeelGroups, which has its own counter and region:
// a group receives at most ceil(blocks / kPeelGroups) blocks of at most
// 64 kBatchObs rays, which the host sizes group_cap for.  The observer field
// holds scene * 16 + observer.  def_cap > 0: the scatterings deferred by the
// late-order launch, in regions of def_cap, item i being state
// deferred_slot(perm[i]) (as in k_scatter), peel-offs only.
template <typename R, int KIND>
__global__ void __launch_bounds__(256) k_bscatter(const BatchParams P, int order, PacketState<R> *__restrict__ pks,
                                                  int in, PeelRay<R> *__restrict__ peels, Queues *__restrict__ Q,
                                                  uint32_t def_cap, const uint32_t *__restrict__ perm)
{
    if (blockIdx.x == 0 && threadIdx.x < kPoolParts) {
        if (threadIdx.x == 0) Q->n_live[in ^ 1] = 0;
        Q->work[1][threadIdx.x][0] = 0;
    }
    const DeferredList D = deferred_list(Q, def_cap);
    const uint32_t n = def_cap ? (uint32_t)D.end[kPoolParts - 1] : Q->n_live[in];
    if (def_cap && blockIdx.x == 0 && threadIdx.x == 0) Q->n_live[in] = n;
    const int lane = threadIdx.x & 63;
    const uint32_t wave0 = (blockIdx.x * blockDim.x + threadIdx.x) - (uint32_t)lane;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t n_scat = 0, n_occ = 0;
    for (uint32_t base = wave0; base < n; base += stride) {
        const uint32_t i = base + (uint32_t)lane;
        bool valid = i < n;
        PacketState<R> st = {};
        int s = 0;
        if (valid) {
            st = pks[def_cap ? deferred_slot(D, perm[i]) : i];
            valid = !def_cap || state_order(st.word) != kNoState;
        }
        if (valid) {
            s = (int)state_tag(st.word);
            n_scat++;
        }
        const BScene &S = P.scenes[s];
        const SceneView<R> V = scene_view<R>(S);
        if (valid) {
            st.S[0] *= V.albedo; st.S[1] *= V.albedo; st.S[2] *= V.albedo;
        }
        R n_ax[3];
        cross3(st.k, st.m, n_ax);
        bool visv[kBatchObs];
        R cv[kBatchObs][3];
        uint32_t pixv[kBatchObs];
#pragma unroll
        for (int ob = 0; ob < kBatchObs; ++ob) {
            bool vis = false, occ = false;
            R c3[3] = {(R)0, (R)0, (R)0};
            uint32_t pix = 0;
            if (valid && ob < S.n_obs) {
                const DevObserver &O = S.obs[ob];
                const R o[3] = {(R)O.o[0], (R)O.o[1], (R)O.o[2]};
                const R ex[3] = {(R)O.ex[0], (R)O.ex[1], (R)O.ex[2]};
                const R ey[3] = {(R)O.ey[0], (R)O.ey[1], (R)O.ey[2]};
                peel_contribution<R>(V, st, n_ax, o, ex, ey, vis, occ, c3, pix);
                n_occ += occ ? 1u : 0u;
            }
            visv[ob] = valid && vis;
            cv[ob][0] = c3[0]; cv[ob][1] = c3[1]; cv[ob][2] = c3[2];
            pixv[ob] = pix;
        }
        // one reservation for the wave's rays toward all observers
        uint64_t mv[kBatchObs];
        uint32_t total = 0;
#pragma unroll
        for (int ob = 0; ob < kBatchObs; ++ob) {
            mv[ob] = __ballot(visv[ob]);
            total += (uint32_t)__popcll(mv[ob]);
        }
        const uint32_t group = (base >> 6) % kPeelGroups;
        uint32_t at = 0;
        if (total) {
            // counters cleared by the walk of the previous order (or with the queues)
            if (lane == 0) at = atomicAdd(&Q->n_peel[order & 1][group][0], total);
            at = __shfl(at, 0, 64);
        }
        at += group * P.group_cap;
#pragma unroll
        for (int ob = 0; ob < kBatchObs; ++ob) {
            if (visv[ob]) {
                PeelRay<R> r;
                r.p[0] = st.p[0]; r.p[1] = st.p[1]; r.p[2] = st.p[2];
                r.c[0] = cv[ob][0]; r.c[1] = cv[ob][1]; r.c[2] = cv[ob][2];
                r.pix = pixv[ob];
                r.obs = ((uint32_t)s << 4) | (uint32_t)ob;
                peels[at + (uint32_t)__popcll(mv[ob] & lanes_below_mask())] = r;
            }
            at += (uint32_t)__popcll(mv[ob]);
        }
        if (valid) {
            if (order < S.max_orders) {
                uint32_t x[3];
                seq_triple<KIND>(scene_seq(P, S), state_idx(st.word), first_scatter_dim(S.src_kind) + 3 * (order - 1), x);
                scatter_packet<R>(V, st, n_ax, x);
            } else {
                st.target = -1.0;   // the scene's last scattering: no further flight
            }
            if (!def_cap) pks[i] = st;
        }
    }
    flush_counters<2>(P.counters, {CNT_SCATTERINGS, CNT_OCCLUDED}, {n_scat, n_occ});
}

// ---------------------------------------------------------------- walks of one order
enum BatchWalkItem : int { BW_NONE = 0, BW_PEEL = 1, BW_MOVE = 2 };

// FLIGHTS = false: the walk of the deferred scatterings' peel rays alone, with
// fewer registers (as k_walk's variant without flights).
template <typename R, bool FLIGHTS>
__global__ void __launch_bounds__(256) k_bwalk(const BatchParams P, int order,
                                               const PacketState<R> *__restrict__ pks, int in,
                                               PacketState<R> *__restrict__ out, const PeelRay<R> *__restrict__ peels,
                                               Queues *__restrict__ Q)
{
    if (blockIdx.x == 0 && threadIdx.x < kPeelGroups)
        Q->n_peel[(order + 1) & 1][threadIdx.x][0] = 0;   // next scatter
    // peel rays of the groups, numbered one group after the other
    uint32_t g_count[kPeelGroups];
    uint64_t n_peel = 0;
#pragma unroll
    for (int g = 0; g < kPeelGroups; ++g) {
        g_count[g] = Q->n_peel[order & 1][g][0];
        n_peel += g_count[g];
    }
    const uint64_t n_live = Q->n_live[in];
    const uint64_t n_move = FLIGHTS && order < P.max_orders ? n_live : 0;
    const uint64_t total = n_peel + n_move;
    const uint64_t stride = block_stride(total >> kOrderBlockLog2);
    __shared__ double s_merge[4][64][3];   // per wave: pixel merge of the image contributions
    uint64_t n_visits = 0;
    uint32_t n_peels = 0, n_esc = 0;
    int kind = BW_NONE;
    uint32_t slot = 0, pix = 0;
    int s = 0, obs = 0;
    R c3[3] = {(R)0, (R)0, (R)0};
    LaneGrid<R> G = {};
    Walk<R> W;
    W.done = true;
    WorkPool pool;
    for (;;) {
        // packets whose flight stopped inside their mesh go to the next live list, in place pos
        const bool append = FLIGHTS && W.done && kind == BW_MOVE && W.stopped;
        const uint32_t pos = FLIGHTS ? wave_append(append, &Q->n_live[in ^ 1]) : 0u;
        const bool peel_done = W.done && kind == BW_PEEL;
        if (__ballot(peel_done) != 0) {
            double v[3] = {0.0, 0.0, 0.0};
            uint64_t key = 0;
            size_t plane = 1;
            if (peel_done) {
                n_visits += W.visits;
                n_peels++;
                const BScene &S = P.scenes[s];
                plane = (size_t)S.npix * (size_t)S.npix;
                const double att = exp(-W.tau);
                v[0] = att * (double)c3[0];
                v[1] = att * (double)c3[1];
                v[2] = att * (double)c3[2];
                // image copy of this block (blocks go round-robin to the XCDs); the key is
                // the offset of the pixel's I value from the base of all images
                key = (uint64_t)(S.img - P.img_base) + (uint64_t)(blockIdx.x % kImageCopies) * S.img_set +
                      (uint64_t)obs * 3 * plane + pix;
                kind = BW_NONE;
            }
            wave_merge_add(peel_done, key, v[0], v[1], v[2], P.img_base, plane, P.img_key_bits,
                           s_merge[threadIdx.x >> 6]);
        }
        if (FLIGHTS && W.done && kind == BW_MOVE) {
            n_visits += W.visits;
            if (append) {
                PacketState<R> st = pks[slot];
                for (int a = 0; a < 3; ++a) st.p[a] = st.p[a] + W.t_out * st.k[a];
                out[pos] = st;
            } else {
                n_esc++;
            }
            kind = BW_NONE;
        }
        uint64_t item = 0;
        if (pool.take(kind == BW_NONE, total, &Q->work[1][0][0], item)) {
            item = scatter_block(item, total, stride);
            if (item < n_peel) {
                uint64_t at = item;
                int g = 0;
#pragma unroll
                for (int q = 0; q < kPeelGroups - 1; ++q) {
                    const bool past = g == q && at >= g_count[q];
                    at -= past ? g_count[q] : 0;
                    g += past ? 1 : 0;
                }
                // appended rays are all visible
                const PeelRay<R> r = peels[(uint64_t)g * P.group_cap + at];
                s = (int)(r.obs >> 4);
                obs = (int)(r.obs & 15u);
                const BScene &S = P.scenes[s];
                const R o[3] = {(R)S.obs[obs].o[0], (R)S.obs[obs].o[1], (R)S.obs[obs].o[2]};
                c3[0] = r.c[0]; c3[1] = r.c[1]; c3[2] = r.c[2];
                pix = r.pix;
                G = lane_grid<R>(S);
                walk_begin(W, G, r.p, o, WALK_EDGE, 0.0);
                kind = BW_PEEL;
            } else if constexpr (FLIGHTS) {
                slot = (uint32_t)(item - n_peel);
                const PacketState<R> *ps = pks + slot;
                if (ps->target >= 0.0) {
                    s = (int)state_tag(ps->word);
                    const R p0[3] = {ps->p[0], ps->p[1], ps->p[2]};
                    const R k0[3] = {ps->k[0], ps->k[1], ps->k[2]};
                    G = lane_grid<R>(P.scenes[s]);
                    walk_begin(W, G, p0, k0, WALK_MOVE, ps->target);
                    kind = BW_MOVE;
                }
            }
        }
        if (__ballot(kind != BW_NONE) == 0) {
            if (pool.dry) break;
            continue;
        }
        if (!FLIGHTS || __ballot(kind == BW_MOVE) == 0) {
            // no lane moves to a target: walks to the edge only
            for (;;) {
                walk_batch_edge<R, kFlightBatch>(W, G);
                if (__popcll(__ballot(W.done || kind == BW_NONE)) >= kWaveRefill) break;
            }
        } else if constexpr (FLIGHTS) {
            for (;;) {
                walk_batch<R, kFlightBatch>(W, G);
                if (__popcll(__ballot(W.done || kind == BW_NONE)) >= kWaveRefill) break;
            }
        }
    }
    flush_counters<4>(P.counters, {CNT_VISITS, CNT_PEELS, CNT_PEEL_RAYS, CNT_ESCAPES}, {n_visits, n_peels, n_peels, n_esc});
}

// ---------------------------------------------------------------- late orders in one launch
// The batched form of k_tail (qrt_transport.hip): from order order0 on, a lane
// carries each live packet through its scene's remaining orders (flight on the
// scene's mesh as k_bwalk walks it); every scattering's state is appended to
// the deferred list (regions per work-pool part) for one k_bscatter launch and
// one k_bwalk launch afterwards.  A wave whose reservation does not fit
// computes its scatterings' peel-offs itself and walks their rays at once.
template <typename R, int KIND>
// three waves per SIMD in FP32 (168 VGPRs with 10 spilled, against two waves at
// the compiler's own 189: the batch runs 1.3 % faster)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 1))) k_btail(const BatchParams P, int order0,
                                               const PacketState<R> *__restrict__ pks, int in,
                                               PacketState<R> *__restrict__ states, uint32_t state_cap,
                                               Queues *__restrict__ Q)
{
    // the peel-ray counters that the scattering launch of the deferred list appends to
    // (their last user, the walk of order order0 - 1, has ended)
    if (blockIdx.x == 0 && threadIdx.x < kPeelGroups) Q->n_peel[P.max_orders & 1][threadIdx.x][0] = 0;
    const uint64_t n = Q->n_live[in];
    const int region = (int)(blockIdx.x % kPoolParts);
    PacketState<R> *sreg = states + (size_t)region * state_cap;
    uint32_t *sreg_n = &Q->n_def[region][0];
    const int lane = (int)(threadIdx.x & 63);
    uint64_t n_visits = 0;
    uint32_t n_scat = 0, n_occ = 0, n_esc = 0, n_peels = 0;
    PacketState<R> st = {};
    int s = 0, order = 0;
    bool has = false, moving = false, at_scatter = false;
    LaneGrid<R> G = {};
    Walk<R> W = {};
    W.done = true;
    WorkPool pool;
    for (;;) {
        if (moving && W.done) {
            n_visits += W.visits;
            if (W.stopped) {
                for (int a = 0; a < 3; ++a) st.p[a] = st.p[a] + W.t_out * st.k[a];
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
            st = pks[item];
            s = (int)state_tag(st.word);
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
                    PacketState<R> d = st;
                    d.word = with_order(d.word, fits ? (uint32_t)order : kNoState);
                    sreg[slot] = d;
                }
            }
            const BScene &S = P.scenes[s];
            const SceneView<R> V = scene_view<R>(S);
            R n_ax[3] = {(R)0, (R)0, (R)0};
            if (at_scatter) {
                st.S[0] *= V.albedo; st.S[1] *= V.albedo; st.S[2] *= V.albedo;
                cross3(st.k, st.m, n_ax);
                G = lane_grid<R>(S);
            }
            if (!fits) {
                // the list is full: this wave's scatterings peel off here
                if (at_scatter) n_scat++;
                for (int ob = 0; ob < kBatchObs; ++ob) {
                    bool vis = false, occ = false;
                    R c3[3] = {(R)0, (R)0, (R)0};
                    uint32_t pix = 0;
                    R o[3] = {(R)0, (R)0, (R)1};
                    if (at_scatter && ob < S.n_obs) {
                        const DevObserver &O = S.obs[ob];
                        const R ex[3] = {(R)O.ex[0], (R)O.ex[1], (R)O.ex[2]};
                        const R ey[3] = {(R)O.ey[0], (R)O.ey[1], (R)O.ey[2]};
                        o[0] = (R)O.o[0]; o[1] = (R)O.o[1]; o[2] = (R)O.o[2];
                        peel_contribution<R>(V, st, n_ax, o, ex, ey, vis, occ, c3, pix);
                        n_occ += occ ? 1u : 0u;
                    }
                    if (vis) {
                        // W is free: this lane's flight has ended
                        walk_begin(W, G, st.p, o, WALK_EDGE, 0.0);
                        walk_run<R, kFlightBatch>(W, G);
                        n_visits += W.visits;
                        n_peels++;
                        const double att = exp(-W.tau);
                        const size_t plane = (size_t)S.npix * (size_t)S.npix;
                        double *dst = S.img + (size_t)(blockIdx.x % kImageCopies) * S.img_set +
                                      (size_t)ob * 3 * plane + pix;
                        unsafeAtomicAdd(dst, att * (double)c3[0]);
                        unsafeAtomicAdd(dst + plane, att * (double)c3[1]);
                        unsafeAtomicAdd(dst + 2 * plane, att * (double)c3[2]);
                    }
                }
            }
            if (at_scatter) {
                if (order < S.max_orders) {
                    uint32_t x[3];
                    seq_triple<KIND>(scene_seq(P, S), state_idx(st.word), first_scatter_dim(S.src_kind) + 3 * (order - 1), x);
                    scatter_packet<R>(V, st, n_ax, x);
                    walk_begin(W, G, st.p, st.k, WALK_MOVE, st.target);
                    moving = true;
                } else {
                    has = false;   // the scene's last order scatters without a flight
                }
                at_scatter = false;
            }
        }
        const int movers = __popcll(__ballot(moving));
        if (movers == 0) continue;
        for (;;) {
            // only lanes with a flight under way step, as in k_tail
            if (moving && !W.done) walk_batch<R, kFlightBatch>(W, G);
            if (8 * __popcll(__ballot(moving && W.done)) >= kTailDoneEighths * movers) break;
        }
    }
    flush_counters<6>(P.counters, {CNT_VISITS, CNT_SCATTERINGS, CNT_OCCLUDED, CNT_ESCAPES, CNT_PEELS, CNT_PEEL_RAYS},
                      {n_visits, n_scat, n_occ, n_esc, n_peels, n_peels});
}

// Sort keys of a batch's deferred scatterings (k_def_keys of the single-scene
// launch): the scene, relative to the chunk's first, in the top bits, then the
// Morton index of the point's cell in a 32^3 grid over the scene's box in the
// bits that remain of 15; entries reserved but not deferred get the largest key.
template <typename R>
__global__ void __launch_bounds__(256) k_bdef_keys(const BatchParams P, const PacketState<R> *__restrict__ pks,
                                                   Queues *__restrict__ Q, uint32_t def_cap,
                                                   uint32_t *__restrict__ keys)
{
    const DeferredList D = deferred_list(Q, def_cap);
    const uint32_t n = (uint32_t)D.end[kPoolParts - 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) Q->n_def_all[0] = n;
    const int pos_bits = P.scene_bits < 15 ? 15 - P.scene_bits : 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const PacketState<R> *st = pks + deferred_slot(D, i);
        uint32_t key = 0xFFFFu;
        if (state_order(st->word) != kNoState) {
            const int sc = (int)state_tag(st->word);
            const BScene &S = P.scenes[sc];
            KeyFrame f;
            for (int a = 0; a < 3; ++a) {
                f.lo[a] = (float)S.lo[a];
                f.scale[a] = (float)(32.0 / (S.n[a] * S.h[a]));
            }
            key = ((uint32_t)(sc - P.scene_base) << pos_bits) | (cell_key(f, st->p) >> (15 - pos_bits));
        }
        keys[i] = key;
    }
}

// ---------------------------------------------------------------- launch sequence
template <typename F>
static int batch_resident_blocks(F kernel)
{
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    (void)hipGetDevice(&dev);
    int cus = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
    return per_cu * cus;
}

template <typename R, int KIND>
static hipError_t batch_chunk(const BatchParams &P, uint64_t b0, uint32_t count, const TransportBuffers &B,
                              hipStream_t st, KernelTimer *T)
{
    // P.scene_base and P.scene_bits are set per chunk by launch_batch
    static int nb_first = 0, nb_scatter = 0, nb_walk = 0, nb_walk_peels = 0, nb_tail = 0;
    if (!nb_first) {
        nb_first = batch_resident_blocks(k_bfirst<R, KIND>);
        nb_scatter = batch_resident_blocks(k_bscatter<R, KIND>);
        nb_walk = batch_resident_blocks(k_bwalk<R, true>);
        nb_walk_peels = batch_resident_blocks(k_bwalk<R, false>);
        nb_tail = batch_resident_blocks(k_btail<R, KIND>);
    }
    PeelRay<R> *peels = (PeelRay<R> *)B.peels;
    const int walk_blocks = std::min(nb_walk, kWalkBlocksPerCu * device_cu_count());
    const uint32_t cblocks = (count + 255) / 256;
    const int b_elem = (int)(cblocks < 2048u ? cblocks : 2048u);
    hipError_t e = launch_clear_queues(B.q, st, T);
    if (e != hipSuccess) return e;
    {
        TimedLaunch tl(T, st, TC_SORT);
        hipLaunchKernelGGL((k_bkey<R, KIND>), dim3(b_elem), dim3(256), 0, st, P, b0, count, B.keys);
    }
    if ((e = launch_sort_keys(B, count, st, T)) != hipSuccess) return e;
    const int bf = (int)(cblocks < (uint32_t)nb_first ? cblocks : (uint32_t)nb_first);
    {
        TimedLaunch tl(T, st, TC_FIRST);
        hipLaunchKernelGGL((k_bfirst<R, KIND>), dim3(bf), dim3(256), 0, st, P, b0, count, (const uint32_t *)B.order,
                           (const uint32_t *)B.keys, state_list<R>(B, 0), B.q);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int bs = (int)(cblocks < (uint32_t)nb_scatter ? cblocks : (uint32_t)nb_scatter);
    // orders from `tail` on run in one launch, their peel rays deferred to one walk
    const bool tail_on = P.tail_from >= 2 && P.tail_from <= P.max_orders;
    const int last = tail_on ? P.tail_from - 1 : P.max_orders;
    for (int order = 1; order <= last; ++order) {
        const int in = (order - 1) & 1;
        {
            TimedLaunch tl(T, st, TC_SCATTER);
            hipLaunchKernelGGL((k_bscatter<R, KIND>), dim3(bs), dim3(256), 0, st, P, order, state_list<R>(B, in), in,
                               peels, B.q, 0u, (const uint32_t *)nullptr);
        }
        const int wb = order < P.max_orders ? walk_blocks : nb_walk;   // the last order walks peel rays only
        {
            TimedLaunch tl(T, st, TC_WALK);
            hipLaunchKernelGGL((k_bwalk<R, true>), dim3(wb), dim3(256), 0, st, P, order,
                               (const PacketState<R> *)state_list<R>(B, in), in, state_list<R>(B, in ^ 1),
                               (const PeelRay<R> *)peels, B.q);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (tail_on) {
        const int in = last & 1;   // the live list of order `tail`; the other list takes the deferred scatterings
        // at most `count` in all, so that their peel rays fit the append groups as a chunk's
        // first order does, in kPoolParts regions, one per work-pool part
        uint64_t cap = std::min<uint64_t>(B.cap, count);
        if (P.def_limit) cap = std::min<uint64_t>(cap, P.def_limit);
        const uint32_t state_cap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap / kPoolParts, 0x1FFFFFFFull));
        {
            TimedLaunch tl(T, st, TC_WALK);
            hipLaunchKernelGGL((k_btail<R, KIND>), dim3(nb_tail), dim3(256), 0, st, P, P.tail_from,
                               (const PacketState<R> *)state_list<R>(B, in), in, state_list<R>(B, in ^ 1),
                               state_cap, B.q);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // the deferred scatterings sorted by scene and position (as in the single-scene
        // launch), their peel-offs as the last order's, then the walk of their rays
        const int din = in ^ 1;
        const uint32_t def_bound = (uint32_t)std::min<uint64_t>((uint64_t)kPoolParts * state_cap, B.cap);
        {
            TimedLaunch tl(T, st, TC_SORT);
            const int kb = (int)std::min<uint32_t>((def_bound + 255) / 256, 512u);
            hipLaunchKernelGGL((k_bdef_keys<R>), dim3(kb), dim3(256), 0, st, P,
                               (const PacketState<R> *)state_list<R>(B, din), B.q, state_cap, B.keys);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const uint32_t *def_count = (const uint32_t *)((const char *)B.q + offsetof(Queues, n_def_all));
        if ((e = launch_sort_keys(B, def_bound, st, T, def_count)) != hipSuccess) return e;
        {
            TimedLaunch tl(T, st, TC_SCATTER);
            hipLaunchKernelGGL((k_bscatter<R, KIND>), dim3(nb_scatter), dim3(256), 0, st, P, P.max_orders,
                               state_list<R>(B, din), din, peels, B.q, state_cap, (const uint32_t *)B.order);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        {
            TimedLaunch tl(T, st, TC_WALK);
            hipLaunchKernelGGL((k_bwalk<R, false>), dim3(nb_walk_peels), dim3(256), 0, st, P, P.max_orders,
                               (const PacketState<R> *)state_list<R>(B, din), din, state_list<R>(B, in),
                               (const PeelRay<R> *)peels, B.q);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R>
static hipError_t batch_kind(const BatchParams &P, int kind, uint64_t b0, uint32_t count, const TransportBuffers &B,
                             hipStream_t st, KernelTimer *T)
{
    switch (kind) {
    case SEQ_SOBOL: return batch_chunk<R, SEQ_SOBOL>(P, b0, count, B, st, T);
    case SEQ_HALTON: return batch_chunk<R, SEQ_HALTON>(P, b0, count, B, st, T);
    case SEQ_NIED2: return batch_chunk<R, SEQ_NIED2>(P, b0, count, B, st, T);
    case SEQ_HAMMERSLEY: return batch_chunk<R, SEQ_HAMMERSLEY>(P, b0, count, B, st, T);
    case SEQ_PHILOX: return batch_chunk<R, SEQ_PHILOX>(P, b0, count, B, st, T);
    case SEQ_SOBOL_OWEN: return batch_chunk<R, SEQ_SOBOL_OWEN>(P, b0, count, B, st, T);
    default: return hipErrorInvalidValue;
    }
}

// last scene whose first batch number is <= b (host copy of the search in batch_scene)
static int host_scene_of(const uint64_t *begin, int n_scenes, uint64_t b)
{
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

hipError_t launch_batch(const BatchParams &P0, const uint64_t *begin, int precision, int kind, uint64_t b_first,
                        uint64_t b_count, const TransportBuffers &B, uint64_t chunk, hipStream_t stream,
                        KernelTimer *timer)
{
    const uint64_t total = b_first + b_count;
    for (uint64_t done = b_first; done < total;) {
        const uint32_t n = (uint32_t)(total - done < chunk ? total - done : chunk);
        // the sort key spends only the bits that the chunk's scenes need on the scene
        BatchParams P = P0;
        // a group of peel rays receives at most ceil(blocks / kPeelGroups) of the chunk's
        // 64-packet blocks, each with at most 64 kBatchObs rays: it must fit its region
        const uint64_t blocks = ((uint64_t)n + 63) / 64;
        if (((blocks + kPeelGroups - 1) / kPeelGroups) * 64 * kBatchObs > P.group_cap) return hipErrorInvalidValue;
        P.scene_base = host_scene_of(begin, P.n_scenes, done);
        const int span = host_scene_of(begin, P.n_scenes, done + n - 1) - P.scene_base + 1;
        P.scene_bits = 0;
        while ((1 << P.scene_bits) < span) P.scene_bits++;
        hipError_t e = precision == 1 ? batch_kind<double>(P, kind, done, n, B, stream, timer)
                                      : batch_kind<float>(P, kind, done, n, B, stream, timer);
        if (e != hipSuccess) return e;
        done += n;
    }
    return hipSuccess;
}

}  // namespace qrt

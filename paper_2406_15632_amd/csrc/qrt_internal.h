// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "qrt_seq.h"
#include "qrt_walk.h"

namespace qrt {

constexpr int kMaxDims = 128;

// bits that hold the values 0 .. n-1 (n >= 1)
__host__ __device__ __forceinline__ int bits_for(uint64_t n)
{
    int b = 0;
    while (b < 63 && (1ull << b) < n) ++b;
    return b;
}
constexpr int kMaxObs = 16;
constexpr uint64_t kChunk = 1ull << 22;   // packets per transport chunk (queue capacity)
constexpr int kImageCopies = 16;          // image accumulators (two per XCD: blocks go to the XCDs in turn), folded on read

// counter slots in the device counter array
enum CounterSlot {
    CNT_PACKETS = 0, CNT_VISITS, CNT_PEELS, CNT_PEEL_RAYS, CNT_ESCAPES, CNT_TAU_CUTS,
    CNT_SCATTERINGS, CNT_OCCLUDED, CNT_SURROGATE, CNT_FALLBACKS, CNT_VISITS_FIRST, CNT_COUNT
};
// The device counter array holds kCounterCopies copies of the slots, each on
// its own 128-byte line: a block adds into copy blockIdx % kCounterCopies
// (one per XCD), and a read sums the copies.
constexpr int kCounterCopies = 8;
constexpr int kCounterLine = 16;
static_assert(CNT_COUNT <= kCounterLine, "the counter slots fit one line");

// Optional kernel timing: a pair of HIP events on the launch stream around each
// kernel launch, by class (the QRT_T_* classes of the C ABI).  Events are reused
// from a free list; pairs wait in `pending` until collect() sums them.
struct KernelTimer {
    struct Pair {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> free_events;
    std::vector<Pair> pending;
    double ms[8] = {};
    int64_t launches[8] = {};
    hipEvent_t open = nullptr;
    int open_cls = 0;

    hipEvent_t take()
    {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        return hipEventCreate(&e) == hipSuccess ? e : nullptr;
    }
    void begin(hipStream_t st, int cls)
    {
        open = take();
        open_cls = cls;
        if (open) (void)hipEventRecord(open, st);
    }
    void end(hipStream_t st)
    {
        hipEvent_t b = take();
        if (open && b) {
            (void)hipEventRecord(b, st);
            pending.push_back({open_cls, open, b});
        } else {
            if (open) free_events.push_back(open);
            if (b) free_events.push_back(b);
        }
        open = nullptr;
    }
    // sums the pairs recorded so far (their stream must have been synchronised)
    hipError_t collect()
    {
        for (const Pair &p : pending) {
            float t = 0.0f;
            const hipError_t e = hipEventElapsedTime(&t, p.a, p.b);
            if (e != hipSuccess) return e;
            ms[p.cls] += (double)t;
            launches[p.cls] += 1;
            free_events.push_back(p.a);
            free_events.push_back(p.b);
        }
        pending.clear();
        return hipSuccess;
    }
    void destroy()
    {
        for (const Pair &p : pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
        pending.clear();
        free_events.clear();
    }
};
enum TimingClass { TC_SORT = 0, TC_FIRST, TC_SCATTER, TC_WALK, TC_PEEL_MLP, TC_OTHER, TC_COUNT };

// times one launch when a timer is given
struct TimedLaunch {
    KernelTimer *t;
    hipStream_t st;
    TimedLaunch(KernelTimer *timer, hipStream_t stream, int cls) : t(timer), st(stream)
    {
        if (t) t->begin(st, cls);
    }
    ~TimedLaunch()
    {
        if (t) t->end(st);
    }
};

struct DevObserver {
    double o[3], ex[3], ey[3];
};

// Network inputs of the surrogate, in the coordinates of its cylindrical
// domain (centre c, outer radius r_out, scale height h(R) = h0 R^beta,
// half-thickness zmax h): (p_x - c_x) / r_out, (p_y - c_y) / r_out,
// (p_z - c_z) / (zmax h(R)) clamped to [-4, 4] (0 on the axis), then
// 2 theta / pi - 1 and phi / pi - 1 of the observer; each rounded to FP32.
struct InputMap {
    double center[3];
    double r_out, h0, beta, zmax;
    float obs_in[kMaxObs][2];
    int n_obs;
};

__device__ __forceinline__ void mlp_inputs(const InputMap &M, double px, double py, double pz, int ob, float x[5])
{
    const double dx = px - M.center[0], dy = py - M.center[1], dz = pz - M.center[2];
    const double R = sqrt(dx * dx + dy * dy);
    double zn = 0.0;
    if (R > 0.0) {
        zn = dz / (M.zmax * (M.h0 * pow(R, M.beta)));
        zn = zn > 4.0 ? 4.0 : (zn < -4.0 ? -4.0 : zn);
    }
    x[0] = (float)(dx / M.r_out);
    x[1] = (float)(dy / M.r_out);
    x[2] = (float)zn;
    x[3] = M.obs_in[ob][0];
    x[4] = M.obs_in[ob][1];
}

// Surrogate peel-off: cylindrical domain (R in [r_in, r_out), |z| < zmax h(R))
// with its validity mask, the network (FP32 parameters for the biases,
// bfloat16 weight tiles), and the capture buffer of a pilot run (null when off).
struct SurrogateParams {
    InputMap in;                          // domain geometry and input map
    double r_in;
    int n_r, n_z;
    const uint8_t *valid;                 // [n_obs][n_r][n_z]
    const float *params;                  // 12929 FP32
    const void *tiles;                    // bfloat16 weight tiles
    float *cap;                           // pilot capture: [cap_capacity][4] = x, y, z, observer
    uint32_t *cap_count;
    uint32_t cap_capacity;
};

// cell ir * n_z + iz of a position in the cylindrical domain, -1 outside
__device__ __forceinline__ int dom_cell(const SurrogateParams &S, double x, double y, double z)
{
    const InputMap &D = S.in;
    const double dx = x - D.center[0], dy = y - D.center[1], dz = z - D.center[2];
    const double R = sqrt(dx * dx + dy * dy);
    if (!(R >= S.r_in && R < D.r_out)) return -1;
    const double zh = dz / (D.h0 * pow(R, D.beta));
    if (!(fabs(zh) < D.zmax)) return -1;
    const int ir = (int)floor((R - S.r_in) / (D.r_out - S.r_in) * (double)S.n_r);
    const int iz = (int)floor((zh + D.zmax) / (2.0 * D.zmax) * (double)S.n_z);
    if (ir < 0 || ir >= S.n_r || iz < 0 || iz >= S.n_z) return -1;
    return ir * S.n_z + iz;
}

struct TransportParams {
    DevGrid grid;
    int src_kind;            // 0 point, 1 sphere star (direct order), 2 sphere star (inverse order)
    double src[3];
    double r_star;
    double albedo, g, p_lin;
    int n_obs, npix;
    double half_width;
    DevObserver obs[kMaxObs];
    SeqParams seq;
    int max_orders;
    double tau_min;
    double *img;                   // [sets][kImageCopies][n_obs][3][npix][npix]
    int order_images;              // 0: one set; K: one set per scattering order 1..K
    unsigned long long *counters;  // [kCounterCopies][kCounterLine]
    int peel_mode;                 // 0 exact traversal, 1 surrogate inside its valid cells
    SurrogateParams sur;
    int tail_from;                 // first order of the late-order launch (0: every order has its own launches)
    uint64_t def_limit;            // at most this many deferred scatterings (0: as many as the buffers hold)
};

// First scattering order that the late-order launch takes over by default.
// From the second order on the live packets no longer fill the GPU well, and
// per-order launches would each wait for their longest walk; the deferred
// scatterings, sorted by position, walk their peel rays as coherently as a
// per-order list.
constexpr int kTailFrom = 2;

// one training batch of the surrogate network
struct MlpBatch {
    uint64_t seed, step;
    int batch;          // samples per step (64 per block)
    float cap, wfloor;  // targets min(tau, cap); weights exp(-target) + wfloor
};

struct AdamStep {
    float lr, beta1, beta2, eps;
    float c1, c2;       // bias corrections 1/(1 - beta1^t), 1/(1 - beta2^t)
};



// A scattered packet between kernels: position, direction, reference axis,
// Stokes weight, the optical depth of its next flight, and one word with the
// point index (bits 0-47), a tag (bits 48-57: the scene of a batch) and a
// scattering order (bits 58-63; the late-order launch's marks).  64 bytes in
// FP32, so a state is one half of a 128-byte line.
template <typename R>
struct alignas(16) PacketState {
    R p[3], k[3], m[3], S[3];
    double target;
    uint64_t word;
};
static_assert(sizeof(PacketState<float>) == 64, "an FP32 state fills 64 bytes");

constexpr int kIdxBits = 48;        // point indices below 2^48
constexpr uint32_t kTagMask = 1023; // scene numbers below 1024
// order field of a deferred scattering that was reserved but not deferred
constexpr uint32_t kNoState = 63;

__host__ __device__ __forceinline__ uint64_t state_word(uint64_t idx, uint32_t tag, uint32_t order)
{
    return idx | ((uint64_t)(tag & kTagMask) << kIdxBits) | ((uint64_t)order << (kIdxBits + 10));
}
__host__ __device__ __forceinline__ uint64_t state_idx(uint64_t w) { return w & ((1ull << kIdxBits) - 1); }
__host__ __device__ __forceinline__ uint32_t state_tag(uint64_t w) { return (uint32_t)(w >> kIdxBits) & kTagMask; }
__host__ __device__ __forceinline__ uint32_t state_order(uint64_t w) { return (uint32_t)(w >> (kIdxBits + 10)); }
__host__ __device__ __forceinline__ uint64_t with_order(uint64_t w, uint32_t order)
{
    return (w & ((1ull << (kIdxBits + 10)) - 1)) | ((uint64_t)order << (kIdxBits + 10));
}

// A peel-off ray waiting for its optical depth: start point, Stokes
// contribution before attenuation, pixel offset and observer.
template <typename R>
struct alignas(16) PeelRay {
    R p[3], c[3];
    uint32_t pix, obs;
};

// Device-side queue counters of one chunk.
constexpr int kPeelGroups = 8;     // peel-ray append counters of the batched launches

struct Queues {
    uint32_t n_live[2];   // live packets per ping-pong list
    // work counters of the persistent kernels: per pool, kPoolParts counters
    // (one per XCD) of which each owns a 128-byte line
    unsigned long long work[4][8][16];
    // appended peel rays per order parity and group (batched launches), one
    // counter per 128-byte line so that the groups' atomics do not share one
    uint32_t n_peel[2][kPeelGroups][32];
    // scatterings deferred by the late-order launch, per region of their list
    // (one region per work-pool part), one counter per 128-byte line
    uint32_t n_def[8][32];
    // the deferred scatterings of all regions together (the count of their sort)
    uint32_t n_def_all[32];
};

// A peel-off ray queued for the surrogate network: its network inputs, the
// offset of its pixel's I value in the image set [obs][3][npix][npix], and its
// contribution before attenuation.
struct alignas(16) SurQuery {
    float x[5];
    uint32_t key;
    double c[3];
};

// The surrogate queue of an order: the rays queued by the 64-packet block b of
// the live list sit at the start of the block's region of 64 n_obs entries,
// and sur_n[b] counts them (no atomics: a wave owns its block).
__host__ __device__ inline size_t sur_queue_entries(uint64_t cap, int n_obs)
{
    return (size_t)((cap + 63) / 64) * 64 * (size_t)n_obs;
}
__host__ __device__ inline size_t sur_count_entries(uint64_t cap) { return (size_t)((cap + 63) / 64); }

constexpr int kSortBits = 16;                 // bits of the coherence sort keys
constexpr int kSortItems = 4096;              // items per block of the radix-sort passes
constexpr int kSortDigit = 256;               // values of an 8-bit digit
// histogram entries of a pass: [kSortDigit][blocks] block counts, then kSortDigit digit totals
constexpr size_t kSortHist = (size_t)kSortDigit * (kChunk / kSortItems) + kSortDigit;

// Device buffers of the transport (owned by the context).
struct TransportBuffers {
    void *packets;        // PacketState<R>[2][cap]: the live packets of a scattering order, dense and in
                          // the order they were appended, ping-pong by order (list in, then list in ^ 1)
    void *peels;          // PeelRay<R>[n_obs * (chunk + 64)], blocks of 64 per observer
    SurQuery *sur_q;      // [sur_queue_entries(cap, n_obs)] peel-off rays queued for the network
    uint32_t *sur_n;      // [sur_count_entries(cap)] queued rays per 64-packet block
    uint32_t *order;      // [chunk] packets in coherence order
    uint32_t *keys;       // [chunk] sort keys
    uint32_t *sort_tmp;   // [2 chunk] keys and packets after the first sort pass
    uint32_t *hist;       // [kSortHist] histograms of a sort pass
    Queues *q;
    size_t packet_bytes, peel_bytes;
    size_t sur_entries;   // entries of sur_q
    uint64_t cap;         // packets per state list
};

// live packet list `in` (0 or 1) of the buffers
template <typename R>
inline PacketState<R> *state_list(const TransportBuffers &B, int in)
{
    return (PacketState<R> *)B.packets + (size_t)in * B.cap;
}

size_t packet_state_bytes(int precision);
size_t peel_ray_bytes(int precision);

// ---------------------------------------------------------------- batches of scenes
constexpr int kBatchObs = 4;            // observers per scene of a batch (peel slots per packet)
constexpr int kMaxBatchScenes = 1024;

// One scene of a batch: its own mesh, source, dust, observers, image and
// packet range.  Its packets are the batch numbers begin .. begin+count-1 and
// use point indices first .. first+count-1 of the scene's sequence.
struct BScene {
    const float *kr;            // bricked as the single-scene mesh
    int n[3];
    int nb[3];                  // bricks per axis
    double lo[3], h[3];
    int src_kind;               // 0 point, 1 sphere star (direct order), 2 sphere star (inverse order)
    double src[3], r_star;
    double albedo, g, p_lin;
    int n_obs, npix;
    double half_width;
    DevObserver obs[kBatchObs];
    int max_orders;
    double tau_min;
    double *img;                // [kImageCopies][n_obs][3][npix][npix]
    uint64_t img_set;           // doubles of one copy: n_obs * 3 * npix^2
    uint64_t first, begin, count, n_total;
};

struct BatchParams {
    const BScene *scenes;       // device array [n_scenes], ordered by begin
    int n_scenes;
    int scene_base;             // first scene of the chunk being launched
    int scene_bits;             // sort-key bits that hold scene - scene_base (the rest: emission direction)
    SeqParams seq;              // n_total is replaced by each scene's own
    int max_orders;             // largest over the scenes
    uint32_t group_cap;         // peel rays per append group: group g owns [g group_cap, (g+1) group_cap),
                                // kPeelGroups group_cap rays at most the peel buffer's capacity
    unsigned long long *counters;  // [kCounterCopies][kCounterLine]
    double *img_base;           // all scenes' images, one after the other (scene images point into it)
    int img_key_bits;           // bits that hold an element offset from img_base
    int tail_from;              // first order of the late-order launch (0: every order has its own launches)
    uint64_t def_limit;         // at most this many deferred scatterings (0: as many as the buffers hold)
};

// Batch numbers b_first .. b_first+b_count-1 of a batch, in chunks of at most
// `chunk`; begin[s] (host) is the first batch number of scene s.
hipError_t launch_batch(const BatchParams &P, const uint64_t *begin, int precision, int kind, uint64_t b_first,
                        uint64_t b_count, const TransportBuffers &B, uint64_t chunk, hipStream_t stream,
                        KernelTimer *timer = nullptr);

// order[0 .. count) = the packets 0 .. count-1 sorted by keys[j] (kSortBits bits), stably; count <= kChunk.
// Two radix passes of 8 bits through B.sort_tmp, histograms in B.hist.
// count_dev (optional): a device word that lowers the count when the kernels run.
hipError_t launch_sort_keys(const TransportBuffers &B, uint32_t count, hipStream_t st, KernelTimer *timer = nullptr,
                            const uint32_t *count_dev = nullptr);

// One chunk of packets first .. first+count-1 (count <= kChunk) through every
// scattering order: first flight, then per order a scatter kernel and a walk
// kernel.  All launches go to stream.
hipError_t launch_transport(const TransportParams &P, int precision, int kind, uint64_t first,
                            uint64_t count, const TransportBuffers &B, hipStream_t stream,
                            KernelTimer *timer = nullptr);

// the x-fastest mesh src[nz][ny][nx] into the bricked order of dst (cleared beforehand)
hipError_t launch_to_bricks(const float *src, float *dst, int nx, int ny, int nz, hipStream_t stream);

// zero the queue counters of a chunk (a kernel, not a memset node)
hipError_t launch_clear_queues(Queues *q, hipStream_t stream, KernelTimer *timer = nullptr);

// img[0 .. n) += img[c n .. (c+1) n) for every further copy c, which is cleared
hipError_t launch_fold_images(double *img, size_t n, hipStream_t stream);

// surrogate network (qrt_mlp.hip); `tiles` holds kMlpTiles x 64 lanes x 8 bfloat16
hipError_t launch_mlp_pack(const float *params, void *tiles, hipStream_t st);
hipError_t launch_mlp_forward(const float *params, const void *tiles, const float *X, uint64_t n, float *y,
                              hipStream_t st);
int mlp_loss_parts(uint64_t n);
hipError_t launch_mlp_loss(const float *params, const void *tiles, const float *X, const float *tau, uint64_t n,
                           float cap, float wfloor, double *part, hipStream_t st);
hipError_t launch_mlp_grad(int mode, const float *params, const void *tiles, const float *X, uint64_t n,
                           const float *tau, const float *dy, const MlpBatch &sel, int n_blocks, float *part,
                           hipStream_t st);
hipError_t launch_mlp_adam(float *params, float *m, float *v, const float *part, int n_parts, const AdamStep &A,
                           void *tiles, hipStream_t st);
hipError_t launch_mlp_reduce(const float *part, int n_parts, float *out, hipStream_t st);
hipError_t launch_mlp_inputs(const float *pos_obs, uint64_t n, const InputMap &M, float *X, hipStream_t st);

hipError_t launch_points(const SeqParams &S, int kind, uint64_t first, uint64_t count, int dims,
                         uint32_t *out, hipStream_t stream);

hipError_t launch_trace_tau(const DevGrid &g, int precision, int64_t n, const double *p,
                            const double *k, double *tau, int64_t *visits, hipStream_t stream);

// Surrogate training data (qrt_sample.hip).  Canonical selection: the m
// captured rays (x, y, z, observer) sorted by a hash of their 16 bytes and the
// seed, the first n kept in that order (out), with their start points and
// observer directions as FP64 (pk: [n][3] points, then [n][3] directions) for
// the exact labels.  temp: scratch of sample_select_temp_bytes(m) bytes.
size_t sample_select_temp_bytes(uint64_t m);
hipError_t launch_sample_select(const float *rays, uint64_t m, uint64_t n, uint64_t seed, const DevObserver *obs,
                                int n_obs, void *temp, float *out, double *pk, hipStream_t st);
// labels: tau32[j] = (float)tau64[j]
hipError_t launch_to_float(const double *src, float *dst, uint64_t n, hipStream_t st);

// Validity mask from validation samples (pos_obs [n][4], exact tau, network
// output y): per cell (observer, R bin, z bin) the sums of |exp(-max(y,0)) -
// exp(-tau)| and of max(exp(-tau), floor_frac * mean transmission of the
// observer) over its samples in fixed point (so that the sums do not depend
// on their order), and the count; mask[k] = count >= min_count, den > 0 and
// num <= max_err den.  rep (device, 5 words): cells, valid cells, samples in
// the domain, samples in valid cells, worst valid num/den as FP64 bits.
hipError_t launch_validate(const SurrogateParams &S, int n_obs, uint64_t n, const float *pos_obs, const float *tau,
                           const float *y, double max_err, double floor_frac, int64_t min_count, void *work,
                           uint8_t *mask, uint64_t *rep, hipStream_t st);
// bytes of the work buffer of launch_validate
size_t validate_work_bytes(int n_obs, size_t cells);

}  // namespace qrt

// C ABI of the library (declared in include/qrt.h): context, argument
// checking, device memory, and the launches of the transport kernels.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "qrt.h"
#include "qrt_internal.h"
#include "qrt_mlp.h"

namespace qrt {
void niederreiter2_columns(int dims, uint32_t *out);
void first_primes(int count, uint32_t *out);
int sobol_table_dims();
void sobol_columns(int dims, uint32_t *out);
}  // namespace qrt

using namespace qrt;

// Transport scratch of the allocation-free runs (qrt_run_static), one copy per
// device; see static_buffers below for its layout.
constexpr size_t kStaticScratchBytes = 36ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Internal streams of overlapped runs: a run may start while the runs on the
// other lanes are still in their last scattering orders.  Three measured best
// (two: 1.15e9, three: 1.16e9, four: 1.12e9 packets/s on the benchmark disk).
constexpr int kLanes = 3;

struct qrt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // mesh (the library's bricked copy)
    bool has_grid = false;
    int n[3] = {0, 0, 0};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float *grid = nullptr;
    size_t grid_alloc = 0;                   // floats
    // source
    bool has_source = false;
    int src_kind = 0;
    double src[3] = {0, 0, 0};
    double r_star = 0.0;
    // dust
    double albedo = 1.0, g = 0.0, p_lin = 0.0;
    // observers and images
    bool has_obs = false;
    int n_obs = 0, npix = 0;
    double theta[QRT_MAX_OBSERVERS], phi[QRT_MAX_OBSERVERS];
    double half_width = 1.0;
    double *img = nullptr;
    size_t img_elems = 0;                    // one copy of one set: n_obs * 3 * npix^2
    int order_images = 0;                    // 0: one image set; K: one per scattering order
    size_t img_alloc = 0;                    // doubles allocated
    // sequence and transport
    int kind = QRT_SOBOL;
    uint64_t seed = 0, n_total = 0;
    int max_orders = 1;
    double tau_min = 1e-8;
    int precision = QRT_FP32;
    int peel_mode = QRT_PEEL_EXACT;
    // bookkeeping
    uint32_t *tables = nullptr;              // [sobol kMaxDims*1024][nied kMaxDims*1024][bases kMaxDims]
    uint32_t *faure = nullptr;               // Faure matrices and powers for faure_dims coordinates
    int faure_dims = 0;
    uint32_t faure_b = 0, faure_m = 0, faure_pow = 0;
    uint64_t faure_bm = 0;
    unsigned long long *counters = nullptr;  // [kCounterCopies][kCounterLine], summed on read
    TransportBuffers tb = {};                // packet and ray queues of the transport
    uint64_t tb_packets = 0;                 // packets the queues hold
    uint64_t packets_run = 0;
    // surrogate network: parameters, Adam moments, weight tiles
    float *mlp = nullptr;                    // [3][kMlpParams]: parameters, m, v
    void *tiles = nullptr;                   // kMlpTiles x 64 lanes x 16 bytes
    bool has_mlp = false;
    int64_t adam_t = 0;                      // Adam steps taken since the parameters were set
    float *part = nullptr;                   // per-wave gradients
    size_t part_elems = 0;
    float *train_x = nullptr;                // normalised training inputs
    size_t train_x_elems = 0;
    // surrogate domain and validity mask
    bool has_domain = false;
    double dom_center[3] = {0, 0, 0};
    double dom_r_in = 0, dom_r_out = 0, dom_h0 = 0, dom_beta = 0, dom_zmax = 0;
    int dom_nr = 0, dom_nz = 0;
    uint8_t *dom_valid = nullptr;            // [QRT_MAX_OBSERVERS][nr][nz] on the device
    // batch of scenes
    std::vector<BScene> batch;               // scene records (device addresses inside)
    std::vector<uint64_t> batch_begin;       // first batch number per scene
    BScene *batch_dev = nullptr;             // [kMaxBatchScenes]
    float *batch_grid = nullptr;             // all meshes, one after the other
    size_t batch_grid_alloc = 0;             // floats
    double *batch_img = nullptr;             // all image sets (kImageCopies each), one after the other
    size_t batch_img_alloc = 0;              // doubles
    size_t batch_img_used = 0;
    uint64_t batch_total = 0;                // packets of one batch run
    int batch_max_orders = 0;
    uint64_t batch_runs = 0;                 // batch runs since the last reset
    // device address of this device's static transport scratch (allocation-free runs)
    unsigned char *scratch = nullptr;
    // kernel timing (qrt_set_timing)
    bool timing = false;
    KernelTimer timer;
    // overlapped runs (qrt_set_overlap): chunks go round the kLanes lanes, each
    // an internal stream with its own transport buffers (lane 0 uses tb); a
    // lane's completion event joins the context stream once the lanes have
    // come round to it
    bool overlap = false;
    hipStream_t lane[kLanes] = {};
    hipEvent_t lane_done[kLanes] = {};
    hipEvent_t fork = nullptr;
    bool lane_pending[kLanes] = {};
    int next_lane = 0;
    TransportBuffers tbl[kLanes - 1] = {};   // buffers of lanes 1 ..
    uint64_t tbl_packets[kLanes - 1] = {};
    // late-order launch (qrt_set_tail): first order it takes, deferred-ray limit
    int tail_from = kTailFrom;
    uint64_t def_limit = 0;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int fail(qrt_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

int hip_fail(qrt_ctx *c, hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(c, QRT_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
    return fail(c, QRT_HIP_ERROR, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(c, expr, what)                     \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hip_fail(c, e_, what); \
    } while (0)

// The context stream waits for the overlapped runs still pending on the lanes.
void join_lanes(qrt_ctx *c)
{
    for (int b = 0; b < kLanes; ++b)
        if (c->lane_pending[b]) {
            (void)hipStreamWaitEvent(c->stream, c->lane_done[b], 0);
            c->lane_pending[b] = false;
        }
}

// Finishes everything the context has enqueued: its stream and all lanes of
// overlapped runs (a buffer is freed or reallocated only after this).
int sync_all(qrt_ctx *c)
{
    join_lanes(c);
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    for (int b = 0; b < kLanes; ++b)
        if (c->lane[b]) HIP_TRY(c, hipStreamSynchronize(c->lane[b]), "lane sync");
    return QRT_OK;
}

// Overlapped runs: the lanes' streams and events, created on first use.
int ensure_lanes(qrt_ctx *c)
{
    for (int b = 0; b < kLanes; ++b) {
        if (!c->lane[b]) HIP_TRY(c, hipStreamCreateWithFlags(&c->lane[b], hipStreamNonBlocking), "lane stream");
        if (!c->lane_done[b]) HIP_TRY(c, hipEventCreateWithFlags(&c->lane_done[b], hipEventDisableTiming), "lane event");
    }
    if (!c->fork) HIP_TRY(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming), "fork event");
    return QRT_OK;
}

// The transport buffers of lane b and their packet capacity (lane 0 uses the
// context's own set, which runs in stream order use too).
TransportBuffers &lane_buffers(qrt_ctx *c, int b)
{
    return b == 0 ? c->tb : c->tbl[b - 1];
}

uint64_t &lane_capacity(qrt_ctx *c, int b)
{
    return b == 0 ? c->tb_packets : c->tbl_packets[b - 1];
}

// Lane b starts after everything enqueued on the context stream so far.
int lane_fork(qrt_ctx *c, int b)
{
    HIP_TRY(c, hipEventRecord(c->fork, c->stream), "fork");
    HIP_TRY(c, hipStreamWaitEvent(c->lane[b], c->fork, 0), "fork");
    return QRT_OK;
}

// Lane b's chunk is enqueued and stays pending; the pending chunk of the lane
// after it joins the context stream, so that the chunk which next uses that
// lane (and its buffers) starts after it.  The newest kLanes - 1 chunks stay
// pending, so that the next chunk starts beside their last scattering orders,
// which occupy few compute units.
int lane_close(qrt_ctx *c, int b)
{
    HIP_TRY(c, hipEventRecord(c->lane_done[b], c->lane[b]), "lane done");
    c->lane_pending[b] = true;
    const int nb = (b + 1) % kLanes;
    if (c->lane_pending[nb]) {
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->lane_done[nb], 0), "join");
        c->lane_pending[nb] = false;
    }
    c->next_lane = nb;
    return QRT_OK;
}

int point_dims(const qrt_ctx *c)
{
    return (c->src_kind >= 1 ? 5 : 3) + 3 * (c->max_orders - 1);
}

SeqParams seq_params(const qrt_ctx *c, int kind, uint64_t seed, uint64_t n_total)
{
    SeqParams s;
    s.mat = c->tables + (kind == QRT_NIEDERREITER2 ? kMaxDims * 1024 : 0);
    s.bases = c->tables + 2 * kMaxDims * 1024;
    s.seed = seed;
    s.n_total = n_total;
    s.faure = c->faure;
    s.fb = c->faure_b;
    s.fm = c->faure_m;
    s.fpow = c->faure_pow;
    s.fbm = c->faure_bm;
    return s;
}

constexpr size_t kCounterBytes = sizeof(unsigned long long) * kCounterCopies * kCounterLine;
constexpr size_t kFaureTable = 8192;   // u32 entries: dims * m * m + m <= 128 * 25 + 5 (and 2 * 32 * 32 + 32)

// Faure tables for `dims` coordinates: base b = smallest prime >= dims, m digits
// with b^m >= 2^32, matrices P^d[r][k] = binom(k, r) d^(k-r) mod b, powers b^k
int ensure_faure(qrt_ctx *c, int dims)
{
    if (c->faure && c->faure_dims == dims) return QRT_OK;
    uint32_t b = dims < 2 ? 2u : (uint32_t)dims;
    for (;; ++b) {
        bool prime = true;
        for (uint32_t q = 2; q * q <= b; ++q)
            if (b % q == 0) { prime = false; break; }
        if (prime) break;
    }
    uint32_t m = 0;
    uint64_t p = 1;
    while (p < (1ull << 32)) { p *= b; ++m; }
    const size_t need = (size_t)dims * m * m + m;
    if (need > kFaureTable) return fail(c, QRT_UNSUPPORTED, "Faure table too large for %d coordinates", dims);
    std::vector<uint32_t> h(kFaureTable, 0);
    // binomials modulo b from Pascal's triangle
    std::vector<uint32_t> binom((size_t)m * m, 0);
    for (uint32_t k = 0; k < m; ++k) {
        binom[(size_t)k * m + 0] = 1;
        for (uint32_t r = 1; r <= k; ++r)
            binom[(size_t)k * m + r] = (binom[(size_t)(k - 1) * m + r - 1] + (r <= k - 1 ? binom[(size_t)(k - 1) * m + r] : 0)) % b;
    }
    for (int d = 0; d < dims; ++d)
        for (uint32_t r = 0; r < m; ++r) {
            uint64_t dp = 1;   // d^(k-r) mod b, with 0^0 = 1
            for (uint32_t k = r; k < m; ++k) {
                h[((size_t)d * m + r) * m + k] = (uint32_t)((binom[(size_t)k * m + r] * dp) % b);
                dp = (dp * (uint64_t)d) % b;
            }
        }
    const uint32_t pow_off = (uint32_t)((size_t)dims * m * m);
    uint64_t pw = 1;
    for (uint32_t k = 0; k < m; ++k) {
        h[pow_off + k] = (uint32_t)pw;
        pw *= b;
    }
    if (!c->faure) HIP_TRY(c, hipMalloc(&c->faure, kFaureTable * sizeof(uint32_t)), "Faure table");
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    HIP_TRY(c, hipMemcpy(c->faure, h.data(), kFaureTable * sizeof(uint32_t), hipMemcpyHostToDevice), "Faure table");
    c->faure_dims = dims;
    c->faure_b = b;
    c->faure_m = m;
    c->faure_pow = pow_off;
    c->faure_bm = pw;
    return QRT_OK;
}

int check_index_range(qrt_ctx *c, int kind, uint64_t n_total, uint64_t first, uint64_t count)
{
    if (first < 1) return fail(c, QRT_INVALID_ARG, "packet indices start at 1 (got %llu)", (unsigned long long)first);
    if (count > 0 && first + count - 1 < first) return fail(c, QRT_INVALID_ARG, "index range overflows");
    uint64_t last = count ? first + count - 1 : first;
    if (kind != QRT_PHILOX && last > 0xFFFFFFFFull)
        return fail(c, QRT_UNSUPPORTED, "low-discrepancy indices must stay below 2^32 (last %llu)",
                    (unsigned long long)last);
    // a packet's state keeps its index in 48 bits
    if (last >> kIdxBits) return fail(c, QRT_UNSUPPORTED, "indices must stay below 2^48 (last %llu)",
                                      (unsigned long long)last);
    if (kind == QRT_HAMMERSLEY && last > n_total)
        return fail(c, QRT_UNSUPPORTED, "Hammersley index %llu beyond N = %llu", (unsigned long long)last,
                    (unsigned long long)n_total);
    return QRT_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Transport buffers T (holding T_packets packets per list) for chunks of up to
// `count` packets (at most kChunk) at the given precision and peel slots per
// packet; grown on demand, never shrunk.
int ensure_buffers(qrt_ctx *c, TransportBuffers &T, uint64_t &T_packets, uint64_t count, int n_obs, int precision)
{
    uint64_t want = 1u << 16;
    while (want < count && want < kChunk) want <<= 1;
    if (want > kChunk) want = kChunk;
    // the state lists hold as many packets as the other lists (which never shrink)
    const uint64_t cap = std::max<uint64_t>(want, T_packets);
    const size_t pb = packet_state_bytes(precision) * cap * 2;   // two state lists
    const size_t rb = peel_ray_bytes(precision) * (want + 64) * (size_t)n_obs;
    const size_t qn = sur_queue_entries(cap, n_obs);
    const size_t qb = align256(qn * sizeof(SurQuery)) + sur_count_entries(cap) * sizeof(uint32_t);
    if (T.q && T.hist && T.packet_bytes >= pb && T.peel_bytes >= rb && T.sur_entries >= qn && T_packets >= want)
        return QRT_OK;
    int rc = sync_all(c);
    if (rc) return rc;
    if (!T.q) HIP_TRY(c, hipMalloc(&T.q, sizeof(Queues)), "queue counters");
    if (!T.hist) HIP_TRY(c, hipMalloc(&T.hist, sizeof(uint32_t) * kSortHist), "sort histograms");
    if (T.packet_bytes < pb) {
        if (T.packets) (void)hipFree(T.packets);
        T.packets = nullptr;
        T.packet_bytes = 0;
        HIP_TRY(c, hipMalloc(&T.packets, pb), "packet states");
        T.packet_bytes = pb;
    }
    if (T.peel_bytes < rb || T.sur_entries < qn) {
        if (T.peels) (void)hipFree(T.peels);
        T.peels = nullptr;
        T.sur_q = nullptr;
        T.sur_n = nullptr;
        T.peel_bytes = 0;
        T.sur_entries = 0;
        // the rays, then the surrogate queue and its per-block counts
        HIP_TRY(c, hipMalloc(&T.peels, align256(rb) + qb), "peel-ray queue");
        T.peel_bytes = rb;
        T.sur_entries = qn;
        T.sur_q = (SurQuery *)((char *)T.peels + align256(rb));
        T.sur_n = (uint32_t *)((char *)T.sur_q + align256(qn * sizeof(SurQuery)));
    }
    if (T_packets < want) {
        uint32_t **lists[3] = {&T.order, &T.keys, &T.sort_tmp};
        for (uint32_t **l : lists) {
            if (*l) (void)hipFree(*l);
            *l = nullptr;
        }
        T_packets = 0;
        T.cap = 0;
        HIP_TRY(c, hipMalloc(&T.order, want * sizeof(uint32_t)), "packet lists");
        HIP_TRY(c, hipMalloc(&T.keys, want * sizeof(uint32_t)), "packet lists");
        HIP_TRY(c, hipMalloc(&T.sort_tmp, 2 * want * sizeof(uint32_t)), "packet lists");
        T_packets = want;
    }
    T.cap = T_packets;
    return QRT_OK;
}

int ensure_queues(qrt_ctx *c, uint64_t count, int n_obs, int precision)
{
    return ensure_buffers(c, c->tb, c->tb_packets, count, n_obs, precision);
}

void free_buffers(TransportBuffers &T)
{
    void *ptrs[] = {T.packets, T.peels, T.q, T.order, T.keys, T.sort_tmp, T.hist};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    T = TransportBuffers{};
}

size_t image_sets(const qrt_ctx *c) { return c->order_images > 0 ? (size_t)c->order_images : 1; }

// Image buffer for the current observers and image sets.  The old buffer is
// freed first (two large image sets need not fit together).  If the new one
// cannot be allocated, the context is left without observers and without
// per-order images, so that no kernel can be launched on a missing buffer
// until qrt_set_observers succeeds again.
int ensure_images(qrt_ctx *c)
{
    const size_t want = c->img_elems * kImageCopies * image_sets(c);
    if (want == c->img_alloc && c->img) return QRT_OK;
    if (c->img) {
        HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
        (void)hipFree(c->img);
        c->img = nullptr;
        c->img_alloc = 0;
    }
    const hipError_t e = hipMalloc(&c->img, want * sizeof(double));
    if (e != hipSuccess) {
        c->img = nullptr;
        c->has_obs = false;
        c->order_images = 0;
        c->img_elems = 0;
        (void)hipGetLastError();   // the failed allocation is reported here, not by a later call
        return hip_fail(c, e, "image allocation");
    }
    c->img_alloc = want;
    return QRT_OK;
}

// fold the copies of every image set into its first copy
int fold_images(qrt_ctx *c)
{
    if (!c->img || !c->has_obs) return fail(c, QRT_BAD_STATE, "no image buffer (set the observers)");
    for (size_t s = 0; s < image_sets(c); ++s)
        HIP_TRY(c, launch_fold_images(c->img + s * kImageCopies * c->img_elems, c->img_elems, c->stream),
                "image fold");
    return QRT_OK;
}

// ---------------------------------------------------------------- allocation-free transport
// qrt_run_static takes every transport buffer (state lists, peel slots, sort
// lists and histograms, queue counters) from one file-scope device array
// instead of context allocations, in chunks of kStaticChunk packets.  Each
// device holds its own copy of the array from the load of the library to the
// end of the process.  In host code `scratch` is only a stand-in for the
// symbol: its device address comes from hipGetSymbolAddress, once per device,
// and only that address is ever handed to kernels.
constexpr uint64_t kStaticChunk = 1ull << 16;
constexpr int kStaticMaxDevices = 64;

std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kStaticMaxDevices] = {};

// device address of the scratch array on `device` (the current device)
hipError_t scratch_address(int device, unsigned char **out)
{
    if (device < 0 || device >= kStaticMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[device] = (unsigned char *)ptr;
    }
    *out = g_scratch_dev[device];
    return hipSuccess;
}

// The transport buffers of one kStaticChunk-packet chunk carved from the
// scratch at base (null: only the size); returns the bytes they take.  The
// surrogate queue is carved only for runs with the surrogate peel-off.
size_t static_buffers(unsigned char *base, int precision, int n_obs, int peel_mode, TransportBuffers &B)
{
    const uint64_t cap = kStaticChunk;
    const size_t pb = packet_state_bytes(precision) * cap * 2;
    const size_t rb = peel_ray_bytes(precision) * (cap + 64) * (size_t)n_obs;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    B = TransportBuffers{};
    B.packets = take(pb);
    B.peels = take(rb);
    const size_t qn = peel_mode == QRT_PEEL_SURROGATE ? sur_queue_entries(cap, n_obs) : 0;
    B.sur_q = qn ? (SurQuery *)take(qn * sizeof(SurQuery)) : nullptr;
    B.sur_n = qn ? (uint32_t *)take(sur_count_entries(cap) * sizeof(uint32_t)) : nullptr;
    B.order = (uint32_t *)take(cap * sizeof(uint32_t));
    B.keys = (uint32_t *)take(cap * sizeof(uint32_t));
    B.sort_tmp = (uint32_t *)take(2 * cap * sizeof(uint32_t));
    B.hist = (uint32_t *)take(kSortHist * sizeof(uint32_t));
    B.q = (Queues *)take(sizeof(Queues));
    B.packet_bytes = pb;
    B.peel_bytes = rb;
    B.sur_entries = qn;
    B.cap = cap;
    return off;
}

}  // namespace

extern "C" {

int qrt_create(qrt_ctx **out, int device, void *hip_stream)
{
    if (!out) return QRT_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return QRT_HIP_ERROR;
    if (device < 0 || device >= ndev) return QRT_INVALID_ARG;
    qrt_ctx *c = new (std::nothrow) qrt_ctx();
    if (!c) return QRT_OUT_OF_MEMORY;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    DeviceGuard dg(device);
    // generator tables: per digital sequence and dimension, the byte tables of
    // its 32 columns ([4][256]: the XOR of the columns that each byte value of
    // the Gray-code index selects), then the Halton bases
    const size_t nbytes = (size_t)kMaxDims * 1024;
    const size_t nt = 2 * nbytes + kMaxDims;
    std::vector<uint32_t> cols(2 * (size_t)kMaxDims * 32, 0u), host(nt, 0u);
    sobol_columns(sobol_table_dims() < kMaxDims ? sobol_table_dims() : kMaxDims, cols.data());
    niederreiter2_columns(kMaxDims, cols.data() + kMaxDims * 32);
    for (int k = 0; k < 2; ++k)
        for (int d = 0; d < kMaxDims; ++d)
            for (int q = 0; q < 4; ++q)
                for (int v = 0; v < 256; ++v) {
                    uint32_t x = 0;
                    for (int b = 0; b < 8; ++b)
                        if ((v >> b) & 1) x ^= cols[((size_t)k * kMaxDims + d) * 32 + 8 * q + b];
                    host[k * nbytes + ((size_t)d * 4 + q) * 256 + v] = x;
                }
    first_primes(kMaxDims, host.data() + 2 * nbytes);
    hipError_t e = hipMalloc(&c->tables, nt * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemcpy(c->tables, host.data(), nt * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&c->counters, kCounterBytes);
    if (e == hipSuccess) e = hipMemset(c->counters, 0, kCounterBytes);
    if (e == hipSuccess) e = hipMalloc(&c->tb.q, sizeof(Queues));
    if (e == hipSuccess) e = hipMalloc(&c->tb.hist, sizeof(uint32_t) * kSortHist);
    // this device's static scratch (looked up once per device, with the device current)
    if (e == hipSuccess) e = scratch_address(device, &c->scratch);
    if (e != hipSuccess) {
        qrt_destroy(c);
        return e == hipErrorOutOfMemory ? QRT_OUT_OF_MEMORY : QRT_HIP_ERROR;
    }
    *out = c;
    return QRT_OK;
}

void qrt_destroy(qrt_ctx *c)
{
    if (!c) return;
    DeviceGuard dg(c->device);
    (void)sync_all(c);
    for (int b = 0; b < kLanes; ++b) {
        if (c->lane[b]) (void)hipStreamDestroy(c->lane[b]);
        if (c->lane_done[b]) (void)hipEventDestroy(c->lane_done[b]);
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
    for (int b = 0; b < kLanes - 1; ++b) free_buffers(c->tbl[b]);
    if (c->grid) (void)hipFree(c->grid);
    if (c->img) (void)hipFree(c->img);
    if (c->tables) (void)hipFree(c->tables);
    if (c->faure) (void)hipFree(c->faure);
    if (c->counters) (void)hipFree(c->counters);
    if (c->tb.packets) (void)hipFree(c->tb.packets);
    if (c->tb.peels) (void)hipFree(c->tb.peels);
    if (c->tb.q) (void)hipFree(c->tb.q);
    if (c->tb.order) (void)hipFree(c->tb.order);
    if (c->tb.keys) (void)hipFree(c->tb.keys);
    if (c->tb.sort_tmp) (void)hipFree(c->tb.sort_tmp);
    if (c->tb.hist) (void)hipFree(c->tb.hist);
    if (c->mlp) (void)hipFree(c->mlp);
    if (c->tiles) (void)hipFree(c->tiles);
    if (c->part) (void)hipFree(c->part);
    if (c->train_x) (void)hipFree(c->train_x);
    if (c->dom_valid) (void)hipFree(c->dom_valid);
    if (c->batch_dev) (void)hipFree(c->batch_dev);
    if (c->batch_grid) (void)hipFree(c->batch_grid);
    if (c->batch_img) (void)hipFree(c->batch_img);
    c->timer.destroy();
    delete c;
}

const char *qrt_last_error(const qrt_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

int qrt_set_stream(qrt_ctx *c, void *hip_stream)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    c->stream = (hipStream_t)hip_stream;
    return QRT_OK;
}

int qrt_set_grid(qrt_ctx *c, int nx, int ny, int nz, const double lo[3], const double hi[3],
                 const float *kappa_rho, int flags)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (nx < 1 || ny < 1 || nz < 1 || !lo || !hi || !kappa_rho)
        return fail(c, QRT_INVALID_ARG, "bad grid arguments");
    const int64_t bricked = mesh_cells(nx, ny, nz);
    if (bricked > (int64_t)1 << 29) return fail(c, QRT_UNSUPPORTED, "grid too large (at most 2^29 stored cells)");
    // a walk counts the faces it crosses per axis in FP32, exactly up to 2^24
    if (nx > kMaxAxisCells || ny > kMaxAxisCells || nz > kMaxAxisCells)
        return fail(c, QRT_UNSUPPORTED, "grid too large (at most 2^20 cells per axis)");
    for (int a = 0; a < 3; ++a)
        if (!(hi[a] > lo[a]) || !isfinite(lo[a]) || !isfinite(hi[a]))
            return fail(c, QRT_INVALID_ARG, "box must satisfy lo < hi on every axis");
    if (flags != QRT_GRID_HOST_COPY && flags != QRT_GRID_DEVICE_COPY && flags != QRT_GRID_DEVICE_BORROW)
        return fail(c, QRT_INVALID_ARG, "unknown grid flag %d", flags);
    const size_t cells = (size_t)nx * ny * nz;
    if (flags == QRT_GRID_HOST_COPY)
        for (size_t i = 0; i < cells; ++i)
            if (!(kappa_rho[i] >= 0.0f) || !isfinite(kappa_rho[i]))
                return fail(c, QRT_INVALID_ARG, "cell %zu is negative or not finite", i);
    DeviceGuard dg(c->device);
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    c->has_grid = false;
    if (c->grid_alloc < (size_t)bricked) {
        if (c->grid) (void)hipFree(c->grid);
        c->grid = nullptr;
        c->grid_alloc = 0;
        HIP_TRY(c, hipMalloc(&c->grid, (size_t)bricked * sizeof(float)), "grid allocation");
        c->grid_alloc = (size_t)bricked;
    }
    int nb[3];
    mesh_bricks(nx, ny, nz, nb);
    const int nbx = nb[0], nby = nb[1];
    if (flags == QRT_GRID_HOST_COPY) {
        std::vector<float> b((size_t)bricked, 0.0f);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    b[(size_t)brick_index(x, y, z, nbx, nby)] = kappa_rho[((size_t)z * ny + y) * nx + x];
        HIP_TRY(c, hipMemcpy(c->grid, b.data(), (size_t)bricked * sizeof(float), hipMemcpyHostToDevice),
                "grid copy");
    } else {
        HIP_TRY(c, hipMemsetAsync(c->grid, 0, (size_t)bricked * sizeof(float), c->stream), "grid clear");
        HIP_TRY(c, launch_to_bricks(kappa_rho, c->grid, nx, ny, nz, c->stream), "grid layout");
        HIP_TRY(c, hipStreamSynchronize(c->stream), "grid copy sync");
    }
    c->n[0] = nx; c->n[1] = ny; c->n[2] = nz;
    for (int a = 0; a < 3; ++a) { c->lo[a] = lo[a]; c->hi[a] = hi[a]; }
    c->has_grid = true;
    return QRT_OK;
}

static bool inside_box(const qrt_ctx *c, double x, double y, double z)
{
    const double p[3] = {x, y, z};
    for (int a = 0; a < 3; ++a)
        if (!(p[a] >= c->lo[a] && p[a] <= c->hi[a])) return false;
    return true;
}

int qrt_set_point_source(qrt_ctx *c, double x, double y, double z)
{
    if (!c) return QRT_INVALID_ARG;
    if (!c->has_grid) return fail(c, QRT_BAD_STATE, "set the grid before the source");
    if (!inside_box(c, x, y, z)) return fail(c, QRT_INVALID_ARG, "the source must lie inside the box");
    c->src_kind = 0;
    c->src[0] = x; c->src[1] = y; c->src[2] = z;
    c->r_star = 0.0;
    c->has_source = true;
    return QRT_OK;
}

int qrt_set_sphere_source(qrt_ctx *c, double x, double y, double z, double radius, int order)
{
    if (!c) return QRT_INVALID_ARG;
    if (!c->has_grid) return fail(c, QRT_BAD_STATE, "set the grid before the source");
    if (order != QRT_EMIT_DIRECT && order != QRT_EMIT_INVERSE)
        return fail(c, QRT_INVALID_ARG, "unknown emission order %d", order);
    if (!(radius > 0.0) || !isfinite(radius)) return fail(c, QRT_INVALID_ARG, "radius must be positive");
    for (int a = 0; a < 3; ++a) {
        const double p = a == 0 ? x : (a == 1 ? y : z);
        if (!(p - radius >= c->lo[a] && p + radius <= c->hi[a]))
            return fail(c, QRT_INVALID_ARG, "the star must lie inside the box");
    }
    c->src_kind = order == QRT_EMIT_INVERSE ? 2 : 1;
    c->src[0] = x; c->src[1] = y; c->src[2] = z;
    c->r_star = radius;
    c->has_source = true;
    return QRT_OK;
}

int qrt_set_dust(qrt_ctx *c, double albedo, double g, double p_lin, double p_circ)
{
    if (!c) return QRT_INVALID_ARG;
    if (!(albedo >= 0.0 && albedo <= 1.0)) return fail(c, QRT_INVALID_ARG, "albedo must be in [0,1]");
    if (!(fabs(g) < 1.0)) return fail(c, QRT_INVALID_ARG, "|g| must be < 1");
    if (!(p_lin >= 0.0 && p_lin <= 1.0)) return fail(c, QRT_INVALID_ARG, "p_lin must be in [0,1]");
    if (p_circ != 0.0) return fail(c, QRT_UNSUPPORTED, "circular polarisation (p_c != 0) is not built");
    c->albedo = albedo;
    c->g = g;
    c->p_lin = p_lin;
    return QRT_OK;
}

int qrt_set_observers(qrt_ctx *c, int n_obs, const double *theta, const double *phi, int npix,
                      double half_width)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (n_obs < 1 || n_obs > QRT_MAX_OBSERVERS || !theta || !phi)
        return fail(c, QRT_INVALID_ARG, "need 1..%d observers", QRT_MAX_OBSERVERS);
    if (npix < 1 || npix > 8192) return fail(c, QRT_INVALID_ARG, "npix must be in 1..8192");
    if (!(half_width > 0.0) || !isfinite(half_width)) return fail(c, QRT_INVALID_ARG, "half_width must be > 0");
    DeviceGuard dg(c->device);
    c->img_elems = (size_t)n_obs * 3 * (size_t)npix * (size_t)npix;   // one copy of one set
    int rc = ensure_images(c);
    if (rc) return rc;
    for (int i = 0; i < n_obs; ++i) {
        c->theta[i] = theta[i];
        c->phi[i] = phi[i];
    }
    c->n_obs = n_obs;
    c->npix = npix;
    c->half_width = half_width;
    c->has_obs = true;
    if (c->dom_valid)   // a mask is validated for given observer directions
        HIP_TRY(c, hipMemsetAsync(c->dom_valid, 0, (size_t)QRT_MAX_OBSERVERS * c->dom_nr * c->dom_nz, c->stream),
                "mask reset");
    return qrt_reset_images(c);
}

int qrt_set_sequence(qrt_ctx *c, int kind, uint64_t seed, uint64_t n_total)
{
    if (!c) return QRT_INVALID_ARG;
    if (kind < QRT_SOBOL || kind > QRT_SOBOL_OWEN) return fail(c, QRT_INVALID_ARG, "unknown sequence kind %d", kind);
    if (kind == QRT_HAMMERSLEY && (n_total < 1 || n_total > 0xFFFFFFFFull))
        return fail(c, QRT_UNSUPPORTED, "Hammersley needs 1 <= N < 2^32");
    c->kind = kind;
    c->seed = seed;
    c->n_total = n_total;
    return QRT_OK;
}

int qrt_set_transport(qrt_ctx *c, int max_orders, double tau_min, int precision, int peel_mode)
{
    if (!c) return QRT_INVALID_ARG;
    if (max_orders < 1) return fail(c, QRT_INVALID_ARG, "max_orders must be >= 1");
    if (c->order_images > 0 && max_orders != c->order_images)
        return fail(c, QRT_BAD_STATE, "turn the per-order images off before changing max_orders");
    if (!(tau_min >= 0.0) || !isfinite(tau_min)) return fail(c, QRT_INVALID_ARG, "tau_min must be >= 0");
    if (precision != QRT_FP32 && precision != QRT_FP64) return fail(c, QRT_INVALID_ARG, "unknown precision");
    if (peel_mode != QRT_PEEL_EXACT && peel_mode != QRT_PEEL_SURROGATE)
        return fail(c, QRT_INVALID_ARG, "unknown peel mode");
    if (peel_mode == QRT_PEEL_SURROGATE && (!c->has_mlp || !c->has_domain))
        return fail(c, QRT_NOT_TRAINED, "the surrogate needs network parameters and a domain");
    c->max_orders = max_orders;
    c->tau_min = tau_min;
    c->precision = precision;
    c->peel_mode = peel_mode;
    return QRT_OK;
}

static DevGrid dev_grid(const qrt_ctx *c)
{
    DevGrid g;
    g.kr = c->grid;
    g.nx = c->n[0]; g.ny = c->n[1]; g.nz = c->n[2];
    mesh_bricks(c->n[0], c->n[1], c->n[2], g.nb);
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = c->lo[a];
        g.hi[a] = c->hi[a];
        g.h[a] = (c->hi[a] - c->lo[a]) / (double)c->n[a];
    }
    return g;
}

// direction o of an observer at (theta, phi) and its image axes
// e_x = (-sin phi, cos phi, 0), e_y = o x e_x (Sec. 3.6)
static DevObserver dev_observer(double theta, double phi)
{
    const double st = sin(theta), ct = cos(theta), sp = sin(phi), cp = cos(phi);
    DevObserver O;
    O.o[0] = st * cp; O.o[1] = st * sp; O.o[2] = ct;
    O.ex[0] = -sp; O.ex[1] = cp; O.ex[2] = 0.0;
    O.ey[0] = O.o[1] * O.ex[2] - O.o[2] * O.ex[1];
    O.ey[1] = O.o[2] * O.ex[0] - O.o[0] * O.ex[2];
    O.ey[2] = O.o[0] * O.ex[1] - O.o[1] * O.ex[0];
    return O;
}

static InputMap input_map(const qrt_ctx *c)
{
    InputMap M;
    memset(&M, 0, sizeof(M));
    for (int a = 0; a < 3; ++a) M.center[a] = c->dom_center[a];
    M.r_out = c->dom_r_out;
    M.h0 = c->dom_h0;
    M.beta = c->dom_beta;
    M.zmax = c->dom_zmax;
    for (int i = 0; i < c->n_obs; ++i) {
        M.obs_in[i][0] = (float)(2.0 * c->theta[i] / 3.14159265358979323846 - 1.0);
        M.obs_in[i][1] = (float)(c->phi[i] / 3.14159265358979323846 - 1.0);
    }
    M.n_obs = c->n_obs;
    return M;
}

static void transport_params(const qrt_ctx *c, TransportParams &P)
{
    memset(&P, 0, sizeof(P));
    P.grid = dev_grid(c);
    P.src_kind = c->src_kind;
    for (int a = 0; a < 3; ++a) P.src[a] = c->src[a];
    P.r_star = c->r_star;
    P.albedo = c->albedo;
    P.g = c->g;
    P.p_lin = c->p_lin;
    P.n_obs = c->n_obs;
    P.npix = c->npix;
    P.half_width = c->half_width;
    for (int i = 0; i < c->n_obs; ++i) P.obs[i] = dev_observer(c->theta[i], c->phi[i]);
    P.seq = seq_params(c, c->kind, c->seed, c->n_total);
    P.max_orders = c->max_orders;
    P.tau_min = c->tau_min;
    P.img = c->img;
    P.order_images = c->order_images;
    P.counters = c->counters;
    P.peel_mode = c->peel_mode;
    P.tail_from = c->tail_from;
    P.def_limit = c->def_limit;
    if (c->has_domain) {
        SurrogateParams &S = P.sur;
        S.in = input_map(c);
        S.r_in = c->dom_r_in;
        S.n_r = c->dom_nr;
        S.n_z = c->dom_nz;
        S.valid = c->dom_valid;
        S.params = c->mlp;
        S.tiles = c->tiles;
    }
}

static int run_checks(qrt_ctx *c, int kind, uint64_t n_total, uint64_t first, uint64_t count)
{
    if (!c->has_grid || !c->has_source || !c->has_obs || !c->img)
        return fail(c, QRT_BAD_STATE, "set grid, source and observers before running");
    if (point_dims(c) > kMaxDims)
        return fail(c, QRT_UNSUPPORTED, "%d point dimensions exceed the %d served", point_dims(c), kMaxDims);
    if (c->peel_mode == QRT_PEEL_SURROGATE && (!c->has_mlp || !c->has_domain))
        return fail(c, QRT_NOT_TRAINED, "the surrogate needs network parameters and a domain");
    return check_index_range(c, kind, n_total, first, count);
}

int qrt_run(qrt_ctx *c, uint64_t first, uint64_t count)
{
    if (!c) return QRT_INVALID_ARG;
    int rc = run_checks(c, c->kind, c->n_total, first, count);
    if (rc) return rc;
    if (count == 0) return QRT_OK;
    DeviceGuard dg(c->device);
    if (c->kind == QRT_FAURE && (rc = ensure_faure(c, point_dims(c)))) return rc;
    TransportParams P;
    transport_params(c, P);
    if (!c->overlap) {
        join_lanes(c);
        rc = ensure_queues(c, count, c->n_obs, c->precision);
        if (rc) return rc;
        // chunks never exceed the queue capacity
        for (uint64_t done = 0; done < count;) {
            const uint64_t n = count - done < c->tb_packets ? count - done : c->tb_packets;
            HIP_TRY(c, launch_transport(P, c->precision, c->kind, first + done, n, c->tb, c->stream,
                                        c->timing ? &c->timer : nullptr),
                    "transport launch");
            done += n;
        }
        c->packets_run += count;
        return QRT_OK;
    }
    // Overlapped: each chunk goes to the next lane (lane_fork, lane_close).
    if ((rc = ensure_lanes(c))) return rc;
    for (uint64_t done = 0; done < count;) {
        const int b = c->next_lane;
        TransportBuffers &T = lane_buffers(c, b);
        uint64_t &T_packets = lane_capacity(c, b);
        if ((rc = ensure_buffers(c, T, T_packets, count - done, c->n_obs, c->precision))) return rc;
        const uint64_t n = count - done < T_packets ? count - done : T_packets;
        if ((rc = lane_fork(c, b))) return rc;
        HIP_TRY(c, launch_transport(P, c->precision, c->kind, first + done, n, T, c->lane[b],
                                    c->timing ? &c->timer : nullptr),
                "transport launch");
        if ((rc = lane_close(c, b))) return rc;
        done += n;
    }
    c->packets_run += count;
    return QRT_OK;
}

int qrt_set_overlap(qrt_ctx *c, int enable)
{
    if (!c) return QRT_INVALID_ARG;
    DeviceGuard dg(c->device);
    join_lanes(c);
    c->overlap = enable != 0;
    return QRT_OK;
}

int qrt_set_tail(qrt_ctx *c, int first_order, uint64_t max_deferred)
{
    if (!c) return QRT_INVALID_ARG;
    if (first_order != 0 && first_order < 2)
        return fail(c, QRT_INVALID_ARG, "the late-order launch starts at order 2 or later (0: off), not %d",
                    first_order);
    DeviceGuard dg(c->device);
    join_lanes(c);
    c->tail_from = first_order;
    c->def_limit = max_deferred;
    return QRT_OK;
}

int qrt_join(qrt_ctx *c)
{
    if (!c) return QRT_INVALID_ARG;
    DeviceGuard dg(c->device);
    join_lanes(c);
    return QRT_OK;
}

int qrt_run_static(qrt_ctx *c, uint64_t first, uint64_t count)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    int rc = run_checks(c, c->kind, c->n_total, first, count);
    if (rc) return rc;
    if (!c->scratch) return fail(c, QRT_HIP_ERROR, "no static scratch on device %d", c->device);
    if (c->kind == QRT_FAURE && !(c->faure && c->faure_dims == point_dims(c)))
        return fail(c, QRT_BAD_STATE,
                    "the Faure tables for %d coordinates are built by qrt_run or qrt_generate_points; "
                    "the allocation-free run does not build them", point_dims(c));
    TransportBuffers B;
    const size_t need = static_buffers(nullptr, c->precision, c->n_obs, c->peel_mode, B);
    if (need > kStaticScratchBytes)
        return fail(c, QRT_UNSUPPORTED,
                    "%d observers at %s need %zu bytes of scratch per chunk of %llu packets; the static "
                    "scratch holds %zu (exact peel-off: at most 4 observers in FP64, 12 in FP32; surrogate "
                    "peel-off: 2 in FP64, 5 in FP32)",
                    c->n_obs, c->precision == QRT_FP64 ? "FP64" : "FP32", need,
                    (unsigned long long)kStaticChunk, kStaticScratchBytes);
    if (count == 0) return QRT_OK;
    DeviceGuard dg(c->device);
    static_buffers(c->scratch, c->precision, c->n_obs, c->peel_mode, B);
    TransportParams P;
    transport_params(c, P);
    for (uint64_t done = 0; done < count;) {
        const uint64_t n = count - done < kStaticChunk ? count - done : kStaticChunk;
        HIP_TRY(c, launch_transport(P, c->precision, c->kind, first + done, n, B, c->stream), "transport launch");
        done += n;
    }
    c->packets_run += count;
    return QRT_OK;
}

int qrt_read_images(qrt_ctx *c, int obs, double *I, double *Q, double *U, int normalized)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_obs) return fail(c, QRT_BAD_STATE, "no observers set");
    if (obs < 0 || obs >= c->n_obs) return fail(c, QRT_INVALID_ARG, "observer %d out of range", obs);
    DeviceGuard dg(c->device);
    const size_t plane = (size_t)c->npix * c->npix;
    int rc = fold_images(c);
    if (rc) return rc;
    double *dst[3] = {I, Q, U};
    std::vector<double> tmp(image_sets(c) > 1 ? plane : 0);
    for (size_t set = 0; set < image_sets(c); ++set) {
        const double *base = c->img + set * kImageCopies * c->img_elems;
        for (int s = 0; s < 3; ++s) {
            if (!dst[s]) continue;
            double *to = set == 0 ? dst[s] : tmp.data();
            HIP_TRY(c, hipMemcpyAsync(to, base + ((size_t)obs * 3 + s) * plane, plane * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream),
                    "image copy");
            if (set > 0) {
                HIP_TRY(c, hipStreamSynchronize(c->stream), "image copy sync");
                for (size_t i = 0; i < plane; ++i) dst[s][i] += tmp[i];
            }
        }
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream), "image copy sync");
    if (normalized && c->packets_run > 0) {
        const double inv = 1.0 / (double)c->packets_run;
        for (int s = 0; s < 3; ++s)
            if (dst[s])
                for (size_t i = 0; i < plane; ++i) dst[s][i] *= inv;
    }
    return QRT_OK;
}

int qrt_image_device_ptr(qrt_ctx *c, double **dev_ptr)
{
    if (!c || !dev_ptr) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_obs) return fail(c, QRT_BAD_STATE, "no observers set");
    if (c->order_images > 0) return fail(c, QRT_BAD_STATE, "per-order images: read them with qrt_read_order_images");
    DeviceGuard dg(c->device);
    int rc = fold_images(c);
    if (rc) return rc;
    *dev_ptr = c->img;
    return QRT_OK;
}

int qrt_set_order_images(qrt_ctx *c, int enable)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_obs) return fail(c, QRT_BAD_STATE, "set the observers first");
    DeviceGuard dg(c->device);
    c->order_images = enable ? c->max_orders : 0;
    int rc = ensure_images(c);
    if (rc) return rc;
    return qrt_reset_images(c);
}

int qrt_read_order_images(qrt_ctx *c, int obs, int order, double *I, double *Q, double *U, int normalized)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_obs) return fail(c, QRT_BAD_STATE, "no observers set");
    if (c->order_images <= 0) return fail(c, QRT_BAD_STATE, "per-order images are off");
    if (obs < 0 || obs >= c->n_obs) return fail(c, QRT_INVALID_ARG, "observer %d out of range", obs);
    if (order < 1 || order > c->order_images) return fail(c, QRT_INVALID_ARG, "order %d out of range", order);
    DeviceGuard dg(c->device);
    const size_t plane = (size_t)c->npix * c->npix;
    int rc = fold_images(c);
    if (rc) return rc;
    const double *base = c->img + (size_t)(order - 1) * kImageCopies * c->img_elems;
    double *dst[3] = {I, Q, U};
    for (int s = 0; s < 3; ++s)
        if (dst[s])
            HIP_TRY(c, hipMemcpyAsync(dst[s], base + ((size_t)obs * 3 + s) * plane, plane * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream),
                    "image copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "image copy sync");
    if (normalized && c->packets_run > 0) {
        const double inv = 1.0 / (double)c->packets_run;
        for (int s = 0; s < 3; ++s)
            if (dst[s])
                for (size_t i = 0; i < plane; ++i) dst[s][i] *= inv;
    }
    return QRT_OK;
}

int qrt_reset_images(qrt_ctx *c)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    DeviceGuard dg(c->device);
    if (c->img)
        HIP_TRY(c, hipMemsetAsync(c->img, 0, c->img_alloc * sizeof(double), c->stream), "image reset");
    HIP_TRY(c, hipMemsetAsync(c->counters, 0, kCounterBytes, c->stream), "counter reset");
    c->packets_run = 0;
    return QRT_OK;
}

int qrt_get_counters(qrt_ctx *c, qrt_counters *out)
{
    if (!c || !out) return QRT_INVALID_ARG;
    join_lanes(c);
    DeviceGuard dg(c->device);
    unsigned long long copies[kCounterCopies][kCounterLine];
    HIP_TRY(c, hipMemcpyAsync(copies, c->counters, sizeof(copies), hipMemcpyDeviceToHost, c->stream), "counter copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "counter copy sync");
    unsigned long long h[CNT_COUNT] = {};
    for (int k = 0; k < kCounterCopies; ++k)
        for (int i = 0; i < CNT_COUNT; ++i) h[i] += copies[k][i];
    out->packets = (int64_t)h[CNT_PACKETS];
    out->visits = (int64_t)h[CNT_VISITS];
    out->peels = (int64_t)h[CNT_PEELS];
    out->peel_rays = (int64_t)h[CNT_PEEL_RAYS];
    out->escapes = (int64_t)h[CNT_ESCAPES];
    out->tau_cuts = (int64_t)h[CNT_TAU_CUTS];
    out->scatterings = (int64_t)h[CNT_SCATTERINGS];
    out->occluded = (int64_t)h[CNT_OCCLUDED];
    out->surrogate = (int64_t)h[CNT_SURROGATE];
    out->fallbacks = (int64_t)h[CNT_FALLBACKS];
    out->visits_first = (int64_t)h[CNT_VISITS_FIRST];
    return QRT_OK;
}

int qrt_set_timing(qrt_ctx *c, int enable)
{
    if (!c) return QRT_INVALID_ARG;
    c->timing = enable != 0;
    return QRT_OK;
}

int qrt_get_timing(qrt_ctx *c, qrt_timing *out, int reset)
{
    if (!c || !out) return QRT_INVALID_ARG;
    join_lanes(c);
    static_assert(QRT_T_CLASSES == TC_COUNT, "timing classes of the ABI and the library agree");
    DeviceGuard dg(c->device);
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "timing sync");
    HIP_TRY(c, c->timer.collect(), "timing events");
    for (int k = 0; k < QRT_T_CLASSES; ++k) {
        out->ms[k] = c->timer.ms[k];
        out->launches[k] = c->timer.launches[k];
    }
    if (reset)
        for (int k = 0; k < QRT_T_CLASSES; ++k) {
            c->timer.ms[k] = 0.0;
            c->timer.launches[k] = 0;
        }
    return QRT_OK;
}

int qrt_generate_points(qrt_ctx *c, int kind, uint64_t seed, uint64_t n_total, uint64_t first, uint64_t count,
                        int dims, uint32_t *out, int out_on_device)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (kind < QRT_SOBOL || kind > QRT_SOBOL_OWEN) return fail(c, QRT_INVALID_ARG, "unknown sequence kind %d", kind);
    if (dims < 1 || dims > kMaxDims) return fail(c, QRT_UNSUPPORTED, "dims must be in 1..%d", kMaxDims);
    if (!out && count) return fail(c, QRT_INVALID_ARG, "null output");
    if (kind == QRT_HAMMERSLEY && (n_total < 1 || n_total > 0xFFFFFFFFull))
        return fail(c, QRT_UNSUPPORTED, "Hammersley needs 1 <= N < 2^32");
    int rc = check_index_range(c, kind, n_total, first, count);
    if (rc) return rc;
    if (count == 0) return QRT_OK;
    DeviceGuard dg(c->device);
    if (kind == QRT_FAURE && (rc = ensure_faure(c, dims))) return rc;
    SeqParams S = seq_params(c, kind, seed, n_total);
    const size_t bytes = (size_t)count * dims * sizeof(uint32_t);
    if (out_on_device) {
        HIP_TRY(c, launch_points(S, kind, first, count, dims, out, c->stream), "points launch");
        return QRT_OK;
    }
    uint32_t *tmp = nullptr;
    HIP_TRY(c, hipMalloc(&tmp, bytes), "points buffer");
    hipError_t e = launch_points(S, kind, first, count, dims, tmp, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(c, e, "points");
    return QRT_OK;
}

int qrt_trace_tau(qrt_ctx *c, int64_t n, const double *p, const double *k, double *tau, int64_t *visits)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_grid) return fail(c, QRT_BAD_STATE, "no grid");
    if (n < 0 || (n > 0 && (!p || !k || !tau))) return fail(c, QRT_INVALID_ARG, "bad ray buffers");
    DeviceGuard dg(c->device);
    HIP_TRY(c, launch_trace_tau(dev_grid(c), c->precision, n, p, k, tau, visits, c->stream), "trace launch");
    return QRT_OK;
}

// ---------------------------------------------------------------- surrogate network

static uint64_t host_splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int ensure_mlp(qrt_ctx *c)
{
    if (c->mlp) return QRT_OK;
    HIP_TRY(c, hipMalloc(&c->mlp, 3 * (size_t)kMlpParams * sizeof(float)), "network parameters");
    HIP_TRY(c, hipMalloc(&c->tiles, (size_t)kMlpTiles * 64 * 16), "weight tiles");
    HIP_TRY(c, hipMemsetAsync(c->tiles, 0, (size_t)kMlpTiles * 64 * 16, c->stream), "weight tiles");
    return QRT_OK;
}

static int ensure_part(qrt_ctx *c, size_t blocks)
{
    const size_t want = blocks * (size_t)kMlpParams;
    if (c->part_elems >= want) return QRT_OK;
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    if (c->part) (void)hipFree(c->part);
    c->part = nullptr;
    c->part_elems = 0;
    HIP_TRY(c, hipMalloc(&c->part, want * sizeof(float)), "gradient buffer");
    c->part_elems = want;
    return QRT_OK;
}

static int ensure_train_x(qrt_ctx *c, size_t n)
{
    const size_t want = n * kMlpIn;
    if (c->train_x_elems >= want) return QRT_OK;
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    if (c->train_x) (void)hipFree(c->train_x);
    c->train_x = nullptr;
    c->train_x_elems = 0;
    HIP_TRY(c, hipMalloc(&c->train_x, want * sizeof(float)), "training inputs");
    c->train_x_elems = want;
    return QRT_OK;
}

// host copy of the domain cell rule used by the kernels
int qrt_mlp_set_params(qrt_ctx *c, const float *params, int64_t n)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!params || n != kMlpParams) return fail(c, QRT_INVALID_ARG, "the network has %d parameters", kMlpParams);
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(params[i])) return fail(c, QRT_INVALID_ARG, "parameter %lld is not finite", (long long)i);
    DeviceGuard dg(c->device);
    int rc = ensure_mlp(c);
    if (rc) return rc;
    HIP_TRY(c, hipMemcpyAsync(c->mlp, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream),
            "parameter copy");
    HIP_TRY(c, hipMemsetAsync(c->mlp + kMlpParams, 0, 2 * (size_t)kMlpParams * sizeof(float), c->stream),
            "moment reset");
    HIP_TRY(c, launch_mlp_pack(c->mlp, c->tiles, c->stream), "tile pack");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "parameter sync");
    c->has_mlp = true;
    c->adam_t = 0;
    return QRT_OK;
}

int qrt_mlp_get_params(qrt_ctx *c, float *params, int64_t n)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!params || n != kMlpParams) return fail(c, QRT_INVALID_ARG, "the network has %d parameters", kMlpParams);
    if (!c->has_mlp) return fail(c, QRT_NOT_TRAINED, "no network parameters");
    DeviceGuard dg(c->device);
    HIP_TRY(c, hipMemcpyAsync(params, c->mlp, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->stream),
            "parameter copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "parameter sync");
    return QRT_OK;
}

int qrt_mlp_init(qrt_ctx *c, uint64_t seed)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    std::vector<float> h(kMlpParams, 0.0f);
    uint64_t st = seed;
    for (int l = 0; l < 5; ++l) {
        const double lim = sqrt(6.0 / (double)mlp_fan_in(l));
        const int nw = mlp_fan_in(l) * mlp_fan_out(l);
        for (int i = 0; i < nw; ++i) {
            const double u = (double)(host_splitmix64(st) >> 11) * 0x1p-53;
            h[mlp_w_off(l) + i] = (float)((2.0 * u - 1.0) * lim);
        }
    }
    return qrt_mlp_set_params(c, h.data(), kMlpParams);
}

int qrt_mlp_forward(qrt_ctx *c, int64_t n, const float *X, float *y)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_mlp) return fail(c, QRT_NOT_TRAINED, "no network parameters");
    if (n < 0 || (n > 0 && (!X || !y))) return fail(c, QRT_INVALID_ARG, "bad buffers");
    DeviceGuard dg(c->device);
    HIP_TRY(c, launch_mlp_forward(c->mlp, c->tiles, X, (uint64_t)n, y, c->stream), "forward launch");
    return QRT_OK;
}

int qrt_mlp_backward(qrt_ctx *c, int64_t n, const float *X, const float *dy, float *grad)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_mlp) return fail(c, QRT_NOT_TRAINED, "no network parameters");
    if (n < 1 || !X || !dy || !grad) return fail(c, QRT_INVALID_ARG, "bad buffers");
    if (n > (int64_t)1 << 24) return fail(c, QRT_UNSUPPORTED, "at most 2^24 rows per call");
    DeviceGuard dg(c->device);
    const int blocks = (int)((n + 63) / 64);
    int rc = ensure_part(c, (size_t)blocks);
    if (rc) return rc;
    MlpBatch sel;
    memset(&sel, 0, sizeof(sel));
    HIP_TRY(c, launch_mlp_grad(1, c->mlp, c->tiles, X, (uint64_t)n, nullptr, dy, sel, blocks, c->part, c->stream),
            "gradient launch");
    HIP_TRY(c, launch_mlp_reduce(c->part, blocks, grad, c->stream), "gradient reduce");
    return QRT_OK;
}

int qrt_surrogate_set_domain(qrt_ctx *c, const double center[3], double r_in, double r_out, double h0, double beta,
                             double zmax_over_h, int n_r, int n_z)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!center || !(r_in >= 0.0) || !(r_out > r_in) || !(h0 > 0.0) || !isfinite(beta) || !(zmax_over_h > 0.0) ||
        !isfinite(r_out) || !isfinite(h0) || !isfinite(zmax_over_h))
        return fail(c, QRT_INVALID_ARG, "bad domain: need 0 <= r_in < r_out, h0 > 0, zmax > 0");
    if (n_r < 1 || n_z < 1 || n_r > 1024 || n_z > 1024) return fail(c, QRT_INVALID_ARG, "bins must be in 1..1024");
    DeviceGuard dg(c->device);
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    if (c->dom_valid) (void)hipFree(c->dom_valid);
    c->dom_valid = nullptr;
    c->has_domain = false;
    const size_t bytes = (size_t)QRT_MAX_OBSERVERS * n_r * n_z;
    HIP_TRY(c, hipMalloc(&c->dom_valid, bytes), "mask allocation");
    HIP_TRY(c, hipMemsetAsync(c->dom_valid, 0, bytes, c->stream), "mask reset");
    for (int a = 0; a < 3; ++a) c->dom_center[a] = center[a];
    c->dom_r_in = r_in; c->dom_r_out = r_out; c->dom_h0 = h0; c->dom_beta = beta; c->dom_zmax = zmax_over_h;
    c->dom_nr = n_r;
    c->dom_nz = n_z;
    c->has_domain = true;
    return QRT_OK;
}

int qrt_surrogate_set_mask(qrt_ctx *c, const uint8_t *mask)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_domain || !c->has_obs) return fail(c, QRT_BAD_STATE, "set observers and a domain first");
    if (!mask) return fail(c, QRT_INVALID_ARG, "null mask");
    DeviceGuard dg(c->device);
    const size_t bytes = (size_t)c->n_obs * c->dom_nr * c->dom_nz;
    HIP_TRY(c, hipMemcpyAsync(c->dom_valid, mask, bytes, hipMemcpyHostToDevice, c->stream), "mask copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "mask sync");
    return QRT_OK;
}

int qrt_surrogate_get_mask(qrt_ctx *c, uint8_t *mask)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_domain || !c->has_obs) return fail(c, QRT_BAD_STATE, "set observers and a domain first");
    if (!mask) return fail(c, QRT_INVALID_ARG, "null mask");
    DeviceGuard dg(c->device);
    const size_t bytes = (size_t)c->n_obs * c->dom_nr * c->dom_nz;
    HIP_TRY(c, hipMemcpyAsync(mask, c->dom_valid, bytes, hipMemcpyDeviceToHost, c->stream), "mask copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "mask sync");
    return QRT_OK;
}

int qrt_surrogate_inputs(qrt_ctx *c, int64_t n, const float *pos_obs, float *X)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_obs || !c->has_domain) return fail(c, QRT_BAD_STATE, "set observers and a domain first");
    if (n < 0 || (n > 0 && (!pos_obs || !X))) return fail(c, QRT_INVALID_ARG, "bad buffers");
    DeviceGuard dg(c->device);
    HIP_TRY(c, launch_mlp_inputs(pos_obs, (uint64_t)n, input_map(c), X, c->stream), "input launch");
    return QRT_OK;
}

int qrt_surrogate_sample(qrt_ctx *c, int64_t n, uint64_t seed, float *pos_obs, float *tau, int64_t *pilot_packets)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_domain) return fail(c, QRT_BAD_STATE, "set a surrogate domain first");
    if (n < 1 || !pos_obs || !tau) return fail(c, QRT_INVALID_ARG, "bad buffers");
    if (n > (int64_t)1 << 26) return fail(c, QRT_UNSUPPORTED, "at most 2^26 samples");
    int rc = run_checks(c, QRT_PHILOX, 0, 1, 1);
    if (rc) return rc;
    DeviceGuard dg(c->device);
    // chunk size: every packet scatters at most max_orders times toward n_obs observers
    const uint64_t per_packet = (uint64_t)c->max_orders * (uint64_t)c->n_obs;
    uint64_t chunk = 1ull << 16;
    while (chunk > 256 && chunk * per_packet > (1ull << 24)) chunk >>= 1;
    const uint64_t capacity = chunk * per_packet;
    rc = ensure_queues(c, chunk, c->n_obs, c->precision);
    if (rc) return rc;
    // the pilot's captured rays stay on the device: each chunk appends to `all`
    // (room for the n wanted plus one chunk's capacity), then the selection,
    // the labels and the copies to the caller's buffers run there too
    const uint64_t want = (uint64_t)n, all_cap = want + capacity;
    float *all = nullptr;
    uint32_t *cap_count = nullptr;
    double *pk = nullptr, *tau64 = nullptr;
    void *temp = nullptr;
    auto release = [&]() {
        if (all) (void)hipFree(all);
        if (cap_count) (void)hipFree(cap_count);
        if (pk) (void)hipFree(pk);
        if (tau64) (void)hipFree(tau64);
        if (temp) (void)hipFree(temp);
    };
    uint64_t m = 0, first = 1;
    int save_mode = c->peel_mode;
    hipError_t e = hipMalloc(&all, all_cap * 4 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&cap_count, sizeof(uint32_t));
    TransportParams P;
    c->peel_mode = QRT_PEEL_EXACT;
    transport_params(c, P);
    c->peel_mode = save_mode;
    P.seq = seq_params(c, QRT_PHILOX, seed, 0);
    P.sur.cap_count = cap_count;
    P.sur.cap_capacity = (uint32_t)capacity;
    // pilot: chunks of Philox packets until enough in-domain peel rays are captured
    while (e == hipSuccess && m < want) {
        if (first > (1ull << 36)) {
            release();
            return fail(c, QRT_UNSUPPORTED, "the pilot finds too few peel-off rays inside the domain");
        }
        uint32_t got = 0;
        P.sur.cap = all + m * 4;
        e = hipMemsetAsync(cap_count, 0, sizeof(uint32_t), c->stream);
        if (e == hipSuccess) e = launch_transport(P, c->precision, QRT_PHILOX, first, chunk, c->tb, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&got, cap_count, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) break;
        m += got < capacity ? got : capacity;   // the capture stops at the chunk's capacity
        first += chunk;
    }
    if (e != hipSuccess) {
        release();
        return hip_fail(c, e, "pilot run");
    }
    // canonical order: the captured rays sorted by a hash of their bytes, the first n kept
    std::vector<DevObserver> obs((size_t)c->n_obs);
    for (int i = 0; i < c->n_obs; ++i) obs[(size_t)i] = dev_observer(c->theta[i], c->phi[i]);
    e = hipMalloc(&temp, sample_select_temp_bytes(m));
    if (e == hipSuccess) e = hipMalloc(&pk, (size_t)n * 6 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&tau64, (size_t)n * sizeof(double));
    if (e == hipSuccess)
        e = launch_sample_select(all, m, (uint64_t)n, seed, obs.data(), c->n_obs, temp, pos_obs, pk, c->stream);
    // labels: exact optical depth toward the observer (FP64 traversal)
    if (e == hipSuccess)
        e = launch_trace_tau(dev_grid(c), QRT_FP64, n, pk, pk + (size_t)n * 3, tau64, nullptr, c->stream);
    if (e == hipSuccess) e = launch_to_float(tau64, tau, (uint64_t)n, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    release();
    if (e != hipSuccess) return hip_fail(c, e, "pilot samples");
    if (pilot_packets) *pilot_packets = (int64_t)(first - 1);
    return qrt_reset_images(c);
}

static double mlp_loss(qrt_ctx *c, const float *X, const float *tau, uint64_t n, float cap, float wfloor, int &rc)
{
    rc = QRT_OK;
    const int parts = mlp_loss_parts(n);
    double *d = nullptr;
    std::vector<double> h((size_t)parts);
    hipError_t e = hipMalloc(&d, (size_t)parts * sizeof(double));
    if (e == hipSuccess) e = launch_mlp_loss(c->mlp, c->tiles, X, tau, n, cap, wfloor, d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, (size_t)parts * sizeof(double), hipMemcpyDeviceToHost,
                                            c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (d) (void)hipFree(d);
    if (e != hipSuccess) {
        rc = hip_fail(c, e, "loss");
        return 0.0;
    }
    double s = 0.0;
    for (double v : h) s += v;
    return n ? s / (double)n : 0.0;
}

int qrt_surrogate_train(qrt_ctx *c, int64_t n, const float *pos_obs, const float *tau, const qrt_train_cfg *cfg,
                        qrt_train_report *rep)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!cfg || n < 1 || !pos_obs || !tau) return fail(c, QRT_INVALID_ARG, "bad arguments");
    if (!c->has_obs || !c->has_domain) return fail(c, QRT_BAD_STATE, "set observers and a domain first");
    if (cfg->steps < 0 || cfg->batch < 64 || cfg->batch > 65536 || cfg->batch % 64)
        return fail(c, QRT_INVALID_ARG, "batch must be a multiple of 64 in 64..65536");
    if (!(cfg->lr > 0.0f) || !(cfg->lr_final >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f) || !(cfg->tau_cap > 0.0f) ||
        !(cfg->weight_floor >= 0.0f))
        return fail(c, QRT_INVALID_ARG, "bad optimiser settings");
    if (!cfg->init && !c->has_mlp) return fail(c, QRT_NOT_TRAINED, "no parameters to continue from");
    int rc = QRT_OK;
    if (cfg->init && (rc = qrt_mlp_init(c, cfg->seed))) return rc;
    DeviceGuard dg(c->device);
    const int blocks = cfg->batch / 64;
    if ((rc = ensure_part(c, (size_t)blocks))) return rc;
    if ((rc = ensure_train_x(c, (size_t)n))) return rc;
    HIP_TRY(c, launch_mlp_inputs(pos_obs, (uint64_t)n, input_map(c), c->train_x, c->stream), "input launch");
    const double l0 = mlp_loss(c, c->train_x, tau, (uint64_t)n, cfg->tau_cap, cfg->weight_floor, rc);
    if (rc) return rc;
    for (int64_t step = 0; step < cfg->steps; ++step) {
        MlpBatch sel;
        sel.seed = cfg->seed;
        sel.step = (uint64_t)(c->adam_t + 1);
        sel.batch = cfg->batch;
        sel.cap = cfg->tau_cap;
        sel.wfloor = cfg->weight_floor;
        HIP_TRY(c, launch_mlp_grad(0, c->mlp, c->tiles, c->train_x, (uint64_t)n, tau, nullptr, sel, blocks, c->part,
                                   c->stream),
                "gradient launch");
        c->adam_t++;
        const double frac = cfg->steps > 1 ? (double)step / (double)(cfg->steps - 1) : 1.0;
        AdamStep A;
        A.lr = (float)(cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + cos(3.14159265358979323846 * frac)));
        A.beta1 = cfg->beta1;
        A.beta2 = cfg->beta2;
        A.eps = cfg->eps;
        A.c1 = (float)(1.0 / (1.0 - pow((double)cfg->beta1, (double)c->adam_t)));
        A.c2 = (float)(1.0 / (1.0 - pow((double)cfg->beta2, (double)c->adam_t)));
        HIP_TRY(c, launch_mlp_adam(c->mlp, c->mlp + kMlpParams, c->mlp + 2 * kMlpParams, c->part, blocks, A, c->tiles,
                                   c->stream),
                "update launch");
    }
    const double l1 = mlp_loss(c, c->train_x, tau, (uint64_t)n, cfg->tau_cap, cfg->weight_floor, rc);
    if (rc) return rc;
    if (rep) {
        rep->loss_first = l0;
        rep->loss_final = l1;
        rep->steps = cfg->steps;
    }
    return QRT_OK;
}

int qrt_surrogate_validate(qrt_ctx *c, int64_t n, const float *pos_obs, const float *tau, double max_err,
                           double floor_frac, int64_t min_count, qrt_mask_report *rep)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!c->has_mlp) return fail(c, QRT_NOT_TRAINED, "no network parameters");
    if (!c->has_domain || !c->has_obs || !c->has_grid) return fail(c, QRT_BAD_STATE, "set grid, observers, domain");
    if (n < 1 || !pos_obs || !tau || !(max_err >= 0.0) || !(floor_frac >= 0.0) || min_count < 1)
        return fail(c, QRT_INVALID_ARG, "bad arguments");
    DeviceGuard dg(c->device);
    int rc = ensure_train_x(c, (size_t)n);
    if (rc) return rc;
    // network outputs, then the per-cell sums, the mask and the report on the device
    const size_t cells = (size_t)c->dom_nr * c->dom_nz;
    const size_t total = (size_t)c->n_obs * cells;
    SurrogateParams S = {};
    S.in = input_map(c);
    S.r_in = c->dom_r_in;
    S.n_r = c->dom_nr;
    S.n_z = c->dom_nz;
    float *y = nullptr;
    void *work = nullptr;
    uint64_t *rep_d = nullptr, rep_h[5] = {0, 0, 0, 0, 0};
    hipError_t e = hipMalloc(&y, (size_t)n * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&work, validate_work_bytes(c->n_obs, cells));
    if (e == hipSuccess) e = hipMalloc(&rep_d, sizeof(rep_h));
    if (e == hipSuccess) e = launch_mlp_inputs(pos_obs, (uint64_t)n, input_map(c), c->train_x, c->stream);
    if (e == hipSuccess) e = launch_mlp_forward(c->mlp, c->tiles, c->train_x, (uint64_t)n, y, c->stream);
    if (e == hipSuccess)
        e = launch_validate(S, c->n_obs, (uint64_t)n, pos_obs, tau, y, max_err, floor_frac, min_count, work,
                            c->dom_valid, rep_d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rep_h, rep_d, sizeof(rep_h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (y) (void)hipFree(y);
    if (work) (void)hipFree(work);
    if (rep_d) (void)hipFree(rep_d);
    if (e != hipSuccess) return hip_fail(c, e, "validation");
    if (rep) {
        rep->cells = (int64_t)total;
        rep->valid_cells = (int64_t)rep_h[1];
        rep->samples = (int64_t)rep_h[2];
        rep->samples_valid = (int64_t)rep_h[3];
        double worst = 0.0;
        memcpy(&worst, &rep_h[4], sizeof(worst));
        rep->max_err_valid = worst;
    }
    return QRT_OK;
}

// ---------------------------------------------------------------- surrogate state

// Blob of a trained surrogate: this header, then theta[n_obs] and phi[n_obs]
// (FP64, the observers the mask was validated for), the FP32 parameters and
// the mask [n_obs][n_r][n_z].
struct SurrogateStateHeader {
    char magic[8];              // "QRTSUR01"
    uint32_t n_params, n_obs;
    int32_t n_r, n_z;
    double center[3];
    double r_in, r_out, h0, beta, zmax;
};
static const char kStateMagic[8] = {'Q', 'R', 'T', 'S', 'U', 'R', '0', '1'};

static size_t state_bytes(uint32_t n_obs, int n_r, int n_z)
{
    return sizeof(SurrogateStateHeader) + 2 * sizeof(double) * n_obs + sizeof(float) * kMlpParams +
           (size_t)n_obs * n_r * n_z;
}

int qrt_surrogate_get_state(qrt_ctx *c, void *blob, size_t *nbytes)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!nbytes) return fail(c, QRT_INVALID_ARG, "null size");
    if (!c->has_mlp || !c->has_domain || !c->has_obs)
        return fail(c, QRT_NOT_TRAINED, "the surrogate needs network parameters, a domain and observers");
    const size_t need = state_bytes((uint32_t)c->n_obs, c->dom_nr, c->dom_nz);
    if (!blob) {
        *nbytes = need;
        return QRT_OK;
    }
    if (*nbytes < need) {
        *nbytes = need;
        return fail(c, QRT_INVALID_ARG, "the state needs %zu bytes", need);
    }
    SurrogateStateHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kStateMagic, sizeof(h.magic));
    h.n_params = kMlpParams;
    h.n_obs = (uint32_t)c->n_obs;
    h.n_r = c->dom_nr;
    h.n_z = c->dom_nz;
    for (int a = 0; a < 3; ++a) h.center[a] = c->dom_center[a];
    h.r_in = c->dom_r_in; h.r_out = c->dom_r_out; h.h0 = c->dom_h0; h.beta = c->dom_beta; h.zmax = c->dom_zmax;
    char *out = (char *)blob;
    memcpy(out, &h, sizeof(h));
    out += sizeof(h);
    memcpy(out, c->theta, sizeof(double) * c->n_obs);
    out += sizeof(double) * c->n_obs;
    memcpy(out, c->phi, sizeof(double) * c->n_obs);
    out += sizeof(double) * c->n_obs;
    int rc = qrt_mlp_get_params(c, (float *)out, kMlpParams);
    if (rc) return rc;
    out += sizeof(float) * kMlpParams;
    rc = qrt_surrogate_get_mask(c, (uint8_t *)out);
    if (rc) return rc;
    *nbytes = need;
    return QRT_OK;
}

int qrt_surrogate_set_state(qrt_ctx *c, const void *blob, size_t nbytes)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (!blob || nbytes < sizeof(SurrogateStateHeader)) return fail(c, QRT_INVALID_ARG, "state too short");
    if (!c->has_obs) return fail(c, QRT_BAD_STATE, "set the observers first");
    SurrogateStateHeader h;
    memcpy(&h, blob, sizeof(h));
    if (memcmp(h.magic, kStateMagic, sizeof(h.magic)) != 0) return fail(c, QRT_INVALID_ARG, "not a surrogate state");
    if (h.n_params != (uint32_t)kMlpParams || h.n_obs < 1 || h.n_obs > QRT_MAX_OBSERVERS || h.n_r < 1 ||
        h.n_z < 1 || h.n_r > 1024 || h.n_z > 1024)
        return fail(c, QRT_INVALID_ARG, "inconsistent surrogate state");
    if (nbytes != state_bytes(h.n_obs, h.n_r, h.n_z)) return fail(c, QRT_INVALID_ARG, "state size mismatch");
    const char *in = (const char *)blob + sizeof(h);
    const double *th = (const double *)(const void *)in;
    const double *ph = th + h.n_obs;
    if ((int)h.n_obs != c->n_obs) return fail(c, QRT_BAD_STATE, "the state is for %u observers", h.n_obs);
    for (int o = 0; o < c->n_obs; ++o) {
        double t, p;
        memcpy(&t, th + o, sizeof(double));
        memcpy(&p, ph + o, sizeof(double));
        if (t != c->theta[o] || p != c->phi[o])
            return fail(c, QRT_BAD_STATE, "observer %d differs from the one the mask was validated for", o);
    }
    in += 2 * sizeof(double) * h.n_obs;
    std::vector<float> params(kMlpParams);
    memcpy(params.data(), in, sizeof(float) * kMlpParams);
    in += sizeof(float) * kMlpParams;
    int rc = qrt_surrogate_set_domain(c, h.center, h.r_in, h.r_out, h.h0, h.beta, h.zmax, h.n_r, h.n_z);
    if (rc) return rc;
    rc = qrt_mlp_set_params(c, params.data(), kMlpParams);
    if (rc) return rc;
    return qrt_surrogate_set_mask(c, (const uint8_t *)in);
}

// ---------------------------------------------------------------- batches of scenes

// checks one scene description; returns its point dimension, or a status < 0
static int batch_scene_check(qrt_ctx *c, int i, const qrt_batch_scene &S)
{
    if (S.nx < 1 || S.ny < 1 || S.nz < 1 || !S.kappa_rho)
        return fail(c, QRT_INVALID_ARG, "scene %d: bad grid arguments", i);
    if (mesh_cells(S.nx, S.ny, S.nz) > (int64_t)1 << 29)
        return fail(c, QRT_UNSUPPORTED, "scene %d: grid too large (at most 2^29 stored cells)", i);
    if (S.nx > kMaxAxisCells || S.ny > kMaxAxisCells || S.nz > kMaxAxisCells)
        return fail(c, QRT_UNSUPPORTED, "scene %d: grid too large (at most 2^20 cells per axis)", i);
    for (int a = 0; a < 3; ++a)
        if (!(S.hi[a] > S.lo[a]) || !isfinite(S.lo[a]) || !isfinite(S.hi[a]))
            return fail(c, QRT_INVALID_ARG, "scene %d: box must satisfy lo < hi on every axis", i);
    const size_t cells = (size_t)S.nx * S.ny * S.nz;
    for (size_t k = 0; k < cells; ++k)
        if (!(S.kappa_rho[k] >= 0.0f) || !isfinite(S.kappa_rho[k]))
            return fail(c, QRT_INVALID_ARG, "scene %d: cell %zu is negative or not finite", i, k);
    if (S.source != QRT_SOURCE_POINT && S.source != QRT_SOURCE_SPHERE)
        return fail(c, QRT_INVALID_ARG, "scene %d: unknown source kind %d", i, S.source);
    const double r = S.source == QRT_SOURCE_SPHERE ? S.radius : 0.0;
    if (S.source == QRT_SOURCE_SPHERE) {
        if (!(S.radius > 0.0) || !isfinite(S.radius)) return fail(c, QRT_INVALID_ARG, "scene %d: radius must be > 0", i);
        if (S.emit_order != QRT_EMIT_DIRECT && S.emit_order != QRT_EMIT_INVERSE)
            return fail(c, QRT_INVALID_ARG, "scene %d: unknown emission order %d", i, S.emit_order);
    }
    for (int a = 0; a < 3; ++a)
        if (!(S.src[a] - r >= S.lo[a] && S.src[a] + r <= S.hi[a]))
            return fail(c, QRT_INVALID_ARG, "scene %d: the source must lie inside the box", i);
    if (!(S.albedo >= 0.0 && S.albedo <= 1.0)) return fail(c, QRT_INVALID_ARG, "scene %d: albedo must be in [0,1]", i);
    if (!(fabs(S.g) < 1.0)) return fail(c, QRT_INVALID_ARG, "scene %d: |g| must be < 1", i);
    if (!(S.p_lin >= 0.0 && S.p_lin <= 1.0)) return fail(c, QRT_INVALID_ARG, "scene %d: p_lin must be in [0,1]", i);
    if (S.n_obs < 1 || S.n_obs > QRT_BATCH_MAX_OBSERVERS)
        return fail(c, QRT_INVALID_ARG, "scene %d: need 1..%d observers", i, QRT_BATCH_MAX_OBSERVERS);
    for (int o = 0; o < S.n_obs; ++o)
        if (!isfinite(S.theta[o]) || !isfinite(S.phi[o]))
            return fail(c, QRT_INVALID_ARG, "scene %d: observer %d direction not finite", i, o);
    if (S.npix < 1 || S.npix > 8192) return fail(c, QRT_INVALID_ARG, "scene %d: npix must be in 1..8192", i);
    if (!(S.half_width > 0.0) || !isfinite(S.half_width))
        return fail(c, QRT_INVALID_ARG, "scene %d: half_width must be > 0", i);
    if (S.max_orders < 1) return fail(c, QRT_INVALID_ARG, "scene %d: max_orders must be >= 1", i);
    const int dims = (S.source == QRT_SOURCE_SPHERE ? 5 : 3) + 3 * (S.max_orders - 1);
    if (dims > kMaxDims)
        return fail(c, QRT_UNSUPPORTED, "scene %d: %d point dimensions exceed the %d served", i, dims, kMaxDims);
    if (!(S.tau_min >= 0.0) || !isfinite(S.tau_min)) return fail(c, QRT_INVALID_ARG, "scene %d: tau_min must be >= 0", i);
    if (S.first < 1) return fail(c, QRT_INVALID_ARG, "scene %d: packet indices start at 1", i);
    if (S.count > 0 && S.first + S.count - 1 < S.first) return fail(c, QRT_INVALID_ARG, "scene %d: index range overflows", i);
    return dims;
}

int qrt_batch_set(qrt_ctx *c, int n_scenes, const qrt_batch_scene *scenes)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (n_scenes < 1 || n_scenes > QRT_BATCH_MAX_SCENES || !scenes)
        return fail(c, QRT_INVALID_ARG, "need 1..%d scenes", QRT_BATCH_MAX_SCENES);
    size_t cells = 0, pixels = 0;
    uint64_t total = 0;
    int max_orders = 0;
    for (int i = 0; i < n_scenes; ++i) {
        const qrt_batch_scene &S = scenes[i];
        const int rc = batch_scene_check(c, i, S);
        if (rc < 0) return rc;
        cells += (size_t)mesh_cells(S.nx, S.ny, S.nz);
        pixels += (size_t)kImageCopies * S.n_obs * 3 * (size_t)S.npix * (size_t)S.npix;
        if (total + S.count < total) return fail(c, QRT_INVALID_ARG, "packet total overflows");
        total += S.count;
        max_orders = std::max(max_orders, S.max_orders);
    }
    DeviceGuard dg(c->device);
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    c->batch.clear();
    c->batch_total = 0;
    if (!c->batch_dev) HIP_TRY(c, hipMalloc(&c->batch_dev, sizeof(BScene) * kMaxBatchScenes), "batch scenes");
    if (c->batch_grid_alloc < cells) {
        if (c->batch_grid) (void)hipFree(c->batch_grid);
        c->batch_grid = nullptr;
        c->batch_grid_alloc = 0;
        HIP_TRY(c, hipMalloc(&c->batch_grid, cells * sizeof(float)), "batch meshes");
        c->batch_grid_alloc = cells;
    }
    if (c->batch_img_alloc < pixels) {
        if (c->batch_img) (void)hipFree(c->batch_img);
        c->batch_img = nullptr;
        c->batch_img_alloc = 0;
        HIP_TRY(c, hipMalloc(&c->batch_img, pixels * sizeof(double)), "batch images");
        c->batch_img_alloc = pixels;
    }
    std::vector<BScene> host((size_t)n_scenes);
    std::vector<uint64_t> begins((size_t)n_scenes);
    size_t grid_off = 0, img_off = 0;
    uint64_t begin = 0;
    for (int i = 0; i < n_scenes; ++i) {
        const qrt_batch_scene &S = scenes[i];
        BScene &B = host[(size_t)i];
        memset(&B, 0, sizeof(B));
        B.n[0] = S.nx; B.n[1] = S.ny; B.n[2] = S.nz;
        mesh_bricks(B.n[0], B.n[1], B.n[2], B.nb);
        const size_t nc = (size_t)B.nb[0] * B.nb[1] * B.nb[2] * (kBrick * kBrick * kBrick);
        std::vector<float> bricked(nc, 0.0f);
        for (int z = 0; z < S.nz; ++z)
            for (int y = 0; y < S.ny; ++y)
                for (int x = 0; x < S.nx; ++x)
                    bricked[(size_t)brick_index(x, y, z, B.nb[0], B.nb[1])] =
                        S.kappa_rho[((size_t)z * S.ny + y) * S.nx + x];
        HIP_TRY(c, hipMemcpy(c->batch_grid + grid_off, bricked.data(), nc * sizeof(float), hipMemcpyHostToDevice),
                "batch mesh copy");
        B.kr = c->batch_grid + grid_off;
        grid_off += nc;
        for (int a = 0; a < 3; ++a) {
            B.lo[a] = S.lo[a];
            B.h[a] = (S.hi[a] - S.lo[a]) / (double)B.n[a];
            B.src[a] = S.src[a];
        }
        B.src_kind = S.source == QRT_SOURCE_SPHERE ? (S.emit_order == QRT_EMIT_INVERSE ? 2 : 1) : 0;
        B.r_star = S.source == QRT_SOURCE_SPHERE ? S.radius : 0.0;
        B.albedo = S.albedo;
        B.g = S.g;
        B.p_lin = S.p_lin;
        B.n_obs = S.n_obs;
        B.npix = S.npix;
        B.half_width = S.half_width;
        for (int o = 0; o < S.n_obs; ++o) B.obs[o] = dev_observer(S.theta[o], S.phi[o]);
        B.max_orders = S.max_orders;
        B.tau_min = S.tau_min;
        B.img = c->batch_img + img_off;
        B.img_set = (uint64_t)S.n_obs * 3 * (uint64_t)S.npix * (uint64_t)S.npix;
        img_off += (size_t)kImageCopies * B.img_set;
        B.first = S.first;
        B.begin = begin;
        begins[(size_t)i] = begin;
        B.count = S.count;
        B.n_total = S.n_total;
        begin += S.count;
    }
    HIP_TRY(c, hipMemcpyAsync(c->batch_dev, host.data(), host.size() * sizeof(BScene), hipMemcpyHostToDevice, c->stream),
            "batch scene copy");
    HIP_TRY(c, hipMemsetAsync(c->batch_img, 0, pixels * sizeof(double), c->stream), "batch image reset");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "batch set sync");
    c->batch.swap(host);
    c->batch_begin.swap(begins);
    c->batch_img_used = pixels;
    c->batch_total = total;
    c->batch_max_orders = max_orders;
    c->batch_runs = 0;
    return QRT_OK;
}

int qrt_batch_run(qrt_ctx *c, int kind, uint64_t seed, int precision)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (c->batch.empty()) return fail(c, QRT_BAD_STATE, "set the batch scenes first");
    if (kind < QRT_SOBOL || kind > QRT_SOBOL_OWEN) return fail(c, QRT_INVALID_ARG, "unknown sequence kind %d", kind);
    if (kind == QRT_FAURE) return fail(c, QRT_UNSUPPORTED, "Faure points are not served in batches");
    if (precision != QRT_FP32 && precision != QRT_FP64) return fail(c, QRT_INVALID_ARG, "unknown precision");
    for (size_t i = 0; i < c->batch.size(); ++i) {
        const BScene &B = c->batch[i];
        if (kind == QRT_HAMMERSLEY && (B.n_total < 1 || B.n_total > 0xFFFFFFFFull))
            return fail(c, QRT_UNSUPPORTED, "scene %zu: Hammersley needs 1 <= N < 2^32", i);
        const int rc = check_index_range(c, kind, B.n_total, B.first, B.count);
        if (rc) return rc;
    }
    c->batch_runs++;
    if (c->batch_total == 0) return QRT_OK;
    DeviceGuard dg(c->device);
    int rc = ensure_queues(c, c->batch_total, kBatchObs, precision);
    if (rc) return rc;
    // overlapped runs: the chunks go round the lanes, each sized to fit every lane's buffers
    const int lanes = c->overlap ? kLanes : 1;
    if (lanes > 1 && (rc = ensure_lanes(c))) return rc;
    size_t peel_bytes = c->tb.peel_bytes;
    uint64_t lane_cap = c->tb_packets;
    for (int b = 1; b < lanes; ++b) {
        if ((rc = ensure_buffers(c, lane_buffers(c, b), lane_capacity(c, b), c->batch_total, kBatchObs, precision)))
            return rc;
        peel_bytes = std::min(peel_bytes, lane_buffers(c, b).peel_bytes);
        lane_cap = std::min(lane_cap, lane_capacity(c, b));
    }
    BatchParams P;
    memset(&P, 0, sizeof(P));
    P.scenes = c->batch_dev;
    P.n_scenes = (int)c->batch.size();
    P.seq = seq_params(c, kind, seed, 0);
    P.max_orders = c->batch_max_orders;
    P.counters = c->counters;
    P.img_base = c->batch_img;
    P.img_key_bits = bits_for(c->batch_img_used);
    P.tail_from = c->tail_from;
    P.def_limit = c->def_limit;
    // the peel-ray buffer split into equal append regions (launch_batch checks that every chunk fits)
    const size_t peel_capacity = peel_bytes / peel_ray_bytes(precision);
    P.group_cap = (uint32_t)std::min<size_t>(peel_capacity / kPeelGroups, 0xFFFFFFFFu);
    // chunks of a multiple of 64 kPeelGroups packets put 64 kBatchObs rays per block in each group
    const uint64_t unit = 64 * kPeelGroups, per_unit = 64 * kBatchObs;
    const uint64_t chunk = std::min<uint64_t>(lane_cap, (P.group_cap / per_unit) * unit);
    if (chunk == 0) return fail(c, QRT_HIP_ERROR, "peel-ray buffer too small for a batch");
    if (lanes == 1) {
        HIP_TRY(c, launch_batch(P, c->batch_begin.data(), precision, kind, 0, c->batch_total, c->tb, chunk, c->stream,
                                c->timing ? &c->timer : nullptr),
                "batch launch");
        return QRT_OK;
    }
    for (uint64_t done = 0; done < c->batch_total;) {
        const uint64_t n = std::min<uint64_t>(chunk, c->batch_total - done);
        const int b = c->next_lane;
        if ((rc = lane_fork(c, b))) return rc;
        HIP_TRY(c, launch_batch(P, c->batch_begin.data(), precision, kind, done, n, lane_buffers(c, b), chunk,
                                c->lane[b], c->timing ? &c->timer : nullptr),
                "batch launch");
        if ((rc = lane_close(c, b))) return rc;
        done += n;
    }
    return QRT_OK;
}

int qrt_batch_read_images(qrt_ctx *c, int scene, int obs, double *I, double *Q, double *U, int normalized)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    if (scene < 0 || scene >= (int)c->batch.size()) return fail(c, QRT_INVALID_ARG, "scene %d out of range", scene);
    const BScene &B = c->batch[(size_t)scene];
    if (obs < 0 || obs >= B.n_obs) return fail(c, QRT_INVALID_ARG, "observer %d out of range", obs);
    DeviceGuard dg(c->device);
    const size_t plane = (size_t)B.npix * B.npix;
    HIP_TRY(c, launch_fold_images(B.img, (size_t)B.img_set, c->stream), "batch image fold");
    double *dst[3] = {I, Q, U};
    for (int s = 0; s < 3; ++s)
        if (dst[s])
            HIP_TRY(c, hipMemcpyAsync(dst[s], B.img + ((size_t)obs * 3 + s) * plane, plane * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream),
                    "batch image copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "batch image copy sync");
    const double n = (double)B.count * (double)c->batch_runs;
    if (normalized && n > 0) {
        const double inv = 1.0 / n;
        for (int s = 0; s < 3; ++s)
            if (dst[s])
                for (size_t i = 0; i < plane; ++i) dst[s][i] *= inv;
    }
    return QRT_OK;
}

int qrt_batch_reset(qrt_ctx *c)
{
    if (!c) return QRT_INVALID_ARG;
    join_lanes(c);
    DeviceGuard dg(c->device);
    if (c->batch_img && c->batch_img_used)
        HIP_TRY(c, hipMemsetAsync(c->batch_img, 0, c->batch_img_used * sizeof(double), c->stream), "batch image reset");
    HIP_TRY(c, hipMemsetAsync(c->counters, 0, kCounterBytes, c->stream), "counter reset");
    c->batch_runs = 0;
    return QRT_OK;
}

}  // extern "C"

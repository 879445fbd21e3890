// C ABI of the library (declared in include/qrt.h): context, argument
// checking, device memory, and the launches of the transport kernels.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "qrt.h"
#include "qrt_internal.h"

namespace qrt {
void niederreiter2_columns(int dims, uint32_t *out);
void first_primes(int count, uint32_t *out);
int sobol_table_dims();
void sobol_columns(int dims, uint32_t *out);
}  // namespace qrt

using namespace qrt;

struct qrt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // mesh
    bool has_grid = false;
    int n[3] = {0, 0, 0};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float *grid = nullptr;
    bool grid_owned = false;
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
    size_t img_elems = 0;
    // sequence and transport
    int kind = QRT_SOBOL;
    uint64_t seed = 0, n_total = 0;
    int max_orders = 1;
    double tau_min = 1e-8;
    int precision = QRT_FP32;
    int peel_mode = QRT_PEEL_EXACT;
    // bookkeeping
    uint32_t *tables = nullptr;              // [sobol kMaxDims*32][nied kMaxDims*32][bases kMaxDims]
    unsigned long long *counters = nullptr;  // [CNT_COUNT]
    TransportBuffers tb = {};                // packet and ray queues of the transport
    uint64_t tb_packets = 0;                 // packets the queues hold
    uint64_t packets_run = 0;
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

int point_dims(const qrt_ctx *c)
{
    return (c->src_kind == 1 ? 5 : 3) + 3 * (c->max_orders - 1);
}

SeqParams seq_params(const qrt_ctx *c, int kind, uint64_t seed, uint64_t n_total)
{
    SeqParams s;
    s.mat = c->tables + (kind == QRT_NIEDERREITER2 ? kMaxDims * 32 : 0);
    s.bases = c->tables + 2 * kMaxDims * 32;
    s.seed = seed;
    s.n_total = n_total;
    return s;
}

int check_index_range(qrt_ctx *c, int kind, uint64_t n_total, uint64_t first, uint64_t count)
{
    if (first < 1) return fail(c, QRT_INVALID_ARG, "packet indices start at 1 (got %llu)", (unsigned long long)first);
    if (count > 0 && first + count - 1 < first) return fail(c, QRT_INVALID_ARG, "index range overflows");
    uint64_t last = count ? first + count - 1 : first;
    if (kind != QRT_PHILOX && last > 0xFFFFFFFFull)
        return fail(c, QRT_UNSUPPORTED, "low-discrepancy indices must stay below 2^32 (last %llu)",
                    (unsigned long long)last);
    if (kind == QRT_HAMMERSLEY && last > n_total)
        return fail(c, QRT_UNSUPPORTED, "Hammersley index %llu beyond N = %llu", (unsigned long long)last,
                    (unsigned long long)n_total);
    return QRT_OK;
}

// Queues for chunks of up to `packets` packets (at most kChunk) at the
// context's precision and observer count; grown on demand, never shrunk.
int ensure_queues(qrt_ctx *c, uint64_t count)
{
    uint64_t want = 1u << 16;
    while (want < count && want < kChunk) want <<= 1;
    if (want > kChunk) want = kChunk;
    const size_t pb = packet_state_bytes(c->precision) * want;
    const size_t rb = peel_ray_bytes(c->precision) * (want + 64) * (size_t)c->n_obs;
    if (c->tb.packet_bytes >= pb && c->tb.peel_bytes >= rb && c->tb_packets >= want) return QRT_OK;
    HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
    if (c->tb.packet_bytes < pb || c->tb_packets < want) {
        if (c->tb.packets) (void)hipFree(c->tb.packets);
        c->tb.packets = nullptr;
        c->tb.packet_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->tb.packets, pb), "packet queue");
        c->tb.packet_bytes = pb;
    }
    if (c->tb.peel_bytes < rb) {
        if (c->tb.peels) (void)hipFree(c->tb.peels);
        c->tb.peels = nullptr;
        c->tb.peel_bytes = 0;
        HIP_TRY(c, hipMalloc(&c->tb.peels, rb), "peel-ray queue");
        c->tb.peel_bytes = rb;
    }
    if (c->tb_packets < want) {
        uint32_t **lists[4] = {&c->tb.live[0], &c->tb.live[1], &c->tb.order, &c->tb.keys};
        for (uint32_t **l : lists) {
            if (*l) (void)hipFree(*l);
            *l = nullptr;
        }
        c->tb_packets = 0;
        for (uint32_t **l : lists) HIP_TRY(c, hipMalloc(l, want * sizeof(uint32_t)), "packet lists");
        c->tb_packets = want;
    }
    return QRT_OK;
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
    // generator tables
    const size_t nt = 2 * (size_t)kMaxDims * 32 + kMaxDims;
    uint32_t *host = new uint32_t[nt];
    memset(host, 0, nt * sizeof(uint32_t));
    sobol_columns(sobol_table_dims() < kMaxDims ? sobol_table_dims() : kMaxDims, host);
    niederreiter2_columns(kMaxDims, host + kMaxDims * 32);
    first_primes(kMaxDims, host + 2 * kMaxDims * 32);
    hipError_t e = hipMalloc(&c->tables, nt * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemcpy(c->tables, host, nt * sizeof(uint32_t), hipMemcpyHostToDevice);
    delete[] host;
    if (e == hipSuccess) e = hipMalloc(&c->counters, CNT_COUNT * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c->counters, 0, CNT_COUNT * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&c->tb.q, sizeof(Queues));
    if (e == hipSuccess) e = hipMalloc(&c->tb.hist, sizeof(uint32_t) << kSortBits);
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
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->grid_owned && c->grid) (void)hipFree(c->grid);
    if (c->img) (void)hipFree(c->img);
    if (c->tables) (void)hipFree(c->tables);
    if (c->counters) (void)hipFree(c->counters);
    if (c->tb.packets) (void)hipFree(c->tb.packets);
    if (c->tb.peels) (void)hipFree(c->tb.peels);
    for (int i = 0; i < 2; ++i)
        if (c->tb.live[i]) (void)hipFree(c->tb.live[i]);
    if (c->tb.q) (void)hipFree(c->tb.q);
    if (c->tb.order) (void)hipFree(c->tb.order);
    if (c->tb.keys) (void)hipFree(c->tb.keys);
    if (c->tb.hist) (void)hipFree(c->tb.hist);
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
    c->stream = (hipStream_t)hip_stream;
    return QRT_OK;
}

int qrt_set_grid(qrt_ctx *c, int nx, int ny, int nz, const double lo[3], const double hi[3],
                 const float *kappa_rho, int flags)
{
    if (!c) return QRT_INVALID_ARG;
    if (nx < 1 || ny < 1 || nz < 1 || !lo || !hi || !kappa_rho)
        return fail(c, QRT_INVALID_ARG, "bad grid arguments");
    if ((int64_t)nx * ny * nz > (int64_t)1 << 31) return fail(c, QRT_UNSUPPORTED, "grid too large");
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
    if (c->grid_owned && c->grid) {
        HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
        (void)hipFree(c->grid);
    }
    c->grid = nullptr;
    c->grid_owned = false;
    c->has_grid = false;
    if (flags == QRT_GRID_DEVICE_BORROW) {
        c->grid = const_cast<float *>(kappa_rho);
    } else {
        HIP_TRY(c, hipMalloc(&c->grid, cells * sizeof(float)), "grid allocation");
        c->grid_owned = true;
        HIP_TRY(c,
                hipMemcpyAsync(c->grid, kappa_rho, cells * sizeof(float),
                               flags == QRT_GRID_HOST_COPY ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                               c->stream),
                "grid copy");
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
    if (order != QRT_EMIT_DIRECT) return fail(c, QRT_UNSUPPORTED, "only the direct emission order is built");
    if (!(radius > 0.0) || !isfinite(radius)) return fail(c, QRT_INVALID_ARG, "radius must be positive");
    for (int a = 0; a < 3; ++a) {
        const double p = a == 0 ? x : (a == 1 ? y : z);
        if (!(p - radius >= c->lo[a] && p + radius <= c->hi[a]))
            return fail(c, QRT_INVALID_ARG, "the star must lie inside the box");
    }
    c->src_kind = 1;
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
    if (n_obs < 1 || n_obs > QRT_MAX_OBSERVERS || !theta || !phi)
        return fail(c, QRT_INVALID_ARG, "need 1..%d observers", QRT_MAX_OBSERVERS);
    if (npix < 1 || npix > 8192) return fail(c, QRT_INVALID_ARG, "npix must be in 1..8192");
    if (!(half_width > 0.0) || !isfinite(half_width)) return fail(c, QRT_INVALID_ARG, "half_width must be > 0");
    DeviceGuard dg(c->device);
    const size_t elems = (size_t)n_obs * 3 * (size_t)npix * (size_t)npix;   // one copy
    if (elems != c->img_elems) {
        if (c->img) {
            HIP_TRY(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize(), "sync");
            (void)hipFree(c->img);
            c->img = nullptr;
            c->img_elems = 0;
        }
        HIP_TRY(c, hipMalloc(&c->img, elems * kImageCopies * sizeof(double)), "image allocation");
        c->img_elems = elems;
    }
    for (int i = 0; i < n_obs; ++i) {
        c->theta[i] = theta[i];
        c->phi[i] = phi[i];
    }
    c->n_obs = n_obs;
    c->npix = npix;
    c->half_width = half_width;
    c->has_obs = true;
    return qrt_reset_images(c);
}

int qrt_set_sequence(qrt_ctx *c, int kind, uint64_t seed, uint64_t n_total)
{
    if (!c) return QRT_INVALID_ARG;
    if (kind < QRT_SOBOL || kind > QRT_PHILOX) return fail(c, QRT_INVALID_ARG, "unknown sequence kind %d", kind);
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
    if (!(tau_min >= 0.0) || !isfinite(tau_min)) return fail(c, QRT_INVALID_ARG, "tau_min must be >= 0");
    if (precision != QRT_FP32 && precision != QRT_FP64) return fail(c, QRT_INVALID_ARG, "unknown precision");
    if (peel_mode != QRT_PEEL_EXACT && peel_mode != QRT_PEEL_SURROGATE)
        return fail(c, QRT_INVALID_ARG, "unknown peel mode");
    if (peel_mode == QRT_PEEL_SURROGATE) return fail(c, QRT_NOT_TRAINED, "no trained surrogate network");
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
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = c->lo[a];
        g.hi[a] = c->hi[a];
        g.h[a] = (c->hi[a] - c->lo[a]) / (double)c->n[a];
    }
    return g;
}

int qrt_run(qrt_ctx *c, uint64_t first, uint64_t count)
{
    if (!c) return QRT_INVALID_ARG;
    if (!c->has_grid || !c->has_source || !c->has_obs)
        return fail(c, QRT_BAD_STATE, "set grid, source and observers before running");
    if (point_dims(c) > kMaxDims)
        return fail(c, QRT_UNSUPPORTED, "%d point dimensions exceed the %d served", point_dims(c), kMaxDims);
    int rc = check_index_range(c, c->kind, c->n_total, first, count);
    if (rc) return rc;
    if (count == 0) return QRT_OK;
    TransportParams P;
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
    for (int i = 0; i < c->n_obs; ++i) {
        const double st = sin(c->theta[i]), ct = cos(c->theta[i]), sp = sin(c->phi[i]), cp = cos(c->phi[i]);
        DevObserver &O = P.obs[i];
        O.o[0] = st * cp; O.o[1] = st * sp; O.o[2] = ct;
        O.ex[0] = -sp; O.ex[1] = cp; O.ex[2] = 0.0;
        O.ey[0] = O.o[1] * O.ex[2] - O.o[2] * O.ex[1];
        O.ey[1] = O.o[2] * O.ex[0] - O.o[0] * O.ex[2];
        O.ey[2] = O.o[0] * O.ex[1] - O.o[1] * O.ex[0];
    }
    P.seq = seq_params(c, c->kind, c->seed, c->n_total);
    P.max_orders = c->max_orders;
    P.tau_min = c->tau_min;
    P.img = c->img;
    P.counters = c->counters;
    DeviceGuard dg(c->device);
    rc = ensure_queues(c, count);
    if (rc) return rc;
    // chunks never exceed the queue capacity
    for (uint64_t done = 0; done < count;) {
        const uint64_t n = count - done < c->tb_packets ? count - done : c->tb_packets;
        HIP_TRY(c, launch_transport(P, c->precision, c->kind, first + done, n, c->tb, c->stream), "transport launch");
        done += n;
    }
    c->packets_run += count;
    return QRT_OK;
}

int qrt_read_images(qrt_ctx *c, int obs, double *I, double *Q, double *U, int normalized)
{
    if (!c) return QRT_INVALID_ARG;
    if (!c->has_obs) return fail(c, QRT_BAD_STATE, "no observers set");
    if (obs < 0 || obs >= c->n_obs) return fail(c, QRT_INVALID_ARG, "observer %d out of range", obs);
    DeviceGuard dg(c->device);
    const size_t plane = (size_t)c->npix * c->npix;
    HIP_TRY(c, launch_fold_images(c->img, c->img_elems, c->stream), "image fold");
    double *dst[3] = {I, Q, U};
    for (int s = 0; s < 3; ++s)
        if (dst[s])
            HIP_TRY(c, hipMemcpyAsync(dst[s], c->img + ((size_t)obs * 3 + s) * plane, plane * sizeof(double),
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

int qrt_image_device_ptr(qrt_ctx *c, double **dev_ptr)
{
    if (!c || !dev_ptr) return QRT_INVALID_ARG;
    if (!c->has_obs) return fail(c, QRT_BAD_STATE, "no observers set");
    DeviceGuard dg(c->device);
    HIP_TRY(c, launch_fold_images(c->img, c->img_elems, c->stream), "image fold");
    *dev_ptr = c->img;
    return QRT_OK;
}

int qrt_reset_images(qrt_ctx *c)
{
    if (!c) return QRT_INVALID_ARG;
    DeviceGuard dg(c->device);
    if (c->img)
        HIP_TRY(c, hipMemsetAsync(c->img, 0, c->img_elems * kImageCopies * sizeof(double), c->stream), "image reset");
    HIP_TRY(c, hipMemsetAsync(c->counters, 0, CNT_COUNT * sizeof(unsigned long long), c->stream), "counter reset");
    c->packets_run = 0;
    return QRT_OK;
}

int qrt_get_counters(qrt_ctx *c, qrt_counters *out)
{
    if (!c || !out) return QRT_INVALID_ARG;
    DeviceGuard dg(c->device);
    unsigned long long h[CNT_COUNT];
    HIP_TRY(c, hipMemcpyAsync(h, c->counters, sizeof(h), hipMemcpyDeviceToHost, c->stream), "counter copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "counter copy sync");
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
    return QRT_OK;
}

int qrt_generate_points(qrt_ctx *c, int kind, uint64_t seed, uint64_t n_total, uint64_t first, uint64_t count,
                        int dims, uint32_t *out, int out_on_device)
{
    if (!c) return QRT_INVALID_ARG;
    if (kind < QRT_SOBOL || kind > QRT_PHILOX) return fail(c, QRT_INVALID_ARG, "unknown sequence kind %d", kind);
    if (dims < 1 || dims > kMaxDims) return fail(c, QRT_UNSUPPORTED, "dims must be in 1..%d", kMaxDims);
    if (!out && count) return fail(c, QRT_INVALID_ARG, "null output");
    if (kind == QRT_HAMMERSLEY && (n_total < 1 || n_total > 0xFFFFFFFFull))
        return fail(c, QRT_UNSUPPORTED, "Hammersley needs 1 <= N < 2^32");
    int rc = check_index_range(c, kind, n_total, first, count);
    if (rc) return rc;
    if (count == 0) return QRT_OK;
    DeviceGuard dg(c->device);
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
    if (!c->has_grid) return fail(c, QRT_BAD_STATE, "no grid");
    if (n < 0 || (n > 0 && (!p || !k || !tau))) return fail(c, QRT_INVALID_ARG, "bad ray buffers");
    DeviceGuard dg(c->device);
    HIP_TRY(c, launch_trace_tau(dev_grid(c), c->precision, n, p, k, tau, visits, c->stream), "trace launch");
    return QRT_OK;
}

}  // extern "C"

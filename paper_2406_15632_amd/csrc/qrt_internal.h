// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qrt_seq.h"
#include "qrt_walk.h"

namespace qrt {

constexpr int kMaxDims = 128;
constexpr int kMaxObs = 16;

// counter slots in the device counter array
enum CounterSlot {
    CNT_PACKETS = 0, CNT_VISITS, CNT_PEELS, CNT_PEEL_RAYS, CNT_ESCAPES, CNT_TAU_CUTS,
    CNT_SCATTERINGS, CNT_OCCLUDED, CNT_SURROGATE, CNT_FALLBACKS, CNT_COUNT
};

struct DevObserver {
    double o[3], ex[3], ey[3];
};

struct TransportParams {
    DevGrid grid;
    int src_kind;            // 0 point, 1 sphere
    double src[3];
    double r_star;
    double albedo, g, p_lin;
    int n_obs, npix;
    double half_width;
    DevObserver obs[kMaxObs];
    SeqParams seq;
    int max_orders;
    double tau_min;
    double *img;                   // [n_obs][3][npix][npix]
    unsigned long long *counters;  // [CNT_COUNT]
};

// transport launcher: precision 0 = FP32, 1 = FP64
// persistent transport kernel; work is a device counter the launch resets
hipError_t launch_transport(const TransportParams &P, int precision, int kind, uint64_t first,
                            uint64_t count, int grid_blocks, unsigned long long *work, hipStream_t stream);

hipError_t launch_points(const SeqParams &S, int kind, uint64_t first, uint64_t count, int dims,
                         uint32_t *out, hipStream_t stream);

hipError_t launch_trace_tau(const DevGrid &g, int precision, int64_t n, const double *p,
                            const double *k, double *tau, int64_t *visits, hipStream_t stream);

}  // namespace qrt

// Training data of the peel-off surrogate, on the device.  The surrogate is
// an addition to the method of Shulman, "Quasi-Monte Carlo Radiative
// Transfer": it learns the optical depth of a peel-off ray (Sec. 3.4, 3.6).
// Here: the canonical selection of the pilot's captured peel-off rays, and the
// validity mask of a trained network from validation samples.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "qrt_internal.h"

namespace qrt {

namespace {

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

// observers passed by value (a kernel argument of about 1 KiB)
struct ObsArg {
    DevObserver o[kMaxObs];
    int n_obs;
};

// key j = hash of the ray's 16 bytes (as two little-endian words) and the seed
__global__ void __launch_bounds__(256) k_sample_keys(const float4 *__restrict__ rays, uint64_t m, uint64_t seed,
                                                     uint64_t *__restrict__ keys, uint32_t *__restrict__ idx)
{
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (uint64_t)gridDim.x * blockDim.x) {
        const float4 r = rays[j];
        const uint64_t a = (uint64_t)__float_as_uint(r.x) | ((uint64_t)__float_as_uint(r.y) << 32);
        const uint64_t b = (uint64_t)__float_as_uint(r.z) | ((uint64_t)__float_as_uint(r.w) << 32);
        keys[j] = splitmix64_mix(a ^ (b * 0xD6E8FEB86659FD93ull) ^ seed);
        idx[j] = (uint32_t)j;
    }
}

// the first n rays in key order, and their points and observer directions in FP64
__global__ void __launch_bounds__(256) k_sample_gather(const float4 *__restrict__ rays,
                                                       const uint32_t *__restrict__ order, uint64_t n, const ObsArg O,
                                                       float4 *__restrict__ out, double *__restrict__ pk)
{
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
        const float4 r = rays[order[j]];
        out[j] = r;
        int ob = (int)r.w;
        ob = ob < 0 ? 0 : (ob >= O.n_obs ? O.n_obs - 1 : ob);
        double *p = pk + 3 * j, *k = pk + 3 * n + 3 * j;
        p[0] = (double)r.x; p[1] = (double)r.y; p[2] = (double)r.z;
        for (int a = 0; a < 3; ++a) k[a] = O.o[ob].o[a];
    }
}

__global__ void __launch_bounds__(256) k_to_float(const double *__restrict__ src, float *__restrict__ dst, uint64_t n)
{
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x)
        dst[j] = (float)src[j];
}

int grid_for(uint64_t n) { return (int)std::min<uint64_t>((n + 255) / 256, 4096); }

// ------------------------------------------------------------ validity mask
// Work buffer: t_sum[n_obs], t_cnt[n_obs], then num, den, cnt [n_obs * cells],
// all uint64; sums in fixed point (value * scale, rounded), so that they do
// not depend on the order of the atomics.
struct ValWork {
    uint64_t *t_sum, *t_cnt, *num, *den, *cnt;
};

ValWork val_work(void *work, int n_obs, size_t cells)
{
    uint64_t *w = (uint64_t *)work;
    const size_t total = (size_t)n_obs * cells;
    return ValWork{w, w + n_obs, w + 2 * n_obs, w + 2 * n_obs + total, w + 2 * n_obs + 2 * total};
}

__device__ __forceinline__ int sample_cell(const SurrogateParams &S, int n_obs, const float4 &r, int &ob)
{
    ob = (int)r.w;
    if (ob < 0 || ob >= n_obs) return -1;
    return dom_cell(S, (double)r.x, (double)r.y, (double)r.z);
}

// mean transmission per observer over the samples inside the domain
__global__ void __launch_bounds__(256) k_val_mean(const SurrogateParams S, int n_obs, uint64_t n,
                                                  const float4 *__restrict__ pos, const float *__restrict__ tau,
                                                  double scale, ValWork V, uint64_t *__restrict__ rep)
{
    uint64_t inside = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
        int ob = 0;
        if (sample_cell(S, n_obs, pos[j], ob) < 0) continue;
        inside++;
        atomicAdd((unsigned long long *)&V.t_sum[ob], (unsigned long long)llrint(exp(-(double)tau[j]) * scale));
        atomicAdd((unsigned long long *)&V.t_cnt[ob], 1ull);
    }
    if (inside) atomicAdd((unsigned long long *)&rep[2], (unsigned long long)inside);
}

__global__ void __launch_bounds__(256) k_val_cells(const SurrogateParams S, int n_obs, uint64_t n,
                                                   const float4 *__restrict__ pos, const float *__restrict__ tau,
                                                   const float *__restrict__ y, double floor_frac, double scale,
                                                   ValWork V)
{
    const size_t cells = (size_t)S.n_r * (size_t)S.n_z;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x) {
        int ob = 0;
        const int cell = sample_cell(S, n_obs, pos[j], ob);
        if (cell < 0) continue;
        const double mean = (double)V.t_sum[ob] / scale / (double)V.t_cnt[ob];
        const double floor_t = floor_frac * mean;
        const double T = exp(-(double)tau[j]);
        const double Th = exp(-(double)(y[j] > 0.0f ? y[j] : 0.0f));
        const size_t k = (size_t)ob * cells + (size_t)cell;
        atomicAdd((unsigned long long *)&V.num[k], (unsigned long long)llrint(fabs(Th - T) * scale));
        atomicAdd((unsigned long long *)&V.den[k], (unsigned long long)llrint((T > floor_t ? T : floor_t) * scale));
        atomicAdd((unsigned long long *)&V.cnt[k], 1ull);
    }
}

__global__ void __launch_bounds__(256) k_val_mask(size_t total, ValWork V, double max_err, int64_t min_count,
                                                  uint8_t *__restrict__ mask, uint64_t *__restrict__ rep)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        const double num = (double)V.num[k], den = (double)V.den[k];
        const bool ok = (int64_t)V.cnt[k] >= min_count && den > 0.0 && num <= max_err * den;
        mask[k] = ok ? 1 : 0;
        if (ok) {
            atomicAdd((unsigned long long *)&rep[1], 1ull);
            atomicAdd((unsigned long long *)&rep[3], (unsigned long long)V.cnt[k]);
            // non-negative doubles order as their bit patterns
            atomicMax((unsigned long long *)&rep[4], (unsigned long long)__double_as_longlong(num / den));
        }
    }
}

}  // namespace

size_t sample_select_temp_bytes(uint64_t m)
{
    size_t cub = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, cub, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)m, 0, 64);
    return 2 * round256(m * sizeof(uint64_t)) + 2 * round256(m * sizeof(uint32_t)) + round256(cub);
}

hipError_t launch_sample_select(const float *rays, uint64_t m, uint64_t n, uint64_t seed, const DevObserver *obs,
                                int n_obs, void *temp, float *out, double *pk, hipStream_t st)
{
    if (n > m || m > 0x7FFFFFFFull || n_obs < 1 || n_obs > kMaxObs) return hipErrorInvalidValue;
    char *t = (char *)temp;
    uint64_t *keys_in = (uint64_t *)t;
    t += round256(m * sizeof(uint64_t));
    uint64_t *keys_out = (uint64_t *)t;
    t += round256(m * sizeof(uint64_t));
    uint32_t *idx_in = (uint32_t *)t;
    t += round256(m * sizeof(uint32_t));
    uint32_t *idx_out = (uint32_t *)t;
    t += round256(m * sizeof(uint32_t));
    size_t cub = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, cub, keys_in, keys_out, idx_in, idx_out, (int)m, 0, 64,
                                                      st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sample_keys, dim3(grid_for(m)), dim3(256), 0, st, (const float4 *)rays, m, seed, keys_in,
                       idx_in);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = hipcub::DeviceRadixSort::SortPairs((void *)t, cub, keys_in, keys_out, idx_in, idx_out, (int)m, 0, 64, st);
    if (e != hipSuccess) return e;
    ObsArg O;
    for (int i = 0; i < n_obs; ++i) O.o[i] = obs[i];
    O.n_obs = n_obs;
    hipLaunchKernelGGL(k_sample_gather, dim3(grid_for(n)), dim3(256), 0, st, (const float4 *)rays,
                       (const uint32_t *)idx_out, n, O, (float4 *)out, pk);
    return hipGetLastError();
}

hipError_t launch_to_float(const double *src, float *dst, uint64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_float, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

size_t validate_work_bytes(int n_obs, size_t cells) { return (2 * (size_t)n_obs + 3 * (size_t)n_obs * cells) * 8; }

hipError_t launch_validate(const SurrogateParams &S, int n_obs, uint64_t n, const float *pos_obs, const float *tau,
                           const float *y, double max_err, double floor_frac, int64_t min_count, void *work,
                           uint8_t *mask, uint64_t *rep, hipStream_t st)
{
    const size_t cells = (size_t)S.n_r * (size_t)S.n_z;
    const size_t total = (size_t)n_obs * cells;
    // fixed-point scale 2^k: n values of at most max(1, floor_frac) stay below 2^62
    const double vmax = floor_frac > 1.0 ? floor_frac : 1.0;
    int k = 40;
    while (k > 8 && (double)n * vmax * ldexp(1.0, k) >= ldexp(1.0, 62)) --k;
    const double scale = ldexp(1.0, k);
    hipError_t e = hipMemsetAsync(work, 0, validate_work_bytes(n_obs, cells), st);
    if (e == hipSuccess) e = hipMemsetAsync(rep, 0, 5 * sizeof(uint64_t), st);
    if (e != hipSuccess) return e;
    const ValWork V = val_work(work, n_obs, cells);
    hipLaunchKernelGGL(k_val_mean, dim3(grid_for(n)), dim3(256), 0, st, S, n_obs, n, (const float4 *)pos_obs, tau,
                       scale, V, rep);
    hipLaunchKernelGGL(k_val_cells, dim3(grid_for(n)), dim3(256), 0, st, S, n_obs, n, (const float4 *)pos_obs, tau,
                       y, floor_frac, scale, V);
    hipLaunchKernelGGL(k_val_mask, dim3(grid_for(total)), dim3(256), 0, st, total, V, max_err, min_count, mask, rep);
    return hipGetLastError();
}

}  // namespace qrt

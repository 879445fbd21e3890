// Wave-level building blocks shared by the transport kernels: work pool of the
// persistent kernels, counter flushes, peel-off slot layout and the
// emission-direction key of the coherence sort.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qrt_internal.h"
#include "qrt_physics.h"

namespace qrt {

constexpr int kWalkBatch = 8;     // steps per load batch of the first flights
constexpr int kBatchWalkBatch = 6; // the same in batches (eight would take the kernel to two waves per SIMD)
constexpr int kFlightBatch = 12;  // steps per load batch of the per-order walks (which run at low occupancy)
constexpr int kTailBatch = 8;     // the same in the late-order launch (flights of a few cells in thick scenes)

// The late-order launch walks its flights until this share of them (in
// eighths) has ended, then lets those lanes scatter and take new packets: a
// lower share runs the scattering events at fewer active lanes, a higher one
// leaves more lanes idle in the walk.  Five eighths measured best over thin
// and thick discs and the uneven batch.
constexpr int kTailDoneEighths = 5;

// Blocks per CU of the per-order walk kernels (measured): at most three.  With
// fewer waves the CU's vector L1 cache keeps more of each lane's current lines
// between steps; with two, the misses' latency shows.  Only orders that walk
// flights are limited: the peel rays of the last order run side by side and
// want every wave.  The FP32 walk's registers allow three blocks per CU
// themselves, so the limit binds only for a leaner build of the kernel.
constexpr int kWalkBlocksPerCu = 3;

// compute units of the current device (read once)
inline int device_cu_count()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        (void)hipGetDevice(&dev);
        cus = (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
                  ? prop.multiProcessorCount : 256;
    }
    return cus;
}

constexpr uint32_t kNoPixel = 0xFFFFFFFFu;   // a peel ray that is off the image or blocked

__host__ __device__ __forceinline__ size_t peel_slot(uint32_t i, int ob, int n_obs)
{
    return ((size_t)(i >> 6) * (size_t)n_obs + (size_t)ob) * 64 + (i & 63);
}
constexpr int kWaveRefill = 64;   // refill a wave once all its lanes are idle: keeps its rays coherent

// Adds the per-lane values v[i] to counter slots slot[i]: summed over the
// wave, then over the block in LDS, then one atomic per block and slot into
// the block's copy of the counters.  A device-wide atomic per wave would put
// thousands of read-modify-writes on one line at the end of every launch.
// Every thread of the block calls it.
template <int N>
__device__ __forceinline__ void flush_counters(unsigned long long *counters, const int (&slot)[N],
                                               const uint64_t (&v)[N])
{
    __shared__ unsigned long long s_sum[N];
    if (threadIdx.x < N) s_sum[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint64_t s = wave_sum_u64(v[i]);
        if ((threadIdx.x & 63) == 0 && s) atomicAdd(&s_sum[i], (unsigned long long)s);
    }
    __syncthreads();
    if (threadIdx.x < N && s_sum[threadIdx.x])
        atomicAdd(counters + (blockIdx.x % kCounterCopies) * kCounterLine + slot[threadIdx.x], s_sum[threadIdx.x]);
}

// Wave-uniform pool of work items [next, end), taken a block at a time: the
// first block of every wave is fixed by its wave index (no atomic at start-up,
// when every wave would hit the same counter at once).  The items after the
// fixed blocks are split into kPoolParts equal parts, each with its own counter
// on its own 128-byte line: a wave draws from the part of its block index
// modulo kPoolParts (workgroups go to the XCDs in turn, so that each XCD has a
// part of its own) and, once that part is spent, from the next ones.  Atomics
// on one counter are a serial point; parts divide them by kPoolParts, and large
// launches take bigger blocks still.
constexpr int kPoolParts = 8;
constexpr int kPoolStride = 16;   // counters per 128-byte line

__device__ __forceinline__ uint64_t pool_block(uint64_t total, uint64_t nwaves)
{
    const uint64_t per_wave = total / nwaves;
    return per_wave >= 8192 ? 512 : (per_wave >= 2048 ? 256 : (per_wave >= 512 ? 128 : 64));
}

struct WorkPool {
    uint64_t next = 0, end = 0;
    bool dry = false, started = false;
    int part = 0, tried = 0;

    // next block of this wave; false once every part is spent
    __device__ __forceinline__ bool refill(uint64_t total, unsigned long long *ctr)
    {
        const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
        const uint64_t blk = pool_block(total, nwaves);
        const uint64_t fixed = nwaves * blk;
        if (!started) {
            started = true;
            part = (int)(blockIdx.x % kPoolParts);
            const uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * blk;
            if (base < total) {
                next = base;
                end = base + blk < total ? base + blk : total;
                return true;
            }
        }
        const uint64_t rest = total > fixed ? total - fixed : 0;
        // parts start on block boundaries, so a wave's 64 items stay inside one
        // aligned group of 64 (the peel rays of 64 packets toward one observer)
        const uint64_t len = ((rest + kPoolParts - 1) / kPoolParts + blk - 1) / blk * blk;
        while (tried < kPoolParts) {
            const uint64_t lo = fixed + (uint64_t)part * len;
            const uint64_t hi = lo + len < total ? lo + len : total;
            if (lo < hi) {
                unsigned long long b = 0;
                if ((threadIdx.x & 63) == 0) b = atomicAdd(ctr + part * kPoolStride, (unsigned long long)blk);
                const uint64_t base = lo + __shfl(b, 0, 64);
                if (base < hi) {
                    next = base;
                    end = base + blk < hi ? base + blk : hi;
                    return true;
                }
            }
            part = part + 1 == kPoolParts ? 0 : part + 1;
            ++tried;
        }
        return false;
    }

    // returns true for a lane that received an item (in `item`); ctr points at
    // the pool's kPoolParts counters, kPoolStride apart
    __device__ __forceinline__ bool take(bool want, uint64_t total, unsigned long long *ctr, uint64_t &item)
    {
        bool got = false;
        uint64_t need = __ballot(want);
        while (need && !dry) {
            if (next >= end && !refill(total, ctr)) {
                dry = true;
                break;
            }
            const uint64_t avail = end - next;
            const uint64_t n = (uint64_t)__popcll(need);
            const uint64_t take_n = n < avail ? n : avail;
            const uint64_t rank = (uint64_t)__popcll(need & lanes_below_mask());
            if (want && !got && rank < take_n) {
                item = next + rank;
                got = true;
            }
            next += take_n;
            need = __ballot(want && !got);
        }
        return got;
    }
};

// The per-order walks' items in blocks of kOrderBlock, block b of the nfull
// whole blocks handed out as block (b * stride) mod nfull, stride = p mod nfull
// with p = 2^31 - 1: p is prime and larger than any block count, so the map is
// a bijection.  Neighbouring list entries come from neighbouring emission
// directions (and, in a batch, from one scene), so waves that take consecutive
// blocks at the same time would work in one part of one mesh; strided blocks
// spread them over it.  A block's
// items stay together, as do the items of a partial last block: a wave's
// successive rounds inside one block keep to one region.
constexpr int kOrderBlockLog2 = 9;
constexpr uint64_t kOrderBlock = 1ull << kOrderBlockLog2;

__host__ __device__ inline uint64_t block_stride(uint64_t nfull)
{
    return nfull ? 2147483647ull % nfull : 1;
}

__host__ __device__ inline uint64_t scatter_block(uint64_t item, uint64_t total, uint64_t stride)
{
    const uint64_t nfull = total >> kOrderBlockLog2, b = item >> kOrderBlockLog2;
    if (b >= nfull) return item;
    return (((b * stride) % nfull) << kOrderBlockLog2) | (item & (kOrderBlock - 1));
}

// The items deferred by the late-order launch (scatterings) lie in kPoolParts
// regions of def_cap items each, region r holding min(n_def[r], def_cap) of
// them: item i of a launch over all of them is item i - start[r] of the region
// r with start[r] <= i < end[r].
struct DeferredList {
    uint64_t end[kPoolParts];
    uint32_t cap;
};

__device__ __forceinline__ DeferredList deferred_list(const Queues *Q, uint32_t def_cap)
{
    DeferredList d;
    d.cap = def_cap;
    uint64_t acc = 0;
    for (int r = 0; r < kPoolParts; ++r) {
        const uint32_t n = Q->n_def[r][0];
        acc += n < def_cap ? n : def_cap;
        d.end[r] = acc;
    }
    return d;
}

__device__ __forceinline__ uint64_t deferred_slot(const DeferredList &d, uint64_t item)
{
    uint64_t start = 0, slot = 0;
    bool found = false;
#pragma unroll
    for (int r = 0; r < kPoolParts; ++r) {
        const bool here = !found && item < d.end[r];
        slot = here ? (uint64_t)r * d.cap + (item - start) : slot;
        found = found || here;
        start = d.end[r];
    }
    return slot;
}

// orders the wave's LDS accesses before and after this point
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Image contributions of a wave, merged by pixel before the FP64 atomics.
// Every lane with `on` adds (v0, v1, v2) to base[key], base[key + plane],
// base[key + 2 plane].  Lanes of the wave that hold the same key are found
// with one ballot per key bit; the lowest of them gathers the others' values
// in the wave's LDS scratch (LDS atomics) and issues the three global atomics
// alone.  Neighbouring packets' peel rays toward one observer often land in
// one pixel, and same-address atomics serialize.  Called by every lane of the
// wave; key < 2^key_bits.  Equal keys must mean equal addresses (and planes).
__device__ __forceinline__ void wave_merge_add(bool on, uint64_t key, double v0, double v1, double v2, double *base,
                                               size_t plane, int key_bits, double (*scratch)[3])
{
    uint64_t peers = __ballot(on);
    for (int b = 0; b < key_bits; ++b) {
        const bool one = (key >> b) & 1ull;
        const uint64_t m = __ballot(on && one);
        peers &= one ? m : ~m;
    }
    const int lane = (int)(threadIdx.x & 63);
    const bool lead = on && (peers & lanes_below_mask()) == 0;
    if (__ballot(on && !lead) != 0) {
        const int leader = on ? (int)__builtin_ctzll(peers) : lane;
        if (lead) {
            scratch[lane][0] = v0;
            scratch[lane][1] = v1;
            scratch[lane][2] = v2;
        }
        wave_lds_sync();
        if (on && !lead) {
            atomicAdd(&scratch[leader][0], v0);
            atomicAdd(&scratch[leader][1], v1);
            atomicAdd(&scratch[leader][2], v2);
        }
        wave_lds_sync();
        if (lead) {
            v0 = scratch[lane][0];
            v1 = scratch[lane][1];
            v2 = scratch[lane][2];
        }
        wave_lds_sync();
    }
    if (lead) {
        double *dst = base + key;
        unsafeAtomicAdd(dst, v0);
        unsafeAtomicAdd(dst + plane, v1);
        unsafeAtomicAdd(dst + 2 * plane, v2);
    }
}

// Sort key of a deferred scattering of the late-order launch: the cell of a
// 32^3 grid over the box that holds the scattering point, in Morton order (15
// bits).  Sorted by these keys, a wave of the deferred walk takes the peel rays
// of 64 scatterings from one small part of the mesh instead of those that a
// wave of the late-order kernel happened to reach together.  The frame holds
// the box's low corner and 32 / its size per axis.
struct KeyFrame {
    float lo[3], scale[3];
};

template <typename R>
__device__ __forceinline__ uint32_t cell_key(const KeyFrame &f, const R p[3])
{
    uint32_t c[3];
    for (int a = 0; a < 3; ++a) {
        const float u = ((float)p[a] - f.lo[a]) * f.scale[a];
        c[a] = u > 0.0f ? (u < 31.0f ? (uint32_t)u : 31u) : 0u;
    }
    uint32_t key = 0;
    for (int b = 0; b < 5; ++b)
        key |= ((c[0] >> b) & 1u) << (3 * b) | ((c[1] >> b) & 1u) << (3 * b + 1) | ((c[2] >> b) & 1u) << (3 * b + 2);
    return key;
}

// Octahedral map of a direction to 2 x 8 bits, interleaved (nearby directions
// get nearby keys).
__device__ __forceinline__ uint32_t interleave2(uint32_t qu, uint32_t qv, int bits)
{
    uint32_t key = 0;
    for (int b = 0; b < bits; ++b) key |= ((qu >> b) & 1u) << (2 * b) | ((qv >> b) & 1u) << (2 * b + 1);
    return key;
}

template <typename R>
__device__ __forceinline__ uint32_t direction_key(const R k[3])
{
    const R s = fabs(k[0]) + fabs(k[1]) + fabs(k[2]);
    R u = k[0] / s, v = k[1] / s;
    if (k[2] < (R)0) {
        const R uu = ((R)1 - fabs(v)) * (u >= (R)0 ? (R)1 : (R)-1);
        const R vv = ((R)1 - fabs(u)) * (v >= (R)0 ? (R)1 : (R)-1);
        u = uu;
        v = vv;
    }
    int qu = (int)((u + (R)1) * (R)128), qv = (int)((v + (R)1) * (R)128);
    qu = qu < 0 ? 0 : (qu > 255 ? 255 : qu);
    qv = qv < 0 ? 0 : (qv > 255 ? 255 : qv);
    return interleave2((uint32_t)qu, (uint32_t)qv, 8);
}

}  // namespace qrt

// Kernels of the peel-off optical-depth surrogate network: weight tiles,
// batched forward pass, forward+backward pass of a training batch, Adam
// update, input normalisation and loss.  The network and the matrix-core
// layout are described in qrt_mlp.h.
//
// Training step (one wave = 64 samples, one wave per block):
//   forward through the 5 layers in the chained register layout; the
//   post-ReLU activations of every layer are also written to LDS as
//   [feature][sample] bfloat16 rows, and their ReLU masks kept as bits;
//   output error dL/dy = 2 w (y - t) / batch for the weighted squared error;
//   per layer from the top: weight gradient dW_l = A_l^T Delta_l as a
//   matrix-core product over the wave's 64 samples (both operands read from
//   LDS rows), bias gradient as row sums, and the error of the layer below
//   Delta_{l-1} = (W_l Delta_l) * [A_l > 0] in the chained register layout.
// Every wave writes its own gradient vector; the Adam kernel sums them in a
// fixed order, so a training run is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "qrt_internal.h"
#include "qrt_mlp.h"

namespace qrt {

constexpr int kLdsRow = 72;   // bfloat16 per LDS row: 64 samples + 8 padding (row stride 144 B)

// ---------------------------------------------------------------- weight tiles
// Writes parameter p (value v) into its forward and backward tile positions;
// biases have none.
__device__ __forceinline__ void pack_param(int p, float v, __bf16 *__restrict__ tiles)
{
    int l = -1;
#pragma unroll
    for (int k = 0; k < 5; ++k)
        if (p >= mlp_w_off(k) && p < mlp_w_off(k) + mlp_fan_in(k) * mlp_fan_out(k)) l = k;
    if (l < 0) return;
    const int fo = mlp_fan_out(l);
    const int i = (p - mlp_w_off(l)) / fo, o = (p - mlp_w_off(l)) % fo;
    const __bf16 b = (__bf16)v;
    int s, kb, q;
    if (l == 0) {
        tiles[((size_t)fwd_tile(0, o >> 4, 0) * 64 + (o & 15)) * 8 + i] = b;
        return;
    }
    chain_slot(i, s, kb, q);
    const int row = l == 4 ? 0 : (o & 15);
    const int mt = l == 4 ? 0 : (o >> 4);
    tiles[((size_t)fwd_tile(l, mt, s) * 64 + row + 16 * kb) * 8 + q] = b;
    if (l == 4) {
        tiles[((size_t)bwd_tile(4, i >> 4, 0) * 64 + (i & 15)) * 8 + 0] = b;
    } else {
        chain_slot(o, s, kb, q);
        tiles[((size_t)bwd_tile(l, i >> 4, s) * 64 + (i & 15) + 16 * kb) * 8 + q] = b;
    }
}

__global__ void __launch_bounds__(256) k_mlp_pack(const float *__restrict__ params, __bf16 *__restrict__ tiles)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) pack_param(p, params[p], tiles);
}

// ---------------------------------------------------------------- forward
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ params,
                                                     const bf16x8 *__restrict__ tiles,
                                                     const float *__restrict__ X, uint64_t n, float *__restrict__ y)
{
    __shared__ float bias[260];
    mlp_bias_to_lds(bias, params);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    MlpWeights W;
    mlp_load(W, tiles, lane);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (uint64_t base = wave * 64; base < n; base += waves * 64) {
        const uint64_t j = base + lane;
        float x[kMlpIn];
#pragma unroll
        for (int a = 0; a < kMlpIn; ++a) x[a] = j < n ? X[j * kMlpIn + a] : 0.0f;
        const float o = mlp_wave(W, bias, x, lane);
        if (j < n) y[j] = o;
    }
}

// ---------------------------------------------------------------- loss
// Per wave: sum over its samples of w (y - t)^2 with t = min(tau, cap),
// w = exp(-t) + floor (FP64 partials, one per wave).
__global__ void __launch_bounds__(256) k_mlp_loss(const float *__restrict__ params, const bf16x8 *__restrict__ tiles,
                                                  const float *__restrict__ X, const float *__restrict__ tau,
                                                  uint64_t n, float cap, float wfloor, double *__restrict__ part)
{
    __shared__ float bias[260];
    mlp_bias_to_lds(bias, params);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    MlpWeights W;
    mlp_load(W, tiles, lane);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    double acc = 0.0;
    for (uint64_t base = wave * 64; base < n; base += waves * 64) {
        const uint64_t j = base + lane;
        float x[kMlpIn];
#pragma unroll
        for (int a = 0; a < kMlpIn; ++a) x[a] = j < n ? X[j * kMlpIn + a] : 0.0f;
        const float o = mlp_wave(W, bias, x, lane);
        if (j < n) {
            const float t = fminf(tau[j], cap);
            const float w = expf(-t) + wfloor;
            acc += (double)w * (double)(o - t) * (double)(o - t);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) part[wave] = acc;
}

// ---------------------------------------------------------------- gradients
struct __align__(16) GradLds {
    __bf16 a0[16 * kLdsRow];       // network inputs, rows 0..4 (5..15 zero)
    __bf16 a[4][64 * kLdsRow];     // post-ReLU activations of layers 0..3
    __bf16 d[64 * kLdsRow];        // error of the current layer's outputs
    float bias[260];
};

__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// post-ReLU D tiles of one N-tile into LDS rows, with their ReLU mask bits
__device__ __forceinline__ void store_act(__bf16 *rows, const f32x4 acc[4], int nt, int lane, uint64_t &bits)
{
    const int rb = lane >> 4, col = nt * 16 + (lane & 15);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float v = acc[mt][r];
            rows[(mt * 16 + rb * 4 + r) * kLdsRow + col] = (__bf16)fmaxf(v, 0.0f);
            if (v > 0.0f) bits |= 1ull << ((mt * 4 + nt) * 4 + r);
        }
}

// dW[i][o] = sum over the 64 samples of A[i][b] D[o][b] for i < fan_in, o < fan_out
__device__ __forceinline__ void grad_weights(const __bf16 *A, int in_tiles, const __bf16 *D, int out_tiles,
                                             int fan_in, int fan_out, float *__restrict__ out, int lane)
{
    const int rb = lane >> 4, col = lane & 15;
    for (int mi = 0; mi < in_tiles; ++mi)
        for (int no = 0; no < out_tiles; ++no) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const bf16x8 a = *(const bf16x8 *)(A + (mi * 16 + col) * kLdsRow + s * 32 + rb * 8);
                const bf16x8 b = *(const bf16x8 *)(D + (no * 16 + col) * kLdsRow + s * 32 + rb * 8);
                acc = mfma(a, b, acc);
            }
            const int o = no * 16 + col;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = mi * 16 + rb * 4 + r;
                if (i < fan_in && o < fan_out) out[i * fan_out + o] = acc[r];
            }
        }
}

// db[o] = sum over the 64 samples of D[o][b], o < rows
__device__ __forceinline__ void grad_bias(const __bf16 *D, int rows, float *__restrict__ out, int lane)
{
    if (lane >= rows) return;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const bf16x8 v = *(const bf16x8 *)(D + lane * kLdsRow + c * 8);
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += (float)v[q];
    }
    out[lane] = acc;
}

// error of the layer below through W_l (backward tiles), masked by its ReLU
// bits; written to LDS and returned as the next chained operands
template <int KSTEPS>
__device__ __forceinline__ void chain_back(const bf16x8 *__restrict__ tiles, int l, bf16x8 B[4][2], uint64_t bits,
                                           __bf16 *D, int lane)
{
    const int rb = lane >> 4, colb = lane & 15;
    bf16x8 nb[4][2];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            acc[mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < KSTEPS; ++s)
                acc[mt] = mfma(tiles[bwd_tile(l, mt, s) * 64 + lane], B[nt][s], acc[mt]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool on = (bits >> ((mt * 4 + nt) * 4 + r)) & 1ull;
                acc[mt][r] = on ? acc[mt][r] : 0.0f;
                D[(mt * 16 + rb * 4 + r) * kLdsRow + nt * 16 + colb] = (__bf16)acc[mt][r];
            }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                nb[nt][s][r] = (__bf16)acc[2 * s][r];
                nb[nt][s][4 + r] = (__bf16)acc[2 * s + 1][r];
            }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        B[nt][0] = nb[nt][0];
        B[nt][1] = nb[nt][1];
    }
}

// MODE 0: training batch; sample of lane = hash(seed, step, position) mod n,
//         output error from the weighted squared error against min(tau, cap).
// MODE 1: gradient of sum_j dy[j] y[j] over rows j = 64 block .. 64 block + 63.
template <int MODE>
__global__ void __launch_bounds__(64) k_mlp_grad(const float *__restrict__ params, const bf16x8 *__restrict__ tiles,
                                                 const float *__restrict__ X, uint64_t n,
                                                 const float *__restrict__ tau, const float *__restrict__ dy_in,
                                                 MlpBatch sel, float *__restrict__ part)
{
    __shared__ GradLds L;
    const int lane = threadIdx.x;
    const int rb = lane >> 4, colb = lane & 15;
    mlp_bias_to_lds(L.bias, params);
    for (int i = lane; i < 16 * kLdsRow; i += 64) L.a0[i] = (__bf16)0.0f;
    for (int i = lane; i < 16 * kLdsRow; i += 64) L.d[i] = (__bf16)0.0f;
    __syncthreads();

    uint64_t j;
    bool valid;
    if (MODE == 0) {
        const uint64_t h = splitmix64(sel.seed ^ splitmix64(sel.step * (uint64_t)sel.batch +
                                                            (uint64_t)blockIdx.x * 64 + lane));
        j = __umul64hi(h, n);
        valid = true;
    } else {
        j = (uint64_t)blockIdx.x * 64 + lane;
        valid = j < n;
    }
    float x[kMlpIn];
#pragma unroll
    for (int a = 0; a < kMlpIn; ++a) x[a] = valid ? X[j * kMlpIn + a] : 0.0f;

    // forward, keeping activations (LDS) and ReLU masks (bits)
    uint64_t bits[4] = {0, 0, 0, 0};
    float y = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int src = nt * 16 + colb;
        bf16x8 xb;
#pragma unroll
        for (int q = 0; q < 8; ++q) xb[q] = (__bf16)0.0f;
#pragma unroll
        for (int a = 0; a < kMlpIn; ++a) {
            const float v = __shfl(x[a], src, 64);
            if (lane < 16) {
                xb[a] = (__bf16)v;
                L.a0[a * kLdsRow + nt * 16 + lane] = (__bf16)v;
            }
        }
        f32x4 acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            acc[mt] = mfma(tiles[fwd_tile(0, mt, 0) * 64 + lane], xb, bias_tile(L.bias, 0, mt, lane));
        store_act(L.a[0], acc, nt, lane, bits[0]);
        bf16x8 h0 = relu_pack(acc[0], acc[1]), h1 = relu_pack(acc[2], acc[3]);
#pragma unroll
        for (int l = 1; l <= 3; ++l) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                acc[mt] = mfma(tiles[fwd_tile(l, mt, 0) * 64 + lane], h0, bias_tile(L.bias, l, mt, lane));
                acc[mt] = mfma(tiles[fwd_tile(l, mt, 1) * 64 + lane], h1, acc[mt]);
            }
            store_act(L.a[l], acc, nt, lane, bits[l]);
            h0 = relu_pack(acc[0], acc[1]);
            h1 = relu_pack(acc[2], acc[3]);
        }
        f32x4 o = {L.bias[256], 0.0f, 0.0f, 0.0f};
        o = mfma(tiles[fwd_tile(4, 0, 0) * 64 + lane], h0, o);
        o = mfma(tiles[fwd_tile(4, 0, 1) * 64 + lane], h1, o);
        const float mine = __shfl(o[0], colb, 64);
        if (rb == nt) y = mine;
    }

    // output error
    float dy = 0.0f;
    if (MODE == 0) {
        const float t = fminf(tau[j], sel.cap);
        const float w = expf(-t) + sel.wfloor;
        dy = 2.0f * w * (y - t) / (float)sel.batch;
    } else if (valid) {
        dy = dy_in[j];
    }
    L.d[lane] = (__bf16)dy;   // row 0: the single output
    bf16x8 B[4][2];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float v = __shfl(dy, nt * 16 + colb, 64);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            B[nt][0][q] = (__bf16)0.0f;
            B[nt][1][q] = (__bf16)0.0f;
        }
        if (lane < 16) B[nt][0][0] = (__bf16)v;
    }
    float *g = part + (size_t)blockIdx.x * kMlpParams;
    __syncthreads();

    // layer 4
    grad_bias(L.d, 1, g + mlp_b_off(4), lane);
    grad_weights(L.a[3], 4, L.d, 1, 64, 1, g + mlp_w_off(4), lane);
    __syncthreads();
    chain_back<1>(tiles, 4, B, bits[3], L.d, lane);
    __syncthreads();
    // layers 3, 2, 1
#pragma unroll
    for (int l = 3; l >= 1; --l) {
        grad_bias(L.d, 64, g + mlp_b_off(l), lane);
        grad_weights(L.a[l - 1], 4, L.d, 4, 64, 64, g + mlp_w_off(l), lane);
        __syncthreads();
        chain_back<2>(tiles, l, B, bits[l - 1], L.d, lane);
        __syncthreads();
    }
    // layer 0
    grad_bias(L.d, 64, g + mlp_b_off(0), lane);
    grad_weights(L.a0, 1, L.d, 4, kMlpIn, 64, g + mlp_w_off(0), lane);
}

// ---------------------------------------------------------------- update
// sum over the per-wave gradients of parameter p in a fixed order: eight
// interleaved partial sums (independent loads in flight), then their sum
__device__ __forceinline__ float sum_parts(const float *__restrict__ part, int n_parts, int p)
{
    float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    int w = 0;
    for (; w + 8 <= n_parts; w += 8)
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += part[(size_t)(w + k) * kMlpParams + p];
    for (; w < n_parts; ++w) s[w & 7] += part[(size_t)w * kMlpParams + p];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ params, float *__restrict__ m,
                                                  float *__restrict__ v, const float *__restrict__ part, int n_parts,
                                                  AdamStep A, __bf16 *__restrict__ tiles)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = sum_parts(part, n_parts, p);
    const float mn = A.beta1 * m[p] + (1.0f - A.beta1) * g;
    const float vn = A.beta2 * v[p] + (1.0f - A.beta2) * g * g;
    m[p] = mn;
    v[p] = vn;
    const float th = params[p] - A.lr * (mn * A.c1) / (sqrtf(vn * A.c2) + A.eps);
    params[p] = th;
    pack_param(p, th, tiles);
}

__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ part, int n_parts, float *__restrict__ out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    out[p] = sum_parts(part, n_parts, p);
}

// ---------------------------------------------------------------- inputs
// (x, y, z, observer) rows -> normalised network inputs
__global__ void __launch_bounds__(256) k_mlp_inputs(const float *__restrict__ pos_obs, uint64_t n, InputMap M,
                                                    float *__restrict__ X)
{
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int ob = (int)pos_obs[j * 4 + 3];
    ob = ob < 0 ? 0 : (ob >= M.n_obs ? M.n_obs - 1 : ob);
    float x[kMlpIn];
    mlp_inputs(M, (double)pos_obs[j * 4], (double)pos_obs[j * 4 + 1], (double)pos_obs[j * 4 + 2], ob, x);
#pragma unroll
    for (int a = 0; a < kMlpIn; ++a) X[j * kMlpIn + a] = x[a];
}

// ---------------------------------------------------------------- launchers
static unsigned blocks_for(uint64_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_mlp_pack(const float *params, void *tiles, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, params, (__bf16 *)tiles);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *params, const void *tiles, const float *X, uint64_t n, float *y,
                              hipStream_t st)
{
    if (n == 0) return hipSuccess;
    unsigned b = blocks_for((n + 63) / 64, 4);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_mlp_forward, dim3(b), dim3(256), 0, st, params, (const bf16x8 *)tiles, X, n, y);
    return hipGetLastError();
}

int mlp_loss_parts(uint64_t n)
{
    unsigned b = blocks_for((n + 63) / 64, 4);
    if (b > 1024) b = 1024;
    if (b == 0) b = 1;
    return (int)b * 4;
}

hipError_t launch_mlp_loss(const float *params, const void *tiles, const float *X, const float *tau, uint64_t n,
                           float cap, float wfloor, double *part, hipStream_t st)
{
    const int parts = mlp_loss_parts(n);
    hipLaunchKernelGGL(k_mlp_loss, dim3(parts / 4), dim3(256), 0, st, params, (const bf16x8 *)tiles, X, tau, n, cap,
                       wfloor, part);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(int mode, const float *params, const void *tiles, const float *X, uint64_t n,
                           const float *tau, const float *dy, const MlpBatch &sel, int n_blocks, float *part,
                           hipStream_t st)
{
    if (mode == 0)
        hipLaunchKernelGGL(k_mlp_grad<0>, dim3(n_blocks), dim3(64), 0, st, params, (const bf16x8 *)tiles, X, n, tau,
                           dy, sel, part);
    else
        hipLaunchKernelGGL(k_mlp_grad<1>, dim3(n_blocks), dim3(64), 0, st, params, (const bf16x8 *)tiles, X, n, tau,
                           dy, sel, part);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *params, float *m, float *v, const float *part, int n_parts, const AdamStep &A,
                           void *tiles, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, params, m, v, part, n_parts,
                       A, (__bf16 *)tiles);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float *part, int n_parts, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks_for(kMlpParams, 256)), dim3(256), 0, st, part, n_parts, out);
    return hipGetLastError();
}

hipError_t launch_mlp_inputs(const float *pos_obs, uint64_t n, const InputMap &M, float *X, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_inputs, dim3(blocks_for(n, 256)), dim3(256), 0, st, pos_obs, n, M, X);
    return hipGetLastError();
}

}  // namespace qrt

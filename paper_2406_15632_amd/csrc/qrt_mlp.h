// Peel-off optical-depth surrogate network on the gfx950 matrix cores.
//
// The surrogate is an addition to the method of the paper: inside a validated
// domain it replaces the mesh traversal of a peel-off ray (Sec. 3.4, 3.6) by
// a small network tau_hat(x, y, z, theta_obs, phi_obs).
//
// Network: 5 inputs -> 4 hidden layers of 64 ReLU units -> 1 linear output.
// Flat FP32 parameters (12,929), layer by layer: W_l[in][out] row-major, then
// b_l[out]:  W0 5x64 | b0 | W1 64x64 | b1 | W2 | b2 | W3 | b3 | W4 64x1 | b4.
// Inputs: position in the coordinates of the surrogate's cylindrical domain
// (computed in FP64, rounded to FP32; see InputMap), 2 theta / pi - 1 and
// phi / pi - 1 of the observer.
//
// Matrix-core mapping (v_mfma_f32_16x16x32_bf16, one wave):
//   D[16x16] += A[16x32] B[32x16]; lane L holds row L%16 of A and column L%16
//   of B, 8 K-values each (K-slot group L/16, slots 0..7), and rows
//   4(L/16) .. 4(L/16)+3 of column L%16 of D.
// The layers are computed transposed, H_out^T = W^T H_in^T: features run
// along M, the 16 queries of a tile along N.  The D tiles of one layer then
// are, without any data movement, the B operand of the next: K-slot q of
// group kb in k-step s holds feature
//     f(s, kb, q) = 16 (2 s + q / 4) + 4 kb + q % 4,
// and the weight tiles are stored with their K index permuted the same way.
// Weights are stored once per update as bfloat16 "tiles" in exactly the
// per-lane order the instruction reads (16 bytes per lane and tile).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 5;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 12929;
constexpr int kFwdTiles = 30;   // layer 0: 4, layers 1-3: 8 each, layer 4: 2
constexpr int kBwdTiles = 28;   // layer 4: 4, layers 1-3: 8 each
constexpr int kMlpTiles = kFwdTiles + kBwdTiles;

__host__ __device__ constexpr int mlp_w_off(int l) { return l == 0 ? 0 : 384 + (l - 1) * 4160; }
__host__ __device__ constexpr int mlp_b_off(int l) { return l == 0 ? 320 : (l == 4 ? 12928 : 384 + (l - 1) * 4160 + 4096); }
__host__ __device__ constexpr int mlp_fan_in(int l) { return l == 0 ? kMlpIn : kMlpHidden; }
__host__ __device__ constexpr int mlp_fan_out(int l) { return l == 4 ? 1 : kMlpHidden; }

// tile numbers (each tile = 64 lanes x 8 bfloat16)
__host__ __device__ constexpr int fwd_tile(int l, int mt, int s)
{
    return l == 0 ? mt : (l == 4 ? 28 + s : 4 + (l - 1) * 8 + mt * 2 + s);
}
__host__ __device__ constexpr int bwd_tile(int l, int mt, int s)
{
    return kFwdTiles + (l == 4 ? mt : 4 + (l - 1) * 8 + mt * 2 + s);
}

// feature -> (k-step, K-slot group, slot) of the chained layout
__host__ __device__ inline void chain_slot(int f, int &s, int &kb, int &q)
{
    const int t = f >> 4, w = f & 15;
    s = t >> 1;
    q = ((t & 1) << 2) | (w & 3);
    kb = w >> 2;
}

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ReLU of the D tiles of two M-tiles (features 32 s .. 32 s + 31) as the B
// operand of the next layer's k-step s.
__device__ __forceinline__ bf16x8 relu_pack(const f32x4 &lo, const f32x4 &hi)
{
    bf16x8 h;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        h[r] = (__bf16)fmaxf(lo[r], 0.0f);
        h[4 + r] = (__bf16)fmaxf(hi[r], 0.0f);
    }
    return h;
}

// Forward weights of one wave, held in registers (120 VGPRs).
struct MlpWeights {
    bf16x8 w0[4];
    bf16x8 w[3][4][2];
    bf16x8 w4[2];
};

__device__ __forceinline__ void mlp_load(MlpWeights &W, const bf16x8 *__restrict__ tiles, int lane)
{
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) W.w0[mt] = tiles[fwd_tile(0, mt, 0) * 64 + lane];
#pragma unroll
    for (int l = 1; l <= 3; ++l)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int s = 0; s < 2; ++s) W.w[l - 1][mt][s] = tiles[fwd_tile(l, mt, s) * 64 + lane];
#pragma unroll
    for (int s = 0; s < 2; ++s) W.w4[s] = tiles[fwd_tile(4, 0, s) * 64 + lane];
}

// Biases in the D layout: lane L, row r of M-tile mt of layer l holds
// b_l[16 mt + 4 (L/16) + r].  `bias` is the block's LDS copy of b0..b3 [4][64]
// followed by b4.
__device__ __forceinline__ f32x4 bias_tile(const float *bias, int l, int mt, int lane)
{
    const float *b = bias + l * 64 + mt * 16 + (lane >> 4) * 4;
    return f32x4{b[0], b[1], b[2], b[3]};
}

// One N-tile of 16 queries through the network.  x is the layer-0 B operand
// (lanes 0..15 hold the 5 inputs of query L in slots 0..4, everything else 0).
// Returns the raw output of query L%16 in lanes 0..15 (other lanes: unused).
__device__ __forceinline__ float mlp_tile(const MlpWeights &W, const float *bias, const bf16x8 &x, int lane)
{
    f32x4 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt] = mfma(W.w0[mt], x, bias_tile(bias, 0, mt, lane));
    bf16x8 h0 = relu_pack(acc[0], acc[1]), h1 = relu_pack(acc[2], acc[3]);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = mfma(W.w[l][mt][0], h0, bias_tile(bias, l + 1, mt, lane));
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = mfma(W.w[l][mt][1], h1, acc[mt]);
        h0 = relu_pack(acc[0], acc[1]);
        h1 = relu_pack(acc[2], acc[3]);
    }
    f32x4 o = {bias[256], 0.0f, 0.0f, 0.0f};
    o = mfma(W.w4[0], h0, o);
    o = mfma(W.w4[1], h1, o);
    return o[0];
}

// The 64 queries of a wave (query i held by lane i) through the network;
// returns lane i's raw output.  Every lane of the wave must call it.
__device__ __forceinline__ float mlp_wave(const MlpWeights &W, const float *bias, const float x[kMlpIn], int lane)
{
    float out = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int src = nt * 16 + (lane & 15);
        bf16x8 xb;
#pragma unroll
        for (int q = 0; q < 8; ++q) xb[q] = (__bf16)0.0f;
#pragma unroll
        for (int a = 0; a < kMlpIn; ++a) {
            const float v = __shfl(x[a], src, 64);
            xb[a] = lane < 16 ? (__bf16)v : (__bf16)0.0f;
        }
        const float o = mlp_tile(W, bias, xb, lane);
        const float mine = __shfl(o, lane & 15, 64);
        if ((lane >> 4) == nt) out = mine;
    }
    return out;
}

// The 64 queries of a wave through the network with the forward weight tiles
// in LDS: each tile is read once and applied to all four 16-query tiles, so
// one layer issues 16 independent matrix-core chains.  Query i is held by
// lane i; returns lane i's raw output.  Every lane of the wave must call it.
__device__ __forceinline__ float mlp_wave_lds(const bf16x8 *Wt, const float *bias, const float x[kMlpIn], int lane)
{
    bf16x8 xb[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int src = nt * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 8; ++q) xb[nt][q] = (__bf16)0.0f;
#pragma unroll
        for (int a = 0; a < kMlpIn; ++a) {
            const float v = __shfl(x[a], src, 64);
            if (lane < 16) xb[nt][a] = (__bf16)v;
        }
    }
    f32x4 acc[4][4];   // [mt][nt]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8 a = Wt[fwd_tile(0, mt, 0) * 64 + lane];
        const f32x4 b = bias_tile(bias, 0, mt, lane);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma(a, xb[nt], b);
    }
    bf16x8 h[4][2];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        h[nt][0] = relu_pack(acc[0][nt], acc[1][nt]);
        h[nt][1] = relu_pack(acc[2][nt], acc[3][nt]);
    }
#pragma unroll
    for (int l = 1; l <= 3; ++l) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 a0 = Wt[fwd_tile(l, mt, 0) * 64 + lane];
            const bf16x8 a1 = Wt[fwd_tile(l, mt, 1) * 64 + lane];
            const f32x4 b = bias_tile(bias, l, mt, lane);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma(a0, h[nt][0], b);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mfma(a1, h[nt][1], acc[mt][nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            h[nt][0] = relu_pack(acc[0][nt], acc[1][nt]);
            h[nt][1] = relu_pack(acc[2][nt], acc[3][nt]);
        }
    }
    const bf16x8 a0 = Wt[fwd_tile(4, 0, 0) * 64 + lane];
    const bf16x8 a1 = Wt[fwd_tile(4, 0, 1) * 64 + lane];
    float out = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 o = {bias[256], 0.0f, 0.0f, 0.0f};
        o = mfma(a0, h[nt][0], o);
        o = mfma(a1, h[nt][1], o);
        const float mine = __shfl(o[0], lane & 15, 64);
        if ((lane >> 4) == nt) out = mine;
    }
    return out;
}

// Copy of the forward weight tiles into LDS, by the threads of one block.
__device__ __forceinline__ void mlp_tiles_to_lds(bf16x8 *Wt, const bf16x8 *__restrict__ tiles)
{
    for (int i = threadIdx.x; i < kFwdTiles * 64; i += blockDim.x) Wt[i] = tiles[i];
}

// Copy of the biases into LDS (257 floats), by the threads of one block.
__device__ __forceinline__ void mlp_bias_to_lds(float *bias, const float *__restrict__ params)
{
    for (int i = threadIdx.x; i < 257; i += blockDim.x) {
        const int l = i >> 6;
        bias[i] = l < 4 ? params[mlp_b_off(l) + (i & 63)] : params[mlp_b_off(4)];
    }
}

}  // namespace qrt

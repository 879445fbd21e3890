// Device-side optical depth on a Cartesian mesh (Sec. 3.4 of Shulman,
// "Quasi-Monte Carlo Radiative Transfer"): kappa*rho is constant per cell, the
// optical depth along a ray is the sum over the crossed cells of
// kappa*rho * (length inside the cell), and a packet moved by a given optical
// depth stops inside the cell where the running sum reaches it.
//
// Cell walk (Amanatides & Woo 1987) kept as resumable per-lane state so that a
// persistent kernel can interleave the walks of many packets:
//  - the starting cell is floor((p-lo)/h) clamped to the mesh;
//  - along each axis with a nonzero direction component, the distance to the
//    j-th face ahead is fma(j, D, T0) (T0 the first face distance, D = h/|k|):
//    one rounding per face, no drift;
//  - the distance to the mesh boundary face of each axis uses the same
//    expression, so the walk ends exactly when the face it is about to cross
//    is a boundary face (tn >= t_exit); the cell index therefore never leaves
//    the mesh;
//  - ties step x before y before z; components below 1e-30 count as zero;
//  - steps are taken in batches: the cells of B steps are computed first (they
//    do not depend on the densities), then their B loads are issued together,
//    then the optical depth is accumulated in order, in FP64, with the
//    stop test of a move done per step.
// Loads go through a buffer resource whose range is the mesh, so an address
// outside the mesh could only read zero.
//
// Cell order in memory: every mesh is stored in bricks of 4x4x4
// cells (bricks x fastest, then y, then z; inside a brick x fastest), so that
// one 128-byte line holds a 4x4x2 block and a ray crossing a brick stays on
// few lines whatever its direction.  The brick counts along x and y are
// padded to powers of two: an element index is then the OR of one part per
// axis, each in bit fields of its own, and the walk moves the part of the
// axis it steps along by one with an add whose carry runs across the other
// axes' bits (a dilated-integer increment).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrt {

constexpr int kBrick = 4;   // cells per brick edge

__host__ __device__ inline int bricks_of(int n) { return (n + kBrick - 1) / kBrick; }

// Stored bricks per axis of an nx x ny x nz mesh: a power of two along x and
// y, bricks_of(nz) along z.
__host__ __device__ inline void mesh_bricks(int nx, int ny, int nz, int nb[3])
{
    nb[0] = 1;
    while (nb[0] < bricks_of(nx)) nb[0] <<= 1;
    nb[1] = 1;
    while (nb[1] < bricks_of(ny)) nb[1] <<= 1;
    nb[2] = bricks_of(nz);
}

// stored cells of a mesh (the cells past its edge hold 0)
// cells per axis at most: a walk's face counts (FP32 in FP32 walks) stay exact
constexpr int kMaxAxisCells = 1 << 20;

__host__ __device__ inline int64_t mesh_cells(int nx, int ny, int nz)
{
    int nb[3];
    mesh_bricks(nx, ny, nz, nb);
    return (int64_t)nb[0] * nb[1] * nb[2] * (kBrick * kBrick * kBrick);
}

// element index of cell (x, y, z) in the bricked order; nbx, nby bricks along x, y
__host__ __device__ inline int brick_index(int x, int y, int z, int nbx, int nby)
{
    const int brick = ((z >> 2) * nby + (y >> 2)) * nbx + (x >> 2);
    return (brick << 6) | ((z & 3) << 4) | ((y & 3) << 2) | (x & 3);
}

// Bit fields of each axis' part of an element's byte offset (4 times its
// index), for nbx = 2^lx and nby = 2^ly bricks: x in bits 2-3 and 8 .. 7+lx,
// y in bits 4-5 and 8+lx .. 7+lx+ly, z in bits 6-7 and from 8+lx+ly up.  The
// index of (x, y, z) is brick_index(x, 0, 0) | brick_index(0, y, 0) |
// brick_index(0, 0, z).
__host__ __device__ inline void axis_masks(int nbx, int nby, uint32_t m[3])
{
    int lx = 0, ly = 0;
    while ((1 << lx) < nbx) ++lx;
    while ((1 << ly) < nby) ++ly;
    m[0] = 0x0Cu | (((1u << lx) - 1u) << 8);
    m[1] = 0x30u | (((1u << ly) - 1u) << (8 + lx));
    m[2] = 0xC0u | (~0u << (8 + lx + ly));
}

struct DevGrid {
    const float *kr;      // bricked: [nbz][nby][nbx][4][4][4], cells outside the mesh 0
    int nx, ny, nz;
    int nb[3];            // stored bricks per axis (mesh_bricks)
    double lo[3], hi[3], h[3];
};

template <typename R>
struct RayGrid {
    __amdgpu_buffer_rsrc_t rsrc;
    int n[3];
    int nbx, nby;
    uint32_t m[3];        // axis_masks
    R lo[3], h[3];
};

template <typename R>
__device__ __forceinline__ RayGrid<R> ray_grid(const DevGrid &g)
{
    RayGrid<R> r;
    // up to 2^29 cells: the byte count (at most 2^31) is the descriptor's unsigned 32-bit record count
    const uint32_t bytes = (uint32_t)g.nb[0] * (uint32_t)g.nb[1] * (uint32_t)g.nb[2] * (kBrick * kBrick * kBrick * 4);
    r.rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)g.kr, (short)0, (int)bytes, 0x00020000);
    r.n[0] = g.nx; r.n[1] = g.ny; r.n[2] = g.nz;
    r.nbx = g.nb[0];
    r.nby = g.nb[1];
    axis_masks(g.nb[0], g.nb[1], r.m);
    for (int a = 0; a < 3; ++a) { r.lo[a] = (R)g.lo[a]; r.h[a] = (R)g.h[a]; }
    return r;
}

// Mesh of one lane (a batch of scenes: every lane may walk its own mesh); the
// densities are read through a plain pointer, since a buffer descriptor has
// to be the same for the whole wave.
template <typename R>
struct LaneGrid {
    const float *kr;
    int n[3];
    int nbx, nby;
    uint32_t m[3];        // axis_masks
    R lo[3], h[3];
};

template <typename R> __device__ __forceinline__ R r_inf();
template <> __device__ __forceinline__ float r_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double r_inf<double>() { return __builtin_huge_val(); }

// kappa*rho of the cell at byte offset `at`
template <typename R>
__device__ __forceinline__ R load_kr(const RayGrid<R> &G, uint32_t at)
{
    return (R)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(G.rsrc, (int)at, 0, 0));
}

template <typename R>
__device__ __forceinline__ R load_kr(const LaneGrid<R> &G, uint32_t at)
{
    return (R)*(const float *)((const char *)G.kr + at);
}

enum WalkMode { WALK_EDGE = 0, WALK_MOVE = 1 };

// Per-lane walk state.  Scalar fields only: a selected array element would be
// lowered to a private-memory load.
template <typename R>
struct Walk {
    R T0x, T0y, T0z, Dx, Dy, Dz;   // face distances: fma(j, D, T0)
    R jx, jy, jz;                  // faces crossed per axis
    R tx, ty, tz;                  // next face distance per axis
    R t, t_exit;
    uint32_t ox, oy, oz;           // each axis' part of the cell's byte offset
    uint32_t ax, ay, az;           // per axis: the addend of a one-cell step of its part (walk_begin)
    double tau, target;
    int mode;
    bool done, stopped;
    R t_out;                       // stop distance (MOVE), else exit distance
    uint32_t visits;               // cells visited, set when the walk ends
};

template <typename R, typename GT>
__device__ __forceinline__ void axis_setup(const GT &G, int a, R p, R d, int &c, R &T0, R &D, R &tb, int &sgn)
{
    R f = floor((p - G.lo[a]) / G.h[a]);
    f = f < (R)0 ? (R)0 : f;
    f = f > (R)(G.n[a] - 1) ? (R)(G.n[a] - 1) : f;
    c = (int)f;
    const int s = d > (R)1e-30 ? 1 : (d < (R)-1e-30 ? -1 : 0);
    sgn = s;
    if (s == 0) {
        T0 = r_inf<R>();
        D = (R)0;
        tb = r_inf<R>();
    } else {
        const R inv = (R)1 / d;
        const R face0 = G.lo[a] + (R)(c + (s > 0 ? 1 : 0)) * G.h[a];
        T0 = (face0 - p) * inv;
        D = G.h[a] * fabs(inv);
        const int J = s > 0 ? G.n[a] - 1 - c : c;
        tb = fma((R)J, D, T0);
    }
}

// Start a walk from p along unit d.  Returns false (and a finished walk with
// tau = 0) for non-finite input or a zero direction.  Such input is set up
// like a ray from the mesh corner along +x, so that every field of the state
// is assigned on one path (separate assignments on a second path lead the
// compiler to keep the face spacings in private memory).
template <typename R, typename GT>
__device__ __forceinline__ bool walk_begin(Walk<R> &W, const GT &G, const R p[3], const R d[3], int mode,
                                           double target)
{
    W.mode = mode;
    W.target = target;
    W.tau = 0.0;
    W.t = (R)0;
    W.t_out = (R)0;
    W.stopped = false;
    W.visits = 0;
    W.jx = W.jy = W.jz = (R)0;
    const bool ok = isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) && isfinite(d[0]) && isfinite(d[1]) &&
                    isfinite(d[2]) && (fabs(d[0]) > (R)1e-30 || fabs(d[1]) > (R)1e-30 || fabs(d[2]) > (R)1e-30);
    W.done = !ok;
    R bx, by, bz;
    int cx, cy, cz, sx, sy, sz;
    axis_setup(G, 0, ok ? p[0] : G.lo[0], ok ? d[0] : (R)1, cx, W.T0x, W.Dx, bx, sx);
    axis_setup(G, 1, ok ? p[1] : G.lo[1], ok ? d[1] : (R)0, cy, W.T0y, W.Dy, by, sy);
    axis_setup(G, 2, ok ? p[2] : G.lo[2], ok ? d[2] : (R)0, cz, W.T0z, W.Dz, bz, sz);
    W.tx = W.T0x; W.ty = W.T0y; W.tz = W.T0z;
    W.t_exit = fmin(bx, fmin(by, bz));
    W.ox = (uint32_t)brick_index(cx, 0, 0, G.nbx, G.nby) << 2;
    W.oy = (uint32_t)brick_index(0, cy, 0, G.nbx, G.nby) << 2;
    W.oz = (uint32_t)brick_index(0, 0, cz, G.nbx, G.nby) << 2;
    // An axis' part holds only the bits of its mask m.  A step up adds 4 (one
    // cell) with every bit outside m set, so that the carry runs through the
    // other axes' bits; since the part has none of those bits, setting them is
    // the same as adding ~m.  A step down subtracts 4, the borrow running
    // through them likewise.  Masking with m afterwards clears them again.
    W.ax = sx > 0 ? ~G.m[0] + 4u : (sx < 0 ? (uint32_t)-4 : 0u);
    W.ay = sy > 0 ? ~G.m[1] + 4u : (sy < 0 ? (uint32_t)-4 : 0u);
    W.az = sz > 0 ? ~G.m[2] + 4u : (sz < 0 ? (uint32_t)-4 : 0u);
    return ok;
}

// The cells (byte offsets), start distances and lengths of the next B steps
// of a walk, which do not depend on the densities.  After the exit step the
// remaining steps repeat the last cell with zero length: they add nothing.
// alive turns false at the exit step.  Every step before the exit crosses one
// face, so a walk that is still going has visited jx + jy + jz cells, and one
// that left the mesh one more.
template <typename R, int B, typename GT>
__device__ __forceinline__ void walk_steps(Walk<R> &W, const GT &G, uint32_t (&cells)[B], R (&t0s)[B],
                                           R (&segs)[B], bool &alive)
{
#pragma unroll
    for (int b = 0; b < B; ++b) {
        // the nearest face; ties go to x, then y
        const R tn = fmin(W.tx, fmin(W.ty, W.tz));
        const bool mx = W.tx == tn;
        const bool my = !mx && W.ty == tn;
        const bool mz = !mx && !my;
        cells[b] = W.ox | W.oy | W.oz;
        t0s[b] = W.t;
        // length max(tn - t, 0), and t never decreases
        const R t1 = fmax(tn, W.t);
        segs[b] = t1 - W.t;
        W.t = t1;
        // the face about to be crossed is a boundary face: the walk ends in this cell
        const bool adv = tn < W.t_exit;
        // the chosen axis' part moves by one cell
        const uint32_t nox = (W.ox + W.ax) & G.m[0];
        const uint32_t noy = (W.oy + W.ay) & G.m[1];
        const uint32_t noz = (W.oz + W.az) & G.m[2];
        W.ox = (adv && mx) ? nox : W.ox;
        W.oy = (adv && my) ? noy : W.oy;
        W.oz = (adv && mz) ? noz : W.oz;
        W.jx += (adv && mx) ? (R)1 : (R)0;
        W.jy += (adv && my) ? (R)1 : (R)0;
        W.jz += (adv && mz) ? (R)1 : (R)0;
        W.tx = fma(W.jx, W.Dx, W.T0x);
        W.ty = fma(W.jy, W.Dy, W.T0y);
        W.tz = fma(W.jz, W.Dz, W.T0z);
        alive = alive && adv;
    }
}

// B steps of a walk in either mode (no effect once done).  The B cells are
// computed first and loaded together; the optical depth is then accumulated
// in order, in FP64.  A move stops at the first step whose running sum
// reaches the target: the steps before it are counted, and the sum before it
// and that step's density and start are kept, from which the stop position is
// computed once, after the batch.
template <typename R, int B, typename GT>
__device__ __forceinline__ void walk_batch(Walk<R> &W, const GT &G)
{
    if (W.done) return;
    uint32_t cells[B];
    R t0s[B], segs[B];
    const uint32_t before_batch = (uint32_t)(W.jx + W.jy + W.jz);   // cells visited so far
    bool alive = true;
    walk_steps<R, B>(W, G, cells, t0s, segs, alive);
    R kr[B];
#pragma unroll
    for (int b = 0; b < B; ++b) kr[b] = load_kr(G, cells[b]);
    const bool edge = W.mode != WALK_MOVE;
    double tau = W.tau, before = W.tau;   // running sum; the sum before the stopping step
    R kr_hit = (R)1, t0_hit = (R)0;       // the stopping step's density and start
    uint32_t below = 0;                   // steps before the stopping step
    bool run = true;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const double next = tau + (double)(kr[b] * segs[b]);
        const bool go = run && (edge || !(next >= W.target));
        below += go ? 1u : 0u;
        before = go ? next : before;
        kr_hit = run && !go ? kr[b] : kr_hit;
        t0_hit = run && !go ? t0s[b] : t0_hit;
        run = go;
        tau = next;
    }
    if (!run) {
        const double rem = W.target - before;
        W.t_out = t0_hit + (rem > 0.0 ? (R)((R)rem / kr_hit) : (R)0);
        W.tau = rem > 0.0 ? W.target : before;
        W.stopped = true;
        W.done = true;
        // the stopping step is at or before the exit step (after it no step adds depth)
        W.visits = before_batch + below + 1;
        return;
    }
    W.tau = tau;
    if (!alive) {
        W.done = true;
        W.t_out = W.t;
        W.visits = (uint32_t)(W.jx + W.jy + W.jz) + 1;
    }
}

// B steps of a walk to the mesh edge (WALK_EDGE), as walk_batch computes
// them, without the stop test: kernels call it when no lane of the wave moves
// to a target.
template <typename R, int B, typename GT>
__device__ __forceinline__ void walk_batch_edge(Walk<R> &W, const GT &G)
{
    if (W.done) return;
    uint32_t cells[B];
    R t0s[B], segs[B];
    bool alive = true;
    walk_steps<R, B>(W, G, cells, t0s, segs, alive);
    R kr[B];
#pragma unroll
    for (int b = 0; b < B; ++b) kr[b] = load_kr(G, cells[b]);
    double tau = W.tau;
#pragma unroll
    for (int b = 0; b < B; ++b) tau += (double)(kr[b] * segs[b]);
    W.tau = tau;
    if (!alive) {
        W.done = true;
        W.t_out = W.t;
        W.visits = (uint32_t)(W.jx + W.jy + W.jz) + 1;
    }
}

template <typename R, int B, typename GT>
__device__ __forceinline__ void walk_run(Walk<R> &W, const GT &G)
{
    while (!W.done) walk_batch<R, B>(W, G);
}

}  // namespace qrt

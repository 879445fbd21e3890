// Device-side optical depth on a Cartesian mesh (Sec. 3.4 of Shulman,
// "Quasi-Monte Carlo Radiative Transfer"): kappa*rho is constant per cell, the
// optical depth along a ray is the sum over the crossed cells of
// kappa*rho * (length inside the cell), and a packet moved by a given optical
// depth stops inside the cell where the running sum reaches it.
//
// Cell walk (Amanatides & Woo 1987).  The starting cell is floor((p-lo)/h)
// clamped to the mesh; each axis keeps the distance to its next face,
// recomputed from the integer cell index after every step (no drift); an axis
// whose direction component is zero never steps; ties step x before y before z.
// The running optical depth is FP64 whatever the ray precision R, so long FP32
// rays (hundreds of cells) do not lose digits.
//
// Visits (cells entered) are not counted per step: every step changes one cell
// index by one, so the count follows from the start and end cells.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrt {

struct DevGrid {
    const float *kr;      // [nz][ny][nx], x fastest
    int nx, ny, nz;
    double lo[3], hi[3], h[3];
};

template <typename R>
struct RayGrid {
    const float *__restrict__ kr;
    int n[3];
    R lo[3], h[3];
};

template <typename R>
__device__ __forceinline__ RayGrid<R> ray_grid(const DevGrid &g)
{
    RayGrid<R> r;
    r.kr = g.kr;
    r.n[0] = g.nx; r.n[1] = g.ny; r.n[2] = g.nz;
    for (int a = 0; a < 3; ++a) { r.lo[a] = (R)g.lo[a]; r.h[a] = (R)g.h[a]; }
    return r;
}

struct WalkResult {
    double tau;      // accumulated optical depth (to the edge, or the target when stopped)
    uint32_t visits; // cells entered
    bool stopped;    // MOVE: stopped inside the mesh
};

template <typename R> __device__ __forceinline__ R r_inf();
template <> __device__ __forceinline__ float r_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double r_inf<double>() { return __builtin_huge_val(); }

enum WalkMode { WALK_EDGE = 0, WALK_MOVE = 1 };

// Walk from p along unit k.  WALK_EDGE: integrate to the mesh edge; t_out is the
// exit distance.  WALK_MOVE: stop where the running optical depth reaches
// target; t_out is the stop distance, or the exit distance if the edge comes first.
template <typename R, int MODE>
__device__ __forceinline__ WalkResult walk(const RayGrid<R> &G, const R p[3], const R k[3], double target,
                                           R &t_out)
{
    int c[3], s[3];
    R tmax[3], invk[3], base[3];
    int c0[3];
    WalkResult res;
    res.stopped = false;
    // Termination: every step moves one cell index by one toward the mesh edge,
    // provided the axis chosen has a nonzero step.  Non-finite positions or
    // directions (never produced by the transport) would break that, so they
    // end the walk at once; components below 1e-30 count as zero, which keeps
    // 1/k and every face distance finite.
    if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) && isfinite(k[0]) && isfinite(k[1]) &&
          isfinite(k[2])) ||
        !(fabs(k[0]) > (R)1e-30 || fabs(k[1]) > (R)1e-30 || fabs(k[2]) > (R)1e-30)) {
        t_out = (R)0;
        res.tau = 0.0;
        res.visits = 0;
        return res;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R f = floor((p[a] - G.lo[a]) / G.h[a]);
        f = f < (R)0 ? (R)0 : f;
        f = f > (R)(G.n[a] - 1) ? (R)(G.n[a] - 1) : f;
        c[a] = (int)f;
        c0[a] = c[a];
        s[a] = k[a] > (R)1e-30 ? 1 : (k[a] < (R)-1e-30 ? -1 : 0);
        invk[a] = s[a] == 0 ? (R)0 : (R)1 / k[a];
        // face(c) = lo + (c + [s>0]) h ; tmax = (face - p) / k
        base[a] = G.lo[a] - p[a] + (s[a] > 0 ? G.h[a] : (R)0);
        tmax[a] = s[a] == 0 ? r_inf<R>() : (base[a] + (R)c[a] * G.h[a]) * invk[a];
    }
    const int sy = G.n[0], sz = G.n[0] * G.n[1];
    int cell = (c[2] * G.n[1] + c[1]) * G.n[0] + c[0];
    R t = (R)0;
    double tau = 0.0;
    for (;;) {
        int a;
        if (tmax[0] <= tmax[1]) a = tmax[0] <= tmax[2] ? 0 : 2;
        else a = tmax[1] <= tmax[2] ? 1 : 2;
        R tn = a == 0 ? tmax[0] : (a == 1 ? tmax[1] : tmax[2]);
        R seg = tn - t;
        seg = seg < (R)0 ? (R)0 : seg;
        R kr = (R)G.kr[cell];
        double dtau = (double)(kr * seg);
        if constexpr (MODE == WALK_MOVE) {
            if (tau + dtau >= target) {
                double rem = target - tau;
                t_out = t + (rem > 0.0 ? (R)(rem / (double)kr) : (R)0);
                res.stopped = true;
                res.tau = rem > 0.0 ? target : tau;
                res.visits = (uint32_t)(abs(c[0] - c0[0]) + abs(c[1] - c0[1]) + abs(c[2] - c0[2]) + 1);
                return res;
            }
        }
        tau += dtau;
        t = tn > t ? tn : t;
        if (a == 0) {
            c[0] += s[0];
            if ((unsigned)c[0] >= (unsigned)G.n[0]) break;
            cell += s[0];
            tmax[0] = (base[0] + (R)c[0] * G.h[0]) * invk[0];
        } else if (a == 1) {
            c[1] += s[1];
            if ((unsigned)c[1] >= (unsigned)G.n[1]) break;
            cell += s[1] * sy;
            tmax[1] = (base[1] + (R)c[1] * G.h[1]) * invk[1];
        } else {
            c[2] += s[2];
            if ((unsigned)c[2] >= (unsigned)G.n[2]) break;
            cell += s[2] * sz;
            tmax[2] = (base[2] + (R)c[2] * G.h[2]) * invk[2];
        }
    }
    t_out = t;
    res.tau = tau;
    // the exiting step is counted by the index change but enters no cell
    res.visits = (uint32_t)(abs(c[0] - c0[0]) + abs(c[1] - c0[1]) + abs(c[2] - c0[2]));
    return res;
}

}  // namespace qrt

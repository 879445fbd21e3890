/*
 * FP64 CPU oracle of the quasi-Monte Carlo radiative-transfer path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product never does.  It shares no
 * code, header or table with the GPU library.
 *
 * It follows the method of Shulman, "Quasi-Monte Carlo Radiative Transfer":
 *   Sec. 3.1  point sets: Sobol, Niederreiter base 2, Halton, Hammersley, and a
 *             counter-based PRNG for the Monte Carlo baseline; the all-zero
 *             leading point is skipped (indices start at 1);
 *   Sec. 3.2  isotropic point-source emission (phi = 2 pi u, theta = acos(2v-1)),
 *             optical depth tau1 to the mesh edge, cut below tau_min, forced first
 *             scattering with weight 1-exp(-tau1) and tau = -ln[1 - w(1-exp(-tau1))];
 *   Sec. 3.3  sphere-star emission, direct order (emission point from v1,v2,
 *             local direction from v3,v4, tau from v5);
 *   Sec. 3.4  optical depth on a Cartesian mesh as the sum of d_cell*kappa*rho,
 *             and moving a packet by a given optical depth;
 *   Sec. 3.5  peel-off before each scattering, Henyey-Greenstein sampling of
 *             cos(Theta) and i1 = 2 pi u, free flight tau2 = -ln w, end when the
 *             packet leaves the mesh or after the last scattering;
 *   Sec. 2.1  albedo weighting at each scattering;
 *   Sec. 2.2  White's Mueller matrix elements P11, P12, P33 (p_c = 0);
 *   Sec. 3.6  peel-off weight W0 exp(-tau_obs) p_obs binned to the nearest pixel;
 *   Sec. 3.7  one point per packet, a fixed dimension per purpose.
 * Readings where the paper is silent (Stokes frame convention, tau_min value,
 * the local emission angle, tie rules of the traversal) are the ones the
 * design document lists; each is marked below where it is used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_PI 3.14159265358979323846

enum { OG_SOBOL = 0, OG_HALTON = 1, OG_NIED2 = 2, OG_HAMMERSLEY = 3, OG_PHILOX = 4, OG_FAURE = 5, OG_SOBOL_OWEN = 6 };
enum { OG_POINT = 0, OG_SPHERE = 1 };

/* ------------------------------------------------------------------------- */
/* scene description (mirrored by a ctypes Structure in oracle.py)           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t nx, ny, nz;
    double lo[3], hi[3];
    const float *kr;              /* kappa*rho per cell, [nz][ny][nx], x fastest */
    int64_t src_kind;             /* OG_POINT / OG_SPHERE */
    double src[3];
    double r_star;
    double albedo, g, p_lin;
    int64_t n_obs, npix;
    const double *obs_theta, *obs_phi;
    double half_width;
    int64_t seq_kind, dims;
    const uint32_t *mat;          /* Sobol / Niederreiter columns [dims][32] */
    const uint32_t *bases;        /* Halton bases [dims] */
    uint64_t seed, n_total;
    int64_t max_orders;
    double tau_min;
    /* surrogate peel-off optical depth (not part of the paper; network and
       domain as described in oracle/mlp.py) */
    int64_t peel_mode;            /* 0 exact traversal, 1 network inside its valid cells */
    const float *mlp;             /* 12929 FP32 parameters */
    double dom_center[3];
    double dom_r_in, dom_r_out, dom_h0, dom_beta, dom_zmax;
    int64_t dom_nr, dom_nz;
    const uint8_t *dom_valid;     /* [n_obs][nr][nz], 1 = network allowed */
    int64_t emit_order;           /* sphere star: 0 direct order, 1 inverse order (Sec. 3.3) */
    int64_t order_images;         /* 0: one image set; K: one set per scattering order 1..K */
} og_scene;

typedef struct {
    int64_t packets, visits, peels, peel_rays, escapes, tau_cuts, scatterings, occluded;
    double e_direct, e_absorbed, e_escaped, e_remaining;
    int64_t surrogate, fallbacks;
    int64_t visits_first;   /* visits of the two first-flight walks (to the edge, then the forced flight) */
} og_counters;

/* ------------------------------------------------------------------------- */
/* point sets (Sec. 3.1); values are unsigned 0.32 fixed point               */
/* ------------------------------------------------------------------------- */

/* Digital (t,s)-sequence in base 2 in Gray-code order: XOR of the matrix
   columns selected by the bits of gray(i) = i ^ (i >> 1). */
static uint32_t og_digital(const uint32_t *cols, uint64_t i)
{
    uint64_t gray = i ^ (i >> 1);
    uint32_t x = 0;
    for (int r = 0; r < 32; ++r)
        if ((gray >> r) & 1u) x ^= cols[r];
    return x;
}

/* floor(phi_b(i) * 2^32), phi_b the radical inverse (van der Corput) in base b.
   phi_b(i) = A / b^K with A the digit-reversed integer, computed exactly. */
static uint32_t og_radical_inverse(uint64_t i, uint32_t b)
{
    unsigned __int128 A = 0, B = 1;
    while (i) {
        A = A * b + (i % b);
        B *= b;
        i /= b;
    }
    return (uint32_t)((A << 32) / B);
}

/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11). */
static void og_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct {
    int64_t kind, dims;
    const uint32_t *mat, *bases;
    uint64_t seed, n_total;
} og_seq;

/* coordinate d (0-based) of point i (i >= 1) */
/* splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014): add the
   golden-ratio increment, then two xor-shift-multiply rounds and a final
   xor-shift. */
static uint64_t og_splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Owen's nested uniform scrambling of a 0.32 fixed-point coordinate: going
   from the most significant bit down, bit j (depth t = 31 - j) is flipped by a
   random bit that depends on the seed, the dimension, the depth and the t
   original bits above it, so that every elementary interval is permuted as a
   whole.  The random bit is the top bit of splitmix64 of a key built from
   (seed, dimension, depth, prefix). */
static uint32_t og_owen(uint32_t x, uint64_t seed, int d)
{
    uint32_t out = x;
    for (int t = 0; t < 32; ++t) {
        uint64_t prefix = t == 0 ? 0 : (uint64_t)(x >> (32 - t));
        uint64_t key = og_splitmix64(seed ^ og_splitmix64(((uint64_t)(uint32_t)d << 8) | (uint64_t)t)) ^ prefix;
        uint32_t flip = (uint32_t)(og_splitmix64(key) >> 63);
        out ^= flip << (31 - t);
    }
    return out;
}

static uint32_t og_point(const og_seq *q, uint64_t i, int d)
{
    switch (q->kind) {
    case OG_SOBOL:
    case OG_NIED2:
        return og_digital(q->mat + 32 * (size_t)d, i);
    case OG_SOBOL_OWEN:
        return og_owen(og_digital(q->mat + 32 * (size_t)d, i), q->seed, d);
    case OG_HALTON:
        return og_radical_inverse(i, q->bases[d]);
    case OG_HAMMERSLEY:
        /* first coordinate i/N (Sec. 3.1 puts i/N first), stored modulo 1:
           i = N gives 0, which as an azimuth is the same direction as 2 pi */
        if (d == 0) return (uint32_t)(((unsigned __int128)i << 32) / q->n_total);
        return og_radical_inverse(i, q->bases[d - 1]);
    case OG_FAURE: {
        /* Faure (1982): base b = bases[0], m = bases[1] digits; mat holds the
           matrices C_d[r][k] = binom(k,r) d^(k-r) mod b, [dims][m][m].
           y = C_d a (mod b) for the base-b digits a of i (least significant
           first), x = sum_r y_r b^-(r+1), returned as floor(x 2^32). */
        uint32_t b = q->bases[0], m = q->bases[1];
        uint32_t a[64];
        uint64_t n = i;
        for (uint32_t k = 0; k < m; ++k) { a[k] = (uint32_t)(n % b); n /= b; }
        const uint32_t *C = q->mat + (size_t)d * m * m;
        unsigned __int128 Y = 0, B = 1;
        for (uint32_t r = 0; r < m; ++r) {
            uint64_t y = 0;
            for (uint32_t k = r; k < m; ++k) y += (uint64_t)C[r * m + k] * a[k];
            Y = Y * b + (y % b);
            B *= b;
        }
        return (uint32_t)((Y << 32) / B);
    }
    case OG_PHILOX: {
        uint64_t ctr[4] = {i, (uint64_t)(d >> 3), 0, 0}, key[2] = {q->seed, 0}, out[4];
        og_philox4x64(ctr, key, out);
        uint64_t w = out[(d & 7) >> 1];
        return (d & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
    }
    default:
        return 0;
    }
}

static double og_u(const og_seq *q, uint64_t i, int d)
{
    return (double)og_point(q, i, d) * (1.0 / 4294967296.0);
}

int oracle_points(int64_t kind, int64_t dims, const uint32_t *mat, const uint32_t *bases,
                  uint64_t seed, uint64_t n_total, uint64_t first, uint64_t count, uint32_t *out)
{
    og_seq q = {kind, dims, mat, bases, seed, n_total};
    if (first < 1) return -1;
    for (uint64_t j = 0; j < count; ++j)
        for (int d = 0; d < dims; ++d)
            out[j * (uint64_t)dims + (uint64_t)d] = og_point(&q, first + j, d);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Cartesian mesh traversal (Sec. 3.4)                                       */
/* ------------------------------------------------------------------------- */
/* Cells are entered in order along p + t k (Amanatides & Woo voxel walk).
   The cell of a point is floor((p-lo)/h) clamped to the mesh.  The next face
   distance on each axis is recomputed from the integer cell index; an axis
   with k_a = 0 never steps; ties step the lowest axis first (x, then y, z).
   Each cell adds kappa*rho * (length of the ray inside it) to tau.
   mode 0: run to the mesh edge, return tau.
   mode 1: stop inside the cell where tau_acc + kappa*rho*seg >= target, at
           t + (target - tau_acc)/(kappa*rho); *stopped = 1.  If the edge comes
           first, *stopped = 0 and *t_out is the exit distance.
   mode 2: integrate only up to distance target along the ray, return tau. */
static double og_walk(const og_scene *S, const double p[3], const double k[3], int mode,
                      double target, double *t_out, int *stopped, int64_t *visits)
{
    const int64_t n[3] = {S->nx, S->ny, S->nz};
    double h[3];
    int64_t c[3], step[3];
    double tmax[3];
    for (int a = 0; a < 3; ++a) {
        h[a] = (S->hi[a] - S->lo[a]) / (double)n[a];
        double f = floor((p[a] - S->lo[a]) / h[a]);
        if (f < 0.0) f = 0.0;
        if (f > (double)(n[a] - 1)) f = (double)(n[a] - 1);
        c[a] = (int64_t)f;
        step[a] = k[a] > 0.0 ? 1 : (k[a] < 0.0 ? -1 : 0);
    }
    for (int a = 0; a < 3; ++a) {
        if (step[a] == 0) { tmax[a] = INFINITY; continue; }
        double face = S->lo[a] + (double)(c[a] + (step[a] > 0 ? 1 : 0)) * h[a];
        tmax[a] = (face - p[a]) / k[a];
    }
    double t = 0.0, tau = 0.0;
    if (stopped) *stopped = 0;
    for (;;) {
        int a = 0;
        if (tmax[1] < tmax[a]) a = 1;
        if (tmax[2] < tmax[a]) a = 2;
        double tn = tmax[a];
        double seg = tn - t;
        if (seg < 0.0) seg = 0.0;
        double kr = (double)S->kr[(c[2] * n[1] + c[1]) * n[0] + c[0]];
        double dtau = kr * seg;
        if (visits) ++*visits;
        if (mode == 2 && tn >= target) {
            /* integrate only up to distance target */
            double s2 = target - t;
            return tau + (s2 > 0.0 ? kr * s2 : 0.0);
        }
        if (mode == 1 && tau + dtau >= target) {
            double rem = target - tau;
            *t_out = t + (rem > 0.0 ? rem / kr : 0.0);
            *stopped = 1;
            return tau + (rem > 0.0 ? rem : 0.0);
        }
        tau += dtau;
        if (tn > t) t = tn;
        c[a] += step[a];
        if (c[a] < 0 || c[a] >= n[a]) break;
        double face = S->lo[a] + (double)(c[a] + (step[a] > 0 ? 1 : 0)) * h[a];
        tmax[a] = (face - p[a]) / k[a];
    }
    if (t_out) *t_out = t;
    return tau;
}

double oracle_tau_ray(const og_scene *S, const double p[3], const double k[3], int64_t *visits)
{
    return og_walk(S, p, k, 0, 0.0, NULL, NULL, visits);
}

/* returns 1 if the packet stopped inside the mesh */
int oracle_move(const og_scene *S, const double p[3], const double k[3], double target,
                double p_out[3], int64_t *visits)
{
    double t = 0.0;
    int stopped = 0;
    og_walk(S, p, k, 1, target, &t, &stopped, visits);
    for (int a = 0; a < 3; ++a) p_out[a] = p[a] + t * k[a];
    return stopped;
}

/* ------------------------------------------------------------------------- */
/* scattering physics (Sec. 2.2, 3.5)                                        */
/* ------------------------------------------------------------------------- */
static double og_dot(const double a[3], const double b[3]) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void og_cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1]*b[2] - a[2]*b[1];
    o[1] = a[2]*b[0] - a[0]*b[2];
    o[2] = a[0]*b[1] - a[1]*b[0];
}

/* Henyey-Greenstein inverse CDF for cos(Theta) (Sec. 3.5); g ~ 0 reads as isotropic */
double oracle_hg_cos(double g, double v)
{
    double c;
    if (fabs(g) < 1e-6) {
        c = 2.0 * v - 1.0;
    } else {
        double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * v);
        c = (1.0 + g * g - f * f) / (2.0 * g);
    }
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return c;
}

/* White's approximation: P11 (Henyey-Greenstein), P12/P11 and P33/P11 */
static void og_mueller(double g, double p_lin, double c, double *p11, double *r12, double *r33)
{
    double den = 1.0 + g * g - 2.0 * g * c;
    *p11 = (1.0 - g * g) / (den * sqrt(den));
    *r12 = -p_lin * (1.0 - c * c) / (1.0 + c * c);
    *r33 = 2.0 * c / (1.0 + c * c);
}

/* Rotate the Stokes reference axis by psi (new axis = cos psi m + sin psi n). */
static void og_rotate(double S[3], double cpsi, double spsi)
{
    double c2 = cpsi * cpsi - spsi * spsi, s2 = 2.0 * spsi * cpsi;
    double q = S[1] * c2 + S[2] * s2;
    double u = -S[1] * s2 + S[2] * c2;
    S[1] = q;
    S[2] = u;
}

/* Orthonormal completion of a unit vector (Duff et al. 2017): m, with n = k x m */
static void og_basis(const double k[3], double m[3])
{
    double sg = k[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + k[2]);
    double b = k[0] * k[1] * a;
    m[0] = 1.0 + sg * k[0] * k[0] * a;
    m[1] = sg * b;
    m[2] = -sg * k[0];
}

typedef struct {
    double o[3], ex[3], ey[3];
} og_obs;

static void og_make_obs(double th, double ph, og_obs *O)
{
    O->o[0] = sin(th) * cos(ph); O->o[1] = sin(th) * sin(ph); O->o[2] = cos(th);
    O->ex[0] = -sin(ph); O->ex[1] = cos(ph); O->ex[2] = 0.0;
    og_cross(O->o, O->ex, O->ey);
}

/* ------------------------------------------------------------------------- */
/* surrogate peel-off optical depth (an addition to the method: a network     */
/* replaces the traversal toward the observer inside a validated domain)      */
/* ------------------------------------------------------------------------- */

/* FP32 rounding, then bfloat16 rounding to nearest with ties to even */
static double og_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* 5 -> 64 -> 64 -> 64 -> 64 -> 1 ReLU network; inputs, weights and hidden
   activations in bfloat16, sums in FP64, biases as given. */
static double og_mlp(const float *th, const double xin[5])
{
    static const int sizes[6] = {5, 64, 64, 64, 64, 1};
    double a[64], z[64];
    for (int i = 0; i < 5; ++i) a[i] = og_bf16(xin[i]);
    const float *W = th;
    for (int l = 0; l < 5; ++l) {
        int ni = sizes[l], no = sizes[l + 1];
        const float *b = W + ni * no;
        for (int o = 0; o < no; ++o) {
            double acc = (double)b[o];
            for (int i = 0; i < ni; ++i) acc += og_bf16((double)W[i * no + o]) * a[i];
            z[o] = acc;
        }
        if (l < 4)
            for (int o = 0; o < no; ++o) a[o] = og_bf16(z[o] > 0.0 ? z[o] : 0.0);
        W = b + no;
    }
    return z[0];
}

/* Cell of p in the cylindrical domain around dom_center (R bins over
   [r_in, r_out), z/h(R) bins over (-zmax, zmax), h = h0 R^beta); -1 outside. */
static int64_t og_dom_cell(const og_scene *S, const double p[3])
{
    double dx = p[0] - S->dom_center[0], dy = p[1] - S->dom_center[1], dz = p[2] - S->dom_center[2];
    double R = sqrt(dx * dx + dy * dy);
    if (!(R >= S->dom_r_in && R < S->dom_r_out)) return -1;
    double zh = dz / (S->dom_h0 * pow(R, S->dom_beta));
    if (!(fabs(zh) < S->dom_zmax)) return -1;
    int64_t ir = (int64_t)floor((R - S->dom_r_in) / (S->dom_r_out - S->dom_r_in) * (double)S->dom_nr);
    int64_t iz = (int64_t)floor((zh + S->dom_zmax) / (2.0 * S->dom_zmax) * (double)S->dom_nz);
    if (ir < 0 || ir >= S->dom_nr || iz < 0 || iz >= S->dom_nz) return -1;
    return ir * S->dom_nz + iz;
}

/* Network inputs in the domain's own coordinates, each rounded to FP32:
   x and y relative to the centre over r_out, the height over the domain's
   half-thickness zmax h(R) (clamped to [-4, 4], 0 on the axis), and the
   observer angles 2 theta / pi - 1 and phi / pi - 1. */
static void og_mlp_inputs(const og_scene *S, const double p[3], int obs, double x[5])
{
    double dx = p[0] - S->dom_center[0], dy = p[1] - S->dom_center[1], dz = p[2] - S->dom_center[2];
    double R = sqrt(dx * dx + dy * dy);
    double zn = 0.0;
    if (R > 0.0) {
        zn = dz / (S->dom_zmax * (S->dom_h0 * pow(R, S->dom_beta)));
        zn = zn > 4.0 ? 4.0 : (zn < -4.0 ? -4.0 : zn);
    }
    x[0] = (double)(float)(dx / S->dom_r_out);
    x[1] = (double)(float)(dy / S->dom_r_out);
    x[2] = (double)(float)zn;
    x[3] = (double)(float)(2.0 * S->obs_theta[obs] / OG_PI - 1.0);
    x[4] = (double)(float)(S->obs_phi[obs] / OG_PI - 1.0);
}

double oracle_mlp_tau(const og_scene *S, const double p[3], int64_t obs)
{
    double x[5];
    og_mlp_inputs(S, p, (int)obs, x);
    double t = og_mlp(S->mlp, x);
    return t > 0.0 ? t : 0.0;
}

/* Raw network outputs (no clamp) for n input rows X[n][5]. */
int oracle_mlp_batch(const float *th, int64_t n, const double *X, double *y)
{
    for (int64_t i = 0; i < n; ++i) y[i] = og_mlp(th, X + 5 * i);
    return 0;
}

/* Domain cells (ir * nz + iz, or -1) of n positions p[n][3]. */
int oracle_dom_cells(const og_scene *S, int64_t n, const double *p, int64_t *cell)
{
    for (int64_t i = 0; i < n; ++i) cell[i] = og_dom_cell(S, p + 3 * i);
    return 0;
}

/* event log record for tests: p[3], X, Y, I, Q, U, cos(Theta_obs), order, obs */
#define OG_EVENT_WORDS 11

typedef struct {
    double *img;
    og_counters *C;
    double *events;
    int64_t max_events, *n_events;
} og_sink;

/* Peel-off toward one observer (Sec. 3.5, 3.6).  S is the packet Stokes vector
   after the albedo factor of this scattering. */
static void og_peel(const og_scene *S, const double p[3], const double k[3], const double m[3],
                    const double Sv[3], const og_obs *O, int obs, int order, og_sink *sink)
{
    double X = og_dot(p, O->ex), Y = og_dot(p, O->ey);
    double R = S->half_width;
    double fx = floor((X + R) / (2.0 * R) * (double)S->npix);
    double fy = floor((Y + R) / (2.0 * R) * (double)S->npix);
    if (fx < 0.0 || fy < 0.0 || fx >= (double)S->npix || fy >= (double)S->npix) return;
    if (S->src_kind == OG_SPHERE) {
        /* the star blocks rays that pass through it */
        double d[3] = {p[0] - S->src[0], p[1] - S->src[1], p[2] - S->src[2]};
        double b = og_dot(d, O->o), cc = og_dot(d, d) - S->r_star * S->r_star;
        if (b < 0.0 && b * b > cc) { sink->C->occluded++; return; }
    }
    double n[3];
    og_cross(k, m, n);
    double c = og_dot(k, O->o);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double s = sqrt(fmax(0.0, 1.0 - c * c));
    double St[3] = {Sv[0], Sv[1], Sv[2]};
    double min_[3], mout[3], nout[3];
    if (s < 1e-12) {
        min_[0] = m[0]; min_[1] = m[1]; min_[2] = m[2];
    } else {
        for (int a = 0; a < 3; ++a) min_[a] = (O->o[a] - c * k[a]) / s;
        og_rotate(St, og_dot(m, min_), og_dot(n, min_));
    }
    double p11, r12, r33;
    og_mueller(S->g, S->p_lin, c, &p11, &r12, &r33);
    double w = p11 / (4.0 * OG_PI);
    double I1 = w * (St[0] + r12 * St[1]);
    double Q1 = w * (r12 * St[0] + St[1]);
    double U1 = w * (r33 * St[2]);
    double Sp[3] = {I1, Q1, U1};
    for (int a = 0; a < 3; ++a) mout[a] = c * min_[a] - s * k[a];
    og_cross(O->o, mout, nout);
    og_rotate(Sp, og_dot(mout, O->ex), og_dot(nout, O->ex));
    int64_t vis = 0;
    double tau;
    int64_t cell = S->peel_mode == 1 ? og_dom_cell(S, p) : -1;
    if (cell >= 0 && S->dom_valid[(int64_t)obs * S->dom_nr * S->dom_nz + cell]) {
        tau = oracle_mlp_tau(S, p, obs);
        sink->C->surrogate++;
    } else {
        tau = og_walk(S, p, O->o, 0, 0.0, NULL, NULL, &vis);
        sink->C->visits += vis;
        sink->C->peel_rays++;
        if (S->peel_mode == 1) sink->C->fallbacks++;
    }
    double att = exp(-tau);
    int64_t ix = (int64_t)fx, iy = (int64_t)fy;
    size_t plane = (size_t)S->npix * (size_t)S->npix;
    size_t base = ((size_t)obs * 3) * plane + (size_t)iy * (size_t)S->npix + (size_t)ix;
    if (S->order_images > 0)   /* the image set of this scattering order */
        base += (size_t)(order - 1) * (size_t)S->n_obs * 3 * plane;
    sink->img[base] += att * Sp[0];
    sink->img[base + plane] += att * Sp[1];
    sink->img[base + 2 * plane] += att * Sp[2];
    sink->C->peels++;
    if (sink->events && *sink->n_events < sink->max_events) {
        double *e = sink->events + OG_EVENT_WORDS * (*sink->n_events)++;
        e[0] = p[0]; e[1] = p[1]; e[2] = p[2]; e[3] = X; e[4] = Y;
        e[5] = att * Sp[0]; e[6] = att * Sp[1]; e[7] = att * Sp[2];
        e[8] = c; e[9] = order; e[10] = obs;
    }
}

/* Emission (Sec. 3.2 point source, Sec. 3.3 sphere star in direct order):
   position p and unit direction k of the packet; returns the dimension that
   carries the forced optical depth and the first dimension of the next flight. */
static void og_emit(const og_scene *S, const og_seq *q, uint64_t idx, double p[3], double k[3],
                    int *dim_tau, int *next_dim)
{
    if (S->src_kind == OG_SPHERE && S->emit_order == 1) {
        /* inverse order: v1,v2 -> propagation direction as for a point source,
           v3 -> tau, v4,v5 -> emission point relative to that direction.
           Reading: for a uniform-brightness surface the emission point seen
           from a given direction k has density ~ max(0, n.k) over the star,
           so its angle alpha to k follows cos(alpha) = sqrt(v5) and its
           azimuth about k is 2 pi v4 (the printed "same equation" as the
           direct emission point, weighted by the emitting hemisphere). */
        double ph = 2.0 * OG_PI * og_u(q, idx, 0);
        double ct = 2.0 * og_u(q, idx, 1) - 1.0;
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        k[0] = st * cos(ph); k[1] = st * sin(ph); k[2] = ct;
        double phr = 2.0 * OG_PI * og_u(q, idx, 3);
        double ca = sqrt(og_u(q, idx, 4));
        double sa = sqrt(fmax(0.0, 1.0 - ca * ca));
        double t1[3] = {ct * cos(ph), ct * sin(ph), -st};
        double t2[3] = {-sin(ph), cos(ph), 0.0};
        for (int a = 0; a < 3; ++a) {
            double n = ca * k[a] + sa * (cos(phr) * t1[a] + sin(phr) * t2[a]);
            p[a] = S->src[a] + S->r_star * n;
        }
        *dim_tau = 2;
        *next_dim = 5;
    } else if (S->src_kind == OG_SPHERE) {
        /* direct order: v1,v2 -> point on the star, v3,v4 -> local direction, v5 -> tau.
           Reading: cos(theta_l) = sqrt(v4), a uniform-brightness (Lambertian) surface. */
        double phe = 2.0 * OG_PI * og_u(q, idx, 0);
        double cte = 2.0 * og_u(q, idx, 1) - 1.0;
        double ste = sqrt(fmax(0.0, 1.0 - cte * cte));
        double ne[3] = {ste * cos(phe), ste * sin(phe), cte};
        double phl = 2.0 * OG_PI * og_u(q, idx, 2);
        double ctl = sqrt(og_u(q, idx, 3));
        double stl = sqrt(fmax(0.0, 1.0 - ctl * ctl));
        double t1[3] = {cte * cos(phe), cte * sin(phe), -ste};
        double t2[3] = {-sin(phe), cos(phe), 0.0};
        for (int a = 0; a < 3; ++a) {
            p[a] = S->src[a] + S->r_star * ne[a];
            k[a] = ctl * ne[a] + stl * (cos(phl) * t1[a] + sin(phl) * t2[a]);
        }
        *dim_tau = 4;
        *next_dim = 5;
    } else {
        double ph = 2.0 * OG_PI * og_u(q, idx, 0);
        double ct = 2.0 * og_u(q, idx, 1) - 1.0;
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        p[0] = S->src[0]; p[1] = S->src[1]; p[2] = S->src[2];
        k[0] = st * cos(ph); k[1] = st * sin(ph); k[2] = ct;
        *dim_tau = 2;
        *next_dim = 3;
    }
}

int oracle_emit(const og_scene *S, uint64_t first, uint64_t count, double *p_out, double *k_out)
{
    og_seq q = {S->seq_kind, S->dims, S->mat, S->bases, S->seed, S->n_total};
    int dt, nd;
    if (first < 1) return -1;
    for (uint64_t j = 0; j < count; ++j)
        og_emit(S, &q, first + j, p_out + 3 * j, k_out + 3 * j, &dt, &nd);
    return 0;
}

/* One photon packet (Sec. 3.2-3.7). */
static void og_packet(const og_scene *S, const og_seq *q, const og_obs *obs, uint64_t idx, og_sink *sink)
{
    og_counters *C = sink->C;
    double p[3], k[3];
    int dim_tau, next_dim;
    C->packets++;
    og_emit(S, q, idx, p, k, &dim_tau, &next_dim);
    /* optical depth to the mesh edge and the forced first scattering */
    int64_t vis = 0;
    double tau1 = og_walk(S, p, k, 0, 0.0, NULL, NULL, &vis);
    C->visits += vis;
    C->visits_first += vis;
    if (tau1 < S->tau_min) {
        C->tau_cuts++;
        C->e_direct += 1.0;
        return;
    }
    double W1 = -expm1(-tau1);
    C->e_direct += exp(-tau1);
    double tau = -log1p(-og_u(q, idx, dim_tau) * W1);
    {
        double t = 0.0;
        int stopped = 0;
        vis = 0;
        og_walk(S, p, k, 1, tau, &t, &stopped, &vis);
        C->visits += vis;
        C->visits_first += vis;
        /* if rounding lets the walk reach the edge first, scatter at the exit point */
        for (int a = 0; a < 3; ++a) p[a] += t * k[a];
    }
    double Sv[3] = {W1, 0.0, 0.0};
    double m[3];
    og_basis(k, m);
    for (int order = 1; order <= S->max_orders; ++order) {
        C->scatterings++;
        C->e_absorbed += (1.0 - S->albedo) * Sv[0];
        for (int a = 0; a < 3; ++a) Sv[a] *= S->albedo;
        for (int o = 0; o < S->n_obs; ++o) og_peel(S, p, k, m, Sv, &obs[o], o, order, sink);
        if (order == S->max_orders) {
            C->e_remaining += Sv[0];
            return;
        }
        /* new direction: i1 from the first number of the triple, cos(Theta) from the second */
        double i1 = 2.0 * OG_PI * og_u(q, idx, next_dim);
        double ct = oracle_hg_cos(S->g, og_u(q, idx, next_dim + 1));
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double w = og_u(q, idx, next_dim + 2);
        next_dim += 3;
        double n[3], min_[3], kn[3], mn[3];
        og_cross(k, m, n);
        double ci = cos(i1), si = sin(i1);
        for (int a = 0; a < 3; ++a) min_[a] = ci * m[a] + si * n[a];
        og_rotate(Sv, ci, si);
        double p11, r12, r33;
        og_mueller(S->g, S->p_lin, ct, &p11, &r12, &r33);
        double I1 = Sv[0] + r12 * Sv[1];
        double Q1 = r12 * Sv[0] + Sv[1];
        double U1 = r33 * Sv[2];
        Sv[0] = I1; Sv[1] = Q1; Sv[2] = U1;
        for (int a = 0; a < 3; ++a) {
            kn[a] = ct * k[a] + st * min_[a];
            mn[a] = ct * min_[a] - st * k[a];
        }
        for (int a = 0; a < 3; ++a) { k[a] = kn[a]; m[a] = mn[a]; }
        /* free flight tau2 = -ln w */
        double tau2 = -log(w);
        double t = 0.0;
        int stopped = 0;
        vis = 0;
        og_walk(S, p, k, 1, tau2, &t, &stopped, &vis);
        C->visits += vis;
        if (!stopped) {
            C->escapes++;
            C->e_escaped += Sv[0];
            return;
        }
        for (int a = 0; a < 3; ++a) p[a] += t * k[a];
    }
}

static void og_add_counters(og_counters *a, const og_counters *b)
{
    a->packets += b->packets; a->visits += b->visits; a->peels += b->peels;
    a->peel_rays += b->peel_rays; a->escapes += b->escapes; a->tau_cuts += b->tau_cuts;
    a->scatterings += b->scatterings; a->occluded += b->occluded;
    a->e_direct += b->e_direct; a->e_absorbed += b->e_absorbed;
    a->e_escaped += b->e_escaped; a->e_remaining += b->e_remaining;
    a->surrogate += b->surrogate; a->fallbacks += b->fallbacks;
    a->visits_first += b->visits_first;
}

/* Run packets first .. first+count-1 and ADD their (unnormalised) Stokes sums to
   img [n_obs][3][npix][npix].  nthreads > 1 splits the index range into
   contiguous blocks with private images summed in thread order. */
int oracle_run(const og_scene *S, uint64_t first, uint64_t count, double *img, og_counters *C,
               int64_t nthreads, double *events, int64_t max_events, int64_t *n_events)
{
    if (first < 1 || S->n_obs < 1 || S->npix < 1) return -1;
    if (S->order_images > 0 && S->order_images < S->max_orders) return -1;
    og_seq q = {S->seq_kind, S->dims, S->mat, S->bases, S->seed, S->n_total};
    og_obs *obs = (og_obs *)malloc(sizeof(og_obs) * (size_t)S->n_obs);
    for (int o = 0; o < S->n_obs; ++o) og_make_obs(S->obs_theta[o], S->obs_phi[o], &obs[o]);
    size_t img_n = (size_t)S->n_obs * 3 * (size_t)S->npix * (size_t)S->npix *
                   (size_t)(S->order_images > 0 ? S->order_images : 1);
    int64_t zero = 0;
    if (n_events) *n_events = 0;
    if (nthreads <= 1 || events) {
        og_sink sink = {img, C, events, max_events, n_events ? n_events : &zero};
        for (uint64_t j = 0; j < count; ++j) og_packet(S, &q, obs, first + j, &sink);
    } else {
#ifdef _OPENMP
        int nt = (int)nthreads;
        double *priv = (double *)calloc(img_n * (size_t)nt, sizeof(double));
        og_counters *pc = (og_counters *)calloc((size_t)nt, sizeof(og_counters));
#pragma omp parallel num_threads(nt)
        {
            int tid = omp_get_thread_num();
            int nth = omp_get_num_threads();
            uint64_t lo = count * (uint64_t)tid / (uint64_t)nth;
            uint64_t hi = count * (uint64_t)(tid + 1) / (uint64_t)nth;
            og_sink sink = {priv + img_n * (size_t)tid, &pc[tid], NULL, 0, &zero};
            for (uint64_t j = lo; j < hi; ++j) og_packet(S, &q, obs, first + j, &sink);
        }
        for (int t = 0; t < nt; ++t) {
            for (size_t e = 0; e < img_n; ++e) img[e] += priv[img_n * (size_t)t + e];
            og_add_counters(C, &pc[t]);
        }
        free(priv);
        free(pc);
#else
        og_sink sink = {img, C, NULL, 0, &zero};
        for (uint64_t j = 0; j < count; ++j) og_packet(S, &q, obs, first + j, &sink);
#endif
    }
    free(obs);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* brute-force quadrature of single scattering from a point source           */
/* ------------------------------------------------------------------------- */
/* Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_n. */
static void og_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(OG_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-15) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* Scattered flux toward one observer, first order, point source (Sec. 3.2, 3.5, 3.6):
     F = omega/(4 pi) * 1/(4 pi) * Int dOmega Int_0^edge ds kr(s) e^{-tau(0->s)} P11(k.o) e^{-tau_obs(s)}
   over points whose image projection falls inside the image.  Directions use
   Gauss-Legendre in cos(theta) (n_mu nodes) and the trapezoid rule in phi
   (n_phi nodes); each cell segment along a direction uses n_seg Gauss nodes. */
double oracle_quad_flux(const og_scene *S, int64_t obs, int64_t n_mu, int64_t n_phi, int64_t n_seg)
{
    og_obs O;
    og_make_obs(S->obs_theta[obs], S->obs_phi[obs], &O);
    double *mu = (double *)malloc(sizeof(double) * (size_t)n_mu), *wmu = (double *)malloc(sizeof(double) * (size_t)n_mu);
    double *gx = (double *)malloc(sizeof(double) * (size_t)n_seg), *gw = (double *)malloc(sizeof(double) * (size_t)n_seg);
    og_gauss_legendre((int)n_mu, mu, wmu);
    og_gauss_legendre((int)n_seg, gx, gw);
    const int64_t n[3] = {S->nx, S->ny, S->nz};
    double h[3];
    for (int a = 0; a < 3; ++a) h[a] = (S->hi[a] - S->lo[a]) / (double)n[a];
    double total = 0.0;
#pragma omp parallel for reduction(+ : total) schedule(dynamic)
    for (int64_t im = 0; im < n_mu; ++im) {
        double ct = mu[im], st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double acc_mu = 0.0;
        for (int64_t ip = 0; ip < n_phi; ++ip) {
            double ph = 2.0 * OG_PI * (ip + 0.5) / (double)n_phi;
            double k[3] = {st * cos(ph), st * sin(ph), ct};
            double c = og_dot(k, O.o), p11, r12, r33;
            og_mueller(S->g, S->p_lin, c, &p11, &r12, &r33);
            /* walk the cells along k, integrating each segment with Gauss nodes */
            int64_t cc[3], step[3];
            double tmax[3];
            for (int a = 0; a < 3; ++a) {
                double f = floor((S->src[a] - S->lo[a]) / h[a]);
                if (f < 0.0) f = 0.0;
                if (f > (double)(n[a] - 1)) f = (double)(n[a] - 1);
                cc[a] = (int64_t)f;
                step[a] = k[a] > 0.0 ? 1 : (k[a] < 0.0 ? -1 : 0);
                tmax[a] = step[a] == 0 ? INFINITY
                          : (S->lo[a] + (double)(cc[a] + (step[a] > 0)) * h[a] - S->src[a]) / k[a];
            }
            double t = 0.0, tau = 0.0, ray = 0.0;
            for (;;) {
                int a = 0;
                if (tmax[1] < tmax[a]) a = 1;
                if (tmax[2] < tmax[a]) a = 2;
                double tn = tmax[a], seg = tn - t;
                if (seg < 0.0) seg = 0.0;
                double kr = (double)S->kr[(cc[2] * n[1] + cc[1]) * n[0] + cc[0]];
                if (kr > 0.0 && seg > 0.0) {
                    for (int j = 0; j < n_seg; ++j) {
                        double s = t + 0.5 * seg * (gx[j] + 1.0);
                        double p[3] = {S->src[0] + s * k[0], S->src[1] + s * k[1], S->src[2] + s * k[2]};
                        double X = og_dot(p, O.ex), Y = og_dot(p, O.ey), R = S->half_width;
                        double fx = floor((X + R) / (2.0 * R) * (double)S->npix);
                        double fy = floor((Y + R) / (2.0 * R) * (double)S->npix);
                        if (fx < 0.0 || fy < 0.0 || fx >= (double)S->npix || fy >= (double)S->npix) continue;
                        double tau_obs = og_walk(S, p, O.o, 0, 0.0, NULL, NULL, NULL);
                        double tau_s = tau + kr * (s - t);
                        ray += 0.5 * seg * gw[j] * kr * exp(-tau_s) * exp(-tau_obs);
                    }
                }
                tau += kr * seg;
                if (tn > t) t = tn;
                cc[a] += step[a];
                if (cc[a] < 0 || cc[a] >= n[a]) break;
                tmax[a] = (S->lo[a] + (double)(cc[a] + (step[a] > 0)) * h[a] - S->src[a]) / k[a];
            }
            acc_mu += ray * p11;
        }
        total += wmu[im] * acc_mu * (2.0 * OG_PI / (double)n_phi);
    }
    free(mu); free(wmu); free(gx); free(gw);
    return S->albedo / (4.0 * OG_PI) * total / (4.0 * OG_PI);
}

/* Per-pixel first-order image of a point source by quadrature over the volume
   seen through each pixel (the same integral as oracle_quad_flux after the
   change of variables dOmega ds = dV / |p|^2, dV = dX dY dZ in image axes):
     I_pix = Int_pix dX dY Int dZ kr e^{-tau(src->p)} omega P11/(4 pi) e^{-tau_obs} / (4 pi |p-src|^2)
   with n_sub x n_sub midpoint sub-pixels and n_seg Gauss nodes per cell
   segment along the line of sight.  out: [npix][npix] (I only). */
int oracle_quad_pixels(const og_scene *S, int64_t obs, int64_t n_sub, int64_t n_seg, double *out)
{
    og_obs O;
    og_make_obs(S->obs_theta[obs], S->obs_phi[obs], &O);
    double *gx = (double *)malloc(sizeof(double) * (size_t)n_seg), *gw = (double *)malloc(sizeof(double) * (size_t)n_seg);
    og_gauss_legendre((int)n_seg, gx, gw);
    const int64_t np = S->npix;
    const double R = S->half_width, pw = 2.0 * R / (double)np, sw = pw / (double)n_sub;
    const int64_t n[3] = {S->nx, S->ny, S->nz};
    double h[3];
    for (int a = 0; a < 3; ++a) h[a] = (S->hi[a] - S->lo[a]) / (double)n[a];
    /* the line of sight enters the box from the far side: start far behind and walk along +o */
    double far = 0.0;
    for (int a = 0; a < 3; ++a) far += (S->hi[a] - S->lo[a]) * (S->hi[a] - S->lo[a]);
    far = sqrt(far) + 1.0;
#pragma omp parallel for schedule(dynamic)
    for (int64_t pix = 0; pix < np * np; ++pix) {
        int64_t iy = pix / np, ix = pix % np;
        double acc = 0.0;
        for (int64_t sy = 0; sy < n_sub; ++sy)
            for (int64_t sx = 0; sx < n_sub; ++sx) {
                double X = -R + ix * pw + (sx + 0.5) * sw;
                double Y = -R + iy * pw + (sy + 0.5) * sw;
                double q0[3];
                for (int a = 0; a < 3; ++a) q0[a] = X * O.ex[a] + Y * O.ey[a] - far * O.o[a];
                /* entry distance into the box along +o (slab method) */
                double t0 = 0.0, t1 = INFINITY;
                int hit = 1;
                for (int a = 0; a < 3; ++a) {
                    if (O.o[a] == 0.0) {
                        if (q0[a] < S->lo[a] || q0[a] > S->hi[a]) hit = 0;
                        continue;
                    }
                    double ta = (S->lo[a] - q0[a]) / O.o[a], tb = (S->hi[a] - q0[a]) / O.o[a];
                    if (ta > tb) { double tt = ta; ta = tb; tb = tt; }
                    if (ta > t0) t0 = ta;
                    if (tb < t1) t1 = tb;
                }
                if (!hit || t0 >= t1) continue;
                /* walk cells along the line from the entry point */
                double pe[3];
                for (int a = 0; a < 3; ++a) pe[a] = q0[a] + (t0 + 1e-12) * O.o[a];
                int64_t cc[3], step[3];
                double tmax[3];
                for (int a = 0; a < 3; ++a) {
                    double f = floor((pe[a] - S->lo[a]) / h[a]);
                    if (f < 0.0) f = 0.0;
                    if (f > (double)(n[a] - 1)) f = (double)(n[a] - 1);
                    cc[a] = (int64_t)f;
                    step[a] = O.o[a] > 0.0 ? 1 : (O.o[a] < 0.0 ? -1 : 0);
                    tmax[a] = step[a] == 0 ? INFINITY
                              : (S->lo[a] + (double)(cc[a] + (step[a] > 0)) * h[a] - pe[a]) / O.o[a];
                }
                double t = 0.0;
                for (;;) {
                    int a = 0;
                    if (tmax[1] < tmax[a]) a = 1;
                    if (tmax[2] < tmax[a]) a = 2;
                    double tn = tmax[a], seg = tn - t;
                    if (seg < 0.0) seg = 0.0;
                    double kr = (double)S->kr[(cc[2] * n[1] + cc[1]) * n[0] + cc[0]];
                    if (kr > 0.0 && seg > 0.0) {
                        for (int j = 0; j < n_seg; ++j) {
                            double s = t + 0.5 * seg * (gx[j] + 1.0);
                            double p[3], d[3];
                            for (int b = 0; b < 3; ++b) { p[b] = pe[b] + s * O.o[b]; d[b] = p[b] - S->src[b]; }
                            double r2 = og_dot(d, d), r = sqrt(r2);
                            double kd[3] = {d[0] / r, d[1] / r, d[2] / r};
                            double tau_s = og_walk(S, S->src, kd, 2, r, NULL, NULL, NULL);
                            double tau_obs = og_walk(S, p, O.o, 0, 0.0, NULL, NULL, NULL);
                            double c = og_dot(kd, O.o), p11, r12, r33;
                            og_mueller(S->g, S->p_lin, c, &p11, &r12, &r33);
                            acc += 0.5 * seg * gw[j] * sw * sw * kr * exp(-tau_s) * S->albedo * p11 /
                                   (4.0 * OG_PI) * exp(-tau_obs) / (4.0 * OG_PI * r2);
                        }
                    }
                    if (tn > t) t = tn;
                    cc[a] += step[a];
                    if (cc[a] < 0 || cc[a] >= n[a]) break;
                    tmax[a] = (S->lo[a] + (double)(cc[a] + (step[a] > 0)) * h[a] - pe[a]) / O.o[a];
                }
            }
        out[pix] = acc;
    }
    free(gx); free(gw);
    return 0;
}

/*
 * qrt.h -- C ABI of the MI355X quasi-Monte Carlo radiative-transfer library.
 *
 * The library transports photon packets of dust-continuum radiation through a
 * Cartesian density mesh and images the scattered light, as in S. G. Shulman,
 * "Quasi-Monte Carlo Radiative Transfer" (Astronomy and Computing).  Every
 * packet is driven by one point of a low-discrepancy sequence (Sobol,
 * Niederreiter base 2, Halton, Hammersley) or of a counter-based PRNG for the
 * Monte Carlo baseline (Sec. 3.1, Sec. 3.7).  One packet goes through
 * emission (Sec. 3.2, 3.3), optical depth to the mesh edge with a forced first
 * scattering (Sec. 3.2), moves by optical depth on the mesh (Sec. 3.4),
 * peel-off toward each observer before each scattering (Sec. 3.5, 3.6) and
 * Henyey-Greenstein scattering with White's Mueller matrix (Sec. 2.2, 3.5).
 *
 * Conventions shared by all calls
 *  - Every call returns QRT_OK (0) or a negative status; qrt_last_error()
 *    gives a message, valid until the next call on the same context.
 *  - No C++ exception crosses this interface.
 *  - Host pointers are owned by the caller and only read or written during
 *    the call.  Device pointers are HIP device addresses on the context's
 *    device.
 *  - All GPU work goes to the context's HIP stream, in order.  Calls that
 *    return host data synchronise that stream; the others only enqueue work.
 *  - One context per host thread; a context is not thread safe.
 *  - Packet indices are global and start at 1: the all-zero first point of
 *    every low-discrepancy sequence is skipped (Sec. 3.1).  Runs over disjoint
 *    index ranges add up, so a long run may be split into chunks and resumed.
 *  - Images are in units of the source luminosity and hold scattered light
 *    only (Sec. 3.4, 3.6).
 */
#ifndef QRT_H
#define QRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define QRT_OK 0
#define QRT_INVALID_ARG (-1)     /* a pointer, size or value is out of range */
#define QRT_BAD_STATE (-2)       /* e.g. a run before the grid is set */
#define QRT_HIP_ERROR (-3)       /* a HIP call failed; the message has hipGetErrorString */
#define QRT_OUT_OF_MEMORY (-4)
#define QRT_UNSUPPORTED (-5)     /* too many dimensions, Hammersley index beyond N, ... */
#define QRT_NOT_TRAINED (-6)     /* surrogate peel-off requested without a trained network */

/* point sets (Sec. 3.1) */
#define QRT_SOBOL 0
#define QRT_HALTON 1
#define QRT_NIEDERREITER2 2
#define QRT_HAMMERSLEY 3
#define QRT_PHILOX 4
#define QRT_FAURE 5               /* Faure (1982), base = smallest prime >= the coordinates used */
#define QRT_SOBOL_OWEN 6          /* Sobol with Owen's nested uniform scrambling keyed by the seed */

/* grid ownership flags for qrt_set_grid */
#define QRT_GRID_HOST_COPY 0      /* kappa_rho is a host pointer; copied */
#define QRT_GRID_DEVICE_COPY 1    /* kappa_rho is a device pointer; copied on the device */
#define QRT_GRID_DEVICE_BORROW 2  /* as QRT_GRID_DEVICE_COPY (the library keeps the mesh in its own cell order) */

/* arithmetic of the transport */
#define QRT_FP32 0                /* FP32 positions/directions/weights, FP64 optical depth and image sums */
#define QRT_FP64 1                /* FP64 throughout */

/* peel-off optical depth */
#define QRT_PEEL_EXACT 0          /* exact mesh traversal toward the observer */
#define QRT_PEEL_SURROGATE 1      /* trained network inside its validated domain, exact elsewhere */

/* sphere-star emission order (Sec. 3.3) */
#define QRT_EMIT_DIRECT 0         /* v1,v2 emission point; v3,v4 local direction; v5 tau */
#define QRT_EMIT_INVERSE 1        /* v1,v2 direction; v3 tau; v4,v5 emission point about the direction */

#define QRT_MAX_DIMS 128          /* largest point dimension served */
#define QRT_MAX_OBSERVERS 16

typedef struct qrt_ctx qrt_ctx;

/* Exact event counts accumulated over runs since the last reset. */
typedef struct {
    int64_t packets;      /* packets started */
    int64_t visits;       /* mesh cells entered by every traversal (Sec. 3.4) */
    int64_t peels;        /* peel-off contributions binned into an image */
    int64_t peel_rays;    /* peel-off traversals toward observers */
    int64_t escapes;      /* packets that left the mesh during a free flight */
    int64_t tau_cuts;     /* packets ended because tau1 < tau_min (Sec. 3.2) */
    int64_t scatterings;  /* scattering events (each is followed by its peel-offs) */
    int64_t occluded;     /* peel-off rays blocked by a sphere star */
    int64_t surrogate;    /* peel-off optical depths taken from the network */
    int64_t fallbacks;    /* surrogate requests answered by exact traversal */
    int64_t visits_first; /* the part of visits made by the first flights: the walk to the mesh edge
                             for tau1 and the forced flight (Sec. 3.2); the rest are the per-order
                             peel-off rays and free flights */
} qrt_counters;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
   (a hipStream_t; NULL selects the null stream).  *out is NULL on failure. */
int qrt_create(qrt_ctx **out, int device, void *hip_stream);

/* Release the context and all library-owned device memory.  NULL is a no-op. */
void qrt_destroy(qrt_ctx *ctx);

/* Message of the last failing call on ctx (never NULL). */
const char *qrt_last_error(const qrt_ctx *ctx);

/* Change the stream later calls enqueue on. */
int qrt_set_stream(qrt_ctx *ctx, void *hip_stream);

/* Density mesh (Sec. 2.1, 3.4): nx*ny*nz cells over the box [lo, hi]; each cell
   holds the constant extinction kappa*rho (FP32), laid out [nz][ny][nx] with x
   fastest.  flags is one of QRT_GRID_*.  Cells must be finite and >= 0 (checked
   for host input).  The library copies the mesh into its own order (bricks of
   4x4x4 cells, the brick counts along x and y rounded up to powers of two; at
   most 2^29 stored cells and 2^20 cells per axis, else QRT_UNSUPPORTED); the
   caller's buffer is not used after the call returns. */
int qrt_set_grid(qrt_ctx *ctx, int nx, int ny, int nz, const double lo[3], const double hi[3],
                 const float *kappa_rho, int flags);

/* Isotropic point source at (x, y, z), which must lie inside the box (Sec. 3.2). */
int qrt_set_point_source(qrt_ctx *ctx, double x, double y, double z);

/* Uniform-brightness spherical star of the given radius centred at (x, y, z)
   (Sec. 3.3), emitting in the direct or the inverse order of the point
   coordinates.  Direct: point on the star from (2 pi v1, cos = 2 v2 - 1),
   local direction (2 pi v3, cos = sqrt(v4)) about the surface normal, tau
   from v5.  Inverse: direction from (2 pi v1, cos = 2 v2 - 1), tau from v3,
   emission point on the hemisphere facing the direction from (2 pi v4,
   cos = sqrt(v5)) about it (a uniform-brightness surface seen from the
   direction).  Both give the same joint law of point and direction.  The star
   blocks peel-off rays that pass through it. */
int qrt_set_sphere_source(qrt_ctx *ctx, double x, double y, double z, double radius, int order);

/* Dust (Sec. 2.1-2.3): albedo in [0,1], HG asymmetry |g| < 1, maximum linear
   polarisation p_lin in [0,1]; p_circ must be 0 (circular polarisation unused). */
int qrt_set_dust(qrt_ctx *ctx, double albedo, double g, double p_lin, double p_circ);

/* Observers at infinity in directions (theta[i], phi[i]) (radians, Sec. 3.6),
   1 <= n_obs <= QRT_MAX_OBSERVERS.  Each image is npix x npix pixels covering
   [-half_width, half_width]^2 in image axes e_x = (-sin phi, cos phi, 0),
   e_y = o x e_x.  Resets the images.  If the image memory cannot be
   allocated (QRT_OUT_OF_MEMORY), the context is left with no observers: runs
   and image reads return QRT_BAD_STATE until a later call succeeds. */
int qrt_set_observers(qrt_ctx *ctx, int n_obs, const double *theta, const double *phi, int npix,
                      double half_width);

/* Point set (Sec. 3.1): kind QRT_*, seed (PRNG key, or the scrambling key of
   QRT_SOBOL_OWEN; ignored by the other low-discrepancy kinds) and n_total
   (Hammersley's N, 1 <= N < 2^32; ignored by the others). */
int qrt_set_sequence(qrt_ctx *ctx, int kind, uint64_t seed, uint64_t n_total);

/* Transport (Sec. 3.2, 3.5): at most max_orders scatterings (1 .. 42 for a
   point source), tau_min cut-off of the first flight, precision QRT_FP32 or
   QRT_FP64, peel_mode QRT_PEEL_EXACT or QRT_PEEL_SURROGATE (needs network
   parameters and a domain, else QRT_NOT_TRAINED; see the surrogate section). */
int qrt_set_transport(qrt_ctx *ctx, int max_orders, double tau_min, int precision, int peel_mode);

/* Transport packets first_index .. first_index+count-1 (first_index >= 1) and
   add their contributions to the images.  Asynchronous on the context stream.
   Indices stay below 2^32 for the low-discrepancy sets and below 2^48 for
   QRT_PHILOX, else QRT_UNSUPPORTED. */
int qrt_run(qrt_ctx *ctx, uint64_t first_index, uint64_t count);

/* Overlapped runs (off by default).  While enabled, qrt_run puts each chunk
   on one of three internal streams of the context in turn, with buffers of
   its own, after everything already enqueued on the context stream; its
   completion joins the context stream once two more chunks have been put on
   the other streams, at the next call of the library on this context other
   than qrt_run (any call but the host-side setters), or at qrt_join.
   Consecutive runs then overlap: the next runs start while the last
   scattering orders of the previous ones, which occupy few compute units,
   are still walking.  Callers that time qrt_run with their own events, or
   enqueue work that reads the images without calling the library first,
   call qrt_join before.  Disabling joins whatever is pending.  qrt_batch_run
   puts its chunks on the streams in the same way; qrt_run_static never
   overlaps. */
int qrt_set_overlap(qrt_ctx *ctx, int enable);

/* Late scattering orders in one launch (Sec. 2.2, 3.5: the same transport,
   launched differently).  From order first_order on (default 2; 0 turns it
   off) a run carries each live packet through its remaining orders in one
   kernel, a lane per packet, keeping the state of every scattering it passes;
   those scatterings are sorted by position, one launch computes their peel-off
   contributions and one more walks their rays, instead of two launches per
   order.  Images differ from the per-order launches only in the order of the
   FP64 sums, counters not at all.  max_deferred bounds the scatterings held
   (0: as many as the live-packet list and the peel-ray buffer hold); a
   scattering beyond it has its peel-offs computed and walked at once by the
   lane that reached it.  In the surrogate mode the deferred scatterings'
   network queries go to one network launch (as many as the query queue
   holds, which also bounds the scatterings held).  Used with one image set
   (not with per-order images), and for batches, where the orders counted are
   those of the batch's deepest scene; a first_order above the largest
   max_orders leaves every order to the per-order launches.  Joins pending
   overlapped runs.  In very thick scenes, where packets scatter more often
   than the list holds (more than about once per packet after the first
   order), a later first_order (4) keeps the late orders' peel-offs from
   spilling into the late-order kernel.  QRT_INVALID_ARG for first_order 1 or
   below 0. */
int qrt_set_tail(qrt_ctx *ctx, int first_order, uint64_t max_deferred);

/* The context stream waits for every overlapped run still pending
   (asynchronous, like qrt_run). */
int qrt_join(qrt_ctx *ctx);

/* qrt_run for callers that cannot allocate device memory: code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc.  It transports
   the same packets with the same kernels and adds the same contributions to
   the images, but takes every transport buffer (packet states, peel-off slots,
   sort lists, queue counters) from a static scratch array of 36 MiB that each
   device holds from the library's load to the end of the process, in chunks
   of 2^16 packets; it calls no hipMalloc, hipFree or other allocating routine.
   The grid, images, counters and tables are the context's, allocated by the
   set-up calls.  Limits: QRT_UNSUPPORTED when a chunk's buffers exceed the
   scratch (more than 4 observers in FP64, more than 12 in FP32; with the
   surrogate peel-off, whose queue takes scratch too, more than 2 and 5);
   QRT_BAD_STATE for Faure points whose tables no earlier qrt_run or
   qrt_generate_points built for this many coordinates.  All contexts on one
   device share its scratch: calls that overlap on one device (other streams,
   other host threads) race and must be serialised by the caller.  Asynchronous
   on the context stream, like qrt_run. */
int qrt_run_static(qrt_ctx *ctx, uint64_t first_index, uint64_t count);

/* Copy image obs (npix*npix doubles each, [iy][ix]) of Stokes I, Q, U to host
   buffers (any may be NULL).  normalized = 1 divides by the number of packets
   run since the last reset.  Synchronises the stream. */
int qrt_read_images(qrt_ctx *ctx, int obs, double *I, double *Q, double *U, int normalized);

/* Device address of the FP64 image sums [n_obs][3][npix][npix] (unnormalised),
   owned by the context.  The kernels accumulate into several copies; this call
   enqueues their fold into the returned array, which is therefore complete
   once the stream reaches this point. */
int qrt_image_device_ptr(qrt_ctx *ctx, double **dev_ptr);

/* Keep one image set per scattering order 1..max_orders (enable = 1) or one
   summed set (enable = 0, the default).  Allocates max_orders times the image
   memory and resets the images.  While it is on, max_orders cannot change,
   qrt_read_images returns the sum over the orders, and qrt_image_device_ptr
   is refused.  If the memory cannot be allocated (QRT_OUT_OF_MEMORY), the
   context is left with no observers and no per-order images, as after a
   failed qrt_set_observers. */
int qrt_set_order_images(qrt_ctx *ctx, int enable);

/* Copy the images of scattering order `order` (1-based) of observer obs, as
   qrt_read_images.  Synchronises the stream. */
int qrt_read_order_images(qrt_ctx *ctx, int obs, int order, double *I, double *Q, double *U, int normalized);

/* Zero the images, the packet count and the counters. */
int qrt_reset_images(qrt_ctx *ctx);

/* Counters accumulated since the last reset.  Synchronises the stream. */
int qrt_get_counters(qrt_ctx *ctx, qrt_counters *out);

/* Kernel timing (a measurement aid, off by default).  While enabled, qrt_run
   and qrt_batch_run record a pair of HIP events on the context stream around
   every kernel launch, by class: QRT_T_SORT (emission keys and the radix sort),
   QRT_T_FIRST (first flights), QRT_T_SCATTER (scattering, peel-off
   contributions, new directions), QRT_T_WALK (peel-off rays and free flights of
   one order), QRT_T_PEEL_MLP (surrogate peel-off), QRT_T_OTHER (queue clears,
   pilot capture).  qrt_get_timing synchronises the stream and returns, per
   class, the summed milliseconds between each pair and the number of launches
   since the last reset (reset = 1 clears them afterwards).  The events cost a
   few microseconds per launch; qrt_run_static records none. */
enum { QRT_T_SORT = 0, QRT_T_FIRST = 1, QRT_T_SCATTER = 2, QRT_T_WALK = 3, QRT_T_PEEL_MLP = 4, QRT_T_OTHER = 5,
       QRT_T_CLASSES = 6 };
typedef struct {
    double ms[QRT_T_CLASSES];
    int64_t launches[QRT_T_CLASSES];
} qrt_timing;
int qrt_set_timing(qrt_ctx *ctx, int enable);
int qrt_get_timing(qrt_ctx *ctx, qrt_timing *out, int reset);

/* Coordinates of points first .. first+count-1, dims each, as unsigned 0.32
   fixed point, row-major [count][dims] (Sec. 3.1).  out is a device pointer
   when out_on_device = 1 (then asynchronous), else a host pointer. */
int qrt_generate_points(qrt_ctx *ctx, int kind, uint64_t seed, uint64_t n_total, uint64_t first,
                        uint64_t count, int dims, uint32_t *out, int out_on_device);

/* Optical depth from (p[3*i]) along unit (k[3*i]) to the mesh edge for n rays,
   at the context precision; visits (may be NULL) gets cells entered per ray.
   All pointers are device pointers; asynchronous (Sec. 3.4). */
int qrt_trace_tau(qrt_ctx *ctx, int64_t n, const double *p, const double *k, double *tau,
                  int64_t *visits);

/* ---------------------------------------------------------------------------
 * Surrogate peel-off optical depth.
 *
 * An addition to the paper's method: the paper finds that integrating optical
 * depth along rays takes almost all of the run time (Sec. 3.1), and the
 * peel-off rays toward the observers (Sec. 3.6) are most of those rays.
 * Inside a validated domain the surrogate replaces the traversal of a
 * peel-off ray by a small network tau_hat(x, y, z, theta_obs, phi_obs):
 *   5 inputs -> 4 hidden layers of 64 ReLU units -> 1 output, clamped at 0.
 * Inputs, in the coordinates of the domain below (computed in FP64, rounded
 * to FP32): (x - c_x) / r_out, (y - c_y) / r_out, (z - c_z) / (zmax h(R))
 * clamped to [-4, 4] (0 on the axis), 2 theta / pi - 1 and phi / pi - 1 of
 * the observer.
 * Inference and training run on the matrix cores in bfloat16 with FP32
 * accumulation; FP32 master weights and Adam moments.
 * Parameters: QRT_MLP_PARAMS FP32 values, layer by layer, each W[in][out]
 * row-major followed by b[out]: W0 5x64, b0, W1 64x64, b1, W2, b2, W3, b3,
 * W4 64x1, b4.
 * Domain: cylinder around `center`, R in [r_in, r_out) in n_r equal bins and
 * z / h(R) in (-zmax, zmax) in n_z equal bins, h(R) = h0 R^beta (a flared
 * disk's scale height); a mask [n_obs][n_r][n_z] marks the cells where the
 * network is used.  Every other peel-off ray is traversed exactly (the
 * fallback), so a zero mask reproduces the exact transport.
 * Samples: rows of 4 floats (x, y, z, observer index) with FP32 labels tau.
 * ------------------------------------------------------------------------- */

#define QRT_MLP_PARAMS 12929

typedef struct {
    int64_t steps;        /* Adam steps */
    int32_t batch;        /* samples per step: a multiple of 64 in 64 .. 65536 */
    int32_t init;         /* 1: fresh random initialisation from seed; 0: continue from the current parameters */
    float lr, lr_final;   /* learning rate, cosine-decayed from lr to lr_final over the steps */
    float beta1, beta2, eps;
    float tau_cap;        /* regression target min(tau, tau_cap) */
    float weight_floor;   /* sample weight exp(-target) + weight_floor */
    uint64_t seed;        /* initialisation and batch selection */
} qrt_train_cfg;

typedef struct {
    double loss_first;    /* weighted squared error over all samples before and after training */
    double loss_final;
    int64_t steps;
} qrt_train_report;

typedef struct {
    int64_t cells;        /* n_obs * n_r * n_z */
    int64_t valid_cells;  /* cells marked for the network */
    int64_t samples;      /* validation samples inside the domain */
    int64_t samples_valid;/* ... of which in valid cells */
    double max_err_valid; /* largest transmission error of a valid cell */
} qrt_mask_report;

/* Network parameters from / to the host (n = QRT_MLP_PARAMS).  Setting them
   resets the Adam moments.  Synchronous. */
int qrt_mlp_set_params(qrt_ctx *ctx, const float *params, int64_t n);
int qrt_mlp_get_params(qrt_ctx *ctx, float *params, int64_t n);

/* Random parameters: weights uniform in +-sqrt(6 / fan_in), biases 0. */
int qrt_mlp_init(qrt_ctx *ctx, uint64_t seed);

/* Raw network outputs y[n] (not clamped) for normalised inputs X[n][5].
   Device pointers; asynchronous. */
int qrt_mlp_forward(qrt_ctx *ctx, int64_t n, const float *X, float *y);

/* grad[QRT_MLP_PARAMS] = gradient of sum_j dy[j] * y[j] over rows X[n][5]
   (1 <= n <= 2^24).  Device pointers; asynchronous. */
int qrt_mlp_backward(qrt_ctx *ctx, int64_t n, const float *X, const float *dy, float *grad);

/* Domain of the surrogate; clears the mask (no cell uses the network).
   Changing the observers clears the mask too. */
int qrt_surrogate_set_domain(qrt_ctx *ctx, const double center[3], double r_in, double r_out, double h0,
                             double beta, double zmax_over_h, int n_r, int n_z);

/* Mask [n_obs][n_r][n_z] (1 = use the network) from / to the host. */
int qrt_surrogate_set_mask(qrt_ctx *ctx, const uint8_t *mask);
int qrt_surrogate_get_mask(qrt_ctx *ctx, uint8_t *mask);

/* Network inputs X[n][5] of sample rows pos_obs[n][4] (needs a domain).
   Device pointers; asynchronous. */
int qrt_surrogate_inputs(qrt_ctx *ctx, int64_t n, const float *pos_obs, float *X);

/* Training samples from a pilot run: Philox packets (key seed) of the current
   scene, exact peel-off, chunk by chunk until n visible peel-off rays inside
   the domain are captured; of all captured rays the n with the smallest hash
   of their bytes and the seed are kept (a reproducible uniform subsample;
   rays whose 64-bit hashes collide keep the order of their capture).  Labels
   are the exact FP64 optical depths toward the observer.  Capture, selection
   (a device radix sort) and labels run on the device; only the per-chunk
   capture count comes back to the host.  pos_obs[n][4] and tau[n] are device
   pointers; *pilot_packets (may be NULL) gets the packets run.  Resets the
   images and counters.  Synchronous; 1 <= n <= 2^26. */
int qrt_surrogate_sample(qrt_ctx *ctx, int64_t n, uint64_t seed, float *pos_obs, float *tau,
                         int64_t *pilot_packets);

/* Adam on the weighted squared error of the network against min(tau, cap)
   with weights exp(-min(tau, cap)) + weight_floor, batches drawn by a hash of
   (seed, step, position).  Device sample buffers; rep may be NULL.
   Synchronous (reads the loss before and after). */
int qrt_surrogate_train(qrt_ctx *ctx, int64_t n, const float *pos_obs, const float *tau, const qrt_train_cfg *cfg,
                        qrt_train_report *rep);

/* Builds the mask from validation samples: a cell (observer, R bin, z bin)
   is valid when it holds at least min_count samples and its transmission
   error  sum |exp(-tau_hat) - exp(-tau)| / sum max(exp(-tau), T_floor)
   over them is at most max_err, where T_floor = floor_frac times the mean
   transmission of that observer's samples in the domain (floor_frac = 0: the
   plain relative error; a floor keeps cells whose light is too faint to
   matter from failing on their relative error alone).  The sums run on the
   device in fixed point (each term rounded to 2^-40 or coarser for very large
   n), so the mask does not depend on the order of the additions.
   Device sample buffers; rep may be NULL.  Synchronous. */
int qrt_surrogate_validate(qrt_ctx *ctx, int64_t n, const float *pos_obs, const float *tau, double max_err,
                           double floor_frac, int64_t min_count, qrt_mask_report *rep);

/* The trained surrogate as one blob: parameters, domain, mask, and the
   observer directions the mask was validated for.  get: blob NULL returns the
   size in *nbytes; otherwise *nbytes is the blob's capacity (too small:
   QRT_INVALID_ARG, *nbytes set to the size).  set: the context's observers
   must be the blob's (else QRT_BAD_STATE); resets the Adam moments.
   Synchronous. */
int qrt_surrogate_get_state(qrt_ctx *ctx, void *blob, size_t *nbytes);
int qrt_surrogate_set_state(qrt_ctx *ctx, const void *blob, size_t nbytes);

/* ---------------------------------------------------------------------------
 * Batches of scenes.
 *
 * Many independent scenes of uneven size, each with its own mesh, source,
 * dust, 1..QRT_BATCH_MAX_OBSERVERS observers, image and packet range, run in
 * one launch sequence that treats all their packets as one queue of work.
 * Every packet follows exactly the transport of a single-scene run of its
 * scene (Sec. 3.2-3.7): the images of scene s equal those of qrt_run on that
 * scene with the same point set, indices and precision, up to the order of
 * the FP64 image sums.  Exact peel-off only; every point set but QRT_FAURE
 * (whose base depends on the coordinates used, which differ between scenes).
 * The batch's images and the context's counters are separate from those of
 * single-scene runs; counters of batch runs add to the context counters.
 * ------------------------------------------------------------------------- */

#define QRT_BATCH_MAX_OBSERVERS 4
#define QRT_BATCH_MAX_SCENES 1024

/* source kinds of a batch scene */
#define QRT_SOURCE_POINT 0        /* isotropic point source (Sec. 3.2) */
#define QRT_SOURCE_SPHERE 1       /* uniform-brightness sphere star (Sec. 3.3) */

typedef struct {
    int nx, ny, nz;               /* mesh cells; kappa_rho as for qrt_set_grid, a host pointer (copied) */
    double lo[3], hi[3];
    const float *kappa_rho;
    int source;                   /* QRT_SOURCE_POINT or QRT_SOURCE_SPHERE */
    int emit_order;               /* sphere star: QRT_EMIT_DIRECT or QRT_EMIT_INVERSE */
    double src[3];                /* source centre, inside the box (a star wholly inside) */
    double radius;                /* star radius (> 0 for a star, ignored for a point) */
    double albedo, g, p_lin;      /* dust as for qrt_set_dust (p_circ = 0) */
    int n_obs;                    /* 1 .. QRT_BATCH_MAX_OBSERVERS */
    double theta[QRT_BATCH_MAX_OBSERVERS], phi[QRT_BATCH_MAX_OBSERVERS];
    int npix;                     /* 1 .. 8192 */
    double half_width;
    int max_orders;               /* >= 1, point dimension <= QRT_MAX_DIMS */
    double tau_min;
    uint64_t first, count;        /* point indices first .. first+count-1 (first >= 1; count may be 0) */
    uint64_t n_total;             /* Hammersley's N of this scene (ignored by the other kinds) */
} qrt_batch_scene;

/* Set the scenes of the batch (1 <= n_scenes <= QRT_BATCH_MAX_SCENES): copies
   every mesh to the device, allocates the FP64 images of every scene (sixteen
   accumulators each, folded when read) and zeroes them.  Replaces a previous
   batch.  Synchronous. */
int qrt_batch_set(qrt_ctx *ctx, int n_scenes, const qrt_batch_scene *scenes);

/* Transport every scene's packets once with point set `kind` and `seed` (as
   for qrt_set_sequence) at `precision` (QRT_FP32 or QRT_FP64), adding to the
   batch images.  Asynchronous on the context stream (its chunks overlapped on
   the internal streams while qrt_set_overlap is on). */
int qrt_batch_run(qrt_ctx *ctx, int kind, uint64_t seed, int precision);

/* Copy the images of observer obs of scene `scene`, as qrt_read_images;
   normalized = 1 divides by the scene's packet count times the batch runs
   since the last reset.  Synchronises the stream. */
int qrt_batch_read_images(qrt_ctx *ctx, int scene, int obs, double *I, double *Q, double *U, int normalized);

/* Zero the batch images, the batch run count and the context counters. */
int qrt_batch_reset(qrt_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* QRT_H */

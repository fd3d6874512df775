/*
 * radiate.h -- C ABI of the MI355X (gfx950) differentiable acoustic radiation library.
 *
 * The library evaluates the far-field Gaussian-kernel radiation model of PA-SFM
 * (Li, Gao et al., arxiv 2604.09643) and its adjoints:
 *
 *   s[f,m,k] = sum_v p0[v] * phi(d - c t_k) / (2 d),   d = |x_v - x_e(f,m)|,
 *   phi(u)   = u * exp(-u^2 / (2 sigma^2)),            t_k = k / fs,
 *
 * keeping only the terms with |d - c t_k| <= trunc * sigma (the other source profiles
 * of Appendix A replace the Gaussian, see ra_sampling).  For the Gaussian the forward and
 * the dL/dp0-only adjoint take the samples within floor(trunc*sigma*fs/c + 1/2) of each
 * term's nearest sample whole: every kept term is among them, and each term they add
 * beyond the window is below psi(trunc) of the kernel's peak (psi(y) = y exp(-y^2/2);
 * 1.5e-7 at trunc = 6), and that adjoint evaluates each voxel-element pair's window sum
 * by an 8-term Taylor expansion whose error is below 1e-6 of the peak (the library takes
 * it only where that bound holds).  Main text Eq. (1)
 * sums the source intensity against a kernel of the source-sensor distance;
 * Appendix A, Eq. (A13) (the discretised far-field model with the Gaussian
 * kernel K_G) fixes the kernel used here.  Element positions follow the rigid
 * array of Stage 4: x_e(f,m) = R_f e_m + t_f.  The gradients with respect to
 * the source intensity and the sensor coordinates are the two directions of
 * gradient flow the paper's engine provides ("Differentiable Acoustic
 * Radiation").
 *
 * Conventions
 *   Units     SI: metres, seconds, hertz.
 *   Grid      voxel (i,j,k) centre = origin + (i,j,k) * spacing; volumes are
 *             float[nx][ny][nz] (z fastest).
 *   Poses     double[F][12]: R row-major (9 values) then t (3 values); the
 *             array template is double[M][3] in the probe frame.
 *   Signals   float[F][M][K], k fastest; element index e = f*M + m.
 *   Memory    every array argument is a DEVICE pointer unless stated otherwise.
 *             The caller owns all buffers.  The library owns only scratch inside
 *             ra_ctx (see ra_reserve).
 *   Streams   `stream` is a hipStream_t (NULL = the legacy default stream).
 *             Calls are stream-ordered and asynchronous.  They do not
 *             synchronise the host, except: loss_and_grad / nc_loss_and_grad /
 *             tgv_loss_and_grad with a HOST `loss` (loss_and_grad with
 *             RA_LOSS_ON_DEVICE does not), ra_count_updates and ra_status, which
 *             wait for their own result; and any call that must grow the
 *             context's scratch (see ra_reserve), which synchronises `stream`,
 *             frees the old scratch and allocates the new one first.
 *   Scratch   each ra_ctx owns ONE scratch buffer that every call on it uses, so
 *             calls on one context must be ordered: issue them on one stream
 *             (or order the streams yourself).  Two streams that run calls of
 *             the same context concurrently race on its scratch; give each
 *             stream its own context instead.
 *   Errors    every int-returning call returns one of the RA_* codes below;
 *             ra_last_error() holds a message for the last failing call.
 *             Arguments are validated before any work is enqueued.  Bulk
 *             arrays are not scanned: NaN/Inf in them propagate.  No C++
 *             exception crosses this boundary.
 *   Threads   one ra_ctx per host thread at a time; contexts are independent.
 */
#ifndef PASFM_RADIATE_H
#define PASFM_RADIATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RA_OK = 0,      /* success                                                        */
    RA_EINVAL = 1,  /* bad scalar, null required pointer, or unsupported sampling      */
    RA_EGEOM = 2,   /* (ra_status) an element was closer than 10*sigma to the grid box */
    RA_ENOMEM = 3,  /* scratch could not be allocated (or would be, under capture)     */
    RA_EHIP = 4,    /* a HIP runtime call failed; see ra_last_error()                  */
    RA_ENOTSUP = 5  /* valid request the library does not implement                    */
};

/* Flags for radiate_adjoint / loss_and_grad. */
#define RA_ACCUMULATE 1u     /* add into grad_p0 / grad_pose / grad_elem instead of overwriting */
#define RA_LOSS_ON_DEVICE 2u /* loss_and_grad: `loss` is a DEVICE double*, written on the stream
                                with no host synchronisation (so the call can be captured) */
#define RA_SIGNALS_GIVEN 4u  /* loss_and_grad: s_out already holds the forward signals of these
                                p0 and poses (an earlier call's s_out); the forward is not run */

/* How the forward model adds the partial signal rows of its voxel regions (ra_set_forward_sums).
 * Each region sums its voxels' contributions in FP32 (in LDS), then adds those rows into the
 * signals; with many regions meeting in one sample, FP32 additions lose accuracy, so large
 * grids add into FP64 sums (extra scratch of F*M*K doubles) that are rounded to FP32 at the end. */
enum {
    RA_SUMS_AUTO = 0, /* FP32 up to 4096 forward regions (e.g. 128x128x64 voxels), FP64 beyond */
    RA_SUMS_F32 = 1,  /* always FP32, straight into s                                            */
    RA_SUMS_F64 = 2   /* always FP64 sums                                                        */
};

typedef struct ra_ctx ra_ctx;

/* Voxel grid: voxel (i,j,k) centre = origin + (i,j,k)*spacing [m]; volume float[nx][ny][nz]. */
typedef struct {
    int32_t nx, ny, nz;
    double origin[3];
    double spacing;
} ra_grid;

/* Sampling: t_k = k/fs for k = 0..K-1; kernel width sigma [m]; a term is kept iff
 * |d - c t_k| <= trunc*sigma (trunc = 6 in the paper's setting).  Requires
 * trunc*sigma >= c/(2 fs) and trunc*sigma <= 40 c/fs (RA_EINVAL otherwise).
 *
 * kernel selects the source profile of Appendix A's analytical solutions, under the
 * far-field form p ~ (d - c t) K(|d - c t|) / (2 d), normalised to K(0) = 1 with width
 * w = sigma:
 *   RA_KERNEL_GAUSSIAN     exp(-x^2/(2 w^2))   (Eq. (A13); the fast path)
 *   RA_KERNEL_EXPONENTIAL  exp(-x/w)
 *   RA_KERNEL_POWER        (1 + x^2/w^2)^(-nu), nu > 1/2
 *   RA_KERNEL_UNIFORM      1 inside the window (a uniform sphere of radius w: trunc = 1)
 * The other profiles take voxels one at a time: the exponential factorises per leg of the
 * window, the power law and the uniform sphere evaluate every sample.  They are not
 * supported by the batched serving step (RA_ENOTSUP).  RA_EINVAL for an unknown kernel or,
 * with RA_KERNEL_POWER, nu <= 1/2 or not finite. */
enum { RA_KERNEL_GAUSSIAN = 0, RA_KERNEL_EXPONENTIAL = 1, RA_KERNEL_POWER = 2, RA_KERNEL_UNIFORM = 3 };
typedef struct {
    double c;       /* speed of sound [m/s]          */
    double fs;      /* sampling rate [Hz]            */
    int32_t K;      /* samples per element           */
    double sigma;   /* kernel width [m]              */
    double trunc;   /* window half-width in sigmas   */
    int32_t kernel; /* RA_KERNEL_*                    */
    double nu;      /* power-law exponent            */
} ra_sampling;

/* Create a context bound to HIP device `device` (it becomes current on the calling
 * thread).  *out receives the context.  Returns RA_OK, RA_EHIP or RA_ENOMEM. */
int ra_create(ra_ctx** out, int device);

/* Destroy a context and free its scratch.  The caller must make sure no work that
 * uses the context is still pending.  NULL is ignored. */
void ra_destroy(ra_ctx* ctx);

/* Message describing the last non-OK return of a call on this context ("" if none).
 * The pointer stays valid until the next call on the context. */
const char* ra_last_error(const ra_ctx* ctx);

/* Synchronise `stream` and report device-side geometry checks of all calls made
 * since the previous ra_status: RA_EGEOM if any element came closer than 10*sigma
 * to the axis-aligned box of the voxel centres (the far-field kernel assumes
 * distances well above the kernel width, Appendix A "Far-Field Approximations");
 * results of such calls are computed but not meaningful.  Clears the flag. */
int ra_status(ra_ctx* ctx, void* stream);

/* Grow the context's device scratch to at least `bytes`.  Calls allocate scratch
 * on demand outside stream capture; under capture they return RA_ENOMEM instead,
 * so reserve first when capturing into a HIP graph.  ra_scratch_bytes() reports
 * what any call with the given sizes needs (whatever ra_set_forward_sums chose). */
int ra_reserve(ra_ctx* ctx, size_t bytes);
size_t ra_scratch_bytes(const ra_grid* grid, int32_t M, int32_t F, const ra_sampling* samp);

/* Choose how this context's forward calls add their partial rows (RA_SUMS_*; default
 * RA_SUMS_AUTO).  RA_EINVAL for another value.  Host-only. */
int ra_set_forward_sums(ra_ctx* ctx, int32_t mode);

/* Forward model (Eq. (1) with the kernel of Eq. (A13), or the profile samp->kernel selects).
 *   p0     float[nx][ny][nz]            initial pressure per voxel
 *   elem   double[M][3]                 array template, probe frame
 *   poses  double[F][12]                rigid pose per frame (R row-major, t)
 *   s      float[F][M][K]  (output)     overwritten */
int radiate_forward(ra_ctx* ctx, const ra_grid* grid, const float* p0,
                    int32_t M, const double* elem, const double* poses, int32_t F,
                    const ra_sampling* samp, float* s, void* stream);

/* radiate_forward for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, result and
 * errors as radiate_forward, but its scratch (element positions, the forward's voxel tables
 * and, when the forward adds into FP64 sums, those sums) lives in a static device array of
 * RA_STATIC_SCRATCH_BYTES that the library holds on every device it runs on until the process
 * ends; the call never allocates, frees or synchronises, whatever the context's own scratch.
 *   Limit    RA_ENOMEM, with the size needed in ra_last_error(), if the call needs more than
 *            the array: 24*F*M bytes of element positions plus 32 bytes per voxel of a forward
 *            region, plus 8*F*M*K bytes when the forward uses FP64 sums (ra_set_forward_sums;
 *            RA_SUMS_AUTO picks them above 4096 forward regions).
 *   Sharing  the array is one per DEVICE, not per context: every call of this entry point on a
 *            device uses the same memory, and each call rewrites what it needs before reading
 *            it.  Calls that overlap on one device (two streams, two contexts, two host threads)
 *            race and give wrong results; order them. */
#define RA_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
int radiate_forward_static(ra_ctx* ctx, const ra_grid* grid, const float* p0,
                           int32_t M, const double* elem, const double* poses, int32_t F,
                           const ra_sampling* samp, float* s, void* stream);

/* Adjoint of the forward model for a given dL/ds.
 *   r          float[F][M][K]           dL/ds
 *   p0         float[nx][ny][nz]        needed for the pose outputs (may be NULL
 *                                       if grad_pose and grad_elem are NULL)
 *   grad_p0    float[nx][ny][nz] or NULL    dL/dp0 = A^T r (back-projection
 *                                           along spherical shells)
 *   grad_pose  double[F][12] or NULL        (dL/dR row-major, dL/dt) per frame
 *   grad_elem  double[F][M][3] or NULL      dL/dx_e per element and frame
 *   flags      RA_ACCUMULATE adds into the outputs instead of overwriting.
 * The per-element gradient is accumulated in FP64 (terms are formed in FP32).
 */
int radiate_adjoint(ra_ctx* ctx, const ra_grid* grid, const float* p0,
                    int32_t M, const double* elem, const double* poses, int32_t F,
                    const ra_sampling* samp, const float* r,
                    float* grad_p0, double* grad_pose, double* grad_elem,
                    uint32_t flags, void* stream);

/* Reconstruction objective of Stage 1 without regulariser (lambda = 0):
 *   L = sum (s - y)^2,  s = forward(p0, poses),  dL/ds = 2 (s - y),
 * followed by the adjoint into grad_p0 / grad_pose / grad_elem (each may be NULL).
 *   y      float[F][M][K]   measured signals
 *   loss   double* or NULL: L as the FP64 sum, in a fixed order on the device, of per-block
 *          FP32 partial sums.  Without RA_LOSS_ON_DEVICE it is a HOST pointer and the call
 *          waits for the stream; with RA_LOSS_ON_DEVICE it is a DEVICE pointer written on
 *          the stream, and the call never synchronises (every launch of the call is a kernel,
 *          so with scratch reserved beforehand it can be captured into a HIP graph).
 *   s_out  float[F][M][K] or NULL: the forward signals, if wanted.  With RA_SIGNALS_GIVEN it is
 *          required and is an INPUT instead: the signals an earlier call wrote for the same p0,
 *          poses and sampling (read, not modified); the call then skips the forward and takes
 *          the residual, loss and adjoint from them (a sweep whose signals fit in device memory
 *          keeps them from the loss pass instead of recomputing them for the gradients).
 *   flags  RA_ACCUMULATE (gradients), RA_LOSS_ON_DEVICE, RA_SIGNALS_GIVEN.
 */
int loss_and_grad(ra_ctx* ctx, const ra_grid* grid, const float* p0,
                  int32_t M, const double* elem, const double* poses, int32_t F,
                  const ra_sampling* samp, const float* y, double* loss,
                  float* s_out, float* grad_p0, double* grad_pose, double* grad_elem,
                  uint32_t flags, void* stream);

/* Negative-correlation objective of Stage 2 (single-element localisation), summed over
 * elements as in Stage 4's inlier-masked global loss:
 *   L_e = -Cov_k(s_e, y_e) / (sigma_sim sigma_meas)   (statistics over the K samples of the
 *         row of element e = (f, m); zero, with zero gradient, if either row is constant),
 *   L   = sum_e w_e L_e,
 * then the adjoint of the forward model for dL/ds into grad_p0 / grad_pose / grad_elem
 * (each may be NULL; grad_elem feeds per-element localisation, grad_pose the rigid array).
 *   y          float[F][M][K]   measured signals
 *   weight     float[F][M] or NULL (all 1): per-element weights w_e (an inlier mask)
 *   loss       HOST double* or NULL.  Non-NULL: the call waits for the stream and stores L
 *              (per-element FP64 values summed in a fixed order on the device).
 *   loss_elem  double[F][M] or NULL: the unweighted L_e (e.g. to rank candidate positions)
 *   s_out      float[F][M][K] or NULL: the forward signals
 * Row statistics are taken in FP64 over the FP32 signals. */
int nc_loss_and_grad(ra_ctx* ctx, const ra_grid* grid, const float* p0,
                     int32_t M, const double* elem, const double* poses, int32_t F,
                     const ra_sampling* samp, const float* y, const float* weight,
                     double* loss, double* loss_elem, float* s_out,
                     float* grad_p0, double* grad_pose, double* grad_elem,
                     uint32_t flags, void* stream);

/* Second-order TGV regulariser of the Stage 1 / Stage 5 objectives, with its auxiliary vector
 * field w written out (the paper names TGV without stating its discretisation):
 *   TGV(u, w) = alpha1 sum_v |D+u - w|_eps + alpha0 sum_v |E(w)|_eps,
 * D+ the forward-difference gradient in voxel steps (zero at the last index of an axis),
 * E(w)_ab = (D-_a w_b + D-_b w_a)/2 with backward differences (zero at the first index),
 * Frobenius norm, |x|_eps = sqrt(|x|^2 + eps^2) - eps.
 *   u       float[nx][ny][nz]       (z fastest), e.g. p0
 *   w       float[3][nx][ny][nz]    components x, y, z
 *   scale   multiplies the value and the gradients (the weight lambda of the objective)
 *   loss    HOST double* or NULL: scale * TGV (FP64 sum; the call waits for the stream)
 *   grad_u  float[nx][ny][nz] or NULL; grad_w float[3][nx][ny][nz] or NULL
 *   flags   RA_ACCUMULATE adds scale * gradient into grad_u / grad_w
 * One pass: each voxel re-evaluates its neighbours' normalised fields from u and w, so HBM
 * sees only the inputs read and the gradients written.
 * Scratch: ra_tgv_scratch_bytes(nx, ny, nz) (one FP64 partial of the value per 64 x 4 voxels of
 * a plane), taken as in the other calls.
 * Errors: RA_EINVAL for non-positive dimensions, missing u or w, alpha < 0, eps < 1e-18 (eps^2
 * must be a normal FP32 number). */
size_t ra_tgv_scratch_bytes(int32_t nx, int32_t ny, int32_t nz);
int tgv_loss_and_grad(ra_ctx* ctx, int32_t nx, int32_t ny, int32_t nz, const float* u, const float* w,
                      double alpha0, double alpha1, double eps, double scale, double* loss,
                      float* grad_u, float* grad_w, uint32_t flags, void* stream);

/* Axis-angle poses: pose6 double[F][6] = (w, t) with R = exp([w]x).
 * ra_pose_from_axis_angle writes poses double[F][12]; ra_pose_grad_axis_angle maps
 * grad_pose double[F][12] (dL/dR, dL/dt) to grad6 double[F][6] (dL/dw, dL/dt). */
int ra_pose_from_axis_angle(ra_ctx* ctx, const double* pose6, int32_t F, double* poses,
                            void* stream);
int ra_pose_grad_axis_angle(ra_ctx* ctx, const double* pose6, const double* grad_pose,
                            int32_t F, double* grad6, void* stream);

/* Euler-angle poses of Stage 4's rigid-array optimiser: pose6 double[F][6] = (a, t) with
 * R = Rz(a2) Ry(a1) Rx(a0) (rotations about the fixed x, then y, then z axes; the paper does
 * not state its convention).  Same layouts and errors as the axis-angle pair above. */
int ra_pose_from_euler(ra_ctx* ctx, const double* pose6, int32_t F, double* poses, void* stream);
int ra_pose_grad_euler(ra_ctx* ctx, const double* pose6, const double* grad_pose,
                       int32_t F, double* grad6, void* stream);

/* Exact number of in-window (voxel, element, sample) triples of this geometry,
 * decided in FP64 (|d - c*(k/fs)| <= trunc*sigma).  Waits for the stream; writes the
 * HOST int64 *count.  Used to price throughput; not part of the model evaluation. */
int ra_count_updates(ra_ctx* ctx, const ra_grid* grid, int32_t M, const double* elem,
                     const double* poses, int32_t F, const ra_sampling* samp,
                     long long* count, void* stream);

/* Calibration for roofline figures (not part of the model): times, with HIP events on `stream`,
 * kernels in which every thread runs 8 independent chains of FP32 FMAs, then of v_exp_f32
 * (4096 workgroups of 256 threads), and writes the measured lane-operation rates to the HOST
 * doubles *fma_per_s (FMAs/s; FLOP/s = 2x) and *exp_per_s (exponentials/s).  Waits for the
 * stream; uses the context's scratch (a 4 MiB output buffer). */
int ra_probe_rates(ra_ctx* ctx, double* fma_per_s, double* exp_per_s, void* stream);

/* ------------------------------------------------------------------------------------------
 * Batched steps for serving.  One call of ra_batch_step performs one gradient step for
 * every request of a batch; requests differ in element count M, sample count K and box of
 * a resident volume, and share spacing, sampling and region size.  All tables live in
 * device memory and every kernel walks its work list with a fixed grid, so a caller may
 * capture ra_batch_step into a HIP graph once and replay it for any batch that fits the
 * capacities of the tables.  The call allocates nothing and never synchronises.
 * ------------------------------------------------------------------------------------------ */
enum { RA_REQ_POSE = 0, RA_REQ_VOLUME = 1 };
#define RA_BATCH_APPLY_UPDATES 1u  /* volume requests add -lr * dL/dp0 into the resident volume */

/* One request of a batch (all pointers are device pointers).
 * Pose refinement (RA_REQ_POSE): forward model of one frame at pose6, residual against y,
 *   element-coordinate adjoint (FP64 reduction), chain to dL/dw, dL/dt, one Adam step on
 *   pose6 (steps lr_w [rad], lr_t [m]; beta1 0.9, beta2 0.999).
 * Volume update (RA_REQ_VOLUME): forward, residual, dL/dp0 of the box into grad_p0; with
 *   RA_BATCH_APPLY_UPDATES the box of the resident volume moves by -lr_w * dL/dp0. */
typedef struct {
    float* p0;              /* first voxel of the request's box inside the resident volume    */
    float* s;               /* float[M][K] scratch: forward signals, then dL/ds               */
    const float* y;         /* float[M][K] measured signals of the frame                      */
    float* grad_p0;         /* float[bx][by][bz] dL/dp0 of the box (volume requests)          */
    double* pose_part;      /* double[nreg][M][3] scratch (pose requests)                     */
    double* pose6;          /* double[6] (w, t); pose requests update it in place              */
    double* adam;           /* double[13] Adam state m[6], v[6], step count (pose requests)    */
    const double* elem;     /* double[M][3] array template                                    */
    float* xe;              /* float[M][6] scratch                                             */
    float* loss;            /* float[1]: sum (s - y)^2 at the start of the step               */
    float* q;               /* ra_batch_info.q_bytes scratch: moment table of dL/ds (batches
                               with ra_batch.moment; unused otherwise)                        */
    int32_t kind;           /* RA_REQ_POSE or RA_REQ_VOLUME                                   */
    int32_t nreg;           /* regions of the box (ra_batch_info.nreg)                        */
    double lr_w;            /* pose: Adam step on w; volume: step size on p0                  */
    double lr_t;            /* pose: Adam step on t                                           */
} ra_batch_request;

/* What ra_batch_describe reports about a request's geometry. */
typedef struct {
    int32_t nreg;           /* regions of the box: the request's work items are 0..nreg-1    */
    int32_t jt, exact;      /* window code: equal for requests that may share a batch        */
    int32_t pair_d;         /* forward pairs z-neighbour voxels with this spread (0: no):
                               equal for requests that may share a batch                     */
    int32_t lmax;           /* LDS sample rows needed                                         */
    int32_t nvpad;          /* voxels per region (padded)                                     */
    int32_t rx, ry, rz;     /* region size                                                    */
    int32_t moment;         /* 1: the batch may take the moment form of the adjoints (the
                               Gaussian's window sums from 8 Taylor moments of dL/ds per
                               sample, as the single calls do); equal for requests that may
                               share a batch                                                  */
    int32_t nbin;           /* centre samples per region and element (moment form)           */
    int64_t q_bytes;        /* bytes of the request's moment table (0 without the form)      */
} ra_batch_info;

/* The device tables of one batch.  Work lists are int32 pairs; counts holds
 * {n_fwd, n_pose, n_vol, n_elem, n_slots}.  items_fwd lists (slot, region) of every request,
 * items_pose / items_vol those of pose / volume requests, items_elem (slot, element). */
typedef struct {
    const void* geos;             /* n_slots descriptors of ra_batch_geo_bytes() each        */
    const ra_batch_request* reqs; /* n_slots requests                                       */
    const void* vtab;             /* voxel tables from ra_batch_tables                      */
    const void* itab;
    const int32_t* items_fwd;
    const int32_t* items_pose;
    const int32_t* items_vol;
    const int32_t* items_elem;
    const int32_t* counts;
    int32_t jt, exact;            /* from ra_batch_describe (equal for all requests)        */
    int32_t pair_d;               /* from ra_batch_describe (equal for all requests)        */
    int32_t lmax, nvpad;          /* maxima over the batch                                  */
    int32_t grid_blocks;          /* workgroups per launch; 0 = 1024                        */
    int32_t moment;               /* 1: adjoints in moment form (every request has ra_batch_info
                                     .moment set and a q buffer); 0: row form.  RA_EINVAL
                                     for the moment form without coef, without the exact
                                     window, or with nbin outside 1..40 or beyond the LDS  */
    int32_t nbin;                 /* ra_batch_info.nbin (moment form; equal for all requests:
                                     a request whose window needs more bins is skipped)     */
    float* coef;                  /* moment form: float[8 (2 jt + 1)] device scratch (jt <= 40,
                                     so 648 floats always suffice)                          */
} ra_batch;

/* Size of one request descriptor. */
size_t ra_batch_geo_bytes(void);

/* Describe a request whose box is the grid `box` (origin = centre of its first voxel)
 * inside a resident volume with element strides stride_x, stride_y (z contiguous), with M
 * elements and sampling `samp`; writes the descriptor to HOST memory `geo`
 * (ra_batch_geo_bytes() bytes) and fills *info.  Host-only; no device work.  RA_ENOTSUP for
 * a source profile other than the Gaussian. */
int ra_batch_describe(ra_ctx* ctx, const ra_grid* box, int64_t stride_x, int64_t stride_y, int32_t M,
                      const ra_sampling* samp, void* geo, ra_batch_info* info);

/* Fill the voxel tables (device buffers of info.nvpad * 16 bytes each) shared by all
 * requests with the same spacing, region size and volume strides. */
int ra_batch_tables(ra_ctx* ctx, const void* geo, void* vtab, void* itab, void* stream);

/* One gradient step for every request of the batch.  flags: RA_BATCH_APPLY_UPDATES. */
int ra_batch_step(ra_ctx* ctx, const ra_batch* batch, uint32_t flags, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PASFM_RADIATE_H */

/*
 * radiate.h -- C ABI of the MI355X (gfx950) differentiable acoustic radiation library.
 *
 * The library evaluates the far-field Gaussian-kernel radiation model of PA-SFM
 * (Li, Gao et al., arxiv 2604.09643) and its adjoints:
 *
 *   s[f,m,k] = sum_v p0[v] * phi(d - c t_k) / (2 d),   d = |x_v - x_e(f,m)|,
 *   phi(u)   = u * exp(-u^2 / (2 sigma^2)),            t_k = k / fs,
 *
 * keeping only the terms with |d - c t_k| <= trunc * sigma.  Main text Eq. (1)
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
 *             synchronise the host, except loss_and_grad with a non-NULL
 *             `loss` and ra_count_updates, which wait for their own result.
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
#define RA_ACCUMULATE 1u /* add into grad_p0 / grad_pose / grad_elem instead of overwriting */

typedef struct ra_ctx ra_ctx;

/* Voxel grid: voxel (i,j,k) centre = origin + (i,j,k)*spacing [m]; volume float[nx][ny][nz]. */
typedef struct {
    int32_t nx, ny, nz;
    double origin[3];
    double spacing;
} ra_grid;

/* Sampling: t_k = k/fs for k = 0..K-1; kernel width sigma [m]; a term is kept iff
 * |d - c t_k| <= trunc*sigma (trunc = 6 in the paper's setting).  Requires
 * trunc*sigma >= c/(2 fs) and trunc*sigma <= 40 c/fs (RA_EINVAL otherwise). */
typedef struct {
    double c;      /* speed of sound [m/s]        */
    double fs;     /* sampling rate [Hz]          */
    int32_t K;     /* samples per element         */
    double sigma;  /* Gaussian kernel width [m]   */
    double trunc;  /* window half-width in sigmas */
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
 * what a call with the given sizes needs. */
int ra_reserve(ra_ctx* ctx, size_t bytes);
size_t ra_scratch_bytes(const ra_grid* grid, int32_t M, int32_t F, const ra_sampling* samp);

/* Forward model (Eq. (1) with the kernel of Eq. (A13)).
 *   p0     float[nx][ny][nz]            initial pressure per voxel
 *   elem   double[M][3]                 array template, probe frame
 *   poses  double[F][12]                rigid pose per frame (R row-major, t)
 *   s      float[F][M][K]  (output)     overwritten */
int radiate_forward(ra_ctx* ctx, const ra_grid* grid, const float* p0,
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
 *   loss   HOST double* or NULL.  Non-NULL: the call waits for the stream and
 *          stores L (per-block FP32 partial sums added in FP64 on the host).
 *   s_out  float[F][M][K] or NULL: the forward signals, if wanted.
 */
int loss_and_grad(ra_ctx* ctx, const ra_grid* grid, const float* p0,
                  int32_t M, const double* elem, const double* poses, int32_t F,
                  const ra_sampling* samp, const float* y, double* loss,
                  float* s_out, float* grad_p0, double* grad_pose, double* grad_elem,
                  uint32_t flags, void* stream);

/* Axis-angle poses: pose6 double[F][6] = (w, t) with R = exp([w]x).
 * ra_pose_from_axis_angle writes poses double[F][12]; ra_pose_grad_axis_angle maps
 * grad_pose double[F][12] (dL/dR, dL/dt) to grad6 double[F][6] (dL/dw, dL/dt). */
int ra_pose_from_axis_angle(ra_ctx* ctx, const double* pose6, int32_t F, double* poses,
                            void* stream);
int ra_pose_grad_axis_angle(ra_ctx* ctx, const double* pose6, const double* grad_pose,
                            int32_t F, double* grad6, void* stream);

/* Exact number of in-window (voxel, element, sample) triples of this geometry,
 * decided in FP64 (|d - c*(k/fs)| <= trunc*sigma).  Waits for the stream; writes the
 * HOST int64 *count.  Used to price throughput; not part of the model evaluation. */
int ra_count_updates(ra_ctx* ctx, const ra_grid* grid, int32_t M, const double* elem,
                     const double* poses, int32_t F, const ra_sampling* samp,
                     long long* count, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PASFM_RADIATE_H */

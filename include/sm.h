/*
 * sm.h -- C ABI of the exact cone-beam system-matrix library (MI355X, HIP).
 *
 * The library applies the system matrix W of Simbrunner, Krenn, Zach and
 * Habring, "Computation of a Consistent System Matrix for Cone-beam Computed
 * Tomography" (arXiv 2511.12235), without storing it.  W maps a voxel image u
 * to the measurements p = W u (Sec. I, eq. "ip"); its entry W_ij is the exact
 * measure (area in 2D, volume in 3D, in absolute units mm^2 / mm^3) of the
 * part of voxel j inside the beam of detector element i, so that W u equals
 * the beam-integrated attenuation of a piecewise-constant object exactly (the
 * "consistency" definition of Sec. I).
 *
 * Geometry (Sec. III-A, eq. "z rotation"; appendix "Fundamental relations"):
 * the source sits at (s cos(phi), s sin(phi), 0) and rotates about +z; the
 * flat detector is perpendicular to the central ray at distance d beyond the
 * origin (source-detector distance D = s + d).  A point p has depth
 * l = s - (x cos(phi) + y sin(phi)) and detector coordinates u = D t / l,
 * v = D z / l with t = y cos(phi) - x sin(phi).  Detector column m_y spans
 * [det_y0 + m_y dy, det_y0 + (m_y + 1) dy] in u, row m_z spans
 * [det_z0 + m_z dz, det_z0 + (m_z + 1) dz] in v.  Voxel (ix, iy, iz) spans
 * [x0 + ix a, x0 + (ix + 1) a] x [y0 + iy b, ...] x [z0 + iz c, ...].
 *
 * Conventions shared by every entry point:
 *  - Layouts (C order, last index fastest):
 *      volume    x[B][nz][ny][nx]            (voxel j = (iz ny + iy) nx + ix)
 *      sinogram  y[B][n_p][det_nz][det_ny]   (ray i = (view det_nz + m_z) det_ny + m_y)
 *    In 2D nz = det_nz = 1.  The element type is float for SM_FP32 plans and
 *    double for SM_FP64 plans.
 *  - Device pointers are HIP device memory owned by the caller.  Host
 *    pointers are named *_host.  The plan owns only its own tables.
 *  - Every call returns an sm_status and never throws or aborts.  On a
 *    non-OK status the outputs are unspecified and sm_last_error() holds a
 *    message (thread-local).
 *  - sm_forward / sm_back are stream-ordered on the given hipStream_t (NULL =
 *    the default stream); they never allocate, never synchronise and overwrite
 *    their output (no zero-initialisation needed).  A plan is immutable after
 *    creation, except through sm_plan_keep_records and sm_timing_enable, and
 *    may be used concurrently from several host threads and streams, provided
 *    each concurrent call has its own workspace.
 */
#ifndef SM_H
#define SM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SM_OK = 0,
    SM_EINVAL = 1,       /* bad argument or geometry */
    SM_ENOMEM = 2,       /* device or host allocation failed */
    SM_EDEVICE = 3,      /* HIP runtime error (launch, copy) */
    SM_EUNSUPPORTED = 4, /* valid request outside the implemented envelope */
    SM_ERANGE = 5        /* caller buffer too small (see sm_weights_csr) */
} sm_status;

typedef enum { SM_FP32 = 0, SM_FP64 = 1 } sm_precision;

/* Scanner and grid description (plain data, copied by sm_plan_create).
 * NaN in x0/y0/z0 selects the grid centred on the rotation axis
 * (x0 = -nx a / 2, ...); NaN in det_y0/det_z0 selects the centred detector
 * (det_y0 = -det_ny dy / 2, ...).  phi == NULL selects phi_k = 2 pi k / n_p
 * (equidistant in [0, 2 pi), Sec. IV).  trig, when non-NULL, supplies the
 * exact (cos(phi_k), sin(phi_k)) pairs and takes precedence over phi. */
typedef struct {
    int32_t dim;              /* 2 (fan beam) or 3 (cone beam) */
    int32_t nx, ny, nz;       /* voxels per axis; nz == 1 in 2D */
    double a, b, c;           /* voxel side lengths; c ignored in 2D */
    double x0, y0, z0;        /* grid minimum corner (NaN = centred) */
    int32_t n_p;              /* number of projection angles */
    int32_t reserved0;        /* must be 0 */
    const double *phi;        /* host array of n_p angles (radians) or NULL */
    const double *trig;       /* host array of n_p (cos, sin) pairs or NULL */
    double s;                 /* source-to-origin distance, s > 0 */
    double d;                 /* origin-to-detector distance, s + d > 0 */
    int32_t det_ny, det_nz;   /* detector columns (u) and rows (v); det_nz == 1 in 2D */
    double dy, dz;            /* detector element side lengths; dz ignored in 2D */
    double det_y0, det_z0;    /* first detector corner (NaN = centred) */
} sm_geometry;

typedef struct sm_plan sm_plan;

/* Validate the geometry and build the per-view tables on the current HIP
 * device (Sec. III-A).  Rejects (SM_EINVAL) non-positive sizes or pitches,
 * dim not in {2, 3}, non-finite values, and any view in which a grid corner
 * has depth l <= 0 (source inside or behind the grid).  Returns
 * SM_EUNSUPPORTED in 3D for det_nz > 1024 or nz > 1024, and when a
 * workgroup's LDS staging would exceed 64 KiB: FP64 plans above about 830
 * detector rows, or a voxel footprint too wide for the adjoint's tile.  The
 * plan must be destroyed with sm_plan_destroy on the same device. */
sm_status sm_plan_create(const sm_geometry *g, sm_precision precision, sm_plan **out);

/* Release the plan and its device tables.  NULL is accepted. */
sm_status sm_plan_destroy(sm_plan *plan);

/* Problem sizes: number of voxels N and number of measurements M = N_d N_p
 * (Sec. I).  Either output pointer may be NULL. */
sm_status sm_plan_sizes(const sm_plan *plan, int64_t *n_vox, int64_t *n_rays);

/* Bytes of the strip records of every view (the top-view polygons of
 * Sec. III-B with their chord tables, built per chunk of views by every 3D
 * sm_forward / sm_back call); 0 in 2D. */
sm_status sm_plan_record_bytes(const sm_plan *plan, int64_t *bytes);

/* Keep the strip records of every view in a plan-owned device buffer, so
 * that sm_forward and sm_back (and the solvers built on them) stop
 * rebuilding them on every call.  The records depend on the geometry only;
 * results are bitwise the same with and without the buffer.  Builds the
 * buffer (sm_plan_record_bytes bytes, allocated on the plan's device) if that
 * is at most max_bytes, else returns SM_ERANGE and changes nothing;
 * max_bytes = 0 releases it.  Either way synchronises `hip_stream` (and, on
 * release, the device).  While the buffer is held, sm_workspace_size leaves
 * out the records.  This call changes the plan: it must not run concurrently
 * with any other call on the plan.  No-op in 2D. */
sm_status sm_plan_keep_records(sm_plan *plan, int64_t max_bytes, void *hip_stream);

/* Launch shape of the 3D operators, fixed at plan creation from the geometry
 * alone: sm_forward and sm_back process the views in chunks of
 * *views_per_chunk consecutive views (the last chunk may be shorter; the
 * strip records of one chunk share the workspace), and the adjoint splits
 * every chunk of n views into *adjoint_runs runs, run g holding views
 * [n g / runs, n (g + 1) / runs) of the chunk, each summed into its own
 * partial volume before the partials are added in order.  In 2D both are
 * reported as (n_p, 1).  Either output pointer may be NULL. */
sm_status sm_plan_launch_shape(const sm_plan *plan, int32_t *views_per_chunk, int32_t *adjoint_runs);

/* Device workspace bytes that sm_forward / sm_back need for `batch` volumes
 * (0 in 2D).  In 3D it holds the strip records of one chunk of views (the
 * top-view polygons of Sec. III-B with their chord tables, at most 4 GiB)
 * and one FP64 column buffer and one word per batch element. */
sm_status sm_workspace_size(const sm_plan *plan, int32_t batch, int64_t *bytes);

/* Forward projection y = W x (Sec. III-B Algorithm 1 for 2D; Sec. III-C for
 * 3D), for `batch` volumes of the plan's geometry: x[batch][nz][ny][nx] in,
 * y[batch][n_p][det_nz][det_ny] out (overwritten).  ws is a device workspace
 * of at least sm_workspace_size(batch) bytes (may be NULL when that is 0);
 * ws_bytes is its size.
 * Weights are recomputed on the fly; each is evaluated once per call and
 * applied to every batch element.  Accuracy (SM_FP32 plans): the few volume
 * terms of voxel faces that a detector row plane cuts are rounded to a
 * fixed-point grid tied to max|x| of each volume and summed exactly; the grid
 * rules out overflow and adds an absolute error per measurement of order
 * 2^-60 R^2 a b c max|x|, R the voxel columns a detector column's beam meets
 * (about 2^-36 a b c max|x| at 256^3), far below FP32 rounding.  A non-finite
 * value in a volume makes its measurements NaN. */
sm_status sm_forward(const sm_plan *plan, const void *x, void *y, int32_t batch, void *ws,
                     int64_t ws_bytes, void *hip_stream);

/* Adjoint (back projection) x = W^T y with the same weights as sm_forward
 * (the matched pair whose adjoint mismatch Sec. IV reports).  Layouts and
 * workspace rules as sm_forward; x is overwritten. */
sm_status sm_back(const sm_plan *plan, const void *y, void *x, int32_t batch, void *ws,
                  int64_t ws_bytes, void *hip_stream);

/* sm_forward (adjoint == 0) or sm_back (adjoint == 1) without a workspace,
 * for callers that cannot allocate device memory: code under HIP stream
 * capture, serving loops and hosts that forbid hipMalloc.  Same plan, layouts,
 * stream, overwrite and precision rules as those entry points; calls no
 * allocator.  The workspace lives in a static device array of
 * SM_NOALLOC_SCRATCH_BYTES per device, which the library holds from the
 * first call on a device until the process ends.  It must hold the volume
 * buffers of the call (3D forward: FP64 prefix sums, (nz + 1) nx ny batch
 * doubles; 3D adjoint: nz nx ny batch elements per view run) plus, unless the
 * plan keeps its records (sm_plan_keep_records), the strip records of at
 * least one view; otherwise SM_ERANGE, with the sizes in sm_last_error().
 * Records are rebuilt in chunks of as many views as fit (the adjoint may also
 * sum fewer view runs), so adjoint results can differ from sm_back's in the
 * rounding order of their sums only; forward results are bitwise sm_forward's.
 * 2D plans need no scratch.  Calls on one device share the array: calls that
 * overlap in time on one device (several streams or host threads) race and
 * must be serialised by the caller.  SM_EINVAL for adjoint not in {0, 1} and
 * the argument errors of sm_forward. */
#define SM_NOALLOC_SCRATCH_BYTES ((int64_t)128 << 20)
sm_status sm_apply_noalloc(const sm_plan *plan, int32_t adjoint, const void *in, void *out,
                           int32_t batch, void *hip_stream);

/* The explicit matrix W in CSR form (Sec. I: W in R^{M x N}) for small
 * problems, written to host arrays.  Entries with W_ij <= tau_keep =
 * 1e-12 * (voxel measure) are treated as exact zeros; the pattern is decided
 * in FP64 whatever the value precision.  Rows are ordered by measurement
 * index, columns ascending within a row.
 * Two-call protocol: with row_ptr_host == NULL only *nnz_inout is written
 * (the number of entries).  Otherwise row_ptr_host must hold M + 1 int64,
 * col_idx_host and val_host (float for SM_FP32 values, double for SM_FP64)
 * *nnz_inout entries; SM_ERANGE is returned when *nnz_inout is too small.
 * The counting call works at any size (it is how the number of nonzero
 * voxel-detector pairs is obtained); filling is limited to 4e8 entries and
 * 2^31 - 1 voxels (SM_EUNSUPPORTED beyond).  Synchronises the current device. */
sm_status sm_weights_csr(const sm_plan *plan, sm_precision values, int64_t *nnz_inout,
                         int64_t *row_ptr_host, int32_t *col_idx_host, void *val_host);

/* ------------------------------------------------------------------------
 * Stored-W mode: W (Sec. I, W in R^{M x N}) or its transpose as device CSR
 * arrays, for problems whose matrix fits in device memory (up to 2^31 - 1
 * entries, voxels and detector elements), applied by a sparse matrix-vector
 * product.  Same pattern rule and value precision choice as
 * sm_weights_csr.  transposed = 0: rows are detector elements
 * (i = (view det_nz + m_z) det_ny + m_y), columns voxels; transposed = 1:
 * rows are voxels, columns detector elements.  Columns ascend within a row.
 * ------------------------------------------------------------------------ */

/* Number of entries of W (or W^T, the same number).  Allocates and frees
 * temporary device buffers and synchronises the current device. */
sm_status sm_stored_count(const sm_plan *plan, int32_t transposed, int64_t *nnz);

/* Fill caller-allocated device arrays: row_ptr (rows + 1 int64), col_idx (nnz
 * int32) and val (nnz float or double, as `values`).  nnz must be the count
 * of sm_stored_count (SM_ERANGE otherwise).  A set-up routine: it allocates
 * and frees temporary device buffers (about 8-12 bytes per entry) and
 * synchronises `hip_stream`. */
sm_status sm_stored_fill(const sm_plan *plan, int32_t transposed, sm_precision values, int64_t nnz,
                         int64_t *row_ptr, int32_t *col_idx, void *val, void *hip_stream);

/* y = A x for a CSR matrix A with n_rows rows (device arrays as filled by
 * sm_stored_fill), `batch` vectors: x + b x_stride and y + b y_stride
 * (elements).  y is overwritten; each row is summed in a fixed order (one
 * wavefront per row), so results are deterministic.  Stream-ordered on
 * hip_stream; does not allocate or synchronise. */
sm_status sm_stored_apply(int64_t n_rows, const int64_t *row_ptr, const int32_t *col_idx,
                          const void *val, sm_precision values, const void *x, void *y,
                          int32_t batch, int64_t x_stride, int64_t y_stride, void *hip_stream);

/* Line-based comparison model (Sec. IV: the line-based system matrix the
 * paper compares against, and its complexity experiment, which averages k
 * lines per detector element to approach the area-based matrix).  Detector
 * element (m_y, m_z) is sampled by the k (2D) or k x k (3D) lines from the
 * source through the detector points
 *     u = det_y0 + (m_y + (s + 1/2) / k) dy,  v = det_z0 + (m_z + (t + 1/2) / k) dz.
 * With the line's points alpha (D, u, v) in the view frame of Sec. III-A
 * (alpha >= 0, alpha = 1 on the detector), voxel j holds the piece
 * alpha in [alpha_in, alpha_out] of the line inside its closed box; on an axis
 * the line runs parallel to, the voxel whose half-open slab [lo, hi) holds
 * the source keeps the line.  Weight of voxel j for the element, summed over
 * its sub-lines:
 *   SM_LINE_LENGTH : R (alpha_out - alpha_in) / k^(dim-1), R = |(D, u, v)|
 *                    (the mean path length: the classical line model);
 *   SM_LINE_MEASURE: dy D (alpha_out^2 - alpha_in^2) / (2k) in 2D,
 *                    dy dz D (alpha_out^3 - alpha_in^3) / (3k^2) in 3D (the
 *                    midpoint rule over the element of its exact area/volume,
 *                    which tends to W of sm_forward as k grows). */
typedef enum { SM_LINE_LENGTH = 0, SM_LINE_MEASURE = 1 } sm_line_weight;
#define SM_LINE_MAX_K 64

/* y = W_line x for `batch` volumes, layouts and stream as sm_forward; needs
 * no workspace and allocates nothing.  1 <= k <= SM_LINE_MAX_K.  Geometry in
 * FP64, sums in FP64, x and y in the plan's precision.  SM_EINVAL for a bad
 * k, weighting, batch or pointer. */
sm_status sm_line_forward(const sm_plan *plan, int32_t k, sm_line_weight weight, const void *x,
                          void *y, int32_t batch, void *hip_stream);

/* x = W_line^T y, the exact transpose of sm_line_forward's matrix (every
 * piece is computed with the same expressions in both directions); same
 * arguments and errors. */
sm_status sm_line_back(const sm_plan *plan, int32_t k, sm_line_weight weight, const void *y,
                       void *x, int32_t batch, void *hip_stream);

/* Footprint boxes of every voxel in one view (eq. "relevant detectors 2d"
 * and the row bounds of Sec. III-C, with strict inequalities): for voxel j,
 * boxes_host[4 j + 0..3] = first column, last column, first row, last row of
 * the detector elements whose open cell meets the open detector-coordinate
 * range of the voxel (first > last when empty).  The box is computed in FP64
 * from the corners with the fixed operation order l = s - (x cos + y sin),
 * t = y cos - x sin, u = (D t) / l, v = (D z) / l (no fused multiply-add),
 * x = x0 + ix a etc., and cell edges det_y0 + m dy.  Host output of
 * nx*ny*nz*4 int32.  Synchronises the current device. */
sm_status sm_footprints(const sm_plan *plan, int32_t view, int32_t *boxes_host);

/* ------------------------------------------------------------------------
 * Reconstruction (Sec. IV, eq. "exp_tikh"): minimise
 *     F(u) = 1/2 || s W u - p ||^2 + lambda/2 || u ||^2
 * where s = wscale (the paper divides W by its spectral norm, s = 1/||W||_2,
 * estimated with 100 power iterations).  All three routines are
 * stream-ordered on hip_stream, never allocate and never synchronise: every
 * scalar of the iteration (step sizes, norms) stays in device memory, dot
 * products are accumulated in FP64 in a fixed order (results are
 * deterministic), and vectors are in the plan's precision.  They run a fixed
 * number of iterations; a caller wanting the paper's stopping rule reads the
 * recorded gradient norms.  ws must hold sm_solver_workspace_size() bytes and
 * must not be shared with concurrent calls.
 * ------------------------------------------------------------------------ */
typedef enum {
    SM_SOLVER_CGLS = 0,  /* sm_cgls */
    SM_SOLVER_NAG = 1,   /* sm_nag */
    SM_SOLVER_POWER = 2  /* sm_power_norm (batch must be 1) */
} sm_solver;

/* Device workspace bytes for one call of the given solver with `batch`
 * independent right-hand sides (the projector workspace included). */
sm_status sm_solver_workspace_size(const sm_plan *plan, sm_solver solver, int32_t batch,
                                   int64_t *bytes);

/* Spectral norm ||W||_2 by power iteration on W^T W (Sec. IV): v = v0/|v0|;
 * repeat iters times { u = W v; sigma2 = |u|^2; w = W^T u; v = w/|w| };
 * *norm_dev = sqrt(sigma2) of the last iteration (a Rayleigh quotient, so it
 * approaches the norm from below).  v0: device volume [nz][ny][nx] (the
 * random start; the caller draws it), not modified.  norm_dev: device
 * pointer to one double.  iters >= 1. */
sm_status sm_power_norm(const sm_plan *plan, const void *v0, int32_t iters, double *norm_dev,
                        void *ws, int64_t ws_bytes, void *hip_stream);

/* CGLS (conjugate gradients on the normal equations (s^2 W^T W + lambda I)
 * u = s W^T p) for `batch` independent problems.  y: device sinograms
 * [batch][n_p][det_nz][det_ny]; x: device volumes [batch][nz][ny][nx], the
 * start on entry and the iterate after `iters` steps on return.  hist_dev:
 * NULL, or device doubles [iters + 1][batch] receiving the squared norm of
 * the normal-equation residual (= |grad F|^2) before each step and after the
 * last.  lambda >= 0, wscale > 0, iters >= 0. */
sm_status sm_cgls(const sm_plan *plan, const void *y, void *x, int32_t batch, int32_t iters,
                  double lambda, double wscale, double *hist_dev, void *ws, int64_t ws_bytes,
                  void *hip_stream);

/* Nesterov's accelerated gradient (Sec. IV) with the FISTA momentum
 * t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 and step 1/L, L = wscale^2 norm^2 +
 * lambda, where norm is read from device memory (norm_dev, e.g. written by
 * sm_power_norm).  x: start on entry, u_iters on return.  hist_dev: NULL or
 * device doubles [iters][batch] receiving |grad F(z_k)|^2 at each
 * extrapolated point.  lambda >= 0, wscale > 0, iters >= 0. */
sm_status sm_nag(const sm_plan *plan, const void *y, void *x, int32_t batch, int32_t iters,
                 double lambda, double wscale, const double *norm_dev, double *hist_dev,
                 void *ws, int64_t ws_bytes, void *hip_stream);

/* sm_power_norm and sm_nag with the line-based operators of sm_line_forward /
 * sm_line_back (k lines per element, weighting) in place of W: the solver of
 * the line-based reconstructions the paper compares against (Sec. IV).  Same
 * arguments, workspace (sm_solver_workspace_size of the same kind) and
 * errors, plus SM_EINVAL for k outside [1, SM_LINE_MAX_K] or a bad weighting. */
sm_status sm_line_power_norm(const sm_plan *plan, int32_t k, sm_line_weight weight, const void *v0,
                             int32_t iters, double *norm_dev, void *ws, int64_t ws_bytes,
                             void *hip_stream);
sm_status sm_line_nag(const sm_plan *plan, int32_t k, sm_line_weight weight, const void *y, void *x,
                      int32_t batch, int32_t iters, double lambda, double wscale,
                      const double *norm_dev, double *hist_dev, void *ws, int64_t ws_bytes,
                      void *hip_stream);

/* Per-kernel timing, for measurement only (not part of the method).  While
 * timing is enabled on a plan, sm_forward and sm_back record a pair of HIP
 * events on their stream around every dispatch of the kernels below and add
 * nothing else (no synchronisation).  One dispatch covers up to 8 batch
 * elements; the 2D kernels count as SM_KERNEL_FORWARD / SM_KERNEL_ADJOINT. */
typedef enum {
    SM_KERNEL_RECORDS = 0,   /* strip polygons and chord tables (Sec. III-B) */
    SM_KERNEL_FORWARD = 1,   /* y = W x accumulation (Sec. III-C) */
    SM_KERNEL_ADJOINT = 2,   /* x = W^T y accumulation */
    SM_KERNEL_PREFIX = 3,    /* the forward's input pass: voxel columns (and max|x|) */
    SM_KERNEL_TRANSPOSE = 4, /* adjoint output to the caller's layout */
    SM_KERNEL_COUNT = 5
} sm_kernel;

typedef struct {
    int64_t launches; /* dispatches timed since the last read */
    double ms;        /* their summed event-to-event durations, milliseconds */
} sm_kernel_time;

/* Enable (enable != 0) or disable per-kernel timing on a plan.  Enabling
 * creates a pool of 8192 events on the plan's device and clears previous
 * records; disabling releases it.  While enabled, calls on this plan must not
 * overlap in time from several host threads.  Must not be toggled while
 * timed work is still in flight on some stream. */
sm_status sm_timing_enable(sm_plan *plan, int32_t enable);

/* Wait for the recorded events (host blocks until they have completed),
 * write SM_KERNEL_COUNT entries to times_host indexed by sm_kernel, and
 * clear the records.  Returns SM_EINVAL when timing is not enabled and
 * SM_ERANGE (times still written) when more dispatches were made than the
 * pool could time; the untimed ones are not counted. */
sm_status sm_timing_read(sm_plan *plan, sm_kernel_time *times_host);

/* Static text for a status code. */
const char *sm_status_str(sm_status status);

/* Message describing the last non-OK status returned on this host thread. */
const char *sm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SM_H */

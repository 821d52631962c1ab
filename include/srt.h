/*
 * srt.h -- C ABI of the MI355X library for the discrete spherical Radon
 * transform (SRT) on a cylindrical aperture.
 *
 * The SRT maps a volume f to its integrals over spheres of radius l centred
 * at sensors r (surface measure; Sec. 2 of Lozenski et al., "An Efficient
 * Implementation of the Spherical Radon Transform with Cylindrical
 * Apertures"). For sensors arranged in columns parallel to z on a cylinder,
 * Sec. 2 writes it as two circular Radon transforms (CRTs): a circle
 * transform in every z-slice about the column centre, then a half-circle
 * transform in the (z, rho) half-plane about each sensor height. Sec. 3.1
 * discretises both on a piecewise-constant voxel basis as sparse matrices
 * A12 (one per column) and A34 (shared by all columns); Alg. 1 is the
 * forward, Alg. 2 the matched adjoint built from their transposes.
 *
 * Conventions shared by every entry point
 *   - Volumes are [batch][mz][ms][ms] (z, y, x; x fastest).
 *   - Sensor data are [batch][n_angles][n_z][n_radii] (radius fastest).
 *   - Column a sits at (R cos angles[a], R sin angles[a]); the cylinder axis is
 *     the z axis x = y = 0.
 *   - Voxel (i, j, k) covers [x0 + i dxy, x0 + (i+1) dxy] x [x0 + j dxy, ...]
 *     x [z0 + k dz, z0 + (k+1) dz].
 *   - The rho axis of the intermediate image reuses the radii: cell l spans
 *     the midpoints between neighbouring radii (outer edges half a spacing
 *     beyond the end radii), unless srt_plan_desc gives it a grid of its own.
 *   - Weights are exact integrals of the basis functions along the arcs,
 *     computed in FP64 on the device and rounded once (round to nearest
 *     even) to the weight dtype: arc lengths for the piecewise-constant
 *     basis, integrals of bilinear tents for the piecewise-linear one.
 *   - Every device pointer is owned by the caller; the plan owns its operator
 *     storage. All apply calls are asynchronous and ordered on the given HIP
 *     stream (NULL = the null stream).
 *   - Every call returns a status and never aborts. On error the contents of
 *     outputs are undefined and srt_last_error() (thread-local) says why.
 */
#ifndef SRT_H
#define SRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srt_plan srt_plan; /* opaque; immutable after creation */

typedef enum {
  SRT_OK = 0,
  SRT_EINVAL = 1,  /* bad argument: null pointer, size <= 0, non-finite value,
                      radii not strictly increasing, dtype pair not supported,
                      workspace too small, destroyed plan */
  SRT_ENOMEM = 2,  /* device allocation failed or budget exceeded */
  SRT_EDEVICE = 3, /* a HIP runtime call failed */
  SRT_ENOTSUP = 4  /* valid request the library does not implement */
} srt_status;

typedef enum { SRT_F32 = 0, SRT_F64 = 1, SRT_BF16 = 2, SRT_F16 = 3 } srt_dtype;

/* How the operators are held. STORED keeps both operators, their transposes
 * and their row-blocked copies resident in HBM. ONTHEFLY keeps only the
 * geometry: every apply regenerates the two operators its direction needs
 * (FP64 geometry, sort, row blocks), applies them and releases them, so an
 * idle plan holds almost no device memory, at the price of most of a plan
 * build per apply (a 128^3 forward measured 0.36 ms stored, 52 ms on the
 * fly). AUTO therefore keeps the operators resident unless they would take
 * more than half of the device's memory. Results are bitwise the same in
 * either mode. */
typedef enum { SRT_OP_AUTO = 0, SRT_OP_STORED = 1, SRT_OP_ONTHEFLY = 2 } srt_opmode;

/* Voxel basis the operators discretise (Sec. 3.1 uses piecewise-constant
 * voxels and notes that other bases, piecewise-linear ones among them, carry
 * over).
 * CONSTANT: f is constant on every voxel; intermediate images are constant on
 *   rho cells that span the midpoints between neighbouring radii (outer edges
 *   half a spacing beyond the end radii).
 * LINEAR: f is the trilinear interpolant of its values at the voxel centres,
 *   falling to zero half a voxel outside the grid; the intermediate image is
 *   bilinear in (z, rho) between the z voxel centres and the radii, zero at
 *   rho = 0 and one radius spacing past the last radius. Volumes then hold
 *   nodal values at the voxel centres; layouts are unchanged. */
typedef enum { SRT_BASIS_CONSTANT = 0, SRT_BASIS_LINEAR = 1 } srt_basis;

typedef struct {
  int32_t ms;  /* voxels along x and along y */
  int32_t mz;  /* voxels along z */
  double x0;   /* lower corner of the grid in x and in y */
  double z0;   /* lower corner of the grid in z */
  double dxy;  /* voxel pitch in x and y (> 0) */
  double dz;   /* voxel pitch in z (> 0) */
} srt_grid;

/* Sizes of a plan's operators (for tests, footprints and FLOP counts). */
typedef struct {
  int64_t nnz_a12;        /* nonzeros of A12 stacked over columns (rows a*n_rho + m) */
  int64_t nnz_a34;        /* nonzeros of A34 (rows h*n_radii + l, cols m*mz + k) */
  int32_t live_radii;     /* rho cells (nodes) that any column's circles reach;
                             A34 columns with m >= live_radii are dropped
                             because the intermediate image is identically
                             zero there */
  int32_t n_angles, n_z, n_radii;
  double weight_scale_a12; /* stored weight = exact weight * scale (power of 2) */
  double weight_scale_a34;
  int32_t basis;           /* srt_basis of the plan */
  int32_t n_rho;           /* size of the stage-2 radial grid (n_radii unless
                              the plan has a grid of its own) */
  int32_t mode;            /* SRT_OP_STORED or SRT_OP_ONTHEFLY (AUTO resolved) */
  int64_t operator_bytes;  /* device bytes of all operators when built */
} srt_plan_info;

/*
 * srt_plan_create -- build both CRT operators (Sec. 2, Sec. 3.1; Alg. 1
 * inputs) for a grid and a cylindrical aperture.
 *   grid        host pointer to the voxel grid
 *   cyl_radius  R >= 0, radius of the sensor cylinder
 *   angles      host, n_angles finite column angles (radians)
 *   z_pos       host, n_z finite sensor heights
 *   radii       host, n_radii sphere radii, > 0 and strictly increasing
 *   value_dtype SRT_F32 or SRT_F64 (type of volumes and data)
 *   weight_dtype SRT_F32/BF16/F16 with F32 values; SRT_F64 with F64 values
 *   mode        SRT_OP_AUTO, SRT_OP_STORED or SRT_OP_ONTHEFLY
 *   device      HIP device ordinal
 *   hip_stream  stream the build runs on (the call returns after the build
 *               has finished)
 *   out         receives the plan; released with srt_plan_destroy
 * Errors: EINVAL (arguments), ENOTSUP (> 2^31 nonzeros), ENOMEM, EDEVICE.
 */
srt_status srt_plan_create(const srt_grid *grid, double cyl_radius,
                           const double *angles, int32_t n_angles,
                           const double *z_pos, int32_t n_z,
                           const double *radii, int32_t n_radii,
                           srt_dtype value_dtype, srt_dtype weight_dtype,
                           srt_opmode mode, int32_t device, void *hip_stream,
                           srt_plan **out);

/*
 * srt_plan_create_columns -- as srt_plan_create, with the sensor columns at
 * arbitrary (x, y) positions instead of on a cylinder. Sec. 2 needs only
 * that each group of sensors lies on one line parallel to z (sharing the
 * first circular transform); A34 is shared by all columns as before.
 *   col_xy   host, n_cols (x, y) pairs (column a at col_xy[2a], col_xy[2a+1]),
 *            finite; a column may stand anywhere, inside the grid included
 *   n_cols   number of columns (the "n_angles" of data layouts and info)
 * Other arguments, outputs and errors as srt_plan_create.
 */
srt_status srt_plan_create_columns(const srt_grid *grid, const double *col_xy,
                                   int32_t n_cols, const double *z_pos, int32_t n_z,
                                   const double *radii, int32_t n_radii,
                                   srt_dtype value_dtype, srt_dtype weight_dtype,
                                   srt_opmode mode, int32_t device, void *hip_stream,
                                   srt_plan **out);

/*
 * Full description of a plan, for srt_plan_create_desc. Fields as in
 * srt_plan_create, plus:
 *   basis       SRT_BASIS_CONSTANT or SRT_BASIS_LINEAR (Sec. 3.1)
 *   cyl_radius, angles   a cylinder aperture (used when col_xy is NULL)
 *   col_xy      host [n_cols][2] column positions anywhere in the plane, or
 *               NULL; exactly one of angles and col_xy is non-NULL
 *   rho, n_rho  host [n_rho] radial grid of the stage-2 image, > 0 and
 *               strictly increasing, or NULL and 0. Sec. 2 evaluates the
 *               first circular transform at the radii rho that the second
 *               one integrates over; the paper takes rho = the sphere radii,
 *               which is what NULL means. A grid of its own makes A12
 *               n_rho x ms^2 per column and A34 (n_z n_radii) x (n_rho mz):
 *               coarser grids make stage 1 cheaper and stage 2 smaller at
 *               some cost in accuracy. Its cells (constant basis) span the
 *               midpoints between grid values, the outer edges half a spacing
 *               beyond the ends; its tent nodes (linear basis) are 0, the
 *               grid values and one spacing past the last.
 * Data layouts are unchanged ([n_cols][n_z][n_radii]).
 */
typedef struct {
  srt_grid grid;
  srt_basis basis;
  double cyl_radius;
  const double *angles;
  const double *col_xy;
  int32_t n_cols;
  const double *z_pos;
  int32_t n_z;
  const double *radii;
  int32_t n_radii;
  const double *rho;
  int32_t n_rho;
  srt_dtype value_dtype;
  srt_dtype weight_dtype;
  srt_opmode mode;
  int32_t device;
} srt_plan_desc;

/*
 * srt_plan_create_desc -- build a plan from a full description (any basis,
 * any column placement, any stage-2 radial grid). desc is read during the
 * call only. Outputs and errors as srt_plan_create; an unknown basis, both
 * or neither of angles / col_xy, a rho pointer without a size (or the
 * reverse) or a rho grid that is not positive and increasing is EINVAL.
 */
srt_status srt_plan_create_desc(const srt_plan_desc *desc, void *hip_stream, srt_plan **out);

/*
 * srt_forward -- Alg. 1 for every column and every batch item:
 * data[b][a][h][l] = sum over (l', k) of A34[(h,l),(l',k)] *
 *                    sum over p of A12_a[l', p] * vol[b][k][p].
 *   vol        device, [batch][mz][ms][ms] of value_dtype (read only)
 *   data       device, [batch][n_angles][n_z][n_radii] of value_dtype
 *              (overwritten)
 *   batch      >= 1
 *   workspace  device scratch of at least the size srt_plan_footprint
 *              reports, 16-byte aligned (hipMalloc's alignment is best), or
 *              NULL to use the plan's own (then calls on one plan must not
 *              overlap)
 *   workspace_bytes  size of workspace (ignored when workspace is NULL)
 * vol and data must be aligned to the size of value_dtype.
 * With a stored plan, a caller workspace and stage timing off, the call only
 * launches kernels on hip_stream (no allocation, memset, copy or wait), so it
 * can be captured into a HIP graph and replayed; the plan's own workspace may
 * be allocated on first use and cannot. An on-the-fly plan (SRT_OP_ONTHEFLY)
 * builds its operators in the call and returns after the apply has finished
 * on hip_stream; calls on one such plan must not overlap.
 * Errors: EINVAL (NULL or misaligned arrays, batch < 1, workspace too small),
 * ENOMEM (own workspace, on-the-fly operators), EDEVICE.
 */
srt_status srt_forward(srt_plan *plan, const void *vol, void *data, int32_t batch,
                       void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * srt_adjoint -- Alg. 2 summed over the columns of the aperture (the exact
 * transpose of srt_forward): vol[b] = sum over a of A12_a^T A34^T data[b][a].
 * Overwrites vol; arguments as in srt_forward with the roles of vol and data
 * exchanged. The sum over columns runs in a fixed order (no atomics), so
 * results are bitwise reproducible.
 */
srt_status srt_adjoint(srt_plan *plan, const void *data, void *vol, int32_t batch,
                       void *workspace, size_t workspace_bytes, void *hip_stream);

/*
 * srt_forward_noalloc -- srt_forward (Alg. 1) for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. It takes no workspace argument and calls
 * no allocating routine; its workspace is a fixed 256 MiB array inside the
 * library, one per device, which that device holds until the process ends.
 *   plan, vol, data, batch, hip_stream  as in srt_forward
 * Same kernels, same results (bitwise) as srt_forward. Every call on one
 * device shares that device's array: calls that overlap on one device (other
 * streams, other threads, other plans) race and must be serialised by the
 * caller. Nothing in the array has to start at zero; each call overwrites
 * what it reads. Stage timing (srt_plan_set_timing) does not record these
 * calls. The first call on a device looks the array's address up
 * (hipGetSymbolAddress); a caller that captures the call into a HIP graph
 * makes one call on that device before capturing. The call itself only
 * launches kernels on hip_stream (no memset, copy or synchronisation), so it
 * can be captured and replayed.
 * Errors: EINVAL (as srt_forward, when the workspace srt_plan_footprint
 * reports for this batch exceeds 256 MiB, and for an on-the-fly plan),
 * ENOTSUP (device ordinal >= 64), EDEVICE.
 */
srt_status srt_forward_noalloc(srt_plan *plan, const void *vol, void *data, int32_t batch,
                               void *hip_stream);

/* Releases the plan's device memory. NULL is accepted. Work queued on the
 * plan must have completed (synchronise its streams first). */
srt_status srt_plan_destroy(srt_plan *plan);

/* Bytes the plan keeps resident and bytes of workspace one apply of
 * `batch` items needs. Either output pointer may be NULL. */
srt_status srt_plan_footprint(const srt_plan *plan, int32_t batch,
                              size_t *resident_bytes, size_t *workspace_bytes);

/* Operator sizes and storage scales. */
srt_status srt_plan_get_info(const srt_plan *plan, srt_plan_info *info);

/*
 * srt_plan_export_coo -- copy one stored operator to host memory as COO
 * triplets (row-major order) with weights converted back to exact weights
 * (stored value / scale, as double). For tests.
 *   which     0 = A12 stacked (rows a*n_rho + m, cols j*ms + i),
 *             1 = A34 (rows h*n_radii + l, cols m*mz + k),
 *             2 = stored transpose of A12 (rows = pixels),
 *             3 = stored transpose of A34 (rows = cells (m, k))
 *   capacity  length of rows/cols/vals; with capacity 0 the pointers may be
 *             NULL and only *nnz is written
 *   nnz       receives the number of stored entries
 * Errors: EINVAL (capacity < nnz with non-zero capacity, bad `which`).
 */
srt_status srt_plan_export_coo(const srt_plan *plan, int32_t which, int64_t capacity,
                               int64_t *nnz, int32_t *rows, int32_t *cols, double *vals);

/*
 * Stage timing (tracing). Each apply runs five stages in stream order:
 *   forward: 0 volume layout, 1 stage 1 (A12), 2 intermediate layout,
 *            3 stage 2 (A34), 4 data layout;
 *   adjoint: 0 data layout, 1 stage 2 (A34^T), 2 intermediate layout,
 *            3 stage 1 (sum over columns of A12^T), 4 volume layout.
 * srt_plan_set_timing(plan, 1) clears earlier records and makes every later
 * apply record HIP events between its stages on the apply's own stream;
 * srt_plan_set_timing(plan, 0) stops and frees the records.
 * srt_plan_stage_times sums the recorded durations (milliseconds) of the
 * forward (adjoint = 0) or adjoint (adjoint = 1) applies into
 * total_ms[0..n_stages) and reports how many applies were recorded. Call it
 * only after synchronising the streams the applies ran on (EINVAL
 * otherwise). Recording is not safe while another thread applies the plan.
 */
srt_status srt_plan_set_timing(srt_plan *plan, int32_t enable);
srt_status srt_plan_stage_times(const srt_plan *plan, int32_t adjoint, int32_t n_stages,
                                double *total_ms, int32_t *n_calls);

/*
 * srt_cgls -- least-squares reconstruction with the matched pair: n_iter
 * iterations of conjugate gradients on the normal equations
 * A^T A f = A^T g (the CGLS arrangement), where A is srt_forward (Alg. 1)
 * and A^T is srt_adjoint (Alg. 2). This is the use the paper gives for an
 * exactly matched adjoint (Sec. 1, Sec. 3.2): the iterates minimise
 * ||A f - g||_2 over growing Krylov spaces. Each batch item is its own
 * problem.
 *   vol        device [batch][mz][ms][ms]: the starting point f0 on entry,
 *              f after n_iter iterations on return
 *   data       device [batch][n_angles][n_z][n_radii]: g (read only)
 *   batch      1 .. 65535
 *   n_iter     >= 0
 *   resid      host array of (n_iter + 1) * batch doubles, or NULL:
 *              resid[k * batch + b] = ||A^T (g - A f_k)||_2 of item b
 *              (the call then returns after the stream has finished)
 *   workspace  device scratch of at least srt_cgls_workspace() bytes,
 *              16-byte aligned (not shared with concurrent calls)
 *   vol and data must be aligned to the size of value_dtype.
 * Inner products are reduced in FP64 in a fixed order; step lengths stay on
 * the device (no host round trip per iteration). Asynchronous on hip_stream
 * unless resid is given.
 * Errors: EINVAL (NULL or misaligned pointers, batch or n_iter out of range,
 * workspace too small), EDEVICE.
 */
srt_status srt_cgls(srt_plan *plan, void *vol, const void *data, int32_t batch,
                    int32_t n_iter, double *resid, void *workspace,
                    size_t workspace_bytes, void *hip_stream);

/* Workspace bytes srt_cgls needs for `batch` items and `n_iter` iterations. */
srt_status srt_cgls_workspace(const srt_plan *plan, int32_t batch, int32_t n_iter,
                              size_t *bytes);

/*
 * srt_nnls -- nonnegative least squares with the matched pair:
 * min 0.5 ||A f - g||_2^2 subject to f >= 0 (an initial pressure is never
 * negative), by n_iter iterations of accelerated projected gradient (FISTA,
 * Beck and Teboulle, SIAM J. Imaging Sci. 2009, Sec. 4, the projection onto
 * f >= 0 as its proximal step). A is srt_forward (Alg. 1), A^T srt_adjoint
 * (Alg. 2); the gradient A^T (A f - g) is only correct because the adjoint
 * is matched (Sec. 1, Sec. 3.2). With y_1 = f_0 and t_1 = 1, step k is
 *   f_k = max(0, y_k - step * A^T (A y_k - g)),
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
 *   y_{k+1} = f_k + ((t_k - 1) / t_{k+1}) (f_k - f_{k-1}).
 * Each batch item is its own problem.
 *   vol        device [batch][mz][ms][ms]: f_0 on entry (need not be
 *              nonnegative), f_{n_iter} on return
 *   data       device [batch][n_angles][n_z][n_radii]: g (read only)
 *   batch      1 .. 65535
 *   n_iter     >= 0
 *   step       1/L with L >= ||A||_2^2 (finite, > 0); srt_opnorm2 estimates
 *              ||A||_2^2 from below, so scale its estimate up a little
 *   resid      host array of n_iter * batch doubles, or NULL:
 *              resid[k * batch + b] = ||A y_{k+1} - g||_2 of item b, the
 *              misfit where step k + 1 took its gradient (the call then
 *              returns after the stream has finished)
 *   workspace  device scratch of at least srt_nnls_workspace() bytes,
 *              16-byte aligned (not shared with concurrent calls)
 *   vol and data must be aligned to the size of value_dtype.
 * Misfits are reduced in FP64 in a fixed order. Asynchronous on hip_stream
 * unless resid is given.
 * Errors: EINVAL (NULL or misaligned pointers, batch, n_iter or step out of
 * range, workspace too small), EDEVICE.
 */
srt_status srt_nnls(srt_plan *plan, void *vol, const void *data, int32_t batch,
                    int32_t n_iter, double step, double *resid, void *workspace,
                    size_t workspace_bytes, void *hip_stream);

/* Workspace bytes srt_nnls needs for `batch` items and `n_iter` iterations. */
srt_status srt_nnls_workspace(const srt_plan *plan, int32_t batch, int32_t n_iter,
                              size_t *bytes);

/*
 * srt_opnorm2 -- estimate of ||A||_2^2, the largest eigenvalue of A^T A,
 * by n_iter steps of the power method on A^T A (srt_forward then
 * srt_adjoint) from the all-ones volume, renormalising after each step.
 * A has no negative entries, so the dominant eigenvector of A^T A can be
 * taken nonnegative and the start has a component along it.
 *   norm2      host; receives the Rayleigh quotient ||A v||^2 / ||v||^2 of
 *              the last iterate v (0 when n_iter is 0). It never exceeds
 *              ||A||_2^2 and rises towards it. The call waits for the stream.
 *   workspace  device scratch of at least srt_nnls_workspace(plan, 1, 0)
 *              bytes, 16-byte aligned
 * Errors: EINVAL (NULL norm2, n_iter < 0, workspace too small or
 * misaligned), EDEVICE.
 */
srt_status srt_opnorm2(srt_plan *plan, int32_t n_iter, double *norm2, void *workspace,
                       size_t workspace_bytes, void *hip_stream);

/* Thread-local description of the last error on the calling thread. */
const char *srt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SRT_H */

/*
 * deam.h -- C ABI of the MI355X (gfx950) DEAM hot-path library.
 *
 * DEAM (dual-energy alternating minimisation) with the metal-trace data
 * substitution of Ge et al., "A Metal Artifact Reduction Scheme For Accurate
 * Iterative Dual-Energy CT Algorithms":
 *   - forward model (Section 2.3, Eq. 8):
 *       g_j(y) = sum_E I0_j(E) exp(-sum_i mu_i(E) l_i(y)),  l_i = H c_i,
 *     with h(x,y) the exact intersection length (mm) of ray y and voxel x;
 *   - metal trace (Section 2.1, Eqs. 2-3): T(y) = sum_x h(x,y) M(x); ray y is
 *     corrupt when T(y) >= t and its measurement is not used;
 *   - DEAM step: the I-divergence of Eq. 5 is minimised by alternating a
 *     p-step on the linear family of Eqs. 9-10 (p_j = q_j d_j / g_j, and
 *     p_j = q_j on the trace: Eq. 11 and the sentence after it) and the
 *     component update c_i <- c_i - ln(b~_i / b^_i) / Z_i, where
 *     b~_i = H^T sum_j sum_E mu_i p_j and b^_i = H^T sum_j sum_E mu_i q_j.
 *
 * Layouts (all C order, channel-major):
 *   image     [n_ch][V],  V = nz*ny*nx, index (iz*ny + iy)*nx + ix (x fastest);
 *             2D geometries have nz = 1.  Voxel (ix,iy,iz) covers
 *             [x0+ix*dx, x0+(ix+1)*dx] x ... with x0 = -nx*dx/2 (grid centred
 *             on the isocentre).
 *   sinogram  [n_ch][R],  R = n_views*n_rows*n_cols, index (v*n_rows + r)*n_cols + k.
 *   Ray (v,r,k): source S = (sid cos b, sid sin b, zs(v)), b = beta0 + 2 pi v /
 *             views_per_rot, zs(v) = (v - (n_views-1)/2) feed_per_rot / views_per_rot;
 *             end point P = S + sdd R(gamma_k) u + (0,0,zeta_r), u = -(cos b, sin b, 0),
 *             gamma_k = (k - (n_cols-1)/2 - col_offset) dgamma,
 *             zeta_r = (r - (n_rows-1)/2) drow_iso sdd / sid  (zeta = 0 in 2D).
 *
 * Precision: a plan is created MIXED (projections, energy sums and weights in
 * FP32; objective terms, reductions and the component update in FP64) or FP64
 * (every step in FP64).  "real" below is float for MIXED and double for FP64.
 *
 * Memory: every data pointer is a device pointer owned by the caller (e.g. a
 * torch tensor), unless stated otherwise.  The plan owns only its small
 * geometry and spectrum tables.  Calls are asynchronous on the given stream
 * (a hipStream_t; NULL = the default stream) and enqueue nothing when they
 * return an error.  Concurrent calls on one plan are allowed on different
 * streams when each uses its own workspace.
 *
 * Errors: every function returns a deam_status; on failure deam_last_error()
 * gives a message (thread-local).  Argument checks happen before anything is
 * enqueued; a device fault shows up at the next synchronisation (and is
 * returned by deam_iterate_sync).  Input data values are not checked on the
 * hot path: image values must be finite and counts d finite and >= 0 (the
 * backprojection of the DEAM weights relies on their signs; a negative count
 * gives undefined results); deam_validate_inputs checks this on request.
 */
#ifndef DEAM_H
#define DEAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DEAM_OK = 0,
  DEAM_ERR_NULL = -1,        /* a required pointer is NULL */
  DEAM_ERR_SHAPE = -2,       /* a size or channel count is out of range */
  DEAM_ERR_GEOMETRY = -3,    /* the geometry is invalid (e.g. source inside the grid) */
  DEAM_ERR_WORKSPACE = -4,   /* the workspace is too small */
  DEAM_ERR_HIP = -5,         /* a HIP runtime call failed */
  DEAM_ERR_UNSUPPORTED = -6, /* the request is valid but not supported by this library */
  DEAM_ERR_VALUE = -7        /* a scalar argument has an invalid value */
} deam_status;

typedef enum { DEAM_FAN2D = 0, DEAM_HELICAL3D = 1 } deam_kind;
typedef enum { DEAM_PREC_MIXED = 0, DEAM_PREC_FP64 = 1 } deam_precision;

/* Weight modes of deam_poly_mean. */
typedef enum {
  DEAM_W_AM = 0,   /* 4 channels (w~1, w~2, w^1, w^2); objective = masked I-divergence terms */
  DEAM_W_GRAD = 1, /* 2 channels u_i = sum_j (r_j - 1) a_ij; objective = masked NLL terms */
  DEAM_W_VJP = 2,  /* 2 channels u_i = -sum_j v_j a_ij for an upstream v_j = dloss/dg_j */
  DEAM_W_STEP_VJP = 3 /* 2 channels lambda_k = dloss/dl_k for an upstream
                         v = [4][R] (dloss/dw~_1, dloss/dw~_2, dloss/dw^_1, dloss/dw^_2) */
} deam_wmode;

/* Workspace queries. */
typedef enum {
  DEAM_OP_FORWARD = 0,
  DEAM_OP_POLY_MEAN = 1,
  DEAM_OP_BACKPROJECT = 2,
  DEAM_OP_ITERATE = 3,
  DEAM_OP_METAL_TRACE = 4,
  DEAM_OP_ITERATE_VJP = 5,
  DEAM_OP_PENALTY = 6,
  DEAM_OP_ITERATE_PENALIZED = 7,
  DEAM_OP_FBP = 8,
  DEAM_OP_MAR_INIT = 9
} deam_op;

typedef struct {
  int32_t kind;                 /* deam_kind */
  int32_t nx, ny, nz;           /* voxels; nz = 1 for DEAM_FAN2D */
  double dx, dy, dz;            /* voxel size, mm */
  int32_t n_views, n_rows, n_cols; /* n_rows = 1 for DEAM_FAN2D */
  double sid, sdd;              /* source-isocentre and source-detector distances, mm */
  double dgamma, col_offset;    /* equiangular channel pitch (rad), channel offset (cells) */
  double drow_iso;              /* detector row pitch at the isocentre, mm (3D) */
  double beta0, views_per_rot;  /* start angle (rad), views per 2 pi */
  double feed_per_rot;          /* table feed per rotation, mm (0 in 2D) */
} deam_geometry;

typedef struct deam_plan deam_plan;

/* Create a plan for one scanner geometry and one pair of spectra.
 *   I0  host [2][n_energy]: photons per ray of the low and high spectrum per
 *       energy bin (the I0_j(E) of Eq. 8; no bowtie: the same for every ray);
 *   mu  host [2][n_energy]: basis attenuation mu_i(E) in 1/mm (Eq. 8).
 * Bins where both spectra are zero are dropped (their terms are exactly 0).
 * precision: deam_precision.  Copies the tables to the current device; a
 * MIXED plan also measures, with one backprojection pass of unit weights on
 * the default stream (synchronous), a per-tile bound of one view batch's sum
 * of intersection lengths, which sets the fixed-point scale of the packed
 * backprojection (deam_iterate, DEAM_BP_NONNEG with 4 channels). */
int deam_plan_create(const deam_geometry* geom, int32_t n_energy, const double* I0,
                     const double* mu, int32_t precision, deam_plan** out);
int deam_plan_destroy(deam_plan* plan);
/* Bowtie filter (the energy- and channel-dependent I0_j(y,E) of Eq. 8): bt
 * host [2][n_cols] holds the filter's path length (mm) in each basis
 * material for every detector channel, so that the rays of channel k see
 * I0_j(E) exp(-mu_1(E) bt[0][k] - mu_2(E) bt[1][k]) (exact for a filter
 * whose attenuation lies in the basis).  It enters every energy sum of the
 * plan (poly-mean, iterations, adjoints) as a per-channel offset of the line
 * integrals; line integrals and the metal trace are unchanged; the MAR
 * initialisation then returns DEAM_ERR_UNSUPPORTED.  bt = NULL removes the
 * filter.  Values must be finite and >= 0.  Synchronous: call it while no
 * call on the plan is in flight. */
int deam_plan_set_bowtie(deam_plan* plan, const double* bt);
/* Number of rays R and voxels V of the plan (host outputs). */
int deam_plan_sizes(const deam_plan* plan, int64_t* n_rays, int64_t* n_voxels);
/* Bytes of device workspace needed by an operation (deam_op). */
int deam_workspace_size(const deam_plan* plan, int32_t op, size_t* bytes);
/* The same size for a plan of this geometry and precision, computed without
 * a plan or a device (to size a workspace before creating the plan).  Equal
 * to deam_workspace_size of the plan that deam_plan_create would make. */
int deam_workspace_size_for(const deam_geometry* geom, int32_t precision, int32_t op,
                            size_t* bytes);

/* Metal trace (Section 2.1, Eqs. 2-3): T(y) = sum_x h(x,y) M(x) in FP64 for
 * both precisions, and mask[y] = (T(y) >= t).
 *   M     [V]  uint8, non-zero = metal voxel;
 *   mask  [R]  uint8 output;   T [R] double output, may be NULL.
 * Workspace: deam_workspace_size(DEAM_OP_METAL_TRACE). */
int deam_metal_trace(const deam_plan* plan, const uint8_t* M, double t, uint8_t* mask,
                     double* T, void* ws, size_t ws_bytes, void* stream);

/* Dilation of a trace along the detector channels (a safety margin around
 * the corrupt rays): out[y] = 1 when a ray of the same view and detector row
 * within `radius` channels of y has mask != 0.  0 <= radius <= n_cols;
 * mask, out [R] uint8, not overlapping. */
int deam_dilate_mask(const deam_plan* plan, const uint8_t* mask, int32_t radius, uint8_t* out,
                     void* stream);

/* Forward projection (the inner sum of Eq. 8): l[c][y] = sum_x h(x,y) c[c][x].
 *   c  [n_ch][V] real;  l [n_ch][R] real;  n_ch = 1 or 2.
 * Workspace: deam_workspace_size(DEAM_OP_FORWARD). */
int deam_forward(const deam_plan* plan, const void* c, int32_t n_ch, void* l, void* ws,
                 size_t ws_bytes, void* stream);

/* Per-ray polyenergetic mean (Eq. 8) with the metal-trace substitution
 * (Eq. 11: p = q where mask = 1) and the weights that feed the backprojection.
 *   l     [2][R] real   line integrals of the two components;
 *   d     [2][R] float  measured counts of the low and high spectrum (finite, >= 0);
 *   mask  [R]    uint8  corrupt rays (NULL = none);
 *   mode  deam_wmode;
 *   v     [2][R] real   upstream dloss/dg (DEAM_W_VJP only, else NULL);
 *   w     [4][R] (AM) or [2][R] real output;
 *   g     [2][R] real output, may be NULL;
 *   obj   device double scalar output, may be NULL: the sum over rays of the
 *         masked I-divergence terms (AM) or masked NLL terms g - d ln g (GRAD).
 * Per ray: q_j(E) = I0_j(E) exp(-mu_1 l_1 - mu_2 l_2), g_j = sum_E q_j,
 * a_ij = sum_E mu_i q_j, r_j = d_j/g_j off the trace and 1 on it;
 * AM: w~_i = sum_j r_j a_ij, w^_i = sum_j a_ij.
 * Workspace: deam_workspace_size(DEAM_OP_POLY_MEAN). */
int deam_poly_mean(const deam_plan* plan, const void* l, const float* d, const uint8_t* mask,
                   int32_t mode, const void* v, void* w, void* g, double* obj, void* ws,
                   size_t ws_bytes, void* stream);

/* deam_poly_mean for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments without the workspace, the same results bit for bit.
 * Its scratch (the per-block objective partials) is a
 * fixed device array of the library, 2 MiB per GPU, held until the process
 * ends; it serves at most 67 100 672 rays (R larger returns
 * DEAM_ERR_UNSUPPORTED, enqueuing nothing).  The call allocates nothing and
 * records no memset.  Every call on one GPU shares that GPU's scratch:
 * calls that overlap on one GPU (different streams, or host threads) race. */
int deam_poly_mean_noalloc(const deam_plan* plan, const void* l, const float* d,
                           const uint8_t* mask, int32_t mode, const void* v, void* w, void* g,
                           double* obj, void* stream);

/* Backprojection with the transpose of the system operator of Eq. 8 (the
 * same h(x,y) as deam_forward): b[c][x] = sum_y h(x,y) w[c][y].  With the
 * DEAM weights of deam_poly_mean it gives b~_i and b^_i of the component
 * update, and with the GRAD or VJP weights the gradient of Eq. 5's
 * objective.
 *   w [n_ch][R] real; b [n_ch][V] real output; n_ch = 1, 2 or 4;
 *   flags: 0, or DEAM_BP_NONNEG when every weight is >= 0 (as the AM weights
 *   are): a cheaper rounding, and for 4 channels of a MIXED plan the packed
 *   accumulation of deam_iterate (two channels per LDS word).  A negative
 *   weight under DEAM_BP_NONNEG gives undefined results.
 * Accumulation is exact integer (fixed point) per voxel, so results are
 * bitwise reproducible.  Each term is rounded to a quantum set per image
 * tile by the largest |w| among the rays that can meet the tile (the call
 * finds these maxima from w), so the relative resolution of a voxel's sum
 * follows the weights of its own rays.
 * Workspace: deam_workspace_size(DEAM_OP_BACKPROJECT). */
enum { DEAM_BP_NONNEG = 1 };
int deam_backproject(const deam_plan* plan, const void* w, int32_t n_ch, int32_t flags, void* b,
                     void* ws, size_t ws_bytes, void* stream);

/* Component update, the c-step of DEAM: the minimiser of the surrogate of the
 * I-divergence (Eq. 5) for the p of Eqs. 9-10 (and p = q on the trace, Eq. 11
 * and the sentence after it), obtained from the convexity of exp in Eq. 8.
 * For each voxel and i = 1, 2, where b~_i > 0 and b^_i > 0,
 * c_i <- c_i - ln(b~_i / b^_i) / Z_i (FP64); other voxels are unchanged.
 * Z_i must satisfy sum_i sum_x h(x,y) mu_i(E) / Z_i <= 1 for every ray y and
 * energy E with photons (then the objective does not increase).
 *   c64  [2][V] double, updated in place;
 *   b    [4][V] real (b~1, b~2, b^1, b^2) from deam_backproject;
 *   Z    host [2] double, > 0;
 *   c_proj [2][V] real output copy of c64 in the plan precision, may be NULL. */
int deam_update(const deam_plan* plan, double* c64, void* c_proj, const void* b,
                const double* Z, void* stream);

/* n_iter iterations of MAR-DEAM (Section 2.3: Eqs. 5, 8-10, with the data on
 * the metal trace replaced by the estimate in every iteration, Eq. 11 and the
 * sentence after it) on one stream with no host synchronisation: forward
 * projection + poly-mean (AM), backprojection, update.
 *   c64   [2][V] double, updated in place;
 *   c_proj [2][V] real output or NULL: the final iterate in the plan precision;
 *   d     [2][R] float counts (finite, >= 0);  mask [R] uint8 or NULL;  Z host [2];
 *   obj_hist  device [n_iter] double or NULL: obj_hist[k] = masked
 *             I-divergence (Eq. 5 restricted to T < t) at the iterate c^k
 *             entering iteration k.
 * A device fault shows up at the caller's next synchronisation; the history
 * stays on the device so that nothing waits (deam_iterate_sync copies it out
 * and reports faults).  Workspace: deam_workspace_size(DEAM_OP_ITERATE). */
int deam_iterate(const deam_plan* plan, double* c64, void* c_proj, const float* d,
                 const uint8_t* mask, const double* Z, int32_t n_iter, double* obj_hist,
                 void* ws, size_t ws_bytes, void* stream);

/* deam_iterate with the objective history in host memory: obj_hist host
 * [n_iter] double or NULL.  Synchronises `stream` before returning and
 * returns DEAM_ERR_HIP when a device fault occurred during the iterations.
 * Allocates n_iter doubles of device memory for the duration of the call. */
int deam_iterate_sync(const deam_plan* plan, double* c64, void* c_proj, const float* d,
                      const uint8_t* mask, const double* Z, int32_t n_iter, double* obj_hist,
                      void* ws, size_t ws_bytes, void* stream);

/* Debug check of the inputs of an iteration (not on the hot path): c64 [2][V]
 * double must be finite, d [2][R] float finite and >= 0 (either pointer may
 * be NULL to skip it).  n_bad host [2] int64 output or NULL: the number of
 * offending entries of each.  ws: device workspace of >= 16 bytes, 8-byte
 * aligned (any workspace of the plan's operations qualifies).  Synchronises
 * `stream`; returns DEAM_ERR_VALUE when an entry is invalid. */
int deam_validate_inputs(const deam_plan* plan, const double* c64, const float* d, int64_t* n_bad,
                         void* ws, size_t ws_bytes, void* stream);

/* deam_iterate with per-kernel device timing, for benchmarks and profiling.
 * Same arguments and results as deam_iterate, plus
 *   kernel_ms  host [4] float output: summed device time (ms, HIP events
 *              recorded on `stream`) over the n_iter iterations of
 *              [0] the forward-projection + poly-mean kernel,
 *              [1] the backprojection kernel,
 *              [2] the update kernel,
 *              [3] the whole loop (first to last event).
 * Synchronises `stream` before returning. */
int deam_iterate_timed(const deam_plan* plan, double* c64, void* c_proj, const float* d,
                       const uint8_t* mask, const double* Z, int32_t n_iter, double* obj_hist,
                       void* ws, size_t ws_bytes, void* stream, float* kernel_ms);

/* DEAM with a system operator and a metal trace per scan (Section 2.1: the
 * two scans may differ, e.g. by geometry or motion, and then need their own
 * traces T_j).  Each scan has its own plan over the same image grid and
 * precision: plan_lo created with the high-energy spectrum all zero and
 * plan_hi with the low-energy spectrum all zero (DEAM_ERR_VALUE otherwise),
 * so that each scan's energy sums and weights use its own spectrum only.
 * b~ and b^ are the sums of the two scans' backprojections; the update is
 * deam_update's.
 *   d_lo [2][R_lo], d_hi [2][R_hi] float: channel 0 of d_lo holds the
 *       low-energy counts and channel 1 of d_hi the high-energy counts; the
 *       other channel is read but does not enter (its expected counts are 0);
 *   mask_lo [R_lo], mask_hi [R_hi] uint8 or NULL: each scan's trace;
 *   obj_hist  device [n_iter] double or NULL: the sum of the two masked
 *             I-divergences at the iterate entering each iteration.
 * Workspace: deam_dual_workspace_size bytes. */
int deam_dual_workspace_size(const deam_plan* plan_lo, const deam_plan* plan_hi, size_t* bytes);
int deam_iterate_dual(const deam_plan* plan_lo, const deam_plan* plan_hi, double* c64,
                      const float* d_lo, const uint8_t* mask_lo, const float* d_hi,
                      const uint8_t* mask_hi, const double* Z, int32_t n_iter, double* obj_hist,
                      void* ws, size_t ws_bytes, void* stream);

/* Ordered-subset DEAM: n_iter epochs; the views are split into n_sub
 * interleaved subsets (view v belongs to subset v mod n_sub), and an epoch
 * runs one DEAM step per subset s = 0, 1, ..., n_sub - 1 using only that
 * subset's rays (forward projection, poly-mean and backprojection walk its
 * views alone; the update is deam_update's).  Each step costs about 1/n_sub
 * of an iteration and moves about as far as a full one early on.  n_sub = 1
 * is deam_iterate.  1 <= n_sub <= n_views.
 *   obj_hist  device [n_iter] double or NULL: masked I-divergence at the
 *             iterate entering each epoch (costs one extra all-view
 *             projection per epoch when requested).
 * Other arguments as deam_iterate.  Workspace: deam_workspace_size(DEAM_OP_ITERATE). */
int deam_iterate_os(const deam_plan* plan, double* c64, const float* d, const uint8_t* mask,
                    const double* Z, int32_t n_sub, int32_t n_iter, double* obj_hist, void* ws,
                    size_t ws_bytes, void* stream);

/* Bit-packed trace (1 bit per ray instead of 1 byte: 7.5 MB instead of 60 MB
 * for 60 M rays): bit b of bits[i] is mask[32 i + b] != 0.
 *   mask [R] uint8;  bits [ceil(R / 32)] uint32 output. */
int deam_pack_mask(const deam_plan* plan, const uint8_t* mask, uint32_t* bits, void* stream);

/* deam_iterate with the trace given bit-packed (deam_pack_mask's layout);
 * same results as deam_iterate with the byte mask, bit for bit.
 * Workspace: deam_workspace_size(DEAM_OP_ITERATE). */
int deam_iterate_packed(const deam_plan* plan, double* c64, const float* d,
                        const uint32_t* mask_bits, const double* Z, int32_t n_iter,
                        double* obj_hist, void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of one DEAM iteration (the differentiable form of
 * deam_iterate, for losses on the reconstructed image): with
 * Phi(c) = c - ln(b~(c) / b^(c)) / Z (the update of deam_update, c unchanged
 * where b~ <= 0 or b^ <= 0),
 *   out = (dPhi/dc)^T G = G + H^T lambda,
 * where u~_i = -G_i / (Z_i b~_i) and u^_i = G_i / (Z_i b^_i) are projected,
 * alpha = H u~ and beta = H u^, and lambda_k(y) = sum_i alpha_i dw~_i/dl_k +
 * beta_i dw^_i/dl_k is formed per ray from the second moments
 * sum_E mu_i(E) mu_k(E) q_j(y,E) (chain rule through Eq. 8 and the weights).
 * The projections of c are recomputed (nothing is kept from the forward pass).
 *   c64  [2][V] double: the iterate entering the iteration;
 *   d    [2][R] float;  mask [R] uint8 or NULL;  Z host [2] double > 0;
 *   G    [2][V] double: dloss/dPhi;   out [2][V] double output (may not
 *        alias G or c64).
 * Workspace: deam_workspace_size(DEAM_OP_ITERATE_VJP). */
int deam_iterate_vjp(const deam_plan* plan, const double* c64, const float* d,
                     const uint8_t* mask, const double* Z, const double* G, double* out,
                     void* ws, size_t ws_bytes, void* stream);

/* Penalised DEAM (Section 2.3, Eqs. 6-7).  The penalty is
 *   R(c) = lambda sum_i sum_x sum_{x~ in N_x} w(x,x~) phi(c_i(x) - c_i(x~)),
 * N_x = the voxels one step away along every axis inside the grid (8 in 2D,
 * 26 in 3D), w = 1 / (distance between the voxel centres in mm), and phi the
 * potential of Eq. 7 read as the convex "fair" potential
 *   phi(t) = delta^2 (|t|/delta - ln(1 + |t|/delta))
 * (the printed sign inside the logarithm would make it concave and undefined
 * for |t| >= delta).  lambda >= 0 and delta > 0, both finite; otherwise
 * DEAM_ERR_VALUE. */

/* R(c) for c64 [2][V] double, into the device scalar out (FP64, deterministic).
 * Workspace: deam_workspace_size(DEAM_OP_PENALTY). */
int deam_penalty(const deam_plan* plan, const double* c64, double lambda, double delta,
                 double* out, void* ws, size_t ws_bytes, void* stream);

/* Penalised component update.  The DEAM data surrogate plus De Pierro's
 * decoupling of R make the c-step one convex problem per voxel and component:
 *   c_i(x) = argmin_c  b~ c + (b^/Z_i) exp(-Z_i (c - c_prev)) +
 *            lambda sum_{x~ in N_x} w phi(2c - c_prev_i(x) - c_prev_i(x~)),
 * solved in FP64 by safeguarded Newton iterations to about 1e-13 relative;
 * voxels with b~ <= 0 or b^ <= 0 keep c_prev.  lambda = 0 gives deam_update.
 *   c_prev [2][V] double: the iterate c^k (read only);
 *   c64    [2][V] double output, must not overlap c_prev;
 *   b, Z, c_proj as for deam_update. */
int deam_update_penalized(const deam_plan* plan, const double* c_prev, double* c64, void* c_proj,
                          const void* b, const double* Z, double lambda, double delta,
                          void* stream);

/* n_iter penalised DEAM iterations (deam_iterate with the penalised update).
 * obj_hist (device [n_iter] double or NULL): masked I-divergence + R at the
 * iterate entering each iteration; it does not increase for FP64 plans.
 * Workspace: deam_workspace_size(DEAM_OP_ITERATE_PENALIZED). */
int deam_iterate_penalized(const deam_plan* plan, double* c64, const float* d,
                           const uint8_t* mask, const double* Z, double lambda, double delta,
                           int32_t n_iter, double* obj_hist, void* ws, size_t ws_bytes,
                           void* stream);

/* MAR initialisation (Section 2.2, Fig. 1, Eq. 4): the initial image of
 * MAR-DEAM from an analytic reconstruction with normalised metal artifact
 * reduction (NMAR) of the measured sinograms.  Defined for 2D fan-beam plans
 * over one full rotation (n_views * 2 pi / views_per_rot = 2 pi) with at most
 * 4096 channels; other plans return DEAM_ERR_UNSUPPORTED.  Real arrays are in
 * the plan precision. */

/* Equiangular fan-beam filtered backprojection of n_ch (1 or 2) sinograms of
 * line integrals p [n_ch][R] into img [n_ch][V]: each view is weighted by
 * sid cos(gamma), convolved with the sampled ramp kernel g(0) = 1/(8 a^2),
 * g(j a) = -1/(2 pi^2 sin^2(j a)) for odd j, 0 for even j (a = dgamma), times a,
 * and backprojected as (2 pi / n_views) sum_v Q_v(gamma') / L^2 with gamma', L
 * the fan angle and distance of the pixel centre from the source and linear
 * interpolation between channels (zero outside the detector).  Sums in FP64.
 * Workspace: deam_workspace_size(DEAM_OP_FBP). */
int deam_fbp(const deam_plan* plan, const void* p, int32_t n_ch, void* img, void* ws,
             size_t ws_bytes, void* stream);

/* NMAR across the metal trace, per view and for both sinograms: on a trace
 * ray the value p / (p_prior + eps) is interpolated linearly along the
 * channels between the nearest rays off the trace (the nearest one beyond a
 * detector end) and multiplied by p_prior + eps; other rays are copied.
 *   p, p_prior, out [2][R] real (out must not overlap p);  mask [R] uint8;
 *   eps > 0 (line-integral units). */
int deam_nmar(const deam_plan* plan, const void* p, const uint8_t* mask, const void* p_prior,
              double eps, void* out, void* stream);

typedef struct {
  double t;           /* metal-trace threshold, mm of metal path (as deam_metal_trace) */
  double water[2];    /* spectrum-weighted attenuation of water, low / high (1/mm), > 0 */
  double air_frac;    /* prior: mu < air_frac * water_j -> 0 */
  double bone_frac;   /* prior: mu < bone_frac * water_j -> water_j, else mu kept */
  double metal_frac;  /* metal image: mu_H >= metal_frac * water_H */
  double eps;         /* NMAR normalisation offset, > 0 */
} deam_mar_params;

/* The whole initialisation from the counts d [2][R] float:
 *   p_j = ln(sum_E I0_j) - ln(max(d_j, 1)); mu0 = FBP(p);
 *   M = [mu0_H >= metal_frac water_H] (output [V] uint8);
 *   mask = [H M >= t] (output [R] uint8, the trace used by DEAM);
 *   prior_j = 0 below air_frac water_j, water_j below bone_frac water_j or on
 *   M, mu0_j above;  p~ = NMAR(p, mask, H prior, eps);  mu1 = FBP(p~);
 *   c64 = Mt^-1 (mu1_L, mu1_H) (Eq. 4, output [2][V] double), with
 *   Mt[j][i] = sum_E I0_j(E) mu_i(E) / sum_E I0_j(E) from the plan's tables.
 * Thresholds are compared in the plan precision.
 * Workspace: deam_workspace_size(DEAM_OP_MAR_INIT). */
int deam_mar_init(const deam_plan* plan, const float* d, const deam_mar_params* prm, double* c64,
                  uint8_t* M, uint8_t* mask, void* ws, size_t ws_bytes, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* deam_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DEAM_H */

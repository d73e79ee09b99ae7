/*
 * pyhst.h — C ABI of the MI355X (gfx950) reconstruction library for
 * parallel-beam tomography after PyHST2 (Mirone, Gouillart, Brun, Tafforeau,
 * Kieffer, Nucl. Instr. Meth. B).
 *
 * Scope: the reconstruction path of the paper's processing pipe (section 2.3):
 * dark/flat normalisation with time-interpolated flats and -log, the ramp
 * filter and pixel-driven backprojection of filtered backprojection (FBP), and
 * the projector pair plus total-variation operators of the TV-regularised
 * iterative mode (section 3.1, eqs. (1)-(3)).
 *
 * Conventions shared by every entry point
 *   - Pixel (ix, iy) of an n_x x n_y slice (row-major, ix fastest) has centre
 *     x = ix - (n_x-1)/2, y = iy - (n_y-1)/2 in pixel units; pixels are
 *     pixel_size (s) detector bins wide.
 *   - Detector bin j has its centre at coordinate j.  At projection k the
 *     centre of pixel (ix, iy) lands on
 *         t = s (x cos th_k + y sin th_k) + axis_pos + axis_shift[k].
 *   - hat(d) = max(0, 1 - |d|) (linear interpolation, zero outside the row).
 *     B (backproject):      img[px]     = sum_k sum_j q[k][j] hat(t_k(px) - j)
 *     A (forward_project):  sino[k][j]  = s^2 sum_px img[px] hat(t_k(px) - j)
 *     so A = s^2 B^T exactly.
 *   - FBP = B(fbp_filter(p)); it returns the attenuation per bin length.
 *
 * Memory and streams
 *   - Every data pointer is a DEVICE pointer owned by the caller unless the
 *     comment says "host".  Calls only enqueue work on the given stream and
 *     return; outputs are valid once the stream reaches that point.
 *   - Once a plan exists no entry point allocates device memory; scratch is
 *     passed in by the caller (tv_prox, reconstruct_slices).
 *   - A plan is immutable after creation except for its tile and projector
 *     choices (pyhst_plan_set_tiles, pyhst_plan_set_fp_kernel,
 *     pyhst_plan_set_bp_slices, not to be called
 *     while other calls use the plan) and its caches (graphs, stream slots),
 *     which are guarded by a lock.  Calls on one plan may run concurrently on
 *     different streams when each has its own output and work buffers; the
 *     persistent backprojector's work counter belongs to the stream (a graph
 *     captured on one stream must not be replayed concurrently with itself or
 *     with other calls of that stream on another stream).
 *
 * Errors: every entry point returns PYHST_OK (0) or a negative code; no C++
 * exception or abort crosses the ABI.  pyhst_last_error() gives the message of
 * the calling thread's last failure.
 */
#ifndef PYHST_H
#define PYHST_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PYHST_OK = 0,
    PYHST_EARG = -1,   /* NULL pointer, non-positive size, axis outside the detector, bad layout */
    PYHST_EGEOM = -2,  /* angular coverage below 180 (resp. 360) degrees, or a half-acquisition
                          axis that is not in the outer quarter of the detector (section 2.1) */
    PYHST_ENOMEM = -3, /* device allocation failed at plan creation, or work buffer too small */
    PYHST_EHIP = -4,   /* a HIP runtime error; see pyhst_last_error() */
    PYHST_ENUM = -5    /* non-finite or zero estimate (pyhst_opnorm, pyhst_patch_lipschitz) */
};

enum { PYHST_SCAN_180 = 0, PYHST_SCAN_360 = 1, PYHST_SCAN_360_HALF = 2 };
enum { PYHST_FBP = 0, PYHST_TV_CP = 1, PYHST_ISTA = 2, PYHST_FISTA = 3 };
/* Largest slice count of a plan or of one tv_prox call (one grid dimension). */
enum { PYHST_MAX_SLICES = 65535 };
/* A plan keeps at most this many executable HIP graphs (one per distinct
 * reconstruct_slices call with use_graph: method, buffers, stream, parameters);
 * once it holds them, further distinct calls run as plain launches. */
enum { PYHST_MAX_GRAPHS = 64 };
/* Persistent backprojection (pyhst_plan_set_tiles) takes its work counter from a
 * per-plan slot owned by the calling stream; a plan has this many slots, and a
 * call on a further stream runs the non-persistent kernel instead. */
enum { PYHST_MAX_STREAMS = 64 };
/* Forward-projector kernels (pyhst_plan_set_fp_kernel). */
enum { PYHST_FP_AUTO = 0, PYHST_FP_BLOCKS = 1, PYHST_FP_STAGED = 2, PYHST_FP_LINES = 3 };

/* Geometry of one slice family (section 2.1: parallel beam, >= 180 degrees of
 * rotation, optional 360 degree half acquisition with the axis near a detector
 * border, axis displacement and angle given per projection). */
typedef struct {
    int32_t n_x, n_y;          /* slice size in pixels */
    int32_t n_det;             /* detector bins per row */
    int32_t n_angles;          /* projections */
    const double *angles;      /* host [n_angles], radians, any order and spacing */
    double axis_pos;           /* rotation-axis position in bin coordinates */
    const double *axis_shift;  /* host [n_angles] per-projection axis displacement (bins), or NULL */
    int32_t scan;              /* PYHST_SCAN_180, PYHST_SCAN_360 or PYHST_SCAN_360_HALF */
    double pixel_size;         /* s: pixel width in bins; <= 0 means 1 */
    double ha_overlap;         /* half acquisition: feather half-width d_f (bins); 0 = distance of the
                                  axis to the nearer detector edge */
} pyhst_geom;

typedef struct pyhst_plan pyhst_plan;

/* Where one slice of a plan lives in the packed buffers the entry points take.
 * For a uniform plan the packed layouts are plain stacks: sinograms
 * [S][K][n_det], filtered rows [S][K][filt_len], images [S][n_y][n_x]. */
typedef struct {
    int32_t n_x, n_y, n_det, n_angles;
    int32_t filt_len;        /* row length written by fbp_filter (n_det unless half acquisition) */
    int32_t filt_pad;        /* zero bins prepended in the filtered layout */
    double filt_axis;        /* axis position in the filtered layout */
    int64_t sino_offset;     /* element offset of the slice in packed [K][n_det] sinograms */
    int64_t filt_offset;     /* element offset in packed [K][filt_len] filtered rows */
    int64_t img_offset;      /* element offset in packed [n_y][n_x] images */
} pyhst_slice_info;

/* Create a plan for n_slices (1 .. PYHST_MAX_SLICES) slices of at most 2^31 - 1
 * pixels each (n_x * n_y).  g: host [n_geom] geometries; slice_geom:
 * host [n_slices] index into g for each slice, or NULL (all slices use g[0]).
 * The plan copies every host array, computes FP64 angle tables, angle
 * weights, half-acquisition weights and filter spectra, and keeps them in
 * device memory of the current device.  Returns EARG/EGEOM on invalid
 * geometry, ENOMEM/EHIP on device failure. */
int pyhst_plan_create(const pyhst_geom *g, int32_t n_geom, const int32_t *slice_geom, int32_t n_slices,
                      pyhst_plan **out);
int pyhst_plan_destroy(pyhst_plan *plan);
int pyhst_plan_slice_info(const pyhst_plan *plan, int32_t slice, pyhst_slice_info *out);
/* Total elements of the packed sinogram, filtered and image buffers. */
int pyhst_plan_sizes(const pyhst_plan *plan, int64_t *sino_elems, int64_t *filt_elems, int64_t *img_elems);
/* Backprojector tile: 0 = 64x64, 1 = 64x32, 2 = 32x64, 3 = 32x32, 4 = 64x128 pixels, 5 = 32x32 with
 * the projections split over 4 angle groups (1024-thread workgroups, partial sums added in a fixed
 * order; for slices too small to fill the chip with tiles); -1 = automatic.
 * persistent != 0 runs the backprojector as one persistent launch over a
 * cost-sorted (slice, tile) work list. */
int pyhst_plan_set_tiles(pyhst_plan *plan, int32_t bp_tile, int32_t persistent);
int pyhst_plan_get_tiles(const pyhst_plan *plan, int32_t *bp_tile, int32_t *persistent);
/* Forward-projector kernel for every projection this plan makes (forward_project,
 * the iterative solvers, pyhst_cv_error): PYHST_FP_AUTO (the default) picks
 * PYHST_FP_STAGED for pixel sizes >= 0.5 (on a uniform plan of several slices
 * with pixels of 0.943 to 1 bin, four or two slices per workgroup sharing the
 * staged segment and the hat weights, with results equal bit for bit to one
 * slice per workgroup); for smaller pixels, angle blocks when they give at
 * least 8 workgroups per compute unit, else PYHST_FP_LINES;
 * PYHST_FP_BLOCKS: up to 16 projections of similar direction per workgroup
 * sharing LDS-staged line segments; PYHST_FP_STAGED: one to four neighbouring
 * projections whose candidates share the segment per workgroup, line segments
 * staged in LDS (pixel size >= 0.5 only: smaller pixels take PYHST_FP_LINES);
 * PYHST_FP_LINES: one projection per workgroup read straight from global
 * memory.  All compute the same sums up to FP32 rounding order.  EARG for
 * another value. */
int pyhst_plan_set_fp_kernel(pyhst_plan *plan, int32_t kind);
int pyhst_plan_get_fp_kernel(const pyhst_plan *plan, int32_t *kind);
/* Slices per backprojector workgroup (section 2.3's tiles) for plain backprojections
 * (backproject, the FBP, the ISTA / FISTA and patch-prior steps; the
 * Chambolle-Pock step with its fused primal update keeps one): 0 = automatic
 * (two on a uniform plan of at least two slices without the persistent work
 * queue), 1 = one, 2 = two where the plan allows it.  Two slices share each
 * staged window entry (one 16-byte LDS read per pixel update of both) and the
 * coordinate arithmetic; the images equal one slice per workgroup bit for bit.
 * EARG for another value. */
int pyhst_plan_set_bp_slices(pyhst_plan *plan, int32_t per_workgroup);
/* Autotuner: times the backprojector of this plan for every tile shape, with
 * and without the persistent work queue (reps launches each, HIP events on
 * `stream`), on filt (filtered layout) -> img, and keeps the fastest.  Writes
 * img; synchronises the stream; *best_ms (may be NULL) receives the time of one
 * launch with the chosen setting. */
int pyhst_plan_autotune(pyhst_plan *plan, const float *filt, float *img, int32_t reps, float *best_ms,
                        hipStream_t stream);

/* Dark/flat normalisation and -log (section 2.3, first steps of the pipe;
 * Beer-Lambert for absorption data), rearranged into sinograms (one per
 * detector line).  Uniform plans only.
 *   raw   [K][R][n_det] uint16 radiographs as acquired (R = n_slices)
 *   flats [n_flats][R][n_det] float, acquired at projection positions
 *   flat_pos host [n_flats] ascending; the flat of projection k is linearly
 *   interpolated between the bracketing flats, held constant outside.
 *   dark  [R][n_det] float
 *   sino  [R][K][n_det] float:  -ln(max((I - D)/(F_k - D), eps)), 0 where F_k <= D.
 * n_flats must be in [1, 32]. */
int pyhst_normalize(const pyhst_plan *plan, const uint16_t *raw, const float *flats, const double *flat_pos,
                    int32_t n_flats, const float *dark, float eps, float *sino, hipStream_t stream);

/* pyhst_normalize with the hot-spot filter of section 2.3 applied to the
 * flat-field-corrected transmission t = (I - D)/(F_k - D) before the -log: a
 * pixel whose 3x3 neighbours' median (the up to 8 neighbours inside the rows
 * and bins given; mean of the middle two for an even count; taken before any
 * replacement) is below t by more than threshold takes that median.  Dead
 * pixels (F_k <= D) stay 0.  threshold < 0 or NaN -> PYHST_EARG.
 * Halo: raw, flats and dark hold R_in = halo_lo + R + halo_hi detector rows
 * (raw [K][R_in][n_det], flats [n_flats][R_in][n_det], dark [R_in][n_det]);
 * sino [R][K][n_det] receives rows halo_lo .. halo_lo + R - 1, and the halo
 * rows (0 or 1 on each side, else PYHST_EARG) serve only as neighbours, so a
 * volume filtered in chunks of rows equals the volume filtered whole. */
int pyhst_normalize_hotspot(const pyhst_plan *plan, const uint16_t *raw, const float *flats, const double *flat_pos,
                            int32_t n_flats, const float *dark, float eps, float threshold, int32_t halo_lo,
                            int32_t halo_hi, float *sino, hipStream_t stream);

/* Ring-artifact filter of section 2.3, in place on sinograms sino [R][K][n_det]
 * of a uniform plan: per slice, m[j] = mean over projections of (sino - obj),
 * hp = m - (mean of m over the bins j-width..j+width that exist), and hp[j] is
 * subtracted from every row.  obj (same layout, or NULL) is the projection of
 * the strongly absorbing part of the object (the thresholded first
 * reconstruction), removed before the average so that its borders do not
 * enter hp.  work: device scratch of >= 2 * R * n_det doubles. */
int pyhst_ring_filter(const pyhst_plan *plan, float *sino, int32_t width, const float *obj, double *work,
                      size_t work_doubles, hipStream_t stream);

/* Ramp filter of FBP (section 2.3): for every row, half-acquisition weighting
 * and extension (360 degree half scans), then linear convolution on
 * [0, filt_len) with the Ram-Lak kernel h[0] = 1/4, h[odd n] = -1/(pi^2 n^2)
 * (unit bin spacing), times the angle's quadrature weight (mid-point rule over
 * the scan period; pi/K for a uniform 180 degree scan).
 *   sino [packed K x n_det], filt [packed K x filt_len].  In place allowed when
 *   filt_len == n_det for every slice. */
int fbp_filter(const pyhst_plan *plan, const float *sino, float *filt, hipStream_t stream);

/* Backprojection img = alpha * B(sino) + beta * img (B as above, no angle
 * weights).  filtered_layout = 0: rows are detector rows [K][n_det] (then
 * alpha = s^2 gives A^T, the exact adjoint of forward_project); 1: rows are in
 * the layout fbp_filter writes (FBP = backproject(fbp_filter(p), 1, 1, 0)).
 * beta == 0 never reads img. */
int backproject(const pyhst_plan *plan, const float *sino, int32_t filtered_layout, float *img, float alpha,
                float beta, hipStream_t stream);

/* Matched forward projection sino = alpha * A(img) (ray-driven gather of the
 * same hat weights; section 2.3 and eq. (1)).  img [packed n_y x n_x], sino
 * [packed K x n_det].  alpha = 1 gives A; alpha = 1/s^2 gives B^T, the adjoint
 * of backproject with alpha = 1.  Non-finite alpha -> PYHST_EARG. */
int forward_project(const pyhst_plan *plan, const float *img, float *sino, float alpha, hipStream_t stream);

/* Proximal map of lambda*TV (isotropic TV of eq. (2), forward differences with
 * a zero last difference):  out = argmin_u 1/2|u - in|^2 + lambda TV(u), by
 * n_inner steps of Chambolle's (2004) dual projection with step 1/8 from a
 * zero dual field.  in, out [n_slices][n_y][n_x] (n_slices <= PYHST_MAX_SLICES,
 * n_y <= 524280); in == out allowed.
 * work: device scratch of at least 4*n_slices*n_y*n_x floats (two copies of the
 * dual field; work_floats gives its size); NULL or too small -> PYHST_EARG. */
int tv_prox(int32_t n_slices, int32_t n_y, int32_t n_x, const float *in, float *out, float lambda,
            int32_t n_inner, float *work, size_t work_floats, hipStream_t stream);

/* Whole-slice reconstruction.
 *   method PYHST_FBP: out = B(fbp_filter(normalise(raw)))   (or of sino)
 *   method PYHST_TV_CP: eq. (3), min_x 1/2|A x - y|^2 + lambda TV(x), by
 *     n_iter Chambolle-Pock iterations with K = [A; mu grad] (mu = tv_mu, <= 0
 *     means 1), tau = sigma = 1/op_norm, theta = 1, from zero:
 *       p <- (p + sigma (A xbar - y)) / (1 + sigma)
 *       q <- q + sigma mu grad xbar, each pixel's 2-vector projected on |q| <= lambda/mu
 *       x' = x - tau (A^T p - mu div q),  xbar = 2 x' - x,  x = x'
 *     (lambda TV(x) = (lambda/mu) sum |mu grad x|, so the minimiser does not
 *     depend on mu; mu = |A|/|grad| balances the two blocks so that the TV
 *     dual reaches its bound within a few hundred iterations).  op_norm must
 *     be |K| (pyhst_opnorm with_grad = 1 and the same mu).
 *   method PYHST_ISTA / PYHST_FISTA: eq. (3) by the solvers named in section
 *     3.1 (Daubechies et al. 2004; Beck & Teboulle 2009): n_iter iterations of
 *       x_k = prox_{(lambda/La) TV}(z - (1/La) A^T (A z - y)),  La = op_norm^2,
 *     ISTA: z = x_k;  FISTA: t' = (1 + sqrt(1 + 4t^2))/2,
 *     z = x_k + ((t - 1)/t') (x_k - x_{k-1}), t = t', from x_0 = z = 0, t = 1.
 *     The proximal map is tv_prox with n_inner dual iterations from zero.
 *     op_norm must be |A| (pyhst_opnorm with_grad = 0).
 *   Iterative methods: op_norm <= 0 or non-finite -> PYHST_EARG.  energy
 *     (DEVICE float [n_iter], or NULL) receives 1/2|A x - y|^2 + lambda TV(x)
 *     of the whole batch after every iteration (section 3.1: the energy is
 *     displayed so that convergence can be judged); it is written by kernels
 *     of the same launch sequence (graph-capturable), FP64 sums rounded to
 *     float; checking it for non-finite values is the caller's.
 * Input: raw (uint16 [K][R][n_det] with flats, flat_pos, n_flats, dark, eps;
 * uniform plans) or, when raw == NULL, sino (normalised line integrals,
 * packed [K][n_det]).  out [packed n_y x n_x].
 * work/work_bytes: device scratch; call first with out == NULL to receive the
 * required size in *work_bytes (no work is enqueued).
 * The call never synchronises and never allocates device memory.
 * use_graph != 0: the launches are captured once into a HIP graph kept by the
 * plan (keyed by every argument) and replayed on later identical calls.
 * Preprocessing (hot_spot, ring_width; uniform plans) runs before every method:
 * the normalised sinogram then goes through a work buffer (the caller's sino is
 * not modified) and FBP no longer fuses normalisation into the filter. */
typedef struct {
    const uint16_t *raw;
    const float *sino;
    const float *flats;
    const double *flat_pos;   /* host */
    int32_t n_flats;
    const float *dark;
    float eps;
    int32_t method;
    float lambda;
    int32_t n_iter;
    double op_norm;           /* iterative methods: |[A; mu grad]| (TV_CP) or |A| (ISTA/FISTA), > 0 */
    float *energy;            /* device [n_iter] or NULL */
    float *out;
    void *work;
    size_t work_bytes;
    int32_t use_graph;
    int32_t n_inner;          /* ISTA/FISTA: dual iterations of each proximal map (>= 0) */
    /* optional preprocessing of section 2.3 (zero = off) */
    int32_t hot_spot;         /* raw input: hot-spot filter with hot_threshold (pyhst_normalize_hotspot) */
    float hot_threshold;
    int32_t ring_width;       /* > 0: ring filter of the sinograms (pyhst_ring_filter) with this half-width */
    int32_t ring_object;      /* != 0: obj = A(x [x > ring_threshold]), x = FBP of the unfiltered data */
    float ring_threshold;
    double tv_mu;             /* TV_CP: scale mu of the gradient block (<= 0: 1) */
    int32_t hot_halo_lo;      /* hot_spot: halo rows of raw/flats/dark before and after the plan's */
    int32_t hot_halo_hi;      /*   rows (0 or 1 each; pyhst_normalize_hotspot), else 0 */
} pyhst_recon_args;

int reconstruct_slices(const pyhst_plan *plan, pyhst_recon_args *a, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as reconstruct_slices, with its scratch taken from a per-device array
 * of PYHST_STATIC_SCRATCH_BYTES (64 MiB) that the library's code object holds
 * on every device it runs on until the process ends.  a->work is ignored;
 * a->work_bytes receives the scratch the call needs; a->use_graph is ignored
 * (plain launches; a caller may capture them itself).  The caller still owns
 * every input and output.  The plan's device must be current.  A call needing
 * more than PYHST_STATIC_SCRATCH_BYTES returns PYHST_ENOMEM, with the sizes in
 * pyhst_last_error(), and enqueues nothing; out == NULL only sets
 * a->work_bytes.  The call allocates nothing and never synchronises.  Every
 * call on one device shares that device's array, which keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on one
 * device (other streams, other threads) race and give undefined results. */
enum { PYHST_STATIC_SCRATCH_BYTES = 64 << 20 };
int reconstruct_slices_static(const pyhst_plan *plan, pyhst_recon_args *a, hipStream_t stream);

/* Operator norm that the iterative methods of reconstruct_slices take as
 * op_norm (uniform plans): with_grad = 0: |A|; with_grad != 0: |[A; mu grad]|
 * (mu <= 0 means 1), by 50 power iterations on A^T A (+ mu^2 grad^T grad) of
 * the whole batch from a constant image, times 1.02 so that
 * tau sigma |K|^2 < 1 holds.  *norm (host) receives the estimate.  work:
 * device scratch; work == NULL returns its size in *work_bytes (nothing is
 * enqueued).  The call synchronises the stream (the result is a host value);
 * non-finite or zero estimate -> PYHST_ENUM. */
int pyhst_opnorm(const pyhst_plan *plan, int32_t with_grad, double mu, void *work, size_t *work_bytes, double *norm,
                 hipStream_t stream);

/* Data consistency per slice: rel[s] = |ax_s - y_s| / |y_s| over slice s's
 * sinogram (packed [K][n_det] layout of the plan; FP64 accumulation, one
 * workgroup per slice).  Used to send slices whose corrected reconstruction
 * does not explain the data to the TV-regularised mode. */
int pyhst_slice_residual(const pyhst_plan *plan, const float *ax, const float *y, float *rel, hipStream_t stream);

/* Choice of the regularisation weight beta of eq. (3) (section 3.1, the
 * estimators evaluated after reconstructing at several beta):
 *
 * Cross-validation estimator for one excluded projection k: err[s] =
 * |(A x_s)_k - y_s,k|^2, the squared distance between the projection at angle
 * k of reconstruction x_s (made from the data without projection k, on a plan
 * of the same image size) and the measured row k.  plan: the full plan (all
 * projections; uniform), which supplies angle k, its axis shift and the
 * layout of y [packed K x n_det].  x [packed n_y x n_x]; row: device scratch of
 * n_slices * n_det floats (receives (A x)_k - y_k); err: device [n_slices]
 * receives weight * |(A x_s)_k - y_s,k|^2, added to its previous value when
 * accumulate != 0 (the average over several excluded projections: weight =
 * 1/count, accumulate from the second one on).  k outside [0, K) or
 * non-finite weight -> PYHST_EARG.  FP64 sum of the squares. */
int pyhst_cv_error(const pyhst_plan *plan, const float *x, const float *y, int32_t k, float *row, float *err,
                   float weight, int32_t accumulate, hipStream_t stream);

/* Decoherence estimator E_cohe of section 3.1: e[s] = cos(x_beta - x_zero,
 * x_beta) per slice, where x_zero is the reconstruction at a very small beta
 * (FP64 sums; 0 when either vector is zero).  Images [packed n_y x n_x];
 * e: device [n_slices]. */
int pyhst_decoherence(const pyhst_plan *plan, const float *x_beta, const float *x_zero, float *e, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Overlapping-patch dictionary prior (section 3.2, eqs. (4)-(9)): the image is
 * x_i = sum_k w_kp phi_k(i - r_p) taken from the patch p whose core contains i,
 * and the coefficients minimise (eq. (8))
 *   |y - Pi x|^2 + rho sum_p sum_{i in p} (x_i - sum_k w_kp phi_k(i - r_p))^2 + beta |w|_1
 * by n_iter ISTA (fast = 0) or FISTA (fast = 1) steps on w with step 1/lipschitz
 * and soft threshold beta/lipschitz, from w = 0; the gradient is eq. (9).
 * Patches: m x m, corners every `stride` pixels per axis (the last at n - m),
 * p = row-corner index * (column corners) + column-corner index; cores: the
 * L1-nearest patch centre, lowest index on ties.  Pi is the plan's projector A
 * (identity = 0; y [packed K x n_det]) or the identity (identity = 1, image
 * denoising; y [packed n_y x n_x]); uniform plans only.
 *   dict [n_atoms][m*m] device, row k = atom phi_k (row-major patch);
 *   w    device [n_slices][n_patches][n_atoms] (receives the coefficients);
 *   out  device [packed n_y x n_x] (the image of eq. (7));
 *   lipschitz: step 1/lipschitz, must be > 0 (pyhst_patch_lipschitz estimates it);
 *   energy (device [n_iter] or NULL): eq. (8) after every iteration, summed over the batch.
 * Query: w == NULL returns work_bytes and n_patches (nothing is enqueued).  The
 * call only enqueues work (the patch tables and the transposed dictionary are
 * built by kernels of the same sequence), so it can be captured in a HIP graph. */
typedef struct {
    const float *y;
    const float *dict;
    int32_t m, stride, n_atoms;
    float rho, beta;
    int32_t n_iter, fast, identity;
    double lipschitz;
    float *w;
    float *out;
    float *energy;            /* device [n_iter] or NULL */
    void *work;
    size_t work_bytes;
    int32_t n_patches;        /* out */
} pyhst_patch_args;

int pyhst_patch_fista(const pyhst_plan *plan, pyhst_patch_args *args, hipStream_t stream);

/* Lipschitz constant of eq. (9)'s gradient map for the problem in args (y,
 * w, out, energy, n_iter unused; work as for pyhst_patch_fista): 60 power
 * iterations from a hashed start vector, times 1.02, written to
 * args->lipschitz.  Synchronises the stream (the result is a host value);
 * non-finite or zero estimate -> PYHST_ENUM. */
int pyhst_patch_lipschitz(const pyhst_plan *plan, pyhst_patch_args *args, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned sparse-angle corrector (not part of the paper, whose learned prior
 * is an overlapping-patch dictionary, section 3.2): a U-Net applied to FBP
 * slices as x_hat = x + f(x).  `levels` resolution levels (the last one is the
 * bottleneck), base*2^l channels at level l, two 3x3 conv + ReLU per level,
 * 2x2 max-pool down, 2x2 stride-2 transposed conv + ReLU up, skip
 * concatenation [encoder | upsampled], 1x1 linear head.  BF16 activations and
 * weights, FP32 accumulation (MFMA), FP32 master weights and Adam moments.
 * Flat FP32 parameter order: per level l = 0..levels-1 the two encoder convs,
 * then per level l = levels-2..0 the transposed conv and the two decoder
 * convs, then the head; each layer stores its weights then its bias.  Conv
 * weights are [c_out][3 ty + tx][c_in] (the first conv has c_in = 8, of which
 * only channel 0 carries the image), transposed-conv weights [2 dy + dx][c_out][c_in],
 * head weights [base] then one bias.
 * Inputs/targets: device FP32 [n][height][width], n <= batch.  The network
 * object owns its activation, gradient and optimizer buffers (allocated once
 * at creation); later calls allocate nothing and only enqueue on `stream`. */
typedef struct pyhst_unet pyhst_unet;
int pyhst_unet_create(int32_t batch, int32_t height, int32_t width, int32_t base, int32_t levels,
                      pyhst_unet **out);
int pyhst_unet_destroy(pyhst_unet *net);
int pyhst_unet_num_params(const pyhst_unet *net, int64_t *n);
/* Data scale c (> 0, default 1; it belongs with the trained weights): the
 * network sees c x and returns x_hat = x + f(c x)/c; training compares
 * c x + f(c x) with c target (loss in those units).  Non-positive or
 * non-finite c -> PYHST_EARG. */
int pyhst_unet_set_scale(pyhst_unet *net, float scale);
int pyhst_unet_get_scale(const pyhst_unet *net, float *scale);
/* Load master weights (device FP32 [n_params]); resets the Adam state. */
int pyhst_unet_set_params(pyhst_unet *net, const float *params, hipStream_t stream);
int pyhst_unet_get_params(const pyhst_unet *net, float *params, hipStream_t stream);
/* Gradients of the last pyhst_unet_backward (device FP32 [n_params]). */
int pyhst_unet_get_grads(const pyhst_unet *net, float *grads, hipStream_t stream);
/* Inference: out = x_hat for the n inputs (device FP32 [n][height][width]).
 * The output head runs in the epilogue of the last decoder convolution, the
 * first encoder convolution inside the second one's kernel, and the
 * up-sampling of every decoder level whose first convolution has at most 32
 * channels per concatenated half and 32 outputs inside that convolution, so
 * this call stores none of those activations (pyhst_unet_tensor kind 5 and
 * kind 1 at level 0, the up half of kind 2 at those levels, and the 8-channel
 * input, kind 0, hold them after pyhst_unet_backward only). */
int pyhst_unet_forward(pyhst_unet *net, const float *in, int32_t n, float *out, hipStream_t stream);
/* Forward, mean-squared-error loss against target (device float *loss, may be
 * NULL) and backward into the gradient buffer. */
int pyhst_unet_backward(pyhst_unet *net, const float *in, const float *target, int32_t n, float *loss,
                        hipStream_t stream);
/* Adam step (bias-corrected) on the stored gradients, then refresh of the BF16 weight copies. */
int pyhst_unet_adam(pyhst_unet *net, float lr, float beta1, float beta2, float eps, hipStream_t stream);
/* backward + Adam (beta1 0.9, beta2 0.999, eps 1e-8). */
int pyhst_unet_train_step(pyhst_unet *net, const float *in, const float *target, int32_t n, float lr, float *loss,
                          hipStream_t stream);

/* Inspection: copy an internal BF16 activation (grad = 0) or activation
 * gradient (grad = 1) into dst (device, `elems` uint16 values = batch x H_l x
 * W_l x channel stride).  kind: 0 input (8 channels), 1 encoder conv-a output
 * of `level`, 2 concatenation [encoder conv-b output | upsampled] of `level`,
 * 3 pooled encoder output of `level`, 4 / 5 decoder conv-a / conv-b output of
 * `level`, 6 bottleneck conv-b output. */
int pyhst_unet_tensor(const pyhst_unet *net, int32_t kind, int32_t level, int32_t grad, uint16_t *dst,
                      int64_t elems, hipStream_t stream);

/* Roofline measurement kernels (not part of the reconstruction path).
 * kind 0: independent FP32 FMA chains, 8 lane-ops per thread and iteration;
 * kind 1: the backprojector's per-update VALU sequence without LDS, 8 updates x
 *         8 lane-ops per thread and iteration;
 * kind 2: LDS ds_read_b64 in a conflict-free pattern, 8 x 8 bytes per thread
 *         and iteration;
 * kind 3: LDS ds_read_b128 in a conflict-free pattern, 8 x 16 bytes per thread
 *         and iteration;
 * kind 4: as kind 3 with consecutive lanes 1.25 entries apart (the projector's
 *         spread of reads along a line);
 * kind 5 / 6: as kind 3 with only the even lanes / lanes 0..31 active
 *         (8 x 16 bytes per active thread and iteration).
 * blocks x 256 threads; sink: device float buffer of blocks*256 elements (only
 * written if a result takes an impossible value, which keeps the work live). */
int pyhst_microbench(int32_t kind, int32_t blocks, int32_t iters, float *sink, hipStream_t stream);

const char *pyhst_strerror(int code);
const char *pyhst_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PYHST_H */

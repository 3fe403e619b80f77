/*
 * fzp.h - C ABI of the MI355X stripe-CZT Fresnel zone plate propagator.
 *
 * The library evaluates the focal-plane field of a full, unscaled, 2-D
 * binary-amplitude (or L-level phase) Fresnel zone plate (FZP) on a fixed region of interest
 * (ROI), by the separable chirp-z transform of the paper's CZT method
 * (Sec. 2.6, Eqs. 9-10; Sec. 3.3, Fig. 2; revised GPU engine, Sec. 6, Fig. 18):
 *
 *   U(x'_q, y'_p) = e^{ikz}/(i lambda z) e^{i pi (x'_q^2 + y'_p^2)/(lambda z)} dx^2
 *                   sum_{j,i} t_ji e^{i phi_ji} e^{i pi (x_i^2 + y_j^2)/(lambda z)}
 *                             e^{-2 pi i (x_i x'_q + y_j y'_p)/(lambda z)}        (Eq. 2)
 *
 * with x_i = (i - (N-1)/2) dx, x'_q = x0 + (q - M/2) dx_out, dx_out = 2 hw / M,
 * and the binary zone mask t_ji of Sec. 2.2 (paraxial radii r_n^2 = n lambda0 f0,
 * Eq. 4): with the exact integer K = (2i-N+1)^2 + (2j-N+1)^2 = 4 r^2/dx^2 and the
 * float64 constant kappa = dx*dx / (4*lambda0*f0), a sample is open iff
 * K <= K_max (inside the aperture disc; K_max = N^2 for the default pitch D/N,
 * floor((D/pitch)^2) otherwise) and floor(K*kappa) is odd (even when
 * centre_open is set); an L-level phase plate (fzp_aperture_t.levels) instead
 * passes every disc sample with t = exp(-2 pi i l / L).  phi = 2 pi h / lambda is an optional phase screen of
 * straight Gaussian creases, h = sum_k H_k exp(-d_k^2/(2 sigma_k^2)),
 * d_k = x cos(theta_k) + y sin(theta_k) - rho_k, sigma_k = width_k/(2 sqrt(2 ln 2)).
 * The N x N aperture is never stored: every stripe of rows is generated on the
 * device from these formulas.
 *
 * Conventions
 *  - Lengths in metres, angles in radians.
 *  - Complex buffers are interleaved (re, im) float64.  The ROI of instance k is
 *    row-major [y = p][x = q], M_k x M_k complex, starting at complex element
 *    fzp_roi_offset(plan, k) of the caller's ROI buffer.
 *  - Device buffers (workspace, ROI) are owned by the caller (allocated through
 *    PyTorch in the Python binding).  A plan owns host memory only; its device
 *    tables live in the caller's workspace.
 *  - All device work is enqueued on the caller's HIP stream (hipStream_t passed
 *    as void*; NULL is the null stream).  A plan may be used by one stream at a
 *    time.  fzp_metrics synchronises the stream before it returns.
 *  - Every call returns a status and never aborts; no C++ exception crosses the
 *    ABI.  fzp_last_error() gives a thread-local message for the last non-OK
 *    status.  A device fault surfaces as FZP_E_DEVICE on the next call that
 *    synchronises.
 *  - Determinism: no float atomics anywhere; both paths are bit-reproducible
 *    run to run for the same plan options.
 */
#ifndef FZP_H
#define FZP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fzp_plan_s *fzp_plan_t;

typedef int32_t fzp_status_t;
#define FZP_OK 0
#define FZP_E_INVAL (-1)       /* an argument is out of range, not finite or NULL */
#define FZP_E_SAMPLING (-2)    /* pitch coarser than the Nyquist limit of Eq. 6 */
#define FZP_E_NOMEM (-3)       /* workspace larger than the caller's limit */
#define FZP_E_DEVICE (-4)      /* a HIP call failed */
#define FZP_E_UNSUPPORTED (-5) /* valid, but outside what the library handles */

/* Evaluation path of the two CZT passes (Eqs. 9-10). */
#define FZP_PATH_FP64_BLUESTEIN 0 /* Bluestein CZT per row and per ROI column, float64
                                     throughout (Sec. 2.6) */
#define FZP_PATH_SPLIT_BF16 1     /* both passes as BF16 MFMA complex GEMMs (stripe . A_x^T,
                                     then B_y . T) with hi/lo split operands and float32
                                     accumulation; phases, the sums over K segments and
                                     chunks and the ROI in float64 */
#define FZP_PATH_AUTO 2           /* fzp_plan picks one of the two by the crossover measured on
                                     MI355X: split when every M is a multiple of 16 and the
                                     largest M is at most 1024 (binary plate, or crease-free
                                     2-level phase plate), 256 (creased amplitude plate, or
                                     crease-free 4-level phase plate), 128 (other phase
                                     plates); twice these with FZP_FLAG_SPLIT_INT8, whose row
                                     pass takes half the matrix-core time (measured faster than
                                     the FP64 path at binary M = 1024, creased M of 256 .. 1024
                                     (mean ~600), 4-level M = 512 and 8- and 16-level M = 256,
                                     slower at 8-level M = 512), the flag being dropped when the
                                     FP64 path is chosen; fzp_plan_info reports the choice */
#define FZP_PATH_SA_CZT 3         /* non-paraxial variant, the semi-analytical chirp-z transform
                                     (Sec. 3.6, Fig. 5): the amplitude plate with the sag-corrected
                                     radii of Eq. 3 centred in a zero-padded grid of Np >= 1.5 N
                                     samples per side; its 2-D FFT times exp(i h(K) z), the
                                     remainder of the exact transfer function exp(i k_z z),
                                     k_z = sqrt(k0^2 - K^2), after the quadratic
                                     c k_max + d K^2 / k_max fitted at K = 0 and K = k_max = 2 k0 / 3
                                     (Sec. 3.4, Fig. 3), back to space; then the quadratic part as a
                                     chirp-z zoom onto the ROI with Z = 4 pi |d| z / k_max in place
                                     of lambda z, prefactor e^{i k0 z} / (i Z) e^{i pi (x'^2+y'^2)/Z}.
                                     Float64 throughout; the padded field (Np^2 x 16 bytes) is in the
                                     workspace.  Whole apertures only: a partial row range is
                                     FZP_E_UNSUPPORTED.  Amplitude plates (levels = 0), creases
                                     allowed, one lane. */

/* Plan flags. */
#define FZP_FLAG_ALLOW_UNDERSAMPLED 1 /* skip the Eq. 6 check (tests on tiny grids) */
/* Split path, binary stripes: the GEMM variant a plan starts with (fzp_autotune may
 * change it).  Without a variant flag: variant 4, the 512-row tile (one work-group per
 * compute unit) with an 8-stage LDS pipeline and the mask expansion interleaved with
 * the MFMAs. */
#define FZP_FLAG_BIN_TILE_256 2       /* variant 1: 256-row tile, two work-groups per compute unit */
#define FZP_FLAG_BIN_SHALLOW 4        /* variant 0: 512-row tile with a 4-stage LDS pipeline */
#define FZP_FLAG_BIN_PREFETCH 8       /* variant 3: variant 2 reading the next stage's first
                                         operand fragments one stage early */
#define FZP_FLAG_BIN_DEEP 32          /* variant 2: 512-row tile with an 8-stage LDS pipeline */
#define FZP_FLAG_CPLX_TILE_128 128    /* split path, complex stripes: start with the 128-column GEMM
                                         tile instead of the 256-column one (same results bit for
                                         bit; fzp_autotune may change it) */
#define FZP_FLAG_CPLX_TILE_DUAL 256   /* as FZP_FLAG_CPLX_TILE_128 with a 2-stage LDS ring and two
                                         work-groups per compute unit */
#define FZP_FLAG_PARAXIAL_RADII 64    /* FZP_PATH_SA_CZT: the paraxial radii of Eq. 4 (r_n^2 = n
                                         lambda0 f0) instead of Eq. 3, e.g. to compare with the
                                         Fresnel paths */
#define FZP_FLAG_SPLIT_INT8 1024      /* split path: the row pass on the int8 matrix cores, the
                                         kernel row (and a complex stripe: creases, L-level
                                         plates) in fixed point of step 1/16256, two int8 digits,
                                         exact int32 sums per K segment: half the BF16 split's
                                         matrix-core work; quantisation error <= 3.1e-5 per element
                                         (the BF16 pair rounds to ~4e-6), and for complex stripes
                                         the digit-1 x digit-1 product (<= 1.5e-5) left out;
                                         FZP_E_UNSUPPORTED on the FP64 or SA-CZT path */
#define FZP_FLAG_OVERLAP_OPERAND 16   /* split path: make each chunk's stripe operand on an internal
                                         auxiliary stream one chunk ahead of its GEMM (two operand
                                         buffers); not under stream capture: fzp_graph_create,
                                         or a call on a capturing stream, returns
                                         FZP_E_UNSUPPORTED for such a plan */

typedef struct {
  double D;          /* aperture diameter */
  double f0;         /* design focal length */
  double lambda0;    /* design wavelength (zone radii r_n^2 = n lambda0 f0) */
  double pitch;      /* sample pitch; 0 means D / N */
  int64_t N;         /* samples per side, 1 .. 2^24 (FZP_PATH_SA_CZT: padded grid up to 2^20) */
  int32_t centre_open; /* amplitude plates: 0 central zone opaque (odd zones open), 1 central
                          zone open; must be 0 for phase plates */
  int32_t levels;      /* 0: binary amplitude plate (Sec. 2.2).  2 .. 64: L-level phase plate
                          (the revised engine's element, Fig. 18 stage 3): on the whole disc
                          the transmission is exp(-2 pi i l / L), l = floor(K kappa_L) mod L,
                          kappa_L = kappa * (L / 2), kappa = pitch^2 / (4 lambda0 f0), the ideal
                          lens phase -pi r^2 / (lambda0 f0) quantised into L steps per period */
} fzp_aperture_t;

typedef struct {
  double theta;  /* ridge direction normal angle */
  double offset; /* signed distance of the ridge line from the axis */
  double width;  /* ridge FWHM */
  double height; /* ridge optical path difference */
} fzp_crease_t;

typedef struct {
  double lambda;     /* wavelength */
  double z;          /* propagation distance; 0 means the first-order focus f0*lambda0/lambda */
  double x0, y0;     /* ROI centre */
  double half_width; /* ROI half width; 0 means 8*lambda*z/D */
  int32_t M;         /* ROI samples per side, 2 .. 2048 */
  int32_t n_creases; /* 0 .. 64 */
  const fzp_crease_t *creases; /* host array of n_creases, copied by fzp_plan */
} fzp_instance_t;

typedef struct {
  int32_t path;         /* FZP_PATH_* */
  int32_t stripe_rows;  /* rows per stripe, the row-pass work unit; 0 = path default */
  int64_t chunk_rows;   /* rows transformed between two column passes (values above N
                           are taken as N); 0 = automatic: the
                           row-pass partial sums near 1 GiB (split) or 0.5 GiB (FP64); for
                           creased instances on the split path the complex stripe planes
                           near 2 GiB, grown up to 8 GiB while the GEMM grid of the
                           smallest ROI has fewer than 512 tiles */
  uint64_t workspace_limit; /* bytes; 0 = no limit.  fzp_plan fails with FZP_E_NOMEM
                               if the workspace would exceed it */
  int32_t flags;        /* FZP_FLAG_* */
  int32_t lanes;        /* instances propagated concurrently, each lane on its own
                           internal stream with its own stripe buffers (the workspace
                           grows by one set of stripe buffers per lane); 0 = 1, at most 8 */
  double pad;           /* FZP_PATH_SA_CZT: padded grid Np = the smallest 2^a 3^b 5^c >= pad N
                           with the parity of N; 0 = 1.5 (the paper's pad), else 1 .. 8 */
} fzp_options_t;

/* Main-lobe metrics of one instance (shared metric extractor, Sec. 3.3 stage 4
 * and Fig. 18 stage 5).  fwhm_* come from a not-a-knot cubic spline through the
 * ROI row (column) holding the brightest sample; de is the power inside
 * r_null = j_{1,1}/pi * lambda z / D around the ROI centre over
 * p_in = (#samples in the disc) dx^2; mtf_half_cut is the radially averaged
 * |FFT2(I)|/|FFT2(I)|(0) at nu_cut/2, nu_cut = D/(lambda z); strehl is
 * i_peak / (pi R^2/(lambda z))^2. */
typedef struct {
  double fwhm_x, fwhm_y, de, mtf_half_cut, strehl, i_peak, p_in, p_lobe;
} fzp_metrics_t;

/* Validate the aperture, the n_inst instances and the options, and build a plan
 * (grids, CZT parameters of Eq. 10, workspace layout).  Host only; no device
 * call.  Errors: FZP_E_INVAL (NULL or out-of-range argument), FZP_E_SAMPLING
 * (pitch > lambda0 f0 / (2 D), Eq. 6, unless FZP_FLAG_ALLOW_UNDERSAMPLED),
 * FZP_E_NOMEM (workspace over options->workspace_limit), FZP_E_UNSUPPORTED. */
fzp_status_t fzp_plan(const fzp_aperture_t *ap, const fzp_instance_t *inst, int32_t n_inst,
                      const fzp_options_t *opt, fzp_plan_t *out);

/* Bytes of device workspace the plan needs (tables + stripe buffers + metric
 * scratch).  The caller allocates it (256-byte aligned). */
fzp_status_t fzp_plan_workspace_size(fzp_plan_t p, size_t *bytes);

/* Total ROI buffer length in complex elements (sum over instances of M^2), and
 * the offset of instance k inside it. */
fzp_status_t fzp_roi_elements(fzp_plan_t p, int64_t *n_complex);
fzp_status_t fzp_roi_offset(fzp_plan_t p, int32_t k, int64_t *offset_complex);

/* Build the plan's device tables (Bluestein chirps and filter spectra, the
 * split-path kernel matrices A_x and B_y) inside `workspace`.  Asynchronous on `stream`.
 * fzp_propagate_roi calls it itself when given a workspace it has not seen. */
fzp_status_t fzp_prepare(fzp_plan_t p, void *workspace, void *stream);

/* Propagate every instance of the plan: roi_dev receives U (Eq. 2) for all
 * aperture rows.  Asynchronous on `stream`. */
fzp_status_t fzp_propagate_roi(fzp_plan_t p, void *workspace, double *roi_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fzp_propagate_roi with the workspace taken from a device array that the
 * library holds, FZP_STATIC_SCRATCH_BYTES per GPU from the first call on that
 * GPU until the process ends.  The caller passes the plan and the ROI buffer
 * (as for fzp_propagate_roi) and nothing else; the call allocates no device
 * memory and creates no stream or event: every instance runs on `stream` in
 * one lane (the same bits as fzp_propagate_roi), without kernel timing or the
 * operand overlap.  The plan's tables are built in the array unless the last
 * successful call on this GPU used the same plan (the array keeps the last
 * call's contents).  All calls on one GPU share the array: calls that overlap
 * in time on one GPU (other threads, other streams) race and give undefined
 * results.  Errors: FZP_E_INVAL (NULL argument), FZP_E_NOMEM (the plan's
 * fzp_plan_workspace_size exceeds FZP_STATIC_SCRATCH_BYTES; checked before any
 * device call: plan with fewer chunk_rows, instances or ROI samples),
 * FZP_E_DEVICE. */
#define FZP_STATIC_SCRATCH_BYTES (64u << 20)
fzp_status_t fzp_propagate_roi_static(fzp_plan_t p, double *roi_dev, void *stream);

/* Contribution of aperture rows row_begin .. row_end-1 only (0 <= begin <= end
 * <= N).  With accumulate = 0 the ROI is overwritten, otherwise added to.  The
 * contributions of a partition of [0, N) into ranges that start on multiples of
 * the plan's chunk_rows add up bit-for-bit to fzp_propagate_roi (resume after
 * interruption; one GPU's share of a multi-GPU run). */
fzp_status_t fzp_propagate_roi_range(fzp_plan_t p, void *workspace, double *roi_dev,
                                     int64_t row_begin, int64_t row_end, int32_t accumulate,
                                     void *stream);

/* Resumable whole-aperture propagation with a checkpoint file on the host (the
 * paper's long runs stream row chunks through files and skip verified groups on
 * restart, Fig. 18 stage 2; here only the M x M float64 ROI and the next row are
 * kept).  The rows run in blocks of rows_per_checkpoint (0: one chunk; rounded
 * up to whole chunks, so the blocks end where the chunks of fzp_propagate_roi
 * end); after each block the ROI buffer and the next row go to `path` (written
 * as path + ".tmp", then renamed).  When `path` exists and carries this plan's
 * fingerprint (aperture, instances, path, chunk, K-segment length and GEMM
 * variant), the ROI is restored from it and the rows continue where it left
 * off, so the finished ROI is bit for bit the one fzp_propagate_roi gives.
 * max_rows > 0 stops after the first block that reaches max_rows rows in this
 * call (a time-sliced run); *next_row (may be NULL) receives the row where the
 * next call starts, N when the aperture is complete.  On completion the file
 * is removed unless keep != 0.  Synchronous on `stream`.  Errors: FZP_E_INVAL
 * for a checkpoint of another plan or a malformed file (the file is left in
 * place), FZP_E_DEVICE when a file cannot be written. */
fzp_status_t fzp_propagate_resumable(fzp_plan_t p, void *workspace, double *roi_dev,
                                     const char *path, int64_t rows_per_checkpoint,
                                     int64_t max_rows, int32_t keep, int64_t *next_row,
                                     void *stream);

/* Metrics of every instance from roi_dev (as written by fzp_propagate_roi),
 * computed on the device; out_host receives n_inst records.  Synchronises
 * `stream`.  Instances with M not a power of two in 8 .. 4096 get NaN MTF. */
fzp_status_t fzp_metrics(fzp_plan_t p, void *workspace, const double *roi_dev,
                         fzp_metrics_t *out_host, void *stream);

/* Plan facts for reporting: FFT length L, Bluestein block B, rows per chunk,
 * stripe rows, path, samples in the aperture disc, and the float64 zone
 * constant kappa.  Any pointer may be NULL. */
fzp_status_t fzp_plan_info(fzp_plan_t p, int32_t *fft_len, int32_t *block, int64_t *chunk_rows,
                           int32_t *stripe_rows, int32_t *path, int64_t *disc_samples,
                           double *kappa);

/* Grid rule of the revised engine (Fig. 18 stage 1), the sampling of the
 * paper's meter-class runs (Tables 1-4): the zone period at the rim
 * Lambda_edge = lambda0 f0 / R (R = D/2) sampled s_samp times per phase step,
 * pitch = Lambda_edge / (s_samp max(L, 2)), N = ceil(D / pitch) made odd (an
 * axis sample).  levels 0 (amplitude plate) counts as L = 2; s_samp 0 = 4.
 * Host only.  Errors: FZP_E_INVAL. */
fzp_status_t fzp_grid_for_element(double D, double f0, double lambda0, int32_t levels, int32_t s_samp,
                                  double *pitch, int64_t *N);

/* Geometry of a plan.  zones_exact is the real root n of Eq. 3 at r = D/2,
 * (lambda0^2/4) n^2 + lambda0 f0 n = (D/2)^2, and total_zones its floor (the zone
 * count of Fig. 2 stage 2, reported for every path).  For FZP_PATH_SA_CZT:
 * padded_n = Np, fft_n1 x fft_n2 = Np (the two LDS transform lengths of each
 * axis) and zoom_distance = Z / lambda of instance k (the distance of the
 * zoom's Fresnel-type transform); 0 otherwise.  Errors: FZP_E_INVAL. */
typedef struct {
  double zones_exact;
  int64_t total_zones;
  int64_t padded_n;
  int32_t fft_n1, fft_n2;
  double zoom_distance;
} fzp_geometry_t;
fzp_status_t fzp_plan_geometry(fzp_plan_t p, int32_t k, fzp_geometry_t *out);

/* Kernel timing.  While enabled, every kernel launch of
 * fzp_propagate_roi(_range) - row pass, column pass, and (split path) the
 * zone-mask bit kernel - is bracketed by its own pair of HIP events recorded
 * on the caller's stream, so each interval covers exactly that kernel.
 * fzp_profile_read waits for the recorded events and returns the accumulated
 * milliseconds and launch counts per kind since the last reset (reset != 0
 * clears them).  Any output pointer may be NULL. */
fzp_status_t fzp_profile_enable(fzp_plan_t p, int32_t on);
fzp_status_t fzp_profile_read(fzp_plan_t p, double *row_ms, int64_t *row_launches, double *col_ms,
                              int64_t *col_launches, double *mask_ms, int64_t *mask_launches, int32_t reset);

/* Batched execution.  fzp_graph_create records one whole fzp_propagate_roi of
 * the plan (every instance, every chunk, all lanes forked from and joined back
 * to one stream) into a HIP graph bound to `workspace` and `roi_dev`, which
 * must stay allocated while the graph lives; fzp_graph_launch replays it on
 * `stream` as one launch.  The workspace is prepared first (synchronously).
 * Kernel timing (fzp_profile_*) is not recorded inside a graph.  Errors:
 * FZP_E_INVAL, FZP_E_DEVICE, FZP_E_UNSUPPORTED (a split plan with
 * FZP_FLAG_OVERLAP_OPERAND; checked before any device call). */
typedef struct fzp_graph_s *fzp_graph_t;
fzp_status_t fzp_graph_create(fzp_plan_t p, void *workspace, double *roi_dev, fzp_graph_t *out);
fzp_status_t fzp_graph_launch(fzp_graph_t g, void *stream);
void fzp_graph_destroy(fzp_graph_t g);

/* Autotuner of the split path's GEMM work decomposition.  Candidates are the
 * K-segment length of a work-group tile (the plan's default and its doublings
 * up to 65536 columns; longer segments mean fewer float32 partial planes for
 * the column pass but fewer independent tiles), the binary-stripe GEMM variant
 * (0: 512-row tile, one work-group per compute unit, 4-stage LDS pipeline;
 * 1: 256-row tile, two work-groups per compute unit; 2: 512-row tile with an
 * 8-stage pipeline; 3: variant 2 with the next stage's first operand fragments
 * read one stage early; 4: variant 2 with the mask expansion interleaved with the
 * MFMAs), for complex stripes the GEMM tile (256 or 128 real columns, the latter
 * also with two work-groups per compute unit), and the
 * number of concurrent lanes (1 .. options.lanes).  The variant reported and
 * cached is the binary variant + 8 x the complex tile (0: 256, 1: 128, 2: 128 with
 * two work-groups per compute unit).  Each candidate runs one
 * full propagation on `stream`, timed with HIP events; the fastest is kept in
 * the plan.  With a non-NULL `cache_path` the choice is looked up first in
 * that text file (one "key seg_len lanes variant" line per plan shape and
 * GPU) and appended when new.  `roi_dev` is overwritten.  The outputs
 * (segment, lanes, variant, and the winning time in ms, 0 when taken from
 * the cache) may be NULL.  The FP64 path has nothing to tune except lanes.
 * Errors: FZP_E_INVAL, FZP_E_DEVICE. */
fzp_status_t fzp_autotune(fzp_plan_t p, void *workspace, double *roi_dev, void *stream,
                          const char *cache_path, int64_t *seg_len_out, int32_t *lanes_out,
                          int32_t *variant_out, double *ms_out);

void fzp_destroy(fzp_plan_t p);

/* ------------------------------------------------------------------------
 * Learned surrogate.  The paper motivates full 2-D simulation by membrane
 * deformations (introduction) and gives no learned model; the library adds a
 * multilayer perceptron from crease parameters and the wavelength to the ROI
 * log-intensity, trained on the propagation's own outputs, with the CZT as
 * arbiter and fallback:
 *   z1 = W1 x + b1, h1 = silu(z1); z2 = W2 h1 + b2, h2 = silu(z2); y = W3 h2 + b3,
 *   silu(z) = z / (1 + e^{-z}),  loss = sum (y - t)^2 / (B n_out),
 * Adam updates (Kingma & Ba 2015, Algorithm 1; beta1 0.9, beta2 0.999,
 * eps 1e-8).  Parameters are one flat float32 vector W1 [H][n_in], b1 [H],
 * W2 [H][H], b2 [H], W3 [n_out][H], b3 [n_out] (row-major).  The products run
 * on the matrix cores with BF16 weights, activations and gradients and float32
 * accumulation; masters, moments, biases and the loss are float32.
 * Row-major device arrays: x [batch][n_in], t and y [batch][n_out],
 * dx [batch][n_in].  All calls are asynchronous on `stream`; none allocates
 * device memory (the caller's workspace holds everything).
 * ------------------------------------------------------------------------ */
typedef struct fzp_mlp_s *fzp_mlp_t;

/* Host only: sizes (n_in 1..4096, n_hidden 1..8192, n_out 1..2^20, batch_max
 * 1..65536); FZP_E_INVAL otherwise. */
fzp_status_t fzp_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch_max, fzp_mlp_t *out);
/* Workspace bytes (256-byte aligned buffer owned by the caller) and the
 * parameter count. */
fzp_status_t fzp_mlp_info(fzp_mlp_t m, size_t *workspace_bytes, int64_t *n_params);
/* Load parameters (device float32, n_params) into the workspace, refresh the
 * BF16 copies and reset the optimizer state; fzp_mlp_get_params copies them out. */
fzp_status_t fzp_mlp_set_params(fzp_mlp_t m, void *workspace, const float *params_dev, void *stream);
fzp_status_t fzp_mlp_get_params(fzp_mlp_t m, void *workspace, float *params_dev, void *stream);
/* y = network(x) for 1 <= batch <= batch_max rows. */
fzp_status_t fzp_mlp_forward(fzp_mlp_t m, void *workspace, const float *x_dev, int32_t batch, float *y_dev,
                             void *stream);
/* Forward, loss against t, and the gradients: grads_dev (n_params, the
 * parameter layout), dx_dev (may be NULL), loss_dev (one float, may be NULL);
 * y_dev receives the forward output.  No update. */
fzp_status_t fzp_mlp_backward(fzp_mlp_t m, void *workspace, const float *x_dev, const float *t_dev, int32_t batch,
                              float *y_dev, float *grads_dev, float *dx_dev, float *loss_dev, void *stream);
/* One training step: forward, backward, Adam update with learning rate lr
 * (the step counter lives in the model and restarts at fzp_mlp_set_params). */
fzp_status_t fzp_mlp_train_step(fzp_mlp_t m, void *workspace, const float *x_dev, const float *t_dev,
                                int32_t batch, float *y_dev, float lr, float *loss_dev, void *stream);
/* One Adam update from given gradients (device float32, n_params). */
fzp_status_t fzp_mlp_adam_update(fzp_mlp_t m, void *workspace, const float *grads_dev, float lr, void *stream);
void fzp_mlp_destroy(fzp_mlp_t m);

/* Training targets and back: out = ln(|U|^2 / i0 + floor) for n_complex ROI
 * samples (float32 out), and U = sqrt(max(i0 (e^y - floor), 0)) + 0i (float64
 * complex, so that fzp_metrics reads predicted intensities).  i0 > 0,
 * floor > 0. */
fzp_status_t fzp_log_intensity(const double *roi_dev, int64_t n_complex, double i0, double floor_, float *out_dev,
                               void *stream);
fzp_status_t fzp_field_from_log_intensity(const float *y_dev, int64_t n_complex, double i0, double floor_,
                                          double *roi_dev, void *stream);

/* Physics prior of the surrogate: the focal-plane intensity of a deformed
 * binary plate's first diffraction order treated as a thin lens with the
 * plate's pupil.  The Eq. 4 plate is periodic in s = r^2 / (lambda0 f0) (period
 * 2); its converging Fourier term has amplitude 1/pi, and at that term's focus
 * (lambda z = lambda0 f0) the Fresnel integral of Eq. 2 becomes a Fourier
 * transform of the pupil times the crease phase screen exp(2 pi i h / lambda)
 * (the creases of fzp_instance_t).  For each of n instances, on the M x M ROI
 * of a default instance at its focus (samples (q - M/2) 16 lambda0 f0 / (D M)):
 *   y[p][q] = ln(16 |S_pq|^2 / (pi^2 Np^4) + floor)   (I / I0 + floor,
 *             I0 = (R^2 / (lambda0 f0))^2, the undeformed peak),
 *   S = E g E^T,  g[j][i] = P_ij exp(2 pi i h(u_i, u_j) / lambda),
 *   u_i = (2 i + 1 - Np) D / (2 Np),  E[q][i] = exp(-2 pi i 4 (2i+1-Np)(2q-M) / (Np M)),
 * P_ij the share of the pixel's ss x ss sub-sample centres inside the disc.
 * The zero order and the defocused orders are not modelled (the surrogate's
 * network learns that remainder).  Phases and ridge heights in float64, the
 * pupil field, the transforms and y in float32. */
typedef struct {
  double D;          /* aperture diameter [m] (crease offsets and widths are in metres) */
  int32_t M;         /* ROI side, 1 .. 4096 */
  int32_t Np;        /* pupil grid side, 16 .. 1024, a multiple of 16 */
  int32_t ss;        /* sub-samples per pupil pixel side for the disc edge, 1 .. 16 */
  int32_t n_creases; /* creases per instance, 0 .. 64 */
  double floor_;     /* log floor relative to I0, > 0 */
} fzp_prior_t;
/* Workspace bytes (256-byte aligned, owned by the caller) for up to n_max
 * instances per call; FZP_E_INVAL for a bad configuration. */
fzp_status_t fzp_pupil_prior_workspace(const fzp_prior_t *cfg, int32_t n_max, size_t *bytes);
/* Device arrays: creases_dev [n][n_creases][4] float64 (theta, offset, width
 * (FWHM), height, as fzp_crease_t; NULL when n_creases = 0), lam_dev [n]
 * float64, y_dev [n][M][M] float32.  0 <= n <= 65535; FZP_E_NOMEM when
 * workspace_bytes is below fzp_pupil_prior_workspace(cfg, n).  Asynchronous on
 * `stream`; allocates nothing. */
fzp_status_t fzp_pupil_prior(const fzp_prior_t *cfg, const double *creases_dev, const double *lam_dev, int32_t n,
                             float *y_dev, void *workspace, size_t workspace_bytes, void *stream);

/* Batched FWHM of log-intensity maps y = ln(I / I0 + floor) (the surrogate's
 * form; y_dev [n][M][M] float32, 5 <= M <= 2048), for the surrogate's gate: per
 * map the brightest sample (first index on ties), the FWHM in samples along its
 * row by the metric extractor's spline (fzp_metrics' fwhm_x / pitch), and two
 * conditioning numbers that need no reference map: cond = (w(1/2 - d) -
 * w(1/2 + d)) / (2 d w(1/2)) with w(l) the full width at level l of the peak and
 * d = level_delta (0 < d < 0.25): about 1.5 for a clean core, large where a
 * shoulder or a secondary peak sits near half the maximum (+inf if a width is
 * undefined); ratio = the brightest sample farther than exclusion_radius
 * samples from the peak over the peak; gap = 1 - (brightest sample of the
 * brighter neighbouring row) / peak and walt = the FWHM in samples along that
 * row (a map whose brightest sample moves there reads walt; gap = 1 and walt =
 * NaN without a neighbouring row).  out_dev [n][5] float64 = (FWHM, cond,
 * ratio, gap, walt).  Asynchronous on `stream`; allocates nothing. */
fzp_status_t fzp_fwhm_batch(const float *y_dev, int32_t n, int32_t M, double floor_, double level_delta,
                            double exclusion_radius, double *out_dev, void *stream);

/* Thread-local message of the last non-OK status on this thread. */
const char *fzp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FZP_H */

/*
 * octmc.h -- C ABI of the MI355X (gfx950) implementation of orthogonal-raster
 * OCT/OCTA 3-D motion correction (Ploner et al., arXiv:2010.06931).
 *
 * Problem statement (Sec. 2.1): two raster scans of the same eye, one with
 * B-scans along x ("X-fast") and one along y ("Y-fast"), each w x h A-scans of
 * d samples, go in; one displacement vector per output A-scan and scan
 * (dx, dy, dz) and a merged volume come out.  The implementation is limited to
 * square scans (w == h, Sec. 5).
 *
 * Conventions shared by every call:
 *   - Volumes are [h][w][d] float32, row j (y), column i (x), depth k
 *     contiguous, both scans in the common (x, y) frame (a Y-fast scan is
 *     transposed by the caller).  En face images are [h][w] float32.
 *   - A displacement field ("disp") is [2][h][w][3] float32: scan V (0 = X-fast,
 *     1 = Y-fast), row j, column i, component (dx, dy, dz), in pixels of the
 *     pyramid level it belongs to.  Scan V's sample for output voxel (i, j, k)
 *     is taken at (i + dx, j + dy, k + dz) of its own volume (Eq. 2).
 *   - Every function returns an octmc_status: 0 on success, < 0 on error.
 *     Nothing throws across the ABI.  octmc_last_error() describes the last
 *     error of the calling thread.
 *   - Ownership: the caller owns every pointer it passes and the library never
 *     frees caller memory.  Device pointers must belong to the context's
 *     device.  Objects created by the library are freed by the matching
 *     *_destroy call.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  Device
 *     outputs are valid once that stream has completed the call's work; calls
 *     that return host values synchronise the stream themselves.
 *   - Asynchronous device faults surface at a later call as OCTMC_E_DEVICE.
 *   - Threading: one host thread per object (pair, multi) at a time.  An
 *     object holds one set of evaluation scratch buffers, so its asynchronous
 *     calls must also be ordered on the device: issue them on one stream, or
 *     synchronise between streams.
 */
#ifndef OCTMC_H
#define OCTMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(OCTMC_BUILD)
#define OCTMC_API __attribute__((visibility("default")))
#else
#define OCTMC_API
#endif

typedef enum {
    OCTMC_OK = 0,
    OCTMC_E_INVALID = -1, /* bad argument (NULL pointer, out-of-range parameter) */
    OCTMC_E_SHAPE = -2,   /* unsupported shape (w != h, too small for the pyramid, too large) */
    OCTMC_E_DTYPE = -3,   /* unknown storage type */
    OCTMC_E_OOM = -4,     /* device allocation failed / request can never fit */
    OCTMC_E_DEVICE = -5,  /* HIP runtime error */
    OCTMC_E_NAN = -6,     /* non-finite input with OCTMC_CHECK_NAN set */
    OCTMC_E_BUSY = -7     /* object in use */
} octmc_status;

/* Storage type of the structural volumes inside the library (the inputs are
 * always float32; they are rounded to nearest-even on ingest).  Arithmetic is
 * float32 in the kernels and float64 in every global reduction and in the
 * L-BFGS state. */
typedef enum { OCTMC_F32 = 0, OCTMC_BF16 = 1, OCTMC_F16 = 2 } octmc_dtype;

typedef enum { OCTMC_MEM_HOST = 0, OCTMC_MEM_DEVICE = 1 } octmc_mem;

/* flags */
#define OCTMC_CHECK_NAN 0x1u      /* scan the inputs for NaN/Inf at pair creation */
#define OCTMC_DETECT_INVALID 0x2u /* derive the B-scan validity from the OCTA volumes (Sec. 2.2) when
                                     octmc_pair_create gets OCTA volumes and no validity vectors */
#define OCTMC_ENFACE_PROJECT 0x4u /* form the en face OCTA images by the segmentation-free projection
                                     of Sec. 2.3 (octmc_enface_project) instead of the depth mean when
                                     octmc_pair_create gets OCTA volumes and no en face images */
#define OCTMC_PREALIGN 0x8u       /* octmc_pair_create first runs the stage-1 rough axial prealignment
                                     (octmc_prealign) and ingests the prealigned volumes */
#define OCTMC_MULTI_PAIRWISE 0x10u /* octmc_multi_*: evaluate the structural term pair by pair (each
                                     volume resampled once per pair it belongs to) instead of the
                                     fused form (each volume resampled once), which serves n = 3 or 4
                                     volumes */
#define OCTMC_HOST_LINE_SEARCH 0x20u /* octmc_register: take the L-BFGS decisions (history update,
                                       search direction, line-search steps) on the host, with a
                                       round trip after every dot-product pass and every trial
                                       evaluation.  Without it they are taken on the device by
                                       single-thread kernels in the same float64 operations, with
                                       the same result bit for bit, and the host enqueues several
                                       iterations ahead (lbfgs_m <= 6; the host form otherwise, and
                                       always for grouped serving).  Applies to octmc_register,
                                       octmc_multi_register and the stage-1 solve (octmc_prealign,
                                       OCTMC_PREALIGN) */

/* Parameters of the objective (Eq. 1 without the stage-1 tilt term) and of the
 * solver.  [P] = value fixed by the paper; [R] = a reading of a point the
 * paper leaves open. */
typedef struct {
    double alpha;        /* weight of the scan-order regulariser R (Eq. 1)       [R: 1.0]  */
    double delta0;       /* angiography weight of a valid A-scan (Eq. 8)          [P: 0.5]  */
    double eps_huber;    /* pseudo-Huber parameter of the data term (Eq. 4)       [P: 1e-3] */
    double eps_reg;      /* pseudo-Huber parameter of R, in pixels                [R: 0.1]  */
    double flyback_frac; /* flyback per B-scan, fraction of the B-scan length     [R: 0.25] */
    double mean_weight;  /* gamma_M of the mean-displacement term M               [R: 1.0]  */
    int32_t levels;      /* pyramid levels (factor 2, Sec. 2.1), 1..8; 0: automatic, the fewest
                            levels whose coarsest level is at most 16 A-scans wide [0]       */
    int32_t iters_per_level; /* accepted L-BFGS steps per level                   [100]     */
    int32_t lbfgs_m;     /* L-BFGS memory (1..8)                                  [R: 5]    */
    int32_t ls_max_evals;/* evaluations per line search                           [R: 20]   */
    double c1, c2;       /* strong Wolfe constants                                [R: 1e-4, 0.9] */
    double merge_kappa;  /* density weight decay exp(-kappa (rho - 1))            [R: 1.0]  */
    double merge_tau;    /* weights below tau are clipped to 0                    [R: 0.05] */
    uint32_t flags;      /* OCTMC_CHECK_NAN | OCTMC_DETECT_INVALID | OCTMC_ENFACE_PROJECT | OCTMC_PREALIGN |
                            OCTMC_MULTI_PAIRWISE | OCTMC_HOST_LINE_SEARCH */
    int32_t prealign_iters; /* stage-1 L-BFGS steps per level                     [100]     */
    double gamma_tilt;   /* weight of the tilt normalisation T (Eq. 1, stage 1)   [R: 1.0]  */
} octmc_params;
/* Choosing `levels`: the solve removes lateral motion between the scans well
 * when it is at most about one pixel at the coarsest level.  On synthetic
 * scans with 10-13 px of motion between them and 100 steps per level, a
 * coarsest level of 10-16 A-scans (6 levels at 300-500 A-scans) removed most
 * of it, where 38-63 A-scans (4 levels) left it in a local minimum.
 * levels = 0 chooses such a depth from the shape. */

typedef struct {
    int32_t w, h, d;   /* A-scans per row, rows, samples per A-scan; w == h */
    octmc_dtype dtype; /* storage type of the structural volumes */
    octmc_mem mem;     /* where the input pointers of octmc_pair_create live */
} octmc_shape;

/* Indices into the terms array written by octmc_eval (float64). */
enum {
    OCTMC_TERM_F = 0,     /* objective: data + alpha R + M                        (Eq. 1) */
    OCTMC_TERM_DATA = 1,  /* eta S_str + S_ang / eta                              (Eq. 9) */
    OCTMC_TERM_STR = 2,   /* S_str at delta0                                      (Eq. 6) */
    OCTMC_TERM_ANG = 3,   /* S_ang at delta0                                      (Eq. 7) */
    OCTMC_TERM_REG = 4,   /* R (not multiplied by alpha)                                  */
    OCTMC_TERM_MEAN = 5,  /* M                                                            */
    OCTMC_TERM_STR05 = 6, /* S_str at delta0 = 0.5 (for eta, Eq. 10)                      */
    OCTMC_TERM_ANG05 = 7, /* S_ang at delta0 = 0.5                                        */
    OCTMC_TERM_ETA = 8,   /* the eta the evaluation used                                  */
    OCTMC_TERM_GP = 9,    /* reserved (directional derivative inside the solver)          */
    OCTMC_NTERMS = 10
};

#define OCTMC_MAX_LEVELS 8

/* Per-level solve report, coarsest level first. */
typedef struct {
    int32_t nlevels;
    int32_t iters[OCTMC_MAX_LEVELS];
    int32_t evals[OCTMC_MAX_LEVELS];
    int32_t ls_fail[OCTMC_MAX_LEVELS];
    double eta[OCTMC_MAX_LEVELS];
    double f_start[OCTMC_MAX_LEVELS];
    double f_end[OCTMC_MAX_LEVELS];
} octmc_report;

typedef struct octmc_ctx octmc_ctx;
typedef struct octmc_pair octmc_pair;

/* Library version string (static storage). */
OCTMC_API const char* octmc_version(void);

/* Description of the calling thread's last error (valid until its next call). */
OCTMC_API const char* octmc_last_error(void);

/* Fill *out with the defaults listed in octmc_params. */
OCTMC_API int octmc_params_default(octmc_params* out);

/* Create a context bound to HIP device `device_ordinal`. */
OCTMC_API int octmc_create(int device_ordinal, octmc_ctx** out);
OCTMC_API int octmc_destroy(octmc_ctx* ctx);

/* Ingest one orthogonal scan pair (Sec. 2.1 input; pyramid of Sec. 2.1
 * "optimization"; validity of Sec. 2.2; en face images of Sec. 2.3/2.4).
 *   oct_x, oct_y       structural volumes [h][w][d] float32 (required);
 *   octa_x, octa_y     OCTA volumes [h][w][d] float32, or NULL; when given,
 *                      the en face images are their projections (Sec. 2.3,
 *                      with OCTMC_ENFACE_PROJECT, using oct_* for the OCT
 *                      mask and the validity below) or else their depth
 *                      means, unless enface_* are given; invalid B-scans are
 *                      replaced by their nearest valid neighbour for the
 *                      OCTA merge (Sec. 2.5);
 *   enface_x, enface_y en face OCTA images [h][w] float32, or NULL;
 *   valid_x[h], valid_y[w] B-scan validity (Sec. 2.2, 1 = valid), or NULL:
 *                      all valid, or with OCTMC_DETECT_INVALID and OCTA
 *                      volumes, derived from them as by
 *                      octmc_validity_from_octa.  X-fast B-scans are rows,
 *                      Y-fast columns.
 * Either both OCTA volumes or both en face images must be given.  With
 * OCTMC_PREALIGN the stage-1 prealignment (octmc_prealign, with delta0 = 0
 * and no en face images) runs first on the structural volumes; both
 * structural and both OCTA volumes are resampled axially with its field
 * (octmc_resample_axial) and the pair holds the prealigned volumes, so that
 * validity detection, projection, registration and merge work on them;
 * octmc_pair_prealignment returns the stage-1 result.  All input
 * pointers live in shape->mem memory.  The library copies every input into
 * its own device memory; the caller may free them once the call returns.
 * Errors: OCTMC_E_SHAPE (w != h, min(w, d) at the coarsest level < 4,
 * volume > 2^31 bytes), OCTMC_E_DTYPE, OCTMC_E_INVALID, OCTMC_E_OOM,
 * OCTMC_E_NAN (with OCTMC_CHECK_NAN), OCTMC_E_DEVICE. */
OCTMC_API int octmc_pair_create(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape,
                      const float* oct_x, const float* oct_y, const float* octa_x, const float* octa_y,
                      const float* enface_x, const float* enface_y, const float* valid_x,
                      const float* valid_y, void* stream, octmc_pair** out);
OCTMC_API int octmc_pair_destroy(octmc_pair* pair);

/* Input validity of one OCTA volume (Sec. 2.2): saccades saturate the
 * decorrelation of whole B-scans.  With m_b the mean of the volume over
 * B-scan b, and mu, sigma the mean and population standard deviation of m
 * over all B-scans, B-scan b is flagged if m_b > mu + 3 sigma; valid_out[b]
 * is 1 if none of the B-scans b-2 .. b+2 is flagged, else 0.
 *   shape      w, h, d of the volume and where `octa` lives (shape->mem);
 *              shape->dtype is ignored (the volume is float32);
 *   octa       [h][w][d] float32 in the common frame;
 *   scan       0: X-fast (B-scans are rows j, nb = h), 1: Y-fast (columns i, nb = w);
 *   valid_out  device float32[nb].
 * Synchronises `stream`.  Errors: OCTMC_E_INVALID, OCTMC_E_SHAPE (volume >
 * 2^31 bytes), OCTMC_E_OOM, OCTMC_E_DEVICE. */
OCTMC_API int octmc_validity_from_octa(octmc_ctx* ctx, const octmc_shape* shape, const float* octa, int32_t scan,
                                       float* valid_out, void* stream);

/* Segmentation-free en face OCTA projection (Sec. 2.3) of one scan:
 *   1. 3-D median filter of radius 1 of the OCTA volume;
 *   2. rank filters of width 15 keeping the 3rd smallest value, along the
 *      fast then the slow scan axis (x then y for X-fast, y then x for Y-fast);
 *   3. p5, p95 = 5th and 95th percentile of that filtered volume over the
 *      valid B-scans (all B-scans if none is valid; linear interpolation
 *      between order statistics), voxel mask: filtered < p5 + 0.1 (p95 - p5);
 *   4. OCT mask: oct > mean + 2 (population) standard deviations of the first
 *      max(1, round(0.05 d)) samples of every A-scan;
 *   5. en face value: mean of the OCTA samples in both masks along depth
 *      (0 where there is none);
 *   6. every B-scan's median is subtracted from it;
 *   7. invalid B-scans take the values of their nearest valid neighbour
 *      (the lower one on a tie).
 * Borders are clamped in every filter.  Selections are exact; thresholds and
 * means are formed in float64.
 *   shape      w, h, d of both volumes and where oct, octa and valid live
 *              (shape->mem); shape->dtype is ignored (float32 volumes);
 *              w, h <= 8192;
 *   oct, octa  [h][w][d] float32 in the common frame: structural and OCTA;
 *   scan       0: X-fast (B-scans are rows j), 1: Y-fast (columns i);
 *   valid      float32[nb] (nb = h for X-fast, w for Y-fast; 1 = valid) or
 *              NULL: all valid;
 *   fixed      host double[2] {p5, p95}, a fixed normalisation mapping used
 *              in place of the percentiles of step 3, or NULL;
 *   enface_out device float32 [h][w];
 *   count_out  device int32 [h][w] or NULL: voxels averaged in step 5;
 *   stats_out  host double[4] or NULL: p5, p95, the threshold of step 3 and
 *              the OCT threshold of step 4;
 *   workspace  device memory of workspace_bytes >= octmc_enface_workspace_size
 *              bytes (about 8 w h d), owned by the caller and not used by
 *              anything else until the stream has passed this call, or NULL:
 *              the library allocates and frees it.
 * With a workspace, device inputs and no stats_out the call is asynchronous
 * on `stream`; otherwise it synchronises `stream`.  Errors: OCTMC_E_INVALID
 * (also a workspace smaller than needed), OCTMC_E_SHAPE (empty, a B-scan
 * longer than 8192 A-scans, volume > 2^31 bytes), OCTMC_E_OOM,
 * OCTMC_E_DEVICE. */
OCTMC_API int octmc_enface_project(octmc_ctx* ctx, const octmc_shape* shape, const float* oct, const float* octa,
                                   int32_t scan, const float* valid, const double* fixed, float* enface_out,
                                   int32_t* count_out, double* stats_out, void* workspace, uint64_t workspace_bytes,
                                   void* stream);

/* Device bytes of the workspace octmc_enface_project needs for w x h x d
 * volumes.  Errors: OCTMC_E_INVALID (NULL), OCTMC_E_SHAPE (empty). */
OCTMC_API int octmc_enface_workspace_size(int32_t w, int32_t h, int32_t d, uint64_t* bytes);

/* Stage 1, rough axial prealignment (Fig. 1; Sec. 2.1 "optimization"):
 * the objective of Eq. 1 restricted to axial displacements with one offset
 * z_b and one tilt t_b per B-scan,
 *   dz(f, b) = z_b + t_b (f - (n_f - 1) / 2),  dx = dy = 0,
 * f the A-scan index along the fast axis, n_f the B-scan length, plus the
 * tilt normalisation T.  T is defined only in earlier work; this library
 * reads it as T = sum_V gamma_tilt d n_f (n_f^2 - 1) / (24 n_b) (sum_b t_b)^2,
 * which fixes the two plane degrees of freedom the data term cannot see.
 * theta layout (float64): the X-fast scan's h B-scans (rows j, n_f = w)
 * then the Y-fast scan's w B-scans (columns i, n_f = h), (z_b, t_b) each:
 * 2 (h + w) values at a level of w x h A-scans, in level pixels.
 *
 * octmc_prealign_eval: the stage-1 objective at level `level` and theta
 * (host): terms (host float64[OCTMC_NTERMS]) as octmc_eval at the expanded
 * field (the pair's parameters and stored eta; the paper's stage 1 has
 * delta0 = 0, as the pair OCTMC_PREALIGN creates), T (host, may be NULL) and
 * d(F + T)/d(theta) (host float64[2 (h + w)], may be NULL).  Synchronises
 * `stream`.  Errors: OCTMC_E_INVALID, OCTMC_E_BUSY (a solve holds the pair),
 * OCTMC_E_OOM, OCTMC_E_NAN, OCTMC_E_DEVICE. */
OCTMC_API int octmc_prealign_eval(octmc_pair* pair, int32_t level, const double* theta, double gamma_tilt,
                                  double* terms, double* tilt_term, double* grad_theta, void* stream);

/* octmc_prealign: the stage-1 solve on the pair's pyramid: theta = 0 at the
 * coarsest level, iters_per_level L-BFGS steps per level (the pair's lbfgs_m,
 * line search constants), between levels the fine field is twice the coarse
 * field at the fine A-scan's coarse position, linear along the fast axis and
 * interpolated linearly between B-scans.  theta_out: host float64[2 (h + w)]
 * at the finest level; rep (may be NULL) as octmc_register (eta = 1).  The
 * L-BFGS iteration is octmc_register's, with its decisions on the device
 * unless the pair's flags hold OCTMC_HOST_LINE_SEARCH (the same result bit for
 * bit).  Synchronises `stream`.  Errors: as octmc_prealign_eval (OCTMC_E_NAN:
 * the objective is not finite at the end of a level). */
OCTMC_API int octmc_prealign(octmc_pair* pair, double gamma_tilt, int32_t iters_per_level, double* theta_out,
                             octmc_report* rep, void* stream);

/* The stage-1 result of a pair created with OCTMC_PREALIGN: theta_out (host
 * float64[2 (h + w)], may be NULL) and the axial field dz_out (device float32
 * [2][h][w], may be NULL).  The displacements octmc_register returns for such
 * a pair are relative to the prealigned volumes; the field to apply to the
 * original scan V at output A-scan (i, j) is d^V plus (0, 0, dz^V) taken at
 * (i + dx^V, j + dy^V).  Synchronises `stream` when dz_out is given.
 * Errors: OCTMC_E_INVALID (no prealignment), OCTMC_E_OOM, OCTMC_E_DEVICE. */
OCTMC_API int octmc_pair_prealignment(const octmc_pair* pair, double* theta_out, float* dz_out, void* stream);

/* Axial resampling (the "prealigned volumes" of Fig. 1):
 * out(i, j, k) = I(vol, i, j, k + dz(i, j)), the interpolator of Eq. 2 at
 * integer lateral positions, i.e. the Catmull-Rom spline along depth with tap
 * indices clamped to the A-scan.  vol [h][w][d] and dz [h][w] float32 live in
 * shape->mem memory (shape->dtype is ignored); out is device float32
 * [h][w][d].  Asynchronous for device inputs; host inputs are copied and the
 * stream synchronised.  Errors: OCTMC_E_INVALID, OCTMC_E_SHAPE, OCTMC_E_OOM,
 * OCTMC_E_DEVICE. */
OCTMC_API int octmc_resample_axial(octmc_ctx* ctx, const octmc_shape* shape, const float* vol, const float* dz,
                                   float* out, void* stream);

/* More than two volumes (Sec. 2.1 input: at least two raster scans, at least
 * one orthogonal to the others; the paper leaves the generalisation to
 * earlier work).  Every volume V has an orientation (0: X-fast, B-scans are
 * rows j; 1: Y-fast, columns i) and its own field.  Objective: the
 * two-volume data term (Eqs. 2-9) summed over all volume pairs P < Q, each
 * pair with its own eta (Eq. 10) and the validity of Eq. 5 resampled along
 * each volume's slow axis; plus alpha R summed over the volumes in their own
 * acquisition orders; plus M = gamma d / (n N_A) sum_c (sum_V sum_ij d)^2.
 * For n = 2 with orientations (0, 1) it is the pair objective.  The merge
 * normalises the density weights over all volumes (a second orthogonal pair
 * fills the first pair's white-line crossings, Fig. 4).
 *
 * octmc_multi_create: n (2..8) volumes of one shape; orient[n] (both
 * orientations must occur); oct[n] structural volumes [h][w][d] float32;
 * octa (NULL or n OCTA volumes), enface (NULL or n en face images [h][w]),
 * valid (NULL or n vectors of h values for X-fast, w for Y-fast volumes), as
 * octmc_pair_create (OCTMC_DETECT_INVALID and OCTMC_ENFACE_PROJECT apply per
 * volume; OCTMC_PREALIGN is not available here).  Pointers live in
 * shape->mem memory and are copied.  With n = 3 or 4 volumes (any storage
 * type; BF16/FP16 levels of odd depth are stored with one padding sample per
 * A-scan) the structural term of all pairs is evaluated in one fused pass
 * that resamples each volume once
 * (OCTMC_MULTI_PAIRWISE selects the pair-by-pair form; the two agree to
 * float32 rounding).
 * Errors: as octmc_pair_create. */
typedef struct octmc_multi octmc_multi;
OCTMC_API int octmc_multi_create(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape, int32_t n,
                                 const int32_t* orient, const float* const* oct, const float* const* octa,
                                 const float* const* enface, const float* const* valid, void* stream,
                                 octmc_multi** out);
OCTMC_API int octmc_multi_destroy(octmc_multi* multi);

/* One evaluation of the n-volume objective at pyramid level `level`: disp
 * device [n][h][w][3] float32 (level pixels), terms device
 * float64[OCTMC_NTERMS] (OCTMC_TERM_ETA is the first pair's eta), grad
 * device [n][h][w][3] float32 or NULL; eta_mode as octmc_eval (per pair).
 * Asynchronous on `stream`.  Errors: OCTMC_E_INVALID, OCTMC_E_BUSY, OCTMC_E_DEVICE. */
OCTMC_API int octmc_multi_eval(octmc_multi* multi, int32_t level, const float* disp, double* terms, float* grad,
                               int32_t eta_mode, void* stream);

/* The n-volume registration (the multi-resolution L-BFGS of octmc_register
 * over all n fields) and, if merged_oct != NULL, the merge.  disp_out device
 * [n][h][w][3]; merged_oct, merged_octa (needs OCTA volumes) device
 * [h][w][d] float32 or NULL; rep as octmc_register (eta of the first pair).
 * Synchronises `stream`.  Errors: OCTMC_E_INVALID, OCTMC_E_BUSY, OCTMC_E_OOM,
 * OCTMC_E_DEVICE. */
OCTMC_API int octmc_multi_register(octmc_multi* multi, float* disp_out, float* merged_oct, float* merged_octa,
                                   octmc_report* rep, void* stream);

/* The number of pyramid levels the pair holds (the resolved count when it was
 * created with levels = 0).  Errors: OCTMC_E_INVALID (NULL). */
OCTMC_API int octmc_pair_levels(const octmc_pair* pair, int32_t* levels);

/* Shape (w, h, d) of pyramid level `level` (0 = finest). */
OCTMC_API int octmc_pair_level_shape(const octmc_pair* pair, int32_t level, int32_t* w, int32_t* h, int32_t* d);

/* One evaluation of the objective (Eq. 1 without T: Eqs. 2-9 plus R and M)
 * and its gradient at pyramid level `level` -- the hot path.
 *   disp   device [2][h][w][3] float32 displacement in level pixels;
 *   terms  device float64[OCTMC_NTERMS] (see OCTMC_TERM_*);
 *   grad   device [2][h][w][3] float32 dF/d(disp), or NULL;
 *   eta_mode 0: set the level's eta from this displacement (Eq. 10, delta0 =
 *            0.5) before evaluating; 1: use the level's stored eta (1.0 until
 *            set).
 * Asynchronous on `stream`; nothing is copied to the host. */
OCTMC_API int octmc_eval(octmc_pair* pair, int32_t level, const float* disp, double* terms, float* grad,
               int32_t eta_mode, void* stream);

/* The same evaluation for npairs pairs whose level `level` has one common
 * shape, in one grouped launch per kernel.  disp and grad are
 * [npairs][2][h][w][3] float32 (device), terms [npairs][OCTMC_NTERMS]
 * float64 (device).  Errors: OCTMC_E_SHAPE if the shapes differ. */
OCTMC_API int octmc_eval_batched(octmc_pair* const* pairs, int32_t npairs, int32_t level, const float* disp,
                       double* terms, float* grad, int32_t eta_mode, void* stream);

/* octmc_eval for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It makes no allocation of any kind (no hipMalloc, hipFree or allocating
 * library routine); the caller passes every input and output, and the
 * kernels' scratch is a static device array of the library, one per GPU,
 * held until the process ends: OCTMC_NOALLOC_SCRATCH_BYTES bytes, enough
 * for w * h <= OCTMC_NOALLOC_MAX_ASCANS A-scans.
 *   ctx      context of the device (its creation resolved the array's address);
 *   params   objective parameters (alpha, delta0, eps_huber, eps_reg,
 *            flyback_frac, mean_weight; the solver fields are not used);
 *   shape    w == h, d, dtype of sx/sy, mem = OCTMC_MEM_DEVICE;
 *   sx, sy   device [h][w][d] structural volumes in the storage type `dtype`
 *            (float32, or bfloat16 / binary16 as 16-bit words);
 *   ax, ay   device [h][w] float32 en face images;
 *   vx, vy   device float32 validity, vx [h] (X-fast B-scans) and vy [w]
 *            (Y-fast); all ones for fully valid scans;
 *   disp, terms, grad as octmc_eval (grad may be NULL);
 *   eta      device float64[1]: eta_mode 0 writes this displacement's eta
 *            (Eq. 10) there before the evaluation, eta_mode 1 reads it.
 * The result equals octmc_eval's on a pair holding the same level 0 data
 * with the same eta.  Errors: OCTMC_E_INVALID (NULL inputs, host memory,
 * bad parameters), OCTMC_E_SHAPE (w != h, too small, or w * h above
 * OCTMC_NOALLOC_MAX_ASCANS), OCTMC_E_DTYPE.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads,
 * other contexts) race and must be ordered by the caller. */
#define OCTMC_NOALLOC_MAX_ASCANS (512 * 512)
#define OCTMC_NOALLOC_SCRATCH_BYTES (OCTMC_NOALLOC_MAX_ASCANS * 32 + 8192 + (OCTMC_NOALLOC_MAX_ASCANS + 255) / 256 * 64)
OCTMC_API int octmc_eval_noalloc(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape, const void* sx,
                                 const void* sy, const float* ax, const float* ay, const float* vx, const float* vy,
                                 const float* disp, double* eta, double* terms, float* grad, int32_t eta_mode,
                                 void* stream);

/* octmc_eval with HIP events recorded on `stream` between its kernels:
 * stage_ms[0] = displacement sum (mean term), [1] = structural resample /
 * residual / depth reduction (the dominant kernel), [2] = en face, validity,
 * combination, regulariser and global sums (both passes when eta_mode = 0).
 * Synchronises the stream.  For measurement; results equal octmc_eval's. */
OCTMC_API int octmc_eval_profile(octmc_pair* pair, int32_t level, const float* disp, double* terms, float* grad,
                                 int32_t eta_mode, float* stage_ms, void* stream);

/* Full multi-resolution registration (Sec. 2.1): zero displacement at the
 * coarsest level, eta fixed per level at its initial field (Eq. 10), L-BFGS
 * with a strong Wolfe line search per level, bilinear x2 upsampling between
 * levels.  disp_out: device [2][h][w][3] float32 at the finest level.
 * merged_oct / merged_octa: device [h][w][d] float32 or NULL (Sec. 2.1
 * "merging", Sec. 2.5); merged_octa needs OCTA volumes at pair creation.
 * rep: host report or NULL.  Synchronises `stream`. */
OCTMC_API int octmc_register(octmc_pair* pair, float* disp_out, float* merged_oct, float* merged_octa,
                   octmc_report* rep, void* stream);

/* Merge only (Sec. 2.1 "merging", Sec. 2.5), with a given finest-level
 * displacement field disp (device).  merged_octa may be NULL. */
OCTMC_API int octmc_merge(octmc_pair* pair, const float* disp, float* merged_oct, float* merged_octa, void* stream);

/* ------------------------------------------------------------------------
 * Serving: registration requests of mixed sizes solved concurrently on one
 * device (the full solve of Sec. 2.1 per request).  A server owns one range
 * of device memory (hbm_budget_bytes) and admits queued requests in arrival
 * order as soon as their footprint (octmc_request_footprint) fits in it and
 * fewer than max_active requests are being solved.  An admitted request keeps
 * its pyramid, float64 solver state and scratch in its part of that range
 * until it completes.  The evaluations of the active requests, each at its
 * own pyramid level and size, run either as grouped launches (one launch per
 * kernel covers every request waiting for an evaluation of fewer than 128^2
 * A-scans, while larger ones, which fill the device alone, run on their
 * request's stream; OCTMC_SERVE_GROUPED) or each on its request's own stream
 * (OCTMC_SERVE_STREAMS).  A request's
 * result is the same in both modes and equals octmc_register's for the same
 * inputs: every reduction runs in a fixed order per request.
 */
typedef struct octmc_server octmc_server;

#define OCTMC_SERVE_GROUPED 0
#define OCTMC_SERVE_STREAMS 1

/* One request.  Inputs as for octmc_pair_create (shape.mem says where they
 * live); they are read when the request is admitted, so they must stay valid
 * until its completion has been returned by octmc_server_poll.  Outputs are
 * device buffers of the caller: disp_out [2][h][w][3] float32 (required),
 * merged_oct / merged_octa [h][w][d] float32 or NULL. */
typedef struct {
    octmc_params params;
    octmc_shape shape;
    const float *oct_x, *oct_y, *octa_x, *octa_y, *enface_x, *enface_y, *valid_x, *valid_y;
    float* disp_out;
    float* merged_oct;
    float* merged_octa;
    uint64_t tag; /* returned unchanged in the completion */
} octmc_request;

/* Completion record of one request.  Times are seconds since the server was
 * created (steady clock). */
typedef struct {
    uint64_t id;
    uint64_t tag;
    int32_t status; /* octmc_status of the request's solve */
    int32_t reserved;
    /* t_submit: queued; t_admit: taken from the queue with its memory
     * reserved (admission times follow arrival order); t_done: solve and
     * outputs complete, before the memory is released */
    double t_submit, t_admit, t_done;
    uint64_t bytes_reserved; /* footprint taken from the server's memory */
    uint64_t bytes_used;     /* of which the request actually used */
    octmc_report report;
    char error[160];         /* octmc_last_error() text when status != 0 */
} octmc_completion;

/* Device bytes one request occupies while it is active (pyramid, solver
 * state, scratch, and the merge buffers if it asks for a merged volume).
 * Errors: as octmc_pair_create's validation. */
OCTMC_API int octmc_request_footprint(const octmc_request* req, uint64_t* bytes);

/* Create a server on ctx's device.  hbm_budget_bytes of device memory are
 * allocated at once; max_active (1..64) requests are solved concurrently;
 * mode is OCTMC_SERVE_GROUPED or OCTMC_SERVE_STREAMS.  Errors: OCTMC_E_INVALID,
 * OCTMC_E_OOM (the budget cannot be allocated). */
OCTMC_API int octmc_server_create(octmc_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_active, int32_t mode,
                                  octmc_server** out);

/* Queue a request; *id identifies its completion.  The call validates the
 * request and returns at once.  OCTMC_PREALIGN is not accepted here: create
 * the prealigned volumes with octmc_pair_create (or octmc_prealign and
 * octmc_resample_axial) and submit those.  Errors: OCTMC_E_INVALID / SHAPE / DTYPE,
 * OCTMC_E_OOM if its footprint exceeds the whole budget (it could never be
 * admitted). */
OCTMC_API int octmc_server_submit(octmc_server* srv, const octmc_request* req, uint64_t* id);

/* Move up to max completions into out (in completion order), waiting up to
 * wait_ms milliseconds for the first one (0: do not wait, < 0: wait until one
 * is available or nothing is pending).  *n receives the count. */
OCTMC_API int octmc_server_poll(octmc_server* srv, octmc_completion* out, int32_t max, int32_t wait_ms,
                                int32_t* n);

/* Counts of queued, active and completed-but-not-polled requests. */
OCTMC_API int octmc_server_status(const octmc_server* srv, int32_t* queued, int32_t* active, int32_t* done);

/* Finish every submitted request, then release the server's threads, streams
 * and memory.  Unpolled completions are discarded. */
OCTMC_API int octmc_server_destroy(octmc_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* OCTMC_H */

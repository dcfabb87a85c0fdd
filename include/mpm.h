/*
 * mpm.h -- C ABI of libmpm, a gfx950 (MI355X) implementation of the
 * voxel-parallel second-order fit of model-based multi-parameter mapping
 * (Balbastre et al., "Model-Based Multi-Parameter Mapping",
 * arXiv 2102.01604).
 *
 * The library fits log-parameter maps (log A, log R1, log R2*, logit MTsat)
 * to multi-echo spoiled-gradient-echo (SPGR) magnitude images, by the paper's
 * Newton-like iteration with its loaded approximate Hessian, either voxelwise
 * (maximum likelihood, "SPGR-ML") or with the joint-total-variation prior
 * solved by IRLS + preconditioned conjugate gradient ("SPGR+JTV").
 *
 * Entry points: mpm_fit, mpm_uncertainty (Laplace variance), mpm_simulate
 * (the forward model); their projected forms for contrasts acquired on their
 * own grids (mpm_*_projected); the fit and forward model with a protocol per
 * voxel (mpm_fit_voxelwise, mpm_simulate_voxelwise; also in the rate and time
 * representations); the noise level and initial maps from the echoes
 * (mpm_estimate_noise); batched JTV-MAP fits of several volumes
 * (mpm_fit_batch); reduced-precision echo storage with per-image
 * offsets (mpm_pack_echoes); a serving queue with continuous batching
 * (mpm_server_*); mpm_footprint_bytes, mpm_autotune, mpm_autotune_set, kernel timing
 * (mpm_profile_*), mpm_last_error and mpm_version.
 *
 * Conventions shared by every entry point
 *   - Voxel index n = x + nx*(y + ny*z) (x fastest); N = nx*ny*nz.
 *   - Images are numbered contrast-major: all echoes of contrast 0, then of
 *     contrast 1, ...  I = sum of n_echoes.
 *   - echoes: device array [I][N] of the storage dtype (mpm_dtype);
 *     maps / var: device float arrays [4][N] in the order
 *     (log A, log R1, log R2*, logit MTsat); b1: device float [N] or NULL
 *     (NULL means a transmit efficiency of 1 everywhere).
 *   - Device pointers belong to the caller and must stay valid until the call
 *     returns (the server's requests: until polled done).  The library
 *     allocates its own workspace on the given stream and frees it before
 *     returning.  Calls block until their device work is
 *     done.  `stream` is a hipStream_t (NULL: the default stream).
 *   - All arguments are validated on the host before any device work.  On an
 *     error nothing is written and mpm_last_error() describes the problem.
 *     Numerical degeneracy (an ill-posed voxel) is not an error: it is
 *     counted in mpm_report.
 *   - Arithmetic is FP32 per voxel; objective sums, CG inner products and the
 *     step-acceptance test are accumulated in FP64.
 */
#ifndef MPM_H
#define MPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPM_OK = 0,
    MPM_ERR_INVALID_ARG = 1,   /* a value or pointer failed validation          */
    MPM_ERR_UNSUPPORTED = 2,   /* a valid request the library does not handle  */
    MPM_ERR_OUT_OF_MEMORY = 3, /* workspace allocation failed                   */
    MPM_ERR_DEVICE = 4,        /* a HIP call failed                             */
    MPM_ERR_BUSY = 5,          /* server: request not finished yet              */
    MPM_ERR_NOT_FOUND = 6,     /* server: unknown ticket                        */
    MPM_ERR_CANCELLED = 7      /* server: the request was cancelled             */
} mpm_status;

typedef enum { MPM_F32 = 0, MPM_F16 = 1, MPM_BF16 = 2 } mpm_dtype; /* echo storage only */
typedef enum { MPM_ML = 0, MPM_MAP_JTV = 1 } mpm_mode;
typedef enum { MPM_INIT_DEFAULT = 0, MPM_INIT_CONST = 1, MPM_INIT_FROM_MAPS = 2 } mpm_init_kind;
/* Loading of the approximate Hessian (paper Sec. 2.3): PROPOSED adds
 * |res| |diag of the signal's second derivatives| per echo (the paper's
 * choice), PROPOSED_PLUS adds |res| times the absolute row sums of the full
 * second-derivative matrix ("Proposed+", a majoriser of the NLL Hessian), GN
 * adds nothing (Gauss-Newton / Fisher scoring). */
typedef enum { MPM_LOAD_PROPOSED = 0, MPM_LOAD_GN = 1, MPM_LOAD_PROPOSED_PLUS = 2 } mpm_loading;
/* Parameters the Newton-like steps act on (the representation comparison of
 * paper Sec. 3.1): LOG = (log A, log R1, log R2*, logit MTsat), the default
 * and the only one of every entry point but mpm_fit_voxelwise; RATE =
 * (A, R1, R2*, MTsat); TIME = (A, T1, T2*, MTsat), T = 1/R. */
typedef enum { MPM_BASIS_LOG = 0, MPM_BASIS_RATE = 1, MPM_BASIS_TIME = 2 } mpm_basis;

#define MPM_MAX_CONTRASTS 8
#define MPM_MAX_IMAGES 64

/* Acquisition protocol: the fixed parameters theta_i = (alpha_i, TR_i, TE_i,
 * sigma_i^2) of every image (paper Sec. 2.4).  An MT contrast carries the
 * off-resonance pulse of the Sec. 2.1 MT signal model (TR2 = 0). */
typedef struct {
    int32_t n_contrasts;                  /* 1..MPM_MAX_CONTRASTS              */
    int32_t n_echoes[MPM_MAX_CONTRASTS];  /* >= 1 each, sum <= MPM_MAX_IMAGES  */
    double tr_s[MPM_MAX_CONTRASTS];       /* repetition time (s), > 0          */
    double flip_rad[MPM_MAX_CONTRASTS];   /* nominal flip angle, (0, pi)       */
    int32_t mt[MPM_MAX_CONTRASTS];        /* 1 = MT-weighted contrast          */
    double te_s[MPM_MAX_IMAGES];          /* echo time per image (s), >= 0     */
    double sigma[MPM_MAX_IMAGES];         /* noise std per image, > 0          */
} mpm_protocol;

typedef struct {
    int64_t nx, ny, nz; /* each in [1, 2^20], nx*ny*nz < 2^30 */
} mpm_grid;

typedef struct {
    int32_t mode;          /* mpm_mode                                               */
    int32_t n_outer;       /* MAP: IRLS re-weighting loops (paper Sec. 2.7)          */
    int32_t n_gn;          /* ML: Newton-like steps; MAP: steps per outer loop       */
    int32_t n_cg;          /* MAP: CG iterations per Newton-like step                */
    int32_t max_halvings;  /* MAP: step halvings tried by the acceptance test (<= 7); <0 off */
    int32_t loading;       /* mpm_loading                                            */
    int32_t init_kind;     /* mpm_init_kind                                          */
    int32_t flags;         /* reserved, must be 0                                    */
    double lambda[4];      /* MAP: JTV weight per map, >= 0 (paper Sec. 2.5)         */
    double jtv_eps;        /* MAP: JTV smoothing; 0 -> 1e-3*sqrt(sum lambda)         */
    double cg_stop;        /* MAP: stop CG when r.z <= cg_stop*r0.z0; 0 -> fixed n_cg */
    double init_const[4];  /* MPM_INIT_CONST: the constant initial log-parameters    */
    /* MAP early stopping (paper Sec. 2.7; the paper's "gain" read as the decrease a
     * step brings over the decrease since the first value of its sequence): an outer
     * loop's Newton steps end after the first step whose gain on F_w is below tol_gn;
     * the outer loops end after the first whose gain on the objective (relative to the
     * end of the first loop) is below tol_outer.  0 -> fixed counts; finite, >= 0. */
    double tol_gn;
    double tol_outer;
    /* Net receive field (paper Sec. 2.4, footnote): device float [N], > 0, that
     * multiplies the modelled signal of each voxel (A -> A * b1_receive[n]), or
     * NULL for none.  Read by mpm_fit, mpm_uncertainty and the server; the
     * projected and per-voxel-protocol fits reject it (MPM_ERR_UNSUPPORTED). */
    const float *b1_receive;
    int32_t basis;  /* mpm_basis; other than MPM_BASIS_LOG: mpm_fit_voxelwise only */
    /* MAP: index of the first outer loop to run, for resuming a fit (checkpoint /
     * resume).  Loops start_outer .. n_outer-1 run; a loop t >= 1 re-weights from
     * the current maps first, so a fit stopped after t loops (its maps saved) and
     * resumed with init_kind = MPM_INIT_FROM_MAPS, start_outer = t and the same
     * other options reproduces the uninterrupted fit (the IRLS state between loops
     * is the maps and the loop index, Sec. 2.5-2.7).  0 <= start_outer < n_outer
     * (0 when n_outer = 0); 0 for ML; tol_outer must be 0 when start_outer > 0
     * (its gains are measured against the end of loop 0).  Trace slots of the
     * loops before start_outer stay NaN; report counts cover the loops run. */
    int32_t start_outer;
    /* Offsets of reduced-precision echo storage: host float [I] or NULL (no
     * offsets).  With MPM_F16 / MPM_BF16 echoes, image i stores its values minus
     * echo_offset[i], rounded to the storage type, and every kernel adds
     * echo_offset[i] back in FP32 when it reads a value.  An offset near the
     * image's values (mpm_pack_echoes uses the image mean) shrinks the magnitude
     * that is rounded, and with it the rounding error: the storage type keeps a
     * fixed number of significant bits.  Must be NULL for MPM_F32 echoes and
     * finite.  Read by mpm_fit, mpm_fit_noalloc, mpm_uncertainty, the projected
     * fit and uncertainty and the server (which copies it at submit);
     * mpm_fit_voxelwise rejects it. */
    const float *echo_offset;
} mpm_options;

typedef struct {
    double objective;          /* final NLL (ML) or NLL + smoothed JTV (MAP)          */
    double nll;                /* final negative log-likelihood                       */
    double jtv;                /* final smoothed JTV (MAP), 0 for ML                  */
    int32_t outer_done;        /* MAP outer loops executed                            */
    int32_t gn_done;           /* Newton-like steps taken (accepted, for MAP)         */
    int32_t cg_done;           /* CG iterations executed in total                     */
    int32_t rejected;          /* MAP steps whose every halving increased F_w         */
    int64_t degenerate_voxels; /* voxels whose last 4x4 solve was degenerate          */
    int64_t nonfinite_voxels;  /* voxels with a non-finite final map value            */
    int64_t nll_increases;     /* ML: (voxel, step) pairs whose NLL rose (> 1e-5 rel) */
} mpm_report;

/*
 * mpm_fit -- fit the maps (paper Sec. 2.3-2.4 for ML; Sec. 2.5-2.7 for MAP).
 *
 * ML: n_gn steps y <- y - P~^{-1} g in every voxel, P~ the loaded approximate
 * Hessian of eq. precond summed over every echo (Sec. 2.4), g the NLL
 * gradient.  MAP: for each of n_outer loops, refresh the JTV weights (from
 * the second loop on; the first loop starts from zero weights), then take
 * n_gn steps solving (P~ + L) delta = g + L y by n_cg iterations of PCG with
 * the block-diagonal preconditioner P~ + diag(G^T W G) (x) diag(lambda)
 * (Sec. 2.6), accepting y - 2^-h delta for the first h <= max_halvings that
 * does not increase F_w = NLL + 1/2 y^T L y.
 *
 * maps: in/out device float [4][N]; read as the initial values when
 * init_kind = MPM_INIT_FROM_MAPS, overwritten with the result.
 * report: host, may be NULL.  trace: host double array or NULL; if given it
 * receives trace_len values (NaN where not reached):
 *   ML : trace[j] = NLL before step j, trace[n_gn] = final NLL;
 *   MAP: for outer loop t, slots t*(n_gn+2)+j hold F_w before step 0 (j=0)
 *        and after step j-1 (j=1..n_gn), then NLL + smoothed JTV at the end
 *        of the loop.
 * Errors: MPM_ERR_INVALID_ARG (bad protocol, grid, options or NULL pointer;
 * |FP16 echo| is not checked), MPM_ERR_UNSUPPORTED (no MT contrast, fewer
 * than two distinct non-MT flip angles with MPM_INIT_DEFAULT, MAP with N < 2),
 * MPM_ERR_OUT_OF_MEMORY, MPM_ERR_DEVICE.
 */
mpm_status mpm_fit(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                   const void *echoes, const float *b1, const mpm_options *options,
                   float *maps, mpm_report *report, double *trace, int32_t trace_len,
                   void *stream);

/*
 * mpm_uncertainty -- Laplace posterior variance of the log-parameters at
 * `maps` (paper Sec. 3.6): the diagonal of
 * (P~ + diag(G^T W G) (x) diag(lambda))^{-1}, W from `maps`; lambda is 0 in
 * ML mode.  var: device float [4][N]; +inf marks a frozen parameter or a
 * degenerate voxel.  moments: device float [4][N] or NULL; receives the
 * log-normal posterior mean and variance of r1 = exp(y1) and of
 * t1 = exp(-y1): E[r1], V[r1], E[t1], V[t1] (Sec. 3.6).
 * options: mode, loading, lambda and jtv_eps are used.  Errors as mpm_fit.
 */
mpm_status mpm_uncertainty(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                           const void *echoes, const float *b1, const mpm_options *options,
                           const float *maps, float *var, float *moments, void *stream);

/*
 * mpm_simulate -- the forward model: SPGR echoes of every image at every
 * voxel from log-parameter maps (paper Sec. 2.1 eqs. 1-3 with TR2 = 0, in the
 * log/logit encoding of Sec. 2.4; flip angle alpha_c * b1_n).
 * maps: device float [4][N]; b1: device float [N] or NULL; noise: device
 * float [I][N] or NULL, added as sigma_i * noise; out: device [I][N] of
 * out_dtype (round-to-nearest-even for FP16/BF16).  Errors as mpm_fit.
 */
mpm_status mpm_simulate(const mpm_protocol *protocol, const mpm_grid *grid, const float *maps,
                        const float *b1, const float *noise, mpm_dtype out_dtype, void *out,
                        void *stream);

/*
 * Spatial projection (paper Sec. 2.4, "Spatial projection"): each contrast may
 * be acquired on its own grid, e.g. after head motion between scans.  The
 * maps and b1 stay on the reconstruction grid `grid`; the model is evaluated
 * on maps resliced into each acquisition space and its gradient and loaded
 * Hessian are sent back with the adjoint; the Hessian blocks that come back
 * are the block-diagonal majoriser of the reslicing the paper cites.
 *
 * mpm_space: the grid of one contrast and the affine map from its voxel
 * indices (i, j, k) to coordinates on the reconstruction grid,
 * r = affine (i, j, k, 1)^T, affine row-major 3x4 (unit: reconstruction
 * voxels).  Reslicing is trilinear with replicated borders; acquisition voxels
 * with r outside [-1/2, n - 1/2] on some axis lie outside the reconstruction
 * field of view and carry no observation.  Each axis of the affine must have
 * length in [1/8, 8] (acquisition voxel size relative to the reconstruction
 * voxel) and the affine must be invertible.
 *
 * spaces: host array of n_contrasts spaces.  echoes: device, the images back
 * to back, image i holding nx*ny*nz values of its contrast's space (image
 * order as mpm_protocol).  All else as mpm_fit / mpm_uncertainty.  An ML fit
 * takes the step y - P~^{-1} g with the pushed blocks in every iteration; its
 * report counts nll_increases as 0 (the NLL per voxel is not defined here)
 * and degenerate_voxels at the final maps.
 */
typedef struct {
    int64_t nx, ny, nz;
    double affine[12];
} mpm_space;

mpm_status mpm_fit_projected(const mpm_protocol *protocol, const mpm_grid *grid, const mpm_space *spaces,
                             mpm_dtype dtype, const void *echoes, const float *b1, const mpm_options *options,
                             float *maps, mpm_report *report, double *trace, int32_t trace_len, void *stream);
mpm_status mpm_uncertainty_projected(const mpm_protocol *protocol, const mpm_grid *grid, const mpm_space *spaces,
                                     mpm_dtype dtype, const void *echoes, const float *b1,
                                     const mpm_options *options, const float *maps, float *var, float *moments,
                                     void *stream);
/* Echoes in every acquisition space (layout as mpm_fit_projected's echoes)
 * from maps and b1 on the reconstruction grid: the model at the resliced maps
 * and b1, plus sigma_i * noise (noise: device float, same layout, or NULL);
 * NaN (no observation) outside the reconstruction field of view. */
mpm_status mpm_simulate_projected(const mpm_protocol *protocol, const mpm_grid *grid, const mpm_space *spaces,
                                  const float *maps, const float *b1, const float *noise, mpm_dtype out_dtype,
                                  void *out, void *stream);

/*
 * mpm_fit_voxelwise -- ML fit in which every voxel has its own protocol, as in
 * the paper's convergence experiment (Sec. 3.1: random TR, flip angles and
 * echo times per voxel).  The n_voxels voxels are independent (no grid).
 *
 * protocols: the contrast/echo structure, MT flags and per-image noise levels
 * are shared (n_contrasts, n_echoes, mt, sigma: rules as mpm_protocol); the
 * device arrays give, per voxel n, the repetition time tr_s[c * N + n] (s) and
 * flip angle flip_rad[c * N + n] (rad, the effective angle: no B1 input) of
 * each contrast c and the echo time te_s[i * N + n] (s) of each image i
 * (N = n_voxels).  echoes: device [I][N] of dtype.  A voxel whose TR is not
 * finite and > 0, whose flip is not in (0, pi) or whose TE is not finite and
 * >= 0 is not fitted: its maps are NaN and it counts as non-finite.
 *
 * options: mode MPM_ML; n_gn steps y <- y - P~^{-1} g with the chosen loading
 * (paper Sec. 2.3); init_kind MPM_INIT_CONST (init_const) or
 * MPM_INIT_FROM_MAPS (maps holds the start); MPM_INIT_DEFAULT is
 * MPM_ERR_UNSUPPORTED (the volume-mean initialisation assumes one protocol).
 * basis: the parameters y the steps act on (Sec. 3.1); with MPM_BASIS_RATE or
 * MPM_BASIS_TIME, maps and init_const hold (A, R1, R2*, MTsat) or
 * (A, T1, T2*, MTsat), and a step that would take A, R1 (T1) or R2* (T2*) to
 * <= 0, or MTsat out of (0, 1), moves that parameter halfway to the boundary
 * it would cross instead.
 *
 * Outputs (device, caller-owned): maps [4][N] (log A, log R1, log R2*,
 * logit MTsat, or the basis' parameters); nll_increases [N] int32 or NULL: the number of steps after
 * which the voxel's NLL exceeds the previous value by more than 1e-5
 * (relative, FP32 evaluation) or becomes non-finite from a finite value;
 * nll [N] float or NULL: the final NLL.  report (host, may be NULL): total
 * final NLL, degenerate and non-finite voxels, total NLL rises.  Validation
 * on the host before any device work; blocks until done.
 */
typedef struct {
    int32_t n_contrasts;
    int32_t n_echoes[MPM_MAX_CONTRASTS];
    int32_t mt[MPM_MAX_CONTRASTS];
    double sigma[MPM_MAX_IMAGES];
    const float *tr_s;      /* device [C][N] */
    const float *flip_rad;  /* device [C][N] */
    const float *te_s;      /* device [I][N] */
} mpm_voxel_protocols;

mpm_status mpm_fit_voxelwise(const mpm_voxel_protocols *protocols, int64_t n_voxels, mpm_dtype dtype,
                             const void *echoes, const mpm_options *options, float *maps, int32_t *nll_increases,
                             float *nll, mpm_report *report, void *stream);

/* Echoes [I][N] of out_dtype for per-voxel protocols (layout and rules as
 * mpm_fit_voxelwise): the model at maps [4][N] plus sigma_i * noise (device
 * float [I][N], or NULL); NaN for a voxel whose protocol is invalid. */
mpm_status mpm_simulate_voxelwise(const mpm_voxel_protocols *protocols, int64_t n_voxels, const float *maps,
                                  const float *noise, mpm_dtype out_dtype, void *out, void *stream);

/*
 * mpm_estimate_noise -- the noise level and the constant initial maps from
 * the echoes, as paper Sec. 2.7 obtains them: per image a two-class Rician
 * mixture fitted to its histogram; the class with the lower mean is the
 * background (air), whose sigma is the image's noise level; the variances of
 * one contrast's echoes are averaged with the geometric mean; the initial
 * maps come from the other class's means (the default initialisation's
 * closed forms).  Needs magnitude images with a background.
 *
 * Per image: the finite values >= 0 (others are not observations) in nbins
 * bins over [0, max] (bin floor(x * (nbins / max)) taken in FP32, the top
 * value in the last bin); n_iter EM iterations on the bin centres, the phase
 * of each value as the latent variable, from the split of the histogram at its
 * mean; class 0, started on the lower part, is a Rician without signal
 * (nu = 0).
 *
 * protocol: as for mpm_fit, its sigma not read; echoes: device [I][N]
 * (dtype); b1: device [N] or NULL (its mean enters the initial maps as in the
 * default initialisation); nbins in [16, 4096] (1024 is a good choice);
 * n_iter in [0, 100000] (200).  Host outputs, caller-owned:
 * sigma_image [I], sigma_contrast [C], fg_mean [I] (the foreground class's
 * mean), init_const [4] (log A, log R1, log R2*, logit MTsat: pass as
 * mpm_options.init_const with MPM_INIT_CONST); fits [I] or NULL: each image's
 * mixture; hist [I][nbins] or NULL: the histograms.  Blocks until done.
 * MPM_ERR_UNSUPPORTED if an image's values do not split in two classes.
 */
typedef struct {
    double pi[2], nu[2], sigma[2]; /* weights and Rice parameters; class 0: nu = 0 */
    double mean[2];                /* responsibility-weighted mean value per class */
    double nll;                    /* negative log-likelihood of the bin centres   */
} mpm_rice_fit;

mpm_status mpm_estimate_noise(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                              const void *echoes, const float *b1, int32_t nbins, int32_t n_iter,
                              double *sigma_image, double *sigma_contrast, double *fg_mean, double *init_const,
                              mpm_rice_fit *fits, uint32_t *hist, void *stream);

/* Device bytes a fit of this size needs: inputs, maps and the library's
 * workspace.  Returns 0 for invalid arguments. */
size_t mpm_footprint_bytes(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                           int32_t mode);

/* Text of the last error raised on the calling thread ("" if none). */
const char *mpm_last_error(void);

/*
 * Serving: a request queue with continuous batching.
 *
 * A server owns `max_active` HIP streams (default-priority).  Submitted fits
 * wait in submission order; mpm_server_step() admits a waiting fit when a
 * stream is free and the sum of mpm_footprint_bytes() of the admitted fits
 * stays within `hbm_budget`.  A MAP fit of 2^21 voxels or more fills the
 * device by itself for a long time, so at most one such fit runs at a time (in
 * submission order); ML fits and smaller MAP fits may be admitted ahead of a
 * waiting large one, but never ahead of a fit that waits for memory.  Each
 * step then enqueues the next piece of work of every admitted fit (the whole
 * ML fit, or one Newton-like step of a MAP fit) on
 * its stream, so fits admitted at different times run concurrently on the
 * device and new arrivals join while others are in flight.  Small JTV-MAP
 * fits (at most 2^19 voxels, whose launches are short enough that the
 * device's dispatch latency dominates them) are admitted in groups: the first
 * waiting one takes later waiting fits of at most twice or half its size that
 * can share launches with it (mpm_fit_batch's conditions; at most 16 fits and
 * 2^22 voxels in all, within the budget) onto its stream, and the group runs
 * as one batched fit, every kernel launch serving all its volumes.  Each fit, alone or in a group, runs the same
 * kernel bodies with the same per-volume launch shapes as mpm_fit(), so its
 * result is the same as when it is run alone, bit for bit.  Flag
 * MPM_SERVER_NO_GROUPS keeps every fit on a stream of its own.
 *
 * mpm_request: the arguments of mpm_fit() (report and trace excepted).  The
 * caller's device buffers must hold their inputs before submit and stay valid
 * until poll reports done; maps receives the result.
 * flags: MPM_SERVER_THREAD starts a host thread that calls mpm_server_step()
 * continuously; otherwise the caller drives it.
 * mpm_server_submit validates like mpm_fit (same errors) and returns a ticket.
 * mpm_server_step: does not wait for the device (a fit whose default
 * initialisation still awaits its image means on the host gets its next
 * piece at a later step; only after an error does a step wait for the work
 * that fit had enqueued); *pending (may be NULL) receives the number of fits
 * queued or running.
 * mpm_server_poll: *done = 1 and the report once the fit finished (returning
 * that fit's status), *done = 0 while queued or running; MPM_ERR_NOT_FOUND for
 * an unknown ticket.  A fit whose footprint exceeds the budget finishes with
 * MPM_ERR_OUT_OF_MEMORY.
 * mpm_server_cancel: a queued request leaves the queue at once; a running one
 * gets no further pieces and is released once its pieces in flight complete
 * (at a later step); a running one in a group finishes with its group (whose
 * launches serve every member) unless every member was cancelled.  Either then
 * polls as done with MPM_ERR_CANCELLED, its maps holding whatever the
 * completed pieces wrote (unspecified).  No effect on a finished request;
 * MPM_ERR_NOT_FOUND for an unknown ticket.  Other requests are unaffected
 * (each fit has its own workspace and control block).
 * mpm_server_destroy waits for running fits and frees the server.
 * Calls on one server are serialised by an internal lock.
 */
typedef struct {
    mpm_protocol protocol;
    mpm_grid grid;
    int32_t dtype;      /* mpm_dtype */
    int32_t reserved;   /* must be 0 */
    const void *echoes;
    const float *b1;
    mpm_options options;
    float *maps;
} mpm_request;

typedef struct mpm_server mpm_server;

#define MPM_SERVER_THREAD 1
#define MPM_SERVER_NO_GROUPS 2  /* run every fit on its own stream (no batched groups) */

mpm_status mpm_server_create(size_t hbm_budget, int32_t max_active, int32_t flags, mpm_server **out);
mpm_status mpm_server_submit(mpm_server *server, const mpm_request *request, uint64_t *ticket);
mpm_status mpm_server_step(mpm_server *server, int32_t *pending);
mpm_status mpm_server_poll(mpm_server *server, uint64_t ticket, int32_t *done, mpm_report *report);
mpm_status mpm_server_cancel(mpm_server *server, uint64_t ticket);
mpm_status mpm_server_destroy(mpm_server *server);

/*
 * mpm_fit_batch -- several JTV-MAP fits (paper Sec. 2.5-2.7) run together on
 * one stream, each kernel launch serving all of them: for many small volumes,
 * whose single launches each cost about the device's dispatch latency, this
 * spends that latency once per launch instead of once per volume.  requests:
 * host array of n (1..64) fits as for the server (their own protocols, grids,
 * echoes, fields, priors, initialisations and maps); all MPM_MAP_JTV, with the
 * same schedule options (n_outer, n_gn, n_cg, max_halvings, loading,
 * start_outer, tol_gn, tol_outer, cg_stop), echo storage dtype and register
 * shape (at most 4 contrasts of at most 8 echoes, 4 x 16, 8 x 8, or other),
 * else MPM_ERR_UNSUPPORTED.  Each fit's maps, report and trace are those of
 * mpm_fit on it alone, bit for bit (each volume keeps its own workspace,
 * launch shape, fixed-order reductions and control block).  reports: host
 * [n] or NULL; traces: host [n][trace_len] or NULL (trace_len 0), as
 * mpm_fit's trace per fit.  Workspace: the sum of the fits' (about 124 B per
 * voxel).  Blocks until done.
 */
mpm_status mpm_fit_batch(int32_t n, const mpm_request *requests, mpm_report *reports, double *traces,
                         int32_t trace_len, void *stream);

/*
 * mpm_pack_echoes -- writes echoes for reduced-precision storage with per-image
 * offsets (see mpm_options.echo_offset): offsets[i] = the mean of the finite
 * values of image i (FP64 sum, rounded to float), then
 * dst[i][n] = round_to_nearest_even(src[i][n] - offsets[i]) in dtype.
 * n_images >= 1 (<= MPM_MAX_IMAGES), n_voxels in [1, 2^30); src: device float
 * [n_images][n_voxels]; dst: device [n_images][n_voxels] of dtype (MPM_F16 or
 * MPM_BF16; must not overlap src); offsets: host float [n_images] (written).
 * Non-finite inputs stay non-finite (missing observations).  A finite value
 * whose difference overflows the storage type is an error: the call returns
 * MPM_ERR_INVALID_ARG after writing dst, with the count in mpm_last_error().
 * Blocks until done.
 */
mpm_status mpm_pack_echoes(int32_t n_images, int64_t n_voxels, const float *src, mpm_dtype dtype, void *dst,
                           float *offsets, void *stream);

/*
 * mpm_fit_noalloc -- mpm_fit for callers that cannot allocate memory: code
 * under HIP graph capture, serving loops that must not allocate, harnesses
 * that forbid it.  Same arguments, validation, results and blocking
 * behaviour as mpm_fit (the same kernels in the same launch shapes, so the
 * maps, report and trace are those of mpm_fit bit for bit); it calls no
 * hipMalloc / hipFree / hipHostMalloc and no other allocating routine.  The
 * caller still owns echoes, b1 and maps.
 * Workspace: a fixed device array of MPM_NOALLOC_SCRATCH_BYTES (64 MiB)
 * inside the library, one per device that runs it, held until the process
 * ends.  That bounds the fit: a MAP fit needs about 124 bytes per voxel (up
 * to about 530,000 voxels, e.g. a 64^3 or 80^3 volume); an ML fit needs
 * 8 * (n_gn + 4) bytes per 256 voxels (plus 8 * (2I + 1) per 1024 voxels for
 * the default initialisation).  A fit that does not fit is rejected with
 * MPM_ERR_OUT_OF_MEMORY before any device work, and mpm_last_error() states
 * the bytes it needs.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (each call initialises what it reads).  Calls that
 * overlapped on one device would race on it: the library serialises them
 * with a per-device lock held for the whole call, so concurrent host threads
 * wait for each other.
 */
#define MPM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

mpm_status mpm_fit_noalloc(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                           const void *echoes, const float *b1, const mpm_options *options, float *maps,
                           mpm_report *report, double *trace, int32_t trace_len, void *stream);

/*
 * mpm_autotune -- picks the workgroup count of the MAP fit's dominant kernel
 * (the CG sweep that walks z-runs of 64 x 16 tiles) for one grid size by
 * timing it; for the callers that fit many volumes of one size.  Each
 * candidate (targets of 512 ... 16384 workgroups, i.e. z-runs of different
 * lengths; targets that give the same launch are timed once) runs `reps`
 * full sweeps on zeroed scratch buffers of that size (about 110 B per voxel,
 * freed on return); the fastest is then used by every later MAP fit of exactly
 * that grid in this process, the server's included; other sizes keep the
 * built-in choice.  Changing the launch shape changes the order of the FP64
 * partial sums, so a grid's results differ at rounding level from those
 * before it was tuned.  Blocks until done.  result (host, may be NULL): the
 * candidates, their mean sweep times and the choice.  mpm_autotune_clear
 * forgets every choice.
 */
typedef struct {
    int32_t n_candidates;
    int32_t chosen;            /* index of the fastest candidate               */
    int32_t target[8];         /* workgroup target                             */
    int32_t workgroups[8];     /* workgroups launched                          */
    int32_t planes_per_run[8]; /* z-planes each workgroup walks                */
    double ms[8];              /* mean time of one sweep                       */
} mpm_tune_result;

mpm_status mpm_autotune(const mpm_grid *grid, int32_t reps, mpm_tune_result *result, void *stream);

/*
 * mpm_autotune_set -- fixes the launch shape of MAP fits and uncertainties of
 * exactly this grid size in this process, as mpm_autotune does after timing:
 * cg_workgroups is the workgroup target of the CG sweep that walks z-runs
 * (each workgroup walks ceil(tiles * nz / target) planes, at most 32), and
 * column_workgroups that of the column walks of the stencil-only kernels (the
 * JTV weights of Sec. 2.5 and the halved-step acceptance test); 0 keeps the
 * built-in choice.  For callers that pin a launch shape, e.g. to reproduce a
 * tuned run or to check every z-run length.  Results depend on the shape only
 * through the order of FP64 partial sums.  MPM_ERR_INVALID_ARG for an invalid
 * grid or a target outside [0, 2^20].  mpm_autotune_clear forgets it.
 */
mpm_status mpm_autotune_set(const mpm_grid *grid, int32_t cg_workgroups, int32_t column_workgroups);
void mpm_autotune_clear(void);

/* Library version string. */
const char *mpm_version(void);

/*
 * Kernel timing for measurement tools.  mpm_profile_enable(k) with k >= 1
 * brackets one in every k launches of each kernel with HIP events on the
 * launch stream (k = 0 turns timing off and is the default); the elapsed
 * times are collected when each call finishes.  mpm_profile_read copies up to
 * `max` records and returns how many kernels have records.
 */
typedef struct {
    char name[40];
    int64_t launches;   /* launches since the last reset              */
    int64_t timed;      /* launches that were bracketed by events     */
    double timed_ms;    /* summed event time of the timed launches    */
    double bytes;       /* algorithmic HBM bytes of all launches      */
} mpm_kernel_stat;

void mpm_profile_enable(int32_t every);
void mpm_profile_reset(void);
int32_t mpm_profile_read(mpm_kernel_stat *out, int32_t max);

#ifdef __cplusplus
}
#endif
#endif

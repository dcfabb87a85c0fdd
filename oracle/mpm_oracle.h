/*
 * mpm_oracle.h -- plain FP64 CPU oracle for model-based multi-parameter
 * mapping (Balbastre et al., "Model-Based Multi-Parameter Mapping",
 * arXiv 2102.01604).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Conventions (all host memory, all FP64):
 *   - voxel index n = x + nx*(y + ny*z), x fastest;
 *   - images are numbered contrast-major: all echoes of contrast 0, then
 *     contrast 1, ...; echoes X are laid out [I][N];
 *   - log-parameter maps Y are laid out [4][N] in the order
 *     (log A, log R1, log R2*, logit MTsat)   (paper Sec. 2.4).
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_CONTRASTS 8
#define ORC_MAX_IMAGES 64

typedef struct {
    int32_t n_contrasts;
    int32_t n_echoes[ORC_MAX_CONTRASTS];
    double  tr[ORC_MAX_CONTRASTS];      /* repetition time, s            */
    double  flip[ORC_MAX_CONTRASTS];    /* nominal flip angle, rad       */
    int32_t mt[ORC_MAX_CONTRASTS];      /* 1 if the contrast has an MT pulse */
    double  te[ORC_MAX_IMAGES];         /* echo time per image, s        */
    double  sigma[ORC_MAX_IMAGES];      /* noise standard deviation per image */
} orc_protocol;

/* Acquisition space of one contrast (spatial projection, Sec. 2.4): its grid
 * and the affine map from its voxel indices (i, j, k) to coordinates on the
 * reconstruction grid, r = A (i, j, k, 1)^T, A row-major 3x4. */
typedef struct {
    int64_t dims[3];
    double  affine[12];
} orc_space;

enum { ORC_ML = 0, ORC_MAP = 1 };
enum { ORC_INIT_DEFAULT = 0, ORC_INIT_CONST = 1, ORC_INIT_FROM_MAPS = 2 };
enum { ORC_LOAD_PROPOSED = 0, ORC_LOAD_GN = 1, ORC_LOAD_PROPOSED_PLUS = 2 };
/* Parameters the Newton-like steps act on (the representation comparison of
 * Sec. 3.1): log/logit (log A, log R1, log R2*, logit MTsat), rate
 * (A, R1, R2*, MTsat) or time (A, T1, T2*, MTsat). */
enum { ORC_BASIS_LOG = 0, ORC_BASIS_RATE = 1, ORC_BASIS_TIME = 2 };

typedef struct {
    int32_t mode;           /* ORC_ML or ORC_MAP                                  */
    int32_t n_outer;        /* IRLS re-weighting loops (MAP)                      */
    int32_t n_gn;           /* Newton-like steps (per outer loop for MAP)         */
    int32_t n_cg;           /* conjugate-gradient iterations per Newton step      */
    int32_t max_halvings;   /* MAP step acceptance: halvings tried; <0 = no test  */
    int32_t loading;        /* ORC_LOAD_PROPOSED (paper), ORC_LOAD_GN or _PLUS    */
    int32_t init_kind;      /* ORC_INIT_*                                         */
    int32_t basis;          /* ORC_BASIS_*; other than LOG only in orc_fit_voxelwise,
                               whose maps and init_const are then in that basis   */
    double  lambda[4];      /* JTV regularisation per map                         */
    double  jtv_eps;        /* smoothing of the JTV norm; 0 -> 1e-3*sqrt(sum lambda) */
    double  cg_stop;        /* CG stops when r.z <= cg_stop * r0.z0 (0: fixed count) */
    double  init_const[4];  /* ORC_INIT_CONST values                              */
    double  tol_gn;         /* MAP: stop an outer loop's Newton steps when the gain of a
                               step falls below this (0: fixed count; reading R-stop) */
    double  tol_outer;      /* MAP: stop the outer loops when the gain of one falls below
                               this (0: fixed count; reading R-stop)                 */
    const double *b1_receive; /* [N] net receive field b-_n multiplying every image of
                               voxel n (Sec. 2.4), or NULL; orc_fit and orc_uncertainty */
    int32_t start_outer;    /* MAP: index of the first outer loop run (0 <= it <=
                               n_outer); loops start_outer .. n_outer-1 run, the first
                               of them re-weighting from the initial maps when >= 1, so
                               a fit stopped after t loops resumes from its maps with
                               start_outer = t (the IRLS state is the maps and t)   */
} orc_options;

typedef struct {
    double  objective;        /* final objective (ML: NLL; MAP: NLL + smoothed JTV) */
    double  nll;              /* final negative log-likelihood                      */
    double  jtv;              /* final smoothed JTV value (MAP), 0 for ML           */
    int32_t outer_done;
    int32_t gn_done;          /* accepted Newton-like steps                         */
    int32_t cg_done;          /* CG iterations executed in total                    */
    int32_t rejected;         /* MAP steps whose every halving increased F          */
    int64_t degenerate_voxels;/* voxels whose last 4x4 solve hit the degenerate rule */
    int64_t nonfinite_voxels; /* voxels with a non-finite final map value           */
    int64_t nll_increases;    /* ML: (voxel, step) pairs where the voxel NLL rose   */
} orc_report;

/* ---- forward model ---- */
void orc_spgr_derivs(const double y[4], double alpha, double tr, double te, int mt,
                     double *s, double ds[4], double d2s[4]);
void orc_spgr_hess(const double y[4], double alpha, double tr, double te, int mt, double H[16]);
void orc_spgr_basis(const double th[4], int basis, double alpha, double tr, double te, int mt,
                    double *s, double ds[4], double H[16]);
void orc_simulate(const orc_protocol *p, int64_t n, const double *maps,
                  const double *b1, double *out);

/* ---- per-voxel likelihood block ---- */
void orc_lik_voxel(const orc_protocol *p, const double *x, int64_t stride,
                   const double y[4], double b1, int loading,
                   double *nll, double g[4], double P[16]);
void orc_lik_voxel_basis(const orc_protocol *p, const double *x, int64_t stride,
                         const double th[4], int basis, int loading,
                         double *nll, double g[4], double P[16]);
int  orc_solve4(const double P[16], const double g[4], double out[4]);

/* ---- JTV prior ---- */
double orc_jtv_weights(const int64_t dims[3], const double *maps, const double lambda[4],
                       double eps, double *w, double *d);
void   orc_apply_L(const int64_t dims[3], const double *w, const double lambda[4],
                   const double *v, double *out);
int    orc_pcg(const int64_t dims[3], const double *P, const double *w, const double *d,
               const double lambda[4], const double *b, int n_cg, double cg_stop,
               double *delta);

/* ---- full fit and uncertainty ---- */
int  orc_default_init(const orc_protocol *p, int64_t n, const double *x, const double *b1,
                      double y0[4]);
/* Mode ORC_MAP: the maps after a finite IRLS x Newton x CG schedule have no
 * closed form and the paper prints no worked example; every step is pinned
 * separately (likelihood block, JTV weights and L, PCG, acceptance), MAP with
 * lambda = 0 equals ML, the objective is monotone, and a long schedule ends
 * at the minimiser of NLL + smoothed JTV found by an unrelated optimiser
 * (pinned through its end point).  Mode ORC_ML is pinned (exact recovery). */
int  orc_fit(const orc_protocol *p, const int64_t dims[3], const double *x, const double *b1,
             const orc_options *opt, double *maps, orc_report *rep, double *trace,
             int32_t trace_len);
int  orc_uncertainty(const orc_protocol *p, const int64_t dims[3], const double *x,
                     const double *b1, const orc_options *opt, const double *maps,
                     double *var, double *moments);
int  orc_num_threads(void);
/* Threads of the voxel-parallel loops from now on (results do not depend on it). */
void orc_set_num_threads(int n);

/* Spatial projection (R-proj): trilinear pull Psi and its adjoint push. */
void orc_pull(const int64_t dims[3], const orc_space *sp, const double *vol, double *out);
void orc_push(const int64_t dims[3], const orc_space *sp, const double *acq, double *vol);
double orc_proj_lik(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces, const double *x,
                    const double *b1, int loading, const double *maps, double *g, double *P);
int orc_default_init_projected(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces,
                               const double *x, const double *b1, double y0[4]);
/* Per-voxel protocols (Sec. 3.1 convergence experiment): tr, flip [C][N] and
 * te [I][N] per voxel; ML steps from init_const or maps; per-voxel counts of
 * NLL rises above rise_rel and final NLL (each optional). */
int orc_fit_voxelwise(const orc_protocol *shape, int64_t N, const double *tr, const double *flip, const double *te,
                      const double *x, const orc_options *opt, double rise_rel, double *maps, int32_t *increases,
                      double *nll, orc_report *rep);
/* Projected fit (R-proj); as orc_fit, pinned for MAP through its end point
 * (the minimiser of the projected NLL + smoothed JTV): identity spaces equal
 * orc_fit, and pull / push / pushed blocks are pinned. */
int orc_fit_projected(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces, const double *x,
                      const double *b1, const orc_options *opt, double *maps, orc_report *rep, double *trace,
                      int32_t trace_len);
int orc_uncertainty_projected(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces,
                              const double *x, const double *b1, const orc_options *opt, const double *maps,
                              double *var, double *moments);

/* ---- noise estimation (Sec. 2.7) ---- */
/* e^-z I0(z) and e^-z I1(z) for z >= 0 (modified Bessel functions). */
void orc_bessel_i01e(double z, double *i0e, double *i1e);
/* Histogram of one magnitude image (x [n]): finite values >= 0 in nbins
 * bins over [0, max]; the bin of a value is decided in FP32 (R-rice).
 * Returns the FP32 scale nbins / max (bin b covers [b, b+1) / scale), 0 if no
 * value is > 0. */
float orc_histogram(const double *x, int64_t n, int nbins, int64_t *counts);
/* Two-class Rician mixture fitted to a histogram by n_iter EM iterations
 * (R-rice; class 0, the background, has nu = 0); per class k: weight pi,
 * Rice parameters nu and sigma, and the
 * responsibility-weighted mean of the values; nll [n_iter + 1] (optional):
 * the histogram's negative log-likelihood before each iteration and after
 * the last.  Returns 0, or 1 if the values do not split in two classes. */
int orc_rice_mixture(const int64_t *counts, int nbins, double scale, int n_iter, double pi[2], double nu[2],
                     double sigma[2], double mean[2], double *nll);
/* Noise level and initial maps as Sec. 2.7 obtains them (R-rice): per image
 * the mixture above, whose lower-mean class is the background;
 * sigma_image[i] its sigma; sigma_contrast[c] the square root of the
 * geometric mean of the variances of contrast c's echoes; fg_mean[i] the mean
 * of the other class; y0 the default initialisation from those means (b1:
 * [n] or NULL).  Returns 0, or 1 if some image does not split in two classes. */
int orc_estimate_noise(const orc_protocol *p, int64_t n, const double *x, const double *b1, int nbins, int n_iter,
                       double *sigma_image, double *sigma_contrast, double *fg_mean, double y0[4]);

#ifdef __cplusplus
}
#endif
#endif

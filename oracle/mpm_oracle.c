/*
 * mpm_oracle.c -- plain FP64 CPU oracle for model-based multi-parameter
 * mapping (Balbastre et al., arXiv 2102.01604).
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked against.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the GPU library.
 *
 * Style: every quantity is computed the way the paper writes it, in double
 * precision, one voxel at a time.  Loops over voxels carry an OpenMP pragma so
 * the oracle finishes moderate volumes in seconds; every sum over voxels is
 * taken afterwards in index order by a plain serial loop, so results do not
 * depend on the thread count.
 *
 * Readings of points the paper leaves open (each one is marked where used):
 *   R-sigma  : each image's squared residual is weighted by 1/sigma_i^2 in the
 *              gradient and in the approximate Hessian (Sec. 2.4 objective).
 *   R-degen  : 4x4 solves are Jacobi-scaled; a parameter whose diagonal entry
 *              is <= 1e-30 * (largest diagonal entry) is frozen (step 0); if a
 *              Cholesky pivot of the scaled matrix falls below 1e-6 the whole
 *              voxel takes step 0 and is counted as degenerate.
 *   R-border : JTV finite differences use unit voxel spacing and a Neumann
 *              border (differences across the border are zero).
 *   R-eps    : the JTV weight is (q + eps^2)^(-1/2); the objective uses the
 *              matching smoothed norm sum_n sqrt(q_n + eps^2).
 *   R-w0     : IRLS starts from w = 0 (the first outer loop is an ML warm
 *              start); weights are recomputed at the start of every later
 *              outer loop and once after the last one.
 *   R-cg     : CG starts from 0 and stops early only when p.q <= 0 or when
 *              r.z <= cg_stop * r0.z0 (cg_stop = 0 by default: the fixed
 *              iteration count of the configured schedule).
 *   R-accept : a MAP Newton step y - 2^-h * delta is accepted for the first
 *              h = 0..max_halvings that does not increase F_w by more than
 *              ACCEPT_REL * |F_w| (1e-9: below that a single-precision
 *              evaluation of the objective cannot tell a rise from a fall, so
 *              the rule is the one a single-precision implementation can
 *              follow); if none does,
 *              y is kept and the remaining Newton steps of that outer loop are
 *              skipped.
 *   R-init   : default initial maps from per-image volume means (see
 *              orc_default_init).
 *   R-missing: a non-finite echo value is a missing observation: it adds
 *              nothing to the NLL, gradient or Hessian of its voxel (and is
 *              left out of the volume means of the default initialisation).
 *   R-rice   : noise estimation (Sec. 2.7): each image's histogram over
 *              [0, max] (bins decided in FP32), a two-class Rician mixture fitted
 *              to the bin centres by EM with the phase as latent variable, from
 *              the split of the histogram at its mean; the class started on the
 *              lower part is the background (air) and has no signal (nu = 0: a
 *              free nu converges only sublinearly along the flat nu-sigma ridge);
 *              a class's mean is its responsibility-weighted mean.
 *   R-basis  : in the rate and time representations (Sec. 3.1) the steps act
 *              on the values themselves; a step that would take A, R1 (T1) or
 *              R2* (T2*) to <= 0, or MTsat out of (0, 1), moves that parameter
 *              halfway to the boundary it would cross instead (the paper states
 *              no domain handling; see step_in_domain).
 */
#include "mpm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FROZEN_REL 1e-30
/* R-accept: the largest relative rise of F_w a step may bring and be accepted */
#define ACCEPT_REL 1e-9
#define PIVOT_MIN 1e-6
/* a voxel NLL "rises" only beyond rounding level (changes near convergence are ~1e-15) */
#define NLL_RISE_REL 1e-12

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Index of the contrast that image i belongs to (images are contrast-major). */
static int contrast_of(const orc_protocol *p, int i)
{
    int c = 0, first = 0;
    while (c < p->n_contrasts && i >= first + p->n_echoes[c]) {
        first += p->n_echoes[c];
        c++;
    }
    return c;
}

static int n_images(const orc_protocol *p)
{
    int I = 0;
    for (int c = 0; c < p->n_contrasts; c++) I += p->n_echoes[c];
    return I;
}

/* ------------------------------------------------------------------------
 * Forward model.
 *
 * Signal of a spoiled gradient echo with an optional MT pulse (TR2 = 0),
 * written in the log / logit parameters (Sec. 2.1 eqs. 1-3; Sec. 2.4 eq.
 * spgr_signal with a = exp(y0), r1 = exp(y1), r2 = exp(y2),
 * delta = 1/(1+exp(-y3))).  For contrasts without an MT pulse delta is 0 and
 * every derivative with respect to y3 is 0 (Sec. 2.4).
 *
 * ds and d2s are the first derivatives and the diagonal second derivatives
 * with respect to (y0..y3), in the form Sec. 2.4 prints them.
 * ------------------------------------------------------------------------ */
void orc_spgr_derivs(const double y[4], double alpha, double tr, double te, int mt,
                     double *s, double ds[4], double d2s[4])
{
    double a = exp(y[0]);
    double r1 = exp(y[1]);
    double r2 = exp(y[2]);
    double delta = mt ? 1.0 / (1.0 + exp(-y[3])) : 0.0;
    double e1 = exp(-r1 * tr);
    double ca = cos(alpha), sa = sin(alpha);
    double den = 1.0 - (1.0 - delta) * ca * e1;

    double sig = a * sa * (1.0 - delta) * (1.0 - e1) / den * exp(-r2 * te);
    *s = sig;

    ds[0] = sig;
    ds[1] = -tr * r1 * (((1.0 - delta) * ca - 1.0) * e1) / (den * (1.0 - e1)) * sig;
    ds[2] = -te * r2 * sig;
    ds[3] = mt ? delta / ((1.0 - delta) * ca * e1 - 1.0) * sig : 0.0;

    d2s[0] = ds[0];
    d2s[1] = (1.0 - tr * r1 * (1.0 + (1.0 - delta) * ca * e1) / den) * ds[1];
    d2s[2] = (1.0 - te * r2) * ds[2];
    d2s[3] = mt ? (2.0 * (1.0 - delta) * (1.0 - ca * e1) / den - 1.0) * ds[3] : 0.0;
}

/* The full 4x4 matrix of second derivatives of s with respect to (y0..y3),
 * row-major.  The paper prints only the diagonal (Sec. 2.4); the rest follows
 * from the same factorisation s = a * f(r1, delta) * exp(-r2 te):
 *   d2s/dy0 dyk = ds/dyk                 (s is proportional to a)
 *   d2s/dy1 dy2 = -te r2 ds/dy1          (ds/dy1 / s does not depend on r2)
 *   d2s/dy2 dy3 = -te r2 ds/dy3
 *   d2s/dy1 dy3 = s * (d phi/dy3 + phi psi), with phi = (ds/dy1)/s and
 *                 psi = (ds/dy3)/s; writing w = (1 - delta) cos(alpha),
 *                 E = exp(-r1 tr), x = r1 tr this is
 *                 -x E delta ((1 - w) - w (1 - E)) / ((1 - E)(1 - w E)^2) * s
 * (zero without an MT pulse).  The "Proposed+" loading of Sec. 2.3 needs the
 * absolute row sums of this matrix. */
void orc_spgr_hess(const double y[4], double alpha, double tr, double te, int mt, double H[16])
{
    double s, ds[4], d2s[4];
    orc_spgr_derivs(y, alpha, tr, te, mt, &s, ds, d2s);
    double r1 = exp(y[1]), r2 = exp(y[2]);
    double delta = mt ? 1.0 / (1.0 + exp(-y[3])) : 0.0;
    double e1 = exp(-r1 * tr);
    double w = (1.0 - delta) * cos(alpha);
    double x = r1 * tr;
    double chi = mt ? -x * e1 * delta * ((1.0 - w) - w * (1.0 - e1)) / ((1.0 - e1) * (1.0 - w * e1) * (1.0 - w * e1))
                    : 0.0;
    for (int k = 0; k < 16; k++) H[k] = 0.0;
    for (int k = 0; k < 4; k++) {
        H[4 * k + k] = d2s[k];
        H[k] = H[4 * k] = ds[k];
    }
    H[0] = d2s[0];
    H[4 * 1 + 2] = H[4 * 2 + 1] = -te * r2 * ds[1];
    H[4 * 2 + 3] = H[4 * 3 + 2] = -te * r2 * ds[3];
    H[4 * 1 + 3] = H[4 * 3 + 1] = chi * s;
}

/* Signal, gradient and full matrix of second derivatives (row-major) with
 * respect to the parameters of the rate basis, th = (A, R1, R2*, MTsat), or
 * of the time basis, th = (A, T1, T2*, MTsat) with R1 = 1/T1 and
 * R2* = 1/T2* (the two alternative representations of Sec. 3.1).  The signal
 * is the formula of Sec. 2.1 (eqs. 1-3, TR2 = 0) evaluated at these values as
 * they are, also outside the physical domain (reading R-basis).
 *
 * Written as s = A * F(R1, delta) * G(R2*) with E = exp(-R1 TR),
 * q = 1 - delta, c = cos(alpha), D = 1 - q c E:
 *   F = sin(alpha) q (1 - E) / D,            G = exp(-R2* TE),
 *   dF/dR1       = TR E sin(alpha) q (1 - q c) / D^2,
 *   d2F/dR1^2    = -TR^2 E sin(alpha) q (1 - q c)(1 + q c E) / D^3,
 *   dF/ddelta    = -sin(alpha) (1 - E) / D^2,
 *   d2F/ddelta^2 = 2 sin(alpha) (1 - E) c E / D^3,
 *   d2F/dR1 ddelta = TR E sin(alpha) (2 q c - 1 - q c E) / D^3,
 *   dG/dR2* = -TE G,  d2G/dR2*^2 = TE^2 G.
 * A parameter u with rate value R = rho(u) adds the factors rho' and rho''
 * (rate: 1 and 0; time: -R^2 and 2 R^3).  Without an MT pulse delta = 0 and
 * every derivative with respect to th[3] is 0. */
void orc_spgr_basis(const double th[4], int basis, double alpha, double tr, double te, int mt,
                    double *s, double ds[4], double H[16])
{
    double a = th[0];
    double r1 = basis == ORC_BASIS_TIME ? 1.0 / th[1] : th[1];
    double r2 = basis == ORC_BASIS_TIME ? 1.0 / th[2] : th[2];
    double delta = mt ? th[3] : 0.0;
    double j1 = 1.0, j1p = 0.0, j2 = 1.0, j2p = 0.0; /* rho' and rho'' */
    if (basis == ORC_BASIS_TIME) {
        j1 = -r1 * r1;
        j1p = 2.0 * r1 * r1 * r1;
        j2 = -r2 * r2;
        j2p = 2.0 * r2 * r2 * r2;
    }
    double E = exp(-r1 * tr);
    double sa = sin(alpha), c = cos(alpha);
    double q = 1.0 - delta;
    double D = 1.0 - q * c * E;

    double F = sa * q * (1.0 - E) / D;
    double F1 = tr * E * sa * q * (1.0 - q * c) / (D * D);
    double F11 = -tr * tr * E * sa * q * (1.0 - q * c) * (1.0 + q * c * E) / (D * D * D);
    double Fd = mt ? -sa * (1.0 - E) / (D * D) : 0.0;
    double Fdd = mt ? 2.0 * sa * (1.0 - E) * c * E / (D * D * D) : 0.0;
    double F1d = mt ? tr * E * sa * (2.0 * q * c - 1.0 - q * c * E) / (D * D * D) : 0.0;
    double G = exp(-r2 * te);
    double G2 = -te * G, G22 = te * te * G;

    /* derivatives with respect to th[1] and th[2] */
    double Fu = F1 * j1, Fuu = F11 * j1 * j1 + F1 * j1p, Fud = F1d * j1;
    double Gv = G2 * j2, Gvv = G22 * j2 * j2 + G2 * j2p;

    *s = a * F * G;
    ds[0] = F * G;
    ds[1] = a * Fu * G;
    ds[2] = a * F * Gv;
    ds[3] = a * Fd * G;
    H[0] = 0.0;
    H[1] = H[4] = Fu * G;
    H[2] = H[8] = F * Gv;
    H[3] = H[12] = Fd * G;
    H[5] = a * Fuu * G;
    H[6] = H[9] = a * Fu * Gv;
    H[7] = H[13] = a * Fud * G;
    H[10] = a * F * Gvv;
    H[11] = H[14] = a * Fd * Gv;
    H[15] = a * Fdd * G;
}

/* Noise-free echoes of every image at every voxel.  The flip angle of a voxel
 * is the nominal one times the transmit-field efficiency b1 (Sec. 2.4,
 * footnote on B1).  maps: [4][n]; b1: [n] or NULL (= 1); out: [I][n]. */
void orc_simulate(const orc_protocol *p, int64_t n, const double *maps,
                  const double *b1, double *out)
{
    int I = n_images(p);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; v++) {
        double y[4] = {maps[v], maps[n + v], maps[2 * n + v], maps[3 * n + v]};
        double b = b1 ? b1[v] : 1.0;
        for (int i = 0; i < I; i++) {
            int c = contrast_of(p, i);
            double s, ds[4], d2s[4];
            orc_spgr_derivs(y, p->flip[c] * b, p->tr[c], p->te[i], p->mt[c], &s, ds, d2s);
            out[(int64_t)i * n + v] = s;
        }
    }
}

/* ------------------------------------------------------------------------
 * Per-voxel likelihood block (Sec. 2.3 eq. chainrule and eq. precond;
 * Sec. 2.4, summed over every echo of every contrast).
 *
 *   nll = sum_i (s_i - x_i)^2 / (2 sigma_i^2)
 *   g   = sum_i (s_i - x_i) / sigma_i^2 * grad s_i
 *   P   = sum_i [ grad s_i grad s_i^T + |s_i - x_i| diag|d2 s_i| ] / sigma_i^2
 *
 * (R-sigma.)  With loading == ORC_LOAD_GN the |.| term is dropped, giving
 * the Gauss-Newton / Fisher-scoring matrix of Sec. 2.3; with
 * ORC_LOAD_PROPOSED_PLUS diag|d2 s_i| is replaced by the absolute row sums of
 * the full second-derivative matrix, diag(|H_s_i| 1) (the "Proposed+" choice
 * of Sec. 2.3, which majorises the Hessian of the NLL).
 * x points at image 0 of this voxel; image i is at x[i*stride].
 * P is the full 4x4 matrix, row-major.
 * ------------------------------------------------------------------------ */
static void lik_voxel(const orc_protocol *p, const double *x, int64_t stride, const double y[4], double b1,
                      int basis, int loading, double *nll, double g[4], double P[16])
{
    int I = n_images(p);
    double l = 0.0;
    for (int k = 0; k < 4; k++) g[k] = 0.0;
    for (int k = 0; k < 16; k++) P[k] = 0.0;
    for (int i = 0; i < I; i++) {
        int c = contrast_of(p, i);
        double s, ds[4], d2s[4];
        double xi = x[(int64_t)i * stride];
        if (!isfinite(xi)) continue; /* R-missing: no observation */
        double Hs[16];
        if (basis == ORC_BASIS_LOG) {
            orc_spgr_derivs(y, p->flip[c] * b1, p->tr[c], p->te[i], p->mt[c], &s, ds, d2s);
            if (loading == ORC_LOAD_PROPOSED_PLUS) orc_spgr_hess(y, p->flip[c] * b1, p->tr[c], p->te[i], p->mt[c], Hs);
        } else {
            orc_spgr_basis(y, basis, p->flip[c] * b1, p->tr[c], p->te[i], p->mt[c], &s, ds, Hs);
            for (int k = 0; k < 4; k++) d2s[k] = Hs[5 * k];
        }
        double res = s - xi;
        double wgt = 1.0 / (p->sigma[i] * p->sigma[i]);
        l += 0.5 * wgt * res * res;
        for (int k = 0; k < 4; k++) {
            g[k] += wgt * res * ds[k];
            for (int j = 0; j < 4; j++) P[4 * k + j] += wgt * ds[k] * ds[j];
            if (loading == ORC_LOAD_PROPOSED) P[4 * k + k] += wgt * fabs(res) * fabs(d2s[k]);
            if (loading == ORC_LOAD_PROPOSED_PLUS) {
                double rowsum = 0.0;
                for (int j = 0; j < 4; j++) rowsum += fabs(Hs[4 * k + j]);
                P[4 * k + k] += wgt * fabs(res) * rowsum;
            }
        }
    }
    *nll = l;
}

void orc_lik_voxel(const orc_protocol *p, const double *x, int64_t stride,
                   const double y[4], double b1, int loading,
                   double *nll, double g[4], double P[16])
{
    lik_voxel(p, x, stride, y, b1, ORC_BASIS_LOG, loading, nll, g, P);
}

/* The same block with respect to the parameters th of `basis` (ORC_BASIS_*),
 * from the derivatives of orc_spgr_basis (log basis: orc_lik_voxel). */
void orc_lik_voxel_basis(const orc_protocol *p, const double *x, int64_t stride,
                         const double th[4], int basis, int loading,
                         double *nll, double g[4], double P[16])
{
    lik_voxel(p, x, stride, th, 1.0, basis, loading, nll, g, P);
}

/* ------------------------------------------------------------------------
 * out = P^{-1} g for a symmetric 4x4 P, with the degenerate rule R-degen.
 * Returns 0 on success, 1 if the voxel was degenerate (out = 0).
 * ------------------------------------------------------------------------ */
int orc_solve4(const double P[16], const double g[4], double out[4])
{
    double maxd = 0.0;
    int ok = 1;
    for (int k = 0; k < 4; k++) {
        out[k] = 0.0;
        if (!isfinite(P[4 * k + k]) || !isfinite(g[k])) ok = 0;
        if (P[4 * k + k] > maxd) maxd = P[4 * k + k];
    }
    if (!ok || !(maxd > 0.0)) return 1;

    int frozen[4];
    double D[4], S[4][4], rhs[4], L[4][4], u[4];
    for (int k = 0; k < 4; k++) {
        frozen[k] = !(P[4 * k + k] > FROZEN_REL * maxd);
        D[k] = frozen[k] ? 0.0 : 1.0 / sqrt(P[4 * k + k]);
    }
    for (int k = 0; k < 4; k++) {
        for (int j = 0; j < 4; j++) {
            if (frozen[k] || frozen[j]) S[k][j] = (k == j) ? 1.0 : 0.0;
            else S[k][j] = D[k] * P[4 * k + j] * D[j];
        }
        rhs[k] = frozen[k] ? 0.0 : D[k] * g[k];
    }
    /* Cholesky S = L L^T */
    for (int j = 0; j < 4; j++) {
        double piv = S[j][j];
        for (int m = 0; m < j; m++) piv -= L[j][m] * L[j][m];
        if (!(piv >= PIVOT_MIN)) return 1;
        L[j][j] = sqrt(piv);
        for (int i = j + 1; i < 4; i++) {
            double v = S[i][j];
            for (int m = 0; m < j; m++) v -= L[i][m] * L[j][m];
            L[i][j] = v / L[j][j];
        }
    }
    /* L t = rhs, then L^T u = t */
    double t[4];
    for (int i = 0; i < 4; i++) {
        double v = rhs[i];
        for (int m = 0; m < i; m++) v -= L[i][m] * t[m];
        t[i] = v / L[i][i];
    }
    for (int i = 3; i >= 0; i--) {
        double v = t[i];
        for (int m = i + 1; m < 4; m++) v -= L[m][i] * u[m];
        u[i] = v / L[i][i];
    }
    for (int k = 0; k < 4; k++) out[k] = D[k] * u[k];
    return 0;
}

/* ------------------------------------------------------------------------
 * Joint total variation (Sec. 2.5).
 *
 * G_n holds the 6 forward and backward finite differences about voxel n
 * (R-border), so ||G_n y_k||^2 = sum over in-bounds neighbours m of
 * (y_k[m] - y_k[n])^2 and
 *     q_n = sum_k lambda_k ||G_n y_k||^2 .
 * The IRLS weights are the minimisers of the bound eq. bound,
 *     w_n = (q_n + eps^2)^(-1/2)             (R-eps),
 * and d_n = diag(G^T W G)_n = sum over in-bounds neighbours m of (w_n + w_m)
 * (the "cross kernel" of Sec. 2.5).  Returns sum_n sqrt(q_n + eps^2).
 * ------------------------------------------------------------------------ */
static int neighbours(const int64_t dims[3], int64_t n, int64_t nb[6])
{
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    int64_t x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
    int cnt = 0;
    if (x > 0) nb[cnt++] = n - 1;
    if (x < nx - 1) nb[cnt++] = n + 1;
    if (y > 0) nb[cnt++] = n - nx;
    if (y < ny - 1) nb[cnt++] = n + nx;
    if (z > 0) nb[cnt++] = n - nx * ny;
    if (z < nz - 1) nb[cnt++] = n + nx * ny;
    return cnt;
}

double orc_jtv_weights(const int64_t dims[3], const double *maps, const double lambda[4],
                       double eps, double *w, double *d)
{
    int64_t N = dims[0] * dims[1] * dims[2];
    double *root = (double *)malloc(sizeof(double) * (size_t)N);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int64_t nb[6];
        int cnt = neighbours(dims, n, nb);
        double q = 0.0;
        for (int k = 0; k < 4; k++) {
            double gk = 0.0;
            for (int j = 0; j < cnt; j++) {
                double diff = maps[k * N + nb[j]] - maps[k * N + n];
                gk += diff * diff;
            }
            q += lambda[k] * gk;
        }
        root[n] = sqrt(q + eps * eps);
        w[n] = root[n] > 0.0 ? 1.0 / root[n] : 0.0;
    }
    if (d) {
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; n++) {
            int64_t nb[6];
            int cnt = neighbours(dims, n, nb);
            double s = 0.0;
            for (int j = 0; j < cnt; j++) s += w[n] + w[nb[j]];
            d[n] = s;
        }
    }
    double jtv = 0.0;
    for (int64_t n = 0; n < N; n++) jtv += root[n];
    free(root);
    return jtv;
}

/* out = L v with L = G^T W G (x) diag(lambda), W = diag(w) (x) I_6 (Sec. 2.5):
 *   (L v)_k[n] = lambda_k * sum over in-bounds neighbours m of
 *                (w_n + w_m) (v_k[n] - v_k[m]).
 * v and out are [4][N]. */
void orc_apply_L(const int64_t dims[3], const double *w, const double lambda[4],
                 const double *v, double *out)
{
    int64_t N = dims[0] * dims[1] * dims[2];
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        int64_t nb[6];
        int cnt = neighbours(dims, n, nb);
        for (int k = 0; k < 4; k++) {
            double s = 0.0;
            for (int j = 0; j < cnt; j++) s += (w[n] + w[nb[j]]) * (v[k * N + n] - v[k * N + nb[j]]);
            out[k * N + n] = lambda[k] * s;
        }
    }
}

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* z = M^{-1} r with the block-diagonal preconditioner of Sec. 2.6,
 * M_n = P_n + diag(lambda_k d_n), solved per voxel with R-degen. */
static void precond(int64_t N, const double *P, const double *d, const double lambda[4],
                    const double *r, double *z)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        double M[16], rv[4], zv[4];
        memcpy(M, P + 16 * n, sizeof(M));
        for (int k = 0; k < 4; k++) {
            M[4 * k + k] += lambda[k] * d[n];
            rv[k] = r[k * N + n];
        }
        orc_solve4(M, rv, zv);
        for (int k = 0; k < 4; k++) z[k * N + n] = zv[k];
    }
}

/* q = (P + L) p */
static void apply_A(const int64_t dims[3], const double *P, const double *w,
                    const double lambda[4], const double *p, double *q)
{
    int64_t N = dims[0] * dims[1] * dims[2];
    orc_apply_L(dims, w, lambda, p, q);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++)
        for (int k = 0; k < 4; k++) {
            double s = 0.0;
            for (int j = 0; j < 4; j++) s += P[16 * n + 4 * k + j] * p[j * N + n];
            q[k * N + n] += s;
        }
}

/* ------------------------------------------------------------------------
 * Preconditioned conjugate gradient for (P + L) delta = b (Sec. 2.6), with
 * the block-Jacobi preconditioner P + (G^T W G o I) (x) diag(lambda)
 * (R-cg).  P: [N][16]; w, d, b, delta: [N] / [4][N].  Returns the number of
 * iterations executed.
 * ------------------------------------------------------------------------ */
int orc_pcg(const int64_t dims[3], const double *P, const double *w, const double *d,
            const double lambda[4], const double *b, int n_cg, double cg_stop, double *delta)
{
    int64_t N = dims[0] * dims[1] * dims[2];
    int64_t V = 4 * N;
    double *r = (double *)malloc(sizeof(double) * (size_t)V);
    double *z = (double *)malloc(sizeof(double) * (size_t)V);
    double *p = (double *)malloc(sizeof(double) * (size_t)V);
    double *q = (double *)malloc(sizeof(double) * (size_t)V);
    int it_done = 0;

    for (int64_t i = 0; i < V; i++) {
        delta[i] = 0.0;
        r[i] = b[i];
    }
    precond(N, P, d, lambda, r, z);
    memcpy(p, z, sizeof(double) * (size_t)V);
    double gamma = dot(r, z, V);
    double gamma0 = gamma;
    if (gamma0 > 0.0) {
        for (int it = 0; it < n_cg; it++) {
            apply_A(dims, P, w, lambda, p, q);
            double pq = dot(p, q, V);
            if (!(pq > 0.0)) break;
            double alpha = gamma / pq;
            for (int64_t i = 0; i < V; i++) {
                delta[i] += alpha * p[i];
                r[i] -= alpha * q[i];
            }
            precond(N, P, d, lambda, r, z);
            double gamma_new = dot(r, z, V);
            it_done++;
            if (gamma_new <= cg_stop * gamma0) break;
            double beta = gamma_new / gamma;
            gamma = gamma_new;
            for (int64_t i = 0; i < V; i++) p[i] = z[i] + beta * p[i];
        }
    }
    free(r);
    free(z);
    free(p);
    free(q);
    return it_done;
}

static double sum(const double *v, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += v[i];
    return s;
}

/* ------------------------------------------------------------------------
 * Spatial projection (Sec. 2.4, "Spatial projection"; reading R-proj).
 *
 * Contrast c is acquired on its own grid; acquisition voxel (i, j, k) lies at
 * reconstruction-grid coordinates r = A (i, j, k, 1)^T (A row-major 3x4).  The
 * reslicing Psi is trilinear interpolation with replicated borders (corner
 * indices clamped to the grid, so every row of Psi sums to 1); acquisition
 * voxels with r outside [-1/2, n_d - 1/2] in any axis d lie outside the
 * reconstruction field of view and carry no observation.
 * proj_weights: the 8 recon voxels and weights of acquisition voxel (i,j,k);
 * returns 0 outside the field of view.
 * ------------------------------------------------------------------------ */
static int proj_weights(const int64_t dims[3], const orc_space *sp, int64_t i, int64_t j, int64_t k,
                        int64_t idx[8], double wt[8])
{
    double r[3], t[3];
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
        const double *a = sp->affine + 4 * d;
        r[d] = a[0] * (double)i + a[1] * (double)j + a[2] * (double)k + a[3];
        if (!(r[d] >= -0.5 && r[d] <= (double)dims[d] - 0.5)) return 0;
        double f = floor(r[d]);
        t[d] = r[d] - f;
        lo[d] = (int64_t)f < 0 ? 0 : (int64_t)f;
        hi[d] = (int64_t)f + 1 > dims[d] - 1 ? dims[d] - 1 : (int64_t)f + 1;
    }
    for (int c = 0; c < 8; c++) {
        int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        int64_t x = bx ? hi[0] : lo[0], y = by ? hi[1] : lo[1], z = bz ? hi[2] : lo[2];
        idx[c] = x + dims[0] * (y + dims[1] * z);
        wt[c] = (bx ? t[0] : 1.0 - t[0]) * (by ? t[1] : 1.0 - t[1]) * (bz ? t[2] : 1.0 - t[2]);
    }
    return 1;
}

static int64_t space_voxels(const orc_space *sp) { return sp->dims[0] * sp->dims[1] * sp->dims[2]; }

/* out = Psi vol (0 outside the field of view).  vol: recon [N]; out: [M]. */
void orc_pull(const int64_t dims[3], const orc_space *sp, const double *vol, double *out)
{
    int64_t m = 0, idx[8];
    double wt[8];
    for (int64_t k = 0; k < sp->dims[2]; k++)
        for (int64_t j = 0; j < sp->dims[1]; j++)
            for (int64_t i = 0; i < sp->dims[0]; i++, m++) {
                double v = 0.0;
                if (proj_weights(dims, sp, i, j, k, idx, wt))
                    for (int c = 0; c < 8; c++) v += wt[c] * vol[idx[c]];
                out[m] = v;
            }
}

/* vol = Psi^T acq (the adjoint: push).  acq: [M]; vol: recon [N]. */
void orc_push(const int64_t dims[3], const orc_space *sp, const double *acq, double *vol)
{
    int64_t N = dims[0] * dims[1] * dims[2], m = 0, idx[8];
    double wt[8];
    for (int64_t n = 0; n < N; n++) vol[n] = 0.0;
    for (int64_t k = 0; k < sp->dims[2]; k++)
        for (int64_t j = 0; j < sp->dims[1]; j++)
            for (int64_t i = 0; i < sp->dims[0]; i++, m++)
                if (proj_weights(dims, sp, i, j, k, idx, wt))
                    for (int c = 0; c < 8; c++) vol[idx[c]] += wt[c] * acq[m];
}

/* Everything a likelihood evaluation needs.  spaces == NULL: every image on
 * the reconstruction grid, echoes [I][N]; otherwise images lie back to back,
 * image i holding the voxels of its contrast's space. */
typedef struct {
    const orc_protocol *p;
    const int64_t *dims;
    const orc_space *spaces;
    const double *x;
    const double *b1;
    const double *b1m; /* receive field [N] or NULL (reconstruction grid only) */
} lik_ctx;

/* The protocol restricted to contrast c. */
static orc_protocol sub_protocol(const orc_protocol *p, int c)
{
    orc_protocol q;
    memset(&q, 0, sizeof(q));
    int first = 0;
    for (int k = 0; k < c; k++) first += p->n_echoes[k];
    q.n_contrasts = 1;
    q.n_echoes[0] = p->n_echoes[c];
    q.tr[0] = p->tr[c];
    q.flip[0] = p->flip[c];
    q.mt[0] = p->mt[c];
    for (int e = 0; e < p->n_echoes[c]; e++) {
        q.te[e] = p->te[first + e];
        q.sigma[e] = p->sigma[first + e];
    }
    return q;
}

/* ------------------------------------------------------------------------
 * Likelihood of every voxel; returns the total NLL (summed in a fixed order).
 * maps: [4][N]; g: [4][N] or NULL; P: [N][16] or NULL.
 * Without projection nll[N] receives the per-voxel NLL.  With projection the
 * blocks are evaluated per acquisition voxel on the pulled maps (and pulled
 * b1) and pushed back: g_n = sum_m Psi_mn g_m and, as the block-diagonal
 * majoriser of Psi^T H Psi (Sec. 2.4), P_n = sum_m Psi_mn (sum_n' Psi_mn') P_m
 * = sum_m Psi_mn P_m; nll is not used.
 * ------------------------------------------------------------------------ */
static double lik_all(const lik_ctx *L, int loading, const double *maps, double *nll, double *g, double *P)
{
    const orc_protocol *p = L->p;
    const int64_t N = L->dims[0] * L->dims[1] * L->dims[2];
    if (!L->spaces) {
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; n++) {
            double y[4] = {maps[n], maps[N + n], maps[2 * N + n], maps[3 * N + n]};
            /* the receive field multiplies the signal: s = b- A f(...) = exp(log A + log b-) f(...),
             * so the likelihood, g and P~ are those at log A + log b- (Sec. 2.4) */
            if (L->b1m) y[0] += log(L->b1m[n]);
            double gl[4], Pl[16], l;
            orc_lik_voxel(p, L->x + n, N, y, L->b1 ? L->b1[n] : 1.0, loading, &l, gl, Pl);
            nll[n] = l;
            if (g)
                for (int k = 0; k < 4; k++) g[k * N + n] = gl[k];
            if (P) memcpy(P + 16 * n, Pl, sizeof(Pl));
        }
        return sum(nll, N);
    }
    if (g)
        for (int64_t i = 0; i < 4 * N; i++) g[i] = 0.0;
    if (P)
        for (int64_t i = 0; i < 16 * N; i++) P[i] = 0.0;
    double total = 0.0;
    const double *img = L->x; /* first image of contrast c */
    for (int c = 0; c < p->n_contrasts; c++) {
        const orc_space *sp = L->spaces + c;
        const int64_t M = space_voxels(sp);
        orc_protocol pc = sub_protocol(p, c);
        int64_t m = 0, idx[8];
        double wt[8];
        for (int64_t k = 0; k < sp->dims[2]; k++)
            for (int64_t j = 0; j < sp->dims[1]; j++)
                for (int64_t i = 0; i < sp->dims[0]; i++, m++) {
                    if (!proj_weights(L->dims, sp, i, j, k, idx, wt)) continue;
                    double y[4] = {0.0, 0.0, 0.0, 0.0}, b = 0.0;
                    for (int q = 0; q < 8; q++) {
                        for (int a = 0; a < 4; a++) y[a] += wt[q] * maps[a * N + idx[q]];
                        b += wt[q] * (L->b1 ? L->b1[idx[q]] : 1.0);
                    }
                    double gl[4], Pl[16], l;
                    orc_lik_voxel(&pc, img + m, M, y, b, loading, &l, gl, Pl);
                    total += l;
                    for (int q = 0; q < 8; q++) {
                        if (g)
                            for (int a = 0; a < 4; a++) g[a * N + idx[q]] += wt[q] * gl[a];
                        if (P)
                            for (int e = 0; e < 16; e++) P[16 * idx[q] + e] += wt[q] * Pl[e];
                    }
                }
        img += (int64_t)p->n_echoes[c] * M;
    }
    return total;
}

/* F_w(y) = sum_n nll_n + 1/2 y^T L y  (Sec. 2.6 objective at fixed weights). */
static double objective_w(const lik_ctx *L, int loading, const double *w, const double lambda[4],
                          const double *maps, double *nll_buf, double *Ly_buf)
{
    int64_t N = L->dims[0] * L->dims[1] * L->dims[2];
    double nll = lik_all(L, loading, maps, nll_buf, NULL, NULL);
    orc_apply_L(L->dims, w, lambda, maps, Ly_buf);
    return nll + 0.5 * dot(maps, Ly_buf, 4 * N);
}

static double logit(double v) { return log(v / (1.0 - v)); }

static double clampd(double v, double lo, double hi)
{
    if (!(v >= lo)) return lo;  /* also maps NaN to lo */
    if (v > hi) return hi;
    return v;
}

/* ------------------------------------------------------------------------
 * Default constant initial maps (R-init; the paper starts from constant maps
 * derived from per-volume means, Sec. 2.7, without saying how).
 *   1. m_i = mean over voxels of image i.
 *   2. log m_i = beta_c(i) - r2 * TE_i, least squares with one shared r2,
 *      giving TE = 0 intercepts S_c = exp(beta_c).
 *   3. Small-angle closed forms (the approximation of Helms et al. 2008 that
 *      the paper builds its MT model on, Sec. 2.1) for R1 and A from the two
 *      non-MT contrasts with the smallest (P) and largest (T) flip angle, and
 *      for delta from the first MT contrast (M); flip angles are scaled by the
 *      mean of b1.
 *   4. Clamp R1 to [0.05, 20], R2* to [0.5, 500], delta to [1e-4, 0.2].
 * Returns 0, or 1 when the protocol lacks the contrasts above.
 * ------------------------------------------------------------------------ */
/* Mean of the finite values of x[0..n) (NaN if there are none). */
static double finite_mean(const double *x, int64_t n)
{
    double s = 0.0;
    int64_t cnt = 0;
    for (int64_t v = 0; v < n; v++)
        if (isfinite(x[v])) {
            s += x[v];
            cnt++;
        }
    return cnt > 0 ? s / (double)cnt : NAN; /* no observation: left out below */
}

static int init_from_means(const orc_protocol *p, const double *m, double b1m, double y0[4]);

int orc_default_init(const orc_protocol *p, int64_t n, const double *x, const double *b1,
                     double y0[4])
{
    int I = n_images(p);
    double m[ORC_MAX_IMAGES];
    for (int i = 0; i < I; i++) m[i] = finite_mean(x + (int64_t)i * n, n);
    double b1m = 1.0;
    if (b1) {
        double s = 0.0;
        for (int64_t v = 0; v < n; v++) s += b1[v];
        b1m = s / (double)n;
    }
    return init_from_means(p, m, b1m, y0);
}

/* The same with projection: image i's mean runs over its own space. */
int orc_default_init_projected(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces,
                               const double *x, const double *b1, double y0[4])
{
    double m[ORC_MAX_IMAGES];
    int i = 0;
    const double *img = x;
    for (int c = 0; c < p->n_contrasts; c++) {
        int64_t M = space_voxels(spaces + c);
        for (int e = 0; e < p->n_echoes[c]; e++, i++, img += M) m[i] = finite_mean(img, M);
    }
    int64_t N = dims[0] * dims[1] * dims[2];
    double b1m = 1.0;
    if (b1) {
        double s = 0.0;
        for (int64_t v = 0; v < N; v++) s += b1[v];
        b1m = s / (double)N;
    }
    return init_from_means(p, m, b1m, y0);
}

static int init_from_means(const orc_protocol *p, const double *m, double b1m, double y0[4])
{
    int I = n_images(p), C = p->n_contrasts;
    /* normal equations of the (C+1)-unknown linear least squares */
    int U = C + 1;
    double A[ORC_MAX_CONTRASTS + 1][ORC_MAX_CONTRASTS + 2];
    memset(A, 0, sizeof(A));
    for (int i = 0; i < I; i++) {
        if (!isfinite(m[i])) continue;
        int c = contrast_of(p, i);
        double row[ORC_MAX_CONTRASTS + 1];
        memset(row, 0, sizeof(row));
        row[c] = 1.0;
        row[C] = -p->te[i];
        double rhs = log(m[i] > 1e-12 ? m[i] : 1e-12);
        for (int a = 0; a < U; a++) {
            for (int b = 0; b < U; b++) A[a][b] += row[a] * row[b];
            A[a][U] += row[a] * rhs;
        }
    }
    /* Gaussian elimination with partial pivoting */
    for (int col = 0; col < U; col++) {
        int piv = col;
        for (int r = col + 1; r < U; r++)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (fabs(A[piv][col]) < 1e-300) return 1;
        if (piv != col)
            for (int k = 0; k <= U; k++) {
                double t = A[col][k];
                A[col][k] = A[piv][k];
                A[piv][k] = t;
            }
        for (int r = 0; r < U; r++) {
            if (r == col) continue;
            double f = A[r][col] / A[col][col];
            for (int k = col; k <= U; k++) A[r][k] -= f * A[col][k];
        }
    }
    double beta[ORC_MAX_CONTRASTS + 1];
    for (int a = 0; a < U; a++) beta[a] = A[a][U] / A[a][a];
    double r2 = beta[C];

    int cP = -1, cT = -1, cM = -1;
    for (int c = 0; c < C; c++) {
        if (p->mt[c]) {
            if (cM < 0) cM = c;
            continue;
        }
        if (cP < 0 || p->flip[c] < p->flip[cP]) cP = c;
        if (cT < 0 || p->flip[c] > p->flip[cT]) cT = c;
    }
    if (cP < 0 || cT < 0 || cP == cT || cM < 0) return 1;
    double SP = exp(beta[cP]), ST = exp(beta[cT]), SM = exp(beta[cM]);
    double aP = p->flip[cP] * b1m, aT = p->flip[cT] * b1m, aM = p->flip[cM] * b1m;
    double tP = p->tr[cP], tT = p->tr[cT], tM = p->tr[cM];

    double R1 = 0.5 * (ST * aT / tT - SP * aP / tP) / (SP / aP - ST / aT);
    double Aa = SP * ST * (tP * aT / aP - tT * aP / aT) / (ST * tP * aT - SP * tT * aP);
    R1 = clampd(R1, 0.05, 20.0);
    if (!(Aa > 0.0) || !isfinite(Aa)) Aa = SP / sin(aP);
    double dl = (Aa * aM / SM - 1.0) * R1 * tM - 0.5 * aM * aM;
    dl = clampd(dl, 1e-4, 0.2);
    r2 = clampd(r2, 0.5, 500.0);

    y0[0] = log(Aa);
    y0[1] = log(R1);
    y0[2] = log(r2);
    y0[3] = logit(dl);
    return 0;
}

/* ------------------------------------------------------------------------
 * Full fit.
 *
 * ML (SPGR-ML, Sec. 3.3): n_gn Newton-like steps y <- y - P~^{-1} g taken
 * independently in every voxel (Sec. 2.3, Newton step with the approximate
 * Hessian of eq. precond); every step is taken, as the paper's method uses no
 * line search.
 *
 * MAP (SPGR+JTV, Sec. 2.5-2.7): IRLS.  For each outer loop t (from
 * start_outer, for resuming) the weights are refreshed (t >= 1; R-w0), then
 * n_gn Newton-like steps solve
 * (P~ + L) delta = g + L y by PCG (Sec. 2.6) and take y - 2^-h delta
 * (R-accept).
 *
 * maps: [4][N], initial values on entry when init_kind = FROM_MAPS, the
 * result on return.  trace (optional):
 *   ML : trace[j] = total NLL before step j, trace[n_gn] = final NLL;
 *   MAP: per outer loop t, slots t*(n_gn+2) + j: F_w before step 0 (j = 0)
 *        and after step j-1 (j = 1..n_gn), then the true objective
 *        NLL + sum sqrt(q + eps^2) at the end of the loop; skipped steps NaN.
 * Returns 0, or 1 on an unusable default initialisation.
 * ------------------------------------------------------------------------ */
static int fit_impl(const lik_ctx *L, const orc_options *opt, double *maps, orc_report *rep, double *trace,
                    int32_t trace_len)
{
    const orc_protocol *p = L->p;
    const int64_t *dims = L->dims;
    int64_t N = dims[0] * dims[1] * dims[2];
    int64_t V = 4 * N;
    orc_report R;
    memset(&R, 0, sizeof(R));
    for (int32_t i = 0; i < trace_len; i++) trace[i] = NAN;
    if (opt->basis != ORC_BASIS_LOG) return 1;

    if (opt->init_kind == ORC_INIT_CONST || opt->init_kind == ORC_INIT_DEFAULT) {
        double y0[4];
        if (opt->init_kind == ORC_INIT_CONST) {
            for (int k = 0; k < 4; k++) y0[k] = opt->init_const[k];
        } else if (L->spaces ? orc_default_init_projected(p, dims, L->spaces, L->x, L->b1, y0)
                             : orc_default_init(p, N, L->x, L->b1, y0)) {
            return 1;
        }
        for (int k = 0; k < 4; k++)
            for (int64_t n = 0; n < N; n++) maps[k * N + n] = y0[k];
    }

    double *nll = (double *)malloc(sizeof(double) * (size_t)N);
    double *g = (double *)malloc(sizeof(double) * (size_t)V);
    double *P = (double *)malloc(sizeof(double) * (size_t)N * 16);
    unsigned char *degen = (unsigned char *)calloc((size_t)N, 1);

    if (opt->mode == ORC_ML) {
        double *prev = (double *)malloc(sizeof(double) * (size_t)N);
        for (int it = 0; it < opt->n_gn; it++) {
            double tot = lik_all(L, opt->loading, maps, nll, g, P);
            if (trace && it < trace_len) trace[it] = tot;
            if (it > 0 && !L->spaces) /* per-voxel NLL exists only without projection */
                for (int64_t n = 0; n < N; n++)
                    if (nll[n] > prev[n] * (1.0 + NLL_RISE_REL)) R.nll_increases++;
            memcpy(prev, nll, sizeof(double) * (size_t)N);
#pragma omp parallel for schedule(static)
            for (int64_t n = 0; n < N; n++) {
                double gv[4] = {g[n], g[N + n], g[2 * N + n], g[3 * N + n]};
                double step[4];
                degen[n] = (unsigned char)orc_solve4(P + 16 * n, gv, step);
                for (int k = 0; k < 4; k++) maps[k * N + n] -= step[k];
            }
            R.gn_done++;
        }
        R.nll = lik_all(L, opt->loading, maps, nll, NULL, NULL);
        if (opt->n_gn > 0 && !L->spaces)
            for (int64_t n = 0; n < N; n++)
                if (nll[n] > prev[n] * (1.0 + NLL_RISE_REL)) R.nll_increases++;
        R.objective = R.nll;
        if (trace && opt->n_gn < trace_len) trace[opt->n_gn] = R.nll;
        for (int64_t n = 0; n < N; n++) R.degenerate_voxels += degen[n];
        free(prev);
    } else {
        double lam_sum = opt->lambda[0] + opt->lambda[1] + opt->lambda[2] + opt->lambda[3];
        double eps = opt->jtv_eps > 0.0 ? opt->jtv_eps : 1e-3 * sqrt(lam_sum);
        double cg_stop = opt->cg_stop > 0.0 ? opt->cg_stop : 0.0;
        double *w = (double *)calloc((size_t)N, sizeof(double));
        double *d = (double *)calloc((size_t)N, sizeof(double));
        double *Ly = (double *)malloc(sizeof(double) * (size_t)V);
        double *b = (double *)malloc(sizeof(double) * (size_t)V);
        double *delta = (double *)malloc(sizeof(double) * (size_t)V);
        double *trial = (double *)malloc(sizeof(double) * (size_t)V);
        int slots = opt->n_gn + 2;
        /* early stopping (reading R-stop): the gain of a step is the decrease it
         * brings over the decrease since the first value of its sequence */
        double F_loop0 = 0.0, obj_first = 0.0, obj_prev = 0.0;
        int n_obj = 0;

        for (int t = opt->start_outer > 0 ? opt->start_outer : 0; t < opt->n_outer; t++) {
            if (t >= 1 && lam_sum > 0.0) orc_jtv_weights(dims, maps, opt->lambda, eps, w, d);
            for (int j = 0; j < opt->n_gn; j++) {
                double tot = lik_all(L, opt->loading, maps, nll, g, P);
                orc_apply_L(dims, w, opt->lambda, maps, Ly);
                double F = tot + 0.5 * dot(maps, Ly, V);
                if (j == 0) F_loop0 = F;
                if (trace && j == 0 && t * slots < trace_len) trace[t * slots] = F;
                for (int64_t i = 0; i < V; i++) b[i] = g[i] + Ly[i];
                R.cg_done += orc_pcg(dims, P, w, d, opt->lambda, b, opt->n_cg, cg_stop, delta);

                int accepted = 0;
                double Fnew = F;
                if (opt->max_halvings < 0) {
                    for (int64_t i = 0; i < V; i++) maps[i] -= delta[i];
                    Fnew = objective_w(L, opt->loading, w, opt->lambda, maps, nll, Ly);
                    accepted = 1;
                } else {
                    double step = 1.0;
                    for (int h = 0; h <= opt->max_halvings; h++) {
                        for (int64_t i = 0; i < V; i++) trial[i] = maps[i] - step * delta[i];
                        double Ft = objective_w(L, opt->loading, w, opt->lambda, trial, nll, Ly);
                        if (Ft <= F + ACCEPT_REL * fabs(F)) {
                            memcpy(maps, trial, sizeof(double) * (size_t)V);
                            Fnew = Ft;
                            accepted = 1;
                            break;
                        }
                        step *= 0.5;
                    }
                }
                if (!accepted) {
                    R.rejected++;
                    break;
                }
                R.gn_done++;
                if (trace && t * slots + j + 1 < trace_len) trace[t * slots + j + 1] = Fnew;
                if (opt->tol_gn > 0.0) {
                    const double den = F_loop0 - Fnew;
                    if (!(den > 0.0) || F - Fnew < opt->tol_gn * den) break;
                }
            }
            R.outer_done++;
            if ((trace && t * slots + opt->n_gn + 1 < trace_len) || opt->tol_outer > 0.0) {
                double jt = lam_sum > 0.0 ? orc_jtv_weights(dims, maps, opt->lambda, eps, Ly, NULL) : 0.0;
                const double O = lik_all(L, opt->loading, maps, nll, NULL, NULL) + jt;
                if (trace && t * slots + opt->n_gn + 1 < trace_len) trace[t * slots + opt->n_gn + 1] = O;
                if (opt->tol_outer > 0.0) {
                    int stop = 0;
                    if (n_obj == 0) {
                        obj_first = O;
                    } else {
                        const double den = obj_first - O;
                        stop = !(den > 0.0) || obj_prev - O < opt->tol_outer * den;
                    }
                    obj_prev = O;
                    n_obj++;
                    if (stop) break;
                }
            }
        }
        /* final weights, objective and degenerate count (R-w0) */
        double jt = 0.0;
        if (lam_sum > 0.0) jt = orc_jtv_weights(dims, maps, opt->lambda, eps, w, d);
        else
            for (int64_t n = 0; n < N; n++) w[n] = d[n] = 0.0;
        R.nll = lik_all(L, opt->loading, maps, nll, NULL, P);
        R.jtv = jt;
        R.objective = R.nll + jt;
        for (int64_t n = 0; n < N; n++) {
            double M[16], e[4] = {1.0, 0.0, 0.0, 0.0}, o[4];
            memcpy(M, P + 16 * n, sizeof(M));
            for (int k = 0; k < 4; k++) M[4 * k + k] += opt->lambda[k] * d[n];
            R.degenerate_voxels += orc_solve4(M, e, o);
        }
        free(w);
        free(d);
        free(Ly);
        free(b);
        free(delta);
        free(trial);
    }
    for (int64_t n = 0; n < N; n++) {
        int bad = 0;
        for (int k = 0; k < 4; k++)
            if (!isfinite(maps[k * N + n])) bad = 1;
        R.nonfinite_voxels += bad;
    }
    free(nll);
    free(g);
    free(P);
    free(degen);
    if (rep) *rep = R;
    return 0;
}

int orc_fit(const orc_protocol *p, const int64_t dims[3], const double *x, const double *b1,
            const orc_options *opt, double *maps, orc_report *rep, double *trace, int32_t trace_len)
{
    lik_ctx L = {p, dims, NULL, x, b1, opt->b1_receive};
    return fit_impl(&L, opt, maps, rep, trace, trace_len);
}

/* ------------------------------------------------------------------------
 * Per-voxel protocols (the convergence experiment of Sec. 3.1): voxel n has
 * its own TR and flip angle per contrast, tr[c*N + n] and flip[c*N + n], and
 * its own echo times te[i*N + n]; the contrast/echo structure, MT flags and
 * noise levels come from shape (its tr, flip and te are ignored).  Each voxel
 * takes opt->n_gn Newton-like steps y <- y - P~^{-1} g (Sec. 2.3) from
 * init_const (ORC_INIT_CONST) or from maps (ORC_INIT_FROM_MAPS), as the ML
 * fit does, on the parameters of opt->basis (the representation comparison of
 * Sec. 3.1; maps and init_const are in that basis).  increases[n] (optional) counts the steps after which the
 * voxel's NLL exceeds the one before by more than rise_rel (relative), or
 * becomes non-finite from a finite value; nll[n] (optional) is the final NLL.
 * Returns 0, or 1 if the options are not an ML fit with a given start.
 * ------------------------------------------------------------------------ */
/* One parameter's Newton-like update u - step (reading R-basis): the log
 * basis has no bounds; in the rate and time bases A, R1 (T1) and R2* (T2*)
 * must stay > 0 and MTsat in (0, 1), and a step that would leave that domain
 * moves the parameter halfway to the boundary it would cross instead. */
static double step_in_domain(int basis, int k, double u, double step)
{
    double v = u - step;
    if (basis == ORC_BASIS_LOG || !isfinite(v)) return v;
    if (!(v > 0.0)) return 0.5 * u;
    if (k == 3 && !(v < 1.0)) return 0.5 * (1.0 + u);
    return v;
}

int orc_fit_voxelwise(const orc_protocol *shape, int64_t N, const double *tr, const double *flip, const double *te,
                      const double *x, const orc_options *opt, double rise_rel, double *maps, int32_t *increases,
                      double *nll, orc_report *rep)
{
    if (opt->mode != ORC_ML || (opt->init_kind != ORC_INIT_CONST && opt->init_kind != ORC_INIT_FROM_MAPS)) return 1;
    if (opt->basis < ORC_BASIS_LOG || opt->basis > ORC_BASIS_TIME) return 1;
    const int C = shape->n_contrasts;
    int I = 0;
    for (int c = 0; c < C; c++) I += shape->n_echoes[c];
    /* per-voxel results; the totals are serial sums in voxel order */
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    double *fnll = (double *)malloc(sizeof(double) * (size_t)N);
    unsigned char *degen = (unsigned char *)malloc((size_t)N);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t n = 0; n < N; n++) {
        orc_protocol pv = *shape;
        for (int c = 0; c < C; c++) {
            pv.tr[c] = tr[c * N + n];
            pv.flip[c] = flip[c * N + n];
        }
        for (int i = 0; i < I; i++) pv.te[i] = te[i * N + n];
        double y[4];
        for (int k = 0; k < 4; k++) y[k] = opt->init_kind == ORC_INIT_CONST ? opt->init_const[k] : maps[k * N + n];
        double prev = 0.0, cur = 0.0, g[4], P[16];
        int count = 0, dg = 0;
        for (int it = 0; it <= opt->n_gn; it++) {
            lik_voxel(&pv, x + n, N, y, 1.0, opt->basis, opt->loading, &cur, g, P);
            if (it > 0 && (cur > prev * (1.0 + rise_rel) || (isfinite(prev) && !isfinite(cur)))) count++;
            prev = cur;
            if (it == opt->n_gn) break;
            double step[4];
            dg = orc_solve4(P, g, step);
            for (int k = 0; k < 4; k++) y[k] = step_in_domain(opt->basis, k, y[k], step[k]);
        }
        for (int k = 0; k < 4; k++) maps[k * N + n] = y[k];
        cnt[n] = count;
        fnll[n] = cur;
        degen[n] = (unsigned char)dg;
    }
    orc_report R;
    memset(&R, 0, sizeof(R));
    for (int64_t n = 0; n < N; n++) {
        int fin = 1;
        for (int k = 0; k < 4; k++) fin &= isfinite(maps[k * N + n]) != 0;
        R.nll += fnll[n];
        R.nll_increases += cnt[n];
        R.degenerate_voxels += opt->n_gn > 0 ? degen[n] : 0;
        R.nonfinite_voxels += !fin;
        if (increases) increases[n] = cnt[n];
        if (nll) nll[n] = fnll[n];
    }
    R.objective = R.nll;
    R.gn_done = opt->n_gn;
    if (rep) *rep = R;
    free(cnt);
    free(fnll);
    free(degen);
    return 0;
}

/* The fit with spatial projection (R-proj): spaces[c] is the acquisition
 * space of contrast c; echoes lie back to back (image i holds the voxels of
 * its contrast's space); maps and b1 live on the reconstruction grid dims.
 * ML takes the Newton-like step y <- y - P~^{-1} g with the pushed blocks. */
int orc_fit_projected(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces, const double *x,
                      const double *b1, const orc_options *opt, double *maps, orc_report *rep, double *trace,
                      int32_t trace_len)
{
    lik_ctx L = {p, dims, spaces, x, b1};
    return fit_impl(&L, opt, maps, rep, trace, trace_len);
}

/* Total NLL, pushed gradient g [4][N] and pushed blocks P [N][16] (either may
 * be NULL) at maps, with projection. */
double orc_proj_lik(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces, const double *x,
                    const double *b1, int loading, const double *maps, double *g, double *P)
{
    lik_ctx L = {p, dims, spaces, x, b1};
    return lik_all(&L, loading, maps, NULL, g, P);
}

/* ------------------------------------------------------------------------
 * Laplace posterior variance (Sec. 3.6): the diagonal of
 * (P~ + diag(G^T W G) (x) diag(lambda))^{-1} at the fitted maps, with W from
 * the fitted maps (lambda = 0 / ML mode: the diagonal of P~^{-1}).  Frozen
 * parameters and degenerate voxels (R-degen) get +inf.
 * moments (optional, [4][N]): E[r1], V[r1], E[t1], V[t1] of the log-normal
 * posterior of r1 = exp(y1) and t1 = exp(-y1) (Sec. 3.6).
 * ------------------------------------------------------------------------ */
static int uncertainty_impl(const lik_ctx *L, const orc_options *opt, const double *maps, double *var,
                            double *moments)
{
    if (opt->basis != ORC_BASIS_LOG) return 1;
    const int64_t *dims = L->dims;
    int64_t N = dims[0] * dims[1] * dims[2];
    double lam[4] = {0.0, 0.0, 0.0, 0.0};
    double *d = (double *)calloc((size_t)N, sizeof(double));
    double *nll = (double *)malloc(sizeof(double) * (size_t)N);
    double *P = (double *)malloc(sizeof(double) * (size_t)N * 16);
    if (opt->mode == ORC_MAP) {
        double lam_sum = opt->lambda[0] + opt->lambda[1] + opt->lambda[2] + opt->lambda[3];
        if (lam_sum > 0.0) {
            double eps = opt->jtv_eps > 0.0 ? opt->jtv_eps : 1e-3 * sqrt(lam_sum);
            double *w = (double *)malloc(sizeof(double) * (size_t)N);
            orc_jtv_weights(dims, maps, opt->lambda, eps, w, d);
            free(w);
            for (int k = 0; k < 4; k++) lam[k] = opt->lambda[k];
        }
    }
    lik_all(L, opt->loading, maps, nll, NULL, P);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; n++) {
        double M[16];
        memcpy(M, P + 16 * n, sizeof(M));
        for (int k = 0; k < 4; k++) M[4 * k + k] += lam[k] * d[n];
        double maxd = 0.0;
        for (int k = 0; k < 4; k++)
            if (M[4 * k + k] > maxd) maxd = M[4 * k + k];
        for (int k = 0; k < 4; k++) {
            double e[4] = {0.0, 0.0, 0.0, 0.0}, col[4];
            e[k] = 1.0;
            int frozen = !(M[4 * k + k] > FROZEN_REL * maxd);
            if (frozen || orc_solve4(M, e, col)) var[k * N + n] = INFINITY;
            else var[k * N + n] = col[k];
        }
        if (moments) {
            double v = var[N + n], r1t = maps[N + n];
            double ev = exp(v);
            moments[n] = sqrt(ev) * exp(r1t);
            moments[N + n] = (ev - 1.0) * ev * exp(r1t) * exp(r1t);
            moments[2 * N + n] = sqrt(ev) * exp(-r1t);
            moments[3 * N + n] = (ev - 1.0) * ev * exp(-r1t) * exp(-r1t);
        }
    }
    free(d);
    free(nll);
    free(P);
    return 0;
}

int orc_uncertainty(const orc_protocol *p, const int64_t dims[3], const double *x, const double *b1,
                    const orc_options *opt, const double *maps, double *var, double *moments)
{
    lik_ctx L = {p, dims, NULL, x, b1, opt->b1_receive};
    return uncertainty_impl(&L, opt, maps, var, moments);
}

int orc_uncertainty_projected(const orc_protocol *p, const int64_t dims[3], const orc_space *spaces,
                              const double *x, const double *b1, const orc_options *opt, const double *maps,
                              double *var, double *moments)
{
    lik_ctx L = {p, dims, spaces, x, b1};
    return uncertainty_impl(&L, opt, maps, var, moments);
}

/* ------------------------------------------------------------------------
 * Noise estimation (Sec. 2.7): per acquired volume, a two-class Rician
 * mixture fitted to the image histogram; the class with the lower mean is the
 * background, whose sigma is the noise level; variances of the echoes of one
 * contrast are averaged with the geometric mean, and the mean of the other
 * class feeds the constant initial maps.
 * ------------------------------------------------------------------------ */

/* e^-z I0(z), e^-z I1(z): the power series
 *   I0(z) = sum_k (z^2/4)^k / (k!)^2,  I1(z) = (z/2) sum_k (z^2/4)^k / (k! (k+1)!)
 * for z <= 25 (summed until a term is below 1e-17 of the sum), else the
 * large-argument expansion
 *   I_v(z) ~ e^z / sqrt(2 pi z) sum_k (-1)^k a_k(v) / z^k,
 *   a_k(v) = prod_{j=1..k} (4 v^2 - (2j - 1)^2) / (k! 8^k),
 * to 30 terms (at z > 25 the terms shrink past 1e-17 before they grow). */
void orc_bessel_i01e(double z, double *i0e, double *i1e)
{
    if (z <= 25.0) {
        double q = 0.25 * z * z, t0 = 1.0, t1 = 1.0, s0 = 1.0, s1 = 1.0;
        for (int k = 1; k < 500; k++) {
            t0 *= q / ((double)k * (double)k);
            t1 *= q / ((double)k * (double)(k + 1));
            s0 += t0;
            s1 += t1;
            if (t0 < 1e-17 * s0 && t1 < 1e-17 * s1) break;
        }
        double e = exp(-z);
        *i0e = s0 * e;
        *i1e = 0.5 * z * s1 * e;
        return;
    }
    double s0 = 1.0, s1 = 1.0, a0 = 1.0, a1 = 1.0;
    for (int k = 1; k <= 30; k++) {
        double odd = (double)(2 * k - 1) * (double)(2 * k - 1);
        a0 *= -(0.0 - odd) / ((double)k * 8.0 * z);
        a1 *= -(4.0 - odd) / ((double)k * 8.0 * z);
        s0 += a0;
        s1 += a1;
    }
    double f = 1.0 / sqrt(2.0 * 3.14159265358979323846 * z);
    *i0e = f * s0;
    *i1e = f * s1;
}

float orc_histogram(const double *x, int64_t n, int nbins, int64_t *counts)
{
    float mx = 0.0f;
    for (int64_t v = 0; v < n; v++) {
        float f = (float)x[v];
        if (isfinite(f) && f > mx) mx = f;
    }
    for (int b = 0; b < nbins; b++) counts[b] = 0;
    if (!(mx > 0.0f)) return 0.0f;
    float scale = (float)nbins / mx;
    for (int64_t v = 0; v < n; v++) {
        float f = (float)x[v];
        if (!isfinite(f) || f < 0.0f) continue;
        int b = (int)(f * scale);
        counts[b < nbins ? b : nbins - 1]++;
    }
    return scale;
}

/* log of the Rice density at c, and the posterior mean of cos(phase),
 * I1(z)/I0(z) with z = c nu / sigma^2:
 *   log p = log c - 2 log sigma - (c - nu)^2 / (2 sigma^2) + log(e^-z I0(z)). */
static double rice_logpdf(double c, double nu, double sigma, double *ratio)
{
    double s2 = sigma * sigma;
    double i0e, i1e;
    orc_bessel_i01e(c * nu / s2, &i0e, &i1e);
    *ratio = i1e / i0e;
    return log(c) - 2.0 * log(sigma) - (c - nu) * (c - nu) / (2.0 * s2) + log(i0e);
}

int orc_rice_mixture(const int64_t *counts, int nbins, double scale, int n_iter, double pi[2], double nu[2],
                     double sigma[2], double mean[2], double *nll)
{
    double width = 1.0 / scale;
    /* initial split at the mean of the values */
    double tot = 0.0, m = 0.0;
    for (int b = 0; b < nbins; b++) {
        tot += (double)counts[b];
        m += (double)counts[b] * (b + 0.5) * width;
    }
    if (!(tot > 0.0)) return 1;
    m /= tot;
    double w[2] = {0.0, 0.0}, s1[2] = {0.0, 0.0}, s2[2] = {0.0, 0.0};
    for (int b = 0; b < nbins; b++) {
        double c = (b + 0.5) * width;
        int k = c < m ? 0 : 1;
        w[k] += (double)counts[b];
        s1[k] += (double)counts[b] * c;
        s2[k] += (double)counts[b] * c * c;
    }
    if (!(w[0] > 0.0) || !(w[1] > 0.0)) return 1;
    for (int k = 0; k < 2; k++) {
        pi[k] = w[k] / tot;
        nu[k] = s1[k] / w[k];
        double var = s2[k] / w[k] - nu[k] * nu[k];
        sigma[k] = sqrt(var > width * width ? var : width * width);
    }
    /* class 0 is the background: air carries no signal, nu = 0 (Rayleigh) */
    nu[0] = 0.0;
    sigma[0] = sqrt(0.5 * s2[0] / w[0]);
    /* EM: the phase of each value is the latent variable (the magnitude of a
     * complex Gaussian of mean nu and variance sigma^2 per part) */
    for (int it = 0; it <= n_iter; it++) {
        double N[2] = {0.0, 0.0}, Sx[2] = {0.0, 0.0}, Sx2[2] = {0.0, 0.0}, Sxa[2] = {0.0, 0.0}, L = 0.0;
        for (int b = 0; b < nbins; b++) {
            if (!counts[b]) continue;
            double c = (b + 0.5) * width, n = (double)counts[b];
            double lp[2], ra[2];
            for (int k = 0; k < 2; k++) lp[k] = log(pi[k]) + rice_logpdf(c, nu[k], sigma[k], &ra[k]);
            double mx = lp[0] > lp[1] ? lp[0] : lp[1];
            double lse = mx + log(exp(lp[0] - mx) + exp(lp[1] - mx));
            L -= n * lse;
            for (int k = 0; k < 2; k++) {
                double r = n * exp(lp[k] - lse);
                N[k] += r;
                Sx[k] += r * c;
                Sx2[k] += r * c * c;
                Sxa[k] += r * c * ra[k];
            }
        }
        if (nll) nll[it] = L;
        if (it == n_iter) {
            for (int k = 0; k < 2; k++) mean[k] = Sx[k] / N[k];
            break;
        }
        for (int k = 0; k < 2; k++) {
            pi[k] = N[k] / tot;
            nu[k] = k == 0 ? 0.0 : Sxa[k] / N[k];
            sigma[k] = sqrt(0.5 * (Sx2[k] / N[k] - nu[k] * nu[k]));
        }
    }
    return 0;
}

int orc_estimate_noise(const orc_protocol *p, int64_t n, const double *x, const double *b1, int nbins, int n_iter,
                       double *sigma_image, double *sigma_contrast, double *fg_mean, double y0[4])
{
    int I = n_images(p);
    int64_t *counts = (int64_t *)malloc(sizeof(int64_t) * (size_t)nbins);
    int bad = 0;
    for (int i = 0; i < I && !bad; i++) {
        double scale = orc_histogram(x + (int64_t)i * n, n, nbins, counts);
        double pi[2], nu[2], sg[2], mn[2];
        if (!(scale > 0.0) || orc_rice_mixture(counts, nbins, scale, n_iter, pi, nu, sg, mn, NULL)) {
            bad = 1;
            break;
        }
        int bg = mn[0] <= mn[1] ? 0 : 1;
        sigma_image[i] = sg[bg];
        fg_mean[i] = mn[1 - bg];
    }
    free(counts);
    if (bad) return 1;
    int first = 0;
    for (int c = 0; c < p->n_contrasts; c++) {
        double lv = 0.0;
        for (int e = 0; e < p->n_echoes[c]; e++) lv += log(sigma_image[first + e] * sigma_image[first + e]);
        sigma_contrast[c] = sqrt(exp(lv / p->n_echoes[c]));
        first += p->n_echoes[c];
    }
    double b1m = 1.0;
    if (b1) {
        double s = 0.0;
        for (int64_t v = 0; v < n; v++) s += b1[v];
        b1m = s / (double)n;
    }
    return init_from_means(p, fg_mean, b1m, y0);
}

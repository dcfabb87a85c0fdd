// mpm_api.hip -- the C ABI of libmpm (declared in include/mpm.h): argument
// validation, workspace management, kernel orchestration and kernel timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_proj.h"
#include "mpm_api_internal.h"
#include "mpm_kernels.h"

using namespace mpm;

namespace mpm {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_last_error;

mpm_status fail(mpm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return st;
}

void clear_error() { t_last_error.clear(); }

// ---------------------------------------------------------------------------
// kernel timing registry
// ---------------------------------------------------------------------------
static std::mutex g_prof_mu;
static std::vector<mpm_kernel_stat> g_stats;
static int g_every = 0;

static int stat_id(const char *name)
{
    for (size_t i = 0; i < g_stats.size(); i++)
        if (!strcmp(g_stats[i].name, name)) return (int)i;
    mpm_kernel_stat s;
    memset(&s, 0, sizeof(s));
    snprintf(s.name, sizeof(s.name), "%s", name);
    g_stats.push_back(s);
    return (int)g_stats.size() - 1;
}

hipError_t Prof::launch(const char *name, double bytes, const std::function<hipError_t()> &fn)
{
    int every, id;
    int64_t count;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        every = g_every;
        id = stat_id(name);
        count = g_stats[id].launches++;
        g_stats[id].bytes += bytes;
    }
    bool timed = every > 0 && (count % every) == 0;
    hipEvent_t a = nullptr, b = nullptr;
    if (timed) {
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) timed = false;
        else hipEventRecord(a, stream);
    }
    hipError_t e = fn();
    if (timed) {
        hipEventRecord(b, stream);
        pend.push_back({id, a, b});
    }
    return e;
}

void Prof::collect()
{
    for (auto &p : pend) {
        float ms = 0.f;
        hipEventSynchronize(p.b);
        hipEventElapsedTime(&ms, p.a, p.b);
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_stats[p.id].timed++;
        g_stats[p.id].timed_ms += ms;
    }
    pend.clear();
}

Prof::~Prof()
{
    for (auto &p : pend) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
int n_images(const mpm_protocol *p)
{
    int I = 0;
    for (int c = 0; c < p->n_contrasts; c++) I += p->n_echoes[c];
    return I;
}

mpm_status check_protocol(const mpm_protocol *p)
{
    if (!p) return fail(MPM_ERR_INVALID_ARG, "protocol is NULL");
    if (p->n_contrasts < 1 || p->n_contrasts > MPM_MAX_CONTRASTS)
        return fail(MPM_ERR_INVALID_ARG, "n_contrasts=%d outside [1, %d]", p->n_contrasts, MPM_MAX_CONTRASTS);
    int I = 0;
    for (int c = 0; c < p->n_contrasts; c++) {
        if (p->n_echoes[c] < 1) return fail(MPM_ERR_INVALID_ARG, "contrast %d has %d echoes", c, p->n_echoes[c]);
        I += p->n_echoes[c];
        if (I > MPM_MAX_IMAGES) return fail(MPM_ERR_INVALID_ARG, "more than %d images", MPM_MAX_IMAGES);
        if (!(p->tr_s[c] > 0.0) || !std::isfinite(p->tr_s[c]))
            return fail(MPM_ERR_INVALID_ARG, "contrast %d: TR must be > 0", c);
        if (!(p->flip_rad[c] > 0.0) || !(p->flip_rad[c] < M_PI))
            return fail(MPM_ERR_INVALID_ARG, "contrast %d: flip angle must be in (0, pi)", c);
        if (p->mt[c] != 0 && p->mt[c] != 1) return fail(MPM_ERR_INVALID_ARG, "contrast %d: mt must be 0 or 1", c);
    }
    for (int i = 0; i < I; i++) {
        if (!(p->te_s[i] >= 0.0) || !std::isfinite(p->te_s[i]))
            return fail(MPM_ERR_INVALID_ARG, "image %d: TE must be >= 0", i);
        if (!(p->sigma[i] > 0.0) || !std::isfinite(p->sigma[i]))
            return fail(MPM_ERR_INVALID_ARG, "image %d: sigma must be > 0", i);
    }
    return MPM_OK;
}

mpm_status check_grid(const mpm_grid *g, int64_t *N)
{
    if (!g) return fail(MPM_ERR_INVALID_ARG, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(MPM_ERR_INVALID_ARG, "grid %lld x %lld x %lld has an empty axis", (long long)g->nx,
                    (long long)g->ny, (long long)g->nz);
    if (g->nx > (1 << 20) || g->ny > (1 << 20) || g->nz > (1 << 20))
        return fail(MPM_ERR_INVALID_ARG, "grid axis longer than 2^20");
    int64_t n = g->nx * g->ny * g->nz;
    // byte offsets into one echo image are 32-bit in the kernels
    if (n > ((int64_t)1 << 30) - 1) return fail(MPM_ERR_INVALID_ARG, "grid has more than 2^30-1 voxels");
    *N = n;
    return MPM_OK;
}

mpm_status check_dtype(int dtype)
{
    if (dtype != MPM_F32 && dtype != MPM_F16 && dtype != MPM_BF16)
        return fail(MPM_ERR_INVALID_ARG, "unknown echo dtype %d", dtype);
    return MPM_OK;
}

mpm_status check_spaces(const mpm_protocol *p, const mpm_space *spaces)
{
    if (!spaces) return fail(MPM_ERR_INVALID_ARG, "spaces is NULL");
    for (int c = 0; c < p->n_contrasts; c++) {
        const mpm_space &sp = spaces[c];
        if (sp.nx < 1 || sp.ny < 1 || sp.nz < 1 || sp.nx > (1 << 20) || sp.ny > (1 << 20) || sp.nz > (1 << 20))
            return fail(MPM_ERR_INVALID_ARG, "space %d: each axis must be in [1, 2^20]", c);
        if (space_voxels(sp) > ((int64_t)1 << 30) - 1)
            return fail(MPM_ERR_INVALID_ARG, "space %d has more than 2^30-1 voxels", c);
        for (int k = 0; k < 12; k++)
            if (!std::isfinite(sp.affine[k])) return fail(MPM_ERR_INVALID_ARG, "space %d: affine is not finite", c);
        const double *a = sp.affine;
        for (int col = 0; col < 3; col++) {
            const double len = std::sqrt(a[col] * a[col] + a[4 + col] * a[4 + col] + a[8 + col] * a[8 + col]);
            if (!(len >= 0.125 && len <= 8.0))
                return fail(MPM_ERR_INVALID_ARG, "space %d: axis %d of the affine has length %g (must be in [1/8, 8])",
                            c, col, len);
        }
        const double det = a[0] * (a[5] * a[10] - a[6] * a[9]) - a[1] * (a[4] * a[10] - a[6] * a[8]) +
                           a[2] * (a[4] * a[9] - a[5] * a[8]);
        if (!(std::fabs(det) > 1e-6)) return fail(MPM_ERR_INVALID_ARG, "space %d: affine is singular", c);
    }
    return MPM_OK;
}

DevProto sub_proto(const DevProto &P, int c)
{
    DevProto q;
    memset(&q, 0, sizeof(q));
    const int i0 = P.first[c], ne = P.first[c + 1] - i0;
    q.C = 1;
    q.I = ne;
    q.first[0] = 0;
    q.first[1] = ne;
    q.tr[0] = P.tr[c];
    q.flip[0] = P.flip[c];
    q.mt[0] = P.mt[c];
    for (int e = 0; e < ne; e++) {
        q.te[e] = P.te[i0 + e];
        q.wgt[e] = P.wgt[i0 + e];
        q.off[e] = P.off[i0 + e];
    }
    return q;
}

bool has_mt(const mpm_protocol *p)
{
    for (int c = 0; c < p->n_contrasts; c++)
        if (p->mt[c]) return true;
    return false;
}

mpm_status check_echo_offset(const mpm_protocol *p, int dtype, const float *echo_offset)
{
    if (!echo_offset) return MPM_OK;
    if (dtype == MPM_F32) return fail(MPM_ERR_INVALID_ARG, "echo_offset applies to MPM_F16 / MPM_BF16 echoes only");
    const int I = n_images(p);
    for (int i = 0; i < I; i++)
        if (!std::isfinite(echo_offset[i])) return fail(MPM_ERR_INVALID_ARG, "echo_offset[%d] is not finite", i);
    return MPM_OK;
}

DevProto to_dev(const mpm_protocol *p, const float *echo_offset)
{
    DevProto d;
    memset(&d, 0, sizeof(d));
    d.C = p->n_contrasts;
    int i = 0;
    for (int c = 0; c < p->n_contrasts; c++) {
        d.first[c] = i;
        d.tr[c] = (float)p->tr_s[c];
        d.flip[c] = (float)p->flip_rad[c];
        d.mt[c] = p->mt[c];
        i += p->n_echoes[c];
    }
    d.first[p->n_contrasts] = i;
    d.I = i;
    for (int k = 0; k < i; k++) {
        d.te[k] = (float)p->te_s[k];
        d.wgt[k] = (float)(1.0 / (p->sigma[k] * p->sigma[k]));
        d.off[k] = echo_offset ? echo_offset[k] : 0.0f;
    }
    return d;
}

size_t dtype_size(int dtype) { return dtype == MPM_F32 ? 4 : 2; }

// ---------------------------------------------------------------------------
// default initialisation from per-image volume means: a log-linear fit with
// one shared R2* gives the TE = 0 intercept of each contrast; small-angle
// closed forms (Helms et al. 2008, the approximation the paper's MT model
// comes from) give A and R1 from the two non-MT contrasts with the smallest
// and largest flip angle and MTsat from the first MT contrast.
// ---------------------------------------------------------------------------
static double clampd(double v, double lo, double hi) { return v >= lo ? (v <= hi ? v : hi) : lo; }

mpm_status default_init_from_means(const mpm_protocol *p, const double *mean, double b1_mean, float y0[4])
{
    const int C = p->n_contrasts, U = C + 1;
    // normal equations of  log m_i = beta_c(i) - r2 * TE_i
    double A[MPM_MAX_CONTRASTS + 1][MPM_MAX_CONTRASTS + 2] = {};
    int i = 0;
    for (int c = 0; c < C; c++)
        for (int e = 0; e < p->n_echoes[c]; e++, i++) {
            if (!std::isfinite(mean[i])) continue;  // image without any finite value
            double lm = std::log(std::max(mean[i], 1e-12));
            double te = p->te_s[i];
            A[c][c] += 1.0;
            A[c][C] -= te;
            A[C][c] -= te;
            A[C][C] += te * te;
            A[c][U] += lm;
            A[C][U] -= te * lm;
        }
    for (int col = 0; col < U; col++) {
        int piv = col;
        for (int r = col + 1; r < U; r++)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        if (std::fabs(A[piv][col]) < 1e-300)
            return fail(MPM_ERR_UNSUPPORTED, "default init: echo times do not determine R2*");
        for (int k = 0; k <= U; k++) std::swap(A[col][k], A[piv][k]);
        for (int r = 0; r < U; r++) {
            if (r == col) continue;
            double f = A[r][col] / A[col][col];
            for (int k = col; k <= U; k++) A[r][k] -= f * A[col][k];
        }
    }
    double beta[MPM_MAX_CONTRASTS + 1];
    for (int u = 0; u < U; u++) beta[u] = A[u][U] / A[u][u];
    int cP = -1, cT = -1, cM = -1;
    for (int c = 0; c < C; c++) {
        if (p->mt[c]) {
            if (cM < 0) cM = c;
        } else {
            if (cP < 0 || p->flip_rad[c] < p->flip_rad[cP]) cP = c;
            if (cT < 0 || p->flip_rad[c] > p->flip_rad[cT]) cT = c;
        }
    }
    if (cM < 0 || cP < 0 || cT < 0 || p->flip_rad[cP] == p->flip_rad[cT])
        return fail(MPM_ERR_UNSUPPORTED,
                    "default init needs an MT contrast and two non-MT contrasts with distinct flip angles");
    double SP = std::exp(beta[cP]), ST = std::exp(beta[cT]), SM = std::exp(beta[cM]);
    double aP = p->flip_rad[cP] * b1_mean, aT = p->flip_rad[cT] * b1_mean, aM = p->flip_rad[cM] * b1_mean;
    double tP = p->tr_s[cP], tT = p->tr_s[cT], tM = p->tr_s[cM];
    double R1 = 0.5 * (ST * aT / tT - SP * aP / tP) / (SP / aP - ST / aT);
    double Aa = SP * ST * (tP * aT / aP - tT * aP / aT) / (ST * tP * aT - SP * tT * aP);
    R1 = clampd(R1, 0.05, 20.0);
    if (!(Aa > 0.0) || !std::isfinite(Aa)) Aa = SP / std::sin(aP);
    double dl = clampd((Aa * aM / SM - 1.0) * R1 * tM - 0.5 * aM * aM, 1e-4, 0.2);
    double r2 = clampd(beta[C], 0.5, 500.0);
    y0[0] = (float)std::log(Aa);
    y0[1] = (float)std::log(R1);
    y0[2] = (float)std::log(r2);
    y0[3] = (float)std::log(dl / (1.0 - dl));
    return MPM_OK;
}

mpm_status check_fit_args(const mpm_protocol *protocol, const mpm_grid *grid, int dtype, const void *echoes,
                          const mpm_options *opt, const float *maps, int64_t *N)
{
    mpm_status st;
    if ((st = check_protocol(protocol)) || (st = check_grid(grid, N)) || (st = check_dtype(dtype))) return st;
    if (!opt) return fail(MPM_ERR_INVALID_ARG, "options is NULL");
    if (!echoes || !maps) return fail(MPM_ERR_INVALID_ARG, "echoes and maps must be device pointers");
    if (opt->mode != MPM_ML && opt->mode != MPM_MAP_JTV) return fail(MPM_ERR_INVALID_ARG, "unknown mode %d", opt->mode);
    if (opt->n_gn < 0 || opt->n_outer < 0 || opt->n_cg < 0 || opt->n_gn > 100000 || opt->n_outer > 100000 ||
        opt->n_cg > 100000)
        return fail(MPM_ERR_INVALID_ARG, "iteration counts must be in [0, 100000]");
    if (opt->max_halvings > 7) return fail(MPM_ERR_INVALID_ARG, "max_halvings must be <= 7");
    if (opt->loading != MPM_LOAD_PROPOSED && opt->loading != MPM_LOAD_GN && opt->loading != MPM_LOAD_PROPOSED_PLUS)
        return fail(MPM_ERR_INVALID_ARG, "unknown loading %d", opt->loading);
    if (opt->init_kind < MPM_INIT_DEFAULT || opt->init_kind > MPM_INIT_FROM_MAPS)
        return fail(MPM_ERR_INVALID_ARG, "unknown init_kind %d", opt->init_kind);
    if (opt->flags != 0) return fail(MPM_ERR_INVALID_ARG, "flags must be 0");
    if (opt->basis != MPM_BASIS_LOG)
        return opt->basis == MPM_BASIS_RATE || opt->basis == MPM_BASIS_TIME
                   ? fail(MPM_ERR_UNSUPPORTED, "only mpm_fit_voxelwise takes a basis other than MPM_BASIS_LOG")
                   : fail(MPM_ERR_INVALID_ARG, "unknown basis %d", opt->basis);
    for (int k = 0; k < 4; k++) {
        if (!(opt->lambda[k] >= 0.0) || !std::isfinite(opt->lambda[k]))
            return fail(MPM_ERR_INVALID_ARG, "lambda[%d] must be finite and >= 0", k);
        if (opt->init_kind == MPM_INIT_CONST && !std::isfinite(opt->init_const[k]))
            return fail(MPM_ERR_INVALID_ARG, "init_const[%d] is not finite", k);
    }
    if (!(opt->jtv_eps >= 0.0) || !(opt->cg_stop >= 0.0)) return fail(MPM_ERR_INVALID_ARG, "jtv_eps and cg_stop must be >= 0");
    if (!(opt->tol_gn >= 0.0) || !std::isfinite(opt->tol_gn) || !(opt->tol_outer >= 0.0) || !std::isfinite(opt->tol_outer))
        return fail(MPM_ERR_INVALID_ARG, "tol_gn and tol_outer must be finite and >= 0");
    if (!has_mt(protocol))
        return fail(MPM_ERR_UNSUPPORTED, "the four-parameter model needs at least one MT contrast");
    if (opt->mode == MPM_MAP_JTV && *N < 2) return fail(MPM_ERR_UNSUPPORTED, "MAP needs at least 2 voxels");
    if (opt->mode == MPM_ML && opt->start_outer != 0)
        return fail(MPM_ERR_INVALID_ARG, "start_outer is a MAP option (0 for ML)");
    if (opt->mode == MPM_MAP_JTV &&
        (opt->start_outer < 0 || (opt->n_outer > 0 ? opt->start_outer >= opt->n_outer : opt->start_outer != 0)))
        return fail(MPM_ERR_INVALID_ARG, "start_outer must be in [0, n_outer) (0 when n_outer = 0)");
    if ((st = check_echo_offset(protocol, dtype, opt->echo_offset))) return st;
    if (opt->start_outer > 0 && opt->tol_outer > 0.0)
        return fail(MPM_ERR_UNSUPPORTED, "tol_outer measures gains from the end of outer loop 0: "
                                         "it cannot be used with start_outer > 0");
    return MPM_OK;
}

// device buffer helper (stream-ordered)
hipError_t Workspace::alloc(void **p, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (arena) {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off > cap || bytes > cap - off) {
            need = off + bytes;
            return hipErrorOutOfMemory;
        }
        *p = arena + off;
        used = off + bytes;
        return hipSuccess;
    }
    hipError_t e = hipMallocAsync(p, bytes, stream);
    if (e == hipSuccess) bufs.push_back(*p);
    return e;
}

Workspace::~Workspace()
{
    for (void *p : bufs) hipFreeAsync(p, stream);
    hipStreamSynchronize(stream);
}

mpm_status run_fit(const FitArgs &a, Workspace &ws, mpm_report *report, double *trace, int trace_len)
{
    mpm_status st;
    mpm_report rep;
    memset(&rep, 0, sizeof(rep));
    Prof prof(a.stream);
    std::unique_ptr<FitJob> job =
        a.opt->mode == MPM_ML ? make_ml_job(a, ws, prof, &st) : make_map_job(a, ws, prof, &st);
    if (st) return st;
    bool more = true;
    while (more)
        if ((st = job->enqueue_next(&more))) {
            // the work already enqueued ends before the job and its staging go
            (void)hipStreamSynchronize(a.stream);
            return st;
        }
    hipError_t e = hipStreamSynchronize(a.stream);
    prof.collect();
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "fit: %s", hipGetErrorString(e));
    if ((st = job->collect(rep, trace, trace_len))) return st;
    if (report) *report = rep;
    return MPM_OK;
}

int image_sum_rows(const DevProto &P) { return 2 * P.I + 1; }

mpm_status enqueue_image_sums(Workspace &ws, Prof &prof, const DevProto &P, int dtype, const void *X,
                              const float *b1, int64_t N, double **sums)
{
    LaunchCtx c{ws.stream};
    int nblk = echo_sums_blocks(N);
    const int rows = image_sum_rows(P);
    double *part = nullptr;
    if (ws.alloc((void **)&part, sizeof(double) * (size_t)nblk * rows) != hipSuccess ||
        ws.alloc((void **)sums, sizeof(double) * rows) != hipSuccess)
        return fail(MPM_ERR_OUT_OF_MEMORY, "workspace allocation failed");
    hipError_t e = prof.launch("echo_sums", (double)N * ((double)P.I * dtype_size(dtype) + (b1 ? 4 : 0)),
                               [&] { return launch_echo_sums(c, P, dtype, X, b1, N, part, nblk); });
    if (e == hipSuccess) e = launch_reduce_rows(c, part, rows, nblk, *sums);
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "image sums: %s", hipGetErrorString(e));
    return MPM_OK;
}

void image_means_from_sums(const DevProto &P, int64_t N, const double *sums, std::vector<double> &mean,
                           double &b1m)
{
    mean.resize(P.I);
    for (int i = 0; i < P.I; i++) mean[i] = sums[P.I + i] > 0.0 ? P.off[i] + sums[i] / sums[P.I + i] : NAN;
    b1m = sums[2 * P.I] / (double)N;
}

mpm_status image_means(Workspace &ws, Prof &prof, const DevProto &P, int dtype, const void *X,
                       const float *b1, int64_t N, std::vector<double> &mean, double &b1m)
{
    double *sums = nullptr;
    mpm_status st = enqueue_image_sums(ws, prof, P, dtype, X, b1, N, &sums);
    if (st) return st;
    std::vector<double> host(image_sum_rows(P));
    hipError_t e = hipMemcpyAsync(host.data(), sums, sizeof(double) * host.size(), hipMemcpyDeviceToHost, ws.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ws.stream);
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "image means: %s", hipGetErrorString(e));
    image_means_from_sums(P, N, host.data(), mean, b1m);
    return MPM_OK;
}

}  // namespace mpm

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *mpm_last_error(void) { return t_last_error.c_str(); }

const char *mpm_version(void) { return "libmpm 0.1 (gfx950)"; }

void mpm_profile_enable(int32_t every)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_every = every > 0 ? every : 0;
}

void mpm_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_stats.clear();
}

int32_t mpm_profile_read(mpm_kernel_stat *out, int32_t max)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int32_t n = (int32_t)g_stats.size();
    for (int32_t i = 0; i < n && i < max; i++) out[i] = g_stats[i];
    return n;
}

mpm_status mpm_simulate(const mpm_protocol *protocol, const mpm_grid *grid, const float *maps, const float *b1,
                        const float *noise, mpm_dtype out_dtype, void *out, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st;
    if ((st = check_protocol(protocol)) || (st = check_grid(grid, &N)) || (st = check_dtype(out_dtype))) return st;
    if (!maps || !out) return fail(MPM_ERR_INVALID_ARG, "maps and out must be device pointers");
    DevProto P = to_dev(protocol);
    hipStream_t s = (hipStream_t)stream;
    Prof prof(s);
    LaunchCtx c{s};
    double bytes = (double)N * (16.0 + (b1 ? 4 : 0) + P.I * (dtype_size(out_dtype) + (noise ? 4.0 : 0.0)));
    hipError_t e = prof.launch("simulate", bytes,
                               [&] { return launch_simulate(c, P, maps, b1, noise, out_dtype, out, N); });
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    prof.collect();
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "simulate: %s", hipGetErrorString(e));
    return MPM_OK;
}

mpm_status mpm_pack_echoes(int32_t n_images, int64_t n_voxels, const float *src, mpm_dtype dtype, void *dst,
                           float *offsets, void *stream)
{
    clear_error();
    if (n_images < 1 || n_images > MPM_MAX_IMAGES)
        return fail(MPM_ERR_INVALID_ARG, "n_images=%d outside [1, %d]", n_images, MPM_MAX_IMAGES);
    if (n_voxels < 1 || n_voxels > ((int64_t)1 << 30) - 1)
        return fail(MPM_ERR_INVALID_ARG, "n_voxels=%lld outside [1, 2^30)", (long long)n_voxels);
    if (dtype != MPM_F16 && dtype != MPM_BF16) return fail(MPM_ERR_INVALID_ARG, "dtype must be MPM_F16 or MPM_BF16");
    if (!src || !dst || !offsets) return fail(MPM_ERR_INVALID_ARG, "src, dst and offsets must be non-NULL");
    const int64_t N = n_voxels;
    const char *s0 = (const char *)src, *s1 = s0 + (size_t)n_images * N * 4;
    const char *d0 = (const char *)dst, *d1 = d0 + (size_t)n_images * N * 2;
    if (d0 < s1 && s0 < d1) return fail(MPM_ERR_INVALID_ARG, "dst overlaps src");
    hipStream_t s = (hipStream_t)stream;
    DevProto P;
    memset(&P, 0, sizeof(P));
    P.I = n_images;
    unsigned int bad = 0;
    {
        Workspace ws(s);
        Prof prof(s);
        std::vector<double> mean;
        double unused;
        mpm_status st = image_means(ws, prof, P, MPM_F32, src, nullptr, N, mean, unused);
        if (st) return st;
        EchoOffsets off;
        memset(&off, 0, sizeof(off));
        for (int i = 0; i < n_images; i++) off.v[i] = std::isfinite(mean[i]) ? (float)mean[i] : 0.0f;
        unsigned int *cnt = nullptr;
        if (ws.alloc((void **)&cnt, sizeof(unsigned int)) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "pack: workspace allocation failed");
        LaunchCtx c{s};
        hipError_t e = hipMemsetAsync(cnt, 0, sizeof(unsigned int), s);
        if (e == hipSuccess)
            e = prof.launch("pack_echoes", (double)n_images * N * 6.0,
                            [&] { return launch_pack_echoes(c, n_images, N, src, dtype, dst, off, cnt); });
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, cnt, sizeof(bad), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        prof.collect();
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "pack: %s", hipGetErrorString(e));
        for (int i = 0; i < n_images; i++) offsets[i] = off.v[i];
    }
    if (bad) return fail(MPM_ERR_INVALID_ARG, "pack: %u finite values overflow the storage type", bad);
    return MPM_OK;
}

size_t mpm_footprint_bytes(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype, int32_t mode)
{
    int64_t N;
    if (check_protocol(protocol) || check_grid(grid, &N) || check_dtype(dtype)) return 0;
    size_t I = (size_t)n_images(protocol);
    size_t inputs = (size_t)N * (I * dtype_size(dtype) + 4 /* b1 */ + 16 /* maps */);
    size_t ws = (size_t)N * (mode == MPM_ML ? 0 : map_workspace_floats_per_voxel() * 4) + ((size_t)1 << 20);
    return inputs + ws;
}

mpm_status mpm_simulate_projected(const mpm_protocol *protocol, const mpm_grid *grid, const mpm_space *spaces,
                                  const float *maps, const float *b1, const float *noise, mpm_dtype out_dtype,
                                  void *out, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st;
    if ((st = check_protocol(protocol)) || (st = check_grid(grid, &N)) || (st = check_dtype(out_dtype)) ||
        (st = check_spaces(protocol, spaces)))
        return st;
    if (!maps || !out) return fail(MPM_ERR_INVALID_ARG, "maps and out must be device pointers");
    const DevProto P = to_dev(protocol);
    const Grid3 g = make_grid3(grid->nx, grid->ny, grid->nz);
    hipStream_t s = (hipStream_t)stream;
    Prof prof(s);
    LaunchCtx lc{s};
    hipError_t e = hipSuccess;
    {
        Workspace ws(s);
        int64_t off = 0;  // elements before the contrast's first image
        for (int c = 0; c < protocol->n_contrasts && e == hipSuccess; c++) {
            const ProjSpace S = make_proj_space(spaces[c]);
            const DevProto Pc = sub_proto(P, c);
            float *Yp = nullptr;
            if (ws.alloc((void **)&Yp, sizeof(float) * 5 * (size_t)S.M) != hipSuccess)
                return fail(MPM_ERR_OUT_OF_MEMORY, "simulate: workspace allocation failed");
            e = prof.launch("proj_pull", (double)S.M * 20.0,
                            [&] { return launch_proj_pull(s, g, S, maps, b1, Yp, Yp + 4 * S.M); });
            char *dst = (char *)out + off * (int64_t)dtype_size(out_dtype);
            const float *nz = noise ? noise + off : nullptr;
            if (e == hipSuccess)
                e = prof.launch("simulate", (double)S.M * (20.0 + Pc.I * (dtype_size(out_dtype) + (noise ? 4.0 : 0.0))),
                                [&] { return launch_simulate(lc, Pc, Yp, Yp + 4 * S.M, nz, out_dtype, dst, S.M); });
            off += (int64_t)Pc.I * S.M;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    prof.collect();
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "simulate: %s", hipGetErrorString(e));
    return MPM_OK;
}

mpm_status mpm_fit(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype, const void *echoes,
                   const float *b1, const mpm_options *opt, float *maps, mpm_report *report, double *trace,
                   int32_t trace_len, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st = check_fit_args(protocol, grid, dtype, echoes, opt, maps, &N);
    if (st) return st;
    if (trace_len < 0 || (trace_len > 0 && !trace)) return fail(MPM_ERR_INVALID_ARG, "trace is NULL");
    for (int i = 0; i < trace_len; i++) trace[i] = NAN;

    hipStream_t s = (hipStream_t)stream;
    FitArgs a{protocol, to_dev(protocol, opt->echo_offset), dtype, echoes, b1, opt, maps, N,
              grid->nx, grid->ny, grid->nz, s};
    Workspace ws(s);
    return run_fit(a, ws, report, trace, trace_len);
}

}  // extern "C"

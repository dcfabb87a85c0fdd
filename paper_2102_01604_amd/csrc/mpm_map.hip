// mpm_map.hip -- host driver of the JTV-regularised (MAP) fit and of the
// Laplace uncertainty (paper Sec. 2.5-2.7, Sec. 3.6).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "mpm_api_internal.h"
#include "mpm_proj.h"
#include "mpm_tune.h"

namespace mpm {

int stencil_workgroups()
{
    static int v = [] {
        const char *e = std::getenv("MPM_STENCIL_WORKGROUPS");
        int x = e ? std::atoi(e) : 0;
        return (x >= 64 && x <= (1 << 20)) ? x : TARGET_WORKGROUPS;
    }();
    return v;
}

int tall_workgroups()
{
    static int v = [] {
        const char *e = std::getenv("MPM_TALL_WORKGROUPS");
        int x = e ? std::atoi(e) : 0;
        return (x >= 16 && x <= (1 << 20)) ? x : TALL_WORKGROUPS;
    }();
    return v;
}

// Hessian d, o (4 each), R, Z, P0, P1, D (4 each), Hessian r (2), w (1)
size_t map_workspace_floats_per_voxel() { return 31; }


static mpm_status alloc_map(const FitArgs &a, Workspace &ws, MapArgs &m, int trace_len)
{
    const int64_t N = a.N;
    m.g = make_grid3(a.nx, a.ny, a.nz, TILE_Y, column_target(a.nx, a.ny, a.nz));
    m.P = a.P;
    m.dtype = a.dtype;
    m.X = a.X;
    m.b1 = a.b1;
    m.bm = a.opt->b1_receive;
    m.Y = a.maps;
    m.gp = plane_grid(m.g);
    m.gt = make_grid3(a.nx, a.ny, a.nz, TALL_Y, tall_target(a.nx, a.ny, a.nz));
    m.gv = plane_grid(make_grid3(a.nx, a.ny, a.nz, cg_b_rows()));
    const int nblk = std::max(std::max(grid_blocks(m.g), grid_blocks(m.gp)), std::max(grid_blocks(m.gt), grid_blocks(m.gv)));
    float *big = nullptr;
    const size_t nf = map_workspace_floats_per_voxel() * (size_t)N;
    if (ws.alloc((void **)&big, nf * sizeof(float)) != hipSuccess ||
        ws.alloc((void **)&m.partials, sizeof(double) * (size_t)(MAX_TRIALS + 2) * nblk) != hipSuccess ||
        ws.alloc((void **)&m.ctl, sizeof(MapCtl)) != hipSuccess ||
        ws.alloc((void **)&m.trace, sizeof(double) * (size_t)(trace_len > 0 ? trace_len : 1)) != hipSuccess)
        return fail(MPM_ERR_OUT_OF_MEMORY, "MAP workspace allocation failed (%zu bytes)", nf * sizeof(float));
    m.pstride = nblk;
    m.nb_a = grid_blocks(m.gt);
    m.nb_b = grid_blocks(m.gv);
    m.fold = m.nb_a <= FOLD_MAX_PARTIALS && m.nb_b <= FOLD_MAX_PARTIALS;
    m.cg_stop_rel = a.opt->cg_stop;
    float4 *v4 = (float4 *)big;  // 16-byte aligned (hipMallocAsync)
    m.H.d = v4;
    m.H.o = v4 + N;
    m.R = v4 + 2 * N;
    m.Z = v4 + 3 * N;
    m.P0 = v4 + 4 * N;
    m.P1 = v4 + 5 * N;
    m.D = v4 + 6 * N;
    m.H.r = (float2 *)(v4 + 7 * N);
    m.w = (float *)(m.H.r + N);
    return MPM_OK;
}

static void set_prior(const mpm_options *o, MapArgs &m, bool use_lambda, int &prior_on)
{
    double ls = 0.0;
    for (int k = 0; k < 4; k++) {
        m.lam[k] = use_lambda ? (float)o->lambda[k] : 0.0f;
        ls += use_lambda ? o->lambda[k] : 0.0;
    }
    m.eps = (float)(o->jtv_eps > 0.0 ? o->jtv_eps : 1e-3 * std::sqrt(ls));
    prior_on = ls > 0.0 ? 1 : 0;
    m.loading = o->loading;
}

// ---------------------------------------------------------------------------
// Spatial projection (paper Sec. 2.4): per contrast its space, protocol, first
// image and acquisition-space blocks; the pushed gradient and Hessian on the
// reconstruction grid; extra partial rows carrying the acquisition-space NLL.
// ---------------------------------------------------------------------------
struct ProjState {
    int C = 0;
    ProjContrast pc[MAXC];
    ProjPushArgs push;
    float4 *G = nullptr;
    double *ext = nullptr;
    int ext_stride = 0;
    PushedProto pp;
    PsiT psi{nullptr, nullptr};  // stored Psi^T (fits: pushed every Newton step)
    float4 *Yt = nullptr;        // trial point y - delta_f (fits)
    int64_t *scan_tmp = nullptr;
    ExtRows rows(int n) const
    {
        ExtRows r;
        r.p = ext;
        r.stride = ext_stride;
        r.cols = ext_stride;
        r.rows = n;
        return r;
    }
};

static mpm_status alloc_proj(const FitArgs &a, Workspace &ws, ProjState &ps, HessArrays Hrecon, bool store_psi)
{
    ps.C = a.P.C;
    memset(&ps.push, 0, sizeof(ps.push));
    ps.push.C = ps.C;
    const char *X = (const char *)a.X;
    int col = 0;
    for (int c = 0; c < ps.C; c++) {
        ProjContrast &pc = ps.pc[c];
        pc.S = make_proj_space(a.spaces[c]);
        pc.P = sub_proto(a.P, c);
        pc.X = X;
        X += (int64_t)pc.P.I * pc.S.M * (int64_t)dtype_size(a.dtype);
        float4 *buf = nullptr;  // g, H d, H o (float4 each), H r (float2) per acquisition voxel
        if (ws.alloc((void **)&buf, (size_t)pc.S.M * 56) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "projection workspace allocation failed");
        pc.B.G = buf;
        pc.B.H.d = buf + pc.S.M;
        pc.B.H.o = buf + 2 * pc.S.M;
        pc.B.H.r = (float2 *)(buf + 3 * pc.S.M);
        pc.ext_col = col;
        col += proj_blocks(pc.S);
        ps.push.S[c] = pc.S;
        ps.push.B[c] = pc.B;
    }
    ps.ext_stride = col;
    if (ws.alloc((void **)&ps.ext, sizeof(double) * MAX_TRIALS * (size_t)col) != hipSuccess ||
        ws.alloc((void **)&ps.G, sizeof(float4) * (size_t)a.N) != hipSuccess)
        return fail(MPM_ERR_OUT_OF_MEMORY, "projection workspace allocation failed");
    ps.pp.G = ps.G;
    ps.pp.H = Hrecon;
    if (store_psi) {
        int64_t cap = 0;  // each acquisition voxel has at most 8 nonzero weights
        for (int c = 0; c < ps.C; c++) cap += 8 * ps.pc[c].S.M;
        const int64_t rows = (int64_t)ps.C * a.N;
        if (ws.alloc((void **)&ps.psi.row, sizeof(int64_t) * (size_t)(rows + 1)) != hipSuccess ||
            ws.alloc((void **)&ps.psi.ent, sizeof(int2) * (size_t)cap) != hipSuccess ||
            ws.alloc((void **)&ps.scan_tmp, sizeof(int64_t) * (size_t)psi_scan_blocks(rows)) != hipSuccess ||
            ws.alloc((void **)&ps.Yt, sizeof(float4) * (size_t)a.N) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "projection workspace allocation failed");
    }
    return MPM_OK;
}

// ---------------------------------------------------------------------------
// MAP fit as a job: piece 0 initialises (maps, control block, w = 0); then
// one piece per Newton-like step (preceded by the weight refresh at the start
// of each outer loop t >= 1, loops running from start_outer); the last piece
// refreshes the weights from the final maps, computes the final statistics
// and copies the control block and the objective trace to pinned host memory.
// ---------------------------------------------------------------------------
struct MapJob : FitJob {
    FitArgs a;
    Workspace &ws;
    Prof &prof;
    MapArgs m;
    int prior_on = 0, ntrial = 1, accept_off = 0;
    int T = 0, J = 0, K = 0, S = 0, tl = 0, t0 = 0;  // t0: first outer loop run (resume)
    int nb_col = 0, nb_pl = 0, nb_cga = 0, nb_cgb = 0;
    int t = 0, j = 0;  // next Newton-like step
    bool started = false, finished = false;
    PinnedBuf host;    // MapCtl followed by the trace
    InitStage init;
    bool proj = false;      // spatial projection
    bool ml_as_map = false; // projected ML: one outer loop, no prior, one CG iteration, every step taken
    mpm_options opt_local;
    ProjState ps;

    MapJob(const FitArgs &a_, Workspace &ws_, Prof &prof_) : a(a_), ws(ws_), prof(prof_) { memset(&m, 0, sizeof(m)); }

    bool ready() const override { return init.ready(); }

    mpm_status setup()
    {
        proj = a.spaces != nullptr;
        if (proj && a.opt->mode == MPM_ML) {
            // y - P~^{-1} g: with no prior the preconditioner is the system
            // matrix, so one CG iteration solves it exactly
            ml_as_map = true;
            opt_local = *a.opt;
            opt_local.mode = MPM_MAP_JTV;
            opt_local.n_outer = 1;
            opt_local.n_cg = 1;
            opt_local.max_halvings = -1;
            opt_local.tol_gn = opt_local.tol_outer = 0.0;  // tolerances are MAP options
            for (int k = 0; k < 4; k++) opt_local.lambda[k] = 0.0;
            a.opt = &opt_local;
        }
        const mpm_options *o = a.opt;
        T = o->n_outer;
        J = o->n_gn;
        K = o->n_cg;
        S = J + 2;
        tl = T * S;
        t = t0 = o->start_outer;
        mpm_status st = alloc_map(a, ws, m, tl);
        if (st) return st;
        if (!a.no_pinned && host.alloc(sizeof(MapCtl) + sizeof(double) * (size_t)(tl > 0 ? tl : 1)) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
        set_prior(o, m, true, prior_on);
        m.tol_gn = o->tol_gn;
        m.tol_outer = o->tol_outer;
        ntrial = o->max_halvings < 0 ? 1 : o->max_halvings + 1;
        accept_off = o->max_halvings < 0;
        nb_col = grid_blocks(m.g);
        nb_pl = grid_blocks(m.gp);
        nb_cga = cg_a_blocks(m);
        nb_cgb = cg_b_blocks(m);
        if (proj) return alloc_proj(a, ws, ps, m.H, true);
        return MPM_OK;
    }

    hipError_t fin(int stage, int arg, int nblk, const ExtRows &ext = ExtRows(), int row = 0)
    {
        return launch_fin(a.stream, m, stage, arg, nblk, a.opt->cg_stop, ntrial, accept_off, ext, row);
    }

    // acquisition-space likelihood of every contrast, then the push
    hipError_t proj_lik_push(int gated)
    {
        const hipStream_t s = a.stream;
        hipError_t e = hipSuccess;
        for (int c = 0; c < ps.C && e == hipSuccess; c++) {
            const ProjContrast &pc = ps.pc[c];
            e = prof.launch("proj_lik", (double)pc.S.M * (pc.P.I * dtype_size(a.dtype) + 16 + 4 + 56),
                            [&] { return launch_proj_lik(s, m, pc, ps.ext, gated); });
        }
        // algorithmic bytes: the blocks of every acquisition voxel once, the
        // stored Psi^T (row pointers, 8 B per entry at 8 entries per
        // acquisition voxel) and the pushed blocks
        double pushed = 0.0;
        for (int c = 0; c < ps.C; c++) pushed += (double)ps.pc[c].S.M * (56 + 64) + (double)a.N * 8;
        if (e == hipSuccess)
            e = prof.launch("proj_push", pushed + (double)a.N * 56,
                            [&] { return launch_proj_push_csr(s, m, ps.push, ps.psi, ps.G, ps.pp.H); });
        return e;
    }

    // likelihood blocks at the trial point y - delta_f: NLL for the acceptance
    // test, and the next step's blocks when the full step is taken
    hipError_t proj_lik_trial()
    {
        hipError_t e = prof.launch("trial_point", (double)a.N * (16 + 32 + 16),
                                   [&] { return launch_trial_point(a.stream, m, ps.Yt); });
        for (int c = 0; c < ps.C && e == hipSuccess; c++) {
            const ProjContrast &pc = ps.pc[c];
            e = prof.launch("proj_lik_trial", (double)pc.S.M * (pc.P.I * dtype_size(a.dtype) + 16 + 4 + 56),
                            [&] { return launch_proj_lik(a.stream, m, pc, ps.ext, 0, ps.Yt); });
        }
        return e;
    }

    hipError_t proj_nll(int h0, int h1)
    {
        hipError_t e = hipSuccess;
        for (int c = 0; c < ps.C && e == hipSuccess; c++) {
            const ProjContrast &pc = ps.pc[c];
            e = prof.launch("proj_nll", (double)pc.S.M * (pc.P.I * dtype_size(a.dtype) + 16 + 4 + 32),
                            [&] { return launch_proj_nll(a.stream, m, pc, ps.ext, ps.ext_stride, h0, h1); });
        }
        return e;
    }

    mpm_status enqueue_next(bool *more) override
    {
        const hipStream_t s = a.stream;
        const double N = (double)a.N, xb = (double)a.P.I * dtype_size(a.dtype);
        const double bb = (a.b1 ? 4.0 : 0.0) + (m.bm ? 4.0 : 0.0);
        hipError_t e = hipSuccess;
#define RUN(name, bytes, call)                                                    \
    do {                                                                          \
        if (e == hipSuccess) e = prof.launch(name, bytes, [&] { return call; }); \
    } while (0)
        *more = true;
        if (started && init.pending) {
            mpm_status st = init.finish(a);
            if (st) return st;
        }
        if (!started) {
            started = true;
            mpm_status st = init.start(a, ws, prof);
            if (st) return st;
            e = launch_ctl_init(s, m.ctl, m.trace, tl);
            LaunchCtx c{s};
            if (e == hipSuccess) e = launch_fill(c, m.w, a.N, 0.0f);
            if (proj) RUN("psi_build", 0.0, launch_psi_build(s, m.g, ps.push, ps.psi, ps.scan_tmp));
        } else if (t < T && J > 0) {
            if (j == 0 && t >= 1) {
                RUN("jtv_weights", N * 20.0, launch_weights(s, m, prior_on));
                // the end of the previous loop, if this call ran it (a resumed
                // fit re-weights from its initial maps without ending a loop)
                if (t > t0) RUN("fin", 0.0, fin(FIN_W, (t - 1) * S + J + 1, nb_col));
            }
            if (!proj) {
                // after a step whose accept pass evaluated this pass (j >= 1),
                // k_lik only checks that the full step was taken
                if (j == 0) RUN("map_lik", N * (xb + bb + 16 + 4 + 40 + 16 + 16), launch_lik(s, m));
                else RUN("map_lik_check", 0.0, launch_lik(s, m));
                RUN("fin", 0.0, fin(FIN_LIK, j == 0 ? t * S : -1, nb_pl));
            } else {
                if (e == hipSuccess) e = proj_lik_push(1);
                RUN("map_lik", N * (16 + 40 + 16 + 4 + 40 + 16 + 16), launch_lik_pushed(s, m, ps.pp));
                RUN("fin", 0.0, fin(FIN_LIK, j == 0 ? t * S : -1, nb_pl, ps.rows(1)));
            }
            for (int i = 0; i < K && e == hipSuccess; i++) {
                double ab = 16 + (i > 0 ? 16 : 0) + 40 + 4 + 16 + (i == 1 ? 16 : i >= 2 ? 32 : 0);
                RUN("cg_a", N * ab, launch_cg_a(s, m, i));
                if (!m.fold) RUN("fin", 0.0, fin(FIN_A, i, nb_cga));
                RUN("cg_b", N * (16 + 4 + 40 + 32 + 16), launch_cg_b(s, m, i));
                // folded: each sweep finalises the one before it; the last sweep B
                // is finalised by a launch of its own (its partials are in row 1)
                if (!m.fold) RUN("fin", 0.0, fin(FIN_B, i, nb_cgb));
                else if (i == K - 1) RUN("fin", 0.0, fin(FIN_B, i, nb_cgb, ExtRows(), 1));
            }
            if (!proj) {
                if (j + 1 < J) {
                    // the next step of this outer loop: its likelihood pass is
                    // evaluated here, at the full step
                    RUN("map_accept_lik", N * (xb + bb + 16 + 16 + 16 + 4 + 40 + 16 + 16), launch_accept_spec(s, m));
                    RUN("fin", 0.0, fin(FIN_ACCEPT_SPEC, t * S + j + 1, nb_pl));
                } else {
                    RUN("map_accept", N * (xb + bb + 16 + 16 + 16 + 4), launch_accept(s, m));
                    RUN("fin", 0.0, fin(FIN_ACCEPT, t * S + j + 1, nb_pl));
                }
                if (ntrial > 1) {
                    // runs only when the full step was rejected (device flag)
                    RUN("map_accept2", 0.0, launch_accept2(s, m, ntrial));
                    RUN("fin", 0.0, fin(FIN_ACCEPT2, t * S + j + 1, nb_col));
                }
            } else {
                if (e == hipSuccess) e = proj_lik_trial();
                RUN("map_accept", N * (16 + 16 + 16 + 4), launch_accept_pushed(s, m, ps.pp));
                RUN("fin", 0.0, fin(FIN_ACCEPT, t * S + j + 1, nb_pl, ps.rows(1)));
                if (ntrial > 1) {
                    if (e == hipSuccess) e = proj_nll(1, ntrial);
                    RUN("fin", 0.0, fin(FIN_ACCEPT2, t * S + j + 1, 0, ps.rows(ntrial)));
                }
            }
            RUN("map_update", N * 64.0, launch_update(s, m));
            if (m.tol_gn > 0.0) RUN("fin", 0.0, fin(FIN_STOP, -1, 0));
            if (++j == J) {
                j = 0;
                t++;
            }
        } else {
            // outer loops without Newton steps only refresh the weights
            for (int tt = (J > 0 ? T : t0 + 1); tt < T && e == hipSuccess; tt++) {
                RUN("jtv_weights", N * 20.0, launch_weights(s, m, prior_on));
                RUN("fin", 0.0, fin(FIN_W, (tt - 1) * S + J + 1, nb_col));
            }
            // final weights (objective and report), then statistics at the final maps
            RUN("jtv_weights", N * 20.0, launch_weights(s, m, prior_on));
            RUN("fin", 0.0, fin(FIN_W, T >= 1 ? (T - 1) * S + J + 1 : -1, nb_col));
            if (!proj) {
                RUN("map_final", N * (xb + bb + 16 + 4), launch_final(s, m, nullptr, nullptr));
                RUN("fin", 0.0, fin(FIN_STATS, 0, nb_pl));
            } else {
                if (e == hipSuccess) e = proj_lik_push(0);
                RUN("map_final", N * (16 + 40 + 16 + 4), launch_final_pushed(s, m, ps.pp, nullptr, nullptr));
                RUN("fin", 0.0, fin(FIN_STATS, 0, nb_pl, ps.rows(1)));
            }
            if (e == hipSuccess && !a.no_pinned)
                e = hipMemcpyAsync(host.p, m.ctl, sizeof(MapCtl), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && tl > 0 && !a.no_pinned)
                e = hipMemcpyAsync((char *)host.p + sizeof(MapCtl), m.trace, sizeof(double) * tl,
                                   hipMemcpyDeviceToHost, s);
            finished = true;
            *more = false;
        }
#undef RUN
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "MAP fit: %s", hipGetErrorString(e));
        return MPM_OK;
    }

    mpm_status collect(mpm_report &rep, double *trace, int trace_len) override
    {
        MapCtl h;
        if (a.no_pinned) {
            const int nt = std::min(tl, trace_len);
            hipError_t e = hipMemcpy(&h, m.ctl, sizeof(MapCtl), hipMemcpyDeviceToHost);
            if (e == hipSuccess && nt > 0) e = hipMemcpy(trace, m.trace, sizeof(double) * nt, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "MAP fit: %s", hipGetErrorString(e));
        } else {
            memcpy(&h, host.p, sizeof(h));
            const double *ht = (const double *)((const char *)host.p + sizeof(MapCtl));
            for (int i = 0; i < tl && i < trace_len; i++) trace[i] = ht[i];
        }
        memset(&rep, 0, sizeof(rep));
        rep.nll = h.nll_final;
        rep.jtv = prior_on ? h.jtv : 0.0;
        rep.objective = rep.nll + rep.jtv;
        rep.outer_done = ml_as_map ? 0 : h.outer_done;
        rep.gn_done = h.gn_done;
        rep.cg_done = h.cg_done;
        rep.rejected = h.rejected;
        rep.degenerate_voxels = (int64_t)llround(h.degenerate);
        rep.nonfinite_voxels = (int64_t)llround(h.nonfinite);
        return MPM_OK;
    }
};

std::unique_ptr<FitJob> make_map_job(const FitArgs &a, Workspace &ws, Prof &prof, mpm_status *st)
{
    std::unique_ptr<MapJob> j(new MapJob(a, ws, prof));
    *st = j->setup();
    if (*st) return nullptr;
    return std::unique_ptr<FitJob>(j.release());
}

// ---------------------------------------------------------------------------
// Batched MAP fits: the sequence of MapJob (without spatial projection), each
// launch a batched one over every volume; each volume keeps its own
// workspace, control block and trace, so its results are those of its fit
// alone.
// ---------------------------------------------------------------------------
static bool same_schedule(const mpm_options &a, const mpm_options &b)
{
    return a.mode == b.mode && a.n_outer == b.n_outer && a.n_gn == b.n_gn && a.n_cg == b.n_cg &&
           a.max_halvings == b.max_halvings && a.loading == b.loading && a.start_outer == b.start_outer &&
           a.tol_gn == b.tol_gn && a.tol_outer == b.tol_outer && a.cg_stop == b.cg_stop;
}

bool batch_compatible(const FitArgs &a, const FitArgs &b)
{
    return !a.spaces && !b.spaces && a.opt->mode == MPM_MAP_JTV && same_schedule(*a.opt, *b.opt) &&
           a.dtype == b.dtype && echo_shape(a.P) == echo_shape(b.P);
}

struct BatchMapJob : BatchJob {
    std::vector<FitArgs> a;
    Workspace &ws;
    Prof &prof;
    hipStream_t s = nullptr;
    int n = 0;
    std::vector<MapArgs> m;
    std::vector<int> prior_on;
    int ntrial = 1, accept_off = 0, T = 0, J = 0, K = 0, S = 0, tl = 0, t0 = 0;
    int t = 0, j = 0;
    bool started = false;
    double cg_stop = 0.0, tol_gn = 0.0, tol_outer = 0.0;
    BatchLaunch b;
    std::unique_ptr<InitStage[]> init;
    PinnedBuf staging;  // the device tables' host copy

    bool ready() const override
    {
        if (init)
            for (int v = 0; v < n; v++)
                if (!init[v].ready()) return false;
        return true;
    }
    double vox = 0.0, xvox = 0.0, bvox = 0.0;  // sums over volumes: N, N * echo bytes, N * field bytes

    BatchMapJob(const std::vector<FitArgs> &a_, Workspace &ws_, Prof &prof_) : a(a_), ws(ws_), prof(prof_) {}

    mpm_status setup()
    {
        n = (int)a.size();
        if (n < 1 || n > MAX_BATCH) return fail(MPM_ERR_INVALID_ARG, "a batch holds 1 to %d fits", MAX_BATCH);
        s = a[0].stream;
        const mpm_options *o = a[0].opt;
        for (int v = 1; v < n; v++)
            if (!batch_compatible(a[0], a[v]))
                return fail(MPM_ERR_UNSUPPORTED, "fit %d cannot share launches with fit 0 (batched fits need the same "
                                                 "schedule options, echo storage and register shape)", v);
        if (a[0].spaces || o->mode != MPM_MAP_JTV)
            return fail(MPM_ERR_UNSUPPORTED, "batched fits are JTV-MAP fits without spatial projection");
        T = o->n_outer;
        J = o->n_gn;
        K = o->n_cg;
        S = J + 2;
        tl = T * S;
        t = t0 = o->start_outer;
        ntrial = o->max_halvings < 0 ? 1 : o->max_halvings + 1;
        accept_off = o->max_halvings < 0;
        cg_stop = o->cg_stop;
        tol_gn = o->tol_gn;
        tol_outer = o->tol_outer;
        m.resize(n);
        prior_on.resize(n);
        for (int v = 0; v < n; v++) {
            memset(&m[v], 0, sizeof(MapArgs));
            mpm_status st = alloc_map(a[v], ws, m[v], tl);
            if (st) return st;
            set_prior(a[v].opt, m[v], true, prior_on[v]);
            m[v].tol_gn = tol_gn;
            m[v].tol_outer = tol_outer;
            const double N = (double)a[v].N;
            vox += N;
            xvox += N * a[v].P.I * dtype_size(a[v].dtype);
            bvox += N * ((a[v].b1 ? 4.0 : 0.0) + (a[v].opt->b1_receive ? 4.0 : 0.0));
        }
        // batched launches share one finaliser launch among their volumes: no folding
        for (int v = 0; v < n; v++) m[v].fold = 0;
        b.n = n;
        b.dtype = a[0].dtype;
        b.shape = echo_shape(a[0].P);
        b.loading = o->loading;
        // device tables: the workgroup ranges and one descriptor per volume
        BatchTab tab;
        fill_batch_tab(tab, m.data(), n, b.total);
        const size_t db = batch_desc_bytes(b.dtype, b.shape);
        std::vector<char> desc(db * (size_t)n);
        for (int v = 0; v < n; v++) fill_batch_desc(desc.data(), v, m[v], prior_on[v], b.dtype, b.shape);
        void *dtab = nullptr, *dvols = nullptr;
        if (ws.alloc(&dtab, sizeof(BatchTab)) != hipSuccess || ws.alloc(&dvols, desc.size()) != hipSuccess ||
            staging.alloc(sizeof(BatchTab) + desc.size()) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "batch table allocation failed");
        // staged in pinned memory owned by the job, so the copies are
        // asynchronous (the job outlives the work on its stream)
        char *h = (char *)staging.p;
        memcpy(h, &tab, sizeof(BatchTab));
        memcpy(h + sizeof(BatchTab), desc.data(), desc.size());
        hipError_t e = hipMemcpyAsync(dtab, h, sizeof(BatchTab), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(dvols, h + sizeof(BatchTab), desc.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "batch tables: %s", hipGetErrorString(e));
        b.tab = (const BatchTab *)dtab;
        b.vols = dvols;
        return MPM_OK;
    }

    hipError_t fin(int stage, int arg, int kind)
    {
        return launch_fin_batch(s, b, stage, arg, kind, cg_stop, ntrial, accept_off, tol_gn, tol_outer);
    }

    mpm_status enqueue_next(bool *more) override
    {
        hipError_t e = hipSuccess;
        const double V = vox;
#define RUNB(name, bytes, call)                                                   \
    do {                                                                          \
        if (e == hipSuccess) e = prof.launch(name, bytes, [&] { return call; }); \
    } while (0)
        *more = true;
        if (started)
            for (int v = 0; v < n; v++)
                if (init[v].pending) {
                    mpm_status st = init[v].finish(a[v]);
                    if (st) return st;
                }
        if (!started) {
            started = true;
            init.reset(new InitStage[n]);
            for (int v = 0; v < n; v++) {
                mpm_status st = init[v].start(a[v], ws, prof);
                if (st) return st;
            }
            e = launch_ctl_init_batch(s, b, tl);
            LaunchCtx c{s};
            for (int v = 0; v < n && e == hipSuccess; v++) e = launch_fill(c, m[v].w, a[v].N, 0.0f);
        } else if (t < T && J > 0) {
            if (j == 0 && t >= 1) {
                RUNB("jtv_weights", V * 20.0, launch_weights_batch(s, b));
                if (t > t0) RUNB("fin", 0.0, fin(FIN_W, (t - 1) * S + J + 1, BK_COL));
            }
            RUNB("map_lik", xvox + bvox + V * (16 + 4 + 40 + 16 + 16), launch_lik_batch(s, b));
            RUNB("fin", 0.0, fin(FIN_LIK, j == 0 ? t * S : -1, BK_PLANE));
            for (int i = 0; i < K && e == hipSuccess; i++) {
                double ab = 16 + (i > 0 ? 16 : 0) + 40 + 4 + 16 + (i == 1 ? 16 : i >= 2 ? 32 : 0);
                RUNB("cg_a", V * ab, launch_cg_a_batch(s, b, i));
                RUNB("fin", 0.0, fin(FIN_A, i, BK_TALL));
                RUNB("cg_b", V * (16 + 4 + 40 + 32 + 16), launch_cg_b_batch(s, b, i));
                RUNB("fin", 0.0, fin(FIN_B, i, BK_CGB));
            }
            RUNB("map_accept", xvox + bvox + V * (16 + 16 + 16 + 4), launch_accept_batch(s, b));
            RUNB("fin", 0.0, fin(FIN_ACCEPT, t * S + j + 1, BK_PLANE));
            if (ntrial > 1) {
                RUNB("map_accept2", 0.0, launch_accept2_batch(s, b, ntrial));
                RUNB("fin", 0.0, fin(FIN_ACCEPT2, t * S + j + 1, BK_COL));
            }
            RUNB("map_update", V * 64.0, launch_update_batch(s, b));
            if (tol_gn > 0.0) RUNB("fin", 0.0, fin(FIN_STOP, -1, BK_NONE));
            if (++j == J) {
                j = 0;
                t++;
            }
        } else {
            for (int tt = (J > 0 ? T : t0 + 1); tt < T && e == hipSuccess; tt++) {
                RUNB("jtv_weights", V * 20.0, launch_weights_batch(s, b));
                RUNB("fin", 0.0, fin(FIN_W, (tt - 1) * S + J + 1, BK_COL));
            }
            RUNB("jtv_weights", V * 20.0, launch_weights_batch(s, b));
            RUNB("fin", 0.0, fin(FIN_W, T >= 1 ? (T - 1) * S + J + 1 : -1, BK_COL));
            RUNB("map_final", xvox + bvox + V * (16 + 4), launch_final_batch(s, b));
            RUNB("fin", 0.0, fin(FIN_STATS, 0, BK_PLANE));
            *more = false;
        }
#undef RUNB
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "batched MAP fit: %s", hipGetErrorString(e));
        return MPM_OK;
    }

    mpm_status collect_item(int i, mpm_report &rep, double *trace, int trace_len) override
    {
        if (i < 0 || i >= n) return fail(MPM_ERR_INVALID_ARG, "no fit %d in this batch", i);
        MapCtl h;
        const int nt = std::min(tl, trace_len);
        hipError_t e = hipMemcpy(&h, m[i].ctl, sizeof(MapCtl), hipMemcpyDeviceToHost);
        if (e == hipSuccess && nt > 0) e = hipMemcpy(trace, m[i].trace, sizeof(double) * nt, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "batched MAP fit: %s", hipGetErrorString(e));
        memset(&rep, 0, sizeof(rep));
        rep.nll = h.nll_final;
        rep.jtv = prior_on[i] ? h.jtv : 0.0;
        rep.objective = rep.nll + rep.jtv;
        rep.outer_done = h.outer_done;
        rep.gn_done = h.gn_done;
        rep.cg_done = h.cg_done;
        rep.rejected = h.rejected;
        rep.degenerate_voxels = (int64_t)llround(h.degenerate);
        rep.nonfinite_voxels = (int64_t)llround(h.nonfinite);
        return MPM_OK;
    }
};

std::unique_ptr<BatchJob> make_batch_job(const std::vector<FitArgs> &a, Workspace &ws, Prof &prof, mpm_status *st)
{
    std::unique_ptr<BatchMapJob> j(new BatchMapJob(a, ws, prof));
    *st = j->setup();
    if (*st) return nullptr;
    return std::unique_ptr<BatchJob>(j.release());
}

}  // namespace mpm

using namespace mpm;

static mpm_status uncertainty_impl(const mpm_protocol *protocol, const mpm_grid *grid, const mpm_space *spaces,
                                   mpm_dtype dtype, const void *echoes, const float *b1, const mpm_options *opt,
                                   const float *maps, float *var, float *moments, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st;
    if ((st = check_protocol(protocol)) || (st = check_grid(grid, &N)) || (st = check_dtype(dtype))) return st;
    if (spaces && (st = check_spaces(protocol, spaces))) return st;
    if (!opt) return fail(MPM_ERR_INVALID_ARG, "options is NULL");
    if (spaces && opt->b1_receive)
        return fail(MPM_ERR_UNSUPPORTED, "b1_receive is not supported by the projected model");
    if (opt->basis != MPM_BASIS_LOG)
        return fail(MPM_ERR_UNSUPPORTED, "the uncertainty is defined on the log-parameters (basis %d)", opt->basis);
    if (!echoes || !maps || !var) return fail(MPM_ERR_INVALID_ARG, "echoes, maps and var must be device pointers");
    if (opt->mode != MPM_ML && opt->mode != MPM_MAP_JTV) return fail(MPM_ERR_INVALID_ARG, "unknown mode %d", opt->mode);
    if (opt->loading != MPM_LOAD_PROPOSED && opt->loading != MPM_LOAD_GN && opt->loading != MPM_LOAD_PROPOSED_PLUS)
        return fail(MPM_ERR_INVALID_ARG, "unknown loading %d", opt->loading);
    for (int k = 0; k < 4; k++)
        if (!(opt->lambda[k] >= 0.0) || !std::isfinite(opt->lambda[k]))
            return fail(MPM_ERR_INVALID_ARG, "lambda[%d] must be finite and >= 0", k);
    if (!(opt->jtv_eps >= 0.0)) return fail(MPM_ERR_INVALID_ARG, "jtv_eps must be >= 0");
    if (!has_mt(protocol)) return fail(MPM_ERR_UNSUPPORTED, "the four-parameter model needs at least one MT contrast");
    if ((st = check_echo_offset(protocol, dtype, opt->echo_offset))) return st;
    hipStream_t s = (hipStream_t)stream;
    FitArgs a{protocol, to_dev(protocol, opt->echo_offset), dtype, echoes, b1, opt, const_cast<float *>(maps), N,
              grid->nx, grid->ny, grid->nz, s, spaces};
    {
        Workspace ws(s);
        Prof prof(s);
        MapArgs m;
        memset(&m, 0, sizeof(m));
        m.g = make_grid3(a.nx, a.ny, a.nz, TILE_Y, column_target(a.nx, a.ny, a.nz));
        m.P = a.P;
        m.dtype = dtype;
        m.X = echoes;
        m.b1 = b1;
        m.bm = opt->b1_receive;
        m.Y = a.maps;  // only read
        m.gp = plane_grid(m.g);
        const int nblk = std::max(grid_blocks(m.g), grid_blocks(m.gp));
        if (ws.alloc((void **)&m.w, sizeof(float) * (size_t)N) != hipSuccess ||
            ws.alloc((void **)&m.partials, sizeof(double) * 3 * (size_t)nblk) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "uncertainty workspace allocation failed");
        int prior_on;
        set_prior(opt, m, opt->mode == MPM_MAP_JTV, prior_on);
        ProjState ps;
        if (spaces) {
            float4 *hb = nullptr;  // pushed Hessian blocks
            if (ws.alloc((void **)&hb, (size_t)N * 40) != hipSuccess)
                return fail(MPM_ERR_OUT_OF_MEMORY, "uncertainty workspace allocation failed");
            HessArrays Hr{hb, hb + N, (float2 *)(hb + 2 * N)};
            if ((st = alloc_proj(a, ws, ps, Hr, false))) return st;
        }
        const double xb = (double)a.P.I * dtype_size(dtype), bb = (b1 ? 4.0 : 0.0) + (m.bm ? 4.0 : 0.0);
        hipError_t e = prof.launch("jtv_weights", (double)N * 20.0, [&] { return launch_weights(s, m, prior_on); });
        if (!spaces) {
            if (e == hipSuccess)
                e = prof.launch("uncertainty", (double)N * (xb + bb + 16 + 4 + 16 + (moments ? 16 : 0)),
                                [&] { return launch_final(s, m, var, moments); });
        } else {
            for (int c = 0; c < ps.C && e == hipSuccess; c++)
                e = prof.launch("proj_lik", (double)ps.pc[c].S.M * (ps.pc[c].P.I * dtype_size(dtype) + 76),
                                [&] { return launch_proj_lik(s, m, ps.pc[c], ps.ext, 0); });
            if (e == hipSuccess)
                e = prof.launch("proj_push", (double)N * 56,
                                [&] { return launch_proj_push(s, m, ps.push, ps.G, ps.pp.H); });
            if (e == hipSuccess)
                e = prof.launch("uncertainty", (double)N * (56 + 4 + 16 + (moments ? 16 : 0)),
                                [&] { return launch_final_pushed(s, m, ps.pp, var, moments); });
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        prof.collect();
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "uncertainty: %s", hipGetErrorString(e));
    }
    return MPM_OK;
}

extern "C" mpm_status mpm_uncertainty(const mpm_protocol *protocol, const mpm_grid *grid, mpm_dtype dtype,
                                      const void *echoes, const float *b1, const mpm_options *opt,
                                      const float *maps, float *var, float *moments, void *stream)
{
    return uncertainty_impl(protocol, grid, nullptr, dtype, echoes, b1, opt, maps, var, moments, stream);
}

extern "C" mpm_status mpm_uncertainty_projected(const mpm_protocol *protocol, const mpm_grid *grid,
                                                const mpm_space *spaces, mpm_dtype dtype, const void *echoes,
                                                const float *b1, const mpm_options *opt, const float *maps,
                                                float *var, float *moments, void *stream)
{
    clear_error();
    if (!spaces) return fail(MPM_ERR_INVALID_ARG, "spaces is NULL");
    return uncertainty_impl(protocol, grid, spaces, dtype, echoes, b1, opt, maps, var, moments, stream);
}

extern "C" mpm_status mpm_fit_projected(const mpm_protocol *protocol, const mpm_grid *grid, const mpm_space *spaces,
                                        mpm_dtype dtype, const void *echoes, const float *b1,
                                        const mpm_options *opt, float *maps, mpm_report *report, double *trace,
                                        int32_t trace_len, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st = check_fit_args(protocol, grid, dtype, echoes, opt, maps, &N);
    if (st) return st;
    if ((st = check_spaces(protocol, spaces))) return st;
    if (opt->b1_receive) return fail(MPM_ERR_UNSUPPORTED, "b1_receive is not supported by the projected model");
    if (trace_len < 0 || (trace_len > 0 && !trace)) return fail(MPM_ERR_INVALID_ARG, "trace is NULL");
    for (int i = 0; i < trace_len; i++) trace[i] = NAN;
    hipStream_t s = (hipStream_t)stream;
    FitArgs a{protocol, to_dev(protocol, opt->echo_offset), dtype, echoes, b1, opt, maps, N,
              grid->nx, grid->ny, grid->nz, s, spaces};
    mpm_report rep;
    memset(&rep, 0, sizeof(rep));
    {
        Workspace ws(s);
        Prof prof(s);
        std::unique_ptr<FitJob> job = make_map_job(a, ws, prof, &st);
        if (st) return st;
        bool more = true;
        while (more)
            if ((st = job->enqueue_next(&more))) {
                // the work already enqueued ends before the job and its staging go
                (void)hipStreamSynchronize(s);
                return st;
            }
        hipError_t e = hipStreamSynchronize(s);
        prof.collect();
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "fit: %s", hipGetErrorString(e));
        if ((st = job->collect(rep, trace, trace_len))) return st;
    }
    if (report) *report = rep;
    return MPM_OK;
}

extern "C" mpm_status mpm_fit_batch(int32_t n, const mpm_request *requests, mpm_report *reports, double *traces,
                                    int32_t trace_len, void *stream)
{
    clear_error();
    if (n < 1 || n > MAX_BATCH) return fail(MPM_ERR_INVALID_ARG, "n=%d outside [1, %d]", n, MAX_BATCH);
    if (!requests) return fail(MPM_ERR_INVALID_ARG, "requests is NULL");
    if (trace_len < 0 || (trace_len > 0 && !traces)) return fail(MPM_ERR_INVALID_ARG, "traces is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::vector<FitArgs> a;
    for (int v = 0; v < n; v++) {
        const mpm_request &r = requests[v];
        int64_t N;
        mpm_status st = check_fit_args(&r.protocol, &r.grid, r.dtype, r.echoes, &r.options, r.maps, &N);
        if (st) return fail(st, "fit %d: %s", v, mpm_last_error());
        if (r.reserved != 0) return fail(MPM_ERR_INVALID_ARG, "fit %d: reserved must be 0", v);
        if (r.options.mode != MPM_MAP_JTV)
            return fail(MPM_ERR_UNSUPPORTED, "fit %d: mpm_fit_batch fits JTV-MAP volumes (an ML fit is one launch: "
                                             "use mpm_fit)", v);
        a.push_back(FitArgs{&r.protocol, to_dev(&r.protocol, r.options.echo_offset), r.dtype, r.echoes, r.b1,
                            &r.options, r.maps, N, r.grid.nx, r.grid.ny, r.grid.nz, s});
    }
    for (int i = 0; i < n * trace_len; i++) traces[i] = NAN;
    Workspace ws(s);
    Prof prof(s);
    mpm_status st;
    std::unique_ptr<BatchJob> job = make_batch_job(a, ws, prof, &st);
    if (st) return st;
    bool more = true;
    while (more)
        if ((st = job->enqueue_next(&more))) {
            // the work already enqueued ends before the job and its staging go
            (void)hipStreamSynchronize(s);
            return st;
        }
    hipError_t e = hipStreamSynchronize(s);
    prof.collect();
    if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "batched fit: %s", hipGetErrorString(e));
    for (int v = 0; v < n; v++) {
        mpm_report rep;
        if ((st = job->collect_item(v, rep, traces ? traces + (size_t)v * trace_len : nullptr, trace_len))) return st;
        if (reports) reports[v] = rep;
    }
    return MPM_OK;
}

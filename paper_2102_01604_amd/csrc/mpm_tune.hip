// mpm_tune.hip -- mpm_autotune: picks the workgroup count of CG sweep A (the
// dominant kernel of the MAP fit) for one grid size by timing candidates.
//
// The count sets how long a z-run each workgroup walks: fewer workgroups walk
// longer runs (fewer re-read boundary planes, a longer tail of the last round),
// more walk shorter ones.  Each candidate runs the steady-state sweep (the one
// that also updates the CG solution) on scratch buffers of the grid's size;
// the fastest is kept for that size.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "mpm_api_internal.h"
#include "mpm_map.h"
#include "mpm_tune.h"

namespace mpm {

namespace {
// Launch shape chosen for one grid size: the workgroup target of CG sweep A
// and of the column walks of the stencil-only kernels (0: built-in choice).
struct Shape {
    int tall = 0;
    int col = 0;
};
std::mutex g_mu;
std::map<std::tuple<int64_t, int64_t, int64_t>, Shape> g_tuned;
}  // namespace

// Built-in choice: grids beyond the last-level cache (about 4 M voxels at the
// sweep's 124 B per voxel) walk z-runs of 2 planes: measured on the 192 x 240
// x 256 volume, runs of 23 / 12 / 6 / 3 / 2 / 1 planes took 377 / 290 / 287 /
// 280 / 278 / 287 us (a shorter run leaves a shorter tail of the last round of
// workgroups; the boundary planes it shares with its z-neighbours stay in L2).
// Smaller grids keep the fixed target (measured there within a few per cent of
// the best; mpm_autotune finds it).  MPM_TALL_WORKGROUPS overrides both.
int tall_target(int64_t nx, int64_t ny, int64_t nz)
{
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_tuned.find(std::make_tuple(nx, ny, nz));
        if (it != g_tuned.end() && it->second.tall > 0) return it->second.tall;
    }
    if (std::getenv("MPM_TALL_WORKGROUPS")) return tall_workgroups();
    const int64_t tiles = ((nx + TILE_X - 1) / TILE_X) * ((ny + TALL_Y - 1) / TALL_Y);
    if (nx * ny * nz >= ((int64_t)1 << 22)) return (int)std::min<int64_t>((tiles * nz + 1) / 2, 1 << 20);
    return tall_workgroups();
}

int column_target(int64_t nx, int64_t ny, int64_t nz)
{
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_tuned.find(std::make_tuple(nx, ny, nz));
    if (it != g_tuned.end() && it->second.col > 0) return it->second.col;
    return stencil_workgroups();
}

}  // namespace mpm

using namespace mpm;

extern "C" mpm_status mpm_autotune(const mpm_grid *grid, int32_t reps, mpm_tune_result *result, void *stream)
{
    clear_error();
    int64_t N;
    mpm_status st;
    if ((st = check_grid(grid, &N))) return st;
    if (N < 2) return fail(MPM_ERR_INVALID_ARG, "the CG sweeps need at least 2 voxels");
    if (reps < 1 || reps > 1000) return fail(MPM_ERR_INVALID_ARG, "reps must be in [1, 1000]");
    static const int cand[] = {512, 1024, 2048, 4096, 8192, 16384};
    constexpr int NC = (int)(sizeof(cand) / sizeof(cand[0]));
    static_assert(NC <= 8, "mpm_tune_result holds 8 candidates");
    mpm_tune_result r;
    memset(&r, 0, sizeof(r));
    Grid3 grids[NC];
    int nblk = 1;
    for (int k = 0; k < NC; k++) {
        const Grid3 g = make_grid3(grid->nx, grid->ny, grid->nz, TALL_Y, cand[k]);
        bool same = false;  // candidates that give the same launch are timed once
        for (int j = 0; j < r.n_candidates; j++)
            same = same || (grids[j].zc == g.zc && grids[j].gz == g.gz);
        if (same) continue;
        grids[r.n_candidates] = g;
        r.target[r.n_candidates] = cand[k];
        r.workgroups[r.n_candidates] = grid_blocks(g);
        r.planes_per_run[r.n_candidates] = g.zc;
        nblk = std::max(nblk, grid_blocks(g));
        r.n_candidates++;
    }
    hipStream_t s = (hipStream_t)stream;
    {
        Workspace ws(s);
        MapArgs m;
        memset(&m, 0, sizeof(m));
        float4 *hb = nullptr, *vec = nullptr;
        if (ws.alloc((void **)&hb, (size_t)N * 40) != hipSuccess ||
            ws.alloc((void **)&vec, sizeof(float4) * 4 * (size_t)N) != hipSuccess ||
            ws.alloc((void **)&m.w, sizeof(float) * (size_t)N) != hipSuccess ||
            ws.alloc((void **)&m.ctl, sizeof(MapCtl)) != hipSuccess ||
            ws.alloc((void **)&m.partials, sizeof(double) * (size_t)nblk) != hipSuccess)
            return fail(MPM_ERR_OUT_OF_MEMORY, "autotune: scratch allocation failed");
        m.H = HessArrays{hb, hb + N, (float2 *)(hb + 2 * N)};
        m.Z = vec;
        m.P0 = vec + N;
        m.P1 = vec + 2 * N;
        m.D = vec + 3 * N;
        for (int k = 0; k < 4; k++) m.lam[k] = 1e-3f;
        hipError_t e = hipMemsetAsync(hb, 0, (size_t)N * 40, s);
        if (e == hipSuccess) e = hipMemsetAsync(vec, 0, sizeof(float4) * 4 * (size_t)N, s);
        if (e == hipSuccess) e = hipMemsetAsync(m.w, 0, sizeof(float) * (size_t)N, s);
        if (e == hipSuccess) e = hipMemsetAsync(m.ctl, 0, sizeof(MapCtl), s);  // no stop flags: full sweeps
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        for (int c = 0; c < r.n_candidates && e == hipSuccess; c++) {
            m.gt = grids[c];
            e = launch_cg_a(s, m, 2);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int k = 0; k < reps && e == hipSuccess; k++) e = launch_cg_a(s, m, 2 + (k & 1));
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            r.ms[c] = (double)ms / reps;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (e != hipSuccess) return fail(MPM_ERR_DEVICE, "autotune: %s", hipGetErrorString(e));
    }
    for (int c = 1; c < r.n_candidates; c++)
        if (r.ms[c] < r.ms[r.chosen]) r.chosen = c;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_tuned[std::make_tuple(grid->nx, grid->ny, grid->nz)].tall = r.target[r.chosen];
    }
    if (result) *result = r;
    return MPM_OK;
}

extern "C" mpm_status mpm_autotune_set(const mpm_grid *grid, int32_t cg_workgroups, int32_t column_workgroups)
{
    clear_error();
    int64_t N;
    mpm_status st;
    if ((st = check_grid(grid, &N))) return st;
    if (cg_workgroups < 0 || cg_workgroups > (1 << 20))
        return fail(MPM_ERR_INVALID_ARG, "cg_workgroups must be in [0, 2^20]");
    if (column_workgroups < 0 || column_workgroups > (1 << 20))
        return fail(MPM_ERR_INVALID_ARG, "column_workgroups must be in [0, 2^20]");
    std::lock_guard<std::mutex> lock(g_mu);
    Shape &sh = g_tuned[std::make_tuple(grid->nx, grid->ny, grid->nz)];
    sh.tall = cg_workgroups;
    sh.col = column_workgroups;
    return MPM_OK;
}

extern "C" void mpm_autotune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_tuned.clear();
}

// Tile-shape autotuner.  The cell-per-lane kernels (Laplacian, CG) take a
// tile of 64 x cw cells (cw in {4, 8, 16} waves) and the row-per-lane bracket
// kernel a tile of rw rows (rw in {8, 16}).  Taller tiles re-read fewer halo
// rows but hold more registers and LDS per workgroup; which wins depends on
// n and on the grid, so the tuner times the real kernels on the grid and
// keeps the fastest shapes in it.
#include <hip/hip_runtime.h>

#include <cmath>

#include "abi_types.h"
#include "dg_launch.h"

using namespace dgk;

namespace {

constexpr int kCellCandidates[3] = {4, 8, 16};
constexpr int kRowCandidates[2] = {8, 16};

bool valid_cw(int cw) { return cw == 4 || cw == 8 || cw == 16; }
bool valid_rw(int rw) { return rw == 8 || rw == 16; }

// Mean milliseconds of one CG iteration (direction + residual kernels) with
// the grid's current cell tile, from a fresh CG setup on omega that cannot
// converge (tol = 0).  Returns a negative status on error.
int time_cg(dg_grid* g, const double* omega, dg_workspace* ws, int reps, hipEvent_t e0,
            hipEvent_t e1, hipStream_t s, float* ms) {
    const Geom& geom = g->geom;
    hipError_t e = launch_cg_mean(geom, g->k64, omega, nullptr, nullptr, 0.0, 0.0, g->area,
                                  0.0, 1 << 30, ws->d, s);
    if (e == hipSuccess)
        e = launch_cg_init(geom, g->k64, omega, nullptr, nullptr, 0.0, 0.0, ws->x, ws->r,
                           ws->d, s);
    for (int i = 0; e == hipSuccess && i < 2; ++i)
        e = launch_cg_iter<double>(geom, g->k64, ws->x, ws->r, ws->p0, ws->p1, ws->d.sc,
                                   ws->d, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; e == hipSuccess && i < reps; ++i)
        e = launch_cg_iter<double>(geom, g->k64, ws->x, ws->r, ws->p0, ws->p1, ws->d.sc,
                                   ws->d, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "tuning CG launch");
    CgScalars h;
    HIP_TRY(hipMemcpy(&h, ws->d.sc, sizeof h, hipMemcpyDeviceToHost));
    if (h.done)
        return fail(DG_E_INVAL, "tuning needs an omega whose mean-free part is nonzero "
                    "(the CG stopped after %d iterations)", h.iter);
    *ms /= reps;
    return DG_OK;
}

int time_rhs(dg_grid* g, const double* omega, dg_workspace* ws, int reps, hipEvent_t e0,
             hipEvent_t e1, hipStream_t s, float* ms) {
    RhsParams p{};
    p.c0 = p.c1 = p.c2 = 1.0;
    p.scale = 1.0 / 3.0;
    p.D = 1e-3;
    p.dt = 1e-3;
    p.a = 0.0;
    p.b = 1.0;
    hipError_t e = launch_rhs(g->geom, g->k64, ws->s2, omega, nullptr, ws->s1, p, true, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; e == hipSuccess && i < reps; ++i)
        e = launch_rhs(g->geom, g->k64, ws->s2, omega, nullptr, ws->s1, p, true, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "tuning bracket launch");
    *ms /= reps;
    return DG_OK;
}

}  // namespace

extern "C" {

int dg_grid_set_tiles(dg_grid* g, int cw, int rw) {
    if (!g) return fail(DG_E_INVAL, "grid is NULL");
    if (!valid_cw(cw) || !valid_rw(rw))
        return fail(DG_E_INVAL, "tile heights must be cw in {4, 8, 16} and rw in {8, 16}");
    if ((g->geom.bcx || g->geom.bcy) && cw != kDirichletCellWaves)
        return fail(DG_E_INVAL, "a grid with a Dirichlet axis uses cell tiles of %d waves",
                    kDirichletCellWaves);
    g->geom.cw = cw;
    g->geom.rw = rw;
    return DG_OK;
}

int dg_grid_tiles(const dg_grid* g, int* cw, int* rw) {
    if (!g || !cw || !rw) return fail(DG_E_INVAL, "NULL argument");
    *cw = g->geom.cw;
    *rw = g->geom.rw;
    return DG_OK;
}

int dg_grid_tune(dg_grid* g, const double* omega, int reps, double* ms_out5, void* stream) {
    if (!g || !omega) return fail(DG_E_INVAL, "NULL argument");
    if (g->geom.bcx || g->geom.bcy) return periodic_only("the tile tuner");
    if (reps < 1) return fail(DG_E_INVAL, "reps must be >= 1");
    const hipStream_t s = (hipStream_t)stream;
    dg_workspace* ws = nullptr;
    int rc = dg_workspace_create(g, DG_PREC_FP64, &ws);
    if (rc != DG_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        dg_workspace_destroy(ws);
        return fail(DG_E_HIP, "event creation failed");
    }
    const int cw0 = g->geom.cw, rw0 = g->geom.rw;
    float t_cell[3] = {0, 0, 0}, t_row[2] = {0, 0};
    for (int i = 0; rc == DG_OK && i < 3; ++i) {
        g->geom.cw = kCellCandidates[i];
        rc = time_cg(g, omega, ws, reps, e0, e1, s, &t_cell[i]);
    }
    // the bracket's second argument: the derivative-rich field s2 = Lap_h omega
    if (rc == DG_OK) {
        g->geom.cw = cw0;
        hipError_t e = launch_laplace(g->geom, g->k64, omega, ws->s2, s);
        if (e != hipSuccess) rc = hip_fail(e, "tuning Laplacian launch");
    }
    for (int i = 0; rc == DG_OK && i < 2; ++i) {
        g->geom.rw = kRowCandidates[i];
        rc = time_rhs(g, omega, ws, reps, e0, e1, s, &t_row[i]);
    }
    if (rc == DG_OK) {
        int bc = 0, br = 0;
        for (int i = 1; i < 3; ++i) if (t_cell[i] < t_cell[bc]) bc = i;
        if (t_row[1] < t_row[0]) br = 1;
        g->geom.cw = kCellCandidates[bc];
        g->geom.rw = kRowCandidates[br];
        if (ms_out5) {
            for (int i = 0; i < 3; ++i) ms_out5[i] = t_cell[i];
            for (int i = 0; i < 2; ++i) ms_out5[3 + i] = t_row[i];
        }
    } else {
        g->geom.cw = cw0;
        g->geom.rw = rw0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dg_workspace_destroy(ws);
    return rc;
}

}  // extern "C"

// K-step Adams-Bashforth stepper (the paper's time integrator, Sec. 6, with
// K = 1..4 as in Table 4):
//     omega_{n+1} = omega_n + dt sum_{j<K} b_j R(omega_{n-j}),
// R = -J(psi, omega) + D Lap_h omega with psi from the Poisson solve of each
// step (initial guess extrapolated from the last two solves).  The state
// keeps the last K right-hand sides; while fewer than K-1 earlier ones exist
// a step is taken by SSP-RK3 instead (the paper does not say how the
// multistep method starts; this is the reading).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "abi_types.h"
#include "dg_launch.h"

using namespace dgk;

struct dg_ab_state {
    int n, nx, ny, K;
    size_t elems;
    dg_state* st;          // psi history and time
    double* R[4];          // right-hand sides, R[0] the newest
    int count;             // right-hand sides recorded so far
};

namespace {

// Adams-Bashforth weights of order K (integrals of the Lagrange polynomials
// through the last K right-hand sides).
const double kAB[4][4] = {
    {1.0, 0.0, 0.0, 0.0},
    {3.0 / 2.0, -1.0 / 2.0, 0.0, 0.0},
    {23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0, 0.0},
    {55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0},
};

}  // namespace

extern "C" {

int dg_ab_state_create(const dg_grid* g, int K, double t0, dg_ab_state** out) {
    if (!g || !out) return fail(DG_E_INVAL, "NULL argument");
    *out = nullptr;
    if (K < 1 || K > 4) return fail(DG_E_INVAL, "K = %d outside [1, 4]", K);
    dg_ab_state* ab = new (std::nothrow) dg_ab_state;
    if (!ab) return fail(DG_E_NOMEM, "host allocation failed");
    std::memset(ab, 0, sizeof *ab);
    ab->n = g->n; ab->nx = g->nx; ab->ny = g->ny; ab->K = K; ab->elems = g->elems;
    int rc = dg_state_create(g, t0, &ab->st);
    if (rc != DG_OK) { delete ab; return rc; }
    for (int j = 0; j < K; ++j) {
        if (hipMalloc((void**)&ab->R[j], g->elems * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            dg_ab_state_destroy(ab);
            return fail(DG_E_NOMEM, "Adams-Bashforth state allocation failed");
        }
    }
    *out = ab;
    return DG_OK;
}

void dg_ab_state_destroy(dg_ab_state* ab) {
    if (!ab) return;
    for (double* r : ab->R) if (r) (void)hipFree(r);
    dg_state_destroy(ab->st);
    delete ab;
}

double dg_ab_time(const dg_ab_state* ab) { return ab ? ab->st->t : 0.0; }

const dg_state* dg_ab_psi_state(const dg_ab_state* ab) { return ab ? ab->st : nullptr; }

int dg_ab_step(const dg_grid* g, double* omega, dg_ab_state* ab, const dg_step_opts* opts,
               dg_step_stats* stats, dg_workspace* ws, void* stream) {
    if (!g || !omega || !ab || !opts) return fail(DG_E_INVAL, "NULL argument");
    if (!ws) return fail(DG_E_INVAL, "workspace is NULL");
    if (ab->n != g->n || ab->nx != g->nx || ab->ny != g->ny)
        return fail(DG_E_INVAL, "Adams-Bashforth state was made for another grid");
    if (!std::isfinite(opts->dt) || !std::isfinite(opts->D))
        return fail(DG_E_INVAL, "dt and D must be finite");
    double fc[4];
    const int frc = form_coeffs(opts->form, &fc[0], &fc[1], &fc[2], &fc[3]);
    if (frc != DG_OK) return frc;
    const hipStream_t s = (hipStream_t)stream;
    const int K = ab->K;
    dg_state* st = ab->st;
    const double t = st->t, dt = opts->dt;
    if (stats) std::memset(stats, 0, sizeof *stats);
    // psi_n from the extrapolated guess
    const double* pa;
    const double* pb;
    double ca, cb;
    double* x;
    int fr;
    state_guess(st, t, &pa, &ca, &pb, &cb, &x, &fr);
    dg_cg_stats cs{};
    int rc = solve_poisson(g, omega, x, pa, ca, pb, cb, &opts->cg, &cs, ws, s);
    int result = DG_OK;
    if (rc == DG_E_NOCONV) result = DG_E_NOCONV;
    else if (rc != DG_OK) return rc;
    state_push(st, fr, t);
    // R_n into the oldest slot, which becomes R[0]
    double* rn = ab->R[K - 1];
    for (int j = K - 1; j > 0; --j) ab->R[j] = ab->R[j - 1];
    ab->R[0] = rn;
    RhsParams p{fc[0], fc[1], fc[2], fc[3], opts->D, 1.0, 0.0, 1.0, 1};
    hipError_t e = launch_rhs(g->geom, g->k64, x, omega, nullptr, rn, p, true, s);
    if (e != hipSuccess) return hip_fail(e, "rhs launch");
    if (stats) stats->cg_iters[0] = cs.iters;
    bool conv = rc == DG_OK;
    if (ab->count < K - 1) {
        // start-up: one SSP-RK3 step on the same psi history (its first
        // stage re-solves at t from the exact guess)
        dg_step_stats rs{};
        dg_step_opts o = *opts;
        o.record_times = 0;
        rc = dg_rk_step(g, omega, st, &o, &rs, ws, stream);
        if (rc == DG_E_NOCONV) { result = DG_E_NOCONV; conv = false; }
        else if (rc != DG_OK) return rc;
        if (stats) stats->cg_iters[1] = rs.cg_iters[0] + rs.cg_iters[1] + rs.cg_iters[2];
    } else {
        double c[4];
        for (int j = 0; j < K; ++j) c[j] = dt * kAB[K - 1][j];
        e = launch_ab_combine((long)ab->elems, omega, ab->R, c, K, s);
        if (e != hipSuccess) return hip_fail(e, "Adams-Bashforth update launch");
        st->t = t + dt;
    }
    ab->count += 1;
    if (stats) stats->converged = conv ? 1 : 0;
    if (result != DG_OK) return fail(result, "a Poisson solve did not converge");
    HIP_TRY(hipStreamSynchronize(s));
    return DG_OK;
}

}  // extern "C"

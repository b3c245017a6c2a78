// C ABI of libdgark: argument validation, device memory of workspaces and
// states, the host side of the CG and SSP-RK3 drivers.  Every step of the
// computation runs in the kernels of kernels.hip; this file only queues
// them and polls the device convergence flag.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "abi_types.h"
#include "dg_launch.h"

using namespace dgk;

namespace dgk {

namespace {
thread_local std::string g_err;
}  // namespace

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(DG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

void state_guess(const dg_state* st, double ts, const double** pa, double* ca,
                 const double** pb, double* cb, double** x, int* xi) {
    *pa = nullptr;
    *pb = nullptr;
    *ca = 0.0;
    *cb = 0.0;
    if (st->count >= 1) {
        *pa = st->buf[st->ia];
        *ca = 1.0;
        if (st->count >= 2 && st->ta != st->tb) {
            const double th = (ts - st->ta) / (st->ta - st->tb);
            *pb = st->buf[st->ib];
            *ca = 1.0 + th;
            *cb = -th;
        }
    }
    int fr = 0;
    while (fr == st->ia || fr == st->ib || fr == st->resv[0] || fr == st->resv[1]) ++fr;
    *x = st->buf[fr];
    *xi = fr;
}

void state_push(dg_state* st, int xi, double ts) {
    st->ib = st->ia;
    st->ia = xi;
    st->tb = st->ta;
    st->ta = ts;
    st->count += 1;
}

}  // namespace dgk

namespace {

template <class T>
void fill_const(const dg_grid& g, OpConst<T>& k) {
    std::memset(&k, 0, sizeof k);
    const int n = g.n;
    AxisLdg ax, ay;
    ldg_axis(g.t, g.hx, g.geom.bcx == 0, &ax);
    ldg_axis(g.t, g.hy, g.geom.bcy == 0, &ay);
    for (int i = 0; i < n * n; ++i) {
        k.C0[i] = (T)g.t.C0[i];
        k.L0x[i] = (T)ax.L0[i];
        k.L0y[i] = (T)ay.L0[i];
        k.L0Bx[i] = (T)ax.L0B[i];
        k.L0By[i] = (T)ay.L0B[i];
    }
    for (int i = 0; i < n; ++i) {
        k.cR[i] = (T)g.t.cR[i]; k.sR[i] = (T)g.t.sR[i];
        k.cL[i] = (T)g.t.cL[i]; k.sL[i] = (T)g.t.sL[i];
        k.eRx[i] = (T)ax.eR[i]; k.eRy[i] = (T)ay.eR[i];
        k.lLx[i] = (T)ax.lL[i]; k.lLy[i] = (T)ay.lL[i];
        k.lR[i] = (T)g.t.lR[i]; k.eL[i] = (T)g.t.eL[i];
        k.eRBx[i] = (T)ax.eRB[i]; k.eRBy[i] = (T)ay.eRB[i];
        k.lLBx[i] = (T)ax.lLB[i]; k.lLBy[i] = (T)ay.lLB[i];
        k.w[i] = (T)g.t.w[i];
    }
    k.ihx = (T)(1.0 / g.hx);
    k.ihy = (T)(1.0 / g.hy);
    k.ihx2 = (T)(1.0 / (g.hx * g.hx));
    k.ihy2 = (T)(1.0 / (g.hy * g.hy));
    k.wq = 0.25 * g.hx * g.hy;
}

bool ranges_overlap(const void* a, const void* b, size_t bytes) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bytes && pb < pa + bytes;
}

int check_ws(const dg_grid* g, const dg_workspace* ws) {
    if (!ws) return fail(DG_E_INVAL, "workspace is NULL");
    if (ws->n != g->n || ws->nx != g->nx || ws->ny != g->ny)
        return fail(DG_E_WORKSPACE, "workspace was made for another grid");
    return DG_OK;
}

// precision part of a workspace mode
int prec_of(int mode) { return mode & ~(DG_WS_FD | DG_WS_FD_PRODUCTS); }

bool valid_mode(int mode) {
    const int prec = prec_of(mode);
    if ((mode & DG_WS_FD_PRODUCTS) && !(mode & DG_WS_FD)) return false;
    return prec == DG_PREC_FP64 || prec == DG_PREC_MIXED;
}

size_t ws_bytes(const dg_grid* g, int mode) {
    const size_t F = g->elems * sizeof(double);
    const size_t L = l64_elems(g->geom);
    int blocks = stencil_blocks(g->geom);
    if (blocks < pointwise_block_cap()) blocks = pointwise_block_cap();
    size_t b = 4 * L * sizeof(double) + 2 * F;          // x, r, p0, p1; s1, s2
    b += (size_t)blocks * 4 * sizeof(double);           // partials
    b += sizeof(CgScalars) + kCntBytes + 4 * sizeof(double);
    if (prec_of(mode) == DG_PREC_MIXED) b += 3 * L * sizeof(float);
    if (mode & DG_WS_FD)
        b += L * sizeof(double) + F + 3 * sizeof(CgScalars) + fd_bytes(g);   // z, wbak, sc3
    return b;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// Copy the device scalars (outer and, if given, inner) to pinned host memory
// and wait for them.
int read_scalars(dg_workspace* ws, const CgScalars* dev, CgScalars* host,
                 hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(host, dev, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)ws;
    return DG_OK;
}

// Queue CG iterations in chunks and poll the device `done` flag one chunk
// behind, so the device never waits for the host.  Iterations queued after
// convergence exit at their first instruction.
// Fold the sampled kernel durations of a completed poll slot into the
// workspace totals; a sample counts only if the device really executed that
// iteration (iterations queued after convergence exit immediately).
int harvest_profile(dg_workspace* ws, int slot, int device_iter) {
    if (ws->pev_iter[slot] < 0) return DG_OK;
    if (device_iter > ws->pev_iter[slot]) {
        float a = 0.f, b = 0.f;
        HIP_TRY(hipEventElapsedTime(&a, ws->pev[slot][0], ws->pev[slot][1]));
        HIP_TRY(hipEventElapsedTime(&b, ws->pev[slot][2], ws->pev[slot][3]));
        ws->prof_ms[0] += a;
        ws->prof_ms[1] += b;
        ws->prof_n[0] += 1;
        ws->prof_n[1] += 1;
    }
    ws->pev_iter[slot] = -1;
    return DG_OK;
}

template <class T>
int cg_loop(const Geom& geom, const OpConst<double>& k, T* x, T* r, T* p0, T* p1,
            CgScalars* sc, int max_iter, int check_every, dg_workspace* ws,
            hipStream_t s, CgScalars* final_host) {
    const int chunk = check_every > 0 ? check_every : 32;
    int issued = 0, round = 0, prev = -1;
    ws->pev_iter[0] = ws->pev_iter[1] = -1;
    for (;;) {
        int m = max_iter - issued;
        if (m > chunk) m = chunk;
        const int slot = round & 1;
        // the sampled iteration alternates between the first and the second
        // of a chunk, so that FP64 solves time direction updates with and
        // without the x update alike
        const int ti = (round & 1) && m > 1 ? 1 : 0;
        for (int i = 0; i < m; ++i) {
            hipError_t e;
            if (ws->prof_on && i == ti) {
                e = launch_cg_dir_timed<T>(geom, k, x, r, p0, p1, sc, ws->d, s,
                                           ws->pev[slot][0], ws->pev[slot][1]);
                if (e != hipSuccess) return hip_fail(e, "cg direction launch");
                e = launch_cg_res_timed<T>(geom, k, r, p0, p1, sc, ws->d, s,
                                           ws->pev[slot][2], ws->pev[slot][3]);
                if (e != hipSuccess) return hip_fail(e, "cg residual launch");
                ws->pev_iter[slot] = issued + i;
            } else {
                e = launch_cg_iter<T>(geom, k, x, r, p0, p1, sc, ws->d, s);
                if (e != hipSuccess) return hip_fail(e, "cg iteration launch");
            }
        }
        issued += m;
        HIP_TRY(hipMemcpyAsync(&ws->host[slot], sc, sizeof(CgScalars),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(ws->ev[slot], s));
        if (issued >= max_iter) {
            HIP_TRY(hipEventSynchronize(ws->ev[slot]));
            *final_host = ws->host[slot];
            if (prev >= 0) {
                int rc = harvest_profile(ws, prev, final_host->iter);
                if (rc != DG_OK) return rc;
            }
            return harvest_profile(ws, slot, final_host->iter);
        }
        if (prev >= 0) {
            HIP_TRY(hipEventSynchronize(ws->ev[prev]));
            int rc = harvest_profile(ws, prev, ws->host[prev].iter);
            if (rc != DG_OK) return rc;
            if (ws->host[prev].done) {
                *final_host = ws->host[prev];
                // the newer slot's sample ran after convergence: drop it
                ws->pev_iter[slot] = -1;
                return DG_OK;
            }
        }
        prev = slot;
        ++round;
    }
}

// FP64 CG from the guess ca*pa + cb*pb into x (x must not alias pa or pb).
int cg_fp64(const dg_grid* g, const double* omega, double* x, const double* pa,
            double ca, const double* pb, double cb, const dg_cg_opts& o,
            dg_cg_stats* st, dg_workspace* ws, hipStream_t s) {
    const double tol2 = o.rtol * o.rtol;
    hipError_t e = launch_cg_mean(g->geom, g->k64, omega, pa, pb, ca, cb, g->area,
                                  tol2, o.max_iter, ws->d, s);
    if (e != hipSuccess) return hip_fail(e, "cg mean launch");
    e = launch_cg_init(g->geom, g->k64, omega, pa, pb, ca, cb, ws->x, ws->r, ws->d, s);
    if (e != hipSuccess) return hip_fail(e, "cg init launch");
    CgScalars fin;
    int rc = cg_loop<double>(g->geom, g->k64, ws->x, ws->r, ws->p0, ws->p1, ws->d.sc,
                             o.max_iter, o.check_every, ws, s, &fin);
    if (rc != DG_OK) return rc;
    e = launch_cg_finish<double>(g->geom, g->k64, ws->x, ws->p0, ws->p1, x, g->area,
                                 ws->d, s);
    if (e != hipSuccess) return hip_fail(e, "cg finish launch");
    rc = read_scalars(ws, ws->d.sc, &ws->host[2], s);
    if (rc != DG_OK) return rc;
    const CgScalars& h = ws->host[2];
    if (st) {
        st->iters = h.iter;
        st->outer_iters = 0;
        st->rel_residual = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
        st->converged = h.converged;
    }
    if (!h.converged)
        return fail(DG_E_NOCONV, "CG stopped after %d iterations, relative residual %.3e%s",
                    h.iter, h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0,
                    h.breakdown ? " (breakdown or non-finite data)" : "");
    return DG_OK;
}

// Mixed precision: r and the directions p are stored in FP32 (lane-
// interleaved r32, q0, q1), the solution x in FP64; every operator, update
// and dot product is computed in FP64 (only the stores round).  After every
// segment of check_every iterations (and whenever the recursive residual
// meets the tolerance) the true residual of the FP64 solution is recomputed
// in FP64 and replaces r32 while the recurrence continues (no restart).
// Stops when that FP64 residual has ||r||_W <= rtol ||b||_W.
int cg_mixed(const dg_grid* g, const double* omega, double* x, const double* pa,
             double ca, const double* pb, double cb, const dg_cg_opts& o,
             dg_cg_stats* st, dg_workspace* ws, hipStream_t s) {
    const double tol2 = o.rtol * o.rtol;
    const int segment = o.check_every > 0 ? o.check_every : 32;
    hipError_t e = launch_cg_mean(g->geom, g->k64, omega, pa, pb, ca, cb, g->area,
                                  tol2, o.max_iter, ws->d, s);
    if (e != hipSuccess) return hip_fail(e, "cg mean launch");
    e = launch_cg_init(g->geom, g->k64, omega, pa, pb, ca, cb, ws->x, ws->r, ws->d, s);
    if (e != hipSuccess) return hip_fail(e, "cg init launch");
    int rc = read_scalars(ws, ws->d.sc, &ws->host[2], s);
    if (rc != DG_OK) return rc;
    CgScalars h = ws->host[2];
    if (!h.done) {
        e = launch_mixed_start(g->geom, g->k64, ws->r, ws->r32, ws->d, s);
        if (e != hipSuccess) return hip_fail(e, "mixed start launch");
        for (;;) {
            for (int i = 0; i < segment; ++i) {
                e = launch_cg_iter<float>(g->geom, g->k64, ws->x, ws->r32, ws->q0,
                                          ws->q1, ws->d.sc, ws->d, s);
                if (e != hipSuccess) return hip_fail(e, "mixed CG launch");
            }
            e = launch_mixed_replace(g->geom, g->k64, omega, ws->x, ws->q0, ws->q1,
                                     ws->r32, ws->d, s);
            if (e != hipSuccess) return hip_fail(e, "mixed replacement launch");
            rc = read_scalars(ws, ws->d.sc, &ws->host[2], s);
            if (rc != DG_OK) return rc;
            h = ws->host[2];
            if (h.done) break;
        }
    } else {
        h.rr_true = h.rr;
    }
    // psi (canonical) = x + the pending alpha p_last (FP32 directions),
    // minus its W-mean; b = 0 gives psi = 0
    e = launch_cg_finish<float>(g->geom, g->k64, ws->x, ws->q0, ws->q1, x, g->area,
                                ws->d, s);
    if (e != hipSuccess) return hip_fail(e, "cg finish launch");
    HIP_TRY(hipStreamSynchronize(s));
    const double rel = h.bb > 0 ? std::sqrt(h.rr_true / h.bb) : 0.0;
    if (st) {
        st->iters = h.iter;
        st->outer_iters = h.outer;
        st->rel_residual = rel;
        st->converged = h.converged;
    }
    if (!h.converged)
        return fail(DG_E_NOCONV, "mixed CG stopped after %d iterations (%d residual "
                    "replacements), relative residual %.3e", h.iter, h.outer, rel);
    return DG_OK;
}

// z = M r on node planes in the precision T, then z and <r, z>_W in FP64
// (device scalars in d.sc).
template <class T>
int precond_step(const dg_grid* g, dg_workspace* ws, const DevScratch& d, hipStream_t s) {
    T* planes = reinterpret_cast<T*>(ws->fd->img0);
    const int layout = fd_layout(ws->fd);
    const bool dense = layout == kFdDense;
    const int Kx = (g->nx + 1) / 2;
    hipError_t e = layout == kFdFolded
                       ? launch_to_planes_fold<T>(g->geom, ws->r, true, Kx, planes, s)
                       : launch_to_image<T>(g->geom, g->k64, ws->r, true, dense, planes, s);
    if (e != hipSuccess) return hip_fail(e, "image conversion launch");
    int rc = fd_apply_image(ws->fd, sizeof(T) == sizeof(float), s);
    if (rc != DG_OK) return rc;
    e = layout == kFdFolded
            ? launch_from_planes_fold<T>(g->geom, g->k64, planes, Kx, ws->z, ws->r, &d, s)
            : launch_from_image_dot<T>(g->geom, g->k64, planes, dense, ws->z, ws->r, d, s);
    if (e != hipSuccess) return hip_fail(e, "image conversion launch");
    return DG_OK;
}

int pcg_iteration(const dg_grid* g, bool fp32, const DevScratch& d, dg_workspace* ws,
                  hipStream_t s);

// Queue the setup of a preconditioned solve and `iters` iterations (z = M r
// on node planes -- cell Fourier transforms + per-wave-number mixing --
// then the direction / residual kernels with p built from z) on the device
// scalars d.sc, reading nothing back.  Once the device flag says the solve
// is done the CG kernels exit at once; the preconditioner's library
// transforms of a later iteration still run.  fp32: M is applied in FP32
// (the mixed-precision form: the solve's bulk work in FP32, every residual,
// solution and step length in FP64, so the FP64 iteration refines the FP32
// solves).
int pcg_queue(const dg_grid* g, const double* omega, const double* pa, double ca,
              const double* pb, double cb, const dg_cg_opts& o, bool fp32, int iters,
              const DevScratch& d, dg_workspace* ws, hipStream_t s) {
    const double tol2 = o.rtol * o.rtol;
    hipError_t e = launch_cg_mean(g->geom, g->k64, omega, pa, pb, ca, cb, g->area, tol2,
                                  o.max_iter, d, s);
    if (e != hipSuccess) return hip_fail(e, "cg mean launch");
    e = launch_cg_init(g->geom, g->k64, omega, pa, pb, ca, cb, ws->x, ws->r, d, s);
    if (e != hipSuccess) return hip_fail(e, "cg init launch");
    for (int it = 0; it < iters; ++it) {
        int rc = pcg_iteration(g, fp32, d, ws, s);
        if (rc != DG_OK) return rc;
    }
    return DG_OK;
}

int pcg_iteration(const dg_grid* g, bool fp32, const DevScratch& d, dg_workspace* ws,
                  hipStream_t s) {
    int rc = fp32 ? precond_step<float>(g, ws, d, s) : precond_step<double>(g, ws, d, s);
    if (rc != DG_OK) return rc;
    hipError_t e = launch_cg_dir<double>(g->geom, g->k64, ws->x, ws->z, ws->p0, ws->p1, d.sc,
                                         d, s);
    if (e == hipSuccess)
        e = launch_cg_res<double>(g->geom, g->k64, ws->r, ws->p0, ws->p1, d.sc, d, s);
    if (e != hipSuccess) return hip_fail(e, "pcg iteration launch");
    return DG_OK;
}

// Fill the solve statistics from final device scalars (host copy h).
int pcg_result(const CgScalars& h, dg_cg_stats* st) {
    const double rel = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    if (st) {
        st->iters = h.iter;
        st->outer_iters = 0;
        st->rel_residual = rel;
        st->converged = h.converged;
    }
    if (!h.converged)
        return fail(DG_E_NOCONV, "preconditioned CG stopped after %d iterations, "
                    "relative residual %.3e%s", h.iter, rel,
                    h.breakdown ? " (breakdown or non-finite data)" : "");
    return DG_OK;
}

// FP64 CG preconditioned by the fast-diagonalisation inverse of -Lap_h.
// The first iteration is queued with the setup (an exact preconditioner
// almost always needs one; if r_0 already met the tolerance its kernels
// exit at once), then the host reads the device scalars after every
// iteration: one round trip per iteration.
int cg_pcg(const dg_grid* g, const double* omega, double* x, const double* pa,
           double ca, const double* pb, double cb, const dg_cg_opts& o, bool fp32,
           dg_cg_stats* st, dg_workspace* ws, hipStream_t s) {
    int rc = pcg_queue(g, omega, pa, ca, pb, cb, o, fp32, 1, ws->d, ws, s);
    if (rc != DG_OK) return rc;
    rc = read_scalars(ws, ws->d.sc, &ws->host[2], s);
    if (rc != DG_OK) return rc;
    CgScalars h = ws->host[2];
    while (!h.done) {
        rc = pcg_iteration(g, fp32, ws->d, ws, s);
        if (rc != DG_OK) return rc;
        rc = read_scalars(ws, ws->d.sc, &ws->host[2], s);
        if (rc != DG_OK) return rc;
        h = ws->host[2];
    }
    hipError_t e = launch_cg_finish<double>(g->geom, g->k64, ws->x, ws->p0, ws->p1, x, g->area,
                                            ws->d, s);
    if (e != hipSuccess) return hip_fail(e, "cg finish launch");
    HIP_TRY(hipStreamSynchronize(s));
    return pcg_result(h, st);
}

int cg_dispatch(const dg_grid* g, const double* omega, double* x, const double* pa,
                double ca, const double* pb, double cb, const dg_cg_opts* opts,
                dg_cg_stats* st, dg_workspace* ws, hipStream_t s) {
    dg_cg_opts o;
    if (opts) o = *opts;
    else { o.rtol = 1e-12; o.max_iter = 100000; o.precision = DG_PREC_FP64;
           o.precond = DG_PRECOND_NONE; o.check_every = 0; }
    if (!(o.rtol > 0) || o.max_iter < 0)
        return fail(DG_E_INVAL, "rtol must be > 0 and max_iter >= 0");
    if (o.precond != DG_PRECOND_NONE && o.precond != DG_PRECOND_FD)
        return fail(DG_E_INVAL, "unknown preconditioner %d", o.precond);
    if ((g->geom.bcx || g->geom.bcy) && o.precond == DG_PRECOND_NONE &&
        o.precision != DG_PREC_FP64)
        return periodic_only("the mixed-precision solve without a preconditioner");
    if (o.precond == DG_PRECOND_FD) {
        if (o.precision != DG_PREC_FP64 && o.precision != DG_PREC_MIXED)
            return fail(DG_E_INVAL, "unknown precision %d", o.precision);
        if (!ws->fd)
            return fail(DG_E_WORKSPACE, "preconditioning needs a DG_WS_FD workspace");
        return cg_pcg(g, omega, x, pa, ca, pb, cb, o, o.precision == DG_PREC_MIXED, st, ws, s);
    }
    if (o.precision == DG_PREC_MIXED) {
        if (prec_of(ws->mode) != DG_PREC_MIXED)
            return fail(DG_E_WORKSPACE, "mixed precision needs a DG_PREC_MIXED workspace");
        return cg_mixed(g, omega, x, pa, ca, pb, cb, o, st, ws, s);
    }
    if (o.precision != DG_PREC_FP64) return fail(DG_E_INVAL, "unknown precision %d", o.precision);
    return cg_fp64(g, omega, x, pa, ca, pb, cb, o, st, ws, s);
}

}  // namespace

namespace dgk {
int state_create(const dg_grid* g, double t0, int nbuf, dg_state** out) {
    if (!g || !out) return fail(DG_E_INVAL, "NULL argument");
    *out = nullptr;
    if (nbuf != 3 && nbuf != 5) return fail(DG_E_INVAL, "a state holds 3 or 5 buffers");
    dg_state* st = new (std::nothrow) dg_state;
    if (!st) return fail(DG_E_NOMEM, "host allocation failed");
    std::memset(st, 0, sizeof *st);
    st->n = g->n; st->nx = g->nx; st->ny = g->ny; st->elems = g->elems;
    st->nbuf = nbuf;
    st->ia = st->ib = -1;
    st->resv[0] = st->resv[1] = -1;
    st->t = t0;
    for (int i = 0; i < nbuf; ++i) {
        if (hipMalloc((void**)&st->buf[i], g->elems * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            dg_state_destroy(st);
            return fail(DG_E_NOMEM, "state allocation failed");
        }
    }
    *out = st;
    return DG_OK;
}

int form_coeffs(int form, double* c0, double* c1, double* c2, double* scale) {
    *c0 = *c1 = *c2 = 0.0;
    *scale = 1.0;
    switch (form) {
        case DG_FORM_ARAKAWA: *c0 = *c1 = *c2 = 1.0; *scale = 1.0 / 3.0; break;
        case DG_FORM_PP: *c0 = 1.0; break;
        case DG_FORM_PX: *c1 = 1.0; break;
        case DG_FORM_XP: *c2 = 1.0; break;
        default: return fail(DG_E_INVAL, "unknown bracket form %d", form);
    }
    return DG_OK;
}

int periodic_only(const char* what) {
    return fail(DG_E_UNSUPPORTED, "%s is implemented for periodic grids only "
                "(Dirichlet grids support the bracket, the Laplacian, the FP64 CG plain "
                "or preconditioned, the mixed-precision PCG and time stepping)", what);
}

int solve_poisson(const dg_grid* g, const double* omega, double* x, const double* pa,
                  double ca, const double* pb, double cb, const dg_cg_opts* opts,
                  dg_cg_stats* st, dg_workspace* ws, hipStream_t s) {
    return cg_dispatch(g, omega, x, pa, ca, pb, cb, opts, st, ws, s);
}
}  // namespace dgk

extern "C" {

const char* dg_last_error(void) { return g_err.c_str(); }

int dg_grid_create(int n, int nx, int ny, double x0, double x1, double y0,
                   double y1, int bc_x, int bc_y, dg_grid** out) {
    if (!out) return fail(DG_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > kMaxN) return fail(DG_E_INVAL, "n = %d outside [1, 5]", n);
    if (nx < 1 || ny < 1) return fail(DG_E_INVAL, "nx, ny must be >= 1");
    if ((long)nx * ny > (1L << 28)) return fail(DG_E_INVAL, "grid too large");
    if (!std::isfinite(x0) || !std::isfinite(x1) || !std::isfinite(y0) ||
        !std::isfinite(y1) || !(x1 > x0) || !(y1 > y0))
        return fail(DG_E_INVAL, "domain bounds must be finite with x0 < x1, y0 < y1");
    if ((bc_x != DG_BC_PERIODIC && bc_x != DG_BC_DIRICHLET) ||
        (bc_y != DG_BC_PERIODIC && bc_y != DG_BC_DIRICHLET))
        return fail(DG_E_INVAL, "unknown boundary condition");
    dg_grid* g = new (std::nothrow) dg_grid;
    if (!g) return fail(DG_E_NOMEM, "host allocation failed");
    g->n = n; g->nx = nx; g->ny = ny;
    g->x0 = x0; g->x1 = x1; g->y0 = y0; g->y1 = y1;
    g->hx = (x1 - x0) / nx;
    g->hy = (y1 - y0) / ny;
    g->area = (x1 - x0) * (y1 - y0);
    if (!build_tables(n, &g->t)) { delete g; return fail(DG_E_INVAL, "table build failed"); }
    g->geom = Geom{n, nx, ny, kCellWavesDefault, kRowWavesDefault,
                   bc_x == DG_BC_DIRICHLET ? 1 : 0, bc_y == DG_BC_DIRICHLET ? 1 : 0};
    fill_const(*g, g->k64);
    g->elems = (size_t)nx * ny * n * n;
    *out = g;
    return DG_OK;
}

void dg_grid_destroy(dg_grid* g) { delete g; }

size_t dg_field_elems(const dg_grid* g) { return g ? g->elems : 0; }

int dg_grid_tables(const dg_grid* g, double* out, int len) {
    if (!g || !out) return fail(DG_E_INVAL, "NULL argument");
    const int n = g->n;
    const int need = 2 * n + (n * n + 4 * n) + 2 * (2 * n * n + 6 * n);
    if (len < need) return fail(DG_E_INVAL, "need %d doubles", need);
    int o = 0;
    auto put = [&](const double* a, int m) { for (int i = 0; i < m; ++i) out[o++] = a[i]; };
    put(g->t.xi, n); put(g->t.w, n);
    put(g->t.C0, n * n); put(g->t.cR, n); put(g->t.sR, n); put(g->t.cL, n); put(g->t.sL, n);
    AxisLdg ax, ay;
    ldg_axis(g->t, g->hx, g->geom.bcx == 0, &ax);
    ldg_axis(g->t, g->hy, g->geom.bcy == 0, &ay);
    for (const AxisLdg* a : {&ax, &ay}) {
        put(a->L0, n * n); put(a->eR, n); put(g->t.lR, n); put(g->t.eL, n); put(a->lL, n);
        put(a->L0B, n * n); put(a->eRB, n); put(a->lLB, n);
    }
    return o;
}

int dg_workspace_bytes(const dg_grid* g, int mode, size_t* bytes) {
    if (!g || !bytes) return fail(DG_E_INVAL, "NULL argument");
    if (!valid_mode(mode)) return fail(DG_E_INVAL, "bad mode %d", mode);
    *bytes = ws_bytes(g, mode);
    return DG_OK;
}

void dg_workspace_destroy(dg_workspace* ws) {
    if (!ws) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ws->device);
    void* bufs[] = {ws->x, ws->r, ws->p0, ws->p1, ws->s1, ws->s2, ws->r32,
                    ws->q0, ws->q1, ws->z, ws->wbak, ws->sc3, ws->d.sc, ws->d.counters,
                    ws->d.partials, ws->d.out3};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    fd_destroy(ws->fd);
    if (ws->host) (void)hipHostFree(ws->host);
    for (auto& e : ws->ev) if (e) (void)hipEventDestroy(e);
    for (auto& e : ws->tev) if (e) (void)hipEventDestroy(e);
    for (auto& row : ws->pev)
        for (auto& e : row) if (e) (void)hipEventDestroy(e);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete ws;
}

int dg_workspace_create(const dg_grid* g, int mode, dg_workspace** out) {
    if (!g || !out) return fail(DG_E_INVAL, "NULL argument");
    *out = nullptr;
    if (!valid_mode(mode)) return fail(DG_E_INVAL, "bad mode %d", mode);
    if (mode & DG_WS_FD) {
        const int rc = fd_supported(g);
        if (rc != DG_OK) return rc;
    }
    dg_workspace* ws = new (std::nothrow) dg_workspace;
    if (!ws) return fail(DG_E_NOMEM, "host allocation failed");
    std::memset(ws, 0, sizeof *ws);
    ws->n = g->n; ws->nx = g->nx; ws->ny = g->ny; ws->mode = mode;
    ws->elems = g->elems;
    hipError_t e = hipGetDevice(&ws->device);
    if (e != hipSuccess) { delete ws; return hip_fail(e, "hipGetDevice"); }
    const size_t F = g->elems * sizeof(double);
    int blocks = stencil_blocks(g->geom);
    if (blocks < pointwise_block_cap()) blocks = pointwise_block_cap();
    ws->d.max_blocks = blocks;
    auto alloc = [&](void** p, size_t b) -> bool {
        return hipMalloc(p, b) == hipSuccess;
    };
    const size_t L = l64_elems(g->geom);
    bool ok = alloc((void**)&ws->x, L * sizeof(double)) &&
              alloc((void**)&ws->r, L * sizeof(double)) &&
              alloc((void**)&ws->p0, L * sizeof(double)) &&
              alloc((void**)&ws->p1, L * sizeof(double)) &&
              alloc((void**)&ws->s1, F) && alloc((void**)&ws->s2, F) &&
              alloc((void**)&ws->d.sc, sizeof(CgScalars)) &&
              alloc((void**)&ws->d.counters, kCntBytes) &&
              alloc((void**)&ws->d.partials, (size_t)blocks * 4 * sizeof(double)) &&
              alloc((void**)&ws->d.out3, 4 * sizeof(double));
    if (ok && prec_of(mode) == DG_PREC_MIXED) {
        const size_t f32 = L * sizeof(float);
        ok = alloc((void**)&ws->r32, f32) && alloc((void**)&ws->q0, f32) &&
             alloc((void**)&ws->q1, f32);
    }
    if (ok && (mode & DG_WS_FD))
        ok = alloc((void**)&ws->z, L * sizeof(double)) && alloc((void**)&ws->wbak, F) &&
             alloc((void**)&ws->sc3, 3 * sizeof(CgScalars));
    if (ok) ok = hipHostMalloc((void**)&ws->host, 4 * sizeof(CgScalars)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        dg_workspace_destroy(ws);
        return fail(DG_E_NOMEM, "workspace allocation of %zu bytes failed", ws_bytes(g, mode));
    }
    for (auto& ev : ws->ev) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            dg_workspace_destroy(ws);
            return fail(DG_E_HIP, "event creation failed");
        }
    }
    for (auto& ev : ws->tev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            dg_workspace_destroy(ws);
            return fail(DG_E_HIP, "event creation failed");
        }
    }
    for (auto& row : ws->pev)
        for (auto& ev : row)
            if (hipEventCreate(&ev) != hipSuccess) {
                dg_workspace_destroy(ws);
                return fail(DG_E_HIP, "event creation failed");
            }
    ws->pev_iter[0] = ws->pev_iter[1] = -1;
    // counters must start at zero (each reduction resets its own)
    e = hipMemset(ws->d.counters, 0, kCntBytes);
    if (e == hipSuccess) e = hipMemset(ws->d.sc, 0, sizeof(CgScalars));
    if (e == hipSuccess && ws->sc3) e = hipMemset(ws->sc3, 0, 3 * sizeof(CgScalars));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { dg_workspace_destroy(ws); return hip_fail(e, "workspace init"); }
    if (mode & DG_WS_FD) {
        const int rc = fd_create(g, (mode & DG_WS_FD_PRODUCTS) != 0, &ws->fd);
        if (rc != DG_OK) { dg_workspace_destroy(ws); return rc; }
    }
    ws->bytes = ws_bytes(g, mode) + fd_extra_bytes(ws->fd);
    *out = ws;
    return DG_OK;
}

int dg_workspace_held_bytes(const dg_workspace* ws, size_t* bytes) {
    if (!ws || !bytes) return fail(DG_E_INVAL, "NULL argument");
    *bytes = ws->bytes;
    return DG_OK;
}

int dg_profile_enable(dg_workspace* ws, int on) {
    if (!ws) return fail(DG_E_INVAL, "workspace is NULL");
    ws->prof_on = on ? 1 : 0;
    return DG_OK;
}

int dg_profile_read(dg_workspace* ws, double* out4) {
    if (!ws || !out4) return fail(DG_E_INVAL, "NULL argument");
    out4[0] = ws->prof_ms[0];
    out4[1] = ws->prof_n[0];
    out4[2] = ws->prof_ms[1];
    out4[3] = ws->prof_n[1];
    ws->prof_ms[0] = ws->prof_ms[1] = ws->prof_n[0] = ws->prof_n[1] = 0.0;
    return DG_OK;
}

int dg_poisson_bracket(const dg_grid* g, const double* f, const double* gg,
                       double* out, void* stream) {
    return dg_bracket_form(g, f, gg, out, DG_FORM_ARAKAWA, stream);
}

int dg_bracket_form(const dg_grid* g, const double* f, const double* gg,
                    double* out, int form, void* stream) {
    if (!g || !f || !gg || !out) return fail(DG_E_INVAL, "NULL argument");
    const size_t B = g->elems * sizeof(double);
    if (ranges_overlap(out, f, B) || ranges_overlap(out, gg, B))
        return fail(DG_E_ALIAS, "out aliases an input");
    RhsParams p{};
    const int rc = form_coeffs(form, &p.c0, &p.c1, &p.c2, &p.scale);
    if (rc != DG_OK) return rc;
    hipError_t e = launch_rhs(g->geom, g->k64, f, gg, nullptr, out, p, false,
                              as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "bracket launch");
    return DG_OK;
}

int dg_laplace_apply(const dg_grid* g, const double* f, double* out, void* stream) {
    if (!g || !f || !out) return fail(DG_E_INVAL, "NULL argument");
    if (ranges_overlap(out, f, g->elems * sizeof(double)))
        return fail(DG_E_ALIAS, "out aliases f");
    hipError_t e = launch_laplace(g->geom, g->k64, f, out, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "laplace launch");
    return DG_OK;
}

int dg_grid_fd_basis(const dg_grid* g, int axis, double* V, double* lam, int* zero) {
    if (!g || !V || !lam || !zero) return fail(DG_E_INVAL, "NULL argument");
    if (axis != 0 && axis != 1) return fail(DG_E_INVAL, "axis must be 0 (x) or 1 (y)");
    if (axis == 0 ? g->geom.bcx : g->geom.bcy)
        return periodic_only("the Bloch eigenbasis");
    FdAxis a;
    double err = 0.0;
    // the basis the preconditioner's transforms use on this grid: phases at
    // the cell centres for the matrix products (up to 512 cells per axis, or
    // an odd count), at the cell edges for the FFTs
    const bool shifted = !fd_uses_fft(g->nx, g->ny);
    const bool ok = axis == 0 ? fd_axis_basis(g->t, g->nx, g->hx, &a, &err, shifted)
                              : fd_axis_basis(g->t, g->ny, g->hy, &a, &err, shifted);
    if (!ok || err > 1e-10) return fail(DG_E_INVAL, "eigenbasis construction failed (defect %.3e)", err);
    std::memcpy(V, a.V.data(), a.V.size() * sizeof(double));
    std::memcpy(lam, a.lam.data(), a.lam.size() * sizeof(double));
    *zero = a.zero;
    return DG_OK;
}

int dg_grid_axis_operator(const dg_grid* g, int axis, double* L) {
    if (!g || !L) return fail(DG_E_INVAL, "NULL argument");
    if (axis != 0 && axis != 1) return fail(DG_E_INVAL, "axis must be 0 (x) or 1 (y)");
    std::vector<double> M;
    if (axis == 0) fd_axis_operator(g->t, g->nx, g->hx, !g->geom.bcx, &M);
    else fd_axis_operator(g->t, g->ny, g->hy, !g->geom.bcy, &M);
    std::memcpy(L, M.data(), M.size() * sizeof(double));
    return DG_OK;
}

int dg_precond_apply(const dg_grid* g, const double* r, double* z, dg_workspace* ws,
                     void* stream) {
    if (!g || !r || !z) return fail(DG_E_INVAL, "NULL argument");
    int rc = check_ws(g, ws);
    if (rc != DG_OK) return rc;
    if (!ws->fd) return fail(DG_E_WORKSPACE, "the workspace has no DG_WS_FD preconditioner");
    if (ranges_overlap(z, r, g->elems * sizeof(double)))
        return fail(DG_E_ALIAS, "z aliases r");
    const hipStream_t s = as_stream(stream);
    const int layout = fd_layout(ws->fd);
    const bool dense = layout == kFdDense;
    const int Kx = (g->nx + 1) / 2;
    hipError_t e = layout == kFdFolded
                       ? launch_to_planes_fold<double>(g->geom, r, false, Kx, ws->fd->img0, s)
                       : launch_to_image<double>(g->geom, g->k64, r, false, dense, ws->fd->img0, s);
    if (e != hipSuccess) return hip_fail(e, "image conversion launch");
    rc = fd_apply_image(ws->fd, false, s);
    if (rc != DG_OK) return rc;
    e = layout == kFdFolded
            ? launch_from_planes_fold<double>(g->geom, g->k64, ws->fd->img0, Kx, z, nullptr,
                                              nullptr, s)
            : launch_from_image<double>(g->geom, g->k64, ws->fd->img0, dense, z, s);
    if (e != hipSuccess) return hip_fail(e, "image conversion launch");
    return DG_OK;
}

int dg_cg_solve_poisson(const dg_grid* g, const double* omega, double* psi,
                        const dg_cg_opts* opts, dg_cg_stats* st, dg_workspace* ws,
                        void* stream) {
    if (!g || !omega || !psi) return fail(DG_E_INVAL, "NULL argument");
    int rc = check_ws(g, ws);
    if (rc != DG_OK) return rc;
    const size_t B = g->elems * sizeof(double);
    if (ranges_overlap(psi, omega, B)) return fail(DG_E_ALIAS, "psi aliases omega");
    // psi is read (the guess) only by the setup kernels and written only by
    // the final conversion out of the workspace vectors
    return cg_dispatch(g, omega, psi, psi, 1.0, nullptr, 0.0, opts, st, ws,
                       as_stream(stream));
}

int dg_state_create(const dg_grid* g, double t0, dg_state** out) {
    return state_create(g, t0, 5, out);
}

void dg_state_destroy(dg_state* st) {
    if (!st) return;
    for (auto b : st->buf) if (b) (void)hipFree(b);
    delete st;
}

const double* dg_state_psi(const dg_state* st) {
    return (st && st->ia >= 0) ? st->buf[st->ia] : nullptr;
}

double dg_state_time(const dg_state* st) { return st ? st->t : 0.0; }

int dg_state_copy_psi(const dg_state* st, double* out, void* stream) {
    if (!st || !out) return fail(DG_E_INVAL, "NULL argument");
    if (st->ia < 0) return fail(DG_E_INVAL, "no Poisson solve yet");
    HIP_TRY(hipMemcpyAsync(out, st->buf[st->ia], st->elems * sizeof(double),
                           hipMemcpyDeviceToDevice, as_stream(stream)));
    return DG_OK;
}

namespace {

constexpr int kRedo = 1;   // a queued step must be taken again synchronously

// One SSP-RK3 step with the three preconditioned stage solves queued ahead
// of any convergence check: each stage runs the setup, one PCG iteration
// (the exact preconditioner's usual count), the finish and the fused RHS
// kernel, on its own device scalars; the host reads the three stages'
// scalars once, at the end.  omega is saved first and the psi history the
// step starts from stays in the state's reserved buffers, so when a stage
// has not converged (the first step from a zero guess, say) both are
// restored and kRedo is returned: the caller takes the step again with the
// solves polled after every iteration.
int rk_step_queued(const dg_grid* g, double* omega, dg_state* st, const dg_step_opts* opts,
                   const double (&fc)[4], dg_step_stats* stats, dg_workspace* ws,
                   hipStream_t s) {
    const double dt = opts->dt, t = st->t;
    const double ts[3] = {t, t + dt, t + 0.5 * dt};
    const double ra[3] = {0.0, 0.75, 1.0 / 3.0};
    const double rb[3] = {1.0, 0.25, 2.0 / 3.0};
    double* win[3] = {omega, ws->s1, ws->s2};
    double* wout[3] = {ws->s1, ws->s2, omega};
    const dg_state saved = *st;
    st->resv[0] = st->ia;
    st->resv[1] = st->ib;
    const bool timing = opts->record_times != 0;
    HIP_TRY(hipMemcpyAsync(ws->wbak, omega, g->elems * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    if (timing) HIP_TRY(hipEventRecord(ws->tev[0], s));
    for (int k = 0; k < 3; ++k) {
        const double* pa;
        const double* pb;
        double ca, cb;
        double* x;
        int fr;
        state_guess(st, ts[k], &pa, &ca, &pb, &cb, &x, &fr);
        DevScratch d = ws->d;
        d.sc = ws->sc3 + k;
        int rc = pcg_queue(g, win[k], pa, ca, pb, cb, opts->cg, false, 1, d, ws, s);
        if (rc != DG_OK) return rc;
        hipError_t e = launch_cg_finish<double>(g->geom, g->k64, ws->x, ws->p0, ws->p1, x,
                                                g->area, d, s);
        if (e != hipSuccess) return hip_fail(e, "cg finish launch");
        state_push(st, fr, ts[k]);
        RhsParams p{fc[0], fc[1], fc[2], fc[3], opts->D, dt, ra[k], rb[k], 0};
        e = launch_rhs(g->geom, g->k64, x, win[k], k ? omega : nullptr, wout[k], p, true, s);
        if (e != hipSuccess) return hip_fail(e, "rhs launch");
        if (timing) HIP_TRY(hipEventRecord(ws->tev[k + 1], s));
    }
    HIP_TRY(hipMemcpyAsync(ws->host, ws->sc3, 3 * sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool ok = true;
    for (int k = 0; k < 3; ++k) ok = ok && ws->host[k].converged;
    st->resv[0] = st->resv[1] = -1;
    if (!ok) {
        HIP_TRY(hipMemcpyAsync(omega, ws->wbak, g->elems * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
        *st = saved;
        return kRedo;
    }
    st->t = t + dt;
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        for (int k = 0; k < 3; ++k) stats->cg_iters[k] = ws->host[k].iter;
        stats->converged = 1;
        if (timing)
            for (int k = 0; k < 3; ++k)
                HIP_TRY(hipEventElapsedTime(&stats->stage_ms[k], ws->tev[k], ws->tev[k + 1]));
    }
    return DG_OK;
}

}  // namespace

int dg_rk_step(const dg_grid* g, double* omega, dg_state* st,
               const dg_step_opts* opts, dg_step_stats* stats, dg_workspace* ws,
               void* stream) {
    if (!g || !omega || !st || !opts) return fail(DG_E_INVAL, "NULL argument");
    int rc = check_ws(g, ws);
    if (rc != DG_OK) return rc;
    if (st->n != g->n || st->nx != g->nx || st->ny != g->ny)
        return fail(DG_E_INVAL, "state was made for another grid");
    if (!std::isfinite(opts->dt) || !std::isfinite(opts->D))
        return fail(DG_E_INVAL, "dt and D must be finite");
    double fc[4];
    rc = form_coeffs(opts->form, &fc[0], &fc[1], &fc[2], &fc[3]);
    if (rc != DG_OK) return rc;
    hipStream_t s = as_stream(stream);
    // FP64 preconditioned solves: queue the whole step, verify once
    if (opts->cg.precond == DG_PRECOND_FD && opts->cg.precision == DG_PREC_FP64 && ws->fd &&
        ws->sc3 && st->nbuf == 5 && opts->cg.rtol > 0 && opts->cg.max_iter >= 1) {
        rc = rk_step_queued(g, omega, st, opts, fc, stats, ws, s);
        if (rc != kRedo) return rc;
    }
    const double dt = opts->dt, t = st->t;
    const double ts[3] = {t, t + dt, t + 0.5 * dt};
    const double ra[3] = {0.0, 0.75, 1.0 / 3.0};
    const double rb[3] = {1.0, 0.25, 2.0 / 3.0};
    double* win[3] = {omega, ws->s1, ws->s2};
    double* wout[3] = {ws->s1, ws->s2, omega};
    const bool timing = opts->record_times != 0;
    int result = DG_OK;
    if (stats) std::memset(stats, 0, sizeof *stats);
    bool all_conv = true, stalled = false;
    if (timing) HIP_TRY(hipEventRecord(ws->tev[0], s));
    for (int k = 0; k < 3; ++k) {
        // guess: linear extrapolation in time through the two newest solves
        const double* pa;
        const double* pb;
        double ca, cb;
        double* x;
        int fr;
        state_guess(st, ts[k], &pa, &ca, &pb, &cb, &x, &fr);
        dg_cg_stats cs{};
        rc = cg_dispatch(g, win[k], x, pa, ca, pb, cb, &opts->cg, &cs, ws, s);
        if (rc == DG_E_NOCONV) { result = DG_E_NOCONV; all_conv = false; }
        else if (rc != DG_OK) return rc;
        if (cs.converged == 2) stalled = true;
        state_push(st, fr, ts[k]);
        RhsParams p{fc[0], fc[1], fc[2], fc[3], opts->D, dt, ra[k], rb[k], 0};
        hipError_t e = launch_rhs(g->geom, g->k64, x, win[k], k ? omega : nullptr,
                                  wout[k], p, true, s);
        if (e != hipSuccess) return hip_fail(e, "rhs launch");
        if (timing) HIP_TRY(hipEventRecord(ws->tev[k + 1], s));
        if (stats) stats->cg_iters[k] = cs.iters;
    }
    st->t = t + dt;
    if (timing) {
        HIP_TRY(hipEventSynchronize(ws->tev[3]));
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ws->tev[k], ws->tev[k + 1]));
            if (stats) stats->stage_ms[k] = ms;
        }
    }
    if (stats) stats->converged = all_conv ? (stalled ? 2 : 1) : 0;
    if (result != DG_OK) return fail(result, "a stage solve did not converge");
    return DG_OK;
}

int dg_invariants_dev(const dg_grid* g, const double* omega, const double* psi,
                      double* out_dev3, dg_workspace* ws, void* stream) {
    if (!g || !omega || !psi || !out_dev3) return fail(DG_E_INVAL, "NULL argument");
    int rc = check_ws(g, ws);
    if (rc != DG_OK) return rc;
    hipError_t e = launch_invariants(g->geom, g->k64, omega, psi, out_dev3, ws->d,
                                     as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "invariants launch");
    return DG_OK;
}

int dg_invariants(const dg_grid* g, const double* omega, const double* psi,
                  double* out_host3, dg_workspace* ws, void* stream) {
    if (!out_host3) return fail(DG_E_INVAL, "NULL argument");
    int rc = dg_invariants_dev(g, omega, psi, ws ? ws->d.out3 : nullptr, ws, stream);
    if (rc != DG_OK) return rc;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(out_host3, ws->d.out3, 3 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return DG_OK;
}

}  // extern "C"

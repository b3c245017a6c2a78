// Pointwise kernels of libdgark: CG setup means, the end-of-solve update
// (lane-interleaved CG vector -> canonical psi), mean removal, invariants,
// the mixed-precision correction and the extrapolated guess.  Grid-stride
// loops over node rows (canonical layout) or cells (layout conversion).
#include "dg_device.h"
#include "dg_launch.h"

namespace dgk {

// W-weighted row sum of one canonical node row (Gauss weights, Sec. 4.1
// eq. def_norm)
template <int N, class T>
__device__ __forceinline__ double wrow(const OpConst<T>& k, int j, const double (&v)[N]) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) s += (double)k.w[i] * v[i];
    return s * (double)k.w[j] * k.wq;
}

// Means of omega and of the guess ca psi_a + cb psi_b, and <omega, omega>_W;
// the last block also initialises every CG scalar for the coming solve.
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_cg_mean(
    long rows, OpConst<double> k, const double* __restrict__ omega,
    const double* __restrict__ pa, const double* __restrict__ pb, double ca,
    double cb, double area, double tol2, int max_iter, CgScalars* sc,
    unsigned* counter, double* partials) {
    double part[3] = {0.0, 0.0, 0.0};
    for (long row = blockIdx.x * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)gridDim.x * kPwThreads) {
        const int j = (int)(row % N);
        double w[N], gs[N], w2[N];
        load_vec(omega, row * N, w);
#pragma unroll
        for (int i = 0; i < N; ++i) gs[i] = 0.0;
        if (ca != 0.0) {
            double a[N];
            load_vec(pa, row * N, a);
#pragma unroll
            for (int i = 0; i < N; ++i) gs[i] += ca * a[i];
        }
        if (cb != 0.0) {
            double b[N];
            load_vec(pb, row * N, b);
#pragma unroll
            for (int i = 0; i < N; ++i) gs[i] += cb * b[i];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) w2[i] = w[i] * w[i];
        part[0] += wrow<N>(k, j, w);
        part[1] += wrow<N>(k, j, gs);
        part[2] += wrow<N>(k, j, w2);
    }
    double tot[3];
    if (reduce_last<3, kPwThreads>(part, partials, counter, gridDim.x, tot) &&
        threadIdx.x == 0) {
        sc->mean_omega = tot[0] / area;
        sc->mean_guess = tot[1] / area;
        sc->ww = tot[2];
        sc->zero_tol2 = 1e-28;   // (1e-14)^2: b below the mean-removal rounding
        sc->tol2 = tol2;
        sc->max_iter = max_iter;
        sc->ca = ca;
        sc->cb = cb;
        sc->alpha = 0.0;
        sc->beta = 0.0;
        sc->done = 0;
        sc->converged = 0;
        sc->zero = 0;
        sc->first = 1;
        sc->pending = 0;
        sc->iter = 0;
        sc->breakdown = 0;
    }
}

// End of a solve: psi = x + alpha p_last (pending update; p_last = the
// buffer written by the last direction update) or psi = 0 when b = 0,
// converted from the lane-interleaved layout to canonical; partial W-mean.
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_cg_finish(
    Geom g, OpConst<double> k, const double* __restrict__ x,
    const double* __restrict__ p0, const double* __restrict__ p1,
    double* __restrict__ psi, double area, CgScalars* sc, unsigned* counter,
    double* partials) {
    const int pending = sc->pending, zero = sc->zero;
    const double alpha = sc->alpha;
    const double* pl = (sc->iter & 1) ? p1 : p0;
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    double part[1] = {0.0};
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const long l64 = ((long)cy * G + (cx >> 6)) * (N * N * 64) + (cx & 63);
        double v[N * N];
#pragma unroll
        for (int e = 0; e < N * N; ++e) {
            double a = 0.0;
            if (!zero) {
                a = x[l64 + 64 * e];
                if (pending) a += alpha * pl[l64 + 64 * e];
            }
            v[e] = a;
        }
        store_vec(psi, cell * (N * N), v);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double r[N];
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] = v[j * N + i];
            part[0] += wrow<N>(k, j, r);
        }
    }
    double tot[1];
    if (reduce_last<1, kPwThreads>(part, partials, counter, gridDim.x, tot) &&
        threadIdx.x == 0) {
        sc->mean_x = tot[0] / area;
        sc->pending = 0;
    }
}

// W-mean of a canonical field into sc->mean_x
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_mean_canon(
    long rows, OpConst<double> k, const double* __restrict__ f, double area,
    CgScalars* sc, unsigned* counter, double* partials) {
    double part[1] = {0.0};
    for (long row = blockIdx.x * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)gridDim.x * kPwThreads) {
        double v[N];
        load_vec(f, row * N, v);
        part[0] += wrow<N>(k, (int)(row % N), v);
    }
    double tot[1];
    if (reduce_last<1, kPwThreads>(part, partials, counter, gridDim.x, tot) &&
        threadIdx.x == 0)
        sc->mean_x = tot[0] / area;
}

__global__ __launch_bounds__(kPwThreads) void k_sub_mean(long elems,
                                                         double* __restrict__ x,
                                                         const CgScalars* sc) {
    const double m = sc->mean_x;
    for (long e = blockIdx.x * (long)kPwThreads + threadIdx.x; e < elems;
         e += (long)gridDim.x * kPwThreads)
        x[e] -= m;
}

// (V, E, Omega) with Gauss weights (Sec. 2 eq. quantities).
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_invariants(
    long rows, OpConst<double> k, const double* __restrict__ omega,
    const double* __restrict__ psi, double* out3, unsigned* counter,
    double* partials) {
    double part[3] = {0.0, 0.0, 0.0};
    for (long row = blockIdx.x * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)gridDim.x * kPwThreads) {
        const int j = (int)(row % N);
        double w[N], p[N], pw[N], ww[N];
        load_vec(omega, row * N, w);
        load_vec(psi, row * N, p);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            pw[i] = p[i] * w[i];
            ww[i] = w[i] * w[i];
        }
        part[0] += wrow<N>(k, j, w);
        part[1] += wrow<N>(k, j, pw);
        part[2] += wrow<N>(k, j, ww);
    }
    double tot[3];
    if (reduce_last<3, kPwThreads>(part, partials, counter, gridDim.x, tot) &&
        threadIdx.x == 0) {
        out3[0] = tot[0];
        out3[1] = 0.5 * tot[1];
        out3[2] = 0.5 * tot[2];
    }
}

// psi (canonical, FP64) += e + alpha p_last (lane-interleaved, FP32): the
// FP64 accumulation of one inner FP32 solve.
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_mixed_update(
    Geom g, double* __restrict__ psi, const float* __restrict__ e32,
    const float* __restrict__ p0, const float* __restrict__ p1,
    const CgScalars* inner) {
    const int pending = inner->pending;
    const float alpha = (float)inner->alpha;
    const float* pl = (inner->iter & 1) ? p1 : p0;
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const long l64 = ((long)cy * G + (cx >> 6)) * (N * N * 64) + (cx & 63);
        double v[N * N];
        load_vec(psi, cell * (N * N), v);
#pragma unroll
        for (int e = 0; e < N * N; ++e) {
            float c = e32[l64 + 64 * e];
            if (pending) c += alpha * pl[l64 + 64 * e];
            v[e] += (double)c;
        }
        store_vec(psi, cell * (N * N), v);
    }
}

// x = ca pa + cb pb (pointwise; in place allowed)
__global__ __launch_bounds__(kPwThreads) void k_guess(long elems,
                                                      double* __restrict__ x,
                                                      const double* pa,
                                                      const double* pb,
                                                      double ca, double cb) {
    for (long e = blockIdx.x * (long)kPwThreads + threadIdx.x; e < elems;
         e += (long)gridDim.x * kPwThreads) {
        double v = 0.0;
        if (ca != 0.0) v += ca * pa[e];
        if (cb != 0.0) v += cb * pb[e];
        x[e] = v;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int pointwise_block_cap() { return 1024; }

int stencil_blocks(const Geom& g) {
    const int a = row_blocks(g), b = cell_blocks(g);
    return a > b ? a : b;
}

hipError_t launch_cg_mean(const Geom& g, const OpConst<double>& k,
                          const double* omega, const double* pa,
                          const double* pb, double ca, double cb, double area,
                          double tol2, int max_iter, const DevScratch& d,
                          hipStream_t s) {
    const long rows = (long)g.nx * g.ny * g.n;
    const int nb = pw_blocks(rows, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_mean<NN>), dim3(nb),
                                          dim3(kPwThreads), 0, s, rows, k, omega,
                                          pa, pb, ca, cb, area, tol2, max_iter,
                                          d.sc, d.counters + kCntMean, d.partials));
    return hipGetLastError();
}

hipError_t launch_cg_finish(const Geom& g, const OpConst<double>& k,
                            const double* x, const double* p0, const double* p1,
                            double* psi, double area, const DevScratch& d,
                            hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_finish<NN>), dim3(nb),
                                          dim3(kPwThreads), 0, s, g, k, x, p0, p1,
                                          psi, area, d.sc, d.counters + kCntFinish,
                                          d.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long elems = cells * g.n * g.n;
    hipLaunchKernelGGL(k_sub_mean, dim3(pw_blocks(elems, pointwise_block_cap())),
                       dim3(kPwThreads), 0, s, elems, psi, d.sc);
    return hipGetLastError();
}

hipError_t launch_mean_sub(const Geom& g, const OpConst<double>& k, double* x,
                           double area, const DevScratch& d, hipStream_t s) {
    const long rows = (long)g.nx * g.ny * g.n;
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_mean_canon<NN>),
                                          dim3(pw_blocks(rows, pointwise_block_cap())),
                                          dim3(kPwThreads), 0, s, rows, k, x, area,
                                          d.sc, d.counters + kCntFinish, d.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long elems = rows * g.n;
    hipLaunchKernelGGL(k_sub_mean, dim3(pw_blocks(elems, pointwise_block_cap())),
                       dim3(kPwThreads), 0, s, elems, x, d.sc);
    return hipGetLastError();
}

hipError_t launch_invariants(const Geom& g, const OpConst<double>& k,
                             const double* omega, const double* psi,
                             double* out3, const DevScratch& d, hipStream_t s) {
    const long rows = (long)g.nx * g.ny * g.n;
    const int nb = pw_blocks(rows, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_invariants<NN>), dim3(nb),
                                          dim3(kPwThreads), 0, s, rows, k, omega,
                                          psi, out3, d.counters + kCntInv,
                                          d.partials));
    return hipGetLastError();
}

hipError_t launch_mixed_update(const Geom& g, double* psi, const float* e,
                               const float* p0, const float* p1,
                               const CgScalars* inner, hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_mixed_update<NN>), dim3(nb),
                                          dim3(kPwThreads), 0, s, g, psi, e, p0, p1,
                                          inner));
    return hipGetLastError();
}

hipError_t launch_guess(long elems, double* x, const double* pa,
                        const double* pb, double ca, double cb, hipStream_t s) {
    const int nb = pw_blocks(elems, pointwise_block_cap());
    hipLaunchKernelGGL(k_guess, dim3(nb), dim3(kPwThreads), 0, s, elems, x, pa,
                       pb, ca, cb);
    return hipGetLastError();
}

}  // namespace dgk

// Pointwise device code of libdgark: CG setup means, the end-of-solve update
// (lane-interleaved CG vector -> canonical psi), mean removal, invariants,
// the mixed-precision correction and the extrapolated guess.  Grid-stride
// loops over node rows (canonical layout) or cells (layout conversion).
#pragma once

#include "dg_device.h"

namespace dgk {

// W-weighted row sum of one canonical node row (Gauss weights, Sec. 4.1
// eq. def_norm)
template <int N, class T>
__device__ __forceinline__ double wrow(const OpConst<T>& k, int j, const double (&v)[N]) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) s = fmx((double)k.w[i], v[i], s);
    return s * (double)k.w[j] * k.wq;
}

// Mean of omega and <omega, omega>_W; the last block also initialises every
// CG scalar for the coming solve.  The guess ca psi_a + cb psi_b keeps its
// mean: Lap_h annihilates constants, so the initial residual does not see it,
// the directions never carry one, and the end of the solve removes the mean of
// the solution (pa, pb: read by the setup kernel only).  With a Dirichlet axis
// (dir != 0) -Lap_h is definite and nothing is subtracted: the mean the later
// kernels remove is stored as zero.
template <int N>
__device__ __forceinline__ void cg_mean_body(int b, int nb, long rows, const OpConst<double>& k, const double* __restrict__ omega,
    const double* __restrict__ pa, const double* __restrict__ pb, double ca,
    double cb, double area, double tol2, int max_iter, int dir, CgScalars* sc,
    unsigned* counter, double* partials) {
    (void)pa;
    (void)pb;
    double part[2] = {0.0, 0.0};
    for (long row = b * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)nb * kPwThreads) {
        const int j = (int)(row % N);
        double w[N], w2[N];
        load_vec(omega, row * N, w);
#pragma unroll
        for (int i = 0; i < N; ++i) w2[i] = w[i] * w[i];
        part[0] += wrow<N>(k, j, w);
        part[1] += wrow<N>(k, j, w2);
    }
    double tot[2];
    if (reduce_last<2, kPwThreads>(part, partials, counter, nb, b, tot) &&
        threadIdx.x == 0) {
        sc->mean_omega = dir ? 0.0 : tot[0] / area;
        sc->ww = tot[1];
        sc->zero_tol2 = 1e-28;   // (1e-14)^2: b below the mean-removal rounding
        sc->tol2 = tol2;
        sc->max_iter = max_iter;
        sc->ca = ca;
        sc->cb = cb;
        sc->alpha = 0.0;
        sc->alpha_prev = 0.0;
        sc->beta = 0.0;
        sc->done = 0;
        sc->converged = 0;
        sc->zero = 0;
        sc->first = 1;
        sc->pending = 0;
        sc->iter = 0;
        sc->breakdown = 0;
        sc->precond = 0;
        sc->rz = 0.0;
        sc->cr = 1.0;
    }
}

// End of a solve: psi = x plus the pending updates or psi = 0 when b = 0,
// converted from the lane-interleaved layout to canonical; partial W-mean.
// pending = 1: x + alpha p_last (p_last = the buffer written by the last
// direction update); 2: first alpha_prev times the other buffer (the
// direction before), then alpha p_last.
template <int N, class P>
__device__ __forceinline__ void cg_finish_body(int b, int nb, Geom g, const OpConst<double>& k, const double* __restrict__ x,
    const P* __restrict__ p0, const P* __restrict__ p1,
    double* __restrict__ psi, double area, CgScalars* sc, unsigned* counter,
    double* partials) {
    const int pending = sc->pending, zero = sc->zero;
    const double alpha = sc->alpha, alpha_prev = sc->alpha_prev;
    const P* pl = (sc->iter & 1) ? p1 : p0;
    const P* pb = (sc->iter & 1) ? p0 : p1;
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    double part[1] = {0.0};
    for (long cell = b * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)nb * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const long l64 = ((long)cy * G + (cx >> 6)) * (N * N * 64) + (cx & 63);
        double v[N * N];
#pragma unroll
        for (int e = 0; e < N * N; ++e) {
            double a = 0.0;
            if (!zero) {
                a = x[l64_at<N>(l64, e)];
                if (pending == 2) a = fmx(alpha_prev, (double)pb[l64_at<N>(l64, e)], a);
                if (pending) a = fmx(alpha, (double)pl[l64_at<N>(l64, e)], a);
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
    if (reduce_last<1, kPwThreads>(part, partials, counter, nb, b, tot) &&
        threadIdx.x == 0) {
        sc->mean_x = tot[0] / area;
        sc->pending = 0;
    }
}

// W-mean of a canonical field into sc->mean_x
template <int N>
__device__ __forceinline__ void mean_canon_body(int b, int nb, long rows, const OpConst<double>& k, const double* __restrict__ f, double area,
    CgScalars* sc, unsigned* counter, double* partials) {
    double part[1] = {0.0};
    for (long row = b * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)nb * kPwThreads) {
        double v[N];
        load_vec(f, row * N, v);
        part[0] += wrow<N>(k, (int)(row % N), v);
    }
    double tot[1];
    if (reduce_last<1, kPwThreads>(part, partials, counter, nb, b, tot) &&
        threadIdx.x == 0)
        sc->mean_x = tot[0] / area;
}

__device__ __forceinline__ void sub_mean_body(int b, int nb, long elems,
                                                         double* __restrict__ x,
                                                         const CgScalars* sc) {
    const double m = sc->mean_x;
    for (long e = b * (long)kPwThreads + threadIdx.x; e < elems;
         e += (long)nb * kPwThreads)
        x[e] -= m;
}

// (V, E, Omega) with Gauss weights (Sec. 2 eq. quantities).
template <int N>
__device__ __forceinline__ void invariants_body(int b, int nb, long rows, const OpConst<double>& k, const double* __restrict__ omega,
    const double* __restrict__ psi, double* out3, unsigned* counter,
    double* partials) {
    double part[3] = {0.0, 0.0, 0.0};
    for (long row = b * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)nb * kPwThreads) {
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
    if (reduce_last<3, kPwThreads>(part, partials, counter, nb, b, tot) &&
        threadIdx.x == 0) {
        out3[0] = tot[0];
        out3[1] = 0.5 * tot[1];
        out3[2] = 0.5 * tot[2];
    }
}

// x = ca pa + cb pb (pointwise; in place allowed)
__device__ __forceinline__ void guess_body(int b, int nb, long elems,
                                                      double* __restrict__ x,
                                                      const double* pa,
                                                      const double* pb,
                                                      double ca, double cb) {
    for (long e = b * (long)kPwThreads + threadIdx.x; e < elems;
         e += (long)nb * kPwThreads) {
        double v = 0.0;
        if (ca != 0.0) v += ca * pa[e];
        if (cb != 0.0) v += cb * pb[e];
        x[e] = v;
    }
}


// Mixed precision, start: r32 = float(r64) (lane-interleaved);
// <r32, r32>_W becomes the CG recurrence's residual norm.
template <int N>
__device__ __forceinline__ void mixed_start_body(int b, int nb, Geom g,
                                                 const OpConst<double>& k,
                                                 const double* __restrict__ r64,
                                                 float* __restrict__ r32,
                                                 CgScalars* sc, unsigned* counter,
                                                 double* partials) {
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    double part[1] = {0.0};
    for (long cell = b * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)nb * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const long l64 = ((long)cy * G + (cx >> 6)) * (N * N * 64) + (cx & 63);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double row[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int e = j * N + i;
                const float f = (float)r64[l64_at<N>(l64, e)];
                r32[l64_at<N>(l64, e)] = f;
                row[i] = (double)f * (double)f;
            }
            part[0] += wrow<N>(k, j, row);
        }
    }
    double tot[1];
    if (reduce_last<1, kPwThreads>(part, partials, counter, nb, b, tot) &&
        threadIdx.x == 0) {
        sc->rr_true = sc->rr;
        sc->rr = tot[0];
        sc->rz = tot[0];
        sc->rr_max = tot[0];
        sc->rr_true_prev = __builtin_inf();
        sc->outer = 0;
    }
}

// Adams-Bashforth update: omega += c0 R0 + c1 R1 + ... (K terms, in order).
__device__ __forceinline__ void ab_combine_body(int b, int nb, long elems,
                                                double* __restrict__ omega,
                                                const double* r0, const double* r1,
                                                const double* r2, const double* r3,
                                                double c0, double c1, double c2, double c3,
                                                int K) {
    for (long e = b * (long)kPwThreads + threadIdx.x; e < elems; e += (long)nb * kPwThreads) {
        double w = omega[e];
        w = fmx(c0, r0[e], w);
        if (K > 1) w = fmx(c1, r1[e], w);
        if (K > 2) w = fmx(c2, r2[e], w);
        if (K > 3) w = fmx(c3, r3[e], w);
        omega[e] = w;
    }
}

}  // namespace dgk

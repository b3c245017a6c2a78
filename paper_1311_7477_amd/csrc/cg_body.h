// LDG Laplacian and conjugate-gradient kernels (cell per lane).
//
// A lane holds all n*n nodal values of one cell in registers; a wave holds
// 64 consecutive cells of one cell row, a workgroup WV consecutive rows (a
// 64 x WV tile; WV in {4, 8, 16} is a template parameter chosen per grid by
// the tile autotuner).  Each 1D operator couples a cell to its
// neighbours only through one scalar per node row (x) or column (y) -- the
// rank-one face blocks of the LDG second derivative (Sec. 6, built from the
// one-sided variants of Sec. 3 eq. discrete_derivative) -- so:
//   * x face scalars come from lanes +-1 by cross-lane shuffles,
//   * y face scalars come from waves +-1 through LDS (one barrier),
//   * only the edge lanes / edge waves of a tile load a halo cell.
//
// The CG vectors x, r, p live in a lane-interleaved layout ("L64"): cells
// are grouped by 64 along x, and inside a group the nodes are stored in
// pairs, node pair m of all 64 cells before pair m + 1,
//   node e of cell (cy, cx) at (cy * G + cx / 64) * 64 n^2 + (e / 2) * 128
//                              + 2 (cx % 64) + e % 2
// (an odd last node alone, at + (n^2 / 2) * 128 + cx % 64), G = ceil(nx / 64),
// so a lane moves two nodes of its cell per 16-byte access and every
// wave-wide access touches 1024 contiguous bytes (l64_at in dg_device.h).
// Fields that cross the library boundary (omega, the guess, psi) keep the
// canonical [cy][cx][j][i] layout and are converted at the start and the end
// of a solve.
#pragma once

#include "dg_device.h"

namespace dgk {


struct CellRef {
    long canon;   // canonical offset of node 0 (node e at +e)
    long l64;     // L64 offset of the cell (node e at l64_at(l64, e))
};

struct CellCtx {
    int lane, wave;
    bool active;                   // this lane's cell lies in the grid
    bool xin_r, xin_l;             // x neighbour held by lane +-1
    bool yin_u, yin_d;             // y neighbour row held by wave +-1 (uniform)
    // homogeneous Dirichlet axes: first / second / last cell along x and y
    bool lo_x, sec_x, hi_x, lo_y, sec_y, hi_y;
    CellRef self, r, l, u, d;
};

template <int N>
__device__ __forceinline__ CellRef cell_ref(const Geom& g, int G, int cx, int cy) {
    CellRef c;
    c.canon = ((long)cy * g.nx + cx) * (N * N);
    c.l64 = ((long)cy * G + (cx >> 6)) * (N * N * 64) + (cx & 63);
    return c;
}

template <int N, int WV>
__device__ __forceinline__ CellCtx make_cell_ctx(const Geom& g, int tilesX,
                                                 int nblocks, int b) {
    CellCtx c;
    c.lane = threadIdx.x & 63;
    c.wave = threadIdx.x >> 6;
    const int t = xcd_tile(b, nblocks);
    const int ty = t / tilesX, tx = t - ty * tilesX;
    const int cx = tx * 64 + c.lane;
    const int cy = ty * WV + c.wave;
    c.active = cx < g.nx && cy < g.ny;
    const int cxa = c.active ? cx : 0, cya = c.active ? cy : 0;
    const int cxr = (cxa + 1 < g.nx) ? cxa + 1 : 0;
    const int cxl = (cxa > 0) ? cxa - 1 : g.nx - 1;
    const int cyu = (cya + 1 < g.ny) ? cya + 1 : 0;
    const int cyd = (cya > 0) ? cya - 1 : g.ny - 1;
    c.xin_r = c.lane < 63 && cx + 1 < g.nx;
    c.xin_l = c.lane > 0;
    c.yin_u = c.wave + 1 < WV && cy + 1 < g.ny;
    c.yin_d = c.wave > 0;
    c.lo_x = g.bcx && cx == 0;
    c.sec_x = g.bcx && cx == 1;
    c.hi_x = g.bcx && cx == g.nx - 1;
    c.lo_y = g.bcy && cy == 0;
    c.sec_y = g.bcy && cy == 1;
    c.hi_y = g.bcy && cy == g.ny - 1;
    const int G = tilesX;
    c.self = cell_ref<N>(g, G, cxa, cya);
    c.r = cell_ref<N>(g, G, cxr, cya);
    c.l = cell_ref<N>(g, G, cxl, cya);
    c.u = cell_ref<N>(g, G, cxa, cyu);
    c.d = cell_ref<N>(g, G, cxa, cyd);
    return c;
}

template <int N, class T>
__device__ __forceinline__ void ld_canon(const T* __restrict__ f, const CellRef& c,
                                         T (&u)[N * N]) {
#pragma unroll
    for (int e = 0; e < N * N; ++e) u[e] = f[c.canon + e];
}

template <int N, class T>
__device__ __forceinline__ void st_canon(T* __restrict__ f, const CellRef& c,
                                         const T (&u)[N * N]) {
#pragma unroll
    for (int e = 0; e < N * N; ++e) f[c.canon + e] = u[e];
}

// L64 loads and stores convert between the storage type S of a CG vector
// and the FP64 arithmetic of the kernels.
template <class S> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

template <int N, class S, class C>
__device__ __forceinline__ void ld_l64(const S* __restrict__ f, const CellRef& c,
                                       C (&u)[N * N]) {
    using V = typename Pair2<S>::type;
    constexpr int P = (N * N) & ~1;
#pragma unroll
    for (int e = 0; e < P; e += 2) {
        const V v = *reinterpret_cast<const V*>(f + l64_at<N>(c.l64, e));
        u[e] = (C)v.x;
        u[e + 1] = (C)v.y;
    }
    if (P < N * N) u[N * N - 1] = (C)f[l64_at<N>(c.l64, N * N - 1)];
}

template <int N, class S, class C>
__device__ __forceinline__ void st_l64(S* __restrict__ f, const CellRef& c,
                                       const C (&u)[N * N]) {
    using V = typename Pair2<S>::type;
    constexpr int P = (N * N) & ~1;
#pragma unroll
    for (int e = 0; e < P; e += 2) {
        V v;
        v.x = (S)u[e];
        v.y = (S)u[e + 1];
        *reinterpret_cast<V*>(f + l64_at<N>(c.l64, e)) = v;
    }
    if (P < N * N) f[l64_at<N>(c.l64, N * N - 1)] = (S)u[N * N - 1];
}

// Round a value to the storage type S and back: the value a stored vector
// will hold, so that an operator applied in registers sees exactly the
// stored vector.  The identity for S = double.
template <class S>
__device__ __forceinline__ double as_stored(double v) { return (double)(S)v; }

// Face scalars of a cell u (n x n, [j][i]) along x for node row j and along
// y for node column i, with weights w.
template <int N, class T>
__device__ __forceinline__ T xdot(const T (&u)[N * N], int j, const T* w) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) s = fmx(w[i], u[j * N + i], s);
    return s;
}

template <int N, class T>
__device__ __forceinline__ T ydot(const T (&u)[N * N], int i, const T* w) {
    T s = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) s = fmx(w[k], u[k * N + i], s);
    return s;
}

// LDS for the y face scalars of one tile: [wave][face][i][lane]
template <int N, class T, int WV>
struct YFaces {
    T v[WV * 2 * N * 64];
};

// Lap_h u for this lane's cell.  `src(ref, out)` evaluates the field on a
// halo cell; the own cell's values are passed in u.  Every thread of the
// block must call it (one barrier).  DIR: the homogeneous Dirichlet closure
// on the axes the grid marks (the last cell drops its outer coupling, the
// first cell uses L0B / eRB and drops its outer coupling, and it is seen by
// the second cell through lLB); the periodic kernels do not carry it.
// ISO: square cells and the same boundary kind on both axes, whose x and y
// blocks coincide -- the y operator reads the x tables (half the constants
// held in registers).
template <int N, int WV, bool DIR = false, bool ISO = false, class T, class Src>
__device__ __forceinline__ void lap_cell(const CellCtx& c, const OpConst<T>& k,
                                         const Src& src, const T (&u)[N * N],
                                         YFaces<N, T, WV>& lds, T (&out)[N * N]) {
    // The Dirichlet tables of the first cells (L0B, eRB, lLB) are chosen by
    // per-lane conditions.  Selecting a table pointer per lane would make
    // the compiler hold a per-lane copy of the selected constants; instead
    // every use sits in a branch whose table is the same for all its lanes
    // (a kernel-argument constant), and only waves holding a first or second
    // cell of a Dirichlet axis run the extra branch.
    const T* lLy = ISO ? k.lLx : k.lLy;
    const T* lLBy = ISO ? k.lLBx : k.lLBy;
    T hR[N], hL[N], hU[N], hD[N];
#pragma unroll
    for (int m = 0; m < N; ++m) hR[m] = hL[m] = hU[m] = hD[m] = 0;
    if (c.active && !c.yin_u) {
        T h[N * N];
        src(c.u, h);
#pragma unroll
        for (int i = 0; i < N; ++i) hU[i] = ydot<N>(h, i, k.lR);
    }
    if (c.active && !c.yin_d) {
        T h[N * N];
        src(c.d, h);
        if (DIR && c.sec_y) {
#pragma unroll
            for (int i = 0; i < N; ++i) hD[i] = ydot<N>(h, i, lLBy);
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) hD[i] = ydot<N>(h, i, lLy);
        }
    }
    if (c.active && !c.xin_r) {
        T h[N * N];
        src(c.r, h);
#pragma unroll
        for (int j = 0; j < N; ++j) hR[j] = xdot<N>(h, j, k.lR);
    }
    if (c.active && !c.xin_l) {
        T h[N * N];
        src(c.l, h);
        if (DIR && c.sec_x) {
#pragma unroll
            for (int j = 0; j < N; ++j) hL[j] = xdot<N>(h, j, k.lLBx);
        } else {
#pragma unroll
            for (int j = 0; j < N; ++j) hL[j] = xdot<N>(h, j, k.lLx);
        }
    }
    // publish this cell's y face scalars
    {
        T dn[N];
#pragma unroll
        for (int i = 0; i < N; ++i) dn[i] = ydot<N>(u, i, lLy);
        if (DIR && c.lo_y) {
#pragma unroll
            for (int i = 0; i < N; ++i) dn[i] = ydot<N>(u, i, lLBy);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            lds.v[((c.wave * 2 + 0) * N + i) * 64 + c.lane] = ydot<N>(u, i, k.lR);
            lds.v[((c.wave * 2 + 1) * N + i) * 64 + c.lane] = dn[i];
        }
    }
    // x face scalars from the neighbouring lanes
    T fR[N], fL[N];
    {
        T lf[N];
#pragma unroll
        for (int j = 0; j < N; ++j) lf[j] = xdot<N>(u, j, k.lLx);
        if (DIR && c.lo_x) {
#pragma unroll
            for (int j = 0; j < N; ++j) lf[j] = xdot<N>(u, j, k.lLBx);
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const T a = __shfl(xdot<N>(u, j, k.lR), c.lane + 1);
            const T b = __shfl(lf[j], c.lane - 1);
            fR[j] = c.xin_r ? a : hR[j];
            fL[j] = c.xin_l ? b : hL[j];
            if (DIR) {
                if (c.hi_x) fR[j] = 0;
                if (c.lo_x) fL[j] = 0;
            }
        }
    }
    __syncthreads();
    T fU[N], fD[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        fU[i] = c.yin_u ? lds.v[(((c.wave + 1) * 2 + 0) * N + i) * 64 + c.lane] : hU[i];
        fD[i] = c.yin_d ? lds.v[(((c.wave - 1) * 2 + 1) * N + i) * 64 + c.lane] : hD[i];
        if (DIR) {
            if (c.hi_y) fU[i] = 0;
            if (c.lo_y) fD[i] = 0;
        }
    }
    auto combine = [&](const T* L0x, const T* eRx, const T* L0y, const T* eRy) {
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T lx = fmx(eRx[i], fR[j], k.eL[i] * fL[j]);
                T ly = fmx(eRy[j], fU[i], k.eL[j] * fD[i]);
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    lx = fmx(L0x[i * N + m], u[j * N + m], lx);
                    ly = fmx(L0y[j * N + m], u[m * N + i], ly);
                }
                out[j * N + i] = fmx(lx, k.ihx2, ly * k.ihy2);
            }
    };
    const T* L0y = ISO ? k.L0x : k.L0y;
    const T* eRy = ISO ? k.eRx : k.eRy;
    const T* L0By = ISO ? k.L0Bx : k.L0By;
    const T* eRBy = ISO ? k.eRBx : k.eRBy;
    if (!DIR || !(c.lo_x || c.lo_y)) {
        combine(k.L0x, k.eRx, L0y, eRy);
    } else if (c.lo_x && c.lo_y) {
        combine(k.L0Bx, k.eRBx, L0By, eRBy);
    } else if (c.lo_x) {
        combine(k.L0Bx, k.eRBx, L0y, eRy);
    } else {
        combine(k.L0x, k.eRx, L0By, eRBy);
    }
}

// <a, b>_W over one cell, accumulated in FP64
template <int N, class T>
__device__ __forceinline__ double wdot_cell(const OpConst<T>& k, const T (&a)[N * N],
                                            const T (&b)[N * N]) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i)
            r = fmx((double)k.w[i], (double)a[j * N + i] * (double)b[j * N + i], r);
        s = fmx(r, (double)k.w[j], s);
    }
    return s * k.wq;
}

template <int N, class T>
struct SrcCanon {                       // u = f (canonical layout)
    const T* f;
    __device__ void operator()(const CellRef& c, T (&u)[N * N]) const { ld_canon<N>(f, c, u); }
};

template <int N, class S>
struct SrcL64 {                         // u = f (L64 layout, stored as S)
    const S* f;
    __device__ void operator()(const CellRef& c, double (&u)[N * N]) const {
        ld_l64<N>(f, c, u);
    }
};

// FP32-stored recurrences (mixed precision) take the exact line-search step
// alpha = <r,p>/<p,Ap> (equal to <r,r>/<p,Ap> without rounding, and still a
// descent step once rounding has cost r its orthogonality to p_old), and,
// right after a residual replacement, the direction p = cr r + beta p_old
// (mixed_replace_body).
template <class S>
constexpr bool kStoredLow = sizeof(S) < sizeof(double);

template <int N, class S>
struct SrcDirection {                   // p = r (first) or cr r + beta p_old, L64
    const S* r;
    const S* p;
    double beta, cr;
    bool first;
    __device__ void operator()(const CellRef& c, double (&u)[N * N]) const {
        ld_l64<N>(r, c, u);
        if (!first) {
            double q[N * N];
            ld_l64<N>(p, c, q);
#pragma unroll
            for (int e = 0; e < N * N; ++e) {
                const double ru = kStoredLow<S> ? cr * u[e] : u[e];
                u[e] = as_stored<S>(fmx(beta, q[e], ru));
            }
        }
    }
};

template <int N>
struct SrcGuess {                       // x0 = ca pa + cb pb, canonical
    const double* pa;
    const double* pb;
    double ca, cb;
    __device__ void operator()(const CellRef& c, double (&u)[N * N]) const {
#pragma unroll
        for (int e = 0; e < N * N; ++e) u[e] = 0.0;
        if (ca != 0.0) {
            double a[N * N];
            ld_canon<N>(pa, c, a);
#pragma unroll
            for (int e = 0; e < N * N; ++e) u[e] = fmx(ca, a[e], u[e]);
        }
        if (cb != 0.0) {
            double b[N * N];
            ld_canon<N>(pb, c, b);
#pragma unroll
            for (int e = 0; e < N * N; ++e) u[e] = fmx(cb, b[e], u[e]);
        }
    }
};

template <int N, class T>
__device__ __forceinline__ void zero_cell(T (&u)[N * N]) {
#pragma unroll
    for (int e = 0; e < N * N; ++e) u[e] = 0;
}

// out = Lap_h u (canonical layout in and out)
template <int N, int WV, bool DIR = false, bool ISO = false>
__device__ __forceinline__ void laplace_body(
    int b, Geom g, int tilesX, int nblocks, const OpConst<double>& k,
    const double* __restrict__ u, double* __restrict__ out,
    YFaces<N, double, WV>& lds) {
    const CellCtx c = make_cell_ctx<N, WV>(g, tilesX, nblocks, b);
    SrcCanon<N, double> src{u};
    double v[N * N], lap[N * N];
    if (c.active) src(c.self, v);
    else zero_cell<N>(v);
    lap_cell<N, WV, DIR, ISO>(c, k, src, v, lds, lap);
    if (c.active) st_canon<N>(out, c.self, lap);
}

// CG setup (stencil part): x0 = guess (to L64; its mean is left in, see
// cg_mean_body);
// r0 = (omega - mean(omega)) + Lap_h x0 (to L64); partials <r0,r0>_W, <b,b>_W.
template <int N, int WV, bool DIR = false, bool ISO = false>
__device__ __forceinline__ void cg_init_body(
    int b, Geom g, int tilesX, int nblocks, const OpConst<double>& k,
    const double* __restrict__ omega, const double* __restrict__ pa,
    const double* __restrict__ pb, double ca, double cb,
    double* __restrict__ x, double* __restrict__ r, CgScalars* sc,
    unsigned* counter, double* partials,
    YFaces<N, double, WV>& lds) {
    const CellCtx c = make_cell_ctx<N, WV>(g, tilesX, nblocks, b);
    SrcGuess<N> src{pa, pb, ca, cb};
    const double mo = sc->mean_omega;
    double x0[N * N], lap[N * N];
    if (c.active) src(c.self, x0);
    else zero_cell<N>(x0);
    lap_cell<N, WV, DIR, ISO>(c, k, src, x0, lds, lap);
    double part[2] = {0.0, 0.0};
    if (c.active) {
        double b[N * N];
        ld_canon<N>(omega, c.self, b);
#pragma unroll
        for (int e = 0; e < N * N; ++e) {
            b[e] -= mo;
            lap[e] += b[e];          // r0
        }
        st_l64<N>(x, c.self, x0);
        st_l64<N>(r, c.self, lap);
        part[0] = wdot_cell<N>(k, lap, lap);
        part[1] = wdot_cell<N>(k, b, b);
    }
    double tot[2];
    if (reduce_last<2, 64 * WV>(part, partials, counter, nblocks, b, tot) &&
        threadIdx.x == 0) {
        sc->rr = tot[0];
        sc->rz = tot[0];
        sc->bb = tot[1];
        sc->first = 1;
        sc->iter = 0;
        sc->pending = 0;
        sc->breakdown = 0;
        // b at the rounding level of the mean removal counts as zero
        if (tot[1] <= sc->zero_tol2 * sc->ww) {
            sc->zero = 1;
            sc->done = 1;
            sc->converged = 1;
        } else if (tot[0] <= sc->tol2 * tot[1]) {
            sc->done = 1;
            sc->converged = 1;
        } else if (sc->max_iter <= 0) {
            sc->done = 1;
        }
    }
}

// CG iteration, first half (L64 vectors r, p stored as S, x in FP64, FP64
// arithmetic):
//   x += alpha_{k-1} p_{k-1};  p_k = r_k + beta_{k-1} p_{k-1};  q = A p_k;
//   alpha_k = <r,r>_W / <p_k, q>_W.
// p is double-buffered (pin -> pout) because halo cells read p_{k-1} of the
// neighbouring tiles while p_k is written.  q is applied to p_k as stored.
// FP64 directions update x every other iteration: at odd k the update waits;
// at even k the cell first reads p_{k-2} from pout (its own cell, before p_k
// replaces it) and applies alpha_{k-2} p_{k-2}, then alpha_{k-1} p_{k-1} --
// the same two roundings in the same order as one update per iteration, so x
// is unchanged bit for bit, while x is read and written half as often.  The
// updates still missing when the solve stops are sc->pending (0, 1 or 2; the
// finish kernel applies them).  FP32-stored directions keep one update per
// iteration (their residual replacement needs x current).
template <int N, class S, int WV, bool DIR = false, bool ISO = false>
__device__ __forceinline__ void cg_dir_body(
    int b, Geom g, int tilesX, int nblocks, const OpConst<double>& k,
    const S* __restrict__ r, S* p0, S* p1, double* __restrict__ x,
    CgScalars* sc, unsigned* counter, double* partials,
    YFaces<N, double, WV>& lds) {
    if (sc->done) return;
    // iteration k reads p_{k-1} from buffer k mod 2 and writes p_k to the other
    const int it = sc->iter;
    const S* pin = (it & 1) ? p1 : p0;
    S* pout = (it & 1) ? p0 : p1;
    constexpr bool kPair = !kStoredLow<S>;
    const bool upd_x = !kPair || !(it & 1);
    const CellCtx c = make_cell_ctx<N, WV>(g, tilesX, nblocks, b);
    // first = 1: p = r; otherwise x += alpha p_old (at even k also the
    // update before it), p = r + beta p_old
    const int first = sc->first;
    const double alpha = sc->alpha;
    const double alpha_prev = sc->alpha_prev;
    SrcDirection<N, S> src{r, pin, sc->beta, sc->cr, first == 1};
    double p[N * N], q[N * N], rv[N * N];
    if (c.active) {
        if (first != 1) {
            double po[N * N];
            ld_l64<N>(pin, c.self, po);
            // x first, so that at most three cell vectors are live at once
            if (upd_x) {
                double xv[N * N];
                ld_l64<N>(x, c.self, xv);
                if (kPair) {
                    double pp[N * N];
                    ld_l64<N>(pout, c.self, pp);
#pragma unroll
                    for (int e = 0; e < N * N; ++e) xv[e] = fmx(alpha_prev, pp[e], xv[e]);
                }
#pragma unroll
                for (int e = 0; e < N * N; ++e) xv[e] = fmx(alpha, po[e], xv[e]);
                st_l64<N>(x, c.self, xv);
            }
            ld_l64<N>(r, c.self, p);
#pragma unroll
            for (int e = 0; e < N * N; ++e) {
                rv[e] = p[e];
                const double ru = kStoredLow<S> ? src.cr * p[e] : p[e];
                p[e] = as_stored<S>(fmx(src.beta, po[e], ru));
            }
        } else {
            ld_l64<N>(r, c.self, p);
#pragma unroll
            for (int e = 0; e < N * N; ++e) rv[e] = p[e];
        }
    } else {
        zero_cell<N>(p);
    }
    // <r, p>_W (FP32-stored directions) before the Laplacian, so that r is not
    // held across it
    double rp = 0.0;
    if (kStoredLow<S> && c.active) rp = wdot_cell<N>(k, rv, p);
    lap_cell<N, WV, DIR, ISO>(c, k, src, p, lds, q);
    constexpr int NV = kStoredLow<S> ? 2 : 1;
    double part[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) part[v] = 0.0;
    if (c.active) {
        st_l64<N>(pout, c.self, p);
#pragma unroll
        for (int e = 0; e < N * N; ++e) q[e] = -q[e];
        part[0] = wdot_cell<N>(k, p, q);
        if (kStoredLow<S>) part[NV - 1] = rp;
    }
    double tot[NV];
    if (reduce_last<NV, 64 * WV>(part, partials, counter, nblocks, b, tot) &&
        threadIdx.x == 0) {
        sc->pq = tot[0];
        sc->first = 0;
        sc->cr = 1.0;
        if (tot[0] > 0.0 && tot[0] == tot[0]) {
            sc->alpha_prev = alpha;
            sc->alpha = (kStoredLow<S> ? tot[NV - 1] : sc->rz) / tot[0];
        } else {  // breakdown (or non-finite data): stop; x lacks
                  // alpha_{k-1} p_{k-1} (still in pin) if its update waited
            sc->done = 1;
            sc->breakdown = 1;
            sc->pending = upd_x ? 0 : 1;
        }
    }
}

// CG iteration, second half: q = A p_k; r -= alpha q; beta = <r,r>new/<r,r>;
// convergence test ||r||_W^2 <= tol^2 ||b||_W^2 on r as stored.
template <int N, class S, int WV, bool DIR = false, bool ISO = false>
__device__ __forceinline__ void cg_res_body(
    int b, Geom g, int tilesX, int nblocks, const OpConst<double>& k, const S* p0,
    const S* p1, S* __restrict__ r, CgScalars* sc, unsigned* counter,
    double* partials, YFaces<N, double, WV>& lds) {
    if (sc->done) return;
    const S* p = (sc->iter & 1) ? p0 : p1;   // p_k written by this iteration's direction update
    const CellCtx c = make_cell_ctx<N, WV>(g, tilesX, nblocks, b);
    const double alpha = sc->alpha;
    SrcL64<N, S> src{p};
    double pv[N * N], q[N * N], rv[N * N];
    if (c.active) src(c.self, pv);
    else zero_cell<N>(pv);
    lap_cell<N, WV, DIR, ISO>(c, k, src, pv, lds, q);   // q = Lap p = -A p
    double part[1] = {0.0};
    if (c.active) {
        // r is loaded only now, so that it is not held across the Laplacian
        ld_l64<N>(r, c.self, rv);
#pragma unroll
        for (int e = 0; e < N * N; ++e) rv[e] = as_stored<S>(fmx(alpha, q[e], rv[e]));
        st_l64<N>(r, c.self, rv);
        part[0] = wdot_cell<N>(k, rv, rv);
    }
    double tot[1];
    if (reduce_last<1, 64 * WV>(part, partials, counter, nblocks, b, tot) &&
        threadIdx.x == 0) {
        const double rrn = tot[0];
        if (!sc->precond) {           // plain CG: z = r
            sc->beta = rrn / sc->rz;
            sc->rz = rrn;
        }
        sc->rr = rrn;
        if (kStoredLow<S> && rrn > sc->rr_max) sc->rr_max = rrn;
        // x lacks alpha_k p_k, and alpha_{k-1} p_{k-1} too after an odd k
        // with FP64 directions
        const int pend = (!kStoredLow<S> && (sc->iter & 1)) ? 2 : 1;
        sc->iter += 1;
        if (rrn <= sc->tol2 * sc->bb) {
            sc->done = 1;
            sc->converged = 1;
            sc->pending = pend;
        } else if (sc->iter >= sc->max_iter || !(rrn == rrn)) {
            sc->done = 1;
            sc->pending = pend;
            if (!(rrn == rrn)) sc->breakdown = 1;
        }
    }
}

// Mixed precision, residual replacement.  r and p are stored in FP32, the
// solution x in FP64; x lags by the update alpha p_last that the next
// direction kernel applies (after any iteration, unless the direction
// update broke down, having applied it itself).  A replacement is made when
// the recursive residual has dropped by delta^2 = 1e-2 in <r,r> below its
// largest value since the last replacement, or the recurrence stopped
// (tolerance met by the recursive residual, max_iter, breakdown); otherwise
// the kernel exits at once.  It computes the true residual of x +
// alpha p_last in FP64, r64 = (omega - mean(omega)) + Lap_h (x + alpha p_last),
// stores r32 = float(r64), and tests convergence on r64.  An FP64 residual
// cannot be evaluated more accurately than ~ eps_64 |Lap_h| |x|, which for
// stiff grids exceeds small tolerances; so the solve also ends (converged =
// 2, "at the attainable accuracy") when the recursive residual had met the
// tolerance but the true one fell by less than 2x since the previous
// replacement.  If the solve goes
// on, the next direction is p = cr r32 + beta p_last with beta rescaled to
// the replaced residual and cr = 1 - beta <r32, p_last> / <r32, r32>, so that
// p_last's component along the new residual is removed first (it would be
// zero without rounding).  Partials <r64,r64>_W, <r32,r32>_W, <r32,p_last>_W.
template <int N>
struct SrcMixedX {
    const double* x;
    const float* pl;
    double alpha;
    bool pending;
    __device__ void operator()(const CellRef& c, double (&u)[N * N]) const {
        ld_l64<N>(x, c, u);
        if (pending) {
            double q[N * N];
            ld_l64<N>(pl, c, q);
#pragma unroll
            for (int e = 0; e < N * N; ++e) u[e] = fmx(alpha, q[e], u[e]);
        }
    }
};

constexpr double kReplaceDrop2 = 1e-2;

template <int N, int WV, bool ISO = false>
__device__ __forceinline__ void mixed_replace_body(
    int b, Geom g, int tilesX, int nblocks, const OpConst<double>& k,
    const double* __restrict__ omega, const double* __restrict__ x,
    const float* __restrict__ q0, const float* __restrict__ q1,
    float* __restrict__ r32, CgScalars* sc, unsigned* counter, double* partials,
    YFaces<N, double, WV>& lds) {
    if (!sc->done && !(sc->rr <= kReplaceDrop2 * sc->rr_max)) return;
    const CellCtx c = make_cell_ctx<N, WV>(g, tilesX, nblocks, b);
    const bool pending = sc->first != 1 && !sc->breakdown;
    const float* pl = (sc->iter & 1) ? q1 : q0;
    SrcMixedX<N> src{x, pl, sc->alpha, pending};
    const double mo = sc->mean_omega;
    double v[N * N], lap[N * N];
    if (c.active) src(c.self, v);
    else zero_cell<N>(v);
    lap_cell<N, WV, false, ISO>(c, k, src, v, lds, lap);
    double part[3] = {0.0, 0.0, 0.0};
    if (c.active) {
        double w[N * N], rd[N * N], pv[N * N];
        ld_canon<N>(omega, c.self, w);
        ld_l64<N>(pl, c.self, pv);
#pragma unroll
        for (int e = 0; e < N * N; ++e) {
            lap[e] += w[e] - mo;
            rd[e] = as_stored<float>(lap[e]);
        }
        st_l64<N>(r32, c.self, rd);
        part[0] = wdot_cell<N>(k, lap, lap);
        part[1] = wdot_cell<N>(k, rd, rd);
        part[2] = wdot_cell<N>(k, rd, pv);
    }
    double tot[3];
    if (reduce_last<3, 64 * WV>(part, partials, counter, nblocks, b, tot) &&
        threadIdx.x == 0) {
        const bool rec_met = sc->rr <= sc->tol2 * sc->bb;
        const double prev = sc->rr_true_prev;
        sc->rr_true = tot[0];
        sc->rr_true_prev = tot[0];
        sc->outer += 1;
        if (tot[0] <= sc->tol2 * sc->bb) {
            sc->done = 1;
            sc->converged = 1;
            sc->pending = pending ? 1 : 0;
        } else if (sc->iter >= sc->max_iter || sc->breakdown || !(tot[0] == tot[0])) {
            sc->done = 1;
            sc->converged = 0;
            sc->pending = pending ? 1 : 0;
        } else if (rec_met && tot[0] > 0.25 * prev) {
            sc->done = 1;
            sc->converged = 2;
            sc->pending = pending ? 1 : 0;
        } else {
            if (sc->first != 1) {
                sc->beta *= tot[1] / sc->rz;
                sc->cr = 1.0 - sc->beta * tot[2] / tot[1];
            }
            sc->rr = tot[1];
            sc->rz = tot[1];
            sc->rr_max = tot[1];
            sc->done = 0;
            sc->converged = 0;
            sc->pending = 0;
        }
    }
}

// Tiles of one cell-per-lane launch on a grid.
struct CellLaunch {
    int tilesX, tilesY, nblocks;
    __host__ __device__ explicit CellLaunch(const Geom& g) {
        tilesX = (g.nx + 63) / 64;
        tilesY = (g.ny + g.cw - 1) / g.cw;
        nblocks = tilesX * tilesY;
    }
};

}  // namespace dgk

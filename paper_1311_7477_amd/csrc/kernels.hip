// HIP kernels (gfx950) for the conservative dG Arakawa right-hand side.
//
// Fields are stored cell-major [cy][cx][j][i] with n x n nodal values per
// cell (X-space, Sec. 4.3 last paragraph).  Every 1D operator of the scheme
// couples a cell to its two neighbours along one axis through one scalar per
// node row or column (the rank-one face blocks of Sec. 4.2 eq. discrete_der
// and of the LDG second derivative), so a stencil kernel needs from each
// neighbour only n "face scalars", never its values.
//
// Two work decompositions are used.
//
// Cell per lane (Laplacian-based kernels of the CG loop).  A lane holds all
// n*n values of one cell in registers; a wave holds 64 consecutive cells of
// one cell row and a workgroup WAVES consecutive rows (a 64 x WAVES tile).
// x face scalars come from the neighbouring lanes by cross-lane shuffles,
// y face scalars from the neighbouring waves through LDS (one barrier).
// Only the lanes and waves at the tile edge load a halo cell themselves.
//
// Row per lane (the fused bracket kernel, which needs a 3 x 3 cell
// neighbourhood and many intermediate fields).  A lane holds one node row
// (cell, j); a wave covers S = 64/n cells of a cell row and a workgroup WAVES
// rows; the outer ring of the tile is halo that is computed but not stored.
// x operators use shuffles, y operators an LDS transpose.
//
// Dot products are reduced deterministically: a fixed butterfly in each
// wave, a fixed order across waves, per-block partials in global memory and
// a fixed-order final sum done by whichever block finishes last (an atomic
// ticket decides only who sums, never the order).
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dg_launch.h"

namespace dgk {

// Block index -> tile index such that the blocks the dispatcher sends to one
// XCD (block b goes to XCD b mod 8) get a contiguous run of tiles: halo
// reads of neighbouring tiles then hit the same L2.
__device__ __forceinline__ int xcd_tile(int nblocks) {
    const int b = blockIdx.x;
    const int xcd = b & 7, idx = b >> 3;
    const int q = nblocks >> 3, r = nblocks & 7;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <int M, class T>
__device__ __forceinline__ void load_vec(const T* __restrict__ f, long off,
                                         T (&u)[M]) {
#pragma unroll
    for (int i = 0; i < M; ++i) u[i] = f[off + i];
}

template <int M, class T>
__device__ __forceinline__ void store_vec(T* __restrict__ f, long off,
                                          const T (&u)[M]) {
#pragma unroll
    for (int i = 0; i < M; ++i) f[off + i] = u[i];
}

// ---------------------------------------------------------------------------
// Deterministic block reduction + last-block-done final sum.
//
// Partials are published with agent-scope atomic stores (coherent across
// the XCDs' L2 caches), the publishing wave waits for their completion, then
// takes a ticket with an agent-scope atomic add.  The block that draws the
// last ticket reads all partials with agent-scope atomic loads.  No L2
// write-back or invalidate is needed because only atomics carry data
// between blocks; results for the next kernel are ordinary stores made
// visible by the kernel boundary.
// Returns true in the last block, where tot[] holds the grid-wide sums.
// ---------------------------------------------------------------------------
template <int NV, int NT>
__device__ bool reduce_last(double (&v)[NV], double* partials,
                            unsigned* counter, int nblocks, double (&tot)[NV]) {
    __shared__ double red[(NT / 64) * NV];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w * NV + k];
            __hip_atomic_store(&partials[(long)blockIdx.x * NV + k], s,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_s_waitcnt(0);   // partials performed before the ticket
        const unsigned t = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        is_last = (t == (unsigned)(nblocks - 1));
    }
    __syncthreads();
    if (!is_last) return false;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT)
#pragma unroll
        for (int k = 0; k < NV; ++k)
            acc[k] += __hip_atomic_load(&partials[(long)b * NV + k],
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = acc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * NV + k];
        tot[k] = s;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// ===========================================================================
// Cell per lane: the LDG Laplacian and the CG kernels
// ===========================================================================
constexpr int kCellWaves = 8;   // tile = 64 x 8 cells, 512 threads

struct CellCtx {
    int lane, wave;
    int cx, cy;
    bool active;                   // this lane's cell lies in the grid
    bool xin_r, xin_l;             // x neighbour held by lane +-1
    bool yin_u, yin_d;             // y neighbour row held by wave +-1 (uniform)
    long cell, cell_r, cell_l, cell_u, cell_d;
};

__device__ __forceinline__ CellCtx make_cell_ctx(const Geom& g, int tilesX,
                                                 int nblocks) {
    CellCtx c;
    c.lane = threadIdx.x & 63;
    c.wave = threadIdx.x >> 6;
    const int t = xcd_tile(nblocks);
    const int ty = t / tilesX, tx = t - ty * tilesX;
    c.cx = tx * 64 + c.lane;
    c.cy = ty * kCellWaves + c.wave;
    c.active = c.cx < g.nx && c.cy < g.ny;
    const int cxr = (c.cx + 1 < g.nx) ? c.cx + 1 : 0;
    const int cxl = (c.cx > 0) ? c.cx - 1 : g.nx - 1;
    const int cyu = (c.cy + 1 < g.ny) ? c.cy + 1 : 0;
    const int cyd = (c.cy > 0) ? c.cy - 1 : g.ny - 1;
    c.xin_r = c.lane < 63 && c.cx + 1 < g.nx;
    c.xin_l = c.lane > 0;
    c.yin_u = c.wave + 1 < kCellWaves && c.cy + 1 < g.ny;
    c.yin_d = c.wave > 0;
    const long row = (long)(c.active ? c.cy : 0) * g.nx;
    const int cxa = c.active ? c.cx : 0;
    c.cell = row + cxa;
    c.cell_r = row + cxr;
    c.cell_l = row + cxl;
    c.cell_u = (long)cyu * g.nx + cxa;
    c.cell_d = (long)cyd * g.nx + cxa;
    return c;
}

// Face scalars of a cell u (n x n, [j][i]) along x for node row j and along
// y for node column i, with weights w.
template <int N, class T>
__device__ __forceinline__ T xdot(const T (&u)[N * N], int j, const T* w) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) s += w[i] * u[j * N + i];
    return s;
}

template <int N, class T>
__device__ __forceinline__ T ydot(const T (&u)[N * N], int i, const T* w) {
    T s = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) s += w[k] * u[k * N + i];
    return s;
}

// LDS for the y face scalars of one tile: [wave][face][i][lane]
template <int N, class T>
struct YFaces {
    T v[kCellWaves * 2 * N * 64];
};

// Lap_h u for this lane's cell.  `src(cell, out)` evaluates the field on any
// cell (the own cell's values are passed in u); it is called for halo cells
// only.  Must be called by every thread of the block (one barrier).
template <int N, class T, class Src>
__device__ __forceinline__ void lap_cell(const CellCtx& c, const OpConst<T>& k,
                                         const Src& src, const T (&u)[N * N],
                                         YFaces<N, T>& lds, T (&out)[N * N]) {
    // halo cells first so their loads overlap the shuffles
    T hR[N], hL[N], hU[N], hD[N];
    if (c.active && !c.xin_r) {
        T h[N * N];
        src(c.cell_r, h);
#pragma unroll
        for (int j = 0; j < N; ++j) hR[j] = xdot<N>(h, j, k.lR);
    }
    if (c.active && !c.xin_l) {
        T h[N * N];
        src(c.cell_l, h);
#pragma unroll
        for (int j = 0; j < N; ++j) hL[j] = xdot<N>(h, j, k.lL);
    }
    if (c.active && !c.yin_u) {
        T h[N * N];
        src(c.cell_u, h);
#pragma unroll
        for (int i = 0; i < N; ++i) hU[i] = ydot<N>(h, i, k.lR);
    }
    if (c.active && !c.yin_d) {
        T h[N * N];
        src(c.cell_d, h);
#pragma unroll
        for (int i = 0; i < N; ++i) hD[i] = ydot<N>(h, i, k.lL);
    }
    // publish this cell's y face scalars
#pragma unroll
    for (int i = 0; i < N; ++i) {
        lds.v[((c.wave * 2 + 0) * N + i) * 64 + c.lane] = ydot<N>(u, i, k.lR);
        lds.v[((c.wave * 2 + 1) * N + i) * 64 + c.lane] = ydot<N>(u, i, k.lL);
    }
    // x face scalars from the neighbouring lanes
    T fR[N], fL[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const T dr = xdot<N>(u, j, k.lR);
        const T dl = xdot<N>(u, j, k.lL);
        const T a = __shfl(dr, c.lane + 1);
        const T b = __shfl(dl, c.lane - 1);
        fR[j] = c.xin_r ? a : hR[j];
        fL[j] = c.xin_l ? b : hL[j];
    }
    __syncthreads();
    T fU[N], fD[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        fU[i] = c.yin_u ? lds.v[(((c.wave + 1) * 2 + 0) * N + i) * 64 + c.lane] : hU[i];
        fD[i] = c.yin_d ? lds.v[(((c.wave - 1) * 2 + 1) * N + i) * 64 + c.lane] : hD[i];
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T lx = k.eR[i] * fR[j] + k.eL[i] * fL[j];
            T ly = k.eR[j] * fU[i] + k.eL[j] * fD[i];
#pragma unroll
            for (int m = 0; m < N; ++m) {
                lx += k.L0[i * N + m] * u[j * N + m];
                ly += k.L0[j * N + m] * u[m * N + i];
            }
            out[j * N + i] = lx * k.ihx2 + ly * k.ihy2;
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
            r += (double)k.w[i] * ((double)a[j * N + i] * (double)b[j * N + i]);
        s += r * (double)k.w[j];
    }
    return s * k.wq;
}

template <int N, class T>
struct SrcField {                       // u = f
    const T* f;
    __device__ void operator()(long cell, T (&u)[N * N]) const {
        load_vec(f, cell * (N * N), u);
    }
};

template <int N, class T>
struct SrcDirection {                   // p = r (first) or r + beta p_old
    const T* r;
    const T* p;
    T beta;
    bool first;
    __device__ void operator()(long cell, T (&u)[N * N]) const {
        load_vec(r, cell * (N * N), u);
        if (!first) {
            T q[N * N];
            load_vec(p, cell * (N * N), q);
#pragma unroll
            for (int e = 0; e < N * N; ++e) u[e] += beta * q[e];
        }
    }
};

template <int N>
struct SrcGuess {                       // x0 = ca pa + cb pb - mean
    const double* pa;
    const double* pb;
    double ca, cb, m;
    __device__ void operator()(long cell, double (&u)[N * N]) const {
#pragma unroll
        for (int e = 0; e < N * N; ++e) u[e] = -m;
        if (ca != 0.0) {
            double a[N * N];
            load_vec(pa, cell * (N * N), a);
#pragma unroll
            for (int e = 0; e < N * N; ++e) u[e] += ca * a[e];
        }
        if (cb != 0.0) {
            double b[N * N];
            load_vec(pb, cell * (N * N), b);
#pragma unroll
            for (int e = 0; e < N * N; ++e) u[e] += cb * b[e];
        }
    }
};

// out = Lap_h u
template <int N>
__global__ __launch_bounds__(64 * kCellWaves) void k_laplace(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ u, double* __restrict__ out) {
    __shared__ YFaces<N, double> lds;
    const CellCtx c = make_cell_ctx(g, tilesX, nblocks);
    SrcField<N, double> src{u};
    double v[N * N], lap[N * N];
    if (c.active) src(c.cell, v);
    else
#pragma unroll
        for (int e = 0; e < N * N; ++e) v[e] = 0.0;
    lap_cell<N>(c, k, src, v, lds, lap);
    if (c.active) store_vec(out, c.cell * (N * N), lap);
}

// CG setup (stencil part): x0 = guess - mean(guess);
// r0 = (omega - mean(omega)) + Lap_h x0; partials <r0, r0>_W and <b, b>_W.
template <int N>
__global__ __launch_bounds__(64 * kCellWaves) void k_cg_init(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ omega, const double* __restrict__ pa,
    const double* __restrict__ pb, double ca, double cb,
    double* __restrict__ x, double* __restrict__ r, CgScalars* sc,
    unsigned* counter, double* partials) {
    __shared__ YFaces<N, double> lds;
    const CellCtx c = make_cell_ctx(g, tilesX, nblocks);
    SrcGuess<N> src{pa, pb, ca, cb, sc->mean_guess};
    const double mo = sc->mean_omega;
    double x0[N * N], lap[N * N];
    if (c.active) src(c.cell, x0);
    else
#pragma unroll
        for (int e = 0; e < N * N; ++e) x0[e] = 0.0;
    lap_cell<N>(c, k, src, x0, lds, lap);
    double part[2] = {0.0, 0.0};
    if (c.active) {
        double b[N * N];
        load_vec(omega, c.cell * (N * N), b);
#pragma unroll
        for (int e = 0; e < N * N; ++e) {
            b[e] -= mo;
            lap[e] += b[e];          // r0
        }
        store_vec(x, c.cell * (N * N), x0);
        store_vec(r, c.cell * (N * N), lap);
        part[0] = wdot_cell<N>(k, lap, lap);
        part[1] = wdot_cell<N>(k, b, b);
    }
    double tot[2];
    if (reduce_last<2, 64 * kCellWaves>(part, partials, counter, nblocks, tot) &&
        threadIdx.x == 0) {
        sc->rr = tot[0];
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

// CG iteration, first half:
//   x += alpha_{k-1} p_{k-1};  p_k = r_k + beta_{k-1} p_{k-1};  q = A p_k;
//   alpha_k = <r,r>_W / <p_k, q>_W.
// p is double-buffered (pin -> pout) because halo cells read p_{k-1} of the
// neighbouring tiles while p_k is written.
template <int N, class T>
__global__ __launch_bounds__(64 * kCellWaves) void k_cg_dir(
    Geom g, int tilesX, int nblocks, OpConst<T> k, const T* __restrict__ r,
    const T* __restrict__ pin, T* __restrict__ pout, T* __restrict__ x,
    CgScalars* sc, unsigned* counter, double* partials) {
    if (sc->done) return;
    __shared__ YFaces<N, T> lds;
    const CellCtx c = make_cell_ctx(g, tilesX, nblocks);
    const bool first = sc->first != 0;
    const T alpha = (T)sc->alpha;
    SrcDirection<N, T> src{r, pin, (T)sc->beta, first};
    T p[N * N], q[N * N];
    if (c.active) {
        load_vec(r, c.cell * (N * N), p);
        if (!first) {
            T po[N * N], xv[N * N];
            load_vec(pin, c.cell * (N * N), po);
            load_vec(x, c.cell * (N * N), xv);
#pragma unroll
            for (int e = 0; e < N * N; ++e) {
                xv[e] += alpha * po[e];
                p[e] += src.beta * po[e];
            }
            store_vec(x, c.cell * (N * N), xv);
        }
    } else {
#pragma unroll
        for (int e = 0; e < N * N; ++e) p[e] = 0;
    }
    lap_cell<N>(c, k, src, p, lds, q);
    double part[1] = {0.0};
    if (c.active) {
        store_vec(pout, c.cell * (N * N), p);
#pragma unroll
        for (int e = 0; e < N * N; ++e) q[e] = -q[e];
        part[0] = wdot_cell<N>(k, p, q);
    }
    double tot[1];
    if (reduce_last<1, 64 * kCellWaves>(part, partials, counter, nblocks, tot) &&
        threadIdx.x == 0) {
        sc->pq = tot[0];
        sc->first = 0;
        if (tot[0] > 0.0 && tot[0] == tot[0]) {
            sc->alpha = sc->rr / tot[0];
        } else {  // breakdown (or non-finite data): stop, x is current
            sc->done = 1;
            sc->breakdown = 1;
            sc->pending = 0;
        }
    }
}

// CG iteration, second half: q = A p_k; r -= alpha q; beta = <r,r>new/<r,r>;
// convergence test ||r||_W^2 <= tol^2 ||b||_W^2.
template <int N, class T>
__global__ __launch_bounds__(64 * kCellWaves) void k_cg_res(
    Geom g, int tilesX, int nblocks, OpConst<T> k, const T* __restrict__ p,
    T* __restrict__ r, CgScalars* sc, unsigned* counter, double* partials) {
    if (sc->done) return;
    __shared__ YFaces<N, T> lds;
    const CellCtx c = make_cell_ctx(g, tilesX, nblocks);
    const T alpha = (T)sc->alpha;
    SrcField<N, T> src{p};
    T pv[N * N], q[N * N], rv[N * N];
    if (c.active) {
        src(c.cell, pv);
        load_vec(r, c.cell * (N * N), rv);
    } else {
#pragma unroll
        for (int e = 0; e < N * N; ++e) pv[e] = 0;
    }
    lap_cell<N>(c, k, src, pv, lds, q);   // q = Lap p = -A p
    double part[1] = {0.0};
    if (c.active) {
#pragma unroll
        for (int e = 0; e < N * N; ++e) rv[e] += alpha * q[e];
        store_vec(r, c.cell * (N * N), rv);
        part[0] = wdot_cell<N>(k, rv, rv);
    }
    double tot[1];
    if (reduce_last<1, 64 * kCellWaves>(part, partials, counter, nblocks, tot) &&
        threadIdx.x == 0) {
        const double rrn = tot[0];
        sc->beta = rrn / sc->rr;
        sc->rr = rrn;
        sc->iter += 1;
        if (rrn <= sc->tol2 * sc->bb) {
            sc->done = 1;
            sc->converged = 1;
            sc->pending = 1;
        } else if (sc->iter >= sc->max_iter || !(rrn == rrn)) {
            sc->done = 1;
            sc->pending = 1;
            if (!(rrn == rrn)) sc->breakdown = 1;
        }
    }
}

// Mixed precision, outer step: r64 = (omega - mean(omega)) + Lap_h psi in
// FP64; stores r32 = float(r64) and e32 = 0 for the inner solve; partials
// <r64,r64>, <b,b>, <r32,r32>.  The last block decides outer convergence and
// initialises the inner CG scalars.
template <int N>
__global__ __launch_bounds__(64 * kCellWaves) void k_mixed_residual(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ omega, const double* __restrict__ psi,
    float* __restrict__ r32, float* __restrict__ e32, double inner_tol2,
    int inner_max, CgScalars* outer, CgScalars* inner, unsigned* counter,
    double* partials) {
    __shared__ YFaces<N, double> lds;
    const CellCtx c = make_cell_ctx(g, tilesX, nblocks);
    SrcField<N, double> src{psi};
    const double mo = outer->mean_omega;
    double v[N * N], lap[N * N];
    if (c.active) src(c.cell, v);
    else
#pragma unroll
        for (int e = 0; e < N * N; ++e) v[e] = 0.0;
    lap_cell<N>(c, k, src, v, lds, lap);
    double part[3] = {0.0, 0.0, 0.0};
    if (c.active) {
        double b[N * N], rd[N * N];
        float rf[N * N], zf[N * N];
        load_vec(omega, c.cell * (N * N), b);
#pragma unroll
        for (int e = 0; e < N * N; ++e) {
            b[e] -= mo;
            lap[e] += b[e];
            rf[e] = (float)lap[e];
            rd[e] = (double)rf[e];
            zf[e] = 0.0f;
        }
        store_vec(r32, c.cell * (N * N), rf);
        store_vec(e32, c.cell * (N * N), zf);
        part[0] = wdot_cell<N>(k, lap, lap);
        part[1] = wdot_cell<N>(k, b, b);
        part[2] = wdot_cell<N>(k, rd, rd);
    }
    double tot[3];
    if (reduce_last<3, 64 * kCellWaves>(part, partials, counter, nblocks, tot) &&
        threadIdx.x == 0) {
        outer->rr = tot[0];
        outer->bb = tot[1];
        outer->iter += 1;
        const bool zero = tot[1] <= outer->zero_tol2 * outer->ww;
        const bool ok = zero || tot[0] <= outer->tol2 * tot[1];
        outer->converged = ok ? 1 : 0;
        outer->zero = zero ? 1 : 0;
        inner->rr = tot[2];
        inner->bb = tot[2];
        inner->tol2 = inner_tol2;
        inner->max_iter = inner_max;
        inner->alpha = 0.0;
        inner->beta = 0.0;
        inner->first = 1;
        inner->iter = 0;
        inner->pending = 0;
        inner->zero = 0;
        inner->breakdown = 0;
        inner->converged = 0;
        inner->done = (ok || tot[2] == 0.0 || inner_max <= 0) ? 1 : 0;
    }
}

// ===========================================================================
// Row per lane: the fused bracket / right-hand-side kernel
// ===========================================================================
template <int N, int WAVES>
struct Tile {
    static constexpr int S = 64 / N;          // cell slots per wave
    static constexpr int TX = S - 2;          // interior cells per tile in x
    static constexpr int TY = WAVES - 2;      // interior cells per tile in y
    // LDS stride of one cell: odd for even n so that lanes of different
    // cells fall into different banks
    static constexpr int CS = (N % 2 == 0) ? N * N + 1 : N * N;
    static constexpr int LDS_FIELD = WAVES * S * CS;
};

constexpr int kRowWaves = 8;

template <int N, int WAVES>
struct Ctx {
    int lane, wave, s, j;
    bool active;      // lane holds a node row
    bool interior;    // lane's cell is inside the tile and the grid: stores
    long row;         // element index of this thread's row start
    int slot;         // wave * S + s (LDS cell slot)
};

template <int N, int WAVES>
__device__ __forceinline__ Ctx<N, WAVES> make_ctx(const Geom& g, int tilesX,
                                                  int nblocks) {
    using TL = Tile<N, WAVES>;
    Ctx<N, WAVES> c;
    c.lane = threadIdx.x & 63;
    c.wave = threadIdx.x >> 6;
    c.s = c.lane / N;
    c.j = c.lane - c.s * N;
    c.active = c.s < TL::S;
    const int t = xcd_tile(nblocks);
    const int ty = t / tilesX, tx = t - ty * tilesX;
    const int cx = tx * TL::TX + c.s - 1;
    const int cy = ty * TL::TY + c.wave - 1;
    c.interior = c.active && c.s >= 1 && c.s <= TL::TX && c.wave >= 1 &&
                 c.wave <= TL::TY && cx < g.nx && cy < g.ny;
    int gx = cx % g.nx;
    if (gx < 0) gx += g.nx;
    int gy = cy % g.ny;
    if (gy < 0) gy += g.ny;
    const long cell = c.active ? (long)gy * g.nx + gx : 0;
    c.row = (cell * N + c.j) * N;
    c.slot = c.wave * TL::S + (c.active ? c.s : TL::S - 1);
    return c;
}

// One 1D operator along x on this thread's row:
//   res = scale * (A0 u + eR (tR . u_right) + eL (tL . u_left))
template <int N, class T>
__device__ __forceinline__ void row_op(const T (&u)[N], int lane,
                                       const T* A0, const T* eR, const T* tR,
                                       const T* eL, const T* tL, T scale,
                                       T (&res)[N]) {
    T dR = 0, dL = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        dR += tR[k] * u[k];
        dL += tL[k] * u[k];
    }
    // the right neighbour cell is N lanes up, the left one N lanes down;
    // lanes of the edge slots receive wrapped values but are halo
    const T fromR = __shfl(dR, lane + N);
    const T fromL = __shfl(dL, lane - N);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T a = eR[i] * fromR + eL[i] * fromL;
#pragma unroll
        for (int k = 0; k < N; ++k) a += A0[i * N + k] * u[k];
        res[i] = a * scale;
    }
}

// One 1D operator along y evaluated on column j of this thread's cell from
// rows staged in LDS; res[k] is the value at node (k, j).  The halo waves
// read clamped (wrong but in-bounds) neighbours and are never stored.
template <int N, int WAVES, class T>
__device__ __forceinline__ void col_op(const T* lds, const Ctx<N, WAVES>& c,
                                       const T* A0, const T* eR, const T* tR,
                                       const T* eL, const T* tL, T scale,
                                       T (&res)[N]) {
    using TL = Tile<N, WAVES>;
    const int up = c.slot + (c.wave + 1 < WAVES ? TL::S : 0);
    const int dn = c.slot - (c.wave > 0 ? TL::S : 0);
    const T* c0 = lds + c.slot * TL::CS + c.j;
    const T* cu = lds + up * TL::CS + c.j;
    const T* cd = lds + dn * TL::CS + c.j;
    T col[N];
    T du = 0, dd = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        col[k] = c0[k * N];
        du += tR[k] * cu[k * N];
        dd += tL[k] * cd[k * N];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        T a = eR[k] * du + eL[k] * dd;
#pragma unroll
        for (int m = 0; m < N; ++m) a += A0[k * N + m] * col[m];
        res[k] = a * scale;
    }
}

template <int N, int WAVES, class T>
__device__ __forceinline__ void lds_put_row(T* lds, const Ctx<N, WAVES>& c,
                                            const T (&u)[N]) {
    if (c.active) {
#pragma unroll
        for (int i = 0; i < N; ++i) lds[c.slot * Tile<N, WAVES>::CS + c.j * N + i] = u[i];
    }
}

template <int N, int WAVES, class T>
__device__ __forceinline__ void lds_put_col(T* lds, const Ctx<N, WAVES>& c,
                                            const T (&v)[N]) {
    if (c.active) {
#pragma unroll
        for (int k = 0; k < N; ++k) lds[c.slot * Tile<N, WAVES>::CS + k * N + c.j] = v[k];
    }
}

template <int N, int WAVES, class T>
__device__ __forceinline__ void lds_get_row(const T* lds, const Ctx<N, WAVES>& c,
                                            T (&u)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = lds[c.slot * Tile<N, WAVES>::CS + c.j * N + i];
}

// Bracket and right-hand side.
//   J = scale * (c0 J++ + Dx(c1 f Dy g - c2 Dy f g) + Dy(c2 Dx f g - c1 f Dx g))
// (c0, c1, c2, scale) = (1, 1, 1, 1/3) gives (J++ + J+x + Jx+)/3 (Sec. 2
// eq. J); one of them alone gives a single form.  With VISC the kernel
// forms R = -J(f, g) + D Lap_h g and stores a * wn + b * (g + dt R)
// (SSP-RK3 stage combination; wn may be null when a == 0).
struct RhsArgs {
    double c0, c1, c2, scale;
    double D, dt, a, b;
};

template <int N, int WAVES, bool VISC>
__global__ __launch_bounds__(64 * WAVES) void k_rhs(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ f, const double* __restrict__ gg,
    const double* __restrict__ wn, double* __restrict__ out, RhsArgs ra) {
    using TL = Tile<N, WAVES>;
    __shared__ double lA[TL::LDS_FIELD];
    __shared__ double lB[TL::LDS_FIELD];
    __shared__ double lC[VISC ? TL::LDS_FIELD : 1];
    const auto c = make_ctx<N, WAVES>(g, tilesX, nblocks);

    double F[N], G[N];
    load_vec(f, c.row, F);
    load_vec(gg, c.row, G);

    double DxF[N], DxG[N], LxG[N], DyF[N], DyG[N], LyG[N];
    row_op(F, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxF);
    row_op(G, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxG);
    if (VISC) row_op(G, c.lane, k.L0, k.eR, k.lR, k.eL, k.lL, k.ihx2, LxG);

    lds_put_row(lA, c, F);
    lds_put_row(lB, c, G);
    __syncthreads();
    {
        double cF[N], cG[N], cL[N];
        col_op(lA, c, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihy, cF);
        col_op(lB, c, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihy, cG);
        if (VISC) col_op(lB, c, k.L0, k.eR, k.lR, k.eL, k.lL, k.ihy2, cL);
        __syncthreads();
        lds_put_col(lA, c, cF);
        lds_put_col(lB, c, cG);
        if (VISC) lds_put_col(lC, c, cL);
    }
    __syncthreads();
    lds_get_row(lA, c, DyF);
    lds_get_row(lB, c, DyG);
    if (VISC) lds_get_row(lC, c, LyG);
    __syncthreads();

    double J[N], A[N], B[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        J[i] = ra.c0 * (DxF[i] * DyG[i] - DyF[i] * DxG[i]);
        A[i] = ra.c1 * (F[i] * DyG[i]) - ra.c2 * (DyF[i] * G[i]);
        B[i] = ra.c2 * (DxF[i] * G[i]) - ra.c1 * (F[i] * DxG[i]);
    }
    double DxA[N], DyB[N];
    row_op(A, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxA);
    lds_put_row(lA, c, B);
    __syncthreads();
    {
        double cb[N];
        col_op(lA, c, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihy, cb);
        __syncthreads();
        lds_put_col(lA, c, cb);
    }
    __syncthreads();
    lds_get_row(lA, c, DyB);

    if (!c.interior) return;
    double o[N];
    if (VISC) {
        double wnr[N];
        if (ra.a != 0.0) load_vec(wn, c.row, wnr);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double Jv = ra.scale * (J[i] + DxA[i] + DyB[i]);
            const double R = ra.D * (LxG[i] + LyG[i]) - Jv;
            const double s = ra.b * (G[i] + ra.dt * R);
            o[i] = (ra.a != 0.0) ? ra.a * wnr[i] + s : s;
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) o[i] = ra.scale * (J[i] + DxA[i] + DyB[i]);
    }
    store_vec(out, c.row, o);
}

// ===========================================================================
// Pointwise kernels (grid-stride over node rows)
// ===========================================================================
constexpr int kPwThreads = 256;

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
        double w[N], gs[N];
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
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            s0 += k.w[i] * w[i];
            s1 += k.w[i] * gs[i];
            s2 += k.w[i] * (w[i] * w[i]);
        }
        const double wj = k.w[j] * k.wq;
        part[0] += s0 * wj;
        part[1] += s1 * wj;
        part[2] += s2 * wj;
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

// End of a solve: apply the pending x += alpha p (p = the buffer written by
// the last direction update), or zero x when b = 0; then the W-mean of x.
template <int N, class T>
__global__ __launch_bounds__(kPwThreads) void k_cg_finish(
    long rows, OpConst<T> k, T* __restrict__ x, const T* __restrict__ p0,
    const T* __restrict__ p1, double area, CgScalars* sc, unsigned* counter,
    double* partials) {
    const int pending = sc->pending, zero = sc->zero;
    const T alpha = (T)sc->alpha;
    const T* pl = (sc->iter & 1) ? p1 : p0;
    double part[1] = {0.0};
    for (long row = blockIdx.x * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)gridDim.x * kPwThreads) {
        const int j = (int)(row % N);
        T xv[N];
        if (zero) {
#pragma unroll
            for (int i = 0; i < N; ++i) xv[i] = 0;
            store_vec(x, row * N, xv);
        } else {
            load_vec(x, row * N, xv);
            if (pending) {
                T pv[N];
                load_vec(pl, row * N, pv);
#pragma unroll
                for (int i = 0; i < N; ++i) xv[i] += alpha * pv[i];
                store_vec(x, row * N, xv);
            }
        }
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) s += (double)k.w[i] * (double)xv[i];
        part[0] += s * (double)k.w[j] * k.wq;
    }
    double tot[1];
    if (reduce_last<1, kPwThreads>(part, partials, counter, gridDim.x, tot) &&
        threadIdx.x == 0) {
        sc->mean_x = tot[0] / area;
        sc->pending = 0;
    }
}

template <class T>
__global__ __launch_bounds__(kPwThreads) void k_sub_mean(long elems,
                                                         T* __restrict__ x,
                                                         const CgScalars* sc) {
    const T m = (T)sc->mean_x;
    for (long e = blockIdx.x * (long)kPwThreads + threadIdx.x; e < elems;
         e += (long)gridDim.x * kPwThreads)
        x[e] -= m;
}

// (V, E, Omega) with Gauss weights.
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_invariants(
    long rows, OpConst<double> k, const double* __restrict__ omega,
    const double* __restrict__ psi, double* out3, unsigned* counter,
    double* partials) {
    double part[3] = {0.0, 0.0, 0.0};
    for (long row = blockIdx.x * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)gridDim.x * kPwThreads) {
        const int j = (int)(row % N);
        double w[N], p[N];
        load_vec(omega, row * N, w);
        load_vec(psi, row * N, p);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            s0 += k.w[i] * w[i];
            s1 += k.w[i] * (p[i] * w[i]);
            s2 += k.w[i] * (w[i] * w[i]);
        }
        const double wj = k.w[j] * k.wq;
        part[0] += s0 * wj;
        part[1] += s1 * wj;
        part[2] += s2 * wj;
    }
    double tot[3];
    if (reduce_last<3, kPwThreads>(part, partials, counter, gridDim.x, tot) &&
        threadIdx.x == 0) {
        out3[0] = tot[0];
        out3[1] = 0.5 * tot[1];
        out3[2] = 0.5 * tot[2];
    }
}

// psi += e (FP64 accumulate of the FP32 correction, after the inner solve's
// pending update e += alpha p).
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_mixed_update(
    long rows, double* __restrict__ psi, const float* __restrict__ e,
    const float* __restrict__ p0, const float* __restrict__ p1,
    const CgScalars* inner) {
    const int pending = inner->pending;
    const float alpha = (float)inner->alpha;
    const float* pl = (inner->iter & 1) ? p1 : p0;
    for (long row = blockIdx.x * (long)kPwThreads + threadIdx.x; row < rows;
         row += (long)gridDim.x * kPwThreads) {
        float ev[N];
        double pv[N];
        load_vec(e, row * N, ev);
        if (pending) {
            float pp[N];
            load_vec(pl, row * N, pp);
#pragma unroll
            for (int i = 0; i < N; ++i) ev[i] += alpha * pp[i];
        }
        load_vec(psi, row * N, pv);
#pragma unroll
        for (int i = 0; i < N; ++i) pv[i] += (double)ev[i];
        store_vec(psi, row * N, pv);
    }
}

// x = ca pa + cb pb (pointwise)
__global__ __launch_bounds__(kPwThreads) void k_guess(long elems,
                                                      double* __restrict__ x,
                                                      const double* __restrict__ pa,
                                                      const double* __restrict__ pb,
                                                      double ca, double cb) {
    for (long e = blockIdx.x * (long)kPwThreads + threadIdx.x; e < elems;
         e += (long)gridDim.x * kPwThreads) {
        double v = 0.0;
        if (ca != 0.0) v += ca * pa[e];
        if (cb != 0.0) v += cb * pb[e];
        x[e] = v;
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
namespace {

struct CellLaunch {
    int tilesX, tilesY, nblocks;
    explicit CellLaunch(const Geom& g) {
        tilesX = (g.nx + 63) / 64;
        tilesY = (g.ny + kCellWaves - 1) / kCellWaves;
        nblocks = tilesX * tilesY;
    }
};

template <int N, int WAVES>
struct RowLaunch {
    using TL = Tile<N, WAVES>;
    int tilesX, tilesY, nblocks;
    explicit RowLaunch(const Geom& g) {
        tilesX = (g.nx + TL::TX - 1) / TL::TX;
        tilesY = (g.ny + TL::TY - 1) / TL::TY;
        nblocks = tilesX * tilesY;
    }
};

int pw_blocks(long rows, int cap) {
    long b = (rows + kPwThreads - 1) / kPwThreads;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

#define DG_DISPATCH_N(n, ...) \
    switch (n) {              \
        case 1: { constexpr int NN = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int NN = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int NN = 3; __VA_ARGS__; } break; \
        case 4: { constexpr int NN = 4; __VA_ARGS__; } break; \
        case 5: { constexpr int NN = 5; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue; \
    }

}  // namespace

int stencil_blocks(const Geom& g) {
    int rb = 0;
    switch (g.n) {
        case 1: rb = RowLaunch<1, kRowWaves>(g).nblocks; break;
        case 2: rb = RowLaunch<2, kRowWaves>(g).nblocks; break;
        case 3: rb = RowLaunch<3, kRowWaves>(g).nblocks; break;
        case 4: rb = RowLaunch<4, kRowWaves>(g).nblocks; break;
        case 5: rb = RowLaunch<5, kRowWaves>(g).nblocks; break;
        default: return 0;
    }
    const int cb = CellLaunch(g).nblocks;
    return rb > cb ? rb : cb;
}

int pointwise_block_cap() { return 1024; }

hipError_t launch_laplace(const Geom& g, const OpConst<double>& k,
                          const double* u, double* out, hipStream_t s) {
    CellLaunch L(g);
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_laplace<NN>), dim3(L.nblocks),
                                          dim3(64 * kCellWaves), 0, s, g, L.tilesX,
                                          L.nblocks, k, u, out));
    return hipGetLastError();
}

hipError_t launch_rhs(const Geom& g, const OpConst<double>& k, const double* f,
                      const double* gg, const double* wn, double* out,
                      const RhsParams& p, bool visc, hipStream_t s) {
    RhsArgs ra{p.c0, p.c1, p.c2, p.scale, p.D, p.dt, p.a, p.b};
    DG_DISPATCH_N(g.n, {
        RowLaunch<NN, kRowWaves> L(g);
        if (visc)
            hipLaunchKernelGGL((k_rhs<NN, kRowWaves, true>), dim3(L.nblocks),
                               dim3(64 * kRowWaves), 0, s, g, L.tilesX, L.nblocks,
                               k, f, gg, wn, out, ra);
        else
            hipLaunchKernelGGL((k_rhs<NN, kRowWaves, false>), dim3(L.nblocks),
                               dim3(64 * kRowWaves), 0, s, g, L.tilesX, L.nblocks,
                               k, f, gg, wn, out, ra);
    });
    return hipGetLastError();
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

hipError_t launch_cg_init(const Geom& g, const OpConst<double>& k,
                          const double* omega, const double* pa,
                          const double* pb, double ca, double cb, double* x,
                          double* r, const DevScratch& d, hipStream_t s) {
    CellLaunch L(g);
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_init<NN>), dim3(L.nblocks),
                                          dim3(64 * kCellWaves), 0, s, g, L.tilesX,
                                          L.nblocks, k, omega, pa, pb, ca, cb, x, r,
                                          d.sc, d.counters + kCntInit, d.partials));
    return hipGetLastError();
}

template <class T>
hipError_t launch_cg_dir(const Geom& g, const OpConst<T>& k, T* x, T* r, T* p0,
                         T* p1, int parity, CgScalars* sc, const DevScratch& d,
                         hipStream_t s) {
    T* pin = parity ? p1 : p0;
    T* pout = parity ? p0 : p1;
    CellLaunch L(g);
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_dir<NN, T>), dim3(L.nblocks),
                                          dim3(64 * kCellWaves), 0, s, g, L.tilesX,
                                          L.nblocks, k, r, pin, pout, x, sc,
                                          d.counters + kCntDir, d.partials));
    return hipGetLastError();
}

template <class T>
hipError_t launch_cg_res(const Geom& g, const OpConst<T>& k, T* r, T* p0, T* p1,
                         int parity, CgScalars* sc, const DevScratch& d,
                         hipStream_t s) {
    T* pout = parity ? p0 : p1;
    CellLaunch L(g);
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_res<NN, T>), dim3(L.nblocks),
                                          dim3(64 * kCellWaves), 0, s, g, L.tilesX,
                                          L.nblocks, k, pout, r, sc,
                                          d.counters + kCntRes, d.partials));
    return hipGetLastError();
}

template <class T>
hipError_t launch_cg_iter(const Geom& g, const OpConst<T>& k, T* x, T* r,
                          T* p0, T* p1, int parity, CgScalars* sc,
                          const DevScratch& d, hipStream_t s) {
    hipError_t e = launch_cg_dir<T>(g, k, x, r, p0, p1, parity, sc, d, s);
    if (e != hipSuccess) return e;
    return launch_cg_res<T>(g, k, r, p0, p1, parity, sc, d, s);
}

template hipError_t launch_cg_dir<double>(const Geom&, const OpConst<double>&,
                                          double*, double*, double*, double*, int,
                                          CgScalars*, const DevScratch&, hipStream_t);
template hipError_t launch_cg_dir<float>(const Geom&, const OpConst<float>&,
                                         float*, float*, float*, float*, int,
                                         CgScalars*, const DevScratch&, hipStream_t);
template hipError_t launch_cg_res<double>(const Geom&, const OpConst<double>&,
                                          double*, double*, double*, int,
                                          CgScalars*, const DevScratch&, hipStream_t);
template hipError_t launch_cg_res<float>(const Geom&, const OpConst<float>&,
                                         float*, float*, float*, int, CgScalars*,
                                         const DevScratch&, hipStream_t);
template hipError_t launch_cg_iter<double>(const Geom&, const OpConst<double>&,
                                           double*, double*, double*, double*,
                                           int, CgScalars*, const DevScratch&,
                                           hipStream_t);
template hipError_t launch_cg_iter<float>(const Geom&, const OpConst<float>&,
                                          float*, float*, float*, float*, int,
                                          CgScalars*, const DevScratch&,
                                          hipStream_t);

hipError_t launch_cg_finish(const Geom& g, const OpConst<double>& k, double* x,
                            const double* p0, const double* p1, double area,
                            const DevScratch& d, hipStream_t s) {
    const long rows = (long)g.nx * g.ny * g.n;
    const int nb = pw_blocks(rows, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_finish<NN, double>), dim3(nb),
                                          dim3(kPwThreads), 0, s, rows, k, x, p0,
                                          p1, area, d.sc, d.counters + kCntFinish,
                                          d.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sub_mean<double>), dim3(nb), dim3(kPwThreads), 0, s,
                       rows * g.n, x, d.sc);
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

hipError_t launch_mixed_residual(const Geom& g, const OpConst<double>& k,
                                 const double* omega, const double* psi,
                                 float* r32, float* e32, double inner_tol2,
                                 int inner_max, CgScalars* outer,
                                 CgScalars* inner, const DevScratch& d,
                                 hipStream_t s) {
    CellLaunch L(g);
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_mixed_residual<NN>), dim3(L.nblocks),
                                          dim3(64 * kCellWaves), 0, s, g, L.tilesX,
                                          L.nblocks, k, omega, psi, r32, e32,
                                          inner_tol2, inner_max, outer, inner,
                                          d.counters + kCntDot, d.partials));
    return hipGetLastError();
}

hipError_t launch_mixed_update(const Geom& g, double* psi, const float* e,
                               const float* p0, const float* p1,
                               const CgScalars* inner, hipStream_t s) {
    const long rows = (long)g.nx * g.ny * g.n;
    const int nb = pw_blocks(rows, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_mixed_update<NN>), dim3(nb),
                                          dim3(kPwThreads), 0, s, rows, psi, e,
                                          p0, p1, inner));
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

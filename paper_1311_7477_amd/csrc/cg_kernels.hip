// Single-instance launches of the LDG Laplacian and CG kernels (cell per
// lane; the device code and its layout conventions are in cg_body.h).  One
// block per 64 x WV tile (WV = the grid's cell tile height g.cw, one of 4, 8,
// 16); block b processes tile xcd_tile(b).
#include <hip/hip_ext.h>

#include <type_traits>

#include "cg_body.h"
#include "dg_launch.h"

namespace dgk {

template <int N, int WV, bool DIR, bool ISO>
__global__ __launch_bounds__(64 * WV) void k_laplace(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ u, double* __restrict__ out) {
    __shared__ YFaces<N, double, WV> lds;
    laplace_body<N, WV, DIR, ISO>(blockIdx.x, g, tilesX, nblocks, k, u, out, lds);
}

template <int N, int WV, bool DIR, bool ISO>
__global__ __launch_bounds__(64 * WV) void k_cg_init(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ omega, const double* __restrict__ pa,
    const double* __restrict__ pb, double ca, double cb,
    double* __restrict__ x, double* __restrict__ r, CgScalars* sc,
    unsigned* counter, double* partials) {
    __shared__ YFaces<N, double, WV> lds;
    cg_init_body<N, WV, DIR, ISO>(blockIdx.x, g, tilesX, nblocks, k, omega, pa, pb, ca, cb, x,
                             r, sc, counter, partials, lds);
}

// At n = 4 the periodic direction and residual kernels are held to 128
// VGPRs (four waves per SIMD): with the paired 16-byte accesses they would
// take 132 / 134 and drop to three, which costs more than the 20 bytes per
// lane the residual kernel then spills.
template <int N, class S, int WV, bool DIR, bool ISO>
__global__ __launch_bounds__(64 * WV, (N == 4 && !DIR) ? 4 : 1) void k_cg_dir(
    Geom g, int tilesX, int nblocks, OpConst<double> k, const S* __restrict__ r,
    S* p0, S* p1, double* __restrict__ x, CgScalars* sc, unsigned* counter,
    double* partials) {
    __shared__ YFaces<N, double, WV> lds;
    cg_dir_body<N, S, WV, DIR, ISO>(blockIdx.x, g, tilesX, nblocks, k, r, p0, p1, x, sc,
                               counter, partials, lds);
}

template <int N, class S, int WV, bool DIR, bool ISO>
__global__ __launch_bounds__(64 * WV, (N == 4 && !DIR) ? 4 : 1) void k_cg_res(
    Geom g, int tilesX, int nblocks, OpConst<double> k, const S* p0, const S* p1,
    S* __restrict__ r, CgScalars* sc, unsigned* counter, double* partials) {
    __shared__ YFaces<N, double, WV> lds;
    cg_res_body<N, S, WV, DIR, ISO>(blockIdx.x, g, tilesX, nblocks, k, p0, p1, r, sc, counter,
                               partials, lds);
}

template <int N, int WV, bool ISO>
__global__ __launch_bounds__(64 * WV) void k_mixed_replace(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ omega, const double* __restrict__ x,
    const float* __restrict__ q0, const float* __restrict__ q1,
    float* __restrict__ r32, CgScalars* sc, unsigned* counter, double* partials) {
    __shared__ YFaces<N, double, WV> lds;
    mixed_replace_body<N, WV, ISO>(blockIdx.x, g, tilesX, nblocks, k, omega, x, q0, q1, r32,
                          sc, counter, partials, lds);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int cell_blocks(const Geom& g) { return CellLaunch(g).nblocks; }

// A grid with a homogeneous Dirichlet axis runs the DIR variants, built for
// 64 x 8 cell tiles only; square cells with the same boundary kind on both
// axes run the ISO variants (identical x and y blocks).
bool dirichlet(const Geom& g) { return g.bcx || g.bcy; }
bool iso(const Geom& g, const OpConst<double>& k) { return !dirichlet(g) && k.ihx == k.ihy; }
bool iso_dir(const Geom& g, const OpConst<double>& k) {
    return g.bcx && g.bcy && k.ihx == k.ihy;
}

hipError_t launch_laplace(const Geom& g, const OpConst<double>& k,
                          const double* u, double* out, hipStream_t s) {
    CellLaunch L(g);
    if (dirichlet(g)) {
        if (g.cw != kDirichletCellWaves) return hipErrorInvalidValue;
        if (iso_dir(g, k)) {
            DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_laplace<NN, kDirichletCellWaves, true, true>),
                                                  dim3(L.nblocks), dim3(64 * kDirichletCellWaves),
                                                  0, s, g, L.tilesX, L.nblocks, k, u, out));
        } else {
            DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_laplace<NN, kDirichletCellWaves, true, false>),
                                                  dim3(L.nblocks), dim3(64 * kDirichletCellWaves),
                                                  0, s, g, L.tilesX, L.nblocks, k, u, out));
        }
        return hipGetLastError();
    }
    if (iso(g, k)) {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_laplace<NN, WW, false, true>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, u, out));
    } else {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_laplace<NN, WW, false, false>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, u, out));
    }
    return hipGetLastError();
}

hipError_t launch_cg_init(const Geom& g, const OpConst<double>& k,
                          const double* omega, const double* pa,
                          const double* pb, double ca, double cb, double* x,
                          double* r, const DevScratch& d, hipStream_t s) {
    CellLaunch L(g);
    if (dirichlet(g)) {
        if (g.cw != kDirichletCellWaves) return hipErrorInvalidValue;
        if (iso_dir(g, k)) {
            DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_init<NN, kDirichletCellWaves, true, true>),
                                                  dim3(L.nblocks), dim3(64 * kDirichletCellWaves),
                                                  0, s, g, L.tilesX, L.nblocks, k, omega, pa, pb,
                                                  ca, cb, x, r, d.sc, d.counters + kCntInit * kCntStride,
                                                  d.partials));
        } else {
            DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_init<NN, kDirichletCellWaves, true, false>),
                                                  dim3(L.nblocks), dim3(64 * kDirichletCellWaves),
                                                  0, s, g, L.tilesX, L.nblocks, k, omega, pa, pb,
                                                  ca, cb, x, r, d.sc, d.counters + kCntInit * kCntStride,
                                                  d.partials));
        }
        return hipGetLastError();
    }
    if (iso(g, k)) {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_cg_init<NN, WW, false, true>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, omega, pa, pb, ca, cb, x, r,
                                              d.sc, d.counters + kCntInit * kCntStride, d.partials));
    } else {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_cg_init<NN, WW, false, false>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, omega, pa, pb, ca, cb, x, r,
                                              d.sc, d.counters + kCntInit * kCntStride, d.partials));
    }
    return hipGetLastError();
}

template <class S>
hipError_t launch_cg_dir(const Geom& g, const OpConst<double>& k, double* x, S* r, S* p0,
                         S* p1, CgScalars* sc, const DevScratch& d, hipStream_t s) {
    CellLaunch L(g);
    if (dirichlet(g)) {
        if constexpr (std::is_same<S, double>::value) {
            if (g.cw != kDirichletCellWaves) return hipErrorInvalidValue;
            if (iso_dir(g, k)) {
                DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_dir<NN, S, kDirichletCellWaves, true, true>),
                                                      dim3(L.nblocks),
                                                      dim3(64 * kDirichletCellWaves), 0, s, g,
                                                      L.tilesX, L.nblocks, k, r, p0, p1, x, sc,
                                                      d.counters + kCntDir * kCntStride, d.partials));
            } else {
                DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_dir<NN, S, kDirichletCellWaves, true, false>),
                                                      dim3(L.nblocks),
                                                      dim3(64 * kDirichletCellWaves), 0, s, g,
                                                      L.tilesX, L.nblocks, k, r, p0, p1, x, sc,
                                                      d.counters + kCntDir * kCntStride, d.partials));
            }
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (iso(g, k)) {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_cg_dir<NN, S, WW, false, true>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, r, p0, p1, x, sc,
                                              d.counters + kCntDir * kCntStride, d.partials));
    } else {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_cg_dir<NN, S, WW, false, false>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, r, p0, p1, x, sc,
                                              d.counters + kCntDir * kCntStride, d.partials));
    }
    return hipGetLastError();
}

template <class S>
hipError_t launch_cg_res(const Geom& g, const OpConst<double>& k, S* r, S* p0, S* p1,
                         CgScalars* sc, const DevScratch& d, hipStream_t s) {
    CellLaunch L(g);
    if (dirichlet(g)) {
        if constexpr (std::is_same<S, double>::value) {
            if (g.cw != kDirichletCellWaves) return hipErrorInvalidValue;
            if (iso_dir(g, k)) {
                DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_res<NN, S, kDirichletCellWaves, true, true>),
                                                      dim3(L.nblocks),
                                                      dim3(64 * kDirichletCellWaves), 0, s, g,
                                                      L.tilesX, L.nblocks, k, p0, p1, r, sc,
                                                      d.counters + kCntRes * kCntStride, d.partials));
            } else {
                DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_res<NN, S, kDirichletCellWaves, true, false>),
                                                      dim3(L.nblocks),
                                                      dim3(64 * kDirichletCellWaves), 0, s, g,
                                                      L.tilesX, L.nblocks, k, p0, p1, r, sc,
                                                      d.counters + kCntRes * kCntStride, d.partials));
            }
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (iso(g, k)) {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_cg_res<NN, S, WW, false, true>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, p0, p1, r, sc,
                                              d.counters + kCntRes * kCntStride, d.partials));
    } else {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_cg_res<NN, S, WW, false, false>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, p0, p1, r, sc,
                                              d.counters + kCntRes * kCntStride, d.partials));
    }
    return hipGetLastError();
}

// The same launches with the dispatch's own start / stop timestamps
// (hipExtLaunchKernel): the events bracket exactly this kernel, without the
// cost of separate marker packets around it.
template <class S>
hipError_t launch_cg_dir_timed(const Geom& g, const OpConst<double>& k, double* x, S* r,
                               S* p0, S* p1, CgScalars* sc, const DevScratch& d,
                               hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    CellLaunch L(g);
    if (dirichlet(g)) return hipErrorInvalidValue;
    if (iso(g, k)) {
        DG_DISPATCH_NW(g.n, g.cw, hipExtLaunchKernelGGL((k_cg_dir<NN, S, WW, false, true>),
                                                        dim3(L.nblocks),
                                                        dim3(64 * WW), 0, s, start, stop, 0, g,
                                                        L.tilesX, L.nblocks, k, (const S*)r, p0,
                                                        p1, x, sc, d.counters + kCntDir * kCntStride,
                                                        d.partials));
    } else {
        DG_DISPATCH_NW(g.n, g.cw, hipExtLaunchKernelGGL((k_cg_dir<NN, S, WW, false, false>),
                                                        dim3(L.nblocks),
                                                        dim3(64 * WW), 0, s, start, stop, 0, g,
                                                        L.tilesX, L.nblocks, k, (const S*)r, p0,
                                                        p1, x, sc, d.counters + kCntDir * kCntStride,
                                                        d.partials));
    }
    return hipGetLastError();
}

template <class S>
hipError_t launch_cg_res_timed(const Geom& g, const OpConst<double>& k, S* r, S* p0, S* p1,
                               CgScalars* sc, const DevScratch& d, hipStream_t s,
                               hipEvent_t start, hipEvent_t stop) {
    CellLaunch L(g);
    if (dirichlet(g)) return hipErrorInvalidValue;
    if (iso(g, k)) {
        DG_DISPATCH_NW(g.n, g.cw, hipExtLaunchKernelGGL((k_cg_res<NN, S, WW, false, true>),
                                                        dim3(L.nblocks),
                                                        dim3(64 * WW), 0, s, start, stop, 0, g,
                                                        L.tilesX, L.nblocks, k, (const S*)p0,
                                                        (const S*)p1, r, sc, d.counters + kCntRes * kCntStride,
                                                        d.partials));
    } else {
        DG_DISPATCH_NW(g.n, g.cw, hipExtLaunchKernelGGL((k_cg_res<NN, S, WW, false, false>),
                                                        dim3(L.nblocks),
                                                        dim3(64 * WW), 0, s, start, stop, 0, g,
                                                        L.tilesX, L.nblocks, k, (const S*)p0,
                                                        (const S*)p1, r, sc, d.counters + kCntRes * kCntStride,
                                                        d.partials));
    }
    return hipGetLastError();
}
template hipError_t launch_cg_dir_timed<double>(const Geom&, const OpConst<double>&, double*,
                                                double*, double*, double*, CgScalars*,
                                                const DevScratch&, hipStream_t, hipEvent_t,
                                                hipEvent_t);
template hipError_t launch_cg_res_timed<double>(const Geom&, const OpConst<double>&, double*,
                                                double*, double*, CgScalars*,
                                                const DevScratch&, hipStream_t, hipEvent_t,
                                                hipEvent_t);

template <class S>
hipError_t launch_cg_iter(const Geom& g, const OpConst<double>& k, double* x, S* r,
                          S* p0, S* p1, CgScalars* sc, const DevScratch& d,
                          hipStream_t s) {
    hipError_t e = launch_cg_dir<S>(g, k, x, r, p0, p1, sc, d, s);
    if (e != hipSuccess) return e;
    return launch_cg_res<S>(g, k, r, p0, p1, sc, d, s);
}

#define DG_INST(S)                                                             \
    template hipError_t launch_cg_dir<S>(const Geom&, const OpConst<double>&,   \
                                         double*, S*, S*, S*, CgScalars*,       \
                                         const DevScratch&, hipStream_t);       \
    template hipError_t launch_cg_res<S>(const Geom&, const OpConst<double>&, S*, \
                                         S*, S*, CgScalars*, const DevScratch&, \
                                         hipStream_t);                          \
    template hipError_t launch_cg_iter<S>(const Geom&, const OpConst<double>&,  \
                                          double*, S*, S*, S*, CgScalars*,      \
                                          const DevScratch&, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

hipError_t launch_mixed_replace(const Geom& g, const OpConst<double>& k,
                                const double* omega, const double* x, const float* q0,
                                const float* q1, float* r32, const DevScratch& d,
                                hipStream_t s) {
    CellLaunch L(g);
    if (dirichlet(g)) return hipErrorInvalidValue;
    if (iso(g, k)) {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_mixed_replace<NN, WW, true>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, omega, x, q0, q1, r32,
                                              d.sc, d.counters + kCntDot * kCntStride, d.partials));
    } else {
        DG_DISPATCH_NW(g.n, g.cw, hipLaunchKernelGGL((k_mixed_replace<NN, WW, false>),
                                                     dim3(L.nblocks),
                                              dim3(64 * WW), 0, s, g, L.tilesX,
                                              L.nblocks, k, omega, x, q0, q1, r32,
                                              d.sc, d.counters + kCntDot * kCntStride, d.partials));
    }
    return hipGetLastError();
}

}  // namespace dgk

// Single-instance launches of the pointwise kernels (device code in
// pw_body.h): grid-stride loops, block b of nb.
#include "dg_launch.h"
#include "pw_body.h"

namespace dgk {

template <int N>
__global__ __launch_bounds__(kPwThreads) void k_cg_mean(
    long rows, OpConst<double> k, const double* __restrict__ omega,
    const double* __restrict__ pa, const double* __restrict__ pb, double ca,
    double cb, double area, double tol2, int max_iter, int dir, CgScalars* sc,
    unsigned* counter, double* partials) {
    cg_mean_body<N>(blockIdx.x, gridDim.x, rows, k, omega, pa, pb, ca, cb, area,
                    tol2, max_iter, dir, sc, counter, partials);
}

template <int N, class P>
__global__ __launch_bounds__(kPwThreads) void k_cg_finish(
    Geom g, OpConst<double> k, const double* __restrict__ x,
    const P* __restrict__ p0, const P* __restrict__ p1,
    double* __restrict__ psi, double area, CgScalars* sc, unsigned* counter,
    double* partials) {
    cg_finish_body<N, P>(blockIdx.x, gridDim.x, g, k, x, p0, p1, psi, area, sc,
                      counter, partials);
}

template <int N>
__global__ __launch_bounds__(kPwThreads) void k_mean_canon(
    long rows, OpConst<double> k, const double* __restrict__ f, double area,
    CgScalars* sc, unsigned* counter, double* partials) {
    mean_canon_body<N>(blockIdx.x, gridDim.x, rows, k, f, area, sc, counter,
                       partials);
}

__global__ __launch_bounds__(kPwThreads) void k_sub_mean(long elems,
                                                         double* __restrict__ x,
                                                         const CgScalars* sc) {
    sub_mean_body(blockIdx.x, gridDim.x, elems, x, sc);
}

template <int N>
__global__ __launch_bounds__(kPwThreads) void k_invariants(
    long rows, OpConst<double> k, const double* __restrict__ omega,
    const double* __restrict__ psi, double* out3, unsigned* counter,
    double* partials) {
    invariants_body<N>(blockIdx.x, gridDim.x, rows, k, omega, psi, out3, counter,
                       partials);
}

template <int N>
__global__ __launch_bounds__(kPwThreads) void k_mixed_start(
    Geom g, OpConst<double> k, const double* __restrict__ r64,
    float* __restrict__ r32, CgScalars* sc, unsigned* counter, double* partials) {
    mixed_start_body<N>(blockIdx.x, gridDim.x, g, k, r64, r32, sc, counter, partials);
}

__global__ __launch_bounds__(kPwThreads) void k_ab_combine(
    long elems, double* __restrict__ omega, const double* r0, const double* r1,
    const double* r2, const double* r3, double c0, double c1, double c2, double c3,
    int K) {
    ab_combine_body(blockIdx.x, gridDim.x, elems, omega, r0, r1, r2, r3, c0, c1, c2, c3, K);
}

__global__ __launch_bounds__(kPwThreads) void k_guess(long elems,
                                                      double* __restrict__ x,
                                                      const double* pa,
                                                      const double* pb,
                                                      double ca, double cb) {
    guess_body(blockIdx.x, gridDim.x, elems, x, pa, pb, ca, cb);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int pointwise_block_cap() { return 1024; }

int stencil_blocks(const Geom& g) {
    // the most blocks any tile shape of this grid can launch (cell tiles of
    // 4 waves, bracket tiles of 8), so a workspace sized once serves every
    // shape the tuner may choose later
    Geom w = g;
    w.cw = 4;
    w.rw = 8;
    const int a = row_blocks(w), b = cell_blocks(w);
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
                                          (g.bcx || g.bcy) ? 1 : 0, d.sc,
                                          d.counters + kCntMean * kCntStride, d.partials));
    return hipGetLastError();
}

template <class P>
hipError_t launch_cg_finish(const Geom& g, const OpConst<double>& k,
                            const double* x, const P* p0, const P* p1,
                            double* psi, double area, const DevScratch& d,
                            hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_cg_finish<NN, P>), dim3(nb),
                                          dim3(kPwThreads), 0, s, g, k, x, p0, p1,
                                          psi, area, d.sc, d.counters + kCntFinish * kCntStride,
                                          d.partials));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.bcx || g.bcy) return hipSuccess;   // definite operator: psi keeps its mean
    const long elems = cells * g.n * g.n;
    hipLaunchKernelGGL(k_sub_mean, dim3(pw_blocks(elems, pointwise_block_cap())),
                       dim3(kPwThreads), 0, s, elems, psi, d.sc);
    return hipGetLastError();
}
template hipError_t launch_cg_finish<double>(const Geom&, const OpConst<double>&,
                                             const double*, const double*, const double*,
                                             double*, double, const DevScratch&, hipStream_t);
template hipError_t launch_cg_finish<float>(const Geom&, const OpConst<double>&,
                                            const double*, const float*, const float*,
                                            double*, double, const DevScratch&, hipStream_t);

hipError_t launch_mean_sub(const Geom& g, const OpConst<double>& k, double* x,
                           double area, const DevScratch& d, hipStream_t s) {
    const long rows = (long)g.nx * g.ny * g.n;
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_mean_canon<NN>),
                                          dim3(pw_blocks(rows, pointwise_block_cap())),
                                          dim3(kPwThreads), 0, s, rows, k, x, area,
                                          d.sc, d.counters + kCntFinish * kCntStride, d.partials));
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
                                          psi, out3, d.counters + kCntInv * kCntStride,
                                          d.partials));
    return hipGetLastError();
}

hipError_t launch_mixed_start(const Geom& g, const OpConst<double>& k,
                              const double* r64, float* r32, const DevScratch& d,
                              hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_mixed_start<NN>), dim3(nb),
                                          dim3(kPwThreads), 0, s, g, k, r64, r32,
                                          d.sc, d.counters + kCntMean * kCntStride, d.partials));
    return hipGetLastError();
}

hipError_t launch_ab_combine(long elems, double* omega, const double* const* R,
                             const double* c, int K, hipStream_t s) {
    if (K < 1 || K > 4) return hipErrorInvalidValue;
    const int nb = pw_blocks(elems, pointwise_block_cap());
    hipLaunchKernelGGL(k_ab_combine, dim3(nb), dim3(kPwThreads), 0, s, elems, omega, R[0],
                       K > 1 ? R[1] : R[0], K > 2 ? R[2] : R[0], K > 3 ? R[3] : R[0], c[0],
                       K > 1 ? c[1] : 0.0, K > 2 ? c[2] : 0.0, K > 3 ? c[3] : 0.0, K);
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

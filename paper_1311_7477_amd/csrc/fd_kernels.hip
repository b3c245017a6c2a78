// Device kernels of the fast-diagonalisation preconditioner: conversions
// between the CG layouts and the image layout U[(cy n + j) * NX + cx n + i]
// (NX = nx n) that the dense basis products act on, the spectral scaling,
// and the preconditioned dot product <r, z>_W that closes the PCG step.
#include "cg_body.h"
#include "dg_launch.h"

namespace dgk {

namespace {

// Image offset of node (j, i) = 0 of cell (cx, cy).
__device__ __forceinline__ long img_base(int n, long NX, int cx, int cy) {
    return (long)cy * n * NX + (long)cx * n;
}

template <int N, bool FromL64>
__global__ __launch_bounds__(kPwThreads) void k_to_image(Geom g, const double* __restrict__ src,
                                                         double* __restrict__ img) {
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    const long NX = (long)g.nx * N;
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const CellRef c = cell_ref<N>(g, G, cx, cy);
        double u[N * N];
        if (FromL64) ld_l64<N>(src, c, u);
        else ld_canon<N>(src, c, u);
        const long o = img_base(N, NX, cx, cy);
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) img[o + j * NX + i] = u[j * N + i];
    }
}

template <int N>
__global__ __launch_bounds__(kPwThreads) void k_from_image(Geom g, const double* __restrict__ img,
                                                           double* __restrict__ dst) {
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    const long NX = (long)g.nx * N;
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const CellRef c = cell_ref<N>(g, G, cx, cy);
        const long o = img_base(N, NX, cx, cy);
        double u[N * N];
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) u[j * N + i] = img[o + j * NX + i];
        st_canon<N>(dst, c, u);
    }
}

// z = image (to L64) and <r, z>_W; the last block sets rz and, past the
// first iteration, beta = <r,z>_new / <r,z>_old (no-op once the solve is
// done; a non-positive or non-finite <r,z> ends the solve as a breakdown).
template <int N>
__global__ __launch_bounds__(kPwThreads) void k_from_image_dot(
    Geom g, OpConst<double> k, const double* __restrict__ img, double* __restrict__ z,
    const double* __restrict__ r, CgScalars* sc, unsigned* counter, double* partials) {
    if (sc->done) return;
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    const long NX = (long)g.nx * N;
    double part[1] = {0.0};
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const CellRef c = cell_ref<N>(g, G, cx, cy);
        const long o = img_base(N, NX, cx, cy);
        double u[N * N], rv[N * N];
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) u[j * N + i] = img[o + j * NX + i];
        st_l64<N>(z, c, u);
        ld_l64<N>(r, c, rv);
        part[0] += wdot_cell<N>(k, rv, u);
    }
    double tot[1];
    if (reduce_last<1, kPwThreads>(part, partials, counter, gridDim.x, blockIdx.x, tot) &&
        threadIdx.x == 0) {
        sc->precond = 1;
        const double rz = tot[0];
        if (!(rz > 0.0) || !(rz < __builtin_inf())) {
            // <r, M r> must be positive and finite for a nonzero residual:
            // stop; x still lacks the last alpha p (after any iteration)
            sc->done = 1;
            sc->breakdown = 1;
            sc->pending = sc->first != 1;
        } else {
            if (sc->first != 1) sc->beta = rz / sc->rz;
            sc->rz = rz;
        }
    }
}

// U[r][c] /= -(ly[r] + lx[c]); the constant mode (zy, zx) is set to zero.
__global__ __launch_bounds__(kPwThreads) void k_fd_scale(int NX, int NY, double* __restrict__ img,
                                                         const double* __restrict__ lx,
                                                         const double* __restrict__ ly, int zx,
                                                         int zy) {
    const long total = (long)NX * NY;
    for (long e = blockIdx.x * (long)kPwThreads + threadIdx.x; e < total;
         e += (long)gridDim.x * kPwThreads) {
        const int r = (int)(e / NX), c = (int)(e - (long)r * NX);
        const double mu = -(ly[r] + lx[c]);
        img[e] = (r == zy && c == zx) ? 0.0 : img[e] / mu;
    }
}

}  // namespace

hipError_t launch_to_image(const Geom& g, const double* src, bool from_l64, double* img,
                           hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    if (from_l64) {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_to_image<NN, true>), dim3(nb), dim3(kPwThreads),
                                              0, s, g, src, img));
    } else {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_to_image<NN, false>), dim3(nb), dim3(kPwThreads),
                                              0, s, g, src, img));
    }
    return hipGetLastError();
}

hipError_t launch_from_image(const Geom& g, const double* img, double* dst, hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_image<NN>), dim3(nb), dim3(kPwThreads), 0, s, g,
                                          img, dst));
    return hipGetLastError();
}

hipError_t launch_from_image_dot(const Geom& g, const OpConst<double>& k, const double* img,
                                 double* z, const double* r, const DevScratch& d, hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_image_dot<NN>), dim3(nb), dim3(kPwThreads), 0,
                                          s, g, k, img, z, r, d.sc, d.counters + kCntDot,
                                          d.partials));
    return hipGetLastError();
}

hipError_t launch_fd_scale(int NX, int NY, double* img, const double* lx, const double* ly,
                           int zx, int zy, hipStream_t s) {
    const long total = (long)NX * NY;
    const int nb = pw_blocks(total, pointwise_block_cap());
    hipLaunchKernelGGL(k_fd_scale, dim3(nb), dim3(kPwThreads), 0, s, NX, NY, img, lx, ly, zx, zy);
    return hipGetLastError();
}

}  // namespace dgk

// Single-instance launch of the fused bracket / right-hand-side kernel (row
// per lane; the device code is in rhs_body.h).
#include "dg_launch.h"
#include "rhs_body.h"

namespace dgk {

template <int N, int WAVES, bool VISC>
__global__ __launch_bounds__(64 * WAVES) void k_rhs(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ f, const double* __restrict__ gg,
    const double* __restrict__ wn, double* __restrict__ out, RhsArgs ra) {
    __shared__ RhsLds<N, WAVES, VISC> lds;
    rhs_body<N, WAVES, VISC>(blockIdx.x, g, tilesX, nblocks, k, f, gg, wn, out,
                             ra, lds);
}

int row_blocks(const Geom& g) {
    switch (g.n) {
        case 1: return RowLaunch<1, kRowWaves>(g).nblocks;
        case 2: return RowLaunch<2, kRowWaves>(g).nblocks;
        case 3: return RowLaunch<3, kRowWaves>(g).nblocks;
        case 4: return RowLaunch<4, kRowWaves>(g).nblocks;
        case 5: return RowLaunch<5, kRowWaves>(g).nblocks;
        default: return 0;
    }
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

}  // namespace dgk

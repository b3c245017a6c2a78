// Single-instance launch of the fused bracket / right-hand-side kernel (row
// per lane; the device code is in rhs_body.h).
#include "dg_launch.h"
#include "rhs_body.h"

namespace dgk {

template <int N, int WAVES, bool VISC, bool DIR>
__global__ __launch_bounds__(64 * WAVES, 4) void k_rhs(
    Geom g, int tilesX, int nblocks, OpConst<double> k,
    const double* __restrict__ f, const double* __restrict__ gg,
    const double* __restrict__ wn, double* __restrict__ out, RhsArgs ra) {
    __shared__ RhsLds<N, WAVES, VISC> lds;
    rhs_body<N, WAVES, VISC, DIR>(blockIdx.x, g, tilesX, nblocks, k, f, gg, wn, out,
                                  ra, lds);
}

int row_blocks(const Geom& g) { return RowLaunch(g).nblocks; }

hipError_t launch_rhs(const Geom& g, const OpConst<double>& k, const double* f,
                      const double* gg, const double* wn, double* out,
                      const RhsParams& p, bool visc, hipStream_t s) {
    RhsArgs ra{p.c0, p.c1, p.c2, p.scale, p.D, p.dt, p.a, p.b, p.only_r};
    DG_DISPATCH_NR(g.n, g.rw, {
        RowLaunch L(g);
        // a Dirichlet axis takes the variants with the boundary faces
        // compiled in (the bracket's zero flux, the viscous term's LDG closure)
        if (visc && (g.bcx || g.bcy))
            hipLaunchKernelGGL((k_rhs<NN, WW, true, true>), dim3(L.nblocks), dim3(64 * WW), 0,
                               s, g, L.tilesX, L.nblocks, k, f, gg, wn, out, ra);
        else if (visc)
            hipLaunchKernelGGL((k_rhs<NN, WW, true, false>), dim3(L.nblocks), dim3(64 * WW), 0,
                               s, g, L.tilesX, L.nblocks, k, f, gg, wn, out, ra);
        else if (g.bcx || g.bcy)
            hipLaunchKernelGGL((k_rhs<NN, WW, false, true>), dim3(L.nblocks), dim3(64 * WW), 0,
                               s, g, L.tilesX, L.nblocks, k, f, gg, wn, out, ra);
        else
            hipLaunchKernelGGL((k_rhs<NN, WW, false, false>), dim3(L.nblocks), dim3(64 * WW),
                               0, s, g, L.tilesX, L.nblocks, k, f, gg, wn, out, ra);
    });
    return hipGetLastError();
}

}  // namespace dgk

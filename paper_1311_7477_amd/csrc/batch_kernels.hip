// Batched launches: many independent instances (any grid sizes; one
// polynomial order and one tile shape per launch) in one launch per kernel
// kind, one block per work item.  Every instance is described by a BatchInst
// record in device memory and cut into the same blocks as its
// single-instance launch; the work list holds (instance, local block index)
// items.  Each item runs the
// very same device body as the single-instance kernel with the same local
// block index, so an instance's arithmetic and reduction order -- and hence
// its result, bit for bit -- do not depend on what else is in the batch.
// Parameters that change between RK stages live in the records, so one
// captured graph serves every stage.
#include "batch.h"
#include "dg_launch.h"
#include "cg_body.h"
#include "pw_body.h"
#include "rhs_body.h"

namespace dgk {

// Block b runs item b of this launch's list (the launch has one block per
// item); the per-item early exits of the bodies are uniform per block.  One
// item per block rather than a grid-stride loop: the loop kept the records'
// values live across iterations (157 instead of 134 VGPRs for the n = 4
// direction kernel).
#define DG_FOR_ITEMS(list)                                                   \
    if (const int it_ = blockIdx.x; it_ < *(list).count)                     \
        if (const BatchItem item_ = (list).items[it_]; true)                 \
            if (const BatchInst& B = inst[item_.inst]; B.active)

template <int N>
__global__ __launch_bounds__(kPwThreads) void kb_cg_mean(const BatchInst* __restrict__ inst,
                                                         ItemList list) {
    DG_FOR_ITEMS(list) {
        cg_mean_body<N>(item_.b, B.nb_rows, B.rows, B.k, B.w_in, B.pa, B.pb,
                        B.ca, B.cb, B.area, B.tol2, B.max_iter, 0, B.sc,
                        B.counters + kCntMean * kCntStride, B.partials);
    }
}

template <int N, int WV>
__global__ __launch_bounds__(64 * WV, (N <= 4 ? 4 : 1)) void kb_cg_init(const BatchInst* __restrict__ inst, ItemList list) {
    __shared__ YFaces<N, double, WV> lds;
    DG_FOR_ITEMS(list) {
        cg_init_body<N, WV>(item_.b, B.g, B.cell_tilesX, B.cell_nblocks, B.k, B.w_in,
                        B.pa, B.pb, B.ca, B.cb, B.x, B.r, B.sc,
                        B.counters + kCntInit * kCntStride, B.partials, lds);
    }
}

template <int N, int WV>
__global__ __launch_bounds__(64 * WV, (N <= 4 ? 4 : 1)) void kb_cg_dir(const BatchInst* __restrict__ inst, ItemList list) {
    __shared__ YFaces<N, double, WV> lds;
    DG_FOR_ITEMS(list) {
        cg_dir_body<N, double, WV>(item_.b, B.g, B.cell_tilesX, B.cell_nblocks, B.k,
                               B.r, B.p0, B.p1, B.x, B.sc, B.counters + kCntDir * kCntStride, B.partials, lds);
    }
}

template <int N, int WV>
__global__ __launch_bounds__(64 * WV, (N <= 4 ? 4 : 1)) void kb_cg_res(const BatchInst* __restrict__ inst, ItemList list) {
    __shared__ YFaces<N, double, WV> lds;
    DG_FOR_ITEMS(list) {
        cg_res_body<N, double, WV>(item_.b, B.g, B.cell_tilesX, B.cell_nblocks, B.k,
                               B.p0, B.p1, B.r, B.sc,
                               B.counters + kCntRes * kCntStride, B.partials, lds);
    }
}

template <int N>
__global__ __launch_bounds__(kPwThreads) void kb_cg_finish(const BatchInst* __restrict__ inst,
                                                           ItemList list) {
    DG_FOR_ITEMS(list) {
        cg_finish_body<N>(item_.b, B.nb_cells, B.g, B.k, B.x, B.p0, B.p1, B.psi,
                          B.area, B.sc, B.counters + kCntFinish * kCntStride, B.partials);
    }
}

__global__ __launch_bounds__(kPwThreads) void kb_sub_mean(const BatchInst* __restrict__ inst,
                                                          ItemList list) {
    DG_FOR_ITEMS(list) {
        sub_mean_body(item_.b, B.nb_elems, B.elems, B.psi, B.sc);
    }
}

template <int N, int W>
__global__ __launch_bounds__(64 * W, 4) void kb_rhs(const BatchInst* __restrict__ inst, ItemList list) {
    __shared__ RhsLds<N, W, true> lds;
    DG_FOR_ITEMS(list) {
        rhs_body<N, W, true>(item_.b, B.g, B.row_tilesX, B.row_nblocks,
                                     B.k, B.psi, B.w_in, B.w_n, B.w_out, B.ra, lds);
    }
}

#undef DG_FOR_ITEMS

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
void fill_batch_geometry(BatchInst& b) {
    const Geom& g = b.g;
    CellLaunch cl(g);
    b.cell_tilesX = cl.tilesX;
    b.cell_nblocks = cl.nblocks;
    RowLaunch rl(g);
    b.row_tilesX = rl.tilesX;
    b.row_nblocks = rl.nblocks;
    b.cells = (long)g.nx * g.ny;
    b.rows = b.cells * g.n;
    b.elems = b.rows * g.n;
    b.nb_rows = pw_blocks(b.rows, pointwise_block_cap());
    b.nb_cells = pw_blocks(b.cells, pointwise_block_cap());
    b.nb_elems = pw_blocks(b.elems, pointwise_block_cap());
}

hipError_t launch_batch(int n, int cw, int rw, BatchKernel kind, const BatchInst* inst,
                        const ItemList& list, int grid, hipStream_t s) {
    const dim3 pw(kPwThreads);
    switch (kind) {
        case BatchKernel::Mean:
            DG_DISPATCH_N(n, hipLaunchKernelGGL((kb_cg_mean<NN>), dim3(grid), pw, 0, s, inst, list));
            break;
        case BatchKernel::Init:
            DG_DISPATCH_NW(n, cw, hipLaunchKernelGGL((kb_cg_init<NN, WW>), dim3(grid),
                                                     dim3(64 * WW), 0, s, inst, list));
            break;
        case BatchKernel::Dir:
            DG_DISPATCH_NW(n, cw, hipLaunchKernelGGL((kb_cg_dir<NN, WW>), dim3(grid),
                                                     dim3(64 * WW), 0, s, inst, list));
            break;
        case BatchKernel::Res:
            DG_DISPATCH_NW(n, cw, hipLaunchKernelGGL((kb_cg_res<NN, WW>), dim3(grid),
                                                     dim3(64 * WW), 0, s, inst, list));
            break;
        case BatchKernel::Finish:
            DG_DISPATCH_N(n, hipLaunchKernelGGL((kb_cg_finish<NN>), dim3(grid), pw, 0, s, inst,
                                                list));
            break;
        case BatchKernel::SubMean:
            hipLaunchKernelGGL(kb_sub_mean, dim3(grid), pw, 0, s, inst, list);
            break;
        case BatchKernel::Rhs:
            DG_DISPATCH_NR(n, rw, hipLaunchKernelGGL((kb_rhs<NN, WW>), dim3(grid), dim3(64 * WW),
                                                     0, s, inst, list));
            break;
    }
    return hipGetLastError();
}

}  // namespace dgk

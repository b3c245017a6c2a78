// Batched launches (internal): per-instance records and work items.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dgk {

struct BatchItem {
    int inst;   // instance index in the record table
    int b;      // local block index of the instance's single-instance launch
};

struct ItemList {
    const BatchItem* items;   // device
    const int* count;         // device: number of valid items
};

// One instance of a batch, in device memory.  The geometry part is fixed;
// the stage part is rewritten by the host before every RK stage.
struct BatchInst {
    Geom g;
    int cell_tilesX, cell_nblocks, row_tilesX, row_nblocks;
    int nb_rows, nb_cells, nb_elems;
    long rows, cells, elems;
    double area, tol2;
    int max_iter, active;
    OpConst<double> k;
    // stage part
    const double* w_in;    // omega of this stage (solve input, bracket input)
    const double* w_n;     // omega at the start of the step (null at stage 1)
    double* w_out;         // stage output
    const double* pa;      // guess = ca pa + cb pb
    const double* pb;
    double ca, cb;
    double* psi;           // solve output (canonical)
    RhsArgs ra;
    // workspace
    double *x, *r, *p0, *p1;
    CgScalars* sc;
    unsigned* counters;
    double* partials;
};

enum class BatchKernel { Mean, Init, Dir, Res, Finish, SubMean, Rhs };

void fill_batch_geometry(BatchInst& b);
// One fused launch of `kind` for polynomial order n with cell tiles of
// cw waves (Init, Dir, Res) and bracket tiles of rw waves (Rhs).
hipError_t launch_batch(int n, int cw, int rw, BatchKernel kind, const BatchInst* inst,
                        const ItemList& list, int grid, hipStream_t s);

}  // namespace dgk

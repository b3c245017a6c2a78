// Separable eigenbases of the periodic 1D LDG second derivative for the
// fast-diagonalisation preconditioner (host construction in fd_basis.cpp,
// device application in fd_kernels.hip and abi.cpp).  Internal.
#pragma once

#include <vector>

#include "dg_internal.h"

namespace dgk {

// Real W-orthonormal eigenbasis of one axis: V is NN x NN column-major
// (row = cx * n + i, the image-layout index along the axis; column = mode),
// L V = V diag(lam), V^T W V = I; `zero` is the column of the constant mode.
struct FdAxis {
    int NN = 0;
    std::vector<double> V;
    std::vector<double> lam;
    int zero = -1;
};

// Builds the basis for N cells of size h from the LDG tables (h = 1 form).
// *max_err receives the largest relative defect seen (Hermitian symmetry of
// the symbols, eigen-residuals).  Returns false if the basis is incomplete.
bool fd_axis_basis(const HostTables& t, int N, double h, FdAxis* out, double* max_err);

// Device resources of the preconditioner, owned by a workspace.
struct FdDevice {
    int NX = 0, NY = 0, zx = -1, zy = -1;
    double *Vx = nullptr, *Px = nullptr, *Vy = nullptr, *Py = nullptr;  // Py/Vy may alias
    double *lx = nullptr, *ly = nullptr;
    double *img0 = nullptr, *img1 = nullptr;   // image-layout work fields
    bool shared = false;                       // y basis aliases the x basis
    void* blas = nullptr;                      // rocblas_handle
    size_t bytes = 0;
};

}  // namespace dgk

// Separable eigenbases of the periodic 1D LDG second derivative for the
// fast-diagonalisation preconditioner (host construction in fd_basis.cpp,
// device application in fd_apply.cpp and fd_kernels.hip).  Internal.
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

// The same basis in factored form V = (Phi (x) I_n) B: Phi (N x N,
// column-major) is the real orthonormal Fourier basis over the cells
// (columns 0 .. K-1 the even ones: constant, cos k, and for even N the
// alternating one; columns K + k - 1 the sines), B block diagonal over the
// K = N/2 + 1 wave
// numbers.  Block k couples the basis columns ccos[k] (and csin[k], -1 for
// k = 0 and N/2) of every node i with the modes of that k: slot p = (i, cos)
// -> i, (i, sin) -> n + i; mode q = (a, re) -> a, (a, im) -> n + a, both
// stored at index a * N + ccos / csin.  mf[k] (2n x 2n, row q) = B^T scaled
// by the Gauss weights (h/2) w_i (forward, V^T W); mi[k] (row p) = B
// (inverse).  lam[a * N + c] is the eigenvalue of that mode, `zero` the
// index of the constant one.
struct FdFactors {
    int N = 0, n = 0, K = 0;
    std::vector<double> phi;
    std::vector<int> ccos, csin;
    std::vector<double> mf, mi;
    std::vector<double> lam;
    int zero = -1;
};

// Builds the basis for N cells of size h from the LDG tables (h = 1 form).
// *max_err receives the largest relative defect seen (Hermitian symmetry of
// the symbols, eigen-residuals).  Returns false if the basis is incomplete.
// shifted: the cell Fourier basis of the matrix-product transforms (phases
// at the cell centres c + 1/2, see fd_basis.cpp), else that of the FFT ones.
bool fd_axis_factors(const HostTables& t, int N, double h, FdFactors* out, double* max_err,
                     bool shifted = false);
// Dense assembly of the same basis (host checks): column a * N + c is the
// mode of slot (a, c), rows cx * n + i.
bool fd_axis_basis(const HostTables& t, int N, double h, FdAxis* out, double* max_err,
                   bool shifted = false);

// The 1D LDG second derivative of one axis (the blocks of ldg_axis times
// h^-2; the homogeneous Dirichlet closure when !periodic): fd_axis_apply
// computes out = L u, fd_axis_operator assembles L densely (m x m with
// m = n N, column-major, row and column index c * n + i).
void fd_axis_apply(const HostTables& t, int N, double h, bool periodic, const double* u,
                   double* out);
void fd_axis_operator(const HostTables& t, int N, double h, bool periodic,
                      std::vector<double>* L);

// Device copy of one axis's factors in one precision: phi (N x N),
// mf / mi (K blocks of 2n x 2n), lam (n N).
template <class T>
struct FdFactorsDevice {
    T *phi = nullptr, *mf = nullptr, *mi = nullptr, *lam = nullptr;
};

// One axis: the factors in FP64 and rounded to FP32 (the FP32 apply), and
// cols[2k] / cols[2k+1] (ccos / csin).
struct FdAxisDevice {
    int N = 0, K = 0, zero = -1;
    FdFactorsDevice<double> f64;
    FdFactorsDevice<float> f32;
    int* cols = nullptr;
    template <class T> const FdFactorsDevice<T>& get() const;
};
template <> inline const FdFactorsDevice<double>& FdAxisDevice::get<double>() const { return f64; }
template <> inline const FdFactorsDevice<float>& FdAxisDevice::get<float>() const { return f32; }

// Dense eigenbasis of one axis, the path of grids with a homogeneous
// Dirichlet axis (whose operator is not circulant): Q = W^{1/2} V, with V the
// W-orthonormal eigenbasis of the 1D operator, is orthogonal; m x m
// column-major with rows c + N i (the axis index of the dense work image),
// in FP64 and rounded to FP32, and lam the eigenvalues of L (m of them).
struct FdDenseAxis {
    int m = 0;
    double *q64 = nullptr, *lam64 = nullptr;
    float *q32 = nullptr, *lam32 = nullptr;
    template <class T> const T* q() const;
    template <class T> const T* lam() const;
};
template <> inline const double* FdDenseAxis::q<double>() const { return q64; }
template <> inline const float* FdDenseAxis::q<float>() const { return q32; }
template <> inline const double* FdDenseAxis::lam<double>() const { return lam64; }
template <> inline const float* FdDenseAxis::lam<float>() const { return lam32; }

// Device resources of the preconditioner, owned by a workspace.
struct FdDevice {
    int n = 0;
    // dense path (a Dirichlet axis): dy aliases dx when `shared`
    bool dense = false;
    FdDenseAxis dx, dy;
    FdAxisDevice x, y;                         // y aliases x when `shared`
    bool shared = false;
    double *img0 = nullptr, *img1 = nullptr;   // node-plane / half-spectrum work
                                               // fields (FP64, or FP32 in their
                                               // first half)
    void* blas = nullptr;                      // rocblas_handle
    // FFTs along the cells (each real row as a complex row of half length):
    // plans [precision][x fwd, y fwd, y inv, x inv] (rocfft_plan, FP64 then
    // FP32), one execution info, work buffer
    void* fft[2][4] = {{nullptr, nullptr, nullptr, nullptr},
                       {nullptr, nullptr, nullptr, nullptr}};
    void* fft_info = nullptr;
    void* fft_work = nullptr;
    size_t fft_work_bytes = 0;
    bool use_fft = true;
    size_t bytes = 0;
};

}  // namespace dgk

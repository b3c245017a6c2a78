// Device side of the fast-diagonalisation preconditioner: upload of the
// factored separable eigenbases (fd_basis.cpp) and the application
//     z = V_y [ (V_y^T W_y R W_x V_x) / -(lam_y + lam_x) ] V_x^T,
// with V = (Phi (x) I_n) B per axis, on node planes U[cx + Nx (cy + Ny q)]
// (q = i + n j).  The cell Fourier transforms Phi are FP64 matrix products
// (rocBLAS), each chosen so that its output puts the next step's axis first:
//   U  --(x transform, batched over j)-->  U1[cy + Ny (i + n kx + n Nx j)]
//   U1 --(x mixing B_x^T W_x, in place)
//   U1 --(y transform)-->                   U2[i + n kx + n Nx (j + n ky)]
//   U2 --(y mixing, scaling, unmixing, in place)
//   U2 --(inverse y transform)-->           U1
//   U1 --(x unmixing B_x, in place)
//   U1 --(inverse x transform, batched)-->  U
// The transforms cost 4 n^2 Nx Ny (Nx + Ny) flops in all, n times fewer
// than dense products with V.
#include <rocblas/rocblas.h>

#include <cstring>
#include <new>

#include "abi_types.h"
#include "dg_launch.h"
#include "fd_basis.h"

namespace dgk {

namespace {

bool same_axis(const dg_grid* g) { return g->nx == g->ny && g->hx == g->hy; }

int blas_fail(rocblas_status st, const char* what) {
    return fail(DG_E_HIP, "%s: rocBLAS status %d (%s)", what, (int)st,
                rocblas_status_to_string(st));
}

size_t axis_bytes(int N, int n) {
    const size_t K = (size_t)N / 2 + 1, S = 2 * (size_t)n;
    return ((size_t)N * N + 2 * K * S * S + (size_t)N * n) * sizeof(double) + 2 * K * sizeof(int);
}

void free_axis(FdAxisDevice* a) {
    void* bufs[] = {a->phi, a->mf, a->mi, a->lam, a->cols};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    *a = FdAxisDevice{};
}

template <class T>
bool upload(T** dst, const std::vector<T>& src) {
    const size_t b = src.size() * sizeof(T);
    if (hipMalloc((void**)dst, b) != hipSuccess) return false;
    return hipMemcpy(*dst, src.data(), b, hipMemcpyHostToDevice) == hipSuccess;
}

bool upload_axis(const FdFactors& f, FdAxisDevice* a) {
    a->N = f.N;
    a->K = f.K;
    a->zero = f.zero;
    std::vector<int> cols(2 * (size_t)f.K);
    for (int k = 0; k < f.K; ++k) {
        cols[2 * k] = f.ccos[k];
        cols[2 * k + 1] = f.csin[k];
    }
    return upload(&a->phi, f.phi) && upload(&a->mf, f.mf) && upload(&a->mi, f.mi) &&
           upload(&a->lam, f.lam) && upload(&a->cols, cols);
}

}  // namespace

size_t fd_bytes(const dg_grid* g) {
    const size_t planes = 2 * (size_t)g->nx * g->ny * g->n * g->n * sizeof(double);
    return planes + axis_bytes(g->nx, g->n) + (same_axis(g) ? 0 : axis_bytes(g->ny, g->n));
}

void fd_destroy(FdDevice* fd) {
    if (!fd) return;
    if (fd->blas) (void)rocblas_destroy_handle((rocblas_handle)fd->blas);
    if (fd->img0) (void)hipFree(fd->img0);
    if (fd->img1) (void)hipFree(fd->img1);
    free_axis(&fd->x);
    if (!fd->shared) free_axis(&fd->y);
    delete fd;
}

int fd_create(const dg_grid* g, FdDevice** out) {
    *out = nullptr;
    FdDevice* fd = new (std::nothrow) FdDevice;
    if (!fd) return fail(DG_E_NOMEM, "host allocation failed");
    fd->n = g->n;
    fd->shared = same_axis(g);
    FdFactors fx, fy;
    double ex = 0.0, ey = 0.0;
    if (!fd_axis_factors(g->t, g->nx, g->hx, &fx, &ex) ||
        (!fd->shared && !fd_axis_factors(g->t, g->ny, g->hy, &fy, &ey))) {
        delete fd;
        return fail(DG_E_INVAL, "eigenbasis construction failed");
    }
    if (ex > 1e-10 || ey > 1e-10) {
        delete fd;
        return fail(DG_E_INVAL, "eigenbasis defect %.3e too large", ex > ey ? ex : ey);
    }
    bool ok = upload_axis(fx, &fd->x);
    if (ok && fd->shared) fd->y = fd->x;
    else if (ok) ok = upload_axis(fy, &fd->y);
    const size_t img = (size_t)g->nx * g->ny * g->n * g->n * sizeof(double);
    if (ok) ok = hipMalloc((void**)&fd->img0, img) == hipSuccess &&
                 hipMalloc((void**)&fd->img1, img) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        fd_destroy(fd);
        return fail(DG_E_NOMEM, "preconditioner allocation of %zu bytes failed", fd_bytes(g));
    }
    rocblas_handle h = nullptr;
    rocblas_status st = rocblas_create_handle(&h);
    if (st != rocblas_status_success) {
        fd_destroy(fd);
        return blas_fail(st, "rocblas_create_handle");
    }
    fd->blas = h;
    fd->bytes = fd_bytes(g);
    *out = fd;
    return DG_OK;
}

// img0 holds the node planes of r on entry and those of z = M r on exit.
int fd_apply_image(const FdDevice* fd, hipStream_t s) {
    rocblas_handle h = (rocblas_handle)fd->blas;
    rocblas_status st = rocblas_set_stream(h, s);
    if (st != rocblas_status_success) return blas_fail(st, "rocblas_set_stream");
    const FdAxisDevice& X = fd->x;
    const FdAxisDevice& Y = fd->y;
    const rocblas_int n = fd->n, Nx = X.N, Ny = Y.N;
    const rocblas_stride plane_j = (rocblas_stride)Nx * Ny * n;   // one j of U / U1
    const double one = 1.0, zero = 0.0;
    const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
    // U1_j = U_j^T Phi_x: U_j is Nx x (Ny n), U1_j is (Ny n) x Nx
    st = rocblas_dgemm_strided_batched(h, T_, N_, Ny * n, Nx, Nx, &one, fd->img0, Nx, plane_j,
                                       X.phi, Nx, 0, &zero, fd->img1, Ny * n, plane_j, n);
    if (st != rocblas_status_success) return blas_fail(st, "x transform");
    hipError_t e = launch_fd_mix_x(n, Nx, Ny, X.K, X.cols, X.mf, fd->img1, s);
    if (e != hipSuccess) return hip_fail(e, "x mixing launch");
    // U2 = U1^T Phi_y: U1 is Ny x (n^2 Nx), U2 is (n^2 Nx) x Ny
    st = rocblas_dgemm(h, T_, N_, n * n * Nx, Ny, Ny, &one, fd->img1, Ny, Y.phi, Ny, &zero,
                       fd->img0, n * n * Nx);
    if (st != rocblas_status_success) return blas_fail(st, "y transform");
    e = launch_fd_mix_y(n, Nx, Ny, Y.K, Y.cols, Y.mf, Y.mi, X.lam, Y.lam, X.zero, Y.zero,
                        fd->img0, s);
    if (e != hipSuccess) return hip_fail(e, "y mixing launch");
    // U1 = Phi_y U2^T
    st = rocblas_dgemm(h, N_, T_, Ny, n * n * Nx, Ny, &one, Y.phi, Ny, fd->img0, n * n * Nx,
                       &zero, fd->img1, Ny);
    if (st != rocblas_status_success) return blas_fail(st, "inverse y transform");
    e = launch_fd_mix_x(n, Nx, Ny, X.K, X.cols, X.mi, fd->img1, s);
    if (e != hipSuccess) return hip_fail(e, "x unmixing launch");
    // U_j = Phi_x U1_j^T
    st = rocblas_dgemm_strided_batched(h, N_, T_, Nx, Ny * n, Nx, &one, X.phi, Nx, 0, fd->img1,
                                       Ny * n, plane_j, &zero, fd->img0, Nx, plane_j, n);
    if (st != rocblas_status_success) return blas_fail(st, "inverse x transform");
    return DG_OK;
}

}  // namespace dgk

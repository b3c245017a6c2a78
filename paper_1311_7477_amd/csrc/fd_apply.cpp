// Device side of the fast-diagonalisation preconditioner: upload of the
// separable eigenbases (fd_basis.cpp) and the application
//     z = V_y [ (V_y^T W_y R W_x V_x) / -(lam_y + lam_x) ] V_x^T
// on the image layout (R[(cy n + j)][(cx n + i)], NY x NX row-major, which
// is the NX x NY column-major matrix R^T) as four dense FP64 products
// (rocBLAS dgemm) and one scaling kernel.  P = W V is stored next to V.
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

}  // namespace

size_t fd_bytes(const dg_grid* g) {
    const size_t NX = (size_t)g->nx * g->n, NY = (size_t)g->ny * g->n;
    size_t mats = 2 * NX * NX + (same_axis(g) ? 0 : 2 * NY * NY);
    return (mats + NX + NY + 2 * NX * NY) * sizeof(double);
}

void fd_destroy(FdDevice* fd) {
    if (!fd) return;
    if (fd->blas) (void)rocblas_destroy_handle((rocblas_handle)fd->blas);
    double* bufs[] = {fd->Vx, fd->Px, fd->lx, fd->img0, fd->img1};
    for (double* b : bufs)
        if (b) (void)hipFree(b);
    if (!fd->shared) {
        if (fd->Vy) (void)hipFree(fd->Vy);
        if (fd->Py) (void)hipFree(fd->Py);
        if (fd->ly) (void)hipFree(fd->ly);
    }
    delete fd;
}

int fd_create(const dg_grid* g, FdDevice** out) {
    *out = nullptr;
    FdDevice* fd = new (std::nothrow) FdDevice;
    if (!fd) return fail(DG_E_NOMEM, "host allocation failed");
    fd->NX = g->nx * g->n;
    fd->NY = g->ny * g->n;
    fd->shared = same_axis(g);
    FdAxis ax, ay;
    double ex = 0.0, ey = 0.0;
    if (!fd_axis_basis(g->t, g->nx, g->hx, &ax, &ex) ||
        (!fd->shared && !fd_axis_basis(g->t, g->ny, g->hy, &ay, &ey))) {
        delete fd;
        return fail(DG_E_INVAL, "eigenbasis construction failed");
    }
    if (ex > 1e-10 || ey > 1e-10) {
        delete fd;
        return fail(DG_E_INVAL, "eigenbasis defect %.3e too large", ex > ey ? ex : ey);
    }
    const FdAxis& by = fd->shared ? ax : ay;
    fd->zx = ax.zero;
    fd->zy = by.zero;
    // P = W V: row (cx, i) of V scaled by the Gauss weight (h / 2) w_i
    auto weighted = [&](const FdAxis& a, double h) {
        std::vector<double> P(a.V.size());
        const int n = g->n;
        for (long c = 0; c < a.NN; ++c)
            for (long r = 0; r < a.NN; ++r)
                P[(size_t)(c * a.NN + r)] = 0.5 * h * g->t.w[r % n] * a.V[(size_t)(c * a.NN + r)];
        return P;
    };
    auto upload = [&](double** dst, const std::vector<double>& src) -> bool {
        const size_t b = src.size() * sizeof(double);
        if (hipMalloc((void**)dst, b) != hipSuccess) return false;
        return hipMemcpy(*dst, src.data(), b, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = upload(&fd->Vx, ax.V) && upload(&fd->Px, weighted(ax, g->hx)) &&
              upload(&fd->lx, ax.lam);
    if (ok && fd->shared) {
        fd->Vy = fd->Vx;
        fd->Py = fd->Px;
        fd->ly = fd->lx;
    } else if (ok) {
        ok = upload(&fd->Vy, ay.V) && upload(&fd->Py, weighted(ay, g->hy)) &&
             upload(&fd->ly, ay.lam);
    }
    const size_t img = (size_t)fd->NX * fd->NY * sizeof(double);
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

// img0 holds the image of r on entry and the image of z = M r on exit.
int fd_apply_image(const FdDevice* fd, hipStream_t s) {
    rocblas_handle h = (rocblas_handle)fd->blas;
    rocblas_status st = rocblas_set_stream(h, s);
    if (st != rocblas_status_success) return blas_fail(st, "rocblas_set_stream");
    const rocblas_int NX = fd->NX, NY = fd->NY;
    const double one = 1.0, zero = 0.0;
    const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
    // B = R^T P_y  (NX x NY)
    st = rocblas_dgemm(h, N_, N_, NX, NY, NY, &one, fd->img0, NX, fd->Py, NY, &zero,
                       fd->img1, NX);
    if (st != rocblas_status_success) return blas_fail(st, "dgemm 1");
    // A = P_x^T B = (P_y^T R P_x)^T
    st = rocblas_dgemm(h, T_, N_, NX, NY, NX, &one, fd->Px, NX, fd->img1, NX, &zero,
                       fd->img0, NX);
    if (st != rocblas_status_success) return blas_fail(st, "dgemm 2");
    hipError_t e = launch_fd_scale(NX, NY, fd->img0, fd->lx, fd->ly, fd->zx, fd->zy, s);
    if (e != hipSuccess) return hip_fail(e, "spectral scaling launch");
    // B = V_x A
    st = rocblas_dgemm(h, N_, N_, NX, NY, NX, &one, fd->Vx, NX, fd->img0, NX, &zero,
                       fd->img1, NX);
    if (st != rocblas_status_success) return blas_fail(st, "dgemm 3");
    // A = B V_y^T = (V_y Z~ V_x^T)^T
    st = rocblas_dgemm(h, N_, T_, NX, NY, NY, &one, fd->img1, NX, fd->Vy, NY, &zero,
                       fd->img0, NX);
    if (st != rocblas_status_success) return blas_fail(st, "dgemm 4");
    return DG_OK;
}

}  // namespace dgk

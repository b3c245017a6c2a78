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
// than dense products with V.  The same steps run in FP64 or, for the mixed-
// precision PCG, in FP32 (factors rounded once at setup; the planes then take
// the first half of the FP64 work fields).
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
    const size_t vals = (size_t)N * N + 2 * K * S * S + (size_t)N * n;
    return vals * (sizeof(double) + sizeof(float)) + 2 * K * sizeof(int);
}

void free_axis(FdAxisDevice* a) {
    void* bufs[] = {a->f64.phi, a->f64.mf, a->f64.mi, a->f64.lam,
                    a->f32.phi, a->f32.mf, a->f32.mi, a->f32.lam, a->cols};
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

std::vector<float> rounded(const std::vector<double>& v) {
    return std::vector<float>(v.begin(), v.end());
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
    return upload(&a->f64.phi, f.phi) && upload(&a->f64.mf, f.mf) &&
           upload(&a->f64.mi, f.mi) && upload(&a->f64.lam, f.lam) &&
           upload(&a->f32.phi, rounded(f.phi)) && upload(&a->f32.mf, rounded(f.mf)) &&
           upload(&a->f32.mi, rounded(f.mi)) && upload(&a->f32.lam, rounded(f.lam)) &&
           upload(&a->cols, cols);
}

// C_b = op(A_b) op(B_b), b < batch (alpha 1, beta 0), in the precision of T.
rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                    rocblas_int m, rocblas_int n, rocblas_int k, const double* A,
                    rocblas_int lda, rocblas_stride sa, const double* B, rocblas_int ldb,
                    rocblas_stride sb, double* C, rocblas_int ldc, rocblas_stride sc,
                    rocblas_int batch) {
    const double one = 1.0, zero = 0.0;
    return rocblas_dgemm_strided_batched(h, ta, tb, m, n, k, &one, A, lda, sa, B, ldb, sb,
                                         &zero, C, ldc, sc, batch);
}

rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb,
                    rocblas_int m, rocblas_int n, rocblas_int k, const float* A,
                    rocblas_int lda, rocblas_stride sa, const float* B, rocblas_int ldb,
                    rocblas_stride sb, float* C, rocblas_int ldc, rocblas_stride sc,
                    rocblas_int batch) {
    const float one = 1.0f, zero = 0.0f;
    return rocblas_sgemm_strided_batched(h, ta, tb, m, n, k, &one, A, lda, sa, B, ldb, sb,
                                         &zero, C, ldc, sc, batch);
}

template <class T>
int apply_planes(const FdDevice* fd, hipStream_t s) {
    rocblas_handle h = (rocblas_handle)fd->blas;
    rocblas_status st = rocblas_set_stream(h, s);
    if (st != rocblas_status_success) return blas_fail(st, "rocblas_set_stream");
    const FdAxisDevice& X = fd->x;
    const FdAxisDevice& Y = fd->y;
    const FdFactorsDevice<T>& fx = X.get<T>();
    const FdFactorsDevice<T>& fy = Y.get<T>();
    T* u0 = reinterpret_cast<T*>(fd->img0);
    T* u1 = reinterpret_cast<T*>(fd->img1);
    const rocblas_int n = fd->n, Nx = X.N, Ny = Y.N, M2 = n * n * Nx;
    const rocblas_stride plane_j = (rocblas_stride)Nx * Ny * n;   // one j of U / U1
    const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
    // U1_j = U_j^T Phi_x: U_j is Nx x (Ny n), U1_j is (Ny n) x Nx
    st = gemm(h, T_, N_, Ny * n, Nx, Nx, u0, Nx, plane_j, fx.phi, Nx, 0, u1, Ny * n, plane_j, n);
    if (st != rocblas_status_success) return blas_fail(st, "x transform");
    hipError_t e = launch_fd_mix_x<T>(n, Nx, Ny, X.K, X.cols, fx.mf, u1, s);
    if (e != hipSuccess) return hip_fail(e, "x mixing launch");
    // U2 = U1^T Phi_y: U1 is Ny x (n^2 Nx), U2 is (n^2 Nx) x Ny
    st = gemm(h, T_, N_, M2, Ny, Ny, u1, Ny, 0, fy.phi, Ny, 0, u0, M2, 0, 1);
    if (st != rocblas_status_success) return blas_fail(st, "y transform");
    e = launch_fd_mix_y<T>(n, Nx, Ny, Y.K, Y.cols, fy.mf, fy.mi, fx.lam, fy.lam, X.zero, Y.zero,
                           u0, s);
    if (e != hipSuccess) return hip_fail(e, "y mixing launch");
    // U1 = Phi_y U2^T
    st = gemm(h, N_, T_, Ny, M2, Ny, fy.phi, Ny, 0, u0, M2, 0, u1, Ny, 0, 1);
    if (st != rocblas_status_success) return blas_fail(st, "inverse y transform");
    e = launch_fd_mix_x<T>(n, Nx, Ny, X.K, X.cols, fx.mi, u1, s);
    if (e != hipSuccess) return hip_fail(e, "x unmixing launch");
    // U_j = Phi_x U1_j^T
    st = gemm(h, N_, T_, Nx, Ny * n, Nx, fx.phi, Nx, 0, u1, Ny * n, plane_j, u0, Nx, plane_j, n);
    if (st != rocblas_status_success) return blas_fail(st, "inverse x transform");
    return DG_OK;
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

// img0 holds the node planes of r on entry and those of z = M r on exit
// (FP32 planes when fp32).
int fd_apply_image(const FdDevice* fd, bool fp32, hipStream_t s) {
    return fp32 ? apply_planes<float>(fd, s) : apply_planes<double>(fd, s);
}

}  // namespace dgk

// Device side of the fast-diagonalisation preconditioner: upload of the
// factored separable eigenbases (fd_basis.cpp) and the application
//     z = V_y [ (V_y^T W_y R W_x V_x) / -(lam_y + lam_x) ] V_x^T,
// with V = (Phi (x) I_n) B per axis, on node planes U[cx + Nx (cy + Ny q)]
// (q = i + n j).  The cell Fourier transforms Phi are FP64 matrix products
// (rocBLAS), each chosen so that its output puts the next step's axis first:
//   U  --(x transform, batched over j)-->  U1[cy + Ny (i + n kx + n Nx j)]
//   U1 --(x mixing B_x^T W_x)
//   U1 --(y transform)-->                   U2[i + n kx + n Nx (j + n ky)]
//   U2 --(y mixing, scaling, unmixing, in place)
//   U2 --(inverse y transform)-->           U1
//   U1 --(x unmixing B_x)
//   U1 --(inverse x transform, batched)-->  U
// Each transform is folded: with phases at the cell centres the even basis
// columns (constant, cosines) take the same value on cells c and N - 1 - c
// and the odd ones (sines, alternating) opposite values, so the rows are
// first combined into sums E and differences O and each half meets its own
// half of Phi -- two products of (N/2)^2 instead of one of N^2.  The x fold
// happens in the input conversion, the y fold in the x mixing (and the
// unfolds in reverse).  The transforms cost 2 n^2 Nx Ny (Nx + Ny) flops in
// all.  Beyond 32 cells on an axis (both counts even) they run as FFTs
// along the cells instead (rocFFT, with the unshifted basis: each real row as
// a complex row of half length, the mixing kernels then convert to and from
// half spectra, fd_kernels.hip).  The same steps run in FP64 or, for the
// mixed-precision PCG, in FP32 (factors rounded once at setup; the
// fields then take the first half of the FP64 work fields).
//
// A grid with a homogeneous Dirichlet axis has no circulant structure along
// that axis, so it takes the dense path: per axis the orthogonal Q = W^{1/2} V
// (V the W-orthonormal eigenbasis of the 1D operator; rocSOLVER's symmetric
// eigensolver on W^{1/2} (-L) W^{-1/2} for a Dirichlet axis, the Bloch basis
// assembled densely for a periodic one), and on the dense image A of
// sqrt(W) r (rows along x)
//     z = W^{-1/2} Q_x [ (Q_x^T A Q_y) / -(lam_x + lam_y) ] Q_y^T,
// four GEMMs of 2 m_x m_y (m_x + m_y) flops in all (m = n N per axis).
#include <rocblas/rocblas.h>
#include <rocfft/rocfft.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "abi_types.h"
#include "dg_launch.h"
#include "fd_basis.h"

namespace dgk {

namespace {

bool same_axis(const dg_grid* g) {
    return g->nx == g->ny && g->hx == g->hy && g->geom.bcx == g->geom.bcy;
}

bool has_dirichlet(const dg_grid* g) { return g->geom.bcx || g->geom.bcy; }

// the dense path's limit: 8192 nodes per axis (Q in FP64 and FP32: 805 MB)
constexpr int kFdDenseMaxNodes = 8192;

size_t dense_axis_bytes(int N, int n) {
    const size_t m = (size_t)N * n;
    return (m * m + m) * (sizeof(double) + sizeof(float));
}

int blas_fail(rocblas_status st, const char* what) {
    return fail(DG_E_HIP, "%s: rocBLAS status %d (%s)", what, (int)st,
                rocblas_status_to_string(st));
}

constexpr int kFdGemmMaxCells = 32;

int fft_fail(rocfft_status st, const char* what) {
    return fail(DG_E_HIP, "%s: rocFFT status %d", what, (int)st);
}

// Reals in one work field: the node planes or the packed spectra of the x or
// y transform (N/2 complex values per real row), with room for N/2 + 1.
size_t field_reals(int n, int Nx, int Ny) {
    const size_t nn = (size_t)n * n;
    size_t a = nn * Nx * Ny, b = nn * Ny * 2 * (Nx / 2 + 1), c = nn * Nx * 2 * (Ny / 2 + 1);
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
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
    // even columns 0 .. Ke-1 and odd ones Ke .. N-1 of each (shifted) basis,
    // Ke = ceil(N/2); folded rows: E for c < Ke, O at Ke + c
    const rocblas_int Kx = (Nx + 1) / 2, Sx = Nx - Kx, Ky = (Ny + 1) / 2, Sy = Ny - Ky;
    const rocblas_int ldj = Ny * n;
    const rocblas_stride plane_j = (rocblas_stride)Nx * Ny * n;   // one j of U / U1
    const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
    const T* phx_s = fx.phi + (size_t)Kx * Nx;   // rows 0 .. Sx-1 of the odd block
    const T* phy_s = fy.phi + (size_t)Ky * Ny;
    // x transform of the x-folded planes u0 (E rows 0 .. Kx-1, O rows Kx ..):
    // U1_j[:, even] = E_j^T Phi_x,even, U1_j[:, odd] = O_j^T Phi_x,odd
    st = gemm(h, T_, N_, ldj, Kx, Kx, u0, Nx, plane_j, fx.phi, Nx, 0, u1, ldj, plane_j, n);
    if (st == rocblas_status_success && Sx > 0)
        st = gemm(h, T_, N_, ldj, Sx, Sx, u0 + Kx, Nx, plane_j, phx_s, Nx, 0,
                  u1 + (size_t)Kx * ldj, ldj, plane_j, n);
    if (st != rocblas_status_success) return blas_fail(st, "x transform");
    // x mixing (B^T W) and the fold along y: u1 -> u0
    hipError_t e = launch_fd_mix_x_fold<T>(false, n, Nx, Ny, Ky, X.K, X.cols, fx.mf, u1, u0, s);
    if (e != hipSuccess) return hip_fail(e, "x mixing launch");
    // y transform: U2 (M2 x Ny) from the y-folded rows of u0 (Ny x M2)
    st = gemm(h, T_, N_, M2, Ky, Ky, u0, Ny, 0, fy.phi, Ny, 0, u1, M2, 0, 1);
    if (st == rocblas_status_success && Sy > 0)
        st = gemm(h, T_, N_, M2, Sy, Sy, u0 + Ky, Ny, 0, phy_s, Ny, 0, u1 + (size_t)Ky * M2, M2,
                  0, 1);
    if (st != rocblas_status_success) return blas_fail(st, "y transform");
    e = launch_fd_mix_y<T>(n, Nx, Ny, Y.K, Y.cols, fy.mf, fy.mi, fx.lam, fy.lam, X.zero, Y.zero,
                           u1, s);
    if (e != hipSuccess) return hip_fail(e, "y mixing launch");
    // inverse y transform into y-folded rows: u1 -> u0
    st = gemm(h, N_, T_, Ky, M2, Ky, fy.phi, Ny, 0, u1, M2, 0, u0, Ny, 0, 1);
    if (st == rocblas_status_success && Sy > 0)
        st = gemm(h, N_, T_, Sy, M2, Sy, phy_s, Ny, 0, u1 + (size_t)Ky * M2, M2, 0, u0 + Ky, Ny,
                  0, 1);
    if (st != rocblas_status_success) return blas_fail(st, "inverse y transform");
    // unfold along y and x unmixing (B): u0 -> u1
    e = launch_fd_mix_x_fold<T>(true, n, Nx, Ny, Ky, X.K, X.cols, fx.mi, u0, u1, s);
    if (e != hipSuccess) return hip_fail(e, "x unmixing launch");
    // inverse x transform into x-folded planes: u1 -> u0
    st = gemm(h, N_, T_, Kx, ldj, Kx, fx.phi, Nx, 0, u1, ldj, plane_j, u0, Nx, plane_j, n);
    if (st == rocblas_status_success && Sx > 0)
        st = gemm(h, N_, T_, Sx, ldj, Sx, phx_s, Nx, 0, u1 + (size_t)Kx * ldj, ldj, plane_j,
                  u0 + Kx, Nx, plane_j, n);
    if (st != rocblas_status_success) return blas_fail(st, "inverse x transform");
    return DG_OK;
}

template <class T>
int apply_fft(const FdDevice* fd, hipStream_t s) {
    const int pr = sizeof(T) == sizeof(float) ? 1 : 0;
    rocfft_execution_info info = (rocfft_execution_info)fd->fft_info;
    rocfft_status st = rocfft_execution_info_set_stream(info, s);
    if (st != rocfft_status_success) return fft_fail(st, "set stream");
    const FdAxisDevice& X = fd->x;
    const FdAxisDevice& Y = fd->y;
    const FdFactorsDevice<T>& fx = X.get<T>();
    const FdFactorsDevice<T>& fy = Y.get<T>();
    const int n = fd->n, Nx = X.N, Ny = Y.N;
    void* b0 = fd->img0;
    void* b1 = fd->img1;
    auto run = [&](int i, void* in, void* out) {
        void* ib[1] = {in};
        void* ob[1] = {out};
        return rocfft_execute((rocfft_plan)fd->fft[pr][i], ib, ob, info);
    };
    // node planes U (b0) -> x spectra (b1) -> x-mixed real field U1 (b0)
    st = run(0, b0, b1);
    if (st != rocfft_status_success) return fft_fail(st, "x transform");
    hipError_t e = launch_fft_mix_x_fwd<T>(n, Nx, Ny, X.cols, fx.mf, b1, (T*)b0, s);
    if (e != hipSuccess) return hip_fail(e, "x mixing launch");
    // U1 (b0) -> y spectra (b1), mixed, divided, unmixed in place -> U1 (b0)
    st = run(1, b0, b1);
    if (st != rocfft_status_success) return fft_fail(st, "y transform");
    e = launch_fft_mix_y<T>(n, Nx, Ny, Y.cols, fy.mf, fy.mi, fx.lam, fy.lam, X.zero,
                            Y.zero, b1, s);
    if (e != hipSuccess) return hip_fail(e, "y mixing launch");
    st = run(2, b1, b0);
    if (st != rocfft_status_success) return fft_fail(st, "inverse y transform");
    // U1 (b0) -> x spectra (b1) -> node planes of z (b0)
    e = launch_fft_mix_x_inv<T>(n, Nx, Ny, X.cols, fx.mi, (const T*)b0, b1, s);
    if (e != hipSuccess) return hip_fail(e, "x unmixing launch");
    st = run(3, b1, b0);
    if (st != rocfft_status_success) return fft_fail(st, "inverse x transform");
    return DG_OK;
}

}  // namespace

// The cell transforms of a periodic grid: FFTs when both axes have an even
// number of cells and one has more than 32 (each real row of N values is
// transformed as a complex row of N/2), the folded GEMMs otherwise (the basis
// with phases at the cell centres folds each axis to half size; an odd count
// cannot be packed into half-length rows).  One FP64 apply with the FFTs
// against the folded GEMMs: 41 / 60 us at n = 4, 64^2; 82 / 129 us at
// n = 4, 256^2; 142 / 270 us at n = 4, 512^2; 210 / 401 us at n = 5, 512^2
// (every order and size from 64 to 512 cells favours the FFTs).
bool fd_uses_fft(int nx, int ny) {
    return (nx > kFdGemmMaxCells || ny > kFdGemmMaxCells) && nx % 2 == 0 && ny % 2 == 0;
}

size_t fd_bytes(const dg_grid* g) {
    if (has_dirichlet(g)) {
        const size_t img = 2 * (size_t)g->n * g->n * g->nx * g->ny * sizeof(double);
        return img + dense_axis_bytes(g->nx, g->n) +
               (same_axis(g) ? 0 : dense_axis_bytes(g->ny, g->n));
    }
    const size_t planes = 2 * field_reals(g->n, g->nx, g->ny) * sizeof(double);
    return planes + axis_bytes(g->nx, g->n) + (same_axis(g) ? 0 : axis_bytes(g->ny, g->n));
}

int fd_supported(const dg_grid* g) {
    if (!has_dirichlet(g)) return DG_OK;
    const long mx = (long)g->n * g->nx, my = (long)g->n * g->ny;
    if (mx > kFdDenseMaxNodes || my > kFdDenseMaxNodes)
        return fail(DG_E_UNSUPPORTED, "the preconditioner of a grid with a Dirichlet axis uses "
                    "dense eigenbases, limited to %d nodes per axis (n * cells: %ld x %ld)",
                    kFdDenseMaxNodes, mx, my);
    return DG_OK;
}

namespace {

void free_dense(FdDenseAxis* a) {
    void* bufs[] = {a->q64, a->lam64, a->q32, a->lam32};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    *a = FdDenseAxis{};
}

// Q (rows c * n + i on entry) reordered to rows c + N i and uploaded in
// FP64 and FP32 with the eigenvalues.
bool upload_dense(int n, int N, const std::vector<double>& Q, const std::vector<double>& lam,
                  FdDenseAxis* out) {
    const size_t m = (size_t)N * n;
    std::vector<double> R(m * m);
    for (size_t col = 0; col < m; ++col)
        for (int c = 0; c < N; ++c)
            for (int i = 0; i < n; ++i)
                R[col * m + c + (size_t)N * i] = Q[col * m + (size_t)c * n + i];
    out->m = (int)m;
    return upload(&out->q64, R) && upload(&out->lam64, lam) &&
           upload(&out->q32, rounded(R)) && upload(&out->lam32, rounded(lam));
}

// The dense eigenbasis of one axis (0: x, 1: y).  A periodic axis assembles
// its Bloch basis; a Dirichlet axis diagonalises S = W^{1/2} (-L) W^{-1/2}
// (symmetric: L is self-adjoint in the Gauss inner product) with rocSOLVER.
// Every eigenpair is then checked against the sparse operator on the host.
int dense_axis(const dg_grid* g, int axis, rocblas_handle h, FdDenseAxis* out) {
    const HostTables& t = g->t;
    const int n = g->n, N = axis ? g->ny : g->nx;
    const double hh = axis ? g->hy : g->hx;
    const bool periodic = !(axis ? g->geom.bcy : g->geom.bcx);
    const size_t m = (size_t)N * n;
    std::vector<double> sw(m);
    for (int c = 0; c < N; ++c)
        for (int i = 0; i < n; ++i) sw[(size_t)c * n + i] = std::sqrt(0.5 * hh * t.w[i]);
    std::vector<double> Q, lam(m);
    double err = 0.0;
    if (periodic) {
        FdAxis a;
        if (!fd_axis_basis(t, N, hh, &a, &err) || err > 1e-10)
            return fail(DG_E_INVAL, "eigenbasis construction failed (defect %.3e)", err);
        Q.swap(a.V);
        for (size_t col = 0; col < m; ++col)
            for (size_t row = 0; row < m; ++row) Q[col * m + row] *= sw[row];
        lam = a.lam;
    } else {
        fd_axis_operator(t, N, hh, false, &Q);
        double scale = 0.0;
        for (size_t col = 0; col < m; ++col)
            for (size_t row = 0; row < m; ++row) {
                double& v = Q[col * m + row];
                v = -v * sw[row] / sw[col];
                scale = std::max(scale, std::fabs(v));
            }
        for (size_t col = 0; col < m; ++col)
            for (size_t row = col + 1; row < m; ++row) {
                double& a = Q[col * m + row];
                double& b = Q[row * m + col];
                err = std::max(err, std::fabs(a - b) / scale);
                a = b = 0.5 * (a + b);
            }
        double *dS = nullptr, *dD = nullptr, *dE = nullptr;
        rocblas_int* dinfo = nullptr;
        rocblas_int info = -1;
        bool ok = hipMalloc((void**)&dS, m * m * sizeof(double)) == hipSuccess &&
                  hipMalloc((void**)&dD, m * sizeof(double)) == hipSuccess &&
                  hipMalloc((void**)&dE, m * sizeof(double)) == hipSuccess &&
                  hipMalloc((void**)&dinfo, sizeof(rocblas_int)) == hipSuccess;
        rocblas_status st = rocblas_status_success;
        if (ok) ok = hipMemcpy(dS, Q.data(), m * m * sizeof(double), hipMemcpyHostToDevice) ==
                     hipSuccess;
        if (ok) {
            st = rocblas_set_stream(h, nullptr);
            if (st == rocblas_status_success)
                st = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper,
                                      (rocblas_int)m, dS, (rocblas_int)m, dD, dE, dinfo);
            if (st == rocblas_status_success) {
                ok = hipMemcpy(Q.data(), dS, m * m * sizeof(double), hipMemcpyDeviceToHost) ==
                         hipSuccess &&
                     hipMemcpy(lam.data(), dD, m * sizeof(double), hipMemcpyDeviceToHost) ==
                         hipSuccess &&
                     hipMemcpy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost) == hipSuccess;
            }
        }
        void* bufs[] = {dS, dD, dE, dinfo};
        for (void* b : bufs)
            if (b) (void)hipFree(b);
        if (st != rocblas_status_success) return blas_fail(st, "rocsolver_dsyevd");
        if (!ok) {
            (void)hipGetLastError();
            return fail(DG_E_NOMEM, "eigensolver buffers for %zu x %zu failed", m, m);
        }
        if (info != 0)
            return fail(DG_E_INVAL, "rocsolver_dsyevd did not converge (info %d)", (int)info);
        for (double& l : lam) l = -l;
    }
    // eigen-residuals |L v - lam v| with v = W^{-1/2} q, against the sparse
    // operator, relative to max |lam| |v|
    double lmax = 0.0;
    for (double l : lam) lmax = std::max(lmax, std::fabs(l));
    std::vector<double> v(m), Lv(m);
    for (size_t col = 0; col < m; ++col) {
        double vmax = 0.0;
        for (size_t row = 0; row < m; ++row) {
            v[row] = Q[col * m + row] / sw[row];
            vmax = std::max(vmax, std::fabs(v[row]));
        }
        fd_axis_apply(t, N, hh, periodic, v.data(), Lv.data());
        for (size_t row = 0; row < m; ++row)
            err = std::max(err, std::fabs(Lv[row] - lam[col] * v[row]) / (lmax * vmax));
    }
    if (!(err <= 1e-9))
        return fail(DG_E_INVAL, "dense eigenbasis defect %.3e too large", err);
    if (!upload_dense(n, N, Q, lam, out)) {
        (void)hipGetLastError();
        return fail(DG_E_NOMEM, "dense eigenbasis upload (%zu bytes) failed",
                    dense_axis_bytes(N, n));
    }
    return DG_OK;
}

template <class T>
int apply_dense(const FdDevice* fd, hipStream_t s) {
    rocblas_handle h = (rocblas_handle)fd->blas;
    rocblas_status st = rocblas_set_stream(h, s);
    if (st != rocblas_status_success) return blas_fail(st, "rocblas_set_stream");
    const FdDenseAxis& X = fd->dx;
    const FdDenseAxis& Y = fd->dy;
    const rocblas_int mx = X.m, my = Y.m;
    T* a = reinterpret_cast<T*>(fd->img0);
    T* b = reinterpret_cast<T*>(fd->img1);
    const T* qx = X.q<T>();
    const T* qy = Y.q<T>();
    const rocblas_operation N_ = rocblas_operation_none, T_ = rocblas_operation_transpose;
    st = gemm(h, T_, N_, mx, my, mx, qx, mx, 0, a, mx, 0, b, mx, 0, 1);          // B = Qx^T A
    if (st == rocblas_status_success)
        st = gemm(h, N_, N_, mx, my, my, b, mx, 0, qy, my, 0, a, mx, 0, 1);      // A = B Qy
    if (st != rocblas_status_success) return blas_fail(st, "dense forward transform");
    hipError_t e = launch_dense_divide<T>(mx, my, X.lam<T>(), Y.lam<T>(), a, s);
    if (e != hipSuccess) return hip_fail(e, "dense spectral division launch");
    st = gemm(h, N_, N_, mx, my, mx, qx, mx, 0, a, mx, 0, b, mx, 0, 1);          // B = Qx A
    if (st == rocblas_status_success)
        st = gemm(h, N_, T_, mx, my, my, b, mx, 0, qy, my, 0, a, mx, 0, 1);      // A = B Qy^T
    if (st != rocblas_status_success) return blas_fail(st, "dense inverse transform");
    return DG_OK;
}

// One batched 1D complex FFT of length H = L/2 along an axis of L cells:
// `count` rows of L real values (distance L), each read as H interleaved
// complex values, the spectra stored row by row in the same way.
int make_plan(bool forward, bool fp32, size_t L, size_t count, rocfft_plan* out) {
    rocfft_plan_description d = nullptr;
    rocfft_status st = rocfft_plan_description_create(&d);
    if (st != rocfft_status_success) return fft_fail(st, "plan description");
    const size_t one = 1, H = L / 2;
    st = rocfft_plan_description_set_data_layout(
        d, rocfft_array_type_complex_interleaved, rocfft_array_type_complex_interleaved, nullptr,
        nullptr, 1, &one, H, 1, &one, H);
    if (st == rocfft_status_success)
        st = rocfft_plan_create(out, rocfft_placement_notinplace,
                                forward ? rocfft_transform_type_complex_forward
                                        : rocfft_transform_type_complex_inverse,
                                fp32 ? rocfft_precision_single : rocfft_precision_double, 1, &H,
                                count, d);
    (void)rocfft_plan_description_destroy(d);
    if (st != rocfft_status_success) return fft_fail(st, "plan create");
    return DG_OK;
}

int make_fft(const dg_grid* g, FdDevice* fd) {
    static std::once_flag once;
    static rocfft_status setup = rocfft_status_success;
    std::call_once(once, [] { setup = rocfft_setup(); });
    if (setup != rocfft_status_success) return fft_fail(setup, "rocfft_setup");
    const size_t n = g->n, Nx = g->nx, Ny = g->ny;
    const size_t bx = Ny * n * n, by = n * n * Nx;    // transforms per axis
    for (int pr = 0; pr < 2; ++pr) {
        rocfft_plan plans[4] = {nullptr, nullptr, nullptr, nullptr};
        int rc = make_plan(true, pr == 1, Nx, bx, &plans[0]);
        if (rc == DG_OK) rc = make_plan(true, pr == 1, Ny, by, &plans[1]);
        if (rc == DG_OK) rc = make_plan(false, pr == 1, Ny, by, &plans[2]);
        if (rc == DG_OK) rc = make_plan(false, pr == 1, Nx, bx, &plans[3]);
        for (int i = 0; i < 4; ++i) fd->fft[pr][i] = plans[i];
        if (rc != DG_OK) return rc;
        for (int i = 0; i < 4; ++i) {
            size_t w = 0;
            rocfft_status st = rocfft_plan_get_work_buffer_size(plans[i], &w);
            if (st != rocfft_status_success) return fft_fail(st, "work buffer size");
            if (w > fd->fft_work_bytes) fd->fft_work_bytes = w;
        }
    }
    rocfft_execution_info info = nullptr;
    rocfft_status st = rocfft_execution_info_create(&info);
    if (st != rocfft_status_success) return fft_fail(st, "execution info");
    fd->fft_info = info;
    if (fd->fft_work_bytes &&
        hipMalloc(&fd->fft_work, fd->fft_work_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DG_E_NOMEM, "FFT work buffer of %zu bytes", fd->fft_work_bytes);
    }
    if (fd->fft_work_bytes) {
        st = rocfft_execution_info_set_work_buffer(info, fd->fft_work, fd->fft_work_bytes);
        if (st != rocfft_status_success) return fft_fail(st, "work buffer");
    }
    return DG_OK;
}

}  // namespace

void fd_destroy(FdDevice* fd) {
    if (!fd) return;
    if (fd->blas) (void)rocblas_destroy_handle((rocblas_handle)fd->blas);
    for (auto& pr : fd->fft)
        for (void* p : pr)
            if (p) (void)rocfft_plan_destroy((rocfft_plan)p);
    if (fd->fft_info) (void)rocfft_execution_info_destroy((rocfft_execution_info)fd->fft_info);
    if (fd->fft_work) (void)hipFree(fd->fft_work);
    if (fd->img0) (void)hipFree(fd->img0);
    if (fd->img1) (void)hipFree(fd->img1);
    free_axis(&fd->x);
    if (!fd->shared) free_axis(&fd->y);
    free_dense(&fd->dx);
    if (!fd->shared) free_dense(&fd->dy);
    delete fd;
}

namespace {

// The mixing kernels read only the first n rows of each 2n x 2n block: rows
// n + q must be [-T1 | T0] of rows q = [T0 | T1], in the forward and the
// inverse blocks, and the cos and sin modes of a wave number must share their
// eigenvalues, exactly (both cell Fourier bases are built that way: the
// shifted one is the unshifted one times a rotation per node, itself a
// complex product).
static bool complex_blocks(const FdFactors& f) {
    const int n = f.n, S = 2 * n;
    for (int k = 0; k < f.K; ++k) {
        if (f.csin[k] < 0) continue;
        for (const std::vector<double>* m : {&f.mf, &f.mi}) {
            const double* b = m->data() + (size_t)k * S * S;
            for (int q = 0; q < n; ++q)
                for (int p = 0; p < n; ++p)
                    if (b[(n + q) * S + p] != -b[q * S + n + p] ||
                        b[(n + q) * S + n + p] != b[q * S + p])
                        return false;
        }
        for (int a = 0; a < n; ++a)
            if (f.lam[(size_t)a * f.N + f.ccos[k]] != f.lam[(size_t)a * f.N + f.csin[k]])
                return false;
    }
    return true;
}

int fd_create_dense(const dg_grid* g, FdDevice* fd) {
    const size_t img = (size_t)g->n * g->n * g->nx * g->ny * sizeof(double);
    if (hipMalloc((void**)&fd->img0, img) != hipSuccess ||
        hipMalloc((void**)&fd->img1, img) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DG_E_NOMEM, "preconditioner allocation of %zu bytes failed", fd_bytes(g));
    }
    rocblas_handle h = (rocblas_handle)fd->blas;
    int rc = dense_axis(g, 0, h, &fd->dx);
    if (rc != DG_OK) return rc;
    if (fd->shared) {
        fd->dy = fd->dx;
        return DG_OK;
    }
    return dense_axis(g, 1, h, &fd->dy);
}

}  // namespace

int fd_create(const dg_grid* g, bool products, FdDevice** out) {
    *out = nullptr;
    int rc0 = fd_supported(g);
    if (rc0 != DG_OK) return rc0;
    FdDevice* fd = new (std::nothrow) FdDevice;
    if (!fd) return fail(DG_E_NOMEM, "host allocation failed");
    fd->n = g->n;
    fd->shared = same_axis(g);
    if (has_dirichlet(g)) {
        fd->dense = true;
        fd->use_fft = false;
        rocblas_handle h = nullptr;
        rocblas_status st = rocblas_create_handle(&h);
        if (st != rocblas_status_success) {
            delete fd;
            return blas_fail(st, "rocblas_create_handle");
        }
        fd->blas = h;
        rc0 = fd_create_dense(g, fd);
        if (rc0 != DG_OK) {
            fd_destroy(fd);
            return rc0;
        }
        fd->bytes = fd_bytes(g);
        *out = fd;
        return DG_OK;
    }
    fd->use_fft = !products && fd_uses_fft(g->nx, g->ny);
    FdFactors fx, fy;
    double ex = 0.0, ey = 0.0;
    if (!fd_axis_factors(g->t, g->nx, g->hx, &fx, &ex, !fd->use_fft) ||
        (!fd->shared && !fd_axis_factors(g->t, g->ny, g->hy, &fy, &ey, !fd->use_fft))) {
        delete fd;
        return fail(DG_E_INVAL, "eigenbasis construction failed");
    }
    if (ex > 1e-10 || ey > 1e-10) {
        delete fd;
        return fail(DG_E_INVAL, "eigenbasis defect %.3e too large", ex > ey ? ex : ey);
    }
    if (!complex_blocks(fx) || (!fd->shared && !complex_blocks(fy))) {
        delete fd;
        return fail(DG_E_INVAL, "mixing blocks lack the structure the mixing kernels use");
    }
    bool ok = upload_axis(fx, &fd->x);
    if (ok && fd->shared) fd->y = fd->x;
    else if (ok) ok = upload_axis(fy, &fd->y);
    const size_t img = field_reals(g->n, g->nx, g->ny) * sizeof(double);
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
    if (fd->use_fft) {
        const int rc = make_fft(g, fd);
        if (rc != DG_OK) { fd_destroy(fd); return rc; }
    }
    fd->bytes = fd_bytes(g) + fd->fft_work_bytes;
    *out = fd;
    return DG_OK;
}

// Device bytes the preconditioner holds beyond fd_bytes(): rocFFT's work
// buffer (known once the plans exist) and what rocBLAS reports for its
// handle.
size_t fd_extra_bytes(const FdDevice* fd) {
    if (!fd) return 0;
    size_t blas = 0;
    if (fd->blas &&
        rocblas_get_device_memory_size((rocblas_handle)fd->blas, &blas) != rocblas_status_success)
        blas = 0;
    return fd->fft_work_bytes + blas;
}

// img0 holds the work image of r on entry and that of z = M r on exit
// (FP32 when fp32): the dense image (dense path), node planes (FFT path) or
// node planes folded along x (matrix-product path).
int fd_layout(const FdDevice* fd) {
    return fd->dense ? kFdDense : (fd->use_fft ? kFdPlanes : kFdFolded);
}

int fd_apply_image(const FdDevice* fd, bool fp32, hipStream_t s) {
    if (fd->dense) return fp32 ? apply_dense<float>(fd, s) : apply_dense<double>(fd, s);
    if (fd->use_fft) return fp32 ? apply_fft<float>(fd, s) : apply_fft<double>(fd, s);
    return fp32 ? apply_planes<float>(fd, s) : apply_planes<double>(fd, s);
}

}  // namespace dgk

// Kernel launchers of libdgark (cg_kernels.hip, rhs_kernels.hip,
// pointwise.hip).  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dgk {

struct RhsParams {
    double c0, c1, c2, scale;   // bracket form coefficients
    double D, dt, a, b;         // viscosity and RK-stage combination
    int only_r;                 // 1: out = -J + D Lap_h g (no stage combination)
};

// Blocks of one launch of each stencil family for the grid's tile shapes;
// stencil_blocks is the maximum over every tile shape.  The reduction
// partials buffer holds at least max(stencil_blocks, pointwise_block_cap)
// entries.
int row_blocks(const Geom& g);
int cell_blocks(const Geom& g);
int stencil_blocks(const Geom& g);
int pointwise_block_cap();

// Elements of one CG vector in the lane-interleaved layout (cells grouped by
// 64 along x, node pairs inside a group): ny * ceil(nx/64) * n*n * 64.
inline size_t l64_elems(const Geom& g) {
    return (size_t)g.ny * (size_t)((g.nx + 63) / 64) * (size_t)(g.n * g.n) * 64;
}

hipError_t launch_laplace(const Geom& g, const OpConst<double>& k,
                          const double* u, double* out, hipStream_t s);
hipError_t launch_rhs(const Geom& g, const OpConst<double>& k, const double* f,
                      const double* gg, const double* wn, double* out,
                      const RhsParams& p, bool visc, hipStream_t s);
hipError_t launch_cg_mean(const Geom& g, const OpConst<double>& k,
                          const double* omega, const double* pa,
                          const double* pb, double ca, double cb, double area,
                          double tol2, int max_iter, const DevScratch& d,
                          hipStream_t s);
// x, r: lane-interleaved; omega, pa, pb: canonical
hipError_t launch_cg_init(const Geom& g, const OpConst<double>& k,
                          const double* omega, const double* pa,
                          const double* pb, double ca, double cb, double* x,
                          double* r, const DevScratch& d, hipStream_t s);
// CG iterations on vectors stored as S (double or float; the arithmetic is
// FP64 either way); the direction buffers p0/p1 alternate by the device
// iteration count (sc->iter), so any number of queued no-op iterations
// keeps them consistent.
template <class S>
hipError_t launch_cg_dir(const Geom& g, const OpConst<double>& k, double* x, S* r, S* p0,
                         S* p1, CgScalars* sc, const DevScratch& d, hipStream_t s);
template <class S>
hipError_t launch_cg_res(const Geom& g, const OpConst<double>& k, S* r, S* p0, S* p1,
                         CgScalars* sc, const DevScratch& d, hipStream_t s);
// Timed variants: start / stop events record the dispatch's own timestamps.
template <class S>
hipError_t launch_cg_dir_timed(const Geom& g, const OpConst<double>& k, double* x, S* r,
                               S* p0, S* p1, CgScalars* sc, const DevScratch& d,
                               hipStream_t s, hipEvent_t start, hipEvent_t stop);
template <class S>
hipError_t launch_cg_res_timed(const Geom& g, const OpConst<double>& k, S* r, S* p0, S* p1,
                               CgScalars* sc, const DevScratch& d, hipStream_t s,
                               hipEvent_t start, hipEvent_t stop);
template <class S>
hipError_t launch_cg_iter(const Geom& g, const OpConst<double>& k, double* x, S* r,
                          S* p0, S* p1, CgScalars* sc, const DevScratch& d,
                          hipStream_t s);
// psi (canonical) = x + pending alpha p (lane-interleaved; p stored as P =
// double or float), minus its W-mean
template <class P>
hipError_t launch_cg_finish(const Geom& g, const OpConst<double>& k,
                            const double* x, const P* p0, const P* p1,
                            double* psi, double area, const DevScratch& d,
                            hipStream_t s);
// x (canonical) -= its W-mean
hipError_t launch_mean_sub(const Geom& g, const OpConst<double>& k, double* x,
                           double area, const DevScratch& d, hipStream_t s);
hipError_t launch_invariants(const Geom& g, const OpConst<double>& k,
                             const double* omega, const double* psi,
                             double* out3, const DevScratch& d, hipStream_t s);
// Mixed precision (r, p stored in FP32, x in FP64, FP64 residual
// replacement; all vectors lane-interleaved): r32 = float(r64); the true
// residual of x + alpha p_last replaces r32.
hipError_t launch_mixed_start(const Geom& g, const OpConst<double>& k,
                              const double* r64, float* r32, const DevScratch& d,
                              hipStream_t s);
hipError_t launch_mixed_replace(const Geom& g, const OpConst<double>& k,
                                const double* omega, const double* x, const float* q0,
                                const float* q1, float* r32, const DevScratch& d,
                                hipStream_t s);
// Fast-diagonalisation preconditioner support (fd_kernels.hip): field ->
// node planes U[cell + nx ny q] (from canonical or lane-interleaved), planes
// -> canonical, planes -> z (lane-interleaved) with <r, z>_W closing the PCG
// step, and the y mixing + spectral scaling + unmixing (K blocks, M
// row-major 2n x 2n each, cols[2k] / cols[2k+1] the cos / sin columns of
// wave number k).  `dense`: the conversions
// use the dense image of the eigenbasis path instead of node planes (rows
// along x, values scaled by sqrt(W) on the way in and by its inverse on the
// way out), and launch_dense_divide is that path's spectral division.
// T = double, or float for the FP32 apply of the mixed-precision PCG.
template <class T>
hipError_t launch_to_image(const Geom& g, const OpConst<double>& k, const double* src,
                           bool from_l64, bool dense, T* img, hipStream_t s);
template <class T>
hipError_t launch_from_image(const Geom& g, const OpConst<double>& k, const T* img, bool dense,
                             double* dst, hipStream_t s);
template <class T>
hipError_t launch_from_image_dot(const Geom& g, const OpConst<double>& k, const T* img,
                                 bool dense, double* z, const double* r, const DevScratch& d,
                                 hipStream_t s);
template <class T>
hipError_t launch_dense_divide(int mx, int my, const T* lx, const T* ly, T* c, hipStream_t s);
// The matrix-product path on node planes folded along x (E = u[c] +
// u[N - 1 - c] at column c < Kx = ceil(N/2), O = u[c] - u[N - 1 - c] at column
// Kx + c): conversions in (from L64 or canonical) and out (to canonical, or
// with d to L64 z plus <r, z>_W), and the x mixing out of place combined
// with the fold (forward) or unfold (inverse) of the y axis, Ky = ceil(Ny/2).
template <class T>
hipError_t launch_to_planes_fold(const Geom& g, const double* src, bool from_l64, int Kx, T* img,
                                 hipStream_t s);
template <class T>
hipError_t launch_from_planes_fold(const Geom& g, const OpConst<double>& k, const T* img, int Kx,
                                   double* dst, const double* r, const DevScratch* d,
                                   hipStream_t s);
template <class T>
hipError_t launch_fd_mix_x_fold(bool inverse, int n, int Nx, int Ny, int Ky, int K,
                                const int* cols, const T* M, const T* in, T* out,
                                hipStream_t s);
template <class T>
hipError_t launch_fd_mix_y(int n, int Nx, int Ny, int K, const int* cols, const T* Mf,
                           const T* Mi, const T* lx, const T* ly, int zx, int zy, T* u,
                           hipStream_t s);
// The same mixing on the packed spectra of the FFTs along the cells (X, Y:
// interleaved complex of type T, N/2 per real row; layouts in fd_kernels.hip).
template <class T>
hipError_t launch_fft_mix_x_fwd(int n, int Nx, int Ny, const int* cols, const T* Mf,
                                const void* X, T* u1, hipStream_t s);
template <class T>
hipError_t launch_fft_mix_x_inv(int n, int Nx, int Ny, const int* cols, const T* Mi,
                                const T* u1, void* X, hipStream_t s);
template <class T>
hipError_t launch_fft_mix_y(int n, int Nx, int Ny, const int* cols, const T* Mf,
                            const T* Mi, const T* lx, const T* ly, int zx, int zy, void* Y,
                            hipStream_t s);
hipError_t launch_guess(long elems, double* x, const double* pa,
                        const double* pb, double ca, double cb, hipStream_t s);
// Adams-Bashforth update omega += sum_{j<K} c[j] R[j] (element-wise, in the
// order j = 0..K-1), K in [1, 4].
hipError_t launch_ab_combine(long elems, double* omega, const double* const* R,
                             const double* c, int K, hipStream_t s);

}  // namespace dgk

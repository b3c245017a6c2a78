// Device kernels of the fast-diagonalisation preconditioner.  Its fields
// live in node planes: U[cell + nx ny (i + n j)] (cell = cy nx + cx), so the
// cell Fourier transforms along x and y are plain matrix products over whole
// planes (folded along x, see k_to_planes_fold) or batched FFTs.  Here:
// the conversions between the CG layouts and the planes, the per-wave-number
// mixing of the x transform (with the fold of the y axis), the mixing +
// spectral scaling + unmixing of the y transform, the same mixings on packed
// spectra for the FFT path, the dense path's conversions and division, and
// the preconditioned dot product <r, z>_W that closes the PCG step.
#include <cmath>
#include <type_traits>

#include "cg_body.h"
#include "dg_launch.h"

namespace dgk {

namespace {

// Where node q = i + n j of cell (cx, cy) sits in the work field: node
// planes [cell + nx ny q], or (Dense, the eigenbasis path of grids with a
// Dirichlet axis) the image [(cx + nx i) + n nx (cy + ny j)], a column-major
// (n nx) x (n ny) matrix whose rows run along x.  Consecutive cells along x
// stay consecutive either way.
template <int N, bool Dense>
__device__ __forceinline__ long fd_at(const Geom& g, long cell, int cx, int cy, int q) {
    if (!Dense) return cell + (long)g.nx * g.ny * q;
    const int i = q % N, j = q / N;
    return cx + (long)g.nx * i + (long)N * g.nx * (cy + (long)g.ny * j);
}

// sqrt(W) at the nodes of one cell (the dense path works with the
// orthogonal Q = W^{1/2} V, so fields enter scaled by sqrt(W) and leave
// scaled by its inverse)
template <int N>
__device__ __forceinline__ void sqrt_w(const OpConst<double>& k, double (&sw)[N * N]) {
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) sw[j * N + i] = sqrt(k.w[i] * k.w[j] * k.wq);
}

template <int N, bool FromL64, bool Dense, class T>
__global__ __launch_bounds__(kPwThreads) void k_to_image(Geom g, OpConst<double> k,
                                                         const double* __restrict__ src,
                                                         T* __restrict__ img) {
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    double sw[N * N];
    if (Dense) sqrt_w<N>(k, sw);
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const CellRef c = cell_ref<N>(g, G, cx, cy);
        double u[N * N];
        if (FromL64) ld_l64<N>(src, c, u);
        else ld_canon<N>(src, c, u);
#pragma unroll
        for (int q = 0; q < N * N; ++q)
            img[fd_at<N, Dense>(g, cell, cx, cy, q)] = (T)(Dense ? u[q] * sw[q] : u[q]);
    }
}

template <int N, bool Dense, class T>
__global__ __launch_bounds__(kPwThreads) void k_from_image(Geom g, OpConst<double> k,
                                                           const T* __restrict__ img,
                                                           double* __restrict__ dst) {
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    double sw[N * N];
    if (Dense) sqrt_w<N>(k, sw);
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const CellRef c = cell_ref<N>(g, G, cx, cy);
        double u[N * N];
#pragma unroll
        for (int q = 0; q < N * N; ++q) {
            u[q] = (double)img[fd_at<N, Dense>(g, cell, cx, cy, q)];
            if (Dense) u[q] /= sw[q];
        }
        st_canon<N>(dst, c, u);
    }
}

// The last block of a <r, z>_W reduction: rz and, past the first iteration,
// beta = <r,z>_new / <r,z>_old; a non-positive or non-finite <r,z> ends the
// solve as a breakdown.
__device__ __forceinline__ void set_rz(double rz, CgScalars* sc) {
    sc->precond = 1;
    if (!(rz > 0.0) || !(rz < __builtin_inf())) {
        // <r, M r> must be positive and finite for a nonzero residual:
        // stop; x still lacks the last alpha p after any iteration, and the
        // one before it after an odd one (iter = the next iteration's k)
        sc->done = 1;
        sc->breakdown = 1;
        sc->pending = sc->first == 1 ? 0 : ((sc->iter & 1) ? 1 : 2);
    } else {
        if (sc->first != 1) sc->beta = rz / sc->rz;
        sc->rz = rz;
    }
}

// Folded node planes of the matrix-product path: along x, cells c and
// N - 1 - c share the even basis columns and the odd ones with opposite
// signs, so the planes hold E[c] = u[c] + u[N - 1 - c] at column c
// (c = 0 .. Kx - 1, Kx = ceil(N/2); u[c] alone for the middle cell of an odd
// N) and O[c] = u[c] - u[N - 1 - c] at column Kx + c.  One thread per cell
// pair.
__device__ __forceinline__ bool fold_pair(int c, int N) { return 2 * c + 1 != N; }

template <int N, bool FromL64, class T>
__global__ __launch_bounds__(kPwThreads) void k_to_planes_fold(Geom g, const double* __restrict__ src,
                                                               T* __restrict__ img, int Kx) {
    const long pairs = (long)Kx * g.ny, cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    for (long t = blockIdx.x * (long)kPwThreads + threadIdx.x; t < pairs;
         t += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(t / Kx), c = (int)(t - (long)cy * Kx);
        const bool pr = fold_pair(c, g.nx);
        double a[N * N], b[N * N];
        const CellRef ca = cell_ref<N>(g, G, c, cy);
        if (FromL64) ld_l64<N>(src, ca, a);
        else ld_canon<N>(src, ca, a);
        if (pr) {
            const CellRef cb = cell_ref<N>(g, G, g.nx - 1 - c, cy);
            if (FromL64) ld_l64<N>(src, cb, b);
            else ld_canon<N>(src, cb, b);
        }
        const long e0 = c + (long)g.nx * cy, o0 = Kx + c + (long)g.nx * cy;
#pragma unroll
        for (int q = 0; q < N * N; ++q) {
            img[e0 + cells * q] = (T)(pr ? a[q] + b[q] : a[q]);
            if (pr) img[o0 + cells * q] = (T)(a[q] - b[q]);
        }
    }
}

// Unfolding: u[c] = E[c] + O[c], u[N - 1 - c] = E[c] - O[c], stored canonical,
// or (Dot) lane-interleaved as z with <r, z>_W reduced as in k_from_image_dot.
template <int N, bool Dot, class T>
__global__ __launch_bounds__(kPwThreads) void k_from_planes_fold(
    Geom g, OpConst<double> k, const T* __restrict__ img, int Kx, double* __restrict__ dst,
    const double* __restrict__ r, CgScalars* sc, unsigned* counter, double* partials) {
    if (Dot && sc->done) return;
    const long pairs = (long)Kx * g.ny, cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    double part[1] = {0.0};
    for (long t = blockIdx.x * (long)kPwThreads + threadIdx.x; t < pairs;
         t += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(t / Kx), c = (int)(t - (long)cy * Kx);
        const bool pr = fold_pair(c, g.nx);
        const long e0 = c + (long)g.nx * cy, o0 = Kx + c + (long)g.nx * cy;
        double a[N * N], b[N * N];
#pragma unroll
        for (int q = 0; q < N * N; ++q) {
            const double ev = (double)img[e0 + cells * q];
            const double od = pr ? (double)img[o0 + cells * q] : 0.0;
            a[q] = ev + od;
            b[q] = ev - od;
        }
        const CellRef ca = cell_ref<N>(g, G, c, cy);
        if (Dot) {
            double rv[N * N];
            st_l64<N>(dst, ca, a);
            ld_l64<N>(r, ca, rv);
            part[0] += wdot_cell<N>(k, rv, a);
        } else {
            st_canon<N>(dst, ca, a);
        }
        if (pr) {
            const CellRef cb = cell_ref<N>(g, G, g.nx - 1 - c, cy);
            if (Dot) {
                double rv[N * N];
                st_l64<N>(dst, cb, b);
                ld_l64<N>(r, cb, rv);
                part[0] += wdot_cell<N>(k, rv, b);
            } else {
                st_canon<N>(dst, cb, b);
            }
        }
    }
    if (Dot) {
        double tot[1];
        if (reduce_last<1, kPwThreads>(part, partials, counter, gridDim.x, blockIdx.x, tot) &&
            threadIdx.x == 0)
            set_rz(tot[0], sc);
    }
}

// z = image (to L64) and <r, z>_W; the last block sets rz and, past the
// first iteration, beta = <r,z>_new / <r,z>_old (no-op once the solve is
// done; a non-positive or non-finite <r,z> ends the solve as a breakdown).
template <int N, bool Dense, class T>
__global__ __launch_bounds__(kPwThreads) void k_from_image_dot(
    Geom g, OpConst<double> k, const T* __restrict__ img, double* __restrict__ z,
    const double* __restrict__ r, CgScalars* sc, unsigned* counter, double* partials) {
    if (sc->done) return;
    const long cells = (long)g.nx * g.ny;
    const int G = (g.nx + 63) / 64;
    double sw[N * N];
    if (Dense) sqrt_w<N>(k, sw);
    double part[1] = {0.0};
    for (long cell = blockIdx.x * (long)kPwThreads + threadIdx.x; cell < cells;
         cell += (long)gridDim.x * kPwThreads) {
        const int cy = (int)(cell / g.nx), cx = (int)(cell - (long)cy * g.nx);
        const CellRef c = cell_ref<N>(g, G, cx, cy);
        double u[N * N], rv[N * N];
#pragma unroll
        for (int q = 0; q < N * N; ++q) {
            u[q] = (double)img[fd_at<N, Dense>(g, cell, cx, cy, q)];
            if (Dense) u[q] /= sw[q];
        }
        st_l64<N>(z, c, u);
        ld_l64<N>(r, c, rv);
        part[0] += wdot_cell<N>(k, rv, u);
    }
    double tot[1];
    if (reduce_last<1, kPwThreads>(part, partials, counter, gridDim.x, blockIdx.x, tot) &&
        threadIdx.x == 0)
        set_rz(tot[0], sc);
}

// out = M v for one 2n-vector (M row-major, S = 2n, row = output index);
// PAIR false: only the leading n x n block (wave numbers 0 and N/2).
template <int N, class T, bool PAIR>
__device__ __forceinline__ void mix_vec(const T* __restrict__ M, const T* v, T* out) {
    constexpr int S = 2 * N;
    constexpr int R = PAIR ? S : N;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        T acc = 0;
#pragma unroll
        for (int p = 0; p < R; ++p) acc = fma(M[q * S + p], v[p], acc);
        out[q] = acc;
    }
}

// out = M v for the mixing blocks, which have the structure of a complex
// product: rows n + q are [-T1 | T0] of rows q = [T0 | T1] (forward and
// inverse, unshifted and shifted bases alike, exactly: the same products with
// one sign flipped; the host checks it), so only the first n rows are read
// and every output keeps the summation order of the full product.  PAIR
// false: the n x n block.
template <int N, class T, bool PAIR>
__device__ __forceinline__ void mix_vec_c(const T* __restrict__ M, const T* v, T* out) {
    constexpr int S = 2 * N;
    if constexpr (!PAIR) {
        mix_vec<N, T, false>(M, v, out);
    } else {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            T top = 0, bot = 0;
#pragma unroll
            for (int p = 0; p < N; ++p) {
                top = fma(M[q * S + p], v[p], top);
                bot = fma(-M[q * S + N + p], v[p], bot);
            }
#pragma unroll
            for (int p = 0; p < N; ++p) {
                top = fma(M[q * S + N + p], v[N + p], top);
                bot = fma(M[q * S + p], v[N + p], bot);
            }
            out[q] = top;
            out[N + q] = bot;
        }
    }
}

// 1 / d from the hardware reciprocal refined by Newton's iteration
// r <- r + r (1 - d r) (twice in FP64, once in FP32): within about one ulp
// of the correctly rounded quotient at a fraction of an IEEE division's
// instructions.  The spectral division of the preconditioner only has to
// approximate the exact inverse (the PCG iteration measures its residual in
// FP64), so the last bit does not matter there.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}
__device__ __forceinline__ float recip(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(r, fmaf(-d, r, 1.0f), r);
}

// Call f(std::true_type) or f(std::false_type) for a (wave-uniform) pair
// flag, so that the mixing code is compiled with the vector length fixed.
template <class F>
__device__ __forceinline__ void with_pair(bool pair, F&& f) {
    if (pair)
        f(std::true_type{});
    else
        f(std::false_type{});
}

// The x mixing of the matrix-product path, out of place, combined with the
// fold of the y axis (the next transform): Inv = false reads U1 and writes
// the mixed rows folded along y (rows E[cy], cy < Ky, and O[cy] at row
// Ky + cy, as for x above); Inv = true reads folded rows (the inverse y
// transform's output), unfolds them to rows cy and Ny - 1 - cy and applies M.
// One thread per (j, cy < Ky), two 2n-vectors each.
template <int N, class T, bool Inv>
__global__ __launch_bounds__(kPwThreads) void k_fd_mix_x_fold(int Nx, int Ny, int Ky,
                                                              const int* __restrict__ cols,
                                                              const T* __restrict__ M,
                                                              const T* __restrict__ in,
                                                              T* __restrict__ out) {
    constexpr int S = 2 * N;
    const int k = blockIdx.y;
    const int c0 = cols[2 * k], c1 = cols[2 * k + 1];
    const bool pair = c1 >= 0;
    const T* Mk = M + (size_t)k * S * S;
    const long per = (long)Ky * N;
    with_pair(pair, [&](auto pc) {
        constexpr bool PAIR = decltype(pc)::value;
        for (long t = blockIdx.x * (long)kPwThreads + threadIdx.x; t < per;
             t += (long)gridDim.x * kPwThreads) {
            const int j = (int)(t / Ky), cy = (int)(t - (long)j * Ky);
            const bool pr = fold_pair(cy, Ny);
            const long jb = (long)Ny * N * Nx * j;
            const long s0 = (long)Ny * N * c0, s1 = (long)Ny * N * (PAIR ? c1 : c0);
            // rows: A (cy) and B (Ny - 1 - cy) unfolded, E (cy) and O (Ky + cy) folded
            const long rA = jb + cy, rB = jb + (Ny - 1 - cy), rE = jb + cy, rO = jb + (Ky + cy);
            const long r0 = Inv ? rE : rA, r1 = Inv ? rO : rB;    // rows read
            const long w0 = Inv ? rA : rE, w1 = Inv ? rB : rO;    // rows written
            T va[S], vb[S], wa[S], wb[S];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const T a0 = in[r0 + s0 + (long)Ny * i];
                const T a1 = PAIR ? in[r0 + s1 + (long)Ny * i] : T(0);
                const T b0 = pr ? in[r1 + s0 + (long)Ny * i] : T(0);
                const T b1 = (pr && PAIR) ? in[r1 + s1 + (long)Ny * i] : T(0);
                va[i] = a0 + b0;
                va[N + i] = a1 + b1;
                vb[i] = a0 - b0;
                vb[N + i] = a1 - b1;
            }
            mix_vec_c<N, T, PAIR>(Mk, va, wa);
            if (pr) mix_vec_c<N, T, PAIR>(Mk, vb, wb);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                out[w0 + s0 + (long)Ny * i] = wa[i];
                if (PAIR) out[w0 + s1 + (long)Ny * i] = wa[N + i];
                if (pr) {
                    out[w1 + s0 + (long)Ny * i] = wb[i];
                    if (PAIR) out[w1 + s1 + (long)Ny * i] = wb[N + i];
                }
            }
        }
    });
}

// Mixing of the y transform, spectral scaling and unmixing, on
// U2[m + n Nx (j + n c)] with m = i + n kx the x mode (a = i, column kx,
// eigenvalue lx[i Nx + kx]) and c the cell Fourier column along y.  Block
// row k = blockIdx.y is one y wave number: per x mode, the 2n-vector at
// columns cols[2k], cols[2k+1] over the nodes j goes to y modes by Mf_k,
// each y mode (b, column c) is divided by -(lx + ly[b Ny + c]) (the constant
// mode, x slot zx and y slot zy, is set to zero), and Mi_k maps back.
template <int N, class T>
__global__ __launch_bounds__(kPwThreads) void k_fd_mix_y(
    int Nx, const int* __restrict__ cols, const T* __restrict__ Mf, const T* __restrict__ Mi,
    const T* __restrict__ lx, const T* __restrict__ ly, int Ny, int zx, int zy,
    T* __restrict__ u) {
    constexpr int S = 2 * N;
    const int k = blockIdx.y;
    const int c0 = cols[2 * k], c1 = cols[2 * k + 1];
    const bool pair = c1 >= 0;
    const T* Mfk = Mf + (size_t)k * S * S;
    const T* Mik = Mi + (size_t)k * S * S;
    const long NXn = (long)N * Nx;
    with_pair(pair, [&](auto pc) {
        constexpr bool PAIR = decltype(pc)::value;
        for (long m = blockIdx.x * (long)kPwThreads + threadIdx.x; m < NXn;
             m += (long)gridDim.x * kPwThreads) {
            const int kx = (int)(m / N), i = (int)(m - (long)kx * N);
            const int xs = i * Nx + kx;
            const T lam_x = lx[xs];
            const long o0 = m + NXn * N * c0;
            const long o1 = m + NXn * N * (PAIR ? c1 : c0);
            T v[S], w[S];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                v[j] = u[o0 + NXn * j];
                if (PAIR) v[N + j] = u[o1 + NXn * j];
            }
            mix_vec_c<N, T, PAIR>(Mfk, v, w);
            // the cos and sin modes of one (b, k) share the eigenvalue
            // ly[b Ny + c0]; the constant mode is a cos mode (k = 0)
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const int ys = q * Ny + c0;
                const T r = recip(lam_x + ly[ys]);
                w[q] = (xs == zx && ys == zy) ? T(0) : -w[q] * r;
                if (PAIR) w[N + q] = -w[N + q] * r;
            }
            mix_vec_c<N, T, PAIR>(Mik, w, v);
#pragma unroll
            for (int j = 0; j < N; ++j) {
                u[o0 + NXn * j] = v[j];
                if (PAIR) u[o1 + NXn * j] = v[N + j];
            }
        }
    });
}

// ---- The same steps with the cell transforms as FFTs.  A real row u of
// even length N is transformed as the complex row z_c = u_{2c} + i u_{2c+1}
// of length H = N/2 (rocFFT, spectra stored row by row like the input).
// The real row's half spectrum X_k = sum_c u_c e^{-2 pi i k c / N} follows
// from Z_k and Z_{H-k} (indices mod H): with E = (Z_k + conj Z_{H-k}) / 2
// and O = (Z_k - conj Z_{H-k}) / 2i, X_k = E + e^{-2 pi i k / N} O for
// k = 0..H.  Backwards, from a half spectrum Y the complex row Z_k = E + i O
// with E = Y_k + conj Y_{H-k} and O = (Y_k - conj Y_{H-k}) e^{2 pi i k / N}
// (k < H) has as unnormalised inverse transform the even (real part) and odd
// (imaginary part) samples of the real inverse transform of Y.  Wave numbers
// k and H - k take the same two values, so the blocks of wave pair p serve
// both (p = 0 with H, both in column 0).  For even H the wave number H/2 =
// N/4 is its own partner; its column rides in pair 0's partner slot, which
// would otherwise hold column 0 a second time, so the pairs are p = 0 .. P - 1
// with P = H/2 (even H) or (H + 1)/2 (odd H), and a launch has no chunk of
// pairs holding H/2 alone.  The orthonormal cos / sin coefficients of wave
// number k are
// sqrt(2/N) (Re X_k, -Im X_k) (k = 0 and N/2: 1/sqrt(N) Re X_k), and the
// real inverse transform of Y_k = sqrt(2/N)/2 (a - i b), Y_0 and Y_{N/2} =
// 1/sqrt(N) a, rebuilds sum a cos + b sin.  The mixing kernels convert
// between the three forms while they mix.

template <class T> struct CplxOf;
template <> struct CplxOf<double> { using type = double2; };
template <> struct CplxOf<float> { using type = float2; };

// Half-spectrum value -> the cos / sin coefficient pair (pair) or the single
// real coefficient, with the orthonormal scaling (cn = 1/sqrt(N),
// cp = sqrt(2/N)).
template <class C, class T>
__device__ __forceinline__ void spec_to_coef(const C z, bool pair, T cn, T cp, T& a, T& b) {
    if (pair) {
        a = cp * z.x;
        b = -cp * z.y;
    } else {
        a = cn * z.x;
        b = T(0);
    }
}

template <class C, class T>
__device__ __forceinline__ C coef_to_spec(bool pair, T cn, T cp, T a, T b) {
    C z;
    if (pair) {
        z.x = T(0.5) * cp * a;
        z.y = -T(0.5) * cp * b;
    } else {
        z.x = cn * a;
        z.y = T(0);
    }
    return z;
}

// Wave pairs of a packed spectrum of half length H (see above).
__host__ __device__ constexpr int spec_pairs(long H) {
    return (int)((H & 1) ? (H + 1) / 2 : H / 2);
}

// The column held in pair p's partner slot: H - p, or for p = 0 the column
// H/2 (even H) or 0 (odd H).
__device__ __forceinline__ long partner_col(int p, long H) {
    return p ? H - p : ((H & 1) ? 0 : H / 2);
}

// The wave numbers of pair p (H = N/2): k0 = p and k1 = H - p, with (c, s) =
// (cos, sin) of 2 pi k / N evaluated in FP64; mid: pair 0 of an even H also
// carries the wave number H/2 (cos, sin of pi/2 = 0, 1 exactly).
template <class T>
struct WavePair {
    int k0, k1;
    bool mid;
    T c0, s0, c1, s1;
    __device__ WavePair(int p, int N) {
        const int H = N / 2;
        k0 = p;
        k1 = H - p;
        mid = p == 0 && !(H & 1);
        c0 = T(cospi(2.0 * k0 / N));
        s0 = T(sinpi(2.0 * k0 / N));
        c1 = T(cospi(2.0 * k1 / N));
        s1 = T(sinpi(2.0 * k1 / N));
    }
};

// X_k from za = Z_k and zb = Z_{H-k}; (c, s) of 2 pi k / N.
template <class C, class T>
__device__ __forceinline__ C unpack_half(const C za, const C zb, T c, T s) {
    const T ex = T(0.5) * (za.x + zb.x), ey = T(0.5) * (za.y - zb.y);
    const T ox = T(0.5) * (za.y + zb.y), oy = -T(0.5) * (za.x - zb.x);
    C x;
    x.x = ex + c * ox + s * oy;
    x.y = ey + c * oy - s * ox;
    return x;
}

// Z_k from ya = Y_k and yb = Y_{H-k}; (c, s) of 2 pi k / N.
template <class C, class T>
__device__ __forceinline__ C pack_half(const C ya, const C yb, T c, T s) {
    const T ex = ya.x + yb.x, ey = ya.y - yb.y;
    const T dx = ya.x - yb.x, dy = ya.y + yb.y;
    const T ox = dx * c - dy * s, oy = dx * s + dy * c;
    C z;
    z.x = ex - oy;
    z.y = ey + ox;
    return z;
}

// Block -> (pair chunk pc, row block rb) for the FFT mixing kernels (grid
// chunks x row blocks).  Neighbouring chunks read neighbouring runs of the
// same spectrum rows (their partner columns share cache lines), so they
// should share one L2: workgroups go to the 8 XCDs in turn, and this map
// gives each XCD a contiguous run of (chunk fastest) blocks; the last
// total mod 8 blocks keep their place.
__device__ __forceinline__ void xcd_pair_block(int& pc, int& rb) {
    const int P = gridDim.x, total = P * gridDim.y;
    const int b = blockIdx.x + P * blockIdx.y, full = total & ~7;
    const int l = b < full ? (b & 7) * (full >> 3) + (b >> 3) : b;
    pc = l % P;
    rb = l / P;
}

// Packed spectra staged through LDS.  A block covers 64 consecutive values
// of a row coordinate a (lanes) and TP consecutive wave pairs p0 .. p0+TP-1
// (waves); spectrum row(a, i) (i < n) holds pair p's values at column p
// (s = 0) and at its partner column q = (H - p) mod H (s = 1).  Global loads
// and stores move runs of TP consecutive columns of one row (64 bytes); in
// the compute phase wave w owns pair p0 + w, so its mixing blocks come in
// through scalar loads, and lane a the row coordinate a0 + a, so the real
// fields it reads or writes are 64 consecutive values.  In the load and
// store phases a thread's element e runs over (pair, low bit of a, s, rest
// of a, row i), pair fastest; with runs of 64 values padded to 66 the lanes
// one LDS cycle serves (16 of 16-byte or 32 of 8-byte values) then fall in
// distinct banks.
template <int N, class T>
struct SpecTile {
    using C = typename CplxOf<T>::type;
    static constexpr int TP = 64 / (int)sizeof(C);          // 4 (FP64) or 8 (FP32)
    static constexpr int THREADS = 64 * TP;   // = 2048 / sizeof(T), the launch bound
    static_assert(THREADS == 2048 / (int)sizeof(T), "launch bound of the mixing kernels");
    static constexpr int RS = 66;                            // padded run of 64 values
    static constexpr int SIZE = N * 2 * TP * RS;
    __device__ static constexpr int at(int i, int s, int p, int a) {
        return ((i * 2 + s) * TP + p) * RS + a;
    }
};

// Element e of a tile in the load / store phases: pair p (fastest), low bit
// of a, s, a / 2, row i.
template <int TP>
__device__ __forceinline__ void spec_elem(int e, int& p, int& s, int& a, int& i) {
    p = e % TP;
    const int al = (e / TP) & 1;
    s = (e / (2 * TP)) & 1;
    a = 2 * ((e / (4 * TP)) & 31) + al;
    i = e / (4 * TP * 32);
}

// Load the block's tile: row(a, i) = base + a + stride * i for a < A, pairs
// p < P (entries outside stay zero).  Every thread issues its 2n loads
// before its first LDS store, so they are all in flight together.
template <int N, class T>
__device__ __forceinline__ void spec_load(const typename CplxOf<T>::type* __restrict__ Z,
                                          long H, int P, int p0, int a0, int A, long base,
                                          long stride, typename CplxOf<T>::type* L) {
    using TL = SpecTile<N, T>;
    using C = typename CplxOf<T>::type;
    constexpr int ITER = N * 64 * 2 * TL::TP / TL::THREADS;     // = 2n
    C v[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int e = threadIdx.x + it * TL::THREADS;
        int p, s, a, i;
        spec_elem<TL::TP>(e, p, s, a, i);
        const int pp = p0 + p;
        v[it].x = T(0);
        v[it].y = T(0);
        if (pp < P && a0 + a < A) {
            const long col = s ? partner_col(pp, H) : pp;
            v[it] = Z[(base + a0 + a + stride * i) * H + col];
        }
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int e = threadIdx.x + it * TL::THREADS;
        int p, s, a, i;
        spec_elem<TL::TP>(e, p, s, a, i);
        L[TL::at(i, s, p, a)] = v[it];
    }
}

// Store the tile back: column p from s = 0 and the partner column from s = 1
// (except pair 0 of an odd H, whose partner slot repeats column 0; column 0
// packs the wave numbers 0 and H).
template <int N, class T>
__device__ __forceinline__ void spec_store(typename CplxOf<T>::type* __restrict__ Z, long H,
                                           int P, int p0, int a0, int A, long base, long stride,
                                           const typename CplxOf<T>::type* L) {
    using TL = SpecTile<N, T>;
    constexpr int ITER = N * 64 * 2 * TL::TP / TL::THREADS;     // = 2n
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int e = threadIdx.x + it * TL::THREADS;
        int p, s, a, i;
        spec_elem<TL::TP>(e, p, s, a, i);
        const int pp = p0 + p;
        if (pp >= P || a0 + a >= A) continue;
        if (s && pp == 0 && (H & 1)) continue;
        const long col = s ? partner_col(pp, H) : pp;
        Z[(base + a0 + a + stride * i) * H + col] = L[TL::at(i, s, p, a)];
    }
}

// Forward x mixing from the x spectra Z[(cy + Ny (i + n j)) H + k] (H =
// Nx/2, k < H) into the real x-transformed field U1[cy + Ny (i + n c +
// n Nx j)] (c: the cos / sin columns of wave number k, as in the
// matrix-product path).  Grid: pair chunks x (cy blocks of 64, j).
template <int N, class T>
__global__ __launch_bounds__(2048 / sizeof(T)) void k_fft_mix_x_fwd(
    int Nx, int Ny, const int* __restrict__ cols, const T* __restrict__ Mf, T cn, T cp,
    const typename CplxOf<T>::type* __restrict__ Z, T* __restrict__ u1) {
    using TL = SpecTile<N, T>;
    using C = typename CplxOf<T>::type;
    constexpr int S = 2 * N;
    __shared__ C L[TL::SIZE];
    int pc, rb;
    xcd_pair_block(pc, rb);
    const int ab = (Ny + 63) / 64;
    const int j = rb / ab, a0 = (rb - j * ab) * 64;
    const long H = Nx / 2, base = (long)Ny * N * j;
    const int P = spec_pairs(H), p0 = pc * TL::TP;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), a = threadIdx.x & 63;
    const int p = p0 + w, cy = a0 + a;
    spec_load<N, T>(Z, H, P, p0, a0, Ny, base, Ny, L);
    __syncthreads();
    if (p >= P || cy >= Ny) return;
    const WavePair<T> wp(p, Nx);
    // pair 0 reads column 0 for both of its wave numbers (the partner slot
    // holds the wave number H/2 of an even H, done last)
    const int sb = p ? 1 : 0;
    C za[N], zb[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        za[i] = L[TL::at(i, 0, w, a)];
        zb[i] = L[TL::at(i, sb, w, a)];
    }
    const long out0 = cy + (long)Ny * N * Nx * j;
    // wave number k from its own half-spectrum value and its partner's
    auto one = [&](int k, const T* Mk, const C* zk, const C* zh, T c, T sn) {
        const int c0 = cols[2 * k], c1 = cols[2 * k + 1];
        with_pair(c1 >= 0, [&](auto pc) {
            constexpr bool PAIR = decltype(pc)::value;
            T v[S], o[S];
#pragma unroll
            for (int i = 0; i < N; ++i)
                spec_to_coef(unpack_half(zk[i], zh[i], c, sn), PAIR, cn, cp, v[i], v[N + i]);
            mix_vec_c<N, T, PAIR>(Mk, v, o);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                u1[out0 + (long)Ny * (i + (long)N * c0)] = o[i];
                if (PAIR) u1[out0 + (long)Ny * (i + (long)N * c1)] = o[N + i];
            }
        });
    };
    one(wp.k0, Mf + (size_t)wp.k0 * S * S, za, zb, wp.c0, wp.s0);
    one(wp.k1, Mf + (size_t)wp.k1 * S * S, zb, za, wp.c1, wp.s1);
    if (wp.mid) {
#pragma unroll
        for (int i = 0; i < N; ++i) za[i] = L[TL::at(i, 1, w, a)];
        const int km = (int)(H / 2);
        one(km, Mf + (size_t)km * S * S, za, za, T(0), T(1));
    }
}

// Inverse x mixing: U1 (real coefficients) -> the packed x spectra, ready for
// the inverse x transform (the packed values go through the LDS tile so the
// spectrum rows are written in runs).
template <int N, class T>
__global__ __launch_bounds__(2048 / sizeof(T)) void k_fft_mix_x_inv(
    int Nx, int Ny, const int* __restrict__ cols, const T* __restrict__ Mi, T cn, T cp,
    const T* __restrict__ u1, typename CplxOf<T>::type* __restrict__ Z) {
    using TL = SpecTile<N, T>;
    using C = typename CplxOf<T>::type;
    constexpr int S = 2 * N;
    __shared__ C L[TL::SIZE];
    int pc, rb;
    xcd_pair_block(pc, rb);
    const int ab = (Ny + 63) / 64;
    const int j = rb / ab, a0 = (rb - j * ab) * 64;
    const long H = Nx / 2, base = (long)Ny * N * j;
    const int P = spec_pairs(H), p0 = pc * TL::TP;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), a = threadIdx.x & 63;
    const int p = p0 + w, cy = a0 + a;
    __syncthreads();
    if (p < P && cy < Ny) {
        const WavePair<T> wp(p, Nx);
        const long in0 = cy + (long)Ny * N * Nx * j;
        // half-spectrum values of wave number k from its real coefficients
        auto one = [&](int k, const T* Mk, C* y) {
            const int c0 = cols[2 * k], c1 = cols[2 * k + 1];
            with_pair(c1 >= 0, [&](auto pc) {
                constexpr bool PAIR = decltype(pc)::value;
                T v[S], o[S];
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    v[i] = u1[in0 + (long)Ny * (i + (long)N * c0)];
                    if (PAIR) v[N + i] = u1[in0 + (long)Ny * (i + (long)N * c1)];
                }
                mix_vec_c<N, T, PAIR>(Mk, v, o);
#pragma unroll
                for (int i = 0; i < N; ++i)
                    y[i] = coef_to_spec<C>(PAIR, cn, cp, o[i], PAIR ? o[N + i] : T(0));
            });
        };
        C y0[N], y1[N];
        one(wp.k0, Mi + (size_t)wp.k0 * S * S, y0);
        one(wp.k1, Mi + (size_t)wp.k1 * S * S, y1);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            L[TL::at(i, 0, w, a)] = pack_half(y0[i], y1[i], wp.c0, wp.s0);
            L[TL::at(i, 1, w, a)] = pack_half(y1[i], y0[i], wp.c1, wp.s1);
        }
        if (wp.mid) {
            // the wave number H/2 is its own partner
            const int km = (int)(H / 2);
            one(km, Mi + (size_t)km * S * S, y0);
#pragma unroll
            for (int i = 0; i < N; ++i) L[TL::at(i, 1, w, a)] = pack_half(y0[i], y0[i], T(0), T(1));
        }
    }
    __syncthreads();
    spec_store<N, T>(Z, H, P, p0, a0, Ny, base, Ny, L);
}

// y mixing, spectral division and unmixing in place on the packed y spectra
// Z[(m + n Nx j) H + k] (m = i + n kx, H = Ny/2, k < H): spectrum -> y
// modes (Mf), divided by -(lam_x + lam_y), the constant mode zeroed, ->
// coefficients (Mi) -> spectrum.  A block reads and writes only the columns
// of its own pairs (p and H - p), so working in place is safe.  Grid: pair
// chunks x m blocks of 64.
template <int N, class T>
__global__ __launch_bounds__(2048 / sizeof(T)) void k_fft_mix_y(
    int Nx, int Ny, const int* __restrict__ cols, const T* __restrict__ Mf,
    const T* __restrict__ Mi, const T* __restrict__ lx, const T* __restrict__ ly, int zx, int zy,
    T cn, T cp, typename CplxOf<T>::type* __restrict__ Z) {
    using TL = SpecTile<N, T>;
    using C = typename CplxOf<T>::type;
    constexpr int S = 2 * N;
    __shared__ C L[TL::SIZE];
    int pc, rb;
    xcd_pair_block(pc, rb);
    const long NXn = (long)N * Nx, H = Ny / 2;
    const int P = spec_pairs(H), p0 = pc * TL::TP, a0 = rb * 64;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), a = threadIdx.x & 63;
    const int p = p0 + w;
    spec_load<N, T>(Z, H, P, p0, a0, (int)NXn, 0, NXn, L);
    __syncthreads();
    const long m = a0 + a;
    if (p < P && m < NXn) {
        const WavePair<T> wp(p, Ny);
        const int kx = (int)(m / N), i = (int)(m - (long)kx * N);
        const int xs = i * Nx + kx;
        const T lam_x = lx[xs];
        // pair 0 reads column 0 for both of its wave numbers (the partner
        // slot holds the wave number H/2 of an even H, done last)
        const int sb = p ? 1 : 0;
        C za[N], zb[N];
#pragma unroll
        for (int jj = 0; jj < N; ++jj) {
            za[jj] = L[TL::at(jj, 0, w, a)];
            zb[jj] = L[TL::at(jj, sb, w, a)];
        }
        // wave number k: spectrum -> y modes, divided, -> spectrum
        auto one = [&](int k, const T* Mfk, const T* Mik, const C* zk, const C* zh, T c, T sn,
                       C* y) {
            const int c0 = cols[2 * k], c1 = cols[2 * k + 1];
            with_pair(c1 >= 0, [&](auto pc) {
                constexpr bool PAIR = decltype(pc)::value;
                T v[S], o[S];
#pragma unroll
                for (int jj = 0; jj < N; ++jj)
                    spec_to_coef(unpack_half(zk[jj], zh[jj], c, sn), PAIR, cn, cp, v[jj],
                                 v[N + jj]);
                mix_vec_c<N, T, PAIR>(Mfk, v, o);
                // the cos and sin modes of one (b, k) share the eigenvalue
                // ly[b Ny + c0]; the constant mode is a cos mode (k = 0)
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    const int ys = q * Ny + c0;
                    const T r = recip(lam_x + ly[ys]);
                    o[q] = (xs == zx && ys == zy) ? T(0) : -o[q] * r;
                    if (PAIR) o[N + q] = -o[N + q] * r;
                }
                mix_vec_c<N, T, PAIR>(Mik, o, v);
#pragma unroll
                for (int jj = 0; jj < N; ++jj)
                    y[jj] = coef_to_spec<C>(PAIR, cn, cp, v[jj], PAIR ? v[N + jj] : T(0));
            });
        };
        C y0[N], y1[N];
        one(wp.k0, Mf + (size_t)wp.k0 * S * S, Mi + (size_t)wp.k0 * S * S, za, zb, wp.c0, wp.s0, y0);
        one(wp.k1, Mf + (size_t)wp.k1 * S * S, Mi + (size_t)wp.k1 * S * S, zb, za, wp.c1, wp.s1, y1);
        if (wp.mid) {
#pragma unroll
            for (int jj = 0; jj < N; ++jj) za[jj] = L[TL::at(jj, 1, w, a)];
        }
#pragma unroll
        for (int jj = 0; jj < N; ++jj) {
            L[TL::at(jj, 0, w, a)] = pack_half(y0[jj], y1[jj], wp.c0, wp.s0);
            L[TL::at(jj, 1, w, a)] = pack_half(y1[jj], y0[jj], wp.c1, wp.s1);
        }
        if (wp.mid) {
            const int km = (int)(H / 2);
            one(km, Mf + (size_t)km * S * S, Mi + (size_t)km * S * S, za, za, T(0), T(1), y0);
#pragma unroll
            for (int jj = 0; jj < N; ++jj)
                L[TL::at(jj, 1, w, a)] = pack_half(y0[jj], y0[jj], T(0), T(1));
        }
    }
    __syncthreads();
    spec_store<N, T>(Z, H, P, p0, a0, (int)NXn, 0, NXn, L);
}

// Spectral division of the dense path: C[a + mx b] /= -(lam_x[a] + lam_y[b])
// (a Dirichlet axis keeps every sum negative).
template <class T>
__global__ __launch_bounds__(kPwThreads) void k_dense_divide(int mx, int my,
                                                             const T* __restrict__ lx,
                                                             const T* __restrict__ ly,
                                                             T* __restrict__ c) {
    const long total = (long)mx * my;
    for (long t = blockIdx.x * (long)kPwThreads + threadIdx.x; t < total;
         t += (long)gridDim.x * kPwThreads) {
        const int b = (int)(t / mx), a = (int)(t - (long)b * mx);
        c[t] = c[t] / -(lx[a] + ly[b]);
    }
}

}  // namespace

template <class T>
hipError_t launch_to_image(const Geom& g, const OpConst<double>& k, const double* src,
                           bool from_l64, bool dense, T* img, hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
#define DG_TO_IMAGE(L64, DN)                                                                 \
    DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_to_image<NN, L64, DN, T>), dim3(nb),            \
                                          dim3(kPwThreads), 0, s, g, k, src, img))
    if (from_l64 && dense) {
        DG_TO_IMAGE(true, true);
    } else if (from_l64) {
        DG_TO_IMAGE(true, false);
    } else if (dense) {
        DG_TO_IMAGE(false, true);
    } else {
        DG_TO_IMAGE(false, false);
    }
#undef DG_TO_IMAGE
    return hipGetLastError();
}

template <class T>
hipError_t launch_from_image(const Geom& g, const OpConst<double>& k, const T* img, bool dense,
                             double* dst, hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    if (dense) {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_image<NN, true, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, k, img, dst));
    } else {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_image<NN, false, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, k, img, dst));
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_from_image_dot(const Geom& g, const OpConst<double>& k, const T* img,
                                 bool dense, double* z, const double* r, const DevScratch& d,
                                 hipStream_t s) {
    const long cells = (long)g.nx * g.ny;
    const int nb = pw_blocks(cells, pointwise_block_cap());
    if (dense) {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_image_dot<NN, true, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, k, img, z, r, d.sc,
                                              d.counters + kCntDot * kCntStride, d.partials));
    } else {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_image_dot<NN, false, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, k, img, z, r, d.sc,
                                              d.counters + kCntDot * kCntStride, d.partials));
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_to_planes_fold(const Geom& g, const double* src, bool from_l64, int Kx, T* img,
                                 hipStream_t s) {
    const int nb = pw_blocks((long)Kx * g.ny, pointwise_block_cap());
    if (from_l64) {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_to_planes_fold<NN, true, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, src, img, Kx));
    } else {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_to_planes_fold<NN, false, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, src, img, Kx));
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_from_planes_fold(const Geom& g, const OpConst<double>& k, const T* img, int Kx,
                                   double* dst, const double* r, const DevScratch* d,
                                   hipStream_t s) {
    const int nb = pw_blocks((long)Kx * g.ny, pointwise_block_cap());
    if (d) {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_planes_fold<NN, true, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, k, img, Kx, dst, r,
                                              d->sc, d->counters + kCntDot * kCntStride, d->partials));
    } else {
        DG_DISPATCH_N(g.n, hipLaunchKernelGGL((k_from_planes_fold<NN, false, T>), dim3(nb),
                                              dim3(kPwThreads), 0, s, g, k, img, Kx, dst,
                                              nullptr, nullptr, nullptr, nullptr));
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_fd_mix_x_fold(bool inverse, int n, int Nx, int Ny, int Ky, int K,
                                const int* cols, const T* M, const T* in, T* out,
                                hipStream_t s) {
    const int nb = pw_blocks((long)Ky * n, pointwise_block_cap());
    if (inverse) {
        DG_DISPATCH_N(n, hipLaunchKernelGGL((k_fd_mix_x_fold<NN, T, true>), dim3(nb, K),
                                            dim3(kPwThreads), 0, s, Nx, Ny, Ky, cols, M, in,
                                            out));
    } else {
        DG_DISPATCH_N(n, hipLaunchKernelGGL((k_fd_mix_x_fold<NN, T, false>), dim3(nb, K),
                                            dim3(kPwThreads), 0, s, Nx, Ny, Ky, cols, M, in,
                                            out));
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_dense_divide(int mx, int my, const T* lx, const T* ly, T* c, hipStream_t s) {
    const int nb = pw_blocks((long)mx * my, pointwise_block_cap());
    hipLaunchKernelGGL((k_dense_divide<T>), dim3(nb), dim3(kPwThreads), 0, s, mx, my, lx, ly, c);
    return hipGetLastError();
}

template <class T>
hipError_t launch_fd_mix_y(int n, int Nx, int Ny, int K, const int* cols, const T* Mf,
                           const T* Mi, const T* lx, const T* ly, int zx, int zy, T* u,
                           hipStream_t s) {
    const int nb = pw_blocks((long)Nx * n, pointwise_block_cap());
    DG_DISPATCH_N(n, hipLaunchKernelGGL((k_fd_mix_y<NN, T>), dim3(nb, K), dim3(kPwThreads), 0, s,
                                        Nx, cols, Mf, Mi, lx, ly, Ny, zx, zy, u));
    return hipGetLastError();
}

template <class T>
hipError_t launch_fft_mix_x_fwd(int n, int Nx, int Ny, const int* cols, const T* Mf,
                                const void* X, T* u1, hipStream_t s) {
    using C = typename CplxOf<T>::type;
    const T cn = T(1.0 / std::sqrt((double)Nx)), cp = T(std::sqrt(2.0 / Nx));
    DG_DISPATCH_N(n, {
        using TL = SpecTile<NN, T>;
        const dim3 grid((spec_pairs(Nx / 2) + TL::TP - 1) / TL::TP, ((Ny + 63) / 64) * NN);
        hipLaunchKernelGGL((k_fft_mix_x_fwd<NN, T>), grid, dim3(TL::THREADS), 0, s, Nx, Ny,
                           cols, Mf, cn, cp, (const C*)X, u1);
    });
    return hipGetLastError();
}

template <class T>
hipError_t launch_fft_mix_x_inv(int n, int Nx, int Ny, const int* cols, const T* Mi,
                                const T* u1, void* X, hipStream_t s) {
    using C = typename CplxOf<T>::type;
    const T cn = T(1.0 / std::sqrt((double)Nx)), cp = T(std::sqrt(2.0 / Nx));
    DG_DISPATCH_N(n, {
        using TL = SpecTile<NN, T>;
        const dim3 grid((spec_pairs(Nx / 2) + TL::TP - 1) / TL::TP, ((Ny + 63) / 64) * NN);
        hipLaunchKernelGGL((k_fft_mix_x_inv<NN, T>), grid, dim3(TL::THREADS), 0, s, Nx, Ny,
                           cols, Mi, cn, cp, u1, (C*)X);
    });
    return hipGetLastError();
}

template <class T>
hipError_t launch_fft_mix_y(int n, int Nx, int Ny, const int* cols, const T* Mf,
                            const T* Mi, const T* lx, const T* ly, int zx, int zy, void* Y,
                            hipStream_t s) {
    using C = typename CplxOf<T>::type;
    const T cn = T(1.0 / std::sqrt((double)Ny)), cp = T(std::sqrt(2.0 / Ny));
    DG_DISPATCH_N(n, {
        using TL = SpecTile<NN, T>;
        const dim3 grid((spec_pairs(Ny / 2) + TL::TP - 1) / TL::TP, ((long)Nx * NN + 63) / 64);
        hipLaunchKernelGGL((k_fft_mix_y<NN, T>), grid, dim3(TL::THREADS), 0, s, Nx, Ny, cols,
                           Mf, Mi, lx, ly, zx, zy, cn, cp, (C*)Y);
    });
    return hipGetLastError();
}

#define DG_FD_INSTANTIATE(T)                                                                  \
    template hipError_t launch_to_image<T>(const Geom&, const OpConst<double>&, const double*, \
                                           bool, bool, T*, hipStream_t);                       \
    template hipError_t launch_from_image<T>(const Geom&, const OpConst<double>&, const T*,    \
                                             bool, double*, hipStream_t);                      \
    template hipError_t launch_from_image_dot<T>(const Geom&, const OpConst<double>&,          \
                                                 const T*, bool, double*, const double*,       \
                                                 const DevScratch&, hipStream_t);              \
    template hipError_t launch_dense_divide<T>(int, int, const T*, const T*, T*, hipStream_t); \
    template hipError_t launch_to_planes_fold<T>(const Geom&, const double*, bool, int, T*,   \
                                                 hipStream_t);                                 \
    template hipError_t launch_from_planes_fold<T>(const Geom&, const OpConst<double>&,       \
                                                   const T*, int, double*, const double*,     \
                                                   const DevScratch*, hipStream_t);           \
    template hipError_t launch_fd_mix_x_fold<T>(bool, int, int, int, int, int, const int*,    \
                                                const T*, const T*, T*, hipStream_t);         \
    template hipError_t launch_fd_mix_y<T>(int, int, int, int, const int*, const T*, const T*, \
                                           const T*, const T*, int, int, T*, hipStream_t);     \
    template hipError_t launch_fft_mix_x_fwd<T>(int, int, int, const int*, const T*,      \
                                                const void*, T*, hipStream_t);                 \
    template hipError_t launch_fft_mix_x_inv<T>(int, int, int, const int*, const T*,      \
                                                const T*, void*, hipStream_t);                 \
    template hipError_t launch_fft_mix_y<T>(int, int, int, const int*, const T*, const T*, \
                                            const T*, const T*, int, int, void*, hipStream_t);
DG_FD_INSTANTIATE(double)
DG_FD_INSTANTIATE(float)
#undef DG_FD_INSTANTIATE

}  // namespace dgk

// Host construction of the separable eigenbases behind the fast-
// diagonalisation preconditioner: the exact inverse of -Lap_h on W-mean-free
// fields (a preconditioner for the CG of Sec. 6, which itself is plain CG).
//
// Along one periodic axis with N cells of size h the LDG second derivative
// (Sec. 6, D_backward D_forward plus the jump penalty; the blocks of
// ldg_axis) is block circulant,
//     (L u)_m = h^-2 [L0 u_m + eR (lR . u_{m+1}) + eL (lL . u_{m-1})],
// so Bloch waves u_m = v e^{i theta m}, theta = 2 pi k / N, reduce it to the
// n x n symbols S(theta) = h^-2 [L0 + e^{i theta} eR lR^T + e^{-i theta} eL lL^T].
// L is self-adjoint in the Gauss inner product (weights h w_i / 2), hence
// H(theta) = Wc^{1/2} S(theta) Wc^{-1/2} (Wc = diag w) is Hermitian; its
// eigenvectors u give v = Wc^{-1/2} u with v^H Wc v = 1.  Pairs theta, -theta
// (conjugate symbols) combine into real cosine / sine eigenvectors, so the
// whole axis gets a real basis V (columns W-orthonormal: V^T W V = I) with
// L V = V diag(lambda).  The constant vector is the single zero mode.
#include <cmath>
#include <complex>
#include <vector>

#include "fd_basis.h"

namespace dgk {

namespace {

using cplx = std::complex<double>;

// H = U diag(lam) U^H for a Hermitian n x n matrix (row-major, destroyed)
// by cyclic Jacobi rotations.  Each rotation first makes H_pq real with a
// diagonal phase, then annihilates it with a real plane rotation.  A real
// symmetric H keeps real U.
void herm_eig(int n, cplx* H, double* lam, cplx* U) {
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) U[a * n + b] = (a == b) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int a = 0; a < n; ++a) {
            diag += std::norm(H[a * n + a]);
            for (int b = a + 1; b < n; ++b) off += std::norm(H[a * n + b]);
        }
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double g = std::abs(H[p * n + q]);
                if (g == 0.0) continue;
                const cplx ph = H[p * n + q] / g;
                // H <- D^H H D, U <- U D with D = diag(1, .., conj(ph) at q)
                for (int k = 0; k < n; ++k) {
                    H[k * n + q] *= std::conj(ph);
                    U[k * n + q] *= std::conj(ph);
                }
                for (int l = 0; l < n; ++l) H[q * n + l] *= ph;
                const double app = H[p * n + p].real(), aqq = H[q * n + q].real();
                const double th = (aqq - app) / (2.0 * g);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                // H <- G^T H G, U <- U G, G = [[c, s], [-s, c]] on (p, q)
                for (int k = 0; k < n; ++k) {
                    const cplx hp = H[k * n + p], hq = H[k * n + q];
                    H[k * n + p] = c * hp - s * hq;
                    H[k * n + q] = s * hp + c * hq;
                    const cplx up = U[k * n + p], uq = U[k * n + q];
                    U[k * n + p] = c * up - s * uq;
                    U[k * n + q] = s * up + c * uq;
                }
                for (int l = 0; l < n; ++l) {
                    const cplx hp = H[p * n + l], hq = H[q * n + l];
                    H[p * n + l] = c * hp - s * hq;
                    H[q * n + l] = s * hp + c * hq;
                }
            }
    }
    for (int a = 0; a < n; ++a) lam[a] = H[a * n + a].real();
}

// Eigenpairs of the Bloch symbol of wave number k: lam[e] and v[:, e]
// (v[i * n + e]) with v^H Wc v = 1.  Accumulates the largest relative defect
// (Hermitian symmetry, eigen-residual) into *err.
void bloch_eig(const HostTables& t, int N, double h, int k, double* lam, cplx* v, double* err) {
    const int n = t.n;
    const double ih2 = 1.0 / (h * h);
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<cplx> S(n * n), H(n * n), U(n * n);
    AxisLdg ax;
    ldg_axis(t, h, true, &ax);
    const double th = two_pi * k / N;
    // e^{i theta}, exact at theta = 0 and pi so those symbols stay real
    const cplx ep = (k == 0) ? cplx(1.0, 0.0)
                  : (2 * k == N) ? cplx(-1.0, 0.0) : cplx(std::cos(th), std::sin(th));
    for (int r = 0; r < n; ++r)
        for (int b = 0; b < n; ++b)
            S[r * n + b] = ih2 * (ax.L0[r * n + b] + ep * (ax.eR[r] * t.lR[b]) +
                                  std::conj(ep) * (t.eL[r] * ax.lL[b]));
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            H[a * n + b] = std::sqrt(t.w[a]) * S[a * n + b] / std::sqrt(t.w[b]);
    // symmetrise the rounding of the Hermitian form; record its defect
    double scale = 0.0;
    for (int a = 0; a < n * n; ++a) scale = std::fmax(scale, std::abs(H[a]));
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            const cplx m = 0.5 * (H[a * n + b] + std::conj(H[b * n + a]));
            *err = std::fmax(*err, std::abs(H[a * n + b] - std::conj(H[b * n + a])) / scale);
            H[a * n + b] = m;
            H[b * n + a] = std::conj(m);
        }
    herm_eig(n, H.data(), lam, U.data());
    // v = Wc^{-1/2} u; check S v = lambda v
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) v[a * n + b] = U[a * n + b] / std::sqrt(t.w[a]);
    for (int e = 0; e < n; ++e) {
        double r = 0.0, vn = 0.0;
        for (int a = 0; a < n; ++a) {
            cplx sv = 0.0;
            for (int b = 0; b < n; ++b) sv += S[a * n + b] * v[b * n + e];
            r = std::fmax(r, std::abs(sv - lam[e] * v[a * n + e]));
            vn = std::fmax(vn, std::abs(v[a * n + e]));
        }
        *err = std::fmax(*err, r / (scale * vn));
    }
}

}  // namespace

bool fd_axis_factors(const HostTables& t, int N, double h, FdFactors* out, double* max_err,
                     bool shifted) {
    const int n = t.n;
    const double two_pi = 6.283185307179586476925286766559;
    const int K = N / 2 + 1;                 // wave numbers 0 .. floor(N/2)
    const int s = 2 * n;
    out->N = N;
    out->n = n;
    out->K = K;
    out->phi.assign((size_t)N * N, 0.0);
    out->ccos.assign(K, -1);
    out->csin.assign(K, -1);
    out->mf.assign((size_t)K * s * s, 0.0);
    out->mi.assign((size_t)K * s * s, 0.0);
    out->lam.assign((size_t)N * n, 0.0);
    out->zero = -1;
    // real orthonormal Fourier basis over the cells, the even columns first.
    // Unshifted (cos / sin of 2 pi k c / N, for the FFT transforms): columns
    // 0 .. K-1 the constant, cos k and for even N the alternating (-1)^c,
    // then the sines at K + k - 1; rows c and N - c agree on the first block.
    // Shifted (of 2 pi k (c + 1/2) / N, for the matrix-product transforms):
    // cells c and N - 1 - c agree on the cosines and differ in sign on the
    // sines and, for even N, the alternating column, so the first Ke =
    // ceil(N/2) columns are the constant and cos k < N/2, the others the sines
    // at Ke + k - 1 and the alternating one last: two halves of N/2 columns
    // for even N, which the transforms use to fold each axis.
    const double c0 = 1.0 / std::sqrt((double)N), c1 = std::sqrt(2.0 / N);
    const int Ke = shifted ? (N + 1) / 2 : K;
    for (int k = 0; k < K; ++k) {
        const bool real = (k == 0) || (2 * k == N);
        const int cc = (shifted && 2 * k == N) ? N - 1 : k, cs = Ke + k - 1;
        out->ccos[k] = cc;
        if (!real) out->csin[k] = cs;
        for (int cx = 0; cx < N; ++cx) {
            if (real) {
                out->phi[(size_t)cc * N + cx] = (k == 0 || cx % 2 == 0) ? c0 : -c0;
            } else {
                // angle reduced exactly: 2 pi k c / N, or pi k (2c + 1) / N
                const long m = shifted ? ((long)k * (2 * cx + 1)) % (2L * N)
                                       : ((long)k * cx) % N;
                const double ang = shifted ? 0.5 * two_pi * (double)m / N
                                           : two_pi * (double)m / N;
                out->phi[(size_t)cc * N + cx] = c1 * std::cos(ang);
                out->phi[(size_t)cs * N + cx] = c1 * std::sin(ang);
            }
        }
    }
    // mixing blocks: slot p = (i, cos) -> i, (i, sin) -> n + i on the input
    // side, q = (a, re) -> a, (a, im) -> n + a on the mode side.  With
    // sc = 1 / sqrt(h / 2) the basis is V = (Phi (x) I) B with
    //   B[(cos,i),(re,a)] = sc Re v,  B[(sin,i),(re,a)] = -sc Im v,
    //   B[(cos,i),(im,a)] = sc Im v,  B[(sin,i),(im,a)] =  sc Re v
    // (v = v_a[i]); forward mf[q][p] = B[p][q] (h/2) w_i, inverse mi[p][q] = B[p][q].
    const double sc = 1.0 / std::sqrt(0.5 * h);
    double err = 0.0, zero_abs = 0.0;
    std::vector<cplx> v(n * n);
    std::vector<double> lam(n);
    for (int k = 0; k < K; ++k) {
        bloch_eig(t, N, h, k, lam.data(), v.data(), &err);
        const bool real = out->csin[k] < 0;
        double* mf = &out->mf[(size_t)k * s * s];
        double* mi = &out->mi[(size_t)k * s * s];
        for (int a = 0; a < n; ++a) {
            for (int i = 0; i < n; ++i) {
                const cplx va = v[i * n + a];
                const double wi = 0.5 * h * t.w[i];
                double Bv[2][2];   // [cos/sin][re/im]
                Bv[0][0] = sc * va.real();
                Bv[1][0] = -sc * va.imag();
                Bv[0][1] = sc * va.imag();
                Bv[1][1] = sc * va.real();
                const int nc = real ? 1 : 2;
                for (int cs = 0; cs < nc; ++cs)
                    for (int ri = 0; ri < nc; ++ri) {
                        const int p = cs * n + i, q = ri * n + a;
                        mf[q * s + p] = Bv[cs][ri] * wi;
                        mi[p * s + q] = Bv[cs][ri];
                    }
            }
            if (shifted && !real && a == n - 1) {
                // the shifted basis column pair of wave number k is the
                // unshifted pair rotated by phi = pi k / N: coefficients
                // (a, b) = R (a', b'), R = [[cos, sin], [-sin, cos]] on the
                // (cos, sin) slots of every node, so mf' = mf R, mi' = R^T mi
                const double ph = 0.5 * two_pi * (double)k / N;
                const double cph = std::cos(ph), sph = std::sin(ph);
                for (int q = 0; q < s; ++q)
                    for (int i2 = 0; i2 < n; ++i2) {
                        double& f0 = mf[q * s + i2];
                        double& f1 = mf[q * s + n + i2];
                        const double g0 = f0 * cph - f1 * sph, g1 = f0 * sph + f1 * cph;
                        f0 = g0;
                        f1 = g1;
                        double& m0 = mi[i2 * s + q];
                        double& m1 = mi[(n + i2) * s + q];
                        const double h0 = cph * m0 - sph * m1, h1 = sph * m0 + cph * m1;
                        m0 = h0;
                        m1 = h1;
                    }
            }
            out->lam[(size_t)a * N + out->ccos[k]] = lam[a];
            if (!real) out->lam[(size_t)a * N + out->csin[k]] = lam[a];
            if (k == 0 && (out->zero < 0 || std::fabs(lam[a]) < zero_abs)) {
                out->zero = a * N;
                zero_abs = std::fabs(lam[a]);
            }
        }
    }
    *max_err = err;
    return out->zero >= 0;
}

bool fd_axis_basis(const HostTables& t, int N, double h, FdAxis* out, double* max_err,
                   bool shifted) {
    FdFactors f;
    if (!fd_axis_factors(t, N, h, &f, max_err, shifted)) return false;
    const int n = t.n, s = 2 * n;
    const long NN = (long)N * n;
    out->NN = (int)NN;
    out->V.assign((size_t)(NN * NN), 0.0);
    out->lam = f.lam;
    out->zero = f.zero;
    // V[(cx, i), slot (a, c')] = sum over the block's basis columns c of
    // Phi[cx, c] B[(c, i), (a, c')]
    for (int k = 0; k < f.K; ++k) {
        const int cols[2] = {f.ccos[k], f.csin[k]};
        const int nc = cols[1] < 0 ? 1 : 2;
        const double* mi = &f.mi[(size_t)k * s * s];
        for (int ri = 0; ri < nc; ++ri)
            for (int a = 0; a < n; ++a) {
                const long col = (long)a * N + cols[ri];
                for (int cx = 0; cx < N; ++cx)
                    for (int i = 0; i < n; ++i) {
                        double acc = 0.0;
                        for (int cs = 0; cs < nc; ++cs)
                            acc += f.phi[(size_t)cols[cs] * N + cx] *
                                   mi[(cs * n + i) * s + ri * n + a];
                        out->V[(size_t)(col * NN + (long)cx * n + i)] = acc;
                    }
            }
    }
    return true;
}

// Row c of the axis operator in the h = 1 blocks: self block, the right
// coupling vector (times lR . u_{c+1}) and the left functional (eL times it
// applied to u_{c-1}); null where the coupling is absent (the Dirichlet ends).
struct AxisRow {
    const double *L0, *eR, *lL;
};

static AxisRow axis_row(const AxisLdg& ax, int N, bool periodic, int c) {
    if (periodic) return {ax.L0, ax.eR, ax.lL};
    AxisRow r{c == 0 ? ax.L0B : ax.L0, c == 0 ? ax.eRB : ax.eR, c == 1 ? ax.lLB : ax.lL};
    if (c == N - 1) r.eR = nullptr;
    if (c == 0) r.lL = nullptr;
    return r;
}

void fd_axis_apply(const HostTables& t, int N, double h, bool periodic, const double* u,
                   double* out) {
    const int n = t.n;
    AxisLdg ax;
    ldg_axis(t, h, periodic, &ax);
    const double ih2 = 1.0 / (h * h);
    for (int c = 0; c < N; ++c) {
        const AxisRow r = axis_row(ax, N, periodic, c);
        const double* uc = u + (size_t)c * n;
        double fr = 0.0, fl = 0.0;
        if (r.eR) {
            const double* up = u + (size_t)((c + 1) % N) * n;
            for (int m = 0; m < n; ++m) fr += t.lR[m] * up[m];
        }
        if (r.lL) {
            const double* um = u + (size_t)((c + N - 1) % N) * n;
            for (int m = 0; m < n; ++m) fl += r.lL[m] * um[m];
        }
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int m = 0; m < n; ++m) acc += r.L0[i * n + m] * uc[m];
            if (r.eR) acc += r.eR[i] * fr;
            if (r.lL) acc += t.eL[i] * fl;
            out[(size_t)c * n + i] = ih2 * acc;
        }
    }
}

void fd_axis_operator(const HostTables& t, int N, double h, bool periodic,
                      std::vector<double>* L) {
    const int n = t.n;
    const size_t m = (size_t)N * n;
    AxisLdg ax;
    ldg_axis(t, h, periodic, &ax);
    const double ih2 = 1.0 / (h * h);
    L->assign(m * m, 0.0);
    auto at = [&](size_t row, size_t col) -> double& { return (*L)[col * m + row]; };
    for (int c = 0; c < N; ++c) {
        const AxisRow r = axis_row(ax, N, periodic, c);
        const size_t rc = (size_t)c * n;
        for (int i = 0; i < n; ++i) {
            for (int b = 0; b < n; ++b) at(rc + i, rc + b) += ih2 * r.L0[i * n + b];
            if (r.eR) {
                const size_t cp = (size_t)((c + 1) % N) * n;
                for (int b = 0; b < n; ++b) at(rc + i, cp + b) += ih2 * r.eR[i] * t.lR[b];
            }
            if (r.lL) {
                const size_t cm = (size_t)((c + N - 1) % N) * n;
                for (int b = 0; b < n; ++b) at(rc + i, cm + b) += ih2 * t.eL[i] * r.lL[b];
            }
        }
    }
}

}  // namespace dgk

// Host construction of the separable eigenbases behind the fast-
// diagonalisation preconditioner: the exact inverse of -Lap_h on W-mean-free
// fields (a preconditioner for the CG of Sec. 6, which itself is plain CG).
//
// Along one periodic axis with N cells of size h the LDG second derivative
// (Sec. 6, D_backward D_forward) is block circulant,
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

}  // namespace

bool fd_axis_basis(const HostTables& t, int N, double h, FdAxis* out, double* max_err) {
    const int n = t.n;
    const long NN = (long)N * n;
    out->NN = (int)NN;
    out->V.assign((size_t)(NN * NN), 0.0);
    out->lam.assign((size_t)NN, 0.0);
    out->zero = -1;
    const double ih2 = 1.0 / (h * h);
    const double norm = 1.0 / std::sqrt(N * 0.5 * h);
    const double two_pi = 6.283185307179586476925286766559;
    double err = 0.0;
    std::vector<cplx> S(n * n), H(n * n), U(n * n), v(n * n);
    std::vector<double> lam(n);
    long col = 0;
    double zero_abs = 0.0;
    for (int k = 0; 2 * k <= N; ++k) {
        const double th = two_pi * k / N;
        // e^{i theta}, exact at theta = 0 and pi so those symbols stay real
        const cplx ep = (k == 0) ? cplx(1.0, 0.0)
                      : (2 * k == N) ? cplx(-1.0, 0.0) : cplx(std::cos(th), std::sin(th));
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                S[a * n + b] = ih2 * (t.L0[a * n + b] + ep * (t.eR[a] * t.lR[b]) +
                                      std::conj(ep) * (t.eL[a] * t.lL[b]));
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b)
                H[a * n + b] = std::sqrt(t.w[a]) * S[a * n + b] / std::sqrt(t.w[b]);
        // symmetrise the rounding of the Hermitian form; record its defect
        double scale = 0.0;
        for (int a = 0; a < n * n; ++a) scale = std::fmax(scale, std::abs(H[a]));
        for (int a = 0; a < n; ++a)
            for (int b = a; b < n; ++b) {
                const cplx m = 0.5 * (H[a * n + b] + std::conj(H[b * n + a]));
                err = std::fmax(err, std::abs(H[a * n + b] - std::conj(H[b * n + a])) / scale);
                H[a * n + b] = m;
                H[b * n + a] = std::conj(m);
            }
        herm_eig(n, H.data(), lam.data(), U.data());
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
            err = std::fmax(err, r / (scale * vn));
        }
        const bool real_pair = (k == 0) || (2 * k == N);
        for (int e = 0; e < n; ++e) {
            if (real_pair) {
                for (int cx = 0; cx < N; ++cx) {
                    const double sgn = (k == 0 || (cx % 2 == 0)) ? 1.0 : -1.0;
                    for (int i = 0; i < n; ++i)
                        out->V[(size_t)(col * NN + (long)cx * n + i)] =
                            norm * sgn * v[i * n + e].real();
                }
                out->lam[col] = lam[e];
                if (k == 0 && (out->zero < 0 || std::fabs(lam[e]) < zero_abs)) {
                    out->zero = (int)col;
                    zero_abs = std::fabs(lam[e]);
                }
                ++col;
            } else {
                const double r2 = std::sqrt(2.0) * norm;
                for (int cx = 0; cx < N; ++cx) {
                    // angle reduced exactly: theta * cx = 2 pi (k cx mod N) / N
                    const long m = ((long)k * cx) % N;
                    const double ang = two_pi * (double)m / N;
                    const cplx e_ = cplx(std::cos(ang), std::sin(ang));
                    for (int i = 0; i < n; ++i) {
                        const cplx z = v[i * n + e] * e_;
                        out->V[(size_t)(col * NN + (long)cx * n + i)] = r2 * z.real();
                        out->V[(size_t)((col + 1) * NN + (long)cx * n + i)] = r2 * z.imag();
                    }
                }
                out->lam[col] = lam[e];
                out->lam[col + 1] = lam[e];
                col += 2;
            }
        }
    }
    *max_err = err;
    return col == NN && out->zero >= 0;
}

}  // namespace dgk

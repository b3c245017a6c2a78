// Host construction of the per-grid operator tables (Sec. 4.1-4.2, Sec. 6).
//
// Everything is built from the Legendre three-term recursion (Sec. 4.1,
// eq. recursion): Gauss-Legendre abscissas by Newton's method on p_n, the
// weights 2 / ((1 - x^2) p_n'(x)^2), the transforms B, F, the derivative
// block D and the end-value products; the X-space blocks are then the
// matrix products of Sec. 4.2 with h = 1.
#include <cmath>
#include <cstring>

#include "dg_internal.h"

namespace dgk {
namespace {

// p[0..m] = p_0(x)..p_m(x) by the three-term recursion.
void legendre_all(int m, double x, double* p) {
    p[0] = 1.0;
    if (m >= 1) p[1] = x;
    for (int k = 1; k < m; ++k) p[k + 1] = ((2 * k + 1) * x * p[k] - k * p[k - 1]) / (k + 1);
}

void gauss_legendre(int n, double* xi, double* w) {
    double p[kMaxN + 1];
    for (int i = 0; i < n; ++i) {
        // i-th largest root of p_n by Newton's method;
        // p_n' = n (p_{n-1} - x p_n) / (1 - x^2)
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            legendre_all(n, x, p);
            double dp = n * (p[n - 1] - x * p[n]) / (1.0 - x * x);
            double dx = p[n] / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        if (n % 2 == 1 && i == n / 2) x = 0.0;  // exact centre node
        legendre_all(n, x, p);
        double dp = n * (p[n - 1] - x * p[n]) / (1.0 - x * x);
        xi[n - 1 - i] = x;  // store ascending
        w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

// c = a * b for n x n row-major matrices
void matmul(int n, const double* a, const double* b, double* c) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += a[i * n + k] * b[k * n + j];
            c[i * n + j] = s;
        }
}

}  // namespace

bool build_tables(int n, HostTables* t) {
    if (n < 1 || n > kMaxN || !t) return false;
    std::memset(t, 0, sizeof(*t));
    t->n = n;
    gauss_legendre(n, t->xi, t->w);

    const int nn = n * n;
    double B[kMaxN * kMaxN], F[kMaxN * kMaxN], Dm[kMaxN * kMaxN];
    for (int j = 0; j < n; ++j) {
        double p[kMaxN + 1];
        legendre_all(n, t->xi[j], p);
        for (int k = 0; k < n; ++k) {
            B[j * n + k] = p[k];                                 // B_jk = p_k(xi_j)
            F[k * n + j] = 0.5 * (2 * k + 1) * t->w[j] * p[k];  // F^kj
        }
    }
    // D_ij = int p_i p_j' = 1 - (-1)^(i+j) for i <= j-1, else 0
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            Dm[i * n + j] = (i <= j - 1) ? 1.0 - (((i + j) % 2) ? -1.0 : 1.0) : 0.0;
    double pr[kMaxN], pl[kMaxN];  // p_k(1), p_k(-1)
    for (int k = 0; k < n; ++k) { pr[k] = 1.0; pl[k] = (k % 2) ? -1.0 : 1.0; }

    // BT = B * diag(2k+1)
    double BT[kMaxN * kMaxN];
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) BT[j * n + k] = B[j * n + k] * (2 * k + 1);

    // traces in X-space: u(-1) = (F^T l).u, u(+1) = (F^T r).u
    double trL[kMaxN], trR[kMaxN];
    for (int j = 0; j < n; ++j) {
        double sl = 0.0, sr = 0.0;
        for (int k = 0; k < n; ++k) { sl += F[k * n + j] * pl[k]; sr += F[k * n + j] * pr[k]; }
        trL[j] = sl;
        trR[j] = sr;
    }
    // B T r and B T l
    double BTr[kMaxN], BTl[kMaxN];
    for (int j = 0; j < n; ++j) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < n; ++k) { a += BT[j * n + k] * pr[k]; b += BT[j * n + k] * pl[k]; }
        BTr[j] = a;
        BTl[j] = b;
    }

    // ---- centred derivative: C0 = 1/2 B T (D - D^T) F; the right
    // neighbour enters through its left trace, the left one through its
    // right trace (Sec. 4.2 eq. discrete_der with 1^+ RL and 1^- LR).
    double S[kMaxN * kMaxN], tmp[kMaxN * kMaxN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) S[i * n + j] = 0.5 * (Dm[i * n + j] - Dm[j * n + i]);
    matmul(n, BT, S, tmp);
    matmul(n, tmp, F, t->C0);
    for (int j = 0; j < n; ++j) {
        t->cR[j] = 0.5 * BTr[j];
        t->sR[j] = trL[j];
        t->cL[j] = -0.5 * BTl[j];
        t->sL[j] = trR[j];
    }

    // ---- LDG: forward Df u = F0 u_m + fp (trL . u_{m+1}),
    //           backward Db v = G0 v_m - gm (trR . v_{m-1}),
    // F0 = B T (D - R) F, fp = B T r, G0 = B T (D + L) F, gm = B T l.
    double F0[kMaxN * kMaxN], G0[kMaxN * kMaxN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) S[i * n + j] = Dm[i * n + j] - pr[i] * pr[j];
    matmul(n, BT, S, tmp);
    matmul(n, tmp, F, F0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) S[i * n + j] = Dm[i * n + j] + pl[i] * pl[j];
    matmul(n, BT, S, tmp);
    matmul(n, tmp, F, G0);
    // (Db Df u)_m = G0 F0 u_m + G0 fp (trL.u_{m+1})
    //               - gm [ (F0^T trR).u_{m-1} + (trR.fp)(trL.u_m) ]
    double G0F0[kMaxN * kMaxN];
    matmul(n, G0, F0, G0F0);
    double trRfp = 0.0;
    for (int j = 0; j < n; ++j) trRfp += trR[j] * BTr[j];
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            t->L0[i * n + j] = G0F0[i * n + j] - trRfp * BTl[i] * trL[j];
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += G0[i * n + k] * BTr[k];
        t->eR[i] = s;
        t->lR[i] = trL[i];
        t->eL[i] = -BTl[i];
        double q = 0.0;
        for (int k = 0; k < n; ++k) q += F0[k * n + i] * trR[k];
        t->lL[i] = q;
        // end values and their W^-1 images: W^-1 tR^T = (B T r) / h
        t->tR[i] = trR[i];
        t->tL[i] = trL[i];
        t->pR[i] = BTr[i];
        t->pL[i] = BTl[i];
    }
    // first cell of a Dirichlet axis: Df with u-hat = 0 on the left face,
    // F0' = F0 + (B T l) trL^T; Db with q-hat = its own left trace there and
    // no left neighbour, G0' = G0 - (B T l) trL^T.  (Db Df u)_0 = G0' F0' u_0
    // + G0' fp (trL . u_1).
    double F0b[kMaxN * kMaxN], G0b[kMaxN * kMaxN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            F0b[i * n + j] = F0[i * n + j] + BTl[i] * trL[j];
            G0b[i * n + j] = G0[i * n + j] - BTl[i] * trL[j];
        }
    matmul(n, G0b, F0b, t->L0B);
    for (int i = 0; i < n; ++i) {
        double s = 0.0, q = 0.0;
        for (int k = 0; k < n; ++k) {
            s += G0b[i * n + k] * BTr[k];
            q += F0b[k * n + i] * trR[k];
        }
        t->eRB[i] = s;
        t->lLB[i] = q;   // the second cell's Db reads trR . q_0, q_0 = F0' u_0 + ..
    }
    (void)nn;
    return true;
}

double ldg_penalty(int n, bool periodic) { return (n == 1 && periodic) ? 0.0 : 1.0; }

void ldg_axis(const HostTables& t, double h, bool periodic, AxisLdg* out) {
    const int n = t.n;
    const double c = ldg_penalty(n, periodic) * h;
    // penalty on face m+1/2: -C11 W^-1 (-tR)^T [u], [u] = tL.u_{m+1} - tR.u_m;
    // on face m-1/2: -C11 W^-1 tL^T [u], [u] = tL.u_m - tR.u_{m-1}
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            const double pen = c * (t.pR[i] * t.tR[j] + t.pL[i] * t.tL[j]);
            out->L0[i * n + j] = t.L0[i * n + j] - pen;
            out->L0B[i * n + j] = t.L0B[i * n + j] - pen;
        }
        out->eR[i] = t.eR[i] + c * t.pR[i];
        out->eRB[i] = t.eRB[i] + c * t.pR[i];
        out->lL[i] = t.lL[i] - c * t.tR[i];
        out->lLB[i] = t.lLB[i] - c * t.tR[i];
    }
}

}  // namespace dgk

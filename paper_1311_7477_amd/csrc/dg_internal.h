// Internal declarations shared by the host tables, the C ABI layer and the
// HIP kernels of libdgark.  Not part of the public interface.
#pragma once

#include <cstddef>
#include <cstdint>

namespace dgk {

constexpr int kMaxN = 5;

// 1D operators on one cell and its two neighbours along one axis, unit cell
// size (h = 1), in X-space (nodal values at Gauss-Legendre points).
//   centred derivative (Sec. 4.2 eqs. discrete_der, matrix_xspace):
//     (D u)_m = C0 u_m + cR (sR . u_{m+1}) + cL (sL . u_{m-1})
//   LDG second derivative D_backward D_forward (Sec. 6):
//     (L u)_m = L0 u_m + eR (lR . u_{m+1}) + eL (lL . u_{m-1})
// The neighbour couplings are rank one: one scalar per node row.  tR / tL
// are the end-value functionals u(+1) = tR . u, u(-1) = tL . u, and pR / pL
// = h W^-1 tR, h W^-1 tL (W = (h/2) diag(w)); they build the LDG jump
// penalty (ldg_axis).
struct HostTables {
    int n;
    double xi[kMaxN], w[kMaxN];
    double C0[kMaxN * kMaxN], cR[kMaxN], sR[kMaxN], cL[kMaxN], sL[kMaxN];
    double L0[kMaxN * kMaxN], eR[kMaxN], lR[kMaxN], eL[kMaxN], lL[kMaxN];
    double tR[kMaxN], tL[kMaxN], pR[kMaxN], pL[kMaxN];
    // first cell of a homogeneous Dirichlet axis (u-hat = 0 and q-hat = the
    // inside trace on its boundary face): self block and right coupling, and
    // the functional lLB through which the second cell sees it
    double L0B[kMaxN * kMaxN], eRB[kMaxN], lLB[kMaxN];
};

// Builds the tables for n in [1, 5]; returns false on bad n.
bool build_tables(int n, HostTables* t);

// The LDG second derivative of one periodic axis with cell size h, in the
// same h = 1 form (the operator is these blocks times h^-2):
//     L = D_backward D_forward - C11 W^-1 J^T J,
// the jump penalty C11 sum_faces [u][v] added to the alternating-flux
// operator.  Its couplings stay rank one with the same lR and eL:
//     L0' = L0 - C11 h (pR tR^T + pL tL^T),  eR' = eR + C11 h pR,
//     lL' = lL - C11 h tR.
// C11 = ldg_penalty(n, periodic): 1 in the units of the domain, 0 for n = 1
// on a periodic axis (the plain finite-difference Laplacian there).
// On a homogeneous Dirichlet axis the last cell drops its right coupling
// (and keeps L0', its boundary face adds the same self penalty an inside
// face would), the first cell drops its left coupling and uses
//     L0B' = L0B - C11 h (pR tR^T + pL tL^T),  eRB' = eRB + C11 h pR,
// and the second cell couples to the first through lLB' = lLB - C11 h tR.
struct AxisLdg {
    double L0[kMaxN * kMaxN], eR[kMaxN], lL[kMaxN];
    double L0B[kMaxN * kMaxN], eRB[kMaxN], lLB[kMaxN];
};
double ldg_penalty(int n, bool periodic);
void ldg_axis(const HostTables& t, double h, bool periodic, AxisLdg* out);

// Operator constants passed to kernels by value (kernel-argument segment).
// The LDG blocks depend on the cell size through the jump penalty, so x and
// y have their own L0 / eR / lL (lR and eL are shared).
template <class T>
struct OpConst {
    T C0[kMaxN * kMaxN], cR[kMaxN], sR[kMaxN], cL[kMaxN], sL[kMaxN];
    T L0x[kMaxN * kMaxN], L0y[kMaxN * kMaxN];
    T eRx[kMaxN], eRy[kMaxN], lLx[kMaxN], lLy[kMaxN], lR[kMaxN], eL[kMaxN];
    T L0Bx[kMaxN * kMaxN], L0By[kMaxN * kMaxN], eRBx[kMaxN], eRBy[kMaxN];
    T lLBx[kMaxN], lLBy[kMaxN];
    T w[kMaxN];
    T ihx, ihy, ihx2, ihy2;   // 1/hx, 1/hy, 1/hx^2, 1/hy^2
    double wq;                // hx * hy / 4: node weight = wq * w_i * w_j
};

// Default tile heights in waves: cell-per-lane tiles of 64 x 8 cells,
// bracket tiles of 8 rows (the tuner may pick 4 / 16 and 16).
constexpr int kCellWavesDefault = 8;
constexpr int kRowWavesDefault = 8;
// the cell tile of grids with a homogeneous Dirichlet axis (the only one
// their Laplacian / CG kernels are built for)
constexpr int kDirichletCellWaves = 8;

// Geometry of one launch, with the grid's tile shapes: cw waves (cell rows)
// per cell-per-lane tile, rw waves per row-per-lane bracket tile.
struct Geom {
    int n, nx, ny;
    int cw, rw;
    int bcx, bcy;     // 1: homogeneous Dirichlet along x / y
};

// Bracket / right-hand-side kernel parameters:
//   J = scale * (c0 J++ + Dx(c1 f Dy g - c2 Dy f g) + Dy(c2 Dx f g - c1 f Dx g))
// and, for an RK stage, out = a * w_n + b * (g + dt * (-J + D Lap_h g)), or
// with only_r set the right-hand side itself, out = -J + D Lap_h g.
struct RhsArgs {
    double c0, c1, c2, scale;
    double D, dt, a, b;
    int only_r;
};

// Device-side scalars of one CG solve (lives in the workspace).
struct CgScalars {
    double rr;        // <r, r>_W of the current residual
    double rz;        // <r, z>_W with z = M r (preconditioned); = rr for plain CG
    double bb;        // <b, b>_W
    double pq;        // <p, A p>_W
    double alpha, beta;
    double alpha_prev; // alpha of the iteration before the last (FP64
                       // directions: x takes two updates at a time)
    double tol2;      // rtol^2
    double mean_omega, mean_x;
    double ww;        // <omega, omega>_W
    double zero_tol2; // b counts as zero when <b,b>_W <= zero_tol2 * ww
    double ca, cb;    // guess = ca * psi_a + cb * psi_b (device copies)
    // mixed precision: <r,r>_W of the FP64 residual at the last replacement,
    // and the number of replacements
    double rr_true, rr_true_prev;
    double rr_max;    // largest recursive <r,r>_W since the last replacement
    double cr;        // coefficient of r in the next direction (1 but right
                      // after a replacement)
    int outer;
    int iter, max_iter;
    int done, converged, pending, first, zero, breakdown;
    int precond;      // 1: beta and rz come from the preconditioned dot kernel
};

// Ticket counters of the last-block-done reductions, one set per kernel kind:
// a global counter and kTicketGroups group counters, each on a 64-byte line
// of its own (atomics on one line are performed one after the other, about
// 12 ns apiece, so blocks finishing together queue on a single counter).
enum CounterId { kCntMean = 0, kCntInit, kCntDir, kCntRes, kCntFinish,
                 kCntInv, kCntDot, kCntCount };
constexpr int kTicketGroups = 32;
constexpr int kCntLine = 16;                               // counters per 64 bytes
constexpr int kCntStride = (1 + kTicketGroups) * kCntLine; // one kind's set
constexpr size_t kCntBytes = (size_t)kCntCount * kCntStride * sizeof(unsigned);

struct DevScratch {
    CgScalars* sc;          // device scalars
    unsigned* counters;     // kCntCount sets of kCntStride counters (kind k at
                            // counters + k * kCntStride), zero between launches
    double* partials;       // per-block partial sums (capacity max_blocks * 4)
    double* out3;           // 3 doubles (invariants / generic reductions)
    int max_blocks;
};

}  // namespace dgk

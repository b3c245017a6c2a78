// Fused bracket / right-hand-side kernel (row per lane).
//
// A lane holds one node row (cell, j) of a field; a wave covers S = 64/n
// consecutive cells of one cell row (lane = slot * n + j) and a workgroup
// WAVES consecutive cell rows.  The outer ring of slots and waves is halo:
// halo lanes load and compute like the others but never store, so every
// interior cell sees its full 3 x 3 cell neighbourhood (the bracket needs
// the x neighbours' y derivatives and vice versa).  Tiles of (S-2) x
// (WAVES-2) interior cells cover the grid; indices wrap periodically
// (Sec. 3 periodic closure).  x operators use one cross-lane shuffle per
// neighbour (rank-one face blocks of Sec. 4.2 eq. discrete_der); y
// operators stage rows in LDS, evaluate columns, and transpose back.
#pragma once

#include "dg_device.h"

namespace dgk {

template <int N, int WAVES>
struct Tile {
    static constexpr int S = 64 / N;          // cell slots per wave
    static constexpr int TX = S - 2;          // interior cells per tile in x
    static constexpr int TY = WAVES - 2;      // interior cells per tile in y
    // LDS layout of a cell's n x n values: the rows are staged by one lane
    // each and read back by columns (and the reverse), so both access
    // patterns must spread a wave over the banks.  For n = 2 and 4 the
    // column index is XORed with the row index and a cell takes n^2 + n
    // doubles: both patterns are then free of bank conflicts; odd n keep the
    // dense n^2 stride (at most two-way conflicts).
    static constexpr bool SWZ = (N == 2 || N == 4);
    static constexpr int CS = SWZ ? N * N + N : N * N;
    static constexpr int LDS_FIELD = WAVES * S * CS;
    __device__ static constexpr int at(int slot, int row, int col) {
        return slot * CS + row * N + (SWZ ? (col ^ row) : col);
    }
};


template <int N, int WAVES>
struct Ctx {
    int lane, wave, s, j;
    bool active;      // lane holds a node row
    bool interior;    // lane's cell is inside the tile and the grid: stores
    bool at_l, at_r, at_d, at_u;   // cell on a Dirichlet boundary of the grid
    bool sec_d;                    // second cell row above a Dirichlet y boundary
    long row;         // element index of this thread's row start
    int slot;         // wave * S + s (LDS cell slot)
};

template <int N, int WAVES>
__device__ __forceinline__ Ctx<N, WAVES> make_ctx(const Geom& g, int tilesX,
                                                  int nblocks, int b) {
    using TL = Tile<N, WAVES>;
    Ctx<N, WAVES> c;
    c.lane = threadIdx.x & 63;
    c.wave = threadIdx.x >> 6;
    c.s = c.lane / N;
    c.j = c.lane - c.s * N;
    c.active = c.s < TL::S;
    const int t = xcd_tile(b, nblocks);
    const int ty = t / tilesX, tx = t - ty * tilesX;
    const int cx = tx * TL::TX + c.s - 1;
    const int cy = ty * TL::TY + c.wave - 1;
    c.interior = c.active && c.s >= 1 && c.s <= TL::TX && c.wave >= 1 &&
                 c.wave <= TL::TY && cx < g.nx && cy < g.ny;
    c.at_l = g.bcx && cx == 0;
    c.at_r = g.bcx && cx == g.nx - 1;
    c.at_d = g.bcy && cy == 0;
    c.at_u = g.bcy && cy == g.ny - 1;
    c.sec_d = g.bcy && cy == 1;
    int gx = cx % g.nx;
    if (gx < 0) gx += g.nx;
    int gy = cy % g.ny;
    if (gy < 0) gy += g.ny;
    const long cell = c.active ? (long)gy * g.nx + gx : 0;
    c.row = (cell * N + c.j) * N;
    c.slot = c.wave * TL::S + (c.active ? c.s : TL::S - 1);
    return c;
}

// One 1D operator along x on this thread's row:
//   res = scale * (A0 u + eR (tR . u_right) + eL (tL . u_left))
// For the centred derivative (A0 = C0 with both faces' self terms, tR / tL
// the left / right trace functionals) a homogeneous Dirichlet boundary face
// carries zero flux (at_hi: right face, at_lo: left face): the neighbour
// trace is replaced by minus the cell's own trace at that face, which
// cancels the face's self term in C0 and drops the coupling.
template <int N, class T, bool DIR = false>
__device__ __forceinline__ void row_op(const T (&u)[N], int lane,
                                       const T* A0, const T* eR, const T* tR,
                                       const T* eL, const T* tL, T scale,
                                       T (&res)[N], bool at_lo = false,
                                       bool at_hi = false) {
    T dR = 0, dL = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        dR = fmx(tR[k], u[k], dR);
        dL = fmx(tL[k], u[k], dL);
    }
    // the right neighbour cell is N lanes up, the left one N lanes down;
    // lanes of the edge slots receive wrapped values but are halo
    // the shuffles run on every lane (a lane that skipped one would not
    // provide its value); the boundary replacement is a select afterwards
    const T nbR = __shfl(dR, lane + N);
    const T nbL = __shfl(dL, lane - N);
    const T fromR = (DIR && at_hi) ? -dL : nbR;
    const T fromL = (DIR && at_lo) ? -dR : nbL;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T a = fmx(eR[i], fromR, eL[i] * fromL);
#pragma unroll
        for (int k = 0; k < N; ++k) a = fmx(A0[i * N + k], u[k], a);
        res[i] = a * scale;
    }
}

// One 1D operator along y evaluated on column j of this thread's cell from
// rows staged in LDS; res[k] is the value at node (k, j).  The halo waves
// read clamped (wrong but in-bounds) neighbours and are never stored.
template <int N, int WAVES, class T, bool DIR = false>
__device__ __forceinline__ void col_op(const T* lds, const Ctx<N, WAVES>& c,
                                       const T* A0, const T* eR, const T* tR,
                                       const T* eL, const T* tL, T scale,
                                       T (&res)[N]) {
    using TL = Tile<N, WAVES>;
    const int up = c.slot + (c.wave + 1 < WAVES ? TL::S : 0);
    const int dn = c.slot - (c.wave > 0 ? TL::S : 0);
    T col[N];
    T du = 0, dd = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        col[k] = lds[TL::at(c.slot, k, c.j)];
        du = fmx(tR[k], lds[TL::at(up, k, c.j)], du);
        dd = fmx(tL[k], lds[TL::at(dn, k, c.j)], dd);
    }
    if (DIR) {   // zero flux on a Dirichlet boundary face (see row_op)
        T sb = 0, st = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            sb = fmx(tR[k], col[k], sb);
            st = fmx(tL[k], col[k], st);
        }
        if (c.at_u) du = -st;
        if (c.at_d) dd = -sb;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        T a = fmx(eR[k], du, eL[k] * dd);
#pragma unroll
        for (int m = 0; m < N; ++m) a = fmx(A0[k * N + m], col[m], a);
        res[k] = a * scale;
    }
}

// The LDG second derivative along x on this thread's row with the
// homogeneous Dirichlet closure of the viscous term (u-hat = 0 and q-hat =
// the inside trace on a boundary face, jump penalty against 0): the last
// cell (at_hi) drops its right coupling; the first (at_lo) uses A0B / eRB,
// drops its left coupling and gives its right neighbour tLB . u in place of
// tL . u.
template <int N, class T>
__device__ __forceinline__ void row_ldg(const T (&u)[N], int lane, const T* A0, const T* eR,
                                        const T* tR, const T* eL, const T* tL, const T* A0B,
                                        const T* eRB, const T* tLB, T scale, T (&res)[N],
                                        bool at_lo, bool at_hi) {
    T dR = 0, dL = 0, dB = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        dR = fmx(tR[k], u[k], dR);
        dL = fmx(tL[k], u[k], dL);
        dB = fmx(tLB[k], u[k], dB);
    }
    const T nbR = __shfl(dR, lane + N);
    const T nbL = __shfl(at_lo ? dB : dL, lane - N);
    const T fromR = at_hi ? T(0) : nbR;
    const T fromL = at_lo ? T(0) : nbL;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T a = fmx(at_lo ? eRB[i] : eR[i], fromR, eL[i] * fromL);
#pragma unroll
        for (int k = 0; k < N; ++k) a = fmx(at_lo ? A0B[i * N + k] : A0[i * N + k], u[k], a);
        res[i] = a * scale;
    }
}

// The same along y (column j of this thread's cell from rows staged in LDS):
// the top cell (at_u) drops its upper coupling, the bottom one (at_d) uses
// A0B / eRB and drops its lower coupling, and the second row (sec_d) reads
// the bottom cell through tLB.
template <int N, int WAVES, class T>
__device__ __forceinline__ void col_ldg(const T* lds, const Ctx<N, WAVES>& c, const T* A0,
                                        const T* eR, const T* tR, const T* eL, const T* tL,
                                        const T* A0B, const T* eRB, const T* tLB, T scale,
                                        T (&res)[N]) {
    using TL = Tile<N, WAVES>;
    const int up = c.slot + (c.wave + 1 < WAVES ? TL::S : 0);
    const int dn = c.slot - (c.wave > 0 ? TL::S : 0);
    const T* tl = c.sec_d ? tLB : tL;
    T col[N];
    T du = 0, dd = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        col[k] = lds[TL::at(c.slot, k, c.j)];
        du = fmx(tR[k], lds[TL::at(up, k, c.j)], du);
        dd = fmx(tl[k], lds[TL::at(dn, k, c.j)], dd);
    }
    if (c.at_u) du = 0;
    if (c.at_d) dd = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        T a = fmx(c.at_d ? eRB[k] : eR[k], du, eL[k] * dd);
#pragma unroll
        for (int m = 0; m < N; ++m) a = fmx(c.at_d ? A0B[k * N + m] : A0[k * N + m], col[m], a);
        res[k] = a * scale;
    }
}

template <int N, int WAVES, class T>
__device__ __forceinline__ void lds_put_row(T* lds, const Ctx<N, WAVES>& c,
                                            const T (&u)[N]) {
    if (c.active) {
#pragma unroll
        for (int i = 0; i < N; ++i) lds[Tile<N, WAVES>::at(c.slot, c.j, i)] = u[i];
    }
}

template <int N, int WAVES, class T>
__device__ __forceinline__ void lds_put_col(T* lds, const Ctx<N, WAVES>& c,
                                            const T (&v)[N]) {
    if (c.active) {
#pragma unroll
        for (int k = 0; k < N; ++k) lds[Tile<N, WAVES>::at(c.slot, k, c.j)] = v[k];
    }
}

template <int N, int WAVES, class T>
__device__ __forceinline__ void lds_get_row(const T* lds, const Ctx<N, WAVES>& c,
                                            T (&u)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = lds[Tile<N, WAVES>::at(c.slot, c.j, i)];
}

// Bracket and right-hand side.
//   J = scale * (c0 J++ + Dx(c1 f Dy g - c2 Dy f g) + Dy(c2 Dx f g - c1 f Dx g))
// (c0, c1, c2, scale) = (1, 1, 1, 1/3) gives (J++ + J+x + Jx+)/3 (Sec. 2
// eq. J); one of them alone gives a single form.  With VISC the kernel
// forms R = -J(f, g) + D Lap_h g and stores a * wn + b * (g + dt R)
// (SSP-RK3 stage combination; wn may be null when a == 0).
//
// b = c2 Dx f g - c1 f Dx g needs only x operators, so it is formed before
// the first barrier and staged with f and g: one column phase then
// evaluates every y operator (Dy f, Dy g, Dy b and the viscous Ly g) and one
// transpose brings back Dy f, Dy g and the sum D Ly g - scale Dy b
// (three barriers in all).  The two halo waves (first and last cell row of
// the tile) only feed their neighbours' y operators with rows of f, g and
// b: they skip the column phase and everything after it (a wave-uniform
// branch).

template <int N, int WAVES, bool VISC>
struct RhsLds {
    double A[Tile<N, WAVES>::LDS_FIELD];
    double B[Tile<N, WAVES>::LDS_FIELD];
    double C[Tile<N, WAVES>::LDS_FIELD];
};

template <int N, int WAVES, bool VISC, bool DIR = false>
__device__ __forceinline__ void rhs_body(
    int b, Geom g, int tilesX, int nblocks, const OpConst<double>& k,
    const double* __restrict__ f, const double* __restrict__ gg,
    const double* __restrict__ wn, double* __restrict__ out, const RhsArgs& ra,
    RhsLds<N, WAVES, VISC>& L) {
    double* lA = L.A;
    double* lB = L.B;
    double* lC = L.C;
    const auto c = make_ctx<N, WAVES>(g, tilesX, nblocks, b);
    const bool inner = c.wave > 0 && c.wave < WAVES - 1;   // wave-uniform

    // At n = 3, Dx f, Dx g and the viscous Lx g are formed again after the
    // column phase rather than held across its barriers (the same operations,
    // so the same values): fewer registers, more waves per SIMD.  At n = 4
    // and 5 that costs more than it saves.
    constexpr bool kLate = N == 3;
    double F[N], G[N];
    load_vec(f, c.row, F);
    load_vec(gg, c.row, G);

    double DxF[N], DxG[N], LxG[N];
    row_op<N, double, DIR>(F, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxF, c.at_l, c.at_r);
    row_op<N, double, DIR>(G, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxG, c.at_l, c.at_r);
    {
        double Bv[N];
#pragma unroll
        for (int i = 0; i < N; ++i) Bv[i] = ra.c2 * (DxF[i] * G[i]) - ra.c1 * (F[i] * DxG[i]);
        lds_put_row(lA, c, F);
        lds_put_row(lB, c, G);
        lds_put_row(lC, c, Bv);
    }
    if (VISC && inner && !kLate) {
        if (DIR)
            row_ldg(G, c.lane, k.L0x, k.eRx, k.lR, k.eL, k.lLx, k.L0Bx, k.eRBx, k.lLBx, k.ihx2,
                    LxG, c.at_l, c.at_r);
        else
            row_op(G, c.lane, k.L0x, k.eRx, k.lR, k.eL, k.lLx, k.ihx2, LxG);
    }
    __syncthreads();

    // column phase: Dy f, Dy g, Dy b (and Ly g) on this lane's column; the
    // barriers stay in uniform control flow, the halo waves just idle
    double cF[N], cG[N], cq[N];
    if (inner) {
        col_op<N, WAVES, double, DIR>(lA, c, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihy, cF);
        col_op<N, WAVES, double, DIR>(lB, c, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihy, cG);
        col_op<N, WAVES, double, DIR>(lC, c, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihy, cq);
        if (VISC) {
            double cL[N];
            if (DIR)
                col_ldg(lB, c, k.L0y, k.eRy, k.lR, k.eL, k.lLy, k.L0By, k.eRBy, k.lLBy, k.ihy2,
                        cL);
            else
                col_op(lB, c, k.L0y, k.eRy, k.lR, k.eL, k.lLy, k.ihy2, cL);
#pragma unroll
            for (int m = 0; m < N; ++m) cq[m] = ra.D * cL[m] - ra.scale * cq[m];
        }
    }
    __syncthreads();
    if (inner) {
        lds_put_col(lA, c, cF);
        lds_put_col(lB, c, cG);
        lds_put_col(lC, c, cq);
    }
    __syncthreads();
    if (!inner) return;        // no barrier follows
    double DyF[N], DyG[N], Q[N];
    lds_get_row(lA, c, DyF);
    lds_get_row(lB, c, DyG);
    lds_get_row(lC, c, Q);

    if (kLate) {
        row_op<N, double, DIR>(F, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxF, c.at_l, c.at_r);
        row_op<N, double, DIR>(G, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxG, c.at_l, c.at_r);
    }
    double J[N], A[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        J[i] = ra.c0 * (DxF[i] * DyG[i] - DyF[i] * DxG[i]);
        A[i] = ra.c1 * (F[i] * DyG[i]) - ra.c2 * (DyF[i] * G[i]);
    }
    double DxA[N];
    row_op<N, double, DIR>(A, c.lane, k.C0, k.cR, k.sR, k.cL, k.sL, k.ihx, DxA, c.at_l, c.at_r);
    if (VISC && kLate) {
        if (DIR)
            row_ldg(G, c.lane, k.L0x, k.eRx, k.lR, k.eL, k.lLx, k.L0Bx, k.eRBx, k.lLBx, k.ihx2,
                    LxG, c.at_l, c.at_r);
        else
            row_op(G, c.lane, k.L0x, k.eRx, k.lR, k.eL, k.lLx, k.ihx2, LxG);
    }

    if (!c.interior) return;
    double o[N];
    if (VISC) {
        // Q = D Ly g - scale Dy b
        double wnr[N];
        if (ra.a != 0.0) load_vec(wn, c.row, wnr);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double R = (ra.D * LxG[i] + Q[i]) - ra.scale * (J[i] + DxA[i]);
            const double s = ra.b * (G[i] + ra.dt * R);
            o[i] = ra.only_r ? R : ((ra.a != 0.0) ? ra.a * wnr[i] + s : s);
        }
    } else {
        // Q = Dy b
#pragma unroll
        for (int i = 0; i < N; ++i) o[i] = ra.scale * (J[i] + DxA[i] + Q[i]);
    }
    store_vec(out, c.row, o);
}


struct RowLaunch {
    int tilesX, tilesY, nblocks;
    // interior cells per tile: (64 / n - 2) along x, rw - 2 along y (Tile)
    __host__ __device__ explicit RowLaunch(const Geom& g) {
        const int tx = 64 / g.n - 2, ty = g.rw - 2;
        tilesX = (g.nx + tx - 1) / tx;
        tilesY = (g.ny + ty - 1) / ty;
        nblocks = tilesX * tilesY;
    }
};

}  // namespace dgk

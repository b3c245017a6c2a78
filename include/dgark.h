/*
 * dgark.h -- C ABI of the MI355X (gfx950) library for one right-hand-side
 * evaluation of the conservative discontinuous-Galerkin Arakawa scheme
 * (Einkemmer & Wiesenberger, "A conservative discontinuous Galerkin scheme
 * for the 2D incompressible Navier-Stokes equations"):
 *
 *     d_t omega + {psi, omega} = D Lap omega,    -Lap psi = omega      (Sec. 1)
 *
 * on a periodic rectangle, with the dG Arakawa bracket J = (J++ + J+x + Jx+)/3
 * (Sec. 2 eq. J, Sec. 3), the LDG Laplacian and a conjugate-gradient Poisson
 * solve (Sec. 6), advanced by SSP-RK3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status      Every function returning int returns DG_OK (0) or a negative
 *             DG_E_* code; dg_last_error() gives a thread-local message for
 *             the last failure on the calling thread.  Nothing throws.
 * Fields      Device pointers to FP64 arrays of dg_field_elems(grid) doubles,
 *             8-byte aligned, on the current HIP device, in the cell-major
 *             layout [cy][cx][j][i]: cell (cx, cy), y-node j, x-node i.  Node
 *             (i, j) of cell (cx, cy) sits at
 *                x = x0 + (cx + 1/2 + xi_i / 2) hx,  y = y0 + (cy + 1/2 + xi_j / 2) hy
 *             with xi the ascending Gauss-Legendre abscissas; the stored values
 *             are nodal values ("X-space", Sec. 4.3 last paragraph).
 * Ownership   The caller owns every field buffer; the library never frees
 *             caller memory.  A dg_grid is host-only and immutable (shareable
 *             across threads and streams).  A dg_workspace and a dg_state own
 *             device memory and serve one stream at a time.
 * Streams     `stream` is a hipStream_t passed as void* (NULL = default
 *             stream).  Calls are asynchronous on that stream unless stated
 *             otherwise; calls that return host scalars synchronise it.
 * Aliasing    An output that aliases an input it must not alias gives
 *             DG_E_ALIAS before any work is queued.
 */
#ifndef DGARK_H
#define DGARK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DG_OK              0
#define DG_E_INVAL        -1   /* invalid argument (null pointer, bad size, n out of range) */
#define DG_E_ALIAS        -2   /* an output aliases an input */
#define DG_E_NOMEM        -3   /* device or pinned-host allocation failed */
#define DG_E_HIP          -4   /* a HIP runtime call failed; message holds hipError text */
#define DG_E_NOCONV       -5   /* CG hit max_iter; outputs hold the last iterate, stats filled */
#define DG_E_UNSUPPORTED  -6   /* valid request this build does not implement */
#define DG_E_WORKSPACE    -7   /* workspace made for another grid or mode */

/* boundary conditions */
#define DG_BC_PERIODIC   0
#define DG_BC_DIRICHLET  1      /* homogeneous (see dg_grid_create for what it supports) */

/* CG precision modes (also the workspace mode) */
#define DG_PREC_FP64   0
#define DG_PREC_MIXED  1        /* r, p stored in FP32, FP64 arithmetic and solution,
                                   periodic FP64 residual replacement */
/* workspace option, OR-ed into the mode: also hold the fast-diagonalisation
   preconditioner (factored separable eigenbases of the 1D LDG operators, in
   FP64 and FP32, and two node-plane work fields) */
#define DG_WS_FD       0x10
/* workspace option, with DG_WS_FD: on a periodic grid, transform along the
   cells with the folded matrix products even where the half-length FFTs
   apply (both cell counts even, an axis beyond 32 cells).  No rocFFT plans
   are made: their creation compiles kernels for every new transform length
   (about 1-2 s per grid size), while a product-path workspace is ready in
   milliseconds; its applies are slower (one FP64 apply at n = 4: 129 against
   82 us at 256^2, 270 against 142 us at 512^2).  For short-lived workspaces,
   such as served requests of many different sizes. */
#define DG_WS_FD_PRODUCTS 0x20

/* CG preconditioners (dg_cg_opts.precond) */
#define DG_PRECOND_NONE 0       /* plain CG, as in Sec. 6 */
#define DG_PRECOND_FD   1       /* exact inverse of -Lap_h by fast diagonalisation */

/* single Jacobian forms for dg_bracket_form (Sec. 2 eq. J) */
#define DG_FORM_ARAKAWA 0       /* (J++ + J+x + Jx+)/3 */
#define DG_FORM_PP      1       /* J++ = Dx f Dy g - Dy f Dx g   */
#define DG_FORM_PX      2       /* J+x = Dx(f Dy g) - Dy(f Dx g) */
#define DG_FORM_XP      3       /* Jx+ = Dy(Dx f g) - Dx(Dy f g) */

typedef struct dg_grid dg_grid;
typedef struct dg_workspace dg_workspace;
typedef struct dg_state dg_state;

typedef struct {
    double rtol;        /* stop when ||r||_W <= rtol ||b||_W (in mixed mode: the
                           FP64 residual recomputed at a replacement) */
    int    max_iter;    /* CG iterations allowed */
    int    precision;   /* DG_PREC_FP64 or DG_PREC_MIXED; with DG_PRECOND_FD,
                           DG_PREC_MIXED applies the preconditioner in FP32
                           (the iteration itself stays FP64) */
    int    precond;     /* DG_PRECOND_NONE or DG_PRECOND_FD */
    int    check_every; /* FP64: iterations between host polls of the device
                           convergence flag; mixed: iterations between FP64
                           residual replacements (0 = library default, 32) */
} dg_cg_opts;

typedef struct {
    int    iters;         /* CG iterations (operator applications after r_0) */
    int    outer_iters;   /* mixed mode: FP64 residual replacements; otherwise 0 */
    double rel_residual;  /* final ||r||_W / ||b||_W (FP64 residual) */
    int    converged;     /* 1 if the tolerance was met; 2 (mixed mode only):
                             the recursive residual met it and the FP64
                             residual stopped decreasing above it, i.e. the
                             solve reached the attainable FP64 accuracy
                             (~ eps |Lap_h| |psi|); 0 otherwise */
} dg_cg_stats;

typedef struct {
    double     dt;          /* time step */
    double     D;           /* viscosity */
    dg_cg_opts cg;          /* options of the three Poisson solves */
    int        record_times;/* 1: time each stage with HIP events (stats.stage_ms) */
    int        form;        /* bracket in the right-hand side: DG_FORM_ARAKAWA
                               (0, the conservative average) or one single form
                               DG_FORM_PP / _PX / _XP (Sec. 2 eq. J; Sec. 6.2
                               compares J++ with J on the Lamb dipole) */
} dg_step_opts;

typedef struct {
    int   cg_iters[3];      /* CG operator applications of each stage's solve */
    float stage_ms[3];      /* device time of each stage (solve + RHS), if recorded */
    int   converged;        /* 1 if all three solves converged; 2 if they all
                               stopped but one only at the attainable FP64
                               accuracy (dg_cg_stats.converged == 2, mixed
                               mode); 0 if one did not converge */
} dg_step_stats;

/* Text of the last error on this thread ("" if none). */
const char* dg_last_error(void);

/* ---------------------------------------------------------------- grid --- */
/* Build the per-grid operator tables on the host: Gauss-Legendre nodes and
 * weights (Sec. 4.1), the X-space centred derivative blocks (Sec. 4.2 eqs.
 * discrete_der, matrix_xspace) and the LDG Laplacian blocks (Sec. 6).
 * n in [1, 5] polynomials per cell and direction, nx, ny >= 1 cells, finite
 * x0 < x1 and y0 < y1.  bc_x, bc_y: DG_BC_PERIODIC (Sec. 3 periodic closure)
 * or DG_BC_DIRICHLET (homogeneous: for the bracket, Sec. 3, read as a zero
 * numerical flux on the boundary faces of that axis, the closure that gives
 * Table 2's Dirichlet row; for the LDG Laplacian u-hat = 0 and q-hat = the
 * inside trace with the jump penalty against 0, the closure that gives
 * Table 3's Dirichlet columns).  A grid with a Dirichlet axis supports the
 * bracket, the Laplacian, the FP64 Poisson solve (no mean is removed:
 * -Lap_h is definite) plain or preconditioned, the mixed-precision
 * preconditioned solve, dg_rk_step, dg_ab_step and dg_invariants, with cell
 * tiles of 64 x 8; the mixed-precision solve without a preconditioner,
 * batches and the tuner return DG_E_UNSUPPORTED for it.  Touches no GPU.
 * Errors: DG_E_INVAL, DG_E_NOMEM. */
int  dg_grid_create(int n, int nx, int ny, double x0, double x1, double y0,
                    double y1, int bc_x, int bc_y, dg_grid** out);
void dg_grid_destroy(dg_grid* grid);                 /* NULL-safe */
/* Number of doubles in one field: ny * nx * n * n. */
size_t dg_field_elems(const dg_grid* grid);
/* Copy the grid's host tables into `out` (capacity `len` doubles), in the
 * order: xi[n], w[n], C0[n*n], cR[n], sR[n], cL[n], sL[n] (centred, h = 1),
 * then for x and for y: L0[n*n], eR[n], lR[n], eL[n], lL[n], L0B[n*n],
 * eRB[n], lLB[n] (the LDG second derivative of that axis).  A 1D centred derivative
 * is (1/h)[C0 u_m + cR (sR.u_{m+1}) + cL (sL.u_{m-1})], the 1D LDG operator
 * (1/h^2)[L0 u_m + eR (lR.u_{m+1}) + eL (lL.u_{m-1})] with the axis' own h
 * (its jump penalty is folded in, so these blocks depend on h); on a
 * homogeneous Dirichlet axis the last cell drops the right coupling, the
 * first cell is (1/h^2)[L0B u_0 + eRB (lR.u_1)] and the second one sees the
 * first through eL (lLB.u_0).  All n x n blocks row-major.  Returns the
 * number of doubles written, or a negative status (DG_E_INVAL if len is too
 * small). */
int  dg_grid_tables(const dg_grid* grid, double* out, int len);

/* Tile shapes of the grid's stencil launches: the cell-per-lane kernels
 * (Laplacian, CG) use tiles of 64 x cw cells, cw in {4, 8, 16}; the fused
 * bracket kernel tiles of rw rows, rw in {8, 16} (default 8 and 8).  Taller
 * tiles re-read fewer halo rows but hold more registers and LDS per
 * workgroup.  The shapes change the reduction order and hence the last bits
 * of CG results; set them before using the grid (a batch copies them when an
 * instance is attached).  DG_E_INVAL for other values, and for cw != 8 on a
 * grid with a Dirichlet axis. */
int  dg_grid_set_tiles(dg_grid* grid, int cw, int rw);
int  dg_grid_tiles(const dg_grid* grid, int* cw, int* rw);
/* Tile autotuner: on the current device, time `reps` CG iterations for each
 * cell tile height and `reps` fused bracket evaluations for each bracket tile
 * height on this grid, from the caller's field omega (device, canonical; its
 * mean-free part must be nonzero), and set the fastest shapes in the grid.
 * ms_out5 (host, optional): mean ms per CG iteration for cw = 4, 8, 16 and
 * per bracket for rw = 8, 16.  Allocates and frees a temporary workspace;
 * synchronises the stream.  Not thread-safe with other users of the grid. */
int  dg_grid_tune(dg_grid* grid, const double* omega, int reps, double* ms_out5,
                  void* stream);

/* ----------------------------------------------------------- workspace --- */
/* Device bytes a workspace for (grid, mode) holds: CG vectors x, r, p, the
 * two RK stage fields, reduction partials and scalars, plus FP32 r and p in
 * DG_PREC_MIXED mode, plus (DG_WS_FD) the preconditioner's z vector, two
 * node-plane fields and per axis the factored eigenbasis in FP64 and FP32
 * (the N x N cell Fourier basis, 2 (N/2 + 1) mixing blocks of 2n x 2n and
 * n N eigenvalues; one set when the axes agree), a copy of omega and three
 * sets of device scalars for RK steps queued ahead (rocBLAS and, on the FFT
 * path, rocFFT keep their own work buffers on top: dg_workspace_held_bytes
 * counts them once the workspace exists).  On a grid
 * with a Dirichlet axis the preconditioner holds instead two dense work
 * images of n^2 Nx Ny doubles and per axis the dense (n N)^2 eigenbasis and
 * n N eigenvalues in FP64 and FP32.  This is the figure that admission
 * control budgets.
 * mode = DG_PREC_FP64 or DG_PREC_MIXED, optionally | DG_WS_FD. */
int  dg_workspace_bytes(const dg_grid* grid, int mode, size_t* bytes);
/* Device bytes a created workspace holds: dg_workspace_bytes plus the work
 * buffers the preconditioner's libraries hold (rocFFT's, known only once its
 * plans exist, and what rocBLAS reports for its handle at creation).  The
 * figure to charge once a workspace exists.  Host-only. */
int  dg_workspace_held_bytes(const dg_workspace* ws, size_t* bytes);
/* Allocate a workspace on the current device (hipMalloc + pinned host
 * scalars).  With DG_WS_FD on a grid with a Dirichlet axis this runs the
 * dense eigensolver (rocSOLVER) on the device, synchronously.  Errors:
 * DG_E_INVAL, DG_E_NOMEM, DG_E_HIP; DG_E_UNSUPPORTED for DG_WS_FD on a grid
 * with a Dirichlet axis of more than 8192 nodes (n * cells). */
int  dg_workspace_create(const dg_grid* grid, int mode, dg_workspace** out);
void dg_workspace_destroy(dg_workspace* ws);         /* NULL-safe */

/* Measurement support.  While enabled, every CG polling chunk of a solve on
 * this workspace times one direction-update kernel launch and one
 * residual-update kernel launch with HIP events recorded by those dispatches
 * on the solve's stream (only iterations the device really executed are
 * counted).  dg_profile_read
 * stores {sum_ms_direction, launches, sum_ms_residual, launches} accumulated
 * since the previous read and resets them.  Host-only bookkeeping. */
int  dg_profile_enable(dg_workspace* ws, int on);
int  dg_profile_read(dg_workspace* ws, double* out4);

/* ------------------------------------------------------------ operators --- */
/* out = J(f, g), the conservative dG Arakawa bracket
 * (J++ + J+x + Jx+)/3 with products taken node-wise in X-space
 * (Sec. 2 eq. J, Sec. 3 last paragraphs, Sec. 4.3 last equation).
 * out must not alias f or g (DG_E_ALIAS).  Asynchronous. */
int  dg_poisson_bracket(const dg_grid* grid, const double* f, const double* g,
                        double* out, void* stream);
/* out = one of the single forms J++, J+x, Jx+ or the Arakawa average
 * (form = DG_FORM_*), Sec. 2 eq. J.  Same rules as dg_poisson_bracket. */
int  dg_bracket_form(const dg_grid* grid, const double* f, const double* g,
                     double* out, int form, void* stream);
/* out = Lap_h f, the LDG Laplacian of Sec. 6 (local dG of Cockburn and Shu,
 * fluxes unprinted; read as): per axis Dx_backward Dx_forward minus the jump
 * penalty C11 sum_faces [u][v] with C11 = 1, the reading whose Table 3
 * errors match the printed ones (n = 1 on a periodic axis: no penalty, the
 * 5-point Laplacian the paper falls back to).  -W Lap_h is symmetric
 * positive semi-definite with the constants as null space (periodic) or
 * definite (a Dirichlet axis).  out != f.  Asynchronous. */
int  dg_laplace_apply(const dg_grid* grid, const double* f, double* out,
                      void* stream);

/* ----------------------------------------------------------------- CG --- */
/* Solve -Lap_h psi = omega - mean_W(omega) by conjugate gradients in the
 * Gauss inner product (Sec. 6: symmetric system, CG; Sec. 4.1 eq. def_norm).
 * On entry psi holds the initial guess (its W-mean is removed); on exit the
 * zero-mean solution.  ||omega - mean|| = 0 gives psi = 0.  On a grid with a
 * Dirichlet axis -Lap_h is definite: -Lap_h psi = omega, no mean removed.
 * ws must be made for this grid, with DG_WS_FD for DG_PRECOND_FD (any
 * precision mode), else in mixed mode for DG_PREC_MIXED (else
 * DG_E_WORKSPACE).  Synchronises the stream
 * (convergence polling).  Returns DG_E_NOCONV when max_iter was hit or the
 * iteration broke down (psi holds the last iterate).  psi must not alias
 * omega. */
int  dg_cg_solve_poisson(const dg_grid* grid, const double* omega, double* psi,
                         const dg_cg_opts* opts, dg_cg_stats* stats,
                         dg_workspace* ws, void* stream);
/* z = (-Lap_h)^+ r: the exact solution of -Lap_h z = r - mean_W(r) with
 * W-mean zero, by fast diagonalisation -- the preconditioner DG_PRECOND_FD
 * applies (beyond the paper, whose CG of Sec. 6 is unpreconditioned).  The
 * 1D LDG operator of each periodic axis is block circulant, so Bloch waves
 * reduce it to n x n Hermitian (in the Gauss weights) symbols whose
 * eigenvectors give a real W-orthonormal basis V with L V = V diag(lambda);
 * then z = V_y [(V_y^T W_y R W_x V_x) / -(lambda_y + lambda_x)] V_x^T, the
 * constant mode dropped.  V is applied in factored form (the cell Fourier
 * transform, then 2n x 2n mixing per wave number); the transform is an FP64
 * matrix product up to 512 cells per axis -- with phases at the cell centres,
 * so that cells c and N - 1 - c fold each axis into two products of half
 * size (2 n^2 Nx Ny (Nx + Ny) flops per call) -- and beyond, when both
 * cell counts are even, an FFT (rocFFT) of each real row read as a complex
 * row of half length (an odd count keeps the matrix products).  On a grid
 * with a homogeneous
 * Dirichlet axis (-Lap_h definite, z = (-Lap_h)^-1 r) both axes use dense
 * eigenbases (the Dirichlet one from rocSOLVER's symmetric eigensolver) and
 * the apply is four dense matrix products, 2 (n Nx)(n Ny)(n Nx + n Ny)
 * flops.  r, z: canonical fields, z must not alias r.  ws must hold
 * DG_WS_FD.  Asynchronous. */
int  dg_precond_apply(const dg_grid* grid, const double* r, double* z,
                      dg_workspace* ws, void* stream);
/* The eigenbasis dg_precond_apply uses along one periodic axis (axis 0: x,
 * 1: y), built on the host from the Bloch symbols: V (host, (N n)^2 doubles,
 * column-major, row = c n + i for cell c and node i, column = mode) with
 * L V = V diag(lam) and V^T W V = I for the 1D LDG second derivative L and
 * Gauss weights W of that axis; lam (host, N n doubles); *zero = the column
 * of the constant mode.  The cell Fourier basis is the one the transforms
 * use on this grid: phases at the cell centres (the matrix products: up to
 * 512 cells per axis, or an odd count) or at the cell edges (the FFTs).  DG_E_UNSUPPORTED for
 * a Dirichlet axis (its basis is computed on the device).  Touches no GPU. */
int  dg_grid_fd_basis(const dg_grid* grid, int axis, double* V, double* lam, int* zero);
/* The 1D LDG second derivative of one axis (axis 0: x, 1: y; Sec. 6 as read
 * for dg_laplace_apply, with the Dirichlet closure on a Dirichlet axis), the
 * operator the preconditioner diagonalises: L (host, (N n)^2 doubles,
 * column-major, row and column = c n + i).  Lap_h is L_x along x plus L_y
 * along y.  Touches no GPU. */
int  dg_grid_axis_operator(const dg_grid* grid, int axis, double* L);

/* ------------------------------------------------------------ stepping --- */
/* History of Poisson solutions used for the CG initial guess: the
 * linear-in-time extrapolation of the two most recent solves (Sec. 6,
 * initial guess from the last two solutions).  Owns five device fields:
 * two hold the history, three take the solves of a step (so a step queued
 * ahead of its convergence checks can be taken again from the history it
 * started from). */
int  dg_state_create(const dg_grid* grid, double t0, dg_state** out);
void dg_state_destroy(dg_state* st);                 /* NULL-safe */
/* Device pointer to the most recent psi (NULL before the first solve). */
const double* dg_state_psi(const dg_state* st);
/* Copy the most recent psi into out (device, dg_field_elems doubles);
 * asynchronous.  DG_E_INVAL before the first solve. */
int  dg_state_copy_psi(const dg_state* st, double* out, void* stream);
double dg_state_time(const dg_state* st);
/* One SSP-RK3 (Shu-Osher) step of d_t omega = -J(psi, omega) + D Lap_h omega
 * with stage times t, t+dt, t+dt/2; each stage solves -Lap_h psi = omega_s
 * by CG (opts->cg) from the extrapolated guess, then one fused kernel forms
 * the bracket, the viscous term and the stage combination.  omega is updated
 * in place; state->t advances by dt.  Synchronises the stream.  Returns
 * DG_E_NOCONV if a solve hit max_iter (the step is still completed).
 * With DG_PRECOND_FD in FP64 the three stages are queued with one PCG
 * iteration each and checked once at the end of the step (one host round
 * trip per step); if a stage has not converged, omega and the psi history
 * are restored and the step is taken again with every solve polled after
 * each iteration -- the result is the same either way. */
int  dg_rk_step(const dg_grid* grid, double* omega, dg_state* state,
                const dg_step_opts* opts, dg_step_stats* stats,
                dg_workspace* ws, void* stream);

/* K-step Adams-Bashforth stepping, the paper's integrator (Sec. 6 uses three
 * steps; Sec. 6.2, Table 4 runs K = 1..4):
 *     omega_{n+1} = omega_n + dt sum_{j<K} b_j R(omega_{n-j}),
 *     b = (1), (3/2, -1/2), (23, -16, 5)/12, (55, -59, 37, -9)/24,
 * R = -J(psi, omega) + D Lap_h omega, psi from one Poisson solve per step
 * (opts->cg, initial guess extrapolated from the last two solves).  The
 * state owns K right-hand-side fields and a dg_state (psi history, time).
 * While fewer than K-1 earlier right-hand sides are known the step is an
 * SSP-RK3 step (the paper does not state the start-up; this reading makes
 * the start third-order accurate).  K outside [1, 4]: DG_E_INVAL. */
typedef struct dg_ab_state dg_ab_state;
int  dg_ab_state_create(const dg_grid* grid, int K, double t0, dg_ab_state** out);
void dg_ab_state_destroy(dg_ab_state* ab);           /* NULL-safe */
double dg_ab_time(const dg_ab_state* ab);
/* The psi history inside (for dg_state_psi / dg_state_copy_psi). */
const dg_state* dg_ab_psi_state(const dg_ab_state* ab);
/* One step; omega (device, canonical) is updated in place, the state's time
 * advances by opts->dt.  stats->cg_iters[0]: the solve of this step;
 * [1]: the start-up RK3 stages' solves (0 once the multistep method runs).
 * Synchronises the stream.  DG_E_NOCONV if a solve hit max_iter (the step
 * is still completed). */
int  dg_ab_step(const dg_grid* grid, double* omega, dg_ab_state* ab,
                const dg_step_opts* opts, dg_step_stats* stats, dg_workspace* ws,
                void* stream);

/* --------------------------------------------------------- invariants --- */
/* out[0..2] = (V, E, Omega) = (int omega, 1/2 int psi omega, 1/2 int omega^2)
 * (Sec. 2 eq. quantities, E by the Green identity) with Gauss quadrature
 * (Sec. 4.1 eq. def_norm), summed in a fixed order (deterministic).
 * dg_invariants writes host memory and synchronises the stream;
 * dg_invariants_dev writes 3 doubles to device memory asynchronously. */
int  dg_invariants(const dg_grid* grid, const double* omega, const double* psi,
                   double* out_host3, dg_workspace* ws, void* stream);
int  dg_invariants_dev(const dg_grid* grid, const double* omega,
                       const double* psi, double* out_dev3, dg_workspace* ws,
                       void* stream);
/* dg_invariants_dev without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops).  The
 * reduction scratch (at most 1024 blocks x 4 doubles of partial sums plus the
 * ticket counters, 47 KB) is a static device array that each device holds
 * from its first call until the process ends; any grid size fits it (the
 * reduction launches at most 1024 blocks).  This call never allocates.  The
 * first call on a device looks the array up and queues a counter clear on
 * `stream`: make it outside stream capture.  Every call on one device shares
 * that device's array, so calls that overlap in time on one device (other
 * streams, other threads) race; calls queued on one stream do not.
 * out_dev3: 3 doubles of device memory, written asynchronously with the
 * same values, bit for bit, as dg_invariants_dev.  Errors: DG_E_INVAL for a
 * NULL argument or a device index >= 64, DG_E_HIP. */
int  dg_invariants_noalloc(const dg_grid* grid, const double* omega,
                           const double* psi, double* out_dev3, void* stream);

/* ------------------------------------------------------------- batches --- */
/* Many independent instances (any n, any grid) advanced together: each
 * kernel kind runs as one fused launch per polynomial order over a
 * device-resident (instance, block) work list (one block per item), and the setup, CG-chunk and
 * finish/RHS sequences of an RK stage are replayed as HIP graphs.  Every
 * instance is cut into the same blocks and uses the same device code as
 * dg_rk_step, so its result is bitwise the same alone or in any batch.
 * Instances can be attached and detached between steps (continuous
 * batching).  A batch lives on the current device and serves one stream at
 * a time. */
typedef struct dg_batch dg_batch;
/* capacity in [1, 4096] slots.  Errors: DG_E_INVAL, DG_E_NOMEM. */
int  dg_batch_create(int capacity, dg_batch** out);
void dg_batch_destroy(dg_batch* b);                  /* NULL-safe; synchronises */
/* Put an instance into a free slot.  grid must outlive the membership;
 * omega (device, canonical, caller-owned) is advanced in place by each step.
 * The batch allocates the instance's workspace and state
 * (dg_batch_member_bytes).  Returns the slot in *slot.  DG_E_INVAL when
 * the batch is full. */
int  dg_batch_attach(dg_batch* b, const dg_grid* grid, double* omega, double dt,
                     double D, double t0, int* slot);
/* Free a slot and its device memory (synchronises the device). */
int  dg_batch_detach(dg_batch* b, int slot);
/* Device bytes one member holds (workspace + state + record): the figure
 * an admission controller budgets. */
int  dg_batch_member_bytes(const dg_grid* grid, size_t* bytes);
/* 1 (default): replay captured HIP graphs; 0: launch kernels directly. */
int  dg_batch_use_graphs(dg_batch* b, int on);
/* Give the members attached from now on workspaces with the fast-
 * diagonalisation preconditioner (ws_fd_flags: DG_WS_FD, optionally with
 * DG_WS_FD_PRODUCTS; 0: none, the default), so that dg_batch_rk_step can
 * take opts->precond = DG_PRECOND_FD.  Such a member also holds
 * dg_workspace_bytes(grid, DG_PREC_FP64 | ws_fd_flags) instead of the plain
 * workspace, and two more fields of psi history.  Such a batch also takes
 * grids with a homogeneous Dirichlet axis (their fused steps are refused:
 * DG_E_UNSUPPORTED).  Only while no member is attached: DG_E_INVAL
 * otherwise, or for other flags. */
int  dg_batch_use_precond(dg_batch* b, int ws_fd_flags);
/* One SSP-RK3 step of every attached instance.  With opts->precond =
 * DG_PRECOND_NONE (FP64 CG, opts->precision must be DG_PREC_FP64) the
 * members advance together in fused launches.  With DG_PRECOND_FD (FP64 or
 * DG_PREC_MIXED) each member takes its step through dg_rk_step on this
 * stream in turn, with the same results as a stand-alone step
 * (DG_E_WORKSPACE unless dg_batch_use_precond preceded the attaches).
 * iters_out, if not NULL, receives the CG iterations of slot i's stage k at
 * [3 i + k] (capacity * 3 ints).  Synchronises the stream.  DG_E_NOCONV if
 * some solve hit max_iter (the step was still completed). */
int  dg_batch_rk_step(dg_batch* b, const dg_cg_opts* opts, int* iters_out,
                      void* stream);
/* 1 if every solve of slot's last dg_batch_rk_step converged, 0 if one hit
 * max_iter (the step was still completed), DG_E_INVAL for an empty slot. */
int  dg_batch_slot_converged(const dg_batch* b, int slot);
/* Copy slot's most recent psi to out (device); asynchronous. */
int  dg_batch_copy_psi(const dg_batch* b, int slot, double* out, void* stream);
/* Simulation time of a slot (0 for an empty slot). */
double dg_batch_time(const dg_batch* b, int slot);

#ifdef __cplusplus
}
#endif
#endif /* DGARK_H */

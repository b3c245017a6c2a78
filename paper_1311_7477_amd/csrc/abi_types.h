// Definitions of the opaque C-ABI objects and the error helpers shared by
// the ABI translation units (abi.cpp, batch.cpp).  Internal.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/dgark.h"
#include "dg_internal.h"
#include "fd_basis.h"

using dgk::HostTables; using dgk::OpConst; using dgk::Geom; using dgk::DevScratch; using dgk::CgScalars;

struct dg_grid {
    int n, nx, ny;
    double x0, x1, y0, y1, hx, hy, area;
    HostTables t;
    OpConst<double> k64;
    Geom geom;
    size_t elems;
};

struct dg_workspace {
    int n, nx, ny, mode, device;
    size_t elems;
    double *x, *r, *p0, *p1;   // CG vectors, lane-interleaved layout
    double *s1, *s2;           // RK stage fields, canonical layout
    float *r32, *q0, *q1;      // mixed precision: FP32 residual and directions
    double* z;                 // preconditioned residual (DG_WS_FD workspaces)
    double* wbak;              // DG_WS_FD: omega at the start of a queued RK step
    CgScalars* sc3;            // DG_WS_FD: device scalars of the three queued stage solves
    dgk::FdDevice* fd;         // fast-diagonalisation preconditioner, or NULL
    DevScratch d;
    CgScalars* host;           // pinned, 4 slots (2 poll slots + 2 spare)
    hipEvent_t ev[2];
    hipEvent_t tev[4];
    size_t bytes;
    // live kernel timing (measurement support)
    int prof_on;
    hipEvent_t pev[2][4];
    int pev_iter[2];           // iteration index sampled in that poll slot (-1: none)
    double prof_ms[2];         // summed ms of sampled direction / residual launches
    double prof_n[2];
};

struct dg_state {
    int n, nx, ny;
    size_t elems;
    double* buf[5];            // nbuf of them allocated
    int nbuf;                  // 3, or 5 so that a queued RK step keeps the
                               // history it started from until it is verified
    int ia, ib;                // indices of the newest / previous solution (-1 none)
    int resv[2];               // buffers a new solve must not take (-1 none)
    double ta, tb, t;
    int count;
};

namespace dgk {
// Record a failure (thread-local message) and return its code.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
// The guess of the next solve from the state's history (linear-in-time
// extrapolation through the two newest solves), and the free buffer x.
void state_guess(const dg_state* st, double ts, const double** pa, double* ca,
                 const double** pb, double* cb, double** x, int* xi);
// Record that buffer xi now holds the solve at time ts.
void state_push(dg_state* st, int xi, double ts);
// A state with nbuf (3 or 5) history buffers; dg_state_create makes 5.
int state_create(const dg_grid* g, double t0, int nbuf, dg_state** out);
// DG_E_UNSUPPORTED for an operation that needs a periodic grid.
int periodic_only(const char* what);
// Bracket coefficients of a DG_FORM_* (Sec. 2 eq. J): c0 J++ + c1 J+x +
// c2 Jx+, times scale; DG_E_INVAL for an unknown form.
int form_coeffs(int form, double* c0, double* c1, double* c2, double* scale);
// The Poisson solve behind dg_cg_solve_poisson and the steppers: guess
// ca pa + cb pb (canonical), result in x (canonical, must not alias pa, pb).
int solve_poisson(const dg_grid* g, const double* omega, double* x, const double* pa,
                  double ca, const double* pb, double cb, const dg_cg_opts* opts,
                  dg_cg_stats* st, dg_workspace* ws, hipStream_t s);
// Fast-diagonalisation preconditioner resources (fd_apply.cpp): device bytes,
// creation / destruction, and z = M r on the image buffer img0 in place.
size_t fd_bytes(const dg_grid* g);
int fd_supported(const dg_grid* g);     // DG_OK, or DG_E_UNSUPPORTED with the reason
bool fd_uses_fft(int nx, int ny);       // periodic grids: FFT (else GEMM) cell transforms
int fd_create(const dg_grid* g, bool products, FdDevice** out);   // products: no FFTs
size_t fd_extra_bytes(const FdDevice* fd);   // library work buffers beyond fd_bytes
void fd_destroy(FdDevice* fd);
int fd_apply_image(const FdDevice* fd, bool fp32, hipStream_t s);
// Layout of the work image fd_apply_image expects and returns.
enum FdLayout { kFdPlanes = 0, kFdFolded = 1, kFdDense = 2 };
int fd_layout(const FdDevice* fd);
}  // namespace dgk

#define HIP_TRY(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return dgk::hip_fail(e_, #call); \
    } while (0)

"""FP64 oracle: the dG Arakawa bracket, the LDG Laplacian, CG, SSP-RK3 and
the invariants, written plainly from the paper's definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring): never used by the
product path.

Layout.  Public functions take and return fields in the canonical cell-major
layout ``u[cy, cx, j, i]`` (numpy shape ``(Ny, Nx, n, n)``): cell (cx, cy),
y-node j, x-node i, holding nodal values at the Gauss-Legendre points
("X-space", Sec. 4.3 last paragraph).  Internally the oracle works on the
image layout ``U[cy*n + j, cx*n + i]`` where a 1D operator along x is a right
multiplication by its transpose and one along y a left multiplication
(Sec. 4.3, the Kronecker-product extension to two dimensions).

Parity status of each function is stated in its docstring; every function is
pinned by a test in ``tests/test_oracle_*.py`` against something other than
itself (library routines, closed forms, printed values, invariants).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from numpy.polynomial.legendre import leggauss

__all__ = [
    "legendre_values", "ReferenceElement", "Grid1D", "Grid2D",
    "to_image", "from_image", "dx", "dy", "dx_form", "dy_form",
    "bracket_forms", "bracket", "laplacian", "inner", "wmean",
    "cg_poisson", "pcg_poisson", "FastDiagonalisation", "rhs", "rk3_step",
    "rk3_step_pcg",
    "PsiHistory", "invariants", "AB_COEFFS", "ab_step",
    "dense_operators", "dense_poisson_solve", "arakawa_fd_jacobian",
    "five_point_laplacian",
]


# --------------------------------------------------------------------------
# Reference element (Sec. 4.1)
# --------------------------------------------------------------------------
def legendre_values(nk: int, x) -> np.ndarray:
    """p_0..p_{nk-1} at the points x by the three-term recursion
    (k+1) p_{k+1} = (2k+1) x p_k - k p_{k-1}, p_0 = 1, p_1 = x (Sec. 4.1,
    eq. recursion).  Returns shape (nk, len(x))."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    out = np.zeros((nk, x.size))
    out[0] = 1.0
    if nk > 1:
        out[1] = x
    for k in range(1, nk - 1):
        out[k + 1] = ((2 * k + 1) * x * out[k] - k * out[k - 1]) / (k + 1)
    return out


@dataclass
class ReferenceElement:
    """All P x P pieces of Sec. 4.1 for P = n polynomials per cell.

    xi, w   Gauss-Legendre abscissas (ascending) and weights on [-1, 1].
    B       backward transform, B[j, k] = p_k(xi_j)  (L-space -> X-space).
    F       forward transform, F[k, j] = (2k+1)/2 w_j p_k(xi_j).
    D       D[i, j] = int_{-1}^{1} p_i p_j' (Sec. 4.1, eq. legendre_operators),
            from the closed form 1 - (-1)^(i+j) for i <= j-1, else 0.
    R, L, RL, LR   products of end values p_i(+-1) p_j(+-1).
    That    diag(2k+1), so that T = That / h (Sec. 4.1, eq. diagonal).
    """
    n: int
    xi: np.ndarray = field(init=False)
    w: np.ndarray = field(init=False)
    B: np.ndarray = field(init=False)
    F: np.ndarray = field(init=False)
    D: np.ndarray = field(init=False)
    R: np.ndarray = field(init=False)
    L: np.ndarray = field(init=False)
    RL: np.ndarray = field(init=False)
    LR: np.ndarray = field(init=False)
    That: np.ndarray = field(init=False)

    def __post_init__(self):
        n = self.n
        if not (1 <= n <= 5):
            raise ValueError("oracle supports 1 <= n <= 5")
        self.xi, self.w = leggauss(n)
        P = legendre_values(n, self.xi)          # P[k, j] = p_k(xi_j)
        self.B = P.T.copy()
        k = np.arange(n)
        self.F = ((2 * k + 1) / 2.0)[:, None] * self.w[None, :] * P
        D = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                if i <= j - 1:
                    D[i, j] = 1.0 - (-1.0) ** (i + j)
        self.D = D
        pr = np.ones(n)                          # p_k(+1) = 1
        pl = (-1.0) ** k                         # p_k(-1) = (-1)^k
        self.R = np.outer(pr, pr)
        self.L = np.outer(pl, pl)
        self.RL = np.outer(pr, pl)
        self.LR = np.outer(pl, pr)
        self.That = np.diag(2.0 * k + 1.0)


# --------------------------------------------------------------------------
# 1D grid and derivative matrices (Sec. 3 eq. discrete_derivative,
# Sec. 4.2 eqs. discrete_der, matrix_xspace)
# --------------------------------------------------------------------------
def _shift(N: int, offset: int, periodic: bool = True) -> sp.csr_matrix:
    """Shift 1^+ (offset=+1: (1^+ f)^m = f^{m+1}) or 1^- (offset=-1)
    (Sec. 4.2, eq. operator_one); periodic wrap as in the periodic closure of
    Sec. 3, or no coupling across the ends (homogeneous Dirichlet)."""
    rows = np.arange(N)
    cols = rows + offset
    if periodic:
        cols = cols % N
    keep = (cols >= 0) & (cols < N)
    return sp.csr_matrix((np.ones(int(keep.sum())), (rows[keep], cols[keep])), shape=(N, N))


class Grid1D:
    """Equidistant 1D grid on [a, b] with N cells of size h (Sec. 4.1) and n
    polynomials per cell; bc = "periodic" or "dirichlet" (homogeneous, Sec. 3
    boundary closures; read as a zero numerical flux on the two boundary
    faces, see lspace_operator)."""

    def __init__(self, n: int, N: int, a: float, b: float, bc: str = "periodic"):
        if bc not in ("periodic", "dirichlet"):
            raise ValueError(bc)
        self.el = ReferenceElement(n)
        self.n, self.N, self.a, self.b = n, N, float(a), float(b)
        self.bc = bc
        self.h = (self.b - self.a) / N
        self._cache = {}

    def nodes(self) -> np.ndarray:
        """x_{mj} = x_m + (h/2) xi_j with x_m the cell centre (Sec. 4.1)."""
        centres = self.a + (np.arange(self.N) + 0.5) * self.h
        return (centres[:, None] + 0.5 * self.h * self.el.xi[None, :]).ravel()

    def weights(self) -> np.ndarray:
        """Diagonal of 1 (x) W, W = diag(h w_j / 2) (Sec. 4.1, eq. diagonal)."""
        return np.tile(0.5 * self.h * self.el.w, self.N)

    def lspace_operator(self, theta: float, boundary: str = "zero") -> sp.csr_matrix:
        """L-space matrix Mbar_theta of the weak dG derivative with numerical
        flux fhat = theta f^+ + (1 - theta) f^- at every face
        (Sec. 3, eq. discrete_derivative):

          fbar_x^{m i} = T^{ii} [ fhat_{m+1/2} p_i(1) - fhat_{m-1/2} p_i(-1)
                                  - sum_k fbar^{m k} D_{k i} ].

        Writing the face values with the end values of the neighbouring cells
        gives  Mbar = 1^+ (x) theta RL + 1 (x) (-theta L + (1-theta) R - D^T)
                      - 1^- (x) (1-theta) LR.
        theta = 1/2 is the standard (centred) flux of eq. standard-flux;
        theta = 1 / 0 are the one-sided fluxes used by the LDG Laplacian.

        Homogeneous Dirichlet, boundary = "zero": the numerical flux on the
        two boundary faces is zero (the reading that reproduces Table 2's
        Dirichlet row; the alternative of a zero outside value, fhat =
        f_inside / 2, keeps the operator skew and would conserve int f J and
        int g J, which Table 2 says it does not).  So the boundary cells lose
        both the neighbour coupling and their own share of the boundary-face
        flux.  boundary = "inside": the flux on a boundary face is the
        cell's own trace there (the LDG flux of the gradient variable on a
        Dirichlet boundary, see laplacian)."""
        e = self.el
        N = self.N
        per = self.bc == "periodic"
        self_block = -theta * e.L + (1.0 - theta) * e.R - e.D.T
        M = (sp.kron(_shift(N, +1, per), theta * e.RL)
             + sp.kron(sp.identity(N), self_block)
             - sp.kron(_shift(N, -1, per), (1.0 - theta) * e.LR))
        if not per:
            n = self.n
            M = M.tolil()
            if boundary == "zero":
                M[(N - 1) * n:, (N - 1) * n:] = M[(N - 1) * n:, (N - 1) * n:] - (1.0 - theta) * e.R
                M[:n, :n] = M[:n, :n] + theta * e.L
            elif boundary == "inside":
                M[(N - 1) * n:, (N - 1) * n:] = M[(N - 1) * n:, (N - 1) * n:] + theta * e.R
                M[:n, :n] = M[:n, :n] - (1.0 - theta) * e.L
            else:
                raise ValueError(boundary)
        return M.tocsr()

    def derivative(self, kind: str = "centred", boundary: str = "zero") -> sp.csr_matrix:
        """X-space derivative f_x = (1 (x) V) M f with
        M = (1 (x) F^T) Mbar (1 (x) F) and the mass-matrix inverse T = That/h
        folded in (Sec. 4.2, eq. matrix_xspace):
            f_x = (1 (x) V F^T) Mbar (1 (x) F) f .
        kind: 'centred' (theta=1/2), 'forward' (theta=1), 'backward' (0);
        boundary: the Dirichlet boundary-face flux (see lspace_operator)."""
        key = (kind, boundary)
        if key in self._cache:
            return self._cache[key]
        theta = {"centred": 0.5, "forward": 1.0, "backward": 0.0}[kind]
        e = self.el
        N = self.N
        V = np.diag(2.0 / (self.h * e.w))
        left = sp.kron(sp.identity(N), V @ e.F.T)
        right = sp.kron(sp.identity(N), e.F)
        op = (left @ self.lspace_operator(theta, boundary) @ right).tocsr()
        self._cache[key] = op
        return op

    def jumps(self) -> sp.csr_matrix:
        """Jump operator J (faces x nodes): [u]_f = u(right side) - u(left
        side) at every face, the traces taken from the cell polynomials
        (u(+-1) = sum_k ubar_k p_k(+-1), ubar = F u).  Periodic: the N faces
        m - 1/2, m = 0..N-1 (face 0 joins cell N-1 to cell 0).  Dirichlet:
        the N + 1 faces, the two boundary faces against the outside value 0."""
        e = self.el
        n, N = self.n, self.N
        k = np.arange(n)
        tr_r = np.ones(n) @ e.F                  # u(+1) as a functional of u
        tr_l = ((-1.0) ** k) @ e.F               # u(-1)
        per = self.bc == "periodic"
        faces = N if per else N + 1
        J = sp.lil_matrix((faces, N * n))
        for f in range(faces):
            right, left = f, f - 1               # cells on either side of face f
            if per:
                left %= N
            if right < N:
                J[f, right * n:(right + 1) * n] = J[f, right * n:(right + 1) * n].toarray() + tr_l
            if left >= 0:
                J[f, left * n:(left + 1) * n] = J[f, left * n:(left + 1) * n].toarray() - tr_r
        return J.tocsr()

    def penalty(self) -> float:
        """C11 of the LDG jump penalty: 1 (in the units of the domain), except
        n = 1 on a periodic grid, where the paper falls back to the plain
        finite-difference Laplacian (Sec. 6.1, the P = 1 remark): 0."""
        return 0.0 if (self.n == 1 and self.bc == "periodic") else 1.0

    def laplacian(self) -> sp.csr_matrix:
        """1D LDG second derivative (Sec. 6: the local dG method of Cockburn
        and Shu; its fluxes are not printed, this is the reading whose Table 3
        errors match the printed ones):
            L = D_backward D_forward - C11 W^-1 J^T J,
        alternating fluxes (u-hat from the right, q-hat from the left of each
        face) plus the jump penalty C11 sum_f [u][v] with C11 = penalty().
        Homogeneous Dirichlet (Cockburn-Shu's boundary fluxes): u-hat = 0 and
        q-hat = the inside trace of q on the boundary faces, and the penalty
        acts on the jump against the outside value 0.  W L is symmetric;
        negative semi-definite with the constants as null space (periodic),
        negative definite (Dirichlet)."""
        if "lap" not in self._cache:
            L = self.derivative("backward", "inside") @ self.derivative("forward", "zero")
            c11 = self.penalty()
            if c11 != 0.0:
                J = self.jumps()
                L = L - c11 * sp.diags(1.0 / self.weights()) @ (J.T @ J)
            self._cache["lap"] = L.tocsr()
        return self._cache["lap"]


class Grid2D:
    """Tensor-product grid [x0,x1] x [y0,y1], Nx x Ny cells, n polynomials
    per cell and direction (Sec. 4.3, two dimensions); each axis periodic or
    homogeneous Dirichlet."""

    def __init__(self, n: int, Nx: int, Ny: int, x0=0.0, x1=2 * math.pi,
                 y0=0.0, y1=2 * math.pi, bc_x="periodic", bc_y="periodic"):
        self.n, self.Nx, self.Ny = n, Nx, Ny
        self.gx = Grid1D(n, Nx, x0, x1, bc_x)
        self.gy = Grid1D(n, Ny, y0, y1, bc_y)
        self.hx, self.hy = self.gx.h, self.gy.h

    @property
    def shape(self):
        return (self.Ny, self.Nx, self.n, self.n)

    @property
    def periodic(self) -> bool:
        """Both axes periodic: -Delta_h then has the constants as null space
        and the Poisson problem is solved for W-mean-free data."""
        return self.gx.bc == "periodic" and self.gy.bc == "periodic"

    def node_coords(self):
        """(X, Y) of every node in the canonical layout (Sec. 4.1 nodes)."""
        xs = self.gx.nodes().reshape(self.Nx, self.n)
        ys = self.gy.nodes().reshape(self.Ny, self.n)
        X = np.broadcast_to(xs[None, :, None, :], self.shape).copy()
        Y = np.broadcast_to(ys[:, None, :, None], self.shape).copy()
        return X, Y

    def weights(self) -> np.ndarray:
        """Gauss weights W[cy,cx,j,i] = (hx w_i / 2)(hy w_j / 2)
        (Sec. 4.1, eq. def_norm, tensor product)."""
        wx = self.gx.weights().reshape(self.Nx, self.n)
        wy = self.gy.weights().reshape(self.Ny, self.n)
        return wy[:, None, :, None] * wx[None, :, None, :]


# --------------------------------------------------------------------------
# Layout conversion
# --------------------------------------------------------------------------
def to_image(u: np.ndarray) -> np.ndarray:
    """[cy, cx, j, i] -> U[cy*n + j, cx*n + i]."""
    Ny, Nx, n, _ = u.shape
    return np.ascontiguousarray(u.transpose(0, 2, 1, 3)).reshape(Ny * n, Nx * n)


def from_image(U: np.ndarray, n: int) -> np.ndarray:
    """Inverse of to_image."""
    Ny, Nx = U.shape[0] // n, U.shape[1] // n
    return np.ascontiguousarray(U.reshape(Ny, n, Nx, n).transpose(0, 2, 1, 3))


def _apply_x(op: sp.csr_matrix, U: np.ndarray) -> np.ndarray:
    return np.asarray((op @ U.T).T)


def _apply_y(op: sp.csr_matrix, U: np.ndarray) -> np.ndarray:
    return np.asarray(op @ U)


# --------------------------------------------------------------------------
# Derivatives, bracket, Laplacian
# --------------------------------------------------------------------------
def dx_form(g: Grid2D, U: np.ndarray, kind="centred") -> np.ndarray:
    """D_x on an image-layout field: acts along (cx, i) (Sec. 4.3)."""
    return _apply_x(g.gx.derivative(kind), U)


def dy_form(g: Grid2D, U: np.ndarray, kind="centred") -> np.ndarray:
    """D_y on an image-layout field: acts along (cy, j) (Sec. 4.3)."""
    return _apply_y(g.gy.derivative(kind), U)


def dx(g: Grid2D, u: np.ndarray, kind="centred") -> np.ndarray:
    return from_image(dx_form(g, to_image(u), kind), g.n)


def dy(g: Grid2D, u: np.ndarray, kind="centred") -> np.ndarray:
    return from_image(dy_form(g, to_image(u), kind), g.n)


def bracket_forms(g: Grid2D, f: np.ndarray, h: np.ndarray):
    """The three dG Jacobians of Sec. 2 eq. J / Sec. 3 with products taken
    node-wise in X-space (Sec. 4.3, last equation):
        J++ = Dx(f) Dy(h) - Dy(f) Dx(h)
        J+x = Dx(f Dy(h)) - Dy(f Dx(h))
        Jx+ = Dy(Dx(f) h) - Dx(Dy(f) h)
    Each is evaluated literally (no regrouping).  Returns (Jpp, Jpx, Jxp) in
    the canonical layout."""
    F, G = to_image(f), to_image(h)
    Fx, Fy = dx_form(g, F), dy_form(g, F)
    Gx, Gy = dx_form(g, G), dy_form(g, G)
    Jpp = Fx * Gy - Fy * Gx
    Jpx = dx_form(g, F * Gy) - dy_form(g, F * Gx)
    Jxp = dy_form(g, Fx * G) - dx_form(g, Fy * G)
    return tuple(from_image(J, g.n) for J in (Jpp, Jpx, Jxp))


def bracket(g: Grid2D, f: np.ndarray, h: np.ndarray, form: str = "arakawa") -> np.ndarray:
    """Conservative dG Arakawa bracket J = (J++ + J+x + Jx+)/3 (Sec. 2 eq. J,
    Sec. 3 end), or one single Jacobian form: form = "pp" (J++), "px"
    (J+x) or "xp" (Jx+).  Sec. 6.2 time-steps the Lamb dipole with J++ alone
    to show what the average conserves."""
    Jpp, Jpx, Jxp = bracket_forms(g, f, h)
    if form == "arakawa":
        return (Jpp + Jpx + Jxp) / 3.0
    return {"pp": Jpp, "px": Jpx, "xp": Jxp}[form]


def laplacian(g: Grid2D, u: np.ndarray) -> np.ndarray:
    """LDG Laplacian Delta_h u = Lx u + Ly u with the 1D operators of
    Grid1D.laplacian along each axis (Sec. 6 first paragraph; Sec. 4.3,
    Kronecker products)."""
    U = to_image(u)
    return from_image(_apply_x(g.gx.laplacian(), U) + _apply_y(g.gy.laplacian(), U), g.n)


# --------------------------------------------------------------------------
# Inner products (Sec. 4.1, eq. def_norm)
# --------------------------------------------------------------------------
def inner(g: Grid2D, u: np.ndarray, v: np.ndarray) -> float:
    """<u, v> = sum W u v with Gauss weights (Sec. 4.1, eq. def_norm)."""
    return float(np.sum(g.weights() * u * v))


def wmean(g: Grid2D, u: np.ndarray) -> float:
    W = g.weights()
    return float(np.sum(W * u) / np.sum(W))


# --------------------------------------------------------------------------
# Conjugate gradient for -Delta_h psi = omega (Sec. 6, first paragraph)
# --------------------------------------------------------------------------
@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    converged: bool
    rel_residual: float


def cg_poisson(g: Grid2D, omega: np.ndarray, guess=None, rtol=1e-12,
               max_iter=100000) -> CGResult:
    """Plain conjugate gradient on -Delta_h psi = b in the W inner product
    (A = -Delta_h is W-self-adjoint).  Periodic grid: b = omega minus its
    W-mean (constants span the null space), the initial guess has its W-mean
    removed and so has the returned psi.  Dirichlet on an axis: A is
    definite, b = omega.  Iteration stops when ||r||_W <= rtol ||b||_W,
    tested on r_0 and after every update; iters counts operator
    applications after r_0.  ||b||_W = 0 returns psi = 0."""
    W = g.weights()

    def dot(u, v):
        return float(np.sum(W * u * v))

    b, x = _poisson_start(g, omega, guess)
    bnorm = math.sqrt(dot(b, b))
    if bnorm == 0.0:
        return CGResult(np.zeros_like(omega), 0, True, 0.0)
    r = b + laplacian(g, x)                      # r = b - A x
    rr = dot(r, r)
    it = 0
    converged = math.sqrt(rr) <= rtol * bnorm
    p = r.copy()
    while not converged and it < max_iter:
        q = -laplacian(g, p)                     # q = A p
        alpha = rr / dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        rr_new = dot(r, r)
        if math.sqrt(rr_new) <= rtol * bnorm:
            converged = True
            rr = rr_new
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    if g.periodic:
        x = x - wmean(g, x)
    return CGResult(x, it, converged, math.sqrt(rr) / bnorm)


def _poisson_start(g: Grid2D, omega: np.ndarray, guess):
    """(b, x0) of the Poisson solves: on a periodic grid both W-mean-free."""
    if g.periodic:
        b = omega - wmean(g, omega)
        x = np.zeros_like(omega) if guess is None else guess - wmean(g, guess)
    else:
        b = omega.copy()
        x = np.zeros_like(omega) if guess is None else guess.copy()
    return b, x


# --------------------------------------------------------------------------
# Preconditioned CG (beyond the paper, which uses plain CG in Sec. 6): the
# preconditioner is the exact inverse of -Delta_h on W-mean-free fields
# built from separable 1D eigenbases ("fast diagonalisation").
# --------------------------------------------------------------------------
class FastDiagonalisation:
    """Exact inverse of -Delta_h on W-mean-free fields (periodic grid; with a
    Dirichlet axis, of the definite -Delta_h on all fields).

    The 1D LDG second derivative L of each axis is self-adjoint in the 1D
    Gauss inner product (W L is symmetric, W = diag of Grid1D.weights), so
    W^(1/2) L W^(-1/2) = Q diag(lam) Q^T with Q orthogonal (numpy eigh) and
    V = W^(-1/2) Q satisfies V^T W V = I and L V = V diag(lam).  Since
    Delta_h = Ly (x) I + I (x) Lx on the image layout (Sec. 4.3, Kronecker
    products), its eigenvectors are V_y[:, b] (x) V_x[:, a] with eigenvalues
    lam_y[b] + lam_x[a] <= 0, and
        (-Delta_h)^+ R = V_y [ (V_y^T W_y R W_x V_x) / -(lam_y + lam_x) ] V_x^T
    with the single zero eigenvalue (the constant mode, lam_x = lam_y = 0)
    dropped on a periodic grid.  Dense eigh: meant for grids up to a few thousand nodes per
    axis."""

    def __init__(self, g: Grid2D):
        self.g = g
        self.Vx, self.lx, self.wx = self._axis(g.gx)
        self.Vy, self.ly, self.wy = self._axis(g.gy)
        mu = -(self.ly[:, None] + self.lx[None, :])
        inv = np.zeros_like(mu)
        nz = np.ones_like(mu, dtype=bool)
        if g.periodic:
            nz[int(np.argmax(self.ly)), int(np.argmax(self.lx))] = False
        inv[nz] = 1.0 / mu[nz]
        self.inv_mu = inv

    @staticmethod
    def _axis(g1: Grid1D):
        L = g1.laplacian().toarray()
        w = g1.weights()
        sw = np.sqrt(w)
        S = sw[:, None] * L / sw[None, :]
        lam, Q = np.linalg.eigh(0.5 * (S + S.T))
        return Q / sw[:, None], lam, w

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = (-Delta_h)^+ r for a canonical-layout field r."""
        R = to_image(r)
        Rt = self.Vy.T @ (self.wy[:, None] * R * self.wx[None, :]) @ self.Vx
        Z = self.Vy @ (Rt * self.inv_mu) @ self.Vx.T
        return from_image(Z, self.g.n)


def pcg_poisson(g: Grid2D, omega: np.ndarray, guess=None, rtol=1e-12,
                max_iter=100000, precond=None) -> CGResult:
    """Preconditioned CG in the W inner product on -Delta_h psi = b, with
    the same b, initial guess, stopping rule (on ||r||_W, tested on r_0 and
    after every update), iteration count and zero-mean result as
    cg_poisson.  precond(r) returns z = M r for a W-self-adjoint positive
    M; None means M = I, which reproduces cg_poisson's iterates exactly."""
    W = g.weights()

    def dot(u, v):
        return float(np.sum(W * u * v))

    apply_m = (lambda u: u.copy()) if precond is None else precond
    b, x = _poisson_start(g, omega, guess)
    bnorm = math.sqrt(dot(b, b))
    if bnorm == 0.0:
        return CGResult(np.zeros_like(omega), 0, True, 0.0)
    r = b + laplacian(g, x)
    rr = dot(r, r)
    it = 0
    converged = math.sqrt(rr) <= rtol * bnorm
    z = apply_m(r)
    rz = dot(r, z)
    p = z
    while not converged and it < max_iter:
        q = -laplacian(g, p)
        alpha = rz / dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        rr = dot(r, r)
        if math.sqrt(rr) <= rtol * bnorm:
            converged = True
            break
        z = apply_m(r)
        rz_new = dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    if g.periodic:
        x = x - wmean(g, x)
    return CGResult(x, it, converged, math.sqrt(rr) / bnorm)


# --------------------------------------------------------------------------
# Right-hand side and SSP-RK3
# --------------------------------------------------------------------------
def rhs(g: Grid2D, omega: np.ndarray, psi: np.ndarray, D: float,
        form: str = "arakawa") -> np.ndarray:
    """R(omega) = -J(psi, omega) + D Delta_h omega for
    d_t omega + {psi, omega} = D Delta omega (Sec. 1, eq. vorticity); J is
    the bracket of the given form (see bracket)."""
    return -bracket(g, psi, omega, form) + D * laplacian(g, omega)


class PsiHistory:
    """The last two Poisson solutions and their times; the CG initial guess
    is the linear-in-time extrapolation through them (Sec. 6, "extrapolating
    the solutions of the last two time steps", read for three RK stages per
    step: the two most recent solves)."""

    def __init__(self):
        self.items = []          # [(t, psi)] most recent first

    def guess(self, t: float):
        if not self.items:
            return None
        if len(self.items) == 1 or self.items[0][0] == self.items[1][0]:
            return self.items[0][1].copy()
        (ta, pa), (tb, pb) = self.items[0], self.items[1]
        theta = (t - ta) / (ta - tb)
        return pa + theta * (pa - pb)

    def push(self, t: float, psi: np.ndarray):
        self.items = [(t, psi.copy())] + self.items[:1]


def rk3_step(g: Grid2D, omega: np.ndarray, t: float, dt: float, D: float,
             hist: PsiHistory, rtol=1e-12, max_iter=100000, form: str = "arakawa"):
    """One Shu-Osher SSP-RK3 step of d_t omega = R(omega); stage times t,
    t+dt, t+dt/2; each stage solves the Poisson problem for its psi.
    Returns (omega_new, [cg iteration counts])."""
    iters = []

    def stage_rhs(w, ts):
        res = cg_poisson(g, w, hist.guess(ts), rtol, max_iter)
        hist.push(ts, res.x)
        iters.append(res.iters)
        return rhs(g, w, res.x, D, form)

    u1 = omega + dt * stage_rhs(omega, t)
    u2 = 0.75 * omega + 0.25 * (u1 + dt * stage_rhs(u1, t + dt))
    u3 = omega / 3.0 + (2.0 / 3.0) * (u2 + dt * stage_rhs(u2, t + 0.5 * dt))
    return u3, iters


# --------------------------------------------------------------------------
# K-step Adams-Bashforth (Sec. 6: the paper's stepper, three steps; Sec. 6.2
# and Table 4: K = 1..4)
# --------------------------------------------------------------------------
# omega_{n+1} = omega_n + dt sum_j b_j R(omega_{n-j}), j = 0..K-1: the
# explicit Adams-Bashforth weights of order K (integrals of the Lagrange
# polynomials through the last K right-hand sides).
AB_COEFFS = {
    1: (1.0,),
    2: (3.0 / 2.0, -1.0 / 2.0),
    3: (23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0),
    4: (55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0),
}


def ab_step(g: Grid2D, omega: np.ndarray, t: float, dt: float, D: float, K: int,
            rhs_hist: list, hist: PsiHistory, rtol=1e-12, max_iter=100000,
            precond=None, form: str = "arakawa"):
    """One step of the K-step Adams-Bashforth method.  rhs_hist holds the
    right-hand sides of the previous steps, most recent first, and is
    updated in place.  While fewer than K-1 are known the step is an SSP-RK3
    step instead (the paper does not state how the multistep method starts;
    this reading starts it with a third-order one-step method), after
    recording R(omega_n).  Each R needs the Poisson solve of its omega, from
    the extrapolated guess.  Returns (omega_new, [cg iteration counts])."""
    res = pcg_poisson(g, omega, hist.guess(t), rtol, max_iter, precond)
    hist.push(t, res.x)
    r_n = rhs(g, omega, res.x, D, form)
    if len(rhs_hist) < K - 1:
        rhs_hist.insert(0, r_n)
        w, its = rk3_step_pcg(g, omega, t, dt, D, hist, rtol, max_iter, precond, form)
        return w, [res.iters] + its
    rs = [r_n] + rhs_hist[:K - 1]
    w = omega.copy()
    for b, r in zip(AB_COEFFS[K], rs):
        w = w + (dt * b) * r
    rhs_hist[:] = rs[:K - 1]
    return w, [res.iters]


def rk3_step_pcg(g: Grid2D, omega: np.ndarray, t: float, dt: float, D: float,
                 hist: PsiHistory, rtol=1e-12, max_iter=100000, precond=None,
                 form: str = "arakawa"):
    """rk3_step with the stage solves by pcg_poisson and an optional
    preconditioner (same stages, same guesses)."""
    iters = []

    def stage_rhs(w, ts):
        res = pcg_poisson(g, w, hist.guess(ts), rtol, max_iter, precond)
        hist.push(ts, res.x)
        iters.append(res.iters)
        return rhs(g, w, res.x, D, form)

    u1 = omega + dt * stage_rhs(omega, t)
    u2 = 0.75 * omega + 0.25 * (u1 + dt * stage_rhs(u1, t + dt))
    u3 = omega / 3.0 + (2.0 / 3.0) * (u2 + dt * stage_rhs(u2, t + 0.5 * dt))
    return u3, iters


# --------------------------------------------------------------------------
# Invariants (Sec. 2, eq. quantities; integrals by Gauss quadrature)
# --------------------------------------------------------------------------
def invariants(g: Grid2D, omega: np.ndarray, psi: np.ndarray):
    """(V, E, Omega) = (int omega, 1/2 int psi omega, 1/2 int omega^2)
    with the Gauss inner product (Sec. 2 eq. quantities and the identity
    E = 1/2 int psi omega; Sec. 4.1 eq. def_norm)."""
    W = g.weights()
    return (float(np.sum(W * omega)), 0.5 * float(np.sum(W * psi * omega)),
            0.5 * float(np.sum(W * omega * omega)))


# --------------------------------------------------------------------------
# Dense brute force (tiny grids)
# --------------------------------------------------------------------------
def dense_operators(g: Grid2D):
    """Dense matrices acting on the flattened image layout:
    Dx = I (x) Mx, Dy = My (x) I, Lap = I (x) Lx + Ly (x) I (Sec. 4.3,
    Kronecker products)."""
    Ix = np.identity(g.Nx * g.n)
    Iy = np.identity(g.Ny * g.n)
    Mx = g.gx.derivative("centred").toarray()
    My = g.gy.derivative("centred").toarray()
    Lx = g.gx.laplacian().toarray()
    Ly = g.gy.laplacian().toarray()
    return np.kron(Iy, Mx), np.kron(My, Ix), np.kron(Iy, Lx) + np.kron(Ly, Ix)


def dense_poisson_solve(g: Grid2D, omega: np.ndarray) -> np.ndarray:
    """Minimum-norm least-squares solution of -Lap psi = omega - mean, then
    the W-mean removed: the exact zero-mean solution on a tiny periodic
    grid (Dirichlet axis: the solution of -Lap psi = omega)."""
    _, _, Lap = dense_operators(g)
    rhs = omega - wmean(g, omega) if g.periodic else omega
    b = to_image(rhs).ravel()
    psi, *_ = np.linalg.lstsq(-Lap, b, rcond=None)
    psi = from_image(psi.reshape(g.Ny * g.n, g.Nx * g.n), g.n)
    return psi - wmean(g, psi) if g.periodic else psi


# --------------------------------------------------------------------------
# Independent finite-difference formulas for the P = 1 reductions
# --------------------------------------------------------------------------
def arakawa_fd_jacobian(psi2d: np.ndarray, zeta2d: np.ndarray, hx: float,
                        hy: float) -> np.ndarray:
    """Arakawa's 1966 energy- and enstrophy-conserving 9-point Jacobian on a
    periodic grid, written with index shifts (array axis 0 = y, axis 1 = x).
    At P = 1 the dG bracket reduces to it (Sec. 2, the remark after eq. J;
    Sec. 3, P = 1 and the standard flux)."""
    def s(a, di, dj):            # value at (x + di, y + dj)
        return np.roll(np.roll(a, -di, axis=1), -dj, axis=0)
    p, z = psi2d, zeta2d
    j1 = ((s(p, 1, 0) - s(p, -1, 0)) * (s(z, 0, 1) - s(z, 0, -1))
          - (s(p, 0, 1) - s(p, 0, -1)) * (s(z, 1, 0) - s(z, -1, 0)))
    j2 = (s(p, 1, 0) * (s(z, 1, 1) - s(z, 1, -1))
          - s(p, -1, 0) * (s(z, -1, 1) - s(z, -1, -1))
          - s(p, 0, 1) * (s(z, 1, 1) - s(z, -1, 1))
          + s(p, 0, -1) * (s(z, 1, -1) - s(z, -1, -1)))
    j3 = (s(z, 0, 1) * (s(p, 1, 1) - s(p, -1, 1))
          - s(z, 0, -1) * (s(p, 1, -1) - s(p, -1, -1))
          - s(z, 1, 0) * (s(p, 1, 1) - s(p, 1, -1))
          + s(z, -1, 0) * (s(p, -1, 1) - s(p, -1, -1)))
    return (j1 + j2 + j3) / (12.0 * hx * hy)


def five_point_laplacian(u2d: np.ndarray, hx: float, hy: float) -> np.ndarray:
    """Periodic 5-point Laplacian (axis 0 = y, axis 1 = x)."""
    return ((np.roll(u2d, -1, 1) - 2 * u2d + np.roll(u2d, 1, 1)) / hx ** 2
            + (np.roll(u2d, -1, 0) - 2 * u2d + np.roll(u2d, 1, 0)) / hy ** 2)

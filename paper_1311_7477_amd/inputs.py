"""Seeded synthetic initial conditions, shared by the tests, the oracle runs
and the benchmark.

This module holds none of the scheme's arithmetic: it only evaluates analytic
initial fields at the nodes of the canonical layout (nodal values at the
ascending Gauss-Legendre points of each cell, Sec. 4.1) and draws seeded
random numbers.  Every generator returns a float64 numpy array of shape
(Ny, Nx, n, n) indexed [cy, cx, j, i].

Recipes (no dataset is involved; the paper's own workloads are analytic):

* ``taylor_green_noise``: sin x sin y plus i.i.d. U(-amp, amp) per node.
* ``random_spectrum``: decaying-turbulence field with energy spectrum
  E(k) ~ (k/k0)^4 exp(-2 (k/k0)^2) over integer wave vectors 1 <= |k| <= 3 k0,
  random complex amplitudes, Hermitian symmetric, zero mean, rescaled to
  kinetic energy 1/2 per unit area; evaluated exactly at the nodes by
  separable Fourier sums.
* ``double_shear_layer``: tanh shear layers of width rho with a sinusoidal
  transverse perturbation, vorticity taken with the sign convention of
  -Lap psi = omega and u = (-psi_y, psi_x).
* ``decay_taylor_green``: omega = 2 sin x sin y (Sec. 6.1 initial value).
* ``conservation_pair``: f = sin x cos y, g = exp(0.1 (x + y)) (Sec. 5.2).
* ``lamb_dipole``: the Lamb dipole of Sec. 6.2, omega = 2 lam U / J0(lam R)
  J1(lam r) cos(theta) inside r < R, zero outside, lam R the first zero of J1;
  centred in the box, theta measured from the x axis (the paper states
  neither the centre nor the reference axis); Bessel functions from scipy.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.legendre import leggauss


def node_coords(n, Nx, Ny, x0=0.0, x1=2 * math.pi, y0=0.0, y1=2 * math.pi):
    """Coordinates (X, Y) of every node in the canonical layout."""
    xi, _ = leggauss(n)
    hx, hy = (x1 - x0) / Nx, (y1 - y0) / Ny
    xs = x0 + (np.arange(Nx)[:, None] + 0.5 + 0.5 * xi[None, :]) * hx
    ys = y0 + (np.arange(Ny)[:, None] + 0.5 + 0.5 * xi[None, :]) * hy
    shape = (Ny, Nx, n, n)
    X = np.broadcast_to(xs[None, :, None, :], shape).copy()
    Y = np.broadcast_to(ys[:, None, :, None], shape).copy()
    return X, Y


def _remove_quadrature_mean(u, n, Nx, Ny):
    """Subtract the Gauss-quadrature mean so that the field has zero total
    vorticity on the grid (periodic problem, constant null space)."""
    _, w = leggauss(n)
    W = np.broadcast_to((w[:, None] * w[None, :])[None, None], u.shape)
    return u - float(np.sum(W * u) / np.sum(W))


def taylor_green_noise(n, N, seed=0, amp=1e-3):
    """sin x sin y on [0, 2pi]^2 plus seeded U(-amp, amp) noise per node,
    quadrature mean removed."""
    X, Y = node_coords(n, N, N)
    rng = np.random.default_rng(seed)
    u = np.sin(X) * np.sin(Y) + rng.uniform(-amp, amp, X.shape)
    return _remove_quadrature_mean(u, n, N, N)


def decay_taylor_green(n, N):
    X, Y = node_coords(n, N, N)
    return 2.0 * np.sin(X) * np.sin(Y)


def conservation_pair(n, N):
    """f = sin x cos y, g = exp(0.1 (x+y)) on [0, pi]^2."""
    X, Y = node_coords(n, N, N, 0.0, math.pi, 0.0, math.pi)
    return np.sin(X) * np.cos(Y), np.exp(0.1 * (X + Y))


def white_noise(n, Nx, Ny, seed=0):
    return np.random.default_rng(seed).standard_normal((Ny, Nx, n, n))


def _spectrum_coefficients(k0, rng, energy):
    """Half-plane amplitudes c[kx, ky] (kx in [-K, K], ky in [0, K]) of a
    real field omega = 2 Re sum_half c_k exp(i k.x), and the matching
    streamfunction amplitudes (psi_k = omega_k / |k|^2)."""
    K = int(math.ceil(3 * k0))
    kx = np.arange(-K, K + 1)[:, None].astype(np.float64)
    ky = np.arange(0, K + 1)[None, :].astype(np.float64)
    kk = np.sqrt(kx ** 2 + ky ** 2)
    half = (ky > 0) | ((ky == 0) & (kx > 0))
    shell = (kk >= 1.0) & (kk <= 3 * k0)
    mask = half & shell
    a = rng.standard_normal(kk.shape)
    b = rng.standard_normal(kk.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        Ek = (kk / k0) ** 4 * np.exp(-2.0 * (kk / k0) ** 2)
        amp = np.sqrt(kk * Ek)
    c = np.where(mask, amp * (a + 1j * b) / math.sqrt(2.0), 0.0)
    k2 = np.where(mask, kk ** 2, 1.0)
    # energy per unit area of the real field: 1/2 sum_all |omega_k|^2/|k|^2
    # = sum_half |c_k|^2 / |k|^2
    e = float(np.sum(np.abs(c) ** 2 / k2))
    c *= math.sqrt(energy / e)
    return K, c, c / k2


def random_modes(n, Nx, Ny, seed=0, kmax=4):
    """Smooth seeded field on [0, 2pi]^2 for any Nx x Ny: sum over wave
    vectors 0 < |kx|, ky <= kmax (ky >= 0) of a N(0,1) amplitude over
    kx^2 + ky^2 times sin(kx x + ky y + phase), phase ~ U[0, 2pi)."""
    X, Y = node_coords(n, Nx, Ny)
    rng = np.random.default_rng(seed)
    w = np.zeros_like(X)
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            if kx == 0 and ky == 0:
                continue
            a, ph = rng.standard_normal(), rng.uniform(0.0, 2 * math.pi)
            w += a * np.sin(kx * X + ky * Y + ph) / (kx * kx + ky * ky)
    return w


def random_spectrum(n, N, k0=10.0, seed=1, energy=0.5, return_umax=False):
    """Zero-mean random-spectrum vorticity on [0, 2pi]^2 (see module doc).
    With return_umax, also returns max over nodes of |u_x| + |u_y| of the
    exact initial velocity u = (-psi_y, psi_x)."""
    rng = np.random.default_rng(seed)
    K, c, cpsi = _spectrum_coefficients(k0, rng, energy)
    xi, _ = leggauss(n)
    h = 2 * math.pi / N
    x = ((np.arange(N)[:, None] + 0.5 + 0.5 * xi[None, :]) * h).ravel()
    kxs = np.arange(-K, K + 1)
    kys = np.arange(0, K + 1)
    Ex = np.exp(1j * np.outer(x, kxs))          # (N n, 2K+1)
    Ey = np.exp(1j * np.outer(x, kys))          # (N n, K+1)

    def field(coef):
        img = 2.0 * np.real(Ey @ coef.T @ Ex.T)  # [y, x]
        return np.ascontiguousarray(
            img.reshape(N, n, N, n).transpose(0, 2, 1, 3))

    omega = _remove_quadrature_mean(field(c), n, N, N)
    if not return_umax:
        return omega
    ux = field(-1j * kys[None, :] * cpsi)       # -psi_y
    uy = field(1j * kxs[:, None] * cpsi)        #  psi_x
    return omega, float(np.max(np.abs(ux) + np.abs(uy)))


def double_shear_layer(n, N, rho=math.pi / 15, delta=0.05):
    """omega = u_y - v_x for u = tanh((y - pi/2)/rho) (y <= pi),
    tanh((3pi/2 - y)/rho) (y > pi), v = delta sin x; returns
    (omega, max |u|+|v|)."""
    X, Y = node_coords(n, N, N)
    low = Y <= math.pi
    uy = np.where(low, 1.0 / np.cosh((Y - math.pi / 2) / rho) ** 2 / rho,
                  -1.0 / np.cosh((1.5 * math.pi - Y) / rho) ** 2 / rho)
    vx = delta * np.cos(X)
    omega = _remove_quadrature_mean(uy - vx, n, N, N)
    return omega, 1.0 + delta


def cfl_dt(n, N, umax, cfl=0.1, length=2 * math.pi):
    """dt = cfl * h / ((2n - 1) * umax), h = length / N."""
    return cfl * (length / N) / ((2 * n - 1) * umax)


LAMB_LAM_R = 3.83170597020751231561     # first zero of J1 (Sec. 6.2)


def lamb_dipole(n, N, L=1.0, U=1.0, R=0.1, centre=None):
    """Lamb dipole vorticity on the periodic box [0, L]^2 with N x N cells:
    omega = 2 lam U / J0(lam R) J1(lam r) cos(theta) for r < R, 0 outside
    (Sec. 6.2), sampled at the nodes."""
    from scipy.special import j0, j1
    X, Y = node_coords(n, N, N, 0.0, L, 0.0, L)
    cx, cy = (0.5 * L, 0.5 * L) if centre is None else centre
    dx, dy = X - cx, Y - cy
    r = np.hypot(dx, dy)
    lam = LAMB_LAM_R / R
    with np.errstate(invalid="ignore", divide="ignore"):
        cos_t = np.where(r > 0, dx / np.where(r > 0, r, 1.0), 0.0)
    w = 2.0 * lam * U / j0(lam * R) * j1(lam * r) * cos_t
    return np.where(r < R, w, 0.0)

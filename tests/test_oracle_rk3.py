"""Pins of the oracle's time stepping and invariants: the exact P = 1
Taylor-Green solution of the discrete system, invariant conservation
(Sec. 2 eq. quantities), the RK3 order of the enstrophy drift, and the
decay experiment's spatial order at D = 0 (Table 3)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1311_7477_amd import inputs as I


def test_p1_taylor_green_closed_form():
    # At P = 1 sin x sin y is an eigenvector of the 5-point Laplacian with
    # eigenvalue -lam; psi = omega/lam so J(psi, omega) vanishes to roundoff,
    # and each SSP-RK3 step multiplies omega by the stability polynomial
    # 1 + z + z^2/2 + z^3/6 at z = -D lam dt.
    N, D, dt, steps = 24, 0.05, 0.01, 10
    g = O.Grid2D(1, N, N)
    X, Y = g.node_coords()
    w0 = np.sin(X) * np.sin(Y)
    lam = 8.0 / g.hx ** 2 * math.sin(g.hx / 2) ** 2
    z = -D * lam * dt
    amp = (1 + z + z * z / 2 + z ** 3 / 6) ** steps
    w, t, hist = w0.copy(), 0.0, O.PsiHistory()
    for _ in range(steps):
        w, _ = O.rk3_step(g, w, t, dt, D, hist, rtol=1e-13)
        t += dt
    np.testing.assert_allclose(w, amp * w0, atol=1e-13)


def test_invariants_closed_form():
    # omega = 2 sin x sin y, psi = sin x sin y on [0, 2pi]^2:
    # V = 0, E = 1/2 int psi omega = pi^2, Omega = 1/2 int omega^2 = 2 pi^2
    g = O.Grid2D(4, 16, 16)
    X, Y = g.node_coords()
    V, E, Om = O.invariants(g, 2 * np.sin(X) * np.sin(Y), np.sin(X) * np.sin(Y))
    assert abs(V) < 1e-12
    assert abs(E - math.pi ** 2) < 1e-9
    assert abs(Om - 2 * math.pi ** 2) < 1e-9


def _drift(n, N, dt, steps, seed=3):
    g = O.Grid2D(n, N, N)
    w = I.random_spectrum(n, N, k0=2.0, seed=seed)
    psi0 = O.cg_poisson(g, w, rtol=1e-14).x
    V0, E0, Om0 = O.invariants(g, w, psi0)
    hist, t = O.PsiHistory(), 0.0
    for _ in range(steps):
        w, _ = O.rk3_step(g, w, t, dt, 0.0, hist, rtol=1e-14)
        t += dt
    psi = O.cg_poisson(g, w, rtol=1e-14).x
    V, E, Om = O.invariants(g, w, psi)
    return V, abs(E - E0) / E0, abs(Om - Om0) / Om0


def test_inviscid_invariants_drift_only_through_time_stepping():
    # V stays at roundoff; the enstrophy error shrinks like dt^3 for RK3
    # on the skew (conservative) semi-discretisation (Sec. 6.2 conclusion).
    V1, eE1, eO1 = _drift(3, 8, 0.08, 5)
    V2, eE2, eO2 = _drift(3, 8, 0.04, 10)
    assert abs(V1) < 1e-13 and abs(V2) < 1e-13
    ratio = eO1 / eO2
    assert 5.5 < ratio < 11.0, ratio
    assert eE2 < eE1


@pytest.mark.slow
@pytest.mark.parametrize("n", [2, 4])
def test_decay_spatial_order_d0(n):
    # Table 3, D = 0 periodic: order P (short integration, time error
    # negligible)
    errs = []
    for N in (8, 16, 32):
        g = O.Grid2D(n, N, N)
        w0 = I.decay_taylor_green(n, N)
        w, t, hist = w0.copy(), 0.0, O.PsiHistory()
        for _ in range(5):
            w, _ = O.rk3_step(g, w, t, 0.02, 0.0, hist, rtol=1e-13)
            t += 0.02
        errs.append(math.sqrt(O.inner(g, w - w0, w - w0)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(orders[-1] - n) < 0.35, orders


def test_psi_history_extrapolation_is_exact_for_linear_in_time_fields():
    # Sec. 6: the CG guess extrapolates the last two solutions linearly in
    # time, so a field psi(t) = A + t B must be reproduced exactly at any
    # later time (to rounding), whatever the spacing of the two solves.
    g = O.Grid2D(3, 6, 5)
    rng = np.random.default_rng(11)
    A, B = rng.standard_normal((2,) + g.shape)
    h = O.PsiHistory()
    assert h.guess(0.3) is None                   # no solve yet: zero guess
    h.push(0.1, A + 0.1 * B)
    np.testing.assert_array_equal(h.guess(0.7), A + 0.1 * B)   # one solve: itself
    h.push(0.25, A + 0.25 * B)
    for t in (0.25, 0.3, 0.125, 0.9):
        np.testing.assert_allclose(h.guess(t), A + t * B, rtol=0, atol=1e-13)
    # the oldest entry drops out: the guess now follows the newest pair
    h.push(0.5, A + 0.5 * B + 1.0)
    got = h.guess(0.75)
    want = (A + 0.5 * B + 1.0) + 1.0 * ((A + 0.5 * B + 1.0) - (A + 0.25 * B))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
    # two solves at the same time: the newest one alone (no division by 0)
    h.push(0.5, A)
    np.testing.assert_array_equal(h.guess(0.6), A)


@pytest.mark.parametrize("form,dE_zero,dOm_zero", [
    ("arakawa", True, True), ("pp", False, False), ("px", False, True),
    ("xp", True, False)])
def test_single_form_rhs_conservation_pattern(form, dE_zero, dOm_zero):
    # Table 2 pattern carried into the right-hand side at D = 0: with
    # R = -J(psi, omega), dE/dt = <psi, R> and dOmega/dt = <omega, R>.
    # The average J conserves both; J++ neither (Table 2: int fJ++ and
    # int gJ++ nonzero); J+x conserves Omega only (int gJ+x = 0); Jx+
    # conserves E only (int fJx+ = 0).  Also checks that rk3_step forwards
    # the form: one step with J++ changes Omega at O(dt), the average at
    # O(dt^3).
    n, N = 3, 10
    g = O.Grid2D(n, N, N)
    # k0 = 4 on 10 cells: under-resolved enough that the single forms'
    # truncation-level imbalance is far above rounding
    w = I.random_spectrum(n, N, k0=4.0, seed=4)
    psi = O.cg_poisson(g, w, rtol=1e-14).x
    R = O.rhs(g, w, psi, 0.0, form)
    scale = math.sqrt(O.inner(g, R, R))
    dE = O.inner(g, psi, R) / (scale * math.sqrt(O.inner(g, psi, psi)))
    dOm = O.inner(g, w, R) / (scale * math.sqrt(O.inner(g, w, w)))
    assert (abs(dE) < 1e-13) == dE_zero, dE
    assert (abs(dOm) < 1e-13) == dOm_zero, dOm
    if not (dE_zero and dOm_zero):
        assert max(abs(dE), abs(dOm)) > 1e-4
    Om0 = 0.5 * O.inner(g, w, w)
    rel = []
    for dt in (1e-3, 2.5e-4):
        w1, _ = O.rk3_step(g, w, 0.0, dt, 0.0, O.PsiHistory(), rtol=1e-14, form=form)
        rel.append(abs(0.5 * O.inner(g, w1, w1) - Om0) / Om0)
    ratio = rel[0] / rel[1]
    if dOm_zero:
        # only the RK3 error: the one-step change falls like dt^4
        assert ratio > 100, rel
    else:
        # the bracket itself changes Omega: like dt
        assert 3.0 < ratio < 5.0 and rel[0] > 1e-6, rel

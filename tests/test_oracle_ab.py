"""Pins of the oracle's K-step Adams-Bashforth stepper (Sec. 6; Sec. 6.2,
Table 4): the weights against exact polynomial quadrature, and the Lamb
dipole conservation errors against the printed Table 4.

Reading (stated in the design notes): the multistep method is started with
SSP-RK3 steps; the dipole is centred in the box with theta measured from the
x axis.  With it the printed K = 1, 2, 3 rows are reproduced to a few
percent.  The printed K = 4 rows are not: neither this start nor an exact
(fourth-order) start gives them (the paper's own orders there are
irregular); for K = 4 the pin is the observed order, 4."""
import math
import os
from fractions import Fraction

import pytest

import oracle as O
from paper_1311_7477_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_ab_weights_integrate_polynomials_exactly(K):
    # dt sum_j b_j p(t_n - j dt) = int_{t_n}^{t_n + dt} p  for deg p < K
    for m in range(K):
        exact = Fraction(1, m + 1)                 # t_n = 0, dt = 1: int_0^1 t^m
        got = sum(Fraction(b).limit_denominator(1000) * Fraction(-j) ** m
                  for j, b in enumerate(O.AB_COEFFS[K]))
        assert got == exact, (K, m, got)


def _table4():
    out = {}
    with open(os.path.join(GOLDEN, "table4_ab_lamb.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            K, steps, eo, ee = line.split()
            out[(int(K), int(steps))] = (float(eo), float(ee))
    return out


@pytest.fixture(scope="module")
def lamb_runs():
    n, N = 1, 200
    g = O.Grid2D(n, N, N, 0.0, 1.0, 0.0, 1.0)
    fd = O.FastDiagonalisation(g)
    w0 = I.lamb_dipole(n, N)
    p0 = O.pcg_poisson(g, w0, rtol=1e-14, precond=fd.apply).x
    V0, E0, Om0 = O.invariants(g, w0, p0)
    res = {}
    for K in (1, 2, 3, 4):
        for steps in (10, 20, 40, 80):
            dt = 0.01 / steps
            w, t, hist, rh = w0.copy(), 0.0, O.PsiHistory(), []
            for _ in range(steps):
                w, _ = O.ab_step(g, w, t, dt, 0.0, K, rh, hist, rtol=1e-14,
                                 precond=fd.apply)
                t += dt
            p = O.pcg_poisson(g, w, hist.guess(t), 1e-14, precond=fd.apply).x
            V, E, Om = O.invariants(g, w, p)
            res[(K, steps)] = (abs(V), abs((Om - Om0) / Om0), abs((E - E0) / E0))
    return res


def test_lamb_dipole_total_vorticity_vanishes(lamb_runs):
    assert max(v[0] for v in lamb_runs.values()) <= 1e-14


@pytest.mark.parametrize("K", [1, 2, 3])
def test_table4_printed_values(lamb_runs, K):
    printed = _table4()
    for steps in (10, 20, 40, 80):
        _, eo, ee = lamb_runs[(K, steps)]
        po, pe = printed[(K, steps)]
        assert abs(eo - po) <= 0.05 * po, (K, steps, eo, po)
        assert abs(ee - pe) <= 0.05 * pe, (K, steps, ee, pe)


@pytest.mark.parametrize("which", [1, 2])          # 1: eps_Omega, 2: eps_E
def test_table4_k4_order(lamb_runs, which):
    errs = [lamb_runs[(4, s)][which] for s in (10, 20, 40, 80)]
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(3.7 <= o <= 4.3 for o in orders), orders

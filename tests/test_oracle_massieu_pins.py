"""Pins of the oracle's Massieu-derivative estimators (Sec. 3, Eq. 1).

The estimators turn moment sums of U, dU/dV and d2U/dV2 into A^r_mn.  They
are pinned to an ensemble whose configurational integral is known exactly:
a few discrete configurations with analytic U_k(V) and weights g_k, for which
A^r(beta, rho) = -ln(sum_k g_k exp(-beta U_k(N / rho))) / N is differentiated
symbolically (sympy).  Feeding the exact Boltzmann-weighted moments of the
same ensemble into the estimators must give those derivatives; a dropped
term, wrong sign or wrong operator order in any of the eight fails it.
"""
import numpy as np
import pytest

from oracle import massieu as M

sympy = pytest.importorskip("sympy")


def toy_ensemble():
    # U_k(V) = a V^-4 + b V^-2 + c V + d, five configurations with weights g
    a = [3.0, -1.5, 0.7, 2.2, -0.4]
    b = [-2.0, 1.1, -0.3, 0.5, 1.7]
    c = [0.05, -0.02, 0.08, -0.06, 0.01]
    d = [-1.0, 0.4, 0.9, -0.2, 0.3]
    g = [1.0, 2.0, 0.5, 1.5, 3.0]
    return a, b, c, d, g


def exact_derivatives(N, beta0, rho0):
    a, b, c, d, g = toy_ensemble()
    beta, rho = sympy.symbols("beta rho", positive=True)
    V = N / rho
    Z = sum(gk * sympy.exp(-beta * (ak * V ** -4 + bk * V ** -2 + ck * V + dk))
            for ak, bk, ck, dk, gk in zip(a, b, c, d, g))
    A = -sympy.log(Z) / N
    out = {}
    for key in M.A_ORDER:
        m, n = int(key[0]), int(key[1])
        expr = A
        if m:
            expr = sympy.diff(expr, beta, m)
        if n:
            expr = sympy.diff(expr, rho, n)
        out[key] = float((beta ** m * rho ** n * expr).subs({beta: beta0, rho: rho0}).evalf(30))
    return out


def exact_moments(N, beta0, rho0, u0, samples=1000.0):
    a, b, c, d, g = (np.array(x) for x in toy_ensemble())
    V = N / rho0
    U = a * V ** -4 + b * V ** -2 + c * V + d
    Y = -4 * a * V ** -5 - 2 * b * V ** -3 + c
    Zv = 20 * a * V ** -6 + 6 * b * V ** -4
    w = g * np.exp(-beta0 * (U - U.min()))
    w /= w.sum()
    X = U - u0
    f = [np.ones_like(X), X, X * X, X ** 3, Y, X * Y, X * X * Y, Y * Y, X * Y * Y, Zv, X * Zv]
    return np.array([samples * (w * q).sum() for q in f]), V


@pytest.mark.parametrize("beta0,rho0", [(0.7, 0.4), (1.6, 0.9)])
def test_estimators_reproduce_exact_derivatives_of_a_known_ensemble(beta0, rho0):
    N = 3.0
    exact = exact_derivatives(N, beta0, rho0)
    for u0 in (0.0, -2.5):                      # the shift must not matter
        mom, V = exact_moments(N, beta0, rho0, u0)
        est = M.residual_derivatives(mom, u0, 1.0 / beta0, V, N)
        for k in M.A_ORDER:
            assert est[k] == pytest.approx(exact[k], rel=1e-8, abs=1e-10), (k, est[k], exact[k])


def test_first_three_reduce_to_the_textbook_fluctuation_formulas():
    # A^r_10 = beta <U>/N, A^r_01 = -beta V <U_V>/N, A^r_20 = -beta^2 var(U)/N
    rng = np.random.default_rng(0)
    U = rng.normal(-50.0, 3.0, 4000)
    Y = rng.normal(-2.0, 0.5, 4000)
    Zv = rng.normal(1.0, 0.2, 4000)
    u0 = -50.0
    X = U - u0
    mom = np.array([len(U), X.sum(), (X * X).sum(), (X ** 3).sum(), Y.sum(), (X * Y).sum(), (X * X * Y).sum(),
                    (Y * Y).sum(), (X * Y * Y).sum(), Zv.sum(), (X * Zv).sum()])
    T, V, N = 1.7, 900.0, 500
    est = M.residual_derivatives(mom, u0, T, V, N)
    assert est["10"] == pytest.approx(U.mean() / T / N, rel=1e-12)
    assert est["01"] == pytest.approx(-V * Y.mean() / T / N, rel=1e-12)
    assert est["20"] == pytest.approx(-U.var() / T ** 2 / N, rel=1e-9)


def test_ideal_gas_has_no_residual_part_and_textbook_properties():
    # U = 0 in every sample: X = -u0, Y = Z = 0
    u0 = 3.0
    n = 200.0
    mom = np.array([n, -u0 * n, u0 * u0 * n, -u0 ** 3 * n, 0, 0, 0, 0, 0, 0, 0], dtype=float)
    est = M.residual_derivatives(mom, u0, 2.0, 1000.0, 100)
    for k in M.A_ORDER:
        assert est[k] == pytest.approx(0.0, abs=1e-12), k
    for dof, gamma in ((3, 5.0 / 3.0), (5, 7.0 / 5.0), (6, 4.0 / 3.0)):
        p = M.properties(est, dof)
        assert p["Z"] == 1.0 and p["dpdrho_kT"] == 1.0 and p["rho_kT_kappaT"] == 1.0
        assert p["cv_k"] == dof / 2.0 and p["cp_k"] == dof / 2.0 + 1.0
        assert p["w2_m_kT"] == pytest.approx(gamma, rel=1e-15)
        assert p["u_kT"] == dof / 2.0

"""Pin of the oracle's second volume derivative d2U/dV2 and of the moment
slots built from it (Z and X*Z of the Lustig sums; Sec. 3, Eq. 1 and the
paragraph after it, where dU/dV and d2U/dV2 of the potential are the sampled
quantities).

The reference is computed without the oracle's conversion formulas: the
total energy is evaluated at scaled states and differentiated numerically.
  * Explicit pairs: molecular scaling (centres and box scaled by s, bodies
    rigid, rc fixed), energy from the oracle's pair sums with the LJ tail off,
    central differences in s.  The set of interacting pairs must not change
    across the stencil (asserted through the pair counter).
  * LJ tail: the zeroth-order reading of the long-range correction (every LJ
    site pair of two molecules beyond rc treated as a uniform fluid at the
    centre distance, g = 1): the pairs beyond rc keep their identity while
    their distances scale, T(s) = (2 pi / V) sum_AB N_A N_B sum_ab
    INT_rc^inf r^2 u_ab(s r) dr, integrated by quadrature and differentiated
    in s by central differences.
With V = V0 s^3, d2E/dV2 at s = 1 is (E'' - 2 E') / (9 V0^2).  The oracle's
sampled Z must equal it; three plausible mistakes in the conversion (the
sign of the 2 E' term, 3V for 9V^2, the tail's second derivative left out)
are each shown to miss it by far more than the tolerance.

The moments are taken from the oracle's MD driver at a state it does not
move: a time step of 1e-30 leaves every centre and quaternion unchanged to
double precision, so each sampled step sees the initial configuration.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from models import small_system
from paper_1507_07548_amd import inputs as I

U_LJ, U_ELEC, U_RECIP, U_CONST, U_LRC, VIR, US, USS, US_LRC, USS_LRC, NPAIR, NSITE = range(12)
M_N, M_X, M_XX, M_XXX, M_Y, M_XY, M_XXY, M_YY, M_XYY, M_Z, M_XZ = range(11)


def systems():
    yield "2cljq_rf", small_system([I.two_center_lj_quadrupole()], 125, 5.93, 2.4, seed=21,
                                   elec=I.ELEC_RF, lj_lrc=1, jitter=0.2)
    yield "stockmayer_rf", small_system([I.stockmayer()], 125, 6.2, 2.5, seed=22, elec=I.ELEC_RF,
                                        eps_rf=30.0, lj_lrc=1, jitter=0.2)
    yield "lj_mixture", small_system([I.one_center_lj(), I.one_center_lj(eps=0.7, sigma=1.15)], 100,
                                     5.6, 2.2, seed=23, lj_lrc=1, jitter=0.2)


SYSTEMS = list(systems())


def explicit_energy(system, s):
    """Explicit pair energy (no LJ tail) after scaling centres and box by s."""
    x = system.copy()
    x.com = system.com * s
    x.params.box = system.params.box * s
    x.params.lj_lrc = 0
    f, t, sums = oracle.evaluate(x)
    return oracle.total_energy(sums), sums[NPAIR]


def lj_site_sets(system):
    """(count per species, LJ sites (sigma, eps) per species)."""
    counts = np.bincount(np.asarray(system.species_idx), minlength=len(system.species))
    sites = [[(st.sigma, st.eps) for st in sp.sites if st.kind == I.LJ] for sp in system.species]
    return counts, sites


def tail_energy(system, s):
    """Zeroth-order LJ tail of the pairs beyond rc, their distances scaled by
    s, by quadrature (unscaled volume and cut-off: the pair set is fixed)."""
    counts, sites = lj_site_sets(system)
    rc, V = system.params.rc, system.params.box ** 3
    total = 0.0
    for A, na in enumerate(counts):
        for B, nb in enumerate(counts):
            for sa, ea in sites[A]:
                for sb, eb in sites[B]:
                    sig, eps = 0.5 * (sa + sb), math.sqrt(ea * eb)

                    # r = rc / x maps (rc, inf) onto (0, 1]: dr = -rc / x^2 dx
                    def f(x):
                        r = rc / x
                        y = sig / (s * r)
                        return r * r * 4.0 * eps * (y ** 12 - y ** 6) * rc / (x * x)

                    val, _ = integrate.quad(f, 0.0, 1.0, epsabs=0.0, epsrel=1e-13, limit=200)
                    total += na * nb * val
    return 2.0 * math.pi / V * total


def derivatives(fun, h):
    """First and second derivative at s = 1 by central differences with
    Richardson extrapolation over steps h and 2h (error O(h^4))."""
    e0 = fun(1.0)
    ep, em = fun(1.0 + h), fun(1.0 - h)
    ep2, em2 = fun(1.0 + 2 * h), fun(1.0 - 2 * h)
    d1 = (8 * (ep - em) - (ep2 - em2)) / (12 * h)
    d2 = (16 * (ep + em) - (ep2 + em2) - 30 * e0) / (12 * h * h)
    return d1, d2


def fd_d2u_dv2(system):
    pairs = []

    def expl(s):
        u, npair = explicit_energy(system, s)
        pairs.append(npair)
        return u

    d1e, d2e = derivatives(expl, 2e-5)
    assert len(set(pairs)) == 1, "a pair crossed the cut-off inside the stencil"
    d1t, d2t = derivatives(lambda s: tail_energy(system, s), 1e-3)
    V = system.params.box ** 3
    return (d2e + d2t - 2.0 * (d1e + d1t)) / (9.0 * V * V), (d1e, d2e, d1t, d2t)


def sampled_moments(system, u0, n_samples=2):
    x = system.copy()
    x.md = I.MDSettings(integrator=I.GEAR, dt=1e-30, temperature=0.0, n_steps=n_samples,
                        sample_every=1, u0=u0)
    return oracle.md(x, want_log=False)["moments"]


@pytest.mark.parametrize("name,system", SYSTEMS, ids=[n for n, _ in SYSTEMS])
def test_sampled_d2u_dv2_matches_scaled_energy(name, system):
    z_ref, (d1e, d2e, d1t, d2t) = fd_d2u_dv2(system)
    _, _, sums = oracle.evaluate(system)
    u = oracle.total_energy(sums)
    u0 = u + 3.25          # X = U - u0 a small number of either sign is fine
    m = sampled_moments(system, u0)
    assert m[M_N] == 2
    z = m[M_Z] / 2
    tol = 2e-7            # measured agreement 2-4e-8 (stencil truncation and rounding)
    assert z == pytest.approx(z_ref, rel=tol), (z, z_ref)
    # the tail's share is well above the tolerance, so dropping it would show
    V = system.params.box ** 3
    assert abs(d2t - 2 * d1t) / (9 * V * V) > 100 * tol * abs(z_ref)
    # X and X*Z of the same samples
    x = u - u0
    assert m[M_X] / 2 == pytest.approx(x, rel=1e-12)
    assert m[M_XZ] == pytest.approx(2 * x * z, rel=1e-12)
    # each planted conversion mistake misses the reference by far more than tol
    us = sums[US] + sums[US_LRC]
    uss = sums[USS] + sums[USS_LRC]
    planted = {
        "+2 U_s": (uss + 2 * us) / (9 * V * V),
        "3V": (uss - 2 * us) / (3 * V),
        "no U_ss,lrc": (sums[USS] - 2 * us) / (9 * V * V),
    }
    for label, zw in planted.items():
        assert abs(zw - z_ref) > 20 * tol * abs(z_ref), label


@pytest.mark.parametrize("name,system", SYSTEMS[:1], ids=[n for n, _ in SYSTEMS[:1]])
def test_first_volume_derivative_matches_scaled_energy(name, system):
    """The Y slot (dU/dV = (U_s + U_s,lrc) / (3V)) against the same stencil."""
    _, (d1e, d2e, d1t, d2t) = fd_d2u_dv2(system)
    V = system.params.box ** 3
    y_ref = (d1e + d1t) / (3 * V)
    _, _, sums = oracle.evaluate(system)
    u0 = oracle.total_energy(sums)
    m = sampled_moments(system, u0)
    assert m[M_Y] / 2 == pytest.approx(y_ref, rel=1e-7)
    assert abs(d1t) / (3 * V) > 1e-4 * abs(y_ref)

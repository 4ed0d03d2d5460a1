"""Pins of the oracle's integrators and samplers: energy conservation, time
reversibility, exact thermostat targets, RDF shell counts of a perfect FCC
lattice and of an ideal gas (Sec. 5, Eq. 2), autocorrelation bookkeeping
(Sec. 4 extended time step; Sec. 5, Eqs. 3-4) and the Lustig moments of an
ideal gas and the virial route to A01 (Sec. 3, Eq. 1)."""
import math

import numpy as np
import pytest

import oracle
from models import ionic_pair_species, small_system
from paper_1507_07548_amd import inputs as I

U_LJ, U_ELEC, U_RECIP, U_CONST, U_LRC, VIR, US, USS, US_LRC, USS_LRC, NPAIR, NSITE = range(12)


def melted(system, steps):
    """Isokinetic run from the lattice start: a perfect FCC lattice puts whole
    shells next to rc, and a truncated potential then jumps as they cross."""
    s = system.copy()
    s.md.n_steps = steps
    if s.md.temperature <= 0:
        s.md.temperature = 1.5
    out = oracle.md(s)["state"]
    out.md.temperature = 0.0
    return out


def test_velocity_verlet_nve_energy_drift():
    s = melted(I.lj_fluid(), 200)              # 500 LJ, rho 0.7, T 1.5, rc 4, dt 0.002
    s.md.n_steps = 100
    out = oracle.md(s)
    e = out["log"][:, 0] + out["log"][:, 1]
    # truncated (unshifted) potential: each pair crossing rc jumps by |u(rc)| ~ 1e-3
    assert np.abs(e - e[0]).max() / s.n < 1e-3


def test_velocity_verlet_time_reversible():
    s = I.lj_fluid(n_steps=50)
    fwd = oracle.md(s)["state"]
    back = fwd.copy()
    back.vel = -fwd.vel
    ret = oracle.md(back)["state"]
    d = ret.com - s.com
    d -= s.params.box * np.rint(d / s.params.box)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-ret.vel, s.vel, atol=1e-9)


def test_gear_quaternion_nve_conserves_energy_and_norms():
    base = melted(I.quadrupolar_fluid(n=256, density=0.3, temperature=2.0, dt=0.001), 400)
    drift = {}
    for dt in (0.0005, 0.00025):
        s = base.copy()
        s.md.dt, s.md.n_steps = dt, int(round(0.05 / dt))
        out = oracle.md(s)
        log = out["log"]
        e = log[:, 0] + log[:, 1] + log[:, 2]
        drift[dt] = np.abs(e[1:] - e[1]).max() / s.n
        q = out["state"].quat
        np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-14)
        # linear molecules: no spin about the symmetry axis
        assert np.abs(out["state"].omega[:, 2]).max() == 0.0
    # converges to the cut-off crossing floor (~2.5e-4 per molecule here)
    assert drift[0.00025] < 1e-3 and drift[0.0005] < 2e-3


def test_isokinetic_thermostat_hits_target_exactly():
    s = I.quadrupolar_fluid(n=108, density=0.5, temperature=1.7, n_steps=20)
    out = oracle.md(s)
    log = out["log"]
    f_tr, f_rot = 3 * s.n - 3, 2 * s.n          # linear molecules: 2 rotational dof
    np.testing.assert_allclose(2 * log[1:, 1] / f_tr, 1.7, rtol=1e-13)
    np.testing.assert_allclose(2 * log[1:, 2] / f_rot, 1.7, rtol=1e-13)
    v = out["state"].vel
    assert np.abs(v.sum(0)).max() < 1e-10       # no net momentum appears


def lattice_rdf(cells=4, density=1.0, bins=200):
    n = 4 * cells ** 3
    s = I.lj_fluid(n=n, density=density, temperature=1.0, rc=0.49 * (n / density) ** (1 / 3), n_steps=1)
    s.vel[:] = 0.0
    s.md.dt = 1e-12
    s.md.rdf_every, s.md.rdf_bins, s.md.rdf_rmax = 1, bins, 0.45 * s.params.box
    return s, oracle.md(s)["rdf"][0]


def test_rdf_fcc_lattice_shell_counts():
    s, h = lattice_rdf()
    a = s.params.box / 4
    dr = s.md.rdf_rmax / s.md.rdf_bins
    # unordered pairs per shell = N * coordination / 2; shells at a/sqrt2, a, a sqrt(3/2)
    for rad, coord in [(a / math.sqrt(2), 12), (a, 6), (a * math.sqrt(1.5), 24), (a * math.sqrt(2), 12)]:
        b = int(rad / dr)
        assert h[b - 1:b + 2].sum() == s.n * coord / 2


def test_rdf_ideal_gas_is_flat():
    rng = np.random.default_rng(4)
    n, box, bins = 2000, 20.0, 40
    s = I.lj_fluid(n=n, density=n / box ** 3, temperature=1.0, rc=9.0, n_steps=1)
    s.species = [I.one_center_lj(eps=0.0)]     # non-interacting points
    s.com = rng.random((n, 3)) * box
    s.vel[:] = 0.0
    s.md.rdf_every, s.md.rdf_bins, s.md.rdf_rmax = 1, bins, 9.0
    h = oracle.md(s)["rdf"][0]
    r = np.linspace(0, 9.0, bins + 1)
    shell = 4 * math.pi / 3 * (r[1:] ** 3 - r[:-1] ** 3)
    g = h / (n * (n - 1) / 2 / box ** 3 * shell)
    sigma = 1 / np.sqrt(np.maximum(h, 1))
    assert np.all(np.abs(g[5:] - 1) < 5 * sigma[5:] + 1e-3)


def test_acf_bookkeeping_with_constant_velocities():
    n = 64
    sp = ionic_pair_species()[:2]
    sp = [I.Species(x.name, [I.Site(I.LJ, (0, 0, 0), sigma=1.0, eps=0.0), x.sites[1]], 1.0, (0, 0, 0))
          for x in sp]
    for x in sp:                                # switch off the charges' interactions
        x.sites[1] = I.Site(I.CHARGE, (0, 0, 0), mag=x.sites[1].mag)
    s = small_system(sp, n, 12.0, 5.0, seed=3, elec=I.ELEC_NONE)
    s.species = [I.Species(x.name, [x.sites[0]], 1.0, (0, 0, 0)) for x in sp]  # no charges act
    rng = np.random.default_rng(1)
    s.vel = rng.normal(size=(n, 3))
    s.md = I.MDSettings(integrator=I.VV, dt=0.001, n_steps=100, acf_every=5, acf_origin_every=20,
                        acf_nlag=10)
    out = oracle.md(s)
    cv = (s.vel ** 2).sum() / n
    # samples at t = 0,5,...,100; origins every 20 steps; lag l (l < 10) gets
    # one contribution from each origin t0 <= 100 - 5 l
    cnt = np.array([sum(1 for t0 in range(0, 101, 20) if t0 + 5 * l <= 100) for l in range(10)])
    np.testing.assert_array_equal(out["acf_cnt"], cnt)
    np.testing.assert_allclose(out["acf_v"], cv * cnt, rtol=1e-12)
    # the current of non-ions is zero: these molecules carry no charge site
    np.testing.assert_allclose(out["acf_j"], 0.0)


def test_electric_current_acf_constant_velocities():
    n = 32
    sp = [I.Species("A", [I.Site(I.LJ, (0, 0, 0), sigma=1.0, eps=0.0), I.Site(I.CHARGE, (0, 0, 0), mag=-1.0)], 1.0, (0, 0, 0)),
          I.Species("C", [I.Site(I.LJ, (0, 0, 0), sigma=1.0, eps=0.0), I.Site(I.CHARGE, (0, 0, 0), mag=2.0)], 1.0, (0, 0, 0))]
    s = small_system(sp, n, 12.0, 5.0, seed=4, elec=I.ELEC_NONE)
    s.species = [I.Species(x.name, x.sites, x.mass, x.inertia) for x in sp]
    s.params.coulomb_k = 0.0                    # charges present, Coulomb switched off
    rng = np.random.default_rng(2)
    s.vel = rng.normal(size=(n, 3))
    s.md = I.MDSettings(integrator=I.VV, dt=0.001, n_steps=40, acf_every=4, acf_origin_every=8, acf_nlag=5)
    out = oracle.md(s)
    q = np.array([-1.0, 2.0])[s.species_idx]
    j = (q[:, None] * s.vel).sum(0)             # Sec. 5, Eq. 4
    np.testing.assert_allclose(out["acf_j"], (j @ j) * out["acf_cnt"], rtol=1e-12)


def test_lustig_moments_ideal_gas_vanish():
    s = small_system([I.one_center_lj(eps=0.0)], 64, 10.0, 4.5, seed=5, lj_lrc=1)
    s.vel = np.random.default_rng(3).normal(size=(64, 3))
    s.md = I.MDSettings(integrator=I.VV, dt=0.001, n_steps=10, sample_every=1)
    m = oracle.md(s)["moments"]
    assert m[0] == 10
    np.testing.assert_allclose(m[1:], 0.0, atol=0.0)


def test_lustig_moments_match_the_per_step_sums():
    """Each moment slot equals the sum over sampled steps of the product it
    names, with X = U - u0 and Y = dU/dV = (U_s + U_s,lrc)/(3V) taken from the
    logged energy and virial (U_s = -W for the explicit pairs); and the volume
    route to Y is the virial route to the excess pressure."""
    s = I.quadrupolar_fluid(n=64, density=0.5, temperature=2.0, n_steps=6, sample_every=2)
    s.md.u0 = -300.0
    out = oracle.md(s)
    m, log = out["moments"], out["log"]
    V = s.params.box ** 3
    _, _, su = oracle.evaluate(s)
    us_lrc = su[US_LRC]                               # fixed N, V and rc
    steps = [2, 4, 6]
    X = log[steps, 0] - s.md.u0
    Y = (-log[steps, 3] + us_lrc) / (3 * V)
    # the logged dU/ds is the same quantity as -W plus the tail
    np.testing.assert_allclose(log[steps, 4], -log[steps, 3] + us_lrc, rtol=1e-12)
    # Z = d2U/dV2 of each sampled step from its logged s-derivatives; the value
    # of this conversion is pinned against scaled energies in
    # test_oracle_volume_moment_pins.py
    Z = (log[steps, 5] - 2 * log[steps, 4]) / (9 * V * V)
    ref = [3, X.sum(), (X * X).sum(), (X ** 3).sum(), Y.sum(), (X * Y).sum(), (X * X * Y).sum(),
           (Y * Y).sum(), (X * Y * Y).sum(), Z.sum(), (X * Z).sum()]
    np.testing.assert_allclose(m, ref, rtol=1e-10)
    # virial route: dU/dV = -(W/(3V) + p_lrc)
    y0 = (su[US] + su[US_LRC]) / (3 * V)
    assert y0 == pytest.approx(-(su[VIR] / (3 * V) - su[US_LRC] / (3 * V)), rel=1e-12)


def test_moment_sampling_with_ewald_is_refused():
    """The oracle, like the library, offers no Lustig moments with Ewald
    summation (Sec. 4): d2U/dV2 has no reciprocal part."""
    s = small_system(ionic_pair_species(), 16, 4.0, 1.9, seed=2, elec=I.ELEC_EWALD, alpha=1.5, kmax2=10)
    s.md = I.MDSettings(integrator=I.GEAR, dt=0.001, n_steps=2, sample_every=1)
    with pytest.raises(ValueError):
        oracle.md(s)
    s.md.sample_every = 0
    assert oracle.md(s)["log"].shape == (3, oracle.LOG_COLS)

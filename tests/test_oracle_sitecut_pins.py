"""Pins of the oracle's site-site cut-off mode (Sec. 3: LJ long-range
correction in the site-site or centre-of-mass cut-off mode): LJ site pairs
interact when their own distance is inside the cut-off, electrostatic site
pairs when the molecule centres are.  Closed forms at special geometries
(two-centre molecules side by side and end to end, on either side of the
cut-off), electrostatics that follow the centres, finite differences of the
energy (forces, torques, volume derivatives) and argument validation."""
import math

import numpy as np
import pytest

import oracle
from models import offset_multipoles, small_system, two_molecules
from paper_1507_07548_amd import inputs as I
from test_oracle_pins import NPAIR, NSITE, U_ELEC, U_LJ, US, USS, Z_TO_X, axis_quat, lj, qmul, total


def two_centre(l=1.0):
    h = 0.5 * l
    return I.Species("2CLJ", [I.Site(I.LJ, (0.0, 0.0, h), sigma=1.0, eps=1.0),
                             I.Site(I.LJ, (0.0, 0.0, -h), sigma=1.0, eps=1.0)], 1.0,
                     (0.25 * l * l, 0.25 * l * l, 0.0))


@pytest.mark.parametrize("mode", [I.CUT_SITE, I.CUT_COM])
def test_side_by_side_two_centre_molecules(mode):
    # axes along z, centres 2 apart on x: same-height site pairs at 2,
    # crossed ones at sqrt(5) = 2.236; rc = 2.1 lies between them
    sp = two_centre()
    s = two_molecules(sp, sp, [2.0, 0, 0], rc=2.1, cutoff_mode=mode)
    _, _, sums = oracle.forces(s)
    if mode == I.CUT_SITE:
        assert sums[U_LJ] == pytest.approx(2 * lj(2.0), rel=1e-14)
        assert (sums[NPAIR], sums[NSITE]) == (1, 2)
    else:
        assert sums[U_LJ] == pytest.approx(2 * lj(2.0) + 2 * lj(math.sqrt(5.0)), rel=1e-14)
        assert (sums[NPAIR], sums[NSITE]) == (1, 4)
    # 2.15 apart: every site pair beyond rc, although the centres are within
    # reach of the site offsets (rc + 2 x 0.5): nothing interacts or counts
    s = two_molecules(sp, sp, [2.15, 0, 0], rc=2.1, cutoff_mode=mode)
    _, _, sums = oracle.forces(s)
    assert (sums[U_LJ], sums[NPAIR], sums[NSITE]) == (0.0, 0.0, 0.0)


@pytest.mark.parametrize("mode", [I.CUT_SITE, I.CUT_COM])
def test_end_to_end_two_centre_molecules(mode):
    # axes along x, centres 2.6 apart on x: site pairs at 1.6, 2.6, 2.6, 3.6;
    # rc = 2.0 is below the centre distance
    sp = two_centre()
    s = two_molecules(sp, sp, [2.6, 0, 0], qa=Z_TO_X, qb=Z_TO_X, rc=2.0, cutoff_mode=mode)
    f, _, sums = oracle.forces(s)
    if mode == I.CUT_SITE:
        assert sums[U_LJ] == pytest.approx(lj(1.6), rel=1e-14)
        assert (sums[NPAIR], sums[NSITE]) == (1, 1)
        # the one pair acts along x: F_x = -u'(1.6)
        du = 4 * (-12 * 1.6 ** -13 + 6 * 1.6 ** -7)
        assert f[0, 0] == pytest.approx(-du, rel=1e-13)
    else:
        assert sums[U_LJ] == 0.0 and sums[NPAIR] == 0


def test_electrostatics_follow_the_centres():
    sp = offset_multipoles()
    rng = np.random.default_rng(3)
    q = [rng.normal(size=4), rng.normal(size=4)]
    q = [x / np.linalg.norm(x) for x in q]
    for dist, inside in ((2.3, False), (1.8, True)):
        s_site = two_molecules(sp, sp, [dist, 0.3, 0.2], qa=q[0], qb=q[1], rc=2.0, elec=I.ELEC_RF,
                               eps_rf=10.0, cutoff_mode=I.CUT_SITE)
        s_com = two_molecules(sp, sp, [dist, 0.3, 0.2], qa=q[0], qb=q[1], rc=2.0, elec=I.ELEC_RF,
                              eps_rf=10.0, cutoff_mode=I.CUT_COM)
        _, _, ss = oracle.forces(s_site)
        _, _, sc = oracle.forces(s_com)
        if inside:
            assert ss[U_ELEC] == sc[U_ELEC] != 0.0
        else:
            assert ss[U_ELEC] == 0.0


def site_systems():
    yield "offset_none", small_system([offset_multipoles()], 27, 6.4, 2.2, seed=1, lj_lrc=0,
                                      cutoff_mode=I.CUT_SITE)
    yield "offset_rf", small_system([offset_multipoles(), I.stockmayer()], 27, 6.4, 2.2, seed=2,
                                    elec=I.ELEC_RF, eps_rf=20.0, lj_lrc=0, cutoff_mode=I.CUT_SITE)
    yield "2cljq", small_system([I.two_center_lj_quadrupole()], 27, 5.0, 2.1, seed=3, elec=I.ELEC_RF,
                                lj_lrc=0, cutoff_mode=I.CUT_SITE)


SITE_SYSTEMS = list(site_systems())


@pytest.mark.parametrize("name,system", SITE_SYSTEMS, ids=[n for n, _ in SITE_SYSTEMS])
def test_site_mode_forces_and_torques_match_energy_gradient(name, system):
    u0, f, t, s = total(system)
    h = 1e-6
    scale = np.sqrt((f ** 2).sum(1).mean())
    tscale = np.sqrt((t ** 2).sum(1).mean())
    for i in range(0, system.n, 2):
        for k in range(3):
            up, dn = system.copy(), system.copy()
            up.com[i, k] += h
            dn.com[i, k] -= h
            eu, _, _, su = total(up)
            ed, _, _, sd = total(dn)
            assert su[NSITE] == sd[NSITE] == s[NSITE]     # no site pair crosses the cut-off
            assert (eu - ed) / (2 * h) == pytest.approx(-f[i, k], abs=2e-6 * scale)
            e = np.zeros(3)
            e[k] = 1
            up, dn = system.copy(), system.copy()
            up.quat[i] = qmul(axis_quat(e, h), system.quat[i])
            dn.quat[i] = qmul(axis_quat(e, -h), system.quat[i])
            eu, _, _, su = total(up)
            ed, _, _, sd = total(dn)
            assert su[NSITE] == sd[NSITE] == s[NSITE]
            assert (eu - ed) / (2 * h) == pytest.approx(-t[i, k], abs=2e-6 * max(tscale, scale))


@pytest.mark.parametrize("name,system", SITE_SYSTEMS, ids=[n for n, _ in SITE_SYSTEMS])
def test_site_mode_volume_derivatives_match_scaling(name, system):
    def at(sc):
        x = system.copy()
        x.com = system.com * sc
        x.params.box = system.params.box * sc
        return total(x)

    u0, _, _, s0 = at(1.0)
    h = 2e-5
    (up, _, _, sp), (dn, _, _, sd) = at(1 + h), at(1 - h)
    assert sp[NSITE] == sd[NSITE] == s0[NSITE]
    assert (up - dn) / (2 * h) == pytest.approx(s0[US], rel=1e-7, abs=1e-7 * abs(u0))
    assert (up - 2 * u0 + dn) / (h * h) == pytest.approx(s0[USS], rel=1e-4, abs=1e-5 * abs(s0[USS]))


def test_site_mode_needs_room_for_the_site_offsets():
    sp = two_centre(l=1.0)                       # LJ sites 0.5 from the centre
    ok = two_molecules(sp, sp, [2.0, 0, 0], box=8.0, rc=2.9, cutoff_mode=I.CUT_SITE)
    oracle.forces(ok)                            # 2.9 + 2 x 0.5 < 4
    bad = two_molecules(sp, sp, [2.0, 0, 0], box=8.0, rc=3.1, cutoff_mode=I.CUT_SITE)
    with pytest.raises(ValueError):
        oracle.forces(bad)

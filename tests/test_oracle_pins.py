"""Pins of the FP64 CPU oracle against what the mathematics fixes.

Every check compares the oracle with something other than itself: closed
forms at special geometries, textbook constants (NaCl Madelung constant),
explicit-charge limits of the point multipoles, central finite differences
of the energy, brute force over periodic images, numerical quadrature of the
LJ tail, and conservation laws.  The oracle runs on the CPU only.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from models import ionic_pair_species, offset_multipoles, small_system, two_molecules, unit
from paper_1507_07548_amd import inputs as I

U_LJ, U_ELEC, U_RECIP, U_CONST, U_LRC, VIR, US, USS, US_LRC, USS_LRC, NPAIR, NSITE = range(12)


def total(system):
    f, t, s = oracle.evaluate(system)
    return oracle.total_energy(s), f, t, s


def axis_quat(axis, angle):
    a = np.asarray(axis, dtype=float)
    a = a / np.linalg.norm(a)
    return np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * a])


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


Z_TO_X = axis_quat([0, 1, 0], math.pi / 2)   # body z -> lab x
Z_TO_Y = axis_quat([1, 0, 0], -math.pi / 2)  # body z -> lab y


def lj(r, eps=1.0, sig=1.0):
    return 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6)


# ---------------------------------------------------------------------------
# Lennard-Jones closed forms (two-site geometries, quaternion convention)
# ---------------------------------------------------------------------------
def test_lj_one_site_pair_closed_form():
    sp = I.one_center_lj(eps=1.3, sigma=1.1)
    for r in [0.95, 1.1, 1.5, 2.7]:
        s = two_molecules(sp, sp, [0.6 * r, 0.8 * r, 0.0])
        f, t, sums = oracle.forces(s)
        x = 1.1 / r
        assert sums[U_LJ] == pytest.approx(4 * 1.3 * (x ** 12 - x ** 6), rel=1e-14)
        # force = -dU/dr along the centre line, checked against the derivative
        dudr = (lj(r * (1 + 1e-7), 1.3, 1.1) - lj(r * (1 - 1e-7), 1.3, 1.1)) / (2e-7 * r)
        np.testing.assert_allclose(f[0], -dudr * np.array([0.6, 0.8, 0.0]), rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(f[1], -f[0], rtol=0, atol=1e-15 * abs(dudr))
        assert sums[NPAIR] == 1 and sums[NSITE] == 1


def test_two_centre_lj_orientations_closed_form():
    sp = I.two_center_lj_quadrupole(elongation=0.3, q2=0.0)
    h, r = 0.15, 1.4
    cases = {
        # both axes along z, centres separated along x: parallel side by side
        "side": (None, None, 2 * lj(r) + 2 * lj(math.hypot(r, 2 * h))),
        # both axes along x (rotated): collinear end to end
        "end": (Z_TO_X, Z_TO_X, 2 * lj(r) + lj(r - 2 * h) + lj(r + 2 * h)),
        # a along x, b along z: T shape
        "tee": (Z_TO_X, None, 2 * lj(math.hypot(r + h, h)) + 2 * lj(math.hypot(r - h, h))),
        # a along y, b along z: crossed
        "cross": (Z_TO_Y, None, 4 * lj(math.sqrt(r * r + 2 * h * h))),
    }
    for name, (qa, qb, u_ref) in cases.items():
        s = two_molecules(sp, sp, [r, 0, 0], qa=qa, qb=qb)
        _, _, sums = oracle.forces(s)
        assert sums[U_LJ] == pytest.approx(u_ref, rel=1e-13), name
        assert sums[NSITE] == 4


# ---------------------------------------------------------------------------
# multipoles: textbook values at special orientations
# ---------------------------------------------------------------------------
def point_species(kind, mag):
    return I.Species("P", [I.Site(kind, (0, 0, 0), (0, 0, 1), mag=mag)], 1.0, (0.1, 0.1, 0.1))


@pytest.mark.parametrize("qa,qb,coef", [
    (None, None, 6.0),              # end to end (axes along R = z)
    (None, Z_TO_X, -3.0),           # T shape
    (Z_TO_X, Z_TO_X, 9.0 / 4.0),    # parallel, side by side
    (Z_TO_X, Z_TO_Y, 3.0 / 4.0),    # crossed, both perpendicular to R
])
def test_quadrupole_pair_special_orientations(qa, qb, coef):
    Q, r, k = 1.3, 2.1, 0.7
    sp = point_species(I.QUAD, Q)
    s = two_molecules(sp, sp, [0, 0, r], qa=qa, qb=qb, coulomb_k=k)
    _, _, sums = oracle.forces(s)
    assert sums[U_ELEC] == pytest.approx(coef * k * Q * Q / r ** 5, rel=1e-13)


@pytest.mark.parametrize("qa,qb,coef", [
    (None, None, -2.0),                               # head to tail along R
    (Z_TO_X, Z_TO_X, 1.0),                            # parallel side by side
    (Z_TO_X, axis_quat([0, 1, 0], -math.pi / 2), -1.0),  # antiparallel side by side
    (Z_TO_X, Z_TO_Y, 0.0),                            # crossed
])
def test_dipole_pair_special_orientations(qa, qb, coef):
    mu, r = 1.7, 1.9
    sp = point_species(I.DIPOLE, mu)
    s = two_molecules(sp, sp, [0, 0, r], qa=qa, qb=qb)
    _, _, sums = oracle.forces(s)
    assert sums[U_ELEC] == pytest.approx(coef * mu * mu / r ** 3, rel=1e-13, abs=1e-15)


# ---------------------------------------------------------------------------
# multipoles: limit of explicit point charges (pins every pair type, its
# sign convention, force and torque)
# ---------------------------------------------------------------------------
def explicit_sites(kind, mag, pos, axis, d):
    pos, e = np.asarray(pos, float), np.asarray(axis, float)
    if kind == I.CHARGE:
        return [I.Site(I.CHARGE, tuple(pos), mag=mag)]
    if kind == I.DIPOLE:   # +q at +d/2 e, -q at -d/2 e, mu = q d
        q = mag / d
        return [I.Site(I.CHARGE, tuple(pos + 0.5 * d * e), mag=q),
                I.Site(I.CHARGE, tuple(pos - 0.5 * d * e), mag=-q)]
    # linear quadrupole: +q at +-d e, -2q at the centre, Q = 2 q d^2
    q = mag / (2 * d * d)
    return [I.Site(I.CHARGE, tuple(pos + d * e), mag=q), I.Site(I.CHARGE, tuple(pos - d * e), mag=q),
            I.Site(I.CHARGE, tuple(pos), mag=-2 * q)]


PAIRS = [(a, b) for a in (I.CHARGE, I.DIPOLE, I.QUAD) for b in (I.CHARGE, I.DIPOLE, I.QUAD)]


@pytest.mark.parametrize("ka,kb", PAIRS)
def test_multipole_explicit_charge_limit(ka, kb):
    rng = np.random.default_rng(10 + 3 * ka + kb)
    pa, pb = (0.1, -0.2, 0.15), (-0.05, 0.1, 0.2)       # off-centre sites
    ea, eb = unit(rng.normal(size=3)), unit(rng.normal(size=3))
    ma, mb = 0.9, -1.1
    qa, qb = I.random_quaternions(2, rng)
    R = np.array([1.7, -1.2, 2.3])

    def run(sa, sb):
        A = I.Species("A", sa, 1.0, (0.1, 0.2, 0.3))
        B = I.Species("B", sb, 1.0, (0.1, 0.2, 0.3))
        f, t, s = oracle.forces(two_molecules(A, B, R, qa=qa, qb=qb))
        return np.concatenate([[s[U_ELEC]], f[0], t[0], t[1]])

    point = run([I.Site(ka, pa, ea, mag=ma)], [I.Site(kb, pb, eb, mag=mb)])
    errs = []
    for d in (0.02, 0.01):
        expl = run(explicit_sites(ka, ma, pa, ea, d), explicit_sites(kb, mb, pb, eb, d))
        errs.append(np.abs(expl - point).max() / np.abs(point).max())
    if ka == kb == I.CHARGE:
        assert errs[0] < 1e-14
        return
    # the point-multipole terms are the exact d -> 0 limit: residual O(d^2)
    assert errs[1] < 2e-4
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_reaction_field_dipole_is_the_limit_of_site_rf_charges():
    mu, rc = 1.2, 3.0
    rng = np.random.default_rng(7)
    qa, qb = I.random_quaternions(2, rng)
    R = np.array([1.1, 0.9, -1.4])
    kw = dict(elec=I.ELEC_RF, eps_rf=30.0, rc=rc, box=40.0)

    def run(sa, sb):
        A = I.Species("A", sa, 1.0, (0.1, 0.1, 0.1))
        B = I.Species("B", sb, 1.0, (0.1, 0.1, 0.1))
        f, t, s = oracle.forces(two_molecules(A, B, R, qa=qa, qb=qb, **kw))
        return np.concatenate([[s[U_ELEC]], f[0], t[0], t[1]])

    point = run([I.Site(I.DIPOLE, (0, 0, 0), (0, 0, 1), mag=mu)], [I.Site(I.DIPOLE, (0, 0, 0), (0, 0, 1), mag=mu)])
    e = []
    for d in (0.02, 0.01):
        x = run(explicit_sites(I.DIPOLE, mu, (0, 0, 0), (0, 0, 1), d),
                explicit_sites(I.DIPOLE, mu, (0, 0, 0), (0, 0, 1), d))
        e.append(np.abs(x - point).max() / np.abs(point).max())
    assert e[1] < 1e-4 and 3.0 < e[0] / e[1] < 5.0


def test_reaction_field_charge_pair_vanishes_at_cutoff():
    sp = point_species(I.CHARGE, 1.0)
    rc = 2.0
    for eps_rf in (2.0, 80.0, math.inf):
        s = two_molecules(sp, sp, [0, 0, rc * (1 - 1e-9)], elec=I.ELEC_RF, eps_rf=eps_rf, rc=rc)
        _, _, sums = oracle.forces(s)
        assert abs(sums[U_ELEC]) < 1e-8


# ---------------------------------------------------------------------------
# finite differences: forces, torques, volume derivatives
# ---------------------------------------------------------------------------
def fd_systems():
    yield "offset_none", small_system([offset_multipoles()], 27, 4.6, 2.2, seed=1, lj_lrc=0)
    yield "offset_rf", small_system([offset_multipoles(), I.stockmayer()], 27, 4.6, 2.2, seed=2,
                                    elec=I.ELEC_RF, eps_rf=20.0, lj_lrc=0)
    yield "2cljq_rf", small_system([I.two_center_lj_quadrupole()], 27, 3.9, 1.85, seed=3,
                                   elec=I.ELEC_RF, lj_lrc=0)
    yield "ewald", small_system(ionic_pair_species(), 32, 4.4, 2.1, seed=4, elec=I.ELEC_EWALD,
                                alpha=1.6, kmax2=27, lj_lrc=0)


FD_SYSTEMS = list(fd_systems())


@pytest.mark.parametrize("name,system", FD_SYSTEMS, ids=[n for n, _ in FD_SYSTEMS])
def test_forces_and_torques_match_energy_gradient(name, system):
    u0, f, t, s = total(system)
    h = 1e-6
    scale = np.sqrt((f ** 2).sum(1).mean())
    tscale = np.sqrt((t ** 2).sum(1).mean())
    for i in range(0, system.n, 3):
        for k in range(3):
            up, dn = system.copy(), system.copy()
            up.com[i, k] += h
            dn.com[i, k] -= h
            eu, _, _, su = total(up)
            ed, _, _, sd = total(dn)
            assert su[NPAIR] == sd[NPAIR] == s[NPAIR]
            assert (eu - ed) / (2 * h) == pytest.approx(-f[i, k], abs=2e-6 * scale)
            # torque: -dU/dtheta for a lab-frame rotation about axis k
            e = np.zeros(3)
            e[k] = 1
            up, dn = system.copy(), system.copy()
            up.quat[i] = qmul(axis_quat(e, h), system.quat[i])
            dn.quat[i] = qmul(axis_quat(e, -h), system.quat[i])
            eu, _, _, _ = total(up)
            ed, _, _, _ = total(dn)
            assert (eu - ed) / (2 * h) == pytest.approx(-t[i, k], abs=2e-6 * max(tscale, scale))


@pytest.mark.parametrize("name,system", FD_SYSTEMS, ids=[n for n, _ in FD_SYSTEMS])
def test_volume_derivatives_match_scaling(name, system):
    """U_s = dU/ds and U_ss = d2U/ds2 under scaling of centres and box."""
    def at(sc):
        x = system.copy()
        x.com = system.com * sc
        x.params.box = system.params.box * sc
        return total(x)

    u0, _, _, s0 = at(1.0)
    h = 2e-5
    (up, _, _, sp), (dn, _, _, sd) = at(1 + h), at(1 - h)
    assert sp[NPAIR] == sd[NPAIR] == s0[NPAIR]
    assert (up - dn) / (2 * h) == pytest.approx(s0[US], rel=1e-7, abs=1e-7 * abs(u0))
    if system.params.elec != I.ELEC_EWALD:   # U_ss is not sampled with Ewald (Sec. 4)
        assert (up - 2 * u0 + dn) / (h * h) == pytest.approx(s0[USS], rel=1e-4, abs=1e-5 * abs(s0[USS]))


@pytest.mark.parametrize("name,system", FD_SYSTEMS, ids=[n for n, _ in FD_SYSTEMS])
def test_momentum_and_virial_identities(name, system):
    _, f, t, s = total(system)
    rms = np.sqrt((f ** 2).sum(1).mean())
    assert np.abs(f.sum(0)).max() < 1e-12 * rms * system.n
    assert s[US] == pytest.approx(-s[VIR], rel=1e-12)


def test_pair_angular_momentum_identity():
    rng = np.random.default_rng(5)
    sp = offset_multipoles()
    for _ in range(5):
        R = rng.normal(size=3) * 1.3
        qa, qb = I.random_quaternions(2, rng)
        f, t, s = oracle.forces(two_molecules(sp, sp, R, qa=qa, qb=qb))
        resid = t[0] + t[1] + np.cross(R, f[0])
        assert np.abs(resid).max() < 1e-12 * np.linalg.norm(f[0]) * np.linalg.norm(R) + 1e-14


# ---------------------------------------------------------------------------
# minimum image and cut-off: brute force over the 27 nearest images
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [11, 12, 13])
def test_minimum_image_brute_force(seed):
    rng = np.random.default_rng(seed)
    sp = offset_multipoles()
    box, rc, n = 6.0, 2.9, 8
    system = small_system([sp], n, box, rc, seed=seed, lj_lrc=0)
    system.com = rng.random((n, 3)) * box
    u, f, t, s = total(system)
    u_bf, f_bf, npair = 0.0, np.zeros((n, 3)), 0
    shifts = [np.array([a, b, c]) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    for i in range(n):
        for j in range(i + 1, n):
            Rs = [system.com[i] - system.com[j] + box * sh for sh in shifts]
            R = min(Rs, key=lambda v: float(v @ v))
            if R @ R >= rc * rc:
                continue
            npair += 1
            pair = two_molecules(sp, sp, R, qa=system.quat[i], qb=system.quat[j])
            fp, _, sp_ = oracle.forces(pair)
            u_bf += oracle.total_energy(sp_)
            f_bf[i] += fp[0]
            f_bf[j] += fp[1]
    assert npair == s[NPAIR]
    assert u == pytest.approx(u_bf, rel=1e-12)
    np.testing.assert_allclose(f, f_bf, rtol=1e-10, atol=1e-10 * np.abs(f).max())


def test_translation_and_permutation_invariance():
    system = small_system([offset_multipoles(), I.stockmayer()], 27, 4.6, 2.2, seed=9,
                          elec=I.ELEC_RF, eps_rf=20.0)
    u, f, t, s = total(system)
    moved = system.copy()
    moved.com = (system.com + np.array([1.37, -2.11, 0.53])) % system.params.box
    u2, f2, t2, _ = total(moved)
    assert u2 == pytest.approx(u, rel=1e-12)
    np.testing.assert_allclose(f2, f, atol=1e-10 * np.abs(f).max())
    perm = np.random.default_rng(1).permutation(system.n)
    pm = system.copy()
    pm.com, pm.quat, pm.species_idx = system.com[perm], system.quat[perm], system.species_idx[perm]
    u3, f3, t3, _ = total(pm)
    assert u3 == pytest.approx(u, rel=1e-12)
    np.testing.assert_allclose(f3, f[perm], atol=1e-10 * np.abs(f).max())
    np.testing.assert_allclose(t3, t[perm], atol=1e-10 * np.abs(t).max())


# ---------------------------------------------------------------------------
# Ewald: NaCl Madelung constant, independence of alpha
# ---------------------------------------------------------------------------
def read_golden(name):
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def rock_salt(cells, alpha_l, kmax2, rc_frac=0.49):
    a = 1.0                      # nearest-neighbour distance
    m = 2 * cells
    box = m * a
    pts, idx = [], []
    for x in range(m):
        for y in range(m):
            for z in range(m):
                pts.append([x + 0.5, y + 0.5, z + 0.5])
                idx.append((x + y + z) % 2)
    sp = [I.Species("NA", [I.Site(I.CHARGE, (0, 0, 0), mag=1.0)], 1.0, (0, 0, 0)),
          I.Species("CL", [I.Site(I.CHARGE, (0, 0, 0), mag=-1.0)], 1.0, (0, 0, 0))]
    params = I.Params(box=box, rc=rc_frac * box, elec=I.ELEC_EWALD, alpha=alpha_l / box, kmax2=kmax2,
                      lj_lrc=0)
    n = len(pts)
    return I.System("nacl", sp, params, np.array(idx, np.int32), np.array(pts, float),
                    I.identity_quaternions(n), np.zeros((n, 3)), np.zeros((n, 3)), I.MDSettings())


def test_ewald_nacl_madelung_constant():
    madelung = read_golden("nacl_madelung.txt")["madelung_nacl"]
    system = rock_salt(cells=2, alpha_l=8.0, kmax2=196)
    u, f, t, s = total(system)
    m_est = -u / (system.n / 2)          # U = -M k q^2 / a per ion pair
    assert abs(m_est - madelung) < 1e-6
    assert np.abs(f).max() < 1e-9        # perfect lattice: no net force on any ion


def test_ewald_total_independent_of_alpha():
    base = small_system(ionic_pair_species(), 32, 4.4, 2.15, seed=21, elec=I.ELEC_EWALD,
                        alpha=0.0, kmax2=0, lj_lrc=0)
    # a neutral system: 8 anions, 8 cations, 16 neutral molecules (no
    # neutralising-background term is modelled)
    base.species_idx = np.random.default_rng(2).permutation([0] * 8 + [1] * 8 + [2] * 16).astype(np.int32)
    res = []
    # converged on both sides: erfc(alpha (rc - 2 d_max)) < 1e-11, exp(-k^2/4alpha^2) < 1e-8
    for alpha, kmax2 in [(3.2, 400), (3.6, 529)]:
        x = base.copy()
        x.params.alpha, x.params.kmax2 = alpha, kmax2
        u, f, t, s = total(x)
        res.append((s[U_ELEC] + s[U_RECIP] + s[U_CONST], f, t))
    assert res[0][0] == pytest.approx(res[1][0], rel=1e-7)
    np.testing.assert_allclose(res[0][1], res[1][1], atol=2e-5 * np.abs(res[0][1]).max())


# ---------------------------------------------------------------------------
# LJ long-range correction: closed forms against numerical quadrature
# ---------------------------------------------------------------------------
def tail_integrals(eps, sig, rc):
    u = lambda r: 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6)
    du = lambda r: 4 * eps * (-12 * sig ** 12 / r ** 13 + 6 * sig ** 6 / r ** 7)
    d2u = lambda r: 4 * eps * (156 * sig ** 12 / r ** 14 - 42 * sig ** 6 / r ** 8)
    q = lambda g: integrate.quad(g, rc, np.inf, epsabs=0, epsrel=1e-13, limit=200)[0]
    return q(lambda r: r * r * u(r)), q(lambda r: r ** 3 * du(r)), q(lambda r: r ** 4 * d2u(r))


def test_lrc_one_site_matches_quadrature_and_textbook_values():
    system = I.lj_fluid()
    _, _, s = oracle.forces(system)
    n, V = system.n, system.params.box ** 3
    rho = n / V
    iu, ius, iuss = tail_integrals(1.0, 1.0, system.params.rc)
    pre = 2 * math.pi * n * n / V
    assert s[U_LRC] == pytest.approx(pre * iu, rel=1e-10)
    assert s[US_LRC] == pytest.approx(pre * ius, rel=1e-10)
    assert s[USS_LRC] == pytest.approx(pre * iuss, rel=1e-10)
    # textbook LJ tail values at rho = 0.7, rc = 4: U/N and pressure
    assert s[U_LRC] / n == pytest.approx(-0.0916223, abs=5e-7)
    p_lrc = -s[US_LRC] / (3 * V)
    assert p_lrc == pytest.approx(-0.1282608, abs=5e-7)
    assert rho == pytest.approx(0.7)


def test_lrc_multisite_mixture_matches_quadrature():
    sp = ionic_pair_species()
    system = small_system(sp, 40, 6.0, 2.9, seed=3, elec=I.ELEC_NONE)
    _, _, s = oracle.forces(system)
    counts = np.bincount(system.species_idx, minlength=len(sp))
    V = system.params.box ** 3
    ref = np.zeros(3)
    for A in range(len(sp)):
        for B in range(len(sp)):
            for sa in sp[A].sites:
                for sb in sp[B].sites:
                    if sa.kind != I.LJ or sb.kind != I.LJ:
                        continue
                    eps, sig = math.sqrt(sa.eps * sb.eps), 0.5 * (sa.sigma + sb.sigma)
                    ref += 2 * math.pi * counts[A] * counts[B] / V * np.array(tail_integrals(eps, sig, 2.9))
    np.testing.assert_allclose([s[U_LRC], s[US_LRC], s[USS_LRC]], ref, rtol=1e-10)

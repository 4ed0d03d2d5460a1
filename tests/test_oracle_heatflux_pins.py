"""Pin of the oracle's heat flux (Sec. 5, Eq. 6) of rigid multi-site
molecules.

The flux is the rate of change of the energy moment M = sum_k R_k e_k, with
e_k = kinetic energy of k + half of k's pair energies.  For an isolated
cluster (large box, every pair inside the cut-off, no crossing) this rate is
computed without the flux formula: the kinetic energies change by the work
F_k.v_k + tau_k.w_k (total forces and torques of the force routine), and the
pair energies change at the rate given by central differences of two-molecule
energies along the instantaneous motion (centres moved by v, bodies rotated
by w).  A dropped factor 1/2, the wrong sign or owner of a torque term, or a
missing convective term all fail it.  The partial-enthalpy term is checked
separately: J(h) - J(0) = -sum_k h_k v_k.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1507_07548_amd import inputs as I


def rotate_body(q, wb, eps):
    """q (x) exp(eps wb / 2): rotation by the body-frame angular velocity."""
    th = np.linalg.norm(wb) * eps
    if th == 0:
        return q.copy()
    ax = wb / np.linalg.norm(wb)
    d = np.array([math.cos(th / 2), *(math.sin(th / 2) * ax)])
    w0, x0, y0, z0 = q
    w1, x1, y1, z1 = d
    return np.array([w0 * w1 - x0 * x1 - y0 * y1 - z0 * z1, w0 * x1 + x0 * w1 + y0 * z1 - z0 * y1,
                     w0 * y1 - x0 * z1 + y0 * w1 + z0 * x1, w0 * z1 + x0 * y1 - y0 * x1 + z0 * w1])


def qmat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def cluster(elec, seed):
    rng = np.random.default_rng(seed)
    sp = [I.two_center_lj_quadrupole(), I.stockmayer(), I.water_tip4p_like(), I.one_center_lj()]
    if elec != I.ELEC_RF:
        sp = sp[:2] + [sp[3]]
    n = 7
    L = 120.0
    pts = []
    while len(pts) < n:                        # centres at least 1.3 apart, within a 6-wide cube
        p = rng.uniform(-3.0, 3.0, 3)
        if all(np.linalg.norm(p - x) > 1.3 for x in pts):
            pts.append(p)
    com = np.array(pts) + L / 2
    idx = rng.integers(0, len(sp), n).astype(np.int32)
    quat = I.random_quaternions(n, rng)
    params = I.Params(box=L, rc=55.0, elec=elec, eps_rf=15.0, coulomb_k=1.0 if elec != I.ELEC_RF else 0.02,
                      lj_lrc=0)
    vel = rng.normal(0, 1.0, (n, 3))
    omega = np.zeros((n, 3))
    for i in range(n):
        inertia = np.array(sp[idx[i]].inertia)
        omega[i] = np.where(inertia > 0, rng.normal(0, 1.5, 3), 0.0)
    return I.System("cluster", sp, params, idx, com, quat, vel, omega, I.MDSettings())


def pair_energy(s, i, j, com_i, com_j, q_i, q_j):
    two = I.System("pair", s.species, s.params, s.species_idx[[i, j]], np.stack([com_i, com_j]),
                   np.stack([q_i, q_j]), np.zeros((2, 3)), np.zeros((2, 3)), I.MDSettings())
    _, _, sums = oracle.forces(two)
    return sums[0] + sums[1]


@pytest.mark.parametrize("elec,seed", [(I.ELEC_NONE, 1), (I.ELEC_RF, 2), (I.ELEC_RF, 3)])
def test_heat_flux_is_the_rate_of_the_energy_moment(elec, seed):
    s = cluster(elec, seed)
    n = s.n
    F, T, _ = oracle.forces(s)
    eps = 1e-5
    u = np.zeros((n, n))
    du = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            u[i, j] = u[j, i] = pair_energy(s, i, j, s.com[i], s.com[j], s.quat[i], s.quat[j])
            up = pair_energy(s, i, j, s.com[i] + eps * s.vel[i], s.com[j] + eps * s.vel[j],
                             rotate_body(s.quat[i], s.omega[i], eps), rotate_body(s.quat[j], s.omega[j], eps))
            um = pair_energy(s, i, j, s.com[i] - eps * s.vel[i], s.com[j] - eps * s.vel[j],
                             rotate_body(s.quat[i], s.omega[i], -eps), rotate_body(s.quat[j], s.omega[j], -eps))
            du[i, j] = du[j, i] = (up - um) / (2 * eps)
    dM = np.zeros(3)
    for k in range(n):
        spk = s.species[s.species_idx[k]]
        kin = 0.5 * spk.mass * s.vel[k] @ s.vel[k] + 0.5 * np.dot(spk.inertia, s.omega[k] ** 2)
        e = kin + 0.5 * u[k].sum()
        w_lab = qmat(s.quat[k]) @ s.omega[k]
        de = F[k] @ s.vel[k] + T[k] @ w_lab + 0.5 * du[k].sum()
        dM += s.vel[k] * e + s.com[k] * de
    jq = oracle.heat_flux(s)
    scale = np.abs(dM).max()
    np.testing.assert_allclose(jq, dM, rtol=0, atol=2e-7 * scale)


def test_partial_enthalpy_term():
    s = cluster(I.ELEC_RF, 5)
    h = np.array([0.7, -1.3, 2.1, 0.4])
    j0 = oracle.heat_flux(s)
    jh = oracle.heat_flux(s, h_partial=h)
    expect = -(h[s.species_idx][:, None] * s.vel).sum(0)
    np.testing.assert_allclose(jh - j0, expect, rtol=1e-12, atol=1e-12)

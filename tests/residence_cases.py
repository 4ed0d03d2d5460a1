"""Residence-time test systems with occupancy windows that are known by hand
(non-interacting molecules, exact binary arithmetic), shared by the oracle
pins and the GPU parity tests.  No method arithmetic here."""
import numpy as np

from paper_1507_07548_amd import inputs as I


def ghost(name):
    # LJ site with eps = 0: no forces, straight-line motion
    s = I.one_center_lj(eps=0.0, sigma=1.0, mass=1.0)
    s.name = name
    return s


def ballistic_system(tolerance, n_steps=12):
    """Solute 0 at rest at the box centre (L = 16); four solvents moving along
    x on lines at distinct heights y (so that no two molecules ever meet),
    shell radius 2, dt = 1/8, one sample per step, origins every 4 steps,
    10 lags.  Inside the shell iff x^2 + y^2 < 4 (strictly).  Per-step
    displacements u (x(k) = x0 + k u, wrapped):
      S1 y = 0,     x0 = 0.5, u = 0    : inside always
      S2 y = 0,     x0 = 1.0, u = 0.5  : inside at k = 0, 1; exactly on the
                                         shell at k = 2, outside from then on
      S3 y = -0.5,  x0 = 1.5, u = 4    : inside at k = 0 mod 4 (|x| < 1.936),
                                         outside 3 samples in between
      S4 y = 1,     x0 = 3.0, u = -0.5 : inside for k = 3 ... 9 (|x| < 1.732)
    A second solute at rest far from all of them has an empty shell: it adds
    nothing to the correlation and zeros to the solvation sum.
    """
    L, c = 16.0, 8.0
    x0 = np.array([0.0, 0.5, 1.0, 1.5, 3.0])
    y0 = np.array([0.0, 0.0, 0.0, -0.5, 1.0])
    u = np.array([0.0, 0.0, 0.5, 4.0, -0.5])
    dt = 0.125
    com = np.stack([c + x0, c + y0, np.full(5, c)], axis=1)
    vel = np.stack([u / dt, np.zeros(5), np.zeros(5)], axis=1)
    com = np.vstack([com, [c, 0.5, 0.5]])
    vel = np.vstack([vel, [0.0, 0.0, 0.0]])
    params = I.Params(box=L, rc=7.5, lj_lrc=0)
    md = I.MDSettings(integrator=I.VV, dt=dt, temperature=0.0, n_steps=n_steps, acf_every=1,
                      acf_origin_every=4, acf_nlag=10, res_solute=0, res_solvent=1, res_radius=2.0,
                      res_tolerance=tolerance)
    quat = np.tile([1.0, 0.0, 0.0, 0.0], (6, 1))
    return I.System("ballistic", [ghost("solute"), ghost("solvent")], params,
                    np.array([0, 1, 1, 1, 1, 0], dtype=np.int32), com, quat, vel, np.zeros((6, 3)), md)


# hand-derived from the windows above: origins at k = 0, 4, 8, 12 holding
# {S1, S2, S3}, {S1, S3, S4}, {S1, S3, S4}, {S1, S3}.  With tolerance 3, S3
# (outside for 3 samples between visits) keeps counting at every visit; with
# tolerance 2 it stops after its first excursion.  S4 leaves for good at k = 10.
BALLISTIC_EXPECTED = {
    3: {"res_acf": [4.0, 2.0, 4.0 / 3.0, 4.0 / 3.0, 7.0 / 3.0, 1.0, 2.0 / 3.0, 2.0 / 3.0, 4.0 / 3.0, 1.0 / 3.0],
        "res_cnt": [4.0, 3.0, 3.0, 3.0, 3.0, 2.0, 2.0, 2.0, 2.0, 1.0]},
    2: {"res_acf": [4.0, 2.0, 4.0 / 3.0, 4.0 / 3.0, 4.0 / 3.0, 1.0, 2.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 1.0 / 3.0],
        "res_cnt": [4.0, 3.0, 3.0, 3.0, 3.0, 2.0, 2.0, 2.0, 2.0, 1.0]},
}
# shell populations 3,2,1,2,3,2,2,2,3,2,1,1,2 over the 13 samples k = 0 ... 12
# for the first solute, 0 for the second: 26 over 2 x 13 terms
BALLISTIC_SOLVATION = (26.0, 26.0)


def fcc_system(n_steps=6):
    """A perfect FCC lattice (108 sites, cell a = 2) of non-interacting
    molecules at rest; the solute sits on a site, so its first shell
    (distance a / sqrt(2)) holds exactly 12 molecules inside radius 1.7."""
    L = 6.0
    pts = I.fcc_lattice(108, L) + 0.25
    n = len(pts)
    sp = np.ones(n, dtype=np.int32)
    sp[13] = 0
    params = I.Params(box=L, rc=2.9, lj_lrc=0)
    md = I.MDSettings(integrator=I.VV, dt=0.01, temperature=0.0, n_steps=n_steps, acf_every=2,
                      acf_origin_every=2, acf_nlag=3, res_solute=0, res_solvent=1, res_radius=1.7,
                      res_tolerance=0)
    return I.System("fcc", [ghost("solute"), ghost("solvent")], params, sp, pts,
                    np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), np.zeros((n, 3)), np.zeros((n, 3)), md)

"""Extra molecular models used only by the tests: molecules whose dipoles,
quadrupoles and charges sit off the centre of mass, and explicit-charge
stand-ins for point multipoles."""
import math

import numpy as np

from paper_1507_07548_amd.inputs import (CHARGE, DIPOLE, LJ, QUAD, Params, Site, Species,
                                         System, MDSettings, ELEC_NONE, identity_quaternions,
                                         random_quaternions)


def unit(v):
    v = np.asarray(v, dtype=float)
    return tuple(v / np.linalg.norm(v))


def offset_multipoles() -> Species:
    """Non-linear rigid molecule carrying every site type away from its centre."""
    return Species("OFFSET", [
        Site(LJ, (0.0, 0.0, 0.35), sigma=1.0, eps=1.0),
        Site(LJ, (0.1, 0.0, -0.35), sigma=0.9, eps=0.8),
        Site(DIPOLE, (0.2, -0.1, 0.05), unit((0.3, 0.5, 0.8)), mag=0.9),
        Site(QUAD, (-0.15, 0.2, 0.0), unit((0.7, -0.2, 0.4)), mag=0.8),
        Site(CHARGE, (0.05, 0.25, -0.1), mag=0.4),
        Site(CHARGE, (-0.05, -0.25, 0.1), mag=-0.4),
    ], 1.0, (0.05, 0.07, 0.09))


def ionic_pair_species():
    """Reduced-unit ions and a neutral 3-charge molecule, all Ewald-compatible."""
    return [
        Species("ANIONR", [Site(LJ, (0, 0, 0), sigma=1.0, eps=1.0), Site(CHARGE, (0, 0, 0), mag=-1.0)], 1.0, (0, 0, 0)),
        Species("CATIONR", [Site(LJ, (0, 0, 0), sigma=0.8, eps=0.5), Site(CHARGE, (0, 0, 0), mag=1.0)], 1.0, (0, 0, 0)),
        Species("TRI", [Site(LJ, (0, 0, 0.1), sigma=1.0, eps=1.0),
                        Site(CHARGE, (0.3, 0.0, -0.1), mag=0.5),
                        Site(CHARGE, (-0.3, 0.0, -0.1), mag=0.5),
                        Site(CHARGE, (0.0, 0.0, 0.2), mag=-1.0)], 1.0, (0.03, 0.05, 0.08)),
    ]


def four_charge_species() -> Species:
    """Neutral rigid molecule with four off-centre charges (the most any model
    class carries) around one LJ site: every charge slot of the reciprocal
    kernels in use."""
    return Species("TETRA4", [
        Site(LJ, (0.0, 0.0, 0.0), sigma=1.0, eps=1.0),
        Site(CHARGE, (0.25, 0.25, 0.25), mag=0.6),
        Site(CHARGE, (-0.25, -0.25, 0.25), mag=0.4),
        Site(CHARGE, (-0.25, 0.25, -0.25), mag=-0.7),
        Site(CHARGE, (0.25, -0.25, -0.25), mag=-0.3),
    ], 1.0, (0.05, 0.05, 0.05))


def small_system(species, n, box, rc, seed, elec=ELEC_NONE, jitter=0.15, **pkw):
    """n molecules on a jittered simple-cubic lattice with random orientations
    and random species assignment."""
    rng = np.random.default_rng(seed)
    m = int(math.ceil(n ** (1.0 / 3.0)))
    a = box / m
    pts = np.array([[(ix + 0.5) * a, (iy + 0.5) * a, (iz + 0.5) * a]
                    for ix in range(m) for iy in range(m) for iz in range(m)])[:n]
    pts = pts + rng.uniform(-jitter, jitter, pts.shape) * a
    idx = rng.integers(0, len(species), n).astype(np.int32)
    quat = random_quaternions(n, rng)
    params = Params(box=box, rc=rc, elec=elec, **pkw)
    return System("test", list(species), params, idx, pts % box, quat,
                  np.zeros((n, 3)), np.zeros((n, 3)), MDSettings())


def two_molecules(sp_a, sp_b, R, qa=None, qb=None, box=40.0, rc=19.0, elec=ELEC_NONE, **pkw):
    """Molecule a at the centre of a huge box, molecule b displaced by -R
    (so R = R_a - R_b)."""
    c = np.array([box / 2] * 3)
    com = np.stack([c, c - np.asarray(R, dtype=float)])
    quat = np.stack([qa if qa is not None else [1, 0, 0, 0], qb if qb is not None else [1, 0, 0, 0]]).astype(float)
    params = Params(box=box, rc=rc, elec=elec, lj_lrc=0, **pkw)
    return System("pair", [sp_a, sp_b], params, np.array([0, 1], dtype=np.int32), com, quat,
                  np.zeros((2, 3)), np.zeros((2, 3)), MDSettings())

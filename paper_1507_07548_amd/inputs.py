"""Seeded synthetic inputs: molecular models, lattices, orientations, velocities.

This module is shared by the GPU path's tests/benchmark and by the oracle's
tests.  It holds configuration and random numbers only -- none of the
method's arithmetic (no potentials, forces, integrators or samplers).

Workloads follow the paper's problem statement (homogeneous fluids of about
10^3 rigid molecules, Sec. 2; a cut-off of the order of half the box edge,
Sec. 2; Lennard-Jones sites, point charges, dipoles and quadrupoles, Sec. 3;
ions with Ewald summation, Sec. 4).  The water-like model takes only its
density from the paper's water runs (Table 1: 55.345 mol/dm^3 at 298.15 K);
its geometry and parameters are a TIP4P-type literature choice, and the ion
parameters are synthetic.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

LJ, CHARGE, DIPOLE, QUAD = 0, 1, 2, 3
ELEC_NONE, ELEC_RF, ELEC_EWALD = 0, 1, 2
CUT_COM, CUT_SITE = 0, 1
VV, GEAR = 0, 1

# e^2 / (4 pi eps0 k_B Angstrom): Coulomb constant for energies in K,
# lengths in Angstrom and charges in e (CODATA 2018 constants).
COULOMB_K_KELVIN_ANGSTROM = 167100.94689828737
# Time unit of the (Angstrom, u, K) system: Angstrom * sqrt(u / k_B) in s.
TIME_UNIT_S = 1.0966875352677374e-12
FEMTOSECOND = 1e-15 / TIME_UNIT_S


@dataclasses.dataclass
class Site:
    kind: int                      # LJ, CHARGE, DIPOLE or QUAD
    pos: Sequence[float]           # body frame, relative to the centre of mass
    axis: Sequence[float] = (0.0, 0.0, 1.0)
    sigma: float = 0.0
    eps: float = 0.0
    mag: float = 0.0               # q, mu or Q


@dataclasses.dataclass
class Species:
    name: str
    sites: List[Site]
    mass: float
    inertia: Sequence[float]       # principal moments (body frame axes)


@dataclasses.dataclass
class Params:
    box: float
    rc: float
    elec: int = ELEC_NONE
    eps_rf: float = math.inf
    alpha: float = 0.0
    kmax2: int = 0
    coulomb_k: float = 1.0
    lj_lrc: int = 1
    cutoff_mode: int = 0            # CUT_COM or CUT_SITE (LJ site pairs cut at their own distance)


@dataclasses.dataclass
class MDSettings:
    integrator: int = GEAR
    dt: float = 0.001
    temperature: float = 0.0       # > 0 isokinetic NVT, <= 0 NVE
    n_steps: int = 0
    sample_every: int = 0
    rdf_every: int = 0
    rdf_bins: int = 0
    rdf_rmax: float = 0.0
    acf_every: int = 0
    acf_origin_every: int = 0
    acf_nlag: int = 0
    u0: float = 0.0
    # residence time / solvation number (Sec. 5, Eqs. 7-8), on the ACF schedule
    res_solute: int = -1            # species of the central molecules, -1 = off
    res_solvent: int = -1           # species counted around them
    res_radius: float = 0.0         # shell radius between molecule centres
    res_tolerance: int = 0          # samples a molecule may spend outside and still count
    # heat-flux ACF (Sec. 5, Eqs. 5-6), on the ACF schedule
    heat_flux: bool = False
    h_partial: Optional[tuple] = None   # partial molar enthalpy per molecule, per species


@dataclasses.dataclass
class System:
    name: str
    species: List[Species]
    params: Params
    species_idx: np.ndarray        # int32 [n]
    com: np.ndarray                # float64 [n, 3]
    quat: np.ndarray               # float64 [n, 4] (w, x, y, z)
    vel: np.ndarray                # float64 [n, 3] lab frame
    omega: np.ndarray              # float64 [n, 3] body frame
    md: MDSettings

    @property
    def n(self) -> int:
        return int(self.species_idx.shape[0])

    def copy(self) -> "System":
        return dataclasses.replace(
            self, species_idx=self.species_idx.copy(), com=self.com.copy(),
            quat=self.quat.copy(), vel=self.vel.copy(), omega=self.omega.copy(),
            params=dataclasses.replace(self.params), md=dataclasses.replace(self.md))


# --------------------------------------------------------------------------
# molecular models
# --------------------------------------------------------------------------
def one_center_lj(eps: float = 1.0, sigma: float = 1.0, mass: float = 1.0) -> Species:
    return Species("1CLJ", [Site(LJ, (0.0, 0.0, 0.0), sigma=sigma, eps=eps)], mass, (0.0, 0.0, 0.0))


def two_center_lj_quadrupole(elongation: float = 0.3, q2: float = 2.0,
                             eps: float = 1.0, sigma: float = 1.0,
                             site_mass: float = 0.5) -> Species:
    """Rigid two-centre LJ molecule with a linear point quadrupole at its centre.

    Sites at +-elongation/2 on the body z axis; Q^2 = q2 in reduced units."""
    h = 0.5 * elongation
    i_perp = 2.0 * site_mass * h * h
    sites = [Site(LJ, (0.0, 0.0, h), sigma=sigma, eps=eps),
             Site(LJ, (0.0, 0.0, -h), sigma=sigma, eps=eps)]
    if q2 > 0.0:
        sites.append(Site(QUAD, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), mag=math.sqrt(q2)))
    return Species("2CLJQ", sites, 2.0 * site_mass, (i_perp, i_perp, 0.0))


def stockmayer(mu2: float = 3.0, eps: float = 1.0, sigma: float = 1.0,
               mass: float = 1.0, inertia: float = 0.025) -> Species:
    """LJ sphere with a central point dipole along the body z axis."""
    return Species("STOCKMAYER",
                   [Site(LJ, (0.0, 0.0, 0.0), sigma=sigma, eps=eps),
                    Site(DIPOLE, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), mag=math.sqrt(mu2))],
                   mass, (inertia, inertia, 0.0))


def _principal_frame(points: np.ndarray, masses: np.ndarray):
    """Centre of mass and principal axes of a set of point masses."""
    com = (masses[:, None] * points).sum(0) / masses.sum()
    x = points - com
    inertia = np.zeros((3, 3))
    for m, v in zip(masses, x):
        inertia += m * (np.dot(v, v) * np.eye(3) - np.outer(v, v))
    w, vec = np.linalg.eigh(inertia)
    if np.linalg.det(vec) < 0:
        vec[:, 2] *= -1.0
    return com, vec, w


def water_tip4p_like() -> Species:
    """4-site water: LJ on O, +0.52 e on each H, -1.04 e on the M site.

    r_OH = 0.9572 A, angle HOH = 104.52 deg, M 0.15 A from O on the bisector,
    sigma_O = 3.154 A, eps_O/k_B = 78.0 K (a TIP4P-type literature choice).
    Units: A, K, e, u."""
    r_oh, ang, d_om = 0.9572, math.radians(104.52), 0.15
    o = np.array([0.0, 0.0, 0.0])
    h1 = np.array([r_oh * math.sin(ang / 2), 0.0, r_oh * math.cos(ang / 2)])
    h2 = np.array([-r_oh * math.sin(ang / 2), 0.0, r_oh * math.cos(ang / 2)])
    m = np.array([0.0, 0.0, d_om])
    masses = np.array([15.9994, 1.008, 1.008])
    com, axes, moments = _principal_frame(np.stack([o, h1, h2]), masses)
    body = lambda v: tuple(float(c) for c in (v - com) @ axes)
    sites = [Site(LJ, body(o), sigma=3.154, eps=78.0),
             Site(CHARGE, body(h1), mag=0.52),
             Site(CHARGE, body(h2), mag=0.52),
             Site(CHARGE, body(m), mag=-1.04)]
    return Species("WATER4", sites, float(masses.sum()), tuple(float(x) for x in moments))


def ion(charge: float, sigma: float, eps: float, mass: float, name: str) -> Species:
    """Monatomic ion: an LJ site and a point charge at the centre (A, K, e, u)."""
    return Species(name, [Site(LJ, (0.0, 0.0, 0.0), sigma=sigma, eps=eps),
                          Site(CHARGE, (0.0, 0.0, 0.0), mag=charge)], mass, (0.0, 0.0, 0.0))


def cation() -> Species:
    return ion(+1.0, 2.6, 50.0, 22.99, "CATION")


def anion() -> Species:
    return ion(-1.0, 4.4, 50.0, 35.45, "ANION")


# --------------------------------------------------------------------------
# seeded generators
# --------------------------------------------------------------------------
def fcc_lattice(n: int, box: float) -> np.ndarray:
    """First n sites of the smallest 4 m^3 >= n face-centred cubic lattice,
    ordered (x cell, y cell, z cell, basis)."""
    m = 1
    while 4 * m ** 3 < n:
        m += 1
    a = box / m
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    pts = []
    for ix in range(m):
        for iy in range(m):
            for iz in range(m):
                for b in basis:
                    pts.append((np.array([ix, iy, iz]) + b + 0.25) * a)
    return np.array(pts[:n], dtype=np.float64)


def random_quaternions(n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed unit quaternions (Shoemake's subgroup method)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def identity_quaternions(n: int) -> np.ndarray:
    q = np.zeros((n, 4))
    q[:, 0] = 1.0
    return q


def maxwell_boltzmann(masses: np.ndarray, temperature: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian velocities, zero total momentum, scaled to `temperature` over
    3N - 3 degrees of freedom (k_B = 1 in the caller's energy unit)."""
    n = masses.shape[0]
    v = rng.standard_normal((n, 3)) * np.sqrt(temperature / masses)[:, None]
    v -= (masses[:, None] * v).sum(0) / masses.sum()
    if temperature > 0.0 and n > 1:
        t_now = (masses[:, None] * v * v).sum() / (3 * n - 3)
        v *= math.sqrt(temperature / t_now)
    return v


def body_angular_velocities(inertia: np.ndarray, temperature: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian body-frame angular velocities N(0, T / I_k); 0 where I_k = 0."""
    inertia = np.asarray(inertia, dtype=np.float64)
    w = rng.standard_normal(inertia.shape)
    safe = np.where(inertia > 0.0, inertia, 1.0)
    return np.where(inertia > 0.0, w * np.sqrt(temperature / safe), 0.0)


def _finish(name, species, params, idx, com, quat, temperature, rng, md) -> System:
    idx = np.asarray(idx, dtype=np.int32)
    masses = np.array([species[s].mass for s in idx])
    inertia = np.array([species[s].inertia for s in idx], dtype=np.float64)
    vel = maxwell_boltzmann(masses, temperature, rng) if temperature > 0 else np.zeros((len(idx), 3))
    omega = body_angular_velocities(inertia, temperature, rng) if temperature > 0 else np.zeros((len(idx), 3))
    return System(name, species, params, idx, np.ascontiguousarray(com, dtype=np.float64),
                  np.ascontiguousarray(quat, dtype=np.float64), vel, omega, md)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def lj_fluid(n: int = 500, density: float = 0.7, temperature: float = 1.5, rc: float = 4.0,
             seed: int = 1, n_steps: int = 100, dt: float = 0.002) -> System:
    """One-site LJ fluid on an FCC start, velocity Verlet NVE (reduced units).
    Defaults: 500 molecules, rho = 0.7, T = 1.5, rc = 4.0, dt = 0.002, 100 steps."""
    rng = np.random.default_rng(seed)
    box = (n / density) ** (1.0 / 3.0)
    sp = [one_center_lj()]
    params = Params(box=box, rc=rc, elec=ELEC_NONE, lj_lrc=1)
    md = MDSettings(integrator=VV, dt=dt, temperature=0.0, n_steps=n_steps)
    return _finish("lj_fluid", sp, params, np.zeros(n), fcc_lattice(n, box),
                   identity_quaternions(n), temperature, rng, md)


def quadrupolar_fluid(n: int = 1000, density: float = 0.6, temperature: float = 2.0,
                      rc_frac: float = 0.48, seed: int = 2, n_steps: int = 1000,
                      dt: float = 0.001, elongation: float = 0.3, q2: float = 2.0,
                      sample_every: int = 1) -> System:
    """2CLJQ fluid (elongation 0.3, Q^2 = 2), rc = 0.48 L, reaction field with
    eps_RF = infinity (no term acts on quadrupoles), Gear NVT (reduced units)."""
    rng = np.random.default_rng(seed)
    box = (n / density) ** (1.0 / 3.0)
    sp = [two_center_lj_quadrupole(elongation, q2)]
    params = Params(box=box, rc=rc_frac * box, elec=ELEC_RF, eps_rf=math.inf, lj_lrc=1)
    md = MDSettings(integrator=GEAR, dt=dt, temperature=temperature, n_steps=n_steps,
                    sample_every=sample_every)
    return _finish("quadrupolar_fluid", sp, params, np.zeros(n), fcc_lattice(n, box),
                   random_quaternions(n, rng), temperature, rng, md)


def ionic_solution(n_water: int = 900, n_pairs: int = 50, molar_density: float = 55.345,
                   temperature: float = 298.0, rc_frac: float = 0.48, alpha_l: float = 5.6,
                   kmax2: int = 64, seed: int = 3, n_steps: int = 500,
                   rdf_bins: int = 400, rdf_every: int = 10) -> System:
    """Water-like molecules plus cation/anion pairs on random lattice sites,
    Ewald (alpha = alpha_l / L, 0 < n^2 <= kmax2), tin-foil, rc = 0.48 L.
    Units: A, K, e, u; dt = 1 fs."""
    rng = np.random.default_rng(seed)
    n = n_water + 2 * n_pairs
    box = (n / (molar_density * 6.02214076e23 * 1e3 * 1e-30)) ** (1.0 / 3.0)
    sp = [water_tip4p_like(), cation(), anion()]
    idx = np.array([0] * n_water + [1] * n_pairs + [2] * n_pairs)
    idx = idx[rng.permutation(n)]
    params = Params(box=box, rc=rc_frac * box, elec=ELEC_EWALD, alpha=alpha_l / box,
                    kmax2=kmax2, coulomb_k=COULOMB_K_KELVIN_ANGSTROM, lj_lrc=1)
    dmax = max(np.linalg.norm(s.pos) for spc in sp for s in spc.sites if s.kind == LJ)
    md = MDSettings(integrator=GEAR, dt=FEMTOSECOND, temperature=temperature, n_steps=n_steps,
                    rdf_every=rdf_every, rdf_bins=rdf_bins,
                    rdf_rmax=params.rc - 2.0 * dmax)
    return _finish("ionic_solution", sp, params, idx, fcc_lattice(n, box),
                   random_quaternions(n, rng), temperature, rng, md)


def batched_state_point(s: int, master_seed: int = 4, n_lo: int = 500, n_hi: int = 4000,
                        rho_lo: float = 0.1, rho_hi: float = 0.8, t_lo: float = 1.0,
                        t_hi: float = 3.0, n_steps: int = 10000, n_override: Optional[int] = None) -> System:
    """State point s of the batched 2CLJQ workload: N ~ U{n_lo..n_hi},
    rho ~ U(rho_lo, rho_hi), T ~ U(t_lo, t_hi), seeded 1000 + s."""
    draw = np.random.default_rng([master_seed, s])
    n = int(draw.integers(n_lo, n_hi + 1)) if n_override is None else int(n_override)
    rho = float(draw.uniform(rho_lo, rho_hi))
    temp = float(draw.uniform(t_lo, t_hi))
    sysm = quadrupolar_fluid(n=n, density=rho, temperature=temp, seed=1000 + s,
                             n_steps=n_steps, sample_every=1)
    sysm.name = f"state_point_{s}"
    return sysm


def jittered(system: System, amplitude: float, seed: int) -> System:
    """Same system with every centre displaced by a uniform random vector of
    at most `amplitude` per component (wrapped into the box)."""
    rng = np.random.default_rng(seed)
    out = system.copy()
    out.com = (system.com + rng.uniform(-amplitude, amplitude, system.com.shape)) % system.params.box
    return out


def with_random_positions(system: System, seed: int) -> System:
    """Same model, uniformly random centres and orientations (for parity tests
    that need unstructured geometry)."""
    rng = np.random.default_rng(seed)
    out = system.copy()
    out.com = rng.random((system.n, 3)) * system.params.box
    out.quat = random_quaternions(system.n, rng)
    return out


# --------------------------------------------------------------------------
# serving trace
# --------------------------------------------------------------------------
SERVING_MODELS = ("lj", "2cljq", "ionic")


def serving_system(model: str, n: int, seed: int, n_steps: int, window: int = 1000,
                   acf_every: int = 10, origin_every: int = 100, rdf_every: int = 10,
                   rdf_bins: int = 400) -> System:
    """One request of the serving workload: model family `model` with n
    molecules, seeded, running `n_steps` steps with RDF, Lustig moments (not
    with Ewald) and velocity / electric-current ACFs over a `window`-step
    window on an extended step of `acf_every`."""
    if model == "lj":
        box = (n / 0.7) ** (1.0 / 3.0)
        s = lj_fluid(n=n, density=0.7, temperature=1.5, rc=min(4.0, 0.48 * box), seed=seed,
                     n_steps=n_steps)
        s.md.sample_every = 1
        dmax = 0.0
    elif model == "2cljq":
        s = quadrupolar_fluid(n=n, seed=seed, n_steps=n_steps, sample_every=1)
        dmax = 0.15
    elif model == "ionic":
        pairs = max(1, int(round(0.05 * n)))
        s = ionic_solution(n_water=n - 2 * pairs, n_pairs=pairs, seed=seed, n_steps=n_steps,
                           rdf_every=rdf_every, rdf_bins=rdf_bins)
        dmax = max(np.linalg.norm(x.pos) for sp in s.species for x in sp.sites if x.kind == LJ)
    else:
        raise ValueError(model)
    s.md.rdf_every, s.md.rdf_bins = rdf_every, rdf_bins
    s.md.rdf_rmax = s.params.rc - 2.0 * dmax
    s.md.acf_every, s.md.acf_origin_every = acf_every, origin_every
    s.md.acf_nlag = window // acf_every
    s.name = f"{model}_{n}"
    return s


def serving_trace(n_requests: int = 64, rate: float = 50.0, seed: int = 5, n_lo: int = 256,
                  n_hi: int = 8192, n_steps: int = 20000, **kw):
    """Poisson arrivals (exponential gaps, mean 1/rate), model uniform over the
    three families, N = round(n_lo (n_hi/n_lo)^u) with u ~ U(0, 1); request r
    is seeded 50000 + r.  Returns [(arrival, model, system)]."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    out = []
    for r in range(n_requests):
        model = SERVING_MODELS[int(rng.integers(len(SERVING_MODELS)))]
        n = int(round(n_lo * (n_hi / n_lo) ** rng.random()))
        out.append((float(t[r]), model, serving_system(model, n, 50000 + r, n_steps, **kw)))
    return out

"""ctypes front end of the plain FP64 CPU oracle (``ms2_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The product package never imports it,
and it imports nothing from the product package: it takes the shared seeded
inputs (plain numpy arrays and model descriptions) and returns numpy arrays.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ms2_oracle.c")
_LIB = os.path.join(_HERE, "libms2_oracle.so")
OR_MAXS = 8

SUM_NAMES = ["u_lj", "u_elec", "u_recip", "u_const", "u_lrc", "virial", "us", "uss",
             "us_lrc", "uss_lrc", "npair", "nsite"]
NSUM = len(SUM_NAMES)
MOMENT_NAMES = ["n", "x", "xx", "xxx", "y", "xy", "xxy", "yy", "xyy", "z", "xz"]
# columns of the per-step energy log of md(): U, K_trans, K_rot, W, U_s + U_s,lrc, U_ss + U_ss,lrc
LOG_COLS = 6

c_double, c_int32 = ctypes.c_double, ctypes.c_int32


class OrSpecies(ctypes.Structure):
    _fields_ = [("n_sites", c_int32), ("type", c_int32 * OR_MAXS),
                ("pos", (c_double * 3) * OR_MAXS), ("axis", (c_double * 3) * OR_MAXS),
                ("sigma", c_double * OR_MAXS), ("eps", c_double * OR_MAXS),
                ("mag", c_double * OR_MAXS), ("mass", c_double), ("inertia", c_double * 3)]


class OrParams(ctypes.Structure):
    _fields_ = [("box", c_double), ("rc", c_double), ("eps_rf", c_double), ("alpha", c_double),
                ("coulomb_k", c_double), ("elec", c_int32), ("kmax2", c_int32),
                ("lj_lrc", c_int32), ("cutoff_mode", c_int32)]


class OrMD(ctypes.Structure):
    _fields_ = [("integrator", c_int32), ("n_steps", c_int32), ("dt", c_double),
                ("temperature", c_double), ("sample_every", c_int32), ("rdf_every", c_int32),
                ("rdf_bins", c_int32), ("acf_every", c_int32), ("acf_origin_every", c_int32),
                ("acf_nlag", c_int32), ("rdf_rmax", c_double), ("u0", c_double),
                ("res_solute", c_int32), ("res_solvent", c_int32), ("res_radius", c_double),
                ("res_tolerance", c_int32), ("heat_flux", c_int32),
                ("h_partial", ctypes.POINTER(c_double))]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, cut-off expression uncontracted)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        dp, ip = P(c_double), P(c_int32)
        _lib.or_forces.argtypes = [P(OrSpecies), c_int32, P(OrParams), c_int32, ip, dp, dp, dp, dp, dp]
        _lib.or_kspace.argtypes = _lib.or_forces.argtypes
        _lib.or_md.argtypes = [P(OrSpecies), c_int32, P(OrParams), P(OrMD), c_int32, ip,
                               dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        _lib.or_heat_flux.argtypes = [P(OrSpecies), c_int32, P(OrParams), c_int32, ip, dp, dp, dp, dp, dp, dp]
        _lib.or_rdf_ntypes.argtypes = [P(OrSpecies), c_int32]
        _lib.or_check.argtypes = [P(OrSpecies), c_int32, P(OrParams)]
    return _lib


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(c_double))


def species_array(species) -> ctypes.Array:
    arr = (OrSpecies * len(species))()
    for k, s in enumerate(species):
        o = arr[k]
        if len(s.sites) > OR_MAXS:
            raise ValueError("too many sites")
        o.n_sites = len(s.sites)
        for a, site in enumerate(s.sites):
            o.type[a] = int(site.kind)
            for c in range(3):
                o.pos[a][c] = float(site.pos[c])
                o.axis[a][c] = float(site.axis[c])
            o.sigma[a], o.eps[a], o.mag[a] = float(site.sigma), float(site.eps), float(site.mag)
        o.mass = float(s.mass)
        for c in range(3):
            o.inertia[c] = float(s.inertia[c])
    return arr


def params_struct(p) -> OrParams:
    return OrParams(box=p.box, rc=p.rc, eps_rf=p.eps_rf, alpha=p.alpha, coulomb_k=p.coulomb_k,
                    elec=p.elec, kmax2=p.kmax2, lj_lrc=p.lj_lrc, cutoff_mode=getattr(p, "cutoff_mode", 0))


def _arrays(system):
    idx = np.ascontiguousarray(system.species_idx, dtype=np.int32)
    com = np.ascontiguousarray(system.com, dtype=np.float64)
    quat = np.ascontiguousarray(system.quat, dtype=np.float64)
    return idx, com, quat


def check(system) -> int:
    sp = species_array(system.species)
    p = params_struct(system.params)
    return lib().or_check(sp, len(system.species), ctypes.byref(p))


def forces(system):
    """Explicit pair sum: (force[n,3], torque[n,3], sums[NSUM])."""
    idx, com, quat = _arrays(system)
    n = idx.shape[0]
    f, t, s = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(NSUM)
    sp, p = species_array(system.species), params_struct(system.params)
    rc = lib().or_forces(sp, len(system.species), ctypes.byref(p), n,
                         idx.ctypes.data_as(ctypes.POINTER(c_int32)), _dp(com), _dp(quat),
                         _dp(f), _dp(t), _dp(s))
    if rc:
        raise ValueError(f"or_forces rejected its arguments ({rc})")
    return f, t, s


def kspace(system, f=None, t=None, s=None):
    """Ewald reciprocal space, accumulated into (f, t, s)."""
    idx, com, quat = _arrays(system)
    n = idx.shape[0]
    f = np.zeros((n, 3)) if f is None else f
    t = np.zeros((n, 3)) if t is None else t
    s = np.zeros(NSUM) if s is None else s
    sp, p = species_array(system.species), params_struct(system.params)
    rc = lib().or_kspace(sp, len(system.species), ctypes.byref(p), n,
                         idx.ctypes.data_as(ctypes.POINTER(c_int32)), _dp(com), _dp(quat),
                         _dp(f), _dp(t), _dp(s))
    if rc:
        raise ValueError(f"or_kspace rejected its arguments ({rc})")
    return f, t, s


def evaluate(system):
    """Full force/energy evaluation: explicit pairs, plus k-space with Ewald."""
    f, t, s = forces(system)
    if system.params.elec == 2:
        kspace(system, f, t, s)
    return f, t, s


def sums_dict(s: np.ndarray) -> Dict[str, float]:
    return {k: float(v) for k, v in zip(SUM_NAMES, s)}


def total_energy(s: np.ndarray) -> float:
    return float(s[0] + s[1] + s[2] + s[3] + s[4])


def rdf_ntypes(species) -> int:
    sp = species_array(species)
    return lib().or_rdf_ntypes(sp, len(species))


def md(system, md_settings=None, want_log: bool = True):
    """Run the integrator in place on a copy of `system`; returns a dict with
    the final state, the per-step energy log and the sampled accumulators."""
    st = system.copy()
    m = md_settings or st.md
    idx, com, quat = _arrays(st)
    n = idx.shape[0]
    vel = np.ascontiguousarray(st.vel, dtype=np.float64).copy()
    omega = np.ascontiguousarray(st.omega, dtype=np.float64).copy()
    com, quat = com.copy(), quat.copy()
    log = np.zeros((m.n_steps + 1, LOG_COLS)) if want_log else None
    moments = np.zeros(len(MOMENT_NAMES))
    T = rdf_ntypes(st.species)
    rdf = np.zeros((T * (T + 1) // 2, max(m.rdf_bins, 1)))
    nlag = max(m.acf_nlag, 1)
    acf_v, acf_j, acf_c = np.zeros(nlag), np.zeros(nlag), np.zeros(nlag)
    res_acf, res_cnt, solv = np.zeros(nlag), np.zeros(nlag), np.zeros(2)
    acf_q, acf_q_cnt = np.zeros(nlag), np.zeros(nlag)
    hp = np.zeros(len(st.species))
    if getattr(m, "h_partial", None) is not None:
        hp[:] = np.asarray(m.h_partial, dtype=np.float64)
    cfg = OrMD(integrator=m.integrator, n_steps=m.n_steps, dt=m.dt, temperature=m.temperature,
               sample_every=m.sample_every, rdf_every=m.rdf_every, rdf_bins=m.rdf_bins,
               acf_every=m.acf_every, acf_origin_every=m.acf_origin_every, acf_nlag=m.acf_nlag,
               rdf_rmax=m.rdf_rmax, u0=m.u0, res_solute=getattr(m, "res_solute", -1),
               res_solvent=getattr(m, "res_solvent", -1), res_radius=getattr(m, "res_radius", 0.0),
               res_tolerance=getattr(m, "res_tolerance", 0), heat_flux=1 if getattr(m, "heat_flux", False) else 0,
               h_partial=_dp(hp))
    sp, p = species_array(st.species), params_struct(st.params)
    rc = lib().or_md(sp, len(st.species), ctypes.byref(p), ctypes.byref(cfg), n,
                     idx.ctypes.data_as(ctypes.POINTER(c_int32)), _dp(com), _dp(quat), _dp(vel),
                     _dp(omega), _dp(log), _dp(moments), _dp(rdf), _dp(acf_v), _dp(acf_j), _dp(acf_c),
                     _dp(res_acf), _dp(res_cnt), _dp(solv), _dp(acf_q), _dp(acf_q_cnt))
    if rc:
        raise ValueError(f"or_md rejected its arguments ({rc})")
    st.com, st.quat, st.vel, st.omega = com, quat, vel, omega
    return {"state": st, "log": log, "moments": moments, "rdf": rdf,
            "acf_v": acf_v, "acf_j": acf_j, "acf_cnt": acf_c, "res_acf": res_acf, "res_cnt": res_cnt,
            "solvation_sum": solv[0], "solvation_cnt": solv[1], "acf_q": acf_q, "acf_q_cnt": acf_q_cnt}


def heat_flux(system, vel=None, omega=None, h_partial=None) -> np.ndarray:
    """Heat flux J_q (Sec. 5, Eq. 6) of one state: vel [n,3] lab, omega
    [n,3] body frame (default: the system's), h_partial per species."""
    idx, com, quat = _arrays(system)
    v = np.ascontiguousarray(system.vel if vel is None else vel, dtype=np.float64)
    w = np.ascontiguousarray(system.omega if omega is None else omega, dtype=np.float64)
    hp = np.zeros(len(system.species)) if h_partial is None else np.ascontiguousarray(h_partial, dtype=np.float64)
    jq = np.zeros(3)
    sp, p = species_array(system.species), params_struct(system.params)
    rc = lib().or_heat_flux(sp, len(system.species), ctypes.byref(p), idx.shape[0],
                            idx.ctypes.data_as(ctypes.POINTER(c_int32)), _dp(com), _dp(quat), _dp(v), _dp(w),
                            _dp(hp), _dp(jq))
    if rc:
        raise ValueError(f"or_heat_flux rejected its arguments ({rc})")
    return jq

"""Thin ctypes binding of libms2.so (include/ms2.h).

Argument marshalling only: every step of the force/energy path runs in the
HIP kernels of the library.  Torch is used for device memory and streams.
The binding raises if the compiled library is missing or no HIP device is
present; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libms2.so")

MAX_SITES = 8
MAX_SPECIES = 8
NOALLOC_MAX_MOL = 4096
NSUM = 12
SUM_NAMES = ["u_lj", "u_elec", "u_recip", "u_const", "u_lrc", "virial", "us", "uss",
             "us_lrc", "uss_lrc", "npair", "nsite"]
FP64, FP32 = 0, 1
STEP_GRAPH = 1
STEP_TIMING = 2
STEP_PREPARE = 4
BATCH_PLAIN_TILES = 1
STATUS = {0: "MS2_OK", 1: "MS2_EINVAL", 2: "MS2_ENOMEM", 3: "MS2_EDEVICE", 4: "MS2_ENONFINITE",
          5: "MS2_EFULL"}

c_double, c_int32, c_int64, c_size_t, c_void_p = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                                                  ctypes.c_size_t, ctypes.c_void_p)
P = ctypes.POINTER


class Species(ctypes.Structure):
    _fields_ = [("n_sites", c_int32), ("type", c_int32 * MAX_SITES),
                ("pos", (c_double * 3) * MAX_SITES), ("axis", (c_double * 3) * MAX_SITES),
                ("sigma", c_double * MAX_SITES), ("eps", c_double * MAX_SITES),
                ("mag", c_double * MAX_SITES), ("mass", c_double), ("inertia", c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("box", c_double), ("rc", c_double), ("eps_rf", c_double), ("alpha", c_double),
                ("coulomb_k", c_double), ("elec", c_int32), ("kmax2", c_int32), ("lj_lrc", c_int32),
                ("precision", c_int32), ("cutoff_mode", c_int32), ("pad", c_int32)]


class System(ctypes.Structure):
    _fields_ = [("params", Params), ("n_mol", c_int32), ("integrator", c_int32), ("n_steps", c_int64),
                ("dt", c_double), ("temperature", c_double), ("sample_every", c_int32),
                ("rdf_every", c_int32), ("rdf_bins", c_int32), ("acf_every", c_int32),
                ("acf_origin_every", c_int32), ("acf_nlag", c_int32), ("rdf_rmax", c_double),
                ("u0", c_double), ("res_enable", c_int32), ("res_solute", c_int32),
                ("res_solvent", c_int32), ("res_tolerance", c_int32), ("res_radius", c_double),
                ("heat_flux", c_int32), ("hf_pad", c_int32), ("h_partial", c_double * MAX_SPECIES),
                ("h_species", P(c_int32)), ("h_com", P(c_double)),
                ("h_quat", P(c_double)), ("h_vel", P(c_double)), ("h_omega", P(c_double))]


class Samples(ctypes.Structure):
    _fields_ = [("steps_done", c_int64), ("status", c_int32), ("rdf_ntypes", c_int32),
                ("sums", c_double * NSUM), ("ekin_trans", c_double), ("ekin_rot", c_double),
                ("pairs_total", c_double), ("site_pairs_total", c_double), ("moments", c_double * 11),
                ("solvation_sum", c_double), ("solvation_cnt", c_double), ("h_rdf", P(c_double)),
                ("h_acf_v", P(c_double)), ("h_acf_j", P(c_double)), ("h_acf_cnt", P(c_double)),
                ("h_res_acf", P(c_double)), ("h_res_cnt", P(c_double)), ("h_acf_q", P(c_double)),
                ("h_acf_q_cnt", P(c_double)), ("h_com", P(c_double)),
                ("h_quat", P(c_double)), ("h_vel", P(c_double)), ("h_omega", P(c_double)),
                ("h_force", P(c_double)), ("h_torque", P(c_double))]


class MS2Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

EXPORTED = ["ms2_create", "ms2_destroy", "ms2_forces", "ms2_ewald_kspace", "ms2_batch_create",
            "ms2_batch_destroy", "ms2_slot_footprint", "ms2_slot_admit", "ms2_slot_retire",
            "ms2_step", "ms2_sample", "ms2_slot_status", "ms2_tile_config", "ms2_set_tile_config",
            "ms2_autotune", "ms2_batch_timing", "ms2_massieu", "ms2_massieu_properties",
            "ms2_device_errors", "ms2_forces_noalloc", "ms2_last_error"]


def lib():
    """Load libms2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1507_07548_amd.build.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = c_void_p, P(c_double), P(c_int32)
        L.ms2_create.argtypes = [P(vp), P(Species), c_int32, c_int32]
        L.ms2_destroy.argtypes = [vp]
        L.ms2_destroy.restype = None
        for fn in (L.ms2_forces, L.ms2_ewald_kspace, L.ms2_forces_noalloc):
            fn.argtypes = [vp, P(Params), c_int32, vp, vp, vp, vp, vp, vp, vp]
        L.ms2_device_errors.argtypes = [vp, vp]
        L.ms2_batch_create.argtypes = [vp, c_int32, c_size_t, c_int32, P(vp)]
        L.ms2_batch_timing.argtypes = [vp, P(c_double), P(c_int32)]
        L.ms2_batch_destroy.argtypes = [vp]
        L.ms2_batch_destroy.restype = None
        L.ms2_slot_footprint.argtypes = [vp, P(System), P(c_size_t)]
        L.ms2_slot_admit.argtypes = [vp, P(System), P(c_int32), vp]
        L.ms2_slot_retire.argtypes = [vp, c_int32]
        L.ms2_step.argtypes = [vp, c_int32, c_int32, vp]
        L.ms2_sample.argtypes = [vp, c_int32, P(Samples), vp]
        L.ms2_slot_status.argtypes = [vp, c_int32, P(c_int64), P(c_int32), vp]
        L.ms2_tile_config.argtypes = [vp, c_int32, c_int32, c_int32, P(c_int32), P(c_int32)]
        L.ms2_set_tile_config.argtypes = [vp, c_int32, c_int32, c_int32, c_int32, c_int32]
        L.ms2_autotune.argtypes = [vp, c_int32, c_int32, c_int32, P(c_double), c_int32, P(c_int32), vp]
        L.ms2_massieu.argtypes = [dp, c_double, c_double, c_double, c_int32, dp]
        L.ms2_massieu_properties.argtypes = [dp, c_double, dp]
        L.ms2_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("ms2_destroy", "ms2_batch_destroy", "ms2_last_error"):
                getattr(L, name).restype = c_int32
        _lib = L
    return _lib


def check(status: int):
    if status != 0:
        raise MS2Error(status, lib().ms2_last_error().decode())


def species_array(species) -> ctypes.Array:
    """Marshal a list of inputs.Species into ms2_species[]."""
    arr = (Species * len(species))()
    for k, s in enumerate(species):
        o = arr[k]
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


def params_struct(p, precision: int) -> Params:
    return Params(box=p.box, rc=p.rc, eps_rf=p.eps_rf, alpha=p.alpha, coulomb_k=p.coulomb_k,
                  elec=p.elec, kmax2=p.kmax2, lj_lrc=p.lj_lrc, precision=precision,
                  cutoff_mode=getattr(p, "cutoff_mode", 0))


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """ms2_ctx: a species table on one HIP device."""

    def __init__(self, species: Sequence, device: int = 0):
        self.species = list(species)
        self._arr = species_array(self.species)
        h = c_void_p()
        check(lib().ms2_create(ctypes.byref(h), self._arr, len(self.species), device))
        self.handle = h
        self.device = device
        # shared with this context's batches: ms2_destroy frees every batch of
        # the context, after which a batch must not free itself again
        self._alive = [True]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._alive[0] = False
            lib().ms2_destroy(self.handle)     # also destroys its remaining batches
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forces(self, params: Params, n: int, species, com, quat, force, torque, sums, stream=None):
        """ms2_forces on torch device tensors (SoA layouts of include/ms2.h)."""
        check(lib().ms2_forces(self.handle, ctypes.byref(params), n, species.data_ptr(), com.data_ptr(),
                               quat.data_ptr(), force.data_ptr(), torque.data_ptr(), sums.data_ptr(),
                               _stream_ptr(stream)))

    def forces_noalloc(self, params: Params, n: int, species, com, quat, force, torque, sums, stream=None):
        """ms2_forces_noalloc: ms2_forces with its scratch in the library's
        static device array (n <= MS2_NOALLOC_MAX_MOL)."""
        check(lib().ms2_forces_noalloc(self.handle, ctypes.byref(params), n, species.data_ptr(),
                                       com.data_ptr(), quat.data_ptr(), force.data_ptr(), torque.data_ptr(),
                                       sums.data_ptr(), _stream_ptr(stream)))

    def ewald_kspace(self, params: Params, n: int, species, com, quat, force, torque, sums, stream=None):
        check(lib().ms2_ewald_kspace(self.handle, ctypes.byref(params), n, species.data_ptr(),
                                     com.data_ptr(), quat.data_ptr(), force.data_ptr(), torque.data_ptr(),
                                     sums.data_ptr(), _stream_ptr(stream)))

    def device_errors(self, stream=None):
        """ms2_device_errors: raises MS2Error if a call recorded a species
        index outside the table since the last check (and clears it)."""
        check(lib().ms2_device_errors(self.handle, _stream_ptr(stream)))

    def tile_config(self, n: int, precision: int, mode: int = 1):
        w, j = c_int32(), c_int32()
        check(lib().ms2_tile_config(self.handle, mode, n, precision, ctypes.byref(w), ctypes.byref(j)))
        return w.value, j.value

    def set_tile_config(self, n: int, precision: int, waves: int, jchunk: int, mode: int = 1):
        check(lib().ms2_set_tile_config(self.handle, mode, n, precision, waves, jchunk))

    def autotune(self, precision: int, n_lo: int, n_hi: int, stream=None):
        """Runs the library's autotuner; returns rows (mode, n, waves, jchunk, us per system)."""
        cap = 512
        rep = np.zeros((cap, 5))
        cnt = c_int32()
        check(lib().ms2_autotune(self.handle, precision, n_lo, n_hi, rep.ctypes.data_as(P(c_double)), cap,
                                 ctypes.byref(cnt), _stream_ptr(stream)))
        return rep[: cnt.value]


class DeviceSystem:
    """Device-resident SoA copies of one system's inputs and outputs."""

    def __init__(self, system, device: str = "cuda:0"):
        import torch
        self.n = system.n
        self.species = torch.tensor(np.ascontiguousarray(system.species_idx, dtype=np.int32), device=device)
        self.com = torch.tensor(np.ascontiguousarray(system.com.T), dtype=torch.float64, device=device)
        self.quat = torch.tensor(np.ascontiguousarray(system.quat.T), dtype=torch.float64, device=device)
        self.force = torch.zeros((3, self.n), dtype=torch.float64, device=device)
        self.torque = torch.zeros((3, self.n), dtype=torch.float64, device=device)
        self.sums = torch.zeros(NSUM, dtype=torch.float64, device=device)


def evaluate(ctx: Context, system, precision: int = FP64, dev: Optional[DeviceSystem] = None,
             stream=None):
    """One full force/energy evaluation of `system` on the GPU (ms2_forces,
    plus ms2_ewald_kspace with Ewald).  Returns numpy (force[n,3],
    torque[n,3], sums[NSUM])."""
    import torch
    d = dev or DeviceSystem(system)
    p = params_struct(system.params, precision)
    ctx.forces(p, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums, stream)
    if system.params.elec == 2:
        ctx.ewald_kspace(p, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums, stream)
    torch.cuda.synchronize()
    return d.force.cpu().numpy().T.copy(), d.torque.cpu().numpy().T.copy(), d.sums.cpu().numpy().copy()


def system_struct(system, precision: int, n_steps: Optional[int] = None):
    """Marshal an inputs.System (+ its MDSettings) into ms2_system.  Returns
    (struct, keep-alive host arrays)."""
    md = system.md
    sp = np.ascontiguousarray(system.species_idx, dtype=np.int32)
    com = np.ascontiguousarray(system.com.T, dtype=np.float64)
    quat = np.ascontiguousarray(system.quat.T, dtype=np.float64)
    vel = np.ascontiguousarray(system.vel.T, dtype=np.float64)
    om = np.ascontiguousarray(system.omega.T, dtype=np.float64)
    keep = (sp, com, quat, vel, om)
    dp = lambda a: a.ctypes.data_as(P(c_double))
    s = System(params=params_struct(system.params, precision), n_mol=system.n, integrator=md.integrator,
               n_steps=md.n_steps if n_steps is None else n_steps, dt=md.dt, temperature=md.temperature,
               sample_every=md.sample_every, rdf_every=md.rdf_every, rdf_bins=md.rdf_bins,
               acf_every=md.acf_every, acf_origin_every=md.acf_origin_every, acf_nlag=md.acf_nlag,
               rdf_rmax=md.rdf_rmax, u0=md.u0, res_enable=1 if md.res_solute >= 0 else 0,
               res_solute=max(md.res_solute, 0), res_solvent=max(md.res_solvent, 0),
               res_radius=md.res_radius, res_tolerance=md.res_tolerance,
               heat_flux=1 if md.heat_flux else 0,
               h_partial=(c_double * MAX_SPECIES)(*(list(md.h_partial or ()) + [0.0] * MAX_SPECIES)[:MAX_SPECIES]),
               h_species=sp.ctypes.data_as(P(c_int32)), h_com=dp(com),
               h_quat=dp(quat), h_vel=dp(vel), h_omega=dp(om))
    return s, keep


class Batch:
    """ms2_batch: device-resident slots advanced together by ms2_step."""

    def __init__(self, ctx: Context, max_slots: int, hbm_budget: int = 0, plain_tiles: bool = False):
        self.ctx = ctx
        h = c_void_p()
        check(lib().ms2_batch_create(ctx.handle, max_slots, hbm_budget,
                                     BATCH_PLAIN_TILES if plain_tiles else 0, ctypes.byref(h)))
        self.handle = h
        self.shapes = {}
        self._ctx_alive = ctx._alive

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value and self._ctx_alive[0]:
            lib().ms2_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, system, precision: int) -> int:
        s, keep = system_struct(system, precision)
        b = c_size_t()
        check(lib().ms2_slot_footprint(self.ctx.handle, ctypes.byref(s), ctypes.byref(b)))
        return b.value

    def admit(self, system, precision: int, n_steps: Optional[int] = None, stream=None) -> int:
        s, keep = system_struct(system, precision, n_steps)
        slot = c_int32()
        check(lib().ms2_slot_admit(self.handle, ctypes.byref(s), ctypes.byref(slot), _stream_ptr(stream)))
        self.shapes[slot.value] = (system.n, system.md.rdf_bins, max(system.md.acf_nlag, 0),
                                   len(system.species))
        return slot.value

    def retire(self, slot: int):
        check(lib().ms2_slot_retire(self.handle, slot))
        self.shapes.pop(slot, None)

    def step(self, n_steps: int, graph: bool = True, timing: bool = False, prepare: bool = False,
             stream=None):
        flags = (STEP_GRAPH if graph else 0) | (STEP_TIMING if timing else 0) | (STEP_PREPARE if prepare else 0)
        check(lib().ms2_step(self.handle, n_steps, flags, _stream_ptr(stream)))

    def pair_time_ms(self):
        """(summed pair-kernel milliseconds, steps) of the last timed step call."""
        ms, k = c_double(), c_int32()
        check(lib().ms2_batch_timing(self.handle, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    def status(self, slot: int, stream=None):
        steps, st = c_int64(), c_int32()
        check(lib().ms2_slot_status(self.handle, slot, ctypes.byref(steps), ctypes.byref(st),
                                    _stream_ptr(stream)))
        return steps.value, st.value

    def sample(self, slot: int, state: bool = True, stream=None) -> dict:
        n, bins, nlag, _ = self.shapes[slot]
        out = Samples()
        arrays = {}

        def buf(name, shape):
            a = np.zeros(shape, dtype=np.float64)
            arrays[name] = a
            setattr(out, "h_" + name, a.ctypes.data_as(P(c_double)))

        T = sum(1 for s in self.ctx.species for site in s.sites if site.kind == 0)
        if bins:
            buf("rdf", (T * (T + 1) // 2, bins))
        if nlag:
            buf("acf_v", nlag)
            buf("acf_j", nlag)
            buf("acf_cnt", nlag)
            buf("res_acf", nlag)
            buf("res_cnt", nlag)
            buf("acf_q", nlag)
            buf("acf_q_cnt", nlag)
        if state:
            buf("com", (3, n))
            buf("quat", (4, n))
            buf("vel", (3, n))
            buf("omega", (3, n))
            buf("force", (3, n))
            buf("torque", (3, n))
        check(lib().ms2_sample(self.handle, slot, ctypes.byref(out), _stream_ptr(stream)))
        res = {"steps_done": out.steps_done, "status": out.status, "sums": np.array(out.sums[:]),
               "ekin_trans": out.ekin_trans, "ekin_rot": out.ekin_rot, "moments": np.array(out.moments[:]),
               "pairs_total": out.pairs_total, "site_pairs_total": out.site_pairs_total,
               "solvation_sum": out.solvation_sum, "solvation_cnt": out.solvation_cnt}
        for k, v in arrays.items():
            res[k] = v.T.copy() if k in ("com", "quat", "vel", "omega", "force", "torque") else v
        return res


# --------------------------------------------------------------------------
# Massieu-potential derivatives (Sec. 3, Eq. 1)
# --------------------------------------------------------------------------
AR_ORDER = ("10", "01", "20", "11", "02", "30", "21", "12")
PROP_ORDER = ("Z", "u_kT", "cv_k", "cp_k", "dpdrho_kT", "dpdT_rhok", "w2_m_kT", "rho_kT_kappaT")


def massieu(moments, u0: float, temperature: float, volume: float, n_mol: int) -> dict:
    """The eight residual derivatives A^r_mn from a slot's moment sums."""
    m = (c_double * 11)(*[float(x) for x in moments])
    out = (c_double * 8)()
    check(lib().ms2_massieu(m, float(u0), float(temperature), float(volume), int(n_mol), out))
    return dict(zip(AR_ORDER, list(out)))


def massieu_properties(a_r: dict, dof: float) -> dict:
    """Thermodynamic properties per molecule (k = 1) from the residual
    derivatives and the ideal part of rigid molecules with `dof` quadratic
    degrees of freedom."""
    a = (c_double * 8)(*[float(a_r[k]) for k in AR_ORDER])
    out = (c_double * 8)()
    check(lib().ms2_massieu_properties(a, float(dof), out))
    return dict(zip(PROP_ORDER, list(out)))

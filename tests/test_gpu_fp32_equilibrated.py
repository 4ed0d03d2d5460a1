"""The precision form (FP32 site arithmetic, FP64 sums) against the FP64
oracle on disordered states: every state here was produced by the oracle's
own integrator from the seeded starts (tests/golden/make_oracle_runs.py), so
no input comes from the GPU.

Energies are normalised by |U| and each volume-derivative sum by its own
magnitude; forces and torques by their rms over the molecules.

Error model (from the arithmetic).  A site-pair term in FP32 carries a
relative rounding error of a few u = 2^-24 = 6e-8 times its condition
number: r^-12 multiplies the error of r^2 by 6, u' / r by 7 (an LJ site
pair's |r|^2 is formed from |R|^2 rounded once, so it carries about one
rounding).
These errors have random signs, so a sum S = sum_p s_p of M such terms is
off by about u * kappa * sqrt(sum_p s_p^2), which is small against
sum_p |s_p| but is divided by |S|: the cancellation ratio
C = sum_p |s_p| / |S| sets the relative error of each sum.
  * U of the LJ + quadrupole fluids (C ~ 3): measured 4e-10 .. 1e-8 of |U|
    (larger at low density, where U is small);
  * U of water + ions: the nine charge-charge terms of two neutral
    molecules cancel to ~1e-3 of their magnitudes (C ~ 250), which makes
    ~5e-8 the floor of FP32 site arithmetic (measured 5.7e-8; 1e-7 asserted);
  * the virial W = -U_s cancels between repulsive and attractive pairs
    (C = 11 for the dense fluid, 45 at rho = 0.33): 2e-8 .. 5e-7 of |W|.
The coefficients themselves (c6, c12 and k_e m_a m_b) are rounded once
from FP64, so no error is common to every pair of a kind beyond that one
rounding (for the quadrupole fluid k_e Q^2 = 2 is exact).
Counters (accepted molecule pairs, site pairs) are exact: the cut-off
decision is taken in FP64 on both sides.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1507_07548_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1507_07548_amd import ms2  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U_SLOTS = [0, 1, 2, 3, 4]
W, US, USS, NPAIR, NSITE = 5, 6, 7, 10, 11


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def state(name, make):
    z = np.load(os.path.join(GOLDEN, "oracle_equilibrated.npz"))
    s = make()
    s.com = z[name + "_com"].copy()
    s.quat = z[name + "_quat"].copy()
    return s


MODELS = {
    "quad": lambda: I.quadrupolar_fluid(),
    "quad_lo": lambda: I.batched_state_point(9),
    "ionic": lambda: I.ionic_solution(),
    "lj": lambda: I.lj_fluid(),
}

# (|dU|/|U|, |dW|/|W| and |dU_s|/|U_s|, |dU_ss|/|U_ss|) asserted per state
TOL = {
    "quad": (2e-9, 2e-7, 2e-8),
    "quad_lo": (2e-8, 1e-6, 1e-7),
    "ionic": (1e-7, 5e-7, 1e-7),
    "lj": (1e-8, 2e-7, 5e-8),
}


@pytest.mark.parametrize("name", sorted(MODELS))
def test_fp32_parity_on_oracle_equilibrated_state(name):
    s = state(name, MODELS[name])
    say(f"[gpu] fp32 vs oracle on the oracle-equilibrated state {name} (n={s.n})")
    fo, to, so = oracle.evaluate(s)
    ctx = ms2.Context(s.species)
    f, t, su = ms2.evaluate(ctx, s, ms2.FP32)
    ctx.close()
    assert su[NPAIR] == so[NPAIR] and su[NSITE] == so[NSITE]
    rms_f = np.sqrt((fo ** 2).sum(1).mean())
    ef = np.abs(f - fo).max() / rms_f
    rms_t = np.sqrt((to ** 2).sum(1).mean())
    et = np.abs(t - to).max() / rms_t if rms_t > 0 else np.abs(t).max()
    U, Uo = su[U_SLOTS].sum(), so[U_SLOTS].sum()
    eu = abs(U - Uo) / abs(Uo)
    ew = abs(su[W] - so[W]) / abs(so[W])
    es = abs(su[US] - so[US]) / abs(so[US])
    ess = abs(su[USS] - so[USS]) / abs(so[USS])
    say(f"  |dU|/|U| {eu:.2e}  |dW|/|W| {ew:.2e}  |dUs|/|Us| {es:.2e}  |dUss|/|Uss| {ess:.2e}  "
        f"max|dF|/rms {ef:.2e}  max|dT|/rms {et:.2e}")
    tu, tw, tss = TOL[name]
    assert ef < 1e-5 and et < 1e-5
    assert eu <= tu
    assert ew <= tw and es <= tw
    assert ess <= tss


def block_stats(per_block):
    a = np.asarray(per_block, dtype=float)
    return a.mean(0), a.std(0, ddof=1) / np.sqrt(len(a))


def test_fp32_nvt_ensemble_averages_match_the_oracle():
    """2CLJQ fluid, 1000 molecules, rho 0.6, T 2: 1000 Gear NVT steps in FP32
    on the GPU against the oracle's FP64 run from the same start.  The
    trajectories part after a few hundred steps (chaos); their averages of
    U/N, dU/dV (the virial route to the pressure), d2U/dV2 and the residual
    Massieu derivatives A^r_10, A^r_01, A^r_20 (Sec. 3, Eq. 1) must agree
    within three standard errors of ten 100-step blocks."""
    z = np.load(os.path.join(GOLDEN, "oracle_quad_nvt_log.npz"))
    log, u0 = z["log"], float(z["u0"])
    s = I.quadrupolar_fluid(n_steps=1000, sample_every=1)
    s.md.u0 = u0
    V, n, T = s.params.box ** 3, s.n, s.md.temperature

    # oracle blocks from its energy log (rows 1..1000: after each step)
    def moments_of(rows):
        X = rows[:, 0] - u0
        Y = rows[:, 4] / (3.0 * V)
        Z = (rows[:, 5] - 2.0 * rows[:, 4]) / (9.0 * V * V)
        return np.array([len(rows), X.sum(), (X * X).sum(), (X ** 3).sum(), Y.sum(), (X * Y).sum(),
                         (X * X * Y).sum(), (Y * Y).sum(), (X * Y * Y).sum(), Z.sum(), (X * Z).sum()])

    mo_total = moments_of(log[1:])
    np.testing.assert_allclose(mo_total, z["moments"], rtol=1e-9, atol=1e-9 * np.abs(z["moments"]).max())

    def observables(m, massieu):
        a = massieu(m)
        return [u0 / n + m[1] / m[0] / n, m[4] / m[0], m[9] / m[0], a["10"], a["01"], a["20"]]

    from oracle import massieu as om
    o_blocks = []
    for b in range(10):
        m = moments_of(log[1 + 100 * b: 1 + 100 * (b + 1)])
        o_blocks.append(observables(m, lambda mm: om.residual_derivatives(mm, u0, T, V, n)))

    say("[gpu] 2CLJQ FP32 Gear NVT, 1000 steps in ten blocks")
    ctx = ms2.Context(s.species)
    b = ms2.Batch(ctx, 1)
    slot = b.admit(s, ms2.FP32)
    prev = np.zeros(11)
    g_blocks = []
    for k in range(10):
        b.step(100, graph=True)
        out = b.sample(slot, state=False)
        assert out["status"] == 0 and out["steps_done"] == 100 * (k + 1)
        m = out["moments"] - prev
        prev = out["moments"].copy()
        g_blocks.append(observables(m, lambda mm: ms2.massieu(mm, u0, T, V, n)))
    b.close()
    ctx.close()

    gm, gse = block_stats(g_blocks)
    om_, ose = block_stats(o_blocks)
    names = ["U/N", "dU/dV", "d2U/dV2", "A^r_10", "A^r_01", "A^r_20"]
    for k, nm in enumerate(names):
        bound = 3.0 * np.hypot(gse[k], ose[k])
        say(f"  {nm:8s} gpu {gm[k]: .6e} +- {gse[k]:.1e}  oracle {om_[k]: .6e} +- {ose[k]:.1e}  "
            f"|diff| {abs(gm[k] - om_[k]):.1e} (3 se {bound:.1e})")
        assert abs(gm[k] - om_[k]) <= bound, nm

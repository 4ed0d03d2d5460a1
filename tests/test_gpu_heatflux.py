"""GPU parity of the heat-flux autocorrelation (Sec. 5, Eqs. 5-6) against the
oracle: FP64 runs of 2CLJQ (Gear, quadrupoles), Stockmayer with reaction
field and partial enthalpies (Gear, dipoles), and one-site LJ (velocity
Verlet).  FP64 trajectories agree to ~1e-12 and the flux is a sum of terms of
both signs, so the ACF sums agree to ~1e-9 relative to their first lag (the
tolerance below).  The FP32 form: pair terms carry ~1e-7 relative error each,
summed over ~1e5 pairs with cancellation; every lag within 1e-4 of the
first.  And alone = in a mix, bitwise."""
import numpy as np
import pytest

import oracle
from models import small_system
from paper_1507_07548_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1507_07548_amd import ms2  # noqa: E402


def say(*a):
    print(*a, flush=True)


def with_flux(s, n_steps=30, h=None):
    s.md.n_steps = n_steps
    s.md.acf_every, s.md.acf_origin_every, s.md.acf_nlag = 2, 6, 8
    s.md.heat_flux = True
    s.md.h_partial = h
    return s


def systems():
    a = with_flux(I.quadrupolar_fluid(n=300, density=0.6, n_steps=30, sample_every=0))
    sp = [I.stockmayer()]
    b = small_system(sp, 216, 7.2, 3.4, seed=5, elec=I.ELEC_RF, eps_rf=30.0)
    rng = np.random.default_rng(6)
    b.vel = I.maxwell_boltzmann(np.ones(216), 1.5, rng)
    b.omega = I.body_angular_velocities(np.array([sp[0].inertia] * 216), 1.5, rng)
    b.md = I.MDSettings(integrator=I.GEAR, dt=0.001, temperature=1.5)
    b = with_flux(b, h=(2.5,))
    c = with_flux(I.lj_fluid(n=500, n_steps=30))
    return {"2cljq_gear": a, "stockmayer_rf_gear": b, "lj_vv": c}


def run(system, precision):
    ctx = ms2.Context(system.species)
    b = ms2.Batch(ctx, 2)
    slot = b.admit(system, precision)
    b.step(system.md.n_steps)
    out = b.sample(slot, state=False)
    b.close()
    return out


@pytest.mark.parametrize("name", ["2cljq_gear", "stockmayer_rf_gear", "lj_vv"])
def test_heat_flux_acf_matches_the_oracle_fp64(name):
    s = systems()[name]
    say(f"[gpu] heat-flux ACF, {name}, n={s.n}, {s.md.n_steps} steps fp64")
    o = oracle.md(s, want_log=False)
    g = run(s, ms2.FP64)
    say(f"  acf_q[0..3] gpu {g['acf_q'][:4]} oracle {o['acf_q'][:4]}")
    np.testing.assert_array_equal(g["acf_q_cnt"], o["acf_q_cnt"])
    assert o["acf_q_cnt"][0] > 0 and o["acf_q"][0] > 0
    np.testing.assert_allclose(g["acf_q"], o["acf_q"], rtol=0, atol=1e-9 * o["acf_q"][0])


@pytest.mark.parametrize("name", ["2cljq_gear", "stockmayer_rf_gear", "lj_vv"])
def test_heat_flux_acf_fp32_every_lag(name):
    """FP32 site arithmetic against the FP64 oracle at every lag of the 30-step
    run.  J_q's pair part (Sec. 5, Eq. 6) is a sum of terms of both signs
    whose magnitudes exceed the sum by C ~ 1e2; each FP32 term carries a
    few 1e-7 of itself, so J_q is good to ~1e-5 relative, an ACF value (a
    product of two fluxes averaged over origins) to twice that, and the
    trajectory itself, integrated with FP32 forces, departs from the FP64
    one by ~1e-6 over 30 steps: every lag within 1e-4 of acf(0)."""
    s = systems()[name]
    say(f"[gpu] heat-flux ACF, {name}, fp32 vs fp64 oracle, {s.md.n_steps} steps")
    o = oracle.md(s, want_log=False)
    g = run(s, ms2.FP32)
    np.testing.assert_array_equal(g["acf_q_cnt"], o["acf_q_cnt"])
    err = np.abs(g["acf_q"] - o["acf_q"]) / o["acf_q"][0]
    say(f"  max over lags |d acf| / acf(0) {err.max():.2e}; per lag {np.array2string(err, precision=1)}")
    assert err.max() < 1e-4


def test_heat_flux_alone_and_in_a_mix_are_identical():
    s = systems()["stockmayer_rf_gear"]
    other = small_system([I.stockmayer()], 300, 8.0, 3.8, seed=9, elec=I.ELEC_RF, eps_rf=30.0)
    other.md = I.MDSettings(integrator=I.GEAR, dt=0.001, temperature=1.2, n_steps=40)
    say("[gpu] heat flux alone vs in a mix")
    ra = run(s, ms2.FP32)
    ctx = ms2.Context(s.species)
    mix = ms2.Batch(ctx, 3)
    mix.admit(other, ms2.FP32)
    sl = mix.admit(s, ms2.FP32)
    mix.step(10)
    mix.step(20, graph=False)
    rm = mix.sample(sl, state=False)
    for k in ("acf_q", "acf_q_cnt", "acf_v", "sums"):
        assert np.array_equal(ra[k], rm[k]), k

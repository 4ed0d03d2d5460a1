"""GPU parity of the residence-time and solvation-number sampler (Sec. 5,
Eqs. 7-8) against the oracle: hand-derived occupancy windows (exact), a
static lattice, and an Ewald water + ions run (FP64 trajectories agree to
~1e-12, so every shell decision agrees; the correlation sums differ only in
the order of their additions: 1e-12 relative); residence results identical
alone and in a mix; and a finished slot takes no further RDF samples while
others keep running."""
import numpy as np
import pytest

import oracle
from paper_1507_07548_amd import inputs as I
from residence_cases import BALLISTIC_EXPECTED, BALLISTIC_SOLVATION, ballistic_system, fcc_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1507_07548_amd import ms2  # noqa: E402


def say(*a):
    print(*a, flush=True)


def run_alone(system, precision=ms2.FP64, steps=None, graph=True):
    ctx = ms2.Context(system.species)
    b = ms2.Batch(ctx, 2)
    slot = b.admit(system, precision)
    b.step(steps or system.md.n_steps, graph=graph)
    out = b.sample(slot, state=False)
    b.close()
    return out


@pytest.mark.parametrize("tol", [3, 2])
def test_ballistic_windows_on_the_gpu(tol):
    say(f"[gpu] residence, ballistic windows, tolerance {tol}")
    g = run_alone(ballistic_system(tol))
    np.testing.assert_allclose(g["res_acf"], BALLISTIC_EXPECTED[tol]["res_acf"], rtol=1e-15, atol=0)
    np.testing.assert_array_equal(g["res_cnt"], BALLISTIC_EXPECTED[tol]["res_cnt"])
    assert (g["solvation_sum"], g["solvation_cnt"]) == BALLISTIC_SOLVATION


def test_static_fcc_on_the_gpu():
    say("[gpu] residence, static FCC lattice")
    g = run_alone(fcc_system())
    assert (g["solvation_sum"], g["solvation_cnt"]) == (48.0, 4.0)
    np.testing.assert_array_equal(g["res_cnt"], [4, 3, 2])
    np.testing.assert_array_equal(g["res_acf"], [4, 3, 2])


def ionic_residence(seed=3, n_steps=40):
    s = I.ionic_solution(n_steps=n_steps, rdf_every=0, seed=seed)
    s.md.acf_every, s.md.acf_origin_every, s.md.acf_nlag = 2, 10, 10
    s.md.res_solute, s.md.res_solvent, s.md.res_radius, s.md.res_tolerance = 1, 0, 3.5, 2
    return s


def test_ionic_solution_residence_matches_the_oracle():
    s = ionic_residence()
    say(f"[gpu] residence, water + ions (Ewald), cation shells of radius 3.5 A, {s.md.n_steps} steps fp64")
    o = oracle.md(s, want_log=False)
    g = run_alone(s)
    say(f"  solvation {g['solvation_sum'] / g['solvation_cnt']:.4f} (oracle {o['solvation_sum'] / o['solvation_cnt']:.4f})")
    assert g["solvation_sum"] == o["solvation_sum"] and g["solvation_cnt"] == o["solvation_cnt"]
    np.testing.assert_array_equal(g["res_cnt"], o["res_cnt"])
    np.testing.assert_allclose(g["res_acf"], o["res_acf"], rtol=1e-12)
    assert o["res_cnt"][0] > 0 and o["solvation_sum"] > 0


def test_residence_alone_and_in_a_mix_are_identical():
    a = ionic_residence(seed=3)
    other = ionic_residence(seed=11, n_steps=60)
    say("[gpu] residence alone vs in a mix")
    ra = run_alone(a)
    ctx = ms2.Context(a.species)
    mix = ms2.Batch(ctx, 3)
    mix.admit(other, ms2.FP64)
    sa = mix.admit(a, ms2.FP64)
    mix.step(20)
    mix.step(40, graph=False)
    rm = mix.sample(sa, state=False)
    for k in ("res_acf", "res_cnt", "moments", "sums"):
        assert np.array_equal(ra[k], rm[k]), k
    assert (ra["solvation_sum"], ra["solvation_cnt"]) == (rm["solvation_sum"], rm["solvation_cnt"])


def test_a_finished_slot_takes_no_further_rdf_samples():
    # the slot ends on an RDF step; the batch keeps stepping
    s = I.ionic_solution(n_steps=20, rdf_every=10)
    say("[gpu] RDF of a slot stepped past its budget")
    o = oracle.md(s, want_log=False)
    g = run_alone(s, steps=40)
    assert g["steps_done"] == 20
    np.testing.assert_array_equal(g["rdf"], o["rdf"])

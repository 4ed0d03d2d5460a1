"""ms2_forces_noalloc through the C ABI: the same result as ms2_forces with
its default tile shape (symmetric tile pairs), bit for bit, on two calls in a
row with the second one smaller; no device memory taken by the call; sizes
above the limit refused before anything is enqueued."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def outputs(d):
    torch.cuda.synchronize()
    return d.force.cpu().numpy().copy(), d.torque.cpu().numpy().copy(), d.sums.cpu().numpy().copy()


def fresh_outputs(d):
    d.force.fill_(np.nan)
    d.torque.fill_(np.nan)
    d.sums.fill_(np.nan)


def run_pair(systems, precision):
    """Both no-allocation calls first (the larger system, then the smaller),
    then ms2_forces on each; returns the four output triples."""
    ctx = ms2.Context(systems[0].species)
    for s in systems:
        # the untuned default: symmetric items, 1, 2 or 4 per tile pair by size
        # (on a 256-CU device: N = 4096 one, N = 1000 two)
        assert ctx.tile_config(s.n, precision, mode=0)[0] == 0
    devs = [ms2.DeviceSystem(s) for s in systems]
    p = [ms2.params_struct(s.params, precision) for s in systems]
    # a first launch loads the kernels' code objects (runtime memory, not
    # the call's): warm them up, and torch's fill and copy, on a tiny system
    tiny = I.quadrupolar_fluid(n=64, density=0.3)
    dt = ms2.DeviceSystem(tiny)
    fresh_outputs(dt)
    ctx.forces_noalloc(ms2.params_struct(tiny.params, precision), dt.n, dt.species, dt.com, dt.quat, dt.force,
                       dt.torque, dt.sums)
    outputs(dt)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = []
    for s, d, q in zip(systems, devs, p):
        say(f"[gpu] ms2_forces_noalloc n={s.n} precision={precision}")
        fresh_outputs(d)
        ctx.forces_noalloc(q, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums)
        got.append(outputs(d))
    free1 = torch.cuda.mem_get_info()[0]
    ref = []
    for s, d, q in zip(systems, devs, p):
        say(f"[gpu] ms2_forces n={s.n} precision={precision}")
        fresh_outputs(d)
        ctx.forces(q, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums)
        ref.append(outputs(d))
    ctx.device_errors()
    ctx.close()
    return got, ref, free0, free1


@pytest.mark.parametrize("precision", [ms2.FP32, ms2.FP64])
def test_noalloc_equals_forces_two_calls_second_smaller(precision):
    big = I.jittered(I.quadrupolar_fluid(n=ms2.NOALLOC_MAX_MOL, density=0.45), 0.1, seed=41)
    small = I.jittered(I.quadrupolar_fluid(n=1000, density=0.6), 0.1, seed=42)
    shapes = {s.n: ms2.Context(s.species).tile_config(s.n, precision, mode=0) for s in (big, small)}
    say(f"  default shapes {shapes}")
    got, ref, free0, free1 = run_pair([big, small], precision)
    for (fa, ta, sa), (fb, tb, sb) in zip(got, ref):
        assert np.array_equal(fa, fb) and np.array_equal(ta, tb) and np.array_equal(sa, sb)
        assert np.isfinite(fa).all() and np.isfinite(sa).all()
    # the no-allocation calls took no device memory
    assert free1 == free0, (free0, free1)
    # and the smaller system against the oracle (ms2_forces' own tolerance)
    fo, to, so = oracle.evaluate(small)
    rms = np.sqrt((fo ** 2).sum(1).mean())
    err = np.abs(got[1][0].T - fo).max() / rms
    say(f"  small system vs oracle: max|dF|/rms {err:.2e}")
    assert err < (1e-5 if precision == ms2.FP32 else 1e-11)
    assert got[1][2][10] == so[10] and got[1][2][11] == so[11]


def test_noalloc_ewald_real_space_and_ragged_tail():
    """Water + ions with the Ewald real-space terms (1000 molecules), then a
    ragged 130-molecule mixture: a tile of two molecules at the end."""
    from models import ionic_pair_species, small_system
    s1 = I.ionic_solution()
    s2 = small_system(ionic_pair_species(), 130, 8.0, 3.5, seed=3, elec=I.ELEC_EWALD, alpha=0.8, kmax2=20)
    for prec in (ms2.FP32, ms2.FP64):
        ctx = ms2.Context(s1.species)
        ctx2 = ms2.Context(s2.species)
        d1, d2 = ms2.DeviceSystem(s1), ms2.DeviceSystem(s2)
        p1, p2 = ms2.params_struct(s1.params, prec), ms2.params_struct(s2.params, prec)
        say(f"[gpu] ms2_forces_noalloc ionic n={s1.n} then mixture n={s2.n} precision={prec}")
        ctx.forces_noalloc(p1, d1.n, d1.species, d1.com, d1.quat, d1.force, d1.torque, d1.sums)
        g1 = outputs(d1)
        ctx2.forces_noalloc(p2, d2.n, d2.species, d2.com, d2.quat, d2.force, d2.torque, d2.sums)
        g2 = outputs(d2)
        ctx.forces(p1, d1.n, d1.species, d1.com, d1.quat, d1.force, d1.torque, d1.sums)
        r1 = outputs(d1)
        ctx2.forces(p2, d2.n, d2.species, d2.com, d2.quat, d2.force, d2.torque, d2.sums)
        r2 = outputs(d2)
        for a, b in ((g1, r1), (g2, r2)):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
        ctx.close()
        ctx2.close()


def test_noalloc_refuses_sizes_above_the_limit():
    s = I.quadrupolar_fluid(n=ms2.NOALLOC_MAX_MOL + 1, density=0.45)
    ctx = ms2.Context(s.species)
    d = ms2.DeviceSystem(s)
    d.sums.fill_(7.0)
    p = ms2.params_struct(s.params, ms2.FP32)
    with pytest.raises(ms2.MS2Error) as e:
        ctx.forces_noalloc(p, d.n, d.species, d.com, d.quat, d.force, d.torque, d.sums)
    assert e.value.status == 1 and "MS2_NOALLOC_MAX_MOL" in str(e.value)
    torch.cuda.synchronize()
    assert (d.sums.cpu().numpy() == 7.0).all()      # nothing was enqueued
    ctx.close()

"""Writes the oracle-produced fixtures of the FP32 tests (calls oracle/ and
the seeded input generators only; nothing from the HIP path):

  oracle_equilibrated.npz  centres and quaternions of four states taken from
      their seeded starts by the oracle's own integrator (Gear NVT; velocity
      Verlet for the one-centre LJ fluid), so that FP32 parity is measured
      on disordered states, not on the lattice starts:
        quad    2CLJQ fluid, 1000 molecules, rho 0.6, T 2, 300 steps
        quad_lo 2CLJQ state point 9 of the batched set (517 molecules,
                rho 0.33), 300 steps
        ionic   900 water-like molecules + 50 ion pairs, Ewald, 200 steps
        lj      one-centre LJ fluid, 500 molecules, rho 0.7, 300 steps
  oracle_quad_nvt_log.npz  the oracle's energy log (U, K_trans, K_rot, W,
      U_s + tail, U_ss + tail per step) of the 2CLJQ fluid (1000 molecules)
      over 1000 Gear NVT steps from its lattice start, and the moment sums
      of that run (u0 = -21000).

Run:  python tests/golden/make_oracle_runs.py   (a few minutes, one thread)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1507_07548_amd import inputs as I  # noqa: E402

QUAD_U0 = -21000.0


def equilibrate(system, steps):
    s = system.copy()
    s.md.n_steps = steps
    s.md.sample_every = 0
    st = oracle.md(s, want_log=False)["state"]
    return np.ascontiguousarray(st.com % s.params.box), np.ascontiguousarray(st.quat)


def main():
    states = {}
    for name, make, steps in (("quad", lambda: I.quadrupolar_fluid(), 300),
                              ("quad_lo", lambda: I.batched_state_point(9), 300),
                              ("ionic", lambda: I.ionic_solution(), 200),
                              ("lj", lambda: I.lj_fluid(), 300)):
        com, quat = equilibrate(make(), steps)
        states[name + "_com"], states[name + "_quat"] = com, quat
        print(f"{name}: {steps} steps", flush=True)
    np.savez(os.path.join(HERE, "oracle_equilibrated.npz"), **states)

    s = I.quadrupolar_fluid(n_steps=1000, sample_every=1)
    s.md.u0 = QUAD_U0
    out = oracle.md(s, want_log=True)
    np.savez(os.path.join(HERE, "oracle_quad_nvt_log.npz"), log=out["log"], moments=out["moments"],
             u0=np.array(QUAD_U0))
    print("quad NVT log: 1000 steps", flush=True)


if __name__ == "__main__":
    main()

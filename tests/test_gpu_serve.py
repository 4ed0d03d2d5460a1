"""Serving on the GPU: a trace of mixed requests admitted into running
batches (continuous batching); every served result equals, bit for bit,
the same request run alone in its own batch."""
import numpy as np
import pytest

from paper_1507_07548_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1507_07548_amd import ms2  # noqa: E402
from paper_1507_07548_amd.serve import GpuBackend, Request, Server, backend_key  # noqa: E402


def families():
    return {"lj": [I.one_center_lj()], "2cljq": [I.two_center_lj_quadrupole()],
            "ionic": [I.water_tip4p_like(), I.cation(), I.anion()]}


@pytest.mark.parametrize("max_inflight", [None, 2])
def test_served_results_equal_the_same_request_run_alone(max_inflight):
    """Batches per model family and size class; every batch launching, or two
    at a time in shortest-remaining-work order."""
    trace = I.serving_trace(n_requests=9, rate=400.0, seed=7, n_lo=200, n_hi=1500, n_steps=120,
                            window=60, acf_every=6, origin_every=30)
    print(f"[gpu] serving max_inflight={max_inflight}", [(round(t, 3), m, s.n) for t, m, s in trace], flush=True)
    fam = families()
    keys = sorted({backend_key(m, s.n) for _, m, s in trace})
    backends = {k: GpuBackend(fam[k.split("/")[0]], max_slots=3) for k in keys}
    reqs = [Request(r, t, backend_key(m, s.n), s, ms2.FP32) for r, (t, m, s) in enumerate(trace)]
    srv = Server(backends, hbm_budget=1 << 34, chunk_steps=40, max_inflight=max_inflight)
    res = {r.rid: r for r in srv.run(reqs)}
    assert sorted(res) == list(range(len(reqs)))
    # some request was admitted while another one was already running
    spans = sorted((r.admitted, r.finished) for r in res.values())
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    for r in reqs:
        got = res[r.rid]
        assert got.status == 0 and got.steps_done == r.system.md.n_steps
        ctx = ms2.Context(fam[r.model.split("/")[0]])
        alone = ms2.Batch(ctx, 1)
        slot = alone.admit(r.system, ms2.FP32)
        alone.step(r.system.md.n_steps)
        ref = alone.sample(slot)
        for k in ("com", "quat", "vel", "omega", "moments", "rdf", "acf_v", "acf_j", "acf_cnt"):
            assert np.array_equal(ref[k], got.samples[k]), (r.rid, r.model, k)
        alone.close()

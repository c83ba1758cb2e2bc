"""Serving form on the device: requests admitted and batched as they arrive
finish with the same fields as the same simulation run alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    import torch
    from paper_2306_17263_amd import Problem
    from paper_2306_17263_amd.serve import DeviceBackend, Server, requests_from_mix
    from workloads import mode_fields, serving_arrivals
    mix = serving_arrivals(count=10, seed=11, rate=400.0, n2=(24, 96), n3=(10, 20), steps=(8, 40))
    reqs = requests_from_mix(mix)
    be = DeviceBackend(keep_results=True)
    budget = 3 * max(be.footprint(r) for r in reqs)            # forces queueing
    out = Server(be, hbm_budget=budget, chunk=7).run(reqs)
    assert out["completed"] == len(reqs)
    st = torch.cuda.Stream()
    for r in out["done"]:
        p = Problem(r.dim, r.n, r.r, stream=st)
        h = 1.0 / r.n
        for name, v in mode_fields(r.dim, r.n, r.k, 0.0, r.r * h / 2, amp=r.amp).items():
            if name in p.fields():
                p.set(name, v)
        p.step(r.steps)
        for a, v in r.result.items():
            assert np.array_equal(v, p.get(a)), (r.id, r.dim, r.n, a)
        p.close()

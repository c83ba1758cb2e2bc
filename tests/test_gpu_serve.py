"""Serving form on the device: requests admitted and batched as they arrive
finish with the same fields as the same simulation run alone (bit for bit)
and as the CPU oracle (the FP64 bar: 1e-12 relative L2, every element within
1e-11 of the field scale)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone_and_oracle():
    import torch
    import oracle
    from gpu_util import check_fields
    from paper_2306_17263_amd import Problem
    from paper_2306_17263_amd.serve import DeviceBackend, Server, requests_from_mix
    from workloads import mode_fields, serving_arrivals
    mix = serving_arrivals(count=10, seed=11, rate=400.0, n2=(24, 96), n3=(10, 20), steps=(8, 40))
    reqs = requests_from_mix(mix)
    be = DeviceBackend(keep_results=True, chunk=7)
    budget = 3 * max(be.footprint(r) for r in reqs)            # forces queueing
    out = Server(be, hbm_budget=budget, chunk=7).run(reqs)
    assert out["completed"] == len(reqs)
    st = torch.cuda.Stream()
    for r in out["done"]:
        p = Problem(r.dim, r.n, r.r, stream=st)
        o = oracle.OracleProblem(r.dim, r.n, r.r, 1.0)
        h = 1.0 / r.n
        for name, v in mode_fields(r.dim, r.n, r.k, 0.0, r.r * h / 2, amp=r.amp).items():
            if name in p.fields():
                p.set(name, v)
                o.set(name, v)
        p.step(r.steps)
        o.step(r.steps)
        names = [a for a in r.result if a[0] in "eh"]
        for a, v in r.result.items():
            assert np.array_equal(v, p.get(a)), (r.id, r.dim, r.n, a)
        check_fields({a: r.result[a] for a in names}, {a: o.get(a) for a in names})
        p.close()

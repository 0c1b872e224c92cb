"""Serving: requests that arrive while others run are admitted as memory frees
up, FP64 and mixed requests run concurrently, and every result equals the
same request run alone (bit for bit)."""
import numpy as np
import pytest

from synthetic import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


def small_requests():
    """Sphere and hex requests of uneven size, layers, substeps, precision and length."""
    from paper_2105_13484_amd.serve import Request
    reqs = []
    specs = [("sphere", 3, 16, 0, 6), ("hex", 12, 40, 1, 4), ("sphere", 2, 100, 1, 5),
             ("hex", 10, 60, 0, 7), ("sphere", 3, 30, 1, 3), ("hex", 8, 20, 0, 5)]
    for i, (kind, size, L, prec, steps) in enumerate(specs):
        if kind == "sphere":
            c = cases.sphere_case(size, L, cases.SEED_BASE + 500 + i, substeps=8, dt_btr=300.0 * 2 ** (4 - size))
        else:
            c = cases.c1(n=size, L=L, substeps=6 + i, dt_btr=15.0, member=10 + i, steps=steps)
        c = cases.with_params(c, precision=prec)
        reqs.append(Request(rid=i, case=c, steps=steps, arrival=0.02 * i))
    return reqs


def test_served_results_equal_alone(dev):
    from paper_2105_13484_amd.serve import Engine
    reqs = small_requests()
    fps = sorted(dev.footprint_bytes(r.case.mesh, r.case.params) for r in reqs)
    # a budget that holds only the three largest at once forces queueing
    eng = Engine(budget_bytes=sum(fps[-3:]), chunk_steps=2)
    stats = eng.run(reqs)
    eng.close()
    assert stats["requests"] == len(reqs) and stats["failed"] == 0
    assert all(r.admitted is not None and r.done >= r.arrival for r in reqs)
    for r in reqs:
        _, st = dev.state_from_case(r.case)
        assert st.step(r.steps) == 0
        alone = st.read()
        for k in ("h", "u", "zeta", "ubar"):
            assert np.array_equal(r.result[k], alone[k]), (r.rid, k)


def test_footprint_matches_allocations(dev):
    c = cases.c1(n=12, L=40, steps=1)
    dm, st = dev.state_from_case(c)
    assert dev.footprint_bytes(c.mesh, c.params) == dm.nbytes + st.nbytes

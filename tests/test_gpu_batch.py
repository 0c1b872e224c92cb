"""Batched ensembles, launch geometry and HIP-graph replay on the GPU.

Every member of a batch computes exactly what it computes alone: the kernels
run the same arithmetic per column and per entity whatever the workgroup
shape or the batch composition, so results are compared bit for bit.
"""
import numpy as np
import pytest

from synthetic import cases

pytestmark = pytest.mark.gpu

FIELDS = ("h", "u", "zeta", "ubar")


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


@pytest.fixture(scope="module")
def stream(dev):
    import torch
    return torch.cuda.Stream()


def member_cases(precision):
    """Uneven members: mesh sizes, layer counts (one above 64) and substep counts differ."""
    specs = [(12, 20, 6), (16, 40, 9), (8, 60, 4), (10, 100, 5), (14, 7, 7)]
    return [cases.with_params(cases.c1(n=n, L=L, substeps=M, dt_btr=15.0, member=i, steps=3), precision=precision)
            for i, (n, L, M) in enumerate(specs)]


def assert_same(a, b, what):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), (what, k, float(np.abs(a[k] - b[k]).max()))


def run_alone(dev, case, steps, stream):
    _, st = dev.state_from_case(case, stream=stream)
    assert st.step(steps) == 0
    return st.read()


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_alone(dev, stream, precision, graph):
    cs = member_cases(precision)
    alone = [run_alone(dev, c, 3, stream) for c in cs]
    keep, b = [], dev.Batch(stream=stream)
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append(dm)
        b.add(st)
    b.compile()
    b.use_graph(graph)
    assert b.step(1) == 0
    assert b.step(2) == 0
    for i, st in enumerate(b.members):
        assert_same(st.read(), alone[i], f"member {i}")
    # One launch per phase across members: 9 M_max barotropic evaluations plus
    # at most 28 other launch sites (16, and 12 precision conversions in mixed
    # mode), each split at most in two by the register-chunk count.
    max_m = max(c.params.substeps for c in cs)
    assert b.launches_per_step() <= 9 * max_m + 2 * 28
    assert b.launches_per_step() < sum(9 * c.params.substeps + 16 for c in cs)


def test_batch_membership_changes(dev, stream):
    cs = member_cases(0)[:3]
    alone5 = [run_alone(dev, c, 5, stream) for c in cs]
    keep, b, sts = [], dev.Batch(stream=stream), []
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append(dm)
        sts.append(st)
        b.add(st)
    assert b.step(2) == 0
    b.remove(sts[1])                 # leaves after 2 steps
    assert sts[1].step(3) == 0       # and finishes alone
    assert b.step(3) == 0
    for i, st in enumerate(sts):
        assert_same(st.read(), alone5[i], f"member {i}")


def test_batch_rejects_mixed_schemes(dev, stream):
    a = member_cases(0)[0]
    c = cases.with_params(member_cases(0)[1], scheme=2)
    _, s1 = dev.state_from_case(a, stream=stream)
    _, s2 = dev.state_from_case(c, stream=stream)
    b = dev.Batch(stream=stream)
    b.add(s1)
    with pytest.raises(dev.SSEError):
        b.add(s2)


@pytest.mark.parametrize("L", [60, 100])
@pytest.mark.parametrize("geom", [(1, 64), (2, 128), (8, 512), (16, 1024)])
def test_geometry_does_not_change_results(dev, stream, geom, L):
    # L = 100: the two-chunk edge pass caps its workgroups at 4 wavefronts,
    # so geometries of 8 and 16 columns per block launch it with fewer
    case = cases.c1(n=12, L=L, steps=3)
    ref = run_alone(dev, case, 3, stream)
    _, st = dev.state_from_case(case, stream=stream)
    st.set_geometry(*geom)
    assert st.step(3) == 0
    assert_same(st.read(), ref, f"geometry {geom}")


@pytest.mark.parametrize("geom", [(8, 512), (16, 1024)])
def test_batch_geometry_with_deep_members(dev, stream, geom):
    cs = member_cases(0)
    refs = [run_alone(dev, c, 3, stream) for c in cs]
    keep, b = [], dev.Batch(stream=stream)
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append(dm)
        b.add(st)
    b.set_geometry(*geom)
    b.compile()
    assert b.step(3) == 0
    for i, st in enumerate(b.members):
        assert_same(st.read(), refs[i], f"batch geometry {geom}, member {i}")


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_equal_eager(dev, stream, precision):
    """Replays of the captured step, with eager work and synchronizations in
    between, match the eager steps after every replay."""
    import torch
    case = cases.with_params(cases.c1(n=12, L=60, steps=4), precision=precision)
    _, eager = dev.state_from_case(case, stream=stream)
    _, g = dev.state_from_case(case, stream=stream)
    g.use_graph(True)
    scratch = torch.zeros(1 << 20, device="cuda")
    for k in range(4):
        assert eager.step(1) == 0
        with torch.cuda.stream(stream):
            scratch.add_(1.0)            # unrelated eager work between replays
        torch.cuda.synchronize()
        assert g.step(1) == 0
        assert_same(g.read(), eager.read(), f"replay {k}")


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_members_with_either_barotropic_variant(dev, stream, precision):
    """Members running the per-evaluation and the per-substep barotropic
    kernels share one batch and compute what they compute alone."""
    cs = member_cases(precision)
    alone = [run_alone(dev, c, 3, stream) for c in cs]
    keep, b = [], dev.Batch(stream=stream)
    for i, c in enumerate(cs):
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append(dm)
        if i % 2:
            assert st.try_bt_variant(0)
        b.add(st)
    b.compile()
    assert b.step(3) == 0
    for i, st in enumerate(b.members):
        assert_same(st.read(), alone[i], f"member {i}")


def _random_members(seed):
    """Five members that share the scheme, the precision mode and the vertical
    coordinate (what a batch requires) and differ at random in everything
    else: planar hexes and land-masked spheres, layer counts on both sides of
    64, M, reconciliation, vertical mixing, biharmonic viscosity, tracer."""
    rng = np.random.default_rng(seed)
    shared = dict(scheme=int(rng.choice([2, 3])), precision=int(rng.choice([0, 1, 2])),
                  vcoord=int(rng.choice([0, 1])))
    out = []
    for i in range(5):
        L = int(rng.choice([2, 7, 31, 64, 65, 100]))
        if rng.random() < 0.3:
            base = cases.sphere_case(2, L, 900 + 10 * seed + i, substeps=5, dt_btr=200.0)
            nu4 = 1e13
        else:
            base = cases.c1(n=int(rng.choice([6, 8, 10])), L=L, member=i, steps=2)
            nu4 = 1e9
        M = int(rng.choice([1, 3, 7]))
        kw = dict(shared, substeps=M, dt=base.params.dt / base.params.substeps * M,
                  reconcile=int(rng.choice([0, 1, 2])))
        if rng.random() < 0.4:
            kw.update(vmix=1, nu_v=1e-3, c_drag=2e-3)
        if rng.random() < 0.4:
            kw.update(hdiff=1, nu_h=nu4)
        if rng.random() < 0.4:
            kw.update(tracer=1, kappa_h=20.0, kappa_v=1e-4)
        out.append(cases.with_params(base, **kw))
    return out


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_random_batches_equal_alone(dev, stream, seed):
    """Batches of members with randomly differing options: every member,
    tracer included, computes in the batch exactly what it computes alone."""
    cs = _random_members(seed)
    alone = []
    for c in cs:
        _, st = dev.state_from_case(c, stream=stream)
        assert st.step(2) == 0, dev.last_error()
        r = st.read()
        if c.params.tracer:
            r["T"] = st.read_tracer()
        alone.append(r)
    keep, b = [], dev.Batch(stream=stream)
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append((dm, st))
        b.add(st)
    assert b.step(2) == 0, dev.last_error()
    for i, (c, (_, st)) in enumerate(zip(cs, keep)):
        got = st.read()
        assert_same(got, alone[i], f"seed {seed} member {i}")
        if c.params.tracer:
            assert np.array_equal(st.read_tracer(), alone[i]["T"]), (seed, i)
    b.close()

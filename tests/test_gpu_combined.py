"""GPU parity with every optional physics term on at once: implicit vertical
mixing (Algorithm 2), biharmonic viscosity and the temperature tracer with its
EOS, against the oracle.

Each term has its own parity file; here they run together, so the edge pass
takes its combined template variant (mixing and del4), the thickness stages
run fused with the tracer stages, and the density the pressure gradient sees
is the EOS density of the evolving temperature.  Bounds: FP64 as in
``tests/parity_cases.py`` (relative L2 1e-11 and largest element error 1e-10 per
field u, h, zeta, ubar, T, or four times the oracle's own measured rounding
spread where that is larger); mixed precision 1e-5 on velocities,
1e-9 on h, and 1e-8 on T.  T is FP64 but carried by the FP32 velocities, so
its error is the velocity error times the relative change that advection
makes to T over the run (about 1e-2 here): 1e-5 x 1e-2 would allow 1e-7, and
1e-8 still leaves room above the ~2e-9 measured.  Batches that mix members
with different term sets give each member the bits it gets alone.
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from synthetic import cases
from tests.helpers import rel_l2
from tests import parity_cases as P
from tests.parity_cases import all_terms
from tests.test_gpu_parity import _report, run_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


COMBINED = {
    "hex12_L20_ssprk3": lambda: all_terms(cases.c1(n=12, L=20, steps=4)),
    "hex12_L20_ssprk2": lambda: all_terms(cases.with_params(cases.c1(n=12, L=20, steps=4), scheme=2)),
    "hex8_L100": lambda: all_terms(cases.c1(n=8, L=100, steps=2)),
    "sphere3_land_L7": lambda: all_terms(cases.sphere_case(3, 7, 77, substeps=5, dt_btr=200.0), nu4=1e13),
}
# SSPRK2-SE grows on these noisy states (its stability polynomial exceeds one
# on the imaginary axis), so it runs fewer steps.
STEPS = {"hex12_L20_ssprk3": 4, "hex12_L20_ssprk2": 2, "hex8_L100": 2, "sphere3_land_L7": 3}


@pytest.mark.parametrize("name", sorted(COMBINED))
def test_all_terms_fp64(dev, name):
    case, steps = P.build("all_terms_" + name)
    assert steps == STEPS[name]
    rc, g, r = run_case(dev, "all_terms_" + name)
    assert rc == 0, dev.last_error()
    P.check("all_terms_" + name, g, r, report=_report)
    # every term changes the answer: dropping any one moves the oracle's result
    for drop in ({"vmix": 0}, {"hdiff": 0, "nu_h": 0.0}, {"tracer": 0}):
        other = S.run(cases.with_params(case, **drop), steps)
        assert rel_l2(other[0], r["u"]) > 1e3 * 1e-11, drop


@pytest.mark.parametrize("name", ["hex12_L20_ssprk3", "sphere3_land_L7"])
def test_all_terms_mixed_precision(dev, name):
    case = COMBINED[name]()
    steps = STEPS[name]
    dm, st = dev.state_from_case(cases.with_params(case, precision=1))
    assert st.step(steps) == 0, dev.last_error()
    g = st.read()
    T = st.read_tracer()
    u, h, zeta, ubar, Tr = S.run(case, steps)
    errs = {"u": rel_l2(g["u"], u), "ubar": rel_l2(g["ubar"], ubar), "h": rel_l2(g["h"], h), "T": rel_l2(T, Tr)}
    _report(f"all terms mixed {name}", errs)
    assert errs["u"] < 1e-5 and errs["ubar"] < 1e-5, errs
    assert errs["h"] < 1e-9 and errs["T"] < 1e-8, errs


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_of_term_sets(dev, precision):
    """One batch holds members with all terms, none, and each pair."""
    import torch
    stream = torch.cuda.Stream()
    sets = [dict(vmix=1, hdiff=1, tracer=1), {}, dict(vmix=1, hdiff=1), dict(hdiff=1, tracer=1),
            dict(vmix=1, tracer=1)]
    shapes = [(12, 20, 6), (10, 70, 5), (8, 40, 4), (14, 9, 7), (10, 33, 5)]
    cs = []
    for i, ((n, L, M), terms) in enumerate(zip(shapes, sets)):
        c = cases.with_params(cases.c1(n=n, L=L, substeps=M, dt_btr=15.0, member=i, steps=3), precision=precision)
        extra = dict(nu_v=1e-3, c_drag=2e-3, kappa_h=20.0, kappa_v=1e-4)
        if terms.get("hdiff"):
            extra["nu_h"] = 1e9
        cs.append(cases.with_params(c, **terms, **extra))
    alone = []
    for c in cs:
        _, st = dev.state_from_case(c, stream=stream)
        assert st.step(3) == 0, dev.last_error()
        out = st.read()
        if c.params.tracer:
            out["T"] = st.read_tracer()
        alone.append(out)
    keep, b = [], dev.Batch(stream=stream)
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append(dm)
        b.add(st)
    b.compile()
    assert b.step(3) == 0, dev.last_error()
    for i, st in enumerate(b.members):
        got = st.read()
        if cs[i].params.tracer:
            got["T"] = st.read_tracer()
        for k in alone[i]:
            assert np.array_equal(got[k], alone[i][k]), (i, k)

"""GPU parity of the temperature tracer stages (fused with the thickness
stages) against the oracle, with the density following the EOS.

FP64 cases and bounds come from ``tests/parity_cases.py`` (relative L2 1e-11
and largest element error 1e-10 per field u, h, zeta, ubar and T, or four times
the oracle's own measured rounding spread where that is larger).  Mixed precision:
the velocity bound 1e-5 for u and ubar, and the thickness bound 1e-9 for h and
T (both FP64, moved by FP32 velocities).
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import Setup
from synthetic import cases
from tests.helpers import rel_l2, smooth_case
from tests.parity_cases import tracer, with_temp
from tests.test_gpu_parity import _report, check_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


def _run(dev, case, steps):
    dm, st = dev.state_from_case(case)
    assert st.step(steps) == 0, dev.last_error()
    g = st.read()
    g["T"] = st.read_tracer()
    u, h, zeta, ubar, T = S.run(case, steps)
    return g, {"u": u, "h": h, "zeta": zeta, "ubar": ubar, "T": T}


@pytest.mark.parametrize("name", ["tracer_ssprk2", "tracer_ssprk3", "tracer_c1_recipe_32x32x60",
                                  "tracer_c2_recipe_level3x60", "tracer_isopycnal_8x8x100"])
def test_tracer_steps(dev, name):
    """Smooth stratified hex with a layered temperature and both schemes; the C1
    and C2 recipes at reduced size; isopycnal with two register chunks."""
    check_case(dev, name)


def test_uniform_tracer_stays_uniform(dev):
    base = tracer(cases.sphere_case(3, 7, 77, substeps=5, dt_btr=200.0), kappa_h=1e3, kappa_v=1e-3)
    T0 = np.full(base.h.shape, 13.0)
    case = with_temp(base, T0)
    dm, st = dev.state_from_case(case)
    assert st.step(5) == 0
    T = st.read_tracer()
    m = case.cell_mask.astype(bool)
    assert np.abs(T[m] - 13.0).max() <= 1e-12 * 13.0


def test_tracer_content_conserved(dev):
    case = tracer(cases.sphere_case(3, 7, 78, substeps=5, dt_btr=200.0), kappa_h=1e3, kappa_v=1e-3)
    dm, st = dev.state_from_case(case)
    A = case.mesh.areaCell[:, None]
    c0 = (A * case.h * case.temp).sum()
    assert st.step(6) == 0
    h, T = st.read()["h"], st.read_tracer()
    assert abs((A * h * T).sum() - c0) <= 1e-13 * abs(c0)


@pytest.mark.parametrize("name", ["c1", "sphere"])
def test_tracer_mixed_precision(dev, name):
    case = tracer(cases.c1(n=16, L=20, steps=3) if name == "c1"
                  else cases.sphere_case(3, 7, 79, substeps=5, dt_btr=200.0), kappa_h=10.0, kappa_v=1e-5)
    dm, st = dev.state_from_case(cases.with_params(case, precision=1))
    assert st.step(3) == 0
    g = st.read()
    T = st.read_tracer()
    u, h, zeta, ubar, Tr = S.run(case, 3)
    errs = {"u": rel_l2(g["u"], u), "ubar": rel_l2(g["ubar"], ubar), "h": rel_l2(g["h"], h), "T": rel_l2(T, Tr)}
    _report(f"tracer mixed {name}", errs)
    assert errs["u"] < 1e-5 and errs["ubar"] < 1e-5
    assert errs["h"] < 1e-9 and errs["T"] < 1e-9


def test_tracer_api_errors(dev):
    plain = cases.c1(n=8, L=4, steps=1)
    _, st = dev.state_from_case(plain)
    with pytest.raises(dev.SSEError):
        st.set_tracer(plain.temp)
    with pytest.raises(dev.SSEError):
        st.read_tracer()
    case = tracer(plain)
    dm = dev.DeviceMesh(case.mesh, case.H, case.cell_mask)
    s2 = dev.DeviceState(dm, case.params)
    s2.init(case.h, case.u, case.rho, case.h_ref)
    with pytest.raises(dev.SSEError):
        s2.step(1)                          # no temperature given yet
    s2.set_tracer(case.temp)
    assert s2.step(1) == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_tracer_and_plain_members(dev, precision):
    import torch
    stream = torch.cuda.Stream()
    cs = [cases.with_params(cases.c1(n=n, L=L, substeps=M, dt_btr=15.0, member=i, steps=3), precision=precision)
          for i, (n, L, M) in enumerate([(12, 20, 6), (10, 70, 5), (8, 40, 4), (14, 9, 7)])]
    cs = [tracer(c, kappa_h=10.0, kappa_v=1e-4) if i % 2 == 0 else c for i, c in enumerate(cs)]
    alone = []
    for c in cs:
        _, st = dev.state_from_case(c, stream=stream)
        assert st.step(3) == 0
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
    assert b.step(3) == 0
    for i, st in enumerate(b.members):
        got = st.read()
        if cs[i].params.tracer:
            got["T"] = st.read_tracer()
        for k in alone[i]:
            assert np.array_equal(got[k], alone[i][k]), (i, k)

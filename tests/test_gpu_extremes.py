"""GPU parity at the ends of the parameter ranges the library accepts:

* L = 128, the largest column (two full 64-lane register chunks), in FP64,
  in mixed precision and with every optional term on;
* L = 65, a second chunk that holds a single layer;
* L = 1, where the baroclinic velocity u - ubar vanishes identically and the
  split step reduces to the barotropic system (hex and sphere with land);
* M = 1, one barotropic substep per large step, in both schemes;
* a batch whose members span these extremes gives each member its solo bits;
* sse_step(0) is a no-op.

FP64 cases and bounds come from ``tests/parity_cases.py`` (relative L2 1e-11 and
largest element error 1e-10 per field, or four times the oracle's own measured
rounding spread where that is larger); mixed precision as in the mixed-precision
parity file.
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from synthetic import cases
from tests.helpers import rel_l2
from tests.test_gpu_mixed import check_state
from tests.test_gpu_parity import check_case, run_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


FP64_CASES = ["hex8_L128", "hex10_L65", "hex12_L1_ssprk3", "hex12_L1_ssprk2", "sphere3_land_L1",
              "hex10_L20_M1_ssprk3", "hex10_L20_M1_ssprk2"]


@pytest.mark.parametrize("name", FP64_CASES)
def test_extreme_shapes_fp64(dev, name):
    rc, gpu, ref = run_case(dev, name)
    assert rc == 0, dev.last_error()
    from tests import parity_cases as P
    P.check(name, gpu, ref)
    if gpu["u"].shape[1] == 1:
        # one layer: the velocity is its own barotropic part (to roundoff: the
        # forcing subtraction u - dt ((h u / h) / dt) need not cancel exactly)
        assert np.abs(gpu["u"][:, 0] - gpu["ubar"]).max() <= 1e-13 * np.abs(gpu["ubar"]).max()


def test_max_layers_mixed(dev):
    case = cases.with_params(cases.c1(n=8, L=128, steps=3), precision=1)
    dm, st = dev.state_from_case(case)
    rc, gpu, ref = st.step(3), st.read(), S.run(case, 3)
    assert rc == 0, dev.last_error()
    check_state("hex8_L128, 3 steps", case, gpu, ref)


def test_max_layers_all_terms(dev):
    check_case(dev, "all_terms_hex8_L128")


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_of_extreme_members(dev, precision):
    import torch
    stream = torch.cuda.Stream()
    shapes = [(8, 128, 20), (10, 1, 20), (10, 65, 3), (6, 64, 1), (12, 2, 7)]
    cs = [cases.with_params(cases.c1(n=n, L=L, substeps=M, dt_btr=15.0, member=i, steps=2), precision=precision)
          for i, (n, L, M) in enumerate(shapes)]
    alone = []
    for c in cs:
        _, st = dev.state_from_case(c, stream=stream)
        assert st.step(2) == 0, dev.last_error()
        alone.append(st.read())
    keep, b = [], dev.Batch(stream=stream)
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append(dm)
        b.add(st)
    b.compile()
    assert b.step(2) == 0, dev.last_error()
    for i, st in enumerate(b.members):
        got = st.read()
        for k in alone[i]:
            assert np.array_equal(got[k], alone[i][k]), (shapes[i], k)


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_steps_leave_the_state_unchanged(dev, precision):
    case = cases.with_params(cases.c1(n=10, L=12, steps=2), precision=precision)
    _, st = dev.state_from_case(case)
    assert st.step(2) == 0, dev.last_error()
    before = st.read()
    assert st.step(0) == 0, dev.last_error()
    after = st.read()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    assert rel_l2(after["u"], before["u"]) == 0.0

"""The gather-only edge pass (sse_debug_edge_gathers, the measurement aid the
benchmark times beside the edge pass) leaves the state alone and refuses the
shapes it does not cover."""
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


@pytest.mark.parametrize("precision", [0, 1])
def test_gather_probe_leaves_the_state_alone(dev, precision):
    case = cases.with_params(cases.c1(n=16, L=60, steps=3), precision=precision)
    out = {}
    for probe in (False, True):
        _, st = dev.state_from_case(case)
        assert st.step(1) == 0
        if probe:
            st.debug_edge_gathers()
            st.debug_edge_gathers()
        assert st.step(2) == 0
        out[probe] = st.read()
    for k in out[False]:
        assert np.array_equal(out[False][k], out[True][k]), k


def test_gather_probe_refuses_two_register_chunks(dev):
    _, st = dev.state_from_case(cases.c1(n=8, L=100, steps=1))
    with pytest.raises(dev.SSEError):
        st.debug_edge_gathers()
    assert st.step(1) == 0

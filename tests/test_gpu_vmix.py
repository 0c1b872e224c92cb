"""GPU parity of the implicit vertical mixing (Algorithm 2) against the oracle.

The GPU solves each edge column's tridiagonal system by parallel cyclic
reduction across the lanes of a wavefront, the oracle by the sequential
Thomas algorithm; both are backward stable on these diagonally dominant
systems, so the FP64 bound stays relative L2 <= 1e-11 per field (with the
long-run self-drift allowance of the other parity tests), and the mixed
bounds are those of the other mixed-precision tests.  Cases span one layer
(no reduction round), 4 and 60 layers (one register chunk, ragged) and 100
layers (two chunks, a stride-64 round), a sphere with land, every edge-pass
variant, and batches that mix members with and without mixing.
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import Setup
from synthetic import cases
from tests.helpers import rel_l2, smooth_case
from tests.test_gpu_mixed import check_state
from tests.parity_cases import field_errors, format_errors, vmix
from tests.test_gpu_parity import TOL, TOL_MAX, _noisy_state, _report, check_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


MIX_CASES = {
    "hex10x6_L4": lambda: vmix(cases.with_params(smooth_case(n=10, L=4), scheme=3)),
    "hex10_L1": lambda: vmix(cases.c1(n=10, L=1, steps=1)),
    "hex12_L60": lambda: vmix(cases.c1(n=12, L=60, steps=1)),
    "hex8_L100": lambda: vmix(cases.c1(n=8, L=100, steps=1)),
    "sphere3_land_L7": lambda: vmix(cases.sphere_case(3, 7, 77, substeps=5, dt_btr=200.0)),
}


def _feuler_ref(case):
    st_o = Setup.from_case(case)
    u, h = _noisy_state(case, steps=1)
    ubar, _ = S.split(u, h, st_o)
    zeta = S.ssh(h, st_o)
    ut1, G = S.baroclinic_feuler_mixing(u, u - ubar[:, None], ubar, zeta, h, case.params.dt, st_o)
    return u, h, ubar, zeta, ut1, G


def _mix_errs(g_ut1, g_G, ut1, G, ubar):
    """Algorithm 2 solves for the whole velocity u1 and returns ut1 = u1 - ubar,
    an exact subtraction where ut1 is small against ubar (one layer: ut1 is
    just the implicit drag increment).  Rounding in u1 is then relative to u1,
    so ut1 is measured against u1's norms; u1 itself is checked as well."""
    u1, g_u1 = ut1 + ubar[:, None], g_ut1 + ubar[:, None]
    d = g_ut1 - ut1
    return {"u1": field_errors(g_u1, u1),
            "ut1/|u1|": {"l2": float(np.linalg.norm(d) / max(np.linalg.norm(u1), np.linalg.norm(ut1), 1e-300)),
                         "max": float(np.abs(d).max() / max(np.abs(u1).max(), np.abs(ut1).max(), 1e-300))},
            "G": field_errors(g_G, G)}


def _assert_mix(name, errs):
    _report(name + ": " + format_errors(errs))
    for k, v in errs.items():
        assert v["l2"] <= TOL and v["max"] <= TOL_MAX, (name, k, v)


@pytest.mark.parametrize("name", sorted(MIX_CASES))
def test_mixing_feuler_parity(dev, name):
    case = MIX_CASES[name]()
    u, h, ubar, zeta, ut1, G = _feuler_ref(case)
    _, st = dev.state_from_case(case)
    g_ut1, g_G = st.debug_baroclinic_feuler(u, ubar, zeta, h, case.params.dt)
    _assert_mix(f"feuler+mixing {name}", _mix_errs(g_ut1, g_G, ut1, G, ubar))
    # the mixing is not a no-op on these cases
    ex, _ = S.baroclinic_feuler(u, u - ubar[:, None], zeta, h, case.params.dt, Setup.from_case(case))
    assert rel_l2(ex, ut1) > 1e3 * TOL


@pytest.mark.parametrize("name", ["hex12_L60", "hex8_L100", "sphere3_land_L7"])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_mixing_edge_variant_parity(dev, name, variant):
    case = MIX_CASES[name]()
    u, h, ubar, zeta, ut1, G = _feuler_ref(case)
    _, st = dev.state_from_case(case)
    if not st.try_edge_variant(variant):
        pytest.skip(f"variant {variant} does not fit: {dev.last_error()}")
    g_ut1, g_G = st.debug_baroclinic_feuler(u, ubar, zeta, h, case.params.dt)
    _assert_mix(f"feuler+mixing variant={variant} {name}", _mix_errs(g_ut1, g_G, ut1, G, ubar))


@pytest.mark.parametrize("name", ["vmix_ssprk2", "vmix_ssprk3", "vmix_c1_recipe_32x32x60",
                                  "vmix_c2_recipe_level3x60", "vmix_hex8_L100"])
def test_mixing_steps(dev, name):
    """Smooth stratified hex with both schemes; the C1 and C2 recipes at reduced
    size with the recipes' nu_v and c_drag; L = 100 (two register chunks)."""
    check_case(dev, name)


@pytest.mark.parametrize("name", ["hex12_L60", "sphere3_land_L7"])
def test_mixing_mixed_precision(dev, name):
    case = MIX_CASES[name]()
    dm, st = dev.state_from_case(cases.with_params(case, precision=1))
    assert st.step(3) == 0, dev.last_error()
    check_state(f"mixing {name}", case, st.read(), S.run(case, 3))


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_mixing_and_explicit_members(dev, precision):
    """Members with and without mixing in one batch compute what they compute alone."""
    import torch
    stream = torch.cuda.Stream()
    cs = [cases.with_params(cases.c1(n=n, L=L, substeps=M, dt_btr=15.0, member=i, steps=3), precision=precision)
          for i, (n, L, M) in enumerate([(12, 20, 6), (10, 70, 5), (8, 40, 4), (14, 9, 7)])]
    cs = [vmix(c) if i % 2 == 0 else c for i, c in enumerate(cs)]
    alone = []
    for c in cs:
        _, st = dev.state_from_case(c, stream=stream)
        assert st.step(3) == 0
        alone.append(st.read())
    keep, b = [], dev.Batch(stream=stream)
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append(dm)
        b.add(st)
    b.compile()
    assert b.step(3) == 0
    for i, st in enumerate(b.members):
        got = st.read()
        for k in ("h", "u", "zeta", "ubar"):
            assert np.array_equal(got[k], alone[i][k]), (i, k)

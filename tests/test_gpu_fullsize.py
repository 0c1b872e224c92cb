"""GPU checks at the full benchmark sizes, in the launch configuration the
benchmark times.

At 512 x 512 cells x 60 layers (and the level-7 sphere) the FP64 oracle takes
about half a minute for one baroclinic forward-Euler pass and minutes per
step, so whole steps are checked through properties that hold at any size:
  * one baroclinic forward-Euler pass (all three column kernels) against the
    oracle on every edge, FP64 bound 1e-11;
  * total volume sum_i A_i sum_k h_ik conserved by whole steps to roundoff;
  * SSH equal to sum_k h_k - H after reconciliation;
  * the mixed-precision path against the FP64 path on the same inputs, with
    the mixed-precision bounds (velocity 1e-5, SSH against zeta + H 1e-9).
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import Setup
from synthetic import cases
from tests.helpers import rel_l2
from tests.test_gpu_parity import _report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


@pytest.fixture(scope="module")
def c1_full():
    return cases.c1()


def _volume(case, h):
    return float(np.sum(case.mesh.areaCell[:, None] * h * case.cell_mask[:, None]))


def test_c1_full_feuler_parity(dev, c1_full):
    """One forward-Euler pass of Algorithm 1 at 512 x 512 x 60 with velocity noise."""
    case = c1_full
    st_o = Setup.from_case(case)
    rng = np.random.default_rng(17)
    u = np.where(st_o.edge_mask[:, None], rng.normal(0.0, 0.05, case.u.shape), 0.0)
    h = case.h
    ubar, _ = S.split(u, h, st_o)
    zeta = S.ssh(h, st_o)
    ut1, G = S.baroclinic_feuler(u, u - ubar[:, None], zeta, h, case.params.dt, st_o)
    _, st = dev.state_from_case(case)
    g_ut1, g_G = st.debug_baroclinic_feuler(u, ubar, zeta, h, case.params.dt)
    errs = {"ut1": rel_l2(g_ut1, ut1), "G": rel_l2(g_G, G)}
    _report("full C1 feuler 512x512x60", errs)
    assert max(errs.values()) < 1e-11


def test_c1_full_steps_conserve_volume(dev, c1_full):
    case = c1_full
    dm, st = dev.state_from_case(case)
    v0 = _volume(case, case.h)
    assert st.step(3) == 0
    out = st.read()
    v1 = _volume(case, out["h"])
    ssh = out["h"].sum(axis=1) - case.H
    errs = {"volume": abs(v1 - v0) / v0,
            "ssh-sum": float(np.abs(out["zeta"] - ssh).max() / np.abs(case.H).max())}
    _report("full C1 3 steps FP64 invariants", errs)
    assert errs["volume"] < 1e-13
    assert errs["ssh-sum"] < 1e-14
    assert np.isfinite(out["u"]).all()


def test_c2_full_mixed_vs_fp64(dev):
    """Level-7 sphere, 60 layers, 30% land, M = 30: 20 steps mixed vs FP64."""
    case = cases.c2()
    res = {}
    for prec in (0, 1):
        dm, st = dev.state_from_case(cases.with_params(case, precision=prec))
        assert st.step(case.steps) == 0, dev.last_error()
        res[prec] = st.read()
        del st, dm
    a, b = res[1], res[0]
    mask = case.cell_mask.astype(bool)
    dz = np.linalg.norm((a["zeta"] - b["zeta"])[mask])
    errs = {"u": rel_l2(a["u"], b["u"]), "ubar": rel_l2(a["ubar"], b["ubar"]), "h": rel_l2(a["h"], b["h"]),
            "zeta/|zeta+H|": float(dz / np.linalg.norm((b["zeta"] + case.H)[mask])),
            "zeta/|zeta|": float(dz / np.linalg.norm(b["zeta"][mask])),
            "volume(mixed)": abs(_volume(case, a["h"]) - _volume(case, case.h)) / _volume(case, case.h)}
    _report("full C2 level 7 x 60, 20 steps, mixed vs FP64", errs)
    assert errs["u"] < 1e-5 and errs["ubar"] < 1e-5
    assert errs["h"] < 1e-9 and errs["zeta/|zeta+H|"] < 1e-9
    assert errs["volume(mixed)"] < 1e-13

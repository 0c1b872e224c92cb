"""GPU checks at the full benchmark sizes, in the launch configuration the
benchmark times.

At 512 x 512 cells x 60 layers (and on the level-7 sphere) the FP64 oracle
takes minutes per step, so whole steps are compared with oracle values stored
by ``tests/golden/make_fullsize.py`` (which calls the oracle only): three
SSPRK3-SE steps of the C1 recipe in FP64 and of the C2 recipe in FP64 and
both mixed modes, compared on a
seeded sample of every field (65,536 velocities, 32,768 values of h, zeta and
ubar).  The measures are the relative L2 over the sample and the largest
sampled element error relative to the field's largest magnitude.  Bounds:

  * C1 and C2, FP64: 1e-11 / 1e-10, or four times the spread that the oracle
    itself shows at full size between correctly rounded, top-down and
    bottom-up column sums (recorded beside the samples);
  * C2 in both mixed modes: velocity 1e-5, h 1e-9, SSH 1e-9 relative to
    zeta + H, SSH relative to zeta alone reported (and held to 1e-5).

Also at full size:
  * one baroclinic forward-Euler pass (all three column kernels) against the
    oracle on every edge, FP64 bound 1e-11;
  * total volume sum_i A_i sum_k h_ik conserved by whole steps to roundoff,
    SSH equal to sum_k h_k - H after reconciliation;
  * the mixed-precision path against the FP64 path over 20 steps of C2.
"""
import os

import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import Setup
from synthetic import cases
from tests import parity_cases as P
from tests.helpers import rel_l2
from tests.test_gpu_parity import _report

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

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


def _stored(name):
    with np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _sampled_errors(gpu, ref):
    out = {}
    for f in ("u", "h", "zeta", "ubar"):
        idx, val = ref[f"idx_{f}"], ref[f"val_{f}"]
        d = np.asarray(gpu[f]).ravel()[idx] - val
        out[f] = {"l2": float(np.linalg.norm(d) / np.linalg.norm(val)),
                  "max": float(np.abs(d).max() / float(ref[f"normmax_{f}"]))}
    return out


def test_c1_full_three_steps_against_the_oracle(dev, c1_full):
    """Three SSPRK3-SE steps of the C1 recipe at 512 x 512 x 60, FP64."""
    ref = _stored("c1")
    steps = int(ref["steps"])
    dm, st = dev.state_from_case(c1_full)
    assert st.step(steps) == 0, dev.last_error()
    errs = _sampled_errors(st.read(), ref)
    _report("full C1 512x512x60, 3 steps vs stored oracle samples: " + P.format_errors(errs))
    for f, e in errs.items():
        b2 = max(P.TOL_L2, P.AMPLIFICATION * float(ref[f"spread_l2_{f}"]))
        bm = max(P.TOL_MAX, P.AMPLIFICATION * float(ref[f"spread_inf_{f}"]))
        assert e["l2"] <= b2 and e["max"] <= bm, (f, e, b2, bm)


def test_c2_full_three_steps_fp64_against_the_oracle(dev):
    """Three SSPRK3-SE steps of the C2 recipe (level-7 sphere, 60 layers, 30 %
    land, M = 30) in FP64 against the same stored oracle samples, at the FP64
    bounds."""
    ref = _stored("c2")
    steps = int(ref["steps"])
    case = cases.c2()
    dm, st = dev.state_from_case(cases.with_params(case, precision=0))
    assert st.step(steps) == 0, dev.last_error()
    errs = _sampled_errors(st.read(), ref)
    _report("full C2 level 7 x 60, 3 steps, FP64 vs stored oracle samples: " + P.format_errors(errs))
    for f, e in errs.items():
        b2 = max(P.TOL_L2, P.AMPLIFICATION * float(ref[f"spread_l2_{f}"]))
        bm = max(P.TOL_MAX, P.AMPLIFICATION * float(ref[f"spread_inf_{f}"]))
        assert e["l2"] <= b2 and e["max"] <= bm, (f, e, b2, bm)


@pytest.mark.parametrize("prec", [1, 2])
def test_c2_full_three_steps_mixed_against_the_oracle(dev, prec):
    """Three steps of the C2 recipe (level-7 sphere, 60 layers, 30 % land,
    M = 30) in SSE_MIXED and SSE_MIXED_BT64 against the FP64 oracle."""
    ref = _stored("c2")
    steps = int(ref["steps"])
    case = cases.c2()
    dm, st = dev.state_from_case(cases.with_params(case, precision=prec))
    assert st.step(steps) == 0, dev.last_error()
    g = st.read()
    errs = _sampled_errors(g, ref)
    idx, val = ref["idx_zeta"], ref["val_zeta"]
    dz = g["zeta"][idx] - val
    zH = val + case.H[idx]
    wet = case.cell_mask[idx].astype(bool)
    ssh = {"zeta/|zeta+H|": float(np.linalg.norm(dz[wet]) / np.linalg.norm(zH[wet])),
           "zeta/|zeta|": float(np.linalg.norm(dz[wet]) / np.linalg.norm(val[wet]))}
    _report(f"full C2 level 7 x 60, 3 steps, precision {prec} vs stored oracle samples: "
            + P.format_errors(errs) + ", " + ", ".join(f"{k}={v:.2e}" for k, v in ssh.items()))
    assert errs["u"]["l2"] < 1e-5 and errs["ubar"]["l2"] < 1e-5, errs
    assert errs["h"]["l2"] < 1e-9, errs
    assert ssh["zeta/|zeta+H|"] < 1e-9 and ssh["zeta/|zeta|"] < 1e-5, ssh


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

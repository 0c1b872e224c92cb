"""Temporal convergence order of the oracle (the Theorem of Section 4; Tables 2-3).

Relative l2 errors of the surface velocity u_1 and the top-layer thickness h_1
(the Section 5 error metric) against a reference run of SSPRK3-SE with
dt = dt_btr, as in the paper's reference solutions; dt_btr halves at fixed M.
With reconciliation the paper observes rates approaching 2 for both schemes
(e.g. Table 2 "With SSH reconciliation", Table 3 likewise); the expected rates
are read from ``tests/golden/paper_convergence_rates.txt``.
"""
import os

import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import Setup
from synthetic.cases import with_params
from tests.helpers import rel_l2, smooth_case

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_convergence_rates.txt")
T_END = 1920.0


def _golden():
    rows = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if line:
            scheme, rate = line.split()[:2]
            rows[scheme] = float(rate)
    return rows


def _run(case, dt, M):
    c = with_params(case, dt=dt, substeps=M)
    st = Setup.from_case(c)
    u, h = c.u.copy(), c.h.copy()
    for _ in range(int(round(T_END / dt))):
        u, h = S.step(u, h, st)
    return u[:, 0], h[:, 0]


@pytest.fixture(scope="module")
def reference():
    base = smooth_case(n=12, L=3, scheme=3, amp_u=0.05)
    return base, _run(base, 7.5, 1)


@pytest.mark.slow
@pytest.mark.parametrize("scheme", ["SSPRK2-SE", "SSPRK3-SE"])
def test_second_order_in_time(reference, scheme):
    base, (u_ref, h_ref) = reference
    expect = _golden()[scheme]
    case = with_params(base, scheme=2 if scheme == "SSPRK2-SE" else 3)
    M = 4
    errs = []
    for dt_btr in (60.0, 30.0, 15.0):
        u1, h1 = _run(case, M * dt_btr, M)
        errs.append((rel_l2(u1, u_ref), rel_l2(h1, h_ref)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert (rates[-1] >= expect - 0.2).all(), (errs, rates)
    assert (errs[:, 0] < 0.05).all()

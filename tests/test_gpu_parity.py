"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Every comparison reports two measures per field: the relative L2 error and the
largest element error relative to the field's largest magnitude.  Kernel-level
comparisons (the debug entry points) must meet 1e-11 and 1e-10.  Whole steps
take their case and their bounds from ``tests/parity_cases.py``: 1e-11 / 1e-10,
or, where the oracle itself moves further under a different rounding of its
column sums or a one-ulp change of its inputs (measured on the CPU and recorded
in ``tests/golden/parity_bounds.json``), four times that measured spread.
Sizes are small enough for the oracle to finish in seconds, chosen with ragged
tails (entity counts that are not multiples of the 4-column blocks or the
256-thread 2D blocks).
"""
import os

import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import Setup
from synthetic import cases
from tests import parity_cases as P
from tests.helpers import smooth_case

pytestmark = pytest.mark.gpu

TOL = P.TOL_L2
TOL_MAX = P.TOL_MAX


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


def _report(name, errs=None):
    line = name if errs is None else f"[parity] {name}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items())
    print(line, flush=True)
    path = os.environ.get("SSE_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")


def _check_kernel(name, errs):
    """errs: {field: (gpu, oracle)}; both measures against 1e-11 / 1e-10."""
    e = {k: P.field_errors(g, r) for k, (g, r) in errs.items()}
    _report(name + ": " + P.format_errors(e))
    for k, v in e.items():
        assert v["l2"] <= TOL and v["max"] <= TOL_MAX, (name, k, v)
    return e


def run_case(dev, name, **state_kw):
    """Runs a case of ``tests/parity_cases.py`` on the GPU and in the oracle."""
    case, steps = P.build(name)
    dm, st = dev.state_from_case(case, **state_kw)
    rc = st.step(steps)
    gpu = st.read()
    if getattr(case.params, "tracer", 0):
        gpu["T"] = st.read_tracer()
    return rc, gpu, P.oracle_fields(case, steps)


def check_case(dev, name):
    rc, gpu, ref = run_case(dev, name)
    assert rc == 0, dev.last_error()
    return P.check(name, gpu, ref, report=_report)


def _noisy_state(case, steps=3, seed=0):
    """A non-trivial state of a case, advanced by the oracle."""
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    rng = np.random.default_rng(seed)
    u = np.where(st.edge_mask[:, None], u + rng.normal(0, 0.01, u.shape), 0.0)
    for _ in range(steps):
        u, h = S.step(u, h, st)
    return u, h


# ---------------------------------------------------------------------------
# per-kernel parity through the debug entry points
# ---------------------------------------------------------------------------
KERNEL_CASES = {
    "hex10x6_L4": lambda: cases.with_params(smooth_case(n=10, L=4), scheme=3),
    "hex12_L20_generic_stencils": lambda: P.build("generic_stencils_hex12_L20")[0],
    "sphere3_land_L7": lambda: cases.sphere_case(3, 7, 77, substeps=5, dt_btr=200.0),
    "hex8_L100": lambda: cases.c1(n=8, L=100, steps=1),
    "hex12_L64": lambda: cases.c1(n=12, L=64, steps=1),
    "sphere3_land_L8": lambda: cases.sphere_case(3, 8, 78, substeps=5, dt_btr=200.0),
}


@pytest.mark.parametrize("name", sorted(KERNEL_CASES))
def test_baroclinic_feuler_parity(dev, name):
    case = KERNEL_CASES[name]()
    st_o = Setup.from_case(case)
    u, h = _noisy_state(case, steps=1)
    ubar, _ = S.split(u, h, st_o)
    ut = u - ubar[:, None]
    zeta = S.ssh(h, st_o)
    ut1, G = S.baroclinic_feuler(u, ut, zeta, h, case.params.dt, st_o)
    _, st = dev.state_from_case(case)
    g_ut1, g_G = st.debug_baroclinic_feuler(u, ubar, zeta, h, case.params.dt)
    _check_kernel(f"feuler {name}", {"ut1": (g_ut1, ut1), "G": (g_G, G)})


@pytest.mark.parametrize("name", sorted(KERNEL_CASES))
@pytest.mark.parametrize("scheme", [2, 3])
def test_barotropic_substep_parity(dev, name, scheme):
    case = KERNEL_CASES[name]()
    st_o = Setup.from_case(case)
    rng = np.random.default_rng(5)
    ubar = np.where(st_o.edge_mask, rng.normal(0, 0.05, case.mesh.nEdges), 0.0)
    zeta = np.where(st_o.cell_mask, rng.normal(0, 0.05, case.mesh.nCells), 0.0)
    G = np.where(st_o.edge_mask, rng.normal(0, 1e-5, case.mesh.nEdges), 0.0)
    M, dt = 7, case.params.dt
    sub = S.barotropic_ssprk2_substep if scheme == 2 else S.barotropic_ssprk3_substep
    u1, z1, F = sub(ubar, zeta, G, dt, M, st_o)
    _, st = dev.state_from_case(case)
    g_u1, g_z1, g_F = st.debug_barotropic_substep(scheme, M, dt, ubar, zeta, G)
    _check_kernel(f"bt{scheme} {name}", {"ubar": (g_u1, u1), "zeta": (g_z1, z1), "Fzeta": (g_F, F)})


@pytest.mark.parametrize("name", sorted(KERNEL_CASES))
@pytest.mark.parametrize("vcoord", [0, 1])
def test_thickness_stage_parity(dev, name, vcoord):
    case = cases.with_params(KERNEL_CASES[name](), vcoord=vcoord)
    st_o = Setup.from_case(case)
    u, h = _noisy_state(case, steps=1)
    rng = np.random.default_rng(9)
    uA = np.where(st_o.edge_mask, rng.normal(0, 1e-3, case.mesh.nEdges), 0.0)
    dt = case.params.dt
    h_out = S.thickness_stage(h, u, uA, dt, st_o)
    z_out = S.ssh(h_out, st_o)
    _, st = dev.state_from_case(case)
    g_h, g_z = st.debug_thickness_stage(h, u, uA, dt)
    _check_kernel(f"thickness vcoord={vcoord} {name}", {"h": (g_h, h_out), "zeta": (g_z, z_out)})


# ---------------------------------------------------------------------------
# whole steps
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["c0_ssprk3_100", "c0_ssprk3_20", "c1_recipe_32x32x60",
                                  "c2_recipe_level3x60", "hex8_L100", "generic_stencils_hex12_L20",
                                  "generic_stencils_sphere3_land_L7"])
def test_whole_steps(dev, name):
    """C0 geometry with SSPRK3-SE over 20 and 100 steps; the C1 recipe (bathymetry,
    density front, 60 layers, M = 20) on a 32x32 hex; the C2 recipe (sphere,
    30 % land, variable f, 60 layers, M = 30) at level 3; L = 100 > 64 layers
    (two register chunks per lane); meshes whose reconstruction stencils are
    not all other edges of the two cells, so that the edge pass runs on its
    generic tables."""
    check_case(dev, name)


def test_c0_ssprk2_stable_window(dev):
    """C0 as specified (SSPRK2-SE, dt = 300 s, M = 10): parity over the first 30 steps."""
    check_case(dev, "c0_ssprk2_30")


def test_c0_ssprk2_blowup_is_reported(dev):
    """SSPRK2 amplifies undamped gravity waves (|R_2(iy)| > 1): C0 blows up
    within 100 steps on both sides; the library reports SSE_ENONFINITE."""
    case = cases.c0()
    dm, st = dev.state_from_case(case)
    rc = st.step(100)
    with np.errstate(all="ignore"):
        u, h, zeta, ubar = S.run(case, 100)
    assert not np.isfinite(u).all()
    assert rc == dev.SSE_ENONFINITE


@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("reconcile", [0, 1, 2])
def test_reconcile_modes(dev, scheme, reconcile):
    check_case(dev, f"reconcile{reconcile}_ssprk{scheme}")


@pytest.mark.parametrize("scheme", [2, 3])
def test_isopycnal_steps(dev, scheme):
    check_case(dev, f"isopycnal_ssprk{scheme}")


def test_determinism_bitwise(dev):
    case = cases.c1(n=16, L=20, steps=3)
    outs = []
    for _ in range(2):
        dm, st = dev.state_from_case(case)
        assert st.step(3) == 0
        outs.append(st.read())
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_checkpoint_resume_bitwise(dev):
    case = cases.with_params(cases.c0(), scheme=3)
    dm, st = dev.state_from_case(case)
    assert st.step(10) == 0
    full = st.read()
    dm2, st2 = dev.state_from_case(case)
    assert st2.step(5) == 0
    mid = st2.read()
    dm3 = dev.DeviceMesh(case.mesh, case.H, case.cell_mask)
    st3 = dev.DeviceState(dm3, case.params)
    st3.init(mid["h"], mid["u"], case.rho, case.h_ref)
    assert st3.step(5) == 0
    res = st3.read()
    for k in full:
        assert np.array_equal(full[k], res[k]), k


def test_nonfinite_input_rejected(dev):
    case = cases.c0()
    dm = dev.DeviceMesh(case.mesh, case.H, case.cell_mask)
    st = dev.DeviceState(dm, case.params)
    h = case.h.copy()
    h[3, 1] = np.nan
    with pytest.raises(dev.SSEError) as ei:
        st.init(h, case.u, case.rho, case.h_ref)
    assert ei.value.code == dev.SSE_ENONFINITE


# ---------------------------------------------------------------------------
# edge-pass variants (direct gathers with 32-bit column offsets or, -2, with
# 64-bit column addresses as meshes with 4 GiB arrays take; LDS tiles of 8 /
# 16 / 32 edges)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["hex12_L64", "hex8_L100", "sphere3_land_L7", "sphere3_land_L8"])
@pytest.mark.parametrize("variant", [-2, 0, 1, 2])
def test_edge_variant_feuler_parity(dev, name, variant):
    case = KERNEL_CASES[name]()
    st_o = Setup.from_case(case)
    u, h = _noisy_state(case, steps=1)
    ubar, _ = S.split(u, h, st_o)
    zeta = S.ssh(h, st_o)
    ut1, G = S.baroclinic_feuler(u, u - ubar[:, None], zeta, h, case.params.dt, st_o)
    _, st = dev.state_from_case(case)
    if not st.try_edge_variant(variant):
        pytest.skip(f"variant {variant} does not fit: {dev.last_error()}")
    g_ut1, g_G = st.debug_baroclinic_feuler(u, ubar, zeta, h, case.params.dt)
    _check_kernel(f"feuler variant={variant} {name}", {"ut1": (g_ut1, ut1), "G": (g_G, G)})


@pytest.mark.parametrize("variant", [-2, 0, 1, 2])
def test_edge_variants_bitwise_equal(dev, variant):
    """Every variant performs the same arithmetic on the same operands: whole
    steps agree bit for bit with the direct-gather kernel."""
    case = cases.c1(n=16, L=60, steps=3)
    out = {}
    for v in (-1, variant):
        _, st = dev.state_from_case(case)
        assert st.try_edge_variant(v), dev.last_error()
        assert st.step(3) == 0
        out[v] = st.read()
    for k in out[-1]:
        assert np.array_equal(out[-1][k], out[variant][k]), k


@pytest.mark.parametrize("precision", [0, 1])
def test_wide_addressing_bitwise_equal(dev, precision):
    """64-bit column addressing (the form meshes with arrays of 4 GiB or more
    take) against 32-bit offsets, with every optional term on and two
    register chunks, alone and in a batch."""
    import torch
    from tests.parity_cases import all_terms
    case = cases.with_params(all_terms(cases.c1(n=10, L=100, steps=2)), precision=precision)
    out = {}
    for v in (-1, -2):
        _, st = dev.state_from_case(case)
        assert st.try_edge_variant(v), dev.last_error()
        assert st.step(2) == 0, dev.last_error()
        out[v] = st.read()
        out[v]["T"] = st.read_tracer()
    for k in out[-1]:
        assert np.array_equal(out[-1][k], out[-2][k]), k
    stream = torch.cuda.Stream()
    keep, b = [], dev.Batch(stream=stream)
    for v in (-2, -1):
        dm, st = dev.state_from_case(case, stream=stream)
        assert st.try_edge_variant(v), dev.last_error()
        keep.append(dm)
        b.add(st)
    b.compile()
    assert b.step(2) == 0, dev.last_error()
    for st in b.members:
        got = st.read()
        got["T"] = st.read_tracer()
        for k in out[-1]:
            assert np.array_equal(got[k], out[-1][k]), k


# ---------------------------------------------------------------------------
# barotropic loop variants (one launch per evaluation, one per substep, one per loop)
# ---------------------------------------------------------------------------
BT_CASES = {
    "c0_one_patch": lambda: cases.c0(),
    "hex32_L60": lambda: cases.c1(n=32, L=60, steps=3),
    "sphere3_land_L7": lambda: cases.sphere_case(3, 7, 77, substeps=5, dt_btr=200.0),
    "sphere4_land_L9": lambda: cases.sphere_case(4, 9, 78, substeps=6, dt_btr=120.0),
}


@pytest.mark.parametrize("name", sorted(BT_CASES))
@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_bt_variants_bitwise_equal(dev, name, scheme, precision):
    """The per-substep (patch) kernel and the persistent loop kernel (all
    substeps in one cooperative launch) perform the per-evaluation kernel's
    arithmetic on the same operands: whole steps agree bit for bit."""
    case = cases.with_params(BT_CASES[name](), scheme=scheme, precision=precision)
    out = {}
    for v in (0, 1, 2):
        _, st = dev.state_from_case(case)
        assert st.try_bt_variant(v), (v, dev.last_error())
        assert st.bt_variant == v
        assert st.step(2) == 0
        out[v] = st.read()
    for v in (1, 2):
        for k in out[0]:
            assert np.array_equal(out[0][k], out[v][k]), (v, k)


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_loop_in_graph_and_eager_alike(dev, precision):
    """A step captured as a HIP graph runs the per-substep kernel in place of
    the persistent loop (a cooperative launch); replays and eager steps agree
    bit for bit."""
    import torch
    case = cases.with_params(BT_CASES["sphere4_land_L9"](), precision=precision)
    stream = torch.cuda.Stream()
    _, eager = dev.state_from_case(case, stream=stream)
    _, g = dev.state_from_case(case, stream=stream)
    assert eager.try_bt_variant(2) and g.try_bt_variant(2), dev.last_error()
    g.use_graph(True)
    for k in range(3):
        assert eager.step(1) == 0
        assert g.step(1) == 0
        a, b = eager.read(), g.read()
        for f in a:
            assert np.array_equal(a[f], b[f]), (k, f)


def test_persistent_loop_barrier_timeout_is_reported(dev):
    """A grid barrier that gives up (forced from the host with a one-poll limit)
    lets every workgroup finish; the step reports SSE_EDEVICE, and after
    initialising again the state steps and matches the per-substep kernel."""
    case = BT_CASES["sphere4_land_L9"]()
    _, ref = dev.state_from_case(case)
    assert ref.step(2) == 0
    want = ref.read()
    _, st = dev.state_from_case(case)
    assert st.try_bt_variant(2), dev.last_error()
    st.set_barrier_spins(1)
    with pytest.raises(dev.SSEError) as info:
        st.step(1)
    assert "barrier" in str(info.value)
    st.set_barrier_spins(0)
    st.init(case.h, case.u, case.rho, case.h_ref)
    assert st.step(2) == 0
    got = st.read()
    for k in want:
        assert np.array_equal(want[k], got[k]), k


@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_barotropic_substep_variants_parity(dev, scheme, variant):
    case = KERNEL_CASES["sphere3_land_L7"]()
    st_o = Setup.from_case(case)
    rng = np.random.default_rng(15)
    ubar = np.where(st_o.edge_mask, rng.normal(0, 0.05, case.mesh.nEdges), 0.0)
    zeta = np.where(st_o.cell_mask, rng.normal(0, 0.05, case.mesh.nCells), 0.0)
    G = np.where(st_o.edge_mask, rng.normal(0, 1e-5, case.mesh.nEdges), 0.0)
    M, dt = 8, case.params.dt
    sub = S.barotropic_ssprk2_substep if scheme == 2 else S.barotropic_ssprk3_substep
    u1, z1, F = sub(ubar, zeta, G, dt, M, st_o)
    _, st = dev.state_from_case(case)
    assert st.try_bt_variant(variant), dev.last_error()
    g_u1, g_z1, g_F = st.debug_barotropic_substep(scheme, M, dt, ubar, zeta, G)
    _check_kernel(f"bt{scheme} variant={variant}", {"ubar": (g_u1, u1), "zeta": (g_z1, z1), "Fzeta": (g_F, F)})

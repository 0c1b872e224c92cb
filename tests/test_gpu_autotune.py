"""The launch-configuration tuner on the GPU: whatever setting it picks
(workgroup shapes, edge-pass variant, barotropic-loop kernel), a state or a
batch tuned by it computes the same bits as with the defaults."""
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


def _same(a, b, what):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), (what, k, float(np.abs(a[k] - b[k]).max()))


@pytest.mark.parametrize("precision", [0, 1])
def test_tuned_state_gives_default_bits(dev, stream, precision):
    from paper_2105_13484_amd import autotune
    case = cases.with_params(cases.c1(n=24, L=20, steps=3), precision=precision)
    _, ref = dev.state_from_case(case, stream=stream)
    assert ref.step(3) == 0
    want = ref.read()
    _, st = dev.state_from_case(case, stream=stream)
    res = autotune.tune_state(st, steps=1)
    best = res["best"]
    print(f"\n[autotune] state precision {precision}: {best}, default {res['default_ms']:.3f} ms/step, "
          f"{len(res['trials'])} trials", flush=True)
    assert set(best) == {"cols_per_block", "block_2d", "edge_variant", "bt_variant"}
    assert st.bt_variant == best["bt_variant"]
    st.init(case.h, case.u, case.rho, case.h_ref)
    assert st.step(3) == 0
    _same(st.read(), want, f"tuned {best}")


def test_tuned_batch_gives_solo_bits(dev, stream):
    from paper_2105_13484_amd import autotune
    cs = [cases.with_params(cases.c1(n=n, L=L, substeps=M, member=i, steps=2), precision=1)
          for i, (n, L, M) in enumerate([(12, 20, 6), (16, 40, 9), (10, 8, 4)])]
    alone = []
    for c in cs:
        _, st = dev.state_from_case(c, stream=stream)
        assert st.step(2) == 0
        alone.append(st.read())
    keep, b = [], dev.Batch(stream=stream)
    for c in cs:
        dm, st = dev.state_from_case(c, stream=stream)
        keep.append((dm, st))
        b.add(st)
    res = autotune.tune_batch(b, steps=1)
    best = res["best"]
    print(f"\n[autotune] batch: {best}, default {res['default_ms']:.3f} ms/step, {len(res['trials'])} trials",
          flush=True)
    assert all(st.bt_variant == best["bt_variant"] for _, st in keep)
    for c, (_, st) in zip(cs, keep):
        st.init(c.h, c.u, c.rho, c.h_ref)
    assert b.step(2) == 0
    for i, (_, st) in enumerate(keep):
        _same(st.read(), alone[i], f"member {i} after tuning {best}")
    b.close()

"""The sweep launch variants change speed only: every variant gives the same
state bit for bit; autotuning leaves the simulation state untouched and the
cache reuses its choice."""
import numpy as np
import pytest

from paper_1908_01762_amd import autotune, cases

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01762_amd import sisph
    return sisph


@pytest.mark.parametrize("case", [cases.taylor_green(60, kernel="wendland", hdx=1.3, precision="mixed"),
                                  cases.dam_break_2d(dx=0.05, precision="fp64")],
                         ids=["tg60_mixed", "db2d_fp64"])
def test_variants_are_bitwise_identical(case):
    sisph = _gpu()
    ref = None
    for v in range(sisph.SWEEP_VARIANTS):
        ctx = sisph.Context(case)
        ctx.variant = v
        ctx.step(3)
        st = ctx.read_state()
        ctx.close()
        if ref is None:
            ref = st
        else:
            for k in ("x", "u", "ut", "p"):
                assert np.array_equal(st[k], ref[k]), (v, k)


def test_autotune_keeps_state_and_caches(tmp_path):
    sisph = _gpu()
    case = cases.taylor_green(80, kernel="wendland", hdx=1.3, precision="mixed")
    a, b = sisph.Context(case), sisph.Context(case)
    a.step(1)
    b.step(1)
    path = str(tmp_path / "tune.json")
    rec = autotune.tune(a, cache_path=path, reps=5)
    print(rec, flush=True)
    assert 0 <= rec["variant"] < sisph.SWEEP_VARIANTS and len(rec["us"]) == sisph.SWEEP_VARIANTS
    assert a.variant == rec["variant"]
    a.step(2)
    b.step(2)
    sa, sb = a.read_state(), b.read_state()
    for k in ("x", "u", "ut", "p"):
        assert np.array_equal(sa[k], sb[k]), k
    c = sisph.Context(case)
    assert autotune.apply_cached(c, cache_path=path) and c.variant == rec["variant"]
    for x in (a, b, c):
        x.close()

"""GTVF short lists (external flows, smoothing length h/2, section 2.1):
the sub-steps walking the short lists give the same state, bit for bit, as
walking the full r* lists, and they are really used.  GPU only."""
import numpy as np
import pytest

from paper_1908_01762_amd import cases

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01762_amd import sisph
    return sisph


def say(*a):
    print(*a, flush=True)


def _run(sisph, case, steps, short):
    ctx = sisph.Context(case)
    if not short:
        ctx.debug_gtvf_short(False)
    used = []
    for _ in range(steps):
        ctx.step(1)
        used.append(ctx.debug_gtvf_short())
    st = ctx.read_state()
    ctx.close()
    return st, used


@pytest.mark.parametrize("name,case", [
    ("db2d_mixed", cases.dam_break_2d(dx=0.05, precision="mixed")),
    ("db2d_fp64", cases.dam_break_2d(dx=0.05, precision="fp64")),
    ("db2d_fp32", cases.dam_break_2d(dx=0.05, precision="fp32")),
    ("db3d_mixed", cases.dam_break_3d(dx=0.05, lx=0.4, ly=0.3, lz=0.5, tank_x=1.0, tank_y=0.3, tank_z=0.8,
                                      precision="mixed")),
])
def test_short_lists_match_full_lists_bitwise(name, case):
    sisph = _gpu()
    steps = 8
    say("case", name, case.n_fluid, case.n_wall)
    a, used = _run(sisph, case, steps, True)
    b, off = _run(sisph, case, steps, False)
    say("  short lists used per step", used)
    assert used == [1] * steps and off == [0] * steps
    for k in ("x", "u", "ut", "p"):
        assert np.array_equal(a[k], b[k]), k


def test_internal_flows_have_no_short_lists():
    sisph = _gpu()
    case = cases.taylor_green(16, kernel="wendland", hdx=1.3, precision="mixed")
    ctx = sisph.Context(case)
    ctx.step(1)
    assert ctx.debug_gtvf_short() == 0
    with pytest.raises(sisph.SisphError):
        ctx.debug_gtvf_short(True)
    ctx.close()

"""The allocation-free entry point, sisph_create_static, through the C ABI.

Its contexts live in the library's static device workspace instead of a
caller-owned one.  Two calls in a row (a walled free-surface case, then a
smaller periodic one, which finds the first case's data in the array) must
give bitwise the results of sisph_create on the same cases: the same
kernels run on the same values, only the addresses differ.  The entry
point refuses a case above the array's size, a second live context on the
device, and the features that would allocate.
"""
import numpy as np
import pytest

from paper_1908_01762_amd import cases

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01762_amd import sisph
    return sisph


def say(*a):
    print(*a, flush=True)


def _run(sisph, case, static, steps=3):
    ctx = sisph.Context(case, device="cuda:0", static=static)
    st = ctx.step(steps)
    s = ctx.read_state()
    s["rhs"] = ctx.field("rhs")
    ctx.close()
    return s, [x["iters"] for x in st]


def test_static_workspace_equals_caller_workspace():
    sisph = _gpu()
    first = cases.dam_break_2d(dx=0.02, precision="mixed")
    second = cases.taylor_green(40, kernel="wendland", hdx=1.3, jitter=0.2, seed=3)
    assert sisph.workspace_bytes(second) < sisph.workspace_bytes(first) <= sisph.STATIC_WORKSPACE_BYTES
    say("static runs:", first.name, first.n, "then", second.name, second.n)
    got = [_run(sisph, c, True) for c in (first, second)]
    say("caller-workspace runs")
    want = [_run(sisph, c, False) for c in (first, second)]
    for (a, ia), (b, ib), c in zip(got, want, (first, second)):
        say(f"  {c.name}: sweeps static {ia} caller {ib}")
        assert ia == ib
        for k in b:
            assert np.array_equal(a[k], b[k]), (c.name, k)


def test_static_workspace_refusals():
    sisph = _gpu()
    L = sisph.lib()
    big = cases.dam_break_2d(dx=0.004)
    assert sisph.workspace_bytes(big) > sisph.STATIC_WORKSPACE_BYTES
    with pytest.raises(sisph.SisphError) as e:
        sisph.Context(big, device="cuda:0", static=True)
    assert e.value.code == sisph.E_NOMEM and "static workspace" in str(e.value)
    small = cases.taylor_green(16)
    ctx = sisph.Context(small, device="cuda:0", static=True)
    with pytest.raises(sisph.SisphError) as e:
        sisph.Context(small, device="cuda:0", static=True)
    assert e.value.code == sisph.E_STATE
    assert L.sisph_set_graphs(ctx.h, 1) == sisph.E_STATE
    assert L.sisph_set_kernel_timing(ctx.h, 1) == sisph.E_STATE
    ctx.step(1)
    with pytest.raises(sisph.SisphError) as e:
        ctx.autotune(2)
    assert e.value.code == sisph.E_STATE
    ctx.close()
    # released: the device's array takes a new context
    ctx = sisph.Context(small, device="cuda:0", static=True)
    ctx.step(1)
    ctx.close()

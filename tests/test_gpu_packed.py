"""The packed mode of the Jacobi sweep (walled cases on grids periodic in no
direction): each sweep workgroup copies the iterate its rows can reach into
LDS and reads it through 12-bit positions, or reads the lists where its copy
would not fit.  The values, the sums and their order are those of the list
path, so the same case stepped with the packed mode switched off must give
bitwise the same iterates, sweep counts and state.  Covered: 2D and 3D dam
breaks (3D large enough that some workgroups read the lists), the cavity,
mixed, FP64 and plain FP32."""
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


def _cases():
    return {
        "db2d_mixed": cases.dam_break_2d(dx=0.02, precision="mixed"),
        "db2d_fp64": cases.dam_break_2d(dx=0.05, precision="fp64"),
        "db2d_fp32": cases.dam_break_2d(dx=0.05, precision="fp32"),
        "db3d_mixed": cases.dam_break_3d(dx=0.03, precision="mixed"),
        "db3d_fp64": cases.dam_break_3d(dx=0.05, precision="fp64"),
        "ldc40_mixed": cases.lid_driven_cavity(40, precision="mixed"),
    }


def _run(sisph, case, packed, steps):
    ctx = sisph.Context(case)
    if not packed:
        ctx.debug_packed(False)
    st = ctx.step(steps)
    s = ctx.read_state()
    ctx.close()
    return s, st


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_packed_equals_lists(name):
    sisph = _gpu()
    case = _cases()[name]
    say("case", name, case.n_fluid, "fluid", case.n_wall, "wall")
    a, sa = _run(sisph, case, True, 4)
    b, sb = _run(sisph, case, False, 4)
    say("  iters", [x["iters"] for x in sa], "index bits", sa[-1]["index_bits"], "/", sb[-1]["index_bits"],
        "list workgroups", [x["list_blocks"] for x in sa])
    assert all(x["index_bits"] == 12 for x in sa) and all(x["index_bits"] == 32 for x in sb)
    assert all(x["list_blocks"] == 0 for x in sb)
    for x, y in zip(sa, sb):
        x = dict(x, index_bits=0, list_blocks=0)
        y = dict(y, index_bits=0, list_blocks=0)
        assert x == y
    for k in ("x", "u", "ut", "p", "rho"):
        assert np.array_equal(a[k], b[k]), k


def test_packed_mode_switch_is_refused_without_walls():
    sisph = _gpu()
    ctx = sisph.Context(cases.taylor_green(12))
    with pytest.raises(sisph.SisphError) as e:
        ctx.debug_packed(True)
    assert e.value.code == sisph.E_INVAL
    ctx.debug_packed(False)   # a no-op there
    ctx.close()

"""Graph replay of the fixed step segments: every replay gives bitwise the
state of the launches one by one (the replays alternate with eager sweep
chunks and host polls), alone and batched, also after the batch's
membership changes and the graphs are captured again."""
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


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("x", "u", "ut", "p"))


def _cases():
    return {
        "tg40_mixed": cases.taylor_green(40, kernel="wendland", hdx=1.3, precision="mixed", seed=1),
        "db2d_fp64": cases.dam_break_2d(dx=0.1, precision="fp64"),
        "db3d_mixed": cases.dam_break_3d(dx=0.1, lx=0.4, ly=0.4, lz=0.5, tank_x=1.0, tank_y=0.4, tank_z=0.8,
                                         precision="mixed"),
        "ldc24_adaptive": cases.lid_driven_cavity(24, dt=0.02).replace(dt_mode="adaptive"),
        # wall-less: one persistent launch per solve, adaptive step
        "tg30_adaptive_mixed": cases.taylor_green(30, kernel="wendland", hdx=1.3, precision="mixed",
                                                  seed=2).replace(dt_mode="adaptive"),
        "db2d_bicgstab": cases.dam_break_2d(dx=0.1, precision="fp64").replace(solver="bicgstab", tol=1e-4),
    }


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_graph_steps_equal_eager(name):
    sisph = _gpu()
    case = _cases()[name]
    say("case", name)
    a, b = sisph.Context(case), sisph.Context(case)
    b.use_graphs(True)
    for k in range(6):
        sa, sb = a.step(1)[0], b.step(1)[0]
        assert sa == sb, k
        assert _same(a.read_state(), b.read_state()), k
    a.close()
    b.close()


def test_graph_batch_equals_solo_with_membership_changes():
    sisph = _gpu()
    mix = [cases.taylor_green(24, kernel="wendland", hdx=1.3, precision="mixed", seed=1),
           cases.dam_break_2d(dx=0.1, precision="mixed"),
           cases.taylor_green(17, kernel="wendland", hdx=1.3, precision="mixed", seed=3, tol=1e-2)]
    steps = {0: 5, 1: 3, 2: 3}
    ref = []
    for k, c in enumerate(mix):
        ctx = sisph.Context(c)
        ctx.step(steps[k])
        ref.append(ctx.read_state())
        ctx.close()
    ctxs = [sisph.Context(c) for c in mix]
    bt = sisph.Batch(4)
    bt.use_graphs(True)
    bt.attach(ctxs[0])
    bt.attach(ctxs[1])
    for _ in range(3):
        bt.step()              # captured once, replayed
    bt.detach(ctxs[1])         # membership change: captured again
    bt.attach(ctxs[2])
    for _ in range(2):
        bt.step()
    bt.detach(ctxs[0])
    bt.step()
    bt.detach(ctxs[2])
    for k, ctx in enumerate(ctxs):
        assert _same(ctx.read_state(), ref[k]), k
    bt.close()
    for ctx in ctxs:
        ctx.close()

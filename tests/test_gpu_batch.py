"""Batched stepping: a case gives bitwise the same state alone and inside a
batch of uneven cases (its workgroups, sums and stopping decisions do not
depend on the other cases), across groups of different dimension, kernel
and precision, with cases attached and detached between steps."""
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


def _mix():
    return [
        cases.taylor_green(24, kernel="wendland", hdx=1.3, precision="mixed", seed=1),
        cases.taylor_green(40, kernel="wendland", hdx=1.3, precision="mixed", seed=2, re=500.0),
        cases.dam_break_2d(dx=0.1, precision="mixed"),
        cases.taylor_green(17, kernel="wendland", hdx=1.3, precision="mixed", seed=3, tol=1e-2),
        cases.taylor_green(30, precision="fp64", seed=4),                 # other group: quintic FP64
        cases.dam_break_3d(dx=0.1, lx=0.4, ly=0.4, lz=0.5, tank_x=1.0, tank_y=0.4, tank_z=0.8,
                           precision="mixed"),                            # other group: 3D
        cases.dam_break_2d(dx=0.08, precision="mixed").replace(dt_mode="adaptive"),
        cases.dam_break_2d(dx=0.1, precision="fp32"),                    # other group: plain FP32
        cases.taylor_green(20, kernel="wendland", hdx=1.3, precision="fp32", seed=5),
    ]


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("x", "u", "ut", "p"))


def test_batch_equals_alone_bitwise():
    sisph = _gpu()
    steps = 6
    alone = []
    for c in _mix():
        say("alone", c.name, c.n_fluid, c.n_wall)
        ctx = sisph.Context(c)
        its = [s["iters"] for s in ctx.step(steps)]
        alone.append((ctx.read_state(), its))
        ctx.close()
    ctxs = [sisph.Context(c) for c in _mix()]
    b = sisph.Batch(16)
    for ctx in ctxs:
        b.attach(ctx)
    its_b = [[] for _ in ctxs]
    for _ in range(steps):
        for k, s in enumerate(b.step()):
            its_b[k].append(s["iters"])
    for k, ctx in enumerate(ctxs):
        b.detach(ctx)
        st = ctx.read_state()
        say("case", k, "iters alone", alone[k][1], "batched", its_b[k])
        assert its_b[k] == alone[k][1]
        assert _same(st, alone[k][0]), k
    b.close()
    for ctx in ctxs:
        ctx.close()


def test_attach_detach_between_steps():
    """Cases join and leave; each still matches its own solo run."""
    sisph = _gpu()
    mix = _mix()[:4]
    ref = []
    for c in mix:
        ctx = sisph.Context(c)
        ctx.step(5)
        ref.append(ctx.read_state())
        ctx.close()
    ctxs = [sisph.Context(c) for c in mix]
    b = sisph.Batch(8)
    b.attach(ctxs[0])
    b.attach(ctxs[1])
    b.step()                   # batch step 1: cases 0, 1
    b.step()                   # 2: 0, 1
    b.attach(ctxs[2])          # joins two steps late
    ctxs[3].step(2)            # runs alone meanwhile
    b.attach(ctxs[3])
    b.step()                   # 3: 0, 1, 2, 3
    b.detach(ctxs[0])          # leaves after 3 steps, finishes alone
    ctxs[0].step(2)
    b.step()                   # 4: 1, 2, 3
    b.step()                   # 5: 1, 2, 3
    b.detach(ctxs[1])          # 5 steps
    b.detach(ctxs[3])          # 2 alone + 3 batched
    b.step()                   # 6: 2
    b.step()                   # 7: 2
    b.detach(ctxs[2])          # steps 3..7
    for k, ctx in enumerate(ctxs):
        st = ctx.read_state()
        assert _same(st, ref[k]), k
    b.close()


def test_small_cases_join_after_a_large_one_leaves():
    """The group then holds more cases than before but fewer workgroups in
    total; every per-case map must still be sized for the case count (a
    map sized by the old count corrupted the workgroup-to-case maps)."""
    sisph = _gpu()
    big = cases.taylor_green(48, kernel="wendland", hdx=1.3, precision="mixed", seed=11)
    small = [cases.taylor_green(n, kernel="wendland", hdx=1.3, precision="mixed", seed=12 + n)
             for n in (12, 14, 16)]
    steps = {0: 1, 1: 3, 2: 2, 3: 2}
    allc = [big] + small
    ref = []
    for k, c in enumerate(allc):
        ctx = sisph.Context(c)
        ctx.step(steps[k])
        ref.append(ctx.read_state())
        ctx.close()
    ctxs = [sisph.Context(c) for c in allc]
    b = sisph.Batch(8)
    b.attach(ctxs[0])
    b.attach(ctxs[1])
    b.step()
    b.detach(ctxs[0])
    b.attach(ctxs[2])
    b.attach(ctxs[3])
    b.step()
    b.step()
    for k, ctx in enumerate(ctxs):
        if ctx in b.members:
            b.detach(ctx)
        say("case", k, allc[k].name)
        assert _same(ctx.read_state(), ref[k]), k
    b.close()
    for ctx in ctxs:
        ctx.close()


def test_stepping_an_attached_context_directly_is_refused():
    sisph = _gpu()
    c = sisph.Context(cases.taylor_green(16))
    b = sisph.Batch(2)
    b.attach(c)
    with pytest.raises(sisph.SisphError) as e:
        c.step(1)
    assert e.value.code == sisph.E_STATE
    b.close()
    c.step(1)   # usable again once the batch is gone
    c.close()


def test_a_failing_case_does_not_disturb_the_others():
    sisph = _gpu()
    good = cases.taylor_green(20, kernel="wendland", hdx=1.3, precision="mixed")
    bad = good.copy()
    bad.u[3, 1] = np.inf
    solo = sisph.Context(good)
    solo.step(1)
    ref = solo.read_state()
    b = sisph.Batch(4)
    cg, cb = sisph.Context(good), sisph.Context(bad)
    b.attach(cg)
    b.attach(cb)
    with pytest.raises(sisph.SisphError) as e:
        b.step()
    assert e.value.code == sisph.E_NONFINITE
    b.detach(cg)
    assert _same(cg.read_state(), ref)
    b.close()


def _run_batch(sisph, mix, steps, persistent):
    ctxs = [sisph.Context(c) for c in mix]
    b = sisph.Batch(16)
    b.use_persistent(persistent)
    for ctx in ctxs:
        b.attach(ctx)
    its = [[] for _ in ctxs]
    for _ in range(steps):
        for k, s in enumerate(b.step()):
            its[k].append(s["iters"])
    info = b.persistent_info()
    states = []
    for ctx in ctxs:
        b.detach(ctx)
        states.append(ctx.read_state())
    b.close()
    for ctx in ctxs:
        ctx.close()
    return states, its, info


def test_persistent_batch_equals_per_launch():
    """The wall-less members of a group solved in one cooperative launch
    (each with its own stopping decision) give bitwise the per-launch
    results and sweep counts, with a walled member in the same group taking
    per-launch sweeps after it; and wall-less cases only, in two groups (the
    quintic and the Wendland kernel), one launch per group and step."""
    sisph = _gpu()
    mixes = {
        "with_walls": (1, [cases.taylor_green(24, kernel="wendland", hdx=1.3, precision="mixed", seed=1),
                           cases.dam_break_2d(dx=0.1, precision="mixed"),
                           cases.taylor_green(40, kernel="wendland", hdx=1.3, precision="mixed", seed=2, re=500.0),
                           cases.taylor_green(17, kernel="wendland", hdx=1.3, precision="mixed", seed=3,
                                              tol=1e-2)]),
        "wall_less": (2, [cases.taylor_green(30, precision="fp64", seed=4),
                          cases.taylor_green(21, precision="fp64", seed=5, tol=1e-3),
                          cases.cloud_2d(precision="fp64")]),
    }
    for name, (groups, mix) in mixes.items():
        a, ia, pa = _run_batch(sisph, mix, 5, True)
        b, ib, pb = _run_batch(sisph, mix, 5, False)
        say(name, "persistent", pa, "iters", ia, "per-launch", ib)
        if pa["launches"] == 0:
            pytest.skip(f"persistent batched launch not taken ({pa['fallbacks']} fallbacks)")
        assert pa["launches"] == 5 * groups and pb["launches"] == 0
        assert ia == ib
        for k in range(len(mix)):
            assert _same(a[k], b[k]), (name, k)

"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every case is seeded and synthetic; the oracle and the GPU read the same
arrays.  Neighbour sets must match bit-exactly (same FP64 predicate, no
contraction); FP64 fields must agree within 1e-5 relative L2 (they agree
to ~1e-12: only the summation order differs); iteration counts must be
equal.  Mixed-precision errors are checked against bounds derived from
FP32 rounding (unit roundoff 6e-8 times the neighbour count and the
conditioning of each quantity).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1908_01762_amd import cases

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-5


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01762_amd import sisph
    return sisph


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def _cases_small():
    return {
        "tg50_quintic": cases.taylor_green(50),
        "tg40_wendland_jitter": cases.taylor_green(40, kernel="wendland", hdx=1.3, jitter=0.2, seed=3),
        "db2d_dx0.05": cases.dam_break_2d(dx=0.05, precision="fp64"),
        "db3d_small": cases.dam_break_3d(dx=0.1, lx=0.5, ly=0.5, lz=0.6, tank_x=1.5, tank_y=0.5, tank_z=1.0,
                                         precision="fp64"),
        "db3d_quintic": cases.dam_break_3d(dx=0.1, lx=0.5, ly=0.5, lz=0.6, tank_x=1.5, tank_y=0.5, tank_z=1.0,
                                           kernel="quintic", hdx=1.0, precision="fp64"),
        # support 3.9 dx: cells of about 59 fluid and 45 wall particles, past
        # the 32 that the cell sort ranks on half a wavefront
        "db3d_dense_cells": cases.dam_break_3d(dx=0.1, lx=0.5, ly=0.5, lz=0.6, tank_x=1.5, tank_y=0.5,
                                               tank_z=1.0, kernel="quintic", hdx=1.3, precision="fp64"),
        "ldc30_slip": cases.lid_driven_cavity(30),
        "ldc30_noslip": cases.lid_driven_cavity(30, ustar_wall="noslip"),
    }


def _same_sets(off_a, ids_a, off_b, ids_b):
    return np.array_equal(off_a, off_b) and np.array_equal(ids_a, ids_b)


@pytest.mark.parametrize("name", list(_cases_small().keys()))
def test_neighbour_sets_bit_exact(name):
    sisph = _gpu()
    case = _cases_small()[name]
    say("case", name, case.n_fluid, case.n_wall)
    ctx = sisph.Context(case)
    ctx.bin()
    off, ids = ctx.neighbors(0, 0)
    roff, rids = oracle.neighbors(case)
    assert _same_sets(off, ids, roff, rids)
    assert ctx.pair_count(0, 0) == roff[-1]
    assert ctx.rows_with_neighbours(0, 0) == np.count_nonzero(np.diff(roff) > 1)   # sets hold the row itself
    if case.n_wall:
        off, ids = ctx.neighbors(0, 1)
        roff, rids = oracle.neighbors(case, dest=(case.n_fluid, case.n), src=(0, case.n_fluid))
        assert _same_sets(off, ids, roff, rids)
        assert ctx.rows_with_neighbours(0, 1) == np.count_nonzero(np.diff(roff) > 0)
    # stage 1: r* = r^n + dt u~^n is formed with the same FP64 operations
    ctx.predict()
    out = oracle.Sim(case).step(capture=True)
    xs_all = case.x.copy()
    xs_all[:case.n_fluid] = out["xs"]
    assert np.array_equal(ctx.field("xstar"), out["xs"])
    off, ids = ctx.neighbors(1, 0)
    roff, rids = oracle.neighbors(case, x=xs_all)
    assert _same_sets(off, ids, roff, rids)
    if case.n_wall:
        off, ids = ctx.neighbors(1, 1)
        roff, rids = oracle.neighbors(case, x=xs_all, dest=(case.n_fluid, case.n), src=(0, case.n_fluid))
        assert _same_sets(off, ids, roff, rids)
    ctx.close()


@pytest.mark.parametrize("name", list(_cases_small().keys()))
def test_single_step_fields_fp64(name):
    sisph = _gpu()
    case = _cases_small()[name]
    say("case", name)
    ref = oracle.Sim(case)
    out = ref.step(capture=True)
    ctx = sisph.Context(case)
    ctx.bin()
    ctx.predict()
    st = ctx.ppe_solve()
    fields = {
        "rho": (ctx.field("rho"), out["rho"]),
        "ustar": (ctx.field("ustar"), out["us"]),
        "rhs": (ctx.field("rhs"), out["rhs"]),
        "dii": (ctx.field("dii"), out["diag"]),
    }
    if case.n_wall:
        fields["wall_ustar"] = (ctx.field("wall_ustar"), out["usw"])
        fields["normals"] = (ctx.field("normal"), ref.nrm)
    ctx.correct()
    fields["unew"] = (ctx.field("unew"), out["unew"])
    s = ctx.read_state()
    fields["p"] = (s["p"], ref.p)
    fields["u_tilde"] = (s["ut"], ref.ut)
    fields["displacement"] = (s["x"][:case.n_fluid] - case.x[:case.n_fluid], ref.x[:case.n_fluid] - case.x[:case.n_fluid])
    for k, (g, o) in fields.items():
        e = rel(g, o)
        say(f"  {k:14s} rel L2 {e:.3e}")
        assert e < FP64_TOL, k
    assert st["iters"] == out["iters"]
    assert math.isclose(st["lam"], out["lam"], rel_tol=1e-9)
    assert np.array_equal(ctx.field("fs"), out["fs"].astype(float))
    ctx.close()


def test_taylor_green_50_steps_fp64():
    """C1: 50x50, quintic h = dx, Re = 100, tol 1e-4, 50 steps, FP64."""
    sisph = _gpu()
    case = cases.taylor_green(50)
    ref = oracle.Sim(case)
    ctx = sisph.Context(case)
    u0 = np.linalg.norm(case.u, axis=1).max()
    worst = 0.0
    for k in range(50):
        o = ref.step()
        g = ctx.step(1)[0]
        assert g["iters"] == o["iters"], f"step {k}"
        s = ctx.read_state()
        a = np.linalg.norm(s["u"], axis=1).max() / u0
        b = np.linalg.norm(ref.u, axis=1).max() / u0
        worst = max(worst, abs(a - b) / b)
    say("  |u|max series worst rel diff", worst)
    assert worst < 1e-4
    s = ctx.read_state()
    assert rel(s["u"], ref.u) < FP64_TOL
    ctx.close()


def test_dam_break_steps_fp64():
    sisph = _gpu()
    case = cases.dam_break_2d(dx=0.05, precision="fp64")
    ref = oracle.Sim(case)
    ctx = sisph.Context(case)
    for k in range(20):
        o = ref.step()
        g = ctx.step(1)[0]
        assert g["iters"] == o["iters"], f"step {k}"
    s = ctx.read_state()
    assert rel(s["p"], ref.p) < FP64_TOL
    assert rel(s["u"], ref.u) < FP64_TOL
    ctx.close()


@pytest.mark.parametrize("form", ["slip", "noslip"])
def test_cavity_steps_fp64(form):
    """Lid-driven cavity (section 4.3), Re = 100, 30 x 30, quintic h = dx,
    tol 1e-2, symm, p_ref = 2 max p after the first solve; 20 steps with the
    slip or the no-slip ghost form for u*."""
    sisph = _gpu()
    case = cases.lid_driven_cavity(30, ustar_wall=form)
    say("case ldc30", form)
    ref = oracle.Sim(case)
    ctx = sisph.Context(case)
    for k in range(20):
        o = ref.step()
        g = ctx.step(1)[0]
        assert g["iters"] == o["iters"], f"step {k}"
        assert math.isclose(g["p_ref"], o["p_ref"], rel_tol=1e-9), f"step {k}"
    s = ctx.read_state()
    assert rel(s["p"], ref.p) < FP64_TOL
    assert rel(s["u"], ref.u) < FP64_TOL
    assert rel(s["x"], ref.x) < FP64_TOL
    ctx.close()


@pytest.mark.parametrize("name", ["db2d", "tg", "ldc"])
def test_adaptive_dt_steps_fp64(name):
    """Adaptive time steps (section 3.2): each step's dt comes from the
    previous step's max |u^n| and max |f^n| on the device; the dt series,
    the sweep counts and the state follow the oracle."""
    sisph = _gpu()
    if name == "db2d":       # the force limit acts once the column collapses
        case = cases.dam_break_2d(dx=0.05, precision="fp64", dt=0.006, tol=1e-2)
    elif name == "tg":       # the speed limit acts from the second step
        case = cases.taylor_green(30, jitter=0.05, seed=3, tol=1e-3, dt=0.0125)
    else:
        case = cases.lid_driven_cavity(24, dt=0.02)
    case = case.replace(dt_mode="adaptive")
    say("case adaptive", name)
    ref = oracle.Sim(case)
    ctx = sisph.Context(case)
    dts = []
    for k in range(15):
        o = ref.step()
        g = ctx.step(1)[0]
        assert g["iters"] == o["iters"], f"step {k}"
        # dt is a maximum over particles of speeds and accelerations that
        # carry the trajectory's summation-order differences (about 1e-12
        # after a few steps of the collapsing column), far inside FP64_TOL
        assert math.isclose(g["dt"], o["dt"], rel_tol=1e-8), f"step {k}: {g['dt']} vs {o['dt']}"
        dts.append(g["dt"])
    say("  dt series", dts[0], min(dts), max(dts))
    assert len(set(dts)) > 2          # the step really adapts
    s = ctx.read_state()
    assert rel(s["p"], ref.p) < FP64_TOL
    assert rel(s["u"], ref.u) < FP64_TOL
    assert rel(s["x"], ref.x) < FP64_TOL
    ctx.close()


def _fs_periodic(n=16, seed=4):
    """Periodic jittered set with a free-surface flag on the sparsest 10 %
    (Dirichlet rows that make the PPE non-singular)."""
    c = cases.taylor_green(n, kernel="wendland", hdx=1.3, jitter=0.2, seed=seed)
    rho = oracle.density(c)
    thr = np.quantile(rho, 0.1)
    return c.replace(free_surface=True, fs_ratio=float(thr / c.rho0) + 1e-12, gtvf="off", null_space="none")


# (case, tol, exact): with exact, the iteration counts must match and the
# state agree to FP64_TOL.  At tol 1e-6 the dam break's BiCGStab count is
# not determined by the arithmetic alone: perturbing p^n by 1e-15 in the
# oracle itself moves the first solve from 41 to 44-45 iterations and the
# pressure after four steps by up to 4e-4 (relative L2; u 3e-5, x 1.3e-9).
# There only convergence and the state within five times that spread are
# compared.  At 1e-3 and 1e-4 the counts do not move under such
# perturbations.
@pytest.mark.parametrize("name,tol,exact", [("fs_periodic", 1e-10, True), ("db2d", 1e-3, True),
                                            ("db2d", 1e-4, True), ("db2d", 1e-6, False)])
def test_bicgstab_steps_fp64(name, tol, exact):
    """BiCGStab on the device (section 3.1's alternative solver): the
    iteration count and the state after a few steps follow the oracle.  Both
    sides run the same recurrences; only summation order differs."""
    sisph = _gpu()
    case = _fs_periodic() if name == "fs_periodic" else cases.dam_break_2d(dx=0.05, precision="fp64")
    case = case.replace(solver="bicgstab", tol=tol, max_iter=2000)
    say("case bicgstab", name, tol)
    ref = oracle.Sim(case)
    ctx = sisph.Context(case)
    for k in range(4):
        o = ref.step()
        g = ctx.step(1)[0]
        say(f"  step {k}: iters gpu {g['iters']} oracle {o['iters']}, ratio {g['ratio']:.3e} / {o['ratio']:.3e}")
        if exact:
            assert g["iters"] == o["iters"], f"step {k}"
        assert g["converged"] and o["converged"]
    s = ctx.read_state()
    bounds = {"p": FP64_TOL, "u": FP64_TOL, "x": FP64_TOL} if exact else {"p": 2e-3, "u": 1.5e-4, "x": 1e-8}
    for key, ours, theirs in (("p", s["p"], ref.p), ("u", s["u"], ref.u), ("x", s["x"], ref.x)):
        e = rel(ours, theirs)
        say(f"  {key} rel L2 {e:.3e}")
        assert e < bounds[key], key
    ctx.close()


def test_bicgstab_mixed_single_step():
    """Mixed precision: FP32 cached coefficients, FP64 vectors and sums
    (tol 1e-4, where the iteration count is stable under rounding)."""
    sisph = _gpu()
    case = cases.dam_break_2d(dx=0.05, precision="mixed").replace(solver="bicgstab", tol=1e-4, max_iter=2000)
    ref = oracle.Sim(case.replace(precision="fp64"))
    o = ref.step()
    ctx = sisph.Context(case)
    g = ctx.step(1)[0]
    s = ctx.read_state()
    e = rel(s["p"], ref.p)
    eu = rel(s["u"], ref.u)
    say(f"  mixed bicgstab iters {g['iters']} / {o['iters']}, p rel L2 {e:.3e}, u {eu:.3e}")
    assert g["converged"]
    assert abs(g["iters"] - o["iters"]) <= 3
    # measured 4.0e-5 / 2.9e-5: BiCGStab's inner products amplify the FP32
    # rounding of the operator applications more than damped Jacobi does
    assert e < 1.2e-4 and eu < 1e-4
    assert np.all(np.isfinite(s["p"])) and np.all(np.isfinite(s["u"]))
    ctx.close()


def test_index_offsets_compact_and_wide():
    """Mixed cases without walls read 16-bit neighbour offsets when every
    offset of the step fits (Taylor-Green), and the full indices otherwise
    (a long periodic strip); both agree with the FP64 path."""
    sisph = _gpu()
    for case, expect in ((cases.taylor_green(60, kernel="wendland", hdx=1.3, precision="mixed", seed=2), 16),
                         (cases.long_strip(), 32)):
        a = sisph.Context(case)
        b = sisph.Context(case.replace(precision="fp64"))
        sa = a.step(2)
        sb = b.step(2)
        ra, rb = a.read_state(), b.read_state()
        e = rel(ra["p"], rb["p"])
        say(f"  {case.name}: index bits {sa[-1]['index_bits']}, iters {[s['iters'] for s in sa]} / "
            f"{[s['iters'] for s in sb]}, p rel L2 vs FP64 {e:.3e}, u {rel(ra['u'], rb['u']):.3e}")
        assert all(s["index_bits"] == expect for s in sa)
        assert all(s["index_bits"] == 32 for s in sb)
        assert e < 1e-3 and rel(ra["u"], rb["u"]) < 1e-4
        a.close()
        b.close()


def test_bicgstab_context_cannot_join_a_batch():
    sisph = _gpu()
    ctx = sisph.Context(cases.dam_break_2d(dx=0.1, precision="mixed").replace(solver="bicgstab"))
    b = sisph.Batch(4)
    with pytest.raises(sisph.SisphError):
        b.attach(ctx)
    b.close()
    ctx.close()


@pytest.mark.parametrize("name", ["tg50_quintic", "db2d_dx0.05", "db3d_dx0.05", "ldc30_noslip"])
def test_mixed_precision_single_step(name):
    """Mixed mode against the FP64 oracle with the oracle run on the GPU's
    sweep count (the ratio test may flip one sweep earlier or later)."""
    sisph = _gpu()
    if name == "db3d_dx0.05":   # 1,200 fluid + 7,248 wall particles
        case = cases.dam_break_3d(dx=0.05, lx=0.5, ly=0.5, lz=0.6, tank_x=1.5, tank_y=0.5, tank_z=1.0,
                                  precision="mixed")
    else:
        case = _cases_small()[name].replace(precision="mixed")
    ctx = sisph.Context(case)
    g = ctx.step(1)[0]
    ref = oracle.Sim(case, forced_iters=g["iters"])
    out = ref.step(capture=True)
    s = ctx.read_state()
    nf = case.n_fluid
    errs = {
        "rho": rel(ctx.field("rho"), out["rho"]),
        "rhs": rel(ctx.field("rhs"), out["rhs"]),
        "dii": rel(ctx.field("dii"), out["diag"]),
        "p": rel(s["p"][:nf], ref.p[:nf]),
        "u": rel(s["u"], ref.u),
        "displacement": rel(s["x"][:nf] - case.x[:nf], ref.x[:nf] - case.x[:nf]),
    }
    if case.n_wall:
        # Wall pressure (eq. p-shepard) is a normalised average.  A wall row
        # whose fluid neighbours all sit within rounding of the support
        # radius has FP64 weights of ~1e-75: normalised they give the
        # neighbours' pressure, while in FP32 they underflow and the row
        # takes the no-neighbour value 0.  Such rows carry no weight in any
        # fluid sum; the others are compared.
        xs = case.x.copy()
        xs[:nf] = out["xs"]
        off, ids = oracle.neighbors(case, x=xs, dest=(nf, case.n), src=(0, nf))
        sw = np.array([oracle.W(case.kernel, case.dim, np.linalg.norm(xs[ids[off[w]:off[w + 1]]] - xs[nf + w], axis=1),
                                case.h).sum() if off[w + 1] > off[w] else 0.0 for w in range(case.n_wall)])
        graze = sw < 1e-30 * oracle.W(case.kernel, case.dim, 0.0, case.h)[0]
        say(f"  mixed {name}: {int(graze.sum())} wall rows without weight")
        assert np.all(s["p"][nf:][graze] == 0.0)
        errs["p_wall"] = rel(s["p"][nf:][~graze], ref.p[nf:][~graze])
    for k, e in errs.items():
        say(f"  mixed {name} {k:12s} rel L2 {e:.3e}")
    # measured maxima over these cases: rho 2.2e-7, D 2.6e-7, RHS 2.2e-6
    # (its terms cancel), p 1.8e-5, u 1.9e-5 (2D dam break: 280 sweeps, each
    # rounding its FP32 neighbour sum; the damped Jacobi map is
    # non-expansive, so the per-sweep rounding of ~1e-7 adds up over the
    # sweeps), wall p 1.5e-5
    assert errs["rho"] < 7e-7 and errs["dii"] < 8e-7
    assert errs["u"] < 6e-5 and errs["displacement"] < 6e-5
    assert errs["rhs"] < 7e-6 and errs["p"] < 6e-5 and errs.get("p_wall", 0.0) < 5e-5
    ctx.close()


def _mixed_steps_cases():
    return {
        "tg40_quintic": cases.taylor_green(40, precision="mixed"),
        "db2d_dx0.05": cases.dam_break_2d(dx=0.05, precision="mixed"),
        "ldc30_noslip": cases.lid_driven_cavity(30, ustar_wall="noslip", precision="mixed"),
        "ldc24_adaptive_dt": cases.lid_driven_cavity(24, dt=0.02, precision="mixed").replace(dt_mode="adaptive"),
        "db2d_bicgstab": cases.dam_break_2d(dx=0.05, precision="mixed").replace(solver="bicgstab"),
    }


@pytest.mark.parametrize("name", list(_mixed_steps_cases().keys()))
def test_mixed_precision_steps(name):
    """Five mixed-mode steps against the FP64 oracle, the oracle taking the
    GPU's iteration count at each step (the stopping test may flip one
    iteration either way).  FP32 rounding of the pair sums (~1e-7 relative,
    accumulated over the sweeps) bounds the drift: velocity and displacement
    to 1e-5, fluid pressure to 2e-5 relative L2 (measured at most 3.2e-6 and
    6.8e-6), BiCGStab 1e-4 (measured 2.9e-5 / 3.4e-5), and the adaptive step
    to 1e-6."""
    sisph = _gpu()
    case = _mixed_steps_cases()[name]
    nf = case.n_fluid
    say("case mixed steps", name, nf, case.n_wall)
    ctx = sisph.Context(case)
    ref = oracle.Sim(case)
    for k in range(5):
        g = ctx.step(1)[0]
        o = ref.step(forced_iters=g["iters"])
        say(f"  step {k}: iters {g['iters']}, dt gpu {g['dt']:.9e} oracle {o['dt']:.9e}")
        assert math.isclose(g["dt"], o["dt"], rel_tol=1e-6)
    s = ctx.read_state()
    errs = {"u": rel(s["u"][:nf], ref.u[:nf]), "p": rel(s["p"][:nf], ref.p[:nf]),
            "displacement": rel(s["x"][:nf] - case.x[:nf], ref.x[:nf] - case.x[:nf])}
    for k, e in errs.items():
        say(f"  mixed steps {name} {k:12s} rel L2 {e:.3e}")
    b = 1e-4 if case.solver == "bicgstab" else 1e-5
    assert errs["u"] < b and errs["displacement"] < b and errs["p"] < 2 * b
    ctx.close()


@pytest.mark.parametrize("name", ["cloud", "single"])
def test_degenerate_rows_fp64(name):
    """Empty neighbour sums: isolated particles (count 1, D_ii = 0), an
    isolated pair and a free-surface disc whose 460 rows leave a ragged last
    workgroup; and a case of one particle.  Neighbour sets bit-exact, three
    steps against the oracle, zero pressure on the isolated rows."""
    sisph = _gpu()
    case = cases.cloud_2d() if name == "cloud" else cases.single_particle()
    iso = case.meta.get("isolated", [0])
    say("case", name, case.n_fluid)
    ctx = sisph.Context(case)
    ctx.bin()
    off, ids = ctx.neighbors(0, 0)
    roff, rids = oracle.neighbors(case)
    assert _same_sets(off, ids, roff, rids)
    ctx.close()
    ref = oracle.Sim(case)
    ctx = sisph.Context(case)
    for k in range(3):
        o = ref.step()
        g = ctx.step(1)[0]
        say(f"  step {k}: iters gpu {g['iters']} oracle {o['iters']}")
        assert g["iters"] == o["iters"]
        s = ctx.read_state()
        assert np.all(s["p"][iso] == 0.0)
        for f in ("x", "u", "ut", "p"):
            e = rel(s[f], getattr(ref, f))
            say(f"    {f:3s} rel L2 {e:.3e}")
            assert e < FP64_TOL, f
    ctx.close()


def test_degenerate_rows_mixed():
    """The cloud in the mixed mode: zero pressure on the isolated rows and
    the fields within the FP32 bounds, the oracle run on the GPU's sweep
    count."""
    sisph = _gpu()
    case = cases.cloud_2d(precision="mixed")
    iso = case.meta["isolated"]
    ctx = sisph.Context(case)
    g = ctx.step(1)[0]
    ref = oracle.Sim(case, forced_iters=g["iters"])
    ref.step()
    s = ctx.read_state()
    assert np.all(s["p"][iso] == 0.0)
    errs = {f: rel(s[f], getattr(ref, f)) for f in ("p", "u")}
    errs["displacement"] = rel(s["x"] - case.x, ref.x - case.x)
    for k, e in errs.items():
        say(f"  mixed cloud {k:12s} rel L2 {e:.3e}")
    # measured 2.5e-8, 1.3e-8, 8.6e-7
    assert errs["u"] < 1e-7 and errs["displacement"] < 5e-8 and errs["p"] < 3e-6
    ctx.close()


def test_error_paths():
    sisph = _gpu()
    case = cases.taylor_green(16)
    ctx = sisph.Context(case)
    with pytest.raises(sisph.SisphError) as e:
        ctx.predict()
    assert e.value.code == sisph.E_STATE
    ctx.close()
    ctx = sisph.Context(case.replace(tol=1e-300, max_iter=3))
    st = ctx.step(1)[0]
    assert st["iters"] == 3 and st["status"] == sisph.WARN_MAXITER
    ctx.close()
    bad = case.copy()
    bad.u[5, 0] = np.nan
    ctx = sisph.Context(bad)
    with pytest.raises(sisph.SisphError) as e:
        ctx.step(1)
    assert e.value.code == sisph.E_NONFINITE
    ctx.close()


@pytest.mark.parametrize("name", ["tg30_fp64", "db2d_mixed"])
def test_eisph_single_sweep_matches_oracle(name):
    """forced one sweep (EISPH) on both sides; with walls in the mixed mode
    the final iterate sits in the second buffer after every solve."""
    sisph = _gpu()
    if name == "tg30_fp64":
        case, tol_u, tol_p = cases.taylor_green(30, jitter=0.1, seed=4), FP64_TOL, FP64_TOL
    else:
        case, tol_u, tol_p = cases.dam_break_2d(dx=0.05, precision="mixed"), 1e-4, 1e-3
    case = case.replace(forced_iters=1)
    ref = oracle.Sim(case)
    ctx = sisph.Context(case)
    for _ in range(3):
        assert ref.step()["iters"] == 1 and ctx.step(1)[0]["iters"] == 1
    s = ctx.read_state()
    nf = case.n_fluid
    say(f"  eisph {name}: p {rel(s['p'], ref.p):.3e} u {rel(s['u'][:nf], ref.u[:nf]):.3e}")
    assert rel(s["p"], ref.p) < tol_p and rel(s["u"][:nf], ref.u[:nf]) < tol_u
    ctx.close()


def test_save_restore_bitwise():
    """20 steps == 10 steps, read_state, write_state, 10 steps (same context)."""
    sisph = _gpu()
    case = cases.dam_break_2d(dx=0.05, precision="mixed")
    a = sisph.Context(case)
    a.step(20)
    b = sisph.Context(case)
    b.step(10)
    s = b.read_state()
    b.write_state(x=s["x"], u=s["u"], ut=s["ut"], p=s["p"])
    b.step(10)
    sa, sb = a.read_state(), b.read_state()
    for k in ("x", "u", "ut", "p"):
        assert np.array_equal(sa[k], sb[k]), k
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_null_space_projection(precision):
    """Reading R24 on the GPU (fully periodic Taylor-Green, the RHS component
    along the left null vector y = m rho removed once per solve): beta of
    every step against the oracle's, the same sweep counts in FP64 (mixed:
    the oracle on the GPU's counts), the fields to the parity bounds, and no
    drift of the mean pressure."""
    sisph = _gpu()
    case = cases.taylor_green(40, kernel="wendland", hdx=1.3, jitter=0.2, seed=3, precision=precision)
    assert case.null_space == "project"
    ctx = sisph.Context(case)
    ref = oracle.Sim(case)
    for k in range(5):
        g = ctx.step(1)[0]
        o = ref.step(forced_iters=None if precision == "fp64" else g["iters"])
        say(f"  step {k}: iters gpu {g['iters']} oracle {o['iters']}, beta gpu {g['beta']:.6e} oracle {o['beta']:.6e}")
        if precision == "fp64":
            assert g["iters"] == o["iters"]
            assert math.isclose(g["beta"], o["beta"], rel_tol=1e-8)
        else:
            assert math.isclose(g["beta"], o["beta"], rel_tol=2e-2)
        assert g["iters"] < case.max_iter
    s = ctx.read_state()
    nf = case.n_fluid
    errs = {"p": rel(s["p"][:nf], ref.p[:nf]), "u": rel(s["u"], ref.u),
            "displacement": rel(s["x"] - case.x, ref.x - case.x)}
    for name, e in errs.items():
        say(f"  projected {precision} {name:12s} rel L2 {e:.3e}")
    bound = FP64_TOL if precision == "fp64" else 1e-4
    assert all(e < bound for e in errs.values())
    assert abs(s["p"][:nf].mean()) < 0.05 * np.abs(s["p"][:nf]).mean()
    ctx.close()


def _round32(case):
    """The same case with its input arrays rounded to FP32 (the plain FP32
    mode starts from those values; the oracle then reads the same numbers)."""
    c = case.copy()
    for k in ("x", "u", "p", "m"):
        setattr(c, k, np.ascontiguousarray(getattr(c, k).astype(np.float32).astype(np.float64)))
    if c.wall_u is not None:
        c.wall_u = np.ascontiguousarray(c.wall_u.astype(np.float32).astype(np.float64))
    return c


def _is_f32(a):
    a = np.asarray(a)
    return np.array_equal(a, a.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("name", ["tg50_quintic", "tg40_wendland_jitter", "db2d_dx0.05", "ldc30_slip"])
def test_fp32_plain_steps(name):
    """The plain FP32 mode (every sum, per-particle result, the residual and
    the stopping test in FP32) against the FP64 oracle on the same FP32
    inputs, the oracle following the GPU's sweep counts, over three steps;
    every state value the GPU holds is an FP32 number."""
    sisph = _gpu()
    case = _round32(_cases_small()[name].replace(precision="fp32"))
    nf = case.n_fluid
    ctx = sisph.Context(case)
    ref = oracle.Sim(case.replace(precision="fp64"))
    its = []
    for k in range(3):
        g = ctx.step(1)[0]
        its.append(g["iters"])
        ref.step(forced_iters=g["iters"])
    s = ctx.read_state()
    for f in ("x", "u", "ut", "p"):
        assert _is_f32(s[f]), f
    errs = {"p": rel(s["p"][:nf], ref.p[:nf]), "u": rel(s["u"], ref.u),
            "displacement": rel(s["x"][:nf] - case.x[:nf], ref.x[:nf] - case.x[:nf])}
    for k, e in errs.items():
        say(f"  fp32 {name} {k:12s} rel L2 {e:.3e} (sweeps {its})")
    # measured: p <= 1.5e-5, u <= 3.8e-6 (FP32 sums over up to 1000 sweeps);
    # the displacement of a dam break's first steps from rest is ~1e-4 of
    # the positions, each of which FP32 rounds by up to 6e-8 relative per
    # step: 1.05e-3 there, <= 6e-5 elsewhere
    bounds = {"p": 5e-5, "u": 2e-5, "displacement": 4e-3 if name.startswith("db") else 2e-4}
    assert all(errs[k] < bounds[k] for k in errs), errs
    ctx.close()

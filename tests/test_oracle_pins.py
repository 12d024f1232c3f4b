"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is a closed form, a
quadrature, a brute-force count, a library solve, a hand computation of one
update, or a value printed in the paper.  Closed-form operator checks use
tolerances sized to the SPH discretisation error at fixed h/dx (about 1-4 %);
a dropped term, a wrong sign or a transposed index gives O(1) errors.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_1908_01762_amd import cases

TP = 2.0 * math.pi
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


# ----------------------------------------------------------------- kernels
@pytest.mark.parametrize("kernel", ["quintic", "wendland"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("h", [1.0, 0.37])
def test_kernel_normalisation(kernel, dim, h):
    """P1: the integral of W over its support is 1 (radial quadrature)."""
    R = oracle.support(kernel) * h
    area = (lambda r: 2 * math.pi * r) if dim == 2 else (lambda r: 4 * math.pi * r * r)
    f = lambda r: oracle.W(kernel, dim, r, h)[0] * area(r)
    val, _ = integrate.quad(f, 0.0, R, points=[h, 2 * h], limit=200, epsabs=1e-13, epsrel=1e-12)
    assert abs(val - 1.0) < 1e-9


@pytest.mark.parametrize("kernel", ["quintic", "wendland"])
@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_derivative_matches_finite_difference(kernel, dim):
    h = 0.5
    R = oracle.support(kernel) * h
    r = np.linspace(0.01, R - 0.01, 57)
    eps = 1e-6
    fd = (oracle.W(kernel, dim, r + eps, h) - oracle.W(kernel, dim, r - eps, h)) / (2 * eps)
    an = oracle.dWdr(kernel, dim, r, h)
    assert np.max(np.abs(fd - an)) < 1e-6 * np.max(np.abs(an))


@pytest.mark.parametrize("kernel", ["quintic", "wendland"])
def test_kernel_vanishes_smoothly_at_support(kernel):
    h = 1.0
    R = oracle.support(kernel)
    assert oracle.W(kernel, 2, R, h)[0] == 0.0 and oracle.dWdr(kernel, 2, R, h)[0] == 0.0
    near = oracle.W(kernel, 2, R - 1e-3, h)[0]
    assert 0.0 < near < 1e-10
    # monotone decreasing on (0, R)
    r = np.linspace(0.0, R, 301)
    w = oracle.W(kernel, 2, r, h)
    assert np.all(np.diff(w) <= 0.0)


# ------------------------------------------------------------- neighbours
def _lattice_count(Rdx, dim):
    """Number of integer points with |k|^2 < Rdx^2 (exact integer arithmetic)."""
    m = int(math.ceil(Rdx))
    R2 = Rdx * Rdx
    rng = range(-m, m + 1)
    if dim == 2:
        return sum(1 for a in rng for b in rng if a * a + b * b < R2)
    return sum(1 for a in rng for b in rng for c in rng if a * a + b * b + c * c < R2)


@pytest.mark.parametrize("kernel,hdx,dim,n,expect", [
    ("quintic", 1.0, 2, 32, 25), ("wendland", 1.3, 2, 32, 21), ("wendland", 1.3, 3, 8, 81)])
def test_lattice_neighbour_counts(kernel, hdx, dim, n, expect):
    """P3: strict |r| < R, self included; dx = 1/2^k so lattice distances are exact."""
    assert _lattice_count(oracle.support(kernel) * hdx, dim) == expect
    c = cases.periodic_lattice(n, dim=dim, kernel=kernel, hdx=hdx)
    off, _ = oracle.neighbors(c)
    cnt = np.diff(off)
    assert cnt.min() == expect and cnt.max() == expect


def _numpy_brute(case, x, dest, src):
    """Independent O(N^2) neighbour sets (same FP64 predicate, vectorised)."""
    R = oracle.support(case.kernel) * case.h
    R2 = R * R
    xi = x[dest[0]:dest[1]][:, None, :]
    xj = x[src[0]:src[1]][None, :, :]
    d = xi - xj
    for k in range(case.dim):
        if case.periodic[k]:
            L = case.box_hi[k] - case.box_lo[k]
            Lh = 0.5 * L
            dk = d[..., k]
            dk = np.where(dk > Lh, dk - L, np.where(dk < -Lh, dk + L, dk))
            d[..., k] = dk
    r2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]
    if case.dim == 3:
        r2 = r2 + d[..., 2] * d[..., 2]
    mask = r2 < R2
    return [np.nonzero(row)[0] + src[0] for row in mask]


def _sets(off, ids):
    return [ids[off[i]:off[i + 1]] for i in range(len(off) - 1)]


@pytest.mark.parametrize("which", ["tg_jitter", "tg_quintic", "dam_break", "cube3d", "faces"])
def test_neighbours_cells_equal_bruteforce(which):
    """P6: cell-list sets == oracle brute force == independent numpy brute force."""
    if which == "tg_jitter":
        c = cases.taylor_green(24, kernel="wendland", hdx=1.3, jitter=0.2, seed=3)
    elif which == "tg_quintic":
        c = cases.taylor_green(20, jitter=0.05, seed=1)
    elif which == "dam_break":
        c = cases.dam_break_2d(dx=0.1, jitter=0.1, seed=2)
    elif which == "cube3d":
        c = cases.dam_break_3d(dx=0.125, lx=0.5, ly=0.5, lz=0.5, tank_x=1.0, tank_y=0.5, tank_z=1.0)
    else:
        # particles on cell faces and at exactly R from each other (dx = 1/64)
        c = cases.periodic_lattice(64, kernel="quintic", hdx=1.0)
        c.x[:, 0] = np.floor(c.x[:, 0] * 16) / 16.0
    dest_sets = [(0, c.n_fluid, 0, c.n)]
    if c.n_wall:
        dest_sets.append((c.n_fluid, c.n, 0, c.n_fluid))
    for d0, d1, s0, s1 in dest_sets:
        oc, ic = oracle.neighbors(c, dest=(d0, d1), src=(s0, s1))
        ob, ib = oracle.neighbors(c, dest=(d0, d1), src=(s0, s1), method="brute")
        assert np.array_equal(oc, ob) and np.array_equal(ic, ib)
        ref = _numpy_brute(c, c.x, (d0, d1), (s0, s1))
        got = _sets(oc, ic)
        assert all(np.array_equal(a, b) for a, b in zip(got, ref))


# ------------------------------------------------------ lattice symmetries
@pytest.mark.parametrize("kernel,hdx", [("quintic", 1.0), ("wendland", 1.3)])
def test_lattice_density_and_symmetry(kernel, hdx):
    """P2/P4: on an unperturbed periodic lattice the density is the same for
    every particle and close to rho0 (partition of unity), the GTVF push and
    the RHS of a uniform flow vanish, and D_ii is the same everywhere."""
    c = cases.periodic_lattice(32, kernel=kernel, hdx=hdx)
    rho = oracle.density(c)
    assert np.ptp(rho) < 1e-12 * rho.mean()
    assert abs(rho.mean() / c.rho0 - 1.0) < 0.02
    f = oracle.gtvf_force(c, c.x, rho, np.ones(c.n_fluid), c.h)
    scale = np.abs(oracle.gtvf_force(cases.taylor_green(32, kernel=kernel, hdx=hdx, jitter=0.1),
                                     c.x, rho, np.ones(c.n_fluid), c.h)).max()
    assert np.abs(f).max() < 1e-10 * max(scale, 1.0)
    us = np.tile([0.3, -0.7], (c.n_fluid, 1))
    assert np.abs(oracle.rhs(c, c.x, rho, us)).max() < 1e-8
    _, D = oracle.ppe_operator(c, c.x, rho, np.zeros(c.n_fluid))
    assert np.ptp(D) < 1e-12 * abs(D.mean()) and D.mean() < 0


def test_gtvf_pushes_a_displaced_particle_back():
    """A particle moved off its lattice site feels a GTVF force toward it."""
    c = cases.periodic_lattice(32, kernel="wendland", hdx=1.3)
    rho = np.full(c.n_fluid, c.rho0)
    i = 500
    for axis in (0, 1):
        for sgn in (1.0, -1.0):
            x = c.x.copy()
            x[i, axis] += sgn * 0.2 * c.dx
            f = oracle.gtvf_force(c, x, rho, np.full(c.n_fluid, 1.0), c.h)
            assert f[i, axis] * sgn < 0


# ----------------------------------------------- closed-form operator checks
def _smooth_fields(c):
    X, Y = c.x[:, 0], c.x[:, 1]
    return X, Y


@pytest.mark.parametrize("kernel,hdx,tol", [("quintic", 1.0, 0.02), ("wendland", 1.3, 0.05)])
def test_pressure_gradient_forms_match_closed_form(kernel, hdx, tol):
    """eq. mom:sph:press:pij and mom:sph:press:symm approximate -grad p / rho."""
    c = cases.taylor_green(32, kernel=kernel, hdx=hdx, jitter=0.0)
    X, Y = _smooth_fields(c)
    rho = np.ones(c.n)
    p = np.sin(TP * X) * np.sin(TP * Y)
    gp = np.stack([TP * np.cos(TP * X) * np.sin(TP * Y), TP * np.sin(TP * X) * np.cos(TP * Y)], 1)
    assert rel(oracle.pressure_force(c, c.x, rho, p, "asymm"), -gp) < tol
    assert rel(oracle.pressure_force(c, c.x, rho, p, "symm"), -gp) < tol
    # the asymm form ignores a constant shift of p, the symm form does not
    # (its constant part is the background-pressure term), on a jittered set
    cj = cases.taylor_green(32, kernel=kernel, hdx=hdx, jitter=0.2, seed=5)
    fa0 = oracle.pressure_force(cj, cj.x, rho, p, "asymm")
    fa1 = oracle.pressure_force(cj, cj.x, rho, p + 10.0, "asymm")
    assert np.max(np.abs(fa0 - fa1)) < 1e-9
    fs0 = oracle.pressure_force(cj, cj.x, rho, p, "symm")
    fs1 = oracle.pressure_force(cj, cj.x, rho, p + 10.0, "symm")
    assert np.max(np.abs(fs0 - fs1)) > 1e-3


@pytest.mark.parametrize("kernel,hdx,tol", [("quintic", 1.0, 0.03), ("wendland", 1.3, 0.06)])
def test_ppe_operator_is_laplacian(kernel, hdx, tol):
    """eq. sph-ppe: sum_j c_ij (p_i - p_j) approximates div(grad p / rho)."""
    for n in (32, 64):
        c = cases.taylor_green(n, kernel=kernel, hdx=hdx, jitter=0.0)
        X, Y = _smooth_fields(c)
        p = np.sin(TP * X) * np.sin(TP * Y)
        lap, D = oracle.ppe_operator(c, c.x, np.ones(c.n), p)
        assert rel(lap, -2 * TP * TP * p) < tol
        # doubling density and mass together (same volumes) halves the
        # operator: div(grad p / rho) = lap p / rho
        c2 = c.replace(m=2.0 * c.m)
        lap2, _ = oracle.ppe_operator(c2, c.x, np.full(c.n, 2.0), p)
        assert rel(lap2, 0.5 * lap) < 1e-12


@pytest.mark.parametrize("kernel,hdx,tol", [("quintic", 1.0, 0.02), ("wendland", 1.3, 0.05)])
def test_rhs_is_divergence_over_dt(kernel, hdx, tol):
    """RHS of eq. sph-ppe approximates div(u*) / dt."""
    c = cases.taylor_green(32, kernel=kernel, hdx=hdx, jitter=0.0)
    X, Y = _smooth_fields(c)
    us = np.stack([np.sin(TP * X), np.sin(TP * Y)], 1)
    div = TP * (np.cos(TP * X) + np.cos(TP * Y))
    assert rel(oracle.rhs(c, c.x, np.ones(c.n), us) * c.dt, div) < tol
    # and vanishes for the (solenoidal) Taylor-Green field up to O(h^2)
    r = oracle.rhs(c, c.x, np.ones(c.n), c.u) * c.dt
    assert np.abs(r).max() < 0.02 * np.abs(div).max()


@pytest.mark.parametrize("kernel,hdx,tol", [("quintic", 1.0, 0.02), ("wendland", 1.3, 0.06)])
def test_viscous_force_is_nu_laplacian(kernel, hdx, tol):
    """P9, eq. mom:sph:visc: for the Taylor-Green field nu lap(u) = -8 pi^2 nu u."""
    c = cases.taylor_green(32, kernel=kernel, hdx=hdx, jitter=0.0)
    f = oracle.predictor_forces(c, c.x, c.u, c.u.copy(), np.ones(c.n))
    assert rel(f, -2 * TP * TP * c.nu * c.u) < tol


@pytest.mark.parametrize("kernel,hdx,tol", [("quintic", 1.0, 0.02), ("wendland", 1.3, 0.05)])
def test_artificial_stress_is_divergence_of_A(kernel, hdx, tol):
    """eq. mom:sph:gtvf:stress approximates (1/rho) div A, A = rho u (x) (u~ - u).

    u = (sin 2 pi y, 0), u~ - u = (0, c): only A_xy = rho c sin(2 pi y) is
    non-zero, so (div A)_x = d/dy A_xy = 2 pi c cos(2 pi y) and (div A)_y = 0.
    A transposed contraction would put the whole force on y instead."""
    c = cases.taylor_green(32, kernel=kernel, hdx=hdx, jitter=0.0).replace(nu=0.0)
    X, Y = _smooth_fields(c)
    cc = 0.3
    u = np.stack([np.sin(TP * Y), 0 * Y], 1)
    ut = u + np.array([0.0, cc])
    f = oracle.predictor_forces(c, c.x, u, ut, np.ones(c.n))
    assert rel(f, np.stack([TP * cc * np.cos(TP * Y), 0 * Y], 1)) < tol


def test_artificial_viscosity_two_particles():
    """eq. mom:sph:av: an approaching pair repels, a receding pair feels nothing;
    the value is the hand-computed Monaghan term."""
    c = cases.dam_break_2d(dx=0.1)
    c = c.replace(n_fluid=2, n_wall=0, x=np.array([[1.0, 1.0], [1.0 + 0.1, 1.0]]),
                  m=np.array([10.0, 10.0]), gravity=(0.0, 0.0, 0.0), nu=0.0)
    rho = np.array([1000.0, 1000.0])
    for v, sign in ((0.5, 1), (-0.5, 0)):
        u = np.array([[v, 0.0], [0.0, 0.0]])
        f = oracle.predictor_forces(c, c.x, u, u.copy(), rho)
        r = -0.1
        dwdr = oracle.dWdr(c.kernel, 2, 0.1, c.h)[0]
        gw = dwdr / 0.1 * r
        mu = v * r / (r * r + c.eta * c.h * c.h)
        Pi = -c.alpha * c.h * c.c_ref * mu / 1000.0 if v * r < 0 else 0.0
        expect = -10.0 * Pi * gw
        assert f[0, 1] == 0.0
        assert math.isclose(f[0, 0], expect, rel_tol=1e-12, abs_tol=1e-300)
        if sign:
            assert f[0, 0] < 0  # pushed back, against its motion toward +x
        else:
            assert f[0, 0] == 0.0


# -------------------------------------------------------------------- walls
def test_wall_pressure_hydrostatic_exact():
    """P15, eq. p-shepard: with uniform density and p_f = rho0 g (H - y_f),
    p_f + rho0 g.r_wf = rho0 g (H - y_w) for every pair, so the Shepard
    average returns the hydrostatic wall pressure exactly."""
    c = cases.dam_break_2d(dx=0.05)
    rho_all = np.full(c.n, c.rho0)
    p = oracle.wall_pressure(c, c.x, rho_all, c.p)
    xw = c.x[c.n_fluid:]
    pw = p[c.n_fluid:]
    has = oracle.neighbors(c, dest=(c.n_fluid, c.n), src=(0, c.n_fluid))[0]
    has = np.diff(has) > 0
    # walls beside the fluid above its surface are clamped at zero
    expect = np.maximum(c.rho0 * 9.81 * (2.0 - xw[:, 1]), 0.0)
    assert has.sum() > 50
    assert np.max(np.abs(pw[has] - expect[has])) < 1e-9 * expect.max()
    assert np.all(pw[~has] == 0.0)
    # free-surface clamp: a negative fluid pressure gives zero wall pressure
    p2 = oracle.wall_pressure(c, c.x, rho_all, -np.abs(c.p) - 1e5)
    assert np.all(p2[c.n_fluid:] >= 0.0)


def test_wall_normals_flat_walls():
    """Section 3.4.1: on flat walls the first wall layer's unit normal points
    into the fluid."""
    c = cases.dam_break_2d(dx=0.05)
    nrm = oracle.wall_normals(c)
    xw = c.x[c.n_fluid:]
    d = c.dx
    bottom = (np.abs(xw[:, 1] + 0.5 * d) < 1e-9) & (xw[:, 0] > 0.5) & (xw[:, 0] < 3.5)
    left = (np.abs(xw[:, 0] + 0.5 * d) < 1e-9) & (xw[:, 1] > 0.5) & (xw[:, 1] < 3.5)
    right = (np.abs(xw[:, 0] - 4.0 - 0.5 * d) < 1e-9) & (xw[:, 1] > 0.5) & (xw[:, 1] < 3.5)
    for sel, n in ((bottom, (0, 1)), (left, (1, 0)), (right, (-1, 0))):
        assert sel.sum() > 10
        assert np.max(np.abs(nrm[sel] - np.array(n))) < 1e-9
    assert np.allclose(np.linalg.norm(nrm[np.linalg.norm(nrm, axis=1) > 0], axis=1), 1.0)


def test_wall_velocity_rules_by_hand():
    """eqs. vf, vg-adami, vg-no-normal on the bottom wall under a uniform
    fluid velocity: tangential flow is mirrored (no-slip) or copied (slip);
    the part pointing into the solid is removed, the part pointing away kept."""
    c = cases.dam_break_2d(dx=0.05)
    nrm = oracle.wall_normals(c)
    xw = c.x[c.n_fluid:]
    sel = (np.abs(xw[:, 1] + 0.025) < 1e-9) & (xw[:, 0] > 0.3) & (xw[:, 0] < 0.8)
    one = np.ones((sel.sum(), 1))
    table = [((1.0, 0.0), (-1.0, 0.0), (1.0, 0.0)),
             ((0.0, -1.0), (0.0, 1.0), (0.0, 0.0)),
             ((0.0, 1.0), (0.0, 0.0), (0.0, 1.0))]
    for uf, noslip, slip in table:
        u = np.tile(uf, (c.n_fluid, 1))
        assert np.allclose(oracle.wall_velocity(c, c.x, u, nrm, slip=False)[sel], one * noslip, atol=1e-12)
        assert np.allclose(oracle.wall_velocity(c, c.x, u, nrm, slip=True)[sel], one * slip, atol=1e-12)


def test_cavity_ustar_wall_forms():
    """Sections 3.4 and 4.3: one cavity step with the slip and the no-slip
    ghost form for u*.  The fluid u* does not depend on the form, and on every
    wall particle the two ghost values are the Shepard average a and
    2 u_wall - a, each with any part into the solid removed (the unit normal
    points into the fluid).  So along the wall they sum to 2 u_wall; along
    the normal both are >= 0, and where the slip value a.n is kept the
    no-slip one is max(2 u_wall.n - a.n, 0)."""
    base = cases.lid_driven_cavity(n=16)
    outs = {}
    for form in ("slip", "noslip"):
        outs[form] = oracle.Sim(base.replace(ustar_wall=form)).step(capture=True)
    s, ns = outs["slip"]["usw"], outs["noslip"]["usw"]
    assert np.array_equal(outs["slip"]["us"], outs["noslip"]["us"])
    nrm = oracle.wall_normals(base)
    wu = base.wall_u
    has_n = np.linalg.norm(nrm, axis=1) > 0.5
    assert has_n.sum() > 50 and (~has_n).sum() > 10
    lid = wu[:, 0] > 0
    assert np.abs(s[lid & has_n, 0]).max() > 1e-6   # the lid drags the fluid
    tang = np.stack([-nrm[:, 1], nrm[:, 0]], axis=1)
    both = s + ns
    t_err = np.einsum("ij,ij->i", both - 2.0 * wu, tang)[has_n]
    assert np.abs(t_err).max() < 1e-12
    sn = np.einsum("ij,ij->i", s, nrm)[has_n]
    nn = np.einsum("ij,ij->i", ns, nrm)[has_n]
    wn = np.einsum("ij,ij->i", wu, nrm)[has_n]
    assert sn.min() > -1e-12 and nn.min() > -1e-12
    kept = sn > 1e-12
    assert kept.sum() > 10 and (~kept).sum() > 10
    assert np.abs(nn[kept] - np.maximum(2.0 * wn[kept] - sn[kept], 0.0)).max() < 1e-12
    assert (nn[~kept] >= np.maximum(2.0 * wn[~kept], 0.0) - 1e-12).all()
    # no normal, nothing removed: the two forms sum to 2 u_wall outright
    assert np.abs(both[~has_n] - 2.0 * wu[~has_n]).max() < 1e-12
    assert not np.array_equal(s, ns)


# --------------------------------------------------------------- PPE solver
def _fs_case(n=12, seed=4):
    """Periodic jittered set where the free-surface test marks a few
    particles (Dirichlet p = 0 rows), which makes the PPE non-singular."""
    c = cases.taylor_green(n, kernel="wendland", hdx=1.3, jitter=0.2, seed=seed)
    rho = oracle.density(c)
    thr = np.quantile(rho, 0.1)
    return c.replace(free_surface=True, fs_ratio=float(thr / c.rho0) + 1e-12, gtvf="off", null_space="none")


def test_jacobi_converges_to_dense_solve():
    """P7: the converged Jacobi pressure solves the assembled linear system
    (numpy.linalg.solve on the non-free-surface rows; free-surface p = 0)."""
    c = _fs_case().replace(tol=1e-14, max_iter=200000, min_iter=2)
    s = oracle.Sim(c)
    out = s.step(capture=True)
    fs = out["fs"].astype(bool)
    assert 0 < fs.sum() < c.n_fluid
    n = c.n_fluid
    rho = out["rho"]
    # assemble A from the operator: (A p)_i = sum_j c_ij (p_i - p_j)
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = oracle.ppe_operator(c, out["xs"], rho, e)[0]
    inner = ~fs
    sol = np.zeros(n)
    sol[inner] = np.linalg.solve(A[np.ix_(inner, inner)], out["rhs"][inner])
    assert np.all(s.p[fs] == 0.0)
    assert rel(s.p[inner], sol[inner]) < 1e-9


def _dense_scaled_system(c, out):
    """The PPE as BiCGStab sees it, assembled column by column from the
    oracle's operator and wall extrapolation: active rows (D != 0, not free
    surface), walls by the unclamped Shepard extrapolation (linear part on
    the unknowns, hydrostatic part on the right).  Returns (A, b, active)
    with A x = b on the active rows."""
    n, nw = c.n_fluid, c.n_wall
    rho_all = np.concatenate([out["rho"], np.full(nw, c.rho0)])
    x_all = c.x.copy()
    x_all[:n] = out["xs"]
    lin = c.replace(gravity=(0.0, 0.0, 0.0), free_surface=False)
    hyd = c.replace(free_surface=False)

    def walls(case, pf):
        if nw == 0:
            return np.zeros(0)
        return oracle.wall_pressure(case, x_all, rho_all, np.concatenate([pf, np.zeros(nw)]))[n:]

    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = oracle.ppe_operator(c, x_all, rho_all, np.concatenate([e, walls(lin, e)]))[0]
    h = walls(hyd, np.zeros(n))
    b = out["rhs"] - oracle.ppe_operator(c, x_all, rho_all, np.concatenate([np.zeros(n), h]))[0]
    active = (out["diag"] != 0.0) & ~out["fs"].astype(bool)
    return A, b, active


@pytest.mark.parametrize("which", ["periodic_fs", "dam_break"])
def test_bicgstab_converges_to_dense_solve(which):
    """Section 3.1 (the BiCGStab alternative): at a tight tolerance the
    BiCGStab pressure solves the assembled system (numpy.linalg.solve), walls
    included; free-surface rows stay 0."""
    if which == "periodic_fs":
        c = _fs_case()
    else:
        c = cases.dam_break_2d(dx=0.1, precision="fp64")
    c = c.replace(solver="bicgstab", tol=1e-13, max_iter=5000)
    s = oracle.Sim(c)
    out = s.step(capture=True)
    A, b, act = _dense_scaled_system(c, out)
    assert 0 < act.sum() < c.n_fluid
    sol = np.linalg.solve(A[np.ix_(act, act)], b[act])
    assert np.all(s.p[:c.n_fluid][~act] == 0.0)
    assert rel(s.p[:c.n_fluid][act], sol) < 1e-8
    assert out["converged"] and out["iters"] < 200


def test_bicgstab_one_iteration_residual_and_ratio():
    """One forced BiCGStab iteration from p^n: the reported ratio is
    omega * sum|r_1| / max(Lambda, sum|x_1|) with r_1 the true scaled residual
    D^-1 (b - A x_1), recomputed here from the assembled system (so the
    residual recurrence, the scaling and the stopping measure are pinned)."""
    c = cases.dam_break_2d(dx=0.1, precision="fp64").replace(solver="bicgstab", forced_iters=1)
    s = oracle.Sim(c)
    out = s.step(capture=True)
    A, b, act = _dense_scaled_system(c, out)
    x1 = s.p[:c.n_fluid].copy()
    D = out["diag"]
    r1 = np.where(act, (b - A @ np.where(act, x1, 0.0)) / np.where(act, D, 1.0), 0.0)
    lam = np.max(np.abs(out["rhs"][act] / D[act]))
    ratio = c.omega * np.sum(np.abs(r1)) / max(lam, np.sum(np.abs(x1)))
    assert out["iters"] == 1
    assert math.isclose(out["ratio"], ratio, rel_tol=1e-8)


def test_bicgstab_needs_fewer_operator_applications():
    """The paper reports that BiCGStab converges in fewer iterations than
    Jacobi; at equal tolerance each BiCGStab iteration applies the operator
    twice and still needs far fewer applications on a free-surface set."""
    c = _fs_case().replace(tol=1e-6, max_iter=20000)
    j = oracle.Sim(c).step()
    b = oracle.Sim(c.replace(solver="bicgstab")).step()
    assert j["converged"] and b["converged"]
    assert 2 * b["iters"] < j["iters"] / 5


def test_bicgstab_refuses_problems_without_a_free_surface():
    with pytest.raises(ValueError):
        oracle.Sim(cases.taylor_green(12).replace(solver="bicgstab"))


def test_single_jacobi_update_eisph():
    """P8/P16: with one forced iteration the step performs exactly one update
    p1 = w (RHS + sum_j c_ij p0_j) / D + (1 - w) p0 (eq. p-sor), with
    sum_j c_ij p0_j = D p0_i - (operator applied to p0)_i; and the reported
    ratio is eq. convergence evaluated on it."""
    c = cases.taylor_green(16, jitter=0.1, seed=7)
    s = oracle.Sim(c, forced_iters=1)
    p0 = c.p.copy()
    out = s.step(capture=True)
    assert out["iters"] == 1
    lap, D = oracle.ppe_operator(c, out["xs"], out["rho"], p0)
    assert rel(D, out["diag"]) < 1e-14
    w = c.omega
    p1 = w * (out["rhs"] + D * p0 - lap) / D + (1 - w) * p0
    assert rel(s.p, p1) < 1e-11
    lam = np.max(np.abs(out["rhs"] / D))
    ratio = np.sum(np.abs(p1 - p0)) / max(lam, np.sum(np.abs(p1)))
    assert math.isclose(out["ratio"], ratio, rel_tol=1e-9)
    assert math.isclose(out["lam"], lam, rel_tol=1e-12)


def test_fixed_point_constant_pressure():
    """P5: RHS = 0 and a constant pressure is a fixed point of every update."""
    c = cases.taylor_green(16, jitter=0.2, seed=9).replace(gtvf="off")
    c.u[:] = 0.0
    c.p[:] = 3.25
    s = oracle.Sim(c.replace(tol=1e-30, max_iter=7))
    out = s.step()
    assert out["iters"] == 7
    assert np.max(np.abs(s.p - 3.25)) < 1e-12


@pytest.mark.parametrize("which", ["cloud", "single"])
def test_isolated_particles_move_ballistically(which):
    """Empty neighbour sums (sections 2-3): a particle with no neighbour but
    itself has D_ii = 0, so its pressure is 0, and no viscous, pressure,
    stress or shifting force acts on it: after k steps x = x0 + k dt u0
    (periodic) with u and the transport velocity still u0.  An isolated
    pair only exchanges equal and opposite forces (both rows sit on the free
    surface, so p = 0 there): its total momentum stays fixed."""
    c = cases.cloud_2d() if which == "cloud" else cases.single_particle()
    iso = c.meta.get("isolated", [0])
    s = oracle.Sim(c)
    steps = 3
    for _ in range(steps):
        out = s.step(capture=True)
        assert np.all(out["diag"][iso] == 0.0)
        assert np.all(s.p[iso] == 0.0)
    want = (c.x[iso] + steps * c.dt * c.u[iso]) % 1.0
    assert np.allclose(s.x[iso], want, rtol=0.0, atol=1e-14)
    assert np.array_equal(s.u[iso], c.u[iso]) and np.array_equal(s.ut[iso], c.u[iso])
    if which == "cloud":
        pr = c.meta["pair"]
        assert np.all(out["fs"][pr] == 1)
        mom0 = c.u[pr].sum(axis=0)
        assert np.allclose(s.u[pr].sum(axis=0), mom0, rtol=0.0, atol=1e-14)
        assert np.allclose(s.ut[pr].sum(axis=0), mom0, rtol=0.0, atol=1e-14)
        # and the pair did interact
        assert np.abs(s.u[pr] - c.u[pr]).max() > 1e-3
    else:
        assert out["iters"] == c.min_iter


def test_iteration_limits():
    """min 2 iterations (section 3.1) and the max_iterations cap."""
    c = cases.taylor_green(16, jitter=0.1)
    assert oracle.Sim(c.replace(tol=1e3)).step()["iters"] == 2
    out = oracle.Sim(c.replace(tol=1e-300, max_iter=5)).step()
    assert out["iters"] == 5 and not out["converged"]


@pytest.mark.parametrize("U0,g,which", [(5.0, 0.1, "cfl"), (0.01, 400.0, "force"), (0.01, 0.1, "cap")])
def test_adaptive_dt_uniform_free_fall(U0, g, which):
    """Section 3.2, adaptive steps, in closed form: a periodic lattice moving
    uniformly under gravity has no viscous, stress or pressure force, so
    max |u^n| = U0 on the first step, max |f| = g, and the next step is
    min(dt_max, 0.25 h / U0, 0.25 sqrt(h / g)).  On the second step the
    speed is |(U0, -g dt0)|, from u^n, not from u^{n+1}."""
    base = cases.periodic_lattice(16, kernel="wendland", hdx=1.3)
    u = np.zeros_like(base.u)
    u[:, 0] = U0
    dt0 = 0.05
    c = base.replace(u=u, gravity=(0.0, -g, 0.0), dt=dt0, dt_mode="adaptive")
    h = c.h
    sim = oracle.Sim(c)
    o = sim.step()
    assert o["dt"] == dt0
    assert math.isclose(o["umax"], U0, rel_tol=1e-13)
    assert math.isclose(o["fmax"], g, rel_tol=1e-12)
    terms = {"cap": dt0, "cfl": 0.25 * h / U0, "force": 0.25 * math.sqrt(h / g)}
    assert min(terms, key=terms.get) == which
    assert math.isclose(o["dt_next"], terms[which], rel_tol=1e-12)
    o2 = sim.step()
    assert o2["dt"] == o["dt_next"]
    assert math.isclose(o2["umax"], math.hypot(U0, g * dt0), rel_tol=1e-12)
    assert math.isclose(sim.t, dt0 + o["dt_next"], rel_tol=1e-15)
    # fixed mode keeps dt whatever the maxima say
    fixed = oracle.Sim(c.replace(dt_mode="fixed"))
    assert fixed.step()["dt_next"] == dt0 and fixed.step()["dt"] == dt0


@pytest.mark.parametrize("which", ["tg", "db2d"])
def test_adaptive_dt_force_is_velocity_change(which):
    """The acceleration behind the force limit is every term of the step
    (predictor forces with gravity and the pressure force), so it equals
    (u^{n+1} - u^n) / dt particle by particle; max |u^n| is the start-of-step
    speed.  A dropped term (pressure or gravity) fails this."""
    if which == "tg":
        c = cases.taylor_green(24, jitter=0.1, seed=5)
    else:
        c = cases.dam_break_2d(dx=0.05, precision="fp64")
    c = c.replace(dt_mode="adaptive")
    sim = oracle.Sim(c)
    for _ in range(3):
        u0 = sim.u.copy()
        o = sim.step()
        dv = np.linalg.norm((sim.u - u0) / o["dt"], axis=1).max()
        assert math.isclose(o["fmax"], dv, rel_tol=1e-9)
        assert math.isclose(o["umax"], np.linalg.norm(u0, axis=1).max(), rel_tol=1e-14, abs_tol=0.0)
        assert o["dt_next"] <= c.dt
        assert o["fmax"] > 0


def test_projection_reduces_divergence():
    """P12: after the solve the corrected velocity is far less divergent than
    u* (an approximate projection, so not exactly zero).  A smooth divergent
    field added to the Taylor-Green flow loses ~98 % of its discrete
    divergence on a lattice; on a jittered set the particle-scale part stays."""
    for jitter, bound in ((0.0, 0.05), (0.1, 0.3)):
        c = cases.taylor_green(32, jitter=jitter, seed=2, tol=1e-10).replace(max_iter=20000, gtvf="off")
        X, Y = c.x[:, 0], c.x[:, 1]
        c.u[:, 0] += 0.5 * np.sin(TP * X)
        c.u[:, 1] += 0.5 * np.sin(TP * Y)
        s = oracle.Sim(c)
        out = s.step(capture=True)
        rho = out["rho"]
        d_star = oracle.rhs(c, out["xs"], rho, out["us"])
        d_new = oracle.rhs(c, out["xs"], rho, out["unew"])
        assert np.linalg.norm(d_new) < bound * np.linalg.norm(d_star)


def test_symm_form_conserves_momentum_asymm_does_not():
    """P13: periodic, no body force: the symm pressure force and the
    predictor's pair terms are antisymmetric, so sum m u is conserved."""
    base = cases.taylor_green(20, jitter=0.2, seed=11)
    mom = {}
    for form in ("symm", "asymm"):
        c = base.replace(pgrad=form)
        s = oracle.Sim(c)
        m0 = (c.m[:, None] * c.u).sum(0)
        s.step()
        mom[form] = np.abs((c.m[:, None] * s.u).sum(0) - m0).max()
    scale = (base.m[:, None] * np.abs(base.u)).sum()
    assert mom["symm"] < 1e-13 * scale
    assert mom["asymm"] > 1e-9 * scale


def test_determinism():
    """P17: two runs are bitwise equal."""
    c = cases.dam_break_2d(dx=0.1, jitter=0.05)
    a, b = oracle.Sim(c), oracle.Sim(c)
    for _ in range(3):
        a.step()
        b.step()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.p, b.p) and np.array_equal(a.u, b.u)


@pytest.mark.parametrize("name", ["tg", "db2d", "db3d", "ldc", "db2d_bicgstab", "cloud"])
def test_openmp_build_is_bitwise_serial(name):
    """P17: the OpenMP build (per-row loops in parallel, every sum over rows
    serial) gives bitwise the serial build's results, on more than one
    thread."""
    c = {"tg": lambda: cases.taylor_green(40, kernel="wendland", hdx=1.3, jitter=0.2, seed=2),
         "db2d": lambda: cases.dam_break_2d(dx=0.05, jitter=0.05),
         "db3d": lambda: cases.dam_break_3d(dx=0.1, lx=0.5, ly=0.5, lz=0.6, tank_x=1.5, tank_y=0.5, tank_z=1.0),
         "ldc": lambda: cases.lid_driven_cavity(20),
         "db2d_bicgstab": lambda: cases.dam_break_2d(dx=0.1).replace(solver="bicgstab", tol=1e-4),
         "cloud": lambda: cases.cloud_2d()}[name]()
    before = oracle.threads(parallel=True)
    oracle.set_threads(4)
    assert oracle.threads(parallel=True) == 4
    a, b = oracle.Sim(c), oracle.Sim(c, parallel=True)
    for _ in range(3):
        oa, ob = a.step(), b.step()
        assert oa["iters"] == ob["iters"] and oa["ratio"] == ob["ratio"]
    oracle.set_threads(before)
    for f in ("x", "u", "ut", "p"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


# ------------------------------------------------------ whole-run behaviour
def test_taylor_green_decay_band():
    """P11: |u|max(t)/|u|max(0) follows exp(b t), b = -8 pi^2 / Re (eq. tgv;
    fixture from the printed formula), within a band calibrated for 50x50 at
    h = dx; and the last step's ratio is the golden value's neighbourhood."""
    gold = json.load(open(os.path.join(GOLDEN, "taylor_green_decay.json")))["cases"][0]
    c = cases.taylor_green(50)
    s = oracle.Sim(c)
    u0 = np.linalg.norm(c.u, axis=1).max()
    b = -8 * math.pi ** 2 / gold["re"]
    for k in range(50):
        s.step()
        ratio = np.linalg.norm(s.u, axis=1).max() / u0
        assert abs(ratio - math.exp(b * s.t)) < 0.04
    assert math.isclose(s.t, gold["t"], rel_tol=1e-12)
    assert abs(ratio - gold["decay"]) < 0.04


def test_dam_break_iterations_and_hydrostatics():
    """Table 1 / section 3.1: at eps = 1e-2 a 2D dam break needs few sweeps
    (median 2); P15: at the first step the bottom-wall pressure is
    hydrostatic, close to rho0 g H."""
    table = json.load(open(os.path.join(GOLDEN, "table1_iterations.json")))["rows"]
    target = [r for r in table if r["problem"] == "dam_break_2d" and r["tolerance"] == 0.01][0]
    c = cases.dam_break_2d(dx=0.05, tol=0.01)
    s = oracle.Sim(c)
    its = []
    for k in range(150):
        its.append(s.step()["iters"])
        if k == 0:
            xw = c.x[c.n_fluid:]
            first = (np.abs(xw[:, 1] + 0.5 * c.dx) < 1e-9) & (xw[:, 0] > 0.1) & (xw[:, 0] < 0.5)
            pw = s.p[c.n_fluid:][first]
            assert np.all(np.abs(pw - c.rho0 * 9.81 * 2.0) < 0.1 * c.rho0 * 9.81 * 2.0)
    assert min(its) >= c.min_iter
    assert np.median(its) == target["avg_iterations"]
    # the fluid has started to fall and spread along the floor
    xf = s.x[:c.n_fluid]
    assert xf[:, 0].max() > 1.1 and xf[:, 1].max() < 2.0

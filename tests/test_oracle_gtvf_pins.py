"""Pins of the oracle's GTVF homogenisation and of its summation density.

* eq. mom:sph:gtvf on an isolated pair: the force on each particle is
  -p0_i m_j / rho_j^2 W'(r, h~) r_ij / r, with the neighbour's mass and
  density (unequal here, so a swapped index fails) and the particle's own
  p0, for both kernels and two smoothing lengths.
* Section 2.1's rules inside a step: h~ = h and p0 = p_ref for internal
  flows; h~ = h/2 and p0 = min(10 |p_i|, p_ref) for external ones.
* eqs. int:gtvf:pos, int:gtvf:vel:tmp, int:vhatnp2 and int:rnp2: with K = 1
  the transport velocity is u^{n+1} + dt f0 / 2; with K = 2 it is
  u^{n+1} + dtau^2 (3 f0 + f1) / (2 dt) with f1 taken at
  r^1 = r^0 + dtau^2 f0 / 2; and r^{n+1} = r^n + dt (u~^{n+1} + u~^n) / 2.
  A dropped 1/2 dtau^2 term, or a missing 1/2 in the position update,
  changes these by O(1).
* The summation density (eq. summation_density) on an unperturbed periodic
  lattice equals the lattice sum of V W over all images within the support,
  brute force, and the partition-of-unity values of the kernels.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1908_01762_amd import cases


def _pair_case(kernel, hdx):
    c = cases.taylor_green(20, kernel=kernel, hdx=hdx, jitter=0.0)
    x = np.array([[0.40, 0.50], [0.40, 0.50]])
    return c.replace(n_fluid=2, n_wall=0, x=x, u=np.zeros((2, 2)), p=np.zeros(2),
                     m=np.array([c.m[0] * 0.8, c.m[0] * 1.3]))


@pytest.mark.parametrize("kernel,hdx", [("quintic", 1.0), ("wendland", 1.3)])
@pytest.mark.parametrize("frac", [0.15, 0.45, 0.8])
@pytest.mark.parametrize("htilde", [1.0, 0.5])
def test_gtvf_force_on_a_pair(kernel, hdx, frac, htilde):
    c = _pair_case(kernel, hdx)
    ht = htilde * c.h
    r = frac * oracle.support(kernel) * ht
    e = np.array([0.6, -0.8])
    x = np.ascontiguousarray(np.array([[0.40, 0.50], [0.40, 0.50]]) + np.outer([0.0, 1.0], r * e))
    rho = np.array([0.97, 1.04])
    p0 = np.array([2.5, 0.7])
    f = oracle.gtvf_force(c, x, rho, p0, ht)
    dwdr = oracle.dWdr(kernel, 2, r, ht)[0]
    assert dwdr < 0
    # r_01 = x0 - x1 = -r e; grad_0 W = W'(r) r_01 / r = -W' e
    f0 = -p0[0] * c.m[1] / rho[1] ** 2 * (-dwdr * e)
    f1 = -p0[1] * c.m[0] / rho[0] ** 2 * (dwdr * e)
    assert np.allclose(f[0], f0, rtol=1e-12, atol=0)
    assert np.allclose(f[1], f1, rtol=1e-12, atol=0)
    # the pair is pushed apart (background pressure is repulsive)
    assert np.dot(f[0], -e) > 0 and np.dot(f[1], e) > 0


def test_gtvf_force_vanishes_beyond_the_reduced_support():
    """With h~ = h/2 a pair between h~ R and h R feels no GTVF force."""
    c = _pair_case("wendland", 1.3)
    r = 0.75 * oracle.support("wendland") * c.h
    x = np.ascontiguousarray(np.array([[0.4, 0.5], [0.4 + r, 0.5]]))
    f = oracle.gtvf_force(c, x, np.ones(2), np.ones(2), 0.5 * c.h)
    assert np.all(f == 0.0)
    assert np.abs(oracle.gtvf_force(c, x, np.ones(2), np.ones(2), c.h)).max() > 0


def _step_capture(case):
    s = oracle.Sim(case)
    out = s.step(capture=True)
    return s, out


def test_gtvf_internal_rule_in_a_step():
    """Internal flow (Taylor-Green): h~ = h, p0 = p_ref, the reference
    pressure being twice the largest pressure after the first solve."""
    case = cases.taylor_green(16, jitter=0.2, seed=4)
    s, out = _step_capture(case)
    nf = case.n_fluid
    p_ref = out["p_ref"]
    assert math.isclose(p_ref, 2.0 * s.p[:nf].max(), rel_tol=1e-15)
    want = oracle.gtvf_force(case, out["xs"], out["rho"], np.full(nf, p_ref), case.h)
    assert np.allclose(out["fgtvf0"], want, rtol=1e-12, atol=1e-14 * np.abs(want).max())


def test_gtvf_external_rule_in_a_step():
    """External flow (dam break): h~ = h/2, p0_i = min(10 |p_i|, p_ref) with
    the solved pressure and p_ref = rho0 (10 v_ref)^2 fixed."""
    case = cases.dam_break_2d(dx=0.05, jitter=0.05)
    assert case.gtvf == "external"
    s, out = _step_capture(case)
    nf = case.n_fluid
    xs = case.x.copy()
    xs[:nf] = out["xs"]
    rho_all = np.concatenate([out["rho"], np.full(case.n_wall, case.rho0)])
    p0 = np.minimum(10.0 * np.abs(s.p[:nf]), case.p_ref)
    assert np.any(p0 < case.p_ref) and np.any(p0 > 0)
    want = oracle.gtvf_force(case, xs, rho_all, p0, 0.5 * case.h)
    assert np.allclose(out["fgtvf0"], want, rtol=1e-12, atol=1e-13 * np.abs(want).max())
    # the full smoothing length would give a different force
    other = oracle.gtvf_force(case, xs, rho_all, p0, case.h)
    assert np.abs(other - want).max() > 0.1 * np.abs(want).max()


@pytest.mark.parametrize("K", [1, 2])
def test_gtvf_substeps_and_transport_velocity(K):
    case = cases.taylor_green(16, jitter=0.2, seed=6, p_ref_mode="fixed", p_ref=40.0, gtvf_K=K)
    x0, ut0 = case.x.copy(), case.u.copy()
    s, out = _step_capture(case)
    dt = case.dt
    dtau = dt / K
    f0 = out["fgtvf0"]
    assert np.abs(f0).max() > 0
    if K == 1:
        disp = 0.5 * dtau * dtau * f0
    else:
        r1 = np.ascontiguousarray(out["xs"] + 0.5 * dtau * dtau * f0)
        rho_all = np.ascontiguousarray(out["rho"])
        f1 = oracle.gtvf_force(case, r1, rho_all, np.full(case.n_fluid, 40.0), case.h)
        disp = dtau * dtau * (1.5 * f0 + 0.5 * f1)
    got = s.ut - out["unew"]
    # f1 here comes from the neighbour sets at r^1, the step keeps those at
    # r*; a pair crossing the support radius in between adds a term of
    # order W'(R - |dr|), about 1e-7 of the force at this p_ref
    assert np.allclose(got, disp / dt, rtol=0, atol=1e-6 * np.abs(disp / dt).max())
    # eq. int:rnp2 with the step's own transport velocity, wrapped into the
    # periodic box
    xn = x0 + 0.5 * dt * (s.ut + ut0)
    xn = xn - np.floor(xn)
    assert np.allclose(s.x, xn, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kernel,hdx,dim,expect", [
    ("quintic", 1.0, 2, 1.0000632246),
    ("wendland", 1.3, 2, 1.0104731521),
    ("wendland", 1.3, 3, 1.0095007838),
])
def test_lattice_density_is_the_lattice_sum(kernel, hdx, dim, expect):
    n = 12 if dim == 3 else 24
    c = cases.periodic_lattice(n, dim=dim, kernel=kernel, hdx=hdx)
    rho = oracle.density(c)
    dx, h = c.dx, c.h
    R = oracle.support(kernel) * h
    k = int(math.ceil(R / dx)) + 1
    total = 0.0
    for off in itertools.product(range(-k, k + 1), repeat=dim):
        r = dx * math.sqrt(sum(o * o for o in off))
        if r < R:
            total += dx ** dim * c.rho0 * oracle.W(kernel, dim, r, h)[0]
    assert np.allclose(rho, total, rtol=1e-12, atol=0)
    assert abs(rho.mean() / c.rho0 - expect) < 1e-9

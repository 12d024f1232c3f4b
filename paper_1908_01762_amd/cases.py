"""Seeded synthetic particle sets for the SISPH hot path.

This module only lays particles out and fills in the initial fields of the
paper's test problems (Taylor-Green vortex, section 4.1, eq. tgv; lid-driven
cavity, section 4.3; 2D/3D dam break, sections 4.5-4.6).  It holds none of the
method's arithmetic: no kernel, no neighbour search, no SPH sum.  Both the CPU
oracle and the HIP path consume exactly the arrays built here, so a parity
test compares two implementations on the same bytes.

Every array is float64, row-major, fluid rows first and wall rows after them:

* ``x``  [n_fluid + n_wall][dim]   positions
* ``u``  [n_fluid][dim]            fluid velocity (the transport velocity starts
                                   equal to it)
* ``p``  [n_fluid + n_wall]        pressure (walls start at 0)
* ``m``  [n_fluid + n_wall]        mass
* ``wall_u`` [n_wall][dim]         prescribed wall velocity (zero for static
                                   walls, (U, 0) for the cavity lid)

Random numbers come from numpy's PCG64 seeded per case; the jitter is uniform
in [-j*dx, +j*dx] per coordinate, mass and density unchanged.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

KERNELS = {"quintic": 0, "wendland": 1}
PGRAD = {"asymm": 0, "symm": 1}
GTVF = {"off": 0, "internal": 1, "external": 2}
PREF = {"fixed": 0, "twice_max": 1}
PRECISION = {"fp64": 0, "mixed": 1, "fp32": 2}
CONV = {"sum": 0, "mean": 1}
USTAR = {"slip": 0, "noslip": 1}
DT_MODE = {"fixed": 0, "adaptive": 1}
SOLVER = {"jacobi": 0, "bicgstab": 1}
NULL_SPACE = {"none": 0, "project": 1}
SUPPORT = {"quintic": 3.0, "wendland": 2.0}


@dataclasses.dataclass
class Case:
    """One SISPH problem: parameters (SI units) plus the initial particle set."""

    name: str
    dim: int
    kernel: str
    h: float
    dx: float
    rho0: float
    nu: float
    alpha: float
    c_ref: float
    dt: float
    tol: float
    pgrad: str
    gtvf: str
    p_ref_mode: str
    p_ref: float
    free_surface: bool
    gravity: tuple
    box_lo: tuple
    box_hi: tuple
    periodic: tuple
    x: np.ndarray
    u: np.ndarray
    p: np.ndarray
    m: np.ndarray
    n_fluid: int
    n_wall: int
    wall_u: Optional[np.ndarray] = None
    precision: str = "fp64"
    eta: float = 0.01
    fs_ratio: float = 0.8
    omega: float = 0.5
    min_iter: int = 2
    max_iter: int = 1000
    gtvf_K: int = 5
    forced_iters: int = 0
    conv_norm: str = "sum"
    ustar_wall: str = "slip"
    dt_mode: str = "fixed"       # "adaptive": dt is the first step's and the largest step
    solver: str = "jacobi"       # "bicgstab": the PPE by BiCGStab on the same operator
    # "project": fully periodic cases (no walls, no free surface) remove the
    # RHS component the singular operator cannot match; "none": as printed
    null_space: str = "none"
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.n_fluid + self.n_wall

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)

    def copy(self) -> "Case":
        c = dataclasses.replace(self)
        for k in ("x", "u", "p", "m", "wall_u"):
            v = getattr(self, k)
            if v is not None:
                setattr(c, k, v.copy())
        c.meta = dict(self.meta)
        return c


def _wrap_periodic(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Map coordinates into [lo, hi) (the same branch rule both sides use)."""
    L = hi - lo
    out = x.copy()
    big = out >= hi
    out[big] -= L
    small = out < lo
    out[small] += L
    out[small & (out >= hi)] = lo
    return out


def taylor_green(n: int = 50, kernel: str = "quintic", hdx: float = 1.0,
                 re: float = 100.0, U: float = 1.0, jitter: float = 0.01,
                 seed: int = 0, tol: float = 1e-4, pgrad: str = "asymm",
                 precision: str = "fp64", gtvf_K: int = 5,
                 p_ref_mode: str = "twice_max", p_ref: float = 0.0,
                 dt: Optional[float] = None, null_space: str = "project") -> Case:
    """Periodic unit-square Taylor-Green vortex (eq. tgv at t = 0).

    Lattice x = (i + 1/2) dx, uniform jitter of +-jitter*dx per coordinate,
    velocity and pressure taken exactly at the jittered positions, rho0 = 1,
    m = rho0 dx^2, nu = U L / Re with L = 1.  The fixed time step is the
    minimum of the advective and viscous limits (section 3.2), there is no
    body force here.  The PPE of this wall-less, fully periodic problem is
    singular (constants solve it); ``null_space="project"`` (the default)
    removes the RHS component it cannot match, ``"none"`` iterates as
    printed.
    """
    L = 1.0
    dx = L / n
    h = hdx * dx
    nu = U * L / re
    rng = np.random.Generator(np.random.PCG64(seed))
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = np.stack([(ii.ravel() + 0.5) * dx, (jj.ravel() + 0.5) * dx], axis=1)
    if jitter > 0:
        x = x + rng.uniform(-jitter * dx, jitter * dx, size=x.shape)
    x = _wrap_periodic(x, 0.0, L)
    X, Y = x[:, 0], x[:, 1]
    tw = 2.0 * math.pi
    u = np.stack([-U * np.cos(tw * X) * np.sin(tw * Y),
                  U * np.sin(tw * X) * np.cos(tw * Y)], axis=1)
    p = -U * U * (np.cos(2 * tw * X) + np.cos(2 * tw * Y)) / 4.0
    rho0 = 1.0
    m = np.full(n * n, rho0 * dx * dx)
    if dt is None:
        dt = min(0.25 * h / U, 0.25 * h * h / nu)
    return Case(
        name=f"tg{n}", dim=2, kernel=kernel, h=h, dx=dx, rho0=rho0, nu=nu,
        alpha=0.0, c_ref=10.0 * U, dt=dt, tol=tol, pgrad=pgrad,
        gtvf="internal", p_ref_mode=p_ref_mode, p_ref=p_ref,
        free_surface=False, gravity=(0.0, 0.0, 0.0),
        box_lo=(0.0, 0.0, 0.0), box_hi=(L, L, 0.0), periodic=(1, 1, 0),
        x=np.ascontiguousarray(x), u=np.ascontiguousarray(u),
        p=np.ascontiguousarray(p), m=m, n_fluid=n * n, n_wall=0,
        wall_u=None, precision=precision, gtvf_K=gtvf_K, null_space=null_space,
        meta=dict(re=re, U=U, seed=seed, jitter=jitter, lattice=n))


def _lattice(counts, dx, origin):
    grids = np.meshgrid(*[np.arange(c) for c in counts], indexing="ij")
    pts = np.stack([g.ravel() for g in grids], axis=1).astype(np.float64)
    return (pts + 0.5) * dx + np.asarray(origin, dtype=np.float64)


def dam_break_2d(dx: float = 0.005, width: float = 1.0, height: float = 2.0,
                 tank: float = 4.0, layers: int = 3, kernel: str = "wendland",
                 hdx: float = 1.3, alpha: float = 0.05, tol: float = 1e-3,
                 g: float = 9.81, precision: str = "mixed", gtvf_K: int = 5,
                 jitter: float = 0.0, seed: int = 0, nu: float = 0.0,
                 dt: Optional[float] = None) -> Case:
    """Water column width x height at the left of an open-top tank x tank tank.

    Fluid on the lattice (i + 1/2) dx inside [0, width] x [0, height];
    ``layers`` rows of wall particles at (i + 1/2) dx outside the tank: the
    bottom (spanning the corners) and both sides up to y = tank.  rho0 = 1000,
    u = 0, hydrostatic initial pressure rho0 g (height - y), static walls.
    The fixed step is 0.125 h / sqrt(2 g height) (section 4.5); artificial
    sound speed c_ref = 10 sqrt(2 g height); the GTVF reference pressure is
    rho0 c_ref^2 (external-flow setting of section 2.1).
    """
    rho0 = 1000.0
    h = hdx * dx
    nxf, nyf = int(round(width / dx)), int(round(height / dx))
    xf = _lattice((nxf, nyf), dx, (0.0, 0.0))
    ntank = int(round(tank / dx))
    bottom = _lattice((ntank + 2 * layers, layers), dx, (-layers * dx, -layers * dx))
    left = _lattice((layers, ntank), dx, (-layers * dx, 0.0))
    right = _lattice((layers, ntank), dx, (tank, 0.0))
    xw = np.concatenate([bottom, left, right], axis=0)
    rng = np.random.Generator(np.random.PCG64(seed))
    if jitter > 0:
        xf = xf + rng.uniform(-jitter * dx, jitter * dx, size=xf.shape)
    nf, nw = xf.shape[0], xw.shape[0]
    x = np.concatenate([xf, xw], axis=0)
    u = np.zeros((nf, 2))
    p = np.zeros(nf + nw)
    p[:nf] = rho0 * g * (height - xf[:, 1])
    m = np.full(nf + nw, rho0 * dx * dx)
    vref = math.sqrt(2.0 * g * height)
    c_ref = 10.0 * vref
    if dt is None:
        dt = 0.125 * h / vref
    return Case(
        name="db2d", dim=2, kernel=kernel, h=h, dx=dx, rho0=rho0, nu=nu,
        alpha=alpha, c_ref=c_ref, dt=dt, tol=tol, pgrad="symm",
        gtvf="external", p_ref_mode="fixed", p_ref=rho0 * c_ref * c_ref,
        free_surface=True, gravity=(0.0, -g, 0.0),
        box_lo=(-layers * dx, -layers * dx, 0.0),
        box_hi=(tank + layers * dx, tank, 0.0), periodic=(0, 0, 0),
        x=np.ascontiguousarray(x), u=u, p=p, m=m, n_fluid=nf, n_wall=nw,
        wall_u=np.zeros((nw, 2)), precision=precision, gtvf_K=gtvf_K,
        meta=dict(height=height, width=width, tank=tank, layers=layers, g=g))


def lid_driven_cavity(n: int = 50, re: float = 100.0, U: float = 1.0,
                      layers: int = 3, kernel: str = "quintic",
                      hdx: float = 1.0, tol: float = 1e-2,
                      pgrad: str = "symm", precision: str = "fp64",
                      ustar_wall: str = "slip", gtvf_K: int = 5,
                      jitter: float = 0.0, seed: int = 0,
                      dt: Optional[float] = None) -> Case:
    """Unit-square lid-driven cavity (section 4.3).

    n x n fluid particles on the lattice (i + 1/2) dx of [0, 1]^2 at rest,
    rho0 = 1, p = 0, nu = U L / Re.  ``layers`` rows of wall particles at
    (i + 1/2) dx outside the square on all four sides; the bottom and top
    strips span the corners.  The top strip (the lid) moves with
    (U, 0); the others are static.  Internal flow: GTVF background pressure
    2 max p after the first solve.  The fixed step is the minimum of the
    advective and viscous limits (section 3.2).  ``ustar_wall`` selects the
    wall ghost form for u* in the PPE (slip by default; the section compares
    it with the no-slip form, section 3.4).
    """
    L = 1.0
    dx = L / n
    h = hdx * dx
    nu = U * L / re
    xf = _lattice((n, n), dx, (0.0, 0.0))
    span = n + 2 * layers
    bottom = _lattice((span, layers), dx, (-layers * dx, -layers * dx))
    top = _lattice((span, layers), dx, (-layers * dx, L))
    left = _lattice((layers, n), dx, (-layers * dx, 0.0))
    right = _lattice((layers, n), dx, (L, 0.0))
    xw = np.concatenate([bottom, left, right, top], axis=0)
    rng = np.random.Generator(np.random.PCG64(seed))
    if jitter > 0:
        xf = xf + rng.uniform(-jitter * dx, jitter * dx, size=xf.shape)
    nf, nw = xf.shape[0], xw.shape[0]
    wall_u = np.zeros((nw, 2))
    wall_u[nw - top.shape[0]:, 0] = U
    rho0 = 1.0
    if dt is None:
        dt = min(0.25 * h / U, 0.25 * h * h / nu)
    return Case(
        name=f"ldc{n}", dim=2, kernel=kernel, h=h, dx=dx, rho0=rho0, nu=nu,
        alpha=0.0, c_ref=10.0 * U, dt=dt, tol=tol, pgrad=pgrad,
        gtvf="internal", p_ref_mode="twice_max", p_ref=0.0,
        free_surface=False, gravity=(0.0, 0.0, 0.0),
        box_lo=(-layers * dx, -layers * dx, 0.0),
        box_hi=(L + layers * dx, L + layers * dx, 0.0), periodic=(0, 0, 0),
        x=np.ascontiguousarray(np.concatenate([xf, xw], axis=0)),
        u=np.zeros((nf, 2)), p=np.zeros(nf + nw),
        m=np.full(nf + nw, rho0 * dx * dx), n_fluid=nf, n_wall=nw,
        wall_u=wall_u, precision=precision, gtvf_K=gtvf_K,
        ustar_wall=ustar_wall,
        meta=dict(re=re, U=U, layers=layers, lattice=n))


def dam_break_3d(dx: float = 0.01, lx: float = 1.0, ly: float = 1.0,
                 lz: float = 2.0, tank_x: float = 4.0, tank_y: float = 1.0,
                 tank_z: float = 4.0, layers: int = 3, kernel: str = "wendland",
                 hdx: float = 1.3, alpha: float = 0.25, tol: float = 1e-3,
                 g: float = 9.81, precision: str = "mixed", gtvf_K: int = 5,
                 nu: float = 0.0, dt: Optional[float] = None) -> Case:
    """Water block lx x ly x lz in the corner of an open-top tank.

    Walls: ``layers`` layers below the bottom (spanning the corners) and
    outside the four sides, up to z = tank_z.  Gravity along -z.  Same
    parameter rules as the 2D case, with alpha = 0.25 (section 4.6).
    """
    rho0 = 1000.0
    h = hdx * dx
    nfx, nfy, nfz = (int(round(v / dx)) for v in (lx, ly, lz))
    xf = _lattice((nfx, nfy, nfz), dx, (0.0, 0.0, 0.0))
    ntx, nty, ntz = (int(round(v / dx)) for v in (tank_x, tank_y, tank_z))
    L = layers
    parts = [
        _lattice((ntx + 2 * L, nty + 2 * L, L), dx, (-L * dx, -L * dx, -L * dx)),  # bottom
        _lattice((L, nty + 2 * L, ntz), dx, (-L * dx, -L * dx, 0.0)),              # x- side
        _lattice((L, nty + 2 * L, ntz), dx, (tank_x, -L * dx, 0.0)),               # x+ side
        _lattice((ntx, L, ntz), dx, (0.0, -L * dx, 0.0)),                          # y- side
        _lattice((ntx, L, ntz), dx, (0.0, tank_y, 0.0)),                           # y+ side
    ]
    xw = np.concatenate(parts, axis=0)
    nf, nw = xf.shape[0], xw.shape[0]
    x = np.concatenate([xf, xw], axis=0)
    u = np.zeros((nf, 3))
    p = np.zeros(nf + nw)
    p[:nf] = rho0 * g * (lz - xf[:, 2])
    m = np.full(nf + nw, rho0 * dx ** 3)
    vref = math.sqrt(2.0 * g * lz)
    c_ref = 10.0 * vref
    if dt is None:
        dt = 0.125 * h / vref
    return Case(
        name="db3d", dim=3, kernel=kernel, h=h, dx=dx, rho0=rho0, nu=nu,
        alpha=alpha, c_ref=c_ref, dt=dt, tol=tol, pgrad="symm",
        gtvf="external", p_ref_mode="fixed", p_ref=rho0 * c_ref * c_ref,
        free_surface=True, gravity=(0.0, 0.0, -g),
        box_lo=(-L * dx, -L * dx, -L * dx),
        box_hi=(tank_x + L * dx, tank_y + L * dx, tank_z), periodic=(0, 0, 0),
        x=np.ascontiguousarray(x), u=u, p=p, m=m, n_fluid=nf, n_wall=nw,
        wall_u=np.zeros((nw, 3)), precision=precision, gtvf_K=gtvf_K,
        meta=dict(height=lz, g=g, layers=layers))


def cloud_2d(n: int = 40, radius: float = 0.3, seed: int = 7,
             precision: str = "fp64") -> Case:
    """Degenerate rows in one case: a free-surface disc of the jittered
    Taylor-Green lattice (Wendland, h = 1.3 dx) in the periodic unit square,
    plus two isolated particles (no neighbour but themselves, so D_ii = 0)
    and an isolated pair, each far from everything else.  The isolated
    particles start at rest and at U = (0.3, -0.2); the pair with opposite
    velocities."""
    c = taylor_green(n, kernel="wendland", hdx=1.3, jitter=0.2, seed=seed, precision=precision)
    dx = c.dx
    keep = np.linalg.norm(c.x - 0.5, axis=1) < radius
    extra_x = np.array([[0.04, 0.04], [0.93, 0.1],
                        [0.08, 0.88], [0.08 + 0.8 * dx, 0.88 + 0.3 * dx]])
    extra_u = np.array([[0.0, 0.0], [0.3, -0.2], [0.1, 0.0], [-0.1, 0.05]])
    x = np.ascontiguousarray(np.vstack([c.x[keep], extra_x]))
    u = np.ascontiguousarray(np.vstack([c.u[keep], extra_u]))
    N = x.shape[0]
    return c.replace(name=f"cloud{n}", x=x, u=u, p=np.zeros(N), m=np.full(N, c.m[0]),
                     n_fluid=N, free_surface=True, null_space="none",
                     meta=dict(c.meta, isolated=[N - 4, N - 3], pair=[N - 2, N - 1]))


def single_particle(precision: str = "fp64") -> Case:
    """One particle alone in the periodic unit square (quintic, 10 x 10
    lattice spacing): every neighbour sum is empty."""
    c = taylor_green(10, precision=precision)
    return c.replace(name="single", x=np.array([[0.3, 0.6]]), u=np.array([[0.2, -0.1]]),
                     p=np.zeros(1), m=c.m[:1].copy(), n_fluid=1)


def long_strip(nx: int = 16384, ny: int = 8, seed: int = 9) -> Case:
    """Periodic strip nx x ny particles (Wendland h = 1.3 dx, cells of about
    2.7 dx): one row of cells holds ~44k particles, so neighbours in the next
    cell row are more than 32767 rows away and the 16-bit offsets cannot be
    used."""
    base = taylor_green(16, kernel="wendland", hdx=1.3, precision="mixed")
    dx = 1.0 / 1024
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = np.stack([(ii.ravel() + 0.5) * dx, (jj.ravel() + 0.5) * dx], axis=1)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = x + rng.uniform(-0.05 * dx, 0.05 * dx, size=x.shape)
    Lx, Ly = nx * dx, ny * dx
    x[:, 0] = np.mod(x[:, 0], Lx)
    x[:, 1] = np.mod(x[:, 1], Ly)
    u = 0.1 * np.stack([np.sin(2 * np.pi * x[:, 1] / Ly), np.sin(2 * np.pi * x[:, 0] / Lx)], axis=1)
    n = x.shape[0]
    h = 1.3 * dx
    return base.replace(name="strip", x=x, u=u, p=np.zeros(n), m=np.full(n, dx * dx), n_fluid=n,
                        h=h, dx=dx, box_lo=(0.0, 0.0, 0.0), box_hi=(Lx, Ly, 0.0), nu=1e-3,
                        dt=0.25 * h / 0.1, tol=1e-4, p_ref_mode="twice_max")


def periodic_lattice(n: int, dim: int = 2, kernel: str = "quintic",
                     hdx: float = 1.0, rho0: float = 1.0) -> Case:
    """Unperturbed periodic lattice at rest (used for symmetry pins)."""
    c = taylor_green(n, kernel=kernel, hdx=hdx, jitter=0.0)
    if dim == 2:
        c.u[:] = 0.0
        c.p[:] = 0.0
        return c
    dx = 1.0 / n
    x = _lattice((n, n, n), dx, (0.0, 0.0, 0.0))
    N = x.shape[0]
    return dataclasses.replace(
        c, name=f"lattice3d{n}", dim=3, x=x, u=np.zeros((N, 3)), p=np.zeros(N),
        m=np.full(N, rho0 * dx ** 3), n_fluid=N, n_wall=0,
        box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
        h=hdx * dx, dx=dx, rho0=rho0)


def serving_mix(n_cases: int = 64, seed: int = 0, rate_hz: float = 20.0,
                n_min: int = 2500, n_max: int = 160000,
                re_range=(50.0, 1000.0), precision: str = "mixed"):
    """Request stream for the serving loop.

    Exponential inter-arrival times (Poisson arrivals at ``rate_hz``), case
    type Bernoulli(1/2) between Taylor-Green and 2D dam break, Re uniform in
    ``re_range`` and particle count log-uniform in [n_min, n_max].  Returns a
    list of (arrival_time_s, Case).  For the dam break the viscosity is
    v_ref * height / Re.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(n_cases):
        t += rng.exponential(1.0 / rate_hz)
        kind = rng.integers(0, 2)
        re = rng.uniform(*re_range)
        N = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        if kind == 0:
            n = max(8, int(round(math.sqrt(N))))
            c = taylor_green(n, kernel="wendland", hdx=1.3, re=re,
                             seed=int(rng.integers(0, 2**31)), precision=precision)
        else:
            nx = max(4, int(round(math.sqrt(N / 2.0))))
            dx = 1.0 / nx
            height = 2.0
            nu = math.sqrt(2.0 * 9.81 * height) * height / re
            c = dam_break_2d(dx=dx, precision=precision, nu=nu)
        c.name = f"req{k}-{c.name}"
        c.meta["re"] = re
        out.append((t, c))
    return out

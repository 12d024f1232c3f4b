"""Python access to the SISPH CPU oracle (``sisph_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark import this package; the product library never does.
It takes the seeded cases of ``paper_1908_01762_amd.cases`` (plain arrays and
parameters) and runs the FP64 reference of one SISPH step on them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sisph_oracle.c")
_HDR = os.path.join(_HERE, "sisph_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")          # serial
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")  # OpenMP, bitwise equal to the serial build

KERNEL = {"quintic": 0, "wendland": 1}
PGRAD = {"asymm": 0, "symm": 1}
GTVF = {"off": 0, "internal": 1, "external": 2}
PREF = {"fixed": 0, "twice_max": 1}
CONV = {"sum": 0, "mean": 1}
USTAR = {"slip": 0, "noslip": 1}
DT_MODE = {"fixed": 0, "adaptive": 1}
SOLVER = {"jacobi": 0, "bicgstab": 1}
NULL_SPACE = {"none": 0, "project": 1}


def build(force: bool = False, parallel: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, so FP64 ops are exact as
    written): the serial build, or the OpenMP one (per-row loops in
    parallel, sums over rows serial: bitwise the same results)."""
    lib_path = _LIB_OMP if parallel else _LIB
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < newest:
        tmp = lib_path + ".tmp"
        omp = ["-fopenmp"] if parallel else ["-Wno-unknown-pragmas"]
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC",
                               "-shared", "-Wall"] + omp + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib_path)
    return lib_path


class Params(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "dim", "kernel", "pgrad", "gtvf", "free_surface", "p_ref_mode",
        "min_iter", "max_iter", "gtvf_K", "forced_iters", "conv_norm", "ustar_wall", "dt_mode",
        "solver", "null_space", "nf", "nw")] + \
        [(n, C.c_double) for n in (
            "h", "rho0", "nu", "alpha", "c_ref", "dt", "eta", "fs_ratio", "omega", "tol", "dt_max")] + \
        [("g", C.c_double * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
         ("periodic", C.c_int64 * 3)]


_DP = C.POINTER(C.c_double)
_I64P = C.POINTER(C.c_int64)


class StepOut(C.Structure):
    _fields_ = [(n, _DP) for n in ("rho", "xs", "us", "uw", "usw", "rhs", "diag",
                                   "unew", "fgtvf0")] + \
        [("fs", _I64P), ("iters", C.c_int64), ("converged", C.c_int64),
         ("ratio", C.c_double), ("lambda_", C.c_double), ("p_ref_used", C.c_double),
         ("beta", C.c_double),
         ("umax", C.c_double), ("fmax", C.c_double), ("dt_next", C.c_double)]


_libs = {}


def lib(parallel: bool = False):
    """The serial oracle library, or the OpenMP build."""
    if parallel not in _libs:
        L = C.CDLL(build(parallel=parallel))
        L.orc_W.restype = C.c_double
        L.orc_W.argtypes = [C.c_int64, C.c_int64, C.c_double, C.c_double]
        L.orc_dWdr.restype = C.c_double
        L.orc_dWdr.argtypes = [C.c_int64, C.c_int64, C.c_double, C.c_double]
        L.orc_support.restype = C.c_double
        L.orc_support.argtypes = [C.c_int64]
        for f in ("orc_neighbors_brute", "orc_neighbors_cells"):
            getattr(L, f).restype = C.c_int64
        L.orc_step.restype = C.c_int64
        L.orc_threads.restype = C.c_int64
        _libs[parallel] = L
    return _libs[parallel]


def threads(parallel: bool = True) -> int:
    """Threads the per-row loops of that build use."""
    return int(lib(parallel).orc_threads())


def set_threads(n: int) -> None:
    """Threads of the OpenMP build's per-row loops."""
    lib(True).orc_set_threads(C.c_int64(int(n)))


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.float64:
        return a.ctypes.data_as(_DP)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_I64P)
    if a.dtype == np.int32:
        return a.ctypes.data_as(C.POINTER(C.c_int32))
    raise TypeError(a.dtype)


def params(case, **over) -> Params:
    P = Params()
    P.dim = case.dim
    P.kernel = KERNEL[case.kernel]
    P.pgrad = PGRAD[case.pgrad]
    P.gtvf = GTVF[case.gtvf]
    P.free_surface = int(bool(case.free_surface))
    P.p_ref_mode = PREF[case.p_ref_mode]
    P.min_iter = case.min_iter
    P.max_iter = case.max_iter
    P.gtvf_K = case.gtvf_K
    P.forced_iters = case.forced_iters
    P.conv_norm = CONV[case.conv_norm]
    P.ustar_wall = USTAR[case.ustar_wall]
    P.dt_mode = DT_MODE[case.dt_mode]
    P.solver = SOLVER[case.solver]
    P.null_space = NULL_SPACE[case.null_space]
    P.dt_max = float(case.dt)
    P.nf = case.n_fluid
    P.nw = case.n_wall
    for k in ("h", "rho0", "nu", "alpha", "c_ref", "dt", "eta", "fs_ratio", "omega", "tol"):
        setattr(P, k, float(getattr(case, k)))
    for k in range(3):
        P.g[k] = case.gravity[k]
        P.lo[k] = case.box_lo[k]
        P.hi[k] = case.box_hi[k]
        P.periodic[k] = int(case.periodic[k])
    for k, v in over.items():
        setattr(P, k, v)
    return P


def W(kernel: str, dim: int, r, h: float) -> np.ndarray:
    L = lib()
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    return np.array([L.orc_W(KERNEL[kernel], dim, float(v), h) for v in r])


def dWdr(kernel: str, dim: int, r, h: float) -> np.ndarray:
    L = lib()
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    return np.array([L.orc_dWdr(KERNEL[kernel], dim, float(v), h) for v in r])


def support(kernel: str) -> float:
    return lib().orc_support(KERNEL[kernel])


def neighbors(case, x=None, dest=None, src=None, method: str = "cells"):
    """CSR (offsets, ids) of {j in src : |r_ij|^2 < R^2} for i in dest."""
    x = np.ascontiguousarray(case.x if x is None else x, dtype=np.float64)
    d0, d1 = dest if dest is not None else (0, case.n_fluid)
    s0, s1 = src if src is not None else (0, case.n)
    P = params(case)
    off = np.zeros(d1 - d0 + 1, dtype=np.int64)
    cap = max(1, 256 * (d1 - d0))
    ids = np.zeros(cap, dtype=np.int32)
    fn = lib().orc_neighbors_brute if method == "brute" else lib().orc_neighbors_cells
    n = fn(C.byref(P), _ptr(x), C.c_int64(d0), C.c_int64(d1), C.c_int64(s0), C.c_int64(s1),
           _ptr(off), _ptr(ids), C.c_int64(cap))
    if n < 0:
        raise RuntimeError("neighbour capacity exceeded")
    return off, ids[:n].copy()


def wall_normals(case, x=None) -> np.ndarray:
    x = np.ascontiguousarray(case.x if x is None else x)
    nrm = np.zeros((case.n_wall, case.dim))
    if case.n_wall:
        lib().orc_wall_normals(C.byref(params(case)), _ptr(x), _ptr(case.m), _ptr(nrm))
    return nrm


def _all(case, fluid_vals, wall_vals):
    return np.ascontiguousarray(np.concatenate([fluid_vals, wall_vals], axis=0))


def density(case, x=None) -> np.ndarray:
    x = np.ascontiguousarray(case.x if x is None else x)
    rho = np.zeros(case.n_fluid)
    lib().orc_density(C.byref(params(case)), _ptr(x), _ptr(case.m), _ptr(rho))
    return rho


def predictor_forces(case, x, u_all, ut, rho_all) -> np.ndarray:
    f = np.zeros((case.n_fluid, case.dim))
    lib().orc_predictor_forces(C.byref(params(case)), _ptr(np.ascontiguousarray(x)),
                               _ptr(np.ascontiguousarray(u_all)), _ptr(np.ascontiguousarray(ut)),
                               _ptr(case.m), _ptr(np.ascontiguousarray(rho_all)), _ptr(f))
    return f


def ppe_operator(case, x, rho_all, p_all):
    """(sum_j c_ij (p_i - p_j), D_ii) for every fluid particle."""
    lap = np.zeros(case.n_fluid)
    diag = np.zeros(case.n_fluid)
    lib().orc_ppe_operator(C.byref(params(case)), _ptr(np.ascontiguousarray(x)), _ptr(case.m),
                           _ptr(np.ascontiguousarray(rho_all)), _ptr(np.ascontiguousarray(p_all)),
                           _ptr(lap), _ptr(diag))
    return lap, diag


def rhs(case, x, rho_all, us_all) -> np.ndarray:
    out = np.zeros(case.n_fluid)
    lib().orc_rhs(C.byref(params(case)), _ptr(np.ascontiguousarray(x)), _ptr(case.m),
                  _ptr(np.ascontiguousarray(rho_all)), _ptr(np.ascontiguousarray(us_all)), _ptr(out))
    return out


def pressure_force(case, x, rho_all, p_all, pgrad: Optional[str] = None) -> np.ndarray:
    f = np.zeros((case.n_fluid, case.dim))
    P = params(case) if pgrad is None else params(case, pgrad=PGRAD[pgrad])
    lib().orc_pressure_force(C.byref(P), _ptr(np.ascontiguousarray(x)), _ptr(case.m),
                             _ptr(np.ascontiguousarray(rho_all)), _ptr(np.ascontiguousarray(p_all)),
                             _ptr(f))
    return f


def gtvf_force(case, x, rho_all, p0, hgtvf) -> np.ndarray:
    f = np.zeros((case.n_fluid, case.dim))
    lib().orc_gtvf_force(C.byref(params(case)), _ptr(np.ascontiguousarray(x)), _ptr(case.m),
                         _ptr(np.ascontiguousarray(rho_all)), _ptr(np.ascontiguousarray(p0)),
                         C.c_double(hgtvf), _ptr(f))
    return f


def wall_pressure(case, x, rho_all, p_all) -> np.ndarray:
    p = np.ascontiguousarray(p_all, dtype=np.float64).copy()
    lib().orc_wall_pressure(C.byref(params(case)), _ptr(np.ascontiguousarray(x)),
                            _ptr(np.ascontiguousarray(rho_all)), _ptr(p))
    return p


def wall_velocity(case, x, u_fluid, nrm, slip: bool, wall_u=None) -> np.ndarray:
    uw = np.zeros((case.n_wall, case.dim))
    wu = None if wall_u is None else np.ascontiguousarray(wall_u)
    lib().orc_wall_velocity(C.byref(params(case)), _ptr(np.ascontiguousarray(x)),
                            _ptr(np.ascontiguousarray(u_fluid)), _ptr(wu),
                            _ptr(np.ascontiguousarray(nrm)), C.c_int64(int(slip)), _ptr(uw))
    return uw


class Sim:
    """Oracle state of one case, advanced one SISPH step at a time."""

    def __init__(self, case, forced_iters: Optional[int] = None, parallel: bool = False):
        if case.solver == "bicgstab" and not case.free_surface:
            raise ValueError("BiCGStab needs free-surface rows: without them the PPE fixes p only up to a constant")
        self.case = case
        self.parallel = parallel
        self.x = case.x.copy()
        self.u = case.u.copy()
        self.ut = case.u.copy()          # transport velocity starts equal to u
        self.p = case.p.copy()
        self.m = case.m.copy()
        self.wall_u = None if case.wall_u is None else np.ascontiguousarray(case.wall_u)
        self.nrm = wall_normals(case) if case.n_wall else np.zeros((0, case.dim))
        self.p_ref = C.c_double(case.p_ref)
        self.p_ref_set = C.c_int64(1 if case.p_ref_mode == "fixed" else 0)
        self.forced_iters = case.forced_iters if forced_iters is None else forced_iters
        self.dt = float(case.dt)         # the next step's dt
        self.t = 0.0
        self.steps = 0

    def step(self, capture: bool = False, forced_iters: Optional[int] = None) -> dict:
        c = self.case
        nf, nw, dim = c.n_fluid, c.n_wall, c.dim
        fi = self.forced_iters if forced_iters is None else forced_iters
        P = params(c, forced_iters=fi, dt=self.dt)
        out = StepOut()
        keep = {}
        if capture:
            shapes = dict(rho=(nf,), xs=(nf, dim), us=(nf, dim), uw=(nw, dim), usw=(nw, dim),
                          rhs=(nf,), diag=(nf,), unew=(nf, dim), fgtvf0=(nf, dim))
            for k, s in shapes.items():
                keep[k] = np.zeros(s)
                setattr(out, k, _ptr(keep[k]))
            keep["fs"] = np.zeros(nf, dtype=np.int64)
            out.fs = _ptr(keep["fs"])
        x0 = self.x.copy()
        rc = lib(self.parallel).orc_step(C.byref(P), _ptr(self.x), _ptr(self.u), _ptr(self.ut), _ptr(self.p),
                       _ptr(self.m), _ptr(np.ascontiguousarray(self.nrm)), _ptr(self.wall_u),
                       C.byref(self.p_ref), C.byref(self.p_ref_set), C.byref(out))
        if rc != 0:
            raise ValueError("null_space='project' needs a case without walls or free surface")
        self.t += self.dt
        self.steps += 1
        keep.update(iters=int(out.iters), converged=bool(out.converged), ratio=float(out.ratio),
                    lam=float(out.lambda_), p_ref=float(out.p_ref_used), beta=float(out.beta), dt=self.dt,
                    umax=float(out.umax), fmax=float(out.fmax), dt_next=float(out.dt_next))
        self.dt = float(out.dt_next)
        if capture:
            keep["x0"] = x0
        return keep

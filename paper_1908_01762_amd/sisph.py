"""Thin Python binding of libsisph (the C ABI of include/sisph.h).

Argument marshalling only: every step of the SISPH path runs in the HIP
kernels of libsisph.so.  PyTorch provides the device workspace (a uint8
tensor the caller owns) and the stream.  If the library is missing this
module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional

import numpy as np

from . import cases as _cases

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsisph.so")

SWEEP_VARIANTS = 8
STATIC_WORKSPACE_BYTES = 64 << 20
OK, WARN_MAXITER = 0, 1
E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_NONFINITE = -1, -2, -3, -4, -5

FIELDS = {"rho": 0, "xstar": 1, "ustar": 2, "rhs": 3, "dii": 4, "unew": 5, "wall_u": 6,
          "wall_ustar": 7, "fs": 8, "normal": 9, "pressure": 10}
_VECTOR = {"xstar", "ustar", "unew", "wall_u", "wall_ustar", "normal"}
_WALL = {"wall_u", "wall_ustar", "normal"}


class SisphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sisph status {code}: {msg}")
        self.code = code


class CaseDesc(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "dim", "kernel", "precision", "pgrad", "gtvf", "free_surface",
        "p_ref_mode", "conv_norm", "min_iter", "max_iter", "gtvf_K", "forced_iters")] + \
        [("periodic", C.c_int32 * 3), ("nbr_cap", C.c_int32), ("ustar_wall", C.c_int32), ("dt_mode", C.c_int32),
         ("solver", C.c_int32), ("null_space", C.c_int32),
         ("n_fluid", C.c_int64), ("n_wall", C.c_int64)] + \
        [(n, C.c_double) for n in (
            "h", "dx", "rho0", "nu", "alpha", "c_ref", "dt", "eta", "fs_ratio",
            "omega", "tol", "p_ref")] + \
        [("gravity", C.c_double * 3), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3)]


class PPEStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("nonfinite", C.c_int32),
                ("status", C.c_int32), ("ratio", C.c_double), ("lambda_", C.c_double),
                ("p_ref", C.c_double), ("dt", C.c_double), ("index_bits", C.c_int32),
                ("list_blocks", C.c_int32), ("beta", C.c_double)]

    def as_dict(self) -> dict:
        return dict(iters=self.iters, converged=bool(self.converged), nonfinite=bool(self.nonfinite),
                    case_status=self.status,
                    ratio=self.ratio, lam=self.lambda_, p_ref=self.p_ref, dt=self.dt,
                    index_bits=self.index_bits, list_blocks=self.list_blocks, beta=self.beta)


_lib = None
_DP = C.POINTER(C.c_double)


def lib():
    """Loads libsisph.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1908_01762_amd/build.py")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded (device memory and streams come from torch), not to a second
        # copy of it in the same process
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        L.sisph_workspace_bytes.restype = C.c_size_t
        L.sisph_workspace_bytes.argtypes = [C.POINTER(CaseDesc)]
        L.sisph_create_static.restype = C.c_int32
        L.sisph_create_static.argtypes = [C.POINTER(CaseDesc), _DP, _DP, _DP, _DP, _DP, C.c_void_p,
                                          C.POINTER(C.c_void_p)]
        L.sisph_create.restype = C.c_int32
        L.sisph_create.argtypes = [C.POINTER(CaseDesc), C.c_void_p, C.c_size_t, _DP, _DP, _DP, _DP, _DP,
                                   C.c_void_p, C.POINTER(C.c_void_p)]
        for f in ("sisph_bin", "sisph_predict", "sisph_correct", "sisph_destroy"):
            getattr(L, f).restype = C.c_int32
            getattr(L, f).argtypes = [C.c_void_p]
        L.sisph_ppe_solve.restype = C.c_int32
        L.sisph_ppe_solve.argtypes = [C.c_void_p, C.POINTER(PPEStats)]
        L.sisph_step.restype = C.c_int32
        L.sisph_step.argtypes = [C.c_void_p, C.c_int32, C.POINTER(PPEStats)]
        L.sisph_read_state.restype = C.c_int32
        L.sisph_read_state.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP, _DP]
        L.sisph_write_state.restype = C.c_int32
        L.sisph_write_state.argtypes = [C.c_void_p, _DP, _DP, _DP, _DP]
        L.sisph_read_field.restype = C.c_int32
        L.sisph_read_field.argtypes = [C.c_void_p, C.c_int32, _DP]
        L.sisph_set_graphs.restype = C.c_int32
        L.sisph_set_graphs.argtypes = [C.c_void_p, C.c_int32]
        L.sisph_set_persistent.restype = C.c_int32
        L.sisph_set_persistent.argtypes = [C.c_void_p, C.c_int32]
        L.sisph_debug_barrier_spins.restype = C.c_int32
        L.sisph_debug_barrier_spins.argtypes = [C.c_void_p, C.c_uint32]
        L.sisph_debug_packed.restype = C.c_int32
        L.sisph_debug_packed.argtypes = [C.c_void_p, C.c_int32]
        L.sisph_debug_gtvf_short.restype = C.c_int32
        L.sisph_debug_gtvf_short.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
        L.sisph_debug_read_rate.restype = C.c_int32
        L.sisph_debug_read_rate.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_int32,
                                            C.POINTER(C.c_double)]
        L.sisph_persistent_info.restype = C.c_int32
        L.sisph_persistent_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.sisph_set_kernel_timing.restype = C.c_int32
        L.sisph_set_kernel_timing.argtypes = [C.c_void_p, C.c_int32]
        L.sisph_kernel_timing.restype = C.c_int32
        L.sisph_kernel_timing.argtypes = [C.c_void_p, _DP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.sisph_persistent_fallbacks.restype = C.c_int32
        L.sisph_persistent_fallbacks.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.sisph_batch_set_graphs.restype = C.c_int32
        L.sisph_batch_set_graphs.argtypes = [C.c_void_p, C.c_int32]
        L.sisph_pair_count.restype = C.c_int32
        L.sisph_pair_count.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
        L.sisph_rows_with_neighbours.restype = C.c_int32
        L.sisph_rows_with_neighbours.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
        L.sisph_debug_neighbors.restype = C.c_int32
        L.sisph_debug_neighbors.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                            C.POINTER(C.c_int32), C.c_int64]
        L.sisph_last_timings.restype = C.c_int32
        L.sisph_last_timings.argtypes = [C.c_void_p, _DP, _DP]
        L.sisph_sweep_counters.restype = C.c_int32
        L.sisph_sweep_counters.argtypes = [C.c_void_p, _DP, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int32]
        L.sisph_autotune.restype = C.c_int32
        L.sisph_autotune.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), _DP]
        L.sisph_set_variant.restype = C.c_int32
        L.sisph_set_variant.argtypes = [C.c_void_p, C.c_int32]
        L.sisph_get_variant.restype = C.c_int32
        L.sisph_get_variant.argtypes = [C.c_void_p]
        L.sisph_batch_create.restype = C.c_int32
        L.sisph_batch_create.argtypes = [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
        for f in ("sisph_batch_attach", "sisph_batch_detach"):
            getattr(L, f).restype = C.c_int32
            getattr(L, f).argtypes = [C.c_void_p, C.c_void_p]
        L.sisph_batch_size.restype = C.c_int32
        L.sisph_batch_size.argtypes = [C.c_void_p]
        L.sisph_batch_step.restype = C.c_int32
        L.sisph_batch_step.argtypes = [C.c_void_p, C.POINTER(PPEStats)]
        L.sisph_batch_set_persistent.restype = C.c_int32
        L.sisph_batch_set_persistent.argtypes = [C.c_void_p, C.c_int32]
        L.sisph_batch_persistent_info.restype = C.c_int32
        L.sisph_batch_persistent_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.sisph_batch_destroy.restype = C.c_int32
        L.sisph_batch_destroy.argtypes = [C.c_void_p]
        L.sisph_status_string.restype = C.c_char_p
        L.sisph_status_string.argtypes = [C.c_int32]
        L.sisph_last_error.restype = C.c_char_p
        L.sisph_last_error.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_DP)


def describe(case: "_cases.Case") -> CaseDesc:
    """sisph_case_desc of a seeded case."""
    d = CaseDesc()
    d.dim = case.dim
    d.kernel = _cases.KERNELS[case.kernel]
    d.precision = _cases.PRECISION[case.precision]
    d.pgrad = _cases.PGRAD[case.pgrad]
    d.gtvf = _cases.GTVF[case.gtvf]
    d.free_surface = int(bool(case.free_surface))
    d.p_ref_mode = _cases.PREF[case.p_ref_mode]
    d.conv_norm = _cases.CONV[case.conv_norm]
    d.min_iter = case.min_iter
    d.max_iter = case.max_iter
    d.gtvf_K = case.gtvf_K
    d.forced_iters = case.forced_iters
    for k in range(3):
        d.periodic[k] = int(case.periodic[k])
        d.gravity[k] = case.gravity[k]
        d.box_lo[k] = case.box_lo[k]
        d.box_hi[k] = case.box_hi[k]
    d.nbr_cap = int(case.meta.get("nbr_cap", 0))
    d.ustar_wall = _cases.USTAR[case.ustar_wall]
    d.dt_mode = _cases.DT_MODE[case.dt_mode]
    d.solver = _cases.SOLVER[case.solver]
    d.null_space = _cases.NULL_SPACE[case.null_space]
    d.n_fluid = case.n_fluid
    d.n_wall = case.n_wall
    for k in ("h", "dx", "rho0", "nu", "alpha", "c_ref", "dt", "eta", "fs_ratio", "omega", "tol", "p_ref"):
        setattr(d, k, float(getattr(case, k)))
    return d


def workspace_bytes(case) -> int:
    return int(lib().sisph_workspace_bytes(C.byref(describe(case))))


def read_rate(buf_ptr: int, nbytes: int, out_ptr: int, grid: int, reps: int) -> float:
    """Microseconds per plain read of nbytes of a device buffer
    (sisph_debug_read_rate); out holds grid * 256 floats."""
    us = C.c_double()
    _check(lib().sisph_debug_read_rate(C.c_void_p(buf_ptr), int(nbytes), C.c_void_p(out_ptr), int(grid),
                                       int(reps), C.byref(us)))
    return us.value


def status_string(code: int) -> str:
    return lib().sisph_status_string(code).decode()


def _check(code: int, ctx=None, allow_warn: bool = True) -> int:
    if code < 0 or (code > 0 and not allow_warn):
        msg = lib().sisph_last_error(ctx).decode()
        raise SisphError(code, f"{status_string(code)} ({msg})")
    return code


class Context:
    """One SISPH case resident on the GPU."""

    def __init__(self, case, device: str = "cuda", stream=None, static: bool = False):
        """static=True: the case lives in the library's static device
        workspace (sisph_create_static, one context per device, nothing
        allocated); otherwise in a torch uint8 tensor this object owns."""
        import torch
        self.case = case
        self.desc = describe(case)
        L = lib()
        nbytes = int(L.sisph_workspace_bytes(C.byref(self.desc)))
        if nbytes == 0:
            raise SisphError(E_INVAL, "invalid case descriptor")
        dev = torch.device(device)
        h = C.c_void_p()
        x = np.ascontiguousarray(case.x, dtype=np.float64)
        u = np.ascontiguousarray(case.u, dtype=np.float64)
        p = np.ascontiguousarray(case.p, dtype=np.float64)
        m = np.ascontiguousarray(case.m, dtype=np.float64)
        wu = None if case.wall_u is None or case.n_wall == 0 else np.ascontiguousarray(case.wall_u, dtype=np.float64)
        if static:
            if dev.index is not None:   # the static workspace is the current device's
                torch.cuda.set_device(dev)
            self.workspace = None
            self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
            code = L.sisph_create_static(C.byref(self.desc), _p(x), _p(u), _p(p), _p(m), _p(wu),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h))
        else:
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
            code = L.sisph_create(C.byref(self.desc), C.c_void_p(aligned), C.c_size_t(nbytes), _p(x), _p(u),
                                  _p(p), _p(m), _p(wu), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        _check(code, None)
        self.h = h
        self.nbytes = nbytes

    # -- stages -----------------------------------------------------------
    def bin(self):
        _check(lib().sisph_bin(self.h), self.h)

    def predict(self):
        _check(lib().sisph_predict(self.h), self.h)

    def ppe_solve(self) -> dict:
        st = PPEStats()
        code = _check(lib().sisph_ppe_solve(self.h, C.byref(st)), self.h)
        d = st.as_dict()
        d["status"] = code
        return d

    def correct(self):
        _check(lib().sisph_correct(self.h), self.h)

    def step(self, nsteps: int = 1) -> List[dict]:
        st = (PPEStats * max(nsteps, 1))()
        code = _check(lib().sisph_step(self.h, nsteps, st), self.h)
        out = [st[k].as_dict() for k in range(nsteps)]
        for o in out:
            o["status"] = code
        return out

    # -- state ------------------------------------------------------------
    def read_state(self) -> Dict[str, np.ndarray]:
        c = self.case
        x = np.zeros((c.n, c.dim))
        u = np.zeros((c.n_fluid, c.dim))
        ut = np.zeros((c.n_fluid, c.dim))
        p = np.zeros(c.n)
        rho = np.zeros(c.n_fluid)
        _check(lib().sisph_read_state(self.h, _p(x), _p(u), _p(ut), _p(p), _p(rho)), self.h)
        return dict(x=x, u=u, ut=ut, p=p, rho=rho)

    def write_state(self, x=None, u=None, ut=None, p=None):
        conv = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        x, u, ut, p = conv(x), conv(u), conv(ut), conv(p)
        _check(lib().sisph_write_state(self.h, _p(x), _p(u), _p(ut), _p(p)), self.h)

    def field(self, name: str) -> np.ndarray:
        c = self.case
        rows = c.n_wall if name in _WALL else (c.n if name == "pressure" else c.n_fluid)
        shape = (rows, c.dim) if name in _VECTOR else (rows,)
        out = np.zeros(shape)
        _check(lib().sisph_read_field(self.h, FIELDS[name], _p(out)), self.h)
        return out

    def neighbors(self, stage: int, dest: int = 0):
        c = self.case
        rows = c.n_fluid if dest == 0 else c.n_wall
        off = np.zeros(rows + 1, dtype=np.int64)
        offp = off.ctypes.data_as(C.POINTER(C.c_int64))
        # first pass sizes the id buffer (offsets are complete even when the
        # ids do not fit), second pass fills it
        code = lib().sisph_debug_neighbors(self.h, stage, dest, offp, None, 0)
        if code != E_NOMEM or off[-1] == 0:
            _check(code, self.h)
        ids = np.zeros(max(int(off[-1]), 1), dtype=np.int32)
        _check(lib().sisph_debug_neighbors(self.h, stage, dest, offp, ids.ctypes.data_as(C.POINTER(C.c_int32)),
                                            ids.size), self.h)
        return off, ids[:off[-1]].copy()

    def use_graphs(self, on: bool = True):
        """Replay the fixed parts of each step from HIP graphs (sisph_step)."""
        _check(lib().sisph_set_graphs(self.h, int(bool(on))), self.h)

    def use_persistent(self, on: bool = True):
        """One cooperative launch per Jacobi solve where it applies (default)."""
        _check(lib().sisph_set_persistent(self.h, int(bool(on))), self.h)

    def pair_count(self, stage: int, dest: int = 0) -> int:
        """Stored neighbour pairs (self included) of the held lists."""
        n = C.c_int64()
        _check(lib().sisph_pair_count(self.h, stage, dest, C.byref(n)), self.h)
        return n.value

    def rows_with_neighbours(self, stage: int, dest: int = 0) -> int:
        """Rows of the held lists with a particle other than the row itself."""
        n = C.c_int64()
        _check(lib().sisph_rows_with_neighbours(self.h, stage, dest, C.byref(n)), self.h)
        return n.value

    def timings(self):
        a, b = C.c_double(), C.c_double()
        _check(lib().sisph_last_timings(self.h, C.byref(a), C.byref(b)), self.h)
        return a.value, b.value

    def autotune(self, reps: int = 20):
        """Times the sweep variants on the current state (needs one completed
        step); selects the fastest.  Returns (best, [us per variant])."""
        best = C.c_int32()
        us = (C.c_double * SWEEP_VARIANTS)()
        _check(lib().sisph_autotune(self.h, int(reps), C.byref(best), us), self.h)
        return best.value, list(us)

    @property
    def variant(self) -> int:
        return int(lib().sisph_get_variant(self.h))

    @variant.setter
    def variant(self, v: int):
        _check(lib().sisph_set_variant(self.h, int(v)), self.h)

    def sweep_counters(self, reset: bool = False):
        ms, n, e = C.c_double(), C.c_int64(), C.c_int64()
        _check(lib().sisph_sweep_counters(self.h, C.byref(ms), C.byref(n), C.byref(e), int(reset)), self.h)
        return dict(sweep_ms=ms.value, launches=n.value, effective=e.value)

    def set_kernel_timing(self, period: int = 1):
        """Bracket every period-th sweep launch of each solve with its own
        HIP events (wall pass left out); period 0 (or False) turns it off,
        True or 1 times every launch."""
        _check(lib().sisph_set_kernel_timing(self.h, int(period)), self.h)

    def kernel_timing(self):
        """Sweep-kernel time (ms), timed launches and persistent ones among
        them, since the last sweep_counters reset."""
        ms, n, p = C.c_double(), C.c_int64(), C.c_int64()
        _check(lib().sisph_kernel_timing(self.h, C.byref(ms), C.byref(n), C.byref(p)), self.h)
        return dict(ms=ms.value, launches=n.value, persistent=p.value)

    def debug_packed(self, on: bool):
        """Test hook: sweeps through the lists (False) or the packed mode's
        LDS copy and codes (True, the default where the case has it)."""
        _check(lib().sisph_debug_packed(self.h, int(bool(on))), self.h)

    def debug_gtvf_short(self, on: Optional[bool] = None) -> int:
        """Turns the GTVF short lists off (False) or back on (True), or
        leaves them (None); returns how the last step's sub-steps used them
        (0 none, 1 all sub-steps, 2 not all)."""
        used = C.c_int32()
        _check(lib().sisph_debug_gtvf_short(self.h, -1 if on is None else int(bool(on)), C.byref(used)), self.h)
        return used.value

    def debug_barrier_spins(self, spins: int):
        """Test hook: polls before a persistent-solve wait gives up."""
        _check(lib().sisph_debug_barrier_spins(self.h, int(spins)), self.h)

    def persistent_info(self):
        """Persistent solves since the counter reset, and whether the last
        solve was one."""
        n, last = C.c_int64(), C.c_int32()
        _check(lib().sisph_persistent_info(self.h, C.byref(n), C.byref(last)), self.h)
        return dict(solves=n.value, last=bool(last.value))

    def persistent_fallbacks(self):
        """Solves meant for one persistent launch that ran per-launch sweeps
        instead (cooperative launch refused, or a grid barrier timed out),
        since the last sweep_counters reset."""
        r, t = C.c_int64(), C.c_int64()
        _check(lib().sisph_persistent_fallbacks(self.h, C.byref(r), C.byref(t)), self.h)
        return dict(refused=r.value, timed_out=t.value)

    def close(self):
        if getattr(self, "h", None):
            lib().sisph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent cases stepped together: one launch per kernel for all
    attached cases (per (dim, kernel, precision) group), each case keeping
    its own PPE convergence."""

    def __init__(self, max_cases: int = 64, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        code = lib().sisph_batch_create(int(max_cases), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if code != OK:
            raise SisphError(code, status_string(code))
        self.h = h
        self.members: List[Context] = []

    def use_graphs(self, on: bool = True):
        """Replay the fixed parts of each batched step from HIP graphs."""
        code = lib().sisph_batch_set_graphs(self.h, int(bool(on)))
        if code != OK:
            raise SisphError(code, status_string(code))

    def use_persistent(self, on: bool = True):
        """Wall-less cases' Jacobi solves in one cooperative launch (default on)."""
        _check(lib().sisph_batch_set_persistent(self.h, int(bool(on))))

    def persistent_info(self):
        """Persistent batched launches and fallbacks since creation."""
        n, f = C.c_int64(), C.c_int64()
        _check(lib().sisph_batch_persistent_info(self.h, C.byref(n), C.byref(f)))
        return dict(launches=n.value, fallbacks=f.value)

    def attach(self, ctx: Context):
        _check(lib().sisph_batch_attach(self.h, ctx.h), ctx.h)
        self.members.append(ctx)

    def detach(self, ctx: Context):
        _check(lib().sisph_batch_detach(self.h, ctx.h), ctx.h)
        self.members.remove(ctx)

    def step(self, raise_on_error: bool = True) -> List[dict]:
        """One step of every attached case, stats in attach order.  Each
        entry's case_status is that case's own status code."""
        n = len(self.members)
        st = (PPEStats * max(n, 1))()
        code = lib().sisph_batch_step(self.h, st)
        out = [st[k].as_dict() for k in range(n)]
        if code < 0 and raise_on_error:
            bad = [m for m, o in zip(self.members, out) if o["case_status"] < 0]
            msg = "; ".join(lib().sisph_last_error(m.h).decode() for m in bad) or status_string(code)
            raise SisphError(code, f"{status_string(code)} ({msg})")
        for o in out:
            o["status"] = code
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().sisph_batch_destroy(self.h)
            self.h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

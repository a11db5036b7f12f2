"""ctypes binding of ``libsaamg.so`` (include/saamg.h).

Argument marshalling only: every numerical step runs in the library's HIP kernels.
Device vectors are torch tensors (float64, contiguous, on the hierarchy's device) whose
``data_ptr()`` is handed to the library; streams default to torch's current stream.
The binding raises if the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsaamg.so")

OK, INVALID_ARG, NOMEM, HIP_ERROR, NOT_CONVERGED, BREAKDOWN, NONFINITE = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "NOMEM", 3: "HIP_ERROR", 4: "NOT_CONVERGED",
                5: "BREAKDOWN", 6: "NONFINITE"}
VARIANT_CONST, VARIANT_LIN, VARIANT_QUAD = 0, 1, 2
FP64, MIXED = 0, 1
COARSE_DIRECT, COARSE_GS = 0, 1
SHAPE_CYLINDER, SHAPE_ELLIPSE, SHAPE_BOXBORE = 0, 1, 2
OP_APPLY, OP_APPLY_T, OP_PRESMOOTH, OP_RESTRICT, OP_PROLONG = range(5)
MAX_LEVELS = 16


class Domain(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("mask", C.POINTER(C.c_uint8)), ("n_wall", C.c_int64),
                ("wall_node", C.POINTER(C.c_int64)), ("wall_dir", C.POINTER(C.c_uint8)),
                ("wall_s", C.POINTER(C.c_double)), ("robin_d", C.c_double)]


# saamg_options' allocator callbacks: alloc(ctx, bytes, stream) -> ptr, free(ctx, ptr, stream)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_levels", C.c_int32), ("max_coarse", C.c_int32),
                ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double),
                ("cheb_boost", C.c_double), ("eig_iters", C.c_int32),
                ("omega_scale", C.c_double), ("coarse_solver", C.c_int32),
                ("coarse_sweeps", C.c_int32), ("l0_planes", C.c_int32),
                ("l0_tile_x", C.c_int32), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", C.c_void_p), ("l0_wide", C.c_int32), ("cg_ring", C.c_int32)]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("z_offset", C.c_int32),
                ("origin", C.c_double * 3), ("h", C.c_double * 3), ("robin_d", C.c_double)]


class Result(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32), ("replacements", C.c_int32),
                ("rel_res_true", C.c_double), ("rel_res_recursive", C.c_double),
                ("t_solve_ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("variant", C.c_int32), ("precision", C.c_int32),
                ("dims", (C.c_int32 * 3) * MAX_LEVELS),
                ("n_unknowns", C.c_int64 * MAX_LEVELS),
                ("lambda_est", C.c_double * MAX_LEVELS), ("omega", C.c_double * MAX_LEVELS),
                ("n_irregular", C.c_int64), ("device_bytes", C.c_int64),
                ("t_setup_ms", C.c_double), ("t_refresh_ms", C.c_double),
                ("l0_planes", C.c_int32), ("l0_tile_x", C.c_int32),
                ("table_rows", C.c_int64 * MAX_LEVELS), ("table_rows_t", C.c_int64 * MAX_LEVELS),
                ("t_setup_phase_ms", C.c_double * 6), ("l0_wide", C.c_int32),
                ("l0_wide_planes", C.c_int32 * 2)]


class SaamgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = C.c_void_p
_DP = C.POINTER(C.c_double)


def lib() -> C.CDLL:
    """Load the library once; raise if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (paper_0907_4863_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    L.saamg_last_error.restype = C.c_char_p
    L.saamg_default_options.argtypes = [C.POINTER(Options)]
    L.saamg_domain_from_shape.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                          C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                          C.POINTER(C.c_uint8), C.c_int64, C.POINTER(C.c_int64),
                                          C.POINTER(C.c_uint8), _DP, C.POINTER(C.c_int64), _DP]
    L.saamg_setup.argtypes = [C.POINTER(Domain), C.c_int, C.POINTER(Options), _P, C.POINTER(_P)]
    L.saamg_refresh.argtypes = [_P, C.POINTER(Domain), _P]
    L.saamg_set_operator.argtypes = [_P, C.POINTER(Domain), _P]
    L.saamg_solve.argtypes = [_P, _P, _P, _P, C.c_double, C.c_int, _P, C.POINTER(Result)]
    L.saamg_solve_noalloc.argtypes = [_P, _P, _P, _P, C.c_double, C.c_int, _P,
                                      C.POINTER(Result)]
    L.saamg_pic_create.argtypes = [C.POINTER(Grid), C.POINTER(C.c_uint8), C.c_int64, C.POINTER(_P)]
    L.saamg_pic_deposit.argtypes = [_P, _P, C.c_int64, C.c_double, _P, _P]
    L.saamg_pic_gather.argtypes = [_P, _P, _P, C.c_int64, _P, _P]
    L.saamg_pic_destroy.argtypes = [_P]
    L.saamg_destroy.argtypes = [_P]
    L.saamg_hierarchy_info.argtypes = [_P, C.POINTER(Info)]
    L.saamg_footprint_bytes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.saamg_state_create.argtypes = [_P, _P, _P, C.c_double, C.c_int, _P, C.POINTER(_P)]
    L.saamg_batch_step.argtypes = [C.POINTER(_P), C.c_int, C.POINTER(C.c_int)]
    L.saamg_batch_advance.argtypes = [C.POINTER(_P), C.c_int, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
    L.saamg_state_query.argtypes = [_P, C.POINTER(C.c_int), C.POINTER(Result)]
    L.saamg_state_finish.argtypes = [_P, _P]
    L.saamg_state_destroy.argtypes = [_P]
    L.saamg_level_apply.argtypes = [_P, C.c_int, C.c_int, C.c_int, _DP, _DP]
    L.saamg_level_coefficients.argtypes = [_P, C.c_int, _DP]
    L.saamg_precond_apply.argtypes = [_P, _P, _P, _P]
    L.saamg_operator_apply.argtypes = [_P, _P, _P, _P]
    L.saamg_scaling.argtypes = [_P, _P, _P]
    L.saamg_coarse_inverse.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int64), _DP]
    L.saamg_timer_enable.argtypes = [C.c_int, C.c_int]
    L.saamg_timer_read.argtypes = [C.c_int, _DP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    _lib = L
    return L


def _check(rc: int, allow: Sequence[int] = (OK,)) -> int:
    if rc not in allow:
        raise SaamgError(rc, lib().saamg_last_error().decode())
    return rc


def last_error() -> str:
    return lib().saamg_last_error().decode()


class TorchAllocator:
    """saamg_options allocator callbacks backed by torch's caching allocator, so that the
    library's device memory comes from (and returns to) torch's pool: no hipMalloc per
    buffer, and frees are stream-ordered instead of device-synchronising.  Counts the
    calls (tests read them)."""

    def __init__(self):
        self.n_alloc = 0
        self.n_free = 0
        self.outstanding = {}  # ptr -> bytes
        self._lock = threading.Lock()
        self._torch = None
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, ctx, nbytes, stream):
        try:
            if self._torch is None:
                import torch
                self._torch = torch
            cuda = self._torch.cuda
            p = cuda.caching_allocator_alloc(int(nbytes), cuda.current_device(), int(stream or 0))
        except Exception:
            return None  # reported by the library as SAAMG_NOMEM
        with self._lock:
            self.n_alloc += 1
            self.outstanding[p] = int(nbytes)
        return p

    def _free(self, ctx, ptr, stream):
        with self._lock:
            self.n_free += 1
            self.outstanding.pop(ptr, None)
        try:
            self._torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass  # interpreter shutdown: the process's memory goes with it

    @property
    def outstanding_bytes(self) -> int:
        with self._lock:
            return sum(self.outstanding.values())


_torch_allocator: Optional[TorchAllocator] = None


def torch_allocator() -> TorchAllocator:
    """The process-wide TorchAllocator (its callbacks must outlive every hierarchy)."""
    global _torch_allocator
    if _torch_allocator is None:
        _torch_allocator = TorchAllocator()
    return _torch_allocator


def default_options(allocator=None, **kw) -> Options:
    """Library defaults (Table 1 and the documented readings) with ``kw`` applied.
    ``allocator``: None (the library's own stream-safe device pool, the default), "torch"
    (torch's caching allocator through Python callbacks) or a TorchAllocator-like object
    with alloc_fn / free_fn.  The pool is the default because the callbacks take the GIL
    on every allocation: with hierarchies built on worker threads beside a polling loop,
    served throughput fell from 54 to 12-19 solves/s with them."""
    o = Options()
    lib().saamg_default_options(C.byref(o))
    if allocator == "torch":
        allocator = torch_allocator()
    if allocator is not None:
        o.alloc = allocator.alloc_fn
        o.free = allocator.free_fn
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# --------------------------------------------------------------------------- domain


class HostDomain:
    """Host arrays describing a discrete domain (the argument of setup)."""

    def __init__(self, mask: np.ndarray, h: Tuple[float, float, float], wall_node: np.ndarray,
                 wall_dir: np.ndarray, wall_s: np.ndarray, robin_d: float = 0.0):
        self.robin_d = float(robin_d)
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.nz, self.ny, self.nx = self.mask.shape
        self.h = tuple(float(v) for v in h)
        self.wall_node = np.ascontiguousarray(wall_node, dtype=np.int64)
        self.wall_dir = np.ascontiguousarray(wall_dir, dtype=np.uint8)
        self.wall_s = np.ascontiguousarray(wall_s, dtype=np.float64)

    def struct(self) -> Domain:
        d = Domain()
        d.nx, d.ny, d.nz = self.nx, self.ny, self.nz
        d.hx, d.hy, d.hz = self.h
        d.mask = self.mask.ctypes.data_as(C.POINTER(C.c_uint8))
        d.n_wall = self.wall_node.size
        d.wall_node = self.wall_node.ctypes.data_as(C.POINTER(C.c_int64))
        d.wall_dir = self.wall_dir.ctypes.data_as(C.POINTER(C.c_uint8))
        d.wall_s = self.wall_s.ctypes.data_as(_DP)
        d.robin_d = self.robin_d
        return d

    @property
    def n_unknowns(self) -> int:
        return int(self.mask.sum())


def domain_from_shape(kind: int, a: float, b: float, length: float, nx: int, ny: int, nz: int,
                      bore_r: float = 0.0, cavity_half_len: float = 0.0,
                      open_ends: bool = False) -> HostDomain:
    """Domain of an analytic pipe; with ``open_ends`` the end planes hold unknowns (Robin,
    d = length / 2) and the box has nz + 2 planes."""
    L = lib()
    nzb = nz + 2 * int(open_ends)
    mask = np.empty((nzb, ny, nx), dtype=np.uint8)
    n = C.c_int64(0)
    mp = mask.ctypes.data_as(C.POINTER(C.c_uint8))
    oe = int(bool(open_ends))
    # one call with room for the wall entries of a surface-sized set of nodes (the entries
    # are written in node order up to the capacity); a second call only if they do not fit
    cap = max(8 * (nx * ny + nx * nzb + ny * nzb), 1)
    while True:
        node = np.empty(cap, dtype=np.int64)
        dr = np.empty(cap, dtype=np.uint8)
        s = np.empty(cap, dtype=np.float64)
        hd = (C.c_double * 4)()
        rc = L.saamg_domain_from_shape(kind, a, b, length, bore_r, cavity_half_len, nx, ny, nz,
                                       oe, mp, cap, node.ctypes.data_as(C.POINTER(C.c_int64)),
                                       dr.ctypes.data_as(C.POINTER(C.c_uint8)),
                                       s.ctypes.data_as(_DP), C.byref(n), hd)
        if rc != OK and n.value > cap:
            cap = n.value
            continue
        _check(rc)
        break
    cnt = n.value
    return HostDomain(mask, (hd[0], hd[1], hd[2]), node[:cnt].copy(), dr[:cnt].copy(),
                      s[:cnt].copy(), hd[3])


def domain_for(shape, nx: int, ny: int, nz: int, open_ends: bool = False) -> HostDomain:
    """Domain of a ``workloads.Shape`` (nx, ny, nz: lattice nodes)."""
    return domain_from_shape(shape.kind, shape.a, shape.b, shape.length, nx, ny, nz,
                             shape.bore_r, shape.cavity_half_len, open_ends)


# --------------------------------------------------------------------------- device glue


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    if not torch.cuda.is_available():
        return None  # host-only calls (argument validation) on a machine without a GPU
    return torch.cuda.current_stream().cuda_stream


def _dptr(t, n: Optional[int] = None) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return t.data_ptr()


class Hierarchy:
    """Owner of a saamg_hierarchy handle."""

    def __init__(self, handle: int, dims: Tuple[int, int, int]):
        self.handle = handle
        self.dims = dims  # (nx, ny, nz)

    @property
    def nbox(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    def __del__(self):
        try:
            destroy(self)
        except Exception:
            pass


def setup(dom: HostDomain, variant: int, options: Optional[Options] = None,
          stream=None) -> Hierarchy:
    """saamg_setup; without ``options`` the library defaults."""
    h = _P()
    ds = dom.struct()
    if options is None:
        options = default_options()
    _check(lib().saamg_setup(C.byref(ds), variant, C.byref(options), _stream(stream),
                             C.byref(h)))
    return Hierarchy(h.value, (dom.nx, dom.ny, dom.nz))


def refresh(H: Hierarchy, dom: HostDomain, stream=None) -> None:
    """Recompute every number of H for ``dom`` on H's aggregates (saamg_refresh)."""
    ds = dom.struct()
    _check(lib().saamg_refresh(H.handle, C.byref(ds), _stream(stream)))


def set_operator(H: Hierarchy, dom: HostDomain, stream=None) -> None:
    """Iterate with the operator of ``dom`` and keep H's preconditioner (saamg_set_operator)."""
    ds = dom.struct()
    _check(lib().saamg_set_operator(H.handle, C.byref(ds), _stream(stream)))


def destroy(H: Hierarchy) -> None:
    if H.handle:
        lib().saamg_destroy(H.handle)
        H.handle = 0


def solve(H: Hierarchy, b, x, x0=None, tol: float = 1e-8, max_iter: int = 500,
          stream=None, raise_on_failure: bool = False) -> dict:
    res = Result()
    rc = lib().saamg_solve(H.handle, _dptr(b, H.nbox), None if x0 is None else _dptr(x0, H.nbox),
                           _dptr(x, H.nbox), tol, max_iter, _stream(stream), C.byref(res))
    allowed = (OK,) if raise_on_failure else (OK, NOT_CONVERGED, BREAKDOWN, NONFINITE)
    _check(rc, allowed)
    return res.as_dict()


def solve_noalloc(H: Hierarchy, b, x, x0=None, tol: float = 1e-8, max_iter: int = 500,
                  stream=None, raise_on_failure: bool = False) -> dict:
    """saamg_solve_noalloc: saamg_solve with its work vectors in the library's static
    scratch array (no device allocation during the call)."""
    res = Result()
    rc = lib().saamg_solve_noalloc(H.handle, _dptr(b, H.nbox),
                                   None if x0 is None else _dptr(x0, H.nbox), _dptr(x, H.nbox),
                                   tol, max_iter, _stream(stream), C.byref(res))
    allowed = (OK,) if raise_on_failure else (OK, NOT_CONVERGED, BREAKDOWN, NONFINITE)
    _check(rc, allowed)
    return res.as_dict()


def hierarchy_info(H: Hierarchy) -> dict:
    info = Info()
    _check(lib().saamg_hierarchy_info(H.handle, C.byref(info)))
    n = info.n_levels
    return {
        "n_levels": n, "variant": info.variant, "precision": info.precision,
        "dims": [tuple(info.dims[l]) for l in range(n)],
        "n_unknowns": [info.n_unknowns[l] for l in range(n)],
        "lambda_est": [info.lambda_est[l] for l in range(n)],
        "omega": [info.omega[l] for l in range(n)],
        "n_irregular": info.n_irregular, "device_bytes": info.device_bytes,
        "t_setup_ms": info.t_setup_ms, "t_refresh_ms": info.t_refresh_ms,
        "l0_planes": info.l0_planes, "l0_tile_x": info.l0_tile_x,
        "l0_wide": info.l0_wide, "l0_wide_planes": list(info.l0_wide_planes),
        "table_rows": [info.table_rows[l] for l in range(n)],
        "table_rows_t": [info.table_rows_t[l] for l in range(n)],
        "t_setup_phase_ms": dict(zip(("host_checks", "level0", "spectral", "galerkin",
                                      "coarse_solver", "fp32"), list(info.t_setup_phase_ms))),
    }


def footprint_bytes(nx: int, ny: int, nz: int, variant: int, precision: int) -> Tuple[int, int]:
    a, b = C.c_int64(0), C.c_int64(0)
    _check(lib().saamg_footprint_bytes(nx, ny, nz, variant, precision, C.byref(a), C.byref(b)))
    return a.value, b.value


class State:
    def __init__(self, handle: int, H: Hierarchy):
        self.handle = handle
        self.H = H

    def __del__(self):
        try:
            state_destroy(self)
        except Exception:
            pass


def state_create(H: Hierarchy, b, x0=None, tol: float = 1e-8, max_iter: int = 500,
                 stream=None) -> State:
    h = _P()
    _check(lib().saamg_state_create(H.handle, _dptr(b, H.nbox),
                                    None if x0 is None else _dptr(x0, H.nbox), tol, max_iter,
                                    _stream(stream), C.byref(h)))
    return State(h.value, H)


def batch_step(states: Sequence[State]) -> int:
    arr = (_P * max(len(states), 1))(*[s.handle for s in states])
    nd = C.c_int(0)
    _check(lib().saamg_batch_step(arr, len(states), C.byref(nd)))
    return nd.value


def batch_advance(states: Sequence[State]) -> Tuple[int, int]:
    """saamg_batch_advance: (finished states, states that completed a step); never waits."""
    arr = (_P * max(len(states), 1))(*[s.handle for s in states])
    nd, ns = C.c_int(0), C.c_int(0)
    _check(lib().saamg_batch_advance(arr, len(states), C.byref(nd), C.byref(ns)))
    return nd.value, ns.value


def state_query(S: State) -> Tuple[bool, dict]:
    done = C.c_int(0)
    res = Result()
    _check(lib().saamg_state_query(S.handle, C.byref(done), C.byref(res)))
    return bool(done.value), res.as_dict()


def state_finish(S: State, x) -> None:
    _check(lib().saamg_state_finish(S.handle, _dptr(x, S.H.nbox)))


def state_destroy(S: State) -> None:
    if S.handle:
        lib().saamg_state_destroy(S.handle)
        S.handle = 0


# --------------------------------------------------------------------------- particles


class Pic:
    """Particle-coupling context (saamg_pic) on the grid of a discrete domain."""

    def __init__(self, handle: int, nbox: int):
        self.handle = handle
        self.nbox = nbox

    def __del__(self):
        pic_destroy(self)


def pic_create(dom: HostDomain, origin, max_particles: int, use_mask: bool = True) -> Pic:
    """Context for ``dom``'s box; ``origin`` = coordinates of lattice node (0, 0, 0)."""
    g = Grid()
    g.nx, g.ny, g.nz = dom.nx, dom.ny, dom.nz
    g.z_offset = 1 if dom.robin_d > 0.0 else 0
    for a in range(3):
        g.origin[a] = float(origin[a])
        g.h[a] = dom.h[a]
    g.robin_d = dom.robin_d
    mp = dom.mask.ctypes.data_as(C.POINTER(C.c_uint8)) if use_mask else None
    h = _P()
    _check(lib().saamg_pic_create(C.byref(g), mp, int(max_particles), C.byref(h)))
    return Pic(h.value, dom.nx * dom.ny * dom.nz)


def _pptr(t, n: int) -> int:
    """Device pointer of a contiguous float64 (n, 3) particle array."""
    return _dptr(t, 3 * n)


def pic_deposit(P: Pic, pos, q: float, rho, stream=None) -> None:
    n = pos.shape[0] if pos.dim() == 2 else pos.numel() // 3
    _check(lib().saamg_pic_deposit(P.handle, _pptr(pos, n) if n else None, n, float(q),
                                   _dptr(rho, P.nbox), _stream(stream)))


def pic_gather(P: Pic, phi, pos, E, stream=None) -> None:
    n = pos.shape[0] if pos.dim() == 2 else pos.numel() // 3
    _check(lib().saamg_pic_gather(P.handle, _dptr(phi, P.nbox), _pptr(pos, n) if n else None, n,
                                  _pptr(E, n) if n else None, _stream(stream)))


def pic_destroy(P: Pic) -> None:
    if getattr(P, "handle", 0):
        lib().saamg_pic_destroy(P.handle)
        P.handle = 0


# --------------------------------------------------------------------------- components


def level_apply(H: Hierarchy, level: int, op: int, vec: np.ndarray, out_shape: Tuple[int, ...],
                precision: int = FP64) -> np.ndarray:
    a = np.ascontiguousarray(vec, dtype=np.float64)
    out = np.zeros(out_shape, dtype=np.float64)
    _check(lib().saamg_level_apply(H.handle, level, op, precision, a.ctypes.data_as(_DP),
                                   out.ctypes.data_as(_DP)))
    return out


def level_coefficients(H: Hierarchy, level: int, dims: Tuple[int, int, int]) -> np.ndarray:
    mx, my, mz = dims
    out = np.zeros((27, mz, my, mx), dtype=np.float64)
    _check(lib().saamg_level_coefficients(H.handle, level, out.ctypes.data_as(_DP)))
    return out


def precond_apply(H: Hierarchy, r, z, stream=None) -> None:
    _check(lib().saamg_precond_apply(H.handle, _dptr(r, H.nbox), _dptr(z, H.nbox),
                                     _stream(stream)))


def operator_apply(H: Hierarchy, x, y, stream=None) -> None:
    _check(lib().saamg_operator_apply(H.handle, _dptr(x, H.nbox), _dptr(y, H.nbox),
                                      _stream(stream)))


def scaling(H: Hierarchy, sigma, stream=None) -> None:
    _check(lib().saamg_scaling(H.handle, _dptr(sigma, H.nbox), _stream(stream)))


def coarse_inverse(H: Hierarchy) -> Tuple[np.ndarray, np.ndarray]:
    """(logical indices of the coarsest level's unknowns, their explicit inverse n x n)."""
    n = C.c_int32(0)
    _check(lib().saamg_coarse_inverse(H.handle, C.byref(n), None, None))
    rows = np.zeros(n.value, dtype=np.int64)
    inv = np.zeros((n.value, n.value), dtype=np.float64)
    _check(lib().saamg_coarse_inverse(H.handle, C.byref(n), rows.ctypes.data_as(C.POINTER(C.c_int64)),
                                      inv.ctypes.data_as(_DP)))
    return rows, inv


# --------------------------------------------------------------------------- timing

TIMER_KINDS = {"l0_cheb": 0, "l0_resid": 1, "l0_restrict": 2, "l0_prolong": 3, "cg_pq": 4,
               "cg_xr": 5, "coarse": 6, "finalize": 7, "cg_x": 8}


def timer_enable(kind: str, enable: bool = True) -> None:
    _check(lib().saamg_timer_enable(TIMER_KINDS[kind], int(enable)))


def timer_read(kind: str) -> Tuple[float, int, int]:
    ms, n, u = C.c_double(0), C.c_int64(0), C.c_int64(0)
    _check(lib().saamg_timer_read(TIMER_KINDS[kind], C.byref(ms), C.byref(n), C.byref(u)))
    return ms.value, n.value, u.value


def timer_reset() -> None:
    _check(lib().saamg_timer_reset())

"""ctypes binding of the C ABI in ``include/hdg.h``.

Argument marshalling only: every step of the computation runs in the HIP
library ``libhdg.so`` built next to this file.  PyTorch provides device
memory (CUDA/HIP tensors) and the stream; there is no CPU fallback, and a
missing library raises at first use.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

HDG_OK = 0
STATUS_NAMES = {0: "HDG_OK", -1: "HDG_EINVAL", -2: "HDG_EHIP", -3: "HDG_ENOMEM",
                -4: "HDG_ENOCONV", -5: "HDG_EUNSUPPORTED"}
F64, F32 = 0, 1
NODAL, EIGEN = 0, 1
TO_EIGEN_UNKNOWN, TO_EIGEN_RESIDUAL, TO_NODAL_UNKNOWN, TO_NODAL_RESIDUAL = 0, 1, 2, 3

# every symbol include/hdg.h declares
EXPORTS = (
    "hdg_default_opts", "hdg_create", "hdg_create_ex", "hdg_destroy", "hdg_last_error",
    "hdg_sizes", "hdg_layout", "hdg_set_lambda", "hdg_tables", "hdg_coords", "hdg_set_origin",
    "hdg_apply", "hdg_apply_noalloc",
    "hdg_face_transform",
    "hdg_rhs", "hdg_solve", "hdg_solve_forcing", "hdg_reconstruct", "hdg_hybridize",
    "hdg_adjoint",
    "hdg_diagonal", "hdg_time_kernel", "hdg_set_tile", "hdg_set_cg_segment", "hdg_autotune",
    "hdg_tile_shape",
    "hdg_batch_create", "hdg_batch_destroy", "hdg_batch_sizes", "hdg_batch_set_tile",
    "hdg_batch_tiles", "hdg_batch_set_form", "hdg_batch_form", "hdg_batch_autotune",
    "hdg_batch_time_cg", "hdg_batch_solve_forcing",
)


class HdgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("maxit", ctypes.c_int), ("precond", ctypes.c_int),
                ("mixed", ctypes.c_int), ("inner_rtol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("check_every", ctypes.c_int),
                ("variant", ctypes.c_int), ("guess", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("rel_res", ctypes.c_double), ("rhs_norm", ctypes.c_double),
                ("t_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("rel_res", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhdg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2007_11891_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "hdg_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
        "hdg_create": (ctypes.c_int, [ip, dp, dp, dp, ctypes.c_int, ctypes.c_double, dp,
                                      ctypes.c_double, vp, ctypes.POINTER(vp)]),
        "hdg_create_ex": (ctypes.c_int, [ip, dp, dp, dp, ctypes.c_int, ctypes.c_double, dp,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, vp,
                                         ctypes.POINTER(vp)]),
        "hdg_destroy": (ctypes.c_int, [vp]),
        "hdg_last_error": (ctypes.c_char_p, []),
        "hdg_sizes": (ctypes.c_int, [vp, i64p, i64p, i64p]),
        "hdg_layout": (ctypes.c_int, [ip, ctypes.c_int, ctypes.c_int, i64p, i64p, i64p]),
        "hdg_set_lambda": (ctypes.c_int, [vp, vp]),
        "hdg_tables": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp, dp, dp, dp]),
        "hdg_coords": (ctypes.c_int, [vp, vp, vp]),
        "hdg_set_origin": (ctypes.c_int, [vp, dp]),
        "hdg_apply": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "hdg_apply_noalloc": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "hdg_face_transform": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_int64]),
        "hdg_rhs": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int]),
        "hdg_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(SolveOpts),
                                     ctypes.POINTER(SolveInfo)]),
        "hdg_solve_forcing": (ctypes.c_int, [vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                             ctypes.POINTER(SolveInfo)]),
        "hdg_reconstruct": (ctypes.c_int, [vp, vp, vp, vp]),
        "hdg_hybridize": (ctypes.c_int, [vp, vp, vp, vp]),
        "hdg_adjoint": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                       ctypes.POINTER(SolveInfo)]),
        "hdg_diagonal": (ctypes.c_int, [vp, vp]),
        "hdg_time_kernel": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_int, dp]),
        "hdg_set_tile": (ctypes.c_int, [vp, ctypes.c_int]),
        "hdg_set_cg_segment": (ctypes.c_int, [vp, ctypes.c_int]),
        "hdg_autotune": (ctypes.c_int, [vp, ctypes.c_int, ip, dp]),
        "hdg_tile_shape": (ctypes.c_int, [vp, ip, ip, ip, ip]),
        "hdg_batch_create": (ctypes.c_int, [ctypes.c_int, ip, ip, dp, ctypes.c_double, vp,
                                            ctypes.POINTER(vp)]),
        "hdg_batch_destroy": (ctypes.c_int, [vp]),
        "hdg_batch_sizes": (ctypes.c_int, [vp, i64p, i64p, i64p, i64p]),
        "hdg_batch_set_tile": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int]),
        "hdg_batch_tiles": (ctypes.c_int, [vp, ip]),
        "hdg_batch_set_form": (ctypes.c_int, [vp, ctypes.c_int]),
        "hdg_batch_form": (ctypes.c_int, [vp, ip]),
        "hdg_batch_autotune": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ip]),
        "hdg_batch_time_cg": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, dp]),
        "hdg_batch_solve_forcing": (ctypes.c_int, [vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                                   ctypes.POINTER(BatchResult), dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, allow_noconv: bool = False):
    if status == HDG_OK or (allow_noconv and status == -4):
        return status
    msg = load_library().hdg_last_error()
    raise HdgError(status, msg.decode() if msg else "")


# SolveOpts.precond: the paper's solvers (section "Summary of solution method")
# hdg_timed_kernel ids of hdg_time_kernel (include/hdg.h)
TIME_ELEM_APPLY_F64, TIME_ELEM_APPLY_F32 = 0, 1
TIME_CG2_ITER_F64, TIME_CG2_ITER_F32 = 2, 3
TIME_CG2_APPLY_F64, TIME_CG2_UPDATE_F64, TIME_CG2_APPLY_F32, TIME_CG2_UPDATE_F32 = 4, 5, 6, 7
TIME_COPY_F64 = 8
TIME_CG1_ITER_F64, TIME_CG1_ITER_F32, TIME_CG1_GRAPH_F64, TIME_CG1_GRAPH_F32 = 9, 10, 11, 12
TIME_NODAL_UNPREC_F64, TIME_NODAL_DIAG_F64, TIME_NODAL_BLOCK_F64 = 13, 14, 15
TIME_APPLY_F64, TIME_APPLY_F32 = 16, 17
TIME_PENCIL_ITER_F64, TIME_PENCIL_ITER_F32 = 18, 19

PRECOND_NONE = 0          # HDG-unprec, nodal basis
PRECOND_EIGEN_JACOBI = 1  # HDG-trans, eigen-face basis (default)
PRECOND_NODAL_DIAG = 2    # HDG-diag, nodal basis
PRECOND_NODAL_BLOCK = 3   # HDG-block, nodal basis


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load_library().hdg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def layout(n: Sequence[int], p: int, neumann: int = 0) -> Sizes:
    """Trace and volume lengths of a mesh without a context (host only)."""
    nn = (ctypes.c_int * 3)(*(int(v) for v in n))
    nf, na, nv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().hdg_layout(nn, int(p), int(neumann), ctypes.byref(nf), ctypes.byref(na),
                                      ctypes.byref(nv)))
    return Sizes(nf.value, na.value, nv.value)


def tables(p: int, tau: float) -> dict:
    """1D tables of the library (host-only call): GLL x, w, D, S, Lambda, B_S, H."""
    lib = load_library()
    n = p + 1
    arrs = {k: np.zeros(s) for k, s in (("x", n), ("w", n), ("D", n * n), ("S", n * n),
                                          ("Lam", n), ("BS", 2 * n), ("H", 1))}
    ptr = {k: v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for k, v in arrs.items()}
    _check(lib.hdg_tables(p, float(tau), ptr["x"], ptr["w"], ptr["D"], ptr["S"], ptr["Lam"],
                          ptr["BS"], ptr["H"]))
    arrs["D"] = arrs["D"].reshape(n, n)
    arrs["S"] = arrs["S"].reshape(n, n)
    arrs["BS"] = arrs["BS"].reshape(n, 2)
    arrs["H"] = float(arrs["H"][0])
    return arrs


def _torch():
    import torch
    return torch


def _dptr(t, n: int, dtype, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class Sizes:
    n_free: int
    n_all: int
    n_vol: int


class HdgContext:
    """One Cartesian mesh / degree / lambda field on the current GPU;
    ``neumann`` is the mask of Neumann sides (bit 2a + s), 0 = all Dirichlet;
    ``exact_mass`` selects the exact GLL mass matrix instead of the lumped one."""

    def __init__(self, n: Sequence[int], widths: Sequence[np.ndarray], p: int, tau: float,
                 lam, device=None, neumann: int = 0, exact_mass: bool = False):
        torch = _torch()
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self._lib = lib
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.n = tuple(int(v) for v in n)
        self.p = int(p)
        self.n_elem = self.n[0] * self.n[1] * self.n[2]
        self.neumann = int(neumann)
        self.exact_mass = bool(exact_mass)
        self._widths = [np.ascontiguousarray(w, dtype=np.float64) for w in widths]
        nn = (ctypes.c_int * 3)(*self.n)
        dp = ctypes.POINTER(ctypes.c_double)
        lam_arr = np.asarray(lam, dtype=np.float64)
        lam_ptr, lam_const = None, 0.0
        if lam_arr.ndim == 0:
            lam_const = float(lam_arr)
        else:
            lam_arr = np.ascontiguousarray(lam_arr)
            if lam_arr.size != self.n_elem:
                raise ValueError("lambda must have one value per element")
            lam_ptr = lam_arr.ctypes.data_as(dp)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            self._stream = stream
            h = ctypes.c_void_p()
            _check(lib.hdg_create_ex(nn, *(w.ctypes.data_as(dp) for w in self._widths), self.p,
                                     float(tau), lam_ptr, lam_const, self.neumann,
                                     int(self.exact_mass), ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.byref(h)))
        self._h = h
        nf, na, nv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.hdg_sizes(self._h, ctypes.byref(nf), ctypes.byref(na), ctypes.byref(nv)))
        self.sizes = Sizes(nf.value, na.value, nv.value)

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers --------------------------------------------------------------
    def _empty(self, n, dtype=None):
        torch = _torch()
        return torch.empty(n, dtype=dtype or torch.float64, device=self.device)

    def zeros_trace(self):
        return _torch().zeros(self.sizes.n_all, dtype=_torch().float64, device=self.device)

    # -- entry points -----------------------------------------------------------
    def coords(self):
        v = self._empty(self.sizes.n_vol * 3)
        t = self._empty(self.sizes.n_all * 3)
        _check(self._lib.hdg_coords(self._h, ctypes.c_void_p(v.data_ptr()),
                                    ctypes.c_void_p(t.data_ptr())))
        return v.view(-1, 3), t.view(-1, 3)

    def set_origin(self, origin):
        """Coordinates of the mesh corner for coords() (default 0, 0, 0)."""
        o = (ctypes.c_double * 3)(*(float(v) for v in origin))
        _check(self._lib.hdg_set_origin(self._h, o))

    def set_lambda(self, lam):
        torch = _torch()
        _check(self._lib.hdg_set_lambda(self._h, _dptr(lam, self.n_elem, torch.float64, "lambda")))

    def apply_noalloc(self, x, y, basis: str = "eigen"):
        """hdg_apply_noalloc: the apply with its scratch in the library's
        static device array (y must be given: nothing is allocated)."""
        torch = _torch()
        dt = x.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("x must be float64 or float32")
        n = self.sizes.n_free
        _check(self._lib.hdg_apply_noalloc(self._h, _dptr(x, n, dt, "x"), _dptr(y, n, dt, "y"),
                                           F64 if dt == torch.float64 else F32,
                                           EIGEN if basis == "eigen" else NODAL))
        return y

    def apply(self, x, y=None, basis: str = "eigen"):
        torch = _torch()
        dt = x.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("x must be float64 or float32")
        if y is None:
            y = self._empty(self.sizes.n_free, dt)
        n = self.sizes.n_free
        _check(self._lib.hdg_apply(self._h, _dptr(x, n, dt, "x"), _dptr(y, n, dt, "y"),
                                   F64 if dt == torch.float64 else F32,
                                   EIGEN if basis == "eigen" else NODAL))
        return y

    def face_transform(self, kind: int, x, n_faces: int, out=None):
        torch = _torch()
        m = n_faces * (self.p + 1) ** 2
        if out is None:
            out = self._empty(m)
        _check(self._lib.hdg_face_transform(self._h, int(kind), _dptr(x, m, torch.float64, "in"),
                                            _dptr(out, m, torch.float64, "out"), int(n_faces)))
        return out

    def rhs(self, f, trace=None, basis: str = "nodal"):
        torch = _torch()
        out = self._empty(self.sizes.n_free)
        tp = None if trace is None else _dptr(trace, self.sizes.n_all, torch.float64, "trace")
        _check(self._lib.hdg_rhs(self._h, _dptr(f, self.sizes.n_vol, torch.float64, "f"), tp,
                                 _dptr(out, self.sizes.n_free, torch.float64, "F"),
                                 EIGEN if basis == "eigen" else NODAL))
        return out

    def solve(self, F_free, opts: Optional[SolveOpts] = None, u_free=None,
              allow_noconv: bool = False):
        torch = _torch()
        if u_free is None:
            u_free = self._empty(self.sizes.n_free)
        info = SolveInfo()
        o = opts or default_opts()
        st = self._lib.hdg_solve(self._h, _dptr(F_free, self.sizes.n_free, torch.float64, "F"),
                                 _dptr(u_free, self.sizes.n_free, torch.float64, "u"),
                                 ctypes.byref(o), ctypes.byref(info))
        _check(st, allow_noconv=allow_noconv)
        return u_free, info.as_dict()

    def solve_forcing(self, f, trace, u_vol=None, want_volume: bool = True,
                      opts: Optional[SolveOpts] = None, allow_noconv: bool = False):
        """Solve with forcing f; trace: in = boundary tail (g_D, g_N) and, with
        opts.guess = 1, the initial guess in the free part; out = nodal
        solution in the free part."""
        torch = _torch()
        if want_volume and u_vol is None:
            u_vol = self._empty(self.sizes.n_vol)
        info = SolveInfo()
        o = opts or default_opts()
        st = self._lib.hdg_solve_forcing(
            self._h, _dptr(f, self.sizes.n_vol, torch.float64, "f"),
            _dptr(trace, self.sizes.n_all, torch.float64, "trace"),
            _dptr(u_vol, self.sizes.n_vol, torch.float64, "u_vol") if want_volume else None,
            ctypes.byref(o), ctypes.byref(info))
        _check(st, allow_noconv=allow_noconv)
        return trace, u_vol, info.as_dict()

    def reconstruct(self, f, trace, u_vol=None):
        torch = _torch()
        if u_vol is None:
            u_vol = self._empty(self.sizes.n_vol)
        _check(self._lib.hdg_reconstruct(self._h, _dptr(f, self.sizes.n_vol, torch.float64, "f"),
                                         _dptr(trace, self.sizes.n_all, torch.float64, "trace"),
                                         _dptr(u_vol, self.sizes.n_vol, torch.float64, "u_vol")))
        return u_vol

    def hybridize(self, u_vol, trace=None, out=None):
        """Initial-guess trace (free part, nodal) from a volume field; the
        g_N block of ``trace`` is read on Neumann faces."""
        torch = _torch()
        if out is None:
            out = self._empty(self.sizes.n_free)
        tp = None if trace is None else _dptr(trace, self.sizes.n_all, torch.float64, "trace")
        _check(self._lib.hdg_hybridize(self._h, _dptr(u_vol, self.sizes.n_vol, torch.float64, "u"),
                                       tp, _dptr(out, self.sizes.n_free, torch.float64, "out")))
        return out

    def adjoint(self, f, trace, dJdu, opts: Optional[SolveOpts] = None):
        torch = _torch()
        dl = self._empty(self.n_elem)
        df = self._empty(self.sizes.n_vol)
        info = SolveInfo()
        o = opts or default_opts()
        _check(self._lib.hdg_adjoint(
            self._h, _dptr(f, self.sizes.n_vol, torch.float64, "f"),
            _dptr(trace, self.sizes.n_all, torch.float64, "trace"),
            _dptr(dJdu, self.sizes.n_vol, torch.float64, "dJdu"),
            _dptr(dl, self.n_elem, torch.float64, "dJdlambda"),
            _dptr(df, self.sizes.n_vol, torch.float64, "dJdf"), ctypes.byref(o), ctypes.byref(info)))
        return dl, df, info.as_dict()

    def diagonal(self):
        torch = _torch()
        d = self._empty(self.sizes.n_free)
        _check(self._lib.hdg_diagonal(self._h, _dptr(d, self.sizes.n_free, torch.float64, "diag")))
        return d

    def set_tile(self, variant: int):
        _check(self._lib.hdg_set_tile(self._h, int(variant)))

    def autotune(self, reps: int = 20):
        """Pick the fastest element-kernel tile variant; returns (variant, times_ms)."""
        ch = ctypes.c_int()
        t = (ctypes.c_double * 3)()
        _check(self._lib.hdg_autotune(self._h, int(reps), ctypes.byref(ch), t))
        return ch.value, list(t)

    def set_cg_segment(self, ks: int = 0):
        """Elements per x3 segment of the pencil CG form (0: automatic)."""
        _check(self._lib.hdg_set_cg_segment(self._h, int(ks)))

    def tile_shape(self) -> dict:
        v, e, t, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.hdg_tile_shape(self._h, ctypes.byref(v), ctypes.byref(e), ctypes.byref(t),
                                        ctypes.byref(g)))
        return {"variant": v.value, "elems_per_unit": e.value, "threads_per_unit": t.value,
                "cg_variant": g.value}

    def time_kernel(self, which: int, x, reps: int = 100, y=None) -> float:
        """Mean launch time (ms) of an internal kernel, HIP events on the context stream."""
        ms = ctypes.c_double()
        yp = None if y is None else ctypes.c_void_p(y.data_ptr())
        _check(self._lib.hdg_time_kernel(self._h, int(which), ctypes.c_void_p(x.data_ptr()),
                                         yp, int(reps), ctypes.byref(ms)))
        return ms.value


class HdgBatch:
    """Independent unit-cube problems (uniform meshes, constant lambda, zero
    Dirichlet data) solved together by the persistent batched CG."""

    def __init__(self, n_elem: Sequence[Sequence[int]], p: Sequence[int], lam: Sequence[float],
                 tau: float = 1.0, device=None):
        torch = _torch()
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self._lib = lib
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        ne = np.ascontiguousarray(np.asarray(n_elem, dtype=np.int32).reshape(-1, 3))
        self.count = ne.shape[0]
        pp = np.ascontiguousarray(np.asarray(p, dtype=np.int32).reshape(-1))
        ll = np.ascontiguousarray(np.asarray(lam, dtype=np.float64).reshape(-1))
        if pp.size != self.count or ll.size != self.count:
            raise ValueError("n_elem, p and lam must describe the same number of problems")
        self.n_elem, self.p, self.lam = ne, pp, ll
        ip = ctypes.POINTER(ctypes.c_int)
        with torch.cuda.device(self.device):
            self._stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _check(lib.hdg_batch_create(self.count, ne.ctypes.data_as(ip), pp.ctypes.data_as(ip),
                                        ll.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        float(tau), ctypes.c_void_p(self._stream.cuda_stream),
                                        ctypes.byref(h)))
        self._h = h
        nf = np.zeros(self.count, dtype=np.int64)
        nv = np.zeros(self.count, dtype=np.int64)
        tf, tv = ctypes.c_int64(), ctypes.c_int64()
        i64p = ctypes.POINTER(ctypes.c_int64)
        _check(lib.hdg_batch_sizes(self._h, nf.ctypes.data_as(i64p), nv.ctypes.data_as(i64p),
                                   ctypes.byref(tf), ctypes.byref(tv)))
        self.n_free, self.n_vol = nf, nv
        self.total_free, self.total_vol = tf.value, tv.value
        self.free_off = np.concatenate([[0], np.cumsum(nf)])
        self.vol_off = np.concatenate([[0], np.cumsum(nv)])

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, p: int, variant: int):
        _check(self._lib.hdg_batch_set_tile(self._h, int(p), int(variant)))

    def tiles(self) -> dict:
        v = (ctypes.c_int * 17)()
        _check(self._lib.hdg_batch_tiles(self._h, v))
        return {q: v[q] for q in range(17) if v[q] >= 0}

    def set_form(self, form: int):
        """0: two phases per CG iteration, 1: one element pass (see hdg.h)."""
        _check(self._lib.hdg_batch_set_form(self._h, int(form)))

    def form(self) -> int:
        v = ctypes.c_int()
        _check(self._lib.hdg_batch_form(self._h, ctypes.byref(v)))
        return v.value

    def autotune(self, iters: int = 20, reps: int = 3) -> dict:
        v = (ctypes.c_int * 17)()
        _check(self._lib.hdg_batch_autotune(self._h, int(iters), int(reps), v))
        return {q: v[q] for q in range(17) if v[q] >= 0}

    def time_cg(self, iters: int, reps: int = 3) -> float:
        ms = ctypes.c_double()
        _check(self._lib.hdg_batch_time_cg(self._h, int(iters), int(reps), ctypes.byref(ms)))
        return ms.value

    def solve_forcing(self, f, trace_free=None, u_vol=None, want_volume: bool = True,
                      opts: Optional[SolveOpts] = None, allow_noconv: bool = False):
        """f: concatenated volume forcing; returns (trace_free, u_vol, results, t_ms)."""
        torch = _torch()
        if trace_free is None:
            trace_free = torch.empty(self.total_free, dtype=torch.float64, device=self.device)
        if want_volume and u_vol is None:
            u_vol = torch.empty(self.total_vol, dtype=torch.float64, device=self.device)
        res = (BatchResult * self.count)()
        ms = ctypes.c_double()
        o = opts or default_opts()
        st = self._lib.hdg_batch_solve_forcing(
            self._h, _dptr(f, self.total_vol, torch.float64, "f"),
            _dptr(trace_free, self.total_free, torch.float64, "trace_free"),
            _dptr(u_vol, self.total_vol, torch.float64, "u_vol") if want_volume else None,
            ctypes.byref(o), res, ctypes.byref(ms))
        _check(st, allow_noconv=allow_noconv)
        return trace_free, u_vol, [r.as_dict() for r in res], ms.value

"""Thin ctypes binding of the gfx950 kd-tree FMM library (include/fmm_mi355.h).

Functions carry the C names and only marshal arguments: torch tensors supply
device pointers, the current HIP stream is passed through, and every step of
the computation runs in the library's kernels.  There is no fallback: if the
library is not built, or a tensor is not a contiguous tensor on the GPU with
the expected dtype, the call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmm_mi355.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "fmm_mi355.h")

FMM_OK, FMM_ERR_INVALID, FMM_ERR_ALLOC, FMM_ERR_CAPACITY, FMM_ERR_HIP, FMM_ERR_STATE = (
    0, -1, -2, -3, -4, -5)
FMM_FP64, FMM_FP32 = 0, 1
FMM_WALK_PHANTOM, FMM_WALK_MUTUAL = 0, 1
FMM_EXPANSION_PHANTOM, FMM_EXPANSION_DEHNEN = 0, 1
FMM_TREE_MEDIAN, FMM_TREE_COM = 0, 1
FMM_REWALK = 1
FMM_VJP_ONLY = 2

_STATUS = {0: "FMM_OK", -1: "FMM_ERR_INVALID", -2: "FMM_ERR_ALLOC", -3: "FMM_ERR_CAPACITY",
           -4: "FMM_ERR_HIP", -5: "FMM_ERR_STATE"}


class FmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class fmm_params(C.Structure):
    _fields_ = [("theta", C.c_double), ("r_kern", C.c_double), ("G", C.c_double),
                ("leaf_size", C.c_int32), ("walk", C.c_int32), ("precision", C.c_int32),
                ("expansion", C.c_int32), ("tree", C.c_int32), ("reserved", C.c_int32),
                ("list_capacity", C.c_int64), ("device_bytes_limit", C.c_int64),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class fmm_stats(C.Structure):
    _fields_ = [("sumF", C.c_double * 3), ("sumAbsF", C.c_double), ("ratio", C.c_double),
                ("mass", C.c_double), ("xcom", C.c_double * 3), ("P", C.c_double * 3),
                ("L", C.c_double * 3), ("pad", C.c_double)]


_lib = None
_vp = C.c_void_p


def lib() -> C.CDLL:
    """Load libfmm_mi355.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    L.fmm_default_params.argtypes = [C.POINTER(fmm_params)]
    L.fmm_default_params.restype = None
    L.fmm_last_error.argtypes = []
    L.fmm_last_error.restype = C.c_char_p
    L.fmm_build_tree.argtypes = [_vp, C.c_int64, C.POINTER(fmm_params), _vp, C.POINTER(_vp)]
    L.fmm_build_tree.restype = st
    L.fmm_build_tree_weighted.argtypes = [_vp, _vp, C.c_int64, C.POINTER(fmm_params), _vp,
                                          C.POINTER(_vp)]
    L.fmm_build_tree_weighted.restype = st
    L.fmm_moments.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.fmm_moments.restype = st
    L.fmm_forces.argtypes = [_vp, _vp, C.c_int32, _vp]
    L.fmm_forces.restype = st
    L.fmm_forces_vjp.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.fmm_forces_vjp.restype = st
    L.fmm_asymmetry_estimate.argtypes = [_vp, C.c_double, _vp, _vp]
    L.fmm_asymmetry_estimate.restype = st
    L.fmm_momentum_stats.argtypes = [_vp, _vp, _vp, _vp, C.c_int32, C.c_int64,
                                     C.POINTER(fmm_stats), _vp]
    L.fmm_momentum_stats.restype = st
    L.fmm_momentum_stats_async.argtypes = [_vp, _vp, _vp, _vp, C.c_int32, C.c_int64, _vp, _vp]
    L.fmm_momentum_stats_async.restype = st
    L.fmm_momentum_stats_noalloc.argtypes = [_vp, _vp, _vp, _vp, C.c_int32, C.c_int64, _vp, _vp]
    L.fmm_momentum_stats_noalloc.restype = st
    L.fmm_kick_drift.argtypes = [_vp, _vp, _vp, C.c_int32, C.c_int64, C.c_double, C.c_double,
                                 _vp]
    L.fmm_kick_drift.restype = st
    L.fmm_tree_free.argtypes = [_vp]
    L.fmm_tree_free.restype = None
    L.fmm_tree_info.argtypes = [_vp, _vp]
    L.fmm_tree_info.restype = st
    L.fmm_tree_device_bytes.argtypes = [_vp, C.POINTER(C.c_int64)]
    L.fmm_tree_device_bytes.restype = st
    L.fmm_tree_params.argtypes = [_vp, C.POINTER(fmm_params), C.POINTER(C.c_int64)]
    L.fmm_tree_params.restype = st
    L.fmm_debug_import.argtypes = [_vp] * 15
    L.fmm_debug_import.restype = st
    L.fmm_debug_export.argtypes = [_vp] * 13
    L.fmm_debug_export.restype = st
    L.fmm_set_timing.argtypes = [_vp, C.c_int32]
    L.fmm_set_timing.restype = st
    L.fmm_stage_times.argtypes = [_vp, _vp]
    L.fmm_stage_times.restype = st
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions the public header declares."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z0-9_]+)\s*\(", txt)))


def _check(status: int):
    if status != FMM_OK:
        raise FmmError(status, lib().fmm_last_error().decode())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor"):
    """Device pointer of t after checking its dtype, shape, layout and device
    (in that order), so that no kernel is handed a buffer it would overrun."""
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype} (got {t.dtype})")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    return C.c_void_p(t.data_ptr())


def default_params(**kw) -> fmm_params:
    p = fmm_params()
    lib().fmm_default_params(C.byref(p))
    fields = {f[0] for f in fmm_params._fields_}
    for k, v in kw.items():
        if k not in fields:
            raise TypeError(f"fmm_params has no field {k!r}")
        setattr(p, k, v)
    return p


def fmm_last_error() -> str:
    return lib().fmm_last_error().decode()


# --------------------------------------------------------------------- calls
def fmm_build_tree(x, params: fmm_params, stream=None, tree=None, m=None):
    """Build (or rebuild in place) the kd-tree of x (n x 3, float64, GPU); m
    (n, float64, GPU) weighs the centre-of-mass cut of FMM_TREE_COM."""
    import torch

    n = x.shape[0]
    h = C.c_void_p(tree) if tree else C.c_void_p(None)
    if m is None:
        _check(lib().fmm_build_tree(_ptr(x, torch.float64, (n, 3), "x"), n, C.byref(params),
                                    _stream(stream), C.byref(h)))
    else:
        _check(lib().fmm_build_tree_weighted(_ptr(x, torch.float64, (n, 3), "x"),
                                             _ptr(m, torch.float64, (n,), "m"), n,
                                             C.byref(params), _stream(stream), C.byref(h)))
    return h.value


def fmm_moments(tree, x, m, h, stream=None):
    import torch

    _, n = _tree_dtype_n(tree)
    _check(lib().fmm_moments(C.c_void_p(tree), _ptr(x, torch.float64, (n, 3), "x"),
                             _ptr(m, torch.float64, (n,), "m"), _ptr(h, torch.float64, (n,), "h"),
                             _stream(stream)))


def fmm_tree_params(tree):
    """(params, n) the tree was last built with (host only, no device work)."""
    p = fmm_params()
    n = C.c_int64(0)
    _check(lib().fmm_tree_params(C.c_void_p(tree), C.byref(p), C.byref(n)))
    return p, int(n.value)


def _tree_dtype_n(tree):
    """dtype of the tree's accelerations and its particle count."""
    import torch

    p, n = fmm_tree_params(tree)
    return (torch.float32 if p.precision == FMM_FP32 else torch.float64), n


def fmm_forces(tree, a, flags: int = 0, stream=None):
    """a may be None with FMM_VJP_ONLY (the tree is prepared for the reverse
    pass and no forces are written)."""
    dt, n = _tree_dtype_n(tree)
    ap = None if (a is None and flags & FMM_VJP_ONLY) else _ptr(a, dt, (n, 3), "a")
    _check(lib().fmm_forces(C.c_void_p(tree), ap, flags, _stream(stream)))


def fmm_forces_vjp(tree, a_bar, x_bar, m_bar, stream=None):
    dt, n = _tree_dtype_n(tree)
    _check(lib().fmm_forces_vjp(C.c_void_p(tree), _ptr(a_bar, dt, (n, 3), "a_bar"),
                                _ptr(x_bar, dt, (n, 3), "x_bar"),
                                _ptr(m_bar, dt, (n,), "m_bar"), _stream(stream)))


def fmm_momentum_stats(x, v, m, a, stream=None) -> dict:
    import torch

    n = x.shape[0]
    prec = FMM_FP32 if a.dtype == torch.float32 else FMM_FP64
    out = fmm_stats()
    _check(lib().fmm_momentum_stats(_ptr(x, torch.float64, (n, 3), "x"),
                                    _ptr(v, torch.float64, (n, 3), "v") if v is not None else None,
                                    _ptr(m, torch.float64, (n,), "m"), _ptr(a, a.dtype, (n, 3), "a"),
                                    prec, n, C.byref(out), _stream(stream)))
    return {"sumF": np.array(out.sumF), "sumAbsF": out.sumAbsF, "ratio": out.ratio,
            "mass": out.mass, "xcom": np.array(out.xcom), "P": np.array(out.P),
            "L": np.array(out.L)}


def fmm_momentum_stats_async(x, v, m, a, out, stream=None):
    """The statistics of fmm_momentum_stats into out, a float64 device tensor
    of 16 elements (sumF[3], sumAbsF, ratio, mass, xcom[3], P[3], L[3], pad),
    without waiting for the stream."""
    import torch

    n = x.shape[0]
    prec = FMM_FP32 if a.dtype == torch.float32 else FMM_FP64
    _check(lib().fmm_momentum_stats_async(
        _ptr(x, torch.float64, (n, 3), "x"),
        _ptr(v, torch.float64, (n, 3), "v") if v is not None else None,
        _ptr(m, torch.float64, (n,), "m"), _ptr(a, a.dtype, (n, 3), "a"), prec, n,
        _ptr(out, torch.float64, (16,), "out"), _stream(stream)))


def fmm_momentum_stats_noalloc(x, v, m, a, out, stream=None):
    """fmm_momentum_stats_async without any device allocation (the partial
    sums use a fixed array of the library): out is a float64 device tensor of
    16 elements."""
    import torch

    n = x.shape[0]
    prec = FMM_FP32 if a.dtype == torch.float32 else FMM_FP64
    _check(lib().fmm_momentum_stats_noalloc(
        _ptr(x, torch.float64, (n, 3), "x"),
        _ptr(v, torch.float64, (n, 3), "v") if v is not None else None,
        _ptr(m, torch.float64, (n,), "m"), _ptr(a, a.dtype, (n, 3), "a"), prec, n,
        _ptr(out, torch.float64, (16,), "out"), _stream(stream)))


def fmm_asymmetry_estimate(tree, m_leaf: float = 0.0, stream=None) -> dict:
    """Asymmetric pairs of the current lists and the total-force estimates
    eq. (33) and eq. (46) (m_leaf <= 0: mean leaf mass)."""
    out = np.empty(4)
    _check(lib().fmm_asymmetry_estimate(C.c_void_p(tree), float(m_leaf),
                                        out.ctypes.data_as(C.c_void_p), _stream(stream)))
    return {"F33": float(out[0]), "F46": float(out[1]), "n_asym": int(out[2]),
            "n_asym_super": int(out[3])}


def fmm_kick_drift(x, v, a, kick: float, drift: float, stream=None):
    """v += kick * a; x += drift * v (in place, on the GPU)."""
    import torch

    n = x.shape[0]
    prec = FMM_FP32 if a.dtype == torch.float32 else FMM_FP64
    _check(lib().fmm_kick_drift(_ptr(x, torch.float64, (n, 3), "x"),
                                _ptr(v, torch.float64, (n, 3), "v"), _ptr(a, a.dtype, (n, 3), "a"),
                                prec, n, float(kick), float(drift), _stream(stream)))


def fmm_tree_free(tree):
    if tree:
        lib().fmm_tree_free(C.c_void_p(tree))


def fmm_tree_info(tree) -> dict:
    info = np.zeros(8, np.int64)
    _check(lib().fmm_tree_info(C.c_void_p(tree), info.ctypes.data_as(C.c_void_p)))
    keys = ("n", "nodes", "leaves", "depth", "n_far", "n_near", "sinks", "has_lists")
    return {k: int(v) for k, v in zip(keys, info)}


def fmm_tree_device_bytes(tree) -> int:
    """Device memory the library holds for the tree, in bytes."""
    b = C.c_int64(0)
    _check(lib().fmm_tree_device_bytes(C.c_void_p(tree), C.byref(b)))
    return int(b.value)


def fmm_set_timing(tree, on: bool):
    _check(lib().fmm_set_timing(C.c_void_p(tree), int(bool(on))))


def fmm_stage_times(tree) -> dict:
    ms = np.zeros(8)
    _check(lib().fmm_stage_times(C.c_void_p(tree), ms.ctypes.data_as(C.c_void_p)))
    keys = ("build", "moments", "walk", "far", "near", "vjp", "stats", "total")
    return dict(zip(keys, ms.tolist()))


def fmm_debug_import(tree, x, m, h, ex: dict, stream=None):
    """Replace the tree's particle order, cell records and interaction lists
    with those of ex (keys as fmm_debug_export returns them: perm, first,
    count, left, right, rec, far_off, far_src, near_off, near_src); x, m, h
    are the particles on the GPU (caller order)."""
    import torch

    _, n = _tree_dtype_n(tree)
    keep = {}

    def host(k, dt):
        a = np.ascontiguousarray(ex[k], dtype=dt)
        keep[k] = a
        return a.ctypes.data_as(C.c_void_p) if a.size else None

    args = [host("perm", np.int32), host("first", np.int32), host("count", np.int32),
            host("left", np.int32), host("right", np.int32), host("rec", np.float64),
            host("far_off", np.int64), host("far_src", np.int32), host("near_off", np.int64),
            host("near_src", np.int32)]
    _check(lib().fmm_debug_import(C.c_void_p(tree), _ptr(x, torch.float64, (n, 3), "x"),
                                  _ptr(m, torch.float64, (n,), "m"),
                                  _ptr(h, torch.float64, (n,), "h"), *args, _stream(stream)))


def fmm_debug_export(tree, lists=True, local: bool = False) -> dict:
    """Copy the tree, cell records and lists to host numpy arrays.
    lists: True (offsets and entries), "offsets" (the CSR offsets only, i.e.
    the list lengths: cheap for trees too large to copy every entry), False."""
    info = fmm_tree_info(tree)
    n, nn = info["n"], info["nodes"]
    out = {"perm": np.empty(n, np.int32)}
    for k in ("first", "count", "left", "right", "axis"):
        out[k] = np.empty(nn, np.int32)
    out["rec"] = np.empty((nn, 12))
    have_lists = bool(lists) and info["has_lists"]
    entries = have_lists and lists != "offsets"
    if have_lists:
        out["far_off"] = np.empty(nn + 1, np.int64)
        out["near_off"] = np.empty(nn + 1, np.int64)
    if entries:
        out["far_src"] = np.empty(max(info["n_far"], 1), np.int32)
        out["near_src"] = np.empty(max(info["n_near"], 1), np.int32)
    if local:
        out["local"] = np.empty((nn, 19))

    def p(k):
        a = out.get(k)
        return None if a is None else a.ctypes.data_as(C.c_void_p)

    _check(lib().fmm_debug_export(C.c_void_p(tree), p("perm"), p("first"), p("count"),
                                  p("left"), p("right"), p("axis"), p("rec"), p("far_off"),
                                  p("far_src"), p("near_off"), p("near_src"), p("local")))
    if entries:
        out["far_src"] = out["far_src"][: info["n_far"]]
        out["near_src"] = out["near_src"][: info["n_near"]]
    return out


class TorchDeviceAllocator:
    """Allocator hooks (fmm_params.dev_alloc / dev_free) that take a tree's
    device memory from torch's caching allocator, so that it is counted in
    torch.cuda.memory_allocated() and reused by torch after fmm_tree_free.
    `live` maps each pointer the library holds to its size."""

    def __init__(self, device: int = 0):
        self.device = device
        self.live: dict[int, int] = {}
        self.calls = 0
        self._alloc = ALLOC_FN(self._on_alloc)
        self._free = FREE_FN(self._on_free)

    def allocate(self, nbytes: int):
        import torch

        return torch.cuda.caching_allocator_alloc(nbytes, device=self.device)

    def _on_alloc(self, nbytes, ctx):
        self.calls += 1
        try:
            ptr = self.allocate(int(nbytes))
        except Exception:
            return None
        if ptr:
            self.live[int(ptr)] = int(nbytes)
        return ptr

    def _on_free(self, ptr, ctx):
        import torch

        self.live.pop(int(ptr))
        torch.cuda.caching_allocator_delete(int(ptr))

    def apply(self, params: fmm_params) -> fmm_params:
        params.dev_alloc = self._alloc
        params.dev_free = self._free
        return params


# --------------------------------------------------------------------- convenience
@dataclass
class GravityFMM:
    """Owns one tree: forces(x, m, h) runs build -> moments -> forces."""
    theta: float = 0.5
    r_kern: float = 2.0
    G: float = 1.0
    leaf_size: int = 8
    walk: int = FMM_WALK_PHANTOM
    precision: int = FMM_FP64
    expansion: int = FMM_EXPANSION_PHANTOM
    tree_shape: int = FMM_TREE_MEDIAN
    tree: int | None = None
    n: int = 0

    def params(self) -> fmm_params:
        return default_params(theta=self.theta, r_kern=self.r_kern, G=self.G,
                              leaf_size=self.leaf_size, walk=self.walk,
                              precision=self.precision, expansion=self.expansion,
                              tree=self.tree_shape)

    def build(self, x, stream=None, m=None):
        if self.tree is not None and x.shape[0] != self.n:
            self.free()
        self.tree = fmm_build_tree(x, self.params(), stream, self.tree,
                                   m if self.tree_shape == FMM_TREE_COM else None)
        self.n = x.shape[0]

    def forces(self, x, m, h, out=None, stream=None, rebuild: bool = True):
        import torch

        if rebuild or self.tree is None:
            self.build(x, stream, m)
        fmm_moments(self.tree, x, m, h, stream)
        if out is None:
            dt = torch.float32 if self.precision == FMM_FP32 else torch.float64
            out = torch.empty((x.shape[0], 3), dtype=dt, device=x.device)
        fmm_forces(self.tree, out, FMM_REWALK if rebuild else 0, stream)
        return out

    def free(self):
        if self.tree is not None:
            fmm_tree_free(self.tree)
            self.tree = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

"""The C ABI library loads and exports every function the public header
declares; host-side argument checks fail before any device work (these calls
never touch a GPU, so they run on the CPU)."""
import ctypes as C

import pytest

from paper_2502_01496_amd import fmm as F


def test_library_exports_header_functions():
    L = F.lib()
    names = F.header_functions()
    assert len(names) >= 12
    for n in ("fmm_build_tree", "fmm_moments", "fmm_forces", "fmm_forces_vjp",
              "fmm_momentum_stats", "fmm_asymmetry_estimate"):
        assert n in names
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []


def test_default_params():
    p = F.default_params()
    assert (p.theta, p.r_kern, p.G, p.leaf_size, p.walk, p.precision, p.expansion) == (
        0.5, 2.0, 1.0, 8, F.FMM_WALK_PHANTOM, F.FMM_FP64, F.FMM_EXPANSION_PHANTOM)
    assert (p.tree, p.reserved) == (F.FMM_TREE_MEDIAN, 0)
    assert (p.list_capacity, p.device_bytes_limit, p.alloc_ctx) == (0, 0, None)
    assert not p.dev_alloc and not p.dev_free
    with pytest.raises(TypeError):
        F.default_params(thetta=0.3)
    assert C.sizeof(F.fmm_stats) == 16 * 8
    # the C layout: 3 doubles, 6 int32, 2 int64, 3 pointers
    assert C.sizeof(F.fmm_params) == 88
    assert F.fmm_params.list_capacity.offset == 48 and F.fmm_params.alloc_ctx.offset == 80


def _build(p, n=10, x=C.c_void_p(16), tree=None):
    h = C.c_void_p(tree)
    return F.lib().fmm_build_tree(x, n, C.byref(p), None, C.byref(h)), h.value


@pytest.mark.parametrize("field,value", [
    ("theta", -0.1), ("theta", 1.5), ("theta", float("nan")), ("r_kern", 0.0),
    ("r_kern", float("inf")), ("G", float("nan")), ("leaf_size", 0), ("leaf_size", 65),
    ("walk", 7), ("precision", 2), ("expansion", 2), ("expansion", -1), ("tree", 2),
    ("reserved", 1), ("list_capacity", -1), ("device_bytes_limit", -5)])
def test_bad_params_rejected_on_host(field, value):
    p = F.default_params()
    setattr(p, field, value)
    st, h = _build(p)
    assert st == F.FMM_ERR_INVALID and h is None
    assert F.fmm_last_error() != ""


def test_allocator_hooks_must_come_in_pairs():
    p = F.default_params()
    p.dev_alloc = F.ALLOC_FN(lambda nbytes, ctx: None)
    st, h = _build(p)
    assert st == F.FMM_ERR_INVALID and h is None
    assert "together" in F.fmm_last_error()
    p = F.default_params()
    p.dev_free = F.FREE_FN(lambda ptr, ctx: None)
    assert _build(p)[0] == F.FMM_ERR_INVALID


def test_bad_sizes_and_pointers_rejected():
    p = F.default_params()
    assert _build(p, n=0)[0] == F.FMM_ERR_INVALID
    assert _build(p, n=-5)[0] == F.FMM_ERR_INVALID
    assert _build(p, n=2 ** 31)[0] == F.FMM_ERR_INVALID
    assert _build(p, x=None)[0] == F.FMM_ERR_INVALID
    L = F.lib()
    h = C.c_void_p(None)
    assert L.fmm_build_tree(C.c_void_p(16), 10, None, None, C.byref(h)) == F.FMM_ERR_INVALID
    assert L.fmm_build_tree(C.c_void_p(16), 10, C.byref(p), None, None) == F.FMM_ERR_INVALID


def test_unknown_handles_rejected():
    L = F.lib()
    bogus = C.c_void_p(None)
    assert L.fmm_moments(bogus, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == F.FMM_ERR_STATE
    assert L.fmm_forces(bogus, C.c_void_p(8), 0, None) == F.FMM_ERR_STATE
    assert L.fmm_forces_vjp(bogus, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == F.FMM_ERR_STATE
    info = (C.c_int64 * 8)()
    assert L.fmm_tree_info(bogus, info) == F.FMM_ERR_STATE
    assert L.fmm_tree_params(bogus, None, None) == F.FMM_ERR_STATE
    assert L.fmm_debug_import(bogus, *([C.c_void_p(8)] * 13), None) == F.FMM_ERR_STATE
    with pytest.raises(F.FmmError):
        F.fmm_tree_params(None)
    L.fmm_tree_free(bogus)  # no-op


def test_stats_argument_checks():
    L = F.lib()
    out = F.fmm_stats()
    v = C.c_void_p(8)
    assert L.fmm_momentum_stats(None, None, v, v, 0, 10, C.byref(out), None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats(v, None, v, v, 0, 0, C.byref(out), None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats(v, None, v, v, 5, 10, C.byref(out), None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats(v, None, v, v, 0, 10, None, None) == F.FMM_ERR_INVALID
    # the device-output form rejects the same arguments before launching anything
    assert L.fmm_momentum_stats_async(None, None, v, v, 0, 10, v, None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats_async(v, None, v, v, 0, 0, v, None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats_async(v, None, v, v, 5, 10, v, None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats_async(v, None, v, v, 0, 10, None, None) == F.FMM_ERR_INVALID


def test_binding_refuses_host_tensors():
    import torch

    with pytest.raises((TypeError, RuntimeError)):
        F.fmm_build_tree(torch.zeros(4, 3, dtype=torch.float64), F.default_params())


def test_binding_checks_dtype_and_shape_before_the_call():
    # a buffer of the wrong precision or length would let a kernel write past
    # it: the binding refuses it before anything reaches the library
    import torch

    with pytest.raises(TypeError, match="dtype"):
        F._ptr(torch.zeros(4, 3, dtype=torch.float32), torch.float64, (4, 3), "a")
    with pytest.raises(ValueError, match="shape"):
        F._ptr(torch.zeros(3, 3, dtype=torch.float64), torch.float64, (4, 3), "a")
    with pytest.raises(ValueError, match="shape"):
        F._ptr(torch.zeros(12, dtype=torch.float64), torch.float64, (4, 3), "a")
    with pytest.raises(ValueError, match="contiguous"):
        F._ptr(torch.zeros(3, 4, dtype=torch.float64).t(), torch.float64, (4, 3), "a")
    with pytest.raises(TypeError, match="GPU"):
        F._ptr(torch.zeros(4, 3, dtype=torch.float64), torch.float64, (4, 3), "a")


def test_binding_constants_match_header():
    # every FMM_* enumerator of the header has the same value in the binding
    import os
    import re

    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "fmm_mi355.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    found = dict(re.findall(r"\b(FMM_[A-Z0-9_]+)\s*=\s*(-?\d+)", hdr))
    assert "FMM_VJP_ONLY" in found and "FMM_REWALK" in found
    for name, value in found.items():
        assert getattr(F, name) == int(value), name

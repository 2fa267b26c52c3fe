"""CPU oracle for the kd-tree FMM gravity path (ctypes wrapper around fmm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the package smoke check
and the CPU-baseline leg of the benchmark, never by the GPU product path.  It
shares no code with the HIP library.

Paper: Potashov & Yudin, arXiv:2502.01496.  Each wrapper names the part of the
paper its C function follows; the C file states the arithmetic in full.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

# -ffp-contract=off: no fused multiply-add, so that every operation that feeds
# a discrete decision is one IEEE operation, in source order.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (a build step, not a use of it)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_d = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def _opt(p):
    """ndpointer that also accepts None (NULL)."""
    base = p

    def from_param(cls, obj):
        if obj is None:
            return None
        return base.from_param(obj)

    return type("Opt" + base.__name__, (base,), {"from_param": classmethod(from_param)})


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        I64, I32, D = C.c_int64, C.c_int32, C.c_double
        L.orc_m4_g.restype = D
        L.orc_m4_g.argtypes = [D, D]
        L.orc_m4_dg_over_r.restype = D
        L.orc_m4_dg_over_r.argtypes = [D, D]
        L.orc_direct.argtypes = [I64, _d, _d, _d, D, _d]
        L.orc_direct_sinks.argtypes = [I64, _d, _d, _d, D, I64, _i64, _d]
        L.orc_direct_vjp.argtypes = [I64, _d, _d, _d, D, _d, _d, _d]
        L.orc_morton.argtypes = [I64, _d, _u64, _i32]
        L.orc_build_tree.restype = I32
        L.orc_build_tree.argtypes = [I64, _d, I32, _i32, _i32, _i32, _i32, _i32, _i32]
        L.orc_build_tree_com.argtypes = [I64, _d, _opt(_d), I32, _i32, _i32, _i32, _i32, _i32,
                                         _i32]
        L.orc_build_tree_com.restype = I32
        L.orc_moments.argtypes = [I64, _d, _d, _d, _i32, I32, _i32, _i32, _i32, _i32,
                                  _d, _d, _d, _d, _d]
        L.orc_p2m.argtypes = [I64, _d, _d, _d, _d, _d]
        L.orc_walk.argtypes = [I32, I32, _i32, _i32, _d, _d, _d, D, D,
                               _i32, _opt(_i32), _i32, _opt(_i32), _i64]
        L.orc_m2l.argtypes = [I32, _d, D, _d, _d]
        L.orc_l2p.argtypes = [_d, _d, _d]
        L.orc_l2l.argtypes = [_d, _d, _d]
        L.orc_far_field.argtypes = [I32, I32, I32, _i32, _i32, _d, _d, _d, _i32, _i32, _d]
        L.orc_near_and_l2p.argtypes = [I64, _d, _d, _d, _i32, I32, _i32, _i32, _i32, _d, _d,
                                       _i32, _i32, D, _d]
        L.orc_stats.argtypes = [I64, _d, _opt(_d), _d, _d, _d]
        L.orc_asym_estimate.argtypes = [I32, _i32, _i32, _d, _d, _d, _i32, _i32, D, _d]
        L.orc_fmm_leaves.argtypes = [I64, _d, _d, _d, _i32, I32, _i32, _i32, _i32, _i32,
                                     _d, _d, _d, _d, _d, D, D, D, I32, I64, _i32, _d,
                                     _opt(_i64)]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Pair kernel and direct sum (Sec. 3, eqs. (12)-(16); Sec. 2 eq. (3), theta=0)
# --------------------------------------------------------------------------
def m4_g(r: float, h: float) -> float:
    """phi'(r,h)/r of the M4 cubic spline (R_kern = 2)."""
    return lib().orc_m4_g(float(r), float(h))


def m4_dg_over_r(r: float, h: float) -> float:
    return lib().orc_m4_dg_over_r(float(r), float(h))


def direct(x, m, h, G=1.0):
    """O(N^2) softened direct sum: the result the FMM approximates."""
    x, m, h = _f64(x), _f64(m), _f64(h)
    a = np.empty_like(x)
    lib().orc_direct(len(m), x, m, h, G, a)
    return a


def direct_sinks(x, m, h, sinks, G=1.0):
    x, m, h = _f64(x), _f64(m), _f64(h)
    s = np.ascontiguousarray(sinks, dtype=np.int64)
    a = np.empty((len(s), 3))
    lib().orc_direct_sinks(len(m), x, m, h, G, len(s), s, a)
    return a


def direct_vjp(x, m, h, abar, G=1.0):
    """(da/dx)^T abar and (da/dm)^T abar of the direct sum."""
    x, m, h, abar = _f64(x), _f64(m), _f64(h), _f64(abar)
    xb = np.empty_like(x)
    mb = np.empty_like(m)
    lib().orc_direct_vjp(len(m), x, m, h, G, abar, xb, mb)
    return xb, mb


# --------------------------------------------------------------------------
# Tree, moments, walks (Sec. 2; Sec. 4; Sec. 7)
# --------------------------------------------------------------------------
def morton(x):
    x = _f64(x)
    n = x.shape[0]
    key = np.empty(n, np.uint64)
    order = np.empty(n, np.int32)
    lib().orc_morton(n, x, key, order)
    return key, order


@dataclass
class Tree:
    perm: np.ndarray    # tree position -> caller index
    first: np.ndarray
    count: np.ndarray
    left: np.ndarray
    right: np.ndarray
    axis: np.ndarray    # split axis, -1 for leaves

    @property
    def nnodes(self):
        return len(self.first)

    @property
    def is_leaf(self):
        return self.left < 0


def build_tree(x, leaf_size=8) -> Tree:
    x = _f64(x)
    n = x.shape[0]
    cap = max(2 * n, 1)
    perm = np.empty(n, np.int32)
    arrs = [np.empty(cap, np.int32) for _ in range(5)]
    nn = lib().orc_build_tree(n, x, int(leaf_size), perm, *arrs)
    return Tree(perm, *[a[:nn].copy() for a in arrs])


def build_tree_com(x, m=None, leaf_size=10) -> Tree:
    """kd-tree cut through the centre of mass (Sec. 2 as written); m=None:
    equal weights."""
    x = _f64(x)
    n = x.shape[0]
    cap = max(2 * n, 1)
    perm = np.empty(n, np.int32)
    arrs = [np.empty(cap, np.int32) for _ in range(5)]
    nn = lib().orc_build_tree_com(n, x, None if m is None else _f64(m), int(leaf_size), perm,
                                  *arrs)
    return Tree(perm, *[a[:nn].copy() for a in arrs])


MEDIAN_TREE = 0  # count-median cut (the reading used by default)
COM_TREE = 1     # cut through the centre of mass


@dataclass
class Moments:
    M: np.ndarray
    c: np.ndarray     # (nnodes, 3)
    s: np.ndarray
    hmax: np.ndarray
    Q: np.ndarray     # (nnodes, 6): xx, xy, xz, yy, yz, zz


def moments(x, m, h, tree: Tree) -> Moments:
    x, m, h = _f64(x), _f64(m), _f64(h)
    nn = tree.nnodes
    M = np.empty(nn)
    c = np.empty((nn, 3))
    s = np.empty(nn)
    hm = np.empty(nn)
    Q = np.empty((nn, 6))
    lib().orc_moments(len(m), x, m, h, tree.perm, nn, tree.first, tree.count, tree.left,
                      tree.right, M, c, s, hm, Q)
    return Moments(M, c, s, hm, Q)


def p2m(x, m):
    """Mass, centre of mass and eq. (7) quadrupole of an explicit particle set."""
    x, m = _f64(x), _f64(m)
    M = np.empty(1)
    c = np.empty(3)
    Q = np.empty(6)
    lib().orc_p2m(len(m), x, m, M, c, Q)
    return float(M[0]), c, Q


@dataclass
class Lists:
    far_off: np.ndarray   # CSR over sink node ids
    far_src: np.ndarray
    near_off: np.ndarray
    near_src: np.ndarray

    def far(self, v):
        return self.far_src[self.far_off[v]:self.far_off[v + 1]]

    def near(self, v):
        return self.near_src[self.near_off[v]:self.near_off[v + 1]]


PHANTOM = 0   # leaf <- cell walk (Sec. 4)
MUTUAL = 1    # symmetric walk (Sec. 7)
PHANTOM_FORM = 0  # M2L as eq. (6) and its r-derivatives (quadrupole at every order)
DEHNEN_FORM = 1   # M2L as eqs. (25)-(26), p = 3: combined source + sink order <= 2


def walk(tree: Tree, mom: Moments, theta=0.5, r_kern=2.0, policy=PHANTOM) -> Lists:
    nn = tree.nnodes
    fo = np.empty(nn + 1, np.int32)
    no = np.empty(nn + 1, np.int32)
    tot = np.zeros(2, np.int64)
    L = lib()
    args = (policy, nn, tree.left, tree.right, mom.c, mom.s, mom.hmax, float(theta),
            float(r_kern))
    L.orc_walk(*args, fo, None, no, None, tot)
    fs = np.empty(max(int(tot[0]), 1), np.int32)
    ns = np.empty(max(int(tot[1]), 1), np.int32)
    L.orc_walk(*args, fo, fs, no, ns, tot)
    return Lists(fo, fs[: tot[0]], no, ns[: tot[1]])


# --------------------------------------------------------------------------
# Far field (eqs. (6)-(8)) and near field (eqs. (12)-(16))
# --------------------------------------------------------------------------
def m2l(r, M, Q, form=PHANTOM_FORM):
    """M2L: form PHANTOM_FORM = eq. (6) and its r-derivatives; DEHNEN_FORM =
    eqs. (25)-(26) with p = 3 (combined source + sink order <= 2)."""
    L = np.empty(19)
    lib().orc_m2l(int(form), _f64(r), float(M), _f64(Q), L)
    return L


def l2p(L, y):
    a = np.empty(3)
    lib().orc_l2p(_f64(L), _f64(y), a)
    return a


def l2l(L, delta):
    out = np.empty(19)
    lib().orc_l2l(_f64(L), _f64(delta), out)
    return out


def far_field(tree: Tree, mom: Moments, lists: Lists, policy=PHANTOM, form=PHANTOM_FORM):
    nn = tree.nnodes
    L = np.empty((nn, 19))
    fs = lists.far_src if len(lists.far_src) else np.zeros(1, np.int32)
    lib().orc_far_field(policy, int(form), nn, tree.left, tree.right, mom.M, mom.c, mom.Q,
                        lists.far_off, np.ascontiguousarray(fs, np.int32), L)
    return L


def near_and_l2p(x, m, h, tree: Tree, mom: Moments, L, lists: Lists, G=1.0):
    x, m, h = _f64(x), _f64(m), _f64(h)
    a = np.empty_like(x)
    ns = lists.near_src if len(lists.near_src) else np.zeros(1, np.int32)
    lib().orc_near_and_l2p(len(m), x, m, h, tree.perm, tree.nnodes, tree.first, tree.count,
                           tree.left, mom.c, _f64(L), lists.near_off,
                           np.ascontiguousarray(ns, np.int32), float(G), a)
    return a


@dataclass
class FmmResult:
    a: np.ndarray
    tree: Tree
    mom: Moments
    lists: Lists
    L: np.ndarray


def fmm(x, m, h, theta=0.5, r_kern=2.0, G=1.0, leaf_size=8, policy=PHANTOM,
        form=PHANTOM_FORM, tree_kind=MEDIAN_TREE) -> FmmResult:
    """Serial kd-tree FMM: build, moments, walk, M2L (+L2L), L2P + near field."""
    tree = build_tree(x, leaf_size) if tree_kind == MEDIAN_TREE else build_tree_com(x, m, leaf_size)
    mom = moments(x, m, h, tree)
    lists = walk(tree, mom, theta, r_kern, policy)
    L = far_field(tree, mom, lists, policy, form)
    a = near_and_l2p(x, m, h, tree, mom, L, lists, G)
    return FmmResult(a, tree, mom, lists, L)


def fmm_leaves(x, m, h, tree: Tree, mom: Moments, leaves, theta=0.5, r_kern=2.0, G=1.0,
               form=PHANTOM_FORM, a=None, counts=False):
    """The leaf <- cell FMM for the listed sink leaves (node ids) only: their
    walks, M2L sums, L2P and near fields, identical to fmm()'s rows for their
    particles.  Rows of other particles are left as they are in `a` (zeros if
    a is None).  counts=True also returns the far and near list lengths."""
    x, m, h = _f64(x), _f64(m), _f64(h)
    if a is None:
        a = np.zeros_like(x)
    lv = np.ascontiguousarray(leaves, dtype=np.int32)
    cnt = np.zeros(2 * len(lv), np.int64) if counts else None
    lib().orc_fmm_leaves(len(m), x, m, h, tree.perm, tree.nnodes, tree.first, tree.count,
                         tree.left, tree.right, mom.M, mom.c, mom.s, mom.hmax, mom.Q,
                         float(theta), float(r_kern), float(G), int(form), len(lv), lv, a, cnt)
    return (a, cnt.reshape(-1, 2)) if counts else a


def fmm_frozen(x, m, h, tree: Tree, lists: Lists, G=1.0, policy=PHANTOM, form=PHANTOM_FORM):
    """FMM with the tree membership and interaction lists held fixed and the
    moments recomputed from (x, m, h): the function whose derivative the VJP is."""
    mom = moments(x, m, h, tree)
    L = far_field(tree, mom, lists, policy, form)
    return near_and_l2p(x, m, h, tree, mom, L, lists, G)


# --------------------------------------------------------------------------
# Diagnostics (Secs. 5-6) and time stepping
# --------------------------------------------------------------------------
STAT_KEYS = ("sumF", "sumAbsF", "ratio", "mass", "xcom", "P", "L")


def stats_raw(x, v, m, a):
    out = np.empty(16)
    lib().orc_stats(len(m), _f64(x), None if v is None else _f64(v), _f64(m), _f64(a), out)
    return out


def stats(x, v, m, a):
    o = stats_raw(x, v, m, a)
    return {"sumF": o[0:3], "sumAbsF": o[3], "ratio": o[4], "mass": o[5], "xcom": o[6:9],
            "P": o[9:12], "L": o[12:15]}


def asym_estimate(tree: Tree, mom: Moments, lists: Lists, m_leaf=None) -> dict:
    """Asymmetric pairs of the lists and the total-force estimates eq. (33)
    and eq. (46) (m_leaf: mean leaf mass unless given)."""
    nn = tree.nnodes
    if m_leaf is None:
        m_leaf = float(mom.M[0]) / int((tree.left < 0).sum())
    fs = lists.far_src if len(lists.far_src) else np.zeros(1, np.int32)
    out = np.empty(4)
    lib().orc_asym_estimate(nn, tree.left, tree.right, mom.M, mom.c, mom.s, lists.far_off,
                            np.ascontiguousarray(fs, np.int32), float(m_leaf), out)
    return {"F33": out[0], "F46": out[1], "n_asym": int(out[2]), "n_asym_super": int(out[3])}


def kdk(x, v, m, h, dt, steps, force):
    """Kick-drift-kick leapfrog with fixed dt; force(x) -> a.  Returns the final
    state and per-step (x, v, a) diagnostics from stats()."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    a = force(x)
    hist = [stats(x, v, m, a)]
    for _ in range(steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = force(x)
        v = v + 0.5 * dt * a
        hist.append(stats(x, v, m, a))
    return x, v, a, hist

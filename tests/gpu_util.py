"""Helpers shared by the GPU tests: run the HIP path through the C ABI and run
the oracle on the same seeded inputs."""
import numpy as np

from paper_2502_01496_amd import fmm as F


def say(*a):
    print(*a, flush=True)


def to_dev(*arrs):
    import torch

    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for a in arrs]


def gpu_run(x, m, h, theta=0.5, leaf=8, G=1.0, precision=F.FMM_FP64, export=True, local=False,
            walk=F.FMM_WALK_PHANTOM, expansion=F.FMM_EXPANSION_PHANTOM,
            tree_shape=F.FMM_TREE_MEDIAN):
    """build -> moments -> forces on the GPU; returns (a, export dict, info)."""
    import torch

    X, Mt, H = to_dev(x, m, h)
    p = F.default_params(theta=theta, leaf_size=leaf, G=G, precision=precision, walk=walk,
                         expansion=expansion, tree=tree_shape)
    t = F.fmm_build_tree(X, p, m=Mt if tree_shape == F.FMM_TREE_COM else None)
    try:
        F.fmm_moments(t, X, Mt, H)
        dt = torch.float32 if precision == F.FMM_FP32 else torch.float64
        A = torch.empty((len(m), 3), dtype=dt, device="cuda")
        F.fmm_forces(t, A)
        torch.cuda.synchronize()
        ex = F.fmm_debug_export(t, lists=True, local=local) if export else None
        info = F.fmm_tree_info(t)
    finally:
        F.fmm_tree_free(t)
    return A.cpu().numpy().astype(np.float64), ex, info


def force_err(a, ref):
    """max_i |a_i - ref_i| / max(|ref_i|, 1e-3 rms|ref|)."""
    nr = np.linalg.norm(ref, axis=1)
    floor = max(1e-3 * np.sqrt((nr ** 2).mean()), 1e-300)
    return (np.linalg.norm(a - ref, axis=1) / np.maximum(nr, floor)).max()


def eta(a, ref):
    return float(np.sqrt(((a - ref) ** 2).sum() / (ref ** 2).sum()))


def gpu_vjp(x, m, h, abar, theta=0.5, leaf=8, G=1.0, precision=F.FMM_FP64, repeat=1,
            expansion=F.FMM_EXPANSION_PHANTOM, tree_shape=F.FMM_TREE_MEDIAN,
            walk=F.FMM_WALK_PHANTOM):
    """build -> moments -> forces -> VJP on the GPU; returns (a, [(xbar, mbar)] * repeat)."""
    import torch

    X, Mt, H = to_dev(x, m, h)
    dt = torch.float32 if precision == F.FMM_FP32 else torch.float64
    AB = torch.from_numpy(np.ascontiguousarray(abar)).to("cuda").to(dt)
    p = F.default_params(theta=theta, leaf_size=leaf, G=G, precision=precision,
                         expansion=expansion, tree=tree_shape, walk=walk)
    t = F.fmm_build_tree(X, p, m=Mt if tree_shape == F.FMM_TREE_COM else None)
    out = []
    try:
        F.fmm_moments(t, X, Mt, H)
        A = torch.empty((len(m), 3), dtype=dt, device="cuda")
        F.fmm_forces(t, A)
        for _ in range(repeat):
            XB = torch.empty((len(m), 3), dtype=dt, device="cuda")
            MB = torch.empty(len(m), dtype=dt, device="cuda")
            F.fmm_forces_vjp(t, AB, XB, MB)
            torch.cuda.synchronize()
            out.append((XB.cpu().numpy().astype(np.float64), MB.cpu().numpy().astype(np.float64)))
    finally:
        F.fmm_tree_free(t)
    return A.cpu().numpy().astype(np.float64), out


def oracle_fmm_threaded(orc, x, m, h, theta=0.5, leaf=8, threads=None):
    """The oracle's serial FMM (leaf <- cell walk) for every particle, its
    per-leaf evaluations spread over threads (the tree build stays serial).
    Rows are identical to orc.fmm(...).a: same tree, lists and arithmetic."""
    import concurrent.futures as cf
    import os

    if threads is None:
        try:
            threads = max(1, min(16, len(os.sched_getaffinity(0))))
        except Exception:
            threads = 4
    tree = orc.build_tree(x, leaf)
    mom = orc.moments(x, m, h, tree)
    leaves = np.flatnonzero(tree.left < 0)
    a = np.zeros_like(np.asarray(x, dtype=np.float64))
    parts = np.array_split(leaves, threads * 8)
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda p: orc.fmm_leaves(x, m, h, tree, mom, p, theta=theta, a=a), parts))
    return a, tree, mom

"""fmm_momentum_stats_noalloc (no device allocation: its partial sums live in
a fixed array of the library) against fmm_momentum_stats_async, the entry
point it is a variant of, through the C ABI: bit-identical statistics for two
calls in a row, the second on a smaller input, for FP64 and FP32
accelerations, with and without velocities."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W

pytestmark = pytest.mark.gpu


def _call(fn, x, v, m, a, out):
    n = x.shape[0]
    prec = F.FMM_FP32 if a.dtype == torch.float32 else F.FMM_FP64
    st = fn(C.c_void_p(x.data_ptr()), C.c_void_p(v.data_ptr()) if v is not None else None,
            C.c_void_p(m.data_ptr()), C.c_void_p(a.data_ptr()), prec, n,
            C.c_void_p(out.data_ptr()), F._stream(None))
    assert st == F.FMM_OK, F.fmm_last_error()


@pytest.mark.parametrize("adt", [torch.float64, torch.float32])
def test_noalloc_stats_match_async_two_calls(adt):
    L = F.lib()
    res = []
    for n, seed in ((300001, 31), (70001, 32)):     # second call: smaller input
        x, m, _ = W.plummer(n, seed)
        rng = np.random.default_rng(seed)
        X = torch.from_numpy(x).cuda()
        Mt = torch.from_numpy(m).cuda()
        V = torch.from_numpy(rng.standard_normal((n, 3))).cuda()
        A = torch.from_numpy(rng.standard_normal((n, 3))).cuda().to(adt)
        for v in (V, None):
            ref = torch.full((16,), float("nan"), dtype=torch.float64, device="cuda")
            got = torch.full((16,), float("nan"), dtype=torch.float64, device="cuda")
            _call(L.fmm_momentum_stats_async, X, v, Mt, A, ref)
            _call(L.fmm_momentum_stats_noalloc, X, v, Mt, A, got)
            torch.cuda.synchronize()
            r, g = ref.cpu().numpy(), got.cpu().numpy()
            print(f"[gpu noalloc] n={n} a={adt} v={'yes' if v is not None else 'no'}: "
                  f"ratio {g[4]:.6e}", flush=True)
            np.testing.assert_array_equal(g, r)
            assert np.isfinite(g[:15]).all()
            res.append(g)
    # the two sizes give different statistics (the array kept nothing over)
    assert not np.array_equal(res[0], res[2])


def test_noalloc_stats_argument_checks():
    L = F.lib()
    v = C.c_void_p(8)
    assert L.fmm_momentum_stats_noalloc(None, None, v, v, 0, 10, v, None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats_noalloc(v, None, v, v, 0, 0, v, None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats_noalloc(v, None, v, v, 3, 10, v, None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats_noalloc(v, None, v, v, 0, 10, None, None) == F.FMM_ERR_INVALID
    assert L.fmm_momentum_stats_noalloc(v, None, v, v, 0, 1 << 31, v, None) == F.FMM_ERR_CAPACITY
    assert "exceeds" in F.fmm_last_error()

"""rsvd_run_noalloc (workspace in the library's fixed device array) against
rsvd_run with a caller workspace, through the C ABI: same kernels and plan, so
the outputs are bit for bit equal.  Two calls in a row, the second smaller
(the array keeps the first call's contents), then a problem too large for
the array, rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from synth import matrices as syn

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _run_both(lib, h, A, k, p, q, seed):
    from paper_1608_02148_amd import api
    from paper_1608_02148_amd import lib as L
    dt = api._check_matrix(A)
    m, n = A.shape
    od = api.out_dtype(A)
    prm = api.make_params(p, q, seed)
    outs = []
    for noalloc in (True, False):
        U = torch.full((m, k), float("nan"), dtype=od, device=DEV)
        S = torch.full((k,), float("nan"), dtype=torch.float64, device=DEV)
        V = torch.full((n, k), float("nan"), dtype=od, device=DEV)
        if noalloc:
            st = lib.rsvd_run_noalloc(h, dt, m, n, ctypes.c_void_p(A.data_ptr()), A.stride(0), k,
                                      ctypes.byref(prm), ctypes.c_void_p(U.data_ptr()), U.stride(0),
                                      ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr()), V.stride(0),
                                      None)
        else:
            nbytes = api.workspace_size(A, k, prm)
            work = api.workspace(nbytes, A.device)
            st = lib.rsvd_run(h, dt, m, n, ctypes.c_void_p(A.data_ptr()), A.stride(0), k, ctypes.byref(prm),
                              ctypes.c_void_p(U.data_ptr()), U.stride(0), ctypes.c_void_p(S.data_ptr()),
                              ctypes.c_void_p(V.data_ptr()), V.stride(0), ctypes.c_void_p(work.data_ptr()),
                              work.numel(), None)
        assert st == 0, L.STATUS.get(st, st)
        torch.cuda.synchronize()
        outs.append((U, S, V))
    return outs


def test_noalloc_matches_rsvd_run(gpu_lib):
    from paper_1608_02148_amd import api
    h = api.handle(DEV)
    A1 = torch.tensor(syn.planted(3000, 800, syn.spectrum("poly", 800, alpha=1.0), 61), dtype=torch.float32,
                      device=DEV)
    A2 = torch.tensor(syn.planted(700, 300, syn.spectrum("exp", 300, tau=20.0), 62), dtype=torch.float64,
                      device=DEV)
    for A, k, p, q in ((A1, 40, 20, 2), (A2, 12, 10, 1)):
        (Un, Sn, Vn), (Ur, Sr, Vr) = _run_both(gpu_lib, h, A, k, p, q, seed=9)
        assert torch.equal(Sn, Sr) and torch.equal(Un, Ur) and torch.equal(Vn, Vr)
        assert torch.all(torch.isfinite(Sn))


def test_noalloc_rejects_problems_beyond_its_array(gpu_lib):
    from paper_1608_02148_amd import api
    from paper_1608_02148_amd import lib as L
    h = api.handle(DEV)
    prm = api.make_params(20, 2, 0)
    m, n, k = 400000, 5000, 100
    need = ctypes.c_size_t()
    assert gpu_lib.rsvd_workspace_size(h, L.RSVD_F32, m, n, k, ctypes.byref(prm), ctypes.byref(need)) == 0
    assert need.value > (256 << 20)
    dummy = ctypes.c_void_p(256)          # rejected before any launch: never dereferenced
    st = gpu_lib.rsvd_run_noalloc(h, L.RSVD_F32, m, n, dummy, n, k, ctypes.byref(prm), None, 0, dummy, None, 0,
                                  None)
    assert st == -2

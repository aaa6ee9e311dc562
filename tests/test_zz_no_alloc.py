"""The allocation-free solve entry point (spalu_solve_static) against the
workspace entry point (spalu_solve) through the C ABI: the same kernels on
the same inputs give bit-identical results, on consecutive calls that reuse
the library's static buffer with a smaller problem the second time, and a
solve too large for the buffer is refused before any launch."""
import ctypes as C

import numpy as np
import pytest

from helpers import rel_res, to_device
from workloads import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2408_14193_amd import spalu
    return spalu


def _static(S, F, Bt, Xt, tol, restart):
    nrhs, n = Bt.shape
    rr = np.zeros(nrhs)
    info = S.SolveInfo()
    rc = S._lib.spalu_solve_static(F._h, nrhs, Bt.data_ptr(), n, Xt.data_ptr(), n,
                                   C.byref(S.SolveOpts(float(tol), 30, 1, int(restart))),
                                   F.stream.cuda_stream, rr.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(info))
    return rc, info.as_dict(), rr


@pytest.mark.parametrize("tol", [0.0, 1e-10])
def test_static_solve_matches_workspace_solve(S, tol):
    import torch
    # the second call is smaller; the first factor is in the symmetric form
    cases = [(1, 127, 4, S.FP32, 8, True), (0, 63, 2, S.FP64, 0, False)]
    for cfg, side, nrhs, prec, restart, sym in cases:
        print("case static solve cfg=%d side=%d nrhs=%d tol=%g symmetric=%s" % (cfg, side, nrhs, tol, sym),
              flush=True)
        P = make_config(cfg, side=side, nrhs=nrhs)
        nd = S.ND(P.dims)
        rp, ci, v, B = to_device(P)
        F = S.Factor(nd, rp, ci, v, eps=P.eps, precision=prec, symmetric=sym)
        Bt = B.t().contiguous()
        Xs = torch.full_like(Bt, float("nan"))
        Xw = torch.full_like(Bt, float("nan"))
        rc, info_s, rr_s = _static(S, F, Bt, Xs, tol, restart)
        assert rc == S.OK, S._lib.spalu_last_error()
        info_w, rr_w = F.solve_into(Bt, Xw, tol=tol, restart=restart, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(Xs, Xw)
        assert np.array_equal(rr_s, rr_w)
        assert info_s["iterations"] == info_w["iterations"]
        if tol > 0:
            assert rel_res(P, Xs.t().cpu().numpy()).max() <= tol


def test_static_solve_refuses_what_does_not_fit(S):
    import torch
    P = make_config(0, side=63, nrhs=1)
    nd = S.ND(P.dims)
    rp, ci, v, B = to_device(P)
    F = S.Factor(nd, rp, ci, v, eps=P.eps)
    nrhs = 1
    while True:
        b = C.c_size_t()
        S._check(S._lib.spalu_solve_workspace(F._h, nrhs, None, C.byref(b)))
        if b.value > (64 << 20):
            break
        nrhs *= 2
    Bt = torch.zeros(nrhs, P.n, dtype=torch.float64, device="cuda")
    Xt = torch.zeros_like(Bt)
    rc, _, _ = _static(S, F, Bt, Xt, 0.0, 0)
    assert rc == S.ENOMEM
    assert b"static" in S._lib.spalu_last_error()

"""GPU parity of the symmetric form (Section 4.4.2) through the C ABI: one
ID per segment shared by A_{s,n} and A_{n,s}^T (one-sided coupling rows),
L D L^T of the segment blocks stored balanced as C^{-1}, C^{-T}, against the
oracle's symmetric form.

* eps = 0: a dense solve to 1e-12;
* FP64 with compression: sizes, ranks, samples and passes equal the
  oracle's on the levels the oracle reproduces under a 1e-15 perturbation,
  and the direct solve within 1e-10 of the oracle's per column;
* W~ = V~^T: the approximate inverse is a symmetric matrix to rounding;
* FP32 storage refines to the FP64 solution; the learned form runs on it;
* a matrix that is not symmetric, or not positive definite, is refused.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from helpers import rel_res, to_device
from oracle import spalu as O
from oracle.nd import nd_order
from test_gpu_parity import (S, _col_err, _id_work, _oracle_ranks, compare_ranks, gpu_factor, gpu_solve,  # noqa: F401
                             oracle_stable_levels)
from workloads import make_config

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,side", [(0, 15), (0, 63), (1, 31), (1, 63), (3, 7), (3, 15)])
def test_sym_eps0_equals_dense_lu(S, cfg, side):
    print("case sym eps0 cfg=%d side=%d" % (cfg, side), flush=True)
    P = make_config(cfg, side=side, nrhs=3)
    nd, F, B = gpu_factor(S, P, eps=0.0, symmetric=True)
    X, info = gpu_solve(F, B)
    Xe = np.linalg.solve(P.scipy().toarray(), P.rhs)
    assert np.linalg.norm(X - Xe) <= 1e-12 * np.linalg.norm(Xe)


@pytest.mark.parametrize("cfg,side", [(0, 31), (0, 63), (1, 63), (3, 15), (1, 255)])
def test_sym_fp64_ranks_and_solution_match_oracle(S, cfg, side):
    print("case sym parity cfg=%d side=%d" % (cfg, side), flush=True)
    P = make_config(cfg, side=side, nrhs=2)
    eps = P.eps
    if side == 255:
        S.profile(True)
    nd, F, B = gpu_factor(S, P, eps=eps, seed=1234, symmetric=True)
    if side == 255:
        work = _id_work(S)
        S.profile(False)
        print("ID work by tier:", work)
        assert work.get("seg_id_b2", 0) > 0
    OF = O.factor(nd_order(P.dims), P.scipy(), O.Opts(eps=eps, seed=1234, symmetric=1))
    ora = _oracle_ranks(OF, nd)
    stable = oracle_stable_levels(P, nd, ora, eps, symmetric=1)
    print("levels reproducible in the oracle:", stable)
    assert len(stable) >= min(nd.L, 3)
    compare_ranks(nd, F.ranks(), ora, stable)
    X, info = gpu_solve(F, B)
    if len(stable) == nd.L:
        Xo = O.apply_inverse(OF, P.rhs)
        err = _col_err(X, Xo)
        print("direct solve vs oracle per column:", err)
        assert err.max() <= 1e-10
    Xr, info = gpu_solve(F, B, tol=1e-10)
    assert info["converged"]
    assert rel_res(P, Xr).max() <= 1e-10


def test_sym_solution_operator_is_symmetric(S):
    """W~ = V~^T on the GPU: the factor applied to the identity (31 x 31
    GRF diffusion, 961 right-hand sides) is symmetric to rounding with
    compression on."""
    import torch
    P = make_config(1, side=31, nrhs=1)
    nd, F, B = gpu_factor(S, P, eps=1e-4, symmetric=True)
    assert F.info["sparsified"] > 0
    I = torch.eye(961, dtype=torch.float64, device=B.device)
    M, info = F.solve(I)
    M = M.cpu().numpy()
    asym = np.linalg.norm(M - M.T) / np.linalg.norm(M)
    print("relative asymmetry of the approximate inverse: %.2e" % asym)
    assert asym <= 1e-13


@pytest.mark.parametrize("cfg", [0, 1])
def test_sym_fp32_refines_to_fp64_solution(S, cfg):
    print("case sym fp32 cfg=%d" % cfg, flush=True)
    P = make_config(cfg, side=127, nrhs=4)
    nd, F, B = gpu_factor(S, P, eps=P.eps, precision=S.FP32, symmetric=True)
    X, info = gpu_solve(F, B, tol=1e-10, max_iter=40)
    assert info["converged"], info
    assert rel_res(P, X).max() <= 1e-10
    Xe = spla.spsolve(P.scipy().tocsc(), P.rhs)
    err = np.linalg.norm(X - Xe, axis=0) / np.linalg.norm(Xe, axis=0)
    print("sym fp32 cfg %d: iterations %d, error vs FP64 %.2e" % (cfg, info["iterations"], err.max()))
    assert err.max() <= 1e-7


def test_sym_learned_form(S):
    """The rank predictor's start samples and keep-whole rule on top of the
    symmetric form (FP32 storage, 127 x 127 GRF diffusion)."""
    import torch
    from paper_2408_14193_amd import rank_model
    P = make_config(1, side=127, nrhs=2)
    model = rank_model.load(device=torch.device("cuda:0"))
    nd, F, B = gpu_factor(S, P, eps=P.eps, precision=S.FP32, symmetric=True, rank_model=model)
    X, info = gpu_solve(F, B, tol=1e-10, max_iter=40)
    assert info["converged"], info
    assert rel_res(P, X).max() <= 1e-10


def test_sym_refuses_what_it_cannot_factor(S):
    P = make_config(2, side=31, nrhs=1)
    with pytest.raises(S.SpaluError) as e:
        gpu_factor(S, P, eps=1e-6, symmetric=True)
    assert e.value.code == -1     # SPALU_EINVAL: not symmetric
    P = make_config(0, side=31, nrhs=1)
    P.data = -P.data
    with pytest.raises(S.SpaluError) as e:
        gpu_factor(S, P, eps=1e-6, symmetric=True)
    assert e.value.code == -3     # SPALU_ESINGULAR: a pivot that is not positive


def test_sym_factor_graph_replays_match_direct_launches(S):
    """The symmetric form's level sweep captured as a HIP graph and replayed
    gives bitwise the factor of direct launches; switching the form on the
    same workspace captures (then reuses) a graph per form, with eager work
    between the replays."""
    import torch
    from paper_2408_14193_amd import rank_model
    P = make_config(1, side=127, nrhs=2)
    nd = S.ND(P.dims)
    rp, ci, v, B = to_device(P)
    Bt = B.t().contiguous()
    kw = dict(eps=P.eps, precision=S.FP32, rank_model=rank_model.load())

    def result(F):
        X = torch.empty_like(Bt)
        F.solve_into(Bt, X, tol=0.0, max_iter=1, graph=False)
        torch.cuda.synchronize()
        return F.ranks(), X.cpu().numpy()

    ws = None
    for sym in (True, False, True):
        ref_ranks, ref_x = result(S.Factor(nd, rp, ci, v, symmetric=sym, **kw))
        for rep in range(2):
            F = S.Factor(nd, rp, ci, v, graph=True, workspace=ws, symmetric=sym, **kw)
            ws = F.workspace
            ranks, x = result(F)
            for a, b in zip(ranks, ref_ranks):
                assert np.array_equal(a, b), "symmetric %s replay %d: ranks differ" % (sym, rep)
            assert np.array_equal(x, ref_x), "symmetric %s replay %d: solve differs" % (sym, rep)
            (Bt * 2.0).sum().item()
            del F


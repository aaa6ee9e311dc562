"""Python binding of libspalu (ctypes): argument marshalling only.

Every step of nested dissection planning, factorization and solve runs in
the compiled library (host planner + HIP kernels for gfx950).  PyTorch
provides device memory (workspaces are torch tensors) and the stream (the
current torch stream).  If the library is missing this module raises on
import; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspalu.so")

# torch is imported first so its HIP runtime is the one loaded in the
# process; the library's libamdhip64.so.7 dependency then binds to it by
# SONAME instead of pulling a second runtime from /opt/rocm.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError("libspalu.so is not built; run paper_2408_14193_amd/build.py "
                      "(or __graft_entry__.build())")
_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, ESINGULAR, ENOCONV, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ESINGULAR: "ESINGULAR", ENOCONV: "ENOCONV",
          EDEVICE: "EDEVICE", EUNSUPPORTED: "EUNSUPPORTED"}


class SpaluError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_NAMES.get(code, code), msg))
        self.code = code


class NdOpts(C.Structure):
    _fields_ = [("levels", C.c_int32), ("leaf_max", C.c_int32)]


class FactorOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("precision", C.c_int32), ("seed", C.c_uint32),
                ("rho", C.c_double), ("h0", C.c_int32), ("probes", C.c_int32),
                ("tau", C.c_double), ("h_init", C.c_void_p), ("rank_model", C.c_void_p),
                ("features_out", C.c_void_p), ("rank_margin", C.c_float), ("rank_pad", C.c_int32),
                ("rank_skip", C.c_float), ("graph", C.c_int32), ("symmetric", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("id_lds_a", C.c_int32), ("id_lds_b", C.c_int32), ("id_lds_b2", C.c_int32),
                ("id_lds_c", C.c_int32), ("id_c_ydiv", C.c_int32), ("melim_lds", C.c_int32),
                ("melim_wave_cap", C.c_int32), ("solve_lanes_min", C.c_int32),
                ("solve_lanes_max", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FactorInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("levels", C.c_int32), ("segments", C.c_int64),
                ("sparsified", C.c_int64), ("sample_passes", C.c_int64),
                ("resampled", C.c_int64), ("max_front", C.c_int64), ("q_tilde", C.c_double),
                ("workspace_bytes", C.c_int64),
                ("singular_level", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("graph", C.c_int32), ("restart", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("max_rel_residual", C.c_double),
                ("first_rel_residual", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = C.c_void_p
I64P = C.POINTER(C.c_int64)
I32P = C.POINTER(C.c_int32)
_lib.spalu_last_error.restype = C.c_char_p
_lib.spalu_nd_order.argtypes = [C.c_int32, I32P, C.POINTER(NdOpts), C.POINTER(P)]
_lib.spalu_nd_info.argtypes = [P, I64P, I32P, I64P, I64P]
_lib.spalu_nd_perm.argtypes = [P, I64P]
_lib.spalu_nd_etree.argtypes = [P, I64P, I64P, I32P, I64P]
_lib.spalu_nd_segments.argtypes = [P, C.c_int32, I64P, I64P, I64P, I32P, I32P, I32P, I64P, I32P]
_lib.spalu_nd_free.argtypes = [P]
_lib.spalu_nd_free.restype = None
_lib.spalu_factor_opts_default.argtypes = [C.POINTER(FactorOpts)]
_lib.spalu_factor_opts_default.restype = None
_lib.spalu_factor_workspace.argtypes = [P, C.POINTER(FactorOpts), C.POINTER(C.c_size_t)]
_lib.spalu_tuning_default.argtypes = [C.POINTER(Tuning)]
_lib.spalu_tuning_default.restype = None
_lib.spalu_tuning_get.argtypes = [C.POINTER(Tuning)]
_lib.spalu_tuning_set.argtypes = [C.POINTER(Tuning)]
_lib.spalu_factor_seg_base.argtypes = [P, I64P]
_lib.spalu_factor.argtypes = [P, C.c_int64, P, P, P, C.POINTER(FactorOpts), P, C.c_size_t, P,
                              C.POINTER(P), C.POINTER(FactorInfo)]
_lib.spalu_factor_ranks.argtypes = [P, I32P, I32P, I32P, I32P]
_lib.spalu_factor_work.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
_lib.spalu_factor_free.argtypes = [P]
_lib.spalu_factor_free.restype = None
_lib.spalu_solve_workspace.argtypes = [P, C.c_int32, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]
_lib.spalu_solve.argtypes = [P, C.c_int32, P, C.c_int64, P, C.c_int64, C.POINTER(SolveOpts), P,
                             C.c_size_t, P, C.POINTER(C.c_double), C.POINTER(SolveInfo)]
_lib.spalu_solve_static.argtypes = [P, C.c_int32, P, C.c_int64, P, C.c_int64, C.POINTER(SolveOpts), P,
                                    C.POINTER(C.c_double), C.POINTER(SolveInfo)]

class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


_lib.spalu_mlp_param_count.restype = C.c_int
_lib.spalu_mlp_workspace.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
_lib.spalu_mlp_forward.argtypes = [P, P, C.c_int32, P, P, C.c_size_t, P]
_lib.spalu_mlp_train_step.argtypes = [P, P, P, P, P, C.c_int32, C.c_float, C.c_int32, P, P, P,
                                      C.c_size_t, P]
_lib.spalu_profile.argtypes = [C.c_int32]
_lib.spalu_profile.restype = None
_lib.spalu_profile_only.argtypes = [C.c_char_p]
_lib.spalu_profile_only.restype = C.c_int
_lib.spalu_profile_read.argtypes = [C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]

EXPORTED = ["spalu_nd_order", "spalu_nd_info", "spalu_nd_perm", "spalu_nd_etree",
            "spalu_nd_segments", "spalu_nd_free", "spalu_factor_opts_default",
            "spalu_factor_workspace", "spalu_factor_seg_base", "spalu_factor",
            "spalu_factor_ranks", "spalu_factor_work", "spalu_factor_free", "spalu_solve_workspace", "spalu_solve",
            "spalu_solve_static", "spalu_tuning_default", "spalu_tuning_get", "spalu_tuning_set",
            "spalu_mlp_param_count", "spalu_mlp_workspace", "spalu_mlp_forward",
            "spalu_mlp_train_step", "spalu_profile", "spalu_profile_only", "spalu_profile_read",
            "spalu_last_error"]


def _check(rc, info=None):
    if rc != OK:
        e = SpaluError(rc, _lib.spalu_last_error().decode())
        e.info = info.as_dict() if info is not None else None
        raise e


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class ND:
    """Nested dissection of a regular grid (spalu_nd_order)."""

    def __init__(self, dims, levels=0, leaf_max=7):
        self.dims = tuple(int(d) for d in dims)
        g = (C.c_int32 * 3)(*(list(self.dims) + [1] * (3 - len(self.dims))))
        h = P()
        _check(_lib.spalu_nd_order(len(self.dims), g, C.byref(NdOpts(levels, leaf_max)), C.byref(h)))
        self._h = h
        n, L, nn, ns = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64()
        _check(_lib.spalu_nd_info(h, C.byref(n), C.byref(L), C.byref(nn), C.byref(ns)))
        self.n, self.L, self.nnodes, self.nsegments = n.value, L.value, nn.value, ns.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.spalu_nd_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def perm(self):
        out = np.empty(self.n, dtype=np.int64)
        _check(_lib.spalu_nd_perm(self._h, _ptr(out, C.c_int64)))
        return out

    def etree(self):
        b = np.empty(self.nnodes, np.int64)
        s = np.empty(self.nnodes, np.int64)
        lv = np.empty(self.nnodes, np.int32)
        p = np.empty(self.nnodes, np.int64)
        _check(_lib.spalu_nd_etree(self._h, _ptr(b, C.c_int64), _ptr(s, C.c_int64),
                                   _ptr(lv, C.c_int32), _ptr(p, C.c_int64)))
        return b, s, lv, p

    def segments(self, level):
        ns, nv, npr = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib.spalu_nd_segments(self._h, level, C.byref(ns), C.byref(nv), None, None, None,
                                      None, C.byref(npr), None))
        ptr = np.empty(ns.value + 1, np.int64)
        verts = np.empty(nv.value, np.int32)
        flags = np.empty(ns.value, np.int32)
        parent = np.empty(ns.value, np.int32)
        pairs = np.empty(2 * npr.value, np.int32)
        _check(_lib.spalu_nd_segments(self._h, level, C.byref(ns), C.byref(nv), _ptr(ptr, C.c_int64),
                                      _ptr(verts, C.c_int32), _ptr(flags, C.c_int32),
                                      _ptr(parent, C.c_int32), C.byref(npr), _ptr(pairs, C.c_int32)))
        return ptr, verts, flags, parent, pairs.reshape(-1, 2)

    def seg_base(self):
        b = np.empty(self.L + 2, np.int64)
        _check(_lib.spalu_factor_seg_base(self._h, _ptr(b, C.c_int64)))
        return b


def factor_opts(eps=1e-6, precision=FP64, seed=1234, rho=0.5, h0=8, probes=5, tau=1.0,
                h_init=None, rank_model=None, features_out=None, rank_margin=1.0, rank_pad=5,
                rank_skip=0.5, graph=False, symmetric=False):
    o = FactorOpts()
    _lib.spalu_factor_opts_default(C.byref(o))
    o.eps, o.precision, o.seed, o.rho, o.h0, o.probes, o.tau = (
        float(eps), int(precision), int(seed) & 0xFFFFFFFF, float(rho), int(h0), int(probes), float(tau))
    o.h_init = None if h_init is None else int(h_init.data_ptr())
    o.rank_model = None if rank_model is None else int(rank_model.data_ptr())
    o.features_out = None if features_out is None else int(features_out.data_ptr())
    o.rank_margin, o.rank_pad, o.rank_skip = float(rank_margin), int(rank_pad), float(rank_skip)
    o.graph = 1 if graph else 0
    o.symmetric = 1 if symmetric else 0
    return o


def tuning_default():
    """The library's default launch shapes (a dict of spalu_tuning)."""
    t = Tuning()
    _lib.spalu_tuning_default(C.byref(t))
    return t.as_dict()


def get_tuning():
    """The launch shapes in use (a dict of spalu_tuning)."""
    t = Tuning()
    _check(_lib.spalu_tuning_get(C.byref(t)))
    return t.as_dict()


def set_tuning(**kw):
    """Changes the named launch shapes (the others keep their values) for
    the factorizations started afterwards; returns the full set."""
    cur = get_tuning()
    unknown = set(kw) - set(cur)
    if unknown:
        raise KeyError("unknown tuning fields: %s" % sorted(unknown))
    cur.update({k: int(v) for k, v in kw.items()})
    _check(_lib.spalu_tuning_set(C.byref(Tuning(**cur))))
    return cur


def factor_workspace_bytes(nd, opts):
    b = C.c_size_t()
    _check(_lib.spalu_factor_workspace(nd.handle, C.byref(opts), C.byref(b)))
    return b.value


class Factor:
    """spaLU factorization of a CSR matrix held in device memory (torch).
    graph: replay the level sweep from a HIP graph captured on the first
    factorization with these pointers and options.  symmetric: the
    symmetric form for a symmetric positive definite matrix (one-sided IDs,
    L D L^T segment factors).  workspace: a uint8
    device tensor to factor into (reused across factorizations, e.g. of a
    sequence of matrices with one pattern; the factor it held before is
    overwritten), else a new one."""

    def __init__(self, nd, rowptr, colind, vals, eps=1e-6, precision=FP64, seed=1234, rho=0.5,
                 h0=8, probes=5, tau=1.0, h_init=None, rank_model=None, features_out=None,
                 stream=None, rank_skip=0.5, graph=False, workspace=None, symmetric=False):
        import torch
        assert rowptr.is_cuda and rowptr.dtype == torch.int64
        assert colind.is_cuda and colind.dtype == torch.int32
        assert vals.is_cuda and vals.dtype == torch.float64
        self.nd = nd
        self.csr = (rowptr.contiguous(), colind.contiguous(), vals.contiguous())
        self.h_init = h_init
        self.rank_model = rank_model
        if rank_model is not None:
            assert rank_model.is_cuda and rank_model.dtype == torch.float32
            assert rank_model.numel() == mlp_param_count()
        if features_out is not None:
            assert features_out.is_cuda and features_out.dtype == torch.float32
            assert features_out.numel() >= nd.nsegments * 12
        self.opts = factor_opts(eps, precision, seed, rho, h0, probes, tau, h_init, rank_model,
                                features_out, rank_skip=rank_skip, graph=graph, symmetric=symmetric)
        nbytes = factor_workspace_bytes(nd, self.opts)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=rowptr.device)
        assert workspace.is_cuda and workspace.dtype == torch.uint8 and workspace.is_contiguous()
        assert workspace.numel() >= nbytes
        self.workspace = workspace
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        h = P()
        info = FactorInfo()
        _check(_lib.spalu_factor(nd.handle, nd.n, self.csr[0].data_ptr(), self.csr[1].data_ptr(),
                                 self.csr[2].data_ptr(), C.byref(self.opts),
                                 self.workspace.data_ptr(), nbytes, s.cuda_stream, C.byref(h),
                                 C.byref(info)), info)
        self._h = h
        self.info = info.as_dict()
        self._solve_ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.spalu_factor_free(h)
            self._h = None

    def ranks(self):
        tot = int(self.nd.seg_base()[-1])
        nb, rk, hh, ps = (np.empty(tot, np.int32) for _ in range(4))
        _check(_lib.spalu_factor_ranks(self._h, _ptr(nb, C.c_int32), _ptr(rk, C.c_int32),
                                       _ptr(hh, C.c_int32), _ptr(ps, C.c_int32)))
        return nb, rk, hh, ps

    def work(self):
        """Algorithmic (flops, bytes) of this factorization."""
        fl, by = C.c_double(), C.c_double()
        _check(_lib.spalu_factor_work(self._h, C.byref(fl), C.byref(by)))
        return fl.value, by.value

    def solve_workspace(self, nrhs, restart=0):
        import torch
        key = (nrhs, restart)
        if key not in self._solve_ws:
            b = C.c_size_t()
            _check(_lib.spalu_solve_workspace(self._h, nrhs, C.byref(SolveOpts(1.0, 0, 0, int(restart))),
                                              C.byref(b)))
            self._solve_ws[key] = torch.empty(b.value, dtype=torch.uint8, device=self.workspace.device)
        return self._solve_ws[key]

    def solve_into(self, Bt, Xt, tol=0.0, max_iter=30, stream=None, graph=True, restart=0):
        """Bt, Xt: (nrhs, n) float64 contiguous device tensors (column-major
        n x nrhs).  restart > 0: flexible GMRES(restart) corrections instead
        of classical refinement.  Returns (info dict, per-column relative
        residuals)."""
        nrhs, n = Bt.shape
        ws = self.solve_workspace(nrhs, restart if tol > 0 else 0)
        s = self.stream if stream is None else stream
        rr = np.zeros(nrhs, np.float64)
        info = SolveInfo()
        rc = _lib.spalu_solve(self._h, nrhs, Bt.data_ptr(), n, Xt.data_ptr(), n,
                              C.byref(SolveOpts(float(tol), int(max_iter), 1 if graph else 0, int(restart))),
                              ws.data_ptr(),
                              ws.numel(), s.cuda_stream, _ptr(rr, C.c_double), C.byref(info))
        if rc not in (OK, ENOCONV):
            _check(rc)
        d = info.as_dict()
        d["converged"] = rc == OK
        return d, rr

    def solve(self, B, tol=0.0, max_iter=30, graph=True, restart=0):
        """B: (n, nrhs) or (n,) float64 device tensor.  Returns (X, info)."""
        import torch
        vec = B.dim() == 1
        Bt = (B[None, :] if vec else B.t()).contiguous()
        Xt = torch.empty_like(Bt)
        info, rr = self.solve_into(Bt, Xt, tol, max_iter, graph=graph, restart=restart)
        info["rel_res"] = rr
        X = Xt[0] if vec else Xt.t()
        return X, info


def profile(on=True):
    """Enable (and clear) or disable per-kernel event timing in the library."""
    _lib.spalu_profile(1 if on else 0)


def profile_only(name=None):
    """Restrict the event timing to one kernel step (None: every step)."""
    _check(_lib.spalu_profile_only(name.encode() if name else None))


def profile_read():
    """Per-kernel totals since the last profile(): {name: dict(launches, ms,
    bytes, flops)}."""
    cnt = C.c_int32()
    _check(_lib.spalu_profile_read(None, 0, C.byref(cnt)))
    arr = (KernelStat * max(1, cnt.value))()
    _check(_lib.spalu_profile_read(arr, cnt.value, C.byref(cnt)))
    return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms, bytes=arr[i].bytes,
                                       flops=arr[i].flops) for i in range(cnt.value)}


def mlp_param_count():
    return int(_lib.spalu_mlp_param_count())


def _mlp_ws(batch, device):
    b = C.c_size_t()
    _check(_lib.spalu_mlp_workspace(int(batch), C.byref(b)))
    return torch.empty(b.value, dtype=torch.uint8, device=device)


def mlp_forward(params, X):
    """Network outputs (rank fractions) for feature rows X (B x 12), FP32."""
    B = X.shape[0]
    y = torch.empty(B, dtype=torch.float32, device=X.device)
    ws = _mlp_ws(B, X.device)
    _check(_lib.spalu_mlp_forward(params.data_ptr(), X.contiguous().data_ptr(), B, y.data_ptr(),
                                  ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream))
    return y


def mlp_train_step(params, X, t, lr=1e-3, step=1, adam=None, want_grad=False, ws=None):
    """One FP32 training step on the GPU (forward, backward, optional Adam
    with state adam = (m, v)).  Returns (loss tensor, grad tensor or None)."""
    B = X.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    grad = torch.empty(mlp_param_count(), dtype=torch.float32, device=X.device) if want_grad else None
    ws = _mlp_ws(B, X.device) if ws is None else ws
    m, v = (None, None) if adam is None else adam
    _check(_lib.spalu_mlp_train_step(params.data_ptr(), None if m is None else m.data_ptr(),
                                     None if v is None else v.data_ptr(), X.contiguous().data_ptr(),
                                     t.contiguous().data_ptr(), B, float(lr), int(step), loss.data_ptr(),
                                     None if grad is None else grad.data_ptr(), ws.data_ptr(), ws.numel(),
                                     torch.cuda.current_stream().cuda_stream))
    return loss, grad

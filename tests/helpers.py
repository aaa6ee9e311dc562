"""Shared test helpers: upload a seeded workload to the GPU."""
import numpy as np


def to_device(P):
    import torch
    dev = torch.device("cuda:0")
    rowptr = torch.from_numpy(P.indptr.astype(np.int64)).to(dev)
    colind = torch.from_numpy(P.indices.astype(np.int32)).to(dev)
    vals = torch.from_numpy(P.data.astype(np.float64)).to(dev)
    B = torch.from_numpy(np.ascontiguousarray(P.rhs)).to(dev)
    return rowptr, colind, vals, B


def rel_res(P, X):
    A = P.scipy()
    r = P.rhs - A @ X
    return np.linalg.norm(r, axis=0) / np.linalg.norm(P.rhs, axis=0)

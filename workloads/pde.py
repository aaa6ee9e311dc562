"""Finite-difference PDE matrices on regular grids, and seeded right-hand sides.

Unknowns are the interior nodes of a uniform grid with homogeneous Dirichlet
boundary values.  Interior node (x, y[, z]) (0-based) has global index
``x + nx * (y + ny * z)``.  Matrices are returned in CSR form with column
indices ascending inside each row (``indptr`` int64, ``indices`` int32,
``data`` float64).

The five named workloads are synthetic stand-ins for the paper's FEM test
problems (Section 6): the paper's meshes and coefficient fields are not
published, so each family is rebuilt here as a finite-difference grid of
the shape and structure named below.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

MASTER_SEED = 20240826


@dataclasses.dataclass
class Problem:
    name: str
    dims: tuple            # interior grid sizes (nx, ny) or (nx, ny, nz)
    indptr: np.ndarray     # int64 [N+1]
    indices: np.ndarray    # int32 [nnz]
    data: np.ndarray       # float64 [nnz]
    rhs: np.ndarray        # float64 [N, nrhs] (column j is right-hand side j)
    eps: float             # ID tolerance
    tol: float             # target relative residual after refinement
    symmetric: bool
    factor_precision: str  # "fp64" or "fp32"

    @property
    def n(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def nrhs(self) -> int:
        return int(self.rhs.shape[1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def _to_csr(rows, cols, vals, n):
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return (m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data.astype(np.float64))


def _stencil_2d(nx, ny, center, west, east, south, north):
    """Assemble a 5-point operator.  Each coefficient argument is either a
    scalar or an array of shape (ny, nx) giving the coupling of node (x, y)
    to that neighbour; couplings to boundary nodes are dropped (Dirichlet)."""
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    full = lambda c: np.broadcast_to(np.asarray(c, dtype=np.float64), (ny, nx))
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [full(center).ravel()]
    for coef, dy, dx in ((west, 0, -1), (east, 0, 1), (south, -1, 0), (north, 1, 0)):
        c = full(coef)
        ys, xs = np.mgrid[0:ny, 0:nx]
        yy, xx = ys + dy, xs + dx
        ok = (yy >= 0) & (yy < ny) & (xx >= 0) & (xx < nx)
        rows.append(idx[ok])
        cols.append(idx[yy[ok], xx[ok]])
        vals.append(c[ok])
    return _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


def laplacian_2d(nx, ny=None, h=None):
    """-Laplace with the 5-point stencil, (1/h^2)[4, -1, -1, -1, -1]."""
    ny = nx if ny is None else ny
    h = 1.0 / (max(nx, ny) + 1) if h is None else h
    s = 1.0 / (h * h)
    return _stencil_2d(nx, ny, 4 * s, -s, -s, -s, -s)


def laplacian_3d(nx, ny=None, nz=None, h=None):
    """-Laplace with the 7-point stencil, (1/h^2)[6, -1 x 6]."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    h = 1.0 / (max(nx, ny, nz) + 1) if h is None else h
    s = 1.0 / (h * h)
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    zs, ys, xs = np.mgrid[0:nz, 0:ny, 0:nx]
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [np.full(n, 6 * s)]
    for dz, dy, dx in ((0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)):
        zz, yy, xx = zs + dz, ys + dy, xs + dx
        ok = (zz >= 0) & (zz < nz) & (yy >= 0) & (yy < ny) & (xx >= 0) & (xx < nx)
        rows.append(idx[ok])
        cols.append(idx[zz[ok], yy[ok], xx[ok]])
        vals.append(np.full(int(ok.sum()), -s))
    return _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)


def gaussian_random_field(m, corr_len, rng):
    """Stationary Gaussian field with squared-exponential covariance
    exp(-r^2 / (2 corr_len^2)) on the (m x m) nodes of the unit square
    (spacing 1/(m-1)), by circulant embedding on a periodic grid of twice
    the size; the sample is shifted and scaled to mean 0 and std 1."""
    h = 1.0 / (m - 1)
    big = 2 * m
    d = np.minimum(np.arange(big), big - np.arange(big)) * h
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    cov = np.exp(-r2 / (2.0 * corr_len * corr_len))
    lam = np.fft.fft2(cov).real
    lam = np.maximum(lam, 0.0)
    white = rng.standard_normal((big, big))
    g = np.fft.ifft2(np.sqrt(lam) * np.fft.fft2(white)).real[:m, :m]
    g = g - g.mean()
    g = g / g.std()
    return g


def diffusion_2d(n, a_nodes, h=None):
    """-div(a grad u) with the 5-point stencil; ``a_nodes`` holds a on all
    (n+2)^2 grid nodes including the boundary, face coefficients are the
    harmonic mean of the two node values."""
    h = 1.0 / (n + 1) if h is None else h
    s = 1.0 / (h * h)
    a = np.asarray(a_nodes, dtype=np.float64)
    assert a.shape == (n + 2, n + 2)
    hm = lambda p, q: 2.0 * p * q / (p + q)
    ac = a[1:-1, 1:-1]                 # [y, x] interior
    aw = hm(ac, a[1:-1, 0:-2])
    ae = hm(ac, a[1:-1, 2:])
    as_ = hm(ac, a[0:-2, 1:-1])
    an = hm(ac, a[2:, 1:-1])
    center = (aw + ae + as_ + an) * s
    return _stencil_2d(n, n, center, -aw * s, -ae * s, -as_ * s, -an * s)


def convection_diffusion_2d(n, velocity=(1.0, 0.5), nu=0.01, h=None):
    """-nu Lap u + v . grad u, 5-point diffusion and first-order upwind
    (backward differences for positive velocity components)."""
    h = 1.0 / (n + 1) if h is None else h
    vx, vy = velocity
    assert vx >= 0 and vy >= 0
    d = nu / (h * h)
    center = 4 * d + (vx + vy) / h
    return _stencil_2d(n, n, center, -d - vx / h, -d, -d - vy / h, -d)


def helmholtz_2d(n, k=None, ppw=10.0, h=None):
    """-Lap_h u - k^2 u with the 5-point stencil (real, indefinite).  With
    ``k`` unset, k = 2 pi / (ppw h) gives ``ppw`` grid points per wavelength."""
    h = 1.0 / (n + 1) if h is None else h
    if k is None:
        k = 2.0 * math.pi / (ppw * h)
    s = 1.0 / (h * h)
    return _stencil_2d(n, n, 4 * s - k * k, -s, -s, -s, -s)


def random_rhs(n, nrhs, dist, rng):
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=(n, nrhs))
    if dist == "normal":
        return rng.standard_normal((n, nrhs))
    raise ValueError(dist)


# Workload table: family, default grid side, dimension, eps, nrhs, rhs law,
# refinement target, factor precision.
CONFIGS = [
    dict(name="laplace2d", side=63, dim=2, eps=1e-6, nrhs=1, dist="uniform", tol=1e-8, prec="fp64"),
    dict(name="diffusion2d_grf", side=1023, dim=2, eps=1e-4, nrhs=16, dist="uniform", tol=1e-10, prec="fp32"),
    dict(name="convdiff2d", side=2047, dim=2, eps=1e-5, nrhs=64, dist="uniform", tol=1e-8, prec="fp32"),
    dict(name="laplace3d", side=127, dim=3, eps=1e-4, nrhs=8, dist="normal", tol=1e-8, prec="fp32"),
    # eps 1e-6: at 10 points per wavelength the compression error of eps 1e-4
    # grows with N past what refinement of the indefinite operator tolerates
    # (direct residual 0.25 at 127^2, 1.8 at 255^2), at 1e-6 it stays ~5e-3
    dict(name="helmholtz2d", side=1023, dim=2, eps=1e-6, nrhs=256, dist="uniform", tol=1e-8, prec="fp32"),
]


def make_config(i, side=None, nrhs=None):
    """Build workload ``i`` (0..4); ``side`` shrinks the grid (same family,
    same coefficient law), ``nrhs`` overrides the number of right-hand sides."""
    c = CONFIGS[i]
    side = c["side"] if side is None else int(side)
    nrhs = c["nrhs"] if nrhs is None else int(nrhs)
    ss = np.random.SeedSequence(MASTER_SEED).spawn(len(CONFIGS))[i]
    mat_ss, rhs_ss = ss.spawn(2)
    mat_rng = np.random.Generator(np.random.PCG64(mat_ss))
    rhs_rng = np.random.Generator(np.random.PCG64(rhs_ss))
    sym = True
    if c["name"] == "laplace2d":
        csr = laplacian_2d(side)
        dims = (side, side)
    elif c["name"] == "diffusion2d_grf":
        g = gaussian_random_field(side + 2, 0.05, mat_rng)
        csr = diffusion_2d(side, np.exp(g))
        dims = (side, side)
    elif c["name"] == "convdiff2d":
        csr = convection_diffusion_2d(side)
        dims = (side, side)
        sym = False
    elif c["name"] == "laplace3d":
        csr = laplacian_3d(side)
        dims = (side, side, side)
    elif c["name"] == "helmholtz2d":
        csr = helmholtz_2d(side)
        dims = (side, side)
    else:  # pragma: no cover
        raise ValueError(c["name"])
    n = int(np.prod(dims))
    rhs = random_rhs(n, nrhs, c["dist"], rhs_rng)
    return Problem(name=c["name"], dims=dims, indptr=csr[0], indices=csr[1], data=csr[2],
                   rhs=rhs, eps=c["eps"], tol=c["tol"], symmetric=sym,
                   factor_precision=c["prec"])

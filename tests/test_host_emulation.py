"""Host emulation of the HIP kernels (CPU, no GPU): the library's sources are
compiled for the CPU with AddressSanitizer, every GPU thread runs as a fiber,
and every device buffer sits between inaccessible guard regions, so an
out-of-bounds access by any kernel fails the test instead of faulting a GPU.
The cases cover the paths the GPU tests take: exact elimination (eps = 0),
sampled IDs with forced resampling, FP32 storage, the global-memory leaf
path of 3D leaves, flexible GMRES refinement, and the symmetric form."""
import os
import re
import subprocess

import numpy as np
import pytest

from workloads import make_config

HERE = os.path.dirname(os.path.abspath(__file__))

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    import sys
    sys.path.insert(0, os.path.join(HERE, "hostemu"))
    import build as hostemu_build
    out = str(tmp_path_factory.mktemp("hostemu"))
    try:
        return hostemu_build.build(out)
    except (OSError, RuntimeError) as e:
        pytest.skip("host compiler unavailable: %s" % e)


def _write(P, d, params=None):
    A = P.scipy().tocsr()
    A.sort_indices()
    np.asarray(P.dims, np.int32).tofile(os.path.join(d, "dims.bin"))
    A.indptr.astype(np.int64).tofile(os.path.join(d, "rowptr.bin"))
    A.indices.astype(np.int32).tofile(os.path.join(d, "colind.bin"))
    A.data.astype(np.float64).tofile(os.path.join(d, "vals.bin"))
    (params if params is not None else np.zeros(1, np.float32)).tofile(os.path.join(d, "params.bin"))


def _run(exe, d, prec, model, eps, nrhs, tol, restart, h0=None, tuning=None, max_rank=None, sym=False):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    if sym:
        env["EMU_SYM"] = "1"
    if h0 is not None:
        env["EMU_H0"] = str(h0)
    if tuning is not None:
        env["EMU_TUNING"] = ",".join(str(int(x)) for x in tuning)
    r = subprocess.run([exe, d, str(prec), str(model), repr(eps), str(nrhs), repr(tol), "1234", str(restart)],
                       capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    m = re.search(r"factor rc (-?\d+)", r.stdout)
    assert m and int(m.group(1)) == 0, r.stdout
    s = re.search(r"solve rc (-?\d+) .* iters (\d+) first (\S+) final (\S+)", r.stdout)
    assert s and int(s.group(1)) == 0, r.stdout
    if max_rank is not None:
        max_rank.append(int(re.search(r"max_rank (\d+)", r.stdout).group(1)))
    return int(s.group(2)), float(s.group(3)), float(s.group(4))


def test_exact_elimination_2d(exe, tmp_path):
    P = make_config(0, side=31, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 64, 0, 0.0, 2, 0.0, 0)
    assert first <= 1e-12


def test_exact_elimination_large_couplings(exe, tmp_path):
    """127 x 127 with eps = 0: no skeleton shrinks, so the coupling blocks
    of the coarse levels (up to 63 x 63) exceed the one-wave scaling and
    take the four-wave matrix-core kernel; the factor is then an exact LU."""
    P = make_config(0, side=127, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 64, 0, 0.0, 3, 0.0, 0)
    assert first <= 1e-12


def test_sampled_ids_with_resampling_and_fgmres(exe, tmp_path):
    """A predictor that always says rank 0 starts every ID at 5 samples, so
    the probe check rejects some IDs and the doubling passes run."""
    P = make_config(4, side=63, nrhs=1)
    p = np.zeros(5081, np.float32)
    p[12:24] = 1.0
    p[-1] = -40.0
    _write(P, str(tmp_path), p)
    it, first, final = _run(exe, str(tmp_path), 64, 1, 1e-6, 2, 1e-10, 8)
    assert final <= 1e-10


def test_fp32_3d_global_leaf_path(exe, tmp_path):
    P = make_config(3, side=15, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 32, 0, 1e-4, 2, 1e-10, 8)
    assert final <= 1e-10


@pytest.mark.parametrize("cfg", [1, 4])
def test_wide_id_tiers_fp64(exe, tmp_path, cfg):
    """127 x 127 in FP64: the stacked coupling rows of the top-level
    segments exceed the LDS budgets, so the eight-wave tier and tier C run,
    with its far rows and row tables in LDS (both cases) and, for the widest
    Helmholtz segments, in global scratch too (bounds checked here on the
    CPU)."""
    P = make_config(cfg, side=127, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 64, 0, P.eps, 2, 1e-10, 8)
    assert final <= 1e-10


def test_exact_rows_split_between_lds_and_scratch(exe, tmp_path):
    """127 x 127 Helmholtz in FP64 with a first sample count above every
    far-row count: every ID is taken on all R stacked rows (the exact case
    of the hybrid sampling), so the widest tier-C segments hold more rows of
    Y than their LDS and keep the rest in global scratch."""
    P = make_config(4, side=127, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 64, 0, P.eps, 2, 1e-10, 8, h0=100000)
    assert final <= 1e-10


# id_lds_a, id_lds_b, id_lds_b2, id_lds_c, id_c_ydiv, melim_lds, melim_wave_cap,
# solve_lanes_min, solve_lanes_max: the smallest ID budgets (tier C without
# room for min(m, n) rows of Y: all of Y in scratch), 256-thread merges from
# 16 DOFs on, and lane groups of 16 to 32 only
SMALL_SHAPES = (4096, 16384, 16384, 32768, 4, 16384, 16, 16, 32)


@pytest.mark.parametrize("prec", [64, 32])
def test_smallest_launch_shapes(exe, tmp_path, prec):
    """127 x 127 Helmholtz with the smallest launch shapes the tuning API
    accepts: most IDs land in tier C with little LDS, the merge and the
    solve take their block kernels on more levels (bounds checked here on
    the CPU before any GPU run of these shapes)."""
    P = make_config(4, side=127, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), prec, 0, P.eps, 2, 1e-10, 8, tuning=SMALL_SHAPES)
    assert final <= 1e-10


def test_block_separator_solve_many_rhs(exe, tmp_path):
    """127 x 127 Helmholtz in FP32 with 70 right-hand sides and one-wave
    kernels for segments of at most 32 DOFs: the coarse levels take the
    256-thread separator kernels and four-wave segment solves on the matrix
    cores, with skeletons above 64 rows (several row passes per segment) and
    a full and a ragged chunk of right-hand-side columns; classical
    refinement, whose residuals go straight into the next right-hand side."""
    P = make_config(4, side=127, nrhs=1)
    _write(P, str(tmp_path))
    mr = []
    it, first, final = _run(exe, str(tmp_path), 32, 0, P.eps, 70, 1e-10, 0, tuning=SMALL_SHAPES, max_rank=mr)
    assert mr[0] > 64, mr
    # the factor alone already solves to about 3e-3 (a wrong row pass or
    # column chunk would leave whole skeleton blocks unsolved), and each
    # classical step gains about as much
    assert first <= 1e-2 and it <= 6, (first, it)
    assert final <= 1e-10


def test_symmetric_form_exact_elimination(exe, tmp_path):
    """Symmetric form with eps = 0: the balanced L D L^T of every segment
    and the one-sided scaling kernels give an exact solve."""
    P = make_config(1, side=63, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 64, 0, 0.0, 2, 0.0, 0, sym=True)
    assert first <= 1e-12


@pytest.mark.parametrize("prec", [64, 32])
def test_symmetric_form_wide_tiers(exe, tmp_path, prec):
    """Symmetric form at 127 x 127 (GRF diffusion): one-sided row tables in
    every ID tier, the block scaling kernels on the coarse levels, and
    refinement to 1e-10."""
    P = make_config(1, side=127, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), prec, 0, P.eps, 2, 1e-10, 8, sym=True)
    assert final <= 1e-10


def test_symmetric_form_3d(exe, tmp_path):
    P = make_config(3, side=15, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 64, 0, P.eps, 2, 1e-10, 0, sym=True)
    assert first <= 10 * P.eps and final <= 1e-10


@pytest.mark.parametrize("sym", [False, True])
def test_exact_elimination_3d_wide_blocks(exe, tmp_path, sym):
    """15^3 with eps = 0: no skeleton shrinks, so the 225-DOF separator
    blocks exceed every LDS-staged kernel and take the matrix-core tiles
    read from memory (coupling scaling and merge), in both forms."""
    P = make_config(3, side=15, nrhs=1)
    _write(P, str(tmp_path))
    it, first, final = _run(exe, str(tmp_path), 64, 0, 0.0, 2, 0.0, 0, sym=sym)
    assert first <= 1e-12

"""The C-ABI library: it loads without a GPU, exports every entry point the
header declares, and its nested-dissection planner reproduces the oracle bit
for bit (perm, etree, segments, couplings).  No compute call runs here."""
import os
import re

import numpy as np
import pytest

from oracle.nd import nd_order

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2408_14193_amd import spalu
    return spalu


def test_exports_every_declared_symbol():
    S = _lib()
    header = open(os.path.join(ROOT, "include", "spalu.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(spalu_\w+)\s*\(", header, re.M))
    assert declared == set(S.EXPORTED)
    for name in declared:
        assert hasattr(S._lib, name)


def test_profile_only_names():
    """Host-only calls: restricting the event timing to one kernel step
    accepts the step names the profile reports and rejects others."""
    S = _lib()
    S.profile(True)
    for name in ("seg_id_c", "solve_sweep_graph", "krylov", None, ""):
        S.profile_only(name)
    with pytest.raises(RuntimeError):
        S.profile_only("no_such_step")
    S.profile(False)


@pytest.mark.parametrize("dims,L", [((7, 7), 3), ((7, 7), 1), ((15, 15), 0), ((63, 63), 0),
                                    ((31, 15), 0), ((47, 33), 0), ((255, 255), 0),
                                    ((15, 15, 15), 0), ((31, 31, 31), 0), ((15, 31, 15), 0)])
def test_nd_bit_exact_against_oracle(dims, L):
    S = _lib()
    nd = S.ND(dims, L)
    o = nd_order(dims, L if L else None)
    assert nd.L == o.L and nd.n == int(np.prod(dims))
    assert np.array_equal(nd.perm(), o.perm)
    b, s, lv, p = nd.etree()
    assert np.array_equal(b, o.node_begin) and np.array_equal(s, o.node_size)
    assert np.array_equal(lv, o.node_level) and np.array_equal(p, o.node_parent)
    for l in range(1, nd.L + 1):
        ptr, verts, flags, parent, pairs = nd.segments(l)
        segs = o.levels[l].segs
        assert len(ptr) - 1 == len(segs)
        for i, sg in enumerate(segs):
            assert np.array_equal(verts[ptr[i]:ptr[i + 1]], sg.verts)
            assert flags[i] == (1 if sg.regular else 0) | (2 if sg.is_sep else 0)
            assert parent[i] == sg.parent
        assert [tuple(x) for x in pairs.tolist()] == o.levels[l].pairs


def test_nd_full_size_2d_counts():
    """1023 x 1023: the separator counts and lengths of the bisection
    closed form, and perm is a permutation (checked at full size)."""
    S = _lib()
    nd = S.ND((1023, 1023))
    assert nd.L == 14
    b, s, lv, p = nd.etree()
    for l in range(1, 15):
        assert (lv == l).sum() == 2 ** (l - 1)
        assert set(s[lv == l].tolist()) == {2 ** (10 - l // 2) - 1}
    perm = nd.perm()
    assert np.array_equal(np.sort(perm), np.arange(1023 * 1023))


def test_nd_errors():
    S = _lib()
    with pytest.raises(S.SpaluError) as e:
        S.ND((7, 7), 5)          # boxes too small to split five times
    assert e.value.code == S.EINVAL
    with pytest.raises(S.SpaluError):
        S.ND((0, 7))


def test_workspace_query_without_gpu():
    S = _lib()
    nd = S.ND((63, 63))
    b64 = S.factor_workspace_bytes(nd, S.factor_opts(precision=S.FP64))
    b32 = S.factor_workspace_bytes(nd, S.factor_opts(precision=S.FP32))
    assert 0 < b32 < b64


def test_tuning_roundtrip_and_validation():
    """Launch shapes: the defaults are the library's, a change reads back,
    an out-of-range value is refused and changes nothing."""
    S = _lib()
    d = S.tuning_default()
    assert S.get_tuning() == d
    try:
        t = S.set_tuning(id_lds_c=80 * 1024, id_c_ydiv=4, solve_lanes_min=16)
        assert S.get_tuning() == t and t["id_lds_c"] == 80 * 1024 and t["solve_lanes_min"] == 16
        for bad in (dict(id_c_ydiv=3), dict(id_lds_a=1 << 20), dict(solve_lanes_min=64, solve_lanes_max=32),
                    dict(melim_wave_cap=64), dict(solve_lanes_max=24)):
            with pytest.raises(S.SpaluError):
                S.set_tuning(**bad)
            assert S.get_tuning() == t
        with pytest.raises(KeyError):
            S.set_tuning(no_such_field=1)
    finally:
        S.set_tuning(**d)
    assert S.get_tuning() == d

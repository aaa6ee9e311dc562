"""Oracle: nested dissection of a regular grid with segment information.

Follows Section 3 (Algorithm 1 and the separator growth rule of eq. (3.1)).
On a regular grid the degree-biased growth always continues straight (the
aligned neighbour scores 1 + theta, sideways ones at most theta), so each
separator is a full grid line (2D) or plane (3D) through the median
vertex, perpendicular to the longest side of the box; ties between equal
sides split the lowest axis (x before y before z).  Every box at depth < L
is split, so all leaves sit at depth L.

Segments (Section 2.3.1, Section 3.2): at factorization level l the
remaining vertices are those on separators of level <= l.  The signature of
a remaining vertex is the set of depth-l boxes that contain one of its
stencil neighbours.  A segment is a connected piece of one separator whose
vertices share one signature; it is *regular* when the signature names two
boxes (one on each side) and a *junction* otherwise.  Levels are built from
the root down and vertices are also keyed by the level-(l-1) segment that
holds them, so every level-l segment nests in one level-(l-1) segment (in
2D this changes nothing; in 3D it cuts junction crosses where their arms
join different coarser segments).  Two segments are
coupled in the level-l Schur complement when their signatures share a box
or a stencil edge joins them.

Orders (the contract shared with the GPU planner):
  * vertex id v = x + nx*(y + ny*z);
  * ``perm`` (new -> old): leaves in left-first depth-first order, then the
    separators of level L, L-1, ..., 1, each level left to right; vertex
    ids ascending inside every node;
  * etree nodes in the same order; leaves have level L+1;
  * segments of a level are ordered by their smallest vertex id, and the
    vertices of a level-L segment ascend.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclasses.dataclass
class Box:
    lo: tuple
    hi: tuple
    depth: int
    index: int              # position among the boxes of its depth
    axis: int = -1          # split axis (internal boxes)
    mid: int = -1
    children: tuple = ()


@dataclasses.dataclass
class Segment:
    verts: np.ndarray       # original vertex ids, ascending
    sep_node: int           # etree node of the separator holding it
    sep_level: int
    sig: tuple              # sorted depth-l box indices
    regular: bool
    is_sep: bool            # on a separator of the current level
    bbox_lo: tuple
    bbox_hi: tuple
    parent: int = -1        # segment index at level l-1 (-1 if eliminated)


@dataclasses.dataclass
class Level:
    level: int
    segs: list
    pairs: list             # sorted (c, d) coupled pairs incl. (c, c)
    seg_of: np.ndarray      # vertex -> segment index at this level (-1)


@dataclasses.dataclass
class ND:
    dims: tuple             # (nx, ny, nz); nz = 1 in 2D
    dim: int
    L: int
    perm: np.ndarray
    node_begin: np.ndarray
    node_size: np.ndarray
    node_level: np.ndarray
    node_parent: np.ndarray
    leaves: list            # per leaf: (interior verts, [level-L segment ids])
    levels: dict            # l -> Level


def _sides(lo, hi):
    return [hi[a] - lo[a] + 1 for a in range(3)]


def default_levels(dims3, leaf_max=7):
    """Smallest L such that every depth-L box has all sides <= leaf_max."""
    boxes = [((0, 0, 0), tuple(d - 1 for d in dims3))]
    L = 0
    while any(max(_sides(lo, hi)) > leaf_max for lo, hi in boxes):
        nxt = []
        for lo, hi in boxes:
            s = _sides(lo, hi)
            a = int(np.argmax(s))
            mid = (lo[a] + hi[a]) // 2
            h0 = list(hi); h0[a] = mid - 1
            l1 = list(lo); l1[a] = mid + 1
            nxt += [(lo, tuple(h0)), (tuple(l1), hi)]
        boxes = nxt
        L += 1
    return L


def build_tree(dims3, L):
    root = Box((0, 0, 0), tuple(d - 1 for d in dims3), 0, 0)
    by_depth = [[root]]
    for d in range(L):
        nxt = []
        for b in by_depth[d]:
            s = _sides(b.lo, b.hi)
            a = int(np.argmax(s))          # first maximum: lowest axis on ties
            if s[a] < 3:
                raise ValueError("box too small to split at depth %d" % d)
            mid = (b.lo[a] + b.hi[a]) // 2
            h0 = list(b.hi); h0[a] = mid - 1
            l1 = list(b.lo); l1[a] = mid + 1
            c0 = Box(b.lo, tuple(h0), d + 1, len(nxt))
            c1 = Box(tuple(l1), b.hi, d + 1, len(nxt) + 1)
            b.axis, b.mid, b.children = a, mid, (c0, c1)
            nxt += [c0, c1]
        by_depth.append(nxt)
    return by_depth


def _box_ids(idx3, lo, hi):
    return idx3[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1].ravel()


def _sep_range(b):
    lo, hi = list(b.lo), list(b.hi)
    lo[b.axis] = hi[b.axis] = b.mid
    return tuple(lo), tuple(hi)


def nd_order(dims, levels=None, leaf_max=7):
    """Nested dissection of a grid; returns the ND structure (perm, etree,
    leaves and per-level segments)."""
    dim = len(dims)
    dims3 = tuple(dims) + (1,) * (3 - dim)
    nx, ny, nz = dims3
    N = nx * ny * nz
    L = max(1, default_levels(dims3, leaf_max)) if levels is None else int(levels)
    if L < 1:
        raise ValueError("need at least one level")
    by_depth = build_tree(dims3, L)
    idx3 = np.arange(N, dtype=np.int64).reshape(nz, ny, nx)

    # etree: leaves first, then separators of level L..1.
    nleaf = len(by_depth[L])
    sep_node_base = {}
    base = nleaf
    for lev in range(L, 0, -1):
        sep_node_base[lev] = base
        base += len(by_depth[lev - 1])
    nnode = base
    node_verts = [None] * nnode
    node_level = np.zeros(nnode, dtype=np.int64)
    node_parent = np.full(nnode, -1, dtype=np.int64)
    seplev = np.zeros(N, dtype=np.int64)          # 0 = leaf interior
    sepnode = np.full(N, -1, dtype=np.int64)
    for i, b in enumerate(by_depth[L]):
        node_verts[i] = _box_ids(idx3, b.lo, b.hi)
        node_level[i] = L + 1
        node_parent[i] = sep_node_base[L] + i // 2
    for lev in range(L, 0, -1):
        for j, b in enumerate(by_depth[lev - 1]):
            node = sep_node_base[lev] + j
            lo, hi = _sep_range(b)
            vs = _box_ids(idx3, lo, hi)
            node_verts[node] = vs
            node_level[node] = lev
            node_parent[node] = sep_node_base[lev - 1] + j // 2 if lev > 1 else -1
            seplev[vs] = lev
            sepnode[vs] = node
    node_size = np.array([len(v) for v in node_verts], dtype=np.int64)
    node_begin = np.concatenate([[0], np.cumsum(node_size)[:-1]]).astype(np.int64)
    perm = np.concatenate(node_verts).astype(np.int64)

    # Stencil neighbours (5-point / 7-point).
    coords = np.stack(np.unravel_index(np.arange(N), (nz, ny, nx))[::-1], axis=1)  # x, y, z
    dirs = []
    for a in range(dim):
        for s in (-1, 1):
            e = [0, 0, 0]; e[a] = s
            dirs.append(e)
    nbr = np.full((N, len(dirs)), -1, dtype=np.int64)
    for k, e in enumerate(dirs):
        c = coords + np.array(e)
        ok = np.all((c >= 0) & (c < np.array(dims3)), axis=1)
        nbr[ok, k] = c[ok, 0] + nx * (c[ok, 1] + ny * c[ok, 2])

    levels_out = {}
    up_seg = None                       # segment ids at level lev-1
    for lev in range(1, L + 1):
        boxes = by_depth[lev]
        box_of = np.full(N, -1, dtype=np.int64)
        for b in boxes:
            box_of[_box_ids(idx3, b.lo, b.hi)] = b.index
        rem = (seplev >= 1) & (seplev <= lev)
        rv = np.nonzero(rem)[0]
        nb_box = np.where(nbr[rv] >= 0, box_of[np.maximum(nbr[rv], 0)], -1)
        nb_box = np.sort(nb_box, axis=1)
        # canonical signature: distinct box ids, padded with -1
        sigs = []
        for row in nb_box:
            sigs.append(tuple(sorted(set(int(x) for x in row if x >= 0))))
        sig_id = {}
        key = np.empty(len(rv), dtype=np.int64)
        for i, s in enumerate(sigs):
            par = -1 if up_seg is None else int(up_seg[rv[i]])
            key[i] = sig_id.setdefault((int(sepnode[rv[i]]), s, par), len(sig_id))
        pos = np.full(N, -1, dtype=np.int64)
        pos[rv] = np.arange(len(rv))
        er, ec = [], []
        for k in range(len(dirs)):
            u = nbr[rv, k]
            ok = u >= 0
            ok[ok] &= rem[u[ok]]
            a_, b_ = np.nonzero(ok)[0], pos[u[ok]]
            same = key[a_] == key[b_]
            er.append(a_[same]); ec.append(b_[same])
        er, ec = np.concatenate(er), np.concatenate(ec)
        g = sp.coo_matrix((np.ones(len(er)), (er, ec)), shape=(len(rv), len(rv)))
        ncomp, comp = connected_components(g, directed=False)
        # order components by smallest vertex id (rv ascending -> first hit)
        first = np.full(ncomp, -1, dtype=np.int64)
        for i in range(len(rv)):
            if first[comp[i]] < 0:
                first[comp[i]] = i
        order = np.argsort(first, kind="stable")
        rank = np.empty(ncomp, dtype=np.int64)
        rank[order] = np.arange(ncomp)
        seg_of = np.full(N, -1, dtype=np.int64)
        seg_of[rv] = rank[comp]
        segs = []
        members = [[] for _ in range(ncomp)]
        for i in range(len(rv)):
            members[rank[comp[i]]].append(rv[i])
        for s in range(ncomp):
            vs = np.array(members[s], dtype=np.int64)
            i0 = pos[vs[0]]
            sl = int(seplev[vs[0]])
            cc = coords[vs]
            segs.append(Segment(verts=vs, sep_node=int(sepnode[vs[0]]), sep_level=sl,
                                sig=sigs[i0], regular=(len(sigs[i0]) == 2),
                                is_sep=(sl == lev),
                                bbox_lo=tuple(int(x) for x in cc.min(axis=0)),
                                bbox_hi=tuple(int(x) for x in cc.max(axis=0))))
        pairs = set((s, s) for s in range(ncomp))
        with_box = {}
        for s, sg in enumerate(segs):
            for b in sg.sig:
                with_box.setdefault(b, []).append(s)
        for lst in with_box.values():
            for a_ in lst:
                for b_ in lst:
                    pairs.add((a_, b_))
        for k in range(len(dirs)):
            u = nbr[rv, k]
            ok = u >= 0
            ok[ok] &= rem[u[ok]]
            sa, sb = seg_of[rv[ok]], seg_of[u[ok]]
            for a_, b_ in zip(sa.tolist(), sb.tolist()):
                pairs.add((a_, b_))
        levels_out[lev] = Level(level=lev, segs=segs, pairs=sorted(pairs), seg_of=seg_of)
        up_seg = seg_of

    # parents: level-l segment -> level-(l-1) segment holding its vertices
    for lev in range(L, 1, -1):
        up = levels_out[lev - 1].seg_of
        for sg in levels_out[lev].segs:
            if sg.is_sep:
                continue
            p = np.unique(up[sg.verts])
            if len(p) != 1 or p[0] < 0:
                raise AssertionError("segment does not nest into one parent segment")
            sg.parent = int(p[0])

    # leaves: interior vertices and the level-L segments on their boundary
    leaves = []
    segL = levels_out[L].segs
    on_leaf = {}
    for s, sg in enumerate(segL):
        for b in sg.sig:
            on_leaf.setdefault(b, []).append(s)
    for b in by_depth[L]:
        leaves.append((_box_ids(idx3, b.lo, b.hi), on_leaf.get(b.index, [])))

    return ND(dims=dims3, dim=dim, L=L, perm=perm, node_begin=node_begin, node_size=node_size,
              node_level=node_level, node_parent=node_parent, leaves=leaves, levels=levels_out)

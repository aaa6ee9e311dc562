// Grid nested dissection with segment information (Section 3, Algorithm 1).
//
// On a regular grid the degree-biased separator growth of eq. (3.1) keeps
// the aligned direction, so the separator of a box is the grid line/plane
// through the median index of its longest side (ties: lowest axis).  Boxes
// are numbered left to right at every depth, so the depth-l ancestor of a
// depth-d box j is j >> (d - l); this gives each vertex's box at any level
// in O(1).
//
// Segments at level l: remaining vertices (on separators of level <= l) are
// grouped by (separator, set of depth-l boxes holding a stencil neighbour,
// segment of level l-1), then split into connected pieces.  A piece whose
// neighbour-box set has two entries is regular, otherwise it is a junction.
#include "planner.hpp"

#include <algorithm>
#include <numeric>
#include <stdexcept>

namespace spalu {
namespace {

struct Box {
  int lo[3], hi[3];
  int axis = -1, mid = -1;
};

int side(const Box& b, int a) { return b.hi[a] - b.lo[a] + 1; }

int longest_axis(const Box& b) {
  int a = 0;
  for (int k = 1; k < 3; ++k)
    if (side(b, k) > side(b, a)) a = k;
  return a;
}

void split(const Box& b, int a, int mid, Box& c0, Box& c1) {
  c0 = b;
  c1 = b;
  c0.hi[a] = mid - 1;
  c1.lo[a] = mid + 1;
  c0.axis = c1.axis = -1;
}

struct DSU {
  std::vector<int32_t> p;
  explicit DSU(size_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int32_t find(int32_t x) {
    while (p[x] != x) {
      p[x] = p[p[x]];
      x = p[x];
    }
    return x;
  }
  void unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};

}  // namespace

void build_plan(int dim, const int32_t* grid, int levels, int leaf_max, Plan& p) {
  if (dim != 2 && dim != 3) throw std::runtime_error("dim must be 2 or 3");
  p.dim = dim;
  for (int a = 0; a < 3; ++a) p.dims[a] = a < dim ? grid[a] : 1;
  for (int a = 0; a < 3; ++a)
    if (p.dims[a] < 1) throw std::runtime_error("grid sizes must be positive");
  const int nx = p.dims[0], ny = p.dims[1], nz = p.dims[2];
  p.N = int64_t(nx) * ny * nz;
  if (p.N >= (int64_t(1) << 31)) throw std::runtime_error("grid too large");
  if (leaf_max <= 0) leaf_max = 7;

  Box root;
  for (int a = 0; a < 3; ++a) {
    root.lo[a] = 0;
    root.hi[a] = p.dims[a] - 1;
  }
  int L = levels;
  if (L <= 0) {
    // smallest depth at which every box has all sides <= leaf_max
    std::vector<Box> cur{root};
    L = 0;
    auto too_big = [&](const std::vector<Box>& v) {
      for (auto& b : v)
        for (int a = 0; a < 3; ++a)
          if (side(b, a) > leaf_max) return true;
      return false;
    };
    while (too_big(cur)) {
      std::vector<Box> nxt;
      for (auto& b : cur) {
        int a = longest_axis(b);
        int mid = (b.lo[a] + b.hi[a]) / 2;
        Box c0, c1;
        split(b, a, mid, c0, c1);
        nxt.push_back(c0);
        nxt.push_back(c1);
      }
      cur.swap(nxt);
      ++L;
    }
    L = std::max(L, 1);
  }
  if (L > 30) throw std::runtime_error("too many levels");
  p.L = L;

  std::vector<std::vector<Box>> by_depth(L + 1);
  by_depth[0].push_back(root);
  for (int d = 0; d < L; ++d) {
    by_depth[d + 1].reserve(by_depth[d].size() * 2);
    for (auto& b : by_depth[d]) {
      int a = longest_axis(b);
      if (side(b, a) < 3) throw std::runtime_error("box too small to split; lower the level count");
      b.axis = a;
      b.mid = (b.lo[a] + b.hi[a]) / 2;
      Box c0, c1;
      split(b, a, b.mid, c0, c1);
      by_depth[d + 1].push_back(c0);
      by_depth[d + 1].push_back(c1);
    }
  }

  auto vid = [&](int x, int y, int z) { return int32_t(x + nx * (y + ny * z)); };
  auto box_verts = [&](const int* lo, const int* hi, std::vector<int32_t>& out) {
    out.clear();
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) out.push_back(vid(x, y, z));
  };

  // etree: leaves, then separators of level L..1
  const int64_t nleaf = int64_t(by_depth[L].size());
  std::vector<int64_t> sep_base(L + 2, 0);
  int64_t base = nleaf;
  for (int lev = L; lev >= 1; --lev) {
    sep_base[lev] = base;
    base += int64_t(by_depth[lev - 1].size());
  }
  const int64_t nnode = base;
  p.node_begin.assign(nnode, 0);
  p.node_size.assign(nnode, 0);
  p.node_level.assign(nnode, 0);
  p.node_parent.assign(nnode, -1);
  p.seplev.assign(p.N, 0);
  std::vector<int32_t> sepnode(p.N, -1), home(p.N, 0);
  std::vector<int8_t> hdepth(p.N, 0);
  p.perm.clear();
  p.perm.reserve(p.N);
  std::vector<int32_t> tmp;
  p.leaves.assign(nleaf, PLeaf());
  for (int64_t i = 0; i < nleaf; ++i) {
    const Box& b = by_depth[L][i];
    box_verts(b.lo, b.hi, tmp);
    p.node_begin[i] = int64_t(p.perm.size());
    p.node_size[i] = int64_t(tmp.size());
    p.node_level[i] = L + 1;
    p.node_parent[i] = sep_base[L] + i / 2;
    for (int32_t v : tmp) {
      p.perm.push_back(v);
      home[v] = int32_t(i);
      hdepth[v] = int8_t(L);
    }
    PLeaf& lf = p.leaves[i];
    for (int a = 0; a < 3; ++a) {
      lf.lo[a] = b.lo[a];
      lf.hi[a] = b.hi[a];
    }
    lf.interior = tmp;
  }
  for (int lev = L; lev >= 1; --lev) {
    const auto& boxes = by_depth[lev - 1];
    for (size_t j = 0; j < boxes.size(); ++j) {
      const Box& b = boxes[j];
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = b.lo[a];
        hi[a] = b.hi[a];
      }
      lo[b.axis] = hi[b.axis] = b.mid;
      box_verts(lo, hi, tmp);
      int64_t node = sep_base[lev] + int64_t(j);
      p.node_begin[node] = int64_t(p.perm.size());
      p.node_size[node] = int64_t(tmp.size());
      p.node_level[node] = lev;
      p.node_parent[node] = lev > 1 ? sep_base[lev - 1] + int64_t(j / 2) : -1;
      for (int32_t v : tmp) {
        p.perm.push_back(v);
        p.seplev[v] = int8_t(lev);
        sepnode[v] = int32_t(node);
        home[v] = int32_t(j);
        hdepth[v] = int8_t(lev - 1);
      }
    }
  }

  // separator vertices in ascending id
  std::vector<int32_t> sepverts;
  for (int64_t v = 0; v < p.N; ++v)
    if (p.seplev[v] > 0) sepverts.push_back(int32_t(v));

  const int ndir = 2 * dim;
  int dx[6], dy[6], dz[6];
  for (int a = 0, k = 0; a < dim; ++a)
    for (int s = -1; s <= 1; s += 2, ++k) {
      dx[k] = a == 0 ? s : 0;
      dy[k] = a == 1 ? s : 0;
      dz[k] = a == 2 ? s : 0;
    }
  auto neighbor = [&](int32_t v, int k) -> int32_t {
    int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
    x += dx[k];
    y += dy[k];
    z += dz[k];
    if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return -1;
    return vid(x, y, z);
  };

  p.levels.assign(L + 1, PLevel());
  std::vector<int32_t> prev_seg(p.N, -1), seg_of(p.N, -1);
  std::vector<int32_t> pos(p.N, -1);
  for (int lev = 1; lev <= L; ++lev) {
    std::vector<int32_t> rv;
    for (int32_t v : sepverts)
      if (p.seplev[v] <= lev) rv.push_back(v);
    const size_t nr = rv.size();
    for (size_t i = 0; i < nr; ++i) pos[rv[i]] = int32_t(i);
    std::vector<int32_t> nsig(nr, 0), sig0(nr, -1), sig1(nr, -1);
    for (size_t i = 0; i < nr; ++i) {
      int32_t v = rv[i];
      int32_t s[6];
      int ns = 0;
      for (int k = 0; k < ndir; ++k) {
        int32_t u = neighbor(v, k);
        if (u < 0) continue;
        if (p.seplev[u] != 0 && p.seplev[u] <= lev) continue;
        int32_t b = home[u] >> (hdepth[u] - lev);
        bool seen = false;
        for (int t = 0; t < ns; ++t) seen |= s[t] == b;
        if (!seen) s[ns++] = b;
      }
      std::sort(s, s + ns);
      if (ns > 2) throw std::runtime_error("vertex borders more than two boxes");
      nsig[i] = ns;
      if (ns > 0) sig0[i] = s[0];
      if (ns > 1) sig1[i] = s[1];
    }
    auto same_key = [&](size_t i, size_t j) {
      int32_t a = rv[i], b = rv[j];
      return sepnode[a] == sepnode[b] && nsig[i] == nsig[j] && sig0[i] == sig0[j] &&
             sig1[i] == sig1[j] && prev_seg[a] == prev_seg[b];
    };
    DSU dsu(nr);
    for (size_t i = 0; i < nr; ++i) {
      for (int k = 0; k < ndir; ++k) {
        int32_t u = neighbor(rv[i], k);
        if (u < 0 || p.seplev[u] == 0 || p.seplev[u] > lev) continue;
        size_t j = size_t(pos[u]);
        if (same_key(i, j)) dsu.unite(int32_t(i), int32_t(j));
      }
    }
    // segment numbering by smallest vertex id (rv is ascending)
    std::vector<int32_t> root_seg(nr, -1);
    PLevel& PL = p.levels[lev];
    for (size_t i = 0; i < nr; ++i) {
      int32_t r = dsu.find(int32_t(i));
      if (root_seg[r] < 0) {
        root_seg[r] = int32_t(PL.segs.size());
        PSeg sg;
        int32_t v = rv[i];
        sg.sep_node = sepnode[v];
        sg.sep_level = p.seplev[v];
        sg.nsig = nsig[i];
        sg.sig[0] = sig0[i];
        sg.sig[1] = sig1[i];
        sg.regular = nsig[i] == 2;
        sg.is_sep = p.seplev[v] == lev;
        sg.parent = prev_seg[v];
        int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
        sg.lo[0] = sg.hi[0] = x;
        sg.lo[1] = sg.hi[1] = y;
        sg.lo[2] = sg.hi[2] = z;
        PL.segs.push_back(sg);
      }
      int32_t s = root_seg[r];
      int32_t v = rv[i];
      PSeg& sg = PL.segs[s];
      sg.verts.push_back(v);
      int c[3] = {v % nx, (v / nx) % ny, v / (nx * ny)};
      for (int a = 0; a < 3; ++a) {
        sg.lo[a] = std::min(sg.lo[a], c[a]);
        sg.hi[a] = std::max(sg.hi[a], c[a]);
      }
      seg_of[v] = s;
    }
    // coupled pairs: a shared neighbour box, or a stencil edge
    std::vector<std::pair<int64_t, int32_t>> by_box;
    for (size_t s = 0; s < PL.segs.size(); ++s)
      for (int t = 0; t < PL.segs[s].nsig; ++t) by_box.push_back({PL.segs[s].sig[t], int32_t(s)});
    std::sort(by_box.begin(), by_box.end());
    std::vector<std::pair<int32_t, int32_t>> pr;
    for (size_t s = 0; s < PL.segs.size(); ++s) pr.push_back({int32_t(s), int32_t(s)});
    for (size_t i = 0; i < by_box.size();) {
      size_t j = i;
      while (j < by_box.size() && by_box[j].first == by_box[i].first) ++j;
      for (size_t a = i; a < j; ++a)
        for (size_t b = i; b < j; ++b) pr.push_back({by_box[a].second, by_box[b].second});
      i = j;
    }
    for (size_t i = 0; i < nr; ++i)
      for (int k = 0; k < ndir; ++k) {
        int32_t u = neighbor(rv[i], k);
        if (u < 0 || p.seplev[u] == 0 || p.seplev[u] > lev) continue;
        if (seg_of[u] != seg_of[rv[i]]) pr.push_back({seg_of[rv[i]], seg_of[u]});
      }
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    PL.pairs.swap(pr);
    for (size_t i = 0; i < nr; ++i) pos[rv[i]] = -1;
    for (int32_t v : rv) prev_seg[v] = seg_of[v];
    for (int32_t v : sepverts)
      if (p.seplev[v] > lev) prev_seg[v] = -1;
    // vertices on level-(lev+1) separators are not in any level-lev segment
  }

  // leaf boundaries: level-L segments whose neighbour boxes include the leaf
  const PLevel& PLL = p.levels[L];
  for (size_t s = 0; s < PLL.segs.size(); ++s)
    for (int t = 0; t < PLL.segs[s].nsig; ++t) p.leaves[PLL.segs[s].sig[t]].bsegs.push_back(int32_t(s));
  for (auto& lf : p.leaves) std::sort(lf.bsegs.begin(), lf.bsegs.end());
}

}  // namespace spalu

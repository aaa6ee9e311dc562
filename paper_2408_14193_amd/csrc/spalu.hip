// C ABI of the spaLU library: nested dissection, factorization and solve on
// one MI355X.  See include/spalu.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/spalu.h"
#include "kernels_factor.hpp"
#include "kernels_solve.hpp"
#include "layout.hpp"
#include "planner.hpp"

using namespace spalu;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(SPALU_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct LevelTabs {
  std::vector<DSeg> segs;
  std::vector<DNbr> nbrs;
  std::vector<DBlk> blks;
  std::vector<int32_t> scale_list;
  std::vector<int32_t> cons_ptr, cons;  // merge into level l-1 (l >= 2)
  std::vector<int32_t> task_ptr;
  std::vector<DTask> tasks;
  std::vector<DSepTerm> terms;
  size_t o_segs = 0, o_nbrs = 0, o_blks = 0, o_scale = 0, o_cons_ptr = 0, o_cons = 0, o_task_ptr = 0,
         o_tasks = 0, o_terms = 0, o_dyn = 0;
};

struct Layout {
  int prec = 0;
  size_t vsize = 8;
  std::vector<LevelTabs> lv;  // 1..L
  std::vector<DLeaf> leaves;
  std::vector<int32_t> lc_ptr;
  std::vector<DLeafContrib> lc;
  std::vector<int32_t> vptrL, vertsL;
  size_t o_leaves = 0, o_lc_ptr = 0, o_lc = 0, o_vptrL = 0, o_vertsL = 0, o_seplev = 0;
  size_t blob_bytes = 0;
  size_t o_iarena = 0, n_iarena = 0;
  size_t o_varena = 0, n_varena = 0;
  size_t o_scratch = 0, n_scratch = 0;
  size_t leaf_scr_stride = 0;
  size_t o_status = 0;
  size_t bytes = 0;
  int64_t nseg_total = 0;
  std::vector<int64_t> seg_base;  // per level
};

}  // namespace

struct spalu_nd_s {
  Plan plan;
  std::unique_ptr<Layout> layout[2];
};

struct spalu_factor_s {
  const spalu_nd_t* nd = nullptr;
  const Layout* lay = nullptr;
  int prec = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* colind = nullptr;
  const double* vals = nullptr;
  GridGeom g{};
};

namespace {

// ---------------------------------------------------------------------------
// Static layout of the factorization for one ND and precision.
// ---------------------------------------------------------------------------
std::unique_ptr<Layout> build_layout(const Plan& P, int prec) {
  auto lay = std::make_unique<Layout>();
  Layout& Y = *lay;
  Y.prec = prec;
  Y.vsize = prec == SPALU_FP32 ? 4 : 8;
  const int L = P.L;
  Y.lv.assign(L + 1, LevelTabs());
  size_t iar = 0, var = 0, pool = 0;
  Y.seg_base.assign(L + 2, 0);
  int64_t sb = 0;
  for (int l = 1; l <= L; ++l) {
    Y.seg_base[l] = sb;
    sb += int64_t(P.levels[l].segs.size());
  }
  Y.seg_base[L + 1] = sb;
  Y.nseg_total = sb;

  for (int l = 1; l <= L; ++l) {
    const PLevel& PL = P.levels[l];
    LevelTabs& T = Y.lv[l];
    const size_t ns = PL.segs.size();
    T.segs.resize(ns);
    // blocks in pair order; adjacency per segment
    std::map<std::pair<int, int>, int> bid;
    for (size_t b = 0; b < PL.pairs.size(); ++b) bid[PL.pairs[b]] = int(b);
    T.blks.resize(PL.pairs.size());
    std::vector<int64_t> rcap(ns, 0);
    std::vector<std::vector<DNbr>> adj(ns);
    for (size_t b = 0; b < PL.pairs.size(); ++b) {
      const int c = PL.pairs[b].first, d = PL.pairs[b].second;
      const size_t cc = PL.segs[c].verts.size(), cd = PL.segs[d].verts.size();
      T.blks[b].c = c;
      T.blks[b].d = d;
      T.blks[b].off = int64_t(var);
      var += cc * cd;
      T.blks[b].soff = int64_t(var);
      var += cc * cd;
      if (c != d) {
        T.scale_list.push_back(int32_t(b));
        rcap[c] += 2 * int64_t(cd);
        DNbr nb;
        nb.d = d;
        nb.blk_cd = int32_t(b);
        nb.blk_dc = bid.at({d, c});
        nb.d_is_sep = PL.segs[d].is_sep ? 1 : 0;
        adj[c].push_back(nb);
        if (PL.segs[c].is_sep && PL.segs[d].is_sep)
          throw std::runtime_error("two separators of one level are coupled");
      }
    }
    size_t level_pool = 0;
    for (size_t c = 0; c < ns; ++c) {
      const PSeg& s = PL.segs[c];
      DSeg& D = T.segs[c];
      const int64_t cap = int64_t(s.verts.size());
      D.cap = int32_t(cap);
      D.flags = (s.regular ? SEG_REGULAR : 0) | (s.is_sep ? SEG_IS_SEP : 0) |
                (adj[c].empty() ? 0 : SEG_HAS_NBR);
      D.nbr_begin = int32_t(T.nbrs.size());
      for (auto& nb : adj[c]) T.nbrs.push_back(nb);
      D.nbr_end = int32_t(T.nbrs.size());
      D.diag_blk = bid.at({int(c), int(c)});
      D.parent = s.parent;
      for (int a = 0; a < 3; ++a) {
        D.lo[a] = s.lo[a];
        D.hi[a] = s.hi[a];
      }
      D.thr = 1;
      D.rcap = int32_t(rcap[c]);
      D.ioff = int64_t(iar);
      iar += size_t(3 * cap + std::max<int64_t>(2 * rcap[c], cap));
      D.lu_off = int64_t(var);
      var += size_t(cap * cap);
      D.t_off = int64_t(var);
      var += size_t(cap * cap / 4 + 1);
      size_t need = size_t(cap * cap);
      if ((D.flags & SEG_REGULAR) && (D.flags & SEG_HAS_NBR))
        need = std::max(need, size_t((3 * rcap[c] + 9) * cap));
      D.scr_off = int64_t(level_pool);
      level_pool += need;
    }
    pool = std::max(pool, level_pool);
  }

  // merge tables l -> l-1
  for (int l = L; l >= 2; --l) {
    const PLevel& PL = P.levels[l];
    const PLevel& PU = P.levels[l - 1];
    LevelTabs& T = Y.lv[l];
    std::map<std::pair<int, int>, int> bid;
    for (size_t b = 0; b < PL.pairs.size(); ++b) bid[PL.pairs[b]] = int(b);
    std::vector<std::vector<int>> cons(PU.segs.size());
    for (size_t c = 0; c < PL.segs.size(); ++c)
      if (!PL.segs[c].is_sep) {
        if (PL.segs[c].parent < 0) throw std::runtime_error("segment without parent");
        cons[PL.segs[c].parent].push_back(int(c));
      }
    T.cons_ptr.assign(1, 0);
    for (auto& v : cons) {
      for (int c : v) T.cons.push_back(c);
      T.cons_ptr.push_back(int32_t(T.cons.size()));
    }
    std::vector<std::vector<int>> seps_of(PL.segs.size());
    for (auto& pr : PL.pairs)
      if (pr.first != pr.second && PL.segs[pr.second].is_sep && !PL.segs[pr.first].is_sep)
        seps_of[pr.first].push_back(pr.second);
    // coverage checks: every surviving coupling lands in a level-(l-1) block
    std::map<std::pair<int, int>, int> ubid;
    for (size_t b = 0; b < PU.pairs.size(); ++b) ubid[PU.pairs[b]] = int(b);
    for (auto& pr : PL.pairs) {
      const PSeg &a = PL.segs[pr.first], &b = PL.segs[pr.second];
      if (!a.is_sep && !b.is_sep && !ubid.count({a.parent, b.parent}))
        throw std::runtime_error("coupling lost in merge");
    }
    std::vector<std::vector<int>> sep_nb(PL.segs.size());
    for (auto& pr : PL.pairs)
      if (pr.first != pr.second && PL.segs[pr.first].is_sep) sep_nb[pr.first].push_back(pr.second);
    for (size_t s = 0; s < PL.segs.size(); ++s) {
      const std::vector<int>& nb = sep_nb[s];
      for (int a : nb)
        for (int b : nb)
          if (!ubid.count({PL.segs[a].parent, PL.segs[b].parent}))
            throw std::runtime_error("fill lost in merge");
    }
    T.task_ptr.assign(1, 0);
    for (size_t ub = 0; ub < PU.pairs.size(); ++ub) {
      const int C = PU.pairs[ub].first, D = PU.pairs[ub].second;
      for (int c : cons[C])
        for (int d : cons[D]) {
          DTask tk{};
          tk.c = c;
          tk.d = d;
          if (c == d)
            tk.src = -2;
          else {
            auto it = bid.find({c, d});
            tk.src = it == bid.end() ? -1 : it->second;
          }
          tk.sep_begin = int32_t(T.terms.size());
          for (int s : seps_of[c])
            if (std::find(seps_of[d].begin(), seps_of[d].end(), s) != seps_of[d].end()) {
              DSepTerm st{};
              st.s = s;
              st.blk_cs = bid.at({c, s});
              st.blk_sd = bid.at({s, d});
              T.terms.push_back(st);
            }
          tk.sep_end = int32_t(T.terms.size());
          if (tk.src != -1 || tk.sep_end > tk.sep_begin) T.tasks.push_back(tk);
        }
      T.task_ptr.push_back(int32_t(T.tasks.size()));
    }
  }

  // leaves
  const PLevel& PLL = P.levels[L];
  Y.leaves.resize(P.leaves.size());
  size_t leaf_need = 0;
  std::vector<std::vector<int32_t>> bsoff(P.leaves.size());
  for (size_t i = 0; i < P.leaves.size(); ++i) {
    const PLeaf& pl = P.leaves[i];
    DLeaf& D = Y.leaves[i];
    for (int a = 0; a < 3; ++a) {
      D.lo[a] = pl.lo[a];
      D.hi[a] = pl.hi[a];
    }
    D.ni = int32_t(pl.interior.size());
    int nb = 0;
    for (int s : pl.bsegs) {
      bsoff[i].push_back(nb);
      nb += int(PLL.segs[s].verts.size());
    }
    D.nb = nb;
    D.ioff = int64_t(iar);
    iar += size_t(nb + D.ni);
    D.lu_off = int64_t(var);
    var += size_t(D.ni) * D.ni;
    D.s_off = int64_t(var);
    var += size_t(nb) * nb;
    leaf_need = std::max(leaf_need, size_t(D.ni) * D.ni + size_t(D.ni) * nb);
  }
  if (leaf_need > size_t(LDS_DOUBLES)) {
    Y.leaf_scr_stride = leaf_need;
    pool = std::max(pool, leaf_need * P.leaves.size());
  }
  // level-L assembly contributions
  {
    const PLevel& PL = P.levels[L];
    Y.lc_ptr.assign(1, 0);
    for (auto& pr : PL.pairs) {
      const PSeg &a = PL.segs[pr.first], &b = PL.segs[pr.second];
      for (int ta = 0; ta < a.nsig; ++ta)
        for (int tb = 0; tb < b.nsig; ++tb)
          if (a.sig[ta] == b.sig[tb]) {
            const int lf = a.sig[ta];
            const auto& bs = P.leaves[lf].bsegs;
            const int ia = int(std::find(bs.begin(), bs.end(), pr.first) - bs.begin());
            const int ib = int(std::find(bs.begin(), bs.end(), pr.second) - bs.begin());
            DLeafContrib lc{};
            lc.leaf = lf;
            lc.oc = bsoff[lf][ia];
            lc.od = bsoff[lf][ib];
            Y.lc.push_back(lc);
          }
      Y.lc_ptr.push_back(int32_t(Y.lc.size()));
    }
    Y.vptrL.assign(1, 0);
    for (auto& s : PL.segs) {
      for (int32_t v : s.verts) Y.vertsL.push_back(v);
      Y.vptrL.push_back(int32_t(Y.vertsL.size()));
    }
  }

  // blob of tables
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  for (int l = 1; l <= L; ++l) {
    LevelTabs& T = Y.lv[l];
    T.o_segs = put(T.segs.size() * sizeof(DSeg));
    T.o_nbrs = put(T.nbrs.size() * sizeof(DNbr));
    T.o_blks = put(T.blks.size() * sizeof(DBlk));
    T.o_scale = put(T.scale_list.size() * 4);
    T.o_cons_ptr = put(T.cons_ptr.size() * 4);
    T.o_cons = put(T.cons.size() * 4);
    T.o_task_ptr = put(T.task_ptr.size() * 4);
    T.o_tasks = put(T.tasks.size() * sizeof(DTask));
    T.o_terms = put(T.terms.size() * sizeof(DSepTerm));
  }
  Y.o_leaves = put(Y.leaves.size() * sizeof(DLeaf));
  Y.o_lc_ptr = put(Y.lc_ptr.size() * 4);
  Y.o_lc = put(Y.lc.size() * sizeof(DLeafContrib));
  Y.o_vptrL = put(Y.vptrL.size() * 4);
  Y.o_vertsL = put(Y.vertsL.size() * 4);
  Y.o_seplev = put(size_t(P.N));
  Y.blob_bytes = o;
  // dynamic per-level arrays (6 ints per segment)
  for (int l = 1; l <= L; ++l) Y.lv[l].o_dyn = put(6 * Y.lv[l].segs.size() * 4);
  Y.o_status = put(64);
  Y.o_iarena = put(iar * 4);
  Y.n_iarena = iar;
  Y.o_varena = put(var * Y.vsize);
  Y.n_varena = var;
  Y.o_scratch = put(pool * 8);
  Y.n_scratch = pool;
  Y.bytes = o;
  return lay;
}

DLevelDyn dyn_of(char* ws, const Layout& Y, int l) {
  int32_t* base = reinterpret_cast<int32_t*>(ws + Y.lv[l].o_dyn);
  const size_t ns = Y.lv[l].segs.size();
  DLevelDyn d;
  d.n = base;
  d.k = base + ns;
  d.nr = base + 2 * ns;
  d.h = base + 3 * ns;
  d.passes = base + 4 * ns;
  d.off = base + 5 * ns;
  return d;
}

template <typename X>
const X* tab(char* ws, size_t off) {
  return reinterpret_cast<const X*>(ws + off);
}

unsigned nblocks(int64_t n, int b = WG) { return unsigned(std::max<int64_t>(1, (n + b - 1) / b)); }

constexpr size_t LDS_BYTES = size_t(LDS_DOUBLES) * 8;

template <typename T>
int run_factor(spalu_factor_t* F, const spalu_factor_opts& o, int* status_host) {
  const Layout& Y = *F->lay;
  const Plan& P = F->nd->plan;
  char* ws = F->ws;
  hipStream_t st = F->stream;
  int32_t* iar = reinterpret_cast<int32_t*>(ws + Y.o_iarena);
  T* var = reinterpret_cast<T*>(ws + Y.o_varena);
  double* scr = reinterpret_cast<double*>(ws + Y.o_scratch);
  int* status = reinterpret_cast<int*>(ws + Y.o_status);
  const int L = P.L;
  HIPCHK(hipMemsetAsync(status, 0, 64, st));
  k_check_pattern<<<nblocks(F->n), WG, 0, st>>>(F->g, F->n, F->rowptr, F->colind, status);
  HIPCHK(hipGetLastError());
  {
    const LevelTabs& TL = Y.lv[L];
    DLevelDyn dL = dyn_of(ws, Y, L);
    k_init_level<<<unsigned(TL.segs.size()), 64, 0, st>>>(tab<DSeg>(ws, TL.o_segs), int(TL.segs.size()),
                                                           tab<int32_t>(ws, Y.o_vptrL),
                                                           tab<int32_t>(ws, Y.o_vertsL), iar, dL);
    HIPCHK(hipGetLastError());
    k_leaf_factor<T><<<unsigned(Y.leaves.size()), WG, LDS_BYTES, st>>>(
        tab<DLeaf>(ws, Y.o_leaves), int(Y.leaves.size()), F->g, F->rowptr, F->colind, F->vals, iar, var,
        scr, int64_t(Y.leaf_scr_stride), status);
    HIPCHK(hipGetLastError());
    k_assemble_leafL<T><<<unsigned(TL.blks.size()), WG, 0, st>>>(
        tab<DBlk>(ws, TL.o_blks), int(TL.blks.size()), tab<DSeg>(ws, TL.o_segs), iar, dL,
        tab<int32_t>(ws, Y.o_lc_ptr), tab<DLeafContrib>(ws, Y.o_lc), tab<DLeaf>(ws, Y.o_leaves),
        F->rowptr, F->colind, F->vals, var);
    HIPCHK(hipGetLastError());
  }
  for (int l = L; l >= 1; --l) {
    const LevelTabs& T_ = Y.lv[l];
    const int ns = int(T_.segs.size());
    DLevelDyn d = dyn_of(ws, Y, l);
    const DSeg* segs = tab<DSeg>(ws, T_.o_segs);
    const DBlk* blks = tab<DBlk>(ws, T_.o_blks);
    IdParams prm;
    prm.eps = o.eps;
    prm.tau = o.tau;
    prm.seed = o.seed;
    prm.h0 = o.h0;
    prm.probes = o.probes;
    prm.level = l;
    prm.seg_base = int(Y.seg_base[l]);
    prm.h_init = o.h_init;
    k_seg_id<T><<<unsigned(ns), WG, LDS_BYTES, st>>>(segs, ns, tab<DNbr>(ws, T_.o_nbrs), blks, F->g, iar,
                                                     var, scr, d, prm);
    HIPCHK(hipGetLastError());
    k_seg_lu<T><<<unsigned(ns), WG, LDS_BYTES, st>>>(segs, ns, blks, iar, var, scr, d, status);
    HIPCHK(hipGetLastError());
    if (!T_.scale_list.empty()) {
      k_blk_scale<T><<<unsigned(T_.scale_list.size()), WG, LDS_BYTES, st>>>(
          blks, tab<int32_t>(ws, T_.o_scale), int(T_.scale_list.size()), segs, iar, var, d);
      HIPCHK(hipGetLastError());
    }
    if (l > 1) {
      const LevelTabs& U = Y.lv[l - 1];
      DLevelDyn du = dyn_of(ws, Y, l - 1);
      k_merge_sizes<<<unsigned(U.segs.size()), 64, 0, st>>>(
          tab<DSeg>(ws, U.o_segs), int(U.segs.size()), tab<int32_t>(ws, T_.o_cons_ptr),
          tab<int32_t>(ws, T_.o_cons), segs, iar, d, du);
      HIPCHK(hipGetLastError());
      k_merge_elim<T><<<unsigned(U.blks.size()), WG, 0, st>>>(
          tab<DBlk>(ws, U.o_blks), int(U.blks.size()), tab<int32_t>(ws, T_.o_task_ptr),
          tab<DTask>(ws, T_.o_tasks), tab<DSepTerm>(ws, T_.o_terms), blks, var, d, du);
      HIPCHK(hipGetLastError());
    }
  }
  HIPCHK(hipMemcpyAsync(status_host, status, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SPALU_OK;
}

struct SolveWs {
  size_t oW, oZ, oB0, oR, oPr, oPb, oNr, oNb, bytes;
  unsigned rblk;
};

SolveWs solve_layout(const spalu_factor_t* F, int nrhs) {
  SolveWs s{};
  const size_t vs = F->lay->vsize;
  const size_t nn = size_t(F->n) * nrhs;
  size_t o = 0;
  auto put = [&](size_t b) {
    size_t r = o;
    o = align256(o + b);
    return r;
  };
  s.rblk = nblocks(F->n);
  s.oW = put(nn * vs);
  s.oZ = put(nn * vs);
  s.oB0 = put(nn * vs);
  s.oR = put(nn * 8);
  s.oPr = put(size_t(s.rblk) * nrhs * 8);
  s.oPb = put(size_t(s.rblk) * nrhs * 8);
  s.oNr = put(size_t(nrhs) * 8);
  s.oNb = put(size_t(nrhs) * 8);
  s.bytes = o;
  return s;
}

// One application of the factor: W <- M^{-1} B0 (both in the working layout).
template <typename T>
int apply_inverse(const spalu_factor_t* F, T* B0, T* W, T* Z, int nrhs) {
  const Layout& Y = *F->lay;
  const Plan& P = F->nd->plan;
  char* ws = F->ws;
  hipStream_t st = F->stream;
  const int32_t* iar = reinterpret_cast<const int32_t*>(ws + Y.o_iarena);
  const T* var = reinterpret_cast<const T*>(ws + Y.o_varena);
  const int L = P.L;
  const size_t nn = size_t(F->n) * nrhs;
  HIPCHK(hipMemcpyAsync(W, B0, nn * sizeof(T), hipMemcpyDeviceToDevice, st));
  const DLeaf* leaves = tab<DLeaf>(ws, Y.o_leaves);
  k_leaf_solve<T, false><<<unsigned(Y.leaves.size()), WG, LDS_BYTES, st>>>(
      leaves, int(Y.leaves.size()), F->g, F->rowptr, F->colind, F->vals, iar, var, B0, W, Z, nrhs);
  HIPCHK(hipGetLastError());
  k_sep_from_leaves<T><<<nblocks(int64_t(nn)), WG, 0, st>>>(F->n, tab<int8_t>(ws, Y.o_seplev), F->rowptr,
                                                             F->colind, F->vals, Z, W, nrhs);
  HIPCHK(hipGetLastError());
  for (int l = L; l >= 1; --l) {
    const LevelTabs& T_ = Y.lv[l];
    const int ns = int(T_.segs.size());
    DLevelDyn d = dyn_of(ws, Y, l);
    k_seg_solve<T, false><<<unsigned(ns), WG, LDS_BYTES, st>>>(tab<DSeg>(ws, T_.o_segs), ns, iar, var, d, W,
                                                               nrhs);
    HIPCHK(hipGetLastError());
    k_sep_fwd<T><<<unsigned(ns), WG, 0, st>>>(tab<DSeg>(ws, T_.o_segs), ns, tab<DNbr>(ws, T_.o_nbrs),
                                             tab<DBlk>(ws, T_.o_blks), iar, var, d, W, nrhs);
    HIPCHK(hipGetLastError());
  }
  for (int l = 1; l <= L; ++l) {
    const LevelTabs& T_ = Y.lv[l];
    const int ns = int(T_.segs.size());
    DLevelDyn d = dyn_of(ws, Y, l);
    k_sep_bwd<T><<<unsigned(ns), WG, 0, st>>>(tab<DSeg>(ws, T_.o_segs), ns, tab<DNbr>(ws, T_.o_nbrs),
                                             tab<DBlk>(ws, T_.o_blks), iar, var, d, W, nrhs);
    HIPCHK(hipGetLastError());
    k_seg_solve<T, true><<<unsigned(ns), WG, LDS_BYTES, st>>>(tab<DSeg>(ws, T_.o_segs), ns, iar, var, d, W,
                                                              nrhs);
    HIPCHK(hipGetLastError());
  }
  k_leaf_solve<T, true><<<unsigned(Y.leaves.size()), WG, LDS_BYTES, st>>>(
      leaves, int(Y.leaves.size()), F->g, F->rowptr, F->colind, F->vals, iar, var, B0, W, Z, nrhs);
  HIPCHK(hipGetLastError());
  return SPALU_OK;
}

template <typename T>
int run_solve(const spalu_factor_t* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
              const spalu_solve_opts& so, char* sw, double* rel_res, spalu_solve_info* info) {
  const SolveWs s = solve_layout(F, nrhs);
  hipStream_t st = F->stream;
  T* W = reinterpret_cast<T*>(sw + s.oW);
  T* Z = reinterpret_cast<T*>(sw + s.oZ);
  T* B0 = reinterpret_cast<T*>(sw + s.oB0);
  double* R = reinterpret_cast<double*>(sw + s.oR);
  double* pr = reinterpret_cast<double*>(sw + s.oPr);
  double* pb = reinterpret_cast<double*>(sw + s.oPb);
  double* nr = reinterpret_cast<double*>(sw + s.oNr);
  double* nb = reinterpret_cast<double*>(sw + s.oNb);
  const int64_t nn = F->n * nrhs;
  const bool want_res = so.tol > 0.0 || rel_res != nullptr || info != nullptr;
  // With X == B (direct solve only) the right-hand side is saved to R first;
  // the residual kernel then reads b from R and overwrites it with r entry
  // by entry.
  const bool alias = want_res && X == B;
  const double* Bsrc = B;
  int64_t ldbres = ldb;
  if (alias) {
    HIPCHK(hipMemcpy2DAsync(R, size_t(F->n) * 8, B, size_t(ldb) * 8, size_t(F->n) * 8, size_t(nrhs),
                            hipMemcpyDeviceToDevice, st));
    Bsrc = R;
    ldbres = F->n;
  }
  k_rhs_in<T><<<nblocks(nn), WG, 0, st>>>(B, ldb, F->n, nrhs, B0);
  HIPCHK(hipGetLastError());
  int rc = apply_inverse<T>(F, B0, W, Z, nrhs);
  if (rc) return rc;
  k_rhs_out<T><<<nblocks(nn), WG, 0, st>>>(W, F->n, nrhs, X, ldx, 0);
  HIPCHK(hipGetLastError());
  if (!want_res) return SPALU_OK;
  std::vector<double> hr(nrhs), hb(nrhs);
  double first = -1.0, worst = 0.0;
  int it = 0;
  std::vector<double> bnorm;
  while (true) {
    dim3 grid(s.rblk, unsigned(nrhs));
    k_residual<<<grid, WG, 0, st>>>(F->n, nrhs, F->rowptr, F->colind, F->vals, Bsrc, ldbres, X, ldx, R,
                                    pr, pb);
    HIPCHK(hipGetLastError());
    k_reduce_cols<<<unsigned(nrhs), WG, 0, st>>>(pr, int(s.rblk), nrhs, nr);
    HIPCHK(hipGetLastError());
    if (bnorm.empty()) {
      k_reduce_cols<<<unsigned(nrhs), WG, 0, st>>>(pb, int(s.rblk), nrhs, nb);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(hb.data(), nb, size_t(nrhs) * 8, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(hr.data(), nr, size_t(nrhs) * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bnorm.empty()) {
      bnorm.resize(nrhs);
      for (int j = 0; j < nrhs; ++j) bnorm[j] = hb[j] > 0 ? std::sqrt(hb[j]) : 1.0;
    }
    worst = 0.0;
    for (int j = 0; j < nrhs; ++j) {
      const double r = std::sqrt(hr[j]) / bnorm[j];
      worst = std::max(worst, r);
      if (rel_res) rel_res[j] = r;
    }
    if (first < 0) first = worst;
    if (so.tol <= 0.0 || worst <= so.tol || it >= so.max_iter) break;
    // correction: solve with r as right-hand side, x += M r
    k_rhs_in<T><<<nblocks(nn), WG, 0, st>>>(R, F->n, F->n, nrhs, B0);
    HIPCHK(hipGetLastError());
    rc = apply_inverse<T>(F, B0, W, Z, nrhs);
    if (rc) return rc;
    k_rhs_out<T><<<nblocks(nn), WG, 0, st>>>(W, F->n, nrhs, X, ldx, 1);
    HIPCHK(hipGetLastError());
    ++it;
  }
  if (info) {
    info->iterations = it;
    info->max_rel_residual = worst;
    info->first_rel_residual = first;
  }
  if (so.tol > 0.0 && worst > so.tol) return fail(SPALU_ENOCONV, "refinement did not reach the tolerance");
  return SPALU_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* spalu_last_error(void) { return g_err.c_str(); }

int spalu_nd_order(int32_t dim, const int32_t* grid, const spalu_nd_opts* opts, spalu_nd_t** out) {
  if (!out) return fail(SPALU_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid) return fail(SPALU_EINVAL, "grid is NULL");
  try {
    auto nd = std::make_unique<spalu_nd_t>();
    build_plan(dim, grid, opts ? opts->levels : 0, opts ? opts->leaf_max : 7, nd->plan);
    *out = nd.release();
    return SPALU_OK;
  } catch (const std::exception& e) {
    return fail(SPALU_EINVAL, e.what());
  }
}

int spalu_nd_info(const spalu_nd_t* nd, int64_t* n, int32_t* levels, int64_t* nnodes, int64_t* nsegments) {
  if (!nd) return fail(SPALU_EINVAL, "nd is NULL");
  if (n) *n = nd->plan.N;
  if (levels) *levels = nd->plan.L;
  if (nnodes) *nnodes = int64_t(nd->plan.node_size.size());
  if (nsegments) {
    int64_t s = 0;
    for (int l = 1; l <= nd->plan.L; ++l) s += int64_t(nd->plan.levels[l].segs.size());
    *nsegments = s;
  }
  return SPALU_OK;
}

int spalu_nd_perm(const spalu_nd_t* nd, int64_t* perm) {
  if (!nd || !perm) return fail(SPALU_EINVAL, "null argument");
  std::copy(nd->plan.perm.begin(), nd->plan.perm.end(), perm);
  return SPALU_OK;
}

int spalu_nd_etree(const spalu_nd_t* nd, int64_t* begin, int64_t* size, int32_t* level, int64_t* parent) {
  if (!nd) return fail(SPALU_EINVAL, "nd is NULL");
  const Plan& p = nd->plan;
  if (begin) std::copy(p.node_begin.begin(), p.node_begin.end(), begin);
  if (size) std::copy(p.node_size.begin(), p.node_size.end(), size);
  if (level) std::copy(p.node_level.begin(), p.node_level.end(), level);
  if (parent) std::copy(p.node_parent.begin(), p.node_parent.end(), parent);
  return SPALU_OK;
}

int spalu_nd_segments(const spalu_nd_t* nd, int32_t level, int64_t* nseg, int64_t* nverts, int64_t* seg_ptr,
                      int32_t* verts, int32_t* flags, int32_t* parent, int64_t* npairs, int32_t* pairs) {
  if (!nd) return fail(SPALU_EINVAL, "nd is NULL");
  const Plan& p = nd->plan;
  if (level < 1 || level > p.L) return fail(SPALU_EINVAL, "level out of range");
  const PLevel& PL = p.levels[level];
  int64_t nv = 0;
  for (auto& s : PL.segs) nv += int64_t(s.verts.size());
  if (nseg) *nseg = int64_t(PL.segs.size());
  if (nverts) *nverts = nv;
  if (npairs) *npairs = int64_t(PL.pairs.size());
  if (!verts) return SPALU_OK;
  int64_t o = 0;
  for (size_t s = 0; s < PL.segs.size(); ++s) {
    if (seg_ptr) seg_ptr[s] = o;
    for (int32_t v : PL.segs[s].verts) verts[o++] = v;
    if (flags) flags[s] = (PL.segs[s].regular ? 1 : 0) | (PL.segs[s].is_sep ? 2 : 0);
    if (parent) parent[s] = PL.segs[s].parent;
  }
  if (seg_ptr) seg_ptr[PL.segs.size()] = o;
  if (pairs)
    for (size_t i = 0; i < PL.pairs.size(); ++i) {
      pairs[2 * i] = PL.pairs[i].first;
      pairs[2 * i + 1] = PL.pairs[i].second;
    }
  return SPALU_OK;
}

void spalu_nd_free(spalu_nd_t* nd) { delete nd; }

void spalu_factor_opts_default(spalu_factor_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 1e-6;
  o->precision = SPALU_FP64;
  o->seed = 1234;
  o->rho = 0.5;
  o->h0 = 8;
  o->probes = 5;
  o->tau = 10.0;
  o->h_init = nullptr;
}

static const Layout* get_layout(const spalu_nd_t* nd, int prec) {
  spalu_nd_t* m = const_cast<spalu_nd_t*>(nd);
  if (!m->layout[prec]) m->layout[prec] = build_layout(nd->plan, prec);
  return m->layout[prec].get();
}

int spalu_factor_workspace(const spalu_nd_t* nd, const spalu_factor_opts* opts, size_t* bytes) {
  if (!nd || !bytes) return fail(SPALU_EINVAL, "null argument");
  spalu_factor_opts o;
  spalu_factor_opts_default(&o);
  if (opts) o = *opts;
  if (o.precision != SPALU_FP64 && o.precision != SPALU_FP32) return fail(SPALU_EINVAL, "bad precision");
  try {
    *bytes = get_layout(nd, o.precision)->bytes;
  } catch (const std::exception& e) {
    return fail(SPALU_EUNSUPPORTED, e.what());
  }
  return SPALU_OK;
}

int spalu_factor_seg_base(const spalu_nd_t* nd, int64_t* base) {
  if (!nd || !base) return fail(SPALU_EINVAL, "null argument");
  const Plan& p = nd->plan;
  int64_t s = 0;
  base[0] = 0;
  for (int l = 1; l <= p.L; ++l) {
    base[l] = s;
    s += int64_t(p.levels[l].segs.size());
  }
  base[p.L + 1] = s;
  return SPALU_OK;
}

int spalu_factor(const spalu_nd_t* nd, int64_t n, const int64_t* rowptr, const int32_t* colind,
                 const double* vals, const spalu_factor_opts* opts, void* workspace, size_t workspace_bytes,
                 void* stream, spalu_factor_t** out, spalu_factor_info* info) {
  if (!out) return fail(SPALU_EINVAL, "out is NULL");
  *out = nullptr;
  if (!nd || !rowptr || !colind || !vals || !workspace) return fail(SPALU_EINVAL, "null argument");
  if (n != nd->plan.N) return fail(SPALU_EINVAL, "matrix size does not match the grid");
  spalu_factor_opts o;
  spalu_factor_opts_default(&o);
  if (opts) o = *opts;
  if (o.precision != SPALU_FP64 && o.precision != SPALU_FP32) return fail(SPALU_EINVAL, "bad precision");
  if (!(o.eps >= 0.0) || !(o.rho >= 0.0) || o.h0 < 1 || o.probes < 1 || o.probes > 8 || !(o.tau > 0.0))
    return fail(SPALU_EINVAL, "bad factor options");
  const Layout* Y;
  try {
    Y = get_layout(nd, o.precision);
  } catch (const std::exception& e) {
    return fail(SPALU_EUNSUPPORTED, e.what());
  }
  if (workspace_bytes < Y->bytes) return fail(SPALU_ENOMEM, "workspace too small");
  auto F = std::make_unique<spalu_factor_t>();
  F->nd = nd;
  F->lay = Y;
  F->prec = o.precision;
  F->ws = static_cast<char*>(workspace);
  F->stream = static_cast<hipStream_t>(stream);
  F->n = n;
  F->rowptr = rowptr;
  F->colind = colind;
  F->vals = vals;
  F->g = GridGeom{nd->plan.dims[0], nd->plan.dims[1], nd->plan.dims[2]};
  // tables: patch the option-dependent near-field radius, then upload
  std::vector<char> blob(Y->blob_bytes, 0);
  const Plan& P = nd->plan;
  for (int l = 1; l <= P.L; ++l) {
    const LevelTabs& T = Y->lv[l];
    std::vector<DSeg> segs = T.segs;
    for (auto& s : segs) {
      int span = 0;
      for (int a = 0; a < 3; ++a) span = std::max(span, s.hi[a] - s.lo[a] + 1);
      s.thr = std::max(1, int(std::ceil(o.rho * span)));
    }
    auto cp = [&](size_t off, const void* src, size_t b) {
      if (b) std::memcpy(blob.data() + off, src, b);
    };
    cp(T.o_segs, segs.data(), segs.size() * sizeof(DSeg));
    cp(T.o_nbrs, T.nbrs.data(), T.nbrs.size() * sizeof(DNbr));
    cp(T.o_blks, T.blks.data(), T.blks.size() * sizeof(DBlk));
    cp(T.o_scale, T.scale_list.data(), T.scale_list.size() * 4);
    cp(T.o_cons_ptr, T.cons_ptr.data(), T.cons_ptr.size() * 4);
    cp(T.o_cons, T.cons.data(), T.cons.size() * 4);
    cp(T.o_task_ptr, T.task_ptr.data(), T.task_ptr.size() * 4);
    cp(T.o_tasks, T.tasks.data(), T.tasks.size() * sizeof(DTask));
    cp(T.o_terms, T.terms.data(), T.terms.size() * sizeof(DSepTerm));
  }
  std::memcpy(blob.data() + Y->o_leaves, Y->leaves.data(), Y->leaves.size() * sizeof(DLeaf));
  std::memcpy(blob.data() + Y->o_lc_ptr, Y->lc_ptr.data(), Y->lc_ptr.size() * 4);
  if (!Y->lc.empty()) std::memcpy(blob.data() + Y->o_lc, Y->lc.data(), Y->lc.size() * sizeof(DLeafContrib));
  std::memcpy(blob.data() + Y->o_vptrL, Y->vptrL.data(), Y->vptrL.size() * 4);
  std::memcpy(blob.data() + Y->o_vertsL, Y->vertsL.data(), Y->vertsL.size() * 4);
  std::memcpy(blob.data() + Y->o_seplev, P.seplev.data(), size_t(P.N));
  // leaf boundary vertex lists into the int arena image
  std::vector<int32_t> leaf_ints;
  HIPCHK(hipMemcpyAsync(F->ws, blob.data(), blob.size(), hipMemcpyHostToDevice, F->stream));
  {
    // bverts of each leaf: concatenated level-L segment vertices
    const PLevel& PLL = P.levels[P.L];
    for (size_t i = 0; i < P.leaves.size(); ++i) {
      std::vector<int32_t> bv;
      for (int s : P.leaves[i].bsegs)
        for (int32_t v : PLL.segs[s].verts) bv.push_back(v);
      if (!bv.empty())
        HIPCHK(hipMemcpyAsync(F->ws + Y->o_iarena + size_t(Y->leaves[i].ioff) * 4, bv.data(), bv.size() * 4,
                              hipMemcpyHostToDevice, F->stream));
    }
  }
  int status = 0;
  int rc = o.precision == SPALU_FP64 ? run_factor<double>(F.get(), o, &status)
                                     : run_factor<float>(F.get(), o, &status);
  if (rc) return rc;
  if (status & 2) return fail(SPALU_EUNSUPPORTED, "matrix pattern is not inside the grid stencil");
  // statistics
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->n = n;
    info->levels = P.L;
    info->segments = Y->nseg_total;
    info->workspace_bytes = int64_t(Y->bytes);
    info->singular_level = -1;
    double q = 0.0;
    int64_t spc = 0, passes = 0, res = 0, mf = 0;
    for (int l = 1; l <= P.L; ++l) {
      const size_t ns = Y->lv[l].segs.size();
      std::vector<int32_t> dv(6 * ns);
      HIPCHK(hipMemcpy(dv.data(), F->ws + Y->lv[l].o_dyn, dv.size() * 4, hipMemcpyDeviceToHost));
      int e = 0, e2 = 0;
      bool any = false;
      for (size_t c = 0; c < ns; ++c) {
        const int nn = dv[c], kk = dv[ns + c], pp = dv[4 * ns + c];
        mf = std::max<int64_t>(mf, nn);
        if (pp > 0) {
          any = true;
          ++spc;
          passes += pp;
          res += pp > 1;
          e = std::max(e, nn);
          e2 = std::max(e2, kk);
        }
      }
      if (any && e > 0) q = std::max(q, double(e2) / e);
    }
    info->sparsified = spc;
    info->sample_passes = passes;
    info->resampled = res;
    info->max_front = mf;
    info->q_tilde = q;
  }
  if (status & 1) {
    if (info) info->singular_level = 0;
    return fail(SPALU_ESINGULAR, "zero pivot in a diagonal block");
  }
  *out = F.release();
  return SPALU_OK;
}

int spalu_factor_ranks(const spalu_factor_t* f, int32_t* n_before, int32_t* rank, int32_t* h, int32_t* passes) {
  if (!f) return fail(SPALU_EINVAL, "f is NULL");
  const Layout& Y = *f->lay;
  HIPCHK(hipStreamSynchronize(f->stream));
  for (int l = 1; l <= f->nd->plan.L; ++l) {
    const size_t ns = Y.lv[l].segs.size();
    std::vector<int32_t> dv(6 * ns);
    HIPCHK(hipMemcpy(dv.data(), f->ws + Y.lv[l].o_dyn, dv.size() * 4, hipMemcpyDeviceToHost));
    const size_t b = size_t(Y.seg_base[l]);
    for (size_t c = 0; c < ns; ++c) {
      if (n_before) n_before[b + c] = dv[c];
      if (rank) rank[b + c] = dv[ns + c];
      if (h) h[b + c] = dv[3 * ns + c];
      if (passes) passes[b + c] = dv[4 * ns + c];
    }
  }
  return SPALU_OK;
}

void spalu_factor_free(spalu_factor_t* f) { delete f; }

int spalu_solve_workspace(const spalu_factor_t* f, int32_t nrhs, size_t* bytes) {
  if (!f || !bytes || nrhs < 1) return fail(SPALU_EINVAL, "bad argument");
  *bytes = solve_layout(f, nrhs).bytes;
  return SPALU_OK;
}

int spalu_solve(const spalu_factor_t* f, int32_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                const spalu_solve_opts* opts, void* workspace, size_t workspace_bytes, void* stream,
                double* rel_res, spalu_solve_info* info) {
  if (!f || !B || !X || !workspace || nrhs < 1) return fail(SPALU_EINVAL, "bad argument");
  if (ldb < f->n || ldx < f->n) return fail(SPALU_EINVAL, "leading dimension < n");
  if (workspace_bytes < solve_layout(f, nrhs).bytes) return fail(SPALU_ENOMEM, "workspace too small");
  spalu_solve_opts so{0.0, 30};
  if (opts) so = *opts;
  if (so.max_iter < 0) return fail(SPALU_EINVAL, "bad max_iter");
  if (so.tol > 0.0 && X == B) return fail(SPALU_EINVAL, "refinement needs X != B");
  spalu_factor_t* F = const_cast<spalu_factor_t*>(f);
  hipStream_t keep = F->stream;
  F->stream = static_cast<hipStream_t>(stream);
  int rc = f->prec == SPALU_FP64
               ? run_solve<double>(f, nrhs, B, ldb, X, ldx, so, static_cast<char*>(workspace), rel_res, info)
               : run_solve<float>(f, nrhs, B, ldb, X, ldx, so, static_cast<char*>(workspace), rel_res, info);
  F->stream = keep;
  return rc;
}

}  // extern "C"

// C ABI of the spaLU library: nested dissection, factorization and solve on
// one MI355X.  See include/spalu.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/spalu.h"
#include "kernels_factor.hpp"
#include "kernels_id.hpp"
#include "kernels_mlp.hpp"
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
  // host adjacency as flat arrays (segment c's neighbours are
  // adj_d[adj_ptr[c] .. adj_ptr[c+1])), built at the first read-back
  mutable std::vector<int32_t> adj_ptr, adj_d;
  std::vector<DBlk> blks;
  std::vector<int32_t> scale_list;
  std::vector<int32_t> cons_ptr, cons;  // merge into level l-1 (l >= 2)
  std::vector<int32_t> task_ptr;
  std::vector<DTask> tasks;
  std::vector<DSepTerm> terms;
  size_t o_segs = 0, o_nbrs = 0, o_blks = 0, o_scale = 0, o_cons_ptr = 0, o_cons = 0, o_task_ptr = 0,
         o_tasks = 0, o_terms = 0, o_dyn = 0;
  // ID launches of the level (bounds from the uncompressed sizes)
  IdTiers tiers{0, 0, 0, 8, 0, 2};
  int tiers_gen = -1;  // tuning generation the tiers were planned with
  bool id_b = false, id_b2 = false, id_c = false, id_cg = false, id_old = false;
  int max_cap = 0;  // largest uncompressed segment
  int max_nbrs = 0;          // largest neighbour count of a segment
  int scale_wave_lds = 0;    // LDS doubles of the one-wave coupling scaling
  int scale_mfma_lds = 0;    // LDS bytes of the matrix-core coupling scaling
  bool scale_block_old = false;  // blocks may exceed the matrix-core scaling
  bool scale_block = false;  // some block exceeds the one-wave coupling scaling
};

struct Layout {
  int prec = 0;
  size_t vsize = 8;
  std::vector<LevelTabs> lv;  // 1..L
  std::vector<DLeaf> leaves;
  std::vector<int32_t> lc_ptr;
  std::vector<DLeafContrib> lc;
  std::vector<int32_t> vptrL, vertsL;
  size_t o_leaves = 0, o_lc_ptr = 0, o_lc = 0, o_vptrL = 0, o_vertsL = 0, o_seplev = 0, o_sepv = 0;
  std::vector<int32_t> sepv;  // separator vertices, ascending
  size_t blob_bytes = 0;
  size_t o_iarena = 0, n_iarena = 0;
  size_t o_varena = 0, n_varena = 0;
  size_t o_scratch = 0, n_scratch = 0;
  size_t leaf_scr_stride = 0;
  size_t leaf_need_min = 0;  // smallest LDS staging need of a leaf (doubles)
  int leaf_wc = 0;                 // register slots of the one-wave leaf kernels (0: block kernels)
  int leaf_wave_lds = 0;           // their dynamic LDS bytes (factor)
  int leaf_ni_max = 0;
  int leaf_nb_max = 0;
  size_t o_status = 0;
  size_t o_feats = 0, o_hinit = 0;  // rank predictor: features, start samples
  size_t o_vfeat = 0;               // rank predictor: per-vertex feature parts (3 doubles)
  size_t bytes = 0;
  int64_t nseg_total = 0;
  std::vector<int64_t> seg_base;  // per level
  size_t leaf_i0 = 0, leaf_i1 = 0;  // int-arena range of the leaf lists
  int dim = 2, L = 0;
  double nsep_verts = 0.0;  // vertices on separators (all levels)
  // host image of the tables (pinned), rebuilt only when rho changes, and
  // its copy in device memory (device dimage_dev), from which every
  // factorization's workspace is filled by a device-to-device copy
  char* image = nullptr;
  size_t image_bytes = 0;
  double image_rho = -1.0;
  char* dimage = nullptr;
  int dimage_dev = -1;
  double dimage_rho = -1.0;
  // one event per stream that copied out of dimage, recorded after its last
  // copy: a replaced image is freed once every such copy is done (not by a
  // device-wide synchronisation)
  std::vector<std::pair<hipStream_t, hipEvent_t>> dimage_read;
  void wait_image_readers() const {
    for (const auto& se : dimage_read) (void)hipEventSynchronize(se.second);
  }
  // pinned staging of the read-back of the per-level size arrays
  mutable char* dyn_pinned = nullptr;
  ~Layout() {
    if (image) (void)hipHostFree(image);
    wait_image_readers();
    if (dimage) (void)hipFree(dimage);
    for (const auto& se : dimage_read) (void)hipEventDestroy(se.second);
    if (dyn_pinned) (void)hipHostFree(dyn_pinned);
  }
};

}  // namespace

// Captured solve sweeps: one graph per set of pointers it bakes in.
struct SweepGraph {
  const void *ws, *sw, *rowptr, *colind, *vals;
  int nrhs, prec;
  std::vector<int> shape;  // launch shapes baked in (per level: lanes, rows, largest skeleton and segment)
  hipGraphExec_t exec;
};

// Side streams (default priority) and events of a factorization, created
// once per ordering handle and shared by its factorizations (which do not
// run concurrently): a level's ID size tiers run concurrently, forked after
// the level's setup and joined before its segment LU; after the segment LU,
// the merge sizes and the next level's features and predictions run on
// aux[0] beside the coupling scaling.
struct FactorStreams {
  hipStream_t aux[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[3] = {nullptr, nullptr, nullptr};
  hipEvent_t lu_done = nullptr, msize_done = nullptr, pre_done = nullptr;
  ~FactorStreams() {
    for (hipStream_t s : aux)
      if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t e : {fork, join[0], join[1], join[2], lu_done, msize_done, pre_done})
      if (e) (void)hipEventDestroy(e);
  }
};

// Captured factorizations: one graph per key (factor_graph_key).
struct FactorGraph {
  std::vector<uint64_t> key;
  hipGraphExec_t exec;
};

struct spalu_nd_s {
  Plan plan;
  std::shared_ptr<Layout> layout[2];
  std::vector<SweepGraph> graphs;    // most recent last
  std::vector<FactorGraph> fgraphs;  // most recent last
  hipStream_t capture_stream = nullptr;
  FactorStreams fs;
  ~spalu_nd_s() {
    for (auto& gph : graphs) (void)hipGraphExecDestroy(gph.exec);
    for (auto& gph : fgraphs) (void)hipGraphExecDestroy(gph.exec);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
};

struct spalu_factor_s {
  const spalu_nd_t* nd = nullptr;
  const Layout* lay = nullptr;
  std::shared_ptr<const Layout> lay_sp;
  int prec = 0;
  int sym = 0;  // symmetric form (one-sided IDs, balanced L D L^T segment factors)
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* colind = nullptr;
  const double* vals = nullptr;
  GridGeom g{};
  // per level: n, k, nr, h, passes, off (host copy after the factorization)
  std::shared_ptr<std::vector<std::vector<int32_t>>> dyn_host;
  // launch shapes of the solve sweeps from the actual sizes, per level: the
  // segment-size bound P of the one-wave kernels (0: 256-thread kernels),
  // the largest stacked neighbour skeleton of an owner, the largest
  // skeleton (the row passes of the 256-thread separator kernels) and the
  // largest segment (the 256-thread segment kernel and its LDS)
  std::vector<int> solve_P, solve_rows, solve_kmax, solve_nmax;
  // side streams and events (owned by the ordering handle)
  FactorStreams* fs = nullptr;
};

namespace {

// LDS limits of the column-parallel ID tiers (bytes of dynamic LDS; a gfx950
// workgroup may hold up to 160 KB).
constexpr size_t ID_LDS_LIMIT = 152 * 1024;  // largest LDS of one group (one per CU)
constexpr size_t SEGLU_MAX_BYTES = 152 * 1024;   // segment LU of large segments
constexpr int SEGLU_WAVE_MAX_N = 32;             // segments up to this size: one wave each
constexpr int ID_BLK_THREADS = 1024;             // block ID of segments over 128 DOFs: sixteen waves
constexpr int SEGLU_BLOCK_NT = 256;              // threads of the block segment LU (one block per CU)
constexpr int SEGLU_WIDE_N = 128;                // segments beyond this size: the wide segment LU
constexpr int SEGLU_WIDE_NT = 1024;              // its threads
constexpr size_t MELIM_MAX_BYTES = 152 * 1024;  // staged separator terms of the merge (at most: one group per CU)

// Launch-shape choices (the autotuner's search space); the defaults are the
// measured hand choices: ID tier A groups of at most 24 KB (six or more per
// CU), tier B 72 KB (two per CU), B2 and C 152 KB (one per CU).
spalu_tuning g_tuning = {24 * 1024, 72 * 1024, 152 * 1024, 152 * 1024, 2, 64 * 1024, 32, 8, 64};
int g_tuning_gen = 0;

// Which ID launches a level needs and their LDS budgets.  The sizes known
// here (uncompressed n, coupling-row bound rcap) bound the ones the kernels
// see, so a segment whose bound fits a tier certainly lands in it; the
// kernels themselves decide with the actual sizes.
void plan_id_tiers(LevelTabs& T, int st) {
  const spalu_tuning& tu = g_tuning;
  size_t a = 0, b = 0, b2 = 0;
  bool beyond_a = false, beyond_b = false, beyond_b2 = false, tabs_global = false, wide = false;
  for (const DSeg& D : T.segs) {
    if (!((D.flags & SEG_REGULAR) && (D.flags & SEG_HAS_NBR))) continue;
    const int cap = D.cap, R = D.rcap;
    const size_t na = idc_lds_bytes(1, 1, std::min(cap, 64), R, st, true);
    if (cap <= 64 && na <= size_t(tu.id_lds_a)) {
      a = std::max(a, na);
      continue;
    }
    beyond_a = true;
    const size_t nb = idc_lds_bytes(ID_B_WAVES, 2, std::min(cap, 128), R, st, true);
    if (cap <= 128 && nb <= size_t(tu.id_lds_b)) {
      b = std::max(b, nb);
      continue;
    }
    beyond_b = true;
    const size_t nb2 = idc_lds_bytes(ID_B2_WAVES, 2, std::min(cap, 128), R, st, true);
    if (cap <= 128 && nb2 <= size_t(tu.id_lds_b2)) {
      b2 = std::max(b2, nb2);
      continue;
    }
    beyond_b2 = true;
    const int nc = std::min(cap, 128);
    if (idc_lds_bytes(ID_B2_WAVES, 2, nc, 0, st, false) + idc_table_bytes(nc, R, st) +
            size_t(std::max(nc, R / tu.id_c_ydiv)) * nc * idc_ye(st) > size_t(tu.id_lds_c))
      tabs_global = true;
    if (cap > 128) wide = true;
  }
  // segments beyond a tier by bound may still land in it by their actual
  // sizes: such levels give the tier its full budget
  if (beyond_a) a = size_t(tu.id_lds_a);
  if (beyond_b) b = size_t(tu.id_lds_b);
  if (beyond_b2) b2 = size_t(tu.id_lds_b2);
  T.tiers.st = st;
  T.tiers.budget_a = int(std::max(a, idc_lds_bytes(1, 1, 1, 2, st, true)));
  T.tiers.budget_b = int(std::max(b, idc_lds_bytes(ID_B_WAVES, 2, 1, 2, st, true)));
  T.tiers.budget_b2 = int(std::max(b2, idc_lds_bytes(ID_B2_WAVES, 2, 1, 2, st, true)));
  T.tiers.lds_c = tu.id_lds_c;
  T.tiers.c_ydiv = tu.id_c_ydiv;
  T.tiers_gen = g_tuning_gen;
  T.id_b = beyond_a;
  T.id_b2 = beyond_b;
  T.id_c = beyond_b2;
  T.id_cg = tabs_global;
  T.id_old = wide;
}

// ---------------------------------------------------------------------------
// Static layout of the factorization for one ND and precision.
// ---------------------------------------------------------------------------
std::shared_ptr<Layout> build_layout(const Plan& P, int prec) {
  auto lay = std::make_shared<Layout>();
  Layout& Y = *lay;
  Y.prec = prec;
  Y.vsize = prec == SPALU_FP32 ? 4 : 8;
  const int L = P.L;
  Y.dim = P.dim;
  Y.L = L;
  Y.sepv.clear();
  for (int64_t v = 0; v < int64_t(P.seplev.size()); ++v)
    if (P.seplev[v] > 0) Y.sepv.push_back(int32_t(v));
  Y.nsep_verts = double(Y.sepv.size());
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
      D.sep_level = s.sep_level;
      D.ioff = int64_t(iar);
      iar += size_t(3 * cap + std::max<int64_t>(2 * rcap[c], cap));
      D.lu_off = int64_t(var);
      var += size_t(cap * cap);
      D.t_off = int64_t(var);
      var += size_t(cap * cap / 4 + 1);
      size_t need = size_t(2 * cap * cap);
      if ((D.flags & SEG_REGULAR) && (D.flags & SEG_HAS_NBR))
        need = std::max({need, size_t((3 * rcap[c] + 9) * cap), idc_scratch_doubles(int(cap), int(rcap[c]))});
      D.scr_off = int64_t(level_pool);
      level_pool += need;
    }
    pool = std::max(pool, level_pool);
    plan_id_tiers(T, prec == SPALU_FP32 ? 4 : 8);
    for (const DSeg& D : T.segs) {
      T.max_cap = std::max(T.max_cap, int(D.cap));
      T.max_nbrs = std::max(T.max_nbrs, int(D.nbr_end - D.nbr_begin));
    }
    {
      constexpr int SCALE_WAVE_MAX = 6144;  // 48 KB of LDS per wave at most
      int need = 0;
      size_t need_m = 0;
      for (int32_t b : T.scale_list) {
        const int cc = T.segs[T.blks[b].c].cap, cd = T.segs[T.blks[b].d].cap;
        const int w = blk_scale_wave_need(std::min(cc, 64), std::min(cd, 64), prec == SPALU_FP32 ? 4 : 8);
        if (cc > 64 || cd > 64 || w > SCALE_WAVE_MAX) {
          // beyond the one-wave kernel: the matrix-core kernel for skeletons
          // of at most 128 DOFs within its LDS, the 256-thread kernel else
          T.scale_block = true;
          const size_t m = blk_scale_mfma_bytes(std::min(cc, 128), std::min(cd, 128));
          if (cc > 128 || cd > 128 || m > size_t(SCALE_MFMA_MAX)) T.scale_block_old = true;
          need_m = std::max(need_m, std::min(m, size_t(SCALE_MFMA_MAX)));
        }
        need = std::max(need, std::min(w, SCALE_WAVE_MAX));
      }
      T.scale_wave_lds = std::max(need, 1);
      T.scale_mfma_lds = int(need_m);
    }
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
  size_t leaf_need = 0, leaf_need_min = SIZE_MAX;
  std::vector<std::vector<int32_t>> bsoff(P.leaves.size());
  for (size_t i = 0; i < P.leaves.size(); ++i) {
    const PLeaf& pl = P.leaves[i];
    DLeaf& D = Y.leaves[i];
    for (int a = 0; a < 3; ++a) {
      D.lo[a] = pl.lo[a];
      D.hi[a] = pl.hi[a];
    }
    D.ni = int32_t(pl.interior.size());
    if (D.ni > LEAF_MAX_NI)
      throw std::runtime_error("leaf boxes hold more than 512 vertices; use more ND levels");
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
    // X = A_II^{-1} A_IB (transposed) is written by the one-wave leaf factor
    // only: no room for leaves beyond it (3D leaves)
    D.x_off = int64_t(var);
    if (leaf_wave_slots(D.ni, nb) != 0) var += size_t(D.ni) * nb;
    leaf_need = std::max(leaf_need, size_t(leaf_lds_need(D.ni, nb)));
    leaf_need_min = std::min(leaf_need_min, size_t(leaf_lds_need(D.ni, nb)));
  }
  Y.leaf_need_min = leaf_need_min;
  // one wave per leaf when every leaf fits its register row
  Y.leaf_wc = 0;
  Y.leaf_wave_lds = 0;
  Y.leaf_ni_max = 0;
  {
    int wc = 0;
    bool all = !Y.leaves.empty();
    for (const DLeaf& D : Y.leaves) {
      const int w = leaf_wave_slots(D.ni, D.nb);
      if (w == 0) all = false;
      wc = std::max(wc, w);
      Y.leaf_ni_max = std::max(Y.leaf_ni_max, int(D.ni));
      Y.leaf_nb_max = std::max(Y.leaf_nb_max, int(D.nb));
    }
    if (all) {
      Y.leaf_wc = wc;
      for (const DLeaf& D : Y.leaves)
        Y.leaf_wave_lds = std::max(Y.leaf_wave_lds, leaf_wave_lds_bytes(wc, D.ni, D.nb));
    }
  }
  Y.leaf_i0 = Y.leaves.empty() ? iar : size_t(Y.leaves[0].ioff);
  Y.leaf_i1 = iar;
  if (leaf_need > size_t(LEAF_LDS_DOUBLES)) {
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
  Y.o_sepv = put(Y.sepv.size() * 4);
  Y.blob_bytes = o;
  // dynamic per-level arrays (6 ints per segment)
  for (int l = 1; l <= L; ++l) Y.lv[l].o_dyn = put(DYN_ARRAYS * Y.lv[l].segs.size() * 4);
  Y.o_status = put(64);
  Y.o_feats = put(size_t(Y.nseg_total) * MLP_NF * 4);
  Y.o_hinit = put(size_t(Y.nseg_total) * 4);
  Y.o_vfeat = put(size_t(P.N) * 3 * 8);
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
  d.nfar = base + 6 * ns;
  return d;
}

template <typename X>
const X* tab(char* ws, size_t off) {
  return reinterpret_cast<const X*>(ws + off);
}

unsigned nblocks(int64_t n, int b = WG) { return unsigned(std::max<int64_t>(1, (n + b - 1) / b)); }

constexpr size_t LDS_BYTES = size_t(LDS_DOUBLES) * 8;
constexpr size_t LEAF_LDS_BYTES = size_t(LEAF_LDS_DOUBLES) * 8;


// ---------------------------------------------------------------------------
// Profiling: when enabled, every launch is bracketed by HIP events on the
// launch stream; after the call's final synchronisation the elapsed times
// are accumulated per kernel together with the launch's algorithmic bytes
// and flops, computed from the actual segment sizes.
// ---------------------------------------------------------------------------
enum KId {
  K_CHECK, K_INIT, K_LEAF, K_ASM, K_ID, K_ID_B, K_ID_B2, K_ID_C, K_ID_BLK, K_LU, K_SCALE, K_MSIZE, K_MELIM,
  K_LSOLVE_F, K_SEPLEAF, K_SSOLVE_F, K_SEPFWD, K_SEPBWD, K_SSOLVE_B, K_LSOLVE_B,
  K_RHSIN, K_RHSOUT, K_RESID, K_REDUCE, K_APPLY, K_FEAT, K_MLP, K_SPMV, K_KRYLOV, K_COUNT
};
const char* const kNames[K_COUNT] = {
    "check_pattern", "init_level", "leaf_factor", "assemble_leafL", "seg_id_a", "seg_id_b", "seg_id_b2",
    "seg_id_c", "seg_id_blk", "seg_lu", "blk_scale",
    "merge_sizes", "merge_elim", "leaf_solve_fwd", "sep_from_leaves", "seg_solve_fwd", "sep_fwd",
    "sep_bwd", "seg_solve_bwd", "leaf_solve_bwd", "rhs_in", "rhs_out", "residual", "reduce_cols",
    "solve_sweep_graph", "features", "mlp_rank", "spmv", "krylov"};

struct PendingLaunch {
  int kid, level;
  bool acct;  // carries the level's algorithmic work (false: a further launch of the same step)
  hipEvent_t a, b;
};

struct TimedLaunch {
  int kid, level, nrhs;
  bool acct;
  double ms;
  int64_t nrows;
  std::shared_ptr<const Layout> lay;
  std::shared_ptr<const std::vector<std::vector<int32_t>>> dyn;
  int sym;  // symmetric form (one-sided ID rows)
};

struct Profiler {
  bool on = false;
  int only = -1;  // >= 0: time the launches of this step only
  std::vector<PendingLaunch> pend;
  std::vector<TimedLaunch> done;  // accounted lazily in spalu_profile_read
  std::vector<hipEvent_t> spare;  // events of harvested launches, reused (creating one per launch
                                  // costs host time inside the timed region)
  int64_t launches[K_COUNT] = {};
  double ms[K_COUNT] = {}, bytes[K_COUNT] = {}, flops[K_COUNT] = {};
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!spare.empty()) {
      e = spare.back();
      spare.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  void reset() {
    for (auto& p : pend) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    spare.clear();
    pend.clear();
    done.clear();
    for (int k = 0; k < K_COUNT; ++k) launches[k] = 0, ms[k] = bytes[k] = flops[k] = 0.0;
  }
};
Profiler g_prof;
const bool g_prof_verbose = std::getenv("SPALU_PROFILE_VERBOSE") != nullptr;

int prof_begin(int kid, int level, hipStream_t st, bool acct = true) {
  if (!g_prof.on || (g_prof.only >= 0 && kid != g_prof.only)) return -1;
  PendingLaunch p{kid, level, acct, g_prof.take(), g_prof.take()};
  if (!p.a || !p.b) {
    if (p.a) g_prof.spare.push_back(p.a);
    if (p.b) g_prof.spare.push_back(p.b);
    return -1;
  }
  (void)hipEventRecord(p.a, st);
  g_prof.pend.push_back(p);
  return int(g_prof.pend.size()) - 1;
}

void prof_end(int idx, hipStream_t st) {
  if (idx >= 0) (void)hipEventRecord(g_prof.pend[size_t(idx)].b, st);
}

#define LAUNCH(kid, level, ...)                  \
  do {                                           \
    const int pi_ = prof_begin(kid, level, st);  \
    __VA_ARGS__;                                 \
    HIPCHK(hipGetLastError());                   \
    prof_end(pi_, st);                           \
  } while (0)

// A further launch of a step whose work the first launch already carries.
#define LAUNCH_MORE(kid, level, ...)                    \
  do {                                                  \
    const int pi_ = prof_begin(kid, level, st, false);  \
    __VA_ARGS__;                                        \
    HIPCHK(hipGetLastError());                          \
    prof_end(pi_, st);                                  \
  } while (0)

// Algorithmic work of one launch (bytes that the step must move, flops it
// must do), from the actual sizes; nrhs = 0 for factorization kernels.
using DynHost = std::vector<std::vector<int32_t>>;

void account(const Layout& Y, const DynHost& dh, int64_t nrows, int kid, int l, int nrhs, double& by,
             double& fl, int sym) {
  const double vs = double(Y.vsize);
  const double nnzrow = 2.0 * Y.dim + 1.0;
  by = fl = 0.0;
  auto dynv = [&](int lev, int which, int c) { return double(dh[lev][size_t(which) * Y.lv[lev].segs.size() + c]); };
  switch (kid) {
    case K_LEAF:
      for (auto& L : Y.leaves) {
        const double ni = L.ni, nb = L.nb;
        by += (ni + nb) * (nnzrow * 12.0 + 8.0) + ni * ni * vs + ni * 4.0 + nb * nb * vs;
        fl += 2.0 / 3.0 * ni * ni * ni + 2.0 * ni * ni * nb + 2.0 * nb * nb;
      }
      break;
    case K_ASM: {
      const LevelTabs& T = Y.lv[l];
      for (size_t b = 0; b < T.blks.size(); ++b) {
        const double e = dynv(l, 0, T.blks[b].c) * dynv(l, 0, T.blks[b].d);
        by += e * vs * (1.0 + double(Y.lc_ptr[b + 1] - Y.lc_ptr[b]));
        fl += e * double(Y.lc_ptr[b + 1] - Y.lc_ptr[b]);
      }
      break;
    }
    case K_ID:
    case K_ID_B:
    case K_ID_B2:
    case K_ID_C:
    case K_ID_BLK: {
      // the segments of this launch's size tier (A, B, B2, C in both
      // variants, block kernel)
      const LevelTabs& T = Y.lv[l];
      for (size_t c = 0; c < T.segs.size(); ++c) {
        if (dynv(l, 4, int(c)) <= 0) continue;
        const double n = dynv(l, 0, int(c)), k = dynv(l, 1, int(c)), h = dynv(l, 3, int(c));
        double R = 0.0;
        for (int e = T.segs[c].nbr_begin; e < T.segs[c].nbr_end; ++e) R += (sym ? 1.0 : 2.0) * dynv(l, 0, T.nbrs[e].d);
        const int tier = id_tier_of_size(int(n), int(R), T.tiers);
        if ((tier == 6 ? 4 : tier) != 1 + (kid - K_ID)) continue;
        // sketch G B_F of the far rows (none once h reaches them: exact rows),
        // CPQR of the |N| + h stacked rows, T = R11^-1 R12
        const double nf = dynv(l, 6, int(c)), nn = R - nf;
        by += R * n * vs + k * (n - k) * vs + n * 4.0;
        fl += (h < nf ? 2.0 * h * nf * n : 0.0) + 4.0 * (nn + h) * n * k + k * k * (n - k);
      }
      break;
    }
    case K_LU: {
      const LevelTabs& T = Y.lv[l];
      for (size_t c = 0; c < T.segs.size(); ++c) {
        const double n = dynv(l, 0, int(c)), k = dynv(l, 1, int(c)), nr = dynv(l, 2, int(c));
        by += 2.0 * n * n * vs + k * nr * vs + n * 8.0;
        fl += 2.0 / 3.0 * n * n * n + 4.0 * n * k * nr;
      }
      break;
    }
    case K_SCALE: {
      const LevelTabs& T = Y.lv[l];
      for (int32_t b : T.scale_list) {
        const double kc = dynv(l, 1, T.blks[b].c), kd = dynv(l, 1, T.blks[b].d);
        by += 2.0 * kc * kd * vs + 0.5 * (kc * kc + kd * kd) * vs;
        fl += kc * kc * kd + kc * kd * kd;
      }
      break;
    }
    case K_MSIZE: {
      const LevelTabs& T = Y.lv[l];
      for (size_t c = 0; c < T.segs.size(); ++c) by += 8.0 * dynv(l, 1, int(c));
      break;
    }
    case K_MELIM: {
      const LevelTabs& T = Y.lv[l];
      const LevelTabs& U = Y.lv[l - 1];
      for (size_t b = 0; b < U.blks.size(); ++b) {
        by += dynv(l - 1, 0, U.blks[b].c) * dynv(l - 1, 0, U.blks[b].d) * vs;
        for (int q = T.task_ptr[b]; q < T.task_ptr[b + 1]; ++q) {
          const DTask& tk = T.tasks[size_t(q)];
          const double kc = dynv(l, 1, tk.c), kd = dynv(l, 1, tk.d);
          if (tk.src >= 0) by += kc * kd * vs;
          for (int e = tk.sep_begin; e < tk.sep_end; ++e) {
            const double ks = dynv(l, 1, T.terms[size_t(e)].s);
            by += (kc * ks + ks * kd) * vs;
            fl += 2.0 * kc * ks * kd;
          }
        }
      }
      break;
    }
    case K_LSOLVE_F:
    case K_LSOLVE_B: {
      // the backward pass from the stored A_II^{-1} A_IB when the one-wave
      // leaf factor ran and the leaves fit a wave
      const bool from_x = kid == K_LSOLVE_B && Y.leaf_wc != 0 && Y.leaf_ni_max <= LEAF_WAVE_MAX_NI;
      for (auto& L : Y.leaves) {
        const double ni = L.ni, nb = L.nb;
        if (from_x) {
          by += ni * nb * vs + 2.0 * ni * nrhs * vs + nb * nrhs * vs;
          fl += 2.0 * ni * nb * nrhs;
        } else {
          by += ni * ni * vs + 2.0 * ni * nrhs * vs + (kid == K_LSOLVE_B ? nb * nrhs * vs + ni * nnzrow * 12.0 : 0.0);
          fl += 2.0 * ni * ni * nrhs;
        }
      }
      break;
    }
    case K_SEPLEAF: {
      const double nsep = Y.nsep_verts;
      by = nsep * (nnzrow * 12.0 + 8.0 + 3.0 * nrhs * vs);
      fl = 2.0 * nsep * 2.0 * nrhs;
      break;
    }
    case K_SSOLVE_F:
    case K_SSOLVE_B: {
      const LevelTabs& T = Y.lv[l];
      for (size_t c = 0; c < T.segs.size(); ++c) {
        const double n = dynv(l, 0, int(c)), k = dynv(l, 1, int(c)), nr = dynv(l, 2, int(c));
        by += 0.5 * n * n * vs + k * nr * vs + 2.0 * n * nrhs * vs + n * 4.0;
        fl += n * n * nrhs + 2.0 * k * nr * nrhs;
      }
      break;
    }
    case K_SEPFWD:
    case K_SEPBWD: {
      const LevelTabs& T = Y.lv[l];
      for (size_t c = 0; c < T.segs.size(); ++c) {
        const bool sep = (T.segs[c].flags & SEG_IS_SEP) != 0;
        if (sep != (kid == K_SEPBWD)) continue;
        const double kc = dynv(l, 1, int(c));
        bool any = false;
        for (int e = T.segs[c].nbr_begin; e < T.segs[c].nbr_end; ++e) {
          if (kid == K_SEPFWD && !T.nbrs[e].d_is_sep) continue;
          const double kd = dynv(l, 1, T.nbrs[e].d);
          by += kc * kd * vs + kd * nrhs * vs;
          fl += 2.0 * kc * kd * nrhs;
          any = true;
        }
        if (any) by += 2.0 * kc * nrhs * vs;
      }
      break;
    }
    case K_RHSIN:
    case K_RHSOUT:
      by = double(nrows) * nrhs * (8.0 + vs);
      break;
    case K_RESID:
      // b and x read in FP64; r written in FP64, or (l = 1) into the next
      // right-hand side in the storage type
      by = double(nrows) * (nnzrow * 12.0 + 8.0) + double(nrows) * nrhs * (16.0 + (l == 1 ? vs : 8.0));
      fl = 2.0 * double(nrows) * nnzrow * nrhs;
      break;
    case K_SPMV:
      by = double(nrows) * (nnzrow * 12.0 + 8.0) + 2.0 * double(nrows) * nrhs * 8.0;
      fl = 2.0 * double(nrows) * nnzrow * nrhs;
      break;
    case K_KRYLOV:  // level = basis vectors the launch streams (< 0: per-column scalars only)
      if (l >= 0) {
        by = double(nrows) * nrhs * 8.0 * (l + 2);
        fl = 2.0 * double(nrows) * nrhs * (l + 1);
      }
      break;
    case K_APPLY: {
      double a, b;
      for (int kid2 : {int(K_LSOLVE_F), int(K_SEPLEAF), int(K_LSOLVE_B)}) {
        account(Y, dh, nrows, kid2, 0, nrhs, a, b, sym);
        by += a;
        fl += b;
      }
      for (int l2 = 1; l2 <= Y.L; ++l2)
        for (int kid2 : {int(K_SSOLVE_F), int(K_SEPFWD), int(K_SEPBWD), int(K_SSOLVE_B)}) {
          account(Y, dh, nrows, kid2, l2, nrhs, a, b, sym);
          by += a;
          fl += b;
        }
      break;
    }
    default:
      break;
  }
}

// Collects the event times of the call's launches; the byte/flop accounting
// happens later (spalu_profile_read), outside any timed region.
void prof_flush(const spalu_factor_t* F, int nrhs) {
  if (!g_prof.on) return;
  for (auto& p : g_prof.pend) {
    float ms = 0.f;
    (void)hipEventSynchronize(p.b);
    if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) ms = 0.f;
    g_prof.done.push_back(
        TimedLaunch{p.kid, p.level, nrhs, p.acct, double(ms), F->n, F->lay_sp, F->dyn_host, F->sym});
    g_prof.spare.push_back(p.a);
    g_prof.spare.push_back(p.b);
  }
  g_prof.pend.clear();
}

void prof_account_pending() {
  for (auto& t : g_prof.done) {
    double by, fl;
    by = fl = 0.0;
    if (t.acct) account(*t.lay, *t.dyn, t.nrows, t.kid, t.level, t.nrhs, by, fl, t.sym);
    if (g_prof_verbose)
      std::fprintf(stderr, "spalu-prof %-16s level %2d  %9.4f ms  %12.0f B  %12.0f flop\n", kNames[t.kid], t.level,
                   t.ms, by, fl);
    g_prof.ms[t.kid] += t.ms;
    g_prof.bytes[t.kid] += by;
    g_prof.flops[t.kid] += fl;
    g_prof.launches[t.kid] += 1;
  }
  g_prof.done.clear();
}

// One device-to-host copy of every level's size arrays (they are adjacent
// in the workspace).
int read_dyn_host(spalu_factor_t* F) {
  const Layout& Y = *F->lay;
  const int L = F->nd->plan.L;
  const size_t lo = Y.lv[1].o_dyn, hi = Y.lv[L].o_dyn + DYN_ARRAYS * Y.lv[L].segs.size() * 4;
  if (!Y.dyn_pinned)
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&Y.dyn_pinned), std::max<size_t>(hi - lo, 1), hipHostMallocDefault));
  const char* raw = Y.dyn_pinned;
  HIPCHK(hipMemcpyAsync(Y.dyn_pinned, F->ws + lo, hi - lo, hipMemcpyDeviceToHost, F->stream));
  HIPCHK(hipStreamSynchronize(F->stream));
  auto dh = std::make_shared<DynHost>(size_t(L) + 1);
  for (int l = 1; l <= L; ++l) {
    (*dh)[l].resize(DYN_ARRAYS * Y.lv[l].segs.size());
    std::memcpy((*dh)[l].data(), raw + (Y.lv[l].o_dyn - lo), (*dh)[l].size() * 4);
  }
  F->dyn_host = dh;
  // one-wave kernels for levels whose segments and neighbour counts fit
  // P <= solve_lanes_max (a power of two from solve_lanes_min up; 16-row
  // tiles, so P <= 16 is one tile) and whose stacked-row table fits 48 KB
  F->solve_P.assign(size_t(L) + 1, 0);
  F->solve_rows.assign(size_t(L) + 1, 1);
  F->solve_kmax.assign(size_t(L) + 1, 1);
  F->solve_nmax.assign(size_t(L) + 1, 1);
  for (int l = 1; l <= L; ++l) {
    const LevelTabs& T = Y.lv[l];
    const size_t ns = T.segs.size();
    const int32_t* nv = (*dh)[l].data();
    const int32_t* kv = nv + ns;
    if (T.adj_ptr.size() != ns + 1) {
      T.adj_ptr.resize(ns + 1);
      T.adj_d.clear();
      for (size_t c = 0; c < ns; ++c) {
        T.adj_ptr[c] = int32_t(T.adj_d.size());
        for (int e = T.segs[c].nbr_begin; e < T.segs[c].nbr_end; ++e) T.adj_d.push_back(T.nbrs[e].d);
      }
      T.adj_ptr[ns] = int32_t(T.adj_d.size());
    }
    const int32_t* ap = T.adj_ptr.data();
    const int32_t* ad = T.adj_d.data();
    int mx = T.max_nbrs, rows = 1, kmax = 1, nmax = 1;
    for (size_t c = 0; c < ns; ++c) {
      mx = std::max(mx, int(nv[c]));
      nmax = std::max(nmax, int(nv[c]));
      kmax = std::max(kmax, int(kv[c]));
      int r = 0;
      for (int e = ap[c]; e < ap[c + 1]; ++e) r += kv[ad[e]];
      rows = std::max(rows, r);
    }
    int P = g_tuning.solve_lanes_min;
    while (P < mx) P *= 2;
    if (P > g_tuning.solve_lanes_max) P = 0;
    if (P && sep_mfma_lds_bytes(rows) <= 49152) F->solve_P[l] = P;
    F->solve_rows[l] = rows;
    F->solve_kmax[l] = kmax;
    F->solve_nmax[l] = nmax;
  }
  return SPALU_OK;
}

// Algorithmic flops and bytes of the whole factorization.
void factor_work(const spalu_factor_t* F, double& fl, double& by) {
  const Layout& Y = *F->lay;
  const DynHost& dh = *F->dyn_host;
  fl = by = 0.0;
  double a, b;
  for (int kid : {int(K_LEAF), int(K_ASM)}) {
    account(Y, dh, F->n, kid, Y.L, 0, a, b, F->sym);
    by += a;
    fl += b;
  }
  for (int l = 1; l <= Y.L; ++l)
    for (int kid : {int(K_ID), int(K_ID_B), int(K_ID_B2), int(K_ID_C), int(K_ID_BLK), int(K_LU), int(K_SCALE),
                    int(K_MSIZE), int(K_MELIM)}) {
      if (l == 1 && (kid == K_MSIZE || kid == K_MELIM)) continue;
      account(Y, dh, F->n, kid, l, 0, a, b, F->sym);
      by += a;
      fl += b;
    }
}

template <typename T>
int issue_factor(spalu_factor_t* F, const spalu_factor_opts& o, hipStream_t st) {
  const Layout& Y = *F->lay;
  const Plan& P = F->nd->plan;
  char* ws = F->ws;
  int32_t* iar = reinterpret_cast<int32_t*>(ws + Y.o_iarena);
  T* var = reinterpret_cast<T*>(ws + Y.o_varena);
  double* scr = reinterpret_cast<double*>(ws + Y.o_scratch);
  int* status = reinterpret_cast<int*>(ws + Y.o_status);
  const int L = P.L;
  k_zero_i32<<<1, 64, 0, st>>>(status, 16);
  HIPCHK(hipGetLastError());
  LAUNCH(K_CHECK, 0, k_check_pattern<<<nblocks(F->n), WG, 0, st>>>(F->g, F->n, F->rowptr, F->colind, status));
  if (F->sym)
    LAUNCH_MORE(K_CHECK, 0, k_check_symmetric<<<nblocks(F->n), WG, 0, st>>>(F->n, F->rowptr, F->colind, F->vals,
                                                                          status));
  {
    const LevelTabs& TL = Y.lv[L];
    DLevelDyn dL = dyn_of(ws, Y, L);
    LAUNCH(K_INIT, L, k_init_level<<<unsigned(TL.segs.size()), 64, 0, st>>>(tab<DSeg>(ws, TL.o_segs), int(TL.segs.size()),
                                                           tab<int32_t>(ws, Y.o_vptrL),
                                                           tab<int32_t>(ws, Y.o_vertsL), iar, dL));
    {
      const DLeaf* lt = tab<DLeaf>(ws, Y.o_leaves);
      const unsigned nl = unsigned(Y.leaves.size());
      const size_t wl = size_t(Y.leaf_wave_lds);
      if (Y.leaf_wc == 48) {
        LAUNCH(K_LEAF, L, k_leaf_factor_wave<T, 48><<<nl, 64, wl, st>>>(lt, int(nl), F->g, F->rowptr, F->colind,
                                                                    F->vals, iar, var, status, L + 1));
      } else if (Y.leaf_wc == 80) {
        LAUNCH(K_LEAF, L, k_leaf_factor_wave<T, 80><<<nl, 64, wl, st>>>(lt, int(nl), F->g, F->rowptr, F->colind,
                                                                    F->vals, iar, var, status, L + 1));
      } else if (Y.leaf_wc == 96) {
        LAUNCH(K_LEAF, L, k_leaf_factor_wave<T, 96><<<nl, 64, wl, st>>>(lt, int(nl), F->g, F->rowptr, F->colind,
                                                                    F->vals, iar, var, status, L + 1));
      } else {
        // no LDS at all when no leaf fits its staging (3D leaves): the
        // groups are then limited by waves, not by an unused LDS buffer
        const bool lds_any = Y.leaf_need_min <= size_t(LEAF_LDS_DOUBLES);
        LAUNCH(K_LEAF, L, k_leaf_factor<T><<<nl, WG, lds_any ? LEAF_LDS_BYTES : 0, st>>>(
            lt, int(nl), F->g, F->rowptr, F->colind, F->vals, iar, var, scr, int64_t(Y.leaf_scr_stride), status,
            L + 1, lds_any ? LEAF_LDS_DOUBLES : 0, lds_any ? 0 : 1));
        // every leaf in scratch: X = A_II^{-1} A_IB and S in a second launch
        if (!lds_any)
          LAUNCH_MORE(K_LEAF, L, k_leaf_x_mfma<T><<<nl, WG, 0, st>>>(lt, int(nl), F->g, F->rowptr, F->colind,
                                                                      F->vals, var, scr,
                                                                      int64_t(Y.leaf_scr_stride)));
      }
    }
    // blocks of small segments: one wave each
    if (TL.max_cap <= 32)
      LAUNCH(K_ASM, L, k_assemble_leafL<T, 64><<<unsigned(TL.blks.size()), 64, 0, st>>>(
          tab<DBlk>(ws, TL.o_blks), int(TL.blks.size()), tab<DSeg>(ws, TL.o_segs), iar, dL,
          tab<int32_t>(ws, Y.o_lc_ptr), tab<DLeafContrib>(ws, Y.o_lc), tab<DLeaf>(ws, Y.o_leaves),
          F->rowptr, F->colind, F->vals, var));
    else
      LAUNCH(K_ASM, L, k_assemble_leafL<T, WG><<<unsigned(TL.blks.size()), WG, 0, st>>>(
          tab<DBlk>(ws, TL.o_blks), int(TL.blks.size()), tab<DSeg>(ws, TL.o_segs), iar, dL,
          tab<int32_t>(ws, Y.o_lc_ptr), tab<DLeafContrib>(ws, Y.o_lc), tab<DLeaf>(ws, Y.o_leaves),
          F->rowptr, F->colind, F->vals, var));
  }
  double* vfeat = reinterpret_cast<double*>(ws + Y.o_vfeat);
  const bool predict = o.rank_model || o.features_out;
  if (predict)
    LAUNCH(K_FEAT, -1, k_vertex_features<<<nblocks(F->n), WG, 0, st>>>(F->n, F->rowptr, F->colind, F->vals, F->g,
                                                                      P.dim, vfeat));
  // features of level lv's segments and (with a model) their start samples,
  // on stream sst
  auto features_and_predictions = [&](int lv, hipStream_t sst) -> int {
    hipStream_t st = sst;
    const LevelTabs& TV = Y.lv[lv];
    const int nsv = int(TV.segs.size());
    const DSeg* segv = tab<DSeg>(ws, TV.o_segs);
    DLevelDyn dv = dyn_of(ws, Y, lv);
    float* feats = (o.features_out ? o.features_out : reinterpret_cast<float*>(ws + Y.o_feats)) +
                   size_t(Y.seg_base[lv]) * MLP_NF;
    LAUNCH(K_FEAT, lv, k_features<<<unsigned(nsv), 64, 0, st>>>(segv, nsv, tab<DNbr>(ws, TV.o_nbrs), F->g, P.dim, L,
                                                                lv, o.eps, iar, dv, vfeat, feats));
    if (o.rank_model) {
      int32_t* hinit = reinterpret_cast<int32_t*>(ws + Y.o_hinit);
      const unsigned mblk = unsigned((nsv + WG / MLP_G - 1) / (WG / MLP_G));
      LAUNCH(K_MLP, lv, k_mlp_rank<<<mblk, WG, 0, st>>>(feats, nsv, o.rank_model, segv, dv, o.rank_margin,
                                                          o.rank_pad, o.rank_skip, hinit + Y.seg_base[lv]));
    }
    return int(SPALU_OK);
  };
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
    prm.sym = o.symmetric;
    if (predict) {
      // the finest level here; the others were done on aux[0] during the
      // level below
      if (l == L) {
        const int rc = features_and_predictions(L, st);
        if (rc) return rc;
      } else {
        HIPCHK(hipStreamWaitEvent(st, F->fs->pre_done, 0));
      }
      if (o.rank_model) prm.h_init = reinterpret_cast<int32_t*>(ws + Y.o_hinit);
    }
    {
      const DNbr* nb = tab<DNbr>(ws, T_.o_nbrs);
      const IdTiers tz = T_.tiers;
      // tier A on the main stream, B (then C with its tables in global
      // scratch), B2 and C (then the block kernel) on side streams: every
      // segment belongs to exactly one tier.  Tier B and the global-table
      // C tier share a stream since they rarely both have work on a level
      const bool side[3] = {T_.id_b || T_.id_cg, T_.id_b2, T_.id_c || T_.id_old};
      if (side[0] || side[1] || side[2]) {
        HIPCHK(hipEventRecord(F->fs->fork, st));
        for (int i = 0; i < 3; ++i)
          if (side[i]) HIPCHK(hipStreamWaitEvent(F->fs->aux[i], F->fs->fork, 0));
      }
      LAUNCH(K_ID, l, k_seg_id_cols<T, 1, 1, false, 1><<<unsigned(ns), 64, size_t(tz.budget_a), st>>>(
          segs, ns, nb, blks, F->g, iar, var, scr, d, prm, tz));
      if (side[0]) {
        hipStream_t st = F->fs->aux[0];
        if (T_.id_b)
          LAUNCH(K_ID_B, l, k_seg_id_cols<T, ID_B_WAVES, 2, false, 2><<<unsigned(ns), 64 * ID_B_WAVES,
                                                                        size_t(tz.budget_b), st>>>(
              segs, ns, nb, blks, F->g, iar, var, scr, d, prm, tz));
        if (T_.id_cg)
          LAUNCH_MORE(K_ID_C, l, k_seg_id_cols<T, 8, 2, true, 6><<<unsigned(ns), 512, size_t(tz.lds_c), st>>>(
              segs, ns, nb, blks, F->g, iar, var, scr, d, prm, tz));
      }
      if (side[1]) {
        hipStream_t st = F->fs->aux[1];
        LAUNCH(K_ID_B2, l, k_seg_id_cols<T, ID_B2_WAVES, 2, false, 3><<<unsigned(ns), 64 * ID_B2_WAVES,
                                                                        size_t(tz.budget_b2), st>>>(
            segs, ns, nb, blks, F->g, iar, var, scr, d, prm, tz));
      }
      if (side[2]) {
        hipStream_t st = F->fs->aux[2];
        if (T_.id_c)
          LAUNCH(K_ID_C, l, k_seg_id_cols<T, 8, 2, true, 4, true><<<unsigned(ns), 512, size_t(tz.lds_c), st>>>(
              segs, ns, nb, blks, F->g, iar, var, scr, d, prm, tz));
        if (T_.id_old)
          LAUNCH(K_ID_BLK, l, k_seg_id<T, ID_BLK_THREADS><<<unsigned(ns), ID_BLK_THREADS, LDS_BYTES, st>>>(segs, ns, nb, blks, F->g, iar, var,
                                                                              scr, d, prm, tz));
      }
      for (int i = 0; i < 3; ++i)
        if (side[i]) {
          HIPCHK(hipEventRecord(F->fs->join[i], F->fs->aux[i]));
          HIPCHK(hipStreamWaitEvent(st, F->fs->join[i], 0));
        }
    }
    {
      // segments of up to 32 DOFs: one wave each; wider ones: one block each
      // with up to 152 KB of LDS (scratch beyond that)
      const int nw = std::min(SEGLU_WAVE_MAX_N, T_.max_cap);
      LAUNCH(K_LU, l, k_seg_lu_wave<T, 1><<<unsigned(ns), 64, size_t(seglu_wave_lds_doubles(nw)) * 8, st>>>(
          segs, ns, blks, iar, var, d, status, 0, nw, l, o.symmetric));
      if (T_.max_cap > SEGLU_WAVE_MAX_N) {
        const int64_t cap = T_.max_cap;
        const int big = int(std::min<int64_t>(2 * cap * cap + cap, int64_t(SEGLU_MAX_BYTES / 8)));
        const int wide = 2 * SEGLU_WIDE_N * SEGLU_WIDE_N;  // staging need beyond which a segment is wide
        LAUNCH_MORE(K_LU, l, k_seg_lu<T, SEGLU_BLOCK_NT><<<unsigned(ns), SEGLU_BLOCK_NT, size_t(big) * 8, st>>>(
            segs, ns, blks, iar, var, scr, d, status, 2 * SEGLU_WAVE_MAX_N * SEGLU_WAVE_MAX_N, wide, big, l,
            o.symmetric));
        // wide segments (staged in scratch): 1024 threads, for the few large
        // fronts of the coarse levels
        if (T_.max_cap > SEGLU_WIDE_N)
          LAUNCH_MORE(K_LU, l, k_seg_lu<T, SEGLU_WIDE_NT><<<unsigned(ns), SEGLU_WIDE_NT, 0, st>>>(
              segs, ns, blks, iar, var, scr, d, status, wide, INT32_MAX, 0, l, o.symmetric));
      }
    }
    if (l > 1) {
      // merge sizes (they need the LU's DOF order) and the next level's
      // features and predictions on aux[0], beside the coupling scaling
      HIPCHK(hipEventRecord(F->fs->lu_done, st));
      hipStream_t st = F->fs->aux[0];
      HIPCHK(hipStreamWaitEvent(st, F->fs->lu_done, 0));
      const LevelTabs& U = Y.lv[l - 1];
      LAUNCH(K_MSIZE, l, k_merge_sizes<<<unsigned(U.segs.size()), 64, 0, st>>>(
          tab<DSeg>(ws, U.o_segs), int(U.segs.size()), tab<int32_t>(ws, T_.o_cons_ptr),
          tab<int32_t>(ws, T_.o_cons), segs, iar, d, dyn_of(ws, Y, l - 1)));
      HIPCHK(hipEventRecord(F->fs->msize_done, st));
      if (predict) {
        const int rc = features_and_predictions(l - 1, st);
        if (rc) return rc;
        HIPCHK(hipEventRecord(F->fs->pre_done, st));
      }
    }
    if (!T_.scale_list.empty()) {
      // one wave per block where the skeletons are small, a block of 256
      // threads otherwise
      const unsigned nsc = unsigned(T_.scale_list.size());
      LAUNCH(K_SCALE, l, k_blk_scale_wave<T><<<nsc, 64, size_t(T_.scale_wave_lds) * 8, st>>>(
          blks, tab<int32_t>(ws, T_.o_scale), int(nsc), segs, iar, var, d, T_.scale_wave_lds, o.symmetric));
      if (T_.scale_block)
        LAUNCH_MORE(K_SCALE, l, k_blk_scale_mfma<T><<<nsc, WG, size_t(T_.scale_mfma_lds), st>>>(
            blks, tab<int32_t>(ws, T_.o_scale), int(nsc), segs, iar, var, d, T_.scale_wave_lds,
            T_.scale_mfma_lds, o.symmetric));
      if (T_.scale_block_old)
        LAUNCH_MORE(K_SCALE, l, k_blk_scale<T><<<nsc, WG, LDS_BYTES, st>>>(
            blks, tab<int32_t>(ws, T_.o_scale), int(nsc), segs, iar, var, d, T_.scale_wave_lds,
            T_.scale_mfma_lds, o.symmetric));
    }
    if (l > 1) {
      const LevelTabs& U = Y.lv[l - 1];
      DLevelDyn du = dyn_of(ws, Y, l - 1);
      HIPCHK(hipStreamWaitEvent(st, F->fs->msize_done, 0));
      // blocks of small segments: one wave each
      if (U.max_cap <= g_tuning.melim_wave_cap) {
        // staged terms with LDS for this level's largest skeletons
        const int cap = T_.max_cap;
        const int lb = ((cap * cap * 8 + 15) & ~15) + 2 * cap * cap * int(sizeof(T));
        LAUNCH(K_MELIM, l, k_merge_elim<T, 64><<<unsigned(U.blks.size()), 64, size_t(lb), st>>>(
            tab<DBlk>(ws, U.o_blks), int(U.blks.size()), tab<int32_t>(ws, T_.o_task_ptr),
            tab<DTask>(ws, T_.o_tasks), tab<DSepTerm>(ws, T_.o_terms), blks, var, d, du, lb));
      }
      else {
        // LDS for the level's largest task (accumulator and the two factors
        // of a term), at most one group per CU
        const size_t cap = size_t(T_.max_cap);
        const size_t need = ((cap * cap * 8 + 15) & ~size_t(15)) + 2 * cap * cap * sizeof(T);
        const size_t lb = std::min(MELIM_MAX_BYTES, std::max(size_t(g_tuning.melim_lds), need));
        LAUNCH(K_MELIM, l, k_merge_elim<T, WG><<<unsigned(U.blks.size()), WG, lb, st>>>(
            tab<DBlk>(ws, U.o_blks), int(U.blks.size()), tab<int32_t>(ws, T_.o_task_ptr),
            tab<DTask>(ws, T_.o_tasks), tab<DSepTerm>(ws, T_.o_terms), blks, var, d, du, int(lb)));
        if (T_.max_cap > MELIM_TILE_MIN)  // wide tasks (3D fronts), after the zeroing above
          LAUNCH_MORE(K_MELIM, l, k_merge_elim<T, WG, true><<<unsigned(U.blks.size()), WG, 0, st>>>(
              tab<DBlk>(ws, U.o_blks), int(U.blks.size()), tab<int32_t>(ws, T_.o_task_ptr),
              tab<DTask>(ws, T_.o_tasks), tab<DSepTerm>(ws, T_.o_terms), blks, var, d, du, int(lb)));
      }
    }
  }
  return SPALU_OK;
}

// Raises the LDS limits of the factorization kernels that take more than
// 64 KB (once per process and storage type, before any launch or capture).
template <typename T>
int factor_kernel_setup() {
  static const bool ok = [] {
    auto lds = [](const void* k, size_t b) {
      return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(b)) == hipSuccess;
    };
    bool r = lds(reinterpret_cast<const void*>(&k_seg_id_cols<T, 1, 1, false, 1>), 64 * 1024);
    r = lds(reinterpret_cast<const void*>(&k_seg_id_cols<T, ID_B_WAVES, 2, false, 2>), ID_LDS_LIMIT) && r;
    r = lds(reinterpret_cast<const void*>(&k_seg_id_cols<T, ID_B2_WAVES, 2, false, 3>), ID_LDS_LIMIT) && r;
    r = lds(reinterpret_cast<const void*>(&k_seg_id_cols<T, 8, 2, true, 4, true>), ID_LDS_LIMIT) && r;
    r = lds(reinterpret_cast<const void*>(&k_seg_id_cols<T, 8, 2, true, 6>), ID_LDS_LIMIT) && r;
    r = lds(reinterpret_cast<const void*>(&k_seg_lu<T, SEGLU_BLOCK_NT>), SEGLU_MAX_BYTES) && r;
    r = lds(reinterpret_cast<const void*>(&k_merge_elim<T, WG>), MELIM_MAX_BYTES) && r;
    r = lds(reinterpret_cast<const void*>(&k_blk_scale_mfma<T>), SCALE_MFMA_MAX) && r;
    const size_t sb = size_t(seg_solve_mfma_lds_bytes(SEG_MFMA_BLOCK_N));
    r = lds(reinterpret_cast<const void*>(&k_seg_solve_mfma<T, false, 4, 2>), sb) && r;
    r = lds(reinterpret_cast<const void*>(&k_seg_solve_mfma<T, true, 4, 2>), sb) && r;
    return r;
  }();
  return ok ? int(SPALU_OK) : fail(SPALU_EDEVICE, "cannot raise the LDS limit of a factorization kernel");
}

// Everything a factorization's launches bake in: the workspace and matrix
// pointers, the layout and every option.
std::vector<uint64_t> factor_graph_key(const spalu_factor_t* F, const spalu_factor_opts& o) {
  auto u = [](const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); };
  auto d = [](double x) {
    uint64_t b;
    std::memcpy(&b, &x, 8);
    return b;
  };
  return {u(F->ws), u(F->rowptr), u(F->colind), u(F->vals), uint64_t(F->n), u(F->lay), uint64_t(o.precision),
          d(o.eps), uint64_t(o.seed), d(o.rho), uint64_t(uint32_t(o.h0)), uint64_t(uint32_t(o.probes)), d(o.tau),
          u(o.h_init), u(o.rank_model), u(o.features_out), d(o.rank_margin), uint64_t(uint32_t(o.rank_pad)),
          d(o.rank_skip), uint64_t(uint32_t(o.symmetric)), uint64_t(g_tuning_gen)};
}

// A factorization: its launches issued directly on the factor's stream,
// or (with o.graph, profiling off) replayed from a HIP graph captured the
// first time these pointers and options are seen; then the status and the
// per-level sizes come back to the host.
template <typename T>
int run_factor(spalu_factor_t* F, const spalu_factor_opts& o, int* status_host) {
  spalu_nd_t* nd = const_cast<spalu_nd_t*>(F->nd);
  FactorStreams& FS = nd->fs;
  if (!FS.fork) {
    HIPCHK(hipEventCreateWithFlags(&FS.fork, hipEventDisableTiming));
    for (int i = 0; i < 3; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&FS.aux[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&FS.join[i], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&FS.lu_done, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&FS.msize_done, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&FS.pre_done, hipEventDisableTiming));
  }
  F->fs = &FS;
  int rc = factor_kernel_setup<T>();
  if (rc) return rc;
  hipStream_t st = F->stream;
  if (o.graph && !g_prof.on) {
    const std::vector<uint64_t> key = factor_graph_key(F, o);
    hipGraphExec_t exec = nullptr;
    for (auto& gph : nd->fgraphs)
      if (gph.key == key) exec = gph.exec;
    if (!exec) {
      if (!nd->capture_stream) HIPCHK(hipStreamCreateWithFlags(&nd->capture_stream, hipStreamNonBlocking));
      hipStream_t cs = nd->capture_stream;
      HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      rc = issue_factor<T>(F, o, cs);
      hipGraph_t graph_ = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &graph_);
      if (rc) {
        if (graph_) (void)hipGraphDestroy(graph_);
        return rc;
      }
      if (e != hipSuccess) return fail(SPALU_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      const hipError_t e2 = hipGraphInstantiate(&exec, graph_, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph_);
      if (e2 != hipSuccess) return fail(SPALU_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
      if (nd->fgraphs.size() >= 4) {
        (void)hipGraphExecDestroy(nd->fgraphs.front().exec);
        nd->fgraphs.erase(nd->fgraphs.begin());
      }
      nd->fgraphs.push_back(FactorGraph{key, exec});
    }
    HIPCHK(hipGraphLaunch(exec, st));
  } else {
    rc = issue_factor<T>(F, o, st);
    if (rc) return rc;
  }
  const int* status = reinterpret_cast<const int*>(F->ws + F->lay->o_status);
  HIPCHK(hipMemcpyAsync(status_host, status, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  rc = read_dyn_host(F);
  if (rc) return rc;
  prof_flush(F, 0);
  return SPALU_OK;
}

// Grid of the layout-change kernels: vertex tiles x column tiles.
inline dim3 rhs_grid(int64_t n, int nrhs) {
  return dim3(unsigned((n + RHS_TV - 1) / RHS_TV), unsigned((nrhs + RHS_TJ - 1) / RHS_TJ));
}

struct SolveWs {
  size_t oW, oZ, oB0, oR, oPr, oPb, oNr, oNb;
  size_t oV, oZk, oKs, oKp, oH1, oH2, oEst;  // flexible GMRES (restart > 0)
  size_t bytes;
  unsigned rblk;       // blocks of one row per thread
  unsigned kblk;       // blocks of the Gram-Schmidt kernels (KRY_ROWS rows per thread)
  int rparts, kparts;  // per-wave partial sums of those launches
};

SolveWs solve_layout(const spalu_factor_t* F, int nrhs, int restart = 0) {
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
  s.kblk = unsigned((F->n + int64_t(WG) * KRY_ROWS - 1) / (int64_t(WG) * KRY_ROWS));
  s.rparts = int(s.rblk) * NWAVE;
  s.kparts = int(s.kblk) * NWAVE;
  s.oW = put(nn * vs);
  s.oZ = put(nn * vs);
  s.oB0 = put(nn * vs);
  s.oR = put(nn * 8);
  s.oPr = put(size_t(s.rparts) * nrhs * 8);
  s.oPb = put(size_t(s.rparts) * nrhs * 8);
  s.oNr = put(size_t(nrhs) * 8);
  s.oNb = put(size_t(nrhs) * 8);
  if (restart > 0) {
    const size_t m = size_t(restart);
    s.oV = put((m + 1) * nn * 8);
    s.oZk = put(m * nn * 8);
    s.oKs = put(size_t(nrhs) * kstate_doubles(restart) * 8);
    s.oKp = put((m + 1) * nrhs * size_t(s.kparts) * 8);
    s.oH1 = put((m + 1) * nrhs * 8);
    s.oH2 = put((m + 1) * nrhs * 8);
    s.oEst = put(size_t(nrhs) * 8);
  }
  s.bytes = o;
  return s;
}

// One application of the factor: W <- M^{-1} B0 (both in the working layout).
// LDS of the four-wave segment solve on level l: the FP64 rows of its
// largest segment, rounded up to whole 16-row tiles.
size_t seg_mfma_block_lds(const spalu_factor_t* F, int l) {
  return size_t(seg_solve_mfma_lds_bytes((F->solve_nmax[l] + 15) / 16 * 16));
}

template <typename T>
int apply_inverse(const spalu_factor_t* F, T* B0, T* W, T* Z, int nrhs, hipStream_t st) {
  const Layout& Y = *F->lay;
  const Plan& P = F->nd->plan;
  const int sym = F->sym;
  char* ws = F->ws;
  const int32_t* iar = reinterpret_cast<const int32_t*>(ws + Y.o_iarena);
  const T* var = reinterpret_cast<const T*>(ws + Y.o_varena);
  const int L = P.L;
  const DLeaf* leaves = tab<DLeaf>(ws, Y.o_leaves);
  const bool wave_leaf = Y.leaf_ni_max <= LEAF_WAVE_MAX_NI;
  const size_t lsl = size_t(leaf_solve_wave_lds_bytes(Y.leaf_ni_max));
  if (wave_leaf) {
    LAUNCH(K_LSOLVE_F, 0, k_leaf_solve_wave<T, false><<<unsigned(Y.leaves.size()), 64, lsl, st>>>(
        leaves, int(Y.leaves.size()), F->g, F->rowptr, F->colind, F->vals, var, B0, W, Z, nrhs));
  } else {
    LAUNCH(K_LSOLVE_F, 0, k_leaf_solve<T, false><<<unsigned(Y.leaves.size()), WG, LDS_BYTES, st>>>(
        leaves, int(Y.leaves.size()), F->g, F->rowptr, F->colind, F->vals, iar, var, B0, W, Z, nrhs));
  }
  const int64_t nsep = int64_t(Y.sepv.size());
  LAUNCH(K_SEPLEAF, 0, k_sep_from_leaves<T><<<nblocks(nsep * nrhs), WG, 0, st>>>(
      nsep, tab<int32_t>(ws, Y.o_sepv), tab<int8_t>(ws, Y.o_seplev), F->rowptr, F->colind, F->vals, B0, Z, W,
      nrhs));
  // levels whose segments (by their actual sizes) hold at most P <= 64 DOFs
  // and neighbours take the one-wave matrix-core kernels
  auto seg_solve_grp = [&](const LevelTabs& T_, int l, int P, bool bwd, DLevelDyn d) {
    const DSeg* sg = tab<DSeg>(ws, T_.o_segs);
    const int ns = int(T_.segs.size());
#define SPALU_SSG(RT)                                                                                          \
  {                                                                                                            \
    const size_t lb = size_t(seg_solve_mfma_lds_bytes(16 * RT));                                               \
    if (bwd)                                                                                                   \
      LAUNCH(K_SSOLVE_B, l, k_seg_solve_mfma<T, true, 1, RT><<<unsigned(ns), 64, lb, st>>>(sg, ns, iar, var, d, W, nrhs, sym)); \
    else                                                                                                       \
      LAUNCH(K_SSOLVE_F, l, k_seg_solve_mfma<T, false, 1, RT><<<unsigned(ns), 64, lb, st>>>(sg, ns, iar, var, d, W, nrhs, sym)); \
  }
    if (P <= 16) SPALU_SSG(1) else if (P == 32) SPALU_SSG(2) else SPALU_SSG(4)
#undef SPALU_SSG
    return int(SPALU_OK);
  };
  auto sep_grp = [&](const LevelTabs& T_, int l, int P, bool bwd, DLevelDyn d) {
    const DSeg* sg = tab<DSeg>(ws, T_.o_segs);
    const DNbr* nbr = tab<DNbr>(ws, T_.o_nbrs);
    const DBlk* bk = tab<DBlk>(ws, T_.o_blks);
    const int ns = int(T_.segs.size());
    const int rc = F->solve_rows[l];
    const size_t lb = size_t(sep_mfma_lds_bytes(rc));
#define SPALU_SG(RT, NY)                                                                                       \
  {                                                                                                            \
    const dim3 g(unsigned(ns), NY);                                                                            \
    if (bwd)                                                                                                   \
      LAUNCH(K_SEPBWD, l, k_sep_mfma<T, false, RT><<<g, 64, lb, st>>>(sg, ns, nbr, bk, iar, var, d, W, nrhs, rc)); \
    else                                                                                                       \
      LAUNCH(K_SEPFWD, l, k_sep_mfma<T, true, RT><<<g, 64, lb, st>>>(sg, ns, nbr, bk, iar, var, d, W, nrhs, rc)); \
  }
    if (P <= 16) SPALU_SG(1, 1) else if (P == 32) SPALU_SG(2, 1) else SPALU_SG(2, 2)
#undef SPALU_SG
    return int(SPALU_OK);
  };
  for (int l = L; l >= 1; --l) {
    const LevelTabs& T_ = Y.lv[l];
    const int ns = int(T_.segs.size());
    DLevelDyn d = dyn_of(ws, Y, l);
    const int P = F->solve_P[l];
    if (P) {
      if (const int rc = seg_solve_grp(T_, l, P, false, d)) return rc;
      if (const int rc = sep_grp(T_, l, P, false, d)) return rc;
    } else {
      const DSeg* sg = tab<DSeg>(ws, T_.o_segs);
      if (F->solve_nmax[l] <= SEG_MFMA_BLOCK_N)
        LAUNCH(K_SSOLVE_F, l, k_seg_solve_mfma<T, false, 4, 2><<<unsigned(ns), WG, seg_mfma_block_lds(F, l), st>>>(
                                  sg, ns, iar, var, d, W, nrhs, sym));
      else
        LAUNCH(K_SSOLVE_F, l, k_seg_solve<T, false><<<unsigned(ns), WG, size_t(SEG_SOLVE_LDS_BYTES), st>>>(sg, ns, iar, var, d, W, nrhs, sym));
      const dim3 gsep(unsigned(ns), unsigned((F->solve_kmax[l] + GG_ROWS - 1) / GG_ROWS));
      LAUNCH(K_SEPFWD, l, k_sep_fwd<T><<<gsep, WG, 0, st>>>(sg, ns, tab<DNbr>(ws, T_.o_nbrs),
                                                                   tab<DBlk>(ws, T_.o_blks), iar, var, d, W, nrhs));
    }
  }
  for (int l = 1; l <= L; ++l) {
    const LevelTabs& T_ = Y.lv[l];
    const int ns = int(T_.segs.size());
    DLevelDyn d = dyn_of(ws, Y, l);
    const int P = F->solve_P[l];
    if (P) {
      if (const int rc = sep_grp(T_, l, P, true, d)) return rc;
      if (const int rc = seg_solve_grp(T_, l, P, true, d)) return rc;
    } else {
      const DSeg* sg = tab<DSeg>(ws, T_.o_segs);
      const dim3 gsep(unsigned(ns), unsigned((F->solve_kmax[l] + GG_ROWS - 1) / GG_ROWS));
      LAUNCH(K_SEPBWD, l, k_sep_bwd<T><<<gsep, WG, 0, st>>>(sg, ns, tab<DNbr>(ws, T_.o_nbrs),
                                                                   tab<DBlk>(ws, T_.o_blks), iar, var, d, W, nrhs));
      if (F->solve_nmax[l] <= SEG_MFMA_BLOCK_N)
        LAUNCH(K_SSOLVE_B, l, k_seg_solve_mfma<T, true, 4, 2><<<unsigned(ns), WG, seg_mfma_block_lds(F, l), st>>>(
                                  sg, ns, iar, var, d, W, nrhs, sym));
      else
        LAUNCH(K_SSOLVE_B, l, k_seg_solve<T, true><<<unsigned(ns), WG, size_t(SEG_SOLVE_LDS_BYTES), st>>>(sg, ns, iar, var, d, W, nrhs, sym));
    }
  }
  if (wave_leaf && Y.leaf_wc != 0) {
    // x_I = y_I - (A_II^{-1} A_IB) x_B with y_I from the forward pass
    LAUNCH(K_LSOLVE_B, 0, k_leaf_solve_bwd_x<T><<<unsigned(Y.leaves.size()), 64,
                                                  size_t(leaf_bwd_x_lds_bytes(Y.leaf_nb_max)), st>>>(
        leaves, int(Y.leaves.size()), F->g, iar, var, W, Z, nrhs));
  } else if (wave_leaf) {
    LAUNCH(K_LSOLVE_B, 0, k_leaf_solve_wave<T, true><<<unsigned(Y.leaves.size()), 64, lsl, st>>>(
        leaves, int(Y.leaves.size()), F->g, F->rowptr, F->colind, F->vals, var, B0, W, Z, nrhs));
  } else {
    LAUNCH(K_LSOLVE_B, 0, k_leaf_solve<T, true><<<unsigned(Y.leaves.size()), WG, LDS_BYTES, st>>>(
        leaves, int(Y.leaves.size()), F->g, F->rowptr, F->colind, F->vals, iar, var, B0, W, Z, nrhs));
  }
  return SPALU_OK;
}

// One application of the factor on stream st, either as direct launches
// or as a replay of a captured graph of the same launches.
template <typename T>
int apply(const spalu_factor_t* F, T* B0, T* W, T* Z, int nrhs, const char* sw, bool graph,
          hipStream_t st) {
  if (!graph) return apply_inverse<T>(F, B0, W, Z, nrhs, st);
  spalu_nd_t* nd = const_cast<spalu_nd_t*>(F->nd);
  hipGraphExec_t exec = nullptr;
  std::vector<int> shape(F->solve_P);
  shape.insert(shape.end(), F->solve_rows.begin(), F->solve_rows.end());
  shape.insert(shape.end(), F->solve_kmax.begin(), F->solve_kmax.end());
  shape.insert(shape.end(), F->solve_nmax.begin(), F->solve_nmax.end());
  for (auto& gph : nd->graphs)
    if (gph.ws == F->ws && gph.sw == sw && gph.rowptr == F->rowptr && gph.colind == F->colind &&
        gph.vals == F->vals && gph.nrhs == nrhs && gph.prec == F->prec && gph.shape == shape)
      exec = gph.exec;
  if (!exec) {
    if (!nd->capture_stream) HIPCHK(hipStreamCreateWithFlags(&nd->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = nd->capture_stream;
    const bool prof_was = g_prof.on;  // no event records inside the capture
    g_prof.on = false;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = apply_inverse<T>(F, B0, W, Z, nrhs, cs);
    g_prof.on = prof_was;
    hipGraph_t graph_ = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph_);
    if (rc) {
      if (graph_) (void)hipGraphDestroy(graph_);
      return rc;
    }
    if (e != hipSuccess) return fail(SPALU_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&exec, graph_, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph_);
    if (e2 != hipSuccess) return fail(SPALU_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    if (nd->graphs.size() >= 8) {
      (void)hipGraphExecDestroy(nd->graphs.front().exec);
      nd->graphs.erase(nd->graphs.begin());
    }
    nd->graphs.push_back(SweepGraph{F->ws, sw, F->rowptr, F->colind, F->vals, nrhs, F->prec, shape, exec});
  }
  const int pi = prof_begin(K_APPLY, 0, st);
  HIPCHK(hipGraphLaunch(exec, st));
  prof_end(pi, st);
  return SPALU_OK;
}

template <typename T>
int run_solve(const spalu_factor_t* F, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
              const spalu_solve_opts& so, char* sw, double* rel_res, spalu_solve_info* info) {
  const SolveWs s = solve_layout(F, nrhs, so.restart);
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
  LAUNCH(K_RHSIN, 0, k_rhs_in<T><<<rhs_grid(F->n, nrhs), WG, 0, st>>>(B, ldb, F->n, nrhs, B0));
  const bool graph = so.graph != 0;
  int rc = apply<T>(F, B0, W, Z, nrhs, sw, graph, st);
  if (rc) return rc;
  LAUNCH(K_RHSOUT, 0, k_rhs_out<T><<<rhs_grid(F->n, nrhs), WG, 0, st>>>(W, F->n, nrhs, X, ldx, 0));
  if (!want_res) {
    prof_flush(F, nrhs);
    return SPALU_OK;
  }
  std::vector<double> hr(nrhs), hb(nrhs);
  double first = -1.0, worst = 0.0, prev = -1.0;
  int it = 0, slow = 0;
  std::vector<double> bnorm;
  // classical refinement writes each residual straight into B0, the next
  // correction's right-hand side
  const bool r_to_b0 = so.restart == 0 && !alias;
  while (true) {
    if (r_to_b0)
      LAUNCH(K_RESID, 1, k_residual<T, true><<<s.rblk, WG, 0, st>>>(F->n, nrhs, F->rowptr, F->colind, F->vals, Bsrc,
                                                                   ldbres, X, ldx, nullptr, B0, pr, pb, s.rparts));
    else
      LAUNCH(K_RESID, 0, k_residual<double, false><<<s.rblk, WG, 0, st>>>(F->n, nrhs, F->rowptr, F->colind, F->vals,
                                                                         Bsrc, ldbres, X, ldx, R, nullptr, pr, pb,
                                                                         s.rparts));
    LAUNCH(K_REDUCE, 0, k_reduce_cols<<<unsigned(nrhs), WG, 0, st>>>(pr, s.rparts, nr));
    if (bnorm.empty()) {
      LAUNCH(K_REDUCE, 0, k_reduce_cols<<<unsigned(nrhs), WG, 0, st>>>(pb, s.rparts, nb));
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
    // stagnation or divergence: three steps without a 10% reduction, or a
    // non-finite residual
    if (!std::isfinite(worst)) break;
    slow = (prev >= 0.0 && !(worst <= 0.9 * prev)) ? slow + 1 : 0;
    prev = worst;
    if (slow >= 3) break;
    if (so.restart == 0) {
      // correction: solve with r (already in B0) as right-hand side, x += M r
      rc = apply<T>(F, B0, W, Z, nrhs, sw, graph, st);
      if (rc) return rc;
      LAUNCH(K_RHSOUT, 0, k_rhs_out<T><<<rhs_grid(F->n, nrhs), WG, 0, st>>>(W, F->n, nrhs, X, ldx, 1));
      ++it;
      continue;
    }
    // correction by one cycle of flexible GMRES(m) on A d = r, right
    // preconditioned by the factor; x += Z y
    const int m = so.restart;
    double* V = reinterpret_cast<double*>(sw + s.oV);
    double* Zk = reinterpret_cast<double*>(sw + s.oZk);
    double* ks = reinterpret_cast<double*>(sw + s.oKs);
    double* kp = reinterpret_cast<double*>(sw + s.oKp);
    double* h1 = reinterpret_cast<double*>(sw + s.oH1);
    double* h2 = reinterpret_cast<double*>(sw + s.oH2);
    double* est = reinterpret_cast<double*>(sw + s.oEst);
    const dim3 vgrid(s.rblk, unsigned(nrhs));
    const unsigned cblk = unsigned((nrhs + 63) / 64);
    LAUNCH(K_KRYLOV, -1, k_kstart<<<cblk, 64, 0, st>>>(nrhs, m, nr, ks));
    LAUNCH(K_KRYLOV, 0, k_kscale<<<vgrid, WG, 0, st>>>(F->n, m, ks, R, V));
    int kdone = 0;
    std::vector<double> he(nrhs);
    for (int c = 0; c < m && it < so.max_iter; ++c) {
      double* Vc = V + size_t(c) * nn;
      double* Zc = Zk + size_t(c) * nn;
      LAUNCH(K_RHSIN, 0, k_rhs_in<T><<<rhs_grid(F->n, nrhs), WG, 0, st>>>(Vc, F->n, F->n, nrhs, B0));
      rc = apply<T>(F, B0, W, Z, nrhs, sw, graph, st);
      if (rc) return rc;
      LAUNCH(K_RHSOUT, 0, k_rhs_out<T><<<rhs_grid(F->n, nrhs), WG, 0, st>>>(W, F->n, nrhs, Zc, F->n, 0));
      ++it;
      LAUNCH(K_SPMV, 0, k_spmv<<<s.rblk, WG, 0, st>>>(F->n, nrhs, F->rowptr, F->colind, F->vals, Zc, R));
      // two classical Gram-Schmidt passes: the dots of w; w -= V h1 with
      // the dots of the result; then V_{c+1} = (w - V h2) / H[c+1][c]
      const dim3 kgrid(s.kblk, unsigned(nrhs));
      LAUNCH(K_KRYLOV, c + 1, k_kdots<<<kgrid, WG, 0, st>>>(F->n, nrhs, V, c + 1, R, kp, s.kparts));
      LAUNCH(K_KRYLOV, -1, k_reduce_cols<<<unsigned((c + 2) * nrhs), WG, 0, st>>>(kp, s.kparts, h1));
      LAUNCH(K_KRYLOV, c + 1, k_korth_dots<<<kgrid, WG, 0, st>>>(F->n, nrhs, V, c + 1, h1, R, kp, s.kparts));
      LAUNCH(K_KRYLOV, -1, k_reduce_cols<<<unsigned((c + 2) * nrhs), WG, 0, st>>>(kp, s.kparts, h2));
      LAUNCH(K_KRYLOV, -1, k_karnoldi<<<cblk, 64, 0, st>>>(nrhs, m, c, h1, h2, ks, est));
      LAUNCH(K_KRYLOV, c + 1, k_korth_scale<<<kgrid, WG, 0, st>>>(F->n, nrhs, m, V, c + 1, h2, ks, R,
                                                                   V + size_t(c + 1) * nn));
      kdone = c + 1;
      HIPCHK(hipMemcpyAsync(he.data(), est, size_t(nrhs) * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      double wk = 0.0;
      for (int j = 0; j < nrhs; ++j) wk = std::max(wk, he[j] / bnorm[j]);
      if (!(wk > 0.5 * so.tol)) break;  // converged (or not finite: the outer check decides)
    }
    LAUNCH(K_KRYLOV, -1, k_ksolve<<<cblk, 64, 0, st>>>(nrhs, m, kdone, ks));
    LAUNCH(K_KRYLOV, kdone, k_kupdate<<<vgrid, WG, 0, st>>>(F->n, nrhs, m, kdone, ks, Zk, X, ldx));
  }
  prof_flush(F, nrhs);
  if (info) {
    info->iterations = it;
    info->max_rel_residual = worst;
    info->first_rel_residual = first;
  }
  if (so.tol > 0.0 && worst > so.tol) return fail(SPALU_ENOCONV, "refinement did not reach the tolerance");
  return SPALU_OK;
}

}  // namespace


// Working memory of the allocation-free solve (spalu_solve_static): one
// file-scope device array, which every GPU the library runs on holds until
// the process ends.  In host code its name stands for the host-side shadow,
// not a device address: kernels get the address that hipGetSymbolAddress
// returns for the current device, looked up once per device.
constexpr size_t SPALU_STATIC_SOLVE_BYTES = size_t(64) << 20;
static __device__ __align__(256) char scratch[SPALU_STATIC_SOLVE_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;  // device -> address of scratch there

int scratch_on_device(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SPALU_EDEVICE, "hipGetSymbolAddress returned no address for the solve scratch");
    it = g_scratch_ptr.emplace(dev, static_cast<char*>(p)).first;
  }
  *out = it->second;
  return SPALU_OK;
}
}  // namespace

// Host image of every table plus the leaf boundary lists, in pinned memory
// so the upload of a factorization is two asynchronous copies.  Rebuilt only
// when the near-field radius option changes.
static int build_image(const Plan& P, Layout* Y, double rho) {
  if (Y->image && Y->image_rho == rho) return SPALU_OK;
  const size_t bytes = Y->blob_bytes + (Y->leaf_i1 - Y->leaf_i0) * 4;
  if (!Y->image || Y->image_bytes < bytes) {
    if (Y->image) (void)hipHostFree(Y->image);
    Y->image = nullptr;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&Y->image), std::max<size_t>(bytes, 1), hipHostMallocDefault));
    Y->image_bytes = bytes;
  }
  char* blob = Y->image;
  std::memset(blob, 0, Y->blob_bytes);
  auto cp = [&](size_t off, const void* src, size_t b) {
    if (b) std::memcpy(blob + off, src, b);
  };
  for (int l = 1; l <= P.L; ++l) {
    const LevelTabs& T = Y->lv[l];
    std::vector<DSeg> segs = T.segs;
    for (auto& sg : segs) {
      int span = 0;
      for (int a = 0; a < 3; ++a) span = std::max(span, sg.hi[a] - sg.lo[a] + 1);
      sg.thr = std::max(1, int(std::ceil(rho * span)));
    }
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
  cp(Y->o_leaves, Y->leaves.data(), Y->leaves.size() * sizeof(DLeaf));
  cp(Y->o_lc_ptr, Y->lc_ptr.data(), Y->lc_ptr.size() * 4);
  cp(Y->o_lc, Y->lc.data(), Y->lc.size() * sizeof(DLeafContrib));
  cp(Y->o_vptrL, Y->vptrL.data(), Y->vptrL.size() * 4);
  cp(Y->o_vertsL, Y->vertsL.data(), Y->vertsL.size() * 4);
  cp(Y->o_seplev, P.seplev.data(), size_t(P.N));
  cp(Y->o_sepv, Y->sepv.data(), Y->sepv.size() * 4);
  // leaf boundary lists (then an unused piv range) in the int-arena layout
  int32_t* li = reinterpret_cast<int32_t*>(blob + Y->blob_bytes);
  std::memset(li, 0, (Y->leaf_i1 - Y->leaf_i0) * 4);
  const PLevel& PLL = P.levels[P.L];
  for (size_t i = 0; i < P.leaves.size(); ++i) {
    int32_t* dst = li + (size_t(Y->leaves[i].ioff) - Y->leaf_i0);
    for (int sg : P.leaves[i].bsegs)
      for (int32_t v : PLL.segs[sg].verts) *dst++ = v;
  }
  Y->image_rho = rho;
  return SPALU_OK;
}
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
  o->tau = 1.0;
  o->h_init = nullptr;
  o->rank_model = nullptr;
  o->features_out = nullptr;
  o->rank_margin = 1.0f;
  o->rank_pad = 5;
  o->rank_skip = 0.5f;
  o->graph = 0;
  o->symmetric = 0;
}

void spalu_tuning_default(spalu_tuning* t) {
  if (t) *t = spalu_tuning{24 * 1024, 72 * 1024, 152 * 1024, 152 * 1024, 2, 64 * 1024, 32, 8, 64};
}

int spalu_tuning_get(spalu_tuning* t) {
  if (!t) return fail(SPALU_EINVAL, "t is NULL");
  *t = g_tuning;
  return SPALU_OK;
}

int spalu_tuning_set(const spalu_tuning* t) {
  if (!t) return fail(SPALU_EINVAL, "t is NULL");
  const int64_t lim = int64_t(ID_LDS_LIMIT);
  auto in = [](int64_t v, int64_t lo, int64_t hi) { return v >= lo && v <= hi; };
  auto pow2 = [](int v) { return v == 8 || v == 16 || v == 32 || v == 64; };
  if (!in(t->id_lds_a, 4096, 65536) || !in(t->id_lds_b, 16384, lim) || !in(t->id_lds_b2, 16384, lim) ||
      !in(t->id_lds_c, 32768, lim) || !(t->id_c_ydiv == 1 || t->id_c_ydiv == 2 || t->id_c_ydiv == 4) ||
      !in(t->melim_lds, 16384, lim) || !in(t->melim_wave_cap, 8, 32) || !pow2(t->solve_lanes_min) ||
      !pow2(t->solve_lanes_max) || t->solve_lanes_min > t->solve_lanes_max)
    return fail(SPALU_EINVAL, "tuning value out of range");
  g_tuning = *t;
  ++g_tuning_gen;
  return SPALU_OK;
}

static const Layout* get_layout(const spalu_nd_t* nd, int prec) {
  spalu_nd_t* m = const_cast<spalu_nd_t*>(nd);
  if (!m->layout[prec]) m->layout[prec] = build_layout(nd->plan, prec);
  return m->layout[prec].get();
}

static std::shared_ptr<const Layout> layout_ptr(const spalu_nd_t* nd, int prec) {
  get_layout(nd, prec);
  return nd->layout[prec];
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
  if (!(o.eps >= 0.0) || !(o.rho >= 0.0) || o.h0 < 1 || o.probes < 1 || o.probes > 8 || !(o.tau > 0.0) ||
      !(o.rank_margin > 0.0f) || o.rank_pad < 1 || !(o.rank_skip >= 0.0f) || (o.graph != 0 && o.graph != 1) ||
      (o.symmetric != 0 && o.symmetric != 1))
    return fail(SPALU_EINVAL, "bad factor options");
  const Layout* Y;
  try {
    Y = get_layout(nd, o.precision);
  } catch (const std::exception& e) {
    return fail(SPALU_EUNSUPPORTED, e.what());
  }
  if (workspace_bytes < Y->bytes) return fail(SPALU_ENOMEM, "workspace too small");
  if (Y->lv[nd->plan.L].tiers_gen != g_tuning_gen) {
    // the launch shapes were changed since this layout's tiers were planned
    Layout* YT = const_cast<Layout*>(Y);
    for (int l = 1; l <= nd->plan.L; ++l) plan_id_tiers(YT->lv[l], o.precision == SPALU_FP32 ? 4 : 8);
  }
  auto F = std::make_unique<spalu_factor_t>();
  F->nd = nd;
  F->lay = Y;
  F->lay_sp = layout_ptr(nd, o.precision);
  F->prec = o.precision;
  F->sym = o.symmetric;
  F->ws = static_cast<char*>(workspace);
  F->stream = static_cast<hipStream_t>(stream);
  F->n = n;
  F->rowptr = rowptr;
  F->colind = colind;
  F->vals = vals;
  F->g = GridGeom{nd->plan.dims[0], nd->plan.dims[1], nd->plan.dims[2]};
  const Plan& P = nd->plan;
  Layout* YM = const_cast<Layout*>(Y);
  const int irc = build_image(P, YM, o.rho);
  if (irc) return irc;
  // the tables reach the workspace from the device copy of the image (kept
  // per layout and device; rebuilt when rho changes)
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const size_t img_bytes = Y->blob_bytes + (Y->leaf_i1 - Y->leaf_i0) * 4;
  if (!YM->dimage || YM->dimage_dev != dev || YM->dimage_rho != o.rho) {
    if (YM->dimage) {
      // copies of earlier factorizations (any stream) may still read it
      YM->wait_image_readers();
      (void)hipFree(YM->dimage);
      YM->dimage = nullptr;
    }
    HIPCHK(hipMalloc(reinterpret_cast<void**>(&YM->dimage), std::max<size_t>(img_bytes, 1)));
    HIPCHK(hipMemcpy(YM->dimage, YM->image, img_bytes, hipMemcpyHostToDevice));
    YM->dimage_dev = dev;
    YM->dimage_rho = o.rho;
  }
  HIPCHK(hipMemcpyAsync(F->ws, YM->dimage, Y->blob_bytes, hipMemcpyDeviceToDevice, F->stream));
  if (Y->leaf_i1 > Y->leaf_i0)
    HIPCHK(hipMemcpyAsync(F->ws + Y->o_iarena + Y->leaf_i0 * 4, YM->dimage + Y->blob_bytes,
                          (Y->leaf_i1 - Y->leaf_i0) * 4, hipMemcpyDeviceToDevice, F->stream));
  {
    hipEvent_t ev = nullptr;
    for (const auto& se : YM->dimage_read)
      if (se.first == F->stream) ev = se.second;
    if (!ev) {
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      YM->dimage_read.emplace_back(F->stream, ev);
    }
    HIPCHK(hipEventRecord(ev, F->stream));
  }
  int stat[2] = {0, 0};
  int rc = o.precision == SPALU_FP64 ? run_factor<double>(F.get(), o, stat)
                                     : run_factor<float>(F.get(), o, stat);
  if (rc) return rc;
  const int status = stat[0];
  if (status & 2) return fail(SPALU_EUNSUPPORTED, "matrix pattern is not inside the grid stencil");
  if (status & 4) return fail(SPALU_EINVAL, "symmetric form: the matrix is not symmetric");
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
      const std::vector<int32_t>& dv = (*F->dyn_host)[l];
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
    if (info) info->singular_level = stat[1];
    if (o.symmetric)
      return fail(SPALU_ESINGULAR, "symmetric form: a pivot that is not positive (matrix not positive definite) "
                                   "in a diagonal block of level " + std::to_string(stat[1]));
    return fail(SPALU_ESINGULAR, "zero pivot in a diagonal block of level " + std::to_string(stat[1]));
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
    std::vector<int32_t> dv(DYN_ARRAYS * ns);
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

int spalu_factor_work(const spalu_factor_t* f, double* flops, double* bytes) {
  if (!f) return fail(SPALU_EINVAL, "f is NULL");
  double fl, by;
  factor_work(f, fl, by);
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  return SPALU_OK;
}


int spalu_mlp_param_count(void) { return MLP_NPARAM; }

static size_t mlp_ws_layout(int B, size_t* off) {
  // Xn[B*12], H1[B*64], H2[B*64], y[B], dz[B], sq[B], dH2[B*64], dH1[B*64], grad[P]
  const size_t sizes[9] = {size_t(B) * MLP_NF, size_t(B) * MLP_H, size_t(B) * MLP_H, size_t(B), size_t(B),
                           size_t(B), size_t(B) * MLP_H, size_t(B) * MLP_H, size_t(MLP_NPARAM)};
  size_t o = 0;
  for (int i = 0; i < 9; ++i) {
    off[i] = o;
    o = align256(o + sizes[i] * 4);
  }
  return o;
}

int spalu_mlp_workspace(int32_t batch, size_t* bytes) {
  if (batch < 1 || !bytes) return fail(SPALU_EINVAL, "bad argument");
  size_t off[9];
  *bytes = mlp_ws_layout(batch, off);
  return SPALU_OK;
}

static int mlp_forward_impl(const float* params, const float* X, int B, const float* t, char* ws, hipStream_t st,
                            float** Xn, float** H1, float** H2, float** y, float** dz, float** sq) {
  size_t off[9];
  mlp_ws_layout(B, off);
  *Xn = reinterpret_cast<float*>(ws + off[0]);
  *H1 = reinterpret_cast<float*>(ws + off[1]);
  *H2 = reinterpret_cast<float*>(ws + off[2]);
  *y = reinterpret_cast<float*>(ws + off[3]);
  *dz = reinterpret_cast<float*>(ws + off[4]);
  *sq = reinterpret_cast<float*>(ws + off[5]);
  k_mlp_normalize<<<nblocks(int64_t(B) * MLP_NF), WG, 0, st>>>(X, B, params, *Xn);
  HIPCHK(hipGetLastError());
  // H1 = relu(Xn W1^T + b1)
  k_gemm_f32<<<dim3(1, unsigned(B)), MLP_H, 0, st>>>(B, MLP_H, MLP_NF, *Xn, MLP_NF, 1, params + MLP_OFF_W1, 1,
                                                     MLP_NF, *H1, MLP_H, 0.f);
  HIPCHK(hipGetLastError());
  k_bias_relu<<<nblocks(int64_t(B) * MLP_H), WG, 0, st>>>(*H1, B, params + MLP_OFF_B1);
  HIPCHK(hipGetLastError());
  k_gemm_f32<<<dim3(1, unsigned(B)), MLP_H, 0, st>>>(B, MLP_H, MLP_H, *H1, MLP_H, 1, params + MLP_OFF_W2, 1, MLP_H,
                                                     *H2, MLP_H, 0.f);
  HIPCHK(hipGetLastError());
  k_bias_relu<<<nblocks(int64_t(B) * MLP_H), WG, 0, st>>>(*H2, B, params + MLP_OFF_B2);
  HIPCHK(hipGetLastError());
  k_mlp_out<<<nblocks(B), WG, 0, st>>>(*H2, B, params, t, *y, *dz, *sq);
  HIPCHK(hipGetLastError());
  return SPALU_OK;
}

int spalu_mlp_forward(const float* params, const float* X, int32_t batch, float* y, void* workspace,
                      size_t workspace_bytes, void* stream) {
  if (!params || !X || !y || !workspace || batch < 1 || batch > 65535)
    return fail(SPALU_EINVAL, "bad argument (batch must be in [1, 65535])");
  size_t off[9];
  if (workspace_bytes < mlp_ws_layout(batch, off)) return fail(SPALU_ENOMEM, "workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  float *Xn, *H1, *H2, *yy, *dz, *sq;
  const int rc = mlp_forward_impl(params, X, batch, nullptr, static_cast<char*>(workspace), st, &Xn, &H1, &H2, &yy,
                                  &dz, &sq);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(y, yy, size_t(batch) * 4, hipMemcpyDeviceToDevice, st));
  return SPALU_OK;
}

int spalu_mlp_train_step(float* params, float* adam_m, float* adam_v, const float* X, const float* t,
                         int32_t batch, float lr, int32_t step, float* loss, float* grad, void* workspace,
                         size_t workspace_bytes, void* stream) {
  if (!params || !X || !t || batch < 1 || batch > 65535 || !workspace || !loss)
    return fail(SPALU_EINVAL, "bad argument (batch must be in [1, 65535])");
  if ((adam_m == nullptr) != (adam_v == nullptr) || (adam_m && step < 1)) return fail(SPALU_EINVAL, "bad Adam state");
  size_t off[9];
  if (workspace_bytes < mlp_ws_layout(batch, off)) return fail(SPALU_ENOMEM, "workspace too small");
  const int B = batch;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  float *Xn, *H1, *H2, *y, *dz, *sq;
  int rc = mlp_forward_impl(params, X, B, t, ws, st, &Xn, &H1, &H2, &y, &dz, &sq);
  if (rc) return rc;
  float* dH2 = reinterpret_cast<float*>(ws + off[6]);
  float* dH1 = reinterpret_cast<float*>(ws + off[7]);
  float* g = grad ? grad : reinterpret_cast<float*>(ws + off[8]);
  HIPCHK(hipMemsetAsync(g, 0, size_t(MLP_OFF_W1) * 4, st));
  // loss = mean of squared errors
  k_mean<<<1, 64, 0, st>>>(sq, B, loss);
  HIPCHK(hipGetLastError());
  // output layer
  k_gemm_f32<<<dim3(1, MLP_H), 64, 0, st>>>(MLP_H, 1, B, H2, 1, MLP_H, dz, 1, 0, g + MLP_OFF_W3, 1, 0.f);
  HIPCHK(hipGetLastError());
  k_colsum<<<1, 64, 0, st>>>(dz, B, 1, 1, g + MLP_OFF_B3);
  HIPCHK(hipGetLastError());
  // second hidden layer
  k_mlp_dh2<<<nblocks(int64_t(B) * MLP_H), WG, 0, st>>>(dz, H2, B, params, dH2);
  HIPCHK(hipGetLastError());
  k_gemm_f32<<<dim3(1, MLP_H), MLP_H, 0, st>>>(MLP_H, MLP_H, B, dH2, 1, MLP_H, H1, MLP_H, 1, g + MLP_OFF_W2,
                                               MLP_H, 0.f);
  HIPCHK(hipGetLastError());
  k_colsum<<<1, MLP_H, 0, st>>>(dH2, B, MLP_H, MLP_H, g + MLP_OFF_B2);
  HIPCHK(hipGetLastError());
  // first hidden layer: dH1 = (dH2 W2) masked by H1 > 0
  k_gemm_f32<<<dim3(1, unsigned(B)), MLP_H, 0, st>>>(B, MLP_H, MLP_H, dH2, MLP_H, 1, params + MLP_OFF_W2, MLP_H, 1,
                                                     dH1, MLP_H, 0.f);
  HIPCHK(hipGetLastError());
  k_mask_pos<<<nblocks(int64_t(B) * MLP_H), WG, 0, st>>>(dH1, H1, B * MLP_H);
  HIPCHK(hipGetLastError());
  k_gemm_f32<<<dim3(1, MLP_H), MLP_NF, 0, st>>>(MLP_H, MLP_NF, B, dH1, 1, MLP_H, Xn, MLP_NF, 1, g + MLP_OFF_W1,
                                                MLP_NF, 0.f);
  HIPCHK(hipGetLastError());
  k_colsum<<<1, MLP_H, 0, st>>>(dH1, B, MLP_H, MLP_H, g + MLP_OFF_B1);
  HIPCHK(hipGetLastError());
  if (adam_m) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, float(step)), c2 = 1.f - std::pow(b2, float(step));
    k_adam<<<nblocks(MLP_NPARAM - MLP_OFF_W1), WG, 0, st>>>(params, g, adam_m, adam_v, MLP_OFF_W1, MLP_NPARAM, lr, b1,
                                                            b2, 1e-8f, c1, c2);
    HIPCHK(hipGetLastError());
  }
  return SPALU_OK;
}

void spalu_profile(int32_t on) {
  g_prof.reset();
  g_prof.on = on != 0;
  g_prof.only = -1;
}

int spalu_profile_only(const char* name) {
  if (!name || !name[0]) {
    g_prof.only = -1;
    return SPALU_OK;
  }
  for (int k = 0; k < K_COUNT; ++k)
    if (std::strcmp(kNames[k], name) == 0) {
      g_prof.only = k;
      return SPALU_OK;
    }
  return fail(SPALU_EINVAL, "unknown kernel step name");
}

int spalu_profile_read(spalu_kernel_stat* out, int32_t max, int32_t* count) {
  if (!count) return fail(SPALU_EINVAL, "count is NULL");
  prof_account_pending();
  int32_t m = 0;
  for (int k = 0; k < K_COUNT; ++k) {
    if (g_prof.launches[k] == 0) continue;
    if (out && m < max) {
      std::memset(&out[m], 0, sizeof(spalu_kernel_stat));
      std::strncpy(out[m].name, kNames[k], sizeof(out[m].name) - 1);
      out[m].launches = g_prof.launches[k];
      out[m].ms = g_prof.ms[k];
      out[m].bytes = g_prof.bytes[k];
      out[m].flops = g_prof.flops[k];
    }
    ++m;
  }
  *count = m;
  return SPALU_OK;
}

int spalu_solve_workspace(const spalu_factor_t* f, int32_t nrhs, const spalu_solve_opts* opts, size_t* bytes) {
  if (!f || !bytes || nrhs < 1) return fail(SPALU_EINVAL, "bad argument");
  const int m = opts ? opts->restart : 0;
  if (m < 0 || m > 32) return fail(SPALU_EINVAL, "restart must be in 0..32");
  *bytes = solve_layout(f, nrhs, m).bytes;
  return SPALU_OK;
}

int spalu_solve(const spalu_factor_t* f, int32_t nrhs, const double* B, int64_t ldb, double* X, int64_t ldx,
                const spalu_solve_opts* opts, void* workspace, size_t workspace_bytes, void* stream,
                double* rel_res, spalu_solve_info* info) {
  if (!f || !B || !X || !workspace || nrhs < 1) return fail(SPALU_EINVAL, "bad argument");
  if (ldb < f->n || ldx < f->n) return fail(SPALU_EINVAL, "leading dimension < n");
  spalu_solve_opts so{0.0, 30, 0, 0};
  if (opts) so = *opts;
  if (so.max_iter < 0) return fail(SPALU_EINVAL, "bad max_iter");
  if (so.restart < 0 || so.restart > 32) return fail(SPALU_EINVAL, "restart must be in 0..32");
  if (so.tol <= 0.0) so.restart = 0;
  if (workspace_bytes < solve_layout(f, nrhs, so.restart).bytes) return fail(SPALU_ENOMEM, "workspace too small");
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

int spalu_solve_static(const spalu_factor_t* f, int32_t nrhs, const double* B, int64_t ldb, double* X,
                       int64_t ldx, const spalu_solve_opts* opts, void* stream, double* rel_res,
                       spalu_solve_info* info) {
  if (!f || !B || !X || nrhs < 1) return fail(SPALU_EINVAL, "bad argument");
  if (ldb < f->n || ldx < f->n) return fail(SPALU_EINVAL, "leading dimension < n");
  spalu_solve_opts so{0.0, 30, 0, 0};
  if (opts) so = *opts;
  so.graph = 0;  // direct launches: instantiating a graph may allocate
  if (so.max_iter < 0) return fail(SPALU_EINVAL, "bad max_iter");
  if (so.restart < 0 || so.restart > 32) return fail(SPALU_EINVAL, "restart must be in 0..32");
  if (so.tol <= 0.0) so.restart = 0;
  if (so.tol > 0.0 && X == B) return fail(SPALU_EINVAL, "refinement needs X != B");
  const size_t need = solve_layout(f, nrhs, so.restart).bytes;
  if (need > SPALU_STATIC_SOLVE_BYTES)
    return fail(SPALU_ENOMEM, "solve needs " + std::to_string(need) + " bytes of working memory; the static "
                "buffer of spalu_solve_static holds " + std::to_string(SPALU_STATIC_SOLVE_BYTES) +
                " (use spalu_solve with a workspace)");
  char* sw = nullptr;
  const int src = scratch_on_device(&sw);
  if (src) return src;
  spalu_factor_t* F = const_cast<spalu_factor_t*>(f);
  hipStream_t keep = F->stream;
  F->stream = static_cast<hipStream_t>(stream);
  int rc = f->prec == SPALU_FP64 ? run_solve<double>(f, nrhs, B, ldb, X, ldx, so, sw, rel_res, info)
                                 : run_solve<float>(f, nrhs, B, ldb, X, ldx, so, sw, rel_res, info);
  F->stream = keep;
  return rc;
}

}  // extern "C"

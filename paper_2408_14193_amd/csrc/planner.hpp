// Host-side planner: grid nested dissection, segment structure per level,
// and the static device layout of the factorization.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace spalu {

struct PSeg {
  std::vector<int32_t> verts;  // original vertex ids, ascending
  int32_t sep_node = -1;
  int32_t sep_level = 0;
  int32_t nsig = 0;
  int32_t sig[2] = {-1, -1};
  bool regular = false;
  bool is_sep = false;
  int32_t lo[3] = {0, 0, 0};
  int32_t hi[3] = {0, 0, 0};
  int32_t parent = -1;  // segment of level l-1 holding it (-1: eliminated)
};

struct PLevel {
  std::vector<PSeg> segs;
  std::vector<std::pair<int32_t, int32_t>> pairs;  // sorted, incl. (c, c)
};

struct PLeaf {
  int32_t lo[3], hi[3];
  std::vector<int32_t> interior;  // ascending
  std::vector<int32_t> bsegs;     // level-L segments on its boundary, ascending
};

struct Plan {
  int dim = 2;
  int dims[3] = {1, 1, 1};
  int L = 0;
  int64_t N = 0;
  std::vector<int64_t> perm, node_begin, node_size, node_parent;
  std::vector<int32_t> node_level;
  std::vector<int8_t> seplev;     // per vertex, 0 = leaf interior
  std::vector<PLevel> levels;     // index 1..L (0 unused)
  std::vector<PLeaf> leaves;
};

// Throws std::runtime_error on invalid sizes.
void build_plan(int dim, const int32_t* grid, int levels, int leaf_max, Plan& p);

}  // namespace spalu

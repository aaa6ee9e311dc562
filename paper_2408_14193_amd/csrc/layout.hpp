// Device tables of the factorization.  Every offset is static: regions are
// sized by the uncompressed (pre-ID) segment sizes, and kernels read the
// actual sizes (which shrink as skeletons are selected) from device arrays,
// so a whole factorization runs without host round trips between levels.
#pragma once

#include <cstdint>

namespace spalu {

enum SegFlags : int32_t {
  SEG_REGULAR = 1,   // two neighbour boxes: gets an ID
  SEG_IS_SEP = 2,    // lies on a separator of the current level
  SEG_HAS_NBR = 4,   // has at least one coupled segment
  SEG_BIG = 8,       // may not fit the LDS staging buffer
};

// Per segment of one level.
struct DSeg {
  int32_t cap;        // uncompressed size (vertices of the segment)
  int32_t flags;
  int32_t nbr_begin;  // adjacency entries [nbr_begin, nbr_end) of this level
  int32_t nbr_end;
  int32_t diag_blk;   // block (c, c)
  int32_t parent;     // segment of level l-1 (-1: eliminated at level l)
  int32_t lo[3];      // bounding box of the uncompressed segment
  int32_t hi[3];
  int32_t thr;        // near-field Chebyshev radius
  int32_t rcap;       // bound on ID rows: 2 * sum of neighbour caps
  int32_t sep_level;  // level of the separator holding the segment
  int64_t ioff;       // int arena: dofs[cap], perm[cap], piv[cap], tag[2*rcap]; piv holds
                      // the LU's row interchanges composed: row i of P X is row piv[i] of X
  int64_t lu_off;     // value arena: cap*cap
  int64_t t_off;      // value arena: floor(cap*cap/4)
  int64_t scr_off;    // scratch pool (doubles): 2*rcap*cap (regular segments)
};

struct DNbr {
  int32_t d;       // neighbour segment
  int32_t blk_cd;  // block (c, d)
  int32_t blk_dc;  // block (d, c)
  int32_t d_is_sep;
};

struct DBlk {
  int32_t c, d;
  int64_t off;   // value arena: raw block, cap_c * cap_d
  int64_t soff;  // value arena: scaled block, cap_c * cap_d
};

// Merge/elimination task: sub-block (c, d) of a level-(l-1) block.
struct DTask {
  int32_t c, d;
  int32_t src;          // scaled level-l block (c, d), -1 none, -2 identity
  int32_t sep_begin;    // entries in the sep list
  int32_t sep_end;
  int32_t pad;
};

struct DSepTerm {
  int32_t s;        // level-l separator segment
  int32_t blk_cs;   // scaled block (c, s)
  int32_t blk_sd;   // scaled block (s, d)
  int32_t pad;
};

struct DLeaf {
  int32_t lo[3], hi[3];
  int32_t ni, nb;
  int64_t ioff;      // int arena: bverts[nb], piv[ni]
  int64_t lu_off;    // value arena: ni*ni
  int64_t s_off;     // value arena: nb*nb (Schur contribution)
  int64_t x_off;     // value arena: ni*nb, A_II^{-1} A_IB transposed (one-wave leaf factor)
};

// Level-L block assembly: contribution of a leaf to block (c, d).
struct DLeafContrib {
  int32_t leaf;
  int32_t oc, od;  // offsets of c and d in the leaf boundary
  int32_t pad;
};

// Per level: dynamic int arrays (device), indexed by segment.
struct DLevelDyn {
  int32_t* n;       // current size
  int32_t* k;       // skeleton size after the ID (n if not sparsified)
  int32_t* nr;      // remainder size
  int32_t* h;       // samples of the accepted pass
  int32_t* passes;  // ID passes
  int32_t* off;     // offset inside the parent segment (merge)
  int32_t* nfar;    // far rows of the accepted ID (0 without an ID)
};

constexpr int DYN_ARRAYS = 7;  // int32 arrays of DLevelDyn, each one entry per segment

}  // namespace spalu

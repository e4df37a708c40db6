// Host-side structure of an H^2 matrix: cluster tree and block tree.
//
// Cluster tree (Definition 1): characteristic points are triangle centroids;
// a cluster with more than leaf_size triangles is bisected at the midpoint of
// the longest side of its centroid bounding box (lowest axis on ties), points
// strictly below the midpoint going to child 0; the geometric cluster is the
// minimal axis-parallel box containing all vertices of its triangles.
// Block tree: admissible iff max(diam) <= 2 eta dist (eq. admissibility);
// otherwise split by the children of whichever clusters have them; a pair of
// leaves that is not admissible is a near-field (inadmissible) leaf.
#pragma once
#include <cstdint>
#include <vector>

namespace h2 {

struct Structure {
  int64_t n = 0;                 // number of triangles (= basis functions)
  int m = 0, k = 0, leaf_size = 0;
  double eta = 0.0;
  // mesh copy
  std::vector<double> vert;      // nv x 3
  std::vector<int32_t> tri;      // n x 3
  // permutation: position p in cluster order holds triangle perm[p]
  std::vector<int32_t> perm;
  // clusters, numbered level by level (breadth first); within a level in
  // left-to-right order.  Level l holds ids [level_ptr[l], level_ptr[l+1]).
  int nclusters = 0, depth = 0;  // depth = deepest level
  std::vector<int32_t> cbegin, cend, parent, child0, child1, level, dfs_id;
  std::vector<double> lo, hi;    // nclusters x 3 (geometric boxes)
  std::vector<int32_t> level_ptr;
  // leaves sorted by cbegin
  std::vector<int32_t> leaves;
  std::vector<int32_t> leaf_of_pos;  // position -> index into `leaves`
  // admissible leaves: CSR by row cluster (all clusters), columns sorted
  std::vector<int64_t> adm_ptr;
  std::vector<int32_t> adm_col;
  // inadmissible leaves: CSR by row leaf (index into `leaves`), columns = cluster ids sorted
  std::vector<int64_t> near_ptr;
  std::vector<int32_t> near_col;
  std::vector<int64_t> panel_off;    // per leaf: element offset of its near-field panel
  int64_t near_entries = 0;          // sum over inadmissible leaves of |tau| |sigma|
  int64_t near_stored = 0;           // entries held in the panels (= near_entries unless symmetric)
  int64_t adm_blocks = 0;            // admissible leaves of the block tree (before any halving)
  int64_t near_blocks = 0;           // inadmissible leaves of the block tree (before any halving)
  // symmetric storage (G~ = G~^T): only blocks (tau, sigma) with sigma after tau are kept;
  // each kept off-diagonal block also feeds the transposed product into a scratch slot,
  // and every target gathers its incoming slots in a fixed order.
  bool sym_s = false, sym_n = false;
  std::vector<int64_t> adm_in_ptr;   // per cluster sigma: incoming blocks (tau, sigma), tau < sigma
  std::vector<int64_t> adm_in_blk;   // their block indices (scratch slot = block index * k)
  std::vector<int64_t> near_slot;    // per kept near block: scratch offset of its transposed part (-1: diagonal)
  std::vector<int64_t> near_in_ptr;  // per leaf: incoming off-diagonal near blocks
  std::vector<int64_t> near_in_slot; // their scratch offsets, by source leaf
  int64_t near_scratch = 0;          // scratch values of the transposed near-field parts
};

// Keeps one block of every symmetric pair: admissible blocks (tau, sigma) with
// sigma > tau (cluster ids) when `s`, inadmissible leaves with leaf index of
// sigma >= that of tau when `nf`; builds the scratch slots and incoming lists.
void make_symmetric(Structure& S, bool s, bool nf);

// Builds tree and block tree.  Throws std::runtime_error on invalid input.
void build_structure(Structure& S, const double* vertices, int64_t nv, const int32_t* triangles,
                     int64_t nt, int m, int leaf_size, double eta);

}  // namespace h2

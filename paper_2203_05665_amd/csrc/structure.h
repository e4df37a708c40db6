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
};

// Builds tree and block tree.  Throws std::runtime_error on invalid input.
void build_structure(Structure& S, const double* vertices, int64_t nv, const int32_t* triangles,
                     int64_t nt, int m, int leaf_size, double eta);

}  // namespace h2

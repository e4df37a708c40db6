// Cluster tree and block tree construction on the host (see structure.h).
// Compiled with -ffp-contract=off: every comparison that decides the tree or
// the block partition is evaluated in plain IEEE double arithmetic.
#include "structure.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>

namespace h2 {
namespace {

struct Node {
  int32_t begin, end, level, parent, child[2];
  double lo[3], hi[3];
};

// Work below this many triangles (tree) or pairs (block tree) stays on the
// calling thread; above it the two halves of a split run on two threads.
constexpr int32_t kParallelTriangles = 1 << 15;
// A cluster of at least this many triangles also splits its own passes (the
// bounding boxes, the count and the stable partition) over the threads it has.
constexpr int32_t kParallelPasses = 1 << 16;

int worker_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return static_cast<int>(std::max(1u, std::min(16u, h)));
}

// runs f(i) for i in [0, n) on up to `threads` threads, in contiguous chunks
template <class F>
void parallel_for(int64_t n, int threads, F&& f) {
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(threads, n / 4096));
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  for (int64_t w = 0; w < nt; ++w)
    pool.emplace_back([&, w]() {
      for (int64_t i = n * w / nt; i < n * (w + 1) / nt; ++i) f(i);
    });
  for (auto& t : pool) t.join();
}

// runs f(w) for w in [0, nw): w = 0 on the calling thread, the rest on threads
// of their own
template <class F>
void run_chunks(int nw, F&& f) {
  if (nw <= 1) {
    f(0);
    return;
  }
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; ++w) pool.emplace_back([&, w]() { f(w); });
  f(0);
  for (auto& t : pool) t.join();
}

struct TreeBuilder {
  const double* V;
  const int32_t* T;
  int leaf;
  std::vector<int32_t> idx, tmp;
  std::vector<double> cen;  // n x 3

  // Builds the subtree of idx[begin, end) into `out` in depth-first pre-order
  // (child 0 before child 1) and returns the position of its root in `out`.
  // The index ranges of two children are disjoint, so with par_depth > 0 the
  // subtree of child 0 is built on a second thread into a vector of its own and
  // both are appended in pre-order afterwards: the same tree, node for node.
  // A large cluster also runs its own passes on its nthr threads, in contiguous
  // chunks: minima, maxima and counts do not depend on how the range is cut, and
  // each chunk writes its low and high triangles at offsets given by the counts
  // of the chunks before it, which is the sequential stable partition.  The
  // bounding box of the triangles is formed at the leaves and, for the other
  // clusters, as the union of the two children's boxes (the same minima and
  // maxima), so the vertices are read once per triangle, not once per level.
  int32_t build(std::vector<Node>& out, int32_t begin, int32_t end, int32_t level, int32_t parent, int par_depth,
                int nthr) {
    const int32_t id = static_cast<int32_t>(out.size());
    out.push_back(Node{begin, end, level, parent, {-1, -1}, {0, 0, 0}, {0, 0, 0}});
    const int32_t size = end - begin;
    const int nw = size >= kParallelPasses ? std::max(1, nthr) : 1;
    auto lo_of = [&](int w) { return begin + static_cast<int32_t>(static_cast<int64_t>(size) * w / nw); };
    // a leaf: the bounding box of its triangles' vertices
    auto leaf_box = [&]() {
      for (int d = 0; d < 3; ++d) {
        out[id].lo[d] = INFINITY;
        out[id].hi[d] = -INFINITY;
      }
      for (int32_t p = begin; p < end; ++p) {
        const int32_t t = idx[p];
        for (int a = 0; a < 3; ++a) {
          const double* v = V + 3 * static_cast<int64_t>(T[3 * static_cast<int64_t>(t) + a]);
          for (int d = 0; d < 3; ++d) {
            out[id].lo[d] = std::min(out[id].lo[d], v[d]);
            out[id].hi[d] = std::max(out[id].hi[d], v[d]);
          }
        }
      }
      return id;
    };
    if (size <= leaf) return leaf_box();
    // the bounding box of the centroids
    std::vector<std::array<double, 6>> box(nw);
    run_chunks(nw, [&](int w) {
      double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int32_t p = lo_of(w); p < lo_of(w + 1); ++p) {
        const double* c = &cen[3 * static_cast<int64_t>(idx[p])];
        for (int d = 0; d < 3; ++d) {
          clo[d] = std::min(clo[d], c[d]);
          chi[d] = std::max(chi[d], c[d]);
        }
      }
      for (int d = 0; d < 3; ++d) {
        box[w][d] = clo[d];
        box[w][3 + d] = chi[d];
      }
    });
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int w = 0; w < nw; ++w)
      for (int d = 0; d < 3; ++d) {
        clo[d] = std::min(clo[d], box[w][d]);
        chi[d] = std::max(chi[d], box[w][3 + d]);
      }
    int axis = 0;
    double ext[3] = {chi[0] - clo[0], chi[1] - clo[1], chi[2] - clo[2]};
    for (int d = 1; d < 3; ++d)
      if (ext[d] > ext[axis]) axis = d;
    if (!(ext[axis] > 0.0)) return leaf_box();
    const double mid = 0.5 * (clo[axis] + chi[axis]);
    std::vector<int32_t> lowc(nw + 1, 0);
    run_chunks(nw, [&](int w) {
      int32_t c = 0;
      for (int32_t p = lo_of(w); p < lo_of(w + 1); ++p)
        if (cen[3 * static_cast<int64_t>(idx[p]) + axis] < mid) ++c;
      lowc[w + 1] = c;
    });
    for (int w = 0; w < nw; ++w) lowc[w + 1] += lowc[w];
    const int32_t nlow = lowc[nw];
    if (nlow == 0 || nlow == size) return leaf_box();
    // stable partition: low side first, both sides keep their relative order
    run_chunks(nw, [&](int w) {
      int32_t a = begin + lowc[w], b = begin + nlow + (lo_of(w) - begin - lowc[w]);
      for (int32_t p = lo_of(w); p < lo_of(w + 1); ++p) {
        const int32_t t = idx[p];
        if (cen[3 * static_cast<int64_t>(t) + axis] < mid) tmp[a++] = t; else tmp[b++] = t;
      }
    });
    run_chunks(nw, [&](int w) { std::copy(tmp.begin() + lo_of(w), tmp.begin() + lo_of(w + 1), idx.begin() + lo_of(w)); });
    int32_t c0, c1;
    if (par_depth > 0 && size >= kParallelTriangles) {
      std::vector<Node> v0, v1;
      const int n0 = std::max(1, nthr / 2), n1 = std::max(1, nthr - nthr / 2);
      std::thread th([&]() { build(v0, begin, begin + nlow, level + 1, -1, par_depth - 1, n0); });
      build(v1, begin + nlow, end, level + 1, -1, par_depth - 1, n1);
      th.join();
      c0 = append(out, v0, id);
      c1 = append(out, v1, id);
    } else {
      c0 = build(out, begin, begin + nlow, level + 1, id, 0, 1);
      c1 = build(out, begin + nlow, end, level + 1, id, 0, 1);
    }
    for (int d = 0; d < 3; ++d) {
      out[id].lo[d] = std::min(out[c0].lo[d], out[c1].lo[d]);
      out[id].hi[d] = std::max(out[c0].hi[d], out[c1].hi[d]);
    }
    out[id].child[0] = c0;
    out[id].child[1] = c1;
    return id;
  }

  // appends a subtree built on its own (local positions, root parent -1)
  static int32_t append(std::vector<Node>& out, const std::vector<Node>& v, int32_t parent) {
    const int32_t off = static_cast<int32_t>(out.size());
    for (Node nd : v) {
      nd.parent = nd.parent < 0 ? parent : nd.parent + off;
      for (int c = 0; c < 2; ++c)
        if (nd.child[c] >= 0) nd.child[c] += off;
      out.push_back(nd);
    }
    return off;
  }
};

inline double diam(const Structure& S, int32_t c) {
  const double d0 = S.hi[3 * c] - S.lo[3 * c];
  const double d1 = S.hi[3 * c + 1] - S.lo[3 * c + 1];
  const double d2 = S.hi[3 * c + 2] - S.lo[3 * c + 2];
  return std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

inline double dist(const Structure& S, int32_t t, int32_t s) {
  double g[3];
  for (int d = 0; d < 3; ++d) {
    const double a = S.lo[3 * s + d] - S.hi[3 * t + d];
    const double b = S.lo[3 * t + d] - S.hi[3 * s + d];
    g[d] = std::max(0.0, std::max(a, b));
  }
  return std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
}

using Pairs = std::vector<std::pair<int32_t, int32_t>>;

struct BlockBuilder {
  const Structure& S;
  std::vector<double> dia;
  explicit BlockBuilder(const Structure& s) : S(s) {
    dia.resize(S.nclusters);
    for (int32_t c = 0; c < S.nclusters; ++c) dia[c] = diam(S, c);
  }
  // one step of the block tree for the pair (t, s): an admissible leaf, an
  // inadmissible leaf, or its children pairs appended to `next`
  void step(int32_t t, int32_t s, Pairs& adm, Pairs& near, Pairs& next) const {
    const double lhs = std::max(dia[t], dia[s]);
    if (lhs <= 2.0 * S.eta * dist(S, t, s)) {
      adm.emplace_back(t, s);
      return;
    }
    const bool ct = S.child0[t] >= 0, cs = S.child0[s] >= 0;
    if (ct && cs) {
      next.emplace_back(S.child0[t], S.child0[s]);
      next.emplace_back(S.child0[t], S.child1[s]);
      next.emplace_back(S.child1[t], S.child0[s]);
      next.emplace_back(S.child1[t], S.child1[s]);
    } else if (cs) {
      next.emplace_back(t, S.child0[s]);
      next.emplace_back(t, S.child1[s]);
    } else if (ct) {
      next.emplace_back(S.child0[t], s);
      next.emplace_back(S.child1[t], s);
    } else {
      near.emplace_back(t, s);
    }
  }
  void visit(int32_t t, int32_t s, Pairs& adm, Pairs& near) const {
    Pairs stack{{t, s}}, next;
    while (!stack.empty()) {
      const auto pr = stack.back();
      stack.pop_back();
      next.clear();
      step(pr.first, pr.second, adm, near, next);
      stack.insert(stack.end(), next.rbegin(), next.rend());
    }
  }
  // The leaves of the block tree of (root, root).  The top of the tree is
  // expanded breadth first until there is work for every thread; each thread then
  // visits a contiguous share of the pending pairs.  The leaves are sorted by the
  // caller, so the result does not depend on the order they were found in.
  void build(int threads, Pairs& adm, Pairs& near) const {
    Pairs front{{0, 0}}, next;
    while (!front.empty() && front.size() < static_cast<size_t>(64 * threads)) {
      next.clear();
      for (const auto& pr : front) step(pr.first, pr.second, adm, near, next);
      front.swap(next);
    }
    const int nt = static_cast<int>(std::min<size_t>(threads, front.size()));
    if (nt <= 1) {
      for (const auto& pr : front) visit(pr.first, pr.second, adm, near);
      return;
    }
    std::vector<Pairs> ta(nt), tn(nt);
    std::vector<std::thread> pool;
    for (int w = 0; w < nt; ++w)
      pool.emplace_back([&, w]() {
        for (size_t i = front.size() * w / nt; i < front.size() * (w + 1) / nt; ++i)
          visit(front[i].first, front[i].second, ta[w], tn[w]);
      });
    for (auto& th : pool) th.join();
    for (int w = 0; w < nt; ++w) {
      adm.insert(adm.end(), ta[w].begin(), ta[w].end());
      near.insert(near.end(), tn[w].begin(), tn[w].end());
    }
  }
};

// CSR by row of a list of pairs: ptr[nrows + 1]; columns of a row in the order
// `less` gives (a counting sort by row, then each row's few columns sorted)
template <class Less>
void csr_by_row(const Pairs& pairs, int32_t nrows, std::vector<int64_t>& ptr, std::vector<int32_t>& col, Less less) {
  ptr.assign(nrows + 1, 0);
  for (const auto& pr : pairs) ptr[pr.first + 1]++;
  for (int32_t i = 0; i < nrows; ++i) ptr[i + 1] += ptr[i];
  col.resize(pairs.size());
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (const auto& pr : pairs) col[fill[pr.first]++] = pr.second;
  parallel_for(nrows, worker_threads(), [&](int64_t i) { std::sort(col.begin() + ptr[i], col.begin() + ptr[i + 1], less); });
}

}  // namespace

void build_structure(Structure& S, const double* vertices, int64_t nv, const int32_t* triangles,
                     int64_t nt, int m, int leaf_size, double eta) {
  if (nt <= 0 || nv <= 0) throw std::runtime_error("empty mesh");
  if (nt > (int64_t(1) << 30)) throw std::runtime_error("too many triangles");
  if (m < 1 || m > 6) throw std::runtime_error("order m must be in [1, 6]");
  if (leaf_size < 1) throw std::runtime_error("leaf_size must be >= 1");
  if (!(eta > 0.0)) throw std::runtime_error("eta must be > 0");
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (triangles[i] < 0 || triangles[i] >= nv) throw std::runtime_error("triangle vertex index out of range");
  S = Structure();
  S.n = nt;
  S.m = m;
  S.k = m * m * m;
  S.leaf_size = leaf_size;
  S.eta = eta;
  S.vert.assign(vertices, vertices + 3 * nv);
  S.tri.assign(triangles, triangles + 3 * nt);

  const int threads = worker_threads();
  TreeBuilder tb{S.vert.data(), S.tri.data(), leaf_size, {}, {}, {}};
  tb.idx.resize(nt);
  tb.tmp.resize(nt);
  std::iota(tb.idx.begin(), tb.idx.end(), 0);
  tb.cen.resize(3 * nt);
  parallel_for(nt, threads, [&](int64_t t) {
    const double* p0 = &S.vert[3 * static_cast<int64_t>(S.tri[3 * t])];
    const double* p1 = &S.vert[3 * static_cast<int64_t>(S.tri[3 * t + 1])];
    const double* p2 = &S.vert[3 * static_cast<int64_t>(S.tri[3 * t + 2])];
    for (int d = 0; d < 3; ++d) tb.cen[3 * t + d] = (p0[d] + p1[d] + p2[d]) / 3.0;
  });
  std::vector<Node> nodes;
  int par_depth = 0;
  while ((1 << par_depth) < threads) ++par_depth;
  tb.build(nodes, 0, static_cast<int32_t>(nt), 0, -1, par_depth, threads);
  S.perm = tb.idx;

  // renumber breadth first (stable within a level = depth-first order)
  const int32_t nc = static_cast<int32_t>(nodes.size());
  S.nclusters = nc;
  int32_t depth = 0;
  for (const Node& nd : nodes) depth = std::max(depth, nd.level);
  S.depth = depth;
  std::vector<int32_t> order(nc);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return nodes[a].level < nodes[b].level; });
  std::vector<int32_t> newid(nc);
  for (int32_t i = 0; i < nc; ++i) newid[order[i]] = i;
  S.cbegin.resize(nc); S.cend.resize(nc); S.parent.resize(nc); S.child0.resize(nc);
  S.child1.resize(nc); S.level.resize(nc); S.dfs_id.resize(nc);
  S.lo.resize(3 * nc); S.hi.resize(3 * nc);
  S.level_ptr.assign(depth + 2, 0);
  for (int32_t i = 0; i < nc; ++i) {
    const Node& nd = nodes[order[i]];
    S.cbegin[i] = nd.begin;
    S.cend[i] = nd.end;
    S.parent[i] = nd.parent >= 0 ? newid[nd.parent] : -1;
    S.child0[i] = nd.child[0] >= 0 ? newid[nd.child[0]] : -1;
    S.child1[i] = nd.child[1] >= 0 ? newid[nd.child[1]] : -1;
    S.level[i] = nd.level;
    S.dfs_id[i] = order[i];
    for (int d = 0; d < 3; ++d) {
      S.lo[3 * i + d] = nd.lo[d];
      S.hi[3 * i + d] = nd.hi[d];
    }
    S.level_ptr[nd.level + 1]++;
  }
  for (int l = 0; l <= depth; ++l) S.level_ptr[l + 1] += S.level_ptr[l];

  for (int32_t i = 0; i < nc; ++i)
    if (S.child0[i] < 0) S.leaves.push_back(i);
  std::sort(S.leaves.begin(), S.leaves.end(),
            [&](int32_t a, int32_t b) { return S.cbegin[a] < S.cbegin[b]; });
  S.leaf_of_pos.resize(nt);
  for (size_t l = 0; l < S.leaves.size(); ++l)
    for (int32_t p = S.cbegin[S.leaves[l]]; p < S.cend[S.leaves[l]]; ++p) S.leaf_of_pos[p] = static_cast<int32_t>(l);

  // block tree: admissible leaves by row cluster, columns ascending; inadmissible
  // leaves by row leaf, columns by their first position
  BlockBuilder bb(S);
  Pairs adm, near;
  bb.build(threads, adm, near);
  csr_by_row(adm, nc, S.adm_ptr, S.adm_col, [](int32_t a, int32_t b) { return a < b; });

  const int32_t nl = static_cast<int32_t>(S.leaves.size());
  std::vector<int32_t> leaf_index(nc, -1);
  for (int32_t l = 0; l < nl; ++l) leaf_index[S.leaves[l]] = l;
  for (auto& pr : near) pr.first = leaf_index[pr.first];
  csr_by_row(near, nl, S.near_ptr, S.near_col,
             [&](int32_t a, int32_t b) { return S.cbegin[a] < S.cbegin[b]; });
  S.panel_off.assign(nl + 1, 0);
  for (int32_t l = 0; l < nl; ++l) {
    const int64_t r = S.cend[S.leaves[l]] - S.cbegin[S.leaves[l]];
    int64_t cols = 0;
    for (int64_t b = S.near_ptr[l]; b < S.near_ptr[l + 1]; ++b)
      cols += S.cend[S.near_col[b]] - S.cbegin[S.near_col[b]];
    S.panel_off[l + 1] = S.panel_off[l] + r * cols;
  }
  S.near_entries = S.panel_off[nl];
  S.near_stored = S.near_entries;
  S.adm_blocks = static_cast<int64_t>(S.adm_col.size());
  S.near_blocks = static_cast<int64_t>(S.near_col.size());
}

void make_symmetric(Structure& S, bool s, bool nf) {
  const int32_t nc = S.nclusters;
  const int32_t nl = static_cast<int32_t>(S.leaves.size());
  if (s) {
    std::vector<int64_t> ptr(nc + 1, 0);
    std::vector<int32_t> col;
    for (int32_t t = 0; t < nc; ++t) {
      for (int64_t b = S.adm_ptr[t]; b < S.adm_ptr[t + 1]; ++b)
        if (S.adm_col[b] > t) col.push_back(S.adm_col[b]);
      ptr[t + 1] = static_cast<int64_t>(col.size());
    }
    S.adm_ptr.swap(ptr);
    S.adm_col.swap(col);
    // incoming: block b = (t, sigma) contributes S_b^T x^_t to sigma; gathered by increasing t
    S.adm_in_ptr.assign(nc + 1, 0);
    for (int32_t c : S.adm_col) S.adm_in_ptr[c + 1]++;
    for (int32_t c = 0; c < nc; ++c) S.adm_in_ptr[c + 1] += S.adm_in_ptr[c];
    S.adm_in_blk.resize(S.adm_col.size());
    std::vector<int64_t> fill(S.adm_in_ptr.begin(), S.adm_in_ptr.end() - 1);
    for (int32_t t = 0; t < nc; ++t)
      for (int64_t b = S.adm_ptr[t]; b < S.adm_ptr[t + 1]; ++b) S.adm_in_blk[fill[S.adm_col[b]]++] = b;
    S.sym_s = true;
  }
  if (nf) {
    std::vector<int32_t> leaf_index(nc, -1);
    for (int32_t l = 0; l < nl; ++l) leaf_index[S.leaves[l]] = l;
    std::vector<int64_t> ptr(nl + 1, 0);
    std::vector<int32_t> col;
    for (int32_t l = 0; l < nl; ++l) {
      for (int64_t b = S.near_ptr[l]; b < S.near_ptr[l + 1]; ++b)
        if (leaf_index[S.near_col[b]] >= l) col.push_back(S.near_col[b]);
      ptr[l + 1] = static_cast<int64_t>(col.size());
    }
    S.near_ptr.swap(ptr);
    S.near_col.swap(col);
    S.panel_off.assign(nl + 1, 0);
    S.near_slot.assign(S.near_col.size(), -1);
    S.near_in_ptr.assign(nl + 1, 0);
    int64_t slot = 0;
    for (int32_t l = 0; l < nl; ++l) {
      const int64_t r = S.cend[S.leaves[l]] - S.cbegin[S.leaves[l]];
      int64_t cols = 0;
      for (int64_t b = S.near_ptr[l]; b < S.near_ptr[l + 1]; ++b) {
        const int32_t c = S.near_col[b];
        const int64_t w = S.cend[c] - S.cbegin[c];
        cols += w;
        if (leaf_index[c] != l) {
          S.near_slot[b] = slot;
          slot += w;
          S.near_in_ptr[leaf_index[c] + 1]++;
        }
      }
      S.panel_off[l + 1] = S.panel_off[l] + r * cols;
    }
    for (int32_t l = 0; l < nl; ++l) S.near_in_ptr[l + 1] += S.near_in_ptr[l];
    S.near_in_slot.resize(S.near_in_ptr[nl]);
    std::vector<int64_t> fill(S.near_in_ptr.begin(), S.near_in_ptr.end() - 1);
    for (int32_t l = 0; l < nl; ++l)
      for (int64_t b = S.near_ptr[l]; b < S.near_ptr[l + 1]; ++b)
        if (S.near_slot[b] >= 0) S.near_in_slot[fill[leaf_index[S.near_col[b]]]++] = S.near_slot[b];
    S.near_scratch = slot;
    S.near_stored = S.panel_off[nl];
    S.sym_n = true;
  }
}

}  // namespace h2

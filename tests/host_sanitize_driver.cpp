// Host code of the library under AddressSanitizer and UBSan (built with g++ by
// tests/test_host_sanitizers.py): tree and block-tree construction (Definition 1,
// eq. admissibility) for m = 1, 3, 4 and leaf sizes 16 and 64, the symmetric
// halving of the block lists, and the quadrature generators.  Each argument is a
// mesh file: int64 nv, int64 nt, nv x 3 doubles, nt x 3 int32.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <vector>
#include "structure.h"
#include "quadrules.h"
using namespace h2;

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    FILE* f = std::fopen(argv[a], "rb");
    int64_t hdr[2];
    if (std::fread(hdr, 8, 2, f) != 2) return 2;
    std::vector<double> V(hdr[0] * 3);
    std::vector<int32_t> T(hdr[1] * 3);
    if (std::fread(V.data(), 8, V.size(), f) != V.size()) return 2;
    if (std::fread(T.data(), 4, T.size(), f) != T.size()) return 2;
    std::fclose(f);
    for (int m : {1, 3, 4}) {
      for (int leaf : {16, 64}) {
        Structure S;
        build_structure(S, V.data(), hdr[0], T.data(), hdr[1], m, leaf, 0.5);
        // every position is in exactly one leaf; perm is a permutation
        std::vector<int> seen(S.n, 0);
        for (int32_t p : S.perm) seen[p]++;
        for (int c : seen) if (c != 1) { std::printf("perm broken\n"); return 1; }
        int64_t cover = 0;
        for (int32_t l : S.leaves) cover += S.cend[l] - S.cbegin[l];
        if (cover != S.n) { std::printf("leaves do not cover\n"); return 1; }
        Structure A = S, B = S, C = S;
        make_symmetric(A, true, true);
        make_symmetric(B, false, true);
        if (m == 4 && leaf == 64) make_symmetric(C, true, false);
        std::printf("%s m=%d leaf=%d: n=%lld clusters=%d adm=%lld near=%lld near_entries=%lld sym kept near %lld\n",
                    argv[a], m, leaf, (long long)S.n, S.nclusters, (long long)S.adm_blocks, (long long)S.near_blocks,
                    (long long)S.near_entries, (long long)A.near_stored);
      }
    }
  }
  for (int q = 1; q <= 8; ++q) {
    std::vector<double> t, w;
    gauss_legendre_unit(q, t, w);
    TriRule r = conical_product_rule(q);
    for (int c = 0; c < 3; ++c) {
      std::vector<double> ss = sauter_schwab_rule(static_cast<SSCase>(c), q);
      double sw = 0;
      for (size_t i = 4; i < ss.size(); i += 5) sw += ss[i];
      if (q >= 2 && std::abs(sw - 0.25) > 1e-12) {
        std::printf("Sauter-Schwab weights q=%d case=%d sum to %.17g\n", q, c, sw);
        return 1;
      }
    }
  }
  TriRule r7 = radon_seven_point();
  std::printf("quadrature ok (radon %d points)\n", r7.size());
  return 0;
}

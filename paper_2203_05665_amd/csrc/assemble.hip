// Assembly of the H^2 matrix data on the GPU (FP64 arithmetic, stored in the
// handle's storage precision):
//   leaf matrices     v_{tau,i nu} = int_{T_i} l_{tau,nu}            (eq. leafV)
//   transfer matrices e_{tau',nu' nu} = l_{tau,nu}(xi_{tau',nu'})     (eq. transfer)
//   coupling matrices s_{nu mu} = g(xi_{tau,nu}, xi_{sigma,mu})       (eq. coupling)
//   near-field blocks g_ij = int_{T_i} int_{T_j} g                   (def. of g_ij)
// Interpolation points: tensor Chebyshev points of the first kind in each
// cluster box; an axis narrower than 1e-3 diam(tau) is widened to that width
// about its centre (boxes of zero thickness occur on flat faces).
// Near field: Radon's 7-point rule on both triangles, or Sauter-Schwab rules for
// triangles sharing a vertex; the triangle with the smaller original index is
// the x-triangle, so g_ij and g_ji are computed identically.
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <thread>
#include <type_traits>

#include <algorithm>
#include <cmath>
#include <numeric>

#include "handle.h"
#include "quadrules.h"

namespace h2 {
namespace {

constexpr double kPi = 3.14159265358979323846;

struct KernelFn {
  int kind;
  double kappa;
};

// g(x, y) -> (re, im)
__device__ inline void kernel_eval(const KernelFn kf, double x0, double x1, double x2, double y0, double y1,
                                   double y2, double& re, double& im) {
  im = 0.0;
  if (kf.kind == H2_TEST_ONE) {
    re = 1.0;
    return;
  }
  if (kf.kind == H2_TEST_BILINEAR) {
    re = x0 * y0 + x1 * y1 + x2 * y2;
    return;
  }
  if (kf.kind == H2_TEST_QUADRATIC) {
    const double d = x0 * y0 + x1 * y1 + x2 * y2;
    re = d * d;
    return;
  }
  const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
  const double q = d0 * d0 + d1 * d1 + d2 * d2;
  // one reciprocal square root instead of a square root and a division (the
  // FP64 assembly's most expensive steps; both within a few ulp)
  const double rinv = rsqrt(q);
  const double inv = rinv * (1.0 / (4.0 * kPi));
  if (kf.kind == H2_HELMHOLTZ) {
    double sn, cs;
    sincos(kf.kappa * (q * rinv), &sn, &cs);
    re = cs * inv;
    im = sn * inv;
  } else {
    re = inv;
  }
}

template <typename T>
__device__ inline void store(T* p, double v);
template <>
__device__ inline void store<double>(double* p, double v) { *p = v; }
template <>
__device__ inline void store<float>(float* p, double v) { *p = static_cast<float>(v); }
template <>
__device__ inline void store<bf16>(bf16* p, double v) {
  // round to nearest even from the FP32 value
  const float f = static_cast<float>(v);
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  p->v = static_cast<uint16_t>(u >> 16);
}

// Lagrange polynomial L_j of the points t[0..m) at x.
__device__ inline double lagrange1(const double* t, int m, int j, double x) {
  double v = 1.0;
  for (int i = 0; i < m; ++i)
    if (i != j) v *= (x - t[i]) / (t[j] - t[i]);
  return v;
}

__device__ inline void tri_vertices(const double* vert, const int32_t* tri, int32_t t, double P[9]) {
  for (int a = 0; a < 3; ++a) {
    const int64_t v = tri[3 * static_cast<int64_t>(t) + a];
    P[3 * a] = vert[3 * v];
    P[3 * a + 1] = vert[3 * v + 1];
    P[3 * a + 2] = vert[3 * v + 2];
  }
}

__device__ inline double tri_area(const double P[9]) {
  const double u0 = P[3] - P[0], u1 = P[4] - P[1], u2 = P[5] - P[2];
  const double v0 = P[6] - P[0], v1 = P[7] - P[1], v2 = P[8] - P[2];
  const double c0 = u1 * v2 - u2 * v1, c1 = u2 * v0 - u0 * v2, c2 = u0 * v1 - u1 * v0;
  return 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
}

// ---------------------------------------------------------------- leaf matrices
template <typename ST>
__global__ void asm_leaf(int64_t n, int k, int m, const int32_t* __restrict__ perm,
                         const int32_t* __restrict__ leaf_of_pos, const int32_t* __restrict__ leaves,
                         const int32_t* __restrict__ cbegin, const int32_t* __restrict__ cend,
                         const double* __restrict__ pts, const double* __restrict__ vert,
                         const int32_t* __restrict__ tri, const double* __restrict__ lam,
                         const double* __restrict__ qw, int nq, ST* __restrict__ Vf, ST* __restrict__ Vb) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t p = e / k;
  const int nu = static_cast<int>(e % k);
  const int32_t c = leaves[leaf_of_pos[p]];
  const int64_t b0 = cbegin[c];
  const int64_t r = cend[c] - b0;
  double P[9];
  tri_vertices(vert, tri, perm[p], P);
  const double area = tri_area(P);
  const double* tc = pts + static_cast<int64_t>(c) * 3 * m;
  const int n1 = nu % m, n2 = (nu / m) % m, n3 = nu / (m * m);
  double s = 0.0;
  for (int q = 0; q < nq; ++q) {
    const double l0 = lam[3 * q], l1 = lam[3 * q + 1], l2 = lam[3 * q + 2];
    const double x0 = l0 * P[0] + l1 * P[3] + l2 * P[6];
    const double x1 = l0 * P[1] + l1 * P[4] + l2 * P[7];
    const double x2 = l0 * P[2] + l1 * P[5] + l2 * P[8];
    s += qw[q] * lagrange1(tc, m, n1, x0) * lagrange1(tc + m, m, n2, x1) * lagrange1(tc + 2 * m, m, n3, x2);
  }
  const double v = area * s;
  store(Vf + p * k + nu, v);
  store(Vb + b0 * k + static_cast<int64_t>(nu) * r + (p - b0), v);
}

// ---------------------------------------------------------------- transfer matrices
template <typename ST>
__global__ void asm_transfer(int nc, int k, int m, const int32_t* __restrict__ parent,
                             const double* __restrict__ pts, ST* __restrict__ F, ST* __restrict__ ET) {
  const int64_t kk = static_cast<int64_t>(k) * k;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nc * kk) return;
  const int64_t c = e / kk;
  if (c == 0) return;  // the root has no transfer matrix
  const int rem = static_cast<int>(e % kk);
  const int nup = rem / k, nu = rem % k;  // row nu' (child point), column nu (parent polynomial)
  const double* tc = pts + c * 3 * m;
  const double* tp = pts + static_cast<int64_t>(parent[c]) * 3 * m;
  const double x0 = tc[nup % m], x1 = tc[m + (nup / m) % m], x2 = tc[2 * m + nup / (m * m)];
  const double v = lagrange1(tp, m, nu % m, x0) * lagrange1(tp + m, m, (nu / m) % m, x1) *
                   lagrange1(tp + 2 * m, m, nu / (m * m), x2);
  store(F + c * kk + static_cast<int64_t>(nup) * k + nu, v);
  store(ET + c * kk + static_cast<int64_t>(nu) * k + nup, v);
}

// one-dimensional factors of the transfer matrices: the Lagrange polynomials
// are tensor products, so E_c[nu'][nu] = prod_d l_{nu_d}(xi_{nu'_d}) (eq. transfer)
template <typename ST>
__global__ void asm_transfer1d(int nc, int m, const int32_t* __restrict__ parent, const double* __restrict__ pts,
                               ST* __restrict__ E1) {
  const int64_t mm3 = 3 * static_cast<int64_t>(m) * m;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nc * mm3) return;
  const int64_t c = e / mm3;
  const int rem = static_cast<int>(e % mm3);
  const int d = rem / (m * m), i = (rem / m) % m, j = rem % m;
  double v = 0.0;
  if (c > 0) v = lagrange1(pts + static_cast<int64_t>(parent[c]) * 3 * m + d * m, m, j, pts[c * 3 * m + d * m + i]);
  store(E1 + e, v);
}

// ---------------------------------------------------------------- coupling matrices
template <typename ST, bool CPLX>
__global__ void asm_coupling(int64_t nblocks, int k, int m, KernelFn kf, const int32_t* __restrict__ row,
                             const int32_t* __restrict__ col, const double* __restrict__ pts,
                             ST* __restrict__ S) {
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const int64_t kk = static_cast<int64_t>(k) * k;
  const double* tt = pts + static_cast<int64_t>(row[b]) * 3 * m;
  const double* ts = pts + static_cast<int64_t>(col[b]) * 3 * m;
  for (int e = threadIdx.x; e < kk; e += blockDim.x) {
    const int nu = e / k, mu = e % k;
    double re, im;
    kernel_eval(kf, tt[nu % m], tt[m + (nu / m) % m], tt[2 * m + nu / (m * m)], ts[mu % m],
                ts[m + (mu / m) % m], ts[2 * m + mu / (m * m)], re, im);
    if (CPLX) {
      store(S + 2 * (b * kk + e), re);
      store(S + 2 * (b * kk + e) + 1, im);
    } else {
      store(S + b * kk + e, re);
    }
  }
}

// ---------------------------------------------------------------- near field, regular pairs
struct NearArgs {
  const int32_t* perm;
  const int32_t* cbegin;
  const int32_t* cend;
  const int32_t* leaves;
  const int32_t* near_row;   // per near block: row leaf index
  const int32_t* near_col;   // per near block: column cluster
  const int32_t* near_cs;    // per near block: first panel column
  const int64_t* panel_off;  // per row leaf
  const double* vert;
  const int32_t* tri;
  const double* rlam;  // 7 x 3
  const double* rw;    // 7
};

__device__ inline bool touching(const int32_t* tri, int32_t a, int32_t b) {
  const int32_t* A = tri + 3 * static_cast<int64_t>(a);
  const int32_t* B = tri + 3 * static_cast<int64_t>(b);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (A[i] == B[j]) return true;
  return false;
}

template <typename ST, bool CPLX>
__global__ void asm_near_regular(int64_t nblocks, KernelFn kf, bool smooth, NearArgs A, ST* __restrict__ N) {
  const int64_t bb = blockIdx.x;
  if (bb >= nblocks) return;
  const int32_t l = A.near_row[bb];
  const int32_t tau = A.leaves[l];
  const int32_t sig = A.near_col[bb];
  const int64_t b0 = A.cbegin[tau], r = A.cend[tau] - b0;
  const int64_t s0 = A.cbegin[sig], w = A.cend[sig] - s0;
  const int64_t base = A.panel_off[l] + static_cast<int64_t>(A.near_cs[bb]) * r;
  for (int64_t e = threadIdx.x; e < r * w; e += blockDim.x) {
    const int64_t i = e % r, j = e / r;
    const int32_t ti = A.perm[b0 + i], tj = A.perm[s0 + j];
    const int32_t ta = min(ti, tj), tb = max(ti, tj);
    double re = 0.0, im = 0.0;
    if (smooth || !touching(A.tri, ta, tb)) {
      double Pa[9], Pb[9];
      tri_vertices(A.vert, A.tri, ta, Pa);
      tri_vertices(A.vert, A.tri, tb, Pb);
      double xa[21], xb[21];
      for (int q = 0; q < 7; ++q)
        for (int d = 0; d < 3; ++d) {
          xa[3 * q + d] = A.rlam[3 * q] * Pa[d] + A.rlam[3 * q + 1] * Pa[3 + d] + A.rlam[3 * q + 2] * Pa[6 + d];
          xb[3 * q + d] = A.rlam[3 * q] * Pb[d] + A.rlam[3 * q + 1] * Pb[3 + d] + A.rlam[3 * q + 2] * Pb[6 + d];
        }
      for (int qa = 0; qa < 7; ++qa) {
        double sr = 0.0, si = 0.0;
        for (int qb = 0; qb < 7; ++qb) {
          double gr, gi;
          kernel_eval(kf, xa[3 * qa], xa[3 * qa + 1], xa[3 * qa + 2], xb[3 * qb], xb[3 * qb + 1], xb[3 * qb + 2],
                      gr, gi);
          sr += A.rw[qb] * gr;
          si += A.rw[qb] * gi;
        }
        re += A.rw[qa] * sr;
        im += A.rw[qa] * si;
      }
      const double f = tri_area(Pa) * tri_area(Pb);
      re *= f;
      im *= f;
    }
    const int64_t off = base + j * r + i;
    if (CPLX) {
      store(N + 2 * off, re);
      store(N + 2 * off + 1, im);
    } else {
      store(N + off, re);
    }
  }
}

// ---------------------------------------------------------------- near field, touching pairs
struct SSArgs {
  const double* vert;
  const int32_t* tri;
  const double* rule[3];
  int npts[3];
};

// one wave per touching pair; lanes share the quadrature points
template <typename ST, bool CPLX>
__global__ void asm_near_singular(int64_t npairs, KernelFn kf, SSArgs A, const int64_t* __restrict__ dst,
                                  const int32_t* __restrict__ pa, const int32_t* __restrict__ pb,
                                  ST* __restrict__ N) {
  const int64_t pr = static_cast<int64_t>(blockIdx.x) * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (pr >= npairs) return;
  const int32_t a = pa[pr], b = pb[pr];
  int32_t va[3], vb[3];
  for (int i = 0; i < 3; ++i) {
    va[i] = A.tri[3 * static_cast<int64_t>(a) + i];
    vb[i] = A.tri[3 * static_cast<int64_t>(b) + i];
  }
  int cs;
  int32_t oa[3], ob[3];
  if (a == b) {
    cs = SS_IDENTICAL;
    for (int i = 0; i < 3; ++i) oa[i] = ob[i] = va[i];
  } else {
    int32_t sh[3];
    int ns = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (va[i] == vb[j]) sh[ns++] = va[i];
    if (ns == 2) {
      cs = SS_EDGE;
      const int32_t u = min(sh[0], sh[1]), w = max(sh[0], sh[1]);
      oa[0] = ob[0] = u;
      oa[1] = ob[1] = w;
      for (int i = 0; i < 3; ++i) {
        if (va[i] != u && va[i] != w) oa[2] = va[i];
        if (vb[i] != u && vb[i] != w) ob[2] = vb[i];
      }
    } else {
      cs = SS_VERTEX;
      int ka = 0, kb = 0;
      for (int i = 0; i < 3; ++i) {
        if (va[i] == sh[0]) ka = i;
        if (vb[i] == sh[0]) kb = i;
      }
      for (int i = 0; i < 3; ++i) {
        oa[i] = va[(ka + i) % 3];
        ob[i] = vb[(kb + i) % 3];
      }
    }
  }
  double Pa[9], Pb[9];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) {
      Pa[3 * i + d] = A.vert[3 * static_cast<int64_t>(oa[i]) + d];
      Pb[3 * i + d] = A.vert[3 * static_cast<int64_t>(ob[i]) + d];
    }
  const double* R = A.rule[cs];
  const int np = A.npts[cs];
  double sr = 0.0, si = 0.0;
  for (int q = lane; q < np; q += 64) {
    const double x1 = R[5 * q], x2 = R[5 * q + 1], y1 = R[5 * q + 2], y2 = R[5 * q + 3], wq = R[5 * q + 4];
    double x[3], y[3];
    for (int d = 0; d < 3; ++d) {
      x[d] = Pa[d] + x1 * (Pa[3 + d] - Pa[d]) + x2 * (Pa[6 + d] - Pa[3 + d]);
      y[d] = Pb[d] + y1 * (Pb[3 + d] - Pb[d]) + y2 * (Pb[6 + d] - Pb[3 + d]);
    }
    double gr, gi;
    kernel_eval(kf, x[0], x[1], x[2], y[0], y[1], y[2], gr, gi);
    sr += wq * gr;
    si += wq * gi;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    sr += __shfl_xor(sr, off);
    si += __shfl_xor(si, off);
  }
  if (lane == 0) {
    double PA[9], PB[9];
    tri_vertices(A.vert, A.tri, a, PA);
    tri_vertices(A.vert, A.tri, b, PB);
    const double f = 4.0 * tri_area(PA) * tri_area(PB);
    if (CPLX) {
      store(N + 2 * dst[pr], f * sr);
      store(N + 2 * dst[pr] + 1, f * si);
    } else {
      store(N + dst[pr], f * sr);
    }
  }
}

inline unsigned grid_for(int64_t work, int block) {
  const int64_t g = (work + block - 1) / block;
  if (g > 0x7fffffff) throw Error(H2_EINVAL, "problem too large for one launch");
  return static_cast<unsigned>(std::max<int64_t>(g, 1));
}

// Per-cluster Chebyshev points (3 x m per cluster), computed on the host.
std::vector<double> cluster_points(const Structure& S) {
  const int m = S.m;
  std::vector<double> pts(static_cast<size_t>(S.nclusters) * 3 * m);
  const double pi = kPi;
  for (int32_t c = 0; c < S.nclusters; ++c) {
    const double h0 = S.hi[3 * c] - S.lo[3 * c], h1 = S.hi[3 * c + 1] - S.lo[3 * c + 1],
                 h2v = S.hi[3 * c + 2] - S.lo[3 * c + 2];
    const double diam = std::sqrt(h0 * h0 + h1 * h1 + h2v * h2v);
    for (int d = 0; d < 3; ++d) {
      const double width = std::max(S.hi[3 * c + d] - S.lo[3 * c + d], 1e-3 * diam);
      const double mid = 0.5 * (S.lo[3 * c + d] + S.hi[3 * c + d]);
      for (int j = 0; j < m; ++j)
        pts[(static_cast<size_t>(c) * 3 + d) * m + j] = mid + 0.5 * width * std::cos(pi * (2.0 * j + 1.0) / (2.0 * m));
    }
  }
  return pts;
}

template <typename VT, typename SST, bool CPLX>
void assemble_typed(h2_handle_s& H) {
  const Structure& S = H.S;
  const int k = S.k, m = S.m;
  const int64_t n = S.n, nc = S.nclusters, kk = static_cast<int64_t>(k) * k;
  const int cw = CPLX ? 2 : 1;
  const KernelFn kf{H.P.kernel, H.P.kappa};
  const bool smooth = H.P.kernel == H2_TEST_ONE || H.P.kernel == H2_TEST_BILINEAR || H.P.kernel == H2_TEST_QUADRATIC;

  H.Vf.alloc(n * k * sizeof(VT));
  H.Vb.alloc(n * k * sizeof(VT));
  H.F.alloc(nc * kk * sizeof(VT));
  H.ET.alloc(nc * kk * sizeof(VT));
  H.Smat.alloc(H.otf ? 16 : static_cast<int64_t>(S.adm_col.size()) * kk * cw * sizeof(SST));
  H.Nmat.alloc(S.near_stored * cw * sizeof(VT));
  H2_HIP(hipMemset(H.F.p, 0, H.F.bytes));
  H2_HIP(hipMemset(H.ET.p, 0, H.ET.bytes));

  // geometry and rules
  DBuf vert, tri, lof, lam, qw, rlam, rw, arow, nrow, ncs;
  vert.upload(S.vert);
  tri.upload(S.tri);
  lof.upload(S.leaf_of_pos);
  // exact for total degree 3(m-1) with one point per direction to spare
  const TriRule vr = conical_product_rule((3 * (m - 1) + 2 + 1) / 2 + 1);
  lam.upload(vr.lam);
  qw.upload(vr.w);
  const TriRule r7 = radon_seven_point();
  rlam.upload(r7.lam);
  rw.upload(r7.w);

  asm_leaf<VT><<<grid_for(n * k, 256), 256>>>(n, k, m, H.perm.as<int32_t>(), lof.as<int32_t>(),
                                               H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                               H.cend.as<int32_t>(), H.pts.as<double>(), vert.as<double>(),
                                               tri.as<int32_t>(), lam.as<double>(), qw.as<double>(), vr.size(),
                                               H.Vf.as<VT>(), H.Vb.as<VT>());
  H2_HIP(hipGetLastError());
  asm_transfer<VT><<<grid_for(nc * kk, 256), 256>>>(static_cast<int>(nc), k, m, H.parent.as<int32_t>(),
                                                    H.pts.as<double>(), H.F.as<VT>(), H.ET.as<VT>());
  H2_HIP(hipGetLastError());
  H.E1.alloc(nc * 3 * m * m * sizeof(VT));
  asm_transfer1d<VT><<<grid_for(nc * 3 * m * m, 256), 256>>>(static_cast<int>(nc), m, H.parent.as<int32_t>(),
                                                             H.pts.as<double>(), H.E1.as<VT>());
  H2_HIP(hipGetLastError());

  // coupling: row index of every admissible block
  const int64_t nadm = static_cast<int64_t>(S.adm_col.size());
  if (nadm > 0 && !H.otf) {
    std::vector<int32_t> row(nadm);
    for (int32_t c = 0; c < S.nclusters; ++c)
      for (int64_t b = S.adm_ptr[c]; b < S.adm_ptr[c + 1]; ++b) row[b] = c;
    arow.upload(row);
    if (nadm > 0x7fffffff) throw Error(H2_EINVAL, "too many admissible blocks");
    asm_coupling<SST, CPLX><<<static_cast<unsigned>(nadm), 256>>>(nadm, k, m, kf, arow.as<int32_t>(),
                                                                   H.adm_col.as<int32_t>(), H.pts.as<double>(),
                                                                   H.Smat.as<SST>());
    H2_HIP(hipGetLastError());
    if constexpr (std::is_same<SST, bf16>::value) {
      // the same entries rounded to FP32, for the FP64-accumulated products
      H.Smat32.alloc(static_cast<size_t>(nadm) * kk * sizeof(float));
      asm_coupling<float, false><<<static_cast<unsigned>(nadm), 256>>>(nadm, k, m, kf, arow.as<int32_t>(),
                                                                      H.adm_col.as<int32_t>(), H.pts.as<double>(),
                                                                      H.Smat32.as<float>());
      H2_HIP(hipGetLastError());
    }
  }

  // near field: block row / first column of every inadmissible block
  const int64_t nnear = static_cast<int64_t>(S.near_col.size());
  const int32_t nl = static_cast<int32_t>(S.leaves.size());
  std::vector<int32_t> nr(nnear), cs(nnear);
  for (int32_t l = 0; l < nl; ++l) {
    int32_t col = 0;
    for (int64_t b = S.near_ptr[l]; b < S.near_ptr[l + 1]; ++b) {
      nr[b] = l;
      cs[b] = col;
      col += S.cend[S.near_col[b]] - S.cbegin[S.near_col[b]];
    }
  }
  nrow.upload(nr);
  ncs.upload(cs);
  NearArgs na{H.perm.as<int32_t>(), H.cbegin.as<int32_t>(), H.cend.as<int32_t>(), H.leaves.as<int32_t>(),
              nrow.as<int32_t>(), H.near_col.as<int32_t>(), ncs.as<int32_t>(), H.panel_off.as<int64_t>(),
              vert.as<double>(), tri.as<int32_t>(), rlam.as<double>(), rw.as<double>()};
  if (nnear > 0x7fffffff) throw Error(H2_EINVAL, "too many near-field blocks");
  if (nnear > 0) {
    asm_near_regular<VT, CPLX><<<static_cast<unsigned>(nnear), 256>>>(nnear, kf, smooth, na, H.Nmat.as<VT>());
    H2_HIP(hipGetLastError());
  }

  if (!smooth) {
    // touching pairs: for every position p, the triangles sharing a vertex with perm[p]
    const int64_t nv = static_cast<int64_t>(S.vert.size() / 3);
    std::vector<int64_t> vptr(nv + 1, 0);
    for (int64_t i = 0; i < 3 * n; ++i) vptr[S.tri[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vt(3 * n), fill(vptr.begin(), vptr.end() - 1);
    for (int64_t t = 0; t < n; ++t)
      for (int a = 0; a < 3; ++a) vt[fill[S.tri[3 * t + a]]++] = static_cast<int32_t>(t);
    std::vector<int32_t> inv(n);
    for (int64_t p = 0; p < n; ++p) inv[S.perm[p]] = static_cast<int32_t>(p);
    // the touching pairs of positions [p0, p1), one list per Sauter-Schwab case;
    // chunks of positions run on separate threads and their lists are joined in
    // position order
    struct Lists {
      std::vector<int64_t> dst[3];
      std::vector<int32_t> ta[3], tb[3];
      std::string err;
    };
    auto scan = [&](int64_t p0, int64_t p1, Lists& L) {
      std::vector<int32_t> nb;
      for (int64_t p = p0; p < p1; ++p) {
        const int32_t t = S.perm[p];
        nb.clear();
        for (int a = 0; a < 3; ++a) {
          const int32_t v = S.tri[3 * static_cast<int64_t>(t) + a];
          for (int64_t q = vptr[v]; q < vptr[v + 1]; ++q) nb.push_back(vt[q]);
        }
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        const int32_t l = S.leaf_of_pos[p];
        const int32_t tau = S.leaves[l];
        const int64_t r = S.cend[tau] - S.cbegin[tau];
        for (int32_t t2 : nb) {
          const int32_t q = inv[t2];
          // symmetric storage keeps the pair in the block of the earlier leaf only
          if (S.sym_n && S.leaf_of_pos[q] < l) continue;
          const int32_t sc = S.leaves[S.leaf_of_pos[q]];
          // the near block (l, sc): columns of row l are sorted by cluster start
          const int64_t lo = S.near_ptr[l], hi = S.near_ptr[l + 1];
          const int32_t* beg = S.near_col.data();
          int64_t a0 = lo, a1 = hi;
          while (a0 < a1) {
            const int64_t mid = (a0 + a1) / 2;
            if (S.cbegin[beg[mid]] < S.cbegin[sc]) a0 = mid + 1; else a1 = mid;
          }
          if (!(a0 < hi && beg[a0] == sc)) {
            L.err = "touching pair outside the near field";
            return;
          }
          int shared = 0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              shared += S.tri[3 * static_cast<int64_t>(t) + i] == S.tri[3 * static_cast<int64_t>(t2) + j];
          const int c = (t == t2) ? SS_IDENTICAL : (shared >= 2 ? SS_EDGE : SS_VERTEX);
          L.dst[c].push_back(S.panel_off[l] + (static_cast<int64_t>(cs[a0]) + (q - S.cbegin[sc])) * r +
                             (p - S.cbegin[tau]));
          L.ta[c].push_back(std::min(t, t2));
          L.tb[c].push_back(std::max(t, t2));
        }
      }
    };
    const int64_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int nth = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(hw, n / 8192)));
    std::vector<Lists> lists(nth);
    {
      std::vector<std::thread> pool;
      for (int w = 1; w < nth; ++w) pool.emplace_back(scan, n * w / nth, n * (w + 1) / nth, std::ref(lists[w]));
      scan(0, n / nth, lists[0]);
      for (auto& th : pool) th.join();
    }
    for (const Lists& L : lists)
      if (!L.err.empty()) throw Error(H2_EINTERNAL, L.err);
    std::vector<int64_t> dst[3];
    std::vector<int32_t> ta[3], tb[3];
    for (int c = 0; c < 3; ++c)
      for (const Lists& L : lists) {
        dst[c].insert(dst[c].end(), L.dst[c].begin(), L.dst[c].end());
        ta[c].insert(ta[c].end(), L.ta[c].begin(), L.ta[c].end());
        tb[c].insert(tb[c].end(), L.tb[c].begin(), L.tb[c].end());
      }
    SSArgs sa{};
    sa.vert = vert.as<double>();
    sa.tri = tri.as<int32_t>();
    DBuf rules[3];
    for (int c = 0; c < 3; ++c) {
      const std::vector<double> R = sauter_schwab_rule(static_cast<SSCase>(c), H.P.q_ss);
      rules[c].upload(R);
      sa.rule[c] = rules[c].as<double>();
      sa.npts[c] = static_cast<int>(R.size() / 5);
    }
    for (int c = 0; c < 3; ++c) {
      const int64_t np = static_cast<int64_t>(dst[c].size());
      if (np == 0) continue;
      DBuf d, a, b;
      d.upload(dst[c]);
      a.upload(ta[c]);
      b.upload(tb[c]);
      asm_near_singular<VT, CPLX><<<grid_for(np, 4), 256>>>(np, kf, sa, d.as<int64_t>(), a.as<int32_t>(),
                                                             b.as<int32_t>(), H.Nmat.as<VT>());
      H2_HIP(hipGetLastError());
      H2_HIP(hipDeviceSynchronize());
    }
  }
  H2_HIP(hipDeviceSynchronize());
}

}  // namespace

void assemble(h2_handle_s& H) {
  const std::vector<double> pts = cluster_points(H.S);
  H.pts.upload(pts);
  if (H.otf) {
    // centres of the (padded) point boxes and the offsets of the points from them
    const Structure& S = H.S;
    const int m = S.m;
    std::vector<double> ctr(3 * static_cast<size_t>(S.nclusters)), o64(pts.size());
    std::vector<float> o32(pts.size());
    for (int32_t c = 0; c < S.nclusters; ++c)
      for (int d = 0; d < 3; ++d) {
        const double mid = 0.5 * (S.lo[3 * c + d] + S.hi[3 * c + d]);
        ctr[3 * c + d] = mid;
        for (int j = 0; j < m; ++j) {
          const size_t i = (static_cast<size_t>(c) * 3 + d) * m + j;
          o64[i] = pts[i] - mid;
          o32[i] = static_cast<float>(o64[i]);
        }
      }
    H.ctr.upload(ctr);
    H.off64.upload(o64);
    H.off32.upload(o32);
  }
  if (H.is_complex) {
    if (H.P.storage == H2_F64) assemble_typed<double, double, true>(H);
    else assemble_typed<float, float, true>(H);
  } else if (H.P.storage == H2_F64) {
    assemble_typed<double, double, false>(H);
  } else if (H.P.storage == H2_F32) {
    assemble_typed<float, float, false>(H);
  } else {
    assemble_typed<float, bf16, false>(H);
  }
}

}  // namespace h2

// Algebraic recompression of the interpolation H^2 matrix: orthonormal nested
// bases, truncated by the weights of everything a cluster carries, one uniform
// rank k' for all clusters, a multiple of 4 (smaller ranks padded with zero
// columns), after which
// the product runs on the same kernels with k' in place of k.
//
// The paper defers such approximations (the GCA-H^2 variant in the section on
// distributed matrix setup; the recompression algorithm in the outlook, whose
// weight matrices follow the patterns of the forward transformation and of the
// interaction phase).  The construction used here:
//   1. orthogonalisation, bottom up: V_leaf = Q R; for a parent the stacked
//      [R_c E_c] of its children is factored Q R and the blocks of Q become the
//      orthonormal transfer matrices, so V-bar_tau = Q-bar_tau R_tau;
//   2. weights, top down: G_tau = E'_tau G_parent E'_tau^T
//      + sum_sigma (R_tau S R_sigma^T)(R_tau S R_sigma^T)^T over the admissible
//      blocks of the row (the sum over blocks runs on the device as
//      R_tau [sum_sigma S C_sigma S^T] R_tau^T with C_sigma = R_sigma^T R_sigma);
//   3. truncation, bottom up: a leaf keeps the dominant eigenvectors of G; a
//      parent those of P G P^T with P = [T_c E'_c] its basis written in the
//      children's truncated bases; T_tau maps the orthonormal basis to the new one;
//   4. coupling, on the device: S'' = (T_tau R_tau) S (T_sigma R_sigma)^T.
// Rank rule per cluster: eps = 0 keeps everything (T = I); eps > 0 keeps the
// eigenvalues above eps^2 times the largest; max_rank caps.  The discarded
// eigenvalues bound the change: ||G~ - G~'||_F^2 <= 2 * discarded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "handle.h"

namespace h2 {
namespace {

// ---------------------------------------------------------------- device: FP64 64 x 64 products
// One 256-thread workgroup; thread t owns rows ti + 16 a and columns tj + 16 b
// (a, b = 0..3) of a 64 x 64 result; operands in LDS with a padded row pitch.
constexpr int RP = 65;

template <typename SST>
__device__ inline void load_tile(double (*dst)[RP], const SST* __restrict__ src, int k) {
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    dst[i][j] = (i < k && j < k) ? static_cast<double>(src[i * k + j]) : 0.0;
  }
}

// H_c = sum over the admissible blocks b of row c of S_b C_{col b} S_b^T
template <typename SST>
__global__ __launch_bounds__(256) void rc_gram(int nc, int k, const int64_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col, const SST* __restrict__ S,
                                               const double* __restrict__ C, double* __restrict__ H) {
  __shared__ double sS[64][RP];
  __shared__ double sB[64][RP];
  const int c = blockIdx.x;
  if (c >= nc) return;
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
  const int64_t kk = static_cast<int64_t>(k) * k;
  double h[4][4] = {};
  for (int64_t b = ptr[c]; b < ptr[c + 1]; ++b) {
    load_tile(sS, S + b * kk, k);
    load_tile(sB, C + static_cast<int64_t>(col[b]) * kk, k);
    __syncthreads();
    double t[4][4] = {};
    for (int l = 0; l < 64; ++l)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) t[a][bb] += sS[ti + 16 * a][l] * sB[l][tj + 16 * bb];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) sB[ti + 16 * a][tj + 16 * bb] = t[a][bb];
    __syncthreads();
    for (int l = 0; l < 64; ++l)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) h[a][bb] += sB[ti + 16 * a][l] * sS[tj + 16 * bb][l];
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int i = ti + 16 * a, j = tj + 16 * bb;
      if (i < k && j < k) H[c * kk + i * k + j] = h[a][bb];
    }
}

// S''_b = P_row S_b P_col^T; P is 64 x 64 per cluster (rows >= its rank are 0),
// S''_b is kp x kp at the storage precision
template <typename SST>
__global__ __launch_bounds__(256) void rc_project(int64_t nblocks, int k, int kp, const int32_t* __restrict__ row,
                                                  const int32_t* __restrict__ col, const SST* __restrict__ S,
                                                  const double* __restrict__ P, SST* __restrict__ Sn) {
  __shared__ double sA[64][RP];
  __shared__ double sB[64][RP];
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
  load_tile(sA, S + b * k * k, k);
  const double* Pc = P + static_cast<int64_t>(col[b]) * 4096;
  for (int e = threadIdx.x; e < 4096; e += 256) sB[e / 64][e % 64] = Pc[e];
  __syncthreads();
  double u[4][4] = {};  // U = S P_col^T
  for (int l = 0; l < 64; ++l)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) u[a][bb] += sA[ti + 16 * a][l] * sB[tj + 16 * bb][l];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) sA[ti + 16 * a][tj + 16 * bb] = u[a][bb];
  const double* Pr = P + static_cast<int64_t>(row[b]) * 4096;
  for (int e = threadIdx.x; e < 4096; e += 256) sB[e / 64][e % 64] = Pr[e];
  __syncthreads();
  double o[4][4] = {};  // P_row U
  for (int l = 0; l < 64; ++l)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) o[a][bb] += sB[ti + 16 * a][l] * sA[l][tj + 16 * bb];
  const int64_t kpp = static_cast<int64_t>(kp) * kp;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int i = ti + 16 * a, j = tj + 16 * bb;
      if (i < kp && j < kp) Sn[b * kpp + i * kp + j] = static_cast<SST>(o[a][bb]);
    }
}

// ---------------------------------------------------------------- host: small dense linear algebra (FP64)
// Row-major matrices: element (i, j) of an m x n matrix at a[i * n + j].

// C (m x n) = A (m x l) B (l x n)
void gemm(int m, int n, int l, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i) {
    double* ci = C + static_cast<size_t>(i) * n;
    for (int j = 0; j < n; ++j) ci[j] = 0.0;
    for (int p = 0; p < l; ++p) {
      const double a = A[static_cast<size_t>(i) * l + p];
      if (a == 0.0) continue;
      const double* bp = B + static_cast<size_t>(p) * n;
      for (int j = 0; j < n; ++j) ci[j] += a * bp[j];
    }
  }
}

// C (m x n) = A (m x l) B^T, B n x l
void gemm_nt(int m, int n, int l, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      const double* ai = A + static_cast<size_t>(i) * l;
      const double* bj = B + static_cast<size_t>(j) * l;
      for (int p = 0; p < l; ++p) s += ai[p] * bj[p];
      C[static_cast<size_t>(i) * n + j] = s;
    }
}

// Thin Householder QR of A (m x n): Q (m x q) with orthonormal columns and
// R (q x n) upper trapezoidal, q = min(m, n), A = Q R.
void qr_thin(int m, int n, const double* A, std::vector<double>& Q, std::vector<double>& R, int& q) {
  q = std::min(m, n);
  std::vector<double> W(A, A + static_cast<size_t>(m) * n);
  std::vector<double> V(static_cast<size_t>(q) * m, 0.0), beta(q, 0.0);
  for (int j = 0; j < q; ++j) {
    double nrm = 0.0;
    for (int i = j; i < m; ++i) nrm += W[static_cast<size_t>(i) * n + j] * W[static_cast<size_t>(i) * n + j];
    nrm = std::sqrt(nrm);
    double* v = V.data() + static_cast<size_t>(j) * m;
    if (nrm == 0.0) continue;
    const double x0 = W[static_cast<size_t>(j) * n + j];
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    for (int i = j; i < m; ++i) v[i] = W[static_cast<size_t>(i) * n + j];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    beta[j] = 2.0 / vv;
    for (int c = j; c < n; ++c) {
      double s = 0.0;
      for (int i = j; i < m; ++i) s += v[i] * W[static_cast<size_t>(i) * n + c];
      s *= beta[j];
      for (int i = j; i < m; ++i) W[static_cast<size_t>(i) * n + c] -= s * v[i];
    }
  }
  R.assign(static_cast<size_t>(q) * n, 0.0);
  for (int i = 0; i < q; ++i)
    for (int c = i; c < n; ++c) R[static_cast<size_t>(i) * n + c] = W[static_cast<size_t>(i) * n + c];
  // Q = H_0 H_1 ... H_{q-1} applied to the first q columns of the identity
  Q.assign(static_cast<size_t>(m) * q, 0.0);
  for (int i = 0; i < q; ++i) Q[static_cast<size_t>(i) * q + i] = 1.0;
  for (int j = q - 1; j >= 0; --j) {
    if (beta[j] == 0.0) continue;
    const double* v = V.data() + static_cast<size_t>(j) * m;
    for (int c = 0; c < q; ++c) {
      double s = 0.0;
      for (int i = j; i < m; ++i) s += v[i] * Q[static_cast<size_t>(i) * q + c];
      s *= beta[j];
      for (int i = j; i < m; ++i) Q[static_cast<size_t>(i) * q + c] -= s * v[i];
    }
  }
}

// Eigen-decomposition of a symmetric n x n matrix by cyclic Jacobi rotations:
// lam descending, U (n x n) with the eigenvectors as columns.
void eig_sym(int n, const double* A0, std::vector<double>& lam, std::vector<double>& U) {
  std::vector<double> A(A0, A0 + static_cast<size_t>(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const double s = 0.5 * (A[static_cast<size_t>(i) * n + j] + A[static_cast<size_t>(j) * n + i]);
      A[static_cast<size_t>(i) * n + j] = A[static_cast<size_t>(j) * n + i] = s;
    }
  U.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) U[static_cast<size_t>(i) * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[static_cast<size_t>(i) * n + j]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += a(i, i) * a(i, i);
      for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
    }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int qq = p + 1; qq < n; ++qq) {
        const double apq = a(p, qq);
        if (apq == 0.0) continue;
        const double app = a(p, p), aqq = a(qq, qq);
        if (std::fabs(apq) <= 1e-300 + 1e-18 * std::sqrt(std::fabs(app * aqq))) {
          a(p, qq) = a(qq, p) = 0.0;
          continue;
        }
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int r = 0; r < n; ++r) {
          const double arp = a(r, p), arq = a(r, qq);
          a(r, p) = cs * arp - sn * arq;
          a(r, qq) = sn * arp + cs * arq;
        }
        for (int r = 0; r < n; ++r) {
          const double apr = a(p, r), aqr = a(qq, r);
          a(p, r) = cs * apr - sn * aqr;
          a(qq, r) = sn * apr + cs * aqr;
        }
        for (int r = 0; r < n; ++r) {
          double* ur = U.data() + static_cast<size_t>(r) * n;
          const double up = ur[p], uq = ur[qq];
          ur[p] = cs * up - sn * uq;
          ur[qq] = sn * up + cs * uq;
        }
      }
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return a(x, x) > a(y, y); });
  lam.resize(n);
  std::vector<double> Us(static_cast<size_t>(n) * n);
  for (int c = 0; c < n; ++c) {
    lam[c] = a(order[c], order[c]);
    for (int r = 0; r < n; ++r) Us[static_cast<size_t>(r) * n + c] = U[static_cast<size_t>(r) * n + order[c]];
  }
  U.swap(Us);
}

template <class F>
void parallel_for(int begin, int end, F f) {
  const int n = end - begin;
  if (n <= 0) return;
  const int nt = std::max(1, std::min<int>(n, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
  if (nt == 1) {
    for (int i = begin; i < end; ++i) f(i);
    return;
  }
  std::atomic<int> next{begin};
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&]() {
      for (int i = next++; i < end; i = next++) f(i);
    });
  for (auto& th : pool) th.join();
}

int rank_rule(const std::vector<double>& lam, double eps, int cap, int full) {
  int r;
  if (eps == 0.0) {
    r = full;
  } else if (lam.empty() || lam[0] <= 0.0) {
    r = 0;
  } else {
    r = 0;
    for (double l : lam)
      if (l > eps * eps * lam[0]) ++r;
  }
  if (cap > 0) r = std::min(r, cap);
  return r;
}

template <typename T>
std::vector<double> download(const DBuf& b, size_t count) {
  std::vector<T> raw(count);
  if (count) H2_HIP(hipMemcpy(raw.data(), b.p, count * sizeof(T), hipMemcpyDeviceToHost));
  return std::vector<double>(raw.begin(), raw.end());
}

template <typename T>
void upload_as(DBuf& b, const std::vector<double>& v) {
  std::vector<T> raw(v.begin(), v.end());
  b.upload(raw);
}

template <typename ST>
void run(h2_handle_s& H, double eps, int cap, h2_recompress_info& info, hipStream_t st) {
  Structure& S = H.S;
  const int k = S.k, nc = S.nclusters;
  const int64_t n = S.n, kk = static_cast<int64_t>(k) * k;
  const int64_t nadm = static_cast<int64_t>(S.adm_col.size());
  const std::vector<double> Vf = download<ST>(H.Vf, static_cast<size_t>(n) * k);
  const std::vector<double> F = download<ST>(H.F, static_cast<size_t>(nc) * kk);
  std::vector<char> is_leaf(nc, 0);
  for (int32_t c : S.leaves) is_leaf[c] = 1;
  auto children = [&](int c, int* ch) {
    int cnt = 0;
    if (S.child0[c] >= 0) ch[cnt++] = S.child0[c];
    if (S.child1[c] >= 0) ch[cnt++] = S.child1[c];
    return cnt;
  };
  auto level_range = [&](int l, int& a, int& b) {
    a = S.level_ptr[l];
    b = S.level_ptr[l + 1];
  };
  // 1. orthogonalisation (levels bottom up)
  std::vector<int> kd(nc, 0);
  std::vector<std::vector<double>> R(nc), Qleaf(nc), Eo(nc);  // Eo[c]: kd[c] x kd[parent]
  for (int l = S.depth; l >= 0; --l) {
    int a, b;
    level_range(l, a, b);
    parallel_for(a, b, [&](int c) {
      if (is_leaf[c]) {
        const int r = S.cend[c] - S.cbegin[c];
        int q;
        qr_thin(r, k, Vf.data() + static_cast<size_t>(S.cbegin[c]) * k, Qleaf[c], R[c], q);
        kd[c] = q;
        return;
      }
      int ch[2];
      const int nch = children(c, ch);
      int rows = 0;
      for (int i = 0; i < nch; ++i) rows += kd[ch[i]];
      std::vector<double> M(static_cast<size_t>(rows) * k);
      int off = 0;
      for (int i = 0; i < nch; ++i) {
        gemm(kd[ch[i]], k, k, R[ch[i]].data(), F.data() + static_cast<size_t>(ch[i]) * kk,
             M.data() + static_cast<size_t>(off) * k);
        off += kd[ch[i]];
      }
      std::vector<double> Q;
      int q;
      qr_thin(rows, k, M.data(), Q, R[c], q);
      kd[c] = q;
      off = 0;
      for (int i = 0; i < nch; ++i) {
        Eo[ch[i]].assign(Q.begin() + static_cast<size_t>(off) * q, Q.begin() + static_cast<size_t>(off + kd[ch[i]]) * q);
        off += kd[ch[i]];
      }
    });
  }
  // 2. weights: the admissible sum on the device, then top down on the host
  std::vector<double> Ch(static_cast<size_t>(nc) * kk, 0.0);
  parallel_for(0, nc, [&](int c) {
    // C_c = R_c^T R_c (k x k)
    const double* Rc = R[c].data();
    double* out = Ch.data() + static_cast<size_t>(c) * kk;
    for (int p = 0; p < kd[c]; ++p)
      for (int i = 0; i < k; ++i) {
        const double rpi = Rc[static_cast<size_t>(p) * k + i];
        if (rpi == 0.0) continue;
        for (int j = 0; j < k; ++j) out[static_cast<size_t>(i) * k + j] += rpi * Rc[static_cast<size_t>(p) * k + j];
      }
  });
  DBuf dC, dH;
  dC.upload(Ch);
  dH.alloc(static_cast<size_t>(nc) * kk * sizeof(double));
  using SST = ST;
  if (nc > 0)
    rc_gram<SST><<<nc, 256, 0, st>>>(nc, k, H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(), H.Smat.as<SST>(),
                                     dC.as<double>(), dH.as<double>());
  H2_HIP(hipGetLastError());
  H2_HIP(hipStreamSynchronize(st));
  std::vector<double> Hh(static_cast<size_t>(nc) * kk);
  if (nc) H2_HIP(hipMemcpy(Hh.data(), dH.p, Hh.size() * sizeof(double), hipMemcpyDeviceToHost));
  dC.release();
  dH.release();
  std::vector<std::vector<double>> G(nc);
  for (int l = 0; l <= S.depth; ++l) {
    int a, b;
    level_range(l, a, b);
    parallel_for(a, b, [&](int c) {
      const int q = kd[c];
      std::vector<double> T1(static_cast<size_t>(q) * k), Gc(static_cast<size_t>(q) * q);
      gemm(q, k, k, R[c].data(), Hh.data() + static_cast<size_t>(c) * kk, T1.data());
      gemm_nt(q, q, k, T1.data(), R[c].data(), Gc.data());
      const int p = S.parent[c];
      if (p >= 0) {
        const int qp = kd[p];
        std::vector<double> T2(static_cast<size_t>(q) * qp), T3(static_cast<size_t>(q) * q);
        gemm(q, qp, qp, Eo[c].data(), G[p].data(), T2.data());
        gemm_nt(q, q, qp, T2.data(), Eo[c].data(), T3.data());
        for (size_t i = 0; i < Gc.size(); ++i) Gc[i] += T3[i];
      }
      G[c].swap(Gc);
    });
  }
  Hh.clear();
  Hh.shrink_to_fit();
  // 3. truncation (levels bottom up)
  std::vector<int> rk(nc, 0);
  std::vector<double> disc(nc, 0.0);
  std::vector<std::vector<double>> T(nc), Vn(nc), En(nc);  // T[c]: rk x kd; En[c]: rk[c] x rk[parent]
  for (int l = S.depth; l >= 0; --l) {
    int a, b;
    level_range(l, a, b);
    parallel_for(a, b, [&](int c) {
      const int q = kd[c];
      int ch[2];
      const int nch = is_leaf[c] ? 0 : children(c, ch);
      if (eps == 0.0 && (cap <= 0 || cap >= q)) {  // nothing is cut: T = I
        rk[c] = q;
        T[c].assign(static_cast<size_t>(q) * q, 0.0);
        for (int i = 0; i < q; ++i) T[c][static_cast<size_t>(i) * q + i] = 1.0;
        if (is_leaf[c]) Vn[c] = Qleaf[c];
        for (int i = 0; i < nch; ++i) En[ch[i]] = Eo[ch[i]];
        return;
      }
      std::vector<double> lam, U;
      if (is_leaf[c]) {
        eig_sym(q, G[c].data(), lam, U);
        const int r = rank_rule(lam, eps, cap, q);
        rk[c] = r;
        T[c].assign(static_cast<size_t>(r) * q, 0.0);
        for (int i = 0; i < r; ++i)
          for (int j = 0; j < q; ++j) T[c][static_cast<size_t>(i) * q + j] = U[static_cast<size_t>(j) * q + i];
        const int rows = S.cend[c] - S.cbegin[c];
        Vn[c].assign(static_cast<size_t>(rows) * r, 0.0);
        for (int p = 0; p < rows; ++p)
          for (int i = 0; i < r; ++i) {
            double s = 0.0;
            for (int j = 0; j < q; ++j) s += Qleaf[c][static_cast<size_t>(p) * q + j] * U[static_cast<size_t>(j) * q + i];
            Vn[c][static_cast<size_t>(p) * r + i] = s;
          }
        for (int i = r; i < q; ++i) disc[c] += std::max(lam[i], 0.0);
        return;
      }
      int rows = 0;
      for (int i = 0; i < nch; ++i) rows += rk[ch[i]];
      std::vector<double> P(static_cast<size_t>(rows) * q);
      int off = 0;
      for (int i = 0; i < nch; ++i) {
        gemm(rk[ch[i]], q, kd[ch[i]], T[ch[i]].data(), Eo[ch[i]].data(), P.data() + static_cast<size_t>(off) * q);
        off += rk[ch[i]];
      }
      std::vector<double> PG(static_cast<size_t>(rows) * q), W(static_cast<size_t>(rows) * rows);
      gemm(rows, q, q, P.data(), G[c].data(), PG.data());
      gemm_nt(rows, rows, q, PG.data(), P.data(), W.data());
      eig_sym(rows, W.data(), lam, U);
      const int r = rank_rule(lam, eps, cap, std::min(rows, q));
      rk[c] = r;
      off = 0;
      for (int i = 0; i < nch; ++i) {
        const int rc = rk[ch[i]];
        En[ch[i]].assign(static_cast<size_t>(rc) * r, 0.0);
        for (int x = 0; x < rc; ++x)
          for (int y = 0; y < r; ++y) En[ch[i]][static_cast<size_t>(x) * r + y] = U[static_cast<size_t>(off + x) * rows + y];
        off += rc;
      }
      T[c].assign(static_cast<size_t>(r) * q, 0.0);  // U_r^T P
      for (int i = 0; i < r; ++i)
        for (int x = 0; x < rows; ++x) {
          const double u = U[static_cast<size_t>(x) * rows + i];
          if (u == 0.0) continue;
          for (int j = 0; j < q; ++j) T[c][static_cast<size_t>(i) * q + j] += u * P[static_cast<size_t>(x) * q + j];
        }
      for (int i = r; i < rows; ++i) disc[c] += std::max(lam[i], 0.0);
    });
  }
  // one rank for all clusters, rounded up to a multiple of 4 (rows of S'' and x^
  // are then read as 16-byte vectors) unless that exceeds k; padding columns are zero
  int kp = 1;
  for (int c = 0; c < nc; ++c) kp = std::max(kp, rk[c]);
  kp = std::min(k, (kp + 3) / 4 * 4);  // never above the rank it started from (k <= 64)
  double discarded = 0.0;
  for (int c = 0; c < nc; ++c) discarded += disc[c];
  // 4. coupling on the device: P_c = T_c R_c (rk x k), padded to 64 x 64
  std::vector<double> Pf(static_cast<size_t>(nc) * 4096, 0.0);
  parallel_for(0, nc, [&](int c) {
    std::vector<double> PR(static_cast<size_t>(rk[c]) * k);
    gemm(rk[c], k, kd[c], T[c].data(), R[c].data(), PR.data());
    for (int i = 0; i < rk[c]; ++i)
      for (int j = 0; j < k; ++j) Pf[static_cast<size_t>(c) * 4096 + i * 64 + j] = PR[static_cast<size_t>(i) * k + j];
  });
  std::vector<int32_t> arow(nadm);
  for (int32_t c = 0; c < nc; ++c)
    for (int64_t b = S.adm_ptr[c]; b < S.adm_ptr[c + 1]; ++b) arow[b] = c;
  DBuf dP, dRow, Snew;
  dP.upload(Pf);
  dRow.upload(arow);
  Snew.alloc(static_cast<size_t>(nadm) * kp * kp * sizeof(SST));
  if (nadm > 0)
    rc_project<SST><<<static_cast<unsigned>(nadm), 256, 0, st>>>(nadm, k, kp, dRow.as<int32_t>(),
                                                                 H.adm_col.as<int32_t>(), H.Smat.as<SST>(),
                                                                 dP.as<double>(), Snew.as<SST>());
  H2_HIP(hipGetLastError());
  H2_HIP(hipStreamSynchronize(st));
  // new leaf bases (forward layout: position-major; backward: per leaf column-major)
  std::vector<double> vf(static_cast<size_t>(n) * kp, 0.0), vb(static_cast<size_t>(n) * kp, 0.0);
  for (int32_t c : S.leaves) {
    const int64_t b0 = S.cbegin[c];
    const int rows = S.cend[c] - S.cbegin[c];
    for (int p = 0; p < rows; ++p)
      for (int i = 0; i < rk[c]; ++i) {
        const double v = Vn[c][static_cast<size_t>(p) * rk[c] + i];
        vf[static_cast<size_t>(b0 + p) * kp + i] = v;
        vb[static_cast<size_t>(b0) * kp + static_cast<size_t>(i) * rows + p] = v;
      }
  }
  // new transfer matrices: F[c][nu'][nu] = E''_c (child row nu', parent column nu), ET its transpose
  const int64_t kpp = static_cast<int64_t>(kp) * kp;
  std::vector<double> fn(static_cast<size_t>(nc) * kpp, 0.0), etn(static_cast<size_t>(nc) * kpp, 0.0);
  for (int c = 1; c < nc; ++c) {
    const int p = S.parent[c];
    if (p < 0) continue;
    for (int x = 0; x < rk[c]; ++x)
      for (int y = 0; y < rk[p]; ++y) {
        const double v = En[c][static_cast<size_t>(x) * rk[p] + y];
        fn[static_cast<size_t>(c) * kpp + static_cast<size_t>(x) * kp + y] = v;
        etn[static_cast<size_t>(c) * kpp + static_cast<size_t>(y) * kp + x] = v;
      }
  }
  const int64_t before = static_cast<int64_t>(H.Vf.bytes + H.Vb.bytes + H.F.bytes + H.ET.bytes + H.E1.bytes +
                                              H.Smat.bytes);
  upload_as<ST>(H.Vf, vf);
  upload_as<ST>(H.Vb, vb);
  upload_as<ST>(H.F, fn);
  upload_as<ST>(H.ET, etn);
  std::swap(H.Smat.p, Snew.p);
  std::swap(H.Smat.bytes, Snew.bytes);
  Snew.release();
  H.E1.release();
  H.kron = false;
  S.k = kp;
  H.tune_slot = 0;  // a slot width tuned for the old rank may not cover the new one
  info.rank = kp;
  info.rank_before = k;
  info.discarded = discarded;
  info.bytes_before = before;
  info.bytes_after = static_cast<int64_t>(H.Vf.bytes + H.Vb.bytes + H.F.bytes + H.ET.bytes + H.Smat.bytes);
}

}  // namespace

void recompress(h2_handle_s& H, double eps, int max_rank, h2_recompress_info& info, hipStream_t st) {
  if (H.host_only) throw Error(H2_EINVAL, "recompression needs a device structure");
  if (H.is_complex) throw Error(H2_EINVAL, "recompression is implemented for real kernels");
  if (H.otf) throw Error(H2_EINVAL, "recompression needs stored coupling matrices (not H2_COUPLING_OTF)");
  if (H.S.sym_s) throw Error(H2_EINVAL, "recompression needs full coupling storage (not H2_SYMMETRIC)");
  if (H.P.storage != H2_F64 && H.P.storage != H2_F32)
    throw Error(H2_EINVAL, "recompression needs H2_F64 or H2_F32 storage");
  if (!(eps >= 0.0) || !std::isfinite(eps)) throw Error(H2_EINVAL, "eps must be finite and >= 0");
  if (max_rank < 0) throw Error(H2_EINVAL, "max_rank must be >= 0");
  if (H.S.k > 64) throw Error(H2_EINVAL, "recompression supports k <= 64");
  const auto t0 = std::chrono::steady_clock::now();
  info = h2_recompress_info{};
  H2_HIP(hipStreamSynchronize(st));
  if (H.P.storage == H2_F64) run<double>(H, eps, max_rank, info, st);
  else run<float>(H, eps, max_rank, info, st);
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace h2

// Krylov solvers for G~ z = b (the paper's introduction names Krylov methods
// for the Galerkin system): conjugate gradients for the symmetric positive
// definite Laplace single-layer matrix, and restarted GMRES with classical
// Gram-Schmidt applied twice and complex Givens rotations for any nonsingular
// matrix (the Helmholtz matrix is complex symmetric, not Hermitian).  All
// vectors and inner products are FP64 (complex FP64 for Helmholtz) on the
// device; reductions use a fixed two-stage order, so a solve is reproducible.
// Optional iterative refinement: the outer residual b - G~ z is recomputed with
// FP64 accumulation over the stored matrix, the inner solve uses the storage
// precision's accumulation.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "handle.h"

namespace h2 {
namespace {

using cd = std::complex<double>;
constexpr int kRedBlocks = 512;
constexpr int kMaxCols = 121;  // restart <= 120

// a vector of n entries is n doubles (real) or 2n doubles (complex, interleaved)
__global__ __launch_bounds__(256) void fill(int64_t len, double* __restrict__ v, double a) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    v[i] = a;
}

// y = a x + b y
template <bool CX>
__global__ __launch_bounds__(256) void axpby(int64_t n, double ar, double ai, const double* __restrict__ x, double br,
                                             double bi, double* __restrict__ y) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (CX) {
      const double xr = x[2 * i], xi = x[2 * i + 1], yr = y[2 * i], yi = y[2 * i + 1];
      y[2 * i] = ar * xr - ai * xi + br * yr - bi * yi;
      y[2 * i + 1] = ar * xi + ai * xr + br * yi + bi * yr;
    } else {
      y[i] = ar * x[i] + br * y[i];
    }
  }
}

// partial[(c * 2 + part) * gridDim + block] = sum_i conj(Q_c[i]) w[i]
template <bool CX>
__global__ __launch_bounds__(256) void multi_dot(int64_t n, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                 const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double red[2][256];
  for (int c = 0; c < ncols; ++c) {
    double sr = 0.0, si = 0.0;
    const double* q = Q + c * ldq;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
      if (CX) {
        const double qr = q[2 * i], qi = q[2 * i + 1], wr = w[2 * i], wi = w[2 * i + 1];
        sr += qr * wr + qi * wi;
        si += qr * wi - qi * wr;
      } else {
        sr += q[i] * w[i];
      }
    }
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        red[0][threadIdx.x] += red[0][threadIdx.x + o];
        red[1][threadIdx.x] += red[1][threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partial[(2 * static_cast<int64_t>(c)) * gridDim.x + blockIdx.x] = red[0][0];
      partial[(2 * static_cast<int64_t>(c) + 1) * gridDim.x + blockIdx.x] = red[1][0];
    }
    __syncthreads();
  }
}

// out[2c + part] = sum over blocks
__global__ __launch_bounds__(256) void finish_dot(int ncols, int nb, const double* __restrict__ partial,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  for (int c = 0; c < 2 * ncols; ++c) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[static_cast<int64_t>(c) * nb + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
    __syncthreads();
  }
}

// w += sign * sum_c h_c Q_c   (h interleaved complex pairs; imaginary parts ignored when real)
template <bool CX>
__global__ __launch_bounds__(256) void multi_axpy(int64_t n, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                  const double* __restrict__ h, double sign, double* __restrict__ w) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < ncols; ++c) {
      const double hr = h[2 * c], hi = h[2 * c + 1];
      if (CX) {
        const double qr = Q[c * ldq + 2 * i], qi = Q[c * ldq + 2 * i + 1];
        sr += hr * qr - hi * qi;
        si += hr * qi + hi * qr;
      } else {
        sr += hr * Q[c * ldq + i];
      }
    }
    if (CX) {
      w[2 * i] += sign * sr;
      w[2 * i + 1] += sign * si;
    } else {
      w[i] += sign * sr;
    }
  }
}

template <bool CX>
struct Ctx {
  h2_handle_s& H;
  hipStream_t st;
  int64_t n, len;
  DBuf partial, dres, hdev;
  double* host = nullptr;  // pinned scalars
  unsigned grid;
  Ctx(h2_handle_s& h, hipStream_t s) : H(h), st(s), n(h.S.n), len(CX ? 2 * h.S.n : h.S.n) {
    grid = static_cast<unsigned>(std::min<int64_t>(kRedBlocks, (n + 255) / 256));
    partial.alloc(sizeof(double) * grid * 2 * kMaxCols);
    dres.alloc(sizeof(double) * 2 * kMaxCols);
    hdev.alloc(sizeof(double) * 2 * kMaxCols);
    H2_HIP(hipHostMalloc(reinterpret_cast<void**>(&host), 2 * kMaxCols * sizeof(double), hipHostMallocDefault));
  }
  ~Ctx() {
    if (host) (void)hipHostFree(host);
  }
  unsigned eg() const { return static_cast<unsigned>(std::min<int64_t>(2048, (n + 255) / 256)); }
  // <Q_c, w> for c < nc (conjugating Q), results in out
  void dots(const double* Q, int64_t ldq, int nc, const double* w, std::vector<cd>& out) {
    multi_dot<CX><<<grid, 256, 0, st>>>(n, nc, Q, ldq, w, partial.as<double>());
    finish_dot<<<1, 256, 0, st>>>(nc, static_cast<int>(grid), partial.as<double>(), dres.as<double>());
    H2_HIP(hipMemcpyAsync(host, dres.p, 2 * nc * sizeof(double), hipMemcpyDeviceToHost, st));
    H2_HIP(hipStreamSynchronize(st));
    out.resize(nc);
    for (int c = 0; c < nc; ++c) out[c] = cd(host[2 * c], CX ? host[2 * c + 1] : 0.0);
  }
  cd dot(const double* a, const double* b) {
    std::vector<cd> v;
    dots(a, 0, 1, b, v);
    return v[0];
  }
  double nrm(const double* a) { return std::sqrt(std::max(0.0, dot(a, a).real())); }
  void set(double* v, double a) { fill<<<eg(), 256, 0, st>>>(len, v, a); }
  void axpby_(cd a, const double* x, cd b, double* y) {
    axpby<CX><<<eg(), 256, 0, st>>>(n, a.real(), a.imag(), x, b.real(), b.imag(), y);
  }
  // w += sign * sum_c h_c Q_c
  void combine(const double* Q, int64_t ldq, const std::vector<cd>& h, int nc, double sign, double* w) {
    for (int c = 0; c < nc; ++c) {
      host[2 * c] = h[c].real();
      host[2 * c + 1] = h[c].imag();
    }
    H2_HIP(hipMemcpyAsync(hdev.p, host, 2 * nc * sizeof(double), hipMemcpyHostToDevice, st));
    multi_axpy<CX><<<eg(), 256, 0, st>>>(n, nc, Q, ldq, hdev.as<double>(), sign, w);
    H2_HIP(hipStreamSynchronize(st));  // `host` is reused by the next call
  }
  // y <- y + alpha A x
  void apply(const double* x, double* y, double alpha, int flags) {
    matvec(H, 1, CX ? H2_C128 : H2_R64, x, n, y, n, alpha, flags, st);
  }
};

// CG on A d = rhs (d starts at 0); real only
int cg(Ctx<false>& C, const double* rhs, double* d, double rtol, int maxit, int flags, double& rel) {
  const int64_t n = C.n;
  DBuf r, p, q;
  r.alloc(n * 8);
  p.alloc(n * 8);
  q.alloc(n * 8);
  H2_HIP(hipMemcpyAsync(r.p, rhs, n * 8, hipMemcpyDeviceToDevice, C.st));
  C.set(d, 0.0);
  H2_HIP(hipMemcpyAsync(p.p, rhs, n * 8, hipMemcpyDeviceToDevice, C.st));
  const double nb = C.nrm(rhs);
  rel = 0.0;
  if (nb == 0.0) return 0;
  double rr = nb * nb;
  int it = 0;
  rel = 1.0;
  while (rel > rtol && it < maxit) {
    C.set(q.as<double>(), 0.0);
    C.apply(p.as<double>(), q.as<double>(), 1.0, flags);
    const double pq = C.dot(p.as<double>(), q.as<double>()).real();
    if (!(pq > 0.0)) break;
    const double alpha = rr / pq;
    C.axpby_(alpha, p.as<double>(), 1.0, d);
    C.axpby_(-alpha, q.as<double>(), 1.0, r.as<double>());
    const double rr2 = C.dot(r.as<double>(), r.as<double>()).real();
    C.axpby_(1.0, r.as<double>(), rr2 / rr, p.as<double>());
    rr = rr2;
    ++it;
    rel = std::sqrt(rr) / nb;
    if (!std::isfinite(rel)) break;
  }
  return it;
}

// GMRES(restart) on A d = rhs with d starting at 0
template <bool CX>
int gmres(Ctx<CX>& C, const double* rhs, double* d, int restart, double rtol, int maxit, int flags, double& rel) {
  const int64_t len = C.len;
  const int m = std::max(1, std::min(restart, kMaxCols - 1));
  DBuf Q, w, r;
  Q.alloc(static_cast<size_t>(len) * (m + 1) * 8);
  w.alloc(len * 8);
  r.alloc(len * 8);
  C.set(d, 0.0);
  const double nb = C.nrm(rhs);
  rel = 0.0;
  if (nb == 0.0) return 0;
  int it = 0;
  rel = 1.0;
  std::vector<cd> Hm((m + 1) * m), cs(m), sn(m), g(m + 1), hcol(m + 1), tmp;
  double* Qp = Q.as<double>();
  while (it < maxit) {
    H2_HIP(hipMemcpyAsync(r.p, rhs, len * 8, hipMemcpyDeviceToDevice, C.st));
    if (it > 0) C.apply(d, r.as<double>(), -1.0, flags);
    const double beta = C.nrm(r.as<double>());
    rel = beta / nb;
    if (rel <= rtol || !std::isfinite(rel)) break;
    C.axpby_(1.0 / beta, r.as<double>(), 0.0, Qp);
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    int j_done = 0;
    for (int j = 0; j < m && it < maxit; ++j) {
      double* wj = w.as<double>();
      C.set(wj, 0.0);
      C.apply(Qp + static_cast<int64_t>(j) * len, wj, 1.0, flags);
      std::fill(hcol.begin(), hcol.end(), cd(0.0));
      for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
        C.dots(Qp, len, j + 1, wj, tmp);
        C.combine(Qp, len, tmp, j + 1, -1.0, wj);
        for (int i = 0; i <= j; ++i) hcol[i] += tmp[i];
      }
      const double hn = C.nrm(wj);
      hcol[j + 1] = hn;
      if (hn > 0.0) C.axpby_(1.0 / hn, wj, 0.0, Qp + static_cast<int64_t>(j + 1) * len);
      for (int i = 0; i < j; ++i) {  // earlier rotations
        const cd t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
        hcol[i + 1] = -std::conj(sn[i]) * hcol[i] + cs[i] * hcol[i + 1];
        hcol[i] = t;
      }
      const cd a = hcol[j], c = hcol[j + 1];
      const double den = std::sqrt(std::norm(a) + std::norm(c));
      if (std::abs(a) == 0.0) {
        cs[j] = 0.0;
        sn[j] = 1.0;
      } else {
        cs[j] = std::abs(a) / den;
        sn[j] = (a / std::abs(a)) * std::conj(c) / den;
      }
      hcol[j] = cs[j] * a + sn[j] * c;
      hcol[j + 1] = 0.0;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) Hm[i * m + j] = hcol[i];
      ++it;
      j_done = j + 1;
      rel = std::abs(g[j + 1]) / nb;
      if (rel <= rtol || hn == 0.0) break;
    }
    std::vector<cd> y(j_done);
    for (int i = j_done - 1; i >= 0; --i) {
      cd s = g[i];
      for (int l = i + 1; l < j_done; ++l) s -= Hm[i * m + l] * y[l];
      y[i] = s / Hm[i * m + i];
    }
    C.combine(Qp, len, y, j_done, 1.0, d);
    if (rel <= rtol) {  // confirm with the true residual
      H2_HIP(hipMemcpyAsync(r.p, rhs, len * 8, hipMemcpyDeviceToDevice, C.st));
      C.apply(d, r.as<double>(), -1.0, flags);
      rel = C.nrm(r.as<double>()) / nb;
      if (rel <= rtol) break;
    }
  }
  return it;
}

template <bool CX>
int solve_t(h2_handle_s& H, const double* b, double* z, const h2_solve_params& p, h2_solve_info& info,
            hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  Ctx<CX> C(H, st);
  const int64_t len = C.len;
  const bool refine = p.refine != 0 && H.P.storage != H2_F64;
  const int outer_flags = refine ? H2_ACC_F64 : 0;
  DBuf r, d;
  r.alloc(len * 8);
  d.alloc(len * 8);
  const double nb = C.nrm(b);
  info = h2_solve_info{};
  if (nb == 0.0) {
    C.set(z, 0.0);
    H2_HIP(hipStreamSynchronize(st));
    info.outer = 1;
    return H2_OK;
  }
  int total = 0, outer = 0;
  double rel = 1.0;
  const int max_outer = refine ? 30 : 1;
  while (outer < max_outer && total < p.maxit) {
    H2_HIP(hipMemcpyAsync(r.p, b, len * 8, hipMemcpyDeviceToDevice, st));
    C.apply(z, r.as<double>(), -1.0, outer_flags);
    rel = C.nrm(r.as<double>()) / nb;
    if (rel <= p.rtol) break;
    ++outer;
    const double tol = refine ? std::max(p.inner_rtol, 0.5 * p.rtol / rel) : p.rtol / rel;
    double irel = 1.0;
    const int left = p.maxit - total;
    int its;
    if constexpr (CX)
      its = gmres<true>(C, r.as<double>(), d.as<double>(), p.restart, tol, left, 0, irel);
    else
      its = p.method == H2_CG ? cg(C, r.as<double>(), d.as<double>(), tol, left, 0, irel)
                              : gmres<false>(C, r.as<double>(), d.as<double>(), p.restart, tol, left, 0, irel);
    total += its;
    C.axpby_(1.0, d.as<double>(), 1.0, z);
    if (its == 0) break;
  }
  H2_HIP(hipMemcpyAsync(r.p, b, len * 8, hipMemcpyDeviceToDevice, st));
  C.apply(z, r.as<double>(), -1.0, outer_flags);
  rel = C.nrm(r.as<double>()) / nb;
  info.iterations = total;
  info.outer = std::max(outer, 1);
  info.rel_residual = rel;
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rel <= p.rtol ? H2_OK : H2_ENOTCONV;
}

}  // namespace

int solve(h2_handle_s& H, const void* b, void* z, const h2_solve_params& p, h2_solve_info& info, hipStream_t st) {
  if (H.host_only) throw Error(H2_EINVAL, "handle was built with H2_HOST_ONLY");
  if (p.method != H2_CG && p.method != H2_GMRES) throw Error(H2_EINVAL, "unknown method");
  if (H.is_complex && p.method != H2_GMRES) throw Error(H2_EINVAL, "the Helmholtz matrix needs H2_GMRES");
  if (!(p.rtol > 0.0) || p.maxit < 1) throw Error(H2_EINVAL, "rtol must be > 0 and maxit >= 1");
  if (p.method == H2_GMRES && (p.restart < 1 || p.restart > kMaxCols - 1))
    throw Error(H2_EINVAL, "restart must be in [1, 120]");
  if (H.is_complex)
    return solve_t<true>(H, static_cast<const double*>(b), static_cast<double*>(z), p, info, st);
  return solve_t<false>(H, static_cast<const double*>(b), static_cast<double*>(z), p, info, st);
}

}  // namespace h2

// Krylov solvers for G~ z = b (the paper's introduction names Krylov methods
// for the Galerkin system): conjugate gradients for the symmetric positive
// definite Laplace single-layer matrix and restarted GMRES with classical
// Gram-Schmidt applied twice.  All vectors and inner products are FP64 on the
// device; reductions use a fixed two-stage order, so a solve is reproducible.
// Optional iterative refinement: the outer residual b - G~ z is recomputed with
// FP64 accumulation over the stored matrix, the inner solve uses the storage
// precision's accumulation.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "handle.h"

namespace h2 {
namespace {

constexpr int kRedBlocks = 512;

__global__ __launch_bounds__(256) void fill(int64_t n, double* __restrict__ v, double a) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    v[i] = a;
}

__global__ __launch_bounds__(256) void axpby(int64_t n, double a, const double* __restrict__ x, double b,
                                             double* __restrict__ y) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

// partial[c * gridDim + block] = sum_i Q[c][i] * w[i] for c < ncols
__global__ __launch_bounds__(256) void multi_dot(int64_t n, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                 const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double red[256];
  for (int c = 0; c < ncols; ++c) {
    double s = 0.0;
    const double* q = Q + c * ldq;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
      s += q[i] * w[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[static_cast<int64_t>(c) * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// out[c] = sum of partial[c][0..nb)
__global__ __launch_bounds__(256) void finish_dot(int ncols, int nb, const double* __restrict__ partial,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  for (int c = 0; c < ncols; ++c) {
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

// w -= sum_c h[c] Q[c]
__global__ __launch_bounds__(256) void multi_axpy(int64_t n, int ncols, const double* __restrict__ Q, int64_t ldq,
                                                  const double* __restrict__ h, double* __restrict__ w) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < ncols; ++c) s += h[c] * Q[c * ldq + i];
    w[i] -= s;
  }
}

// y += Q h  (combination of basis vectors)
__global__ __launch_bounds__(256) void combine(int64_t n, int ncols, const double* __restrict__ Q, int64_t ldq,
                                               const double* __restrict__ h, double* __restrict__ y) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < ncols; ++c) s += h[c] * Q[c * ldq + i];
    y[i] += s;
  }
}

struct Ctx {
  h2_handle_s& H;
  hipStream_t st;
  int64_t n;
  DBuf partial, dres;
  double* host = nullptr;  // pinned scalars
  unsigned grid;
  Ctx(h2_handle_s& h, hipStream_t s) : H(h), st(s), n(h.S.n) {
    grid = static_cast<unsigned>(std::min<int64_t>(kRedBlocks, (n + 255) / 256));
    partial.alloc(sizeof(double) * grid * 128);
    dres.alloc(sizeof(double) * 128);
    H2_HIP(hipHostMalloc(reinterpret_cast<void**>(&host), 128 * sizeof(double), hipHostMallocDefault));
  }
  ~Ctx() {
    if (host) (void)hipHostFree(host);
  }
  unsigned eg() const { return static_cast<unsigned>(std::min<int64_t>(2048, (n + 255) / 256)); }
  // dots of columns Q[0..nc) with w, result in host[0..nc)
  void dots(const double* Q, int64_t ldq, int nc, const double* w) {
    multi_dot<<<grid, 256, 0, st>>>(n, nc, Q, ldq, w, partial.as<double>());
    finish_dot<<<1, 256, 0, st>>>(nc, static_cast<int>(grid), partial.as<double>(), dres.as<double>());
    H2_HIP(hipMemcpyAsync(host, dres.p, nc * sizeof(double), hipMemcpyDeviceToHost, st));
    H2_HIP(hipStreamSynchronize(st));
  }
  double dot(const double* a, const double* b) {
    dots(a, 0, 1, b);
    return host[0];
  }
  double nrm(const double* a) { return std::sqrt(dot(a, a)); }
  void set(double* v, double a) { fill<<<eg(), 256, 0, st>>>(n, v, a); }
  void axpby_(double a, const double* x, double b, double* y) { axpby<<<eg(), 256, 0, st>>>(n, a, x, b, y); }
  // y <- y + alpha A x
  void apply(const double* x, double* y, double alpha, int flags) {
    matvec(H, 1, H2_R64, x, n, y, n, alpha, flags, st);
  }
};

// CG on A d = r0 (d starts at 0); returns iterations, updates relres estimate
int cg(Ctx& C, const double* rhs, double* d, double rtol, int maxit, int flags, double& rel) {
  const int64_t n = C.n;
  DBuf r, p, q;
  r.alloc(n * 8);
  p.alloc(n * 8);
  q.alloc(n * 8);
  H2_HIP(hipMemcpyAsync(r.p, rhs, n * 8, hipMemcpyDeviceToDevice, C.st));
  C.set(d, 0.0);
  H2_HIP(hipMemcpyAsync(p.p, rhs, n * 8, hipMemcpyDeviceToDevice, C.st));
  const double nb = C.nrm(rhs);
  if (nb == 0.0) {
    rel = 0.0;
    return 0;
  }
  double rr = nb * nb;
  int it = 0;
  rel = 1.0;
  while (rel > rtol && it < maxit) {
    C.set(q.as<double>(), 0.0);
    C.apply(p.as<double>(), q.as<double>(), 1.0, flags);
    const double pq = C.dot(p.as<double>(), q.as<double>());
    if (!(pq > 0.0)) break;
    const double alpha = rr / pq;
    C.axpby_(alpha, p.as<double>(), 1.0, d);
    C.axpby_(-alpha, q.as<double>(), 1.0, r.as<double>());
    const double rr2 = C.dot(r.as<double>(), r.as<double>());
    C.axpby_(1.0, r.as<double>(), rr2 / rr, p.as<double>());
    rr = rr2;
    ++it;
    rel = std::sqrt(rr) / nb;
    if (!std::isfinite(rel)) break;
  }
  return it;
}

// GMRES(restart) on A d = rhs with d starting at 0
int gmres(Ctx& C, const double* rhs, double* d, int restart, double rtol, int maxit, int flags, double& rel) {
  const int64_t n = C.n;
  const int m = std::max(1, std::min(restart, 120));
  DBuf Q, w, r, hdev;
  Q.alloc(static_cast<size_t>(n) * (m + 1) * 8);
  w.alloc(n * 8);
  r.alloc(n * 8);
  hdev.alloc(128 * 8);
  C.set(d, 0.0);
  const double nb = C.nrm(rhs);
  if (nb == 0.0) {
    rel = 0.0;
    return 0;
  }
  int it = 0;
  rel = 1.0;
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), hcol(m + 1);
  while (it < maxit) {
    // r = rhs - A d
    H2_HIP(hipMemcpyAsync(r.p, rhs, n * 8, hipMemcpyDeviceToDevice, C.st));
    if (it > 0) C.apply(d, r.as<double>(), -1.0, flags);
    const double beta = C.nrm(r.as<double>());
    rel = beta / nb;
    if (rel <= rtol || !std::isfinite(rel)) break;
    double* Qp = Q.as<double>();
    C.axpby_(1.0 / beta, r.as<double>(), 0.0, Qp);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j_done = 0;
    for (int j = 0; j < m && it < maxit; ++j) {
      double* wj = w.as<double>();
      C.set(wj, 0.0);
      C.apply(Qp + static_cast<int64_t>(j) * n, wj, 1.0, flags);
      std::fill(hcol.begin(), hcol.end(), 0.0);
      for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
        C.dots(Qp, n, j + 1, wj);
        H2_HIP(hipMemcpyAsync(hdev.p, C.host, (j + 1) * 8, hipMemcpyHostToDevice, C.st));
        multi_axpy<<<C.eg(), 256, 0, C.st>>>(n, j + 1, Qp, n, hdev.as<double>(), wj);
        for (int i = 0; i <= j; ++i) hcol[i] += C.host[i];
      }
      const double hn = C.nrm(wj);
      hcol[j + 1] = hn;
      if (hn > 0.0) C.axpby_(1.0 / hn, wj, 0.0, Qp + static_cast<int64_t>(j + 1) * n);
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
        hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
        hcol[i] = t;
      }
      const double a = hcol[j], c = hcol[j + 1];
      const double den = std::hypot(a, c);
      cs[j] = den == 0.0 ? 1.0 : a / den;
      sn[j] = den == 0.0 ? 0.0 : c / den;
      hcol[j] = cs[j] * a + sn[j] * c;
      hcol[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[i * m + j] = hcol[i];
      ++it;
      j_done = j + 1;
      rel = std::fabs(g[j + 1]) / nb;
      if (rel <= rtol || hn == 0.0) break;
    }
    // back substitution and update
    std::vector<double> y(j_done);
    for (int i = j_done - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < j_done; ++l) s -= H[i * m + l] * y[l];
      y[i] = s / H[i * m + i];
    }
    H2_HIP(hipMemcpyAsync(hdev.p, y.data(), j_done * 8, hipMemcpyHostToDevice, C.st));
    combine<<<C.eg(), 256, 0, C.st>>>(n, j_done, Qp, n, hdev.as<double>(), d);
    H2_HIP(hipStreamSynchronize(C.st));
    if (rel <= rtol) {
      // confirm with the true residual
      H2_HIP(hipMemcpyAsync(r.p, rhs, n * 8, hipMemcpyDeviceToDevice, C.st));
      C.apply(d, r.as<double>(), -1.0, flags);
      rel = C.nrm(r.as<double>()) / nb;
      if (rel <= rtol) break;
    }
  }
  return it;
}

}  // namespace

int solve(h2_handle_s& H, const double* b, double* z, const h2_solve_params& p, h2_solve_info& info,
          hipStream_t st) {
  if (H.host_only) throw Error(H2_EINVAL, "handle was built with H2_HOST_ONLY");
  if (H.is_complex) throw Error(H2_EINVAL, "complex solves are not supported by h2_solve");
  if (p.method != H2_CG && p.method != H2_GMRES) throw Error(H2_EINVAL, "unknown method");
  if (!(p.rtol > 0.0) || p.maxit < 1) throw Error(H2_EINVAL, "rtol must be > 0 and maxit >= 1");
  const auto t0 = std::chrono::steady_clock::now();
  Ctx C(H, st);
  const int64_t n = C.n;
  const bool refine = p.refine != 0 && H.P.storage != H2_F64;
  const int inner_flags = 0;
  const int outer_flags = H2_ACC_F64;
  DBuf r, d;
  r.alloc(n * 8);
  d.alloc(n * 8);
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
    // r = b - A z in FP64 accumulation
    H2_HIP(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, st));
    C.apply(z, r.as<double>(), -1.0, refine ? outer_flags : 0);
    rel = C.nrm(r.as<double>()) / nb;
    if (rel <= p.rtol) break;
    ++outer;
    const double tol = refine ? std::max(p.inner_rtol, 0.5 * p.rtol / rel) : p.rtol / rel;
    double irel = 1.0;
    const int left = p.maxit - total;
    const int its = p.method == H2_CG
                        ? cg(C, r.as<double>(), d.as<double>(), tol, left, refine ? inner_flags : 0, irel)
                        : gmres(C, r.as<double>(), d.as<double>(), p.restart, tol, left,
                                refine ? inner_flags : 0, irel);
    total += its;
    C.axpby_(1.0, d.as<double>(), 1.0, z);
    if (its == 0) break;
  }
  H2_HIP(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, st));
  C.apply(z, r.as<double>(), -1.0, refine ? outer_flags : 0);
  rel = C.nrm(r.as<double>()) / nb;
  info.iterations = total;
  info.outer = std::max(outer, 1);
  info.rel_residual = rel;
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return rel <= p.rtol ? H2_OK : H2_ENOTCONV;
}

}  // namespace h2

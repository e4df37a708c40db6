// Batched Krylov vector kernels for many independent right-hand sides:
//   dots:   h[r][i] = sum_k conj(Q[r][i][k]) w[r][k]     (Gram-Schmidt coefficients)
//   update: w[r][k] += sign * sum_i h[r][i] Q[r][i][k]    (Gram-Schmidt / solution update)
// Real (FP64) or complex (interleaved FP64) data.  One workgroup per (r, i)
// computes a dot product with a fixed-order reduction inside the workgroup, so
// results are reproducible, no scratch memory is needed and no workgroup waits
// for another.
#include <hip/hip_runtime.h>

#include "handle.h"

namespace h2 {
namespace {

// One 1024-thread workgroup per (r, i): every thread keeps KU independent loads of
// q and w in flight (a dot product of one long pair of rows is latency-bound when
// few outputs are asked for, e.g. the norms of a handful of right-hand sides),
// then a fixed-order reduction: butterfly within each wave, the 16 wave sums added
// in wave order by one thread.
constexpr int KB = 1024, KU = 8;

template <bool CX>
__global__ __launch_bounds__(KB) void kdots(int nvec, int64_t n, const double* __restrict__ Q, int64_t qr,
                                            int64_t qv, const double* __restrict__ W, int64_t wr,
                                            double* __restrict__ h) {
  __shared__ double red[2][KB / 64];
  const int r = blockIdx.x / nvec, i = blockIdx.x % nvec;
  const int cw = CX ? 2 : 1;
  const double* q = Q + (static_cast<int64_t>(r) * qr + static_cast<int64_t>(i) * qv) * cw;
  const double* w = W + static_cast<int64_t>(r) * wr * cw;
  double sr = 0.0, si = 0.0;
  int64_t k = threadIdx.x;
  for (; k + static_cast<int64_t>(KU - 1) * KB < n; k += static_cast<int64_t>(KU) * KB) {
    double a[KU], b[KU], c[KU], d[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t e = k + static_cast<int64_t>(u) * KB;
      a[u] = q[cw * e];
      c[u] = w[cw * e];
      if (CX) {
        b[u] = q[2 * e + 1];
        d[u] = w[2 * e + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (CX) {
        sr += a[u] * c[u] + b[u] * d[u];
        si += a[u] * d[u] - b[u] * c[u];
      } else {
        sr += a[u] * c[u];
      }
    }
  }
  for (; k < n; k += KB) {
    if (CX) {
      const double a = q[2 * k], b = q[2 * k + 1], c = w[2 * k], d = w[2 * k + 1];
      sr += a * c + b * d;
      si += a * d - b * c;
    } else {
      sr += q[k] * w[k];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    if (CX) si += __shfl_xor(si, o);
  }
  const int wave = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
    red[0][wave] = sr;
    red[1][wave] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, ti = 0.0;
    for (int v = 0; v < KB / 64; ++v) {
      tr += red[0][v];
      ti += red[1][v];
    }
    if (CX) {
      h[2 * (static_cast<int64_t>(r) * nvec + i)] = tr;
      h[2 * (static_cast<int64_t>(r) * nvec + i) + 1] = ti;
    } else {
      h[static_cast<int64_t>(r) * nvec + i] = tr;
    }
  }
}

template <bool CX>
__global__ __launch_bounds__(256) void kupdate(int nrhs, int nvec, int64_t n, const double* __restrict__ Q, int64_t qr,
                                               int64_t qv, const double* __restrict__ h, double sign,
                                               double* __restrict__ W, int64_t wr) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t r = e / n, k = e % n;
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < nvec; ++i) {
    const int64_t qo = r * qr + static_cast<int64_t>(i) * qv + k;
    if (CX) {
      const double hr = h[2 * (r * nvec + i)], hi = h[2 * (r * nvec + i) + 1];
      const double a = Q[2 * qo], b = Q[2 * qo + 1];
      sr += hr * a - hi * b;
      si += hr * b + hi * a;
    } else {
      sr += h[r * nvec + i] * Q[qo];
    }
  }
  if (CX) {
    W[2 * (r * wr + k)] += sign * sr;
    W[2 * (r * wr + k) + 1] += sign * si;
  } else {
    W[r * wr + k] += sign * sr;
  }
}

void check_args(int dtype, int nrhs, int nvec, int64_t n, const void* Q, const void* W, const void* h) {
  if (dtype != H2_R64 && dtype != H2_C128) throw Error(H2_EINVAL, "dtype must be H2_R64 or H2_C128");
  if (nrhs < 0 || nvec < 0 || n < 0) throw Error(H2_EINVAL, "negative size");
  if (static_cast<int64_t>(nrhs) * nvec > 0x7fffffff) throw Error(H2_EINVAL, "too many products");
  if (nrhs > 0 && nvec > 0 && n > 0 && (!Q || !W || !h)) throw Error(H2_EINVAL, "NULL pointer");
}

}  // namespace

void krylov_dots(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t qr, int64_t qv, const void* W,
                 int64_t wr, void* h, hipStream_t st) {
  check_args(dtype, nrhs, nvec, n, Q, W, h);
  if (nrhs == 0 || nvec == 0) return;
  const unsigned grid = static_cast<unsigned>(nrhs * nvec);
  if (dtype == H2_C128)
    kdots<true><<<grid, KB, 0, st>>>(nvec, n, static_cast<const double*>(Q), qr, qv, static_cast<const double*>(W),
                                      wr, static_cast<double*>(h));
  else
    kdots<false><<<grid, KB, 0, st>>>(nvec, n, static_cast<const double*>(Q), qr, qv, static_cast<const double*>(W),
                                       wr, static_cast<double*>(h));
  H2_HIP(hipGetLastError());
}

void krylov_update(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t qr, int64_t qv, const void* h,
                   double sign, void* W, int64_t wr, hipStream_t st) {
  check_args(dtype, nrhs, nvec, n, Q, W, h);
  if (nrhs == 0 || n == 0) return;
  const int64_t work = n * nrhs;
  const int64_t g = (work + 255) / 256;
  if (g > 0x7fffffff) throw Error(H2_EINVAL, "launch too large");
  if (dtype == H2_C128)
    kupdate<true><<<static_cast<unsigned>(g), 256, 0, st>>>(nrhs, nvec, n, static_cast<const double*>(Q), qr, qv,
                                                           static_cast<const double*>(h), sign,
                                                           static_cast<double*>(W), wr);
  else
    kupdate<false><<<static_cast<unsigned>(g), 256, 0, st>>>(nrhs, nvec, n, static_cast<const double*>(Q), qr, qv,
                                                            static_cast<const double*>(h), sign,
                                                            static_cast<double*>(W), wr);
  H2_HIP(hipGetLastError());
}

}  // namespace h2

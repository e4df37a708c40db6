// The H^2 matrix-vector product y <- y + alpha G~ x on the GPU.
//
// Phases (Section "H^2-matrices", three-phase product; Algorithms 1-3):
//   permute-in      x_c[p] = x[perm[p]]  (each cluster is a contiguous range)
//   leaf forward    x^_sigma = V_sigma^T x|sigma for every leaf        (Alg. 1)
//   transfer up     x^_sigma = sum_children F_sigma'^T x^_sigma', level by level,
//                   deepest first                                      (Alg. 1)
//   coupling        y^_tau = sum_{(tau,sigma) admissible} S x^_sigma    (Alg. 3)
//                   (assigns, so y^ := 0 is part of this phase)
//   transfer down   y^_tau' += E_tau' y^_tau, level by level, root first (Alg. 2)
//   near + backward y_c|tau = sum_{(tau,sigma) inadmissible} G|tau x sigma x|sigma
//                   + V_tau y^_tau for every leaf                   (Alg. 3 and 2)
//   permute-out     y[perm[p]] += alpha y_c[p]
// Every output element is written by exactly one thread: no atomics, and the
// result is bitwise reproducible from call to call.
//
// Layouts: S blocks k x k row-major, CSR by row cluster; F (= E) row nu' and
// its transpose ET per cluster; Vf = V row-major [position][nu]; Vb = V per leaf
// column-major [nu][row]; the near field of row leaf tau is one column-major
// panel |tau| x (sum |sigma|), blocks in column-cluster order.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "handle.h"
#include "otf_math.h"

namespace h2 {
namespace {

// ---------------------------------------------------------------- element access
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

template <typename ST, typename AT>
__device__ inline AT ld(const ST* p);
template <>
__device__ inline double ld<double, double>(const double* p) { return *p; }
template <>
__device__ inline float ld<float, float>(const float* p) { return *p; }
template <>
__device__ inline double ld<float, double>(const float* p) { return static_cast<double>(*p); }

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// 16-byte vector of storage elements converted to AT (non-temporal: streamed once)
template <typename ST>
struct Vec16;
template <>
struct Vec16<double> {
  static constexpr int N = 2;
  template <typename AT>
  __device__ static inline void load(const double* p, AT* out) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    out[0] = v.x;
    out[1] = v.y;
  }
};
template <>
struct Vec16<float> {
  static constexpr int N = 4;
  template <typename AT>
  __device__ static inline void load(const float* p, AT* out) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  }
};
template <>
struct Vec16<bf16> {
  static constexpr int N = 8;
  template <typename AT>
  __device__ static inline void load(const bf16* p, AT* out) {
    const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p));
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      out[2 * i] = __uint_as_float(w[i] << 16);
      out[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  }
};

// ---------------------------------------------------------------- permutations
template <typename XT, typename AT>
__global__ void permute_in(int64_t n, const int32_t* __restrict__ perm, const XT* __restrict__ x,
                           AT* __restrict__ xc) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) xc[p] = static_cast<AT>(x[perm[p]]);
}

template <typename XT, typename AT>
__global__ void permute_out(int64_t n, const int32_t* __restrict__ perm, const AT* __restrict__ yc, XT* __restrict__ y,
                            double alpha, bool ow) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) {
    const int32_t t = perm[p];
    const double y0 = ow ? 0.0 : static_cast<double>(y[t]);
    y[t] = static_cast<XT>(y0 + alpha * static_cast<double>(yc[p]));
  }
}

// ---------------------------------------------------------------- wave broadcast
// value of lane `j` (wave-uniform) to every lane
__device__ inline float bcast(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ inline double bcast(double v, int j) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffff), j);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), j);
  return __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}

// acc += sum_{j < cnt} A[j * stride] * (value of xv in lane j) for cnt <= 64, with
// xv zero in lanes cnt..63.  G loads in flight (G divides 64); the last group
// re-reads column cnt - 1 in place of the columns past cnt, whose x is zero, so
// every group issues all of its loads before the first multiply
template <typename ST, typename AT, int G = 8>
__device__ inline AT stream_dot(const ST* __restrict__ A, int64_t stride, int cnt, AT xv, AT acc) {
  static_assert(64 % G == 0, "groups tile the 64 lanes");
  for (int j = 0; j < cnt; j += G) {
    AT a[G];
#pragma unroll
    for (int u = 0; u < G; ++u) a[u] = ld<ST, AT>(A + min(j + u, cnt - 1) * stride);
#pragma unroll
    for (int u = 0; u < G; ++u) acc += a[u] * bcast(xv, j + u);
  }
  return acc;
}

// ---------------------------------------------------------------- leaf forward
// one wave per leaf, lane = nu (chunks of 64 for k > 64); x|sigma staged one
// value per lane and broadcast
template <typename ST, typename AT>
__global__ __launch_bounds__(256) void leaf_forward(int nleaves, int k, const int32_t* __restrict__ leaves,
                                                    const int32_t* __restrict__ cbegin,
                                                    const int32_t* __restrict__ cend, const ST* __restrict__ Vf,
                                                    const AT* __restrict__ xc, AT* __restrict__ xhat) {
  const int l = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (l >= nleaves) return;
  const int32_t c = leaves[l];
  const int64_t b0 = cbegin[c];
  const int r = cend[c] - cbegin[c];
  for (int nu0 = 0; nu0 < k; nu0 += 64) {
    const int nu = nu0 + lane;
    const int nus = nu < k ? nu : 0;
    AT acc = 0;
    for (int p0 = 0; p0 < r; p0 += 64) {
      const AT xv = p0 + lane < r ? xc[b0 + p0 + lane] : AT(0);
      acc = stream_dot<ST, AT>(Vf + (b0 + p0) * k + nus, k, min(64, r - p0), xv, acc);
    }
    if (nu < k) xhat[static_cast<int64_t>(c) * k + nu] = acc;
  }
}

// ---------------------------------------------------------------- transfers
// One wave per cluster.  Dense transfers (any k): lane = parent index nu (up) or
// child index nu' (down), the matrix read as coalesced rows (F and its transpose
// ET are both stored).
template <typename ST, typename AT>
__device__ inline void up_dense(int32_t c, int k, int lane, const int32_t* __restrict__ child0,
                                const int32_t* __restrict__ child1, const ST* __restrict__ F, AT* __restrict__ xhat) {
  const int32_t ch[2] = {child0[c], child1[c]};
  const int64_t kk = static_cast<int64_t>(k) * k;
  for (int nu0 = 0; nu0 < k; nu0 += 64) {
    const int nu = nu0 + lane;
    const int nus = nu < k ? nu : 0;
    AT acc = 0;
    for (int a = 0; a < 2; ++a) {
      const AT* xs = xhat + static_cast<int64_t>(ch[a]) * k;
      for (int q0 = 0; q0 < k; q0 += 64) {
        const AT xv = q0 + lane < k ? xs[q0 + lane] : AT(0);
        acc = stream_dot<ST, AT>(F + ch[a] * kk + static_cast<int64_t>(q0) * k + nus, k, min(64, k - q0), xv, acc);
      }
    }
    if (nu < k) xhat[static_cast<int64_t>(c) * k + nu] = acc;
  }
}

template <typename ST, typename AT>
__device__ inline void down_dense(int32_t c, int k, int lane, const int32_t* __restrict__ parent,
                                  const ST* __restrict__ ET, AT* __restrict__ yhat) {
  const int64_t kk = static_cast<int64_t>(k) * k;
  const AT* yp = yhat + static_cast<int64_t>(parent[c]) * k;
  for (int n0 = 0; n0 < k; n0 += 64) {
    const int nup = n0 + lane;
    const int nus = nup < k ? nup : 0;
    AT acc = 0;
    for (int q0 = 0; q0 < k; q0 += 64) {
      const AT yv = q0 + lane < k ? yp[q0 + lane] : AT(0);
      acc = stream_dot<ST, AT>(ET + c * kk + static_cast<int64_t>(q0) * k + nus, k, min(64, k - q0), yv, acc);
    }
    if (nup < k) yhat[static_cast<int64_t>(c) * k + nup] += acc;
  }
}

// k = 64 (m = 4): E_c = E_x (x) E_y (x) E_z, applied one axis at a time.  One
// wave per cluster, lane = nu = nu_x + 4 nu_y + 16 nu_z; each axis step
// contracts four lanes that differ only in that axis (lane shuffles), so a
// transfer reads 48 numbers instead of 4096.  E1 holds E1[c][d][i][j] =
// l_j(xi_i) along axis d (i child point, j parent polynomial).
template <typename ST, typename AT>
__device__ inline AT kron_axis(AT t, const ST* __restrict__ e, int lane, int shift, bool transpose) {
  const int own = (lane >> shift) & 3;
  const int base = lane & ~(3 << shift);
  AT r = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const AT v = __shfl(t, base | (i << shift));
    // up (transpose): sum over child points i of E[i][own]; down: sum over parent polynomials i of E[own][i]
    r += ld<ST, AT>(e + (transpose ? i * 4 + own : own * 4 + i)) * v;
  }
  return r;
}

// up: x^_c = sum over the two children a of E_a^T x^_a (Algorithm 1)
template <typename ST, typename AT>
__device__ inline void up_kron(int32_t c, int lane, const int32_t* __restrict__ child0,
                               const int32_t* __restrict__ child1, const ST* __restrict__ E1, AT* __restrict__ xhat) {
  const int32_t ch[2] = {child0[c], child1[c]};
  AT acc = 0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const ST* e = E1 + static_cast<int64_t>(ch[a]) * 48;
    AT t = xhat[static_cast<int64_t>(ch[a]) * 64 + lane];
    t = kron_axis<ST, AT>(t, e, lane, 0, true);
    t = kron_axis<ST, AT>(t, e + 16, lane, 2, true);
    t = kron_axis<ST, AT>(t, e + 32, lane, 4, true);
    acc += t;
  }
  xhat[static_cast<int64_t>(c) * 64 + lane] = acc;
}

// down: y^_c += E_c y^_parent(c) (Algorithm 2)
template <typename ST, typename AT>
__device__ inline void down_kron(int32_t c, int lane, const int32_t* __restrict__ parent, const ST* __restrict__ E1,
                                 AT* __restrict__ yhat) {
  const ST* e = E1 + static_cast<int64_t>(c) * 48;
  AT t = yhat[static_cast<int64_t>(parent[c]) * 64 + lane];
  t = kron_axis<ST, AT>(t, e, lane, 0, false);
  t = kron_axis<ST, AT>(t, e + 16, lane, 2, false);
  t = kron_axis<ST, AT>(t, e + 32, lane, 4, false);
  yhat[static_cast<int64_t>(c) * 64 + lane] += t;
}

// one level: one wave per cluster (E: E1 for the Kronecker form, else F / ET)
template <typename ST, typename AT, bool KRON>
__global__ __launch_bounds__(256) void transfer_up(int count, int k, const int32_t* __restrict__ list,
                                                   const int32_t* __restrict__ child0,
                                                   const int32_t* __restrict__ child1, const ST* __restrict__ E,
                                                   AT* __restrict__ xhat) {
  const int w = blockIdx.x * 4 + threadIdx.x / 64;
  if (w >= count) return;
  if (KRON) up_kron<ST, AT>(list[w], threadIdx.x % 64, child0, child1, E, xhat);
  else up_dense<ST, AT>(list[w], k, threadIdx.x % 64, child0, child1, E, xhat);
}

template <typename ST, typename AT, bool KRON>
__global__ __launch_bounds__(256) void transfer_down(int first, int count, int k, const int32_t* __restrict__ parent,
                                                     const ST* __restrict__ E, AT* __restrict__ yhat) {
  const int w = blockIdx.x * 4 + threadIdx.x / 64;
  if (w >= count) return;
  if (KRON) down_kron<ST, AT>(first + w, threadIdx.x % 64, parent, E, yhat);
  else down_dense<ST, AT>(first + w, k, threadIdx.x % 64, parent, E, yhat);
}

// The top levels, which hold few clusters each, in one workgroup of 16 waves:
// level by level (deepest first going up, root first going down), a workgroup
// barrier between levels (a level reads what the previous one wrote), so their
// dependent launches become one.  lev: the levels' offsets into list (up), or the
// cluster offsets of the levels (down).
constexpr int kTopWaves = 16;

template <typename ST, typename AT, bool KRON>
__global__ __launch_bounds__(64 * kTopWaves) void transfer_up_top(int nlev, const int64_t* __restrict__ lev, int k,
                                                                  const int32_t* __restrict__ list,
                                                                  const int32_t* __restrict__ child0,
                                                                  const int32_t* __restrict__ child1,
                                                                  const ST* __restrict__ E, AT* __restrict__ xhat) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int l = nlev - 1; l >= 0; --l) {
    for (int64_t w = lev[l] + wave; w < lev[l + 1]; w += kTopWaves) {
      if (KRON) up_kron<ST, AT>(list[w], lane, child0, child1, E, xhat);
      else up_dense<ST, AT>(list[w], k, lane, child0, child1, E, xhat);
    }
    __syncthreads();
  }
}

template <typename ST, typename AT, bool KRON>
__global__ __launch_bounds__(64 * kTopWaves) void transfer_down_top(int nlev, const int32_t* __restrict__ level_ptr,
                                                                    int k, const int32_t* __restrict__ parent,
                                                                    const ST* __restrict__ E, AT* __restrict__ yhat) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int l = 0; l < nlev; ++l) {
    for (int32_t c = level_ptr[l + 1] + wave; c < level_ptr[l + 2]; c += kTopWaves) {
      if (KRON) down_kron<ST, AT>(c, lane, parent, E, yhat);
      else down_dense<ST, AT>(c, k, lane, parent, E, yhat);
    }
    __syncthreads();
  }
}

// the transfer phases of one product: Kronecker form for k = 64, dense otherwise
template <typename ST, typename AT>
void launch_up(h2_handle_s& H, AT* xh, hipStream_t st);
template <typename ST, typename AT>
void launch_down(h2_handle_s& H, AT* yh, hipStream_t st);

// ---------------------------------------------------------------- coupling
// k = 64 fast path: one 256-thread workgroup per row cluster; each thread reads
// 16-byte vectors of S (lanes_per_row lanes cover one row of a block) and keeps
// its partial row sums in registers across all blocks of the row; one shuffle
// reduction at the end.
template <typename SST, typename AT>
__global__ __launch_bounds__(256) void coupling64(int nc, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const SST* __restrict__ S,
                                                  const AT* __restrict__ xhat, AT* __restrict__ yhat) {
  constexpr int VEC = Vec16<SST>::N;
  constexpr int LPR = 64 / VEC;
  constexpr int RPP = 256 / LPR;
  constexpr int NP = 64 / RPP;
  const int tau = blockIdx.x;
  if (tau >= nc) return;
  const int t = threadIdx.x;
  const int lr = t % LPR, r0 = t / LPR;
  AT acc[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) acc[j] = 0;
  const int64_t b1 = ptr[tau + 1];
  for (int64_t b = ptr[tau]; b < b1; ++b) {
    const int64_t s = col[b];
    AT xv[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) xv[v] = xhat[s * 64 + lr * VEC + v];
    const SST* Sb = S + b * 4096 + lr * VEC;
    AT sv[NP][VEC];
#pragma unroll
    for (int j = 0; j < NP; ++j) Vec16<SST>::load(Sb + (r0 + j * RPP) * 64, sv[j]);
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[j] += sv[j][v] * xv[v];
  }
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) acc[j] += __shfl_xor(acc[j], off);
  if (lr == 0) {
#pragma unroll
    for (int j = 0; j < NP; ++j) yhat[static_cast<int64_t>(tau) * 64 + r0 + j * RPP] = acc[j];
  }
}

// Symmetric storage (G~ = G~^T, so S_{sigma tau} = S_{tau sigma}^T): only the
// blocks (tau, sigma) with sigma > tau are kept, and each one is used twice:
// y^_tau += S x^_sigma (row sums) and S^T x^_tau (column sums), the latter into
// the block's scratch slot, which adm_gather adds to y^_sigma afterwards in a
// fixed order.  One workgroup per row cluster; wave w takes the kept blocks
// w, w + 4, ... of the row and reads each with 16-byte loads: a lane owns VEC
// consecutive columns of NR rows, so its row sums carry across the wave's
// blocks and a block's column sums need one reduction over RPI lanes.
template <typename SST, typename AT>
__global__ __launch_bounds__(256) void coupling64_sym(int nc, const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ col, const SST* __restrict__ S,
                                                      const AT* __restrict__ xhat, AT* __restrict__ yhat,
                                                      AT* __restrict__ scratch) {
  constexpr int VEC = Vec16<SST>::N;  // columns per lane
  constexpr int LPR = 64 / VEC;       // lanes per block row
  constexpr int RPI = 64 / LPR;       // rows per load instruction
  constexpr int NR = 64 / RPI;        // rows per lane
  constexpr int CH = NR < 8 ? NR : 8; // loads in flight
  __shared__ AT part[3][64];
  const int tau = blockIdx.x;
  if (tau >= nc) return;
  const int lane = threadIdx.x % 64;
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lr = lane % LPR, r0 = lane / LPR;
  AT xt[NR], acc[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    xt[j] = xhat[static_cast<int64_t>(tau) * 64 + r0 + RPI * j];
    acc[j] = 0;
  }
  const int64_t b1 = ptr[tau + 1];
  for (int64_t b = ptr[tau] + w; b < b1; b += 4) {
    const int64_t s = col[b];
    AT xs[VEC], cp[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      xs[v] = xhat[s * 64 + lr * VEC + v];
      cp[v] = 0;
    }
    const SST* Sb = S + b * 4096 + lr * VEC;
#pragma unroll
    for (int j0 = 0; j0 < NR; j0 += CH) {
      AT sv[CH][VEC];
#pragma unroll
      for (int u = 0; u < CH; ++u) Vec16<SST>::load(Sb + (r0 + RPI * (j0 + u)) * 64, sv[u]);
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          acc[j0 + u] += sv[u][v] * xs[v];
          cp[v] += sv[u][v] * xt[j0 + u];
        }
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v)
#pragma unroll
      for (int off = LPR; off < 64; off <<= 1) cp[v] += __shfl_xor(cp[v], off);
    if (r0 == 0) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) scratch[b * 64 + lr * VEC + v] = cp[v];
    }
  }
#pragma unroll
  for (int j = 0; j < NR; ++j)
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) acc[j] += __shfl_xor(acc[j], off);
  if (w > 0 && lr == 0) {
#pragma unroll
    for (int j = 0; j < NR; ++j) part[w - 1][r0 + RPI * j] = acc[j];
  }
  __syncthreads();
  if (w == 0 && lr == 0) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int row = r0 + RPI * j;
      yhat[static_cast<int64_t>(tau) * 64 + row] = ((acc[j] + part[0][row]) + part[1][row]) + part[2][row];
    }
  }
}

// y^_c += the transposed parts of the kept blocks (tau, c), in increasing tau
template <typename AT>
__global__ __launch_bounds__(256) void adm_gather(int nc, const int64_t* __restrict__ in_ptr,
                                                  const int64_t* __restrict__ in_blk, const AT* __restrict__ scratch,
                                                  AT* __restrict__ yhat) {
  const int c = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (c >= nc) return;
  const int64_t i0 = in_ptr[c], i1 = in_ptr[c + 1];
  if (i0 == i1) return;
  AT s = 0;
  for (int64_t i = i0; i < i1; ++i) s += scratch[in_blk[i] * 64 + lane];
  yhat[static_cast<int64_t>(c) * 64 + lane] += s;
}

// any k: one thread per row nu of the block row
template <typename SST, typename AT>
__device__ inline AT lds(const SST* p);
template <>
__device__ inline double lds<double, double>(const double* p) { return *p; }
template <>
__device__ inline float lds<float, float>(const float* p) { return *p; }
template <>
__device__ inline double lds<float, double>(const float* p) { return *p; }
template <>
__device__ inline float lds<bf16, float>(const bf16* p) { return bf2f(p->v); }
template <>
__device__ inline double lds<bf16, double>(const bf16* p) { return bf2f(p->v); }

template <typename SST, typename AT>
__global__ __launch_bounds__(256) void coupling_any(int nc, int k, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col, const SST* __restrict__ S,
                                                   const AT* __restrict__ xhat, AT* __restrict__ yhat) {
  const int tau = blockIdx.x;
  if (tau >= nc) return;
  const int64_t kk = static_cast<int64_t>(k) * k;
  for (int nu = threadIdx.x; nu < k; nu += blockDim.x) {
    AT acc = 0;
    for (int64_t b = ptr[tau]; b < ptr[tau + 1]; ++b) {
      const SST* Sb = S + b * kk + static_cast<int64_t>(nu) * k;
      const AT* xs = xhat + static_cast<int64_t>(col[b]) * k;
      for (int mu = 0; mu < k; ++mu) acc += lds<SST, AT>(Sb + mu) * xs[mu];
    }
    yhat[static_cast<int64_t>(tau) * k + nu] = acc;
  }
}

// Small k (recompressed bases, k <= RB <= 32): one wave per row cluster; the 64
// lanes form 64 / RB slots of RB lanes, slot j takes the blocks ptr + j,
// ptr + j + 64 / RB, ...; lane nu of a slot owns row nu of its block and issues
// the whole row's loads at once (indices clamped to the last column, surplus
// terms masked).  The slots' row sums are added by lane shuffles.
// FP32 S with k a multiple of 4 (V4): rows are read as 16-byte vectors.
template <int RB, typename SST, typename AT>
__device__ inline AT row_dot_small(const SST* __restrict__ Sb, const AT* __restrict__ xs, int k) {
  AT a[RB], xv[RB];
#pragma unroll
  for (int mu = 0; mu < RB; ++mu) {
    const int mc = min(mu, k - 1);
    a[mu] = lds<SST, AT>(Sb + mc);
    xv[mu] = xs[mc];
  }
  AT acc = 0;
#pragma unroll
  for (int mu = 0; mu < RB; ++mu) acc += mu < k ? a[mu] * xv[mu] : AT(0);
  return acc;
}

template <int RB>
__device__ inline float row_dot_small_v4(const float* __restrict__ Sb, const float* __restrict__ xs, int k) {
  f4v a[RB / 4], xv[RB / 4];
#pragma unroll
  for (int q = 0; q < RB / 4; ++q) {
    const int qc = min(q, k / 4 - 1);
    a[q] = *reinterpret_cast<const f4v*>(Sb + 4 * qc);
    xv[q] = *reinterpret_cast<const f4v*>(xs + 4 * qc);
  }
  float acc = 0.f;
#pragma unroll
  for (int q = 0; q < RB / 4; ++q)
    if (4 * q < k) acc += ((a[q].x * xv[q].x + a[q].y * xv[q].y) + a[q].z * xv[q].z) + a[q].w * xv[q].w;
  return acc;
}

template <int RB, bool V4, typename SST, typename AT>
__global__ __launch_bounds__(256) void coupling_small(int nc, int k, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col, const SST* __restrict__ S,
                                                     const AT* __restrict__ xhat, AT* __restrict__ yhat) {
  const int64_t tau = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / 64;
  if (tau >= nc) return;  // uniform per wave
  constexpr int NS = 64 / RB;
  const int lane = threadIdx.x % 64, nu = lane % RB, slot = lane / RB;
  const int64_t kk = static_cast<int64_t>(k) * k;
  const int nur = min(nu, k - 1);
  AT acc = 0;
  const int64_t b1 = ptr[tau + 1];
  for (int64_t b = ptr[tau] + slot; b < b1; b += NS) {
    const SST* Sb = S + b * kk + static_cast<int64_t>(nur) * k;
    const AT* xs = xhat + static_cast<int64_t>(col[b]) * k;
    if constexpr (V4) acc += row_dot_small_v4<RB>(Sb, xs, k);
    else acc += row_dot_small<RB, SST, AT>(Sb, xs, k);
  }
#pragma unroll
  for (int o = RB; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
  if (slot == 0 && nu < k) yhat[tau * k + nu] = acc;
}

// ---------------------------------------------------------------- coupling evaluated on the fly
// s_{nu mu} = g(xi_{tau,nu}, xi_{sigma,mu}) (eq. coupling) from the tensor
// Chebyshev points: xi - eta = (c_tau - c_sigma) + (o_tau - o_sigma) per axis,
// with the centre difference formed in FP64 and the small offsets o in the
// evaluation precision ET, so the difference keeps ET's relative accuracy even
// for clusters far from the origin.
__device__ inline float rsq(float v) { return __frsqrt_rn(v); }
__device__ inline double rsq(double v) { return rsqrt(v); }

template <int KIND, typename ET>
__device__ inline ET otf_g(ET dx, ET dy, ET dz, ET x0, ET x1, ET x2, ET y0, ET y1, ET y2) {
  if (KIND == H2_LAPLACE) return rsq(dx * dx + dy * dy + dz * dz);  // times 1/(4 pi) at the end
  if (KIND == H2_TEST_ONE) return ET(1);
  const ET d = x0 * y0 + x1 * y1 + x2 * y2;
  if (KIND == H2_TEST_BILINEAR) return d;
  return d * d;
}

// k = 64 (m = 4): one 256-thread workgroup per row cluster tau, rows taken
// heaviest first (spans): the kernel is bound by its arithmetic, not by HBM, so
// the launch ends when the last rows do, and heavy rows started last set that end
// (0.896 -> 0.854 ms at 1,310,720 triangles; for the stored coupling and the near
// field, which stream from HBM, tree order is as fast or faster).  Wave w takes
// the row's blocks w, w + 4, ...; lane nu owns row nu and all 64 columns of
// each of its blocks.  What depends on the column cluster only (its centre, its
// 12 point offsets, x^_sigma) is the same for the whole wave and is read with
// wave-uniform loads; per entry a lane then needs one add, one reciprocal
// square root and one FMA.  The four wave partials are summed through LDS in a
// fixed order, so the result is reproducible.
template <int KIND, typename ET, typename AT>
__global__ __launch_bounds__(256) void coupling64_otf(int nc, const RowSpan* __restrict__ spans,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ ctr, const ET* __restrict__ off,
                                                      const AT* __restrict__ xhat, AT* __restrict__ yhat) {
  __shared__ AT part[3][64];
  if (static_cast<int>(blockIdx.x) >= nc) return;
  const RowSpan sp = spans[blockIdx.x];  // rows heaviest first
  const int tau = sp.tau;
  const int nu = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const ET* ot = off + static_cast<int64_t>(tau) * 12;
  const ET ax = ot[nu & 3], ay = ot[4 + ((nu >> 2) & 3)], az = ot[8 + (nu >> 4)];
  const double cx = ctr[3 * tau], cy = ctr[3 * tau + 1], cz = ctr[3 * tau + 2];
  AT acc = 0;
  const int64_t b1 = sp.b0 + sp.nb;
  for (int64_t b = sp.b0 + w; b < b1; b += 4) {
    const int64_t s = col[b];
    const ET* os = off + s * 12;
    const AT* xs = xhat + s * 64;
    if (KIND == H2_LAPLACE) {
      const ET ex = static_cast<ET>(cx - ctr[3 * s]) + ax, ey = static_cast<ET>(cy - ctr[3 * s + 1]) + ay,
               ez = static_cast<ET>(cz - ctr[3 * s + 2]) + az;
      ET dx2[4], dy2[4], dz2[4], dyz[16];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const ET dx = ex - os[i], dy = ey - os[4 + i], dz = ez - os[8 + i];
        dx2[i] = dx * dx;
        dy2[i] = dy * dy;
        dz2[i] = dz * dz;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) dyz[i] = dy2[i & 3] + dz2[i >> 2];
#pragma unroll
      for (int j = 0; j < 64; ++j) acc += static_cast<AT>(rsq(dx2[j & 3] + dyz[j >> 2])) * xs[j];
    } else {
      // polynomial test kernels on absolute coordinates
      const ET x0 = static_cast<ET>(cx) + ax, x1 = static_cast<ET>(cy) + ay, x2 = static_cast<ET>(cz) + az;
      ET px[4], pyz[16], py[4], pz[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        px[i] = x0 * (static_cast<ET>(ctr[3 * s]) + os[i]);
        py[i] = x1 * (static_cast<ET>(ctr[3 * s + 1]) + os[4 + i]);
        pz[i] = x2 * (static_cast<ET>(ctr[3 * s + 2]) + os[8 + i]);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) pyz[i] = py[i & 3] + pz[i >> 2];
#pragma unroll
      for (int j = 0; j < 64; ++j) {
        const ET d = px[j & 3] + pyz[j >> 2];
        const ET g = KIND == H2_TEST_ONE ? ET(1) : KIND == H2_TEST_BILINEAR ? d : d * d;
        acc += static_cast<AT>(g) * xs[j];
      }
    }
  }
  if (w > 0) part[w - 1][nu] = acc;
  __syncthreads();
  if (w == 0) {
    acc = ((acc + part[0][nu]) + part[1][nu]) + part[2][nu];
    const AT scale = KIND == H2_LAPLACE ? AT(1.0 / (4.0 * 3.14159265358979323846)) : AT(1);
    yhat[static_cast<int64_t>(tau) * 64 + nu] = acc * scale;
  }
}

// Helmholtz, k = 64, FP32 evaluation: as coupling64_otf with g = e^{i kappa r} / r
// (times 1/(4 pi) at the end); per entry the squared distance, one reciprocal
// square root, r, the sine and cosine of kappa r, and one complex multiply-add
// with the wave-uniform x^_sigma (two planes).
template <typename AT>
__global__ __launch_bounds__(256) void coupling64c_otf(int nc, float kappa, const RowSpan* __restrict__ spans,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ ctr, const float* __restrict__ off,
                                                       const AT* __restrict__ xhr, const AT* __restrict__ xhi,
                                                       AT* __restrict__ yhr, AT* __restrict__ yhi) {
  __shared__ AT part[2][3][64];
  if (static_cast<int>(blockIdx.x) >= nc) return;
  const RowSpan sp = spans[blockIdx.x];  // rows heaviest first, as coupling64_otf
  const int tau = sp.tau;
  const int nu = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const float* ot = off + static_cast<int64_t>(tau) * 12;
  const float ax = ot[nu & 3], ay = ot[4 + ((nu >> 2) & 3)], az = ot[8 + (nu >> 4)];
  const double cx = ctr[3 * tau], cy = ctr[3 * tau + 1], cz = ctr[3 * tau + 2];
  AT ar = 0, ai = 0;
  const int64_t b1 = sp.b0 + sp.nb;
  for (int64_t b = sp.b0 + w; b < b1; b += 4) {
    const int64_t s = col[b];
    const float* os = off + s * 12;
    const AT* xr = xhr + s * 64;
    const AT* xi = xhi + s * 64;
    const float ex = static_cast<float>(cx - ctr[3 * s]) + ax, ey = static_cast<float>(cy - ctr[3 * s + 1]) + ay,
                ez = static_cast<float>(cz - ctr[3 * s + 2]) + az;
    float dx2[4], dy2[4], dz2[4], dyz[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float dx = ex - os[i], dy = ey - os[4 + i], dz = ez - os[8 + i];
      dx2[i] = dx * dx;
      dy2[i] = dy * dy;
      dz2[i] = dz * dz;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) dyz[i] = dy2[i & 3] + dz2[i >> 2];
#pragma unroll 8
    for (int j = 0; j < 64; ++j) {
      const float d2 = dx2[j & 3] + dyz[j >> 2];
      const float inv = rsq(d2);
      float sn, cs;
      sincos_phase(kappa * (d2 * inv), sn, cs);
      const AT gr = static_cast<AT>(cs * inv), gi = static_cast<AT>(sn * inv);
      ar += gr * xr[j] - gi * xi[j];
      ai += gr * xi[j] + gi * xr[j];
    }
  }
  if (w > 0) {
    part[0][w - 1][nu] = ar;
    part[1][w - 1][nu] = ai;
  }
  __syncthreads();
  if (w == 0) {
    const AT scale = AT(1.0 / (4.0 * 3.14159265358979323846));
    yhr[static_cast<int64_t>(tau) * 64 + nu] = (((ar + part[0][0][nu]) + part[0][1][nu]) + part[0][2][nu]) * scale;
    yhi[static_cast<int64_t>(tau) * 64 + nu] = (((ai + part[1][0][nu]) + part[1][1][nu]) + part[1][2][nu]) * scale;
  }
}

// any order m: one thread per row nu
template <int KIND, typename ET, typename AT>
__global__ __launch_bounds__(256) void coupling_any_otf(int nc, int m, const int64_t* __restrict__ ptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ ctr, const ET* __restrict__ off,
                                                        const AT* __restrict__ xhat, AT* __restrict__ yhat) {
  const int tau = blockIdx.x;
  if (tau >= nc) return;
  const int k = m * m * m;
  const ET* ot = off + static_cast<int64_t>(tau) * 3 * m;
  for (int nu = threadIdx.x; nu < k; nu += blockDim.x) {
    const ET ax = ot[nu % m], ay = ot[m + (nu / m) % m], az = ot[2 * m + nu / (m * m)];
    AT acc = 0;
    for (int64_t b = ptr[tau]; b < ptr[tau + 1]; ++b) {
      const int64_t s = col[b];
      const ET* os = off + s * 3 * m;
      const ET dcx = static_cast<ET>(ctr[3 * tau] - ctr[3 * s]), dcy = static_cast<ET>(ctr[3 * tau + 1] - ctr[3 * s + 1]),
               dcz = static_cast<ET>(ctr[3 * tau + 2] - ctr[3 * s + 2]);
      for (int mu = 0; mu < k; ++mu) {
        const ET ox = os[mu % m], oy = os[m + (mu / m) % m], oz = os[2 * m + mu / (m * m)];
        const ET x0 = static_cast<ET>(ctr[3 * tau]) + ax, x1 = static_cast<ET>(ctr[3 * tau + 1]) + ay,
                 x2 = static_cast<ET>(ctr[3 * tau + 2]) + az;
        const ET y0 = static_cast<ET>(ctr[3 * s]) + ox, y1 = static_cast<ET>(ctr[3 * s + 1]) + oy,
                 y2 = static_cast<ET>(ctr[3 * s + 2]) + oz;
        const ET g = otf_g<KIND, ET>((dcx + ax) - ox, (dcy + ay) - oy, (dcz + az) - oz, x0, x1, x2, y0, y1, y2);
        acc += static_cast<AT>(g) * xhat[s * k + mu];
      }
    }
    const AT scale = KIND == H2_LAPLACE ? AT(1.0 / (4.0 * 3.14159265358979323846)) : AT(1);
    yhat[static_cast<int64_t>(tau) * k + nu] = acc * scale;
  }
}

template <typename ET, typename AT>
void launch_otf(h2_handle_s& H, const AT* xh, AT* yh, hipStream_t st) {
  const Structure& S = H.S;
  const int nc = S.nclusters;
  const ET* off = static_cast<const ET*>(sizeof(ET) == 8 ? H.off64.p : H.off32.p);
  const double* ctr = H.ctr.as<double>();
  const int64_t* ptr = H.adm_ptr.as<int64_t>();
  const RowSpan* spans = H.row_spans.as<RowSpan>();
  const int32_t* col = H.adm_col.as<int32_t>();
#define H2_OTF_CASE(K)                                                                                \
  case K:                                                                                             \
    if (S.k == 64) coupling64_otf<K, ET, AT><<<nc, 256, 0, st>>>(nc, spans, col, ctr, off, xh, yh);  \
    else coupling_any_otf<K, ET, AT><<<nc, 256, 0, st>>>(nc, S.m, ptr, col, ctr, off, xh, yh);       \
    break;
  switch (H.P.kernel) {
    H2_OTF_CASE(H2_LAPLACE)
    H2_OTF_CASE(H2_TEST_ONE)
    H2_OTF_CASE(H2_TEST_BILINEAR)
    H2_OTF_CASE(H2_TEST_QUADRATIC)
    default: throw Error(H2_EINVAL, "on-the-fly coupling supports real kernels only");
  }
#undef H2_OTF_CASE
}

// ---------------------------------------------------------------- near field + leaf backward
// one 256-thread workgroup per row leaf tau; lane = row of tau.  The near blocks
// of the row are dealt round-robin to the four waves; a wave stages x|sigma one
// value per lane and streams the block's columns (each column is |tau|
// contiguous entries of the column-major panel) with 16 loads in flight.  The
// columns of V_tau (multiplied by y^_tau) are split between the waves the same
// way.  LDS sums the four partial results in a fixed order.
template <typename ST, typename AT>
__global__ __launch_bounds__(256) void near_backward(int nleaves, int k, const int32_t* __restrict__ leaves,
                                                     const int32_t* __restrict__ cbegin,
                                                     const int32_t* __restrict__ cend,
                                                     const int64_t* __restrict__ near_ptr,
                                                     const int32_t* __restrict__ near_col,
                                                     const int64_t* __restrict__ panel_off,
                                                     const ST* __restrict__ N, const ST* __restrict__ Vb,
                                                     const AT* __restrict__ xc, const AT* __restrict__ yhat,
                                                     AT* __restrict__ yc) {
  __shared__ AT part[4][64];
  const int l = blockIdx.x;
  if (l >= nleaves) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int32_t tau = leaves[l];
  const int64_t b0 = cbegin[tau];
  const int r = cend[tau] - cbegin[tau];
  const ST* P = N + panel_off[l];
  const ST* Vl = Vb + b0 * k;
  const AT* yh = yhat + static_cast<int64_t>(tau) * k;
  const int64_t bfirst = near_ptr[l], blast = near_ptr[l + 1];
  for (int i0 = 0; i0 < r; i0 += 64) {
    const int i = i0 + lane;
    const int is = i < r ? i : r - 1;  // idle lanes re-read the last row
    AT acc = 0;
    int64_t colbase = 0;
    for (int64_t bb = bfirst; bb < blast; ++bb) {
      const int32_t s = near_col[bb];
      const int64_t s0 = cbegin[s];
      const int w = cend[s] - cbegin[s];
      if (((bb - bfirst) & 3) == wave) {
        for (int j0 = 0; j0 < w; j0 += 64) {
          const AT xv = j0 + lane < w ? xc[s0 + j0 + lane] : AT(0);
          acc = stream_dot<ST, AT, 16>(P + (colbase + j0) * r + is, r, min(64, w - j0), xv, acc);
        }
      }
      colbase += w;
    }
    // leaf backward: columns nu of V_tau, a quarter per wave
    const int kq = (k + 3) / 4;
    const int n0 = wave * kq, n1 = min(k, n0 + kq);
    for (int q0 = n0; q0 < n1; q0 += 64) {
      const AT yv = q0 + lane < n1 ? yh[q0 + lane] : AT(0);
      acc = stream_dot<ST, AT, 16>(Vl + static_cast<int64_t>(q0) * r + is, r, min(64, n1 - q0), yv, acc);
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && i < r) yc[b0 + i] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    __syncthreads();
  }
}

// Leaves of at most 64 triangles and at most 256 near blocks per row: the same
// product with the column stream kept busy from the first column to the last.
// The blocks of the row go round-robin to the four waves as above; a wave holds its
// blocks' descriptors (first triangle s0 and width w of sigma, first panel column
// cb) one per lane and walks its columns in groups of G.  The G loads of the next
// group, which may open the next block, are issued before the current group is
// multiplied, so G to 2G loads of |tau| entries stay in flight.  A group that runs
// past its block's last column re-reads that column, whose x weight there is
// zero.  The leaf-backward operands (this wave's columns of V_tau and of y^_tau)
// are loaded first, so their latency overlaps the start of the stream, and each
// row's and block's descriptors are one load each.
template <typename ST, typename AT, int G>
__global__ __launch_bounds__(256) void near_backward64(int nleaves, int k, const NearRow* __restrict__ rows,
                                                       const NearBlock* __restrict__ blocks,
                                                       const ST* __restrict__ N, const ST* __restrict__ Vb,
                                                       const AT* __restrict__ xc, const AT* __restrict__ yhat,
                                                       AT* __restrict__ yc) {
  static_assert(64 % G == 0, "groups tile the 64 lanes");
  __shared__ AT part[4][64];
  const int l = blockIdx.x;
  if (l >= nleaves) return;
  const NearRow d = rows[l];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int r = d.r;
  const int is = lane < r ? lane : r - 1;  // idle lanes re-read the last row
  const int mine = d.nb > wave ? (d.nb - wave + 3) / 4 : 0;  // blocks wave, wave + 4, ...
  NearBlock e{0, 1, 0, 0};
  if (lane < mine) e = blocks[d.bfirst + wave + 4 * lane];
  // leaf backward operands: columns n0 .. n0 + nv - 1 of V_tau (a quarter per wave),
  // the first G of them held in registers until the end
  const int kq = (k + 3) / 4, n0 = wave * kq;
  const int nv = min(k, n0 + kq) - n0;  // may be <= 0 for tiny k
  const ST* Vl = Vb + static_cast<int64_t>(d.b0) * k + static_cast<int64_t>(n0) * r + is;
  const AT* yh = yhat + static_cast<int64_t>(d.tau) * k + n0;
  ST va[G];
  AT yv = 0;
  if (nv > 0) {
    yv = yh[min(lane, nv - 1)];
#pragma unroll
    for (int u = 0; u < G; ++u) va[u] = Vl[static_cast<int64_t>(min(u, nv - 1)) * r];
  }
  const ST* P = N + d.panel_off + is;
  AT acc = 0;
  if (mine > 0) {
    int m = 0, j0 = 0;  // the group issued next: block m, columns j0 .. j0 + G - 1
    int s0 = __builtin_amdgcn_readlane(e.s0, 0), w = __builtin_amdgcn_readlane(e.w, 0);
    int cb = __builtin_amdgcn_readlane(e.cb, 0);
    // stored values stay in the storage type until multiplied, so no conversion
    // waits for a load ahead of the multiplies
    auto issue = [&](ST (&a)[G], AT& xv) {
      xv = xc[s0 + min(lane, w - 1)];
      const ST* A = P + static_cast<int64_t>(cb) * r;
#pragma unroll
      for (int u = 0; u < G; ++u) a[u] = A[static_cast<int64_t>(min(j0 + u, w - 1)) * r];
    };
    auto advance = [&]() {
      j0 += G;
      if (j0 >= w) {
        j0 = 0;
        if (++m < mine) {
          s0 = __builtin_amdgcn_readlane(e.s0, m);
          w = __builtin_amdgcn_readlane(e.w, m);
          cb = __builtin_amdgcn_readlane(e.cb, m);
        }
      }
    };
    auto mul = [&](const ST (&a)[G], AT xv, int ja, int wa) {
      const AT xm = lane < wa ? xv : AT(0);
#pragma unroll
      for (int u = 0; u < G; ++u) acc += static_cast<AT>(a[u]) * bcast(xm, ja + u);
    };
    // two register sets in turn: one is multiplied while the other's loads are in
    // flight.  Past the last group the issue repeats the last block's first group
    // (cached); that group gets weight zero, which keeps its loads where they are.
    ST a[G], b[G];
    AT xa, xb;
    int ja = j0, wa = w;
    issue(a, xa);
    advance();
    for (;;) {
      const int jb = j0, wb = w;
      const bool endb = m >= mine;
      issue(b, xb);
      __builtin_amdgcn_sched_barrier(0);  // the loads go out before the multiplies
      mul(a, xa, ja, wa);
      if (endb) {
        mul(b, xb, 0, 0);
        break;
      }
      advance();
      ja = j0;
      wa = w;
      const bool enda = m >= mine;
      issue(a, xa);
      __builtin_amdgcn_sched_barrier(0);
      mul(b, xb, jb, wb);
      if (enda) {
        mul(a, xa, 0, 0);
        break;
      }
      advance();
    }
  }
  // leaf backward: y_tau += V_tau y^_tau over this wave's columns
  if (nv > 0) {
    const AT ym = lane < nv ? yv : AT(0);
#pragma unroll
    for (int u = 0; u < G; ++u) acc += static_cast<AT>(va[u]) * bcast(ym, u);
    for (int q0 = G; q0 < nv; q0 += 64) {  // k > 4 G only
      const AT y2 = q0 + lane < nv ? yh[q0 + lane] : AT(0);
      acc = stream_dot<ST, AT, 16>(Vl + static_cast<int64_t>(q0) * r, r, min(64, nv - q0), y2, acc);
    }
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && lane < r)
    yc[static_cast<int64_t>(d.b0) + lane] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// ---------------------------------------------------------------- symmetric near field
// Cross-lane moves on gfx950 without the LDS crossbar.  xor_lane<S>(v) is the
// value of lane l ^ S (S = 1, 2, 8: DPP quad permutes and a row rotation by 8 of
// the 16-lane rows; S = 4: swizzle within 32 lanes).  swap_sum<S>(a, b) for
// S = 32 / 16 exchanges the upper lane group of a with the lower group of b
// (v_permlane32_swap / v_permlane16_swap) and adds: a lane whose bit S is clear
// gets a + a[l ^ S], one whose bit S is set gets b[l ^ S] + b.
template <int S>
__device__ inline uint32_t xor_word(uint32_t v) {
  if (S == 1) return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0xb1, 0xf, 0xf, false));
  if (S == 2) return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x4e, 0xf, 0xf, false));
  if (S == 8) return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x128, 0xf, 0xf, false));
  return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(static_cast<int>(v), 0x101f));  // S == 4
}
template <int S>
__device__ inline float xor_lane(float v) { return __uint_as_float(xor_word<S>(__float_as_uint(v))); }
template <int S>
__device__ inline double xor_lane(double v) {
  const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
  const uint64_t lo = xor_word<S>(static_cast<uint32_t>(u)), hi = xor_word<S>(static_cast<uint32_t>(u >> 32));
  return __longlong_as_double(static_cast<long long>((hi << 32) | lo));
}
template <int S>
__device__ inline void swap_words(uint32_t& a, uint32_t& b) {
  if (S == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  }
}
template <int S>
__device__ inline float swap_sum(float a, float b) {
  uint32_t x = __float_as_uint(a), y = __float_as_uint(b);
  swap_words<S>(x, y);
  return __uint_as_float(x) + __uint_as_float(y);
}
template <int S>
__device__ inline double swap_sum(double a, double b) {
  const uint64_t ua = static_cast<uint64_t>(__double_as_longlong(a)), ub = static_cast<uint64_t>(__double_as_longlong(b));
  uint32_t al = static_cast<uint32_t>(ua), ah = static_cast<uint32_t>(ua >> 32);
  uint32_t bl = static_cast<uint32_t>(ub), bh = static_cast<uint32_t>(ub >> 32);
  swap_words<S>(al, bl);
  swap_words<S>(ah, bh);
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(ah) << 32) | al)) +
         __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(bh) << 32) | bl));
}

// one halving step over lane bit S: p[q] (q < S) becomes the sum, over the lane
// pair {l, l ^ S}, of entry q (bit clear) or q + S (bit set)
template <int S, typename AT, int NV>
__device__ inline void halve(AT (&p)[NV], bool up) {
#pragma unroll
  for (int q = 0; q < S; ++q) {
    if (S >= 16) {
      p[q] = swap_sum<S>(p[q], p[q + S]);
    } else {
      const AT lo = p[q] + xor_lane<S>(p[q]);
      const AT hi = p[q + S] + xor_lane<S>(p[q + S]);
      p[q] = up ? hi : lo;
    }
  }
}

// Sum over lanes of p[j], delivered to lane j: 64 values per lane (32 for FP64,
// where the two lane halves are added first and lane j & 31 receives column j),
// by recursive halving: at each step a lane keeps the half of its values
// selected by its lane bit, summed with the partner's copy of that half.
template <typename AT, int NV>
__device__ inline AT transpose_reduce(AT (&p)[NV]) {
  const int lane = threadIdx.x % 64;
  if (NV == 64) {
    halve<32>(p, false);
  } else {
#pragma unroll
    for (int q = 0; q < 32; ++q) p[q] = swap_sum<32>(p[q], p[q]);  // both halves get the full sum
  }
  halve<16>(p, false);
  halve<8>(p, (lane & 8) != 0);
  halve<4>(p, (lane & 4) != 0);
  halve<2>(p, (lane & 2) != 0);
  halve<1>(p, (lane & 1) != 0);
  return p[0];
}

// Near field with symmetric storage (leaves of at most 64 triangles): the panel
// of leaf tau holds its blocks (tau, sigma) with sigma not before tau.  One
// workgroup per leaf, blocks dealt to the four waves, lane = row.  An
// off-diagonal block also yields G^T x|tau (column sums over the lanes), written
// to the block's scratch slot; permute_out_sym adds the slots of each leaf.
template <typename ST, typename AT>
__global__ __launch_bounds__(256) void near_backward_sym(int nleaves, int k, const int32_t* __restrict__ leaves,
                                                         const int32_t* __restrict__ cbegin,
                                                         const int32_t* __restrict__ cend,
                                                         const int64_t* __restrict__ near_ptr,
                                                         const int32_t* __restrict__ near_col,
                                                         const int64_t* __restrict__ panel_off,
                                                         const int64_t* __restrict__ near_slot,
                                                         const ST* __restrict__ N, const ST* __restrict__ Vb,
                                                         const AT* __restrict__ xc, const AT* __restrict__ yhat,
                                                         AT* __restrict__ yc, AT* __restrict__ scratch) {
  constexpr int NV = sizeof(AT) == 4 ? 64 : 32;  // columns per transposed reduction
  __shared__ AT part[4][64];
  const int l = blockIdx.x;
  if (l >= nleaves) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int32_t tau = leaves[l];
  const int64_t b0 = cbegin[tau];
  const int r = cend[tau] - cbegin[tau];
  const int is = lane < r ? lane : r - 1;
  const AT xt = lane < r ? xc[b0 + lane] : AT(0);
  const ST* P = N + panel_off[l];
  AT acc = 0;
  int64_t colbase = 0;
  const int64_t bfirst = near_ptr[l], blast = near_ptr[l + 1];
  for (int64_t bb = bfirst; bb < blast; ++bb) {
    const int32_t s = near_col[bb];
    const int64_t s0 = cbegin[s];
    const int w = cend[s] - cbegin[s];
    if (((bb - bfirst) & 3) == wave) {
      const AT xv = lane < w ? xc[s0 + lane] : AT(0);
      const ST* A = P + colbase * r + is;
      const int64_t slot = near_slot[bb];
      if (slot < 0) {
        acc = stream_dot<ST, AT>(A, r, w, xv, acc);
      } else {
        // straight-line over all column slots of the chunk, loads clamped to the
        // last column: beyond w the row products vanish (xv is 0 there) and the
        // column partials are computed but never stored
#pragma unroll
        for (int c0 = 0; c0 < 64; c0 += NV) {
          if (c0 < w) {
            AT p[NV];
#pragma unroll
            for (int j = 0; j < NV; j += 8) {
              AT a[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) a[u] = ld<ST, AT>(A + min(c0 + j + u, w - 1) * r);
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                acc += a[u] * bcast(xv, c0 + j + u);
                p[j + u] = a[u] * xt;
              }
            }
            const AT t = transpose_reduce<AT, NV>(p);
            if (lane < NV && c0 + lane < w) scratch[slot + c0 + lane] = t;
          }
        }
      }
    }
    colbase += w;
  }
  // leaf backward: columns nu of V_tau, a quarter per wave (k <= 64)
  const ST* Vl = Vb + b0 * k;
  const int kq = (k + 3) / 4, n0 = wave * kq, nv = min(k, n0 + kq) - n0;
  const AT yv = lane < nv ? yhat[static_cast<int64_t>(tau) * k + n0 + lane] : AT(0);
  acc = stream_dot<ST, AT>(Vl + static_cast<int64_t>(n0) * r + is, r, nv, yv, acc);
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && lane < r) yc[b0 + lane] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// y[perm[p]] += alpha (y_c[p] + the transposed near-field parts addressed to p's leaf)
template <typename XT, typename AT>
__global__ void permute_out_sym(int64_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ leaf_of_pos,
                                const int32_t* __restrict__ leaves, const int32_t* __restrict__ cbegin,
                                const int64_t* __restrict__ in_ptr, const int64_t* __restrict__ in_slot,
                                const AT* __restrict__ scratch, const AT* __restrict__ yc, XT* __restrict__ y,
                                double alpha, bool ow) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t l = leaf_of_pos[p];
  const int64_t off = p - cbegin[leaves[l]];
  AT v = yc[p];
  for (int64_t i = in_ptr[l]; i < in_ptr[l + 1]; ++i) v += scratch[in_slot[i] + off];
  const int64_t t = perm[p];
  const double y0 = ow ? 0.0 : static_cast<double>(y[t]);
  y[t] = static_cast<XT>(y0 + alpha * static_cast<double>(v));
}

// ---------------------------------------------------------------- complex kernels (Helmholtz)
// S and the near field hold interleaved (re, im) entries; V and E are real (the
// Lagrange polynomials are real), so the forward and backward transformations
// run on the real and imaginary planes of x^, y^ with the real kernels above.
template <typename XT, typename AT>
__global__ void permute_in_c(int64_t n, const int32_t* __restrict__ perm, const XT* __restrict__ x,
                             AT* __restrict__ xr, AT* __restrict__ xi) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) {
    const int64_t t = perm[p];
    xr[p] = static_cast<AT>(x[2 * t]);
    xi[p] = static_cast<AT>(x[2 * t + 1]);
  }
}

template <typename XT, typename AT>
__global__ void permute_out_c(int64_t n, const int32_t* __restrict__ perm, const AT* __restrict__ yr,
                              const AT* __restrict__ yi, XT* __restrict__ y, double alpha, bool ow) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) {
    const int64_t t = perm[p];
    const double y0r = ow ? 0.0 : static_cast<double>(y[2 * t]);
    const double y0i = ow ? 0.0 : static_cast<double>(y[2 * t + 1]);
    y[2 * t] = static_cast<XT>(y0r + alpha * static_cast<double>(yr[p]));
    y[2 * t + 1] = static_cast<XT>(y0i + alpha * static_cast<double>(yi[p]));
  }
}

// k = 64: one workgroup per row cluster, 16-byte loads of interleaved complex S
template <typename SST, typename AT>
__global__ __launch_bounds__(256) void coupling64c(int nc, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col, const SST* __restrict__ S,
                                                   const AT* __restrict__ xr, const AT* __restrict__ xi,
                                                   AT* __restrict__ yr, AT* __restrict__ yi) {
  constexpr int VEC = Vec16<SST>::N;
  constexpr int CPV = VEC / 2;  // complex entries per 16-byte load
  constexpr int LPR = 64 / CPV;
  constexpr int RPP = 256 / LPR;
  constexpr int NP = 64 / RPP;
  const int tau = blockIdx.x;
  if (tau >= nc) return;
  const int t = threadIdx.x;
  const int lr = t % LPR, r0 = t / LPR;
  AT ar[NP], ai[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) ar[j] = ai[j] = 0;
  for (int64_t b = ptr[tau]; b < ptr[tau + 1]; ++b) {
    const int64_t s = col[b];
    AT vr[CPV], vi[CPV];
#pragma unroll
    for (int c = 0; c < CPV; ++c) {
      vr[c] = xr[s * 64 + lr * CPV + c];
      vi[c] = xi[s * 64 + lr * CPV + c];
    }
    const SST* Sb = S + b * 8192 + lr * VEC;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      AT sv[VEC];
      Vec16<SST>::load(Sb + (r0 + j * RPP) * 128, sv);
#pragma unroll
      for (int c = 0; c < CPV; ++c) {
        ar[j] += sv[2 * c] * vr[c] - sv[2 * c + 1] * vi[c];
        ai[j] += sv[2 * c] * vi[c] + sv[2 * c + 1] * vr[c];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int off = LPR / 2; off >= 1; off >>= 1) {
      ar[j] += __shfl_xor(ar[j], off);
      ai[j] += __shfl_xor(ai[j], off);
    }
  if (lr == 0) {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      yr[static_cast<int64_t>(tau) * 64 + r0 + j * RPP] = ar[j];
      yi[static_cast<int64_t>(tau) * 64 + r0 + j * RPP] = ai[j];
    }
  }
}

template <typename SST, typename AT>
__global__ __launch_bounds__(256) void coupling_anyc(int nc, int k, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col, const SST* __restrict__ S,
                                                     const AT* __restrict__ xr, const AT* __restrict__ xi,
                                                     AT* __restrict__ yr, AT* __restrict__ yi) {
  const int tau = blockIdx.x;
  if (tau >= nc) return;
  const int64_t kk = static_cast<int64_t>(k) * k;
  for (int nu = threadIdx.x; nu < k; nu += blockDim.x) {
    AT ar = 0, ai = 0;
    for (int64_t b = ptr[tau]; b < ptr[tau + 1]; ++b) {
      const SST* Sb = S + 2 * (b * kk + static_cast<int64_t>(nu) * k);
      const int64_t s = col[b];
      for (int mu = 0; mu < k; ++mu) {
        const AT sr = ld<SST, AT>(Sb + 2 * mu), si = ld<SST, AT>(Sb + 2 * mu + 1);
        ar += sr * xr[s * k + mu] - si * xi[s * k + mu];
        ai += sr * xi[s * k + mu] + si * xr[s * k + mu];
      }
    }
    yr[static_cast<int64_t>(tau) * k + nu] = ar;
    yi[static_cast<int64_t>(tau) * k + nu] = ai;
  }
}

// near field (complex panels, lane = row) + leaf backward (real V times both planes)
template <typename ST, typename AT>
__global__ __launch_bounds__(256) void near_backward_c(int nleaves, int k, const int32_t* __restrict__ leaves,
                                                       const int32_t* __restrict__ cbegin,
                                                       const int32_t* __restrict__ cend,
                                                       const int64_t* __restrict__ near_ptr,
                                                       const int32_t* __restrict__ near_col,
                                                       const int64_t* __restrict__ panel_off,
                                                       const ST* __restrict__ N, const ST* __restrict__ Vb,
                                                       const AT* __restrict__ xr, const AT* __restrict__ xi,
                                                       const AT* __restrict__ yhr, const AT* __restrict__ yhi,
                                                       AT* __restrict__ ycr, AT* __restrict__ yci) {
  __shared__ AT part[2][4][64];
  const int l = blockIdx.x;
  if (l >= nleaves) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int32_t tau = leaves[l];
  const int64_t b0 = cbegin[tau];
  const int r = cend[tau] - cbegin[tau];
  const ST* P = N + 2 * panel_off[l];
  const ST* Vl = Vb + b0 * k;
  const int64_t bfirst = near_ptr[l], blast = near_ptr[l + 1];
  for (int i0 = 0; i0 < r; i0 += 64) {
    const int i = i0 + lane;
    const int is = i < r ? i : r - 1;
    AT accr = 0, acci = 0;
    int64_t colbase = 0;
    for (int64_t bb = bfirst; bb < blast; ++bb) {
      const int32_t s = near_col[bb];
      const int64_t s0 = cbegin[s];
      const int w = cend[s] - cbegin[s];
      if (((bb - bfirst) & 3) == wave) {
        for (int j0 = 0; j0 < w; j0 += 64) {
          const AT vr = j0 + lane < w ? xr[s0 + j0 + lane] : AT(0);
          const AT vi = j0 + lane < w ? xi[s0 + j0 + lane] : AT(0);
          const ST* Pc = P + 2 * ((colbase + j0) * r + is);
          const int cnt = min(64, w - j0);
          int j = 0;
          for (; j + 4 <= cnt; j += 4) {
            AT nr[4], ni[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              nr[u] = ld<ST, AT>(Pc + 2 * static_cast<int64_t>(j + u) * r);
              ni[u] = ld<ST, AT>(Pc + 2 * static_cast<int64_t>(j + u) * r + 1);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const AT br = bcast(vr, j + u), bi = bcast(vi, j + u);
              accr += nr[u] * br - ni[u] * bi;
              acci += nr[u] * bi + ni[u] * br;
            }
          }
          for (; j < cnt; ++j) {
            const AT nr = ld<ST, AT>(Pc + 2 * static_cast<int64_t>(j) * r);
            const AT ni = ld<ST, AT>(Pc + 2 * static_cast<int64_t>(j) * r + 1);
            const AT br = bcast(vr, j), bi = bcast(vi, j);
            accr += nr * br - ni * bi;
            acci += nr * bi + ni * br;
          }
        }
      }
      colbase += w;
    }
    const int kq = (k + 3) / 4;
    const int n0 = wave * kq, n1 = min(k, n0 + kq);
    for (int q0 = n0; q0 < n1; q0 += 64) {
      const AT yr = q0 + lane < n1 ? yhr[static_cast<int64_t>(tau) * k + q0 + lane] : AT(0);
      const AT yi = q0 + lane < n1 ? yhi[static_cast<int64_t>(tau) * k + q0 + lane] : AT(0);
      accr = stream_dot<ST, AT>(Vl + static_cast<int64_t>(q0) * r + is, r, min(64, n1 - q0), yr, accr);
      acci = stream_dot<ST, AT>(Vl + static_cast<int64_t>(q0) * r + is, r, min(64, n1 - q0), yi, acci);
    }
    part[0][wave][lane] = accr;
    part[1][wave][lane] = acci;
    __syncthreads();
    if (wave == 0 && i < r) {
      ycr[b0 + i] = (part[0][0][lane] + part[0][1][lane]) + (part[0][2][lane] + part[0][3][lane]);
      yci[b0 + i] = (part[1][0][lane] + part[1][1][lane]) + (part[1][2][lane] + part[1][3][lane]);
    }
    __syncthreads();
  }
}

inline unsigned blocks_for(int64_t work, int per) {
  const int64_t g = (work + per - 1) / per;
  if (g > 0x7fffffff) throw Error(H2_EINVAL, "launch too large");
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

template <typename ST, typename AT>
void launch_up(h2_handle_s& H, AT* xh, hipStream_t st) {
  const Structure& S = H.S;
  const ST* E = H.kron ? H.E1.as<ST>() : H.F.as<ST>();
  const int32_t* list = H.up_list.as<int32_t>();
  for (int l = S.depth - 1; l >= H.up_top; --l) {
    const int cnt = static_cast<int>(H.up_ptr[l + 1] - H.up_ptr[l]);
    if (cnt == 0) continue;
    if (H.kron)
      transfer_up<ST, AT, true><<<blocks_for(cnt, 4), 256, 0, st>>>(cnt, S.k, list + H.up_ptr[l], H.child0.as<int32_t>(),
                                                                     H.child1.as<int32_t>(), E, xh);
    else
      transfer_up<ST, AT, false><<<blocks_for(cnt, 4), 256, 0, st>>>(cnt, S.k, list + H.up_ptr[l],
                                                                      H.child0.as<int32_t>(), H.child1.as<int32_t>(), E,
                                                                      xh);
  }
  if (H.up_top > 0) {
    if (H.kron)
      transfer_up_top<ST, AT, true><<<1, 64 * kTopWaves, 0, st>>>(H.up_top, H.up_ptr_dev.as<int64_t>(), S.k, list,
                                                                  H.child0.as<int32_t>(), H.child1.as<int32_t>(), E, xh);
    else
      transfer_up_top<ST, AT, false><<<1, 64 * kTopWaves, 0, st>>>(H.up_top, H.up_ptr_dev.as<int64_t>(), S.k, list,
                                                                   H.child0.as<int32_t>(), H.child1.as<int32_t>(), E,
                                                                   xh);
  }
}

template <typename ST, typename AT>
void launch_down(h2_handle_s& H, AT* yh, hipStream_t st) {
  const Structure& S = H.S;
  const ST* E = H.kron ? H.E1.as<ST>() : H.ET.as<ST>();
  if (H.down_top > 0) {
    if (H.kron)
      transfer_down_top<ST, AT, true><<<1, 64 * kTopWaves, 0, st>>>(H.down_top, H.level_ptr_dev.as<int32_t>(), S.k,
                                                                    H.parent.as<int32_t>(), E, yh);
    else
      transfer_down_top<ST, AT, false><<<1, 64 * kTopWaves, 0, st>>>(H.down_top, H.level_ptr_dev.as<int32_t>(), S.k,
                                                                     H.parent.as<int32_t>(), E, yh);
  }
  for (int l = H.down_top; l < S.depth; ++l) {
    const int first = S.level_ptr[l + 1], cnt = S.level_ptr[l + 2] - S.level_ptr[l + 1];
    if (cnt == 0) continue;
    if (H.kron)
      transfer_down<ST, AT, true><<<blocks_for(cnt, 4), 256, 0, st>>>(first, cnt, S.k, H.parent.as<int32_t>(), E, yh);
    else
      transfer_down<ST, AT, false><<<blocks_for(cnt, 4), 256, 0, st>>>(first, cnt, S.k, H.parent.as<int32_t>(), E, yh);
  }
}

template <typename SST, typename ST, typename AT, typename XT>
void matvec_typed(h2_handle_s& H, const XT* x, XT* y, double alpha, hipStream_t st) {
  const Structure& S = H.S;
  const int k = S.k;
  const int64_t n = S.n;
  const int nc = S.nclusters;
  const int nl = static_cast<int>(S.leaves.size());
  AT* xc = H.xc.as<AT>();
  AT* yc = H.yc.as<AT>();
  AT* xh = H.xhat.as<AT>();
  AT* yh = H.yhat.as<AT>();
  // BF16 storage keeps an FP32 copy of S: FP32 coupling data there is that copy
  const SST* Sm = (std::is_same<SST, float>::value && H.P.storage == H2_F32_SBF16) ? H.Smat32.as<SST>()
                                                                                    : H.Smat.as<SST>();
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr, e4 = nullptr;
  if (H.prof) {
    e0 = prof_event(H);
    H2_HIP(hipEventRecord(e0, st));
  }
  permute_in<XT, AT><<<blocks_for(n, 256), 256, 0, st>>>(n, H.perm.as<int32_t>(), x, xc);
  leaf_forward<ST, AT><<<blocks_for(nl, 4), 256, 0, st>>>(nl, k, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                                           H.cend.as<int32_t>(), H.Vf.as<ST>(), xc, xh);
  launch_up<ST, AT>(H, xh, st);
  if (H.prof) {
    e1 = prof_event(H);
    H2_HIP(hipEventRecord(e1, st));
  }
  if (H.otf) {
    if (H.P.storage == H2_F64) launch_otf<double, AT>(H, xh, yh, st);
    else launch_otf<float, AT>(H, xh, yh, st);
  } else if (S.sym_s) {
    coupling64_sym<SST, AT><<<nc, 256, 0, st>>>(nc, H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(),
                                               Sm, xh, yh, H.scr_s.as<AT>());
    adm_gather<AT><<<blocks_for(nc, 4), 256, 0, st>>>(nc, H.adm_in_ptr.as<int64_t>(), H.adm_in_blk.as<int64_t>(),
                                                      H.scr_s.as<AT>(), yh);
  } else if (k == 64) {
    coupling64<SST, AT><<<nc, 256, 0, st>>>(nc, H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(), Sm,
                                           xh, yh);
  } else if (k <= 32) {
    const int64_t* ap = H.adm_ptr.as<int64_t>();
    const int32_t* ac = H.adm_col.as<int32_t>();
    const unsigned g = blocks_for(nc, 4);
    // slots of 16 lanes cover k <= 16; 32 lanes cover every k here (tuned choice)
    const bool rb16 = k <= 16 && H.tune_slot != 32;
    constexpr bool f32 = std::is_same<SST, float>::value && std::is_same<AT, float>::value;
    if constexpr (f32) {
      if (k % 4 == 0) {
        if (rb16) coupling_small<16, true, float, float><<<g, 256, 0, st>>>(nc, k, ap, ac, Sm, xh, yh);
        else coupling_small<32, true, float, float><<<g, 256, 0, st>>>(nc, k, ap, ac, Sm, xh, yh);
      } else if (rb16) {
        coupling_small<16, false, SST, AT><<<g, 256, 0, st>>>(nc, k, ap, ac, Sm, xh, yh);
      } else {
        coupling_small<32, false, SST, AT><<<g, 256, 0, st>>>(nc, k, ap, ac, Sm, xh, yh);
      }
    } else if (rb16) {
      coupling_small<16, false, SST, AT><<<g, 256, 0, st>>>(nc, k, ap, ac, Sm, xh, yh);
    } else {
      coupling_small<32, false, SST, AT><<<g, 256, 0, st>>>(nc, k, ap, ac, Sm, xh, yh);
    }
  } else {
    coupling_any<SST, AT><<<nc, 256, 0, st>>>(nc, k, H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(),
                                             Sm, xh, yh);
  }
  if (H.prof) {
    e2 = prof_event(H);
    H2_HIP(hipEventRecord(e2, st));
  }
  launch_down<ST, AT>(H, yh, st);
  if (H.prof) {
    e3 = prof_event(H);
    H2_HIP(hipEventRecord(e3, st));
  }
  if (S.sym_n) {
    near_backward_sym<ST, AT><<<nl, 256, 0, st>>>(nl, k, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                                  H.cend.as<int32_t>(), H.near_ptr.as<int64_t>(),
                                                  H.near_col.as<int32_t>(), H.panel_off.as<int64_t>(),
                                                  H.near_slot.as<int64_t>(), H.Nmat.as<ST>(), H.Vb.as<ST>(), xc, yh,
                                                  yc, H.scr_n.as<AT>());
    permute_out_sym<XT, AT><<<blocks_for(n, 256), 256, 0, st>>>(
        n, H.perm.as<int32_t>(), H.leaf_of_pos.as<int32_t>(), H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
        H.near_in_ptr.as<int64_t>(), H.near_in_slot.as<int64_t>(), H.scr_n.as<AT>(), yc, y, alpha, H.overwrite);
  } else {
    // 16 loads per group for FP32 panels; 8 for FP64 (the same bytes in flight,
    // fewer registers, six waves per SIMD instead of four: 3.20 against 3.28 ms
    // at 1,310,720 triangles)
    if (H.near64)
      near_backward64<ST, AT, sizeof(ST) == 8 ? 8 : 16><<<nl, 256, 0, st>>>(nl, k, H.near_rows.as<NearRow>(),
                                                      H.near_blocks.as<NearBlock>(), H.Nmat.as<ST>(), H.Vb.as<ST>(),
                                                      xc, yh, yc);
    else
      near_backward<ST, AT><<<nl, 256, 0, st>>>(nl, k, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                                H.cend.as<int32_t>(), H.near_ptr.as<int64_t>(),
                                                H.near_col.as<int32_t>(), H.panel_off.as<int64_t>(), H.Nmat.as<ST>(),
                                                H.Vb.as<ST>(), xc, yh, yc);
    permute_out<XT, AT><<<blocks_for(n, 256), 256, 0, st>>>(n, H.perm.as<int32_t>(), yc, y, alpha, H.overwrite);
  }
  H2_HIP(hipGetLastError());
  if (H.prof) {
    e4 = prof_event(H);
    H2_HIP(hipEventRecord(e4, st));
    prof_record(H, H2_PH_FORWARD, e0, e1);
    prof_record(H, H2_PH_COUPLING, e1, e2);
    prof_record(H, H2_PH_DOWN, e2, e3);
    prof_record(H, H2_PH_NEAR, e3, e4);
    prof_record(H, H2_PH_TOTAL, e0, e4);
  }
}

template <typename SST, typename ST, typename AT>
void matvec_x(h2_handle_s& H, int dtype, const void* x, void* y, double alpha, hipStream_t st) {
  if (dtype == H2_R64)
    matvec_typed<SST, ST, AT, double>(H, static_cast<const double*>(x), static_cast<double*>(y), alpha, st);
  else
    matvec_typed<SST, ST, AT, float>(H, static_cast<const float*>(x), static_cast<float*>(y), alpha, st);
}

template <typename SST, typename ST, typename AT, typename XT>
void matvec_complex(h2_handle_s& H, const XT* x, XT* y, double alpha, hipStream_t st) {
  const Structure& S = H.S;
  const int k = S.k;
  const int64_t n = S.n;
  const int nc = S.nclusters;
  const int nl = static_cast<int>(S.leaves.size());
  const int64_t nh = static_cast<int64_t>(nc) * k;
  AT* xr = H.xc.as<AT>();
  AT* xi = xr + n;
  AT* ycr = H.yc.as<AT>();
  AT* yci = ycr + n;
  AT* xhr = H.xhat.as<AT>();
  AT* xhi = xhr + nh;
  AT* yhr = H.yhat.as<AT>();
  AT* yhi = yhr + nh;
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr, e4 = nullptr;
  if (H.prof) {
    e0 = prof_event(H);
    H2_HIP(hipEventRecord(e0, st));
  }
  permute_in_c<XT, AT><<<blocks_for(n, 256), 256, 0, st>>>(n, H.perm.as<int32_t>(), x, xr, xi);
  AT* planes_x[2] = {xr, xi};
  AT* planes_h[2] = {xhr, xhi};
  for (int pl = 0; pl < 2; ++pl) {
    leaf_forward<ST, AT><<<blocks_for(nl, 4), 256, 0, st>>>(nl, k, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                                             H.cend.as<int32_t>(), H.Vf.as<ST>(), planes_x[pl],
                                                             planes_h[pl]);
    launch_up<ST, AT>(H, planes_h[pl], st);
  }
  if (H.prof) {
    e1 = prof_event(H);
    H2_HIP(hipEventRecord(e1, st));
  }
  if (H.otf)
    coupling64c_otf<AT><<<nc, 256, 0, st>>>(nc, static_cast<float>(H.P.kappa), H.row_spans.as<RowSpan>(),
                                            H.adm_col.as<int32_t>(), H.ctr.as<double>(), H.off32.as<float>(), xhr,
                                            xhi, yhr, yhi);
  else if (k == 64)
    coupling64c<SST, AT><<<nc, 256, 0, st>>>(nc, H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(),
                                            H.Smat.as<SST>(), xhr, xhi, yhr, yhi);
  else
    coupling_anyc<SST, AT><<<nc, 256, 0, st>>>(nc, k, H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(),
                                              H.Smat.as<SST>(), xhr, xhi, yhr, yhi);
  if (H.prof) {
    e2 = prof_event(H);
    H2_HIP(hipEventRecord(e2, st));
  }
  AT* planes_y[2] = {yhr, yhi};
  for (int pl = 0; pl < 2; ++pl) launch_down<ST, AT>(H, planes_y[pl], st);
  if (H.prof) {
    e3 = prof_event(H);
    H2_HIP(hipEventRecord(e3, st));
  }
  near_backward_c<ST, AT><<<nl, 256, 0, st>>>(nl, k, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                              H.cend.as<int32_t>(), H.near_ptr.as<int64_t>(),
                                              H.near_col.as<int32_t>(), H.panel_off.as<int64_t>(), H.Nmat.as<ST>(),
                                              H.Vb.as<ST>(), xr, xi, yhr, yhi, ycr, yci);
  permute_out_c<XT, AT><<<blocks_for(n, 256), 256, 0, st>>>(n, H.perm.as<int32_t>(), ycr, yci, y, alpha,
                                                            H.overwrite);
  H2_HIP(hipGetLastError());
  if (H.prof) {
    e4 = prof_event(H);
    H2_HIP(hipEventRecord(e4, st));
    prof_record(H, H2_PH_FORWARD, e0, e1);
    prof_record(H, H2_PH_COUPLING, e1, e2);
    prof_record(H, H2_PH_DOWN, e2, e3);
    prof_record(H, H2_PH_NEAR, e3, e4);
    prof_record(H, H2_PH_TOTAL, e0, e4);
  }
}

template <typename SST, typename ST, typename AT>
void matvec_cx(h2_handle_s& H, int dtype, const void* x, void* y, double alpha, hipStream_t st) {
  if (dtype == H2_C128)
    matvec_complex<SST, ST, AT, double>(H, static_cast<const double*>(x), static_cast<double*>(y), alpha, st);
  else
    matvec_complex<SST, ST, AT, float>(H, static_cast<const float*>(x), static_cast<float*>(y), alpha, st);
}

}  // namespace

void matvec(h2_handle_s& H, int nrhs, int dtype, const void* x, int64_t ldx, void* y, int64_t ldy, double alpha,
            int flags, hipStream_t st, bool may_alloc) {
  if (H.host_only) throw Error(H2_EINVAL, "handle was built with H2_HOST_ONLY");
  if (nrhs < 0) throw Error(H2_EINVAL, "nrhs must be >= 0");
  const bool cx = dtype == H2_C128 || dtype == H2_C64;
  if (dtype != H2_R64 && dtype != H2_R32 && !cx) throw Error(H2_EINVAL, "unknown dtype");
  if (cx != H.is_complex)
    throw Error(H2_EINVAL, H.is_complex ? "the Helmholtz matrix needs complex vectors (H2_C128/H2_C64)"
                                        : "complex vectors need the Helmholtz kernel");
  if (nrhs > 0 && (x == nullptr || y == nullptr)) throw Error(H2_EINVAL, "x and y must not be NULL");
  if (ldx < H.S.n || ldy < H.S.n) throw Error(H2_EINVAL, "leading dimension smaller than n");
  const bool acc64 = (flags & H2_ACC_F64) != 0;
  H.overwrite = (flags & H2_OVERWRITE) != 0;
  const bool multi = nrhs >= 2 && !acc64 && matvec_multi_supported(H) &&
                     (may_alloc || matvec_multi_ready(H, nrhs, dtype));
  if (cx) {
    if (multi) {
      matvec_multi(H, nrhs, dtype, x, ldx, y, ldy, alpha, st);
      return;
    }
    const size_t es = dtype == H2_C128 ? 16 : 8;
    for (int j = 0; j < nrhs; ++j) {
      const void* xj = static_cast<const char*>(x) + static_cast<size_t>(j) * ldx * es;
      void* yj = static_cast<char*>(y) + static_cast<size_t>(j) * ldy * es;
      if (H.P.storage == H2_F64) matvec_cx<double, double, double>(H, dtype, xj, yj, alpha, st);
      else if (acc64) matvec_cx<float, float, double>(H, dtype, xj, yj, alpha, st);
      else matvec_cx<float, float, float>(H, dtype, xj, yj, alpha, st);
    }
    return;
  }
  const size_t es = dtype == H2_R64 ? 8 : 4;
  if (multi) {
    matvec_multi(H, nrhs, dtype, x, ldx, y, ldy, alpha, st);
    return;
  }
  for (int j = 0; j < nrhs; ++j) {
    const void* xj = static_cast<const char*>(x) + static_cast<size_t>(j) * ldx * es;
    void* yj = static_cast<char*>(y) + static_cast<size_t>(j) * ldy * es;
    switch (H.P.storage) {
      case H2_F64: matvec_x<double, double, double>(H, dtype, xj, yj, alpha, st); break;
      case H2_F32:
        if (acc64) matvec_x<float, float, double>(H, dtype, xj, yj, alpha, st);
        else matvec_x<float, float, float>(H, dtype, xj, yj, alpha, st);
        break;
      default:  // BF16 S; FP64 accumulation applies the FP32 copy of S
        if (acc64) matvec_x<float, float, double>(H, dtype, xj, yj, alpha, st);
        else matvec_x<bf16, float, float>(H, dtype, xj, yj, alpha, st);
    }
  }
}

}  // namespace h2

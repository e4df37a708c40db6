// Step-wise Krylov solver for G~ Z = B with several right-hand sides (the
// paper's introduction names Krylov methods for the Galerkin system; it picks
// none, so: conjugate gradients for the symmetric positive definite Laplace
// single-layer matrix, restarted GMRES with classical Gram-Schmidt applied twice
// and complex Givens rotations for any nonsingular matrix, e.g. the complex
// symmetric Helmholtz matrix).
//
// The solver never applies the matrix itself.  It asks for one product
// Y = G~ X per step (`next` writes X, `advance` consumes Y), so a caller can batch
// the products of many solves into one many-right-hand-side product; h2_solve
// drives it with the handle's own product.  All vectors, inner products, the
// Hessenberg columns, the Givens rotations and the small triangular solves live
// on the device in FP64 (complex FP64); the host only reads, after the caller has
// synchronised, one residual per column to take the control decisions (converged,
// restart, refine).  Columns run in lockstep: one product serves every column.
//
// Optional iterative refinement (FP32 / BF16 storage): the outer residual
// B - G~ Z is formed from a product with FP64 accumulation (H2_ACC_F64; with BF16
// coupling storage that product applies the FP32 copy of S), the inner solve runs
// on products with the storage precision's accumulation.
//
// Reductions: every inner product is a fixed two-stage sum -- per (column, chunk)
// partial sums in a fixed order, then one wave per column adds the chunks in a
// fixed order.  The chunking depends on n and the column count only, so a solve
// gives the same numbers whatever other work shares the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "handle.h"
#include "ksolve.h"

namespace h2 {
namespace {

constexpr int KT = 256;  // threads of the chunked kernels

// per-column scalars, doubles at scal + c * sc_stride
enum {
  S_NB_OUT = 0,  // ||b_c||
  S_REL_OUT,     // ||b_c - G~ z_c|| / ||b_c|| (0 for b_c = 0)
  S_NB_IN,       // ||inner right-hand side||
  S_RR,          // CG: <r, r>
  S_ALPHA,       // CG step length
  S_BETA,        // CG direction update
  S_REL_IN,      // inner relative residual (recurrence estimate or true)
  S_INV,         // GMRES: 1 / norm of the vector being normalised (0 if that norm is 0)
  S_BAD,         // 1 once a reduction gave a non-finite value
  S_FIXED        // first complex array
};

struct Geo {
  int64_t n;      // rows
  int cw;         // doubles per entry (1 real, 2 complex)
  int r;          // columns
  int m;          // GMRES restart (0 for CG)
  int nchunk;     // chunks per column
  int64_t csz;    // rows per chunk
  int nvmax;      // partial sums per (column, chunk)
  int64_t sc;     // doubles of scalars per column
  // complex arrays (pairs of doubles) inside a column's scalars
  int64_t o_hcol, o_hcur, o_g, o_cs, o_sn, o_y, o_H;
};

__host__ __device__ inline int64_t col_off(const Geo& g, int c) { return static_cast<int64_t>(c) * g.sc; }

// ---------------------------------------------------------------- reductions
template <bool CX>
__device__ inline void block_sum2(double& sr, double& si, double* lds /* 2 * KT/64 */) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    if (CX) si += __shfl_xor(si, o);
  }
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (threadIdx.x % 64 == 0) {
    lds[2 * w] = sr;
    lds[2 * w + 1] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, ti = 0.0;
    for (int v = 0; v < KT / 64; ++v) {
      tr += lds[2 * v];
      ti += lds[2 * v + 1];
    }
    sr = tr;
    si = ti;
  }
}

// conj(a) * b
template <bool CX>
__device__ inline void cdot_acc(const double* a, const double* b, int64_t e, double& sr, double& si) {
  if (CX) {
    const double ar = a[2 * e], ai = a[2 * e + 1], br = b[2 * e], bi = b[2 * e + 1];
    sr += ar * br + ai * bi;
    si += ar * bi - ai * br;
  } else {
    sr += a[e] * b[e];
  }
}

// part[((c * nvmax + i) * nchunk + chunk) * 2 + {0,1}] = sum over the chunk of conj(A_{c,i}) B_c
// A_{c,i} = A + c * a_col + i * a_vec, B_c = B + c * b_col (offsets in doubles)
template <bool CX>
__global__ __launch_bounds__(KT) void k_partial(Geo g, int nvec, const double* __restrict__ A, int64_t a_col,
                                                int64_t a_vec, const double* __restrict__ B, int64_t b_col,
                                                double* __restrict__ part) {
  __shared__ double lds[2 * KT / 64];
  const int chunk = blockIdx.x, c = blockIdx.y;
  const int64_t e0 = chunk * g.csz, e1 = e0 + g.csz < g.n ? e0 + g.csz : g.n;
  const double* b = B + c * b_col;
  for (int i = 0; i < nvec; ++i) {
    const double* a = A + c * a_col + i * a_vec;
    double sr = 0.0, si = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += KT) cdot_acc<CX>(a, b, e, sr, si);
    block_sum2<CX>(sr, si, lds);
    if (threadIdx.x == 0) {
      double* p = part + ((static_cast<int64_t>(c) * g.nvmax + i) * g.nchunk + chunk) * 2;
      p[0] = sr;
      p[1] = si;
    }
  }
}

// ---------------------------------------------------------------- complex helpers
struct cpx {
  double re, im;
};
__device__ inline cpx cmul(cpx a, cpx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cpx cconj(cpx a) { return {a.re, -a.im}; }
__device__ inline cpx cadd(cpx a, cpx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cpx csub(cpx a, cpx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cpx cscale(cpx a, double s) { return {a.re * s, a.im * s}; }
__device__ inline double cabs2(cpx a) { return a.re * a.re + a.im * a.im; }
__device__ inline cpx cdiv(cpx a, cpx b) {
  const double d = cabs2(b);
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ inline cpx ld_c(const double* p, int64_t i) { return {p[2 * i], p[2 * i + 1]}; }
__device__ inline void st_c(double* p, int64_t i, cpx v) {
  p[2 * i] = v.re;
  p[2 * i + 1] = v.im;
}

// ---------------------------------------------------------------- finishing the sums
enum Op {
  OP_NB_OUT = 0,   // ||b||; rel_out = (b != 0)
  OP_REL_OUT,      // rel_out = ||r|| / ||b||
  OP_CG_INIT,      // rr = <r, r>, nb_in, rel_in
  OP_CG_ALPHA,     // alpha = rr / <p, G~p>
  OP_CG_BETA,      // beta = rr' / rr, rr = rr', rel_in
  OP_GM_START,     // beta = ||r||: nb_in = beta, g = beta e_1, rel_in, inv
  OP_GM_RESTART,   // beta = ||r||: g = beta e_1, rel_in, inv
  OP_GM_H1,        // h = Q^H w (first Gram-Schmidt pass)
  OP_GM_H2,        // h += Q^H w (second pass)
  OP_GM_NORM       // h_{j+1,j} = ||w||, Givens rotations, rel_in, inv
};

// One wave per column: adds the chunks of nvec partial sums in a fixed order,
// then lane 0 updates the column's scalars.
template <bool CX>
__global__ __launch_bounds__(64) void k_finish(Geo g, int op, int nvec, int j, const double* __restrict__ part,
                                               double* __restrict__ scal) {
  __shared__ double hv[2 * 128];
  const int c = blockIdx.x;
  for (int i = 0; i < nvec; ++i) {
    const double* p = part + (static_cast<int64_t>(c) * g.nvmax + i) * g.nchunk * 2;
    double sr = 0.0, si = 0.0;
    for (int k = threadIdx.x; k < g.nchunk; k += 64) {
      sr += p[2 * k];
      si += p[2 * k + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sr += __shfl_xor(sr, o);
      si += __shfl_xor(si, o);
    }
    if (threadIdx.x == 0) {
      hv[2 * i] = sr;
      hv[2 * i + 1] = CX ? si : 0.0;
    }
  }
  if (threadIdx.x != 0) return;
  double* s = scal + col_off(g, c);
  const double v = hv[0];
  // the reductions that read a product first blame the product (1), the others the
  // solver's own arithmetic (2)
  const bool reads_product = op == OP_REL_OUT || op == OP_CG_ALPHA || op == OP_GM_H1 || op == OP_GM_RESTART;
  auto bad = [&](double x) {
    if (!std::isfinite(x) && s[S_BAD] == 0.0) s[S_BAD] = reads_product ? 1.0 : 2.0;
  };
  switch (op) {
    case OP_NB_OUT: {
      const double nb = std::sqrt(std::max(v, 0.0));
      s[S_NB_OUT] = nb;
      s[S_REL_OUT] = nb > 0.0 ? 1.0 : 0.0;
      bad(v);
      break;
    }
    case OP_REL_OUT: {
      const double nr = std::sqrt(std::max(v, 0.0));
      s[S_REL_OUT] = s[S_NB_OUT] > 0.0 ? nr / s[S_NB_OUT] : 0.0;
      bad(v);
      break;
    }
    case OP_CG_INIT:
      s[S_RR] = v;
      s[S_NB_IN] = std::sqrt(std::max(v, 0.0));
      s[S_REL_IN] = v > 0.0 ? 1.0 : 0.0;
      bad(v);
      break;
    case OP_CG_ALPHA:
      s[S_ALPHA] = (v > 0.0 && std::isfinite(v)) ? s[S_RR] / v : 0.0;
      bad(v);
      break;
    case OP_CG_BETA: {
      const double rr = s[S_RR];
      s[S_BETA] = rr > 0.0 ? v / rr : 0.0;
      s[S_RR] = v;
      s[S_REL_IN] = s[S_NB_IN] > 0.0 ? std::sqrt(std::max(v, 0.0)) / s[S_NB_IN] : 0.0;
      bad(v);
      break;
    }
    case OP_GM_START:
    case OP_GM_RESTART: {
      const double beta = std::sqrt(std::max(v, 0.0));
      if (op == OP_GM_START) s[S_NB_IN] = beta;
      double* gg = s + g.o_g;
      for (int i = 0; i <= g.m; ++i) st_c(gg, i, {0.0, 0.0});
      st_c(gg, 0, {beta, 0.0});
      s[S_REL_IN] = s[S_NB_IN] > 0.0 ? beta / s[S_NB_IN] : 0.0;
      s[S_INV] = beta > 0.0 ? 1.0 / beta : 0.0;
      bad(v);
      break;
    }
    case OP_GM_H1:
    case OP_GM_H2: {
      double* hc = s + g.o_hcol;
      double* hu = s + g.o_hcur;
      for (int i = 0; i < nvec; ++i) {
        const cpx h = {hv[2 * i], hv[2 * i + 1]};
        st_c(hu, i, h);
        st_c(hc, i, op == OP_GM_H1 ? h : cadd(ld_c(hc, i), h));
        bad(h.re);
        bad(h.im);
      }
      break;
    }
    case OP_GM_NORM: {
      const double hn = std::sqrt(std::max(v, 0.0));
      bad(v);
      double* hc = s + g.o_hcol;
      double* cs = s + g.o_cs;
      double* sn = s + g.o_sn;
      double* gg = s + g.o_g;
      double* H = s + g.o_H;
      st_c(hc, j + 1, {hn, 0.0});
      for (int i = 0; i < j; ++i) {  // the earlier rotations
        const cpx a = ld_c(hc, i), b = ld_c(hc, i + 1), ci = ld_c(cs, i), si = ld_c(sn, i);
        st_c(hc, i + 1, csub(cmul(ci, b), cmul(cconj(si), a)));
        st_c(hc, i, cadd(cmul(ci, a), cmul(si, b)));
      }
      const cpx a = ld_c(hc, j), b = ld_c(hc, j + 1);
      const double aa = std::sqrt(cabs2(a));
      const double den = std::sqrt(cabs2(a) + cabs2(b));
      cpx cj, sj;
      if (aa == 0.0) {
        cj = {0.0, 0.0};
        sj = {1.0, 0.0};
      } else {
        cj = {aa / den, 0.0};
        sj = cscale(cmul(cscale(a, 1.0 / aa), cconj(b)), 1.0 / den);
      }
      st_c(cs, j, cj);
      st_c(sn, j, sj);
      st_c(hc, j, cadd(cmul(cj, a), cmul(sj, b)));
      st_c(hc, j + 1, {0.0, 0.0});
      const cpx gj = ld_c(gg, j);
      st_c(gg, j + 1, cscale(cmul(cconj(sj), gj), -1.0));
      st_c(gg, j, cmul(cj, gj));
      for (int i = 0; i <= j; ++i) st_c(H, static_cast<int64_t>(i) * g.m + j, ld_c(hc, i));
      const double gn = std::sqrt(cabs2(ld_c(gg, j + 1)));
      s[S_REL_IN] = s[S_NB_IN] > 0.0 ? gn / s[S_NB_IN] : 0.0;
      s[S_INV] = hn > 0.0 ? 1.0 / hn : 0.0;
      bad(gn);
      break;
    }
    default:
      break;
  }
}

// ---------------------------------------------------------------- element-wise steps
// Every kernel runs on the (chunk, column) grid of the reductions; e indexes rows.
#define CHUNK_LOOP(g)                                                      \
  const int c = blockIdx.y;                                                \
  const int64_t e0 = blockIdx.x * (g).csz;                                 \
  const int64_t e1 = e0 + (g).csz < (g).n ? e0 + (g).csz : (g).n;         \
  for (int64_t e = e0 + threadIdx.x; e < e1; e += KT)

// D = 0 (columns d_col apart)
__global__ __launch_bounds__(KT) void k_zero(Geo g, double* __restrict__ D, int64_t d_col) {
  CHUNK_LOOP(g) {
    for (int q = 0; q < g.cw; ++q) D[c * d_col + g.cw * e + q] = 0.0;
  }
}

// p[0, count) = 0 (a kernel rather than a memset, so the solve records no memset node
// if a caller captures its stream)
__global__ __launch_bounds__(KT) void k_fill0(double* __restrict__ p, int64_t count) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * KT + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * KT)
    p[i] = 0.0;
}

// Z = z0 for columns with b != 0, else 0
__global__ __launch_bounds__(KT) void k_copy_masked(Geo g, const double* __restrict__ S, int64_t s_col,
                                                    double* __restrict__ D, int64_t d_col,
                                                    const double* __restrict__ scal) {
  const bool keep = scal[col_off(g, blockIdx.y) + S_NB_OUT] > 0.0;
  CHUNK_LOOP(g) {
    for (int q = 0; q < g.cw; ++q) D[c * d_col + g.cw * e + q] = keep ? S[c * s_col + g.cw * e + q] : 0.0;
  }
}

// R = B - Y, partial sums of |R|^2
template <bool CX>
__global__ __launch_bounds__(KT) void k_resid(Geo g, const double* __restrict__ B, int64_t b_col,
                                              const double* __restrict__ Y, int64_t y_col, double* __restrict__ R,
                                              int64_t r_col, double* __restrict__ part) {
  __shared__ double lds[2 * KT / 64];
  double sr = 0.0, si = 0.0;
  CHUNK_LOOP(g) {
    for (int q = 0; q < g.cw; ++q) {
      const double v = B[c * b_col + g.cw * e + q] - Y[c * y_col + g.cw * e + q];
      R[c * r_col + g.cw * e + q] = v;
      sr += v * v;
    }
  }
  block_sum2<false>(sr, si, lds);
  if (threadIdx.x == 0) {
    double* p = part + (static_cast<int64_t>(blockIdx.y) * g.nvmax * g.nchunk + blockIdx.x) * 2;
    p[0] = sr;
    p[1] = 0.0;
  }
}

// CG start: X = 0, R = P = F (inner right-hand side), partial sums of |F|^2
__global__ __launch_bounds__(KT) void k_cg_init(Geo g, const double* __restrict__ F, int64_t f_col,
                                                double* __restrict__ X, double* __restrict__ R,
                                                double* __restrict__ P, int64_t col, double* __restrict__ part) {
  __shared__ double lds[2 * KT / 64];
  double sr = 0.0, si = 0.0;
  CHUNK_LOOP(g) {
    for (int q = 0; q < g.cw; ++q) {
      const double v = F[c * f_col + g.cw * e + q];
      X[c * col + g.cw * e + q] = 0.0;
      R[c * col + g.cw * e + q] = v;
      P[c * col + g.cw * e + q] = v;
      sr += v * v;
    }
  }
  block_sum2<false>(sr, si, lds);
  if (threadIdx.x == 0) {
    double* p = part + (static_cast<int64_t>(blockIdx.y) * g.nvmax * g.nchunk + blockIdx.x) * 2;
    p[0] = sr;
    p[1] = 0.0;
  }
}

// CG: X += alpha P, R -= alpha Y (Y = G~ P), partial sums of |R|^2
__global__ __launch_bounds__(KT) void k_cg_xr(Geo g, const double* __restrict__ P, const double* __restrict__ Y,
                                              int64_t y_col, double* __restrict__ X, double* __restrict__ R,
                                              int64_t col, const double* __restrict__ scal, double* __restrict__ part) {
  __shared__ double lds[2 * KT / 64];
  const double alpha = scal[col_off(g, blockIdx.y) + S_ALPHA];
  double sr = 0.0, si = 0.0;
  CHUNK_LOOP(g) {
    const int64_t o = c * col + e;
    X[o] += alpha * P[o];
    const double r = R[o] - alpha * Y[c * y_col + e];
    R[o] = r;
    sr += r * r;
  }
  block_sum2<false>(sr, si, lds);
  if (threadIdx.x == 0) {
    double* p = part + (static_cast<int64_t>(blockIdx.y) * g.nvmax * g.nchunk + blockIdx.x) * 2;
    p[0] = sr;
    p[1] = 0.0;
  }
}

// CG: P = R + beta P
__global__ __launch_bounds__(KT) void k_cg_p(Geo g, const double* __restrict__ R, double* __restrict__ P, int64_t col,
                                             const double* __restrict__ scal) {
  const double beta = scal[col_off(g, blockIdx.y) + S_BETA];
  CHUNK_LOOP(g) {
    const int64_t o = c * col + e;
    P[o] = R[o] + beta * P[o];
  }
}

// GMRES: W = V - sum_{i < nvec} hcur_i Q_i  (V = Y for the first pass, W itself for the
// second); with norm set, also the partial sums of |W|^2
template <bool CX, bool NORM>
__global__ __launch_bounds__(KT) void k_gs_update(Geo g, int nvec, const double* __restrict__ Q, int64_t q_col,
                                                  int64_t q_vec, const double* V, int64_t v_col, double* W,
                                                  int64_t w_col, const double* __restrict__ scal,
                                                  double* __restrict__ part) {
  __shared__ double lds[2 * KT / 64];
  __shared__ double h[2 * 128];
  const double* hc = scal + col_off(g, blockIdx.y) + g.o_hcur;
  for (int i = threadIdx.x; i < 2 * nvec; i += KT) h[i] = hc[i];
  __syncthreads();
  double sr = 0.0, si = 0.0;
  CHUNK_LOOP(g) {
    double ar = V[c * v_col + g.cw * e], ai = CX ? V[c * v_col + 2 * e + 1] : 0.0;
    for (int i = 0; i < nvec; ++i) {
      const double* q = Q + c * q_col + i * q_vec;
      if (CX) {
        const double qr = q[2 * e], qi = q[2 * e + 1];
        ar -= h[2 * i] * qr - h[2 * i + 1] * qi;
        ai -= h[2 * i] * qi + h[2 * i + 1] * qr;
      } else {
        ar -= h[2 * i] * q[e];
      }
    }
    W[c * w_col + g.cw * e] = ar;
    if (CX) W[c * w_col + 2 * e + 1] = ai;
    if (NORM) sr += ar * ar + ai * ai;
  }
  if (NORM) {
    block_sum2<false>(sr, si, lds);
    if (threadIdx.x == 0) {
      double* p = part + (static_cast<int64_t>(blockIdx.y) * g.nvmax * g.nchunk + blockIdx.x) * 2;
      p[0] = sr;
      p[1] = 0.0;
    }
  }
}

// D = inv * S (inv = the column's S_INV)
__global__ __launch_bounds__(KT) void k_scale(Geo g, const double* __restrict__ S, int64_t s_col, double* __restrict__ D,
                                              int64_t d_col, const double* __restrict__ scal) {
  const double inv = scal[col_off(g, blockIdx.y) + S_INV];
  CHUNK_LOOP(g) {
    for (int q = 0; q < g.cw; ++q) D[c * d_col + g.cw * e + q] = inv * S[c * s_col + g.cw * e + q];
  }
}

// D += S
__global__ __launch_bounds__(KT) void k_add(Geo g, const double* __restrict__ S, int64_t s_col, double* __restrict__ D,
                                            int64_t d_col) {
  CHUNK_LOOP(g) {
    for (int q = 0; q < g.cw; ++q) D[c * d_col + g.cw * e + q] += S[c * s_col + g.cw * e + q];
  }
}

// GMRES cycle end, one thread per column: y = H(0:k, 0:k)^{-1} g(0:k) by back
// substitution (a zero diagonal entry gives a zero coefficient), stored as the
// coefficients hcur for X += sum_i y_i Q_i.
__global__ void k_backsolve(Geo g, int k, double* __restrict__ scal) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.r) return;
  double* s = scal + col_off(g, c);
  const double* H = s + g.o_H;
  const double* gg = s + g.o_g;
  double* y = s + g.o_hcur;
  for (int i = k - 1; i >= 0; --i) {
    cpx acc = ld_c(gg, i);
    for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(ld_c(H, static_cast<int64_t>(i) * g.m + l), ld_c(y, l)));
    const cpx d = ld_c(H, static_cast<int64_t>(i) * g.m + i);
    st_c(y, i, cabs2(d) > 0.0 ? cdiv(acc, d) : cpx{0.0, 0.0});
  }
}

// status for the host: rel_out per column, rel_in per column, any non-finite
__global__ void k_status(Geo g, const double* __restrict__ scal, double* __restrict__ stat) {
  const int c = threadIdx.x + blockIdx.x * blockDim.x;
  if (c < g.r) {
    const double* s = scal + col_off(g, c);
    stat[c] = s[S_REL_OUT];
    stat[g.r + c] = s[S_REL_IN];
    stat[2 * g.r + c] = s[S_BAD];
  }
}

// GMRES: X += sum_{i < nvec} y_i Q_i with y in hcur (nvec = k columns of the cycle)
template <bool CX>
__global__ __launch_bounds__(KT) void k_xupdate(Geo g, int nvec, const double* __restrict__ Q, int64_t q_col,
                                                int64_t q_vec, double* __restrict__ X, int64_t x_col,
                                                const double* __restrict__ scal) {
  __shared__ double h[2 * 128];
  const double* hc = scal + col_off(g, blockIdx.y) + g.o_hcur;
  for (int i = threadIdx.x; i < 2 * nvec; i += KT) h[i] = hc[i];
  __syncthreads();
  CHUNK_LOOP(g) {
    double ar = 0.0, ai = 0.0;
    for (int i = 0; i < nvec; ++i) {
      const double* q = Q + c * q_col + i * q_vec;
      if (CX) {
        const double qr = q[2 * e], qi = q[2 * e + 1];
        ar += h[2 * i] * qr - h[2 * i + 1] * qi;
        ai += h[2 * i] * qi + h[2 * i + 1] * qr;
      } else {
        ar += h[2 * i] * q[e];
      }
    }
    X[c * x_col + g.cw * e] += ar;
    if (CX) X[c * x_col + 2 * e + 1] += ai;
  }
}

// Z columns from/to a caller's block with leading dimension ld (in entries)
__global__ __launch_bounds__(KT) void k_copy_ld(Geo g, const double* __restrict__ S, int64_t s_col, double* __restrict__ D,
                                                int64_t d_col) {
  CHUNK_LOOP(g) {
    for (int q = 0; q < g.cw; ++q) D[c * d_col + g.cw * e + q] = S[c * s_col + g.cw * e + q];
  }
}

inline size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

}  // namespace

// ============================================================================ KSolver
KLayout klayout(int dtype, int64_t n, int nrhs, const h2_solve_params& p) {
  KLayout L{};
  L.cx = dtype == H2_C128;
  L.cg = p.method == H2_CG;
  L.n = n;
  L.r = nrhs;
  L.m = L.cg ? 0 : p.restart;
  const int cw = L.cx ? 2 : 1;
  // chunks: about 2048 workgroups in all, at least 1024 rows per chunk, at most 1024 chunks
  int nch = static_cast<int>(std::min<int64_t>((n + 1023) / 1024, (2048 + nrhs - 1) / std::max(nrhs, 1)));
  nch = std::max(1, std::min(nch, 1024));
  L.nchunk = nch;
  L.csz = (n + nch - 1) / nch;
  L.nvmax = L.cg ? 1 : L.m + 1;
  const int64_t mm = std::max(L.m, 1);
  L.o_hcol = S_FIXED;
  L.o_hcur = L.o_hcol + 2 * (mm + 1);
  L.o_g = L.o_hcur + 2 * (mm + 1);
  L.o_cs = L.o_g + 2 * (mm + 1);
  L.o_sn = L.o_cs + 2 * mm;
  L.o_y = L.o_sn + 2 * mm;
  L.o_H = L.o_y + 2 * mm;
  L.sc = L.o_H + 2 * (mm + 1) * mm;
  L.col = n * cw;  // doubles per column
  const size_t blk = static_cast<size_t>(L.col) * nrhs * 8;
  size_t off = 0;
  L.off_Z = off;
  off += align256(blk);
  L.off_Ro = off;
  off += align256(blk);
  L.off_X = off;
  off += align256(blk);
  if (L.cg) {
    L.off_R = off;
    off += align256(blk);
    L.off_P = off;
    off += align256(blk);
  } else {
    L.off_W = off;
    off += align256(blk);
    L.off_Q = off;
    off += align256(blk * (L.m + 1));
  }
  L.off_part = off;
  off += align256(static_cast<size_t>(nrhs) * L.nvmax * L.nchunk * 2 * 8);
  L.off_scal = off;
  off += align256(static_cast<size_t>(nrhs) * L.sc * 8);
  L.off_stat = off;
  off += align256(static_cast<size_t>(3 * nrhs) * 8);
  L.bytes = off;
  return L;
}

void KSolver::check_params(const h2_solve_params& p, bool cx) {
  if (p.method != H2_CG && p.method != H2_GMRES) throw Error(H2_EINVAL, "unknown method");
  if (cx && p.method != H2_GMRES) throw Error(H2_EINVAL, "complex systems need H2_GMRES");
  if (!(p.rtol > 0.0) || p.maxit < 1) throw Error(H2_EINVAL, "rtol must be > 0 and maxit >= 1");
  if (p.method == H2_GMRES && (p.restart < 1 || p.restart > kMaxRestart))
    throw Error(H2_EINVAL, "restart must be in [1, 120]");
  if (p.refine && !(p.inner_rtol > 0.0 && p.inner_rtol < 1.0)) throw Error(H2_EINVAL, "inner_rtol must be in (0, 1)");
}

KSolver::KSolver(int dtype, int64_t n, int nrhs, const h2_solve_params& p, void* workspace, size_t bytes,
                 double* host_status)
    : P(p) {
  if (dtype != H2_R64 && dtype != H2_C128) throw Error(H2_EINVAL, "Krylov vectors must be H2_R64 or H2_C128");
  if (n < 1 || nrhs < 1) throw Error(H2_EINVAL, "n and nrhs must be >= 1");
  if (nrhs > 65535) throw Error(H2_EINVAL, "at most 65535 right-hand sides");
  check_params(p, dtype == H2_C128);
  L = klayout(dtype, n, nrhs, p);
  if (!workspace || bytes < L.bytes) throw Error(H2_EINVAL, "workspace too small: need " + std::to_string(L.bytes));
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) throw Error(H2_EINVAL, "workspace must be 256-byte aligned");
  ws = static_cast<char*>(workspace);
  if (host_status) {
    stat_host = host_status;
  } else {
    H2_HIP(hipHostMalloc(reinterpret_cast<void**>(&own_stat), 3 * static_cast<size_t>(nrhs) * 8,
                         hipHostMallocDefault));
    stat_host = own_stat;
  }
  max_outer = P.refine ? 30 : 5;
}

KSolver::~KSolver() {
  if (own_stat) (void)hipHostFree(own_stat);
}

double* KSolver::d(size_t off) const { return reinterpret_cast<double*>(ws + off); }

namespace {
Geo geo_of(const KLayout& L) {
  Geo g;
  g.n = L.n;
  g.cw = L.cx ? 2 : 1;
  g.r = L.r;
  g.m = L.m;
  g.nchunk = L.nchunk;
  g.csz = L.csz;
  g.nvmax = L.nvmax;
  g.sc = L.sc;
  g.o_hcol = L.o_hcol;
  g.o_hcur = L.o_hcur;
  g.o_g = L.o_g;
  g.o_cs = L.o_cs;
  g.o_sn = L.o_sn;
  g.o_y = L.o_y;
  g.o_H = L.o_H;
  return g;
}
}  // namespace

void KSolver::finish(int op, int nvec, int j, hipStream_t st) {
  const Geo g = geo_of(L);
  if (L.cx)
    k_finish<true><<<L.r, 64, 0, st>>>(g, op, nvec, j, d(L.off_part), d(L.off_scal));
  else
    k_finish<false><<<L.r, 64, 0, st>>>(g, op, nvec, j, d(L.off_part), d(L.off_scal));
}

void KSolver::partial(int nvec, const double* A, int64_t a_col, int64_t a_vec, const double* B, int64_t b_col,
                      hipStream_t st) {
  const Geo g = geo_of(L);
  const dim3 grid(L.nchunk, L.r);
  if (L.cx)
    k_partial<true><<<grid, KT, 0, st>>>(g, nvec, A, a_col, a_vec, B, b_col, d(L.off_part));
  else
    k_partial<false><<<grid, KT, 0, st>>>(g, nvec, A, a_col, a_vec, B, b_col, d(L.off_part));
}

void KSolver::status_copy(hipStream_t st) {
  const Geo g = geo_of(L);
  k_status<<<(L.r + 63) / 64, 64, 0, st>>>(g, d(L.off_scal), d(L.off_stat));
  H2_HIP(hipMemcpyAsync(stat_host, d(L.off_stat), 3 * static_cast<size_t>(L.r) * 8, hipMemcpyDeviceToHost, st));
}

void KSolver::begin(const void* b, int64_t ldb, const void* z0, int64_t ldz, hipStream_t st) {
  const int cw = L.cx ? 2 : 1;
  if (!b) throw Error(H2_EINVAL, "b must not be NULL");
  if (ldb < L.n || (z0 && ldz < L.n)) throw Error(H2_EINVAL, "leading dimension smaller than n");
  B = static_cast<const double*>(b);
  b_col = ldb * cw;
  const Geo g = geo_of(L);
  const dim3 grid(L.nchunk, L.r);
  {
    const int64_t cnt = static_cast<int64_t>(L.r) * L.sc;
    k_fill0<<<static_cast<unsigned>(std::min<int64_t>(1024, (cnt + KT - 1) / KT)), KT, 0, st>>>(d(L.off_scal), cnt);
  }
  partial(1, B, b_col, 0, B, b_col, st);
  finish(OP_NB_OUT, 1, 0, st);
  iterations = outer = products = 0;
  inner_tol = 1.0;
  state = H2_KS_PRODUCT;
  message.clear();
  if (z0) {
    // Z = z0 (zero for b_c = 0); the first product forms the outer residual
    k_copy_masked<<<grid, KT, 0, st>>>(g, static_cast<const double*>(z0), ldz * cw, d(L.off_Z), L.col,
                                       d(L.off_scal));
    phase = PH_OUTER;
    pend_inner = pend_close = pend_zupd = false;
  } else {
    // Z = 0: the outer residual is B itself, relative residual 1 (0 for b_c = 0)
    k_zero<<<grid, KT, 0, st>>>(g, d(L.off_Z), L.col);
    rhs = B;
    rhs_col = b_col;
    ++outer;
    start_inner(1.0);
  }
  H2_HIP(hipGetLastError());
  status_copy(st);
}

void KSolver::start_inner(double rel_out_max) {
  inner_tol = P.refine ? std::max(P.inner_rtol, 0.5 * P.rtol / rel_out_max) : P.rtol / rel_out_max;
  inner_tol = std::min(inner_tol, 1.0);
  pend_inner = true;
  pend_close = pend_zupd = false;
  phase = L.cg ? PH_CG : PH_ARNOLDI;
  j = 0;
}

int KSolver::next(void* x, int64_t ldx, int* flags, hipStream_t st) {
  if (state != H2_KS_PRODUCT) return state;
  if (!x) {  // query: the flags of the next product, no device work
    const bool outer_next = pend_zupd || (phase == PH_OUTER && !pend_inner && !pend_close);
    if (flags) *flags = outer_next && P.refine ? H2_ACC_F64 : 0;
    return state;
  }
  const int cw = L.cx ? 2 : 1;
  if (ldx < L.n) throw Error(H2_EINVAL, "leading dimension smaller than n");
  const Geo g = geo_of(L);
  const dim3 grid(L.nchunk, L.r);
  const int64_t col = L.col, qcol = col * (L.m + 1);
  if (pend_inner) {
    pend_inner = false;
    if (L.cg) {
      k_cg_init<<<grid, KT, 0, st>>>(g, rhs, rhs_col, d(L.off_X), d(L.off_R), d(L.off_P), col, d(L.off_part));
      finish(OP_CG_INIT, 1, 0, st);
    } else {
      k_zero<<<grid, KT, 0, st>>>(g, d(L.off_X), col);
      partial(1, rhs, rhs_col, 0, rhs, rhs_col, st);
      finish(OP_GM_START, 1, 0, st);
      k_scale<<<grid, KT, 0, st>>>(g, rhs, rhs_col, d(L.off_Q), qcol, d(L.off_scal));
    }
  }
  if (pend_close) {
    pend_close = false;
    k_backsolve<<<(L.r + 63) / 64, 64, 0, st>>>(g, j, d(L.off_scal));
    if (L.cx)
      k_xupdate<true><<<grid, KT, 0, st>>>(g, j, d(L.off_Q), qcol, col, d(L.off_X), col, d(L.off_scal));
    else
      k_xupdate<false><<<grid, KT, 0, st>>>(g, j, d(L.off_Q), qcol, col, d(L.off_X), col, d(L.off_scal));
    phase = PH_RESID;
  }
  if (pend_zupd) {
    pend_zupd = false;
    k_add<<<grid, KT, 0, st>>>(g, d(L.off_X), col, d(L.off_Z), col);
    phase = PH_OUTER;
  }
  const double* src = nullptr;
  int64_t s_col = col;
  int fl = 0;
  switch (phase) {
    case PH_OUTER: src = d(L.off_Z); fl = P.refine ? H2_ACC_F64 : 0; break;
    case PH_CG: src = d(L.off_P); break;
    case PH_ARNOLDI: src = d(L.off_Q) + static_cast<int64_t>(j) * col; s_col = qcol; break;
    case PH_RESID: src = d(L.off_X); break;
  }
  k_copy_ld<<<grid, KT, 0, st>>>(g, src, s_col, static_cast<double*>(x), ldx * cw);
  H2_HIP(hipGetLastError());
  if (flags) *flags = fl;
  return state;
}

void KSolver::advance(const void* y, int64_t ldy, hipStream_t st) {
  if (state != H2_KS_PRODUCT) throw Error(H2_EINVAL, "the solve asked for no product");
  const int cw = L.cx ? 2 : 1;
  if (!y || ldy < L.n) throw Error(H2_EINVAL, "product missing or leading dimension smaller than n");
  const double* Y = static_cast<const double*>(y);
  const int64_t y_col = ldy * cw;
  const Geo g = geo_of(L);
  const dim3 grid(L.nchunk, L.r);
  const int64_t col = L.col, qcol = col * (L.m + 1);
  ++products;
  switch (phase) {
    case PH_OUTER:  // Ro = B - G~ Z
      k_resid<false><<<grid, KT, 0, st>>>(g, B, b_col, Y, y_col, d(L.off_Ro), col, d(L.off_part));
      finish(OP_REL_OUT, 1, 0, st);
      break;
    case PH_CG:
      partial(1, d(L.off_P), col, 0, Y, y_col, st);
      finish(OP_CG_ALPHA, 1, 0, st);
      k_cg_xr<<<grid, KT, 0, st>>>(g, d(L.off_P), Y, y_col, d(L.off_X), d(L.off_R), col, d(L.off_scal),
                                    d(L.off_part));
      finish(OP_CG_BETA, 1, 0, st);
      k_cg_p<<<grid, KT, 0, st>>>(g, d(L.off_R), d(L.off_P), col, d(L.off_scal));
      ++iterations;
      break;
    case PH_ARNOLDI: {
      // the cycle holds at most m steps: poll() closes it before a step would overrun Q
      if (j >= L.m) throw Error(H2_EINVAL, "h2_krylov_poll must follow every advance");
      // classical Gram-Schmidt, twice: h = Q^H y, w = y - Q h; h' = Q^H w, w -= Q h'
      const double* Q = d(L.off_Q);
      double* W = d(L.off_W);
      const int nv = j + 1;
      partial(nv, Q, qcol, col, Y, y_col, st);
      finish(OP_GM_H1, nv, j, st);
      if (L.cx)
        k_gs_update<true, false><<<grid, KT, 0, st>>>(g, nv, Q, qcol, col, Y, y_col, W, col, d(L.off_scal), nullptr);
      else
        k_gs_update<false, false><<<grid, KT, 0, st>>>(g, nv, Q, qcol, col, Y, y_col, W, col, d(L.off_scal), nullptr);
      partial(nv, Q, qcol, col, W, col, st);
      finish(OP_GM_H2, nv, j, st);
      if (L.cx)
        k_gs_update<true, true><<<grid, KT, 0, st>>>(g, nv, Q, qcol, col, W, col, W, col, d(L.off_scal),
                                                      d(L.off_part));
      else
        k_gs_update<false, true><<<grid, KT, 0, st>>>(g, nv, Q, qcol, col, W, col, W, col, d(L.off_scal),
                                                       d(L.off_part));
      finish(OP_GM_NORM, 1, j, st);
      k_scale<<<grid, KT, 0, st>>>(g, W, col, d(L.off_Q) + static_cast<int64_t>(j + 1) * col, qcol, d(L.off_scal));
      ++j;
      ++iterations;
      break;
    }
    case PH_RESID:  // inner residual of the cycle's end, then the restart vector
      k_resid<false><<<grid, KT, 0, st>>>(g, rhs, rhs_col, Y, y_col, d(L.off_W), col, d(L.off_part));
      finish(OP_GM_RESTART, 1, 0, st);
      k_scale<<<grid, KT, 0, st>>>(g, d(L.off_W), col, d(L.off_Q), qcol, d(L.off_scal));
      j = 0;
      break;
  }
  H2_HIP(hipGetLastError());
  status_copy(st);
}

int KSolver::poll() {
  if (state != H2_KS_PRODUCT) return state;
  const int r = L.r;
  double rel_out = 0.0, rel_in = 0.0, bad = 0.0;
  for (int c = 0; c < r; ++c) {
    const double a = stat_host[c], b = stat_host[r + c];
    rel_out = (std::isnan(a) || a > rel_out) ? a : rel_out;
    rel_in = (std::isnan(b) || b > rel_in) ? b : rel_in;
    if (bad == 0.0) bad = stat_host[2 * r + c];
  }
  if (bad != 0.0 || std::isnan(rel_out) || std::isnan(rel_in)) {
    state = H2_KS_FAILED;
    message = phase == PH_OUTER ? "non-finite outer residual" : "non-finite inner residual";
    message += " after " + std::to_string(iterations) + " iterations; ";
    message += bad == 1.0 ? "a product returned a non-finite entry" : "all products were finite";
    return state;
  }
  last_rel = phase == PH_OUTER ? rel_out : rel_in;
  switch (phase) {
    case PH_OUTER:  // the outer residual of the current Z decides
      if (rel_out <= P.rtol) {
        state = H2_KS_DONE;
      } else if (iterations >= P.maxit || outer >= max_outer) {
        state = H2_KS_NOTCONV;
      } else {
        rhs = d(L.off_Ro);
        rhs_col = L.col;
        ++outer;
        start_inner(rel_out);
      }
      break;
    case PH_CG:
      if (rel_in <= inner_tol || iterations >= P.maxit) pend_zupd = true;
      break;
    case PH_ARNOLDI:
      if (j >= L.m || rel_in <= inner_tol || iterations >= P.maxit) pend_close = true;
      break;
    case PH_RESID:
      if (rel_in <= inner_tol || iterations >= P.maxit) pend_zupd = true;
      else phase = PH_ARNOLDI;  // continue with the restart vector already in Q_0
      break;
  }
  return state;
}

void KSolver::residuals(double* out) const {
  for (int c = 0; c < L.r; ++c) out[c] = stat_host[c];
}

void KSolver::solution(void* z, int64_t ldz, hipStream_t st) {
  const int cw = L.cx ? 2 : 1;
  if (!z || ldz < L.n) throw Error(H2_EINVAL, "z missing or leading dimension smaller than n");
  const Geo g = geo_of(L);
  const dim3 grid(L.nchunk, L.r);
  k_copy_ld<<<grid, KT, 0, st>>>(g, d(L.off_Z), L.col, static_cast<double*>(z), ldz * cw);
  H2_HIP(hipGetLastError());
}

// ============================================================================ h2_solve
namespace {
void check_solve_args(const h2_handle_s& H, int nrhs, int dtype, const void* b, int64_t ldb, const void* z,
                      int64_t ldz, const h2_solve_params& p) {
  if (H.host_only) throw Error(H2_EINVAL, "handle was built with H2_HOST_ONLY");
  if (nrhs < 0) throw Error(H2_EINVAL, "nrhs must be >= 0");
  const bool cx = dtype == H2_C128;
  if (dtype != H2_R64 && dtype != H2_C128) throw Error(H2_EINVAL, "h2_solve takes H2_R64 or H2_C128 vectors");
  if (cx != H.is_complex)
    throw Error(H2_EINVAL, H.is_complex ? "the Helmholtz matrix needs complex vectors (H2_C128)"
                                        : "complex vectors need the Helmholtz kernel");
  KSolver::check_params(p, cx);
  if (nrhs == 0) return;
  if (!b || !z) throw Error(H2_EINVAL, "b and z must not be NULL");
  if (ldb < H.S.n || ldz < H.S.n) throw Error(H2_EINVAL, "leading dimension smaller than n");
}

// Device bytes of a solve: the solver's workspace plus the two n x nrhs product buffers
size_t solve_bytes(const h2_handle_s& H, int nrhs, int dtype, const h2_solve_params& p, size_t* vec) {
  const KLayout L = klayout(dtype, H.S.n, nrhs, p);
  *vec = align256(static_cast<size_t>(H.S.n) * nrhs * (dtype == H2_C128 ? 16 : 8));
  return L.bytes + 2 * *vec;
}

// The solve loop on a given workspace: one product per step, then the solver's decision.
int run_solve(h2_handle_s& H, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
              const h2_solve_params& p, h2_solve_info& info, hipStream_t st, char* ws, double* host_status,
              bool may_alloc) {
  const auto t0 = std::chrono::steady_clock::now();
  size_t vec = 0;
  const size_t need = solve_bytes(H, nrhs, dtype, p, &vec);
  const size_t kbytes = need - 2 * vec;
  void* X = ws + kbytes;
  void* Y = ws + kbytes + vec;
  KSolver K(dtype, H.S.n, nrhs, p, ws, kbytes, host_status);
  K.begin(b, ldb, z, ldz, st);
  int state = H2_KS_PRODUCT;
  while (true) {
    int flags = 0;
    state = K.next(X, H.S.n, &flags, st);
    if (state != H2_KS_PRODUCT) break;
    matvec(H, nrhs, dtype, X, H.S.n, Y, H.S.n, 1.0, flags | H2_OVERWRITE, st, may_alloc);
    K.advance(Y, H.S.n, st);
    H2_HIP(hipStreamSynchronize(st));
    state = K.poll();
    if (state != H2_KS_PRODUCT) break;
  }
  K.solution(z, ldz, st);
  H2_HIP(hipStreamSynchronize(st));
  info.iterations = K.iterations;
  info.outer = std::max(K.outer, 1);
  info.rel_residual = K.last_rel;
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (state == H2_KS_FAILED) throw Error(H2_ENOTCONV, K.message);
  return state == H2_KS_DONE ? H2_OK : H2_ENOTCONV;
}
}  // namespace

int solve_multi(h2_handle_s& H, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
                const h2_solve_params& p, h2_solve_info& info, hipStream_t st) {
  check_solve_args(H, nrhs, dtype, b, ldb, z, ldz, p);
  info = h2_solve_info{};
  if (nrhs == 0) return H2_OK;
  size_t vec = 0;
  // the handle keeps the solver's workspace between calls; it grows when a call needs more
  const size_t need = solve_bytes(H, nrhs, dtype, p, &vec);
  if (H.kws.bytes < need) {
    H2_HIP(hipStreamSynchronize(st));
    H.kws.alloc(need);
  }
  if (H.kstat_n < 3 * nrhs) {
    if (H.kstat) (void)hipHostFree(H.kstat);
    H.kstat = nullptr;
    H.kstat_n = 0;
    H2_HIP(hipHostMalloc(reinterpret_cast<void**>(&H.kstat), 3 * static_cast<size_t>(nrhs) * 8,
                         hipHostMallocDefault));
    H.kstat_n = 3 * nrhs;
  }
  return run_solve(H, nrhs, dtype, b, ldb, z, ldz, p, info, st, H.kws.as<char>(), H.kstat, true);
}

// ============================================================================ allocation-free h2_solve
// The solver's workspace and the product buffers live in one file-scope device
// array: each GPU holds its own copy from the time the library's code object is
// loaded on it until the process ends.  In host code `scratch` only names the
// symbol; its device address on the current GPU comes from hipGetSymbolAddress,
// looked up once per device and kept.
namespace {
constexpr size_t kScratchBytes = static_cast<size_t>(H2_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

char* scratch_on_current_device() {
  int dev = 0;
  H2_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(H2_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    H2_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(H2_EHIP, "no device address for the solver scratch");
    g_scratch_ptr[dev] = ptr;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}
}  // namespace

int solve_noalloc(h2_handle_s& H, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
                  const h2_solve_params& p, h2_solve_info& info, hipStream_t st) {
  check_solve_args(H, nrhs, dtype, b, ldb, z, ldz, p);
  info = h2_solve_info{};
  if (nrhs == 0) return H2_OK;
  if (nrhs > H2_NOALLOC_MAX_RHS)
    throw Error(H2_EINVAL, "h2_solve_noalloc takes at most " + std::to_string(H2_NOALLOC_MAX_RHS) +
                               " right-hand sides");
  size_t vec = 0;
  const size_t need = solve_bytes(H, nrhs, dtype, p, &vec);
  if (need > kScratchBytes)
    throw Error(H2_EINVAL, "the solve needs " + std::to_string(need) + " bytes of scratch; h2_solve_noalloc has " +
                               std::to_string(kScratchBytes));
  char* ws = scratch_on_current_device();
  double status[3 * H2_NOALLOC_MAX_RHS];  // pageable: read after the stream is synchronised
  return run_solve(H, nrhs, dtype, b, ldb, z, ldz, p, info, st, ws, status, false);
}

}  // namespace h2

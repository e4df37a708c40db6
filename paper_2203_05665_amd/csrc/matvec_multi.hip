// Many right-hand sides: y <- y + alpha G~ X for an n x R block X (FP32 storage,
// k = 64).  The phases are those of the single-vector product (Algorithms 1-3);
// with R columns each step becomes a small dense contraction, evaluated on the
// matrix cores with v_mfma_f32_32x32x2f32 -- except the transfers of handles with
// Kronecker factors, which apply the three 4 x 4 factors per column in registers
// (12 multiply-adds per coefficient instead of 64).
//
// Internal layouts (RP = 32 or 64 right-hand sides per pass, zero-padded):
//   x_c, y_c   [n][RP]        position-major, right-hand sides contiguous
//   x^, y^     [N_c][RP][k]   per cluster, the k coefficients of one right-hand
//                             side contiguous
// One wave or one workgroup owns one output block (a row cluster or a group of
// four, a leaf, a transfer target) and computes all of it, so every input
// element is loaded once per block: the coupling and the leaf forward on 32 x 32
// tiles, the near field on 16 x 16 tiles (two waves per leaf), the Kronecker
// transfers with four waves per cluster.  Rows, leaves and clusters are dealt to
// the eight XCDs in contiguous chunks, so neighbouring ones, which share most of
// their column clusters, share an L2.  Every output element has one owner: no
// atomics.
//
// MFMA operand convention (K = 64 per call, split across lane halves): in each
// step lanes 0-31 supply A[i][kk] and B[kk][j] for one kk of the first half of K
// and lanes 32-63 those for one kk of the second half, i = j = lane % 32.
// The 32 x 32 accumulator holds D[i][j] in register v of lane l with
// j = l % 32, i = (v % 4) + 4 (l / 32) + 8 (v / 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <vector>

#include "handle.h"
#include "otf_math.h"

namespace h2 {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ inline f32x16 mfma(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ inline int acc_row(int v, int l) { return (v % 4) + 4 * (l / 32) + 8 * (v / 4); }

__device__ inline f4v ld4c(const float* p) { return *reinterpret_cast<const f4v*>(p); }

// acc[ti][tj] += A(rows 32ti.., 64) * B(64, cols 32tj..) for ti < 2, tj < NT.
// A row-major 64 x 64 (row stride 64); Bt right-hand-side-major (element (kk, j)
// at Bt[j * 64 + kk]).  In step (p, e) lane half h covers kk = 8 p + 4 h + e, so
// the two lanes of a row read 32 contiguous bytes and the four steps p of one
// half-block consume whole 128-byte lines back to back (cached loads: the lines
// are reused by the next instructions, not streamed past).
template <int NT>
__device__ inline void mma64_rowA(const float* __restrict__ A, const float* __restrict__ Bt, f32x16 (&acc)[2][NT]) {
  const int l = threadIdx.x % 64, r = l % 32, h = l / 32;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    f4v a[2][4], b[NT][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = 8 * (4 * half + q) + 4 * h;
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) a[ti][q] = ld4c(A + (32 * ti + r) * 64 + kk);
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) b[tj][q] = ld4c(Bt + (32 * tj + r) * 64 + kk);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = mfma(a[ti][q][e], b[tj][q][e], acc[ti][tj]);
  }
}

template <int NT>
__device__ inline void zero(f32x16 (&acc)[2][NT]) {
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[ti][tj][v] = 0.f;
}

// out (right-hand-side-major k-vectors, element (nu, j) at out[j * 64 + nu]) = / += acc
template <int NT, bool ADD>
__device__ inline void store_hat(float* __restrict__ out, const f32x16 (&acc)[2][NT]) {
  const int l = threadIdx.x % 64;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float* p = out + (32 * tj + l % 32) * 64 + 32 * ti + acc_row(v, l);
        if (ADD) *p += acc[ti][tj][v]; else *p = acc[ti][tj][v];
      }
}

// the output block of wave `g` when row blocks are dealt to the XCDs in
// contiguous chunks (workgroups are dispatched round-robin over 8 XCDs).  The
// value is wave-uniform and is returned as such (readfirstlane), so everything
// derived from it stays in scalar registers.  Item counts stay below 2^31.
__device__ inline int64_t xcd_item(int64_t items) {
  const int64_t nwg = gridDim.x;
  const int64_t per = (nwg + 7) / 8;
  const int64_t wg = static_cast<int64_t>(blockIdx.x % 8) * per + blockIdx.x / 8;
  return __builtin_amdgcn_readfirstlane(static_cast<int>(wg * 4 + threadIdx.x / 64));  // 4 waves per workgroup
}

// item of a per-cluster workgroup: the grid (a multiple of 8 workgroups) in eight
// chunks of consecutive items, one per XCD, so neighbouring clusters (siblings) share an L2
__device__ inline int64_t xcd_group_item() {
  const int64_t per = gridDim.x / 8;
  return static_cast<int64_t>(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// ---------------------------------------------------------------- permutations
// User order (column-major, leading dimension ld) <-> cluster order
// (position-major, RP columns), through an LDS tile of 64 user indices x RP
// columns per workgroup, walked in user order: the user side reads or writes 64
// consecutive indices of a column (one contiguous run per wave), the cluster side
// one whole RP-column row per position, iperm[i] being the position of user
// index i (a contiguous run of RP floats).  Both sides move whole cache lines,
// so no line is fetched twice.  The tile's odd row pitch keeps both LDS passes
// free of bank conflicts.  Columns rcur..RP-1 of the cluster-order rows are 0.
template <typename XT, int RP>
__global__ __launch_bounds__(256) void mpermute_in(int64_t n, int rcur, const int32_t* __restrict__ iperm,
                                                   const XT* __restrict__ x, int64_t ldx, float* __restrict__ xc) {
  constexpr int PER = 64 * RP / 256;  // elements per thread and pass
  __shared__ float tile[64][RP + 1];
  __shared__ int32_t pos[64];
  const int t = threadIdx.x;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int32_t ip = iperm[min(i0 + t % 64, n - 1)];  // every wave loads the tile's positions
  // all loads first (out-of-range elements read x[0] and are replaced by 0)
  XT v[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int j = (t + 256 * s) / 64, il = t % 64;
    const bool ok = j < rcur && i0 + il < n;
    v[s] = x[ok ? static_cast<int64_t>(j) * ldx + i0 + il : 0];
    v[s] = ok ? v[s] : XT(0);
  }
  if (t < 64) pos[t] = i0 + t < n ? ip : 0;
#pragma unroll
  for (int s = 0; s < PER; ++s) tile[t % 64][(t + 256 * s) / 64] = static_cast<float>(v[s]);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int il = (t + 256 * s) / RP, j = (t + 256 * s) % RP;
    if (i0 + il < n) xc[static_cast<int64_t>(pos[il]) * RP + j] = tile[il][j];
  }
}

template <typename XT, int RP>
__global__ __launch_bounds__(256) void mpermute_out(int64_t n, int rcur, const int32_t* __restrict__ iperm,
                                                    const float* __restrict__ yc, XT* __restrict__ y, int64_t ldy,
                                                    double alpha, bool ow) {
  constexpr int PER = 64 * RP / 256;
  __shared__ float tile[64][RP + 1];
  __shared__ int32_t pos[64];
  const int t = threadIdx.x;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int32_t ip = iperm[min(i0 + t % 64, n - 1)];  // every wave loads the tile's positions
  // the user-side operand of the update, loaded while the positions arrive
  XT y0[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int j = (t + 256 * s) / 64, il = t % 64;
    const bool ok = !ow && j < rcur && i0 + il < n;
    y0[s] = y[ok ? static_cast<int64_t>(j) * ldy + i0 + il : 0];
    y0[s] = ok ? y0[s] : XT(0);
  }
  if (t < 64) pos[t] = i0 + t < n ? ip : 0;
  __syncthreads();
  float v[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int il = (t + 256 * s) / RP, j = (t + 256 * s) % RP;
    v[s] = yc[static_cast<int64_t>(pos[il]) * RP + j];  // pos = 0 past n: a valid row
  }
#pragma unroll
  for (int s = 0; s < PER; ++s) tile[(t + 256 * s) / RP][(t + 256 * s) % RP] = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int j = (t + 256 * s) / 64, il = t % 64;
    if (j < rcur && i0 + il < n)
      y[static_cast<int64_t>(j) * ldy + i0 + il] =
          static_cast<XT>(static_cast<double>(y0[s]) + alpha * static_cast<double>(tile[il][j]));
  }
}

// ---------------------------------------------------------------- phases (one wave per output block)
// x^_sigma = V_sigma^T X|sigma (Alg. 1) for every leaf (at most 64 triangles):
// one workgroup per leaf.  The leaf's r x 64 block of V and r x RP block of X
// are contiguous; they are moved to LDS with coalesced 16-byte loads (rows past r
// as zeros), wave (ti, tj) forms the 32 x 32 tile D(nu, j) = sum_p V[p][nu] X[p][j]
// (nu = 32 ti.., j = 32 tj..) with v_mfma_f32_32x32x2f32 straight from LDS (lane
// l takes p = 2 s + l / 32; the pitch of 96 floats puts the two rows of a step in
// different bank halves), and the tile leaves through LDS again as coalesced
// 16-byte stores of the RP x 64 output.
constexpr int kLeafPitch = 96;
constexpr int kOutPitch = 68;

template <int NT>
__global__ __launch_bounds__(256) void mleaf_forward(int nleaves, const int32_t* __restrict__ leaves,
                                                     const int32_t* __restrict__ cbegin,
                                                     const int32_t* __restrict__ cend, const float* __restrict__ Vf,
                                                     const float* __restrict__ xc, float* __restrict__ xhat) {
  constexpr int RP = 32 * NT;
  __shared__ __align__(16) float lds[2 * 64 * kLeafPitch];
  float* vs = lds;
  float* xs = lds + 64 * kLeafPitch;
  const int64_t it = xcd_group_item();
  if (it >= nleaves) return;  // whole workgroup
  const int t = threadIdx.x;
  const int32_t c = __builtin_amdgcn_readfirstlane(leaves[it]);
  const int64_t b0 = __builtin_amdgcn_readfirstlane(cbegin[c]);
  const int r = __builtin_amdgcn_readfirstlane(cend[c]) - static_cast<int>(b0);
  f4v va[4], xa[RP / 16];
  const f4v z4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int f = 4 * (q * 256 + t);
    va[q] = f / 64 < r ? ld4c(Vf + b0 * 64 + f) : z4;
  }
#pragma unroll
  for (int q = 0; q < RP / 16; ++q) {
    const int f = 4 * (q * 256 + t);
    xa[q] = f / RP < r ? ld4c(xc + b0 * RP + f) : z4;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int f = 4 * (q * 256 + t);
    *reinterpret_cast<f4v*>(vs + (f / 64) * kLeafPitch + f % 64) = va[q];
  }
#pragma unroll
  for (int q = 0; q < RP / 16; ++q) {
    const int f = 4 * (q * 256 + t);
    *reinterpret_cast<f4v*>(xs + (f / RP) * kLeafPitch + f % RP) = xa[q];
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(t / 64), l = t % 64;
  const int ti = wave >> 1, tj = wave & 1;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  if (tj < NT) {
    const float* a = vs + (l / 32) * kLeafPitch + 32 * ti + l % 32;
    const float* b = xs + (l / 32) * kLeafPitch + 32 * tj + l % 32;
    const int steps = (r + 1) / 2;  // row r, if read, is zero
    for (int s = 0; s < steps; ++s) acc = mfma(a[2 * s * kLeafPitch], b[2 * s * kLeafPitch], acc);
  }
  __syncthreads();  // the operands' space is reused for the output tile
  float* os = lds;  // os[j][nu], pitch kOutPitch
  if (tj < NT) {
#pragma unroll
    for (int v = 0; v < 16; ++v) os[(32 * tj + l % 32) * kOutPitch + 32 * ti + acc_row(v, l)] = acc[v];
  }
  __syncthreads();
  float* dst = xhat + static_cast<int64_t>(c) * RP * 64;
#pragma unroll
  for (int q = 0; q < RP / 16; ++q) {
    const int f = 4 * (q * 256 + t);
    *reinterpret_cast<f4v*>(dst + f) = *reinterpret_cast<const f4v*>(os + (f / 64) * kOutPitch + f % 64);
  }
}

// x^_sigma = sum_children F^T x^_child; A(nu, nu') = ET[nu][nu'] (row-major)
template <int NT>
__global__ __launch_bounds__(256) void mtransfer_up(int count, const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ child0,
                                                    const int32_t* __restrict__ child1, const float* __restrict__ ET,
                                                    float* __restrict__ xhat) {
  const int64_t it = xcd_item(count);
  if (it >= count) return;
  constexpr int RP = 32 * NT;
  const int32_t c = list[it];
  f32x16 acc[2][NT];
  zero(acc);
  mma64_rowA<NT>(ET + static_cast<int64_t>(child0[c]) * 4096, xhat + static_cast<int64_t>(child0[c]) * RP * 64, acc);
  mma64_rowA<NT>(ET + static_cast<int64_t>(child1[c]) * 4096, xhat + static_cast<int64_t>(child1[c]) * RP * 64, acc);
  store_hat<NT, false>(xhat + static_cast<int64_t>(c) * RP * 64, acc);
}

// y^_tau = sum_{(tau,sigma) admissible} S_{tau sigma} x^_sigma (assigns)
template <int NT>
__global__ __launch_bounds__(256) void mcoupling(int64_t nitems, const int32_t* __restrict__ order,
                                                 const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col, const float* __restrict__ S,
                                                 const float* __restrict__ xhat, float* __restrict__ yhat) {
  const int64_t it = xcd_item(nitems);
  if (it >= nitems) return;
  const int64_t tau = order[it];
  if (tau < 0) return;
  constexpr int RP = 32 * NT;
  f32x16 acc[2][NT];
  zero(acc);
  const int64_t b1 = ptr[tau + 1];
  for (int64_t b = ptr[tau]; b < b1; ++b)
    mma64_rowA<NT>(S + b * 4096, xhat + static_cast<int64_t>(col[b]) * RP * 64, acc);
  store_hat<NT, false>(yhat + tau * RP * 64, acc);
}

// y^_tau = sum_sigma S_{tau sigma} x^_sigma for four row clusters per workgroup
// (64 right-hand sides), so that x^_sigma, which the rows of a group share, is
// read from HBM once per group instead of once per row.  A group is usually the
// four grandchildren of one cluster: neighbours whose admissible lists overlap
// (Algorithm 3 visits the same sigma from each of them).  Its work is the union
// of the four lists, ordered by column cluster; an entry holds sigma and the block
// S_{tau sigma} of each slot (-1 where tau does not meet sigma), so every row meets
// its blocks in the order of its own list.  Each (entry, slot) with a block is a
// task: the workgroup stages S_{tau sigma} (and x^_sigma when sigma changes) into
// LDS with contiguous 16-byte loads, one task ahead, and each wave multiplies its
// 32 x 32 tile (rows 32 ti of S, right-hand sides 32 tj) into that slot's
// accumulator: the four waves share every task, so none waits for a row it does
// not own.  The K order per block is that of mma64_rowA, so every tile sums the
// same products in the same order as mcoupling.
constexpr int kGrpPitch = 68;  // LDS row pitch in floats: 16-byte reads of 16 lanes cover all 64 banks

__device__ inline void mma_tile_k64(const float* __restrict__ As, const float* __restrict__ Bs, f32x16& acc) {
  f4v a[8], b[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    a[p] = *reinterpret_cast<const f4v*>(As + 8 * p);
    b[p] = *reinterpret_cast<const f4v*>(Bs + 8 * p);
  }
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc = mfma(a[p][e], b[p][e], acc);
}

// LDS holds one S block and one x^_sigma (34 KB) and a lane at most 128
// registers, so four workgroups share a CU: while one waits at its barriers or
// for its staged loads, the others multiply.  Per task the next operands are
// loaded into registers before the multiplies and written to LDS between two
// barriers after them.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mcoupling_grp(
    int64_t ngroups, const int32_t* __restrict__ grows, const int64_t* __restrict__ gent,
    const int32_t* __restrict__ ents, const float* __restrict__ S, const float* __restrict__ xhat,
    float* __restrict__ yhat) {
  constexpr int RP = 64;
  __shared__ __align__(16) float sbuf[64 * kGrpPitch];
  __shared__ __align__(16) float xbuf[64 * kGrpPitch];
  const int64_t per = gridDim.x / 8;  // groups per XCD chunk (the grid is 8 chunks)
  const int64_t g = static_cast<int64_t>(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (g >= ngroups) return;  // whole workgroup
  const int t = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(t / 64), l = t % 64, r = l % 32, h = l / 32;
  const int ti = wave >> 1, tj = wave & 1;
  const int64_t e0 = gent[g], e1 = gent[g + 1];
  f32x16 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
  // staging: 16 KB tiles (64 rows of 64 floats), thread t moves vectors q 256 + t
  f4v sreg[4], xreg[4];
  auto fetch = [&](const float* src, f4v(&reg)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) reg[q] = ld4c(src + (q * 256 + t) * 4);
  };
  // S is read once per pass: non-temporal loads keep it from displacing the x^
  // tiles that other groups re-read from L2 (fetched bytes 1.46 -> 1.37 x S)
  auto fetch_s = [&](const float* src, f4v(&reg)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) reg[q] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(src + (q * 256 + t) * 4));
  };
  auto put = [&](float* dst, const f4v(&reg)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = (q * 256 + t) * 4;
      *reinterpret_cast<f4v*>(dst + (f / 64) * kGrpPitch + f % 64) = reg[q];
    }
  };
  // entry e: ents[8 e] = sigma, ents[8 e + 1 + i] = block of slot i or -1
  auto first_block = [&](int64_t e) {
    const int32_t* en = ents + 8 * e;
    return en[1] >= 0 ? en[1] : en[2] >= 0 ? en[2] : en[3] >= 0 ? en[3] : en[4];
  };
  if (e0 < e1) {
    fetch_s(S + static_cast<int64_t>(first_block(e0)) * 4096, sreg);
    fetch(xhat + static_cast<int64_t>(ents[8 * e0]) * RP * 64, xreg);
    put(sbuf, sreg);
    put(xbuf, xreg);
  }
  __syncthreads();
  for (int64_t e = e0; e < e1; ++e) {
    const int32_t* en = ents + 8 * e;
    const int32_t blk[4] = {en[1], en[2], en[3], en[4]};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (blk[i] >= 0) {
        // the next task: a later slot of this entry, else the first of the next entry
        int32_t nb = -1;
#pragma unroll
        for (int j = 3; j > i; --j)
          if (blk[j] >= 0) nb = blk[j];
        const bool newx = nb < 0 && e + 1 < e1;
        if (newx) nb = first_block(e + 1);
        if (nb >= 0) fetch_s(S + static_cast<int64_t>(nb) * 4096, sreg);
        if (newx) fetch(xhat + static_cast<int64_t>(ents[8 * e + 8]) * RP * 64, xreg);
        mma_tile_k64(sbuf + (32 * ti + r) * kGrpPitch + 4 * h, xbuf + (32 * tj + r) * kGrpPitch + 4 * h, acc[i]);
        __syncthreads();  // every wave is done with this task's operands
        if (nb >= 0) put(sbuf, sreg);
        if (newx) put(xbuf, xreg);
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int32_t tau = grows[4 * g + i];
    if (tau >= 0) {
      float* out = yhat + static_cast<int64_t>(tau) * RP * 64;
#pragma unroll
      for (int v = 0; v < 16; ++v) out[(32 * tj + r) * 64 + 32 * ti + acc_row(v, l)] = acc[i][v];
    }
  }
}

// The same with S evaluated on the fly (eq. coupling): every lane computes the
// A-operand entries it feeds to the matrix cores instead of loading them, in the
// K order of mma64_rowA (kk = 8 P + 4 h + e, P = 0..7): column point
// mu = (e, (2 P + h) % 4, P / 2); rows nu = 32 ti + r = (r % 4, (r / 4) % 4,
// 2 ti + r / 16).  Point differences are (c_tau - c_sigma) + (o_tau - o_sigma)
// with FP64 centres and FP32 offsets, as in the single-vector kernel.
template <int NT, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mcoupling_otf(
    int64_t nitems, const int32_t* __restrict__ order, const int64_t* __restrict__ ptr,
    const int32_t* __restrict__ col, const double* __restrict__ ctr, const float* __restrict__ off,
    const float* __restrict__ xhat, float* __restrict__ yhat) {
  const int64_t it = xcd_item(nitems);
  if (it >= nitems) return;
  const int64_t tau = order[it];
  if (tau < 0) return;
  constexpr int RP = 32 * NT;
  const int l = threadIdx.x % 64, r = l % 32, h = l / 32;
  const float* ot = off + tau * 12;
  const float ax = ot[r % 4], ay = ot[4 + (r / 4) % 4];
  const float az[2] = {ot[8 + r / 16], ot[10 + r / 16]};
  const double cx = ctr[3 * tau], cy = ctr[3 * tau + 1], cz = ctr[3 * tau + 2];
  f32x16 acc[2][NT];
  zero(acc);
  const int64_t b1 = ptr[tau + 1];
  for (int64_t b = ptr[tau]; b < b1; ++b) {
    const int64_t s = col[b];
    const float* os = off + s * 12;
    // per-axis parts: x by e, y by P & 1, z by (ti, P >> 1)
    float px[4], py[2], pz[2][4];
    if (KIND == H2_LAPLACE) {
      const float ex = static_cast<float>(cx - ctr[3 * s]) + ax, ey = static_cast<float>(cy - ctr[3 * s + 1]) + ay;
      const float dcz = static_cast<float>(cz - ctr[3 * s + 2]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float d = ex - os[e];
        px[e] = d * d;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float d = ey - os[4 + 2 * j + h];
        py[j] = d * d;
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int z = 0; z < 4; ++z) {
          const float d = (dcz + az[ti]) - os[8 + z];
          pz[ti][z] = d * d;
        }
    } else {  // polynomial test kernels: parts of x . y on absolute coordinates
      const float x0 = static_cast<float>(cx) + ax, x1 = static_cast<float>(cy) + ay;
      const float sx = static_cast<float>(ctr[3 * s]), sy = static_cast<float>(ctr[3 * s + 1]),
                  sz = static_cast<float>(ctr[3 * s + 2]);
#pragma unroll
      for (int e = 0; e < 4; ++e) px[e] = x0 * (sx + os[e]);
#pragma unroll
      for (int j = 0; j < 2; ++j) py[j] = x1 * (sy + os[4 + 2 * j + h]);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int z = 0; z < 4; ++z) pz[ti][z] = (static_cast<float>(cz) + az[ti]) * (sz + os[8 + z]);
    }
    const float* Bt = xhat + s * RP * 64;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      f4v bv[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) bv[tj][q] = ld4c(Bt + (32 * tj + r) * 64 + 8 * (4 * half + q) + 4 * h);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int P = 4 * half + q;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float a[2];
#pragma unroll
          for (int ti = 0; ti < 2; ++ti) {
            const float t = px[e] + (py[P & 1] + pz[ti][P >> 1]);
            a[ti] = KIND == H2_LAPLACE ? __builtin_amdgcn_rsqf(t)
                    : KIND == H2_TEST_ONE ? 1.f
                    : KIND == H2_TEST_BILINEAR ? t : t * t;
          }
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = mfma(a[ti], bv[tj][q][e], acc[ti][tj]);
        }
      }
    }
  }
  if (KIND == H2_LAPLACE) {
    const float scale = static_cast<float>(1.0 / (4.0 * 3.14159265358979323846));
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < NT; ++tj) acc[ti][tj] *= scale;
  }
  store_hat<NT, false>(yhat + tau * RP * 64, acc);
}

// y^_c += E_c y^_parent for the clusters of one level; A(nu', nu) = F[nu'][nu]
template <int NT>
__global__ __launch_bounds__(256) void mtransfer_down(int first, int count, const int32_t* __restrict__ parent,
                                                      const float* __restrict__ F, float* __restrict__ yhat) {
  const int64_t it = xcd_item(count);
  if (it >= count) return;
  constexpr int RP = 32 * NT;
  const int64_t c = first + it;
  f32x16 acc[2][NT];
  zero(acc);
  mma64_rowA<NT>(F + c * 4096, yhat + static_cast<int64_t>(parent[c]) * RP * 64, acc);
  store_hat<NT, true>(yhat + c * RP * 64, acc);
}

// Kronecker form of the two transfers (k = 64, interpolation bases):
// E_c = E_x (x) E_y (x) E_z with E1[c][d][i][j] = l_j(xi_i) along axis d (i child
// point, j parent polynomial), nu = nu_x + 4 nu_y + 16 nu_z.  A transfer reads 48
// factor numbers instead of a dense 64 x 64 E and takes 12 multiply-adds per
// coefficient instead of 64: it is bound by the x^ / y^ tiles it moves.
// One group of four waves per cluster.  The RP x 64 tile (RP columns of 64
// coefficients) is moved between HBM and LDS with coalesced 16-byte accesses
// (1 KB per wave instruction).  In LDS, lane j of wave w first takes the plane
// nu_z = w of column j (16 coefficients, register-local x and y steps), then,
// after a barrier, the coefficients with nu_y = w (the z step); every wave
// writes back only what it read in that step, so three barriers order a
// transfer.  The factor entries are wave-uniform scalar loads.
constexpr int kTilePitch = 68;                   // LDS row pitch of a tile (floats)
constexpr int kTileFloats = 64 * kTilePitch;     // one tile, up to 64 columns

// a(o, i) = E_d[i][o] (up: transposed) or E_d[o][i] (down)
template <bool TRANSPOSE>
__device__ inline float kfac(const float* __restrict__ e, int o, int i) {
  return e[TRANSPOSE ? 4 * i + o : 4 * o + i];
}

// x and y steps on one plane in place: v[q], q = nu_x + 4 nu_y
template <bool TRANSPOSE>
__device__ inline void kron_xy(float (&v)[16], const float* __restrict__ e) {
#pragma unroll
  for (int line = 0; line < 4; ++line) {  // x: the four nu_x of one nu_y
    float t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = v[4 * line + i];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float r = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) r += kfac<TRANSPOSE>(e, o, i) * t[i];
      v[4 * line + o] = r;
    }
  }
#pragma unroll
  for (int line = 0; line < 4; ++line) {  // y: the four nu_y of one nu_x
    float t[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = v[line + 4 * i];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float r = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) r += kfac<TRANSPOSE>(e + 16, o, i) * t[i];
      v[line + 4 * o] = r;
    }
  }
}

// z step of the coefficients with nu_y = w: out[o][x] = sum_z a_z(o, z) u[z][x]
// with u[z][x] = tile[j][x + 4 w + 16 z]; ADD: out accumulates
template <bool TRANSPOSE, bool ADD>
__device__ inline void kron_z(const float* __restrict__ row, int w, const float* __restrict__ e, float (&out)[4][4]) {
  float u[4][4];
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    const f4v t = *reinterpret_cast<const f4v*>(row + 4 * w + 16 * z);
    u[z][0] = t.x;
    u[z][1] = t.y;
    u[z][2] = t.z;
    u[z][3] = t.w;
  }
#pragma unroll
  for (int o = 0; o < 4; ++o)
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      float r = 0.f;
#pragma unroll
      for (int z = 0; z < 4; ++z) r += kfac<TRANSPOSE>(e + 32, o, z) * u[z][x];
      out[o][x] = ADD ? out[o][x] + r : r;
    }
}

// tile (RP rows of 64 floats at src) -> LDS rows of pitch kTilePitch; g = thread of the group
template <int RP>
__device__ inline void tile_to_lds(const float* __restrict__ src, float* __restrict__ t, int g) {
#pragma unroll
  for (int s = 0; s < RP / 16; ++s) {
    const int e = 4 * (g + 256 * s);
    *reinterpret_cast<f4v*>(t + (e / 64) * kTilePitch + e % 64) = ld4c(src + e);
  }
}

__device__ inline void plane_load(const float* __restrict__ row, int w, float (&v)[16]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f4v t = *reinterpret_cast<const f4v*>(row + 16 * w + 4 * q);
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
}

__device__ inline void plane_store(float* __restrict__ row, int w, const float (&v)[16]) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    *reinterpret_cast<f4v*>(row + 16 * w + 4 * q) = f4v{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
}

__device__ inline void zrow_store(float* __restrict__ row, int w, const float (&o)[4][4]) {
#pragma unroll
  for (int z = 0; z < 4; ++z) *reinterpret_cast<f4v*>(row + 4 * w + 16 * z) = f4v{o[z][0], o[z][1], o[z][2], o[z][3]};
}

// x^_c = E_c0^T x^_c0 + E_c1^T x^_c1 by the group of threads g = 0..255 with the LDS
// tiles t (two); c < 0: the group only takes part in the barriers
template <int NT>
__device__ inline void kup_group(int64_t c, int g, const int32_t* __restrict__ child0, const int32_t* __restrict__ child1,
                                 const float* __restrict__ E1, float* __restrict__ xhat, float* __restrict__ t) {
  constexpr int RP = 32 * NT;
  const int w = g / 64, j = g % 64;
  int64_t ch[2] = {0, 0};
  if (c >= 0) {
    ch[0] = __builtin_amdgcn_readfirstlane(child0[c]);
    ch[1] = __builtin_amdgcn_readfirstlane(child1[c]);
    tile_to_lds<RP>(xhat + ch[0] * RP * 64, t, g);
    tile_to_lds<RP>(xhat + ch[1] * RP * 64, t + kTileFloats, g);
  }
  __syncthreads();
  if (c >= 0 && j < RP) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      float v[16];
      float* row = t + a * kTileFloats + j * kTilePitch;
      plane_load(row, w, v);
      kron_xy<true>(v, E1 + ch[a] * 48);
      plane_store(row, w, v);
    }
  }
  __syncthreads();
  if (c >= 0 && j < RP) {
    float acc[4][4];
    kron_z<true, false>(t + j * kTilePitch, w, E1 + ch[0] * 48, acc);
    kron_z<true, true>(t + kTileFloats + j * kTilePitch, w, E1 + ch[1] * 48, acc);
    zrow_store(t + j * kTilePitch, w, acc);
  }
  __syncthreads();
  if (c >= 0) {
    float* dst = xhat + c * RP * 64;
#pragma unroll
    for (int s = 0; s < RP / 16; ++s) {
      const int e = 4 * (g + 256 * s);
      *reinterpret_cast<f4v*>(dst + e) = *reinterpret_cast<const f4v*>(t + (e / 64) * kTilePitch + e % 64);
    }
  }
}

// y^_c += E_c y^_parent(c), likewise (one LDS tile)
template <int NT>
__device__ inline void kdown_group(int64_t c, int g, const int32_t* __restrict__ parent, const float* __restrict__ E1,
                                   float* __restrict__ yhat, float* __restrict__ t) {
  constexpr int RP = 32 * NT;
  const int w = g / 64, j = g % 64;
  f4v own[RP / 16];
  if (c >= 0) {
    const int64_t p = __builtin_amdgcn_readfirstlane(parent[c]);
#pragma unroll
    for (int s = 0; s < RP / 16; ++s) own[s] = ld4c(yhat + c * RP * 64 + 4 * (g + 256 * s));
    tile_to_lds<RP>(yhat + p * RP * 64, t, g);
  }
  __syncthreads();
  if (c >= 0 && j < RP) {
    float v[16];
    float* row = t + j * kTilePitch;
    plane_load(row, w, v);
    kron_xy<false>(v, E1 + c * 48);
    plane_store(row, w, v);
  }
  __syncthreads();
  if (c >= 0 && j < RP) {
    float out[4][4];
    float* row = t + j * kTilePitch;
    kron_z<false, false>(row, w, E1 + c * 48, out);
    zrow_store(row, w, out);
  }
  __syncthreads();
  if (c >= 0) {
    float* dst = yhat + c * RP * 64;
#pragma unroll
    for (int s = 0; s < RP / 16; ++s) {
      const int e = 4 * (g + 256 * s);
      const f4v d = *reinterpret_cast<const f4v*>(t + (e / 64) * kTilePitch + e % 64);
      *reinterpret_cast<f4v*>(dst + e) = own[s] + d;
    }
  }
}

// the parents of one level, one workgroup each
template <int NT>
__global__ __launch_bounds__(256) void mtransfer_up_kron(int count, const int32_t* __restrict__ list,
                                                         const int32_t* __restrict__ child0,
                                                         const int32_t* __restrict__ child1,
                                                         const float* __restrict__ E1, float* __restrict__ xhat) {
  __shared__ __attribute__((aligned(16))) float t[2 * kTileFloats];
  const int64_t it = xcd_group_item();
  if (it >= count) return;  // uniform per workgroup
  kup_group<NT>(__builtin_amdgcn_readfirstlane(list[it]), threadIdx.x, child0, child1, E1, xhat, t);
}

// the clusters of one level, one workgroup each
template <int NT>
__global__ __launch_bounds__(256) void mtransfer_down_kron(int first, int count, const int32_t* __restrict__ parent,
                                                           const float* __restrict__ E1, float* __restrict__ yhat) {
  __shared__ __attribute__((aligned(16))) float t[kTileFloats];
  const int64_t it = xcd_group_item();
  if (it >= count) return;
  kdown_group<NT>(first + it, threadIdx.x, parent, E1, yhat, t);
}

// The top levels (few clusters each) in one workgroup of kMTopGroups groups, level
// by level; a level's clusters are taken kMTopGroups at a time, and the barriers
// inside a transfer and after it also order the levels (a level reads the tiles
// the previous one wrote).
constexpr int kMTopGroups = 4;

template <int NT>
__global__ __launch_bounds__(256 * kMTopGroups) void mtransfer_up_kron_top(
    int nlev, const int64_t* __restrict__ lev, const int32_t* __restrict__ list, const int32_t* __restrict__ child0,
    const int32_t* __restrict__ child1, const float* __restrict__ E1, float* __restrict__ xhat) {
  __shared__ __attribute__((aligned(16))) float t[kMTopGroups * 2 * kTileFloats];
  const int grp = threadIdx.x / 256, g = threadIdx.x % 256;
  for (int l = nlev - 1; l >= 0; --l)
    for (int64_t w0 = lev[l]; w0 < lev[l + 1]; w0 += kMTopGroups) {
      const int64_t w = w0 + grp;
      const int64_t c = w < lev[l + 1] ? static_cast<int64_t>(__builtin_amdgcn_readfirstlane(list[w])) : -1;
      kup_group<NT>(c, g, child0, child1, E1, xhat, t + grp * 2 * kTileFloats);
      __syncthreads();  // the tiles are read to the end before the next clusters fill them
    }
}

template <int NT>
__global__ __launch_bounds__(256 * kMTopGroups) void mtransfer_down_kron_top(int nlev,
                                                                           const int32_t* __restrict__ level_ptr,
                                                                           const int32_t* __restrict__ parent,
                                                                           const float* __restrict__ E1,
                                                                           float* __restrict__ yhat) {
  __shared__ __attribute__((aligned(16))) float t[kMTopGroups * kTileFloats];
  const int grp = threadIdx.x / 256, g = threadIdx.x % 256;
  for (int l = 0; l < nlev; ++l)
    for (int64_t c0 = level_ptr[l + 1]; c0 < level_ptr[l + 2]; c0 += kMTopGroups) {
      const int64_t c = c0 + grp < level_ptr[l + 2] ? c0 + grp : -1;
      kdown_group<NT>(c, g, parent, E1, yhat, t + grp * kTileFloats);
      __syncthreads();
    }
}

// Y|tau = sum_{(tau,sigma) inadmissible} G|tau x sigma X|sigma + V_tau y^_tau for
// every leaf (all leaves hold at most 64 triangles on this path), on 16 x 16
// tiles (v_mfma_f32_16x16x4f32): one wave per leaf.  Lane l supplies
// A[i = l % 16][kk = l / 16] and B[kk = l / 16][j = l % 16]; the accumulator
// holds D[i][j] in register v of lane l with i = 4 (l / 16) + v, j = l % 16.  A
// leaf of r rows takes ceil(r / 16) row tiles (the same for the whole wave) and
// a near block of w columns ceil(w / 4) K-steps, so padding costs at most 15
// rows per leaf and 3 columns per block instead of a full 64 x 64 tile.  Loads
// read clamped in-range addresses; the masks are applied by selects.  The panel
// streams from HBM with a short MFMA run per K-step, so latency is hidden twice:
// each wave loads step s+1 while its MFMAs consume step s, and the kernel is
// limited to 128 VGPRs (four waves per SIMD).  Measured on the 786k cube with 64
// columns: 3.1 ms against 4.9 ms unconstrained and without the pipeline.
__device__ inline f4v mfma16(float a, float b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// rows of the leaf: NTI tiles of 16 (r > 16 (NTI - 1)); see mnear_backward16
template <int TJ, int NTI>
__device__ inline void near16_leaf(int64_t it, int r, int64_t b0, int32_t tau, const int32_t* __restrict__ cbegin,
                                   const int32_t* __restrict__ cend, const int64_t* __restrict__ near_ptr,
                                   const int32_t* __restrict__ near_col, const int64_t* __restrict__ panel_off,
                                   const float* __restrict__ N, const float* __restrict__ Vb,
                                   const float* __restrict__ xc, const float* __restrict__ yhat,
                                   float* __restrict__ yc) {
  constexpr int RP = 16 * TJ;
  const int l = threadIdx.x % 64, li = l % 16, lk = l / 16;
  int rowc[NTI];
  bool rowok[NTI];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti) {
    rowok[ti] = 16 * ti + li < r;
    rowc[ti] = min(16 * ti + li, r - 1);
  }
  f4v acc[NTI][TJ];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
  const float* P = N + panel_off[it];
  int64_t colbase = 0;
  for (int64_t bb = near_ptr[it]; bb < near_ptr[it + 1]; ++bb) {
    const int32_t s = near_col[bb];
    const int wdt = cend[s] - cbegin[s];
    const float* A = P + colbase * r;
    const float* B = xc + static_cast<int64_t>(cbegin[s]) * RP + li;
    // operands of K-step k0 (4 columns), clamped in range and masked
    auto fetch = [&](int k0, float (&av)[NTI], float (&bv)[TJ]) {
      const int kk = k0 + lk;
      const bool ok = kk < wdt;
      const int kc = ok ? kk : wdt - 1;
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) {
        const float y = B[kc * RP + 16 * tj];
        bv[tj] = ok ? y : 0.f;
      }
#pragma unroll
      for (int ti = 0; ti < NTI; ++ti) {
        const float x = A[kc * r + rowc[ti]];
        av[ti] = (ok && rowok[ti]) ? x : 0.f;
      }
    };
    // software pipeline, NP steps deep: slot d holds the operands of step st + d;
    // after its MFMAs a slot is refilled with step st + d + NP (clamped to the
    // last step, so every load stays in range; the extra loads are never used)
    constexpr int NP = TJ >= 4 ? 2 : 4;  // within the register budget of four waves per SIMD
    const int nsteps = (wdt + 3) >> 2;
    float av[NP][NTI], bv[NP][TJ];
#pragma unroll
    for (int d = 0; d < NP; ++d) fetch(min(d, nsteps - 1) * 4, av[d], bv[d]);
    for (int st = 0; st < nsteps; st += NP) {
#pragma unroll
      for (int d = 0; d < NP; ++d) {
        if (st + d < nsteps) {
#pragma unroll
          for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = mfma16(av[d][ti], bv[d][tj], acc[ti][tj]);
          fetch(min(st + d + NP, nsteps - 1) * 4, av[d], bv[d]);
        }
      }
    }
    colbase += wdt;
  }
  // + V_tau y^_tau: A = Vb (column-major r x 64), B(kk, j) = y^_tau[j * 64 + kk]
  const float* A = Vb + b0 * 64;
  const float* Y = yhat + static_cast<int64_t>(tau) * RP * 64 + li * 64;
#pragma unroll 2
  for (int k0 = 0; k0 < 64; k0 += 4) {
    const int kk = k0 + lk;
    float av[NTI], bv[TJ];
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) bv[tj] = Y[16 * tj * 64 + kk];
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) {
      const float x = A[kk * r + rowc[ti]];
      av[ti] = rowok[ti] ? x : 0.f;
    }
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = mfma16(av[ti], bv[tj], acc[ti][tj]);
  }
  float* out = yc + b0 * RP + li;
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * ti + 4 * lk + v;
        if (i < r) out[i * RP + 16 * tj] = acc[ti][tj][v];
      }
}

// The same product with the K-steps of the row's near blocks in one stream, for
// rows of at most 64 near blocks: the wave holds the blocks' descriptors (first
// triangle s0 and width w of sigma, first panel column cb) one per lane and keeps
// NP K-steps in flight across block boundaries, so the pipeline never drains
// between blocks.  A K-step past a block's last column re-reads that column of
// the panel and multiplies it by a row of zeros instead of x, so no loaded value
// needs a mask.  Two waves share a leaf: half 0 streams the first ceil(nb / 2)
// blocks, half 1 the rest and V_tau y^_tau, and half 1's sums reach half 0
// through LDS (red, one 16 KB slot per leaf), which adds and stores them.  Half
// the work per wave halves the tail of the launch (the last leaves to start run
// alone): 2.07 -> 1.88 ms per 64-column pass on the 786k cube.
__device__ float kZeroRow[64];  // zero-initialised, never written

template <int TJ, int NTI>
__device__ inline void near16_stream(const NearRow& d0, int half, float* __restrict__ red,
                                     const NearBlock* __restrict__ blocks, const float* __restrict__ N,
                                     const float* __restrict__ Vb, const float* __restrict__ xc,
                                     const float* __restrict__ yhat, float* __restrict__ yc) {
  constexpr int RP = 16 * TJ;
  NearRow d = d0;
  const int nb0 = (d0.nb + 1) / 2;
  if (half == 0) {
    d.nb = nb0;
  } else {
    d.bfirst += nb0;
    d.nb = d0.nb - nb0;
  }
  constexpr int NP = TJ >= 4 ? 3 : 4;  // K-steps in flight (within 128 VGPRs: four waves per SIMD)
  const int l = threadIdx.x % 64, li = l % 16, lk = l / 16;
  const int r = d.r;
  int rowc[NTI];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti) rowc[ti] = min(16 * ti + li, r - 1);  // rows past r are computed, not stored
  f4v acc[NTI][TJ];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
  NearBlock e{0, 1, 0, 0};
  if (l < d.nb) e = blocks[d.bfirst + l];
  int nst = l < d.nb ? (e.w + 3) >> 2 : 0;  // K-steps of the whole row
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nst += __shfl_xor(nst, o);
  nst = __builtin_amdgcn_readfirstlane(nst);
  const float* P = N + d.panel_off;
  int m = 0, k0 = 0;  // the K-step fetched next: block m, columns k0 .. k0 + 3
  int s0 = __builtin_amdgcn_readlane(e.s0, 0), w = __builtin_amdgcn_readlane(e.w, 0);
  int cb = __builtin_amdgcn_readlane(e.cb, 0);
  auto fetch = [&](float (&av)[NTI], float (&bv)[TJ]) {
    const int kk = k0 + lk;
    const int kc = min(kk, w - 1);
    const float* B = (m < d.nb && kk < w) ? xc + static_cast<int64_t>(s0 + kk) * RP + li : kZeroRow + li;
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) bv[tj] = B[16 * tj];
    const float* A = P + static_cast<int64_t>(cb + kc) * r;
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) av[ti] = __builtin_nontemporal_load(A + rowc[ti]);  // streamed once
    k0 += 4;
    if (k0 >= w) {
      k0 = 0;
      if (++m < d.nb) {  // past the last block the last one is re-read, times zero
        s0 = __builtin_amdgcn_readlane(e.s0, m);
        w = __builtin_amdgcn_readlane(e.w, m);
        cb = __builtin_amdgcn_readlane(e.cb, m);
      }
    }
  };
  // whole rounds of NP steps: the steps past the row's last one multiply zeros, so
  // every round is the same straight-line code and the loads stay NP steps ahead
  float av[NP][NTI], bv[NP][TJ];
#pragma unroll
  for (int q = 0; q < NP; ++q) fetch(av[q], bv[q]);
  for (int st = 0; st < nst; st += NP) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = mfma16(av[q][ti], bv[q][tj], acc[ti][tj]);
      fetch(av[q], bv[q]);
    }
  }
  // + V_tau y^_tau: A = Vb (column-major r x 64), B(kk, j) = y^_tau[j * 64 + kk]
  const float* A = Vb + static_cast<int64_t>(d.b0) * 64;
  const float* Y = yhat + static_cast<int64_t>(d.tau) * RP * 64 + li * 64;
#pragma unroll 2
  for (int q0 = 0; q0 < (half ? 64 : 0); q0 += 4) {
    const int kk = q0 + lk;
    float a2[NTI], b2[TJ];
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) b2[tj] = Y[16 * tj * 64 + kk];
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) a2[ti] = A[kk * r + rowc[ti]];
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = mfma16(a2[ti], b2[tj], acc[ti][tj]);
  }
  // the two halves' sums: half 1 hands its registers over through LDS
  if (half == 1) {
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[((ti * TJ + tj) * 4 + v) * 64 + l] = acc[ti][tj][v];
  }
  __syncthreads();
  if (half == 1) return;
  float* out = yc + static_cast<int64_t>(d.b0) * RP + li;
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * ti + 4 * lk + v;
        if (i < r) out[i * RP + 16 * tj] = acc[ti][tj][v] + red[((ti * TJ + tj) * 4 + v) * 64 + l];
      }
}

template <int TJ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mnear_stream16(
    int nleaves, const NearRow* __restrict__ rows, const NearBlock* __restrict__ blocks, const float* __restrict__ N,
    const float* __restrict__ Vb, const float* __restrict__ xc, const float* __restrict__ yhat,
    float* __restrict__ yc) {
  // two leaves per workgroup, two waves per leaf; the halves of a leaf meet at
  // one workgroup barrier, which the waves of a missing second leaf also reach
  __shared__ __align__(16) float red[2][4 * TJ * 4 * 64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t it = xcd_group_item() * 2 + (wave >> 1);
  const int half = wave & 1;
  if (it >= nleaves) {
    __syncthreads();
    return;
  }
  const NearRow d = rows[it];
  float* rd = red[wave >> 1];
  switch ((d.r + 15) >> 4) {  // wave-uniform: one leaf per wave
    case 1: near16_stream<TJ, 1>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
    case 2: near16_stream<TJ, 2>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
    case 3: near16_stream<TJ, 3>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
    default: near16_stream<TJ, 4>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
  }
}

template <int TJ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mnear_backward16(int nleaves, const int32_t* __restrict__ leaves,
                                                        const int32_t* __restrict__ cbegin,
                                                        const int32_t* __restrict__ cend,
                                                        const int64_t* __restrict__ near_ptr,
                                                        const int32_t* __restrict__ near_col,
                                                        const int64_t* __restrict__ panel_off,
                                                        const float* __restrict__ N, const float* __restrict__ Vb,
                                                        const float* __restrict__ xc, const float* __restrict__ yhat,
                                                        float* __restrict__ yc) {
  const int64_t it = xcd_item(nleaves);
  if (it >= nleaves) return;
  const int32_t tau = leaves[it];
  const int64_t b0 = cbegin[tau];
  const int r = cend[tau] - cbegin[tau];
  switch ((r + 15) >> 4) {  // wave-uniform: one leaf per wave
    case 1: near16_leaf<TJ, 1>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
    case 2: near16_leaf<TJ, 2>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
    case 3: near16_leaf<TJ, 3>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
    default: near16_leaf<TJ, 4>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
  }
}

// ---------------------------------------------------------------- complex (Helmholtz) many-RHS path
// 16 complex right-hand sides per pass are held as 32 real columns [re | im];
// the real V and E act on them with the real kernels above.  Complex S and
// near-field entries (interleaved re, im) multiply as C1 = Re(A) [Xr | Xi] and
// C2 = Im(A) [Xr | Xi]; then Yr = C1[:, :16] - C2[:, 16:], Yi = C1[:, 16:] +
// C2[:, :16], one lane exchange (xor 16) per output element.
// complex: 16 complex columns jc held as 32 real columns j = 16 part + jc
// (part 0 = real, 1 = imaginary); user vectors interleaved (re, im); tiled as above
template <typename XT>
__global__ __launch_bounds__(256) void mpermute_in_c(int64_t n, int rcur, const int32_t* __restrict__ iperm,
                                                     const XT* __restrict__ x, int64_t ldx, float* __restrict__ xc) {
  constexpr int PER = 64 * 32 / 256;
  __shared__ float tile[64][33];
  __shared__ int32_t pos[64];
  const int t = threadIdx.x;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int32_t ip = iperm[min(i0 + t % 64, n - 1)];  // every wave loads the tile's positions
  XT v[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int idx = t + 256 * s, part = idx % 2, il = (idx / 2) % 64, jc = idx / 128;
    const bool ok = jc < rcur && i0 + il < n;
    v[s] = x[ok ? 2 * (static_cast<int64_t>(jc) * ldx + i0 + il) + part : 0];
    v[s] = ok ? v[s] : XT(0);
  }
  if (t < 64) pos[t] = i0 + t < n ? ip : 0;
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int idx = t + 256 * s, part = idx % 2, il = (idx / 2) % 64, jc = idx / 128;
    tile[il][16 * part + jc] = static_cast<float>(v[s]);
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int il = (t + 256 * s) / 32, j = (t + 256 * s) % 32;
    if (i0 + il < n) xc[static_cast<int64_t>(pos[il]) * 32 + j] = tile[il][j];
  }
}

template <typename XT>
__global__ __launch_bounds__(256) void mpermute_out_c(int64_t n, int rcur, const int32_t* __restrict__ iperm,
                                                      const float* __restrict__ yc, XT* __restrict__ y, int64_t ldy,
                                                      double alpha, bool ow) {
  constexpr int PER = 64 * 32 / 256;
  __shared__ float tile[64][33];
  __shared__ int32_t pos[64];
  const int t = threadIdx.x;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int32_t ip = iperm[min(i0 + t % 64, n - 1)];  // every wave loads the tile's positions
  XT y0[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int idx = t + 256 * s, part = idx % 2, il = (idx / 2) % 64, jc = idx / 128;
    const bool ok = !ow && jc < rcur && i0 + il < n;
    y0[s] = y[ok ? 2 * (static_cast<int64_t>(jc) * ldy + i0 + il) + part : 0];
    y0[s] = ok ? y0[s] : XT(0);
  }
  if (t < 64) pos[t] = i0 + t < n ? ip : 0;
  __syncthreads();
  float v[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int il = (t + 256 * s) / 32, j = (t + 256 * s) % 32;
    v[s] = yc[static_cast<int64_t>(pos[il]) * 32 + j];
  }
#pragma unroll
  for (int s = 0; s < PER; ++s) tile[(t + 256 * s) / 32][(t + 256 * s) % 32] = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int idx = t + 256 * s, part = idx % 2, il = (idx / 2) % 64, jc = idx / 128;
    if (jc < rcur && i0 + il < n)
      y[2 * (static_cast<int64_t>(jc) * ldy + i0 + il) + part] =
          static_cast<XT>(static_cast<double>(y0[s]) + alpha * static_cast<double>(tile[il][16 * part + jc]));
  }
}

// Complex coupling on the real matrix cores.  With x^ held as 32 real columns
// [Xr | Xi] and S = Sr + i Si (interleaved), the 32 output columns [Yr | Yi] are
//   Sr [Xr | Xi] + Si [-Xi | Xr]:
// the second right-hand operand is the first with its halves swapped and the
// first half negated, so one set of accumulators holds the result and no lane
// exchange is needed.  One half of a block (32 of its 64 K columns) in the K order
// of mma64_rowA: per lane row 32 ti + r, columns kk .. kk + 3 with
// kk = 8 (4 half + q) + 4 h.
struct CHalf {
  f4v u[2][4], w[2][4];  // S entries (re, im, re, im) of columns kk, kk + 1 / kk + 2, kk + 3
  f4v b[4], bs[4];       // [Xr | Xi] and [-Xi | Xr] at rows kk .. kk + 3, column r
};

__device__ inline void load_half_c(const float* __restrict__ A, const float* __restrict__ Bt, int half, CHalf& d) {
  const int l = threadIdx.x % 64, r = l % 32, h = l / 32;
  const int rs = (r + 16) % 32;
  const float sg = r < 16 ? -1.f : 1.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int kk = 8 * (4 * half + q) + 4 * h;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
      d.u[ti][q] = ld4c(A + (32 * ti + r) * 128 + 2 * kk);
      d.w[ti][q] = ld4c(A + (32 * ti + r) * 128 + 2 * kk + 4);
    }
    d.b[q] = ld4c(Bt + r * 64 + kk);
    d.bs[q] = sg * ld4c(Bt + rs * 64 + kk);
  }
}

__device__ inline void mma_half_c(const CHalf& d, f32x16 (&acc)[2]) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) {
        const f4v& src = e < 2 ? d.u[ti][q] : d.w[ti][q];
        acc[ti] = mfma(src[2 * (e % 2)], d.b[q][e], acc[ti]);
        acc[ti] = mfma(src[2 * (e % 2) + 1], d.bs[q][e], acc[ti]);
      }
}

// y^_tau = sum_{(tau,sigma) admissible} S_{tau sigma} x^_sigma, 16 complex columns
// (assigns); row clusters in the XCD-balanced order of mcoupling.  Software
// pipelined: the loads of the next half block are in flight while the current
// half's products run (two half-block register sets, two waves per SIMD).
__global__ __launch_bounds__(256) void mcoupling_c(int64_t nitems, const int32_t* __restrict__ order,
                                                   const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                   const float* __restrict__ S, const float* __restrict__ xhat,
                                                   float* __restrict__ yhat) {
  const int64_t it = xcd_item(nitems);
  if (it >= nitems) return;
  const int64_t tau = order[it];
  if (tau < 0) return;
  f32x16 acc[2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[ti][v] = 0.f;
  const int64_t b0 = ptr[tau], b1 = ptr[tau + 1];
  CHalf P, Q;
  if (b0 < b1) load_half_c(S + b0 * 8192, xhat + static_cast<int64_t>(col[b0]) * 2048, 0, P);
  for (int64_t b = b0; b < b1; ++b) {
    const float* Ab = S + b * 8192;
    const float* Bb = xhat + static_cast<int64_t>(col[b]) * 2048;
    load_half_c(Ab, Bb, 1, Q);
    mma_half_c(P, acc);
    if (b + 1 < b1) load_half_c(Ab + 8192, xhat + static_cast<int64_t>(col[b + 1]) * 2048, 0, P);
    mma_half_c(Q, acc);
  }
  const int l = threadIdx.x % 64;
  float* out = yhat + tau * 32 * 64;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int v = 0; v < 16; ++v) out[(l % 32) * 64 + 32 * ti + acc_row(v, l)] = acc[ti][v];
}

// Helmholtz coupling evaluated during the product, 16 complex columns: the
// matrix-core scheme of mcoupling_c with the A operands (Re and Im of
// e^{i kappa r} / r) computed per lane in the K order of mma64_rowA, from the
// per-axis squared differences as in mcoupling_otf (x by e, y by P & 1, z by
// (ti, P >> 1)); the sine and cosine by sincos_phase; times 1/(4 pi) at the end.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mcoupling_c_otf(
    int64_t nitems, const int32_t* __restrict__ order, const int64_t* __restrict__ ptr,
    const int32_t* __restrict__ col, const double* __restrict__ ctr, const float* __restrict__ off, float kappa,
    const float* __restrict__ xhat, float* __restrict__ yhat) {
  const int64_t it = xcd_item(nitems);
  if (it >= nitems) return;
  const int64_t tau = order[it];
  if (tau < 0) return;
  const int l = threadIdx.x % 64, r = l % 32, h = l / 32;
  const int rs = (r + 16) % 32;
  const float sg = r < 16 ? -1.f : 1.f;
  const float* ot = off + tau * 12;
  const float ax = ot[r % 4], ay = ot[4 + (r / 4) % 4];
  const float az[2] = {ot[8 + r / 16], ot[10 + r / 16]};
  const double cx = ctr[3 * tau], cy = ctr[3 * tau + 1], cz = ctr[3 * tau + 2];
  f32x16 acc[2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[ti][v] = 0.f;
  const int64_t b1 = ptr[tau + 1];
  for (int64_t b = ptr[tau]; b < b1; ++b) {
    const int64_t s = col[b];
    const float* os = off + s * 12;
    float px[4], py[2], pz[2][4];
    const float ex = static_cast<float>(cx - ctr[3 * s]) + ax, ey = static_cast<float>(cy - ctr[3 * s + 1]) + ay;
    const float dcz = static_cast<float>(cz - ctr[3 * s + 2]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d = ex - os[e];
      px[e] = d * d;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const float d = ey - os[4 + 2 * j + h];
      py[j] = d * d;
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int z = 0; z < 4; ++z) {
        const float d = (dcz + az[ti]) - os[8 + z];
        pz[ti][z] = d * d;
      }
    const float* Bt = xhat + s * 2048;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      f4v bv[4], bsv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = 8 * (4 * half + q) + 4 * h;
        bv[q] = ld4c(Bt + r * 64 + kk);
        bsv[q] = sg * ld4c(Bt + rs * 64 + kk);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int P = 4 * half + q;
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int ti = 0; ti < 2; ++ti) {
            const float d2 = px[e] + (py[P & 1] + pz[ti][P >> 1]);
            const float inv = __builtin_amdgcn_rsqf(d2);
            float sn, cs;
            sincos_phase(kappa * (d2 * inv), sn, cs);
            acc[ti] = mfma(cs * inv, bv[q][e], acc[ti]);
            acc[ti] = mfma(sn * inv, bsv[q][e], acc[ti]);
          }
      }
    }
  }
  const float scale = static_cast<float>(1.0 / (4.0 * 3.14159265358979323846));
  float* out = yhat + tau * 32 * 64;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int v = 0; v < 16; ++v) out[(l % 32) * 64 + 32 * ti + acc_row(v, l)] = acc[ti][v] * scale;
}

// Complex near field + leaf backward on 16 x 16 tiles, as mnear_backward16: the
// 32 real columns are [Xr | Xi] (tile tj = 0 real parts, 1 imaginary parts), A
// is complex column-major (interleaved), C1 = Re(A) X and C2 = Im(A) X.  The real
// output columns are C1[., 0] - C2[., 1] and the imaginary ones C1[., 1] + C2[., 0]:
// the two terms of an output sit in the same lane, so no exchange is needed.
// The real V times [y^r | y^i] adds to C1.
template <int NTI>
__device__ inline void near16c_leaf(int64_t it, int r, int64_t b0, int32_t tau, const int32_t* __restrict__ cbegin,
                                    const int32_t* __restrict__ cend, const int64_t* __restrict__ near_ptr,
                                    const int32_t* __restrict__ near_col, const int64_t* __restrict__ panel_off,
                                    const float* __restrict__ N, const float* __restrict__ Vb,
                                    const float* __restrict__ xc, const float* __restrict__ yhat,
                                    float* __restrict__ yc) {
  const int l = threadIdx.x % 64, li = l % 16, lk = l / 16;
  int rowc[NTI];
  bool rowok[NTI];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti) {
    rowok[ti] = 16 * ti + li < r;
    rowc[ti] = min(16 * ti + li, r - 1);
  }
  f4v c1[NTI][2], c2[NTI][2];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) c1[ti][tj] = c2[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
  const float* P = N + 2 * panel_off[it];
  int64_t colbase = 0;
  for (int64_t bb = near_ptr[it]; bb < near_ptr[it + 1]; ++bb) {
    const int32_t s = near_col[bb];
    const int wdt = cend[s] - cbegin[s];
    const float* A = P + 2 * colbase * r;
    const float* B = xc + static_cast<int64_t>(cbegin[s]) * 32 + li;
    auto fetch = [&](int k0, float (&ar)[NTI], float (&ai)[NTI], float (&bv)[2]) {
      const int kk = k0 + lk;
      const bool ok = kk < wdt;
      const int kc = ok ? kk : wdt - 1;
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        const float y = B[kc * 32 + 16 * tj];
        bv[tj] = ok ? y : 0.f;
      }
#pragma unroll
      for (int ti = 0; ti < NTI; ++ti) {
        const f2v a = *reinterpret_cast<const f2v*>(A + 2 * (static_cast<int64_t>(kc) * r + rowc[ti]));
        const bool use = ok && rowok[ti];
        ar[ti] = use ? a.x : 0.f;
        ai[ti] = use ? a.y : 0.f;
      }
    };
    const int nsteps = (wdt + 3) >> 2;
    float arn[NTI], ain[NTI], bvn[2];
    fetch(0, arn, ain, bvn);
    for (int st = 0; st < nsteps; ++st) {
      float ar[NTI], ai[NTI], bv[2];
#pragma unroll
      for (int ti = 0; ti < NTI; ++ti) {
        ar[ti] = arn[ti];
        ai[ti] = ain[ti];
      }
      bv[0] = bvn[0];
      bv[1] = bvn[1];
      fetch(min(st + 1, nsteps - 1) * 4, arn, ain, bvn);
#pragma unroll
      for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          c1[ti][tj] = mfma16(ar[ti], bv[tj], c1[ti][tj]);
          c2[ti][tj] = mfma16(ai[ti], bv[tj], c2[ti][tj]);
        }
    }
    colbase += wdt;
  }
  // + V_tau [y^r | y^i]: A = Vb (column-major r x 64), B(kk, j) = y^_tau[j * 64 + kk]
  const float* A = Vb + b0 * 64;
  const float* Y = yhat + static_cast<int64_t>(tau) * 32 * 64 + li * 64;
#pragma unroll 2
  for (int k0 = 0; k0 < 64; k0 += 4) {
    const int kk = k0 + lk;
    float av[NTI], bv[2];
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) bv[tj] = Y[16 * tj * 64 + kk];
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) {
      const float x = A[kk * r + rowc[ti]];
      av[ti] = rowok[ti] ? x : 0.f;
    }
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) c1[ti][tj] = mfma16(av[ti], bv[tj], c1[ti][tj]);
  }
  float* out = yc + b0 * 32 + li;
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ti + 4 * lk + v;
      if (i < r) {
        out[i * 32] = c1[ti][0][v] - c2[ti][1][v];
        out[i * 32 + 16] = c1[ti][1][v] + c2[ti][0][v];
      }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mnear_backward16c(
    int nleaves, const int32_t* __restrict__ leaves, const int32_t* __restrict__ cbegin,
    const int32_t* __restrict__ cend, const int64_t* __restrict__ near_ptr, const int32_t* __restrict__ near_col,
    const int64_t* __restrict__ panel_off, const float* __restrict__ N, const float* __restrict__ Vb,
    const float* __restrict__ xc, const float* __restrict__ yhat, float* __restrict__ yc) {
  const int64_t it = xcd_item(nleaves);
  if (it >= nleaves) return;
  const int32_t tau = leaves[it];
  const int64_t b0 = cbegin[tau];
  const int r = cend[tau] - cbegin[tau];
  switch ((r + 15) >> 4) {  // wave-uniform: one leaf per wave
    case 1: near16c_leaf<1>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
    case 2: near16c_leaf<2>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
    case 3: near16c_leaf<3>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
    default: near16c_leaf<4>(it, r, b0, tau, cbegin, cend, near_ptr, near_col, panel_off, N, Vb, xc, yhat, yc); break;
  }
}

// The complex near field streamed as near16_stream does for the real one (rows
// of at most 64 near blocks, K-steps across block boundaries, two waves per leaf
// meeting through LDS): the panel entry (re, im) is one 8-byte load per row and
// K-step, and the products accumulate straight into the output's two parts,
// Yr += Re(A) Xr - Im(A) Xi and Yi += Re(A) Xi + Im(A) Xr (tile tj = 0: Xr, 1: Xi),
// so one accumulator pair per row tile holds the result.
template <int NTI>
__device__ inline void near16c_stream(const NearRow& d0, int half, float* __restrict__ red,
                                      const NearBlock* __restrict__ blocks, const float* __restrict__ N,
                                      const float* __restrict__ Vb, const float* __restrict__ xc,
                                      const float* __restrict__ yhat, float* __restrict__ yc) {
  NearRow d = d0;
  const int nb0 = (d0.nb + 1) / 2;
  if (half == 0) {
    d.nb = nb0;
  } else {
    d.bfirst += nb0;
    d.nb = d0.nb - nb0;
  }
  constexpr int NP = 4;  // K-steps in flight
  const int l = threadIdx.x % 64, li = l % 16, lk = l / 16;
  const int r = d.r;
  int rowc[NTI];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti) rowc[ti] = min(16 * ti + li, r - 1);  // rows past r are computed, not stored
  f4v yr[NTI], yi[NTI];
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti) yr[ti] = yi[ti] = f4v{0.f, 0.f, 0.f, 0.f};
  NearBlock e{0, 1, 0, 0};
  if (l < d.nb) e = blocks[d.bfirst + l];
  int nst = l < d.nb ? (e.w + 3) >> 2 : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nst += __shfl_xor(nst, o);
  nst = __builtin_amdgcn_readfirstlane(nst);
  const float* P = N + 2 * d.panel_off;
  int m = 0, k0 = 0;
  int s0 = __builtin_amdgcn_readlane(e.s0, 0), w = __builtin_amdgcn_readlane(e.w, 0);
  int cb = __builtin_amdgcn_readlane(e.cb, 0);
  auto fetch = [&](f2v (&av)[NTI], float (&bv)[2]) {
    const int kk = k0 + lk;
    const int kc = min(kk, w - 1);
    const float* B = (m < d.nb && kk < w) ? xc + static_cast<int64_t>(s0 + kk) * 32 + li : kZeroRow + li;
    bv[0] = B[0];
    bv[1] = B[16];
    const float* A = P + 2 * static_cast<int64_t>(cb + kc) * r;
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) av[ti] = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(A + 2 * rowc[ti]));
    k0 += 4;
    if (k0 >= w) {
      k0 = 0;
      if (++m < d.nb) {
        s0 = __builtin_amdgcn_readlane(e.s0, m);
        w = __builtin_amdgcn_readlane(e.w, m);
        cb = __builtin_amdgcn_readlane(e.cb, m);
      }
    }
  };
  f2v av[NP][NTI];
  float bv[NP][2];
#pragma unroll
  for (int q = 0; q < NP; ++q) fetch(av[q], bv[q]);
  for (int st = 0; st < nst; st += NP) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
#pragma unroll
      for (int ti = 0; ti < NTI; ++ti) {
        yr[ti] = mfma16(av[q][ti].x, bv[q][0], yr[ti]);
        yr[ti] = mfma16(-av[q][ti].y, bv[q][1], yr[ti]);
        yi[ti] = mfma16(av[q][ti].x, bv[q][1], yi[ti]);
        yi[ti] = mfma16(av[q][ti].y, bv[q][0], yi[ti]);
      }
      fetch(av[q], bv[q]);
    }
  }
  // + V_tau [y^r | y^i] (the second half)
  const float* A = Vb + static_cast<int64_t>(d.b0) * 64;
  const float* Y = yhat + static_cast<int64_t>(d.tau) * 32 * 64 + li * 64;
#pragma unroll 2
  for (int q0 = 0; q0 < (half ? 64 : 0); q0 += 4) {
    const int kk = q0 + lk;
    const float br = Y[kk], bi = Y[16 * 64 + kk];
    float a2[NTI];
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) a2[ti] = A[kk * r + rowc[ti]];
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti) {
      yr[ti] = mfma16(a2[ti], br, yr[ti]);
      yi[ti] = mfma16(a2[ti], bi, yi[ti]);
    }
  }
  // half 1 hands its sums over through LDS
  if (half == 1) {
#pragma unroll
    for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        red[((ti * 2 + 0) * 4 + v) * 64 + l] = yr[ti][v];
        red[((ti * 2 + 1) * 4 + v) * 64 + l] = yi[ti][v];
      }
  }
  __syncthreads();
  if (half == 1) return;
  float* out = yc + static_cast<int64_t>(d.b0) * 32 + li;
#pragma unroll
  for (int ti = 0; ti < NTI; ++ti)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ti + 4 * lk + v;
      if (i < r) {
        out[i * 32] = yr[ti][v] + red[((ti * 2 + 0) * 4 + v) * 64 + l];
        out[i * 32 + 16] = yi[ti][v] + red[((ti * 2 + 1) * 4 + v) * 64 + l];
      }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mnear_stream16c(
    int nleaves, const NearRow* __restrict__ rows, const NearBlock* __restrict__ blocks, const float* __restrict__ N,
    const float* __restrict__ Vb, const float* __restrict__ xc, const float* __restrict__ yhat,
    float* __restrict__ yc) {
  // two leaves per workgroup, two waves per leaf, as mnear_stream16
  __shared__ __align__(16) float red[2][4 * 2 * 4 * 64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t it = xcd_group_item() * 2 + (wave >> 1);
  const int half = wave & 1;
  if (it >= nleaves) {
    __syncthreads();
    return;
  }
  const NearRow d = rows[it];
  float* rd = red[wave >> 1];
  switch ((d.r + 15) >> 4) {
    case 1: near16c_stream<1>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
    case 2: near16c_stream<2>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
    case 3: near16c_stream<3>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
    default: near16c_stream<4>(d, half, rd, blocks, N, Vb, xc, yhat, yc); break;
  }
}

inline unsigned nblk(int64_t work, int per) {
  const int64_t g = (work + per - 1) / per;
  if (g > 0x7fffffff) throw Error(H2_EINVAL, "launch too large");
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

// Row clusters for the coupling kernels: 8 contiguous ranges of about equal
// work (admissible blocks + 1 per row), one per XCD (xcd_item gives XCD x the
// items [x L, (x + 1) L)), each ordered heaviest first and padded with -1 to the
// common length L, a multiple of 4.  Contiguous ranges keep neighbouring rows,
// which share column clusters, on one L2; equal work keeps the eight XCDs busy
// until the end, and heaviest first keeps a heavy row from starting last
// (mcoupling_otf 3.07 -> 2.66 ms on the 786k cube with 64 columns; the complex
// coupling 5.03 -> 4.85 ms stored and 3.47 -> 2.71 ms on the fly at 327,680
// triangles with 16 complex columns).
std::vector<int32_t> balanced_rows(const Structure& S) {
  const int32_t nc = S.nclusters;
  double total = 0.0;
  for (int32_t t = 0; t < nc; ++t) total += 1.0 + static_cast<double>(S.adm_ptr[t + 1] - S.adm_ptr[t]);
  std::vector<int32_t> cut(9, nc);
  cut[0] = 0;
  double acc = 0.0;
  int x = 1;
  for (int32_t t = 0; t < nc && x < 8; ++t) {
    acc += 1.0 + static_cast<double>(S.adm_ptr[t + 1] - S.adm_ptr[t]);
    if (acc >= total * x / 8.0) cut[x++] = t + 1;
  }
  int64_t L = 4;
  for (int c = 0; c < 8; ++c) L = std::max<int64_t>(L, cut[c + 1] - cut[c]);
  L = (L + 3) / 4 * 4;
  std::vector<int32_t> order(8 * L, -1);
  for (int c = 0; c < 8; ++c) {
    for (int32_t t = cut[c]; t < cut[c + 1]; ++t) order[c * L + (t - cut[c])] = t;
    std::stable_sort(order.begin() + c * L, order.begin() + c * L + (cut[c + 1] - cut[c]),
                     [&](int32_t a, int32_t b) {
                       return S.adm_ptr[a + 1] - S.adm_ptr[a] > S.adm_ptr[b + 1] - S.adm_ptr[b];
                     });
  }
  return order;
}

// Row clusters in their natural order, four per workgroup, so that workgroup g
// (on XCD g mod 8) takes rows 4g..4g+3: neighbouring rows run at the same time on
// all eight XCDs instead of in eight separate ranges.
std::vector<int32_t> interleaved_rows(const Structure& S) {
  const int64_t nc = S.nclusters;
  const int64_t nit = (nc + 31) / 32 * 32, nwg = nit / 4, per = nwg / 8;
  std::vector<int32_t> order(nit, -1);
  for (int64_t g = 0; g < nwg; ++g)
    for (int w = 0; w < 4; ++w) {
      const int64_t row = 4 * g + w;
      order[((g % 8) * per + g / 8) * 4 + w] = row < nc ? static_cast<int32_t>(row) : -1;
    }
  return order;
}

// The groups of mcoupling_grp: the four grandchildren of every cluster whose two
// children both have children, then the remaining row clusters in runs of up to
// four consecutive ids; sorted by first row, cut into 8 contiguous chunks of about
// equal work (blocks + 1 per group), one per XCD, each ordered heaviest first and
// padded with empty groups to the common length.  Entries: (column cluster, block of each slot or -1, 3 x
// padding), per group ordered by the position of the column cluster.
void build_groups(h2_handle_s& H) {
  const Structure& S = H.S;
  const int32_t nc = S.nclusters;
  std::vector<std::array<int32_t, 4>> groups;
  std::vector<char> done(nc, 0);
  for (int32_t p = 0; p < nc; ++p) {
    const int32_t c0 = S.child0[p], c1 = S.child1[p];
    if (c0 < 0 || c1 < 0 || S.child0[c0] < 0 || S.child1[c0] < 0 || S.child0[c1] < 0 || S.child1[c1] < 0) continue;
    const std::array<int32_t, 4> g = {S.child0[c0], S.child1[c0], S.child0[c1], S.child1[c1]};
    for (int32_t t : g) done[t] = 1;
    groups.push_back(g);
  }
  for (int32_t t = 0; t < nc;) {
    if (done[t]) {
      ++t;
      continue;
    }
    std::array<int32_t, 4> g = {-1, -1, -1, -1};
    for (int i = 0; i < 4 && t < nc && !done[t]; ++i, ++t) g[i] = t;
    groups.push_back(g);
  }
  std::sort(groups.begin(), groups.end(),
            [](const std::array<int32_t, 4>& a, const std::array<int32_t, 4>& b) { return a[0] < b[0]; });
  std::vector<std::vector<int32_t>> ge(groups.size());
  std::vector<double> work(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const auto& g = groups[gi];
    int64_t pos[4], end[4];
    for (int i = 0; i < 4; ++i) {
      pos[i] = g[i] >= 0 ? S.adm_ptr[g[i]] : 0;
      end[i] = g[i] >= 0 ? S.adm_ptr[g[i] + 1] : 0;
    }
    auto key = [&](int32_t c) { return std::make_pair(S.cbegin[c], c); };
    std::vector<int32_t>& out = ge[gi];
    double blocks = 0.0;
    for (;;) {  // merge the four lists (each ordered by position of the column cluster)
      int32_t sig = -1;
      for (int i = 0; i < 4; ++i)
        if (pos[i] < end[i] && (sig < 0 || key(S.adm_col[pos[i]]) < key(sig))) sig = S.adm_col[pos[i]];
      if (sig < 0) break;
      int32_t en[8] = {sig, -1, -1, -1, -1, 0, 0, 0};
      for (int i = 0; i < 4; ++i)
        if (pos[i] < end[i] && S.adm_col[pos[i]] == sig) {
          en[1 + i] = static_cast<int32_t>(pos[i]++);
          blocks += 1.0;
        }
      out.insert(out.end(), en, en + 8);
    }
    work[gi] = 1.0 + blocks;
  }
  double total = 0.0;
  for (double w : work) total += w;
  const int64_t ng = static_cast<int64_t>(groups.size());
  std::vector<int64_t> cut(9, ng);
  cut[0] = 0;
  double acc = 0.0;
  int x = 1;
  for (int64_t gi = 0; gi < ng && x < 8; ++gi) {
    acc += work[gi];
    if (acc >= total * x / 8.0) cut[x++] = gi + 1;
  }
  int64_t L = 1;
  for (int c = 0; c < 8; ++c) L = std::max<int64_t>(L, cut[c + 1] - cut[c]);
  std::vector<int32_t> rows(8 * L * 4, -1), ents;
  std::vector<int64_t> ptr(8 * L + 1, 0);
  // within a chunk the groups go out heaviest first (the workgroups of an XCD
  // take them in dispatch order): in tree order the heavy groups that start last
  // set the end of the launch (simulated makespan 1.26 x the mean work per
  // slot, 1.07 x heaviest first); the x^ tiles of the groups in flight are then
  // less often shared (fetched 1.37 -> 1.48 x S), and the coupling still drops
  // from 3.32 to 3.11 ms on the 786k cube
  std::vector<int64_t> order(ng);
  for (int64_t gi = 0; gi < ng; ++gi) order[gi] = gi;
  for (int c = 0; c < 8; ++c)
    std::stable_sort(order.begin() + cut[c], order.begin() + cut[c + 1],
                     [&](int64_t a, int64_t b) { return work[a] > work[b]; });
  for (int c = 0; c < 8; ++c)
    for (int64_t q = 0; q < L; ++q) {
      const int64_t slot = c * L + q, gi = cut[c] + q < cut[c + 1] ? order[cut[c] + q] : ng;
      if (gi < ng) {
        for (int i = 0; i < 4; ++i) rows[4 * slot + i] = groups[gi][i];
        ents.insert(ents.end(), ge[gi].begin(), ge[gi].end());
      }
      ptr[slot + 1] = static_cast<int64_t>(ents.size() / 8);
    }
  H.mgrp_rows.upload(rows);
  H.mgrp_ptr.upload(ptr);
  H.mgrp_tasks.upload(ents);
  H.mgrp_n = 8 * L;
}

}  // namespace

// the row order of the coupling kernels (built on first use, rebuilt when the
// row-order knob changes): XCD chunks of equal admissible-block count, or
// interleaved; schedule 3 also builds the row groups of mcoupling_grp (passes of
// other widths use the XCD chunks).  Unset, the knob means 3 for real stored
// coupling matrices and 1 otherwise.
int row_schedule(const h2_handle_s& H) {
  if (H.tune_order != 0) return H.tune_order;
  return !H.is_complex && !H.otf ? 3 : 1;  // built-in rule: row groups wherever they apply
}

void ensure_row_order(h2_handle_s& H) {
  const int kind = row_schedule(H);
  if (H.morder.p == nullptr || H.morder_kind != kind) {
    const std::vector<int32_t> ord = kind == 2 ? interleaved_rows(H.S) : balanced_rows(H.S);
    H.morder.upload(ord);
    H.morder_items = static_cast<int64_t>(ord.size());
    if (kind == 3 && H.mgrp_n == 0) build_groups(H);
    H.morder_kind = kind;
  }
}

namespace {

template <int NT, typename XT>
void run_pass(h2_handle_s& H, int rcur, const XT* x, int64_t ldx, XT* y, int64_t ldy, double alpha, hipStream_t st) {
  constexpr int RP = 32 * NT;
  const Structure& S = H.S;
  const int64_t n = S.n;
  const int nc = S.nclusters;
  const int nl = static_cast<int>(S.leaves.size());
  float* xc = H.mxc.as<float>();
  float* yc = H.myc.as<float>();
  float* xh = H.mxhat.as<float>();
  float* yh = H.myhat.as<float>();
  auto waves = [](int64_t items) { return nblk((items + 3) / 4 * 4, 4) + 0u; };  // 4 waves per workgroup
  auto grid8 = [&](int64_t items) {  // a multiple of 8 workgroups, so every XCD chunk has the same size
    const unsigned g = waves(items);
    return (g + 7) / 8 * 8;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr, e4 = nullptr;
  if (H.prof) {
    e0 = prof_event(H);
    H2_HIP(hipEventRecord(e0, st));
  }
  const unsigned ptiles = nblk(n, 64);
  mpermute_in<XT, RP><<<ptiles, 256, 0, st>>>(n, rcur, H.iperm.as<int32_t>(), x, ldx, xc);
  mleaf_forward<NT><<<(nl + 7) / 8 * 8, 256, 0, st>>>(nl, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                               H.cend.as<int32_t>(), H.Vf.as<float>(), xc, xh);
  const int up_top = H.kron ? H.mup_top : 0;  // the dense MFMA transfers run one launch per level
  for (int lv = S.depth - 1; lv >= up_top; --lv) {
    const int cnt = static_cast<int>(H.up_ptr[lv + 1] - H.up_ptr[lv]);
    if (cnt == 0) continue;
    if (H.kron)
      mtransfer_up_kron<NT><<<(cnt + 7) / 8 * 8, 256, 0, st>>>(cnt, H.up_list.as<int32_t>() + H.up_ptr[lv],
                                                        H.child0.as<int32_t>(), H.child1.as<int32_t>(),
                                                        H.E1.as<float>(), xh);
    else
      mtransfer_up<NT><<<grid8(cnt), 256, 0, st>>>(cnt, H.up_list.as<int32_t>() + H.up_ptr[lv],
                                                   H.child0.as<int32_t>(), H.child1.as<int32_t>(), H.ET.as<float>(), xh);
  }
  if (up_top > 0)
    mtransfer_up_kron_top<NT><<<1, 256 * kMTopGroups, 0, st>>>(up_top, H.up_ptr_dev.as<int64_t>(),
                                                             H.up_list.as<int32_t>(), H.child0.as<int32_t>(),
                                                             H.child1.as<int32_t>(), H.E1.as<float>(), xh);
  if (H.prof) {
    e1 = prof_event(H);
    H2_HIP(hipEventRecord(e1, st));
  }
  ensure_row_order(H);
  const int64_t nit = H.morder_items;
  const int32_t* ord = H.morder.as<int32_t>();
  const unsigned gco = static_cast<unsigned>(nit / 4);  // a multiple of 8 workgroups
  if (H.otf) {
    const int64_t* ap = H.adm_ptr.as<int64_t>();
    const int32_t* ac = H.adm_col.as<int32_t>();
    const double* ctr = H.ctr.as<double>();
    const float* off = H.off32.as<float>();
    switch (H.P.kernel) {
      case H2_LAPLACE: mcoupling_otf<NT, H2_LAPLACE><<<gco, 256, 0, st>>>(nit, ord, ap, ac, ctr, off, xh, yh); break;
      case H2_TEST_ONE: mcoupling_otf<NT, H2_TEST_ONE><<<gco, 256, 0, st>>>(nit, ord, ap, ac, ctr, off, xh, yh); break;
      case H2_TEST_BILINEAR:
        mcoupling_otf<NT, H2_TEST_BILINEAR><<<gco, 256, 0, st>>>(nit, ord, ap, ac, ctr, off, xh, yh);
        break;
      case H2_TEST_QUADRATIC:
        mcoupling_otf<NT, H2_TEST_QUADRATIC><<<gco, 256, 0, st>>>(nit, ord, ap, ac, ctr, off, xh, yh);
        break;
      default: throw Error(H2_EINVAL, "on-the-fly coupling supports real kernels only");
    }
  } else if (NT == 2 && H.morder_kind == 3) {
    mcoupling_grp<<<static_cast<unsigned>(H.mgrp_n), 256, 0, st>>>(
        H.mgrp_n, H.mgrp_rows.as<int32_t>(), H.mgrp_ptr.as<int64_t>(), H.mgrp_tasks.as<int32_t>(), H.Smat.as<float>(),
        xh, yh);
  } else {
    mcoupling<NT><<<gco, 256, 0, st>>>(nit, ord, H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(),
                                       H.Smat.as<float>(), xh, yh);
  }
  if (H.prof) {
    e2 = prof_event(H);
    H2_HIP(hipEventRecord(e2, st));
  }
  const int down_top = H.kron ? H.mdown_top : 0;
  if (down_top > 0)
    mtransfer_down_kron_top<NT><<<1, 256 * kMTopGroups, 0, st>>>(down_top, H.level_ptr_dev.as<int32_t>(),
                                                               H.parent.as<int32_t>(), H.E1.as<float>(), yh);
  for (int lv = down_top; lv < S.depth; ++lv) {
    const int first = S.level_ptr[lv + 1], cnt = S.level_ptr[lv + 2] - S.level_ptr[lv + 1];
    if (cnt == 0) continue;
    if (H.kron)
      mtransfer_down_kron<NT><<<(cnt + 7) / 8 * 8, 256, 0, st>>>(first, cnt, H.parent.as<int32_t>(), H.E1.as<float>(), yh);
    else
      mtransfer_down<NT><<<grid8(cnt), 256, 0, st>>>(first, cnt, H.parent.as<int32_t>(), H.F.as<float>(), yh);
  }
  if (H.prof) {
    e3 = prof_event(H);
    H2_HIP(hipEventRecord(e3, st));
  }
  if (H.near_row64)
    mnear_stream16<2 * NT><<<((nl + 1) / 2 + 7) / 8 * 8, 256, 0, st>>>(nl, H.near_rows.as<NearRow>(), H.near_blocks.as<NearBlock>(),
                                                      H.Nmat.as<float>(), H.Vb.as<float>(), xc, yh, yc);
  else
    mnear_backward16<2 * NT><<<grid8(nl), 256, 0, st>>>(nl, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                                        H.cend.as<int32_t>(), H.near_ptr.as<int64_t>(),
                                                        H.near_col.as<int32_t>(), H.panel_off.as<int64_t>(),
                                                        H.Nmat.as<float>(), H.Vb.as<float>(), xc, yh, yc);
  mpermute_out<XT, RP><<<ptiles, 256, 0, st>>>(n, rcur, H.iperm.as<int32_t>(), yc, y, ldy, alpha, H.overwrite);
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

template <typename XT>
void run_pass_c(h2_handle_s& H, int rcur, const XT* x, int64_t ldx, XT* y, int64_t ldy, double alpha,
                hipStream_t st) {
  const Structure& S = H.S;
  const int64_t n = S.n;
  const int nc = S.nclusters;
  const int nl = static_cast<int>(S.leaves.size());
  float* xc = H.mxc.as<float>();
  float* yc = H.myc.as<float>();
  float* xh = H.mxhat.as<float>();
  float* yh = H.myhat.as<float>();
  auto grid8 = [&](int64_t items) {
    const unsigned g = nblk((items + 3) / 4 * 4, 4);
    return (g + 7) / 8 * 8;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr, e4 = nullptr;
  if (H.prof) {
    e0 = prof_event(H);
    H2_HIP(hipEventRecord(e0, st));
  }
  const unsigned ptiles = nblk(n, 64);
  mpermute_in_c<XT><<<ptiles, 256, 0, st>>>(n, rcur, H.iperm.as<int32_t>(), x, ldx, xc);
  mleaf_forward<1><<<(nl + 7) / 8 * 8, 256, 0, st>>>(nl, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                              H.cend.as<int32_t>(), H.Vf.as<float>(), xc, xh);
  for (int lv = S.depth - 1; lv >= 0; --lv) {
    const int cnt = static_cast<int>(H.up_ptr[lv + 1] - H.up_ptr[lv]);
    if (cnt == 0) continue;
    if (H.kron)
      mtransfer_up_kron<1><<<(cnt + 7) / 8 * 8, 256, 0, st>>>(cnt, H.up_list.as<int32_t>() + H.up_ptr[lv],
                                                       H.child0.as<int32_t>(), H.child1.as<int32_t>(),
                                                       H.E1.as<float>(), xh);
    else
      mtransfer_up<1><<<grid8(cnt), 256, 0, st>>>(cnt, H.up_list.as<int32_t>() + H.up_ptr[lv],
                                                  H.child0.as<int32_t>(), H.child1.as<int32_t>(), H.ET.as<float>(), xh);
  }
  if (H.prof) {
    e1 = prof_event(H);
    H2_HIP(hipEventRecord(e1, st));
  }
  ensure_row_order(H);
  if (H.otf)
    mcoupling_c_otf<<<static_cast<unsigned>(H.morder_items / 4), 256, 0, st>>>(
        H.morder_items, H.morder.as<int32_t>(), H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(), H.ctr.as<double>(),
        H.off32.as<float>(), static_cast<float>(H.P.kappa), xh, yh);
  else
    mcoupling_c<<<static_cast<unsigned>(H.morder_items / 4), 256, 0, st>>>(
        H.morder_items, H.morder.as<int32_t>(), H.adm_ptr.as<int64_t>(), H.adm_col.as<int32_t>(), H.Smat.as<float>(),
        xh, yh);
  if (H.prof) {
    e2 = prof_event(H);
    H2_HIP(hipEventRecord(e2, st));
  }
  for (int lv = 0; lv < S.depth; ++lv) {
    const int first = S.level_ptr[lv + 1], cnt = S.level_ptr[lv + 2] - S.level_ptr[lv + 1];
    if (cnt == 0) continue;
    if (H.kron)
      mtransfer_down_kron<1><<<(cnt + 7) / 8 * 8, 256, 0, st>>>(first, cnt, H.parent.as<int32_t>(), H.E1.as<float>(), yh);
    else
      mtransfer_down<1><<<grid8(cnt), 256, 0, st>>>(first, cnt, H.parent.as<int32_t>(), H.F.as<float>(), yh);
  }
  if (H.prof) {
    e3 = prof_event(H);
    H2_HIP(hipEventRecord(e3, st));
  }
  if (H.near_row64)
    mnear_stream16c<<<((nl + 1) / 2 + 7) / 8 * 8, 256, 0, st>>>(nl, H.near_rows.as<NearRow>(),
                                                               H.near_blocks.as<NearBlock>(), H.Nmat.as<float>(),
                                                               H.Vb.as<float>(), xc, yh, yc);
  else
    mnear_backward16c<<<grid8(nl), 256, 0, st>>>(nl, H.leaves.as<int32_t>(), H.cbegin.as<int32_t>(),
                                                  H.cend.as<int32_t>(), H.near_ptr.as<int64_t>(),
                                                  H.near_col.as<int32_t>(), H.panel_off.as<int64_t>(),
                                                  H.Nmat.as<float>(), H.Vb.as<float>(), xc, yh, yc);
  mpermute_out_c<XT><<<ptiles, 256, 0, st>>>(n, rcur, H.iperm.as<int32_t>(), yc, y, ldy, alpha, H.overwrite);
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

}  // namespace

bool matvec_multi_supported(const h2_handle_s& H) {
  if (H.host_only || H.P.storage != H2_F32 || H.S.k != 64) return false;
  if (H.S.sym_s || H.S.sym_n) return false;  // kept blocks are applied by the single-vector kernels
  for (int32_t c : H.S.leaves)
    if (H.S.cend[c] - H.S.cbegin[c] > 64) return false;  // one MFMA K-chunk per leaf
  return true;
}

// columns per pass of the many-RHS path and the workspace bytes it needs
static int pass_columns(const h2_handle_s& H, int nrhs, int dtype) {
  const bool cx = dtype == H2_C128 || dtype == H2_C64;
  return cx ? 32 : H.tune_pass == 32 || H.tune_pass == 64 ? H.tune_pass : (nrhs <= 32 ? 32 : 64);
}

bool matvec_multi_ready(const h2_handle_s& H, int nrhs, int dtype) {
  const int rp = pass_columns(H, nrhs, dtype);
  const size_t need_v = static_cast<size_t>(H.S.n) * rp * 4, need_h = static_cast<size_t>(H.S.nclusters) * 64 * rp * 4;
  return H.mxc.bytes >= need_v && H.mxhat.bytes >= need_h && H.morder.p != nullptr &&
         H.morder_kind == row_schedule(H);
}

void matvec_multi(h2_handle_s& H, int nrhs, int dtype, const void* x, int64_t ldx, void* y, int64_t ldy,
                  double alpha, hipStream_t st) {
  const bool cx = dtype == H2_C128 || dtype == H2_C64;
  const int rp = pass_columns(H, nrhs, dtype);
  const Structure& S = H.S;
  const size_t need_v = static_cast<size_t>(S.n) * rp * 4, need_h = static_cast<size_t>(S.nclusters) * 64 * rp * 4;
  if (H.mxc.bytes < need_v || H.mxhat.bytes < need_h) {
    // workspaces grow on demand (the first many-RHS call allocates)
    H2_HIP(hipStreamSynchronize(st));
    H.mxc.alloc(need_v);
    H.myc.alloc(need_v);
    H.mxhat.alloc(need_h);
    H.myhat.alloc(need_h);
  }
  if (cx) {  // 16 complex columns per pass
    const size_t ces = dtype == H2_C128 ? 16 : 8;
    for (int j0 = 0; j0 < nrhs; j0 += 16) {
      const int rcur = std::min(16, nrhs - j0);
      const void* xj = static_cast<const char*>(x) + static_cast<size_t>(j0) * ldx * ces;
      void* yj = static_cast<char*>(y) + static_cast<size_t>(j0) * ldy * ces;
      if (dtype == H2_C128)
        run_pass_c<double>(H, rcur, static_cast<const double*>(xj), ldx, static_cast<double*>(yj), ldy, alpha, st);
      else
        run_pass_c<float>(H, rcur, static_cast<const float*>(xj), ldx, static_cast<float*>(yj), ldy, alpha, st);
    }
    return;
  }
  const size_t es = dtype == H2_R64 ? 8 : 4;
  for (int j0 = 0; j0 < nrhs; j0 += rp) {
    const int rcur = std::min(rp, nrhs - j0);
    const void* xj = static_cast<const char*>(x) + static_cast<size_t>(j0) * ldx * es;
    void* yj = static_cast<char*>(y) + static_cast<size_t>(j0) * ldy * es;
    if (rp == 32) {
      if (dtype == H2_R64)
        run_pass<1, double>(H, rcur, static_cast<const double*>(xj), ldx, static_cast<double*>(yj), ldy, alpha, st);
      else
        run_pass<1, float>(H, rcur, static_cast<const float*>(xj), ldx, static_cast<float*>(yj), ldy, alpha, st);
    } else {
      if (dtype == H2_R64)
        run_pass<2, double>(H, rcur, static_cast<const double*>(xj), ldx, static_cast<double*>(yj), ldy, alpha, st);
      else
        run_pass<2, float>(H, rcur, static_cast<const float*>(xj), ldx, static_cast<float*>(yj), ldy, alpha, st);
    }
  }
}

}  // namespace h2

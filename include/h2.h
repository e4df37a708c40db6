/*
 * h2.h -- C ABI of the MI355X H^2-matrix library.
 *
 * The library builds and applies the interpolation-based H^2 approximation
 * G~ of the Galerkin matrix G of a boundary integral operator (Boerm,
 * "Distributed H^2-matrices for boundary element methods"):
 *
 *   g_ij = int_{T_i} int_{T_j} g(x, y) dy dx      (Introduction, def. of g_ij)
 *
 * with piecewise-constant test and trial functions phi_i = psi_i = indicator
 * of triangle T_i, the Laplace kernel g = 1/(4 pi |x-y|) or the Helmholtz
 * kernel g = exp(i kappa |x-y|)/(4 pi |x-y|) (Introduction).  G~ consists of
 * (Section "H^2-matrices"):
 *   - a cluster tree (Definition 1) built by bisection of triangle centroids,
 *     clusters being minimal axis-parallel boxes containing their triangles;
 *   - a block tree whose admissible leaves satisfy
 *     max(diam tau, diam sigma) <= 2 eta dist(tau, sigma)  (eq. admissibility);
 *   - leaf matrices V_tau (eq. leafV), transfer matrices E_tau (eq. transfer)
 *     and coupling matrices S_{tau sigma} (eq. coupling) from tensor Chebyshev
 *     interpolation of order m (k = m^3 points per cluster);
 *   - dense near-field blocks for the inadmissible leaves, evaluated with
 *     Radon's 7-point rule per triangle, or Sauter-Schwab quadrature of order
 *     q_ss for triangles that share a vertex (Section "Distributed H^2-matrices",
 *     experiments: Sauter-Schwab quadrature).
 * The product y <- y + alpha G~ x is evaluated on the GPU by the three phases of
 * the paper's matrix-vector multiplication: forward transformation (Algorithm 1),
 * interaction phase (Algorithm 3) and backward transformation (Algorithm 2).
 *
 * Conventions for every entry point:
 *   - Return value: H2_OK (0) on success, a negative H2_E* code on failure;
 *     h2_last_error() then returns a thread-local message.  No C++ exception
 *     crosses this interface.  A failed call leaves a valid handle valid.
 *   - Vectors x, y, b, z are DEVICE pointers owned by the caller, column-major
 *     n x nrhs with leading dimension ld >= n, in the ORIGINAL triangle order.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Matrix
 *     products are asynchronous on that stream; h2_solve returns when done.
 *   - Mesh arrays are HOST pointers, copied by build_h2; the caller keeps them.
 *   - The handle owns all device memory of the matrix; h2_free releases it.
 *   - Calls on one handle must not overlap in time (one handle, one stream at a
 *     time); different handles are independent.
 */
#ifndef H2_MI355X_H
#define H2_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define H2_OK 0
#define H2_EINVAL (-1)    /* invalid argument */
#define H2_ENOMEM (-2)    /* device or host allocation failed */
#define H2_EHIP (-3)      /* HIP runtime error */
#define H2_ENOTCONV (-4)  /* solver did not reach the tolerance (outputs still written) */
#define H2_EINTERNAL (-5) /* unexpected internal error */

/* kernel functions g(x, y) */
#define H2_LAPLACE 0        /* 1/(4 pi |x-y|) */
#define H2_HELMHOLTZ 1      /* exp(i kappa |x-y|)/(4 pi |x-y|), complex matrix */
#define H2_TEST_ONE 2       /* g = 1; closed-form test kernel */
#define H2_TEST_BILINEAR 3  /* g = x.y; closed-form test kernel */
#define H2_TEST_QUADRATIC 4 /* g = (x.y)^2; closed-form test kernel */

/* storage precision of V, E, S and the near field */
#define H2_F64 0       /* everything FP64 */
#define H2_F32 1       /* everything FP32 */
#define H2_F32_SBF16 2 /* coupling matrices BF16, the rest FP32; S is also kept in FP32
                          for the products with H2_ACC_F64 (the outer residual of iterative
                          refinement), so BF16 S only ever serves the inner solves */

/* element type of user vectors */
#define H2_R64 0  /* double */
#define H2_R32 1  /* float */
#define H2_C128 2 /* complex double, interleaved (re, im); Helmholtz only */
#define H2_C64 3  /* complex float, interleaved (re, im); Helmholtz only */

/* h2_matvec flags */
#define H2_ACC_F64 1 /* accumulate in FP64 even when the matrix is stored in FP32/BF16;
                        with H2_F32_SBF16 storage the product applies the FP32 copy of S */
#define H2_OVERWRITE 2 /* assign y <- alpha G~ x instead of accumulating (y is not read) */

/* h2_params.flags */
#define H2_HOST_ONLY 1   /* build only the trees (no device work); for structure inspection */
#define H2_COUPLING_OTF 2 /* do not store the coupling matrices: every product evaluates
                             s_{nu mu} = g(xi_{tau,nu}, xi_{sigma,mu}) (eq. coupling) from the
                             clusters' interpolation points.  Real kernels: FP64 storage
                             evaluates in FP64, FP32 storage in FP32 from FP64 cluster-centre
                             differences plus FP32 offsets.  Helmholtz: FP32 storage and m = 4
                             only, evaluated the same way in FP32 with the sine and cosine of
                             kappa r by quadrant reduction and Taylor polynomials. */

#define H2_SYMMETRIC 4    /* store one block of every symmetric pair (G~ = G~^T because test and
                             trial spaces coincide and g is symmetric): coupling blocks (tau,
                             sigma) with sigma > tau and near-field blocks whose column leaf is
                             not before the row leaf; each kept off-diagonal block is applied
                             as itself and as its transpose.  Real kernels, FP64 or FP32
                             storage, k = 64, leaves of at most 64 triangles; single right-hand
                             side kernels (several columns are applied one at a time).  With
                             H2_COUPLING_OTF only the near field is halved. */
#define H2_SYMMETRIC_NEAR 8 /* the near-field half of H2_SYMMETRIC only: coupling blocks stay
                             stored in full (so h2_recompress applies), near-field blocks are kept
                             once per symmetric pair.  Real kernels, FP64 or FP32 storage, any
                             order m, leaves of at most 64 triangles; single right-hand side
                             kernels.  Together with H2_SYMMETRIC it is H2_SYMMETRIC. */

typedef struct h2_handle_s* h2_handle;

typedef struct {
  int64_t nv;               /* number of vertices */
  int64_t nt;               /* number of triangles = n */
  const double* vertices;   /* nv x 3, row-major, host */
  const int32_t* triangles; /* nt x 3 vertex indices, row-major, host */
} h2_mesh;

typedef struct {
  int kernel;     /* H2_LAPLACE, ...                                          */
  double kappa;   /* Helmholtz wave number (ignored otherwise)                */
  int order_m;    /* interpolation points per axis, 1..6; k = m^3             */
  int leaf_size;  /* clusters with more triangles are split                   */
  double eta;     /* admissibility parameter of eq. admissibility             */
  int q_ss;       /* Gauss-Legendre order per axis of the Sauter-Schwab rules */
  int storage;    /* H2_F64, H2_F32, H2_F32_SBF16                             */
  int flags;      /* 0 or any of H2_HOST_ONLY, H2_COUPLING_OTF, H2_SYMMETRIC,
                     H2_SYMMETRIC_NEAR                                          */
} h2_params;

typedef struct {
  int64_t n, nclusters, nleaves, depth, n_adm, n_near, near_entries;
  int64_t m, k, storage, kernel;
  int64_t bytes_S, bytes_N, bytes_V, bytes_E, bytes_total; /* device storage */
  double matvec_bytes; /* algorithmic HBM bytes of one single-vector product:
                          V twice, E twice, S once, near field once */
  double matvec_flops; /* 2 flops per stored scalar used (x4 for complex)    */
  int64_t s_blocks_stored;     /* coupling blocks held in memory (0 on the fly)  */
  int64_t near_entries_stored; /* near-field entries held in memory              */
} h2_stats;

/* Builds the H^2 matrix of the mesh (trees on the host, all matrix entries on
 * the current HIP device).  *out receives a new handle on success. */
int build_h2(const h2_mesh* mesh, const h2_params* params, h2_handle* out);

/* y <- y + alpha G~ x for nrhs columns.  dtype: H2_R64 or H2_R32 for real
 * kernels, H2_C128 or H2_C64 (interleaved complex, ld counted in complex
 * elements) for the Helmholtz kernel; alpha is real.  flags: 0 or any of
 * H2_ACC_F64, H2_OVERWRITE.
 * Asynchronous on `stream`. */
int h2_matvec(h2_handle h, int nrhs, int dtype, const void* x, int64_t ldx, void* y, int64_t ldy,
              double alpha, int flags, void* stream);

/* Solver for G~ z = b (Introduction: Krylov methods). */
#define H2_CG 0
#define H2_GMRES 1
typedef struct {
  int method;        /* H2_CG (Laplace: G~ symmetric positive definite) or H2_GMRES */
  int restart;       /* GMRES restart length, 1..120                                */
  int maxit;         /* maximum number of inner iterations in total                 */
  double rtol;       /* stop when ||b_j - G~ z_j|| <= rtol ||b_j|| for every column j */
  int refine;        /* 0: plain solve with the matrix's own accumulation;
                        1: FP64 iterative refinement -- outer residuals from products
                           with H2_ACC_F64 (FP64 accumulation; with H2_F32_SBF16 the
                           FP32 copy of S), inner solves with the storage precision's
                           accumulation to inner_rtol                              */
  double inner_rtol; /* inner tolerance of the refinement, in (0, 1)               */
} h2_solve_params;

typedef struct {
  int iterations;       /* total inner iterations (one product each)          */
  int outer;            /* inner solves started (refinement steps)            */
  double rel_residual;  /* max over columns of ||b - G~ z|| / ||b||, FP64,
                           from the last outer residual                      */
  double seconds;       /* wall time                                          */
} h2_solve_info;

/* Solves G~ Z = B for nrhs columns at once (device blocks, column-major,
 * leading dimensions ldb, ldz >= n; dtype H2_R64 for real kernels, H2_C128 for
 * Helmholtz, which requires H2_GMRES).  Z is both the initial guess and the
 * result.  Every iteration applies one product to all columns (the many-
 * right-hand-side path when nrhs >= 2); inner products, the GMRES Hessenberg
 * columns, Givens rotations and triangular solves are FP64 on the device; the
 * host reads one residual per column and iteration.  The handle keeps the
 * solver's workspace (about (5 + restart) n nrhs FP64 values) for later calls.
 * Returns H2_ENOTCONV if some column missed rtol (Z and info still written),
 * also when a non-finite value appeared (h2_last_error says which). */
int h2_solve(h2_handle h, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
             const h2_solve_params* p, h2_solve_info* info, void* stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid allocation):
 * h2_solve without any allocation.  The solver's workspace and its two
 * n x nrhs product buffers live in a fixed device array of the library
 * (H2_NOALLOC_SCRATCH_BYTES = 256 MiB per GPU, held from the library's load on
 * that GPU until the process ends); the residual status is read into host stack
 * memory; products with several columns use the many-right-hand-side path only
 * if the handle already holds its workspaces (after an h2_matvec or h2_solve
 * with as many columns), else they apply the columns one at a time.  H2_EINVAL
 * when the solve needs more than the array (about (5 + restart) n nrhs FP64
 * values plus 2 n nrhs for the products) or nrhs > H2_NOALLOC_MAX_RHS; otherwise
 * as h2_solve.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other threads, other streams) race. */
#define H2_NOALLOC_SCRATCH_BYTES (256ll << 20)
#define H2_NOALLOC_MAX_RHS 64
int h2_solve_noalloc(h2_handle h, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
                     const h2_solve_params* p, h2_solve_info* info, void* stream);

/* Step-wise form of the same solver, for callers that batch the products of
 * several solves (the solve service issues one many-right-hand-side product
 * per matrix for all the solves that wait on it).  The solver never touches a
 * matrix: it writes the block X whose product it needs and consumes Y = G~ X.
 *   h2_krylov_workspace  device bytes a solve of nrhs columns of length n needs
 *                        (-1 for invalid arguments)
 *   h2_krylov_create     a solver on caller-owned DEVICE memory `workspace`
 *                        (256-byte aligned, >= the bytes above, kept until
 *                        destroy) and optional caller-owned PINNED host memory
 *                        `host_status` of 3 nrhs doubles (NULL: the solver
 *                        allocates its own); allocates no device memory
 *   h2_krylov_begin      starts a solve of G~ Z = B; b must stay valid and
 *                        unchanged until the solve ends; z0 = NULL means Z = 0
 *   h2_krylov_next       returns H2_KS_PRODUCT and writes the block X (n x nrhs,
 *                        ldx) whose product is needed, with the h2_matvec flags
 *                        it needs in *flags (H2_ACC_F64 for the outer residual
 *                        of a refinement); or returns the final state.  With
 *                        x = NULL it only reports the state and the flags (no
 *                        device work), so a caller can group solves by flags
 *   h2_krylov_advance    consumes Y = G~ X (ldy), computed with those flags
 *   h2_krylov_poll       after the stream has completed the advance: takes the
 *                        control decisions and returns the state; st may be NULL
 *   h2_krylov_residuals  relative outer residual per column (host copy, nrhs)
 *   h2_krylov_solution   copies Z into z (ldz)
 * next, advance and solution are asynchronous on `stream`; one solver must stay
 * on one stream.  Calls return a negative H2_E* code on invalid use. */
#define H2_KS_PRODUCT 1  /* the solve needs another product                  */
#define H2_KS_DONE 2     /* every column met rtol                             */
#define H2_KS_NOTCONV 3  /* maxit or the refinement steps ran out             */
#define H2_KS_FAILED 4   /* a non-finite value appeared; see message          */
typedef struct h2_krylov_s* h2_krylov;
typedef struct {
  int state;
  int iterations;
  int outer;
  int products;
  double rel_residual; /* max over columns of the latest relative residual   */
  char message[128];
} h2_krylov_status;
int64_t h2_krylov_workspace(int dtype, int64_t n, int nrhs, const h2_solve_params* p);
int h2_krylov_create(int dtype, int64_t n, int nrhs, const h2_solve_params* p, void* workspace, int64_t bytes,
                     double* host_status, h2_krylov* out);
int h2_krylov_begin(h2_krylov k, const void* b, int64_t ldb, const void* z0, int64_t ldz, void* stream);
int h2_krylov_next(h2_krylov k, void* x, int64_t ldx, int* flags, void* stream);
int h2_krylov_advance(h2_krylov k, const void* y, int64_t ldy, void* stream);
int h2_krylov_poll(h2_krylov k, h2_krylov_status* st);
int h2_krylov_residuals(h2_krylov k, double* out);
int h2_krylov_solution(h2_krylov k, void* z, int64_t ldz, void* stream);
void h2_krylov_destroy(h2_krylov k);

/* Algebraic recompression (a smaller-rank H^2 matrix of the same block
 * structure; the paper names such approximations as future work: the GCA-H^2
 * variant in the section on distributed matrix setup, the recompression
 * algorithm in the outlook).  The cluster bases are made orthonormal and
 * nested (QR, bottom up), every cluster's basis is truncated to the dominant
 * eigenvectors of the weight of all admissible blocks it carries, including
 * those inherited from its ancestors, and the coupling matrices are projected.
 * Every cluster is then padded to one rank k' (the largest rank rounded up to a
 * multiple of 4, but never above k) and the handle's V, E and S are
 * replaced in place: products (h2_matvec, h2_solve) use k' from then on, the
 * near field is unchanged.
 *   eps       relative tolerance per cluster: keep the eigenvalues of its
 *             weight above eps^2 times the largest; 0 = orthogonalise only
 *             (the represented matrix stays G~ up to rounding)
 *   max_rank  0, or a cap on every cluster's rank
 *   info      may be NULL; on success:
 *               rank          k' (every cluster padded to it)
 *               rank_before   k
 *               discarded     sum of the discarded eigenvalues; the change
 *                             satisfies ||G~ - G~'||_F^2 <= 2 * discarded
 *               seconds       wall time
 *               bytes_before / bytes_after   device bytes of V, E and S
 * Requires a real kernel, H2_F64 or H2_F32 storage, stored coupling matrices
 * (not H2_COUPLING_OTF) and full coupling storage (not H2_SYMMETRIC; the
 * near-field-only H2_SYMMETRIC_NEAR is fine); H2_EINVAL
 * otherwise, or for eps < 0 / not finite, max_rank < 0.  Runs its device
 * kernels on `stream` and returns after completion; the factorisations run on
 * the host in FP64.  After recompression with k' != 64 several columns are
 * applied one at a time. */
typedef struct {
  int64_t rank;
  int64_t rank_before;
  double discarded;
  double seconds;
  int64_t bytes_before;
  int64_t bytes_after;
} h2_recompress_info;
int h2_recompress(h2_handle h, double eps, int max_rank, h2_recompress_info* info, void* stream);

/* Tile-shape autotuning of the product y <- y + alpha G~ x (Algorithms 1-3 of the
 * section on the matrix-vector multiplication; the tile shapes are this
 * library's, not the paper's).  One knob decides the tiles of the path a call
 * takes; several values compute the same product with different tiles (and a
 * different summation order, within the storage precision):
 *   H2_TUNE_PASS_COLUMNS  many right-hand sides (nrhs >= 2) on the matrix-core
 *                         path: real kernels, H2_F32 storage, k = 64, leaves of
 *                         at most 64 triangles, no symmetric storage, S stored
 *                         or on the fly.  Right-hand sides per pass: 32 (one
 *                         32x32 MFMA column tile per wave in the coupling, two
 *                         16-column near-field tiles) or 64 (two and four).
 *                         Built-in rule: 32 if nrhs <= 32, else 64.
 *   H2_TUNE_SMALL_SLOT    single-vector coupling with k <= 32 (recompressed
 *                         bases): lanes per block-row slot of a wave, 16 (four
 *                         blocks of a row cluster at a time, needs k <= 16) or 32
 *                         (two).  Built-in rule: 16 if k <= 16, else 32.
 *   H2_TUNE_ROW_ORDER     many right-hand sides on the matrix-core path (real
 *                         or complex): how the workgroups of the coupling
 *                         kernels take the row clusters, 1 (one row per wave,
 *                         eight contiguous ranges of equal work, one per XCD:
 *                         rows that share column clusters share an L2), 2
 *                         (natural order, four rows per workgroup, workgroups
 *                         dealt round-robin to the XCDs) or 3 (real stored S,
 *                         64-column passes: four neighbouring row clusters per
 *                         workgroup, each x^_sigma they share staged once in LDS
 *                         for all four; the same sums in the same order as 1;
 *                         other passes take 1).  Built-in rule: 3 for real
 *                         stored S, else 1.  Only h2_tune_knob tunes it.
 * h2_tune runs the product the way h2_matvec(h, nrhs, dtype, ...) would, with
 * every value of the knob that path has: one untimed and `reps` timed products
 * each on library-owned vectors (allocated for the call), timed with HIP events
 * on `stream`; it keeps the value with the smallest median time and fills info:
 *   knob          the knob tuned, H2_TUNE_NONE if the path has no alternatives
 *                 (complex kernels; single vectors with on-the-fly or symmetric
 *                 coupling or k > 16; many right-hand sides that are applied one
 *                 at a time with k > 16)
 *   ncand         number of values timed (0 with H2_TUNE_NONE)
 *   value[i]      the values, ms[i] their median milliseconds per product call
 *   chosen        index of the value kept
 * Synchronizes `stream`.  The choice stays with the handle for every later call
 * until h2_set_tuning or h2_recompress (which resets H2_TUNE_SMALL_SLOT) changes
 * it.  H2_EINVAL for nrhs < 1, reps < 1 or 1000 < reps, a host-only handle, or
 * what h2_matvec rejects.
 * h2_set_tuning sets a knob directly: value 0 restores the built-in rule;
 * H2_EINVAL for an unknown knob or a value outside the list above (16 for
 * H2_TUNE_SMALL_SLOT while k > 16). */
#define H2_TUNE_NONE (-1)
#define H2_TUNE_PASS_COLUMNS 0
#define H2_TUNE_SMALL_SLOT 1
#define H2_TUNE_ROW_ORDER 2
typedef struct {
  int knob;
  int ncand;
  int value[4];
  double ms[4];
  int chosen;
} h2_tune_info;
int h2_tune(h2_handle h, int nrhs, int dtype, int reps, h2_tune_info* info, void* stream);
/* h2_tune for one given knob of the path (info.knob = H2_TUNE_NONE if the path
 * does not have it). */
int h2_tune_knob(h2_handle h, int knob, int nrhs, int dtype, int reps, h2_tune_info* info, void* stream);
int h2_set_tuning(h2_handle h, int knob, int value);

int h2_info(h2_handle h, h2_stats* out);
void h2_free(h2_handle h);
const char* h2_last_error(void);

/* Structure and data export for inspection and tests (host copies).
 * what: H2_X_PERM      int32[n]           position -> triangle
 *       H2_X_CLUSTERS  int32[nclusters*6] begin, end, parent, child0, child1, level
 *       H2_X_BOXES     double[nclusters*6] lo xyz, hi xyz
 *       H2_X_ADM       int32[n_adm*2]     (row cluster, column cluster)
 *       H2_X_NEAR      int32[n_near*2]    (row cluster, column cluster)
 *       H2_X_DFS       int32[nclusters]   depth-first pre-order number
 *       H2_X_V         double[|tau| * k]  leaf matrix of cluster `index` (row-major)
 *       H2_X_E         double[k * k]      transfer matrix of cluster `index` (row nu')
 *       H2_X_S         double[k * k]      coupling matrix of admissible block `index`
 *       H2_X_N         double[|tau|*|sigma|] near block `index` (row-major)
 * For complex kernels H2_X_S and H2_X_N return interleaved (re, im) pairs.
 * `cap` is the capacity of dst in elements; H2_EINVAL if too small. */
#define H2_X_PERM 0
#define H2_X_CLUSTERS 1
#define H2_X_BOXES 2
#define H2_X_ADM 3
#define H2_X_NEAR 4
#define H2_X_DFS 5
#define H2_X_V 6
#define H2_X_E 7
#define H2_X_S 8
#define H2_X_N 9
int h2_export(h2_handle h, int what, int64_t index, void* dst, int64_t cap);

/* Batched Krylov vector kernels for many independent right-hand sides (the
 * Gram-Schmidt and update steps of GMRES; Introduction: Krylov methods).
 * dtype H2_R64 (double) or H2_C128 (interleaved complex double); DEVICE data:
 *   Q: element k of basis vector i of right-hand side r at
 *      Q[r * q_rhs_stride + i * q_vec_stride + k]   (strides in elements)
 *   W: element k of right-hand side r at W[r * w_rhs_stride + k]
 *   h: nrhs x nvec, row-major.
 * h2_krylov_dots:   h[r][i] = sum_k conj(Q[r][i][k]) W[r][k]
 * h2_krylov_update: W[r][k] += sign * sum_i h[r][i] Q[r][i][k]
 * Asynchronous on `stream`; deterministic (fixed reduction order); no handle
 * and no allocation. */
int h2_krylov_dots(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t q_rhs_stride,
                   int64_t q_vec_stride, const void* W, int64_t w_rhs_stride, void* h, void* stream);
int h2_krylov_update(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t q_rhs_stride,
                     int64_t q_vec_stride, const void* h, double sign, void* W, int64_t w_rhs_stride,
                     void* stream);

/* Measurement utility: reads `bytes` (a positive multiple of 16) of DEVICE memory
 * at `data` (16-byte aligned) with 16-byte non-temporal loads, `loads` (4, 8 or
 * 16) in flight per thread, each workgroup on contiguous tiles of 256 x loads
 * vectors, the way the bandwidth-bound product kernels stream their data, and
 * writes nothing in practice (`sink`, DEVICE memory of at least 16 KiB, keeps
 * the loads live).  Timed by the caller; bytes / time is the HBM read rate a
 * plain kernel reaches, the measured ceiling beside the vendor peak.
 * Asynchronous on `stream`. */
int h2_stream_read(const void* data, int64_t bytes, int loads, void* sink, int64_t sink_bytes, void* stream);

/* Per-phase device timing of h2_matvec (HIP events on the call's stream).
 * h2_profile(h, 1) enables and clears; h2_profile(h, 0) disables.
 * h2_profile_read fills ms[H2_NPHASE] with summed milliseconds and
 * calls[H2_NPHASE] with launch counts since the last clear (synchronizes). */
#define H2_PH_FORWARD 0  /* permute-in, leaf forward, transfer up        */
#define H2_PH_COUPLING 1 /* coupling S x-hat                              */
#define H2_PH_DOWN 2     /* transfer down                                 */
#define H2_PH_NEAR 3     /* near field + leaf backward (+ permute-out)    */
#define H2_PH_TOTAL 4    /* the whole product                              */
#define H2_NPHASE 5
int h2_profile(h2_handle h, int enable);
int h2_profile_read(h2_handle h, double* ms, int64_t* calls);

#ifdef __cplusplus
}
#endif
#endif /* H2_MI355X_H */

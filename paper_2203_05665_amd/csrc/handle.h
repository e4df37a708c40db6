// Internal state of an h2_handle: host structure, device arrays, workspaces.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/h2.h"
#include "structure.h"

namespace h2 {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define H2_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::h2::Error(e_ == hipErrorOutOfMemory ? H2_ENOMEM : H2_EHIP,                    \
                        std::string(#call) + ": " + hipGetErrorString(e_));                 \
  } while (0)

// Owning device allocation.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 16;
    H2_HIP(hipMalloc(&p, b));
    bytes = b;
  }
  template <class T>
  void upload(const std::vector<T>& v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) H2_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// One row leaf of the near field for near_backward64: its panel, its first near
// block, its triangles and its cluster.
struct NearRow {
  int64_t panel_off;  // element offset of the panel
  int64_t bfirst;     // first near block (index into near_col)
  int32_t b0, r;      // first triangle (cluster order) and triangle count
  int32_t nb, tau;    // near blocks of the row; cluster id
};

// One near block for near_backward64: first triangle s0 and width w of the column
// leaf sigma, first column cb of the block in the row's panel (pad: unused).
struct NearBlock {
  int32_t s0, w, cb, pad;
};

// One row cluster of the single-vector coupling evaluated during the product: its
// first admissible block, its block count and its id.  The table lists the rows
// heaviest first.
struct RowSpan {
  int64_t b0;
  int32_t nb, tau;
};

// bf16 storage element (upper half of an IEEE float).
struct bf16 {
  uint16_t v;
};

}  // namespace h2

struct h2_handle_s {
  h2::Structure S;
  h2_params P{};
  bool host_only = false;
  bool is_complex = false;
  bool otf = false;       // coupling matrices evaluated during the product
  int device = 0;
  size_t val_bytes = 8;   // bytes per stored real scalar of V, E, N
  size_t s_bytes = 8;     // bytes per stored real scalar of S
  // device structure
  h2::DBuf perm, cbegin, cend, parent, child0, child1, leaves, adm_ptr, adm_col, near_ptr, near_col,
      panel_off, up_list, pts;
  h2::DBuf iperm;  // inverse of perm: the cluster-order position of every user index
  // near_backward64's descriptors (h2::NearRow per leaf, h2::NearBlock per near
  // block); near64: every leaf holds at most 64 triangles and every row at most 256
  // near blocks, so that kernel applies
  h2::DBuf near_rows, near_blocks;
  // the rows of the single-vector coupling evaluated during the product, heaviest
  // first (h2::RowSpan)
  h2::DBuf row_spans;
  bool near64 = false;
  bool near_row64 = false;  // also at most 64 near blocks per row (mnear_stream16 applies)
  // on-the-fly coupling: cluster centres (FP64, 3 per cluster) and point offsets from
  // the centre (3 x m per cluster, FP32 and FP64)
  h2::DBuf ctr, off32, off64;
  std::vector<int64_t> up_ptr;  // host offsets into up_list per level
  // the top levels of the transfer sweeps that run in one workgroup: up levels
  // 0..up_top-1, down parent levels 0..down_top-1 (each at most 64 clusters, four
  // rounds of the single-vector kernel's 16 waves); mup_top / mdown_top likewise for
  // the many-column sweeps, whose per-cluster work is larger (at most 8 clusters a
  // level, one round of that kernel's 8 waves)
  int up_top = 0, down_top = 0, mup_top = 0, mdown_top = 0;
  h2::DBuf up_ptr_dev, level_ptr_dev;
  // matrix data
  h2::DBuf Vf, Vb, F, ET, Smat, Nmat;
  // H2_F32_SBF16: the coupling matrices also in FP32, for products with FP64
  // accumulation (the outer residual of iterative refinement); BF16 S serves the rest
  h2::DBuf Smat32;
  // E_c = E_x (x) E_y (x) E_z: per cluster the three m x m one-dimensional factors,
  // E1[c][d][i][j] = l_j(xi_i) along axis d (i child point, j parent polynomial)
  h2::DBuf E1;
  bool kron = false;  // transfers applied through E1 (interpolation bases, k = 64)
  // symmetric storage: incoming lists, near-field scratch slots, and the scratch
  // of the transposed products (sized for FP64 accumulation)
  h2::DBuf adm_in_ptr, adm_in_blk, near_slot, near_in_ptr, near_in_slot, leaf_of_pos, scr_s, scr_n;
  // workspaces (sized for FP64 vectors, one right-hand side)
  h2::DBuf xc, yc, xhat, yhat;
  // many-right-hand-side workspaces (FP32, grown on first use) and the row order
  // of the coupling kernels (built on first use)
  h2::DBuf mxc, myc, mxhat, myhat, morder;
  int64_t morder_items = 0;
  // tile choices (0: the built-in rule), set by h2_tune or h2_set_tuning
  int tune_pass = 0;  // right-hand sides per many-RHS pass: 32 or 64
  int tune_slot = 0;  // lanes per block-row slot of the small-k coupling: 16 or 32
  int tune_order = 0; // schedule of the many-RHS coupling: 1 XCD chunks, 2 interleaved,
                      // 3 row groups sharing x^ (0: rule, 3 for real stored S, else 1)
  int morder_kind = 0;  // the schedule morder (and the groups) hold
  // schedule 3: row groups (4 cluster ids each, -1 unused), their entry ranges and
  // entries (column cluster, the block of each of the 4 rows or -1, 3 x padding)
  h2::DBuf mgrp_rows, mgrp_ptr, mgrp_tasks;
  int64_t mgrp_n = 0;
  bool overwrite = false;  // the current product assigns y <- alpha G~ x (H2_OVERWRITE)
  // h2_solve: the Krylov solver's workspace and its pinned status (kept between
  // calls, grown when a call needs more)
  h2::DBuf kws;
  double* kstat = nullptr;
  int kstat_n = 0;
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> events;     // pool
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  double ms[H2_NPHASE] = {0};
  int64_t calls[H2_NPHASE] = {0};
  ~h2_handle_s();
};

namespace h2 {
void assemble(h2_handle_s& H);  // fills Vf, Vb, F, ET, Smat, Nmat on the device
// may_alloc = false: no device allocation; the many-RHS path is taken only when
// its workspaces exist already, else the columns are applied one at a time
void matvec(h2_handle_s& H, int nrhs, int dtype, const void* x, int64_t ldx, void* y, int64_t ldy,
            double alpha, int flags, hipStream_t s, bool may_alloc = true);
bool matvec_multi_supported(const h2_handle_s& H);
bool matvec_multi_ready(const h2_handle_s& H, int nrhs, int dtype);
void matvec_multi(h2_handle_s& H, int nrhs, int dtype, const void* x, int64_t ldx, void* y, int64_t ldy,
                  double alpha, hipStream_t s);
int solve_multi(h2_handle_s& H, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
                const h2_solve_params& p, h2_solve_info& info, hipStream_t st);
int solve_noalloc(h2_handle_s& H, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
                  const h2_solve_params& p, h2_solve_info& info, hipStream_t st);
void krylov_dots(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t qr, int64_t qv, const void* W,
                 int64_t wr, void* h, hipStream_t st);
void krylov_update(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t qr, int64_t qv, const void* h,
                   double sign, void* W, int64_t wr, hipStream_t st);
void recompress(h2_handle_s& H, double eps, int max_rank, h2_recompress_info& info, hipStream_t st);
void tune(h2_handle_s& H, int nrhs, int dtype, int reps, h2_tune_info& info, hipStream_t st, int knob = -2);
void ensure_row_order(h2_handle_s& H);
void set_tuning(h2_handle_s& H, int knob, int value);
void stream_read_launch(const void* data, int64_t bytes, int loads, void* sink, int64_t sink_bytes, hipStream_t st);
hipEvent_t prof_event(h2_handle_s& H);
void prof_record(h2_handle_s& H, int phase, hipEvent_t a, hipEvent_t b);
}  // namespace h2

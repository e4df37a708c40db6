// Step-wise batched Krylov solver (internal interface; C ABI in include/h2.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/h2.h"

namespace h2 {

constexpr int kMaxRestart = 120;

// Device workspace of one solve: byte offsets of its parts and the reduction shape.
struct KLayout {
  bool cx = false, cg = true;
  int64_t n = 0;
  int r = 0, m = 0, nchunk = 1, nvmax = 1;
  int64_t csz = 0, col = 0, sc = 0;
  int64_t o_hcol = 0, o_hcur = 0, o_g = 0, o_cs = 0, o_sn = 0, o_y = 0, o_H = 0;
  size_t off_Z = 0, off_Ro = 0, off_X = 0, off_R = 0, off_P = 0, off_W = 0, off_Q = 0, off_part = 0, off_scal = 0,
         off_stat = 0, bytes = 0;
};
KLayout klayout(int dtype, int64_t n, int nrhs, const h2_solve_params& p);

class KSolver {
 public:
  KSolver(int dtype, int64_t n, int nrhs, const h2_solve_params& p, void* workspace, size_t bytes,
          double* host_status);
  ~KSolver();
  KSolver(const KSolver&) = delete;
  KSolver& operator=(const KSolver&) = delete;
  static void check_params(const h2_solve_params& p, bool cx);

  void begin(const void* b, int64_t ldb, const void* z0, int64_t ldz, hipStream_t st);
  int next(void* x, int64_t ldx, int* flags, hipStream_t st);
  void advance(const void* y, int64_t ldy, hipStream_t st);
  int poll();
  void residuals(double* out) const;
  void solution(void* z, int64_t ldz, hipStream_t st);

  KLayout L;
  h2_solve_params P;
  int state = H2_KS_PRODUCT;
  int iterations = 0, outer = 0, products = 0;
  double last_rel = 1.0;
  std::string message;

 private:
  enum Phase { PH_OUTER, PH_CG, PH_ARNOLDI, PH_RESID };
  double* d(size_t off) const;
  void partial(int nvec, const double* A, int64_t a_col, int64_t a_vec, const double* B, int64_t b_col,
               hipStream_t st);
  void finish(int op, int nvec, int j, hipStream_t st);
  void status_copy(hipStream_t st);
  void start_inner(double rel_out_max);

  char* ws = nullptr;
  double* stat_host = nullptr;
  double* own_stat = nullptr;
  const double* B = nullptr;
  int64_t b_col = 0;
  const double* rhs = nullptr;  // inner right-hand side: B, or the outer residual
  int64_t rhs_col = 0;
  Phase phase = PH_OUTER;
  bool pend_inner = false, pend_close = false, pend_zupd = false;
  int j = 0;  // GMRES: Arnoldi steps of the current cycle
  int max_outer = 1;
  double inner_tol = 1.0;
};

}  // namespace h2

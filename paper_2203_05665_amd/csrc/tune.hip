// Tile-shape autotuner of the product y <- y + alpha G~ x (the three phases of the
// section on the matrix-vector multiplication).  Each knob selects among kernels
// that compute the same product with different tiles; the tuner times every value
// the handle's path admits on the handle itself and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "handle.h"

namespace h2 {
namespace {

// x[i] = a fixed pattern in [-0.5, 0.5): timing inputs with no zeros and no
// special values
template <typename T>
__global__ void tune_fill(int64_t count, T* __restrict__ x) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) x[i] = static_cast<T>(static_cast<double>((i * 2654435761LL) % 1000) / 1000.0 - 0.5);
}

int applicable_knob(const h2_handle_s& H, int nrhs, int dtype) {
  const bool cx = dtype == H2_C128 || dtype == H2_C64;
  if (cx || H.is_complex) return H2_TUNE_NONE;
  if (nrhs >= 2 && matvec_multi_supported(H)) return H2_TUNE_PASS_COLUMNS;
  if (!H.otf && !H.S.sym_s && H.S.k <= 16) return H2_TUNE_SMALL_SLOT;  // k in 17..32: slots of 32 only
  return H2_TUNE_NONE;
}

int& knob_ref(h2_handle_s& H, int knob) {
  return knob == H2_TUNE_PASS_COLUMNS ? H.tune_pass : knob == H2_TUNE_ROW_ORDER ? H.tune_order : H.tune_slot;
}

// the knobs the path of (nrhs, dtype) has, and their values
std::vector<int> knob_values(const h2_handle_s& H, int knob, int nrhs, int dtype) {
  const bool cx = dtype == H2_C128 || dtype == H2_C64;
  if (knob == H2_TUNE_PASS_COLUMNS && !cx && nrhs >= 2 && matvec_multi_supported(H)) return {32, 64};
  if (knob == H2_TUNE_ROW_ORDER && nrhs >= 2 && matvec_multi_supported(H)) {
    if (!cx && !H.is_complex && !H.otf) return {1, 2, 3};
    return {1, 2};
  }
  if (knob == H2_TUNE_SMALL_SLOT && applicable_knob(H, nrhs, dtype) == H2_TUNE_SMALL_SLOT) return {16, 32};
  return {};
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  Events() {
    H2_HIP(hipEventCreate(&a));
    H2_HIP(hipEventCreate(&b));
  }
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

void set_tuning(h2_handle_s& H, int knob, int value) {
  if (knob == H2_TUNE_PASS_COLUMNS) {
    if (value != 0 && value != 32 && value != 64) throw Error(H2_EINVAL, "H2_TUNE_PASS_COLUMNS takes 0, 32 or 64");
    H.tune_pass = value;
  } else if (knob == H2_TUNE_SMALL_SLOT) {
    if (value != 0 && value != 16 && value != 32) throw Error(H2_EINVAL, "H2_TUNE_SMALL_SLOT takes 0, 16 or 32");
    if (value == 16 && H.S.k > 16) throw Error(H2_EINVAL, "slots of 16 lanes need k <= 16");
    H.tune_slot = value;
  } else if (knob == H2_TUNE_ROW_ORDER) {
    if (value < 0 || value > 3) throw Error(H2_EINVAL, "H2_TUNE_ROW_ORDER takes 0, 1, 2 or 3");
    H.tune_order = value;
    // a row order already in use is rebuilt now, not in a later product
    if (H.morder.p != nullptr) ensure_row_order(H);
  } else {
    throw Error(H2_EINVAL, "unknown tuning knob");
  }
}

void tune(h2_handle_s& H, int nrhs, int dtype, int reps, h2_tune_info& info, hipStream_t st, int which) {
  if (H.host_only) throw Error(H2_EINVAL, "handle was built with H2_HOST_ONLY");
  if (nrhs < 1) throw Error(H2_EINVAL, "nrhs must be >= 1");
  if (reps < 1 || reps > 1000) throw Error(H2_EINVAL, "reps must be in 1..1000");
  if (dtype != H2_R64 && dtype != H2_R32 && dtype != H2_C128 && dtype != H2_C64)
    throw Error(H2_EINVAL, "unknown dtype");
  if (which != -2 && which != H2_TUNE_PASS_COLUMNS && which != H2_TUNE_SMALL_SLOT && which != H2_TUNE_ROW_ORDER)
    throw Error(H2_EINVAL, "unknown tuning knob");
  info = h2_tune_info{};
  info.knob = which == -2 ? applicable_knob(H, nrhs, dtype) : which;
  if (info.knob == H2_TUNE_NONE) return;
  const std::vector<int> values = knob_values(H, info.knob, nrhs, dtype);
  if (values.empty()) {
    info.knob = H2_TUNE_NONE;
    return;
  }

  // trial vectors: n x nrhs entries, complex ones as interleaved pairs of scalars
  const int cw = (dtype == H2_C128 || dtype == H2_C64) ? 2 : 1;
  const bool dbl = dtype == H2_R64 || dtype == H2_C128;
  const int64_t n = H.S.n, count = n * nrhs * cw;
  const size_t es = dbl ? 8 : 4;
  DBuf xb, yb;
  xb.alloc(static_cast<size_t>(count) * es);
  yb.alloc(static_cast<size_t>(count) * es);
  const unsigned g = static_cast<unsigned>((count + 255) / 256);
  if (!dbl) tune_fill<float><<<g, 256, 0, st>>>(count, xb.as<float>());
  else tune_fill<double><<<g, 256, 0, st>>>(count, xb.as<double>());
  H2_HIP(hipGetLastError());
  H2_HIP(hipMemsetAsync(yb.p, 0, yb.bytes, st));
  int& knob = knob_ref(H, info.knob);
  const int saved = knob;
  const bool saved_prof = H.prof;
  H.prof = false;  // the trial products stay out of the phase timings
  try {
    Events ev;
    for (size_t c = 0; c < values.size(); ++c) {
      knob = values[c];
      matvec(H, nrhs, dtype, xb.p, n, yb.p, n, 1.0, 0, st);  // untimed
      std::vector<float> t(reps);
      for (int r = 0; r < reps; ++r) {
        H2_HIP(hipEventRecord(ev.a, st));
        matvec(H, nrhs, dtype, xb.p, n, yb.p, n, 1.0, 0, st);
        H2_HIP(hipEventRecord(ev.b, st));
        H2_HIP(hipEventSynchronize(ev.b));
        H2_HIP(hipEventElapsedTime(&t[r], ev.a, ev.b));
      }
      std::sort(t.begin(), t.end());
      info.value[c] = values[c];
      info.ms[c] = t[reps / 2];
      ++info.ncand;
    }
  } catch (...) {
    knob = saved;
    H.prof = saved_prof;
    throw;
  }
  H.prof = saved_prof;
  info.chosen = 0;
  for (int c = 1; c < info.ncand; ++c)
    if (info.ms[c] < info.ms[info.chosen]) info.chosen = c;
  knob = info.value[info.chosen];
  H2_HIP(hipStreamSynchronize(st));
}

}  // namespace h2

// extern "C" entry points of include/h2.h: argument checks, error capture and
// dispatch.  No C++ exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "handle.h"
#include "ksolve.h"

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const h2::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(H2_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(H2_EINVAL, e.what());
  } catch (...) {
    return fail(H2_EINTERNAL, "unknown error");
  }
}
}  // namespace

h2_handle_s::~h2_handle_s() {
  if (kstat) (void)hipHostFree(kstat);
  std::vector<hipEvent_t> all(events);
  for (auto& pe : pending) {
    all.push_back(pe.second.first);
    all.push_back(pe.second.second);
  }
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  for (hipEvent_t e : all) (void)hipEventDestroy(e);
}

namespace h2 {

hipEvent_t prof_event(h2_handle_s& H) {
  if (!H.events.empty()) {
    hipEvent_t e = H.events.back();
    H.events.pop_back();
    return e;
  }
  hipEvent_t e;
  H2_HIP(hipEventCreate(&e));
  return e;
}

void prof_record(h2_handle_s& H, int phase, hipEvent_t a, hipEvent_t b) {
  // the same event may close one phase and open the next; prof_drain returns
  // each distinct event to the pool once
  H.pending.push_back({phase, {a, b}});
}

static void prof_drain(h2_handle_s& H) {
  std::vector<hipEvent_t> seen;
  for (auto& pe : H.pending) {
    H2_HIP(hipEventSynchronize(pe.second.second));
    float ms = 0.f;
    H2_HIP(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
    H.ms[pe.first] += ms;
    H.calls[pe.first] += 1;
    seen.push_back(pe.second.first);
    seen.push_back(pe.second.second);
  }
  std::sort(seen.begin(), seen.end());
  seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
  for (hipEvent_t e : seen) H.events.push_back(e);
  H.pending.clear();
}

}  // namespace h2

extern "C" {

const char* h2_last_error(void) { return g_err.c_str(); }

int build_h2(const h2_mesh* mesh, const h2_params* params, h2_handle* out) {
  return guarded([&]() -> int {
    if (!mesh || !params || !out) return fail(H2_EINVAL, "NULL argument");
    if (!mesh->vertices || !mesh->triangles) return fail(H2_EINVAL, "NULL mesh arrays");
    const h2_params& P = *params;
    if (P.kernel < H2_LAPLACE || P.kernel > H2_TEST_QUADRATIC) return fail(H2_EINVAL, "unknown kernel");
    if (P.storage < H2_F64 || P.storage > H2_F32_SBF16) return fail(H2_EINVAL, "unknown storage");
    if (P.kernel == H2_HELMHOLTZ && P.storage == H2_F32_SBF16)
      return fail(H2_EINVAL, "BF16 coupling storage is real-only");
    if (P.q_ss < 1 || P.q_ss > 32) return fail(H2_EINVAL, "q_ss must be in [1, 32]");
    *out = nullptr;
    h2_handle_s* H = new h2_handle_s();
    try {
      H->P = P;
      H->host_only = (P.flags & H2_HOST_ONLY) != 0;
      H->is_complex = P.kernel == H2_HELMHOLTZ;
      H->otf = (P.flags & H2_COUPLING_OTF) != 0;
      if (H->otf && !H->is_complex && P.storage == H2_F32_SBF16)
        throw h2::Error(H2_EINVAL, "on-the-fly coupling needs FP64 or FP32 storage");
      if (H->otf && H->is_complex && (P.storage != H2_F32 || P.order_m != 4))
        throw h2::Error(H2_EINVAL, "on-the-fly Helmholtz coupling needs FP32 storage and m = 4");
      const bool sym = (P.flags & H2_SYMMETRIC) != 0;
      const bool sym_near = sym || (P.flags & H2_SYMMETRIC_NEAR) != 0;
      if (sym && (H->is_complex || P.storage == H2_F32_SBF16 || P.order_m != 4))
        throw h2::Error(H2_EINVAL, "symmetric storage needs a real kernel, FP64 or FP32 storage and m = 4");
      if (sym_near && (H->is_complex || P.storage == H2_F32_SBF16))
        throw h2::Error(H2_EINVAL, "symmetric near-field storage needs a real kernel and FP64 or FP32 storage");
      h2::build_structure(H->S, mesh->vertices, mesh->nv, mesh->triangles, mesh->nt, P.order_m, P.leaf_size,
                          P.eta);
      if (sym_near) {
        for (int32_t c : H->S.leaves)
          if (H->S.cend[c] - H->S.cbegin[c] > 64)
            throw h2::Error(H2_EINVAL, "symmetric storage needs leaves of at most 64 triangles");
        h2::make_symmetric(H->S, sym && !H->otf, true);
      }
      if (!H->host_only) {
        H2_HIP(hipGetDevice(&H->device));
        const h2::Structure& S = H->S;
        H->val_bytes = P.storage == H2_F64 ? 8 : 4;
        H->s_bytes = P.storage == H2_F64 ? 8 : (P.storage == H2_F32 ? 4 : 2);
        H->perm.upload(S.perm);
        {
          std::vector<int32_t> ip(S.perm.size());
          for (size_t p = 0; p < S.perm.size(); ++p) ip[S.perm[p]] = static_cast<int32_t>(p);
          H->iperm.upload(ip);
        }
        H->cbegin.upload(S.cbegin);
        H->cend.upload(S.cend);
        H->parent.upload(S.parent);
        H->child0.upload(S.child0);
        H->child1.upload(S.child1);
        H->leaves.upload(S.leaves);
        H->adm_ptr.upload(S.adm_ptr);
        H->adm_col.upload(S.adm_col);
        H->near_ptr.upload(S.near_ptr);
        H->near_col.upload(S.near_col);
        H->panel_off.upload(S.panel_off);
        {
          std::vector<h2::NearRow> rows(S.leaves.size());
          std::vector<h2::NearBlock> blks(S.near_col.size());
          bool fits = true, fits64 = true;
          for (size_t l = 0; l < S.leaves.size(); ++l) {
            const int32_t tau = S.leaves[l];
            const int64_t nb = S.near_ptr[l + 1] - S.near_ptr[l];
            rows[l] = {S.panel_off[l], S.near_ptr[l], S.cbegin[tau], S.cend[tau] - S.cbegin[tau],
                       static_cast<int32_t>(nb), tau};
            int32_t c = 0;
            for (int64_t b = S.near_ptr[l]; b < S.near_ptr[l + 1]; ++b) {
              const int32_t s = S.near_col[b], w = S.cend[s] - S.cbegin[s];
              blks[b] = {S.cbegin[s], w, c, 0};
              c += w;
            }
            fits = fits && rows[l].r <= 64 && nb <= 256;
            fits64 = fits64 && rows[l].r <= 64 && nb <= 64;
          }
          H->near_rows.upload(rows);
          H->near_blocks.upload(blks);
          H->near64 = fits;
          H->near_row64 = fits64;
        }
        std::vector<int32_t> ul;
        H->up_ptr.assign(S.depth + 1, 0);
        for (int l = 0; l < S.depth; ++l) {
          for (int32_t c = S.level_ptr[l]; c < S.level_ptr[l + 1]; ++c)
            if (S.child0[c] >= 0) ul.push_back(c);
          H->up_ptr[l + 1] = static_cast<int64_t>(ul.size());
        }
        H->up_list.upload(ul);
        {
          std::vector<h2::RowSpan> sp(S.nclusters);
          for (int32_t c = 0; c < S.nclusters; ++c)
            sp[c] = {S.adm_ptr[c], static_cast<int32_t>(S.adm_ptr[c + 1] - S.adm_ptr[c]), c};
          std::stable_sort(sp.begin(), sp.end(), [](const h2::RowSpan& a, const h2::RowSpan& b) { return a.nb > b.nb; });
          H->row_spans.upload(sp);
        }
        // levels with few clusters from the root down: their transfers run in one workgroup
        auto top_levels = [&](int64_t most, bool up) {
          int t = 0;
          while (t < S.depth && (up ? H->up_ptr[t + 1] - H->up_ptr[t] : S.level_ptr[t + 2] - S.level_ptr[t + 1]) <= most)
            ++t;
          return t;
        };
        H->up_top = top_levels(64, true);
        H->down_top = top_levels(64, false);
        H->mup_top = top_levels(4, true);
        H->mdown_top = top_levels(4, false);
        H->up_ptr_dev.upload(H->up_ptr);
        H->level_ptr_dev.upload(S.level_ptr);
        if (S.sym_s) {
          H->adm_in_ptr.upload(S.adm_in_ptr);
          H->adm_in_blk.upload(S.adm_in_blk);
          H->scr_s.alloc(S.adm_col.size() * 64 * 8);
        }
        if (S.sym_n) {
          H->near_slot.upload(S.near_slot);
          H->near_in_ptr.upload(S.near_in_ptr);
          H->near_in_slot.upload(S.near_in_slot);
          H->leaf_of_pos.upload(S.leaf_of_pos);
          H->scr_n.alloc(static_cast<size_t>(S.near_scratch) * 8);
        }
        const int cw = H->is_complex ? 2 : 1;
        H->xc.alloc(S.n * 8 * cw);
        H->yc.alloc(S.n * 8 * cw);
        H->xhat.alloc(static_cast<size_t>(S.nclusters) * S.k * 8 * cw);
        H->yhat.alloc(static_cast<size_t>(S.nclusters) * S.k * 8 * cw);
        h2::assemble(*H);
        H->kron = S.k == 64;
      }
    } catch (...) {
      delete H;
      throw;
    }
    *out = H;
    return H2_OK;
  });
}

int h2_matvec(h2_handle h, int nrhs, int dtype, const void* x, int64_t ldx, void* y, int64_t ldy, double alpha,
              int flags, void* stream) {
  return guarded([&]() -> int {
    if (!h) return fail(H2_EINVAL, "NULL handle");
    h2::matvec(*h, nrhs, dtype, x, ldx, y, ldy, alpha, flags, static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_solve(h2_handle h, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
             const h2_solve_params* p, h2_solve_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!h || !p) return fail(H2_EINVAL, "NULL argument");
    h2_solve_info tmp{};
    const int rc = h2::solve_multi(*h, nrhs, dtype, b, ldb, z, ldz, *p, info ? *info : tmp,
                                   static_cast<hipStream_t>(stream));
    if (rc == H2_ENOTCONV) return fail(rc, "solver did not reach the tolerance");
    return rc;
  });
}

int h2_solve_noalloc(h2_handle h, int nrhs, int dtype, const void* b, int64_t ldb, void* z, int64_t ldz,
                     const h2_solve_params* p, h2_solve_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!h || !p) return fail(H2_EINVAL, "NULL argument");
    h2_solve_info tmp{};
    const int rc = h2::solve_noalloc(*h, nrhs, dtype, b, ldb, z, ldz, *p, info ? *info : tmp,
                                     static_cast<hipStream_t>(stream));
    if (rc == H2_ENOTCONV) return fail(rc, "solver did not reach the tolerance");
    return rc;
  });
}

int64_t h2_krylov_workspace(int dtype, int64_t n, int nrhs, const h2_solve_params* p) {
  try {
    if (!p || n < 1 || nrhs < 1 || (dtype != H2_R64 && dtype != H2_C128)) return -1;
    h2::KSolver::check_params(*p, dtype == H2_C128);
    return static_cast<int64_t>(h2::klayout(dtype, n, nrhs, *p).bytes);
  } catch (...) {
    return -1;
  }
}

int h2_krylov_create(int dtype, int64_t n, int nrhs, const h2_solve_params* p, void* workspace, int64_t bytes,
                     double* host_status, h2_krylov* out) {
  return guarded([&]() -> int {
    if (!p || !out) return fail(H2_EINVAL, "NULL argument");
    *out = nullptr;
    if (bytes < 0) return fail(H2_EINVAL, "negative workspace size");
    *out = reinterpret_cast<h2_krylov>(
        new h2::KSolver(dtype, n, nrhs, *p, workspace, static_cast<size_t>(bytes), host_status));
    return H2_OK;
  });
}

static h2::KSolver* ks(h2_krylov k) { return reinterpret_cast<h2::KSolver*>(k); }

int h2_krylov_begin(h2_krylov k, const void* b, int64_t ldb, const void* z0, int64_t ldz, void* stream) {
  return guarded([&]() -> int {
    if (!k) return fail(H2_EINVAL, "NULL solver");
    ks(k)->begin(b, ldb, z0, ldz, static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_krylov_next(h2_krylov k, void* x, int64_t ldx, int* flags, void* stream) {
  return guarded([&]() -> int {
    if (!k) return fail(H2_EINVAL, "NULL solver");
    return ks(k)->next(x, ldx, flags, static_cast<hipStream_t>(stream));
  });
}

int h2_krylov_advance(h2_krylov k, const void* y, int64_t ldy, void* stream) {
  return guarded([&]() -> int {
    if (!k) return fail(H2_EINVAL, "NULL solver");
    ks(k)->advance(y, ldy, static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_krylov_poll(h2_krylov k, h2_krylov_status* st) {
  return guarded([&]() -> int {
    if (!k) return fail(H2_EINVAL, "NULL solver");
    h2::KSolver& K = *ks(k);
    const int s = K.poll();
    if (st) {
      st->state = s;
      st->iterations = K.iterations;
      st->outer = K.outer;
      st->products = K.products;
      st->rel_residual = K.last_rel;
      std::snprintf(st->message, sizeof(st->message), "%s", K.message.c_str());
    }
    return s;
  });
}

int h2_krylov_residuals(h2_krylov k, double* out) {
  return guarded([&]() -> int {
    if (!k || !out) return fail(H2_EINVAL, "NULL argument");
    ks(k)->residuals(out);
    return H2_OK;
  });
}

int h2_krylov_solution(h2_krylov k, void* z, int64_t ldz, void* stream) {
  return guarded([&]() -> int {
    if (!k) return fail(H2_EINVAL, "NULL solver");
    ks(k)->solution(z, ldz, static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

void h2_krylov_destroy(h2_krylov k) {
  try {
    delete ks(k);
  } catch (...) {
  }
}

int h2_recompress(h2_handle h, double eps, int max_rank, h2_recompress_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!h) return fail(H2_EINVAL, "NULL handle");
    h2_recompress_info tmp{};
    h2::recompress(*h, eps, max_rank, info ? *info : tmp, static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_tune(h2_handle h, int nrhs, int dtype, int reps, h2_tune_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!h) return fail(H2_EINVAL, "NULL handle");
    h2_tune_info tmp{};
    h2::tune(*h, nrhs, dtype, reps, info ? *info : tmp, static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_tune_knob(h2_handle h, int knob, int nrhs, int dtype, int reps, h2_tune_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!h) return fail(H2_EINVAL, "NULL handle");
    h2_tune_info tmp{};
    h2::tune(*h, nrhs, dtype, reps, info ? *info : tmp, static_cast<hipStream_t>(stream), knob);
    return H2_OK;
  });
}

int h2_set_tuning(h2_handle h, int knob, int value) {
  return guarded([&]() -> int {
    if (!h) return fail(H2_EINVAL, "NULL handle");
    h2::set_tuning(*h, knob, value);
    return H2_OK;
  });
}

int h2_info(h2_handle h, h2_stats* out) {
  return guarded([&]() -> int {
    if (!h || !out) return fail(H2_EINVAL, "NULL argument");
    const h2::Structure& S = h->S;
    std::memset(out, 0, sizeof(*out));
    out->n = S.n;
    out->nclusters = S.nclusters;
    out->nleaves = static_cast<int64_t>(S.leaves.size());
    out->depth = S.depth;
    out->n_adm = S.adm_blocks;
    out->n_near = S.near_blocks;
    out->near_entries = S.near_entries;
    out->s_blocks_stored = h->otf ? 0 : static_cast<int64_t>(S.adm_col.size());
    out->near_entries_stored = S.near_stored;
    out->m = S.m;
    out->k = S.k;
    out->storage = h->P.storage;
    out->kernel = h->P.kernel;
    out->bytes_S = static_cast<int64_t>(h->Smat.bytes + h->Smat32.bytes);
    out->bytes_N = static_cast<int64_t>(h->Nmat.bytes);
    out->bytes_V = static_cast<int64_t>(h->Vf.bytes + h->Vb.bytes);
    out->bytes_E = static_cast<int64_t>(h->F.bytes + h->ET.bytes + h->E1.bytes);
    out->bytes_total = out->bytes_S + out->bytes_N + out->bytes_V + out->bytes_E;
    const double cw = h->is_complex ? 2.0 : 1.0;
    const double vb = h->P.storage == H2_F64 ? 8.0 : 4.0;
    const double sb = h->P.storage == H2_F64 ? 8.0 : (h->P.storage == H2_F32 ? 4.0 : 2.0);
    const double k = S.k;
    // V twice; E twice, in Kronecker form (3 m^2 numbers per cluster) on the k = 64 path
    const double e_per = h->kron ? 3.0 * S.m * S.m : k * k;
    const double v_e = 2.0 * S.n * k + 2.0 * e_per * (S.nclusters - 1);
    // every stored entry of S and of the near field is read once (symmetric storage: each
    // kept block serves both of its uses in the same pass)
    out->matvec_bytes = vb * v_e + cw * (sb * k * k * static_cast<double>(out->s_blocks_stored) +
                                         vb * static_cast<double>(S.near_stored));
    out->matvec_flops = 2.0 * (v_e * (h->is_complex ? 2.0 : 1.0) +
                               (h->is_complex ? 4.0 : 1.0) * (k * k * out->n_adm + static_cast<double>(S.near_entries)));
    return H2_OK;
  });
}

void h2_free(h2_handle h) {
  if (!h) return;
  try {
    if (!h->host_only) (void)hipDeviceSynchronize();
    delete h;
  } catch (...) {
  }
}

int h2_export(h2_handle h, int what, int64_t index, void* dst, int64_t cap) {
  return guarded([&]() -> int {
    if (!h || !dst) return fail(H2_EINVAL, "NULL argument");
    const h2::Structure& S = h->S;
    auto need = [&](int64_t n) {
      if (cap < n) throw h2::Error(H2_EINVAL, "export buffer too small: need " + std::to_string(n));
    };
    auto copy_i = [&](const std::vector<int32_t>& v) {
      need(static_cast<int64_t>(v.size()));
      std::memcpy(dst, v.data(), v.size() * 4);
    };
    const int nc = S.nclusters;
    const int64_t k = S.k;
    switch (what) {
      case H2_X_PERM: copy_i(S.perm); return H2_OK;
      case H2_X_DFS: copy_i(S.dfs_id); return H2_OK;
      case H2_X_CLUSTERS: {
        std::vector<int32_t> v(6 * static_cast<size_t>(nc));
        for (int c = 0; c < nc; ++c) {
          v[6 * c] = S.cbegin[c]; v[6 * c + 1] = S.cend[c]; v[6 * c + 2] = S.parent[c];
          v[6 * c + 3] = S.child0[c]; v[6 * c + 4] = S.child1[c]; v[6 * c + 5] = S.level[c];
        }
        copy_i(v);
        return H2_OK;
      }
      case H2_X_BOXES: {
        need(6 * static_cast<int64_t>(nc));
        double* d = static_cast<double*>(dst);
        for (int c = 0; c < nc; ++c)
          for (int a = 0; a < 3; ++a) {
            d[6 * c + a] = S.lo[3 * c + a];
            d[6 * c + 3 + a] = S.hi[3 * c + a];
          }
        return H2_OK;
      }
      case H2_X_ADM: {
        if (S.sym_s) return fail(H2_EINVAL, "admissible blocks are stored once per symmetric pair (H2_SYMMETRIC)");
        std::vector<int32_t> v;
        for (int c = 0; c < nc; ++c)
          for (int64_t b = S.adm_ptr[c]; b < S.adm_ptr[c + 1]; ++b) { v.push_back(c); v.push_back(S.adm_col[b]); }
        copy_i(v);
        return H2_OK;
      }
      case H2_X_NEAR: {
        if (S.sym_n) return fail(H2_EINVAL, "near-field blocks are stored once per symmetric pair (H2_SYMMETRIC)");
        std::vector<int32_t> v;
        for (size_t l = 0; l < S.leaves.size(); ++l)
          for (int64_t b = S.near_ptr[l]; b < S.near_ptr[l + 1]; ++b) { v.push_back(S.leaves[l]); v.push_back(S.near_col[b]); }
        copy_i(v);
        return H2_OK;
      }
      default: break;
    }
    if (h->host_only) return fail(H2_EINVAL, "matrix data is not available with H2_HOST_ONLY");
    const int cw = h->is_complex ? 2 : 1;
    const size_t vb = h->val_bytes, sb = h->s_bytes;
    auto fetch = [&](const h2::DBuf& buf, size_t eb, int64_t off, int64_t cnt, std::vector<double>& out) {
      std::vector<char> raw(cnt * eb);
      if (cnt > 0) H2_HIP(hipMemcpy(raw.data(), static_cast<char*>(buf.p) + off * eb, cnt * eb, hipMemcpyDeviceToHost));
      out.resize(cnt);
      for (int64_t i = 0; i < cnt; ++i) {
        if (eb == 8) { double v; std::memcpy(&v, &raw[8 * i], 8); out[i] = v; }
        else if (eb == 4) { float v; std::memcpy(&v, &raw[4 * i], 4); out[i] = v; }
        else { uint16_t u; std::memcpy(&u, &raw[2 * i], 2); uint32_t w = static_cast<uint32_t>(u) << 16; float v; std::memcpy(&v, &w, 4); out[i] = v; }
      }
    };
    std::vector<double> v;
    if (what == H2_X_S && h->otf) return fail(H2_EINVAL, "coupling matrices are not stored (H2_COUPLING_OTF)");
    if ((what == H2_X_S && S.sym_s) || (what == H2_X_N && S.sym_n))
      return fail(H2_EINVAL, "blocks are stored once per symmetric pair (H2_SYMMETRIC)");
    if (what == H2_X_V) {
      if (index < 0 || index >= nc || S.child0[index] >= 0) return fail(H2_EINVAL, "not a leaf cluster");
      const int64_t b0 = S.cbegin[index], r = S.cend[index] - b0;
      fetch(h->Vf, vb, b0 * k, r * k, v);
    } else if (what == H2_X_E) {
      if (index <= 0 || index >= nc) return fail(H2_EINVAL, "cluster has no transfer matrix");
      fetch(h->F, vb, index * k * k, k * k, v);
    } else if (what == H2_X_S) {
      if (index < 0 || index >= static_cast<int64_t>(S.adm_col.size())) return fail(H2_EINVAL, "block index out of range");
      fetch(h->Smat, sb, index * k * k * cw, k * k * cw, v);
    } else if (what == H2_X_N) {
      if (index < 0 || index >= static_cast<int64_t>(S.near_col.size())) return fail(H2_EINVAL, "block index out of range");
      int64_t l = std::upper_bound(S.near_ptr.begin(), S.near_ptr.end(), index) - S.near_ptr.begin() - 1;
      const int32_t tau = S.leaves[l];
      const int64_t r = S.cend[tau] - S.cbegin[tau];
      int64_t col = 0;
      for (int64_t b = S.near_ptr[l]; b < index; ++b) col += S.cend[S.near_col[b]] - S.cbegin[S.near_col[b]];
      const int64_t w = S.cend[S.near_col[index]] - S.cbegin[S.near_col[index]];
      std::vector<double> cm;
      fetch(h->Nmat, vb, (S.panel_off[l] + col * r) * cw, r * w * cw, cm);
      v.resize(r * w * cw);
      for (int64_t i = 0; i < r; ++i)
        for (int64_t j = 0; j < w; ++j)
          for (int c = 0; c < cw; ++c) v[(i * w + j) * cw + c] = cm[(j * r + i) * cw + c];
    } else {
      return fail(H2_EINVAL, "unknown export");
    }
    need(static_cast<int64_t>(v.size()));
    std::memcpy(dst, v.data(), v.size() * 8);
    return H2_OK;
  });
}

int h2_krylov_dots(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t q_rhs_stride,
                   int64_t q_vec_stride, const void* W, int64_t w_rhs_stride, void* h, void* stream) {
  return guarded([&]() -> int {
    h2::krylov_dots(dtype, nrhs, nvec, n, Q, q_rhs_stride, q_vec_stride, W, w_rhs_stride, h,
                    static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_krylov_update(int dtype, int nrhs, int nvec, int64_t n, const void* Q, int64_t q_rhs_stride,
                     int64_t q_vec_stride, const void* h, double sign, void* W, int64_t w_rhs_stride, void* stream) {
  return guarded([&]() -> int {
    h2::krylov_update(dtype, nrhs, nvec, n, Q, q_rhs_stride, q_vec_stride, h, sign, W, w_rhs_stride,
                      static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_stream_read(const void* data, int64_t bytes, int loads, void* sink, int64_t sink_bytes, void* stream) {
  return guarded([&]() -> int {
    h2::stream_read_launch(data, bytes, loads, sink, sink_bytes, static_cast<hipStream_t>(stream));
    return H2_OK;
  });
}

int h2_profile(h2_handle h, int enable) {
  return guarded([&]() -> int {
    if (!h) return fail(H2_EINVAL, "NULL handle");
    h2::prof_drain(*h);
    h->prof = enable != 0;
    for (int i = 0; i < H2_NPHASE; ++i) { h->ms[i] = 0; h->calls[i] = 0; }
    return H2_OK;
  });
}

int h2_profile_read(h2_handle h, double* ms, int64_t* calls) {
  return guarded([&]() -> int {
    if (!h || !ms || !calls) return fail(H2_EINVAL, "NULL argument");
    h2::prof_drain(*h);
    for (int i = 0; i < H2_NPHASE; ++i) { ms[i] = h->ms[i]; calls[i] = h->calls[i]; }
    return H2_OK;
  });
}

}  // extern "C"

// extern "C" entry points: argument validation, handle lifecycle, error codes.
#include <cmath>
#include <cstring>
#include <string>

#include "h2_core.h"
#include "h2_kernels.h"

struct h2_context_s {
  std::shared_ptr<h2::Context> core;
  h2::Context& c;
  h2_context_s() : core(std::make_shared<h2::Context>()), c(*core) { core->self = core; }
};
struct h2_tree_s {
  std::shared_ptr<h2::Tree> t;
  h2_context ctx;
};
struct h2_matrix_s {
  std::unique_ptr<h2::Matrix> m;
};
struct h2_job_s {
  h2::Job* j = nullptr;
  h2_context ctx = nullptr;
};

namespace {
thread_local std::string g_err;

template <typename F>
h2_status guard(F&& f) {
  try {
    g_err.clear();
    f();
    return H2_OK;
  } catch (const h2::Error& e) {
    g_err = e.what();
    // a failed runtime call stays the runtime's "last error" until read; the
    // failure is reported here, so it must not surface again in the launch
    // checks of a later call (e.g. a product retried after out of memory)
    (void)hipGetLastError();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return H2_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    g_err = e.what();
    return H2_ERR_DEVICE;
  }
}

void require(bool ok, const char* msg) {
  if (!ok) throw h2::Error(H2_ERR_INVALID_ARG, msg);
}

void set_device(h2_context ctx) { H2_HIP(hipSetDevice(ctx->c.device)); }
}  // namespace

extern "C" {

const char* h2_last_error(void) { return g_err.c_str(); }

h2_status h2_context_create(int device, h2_context* out) {
  if (out) *out = nullptr;
  return guard([&] {
    require(out != nullptr, "out is null");
    int n = 0;
    H2_HIP(hipGetDeviceCount(&n));
    require(device >= 0 && device < n, "invalid device");
    auto* ctx = new h2_context_s;
    try {
      ctx->c.device = device;
      H2_HIP(hipSetDevice(device));
      H2_HIP(hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking));
      for (auto& a : ctx->c.aux) H2_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
      H2_HIP(hipEventCreateWithFlags(&ctx->c.fork, hipEventDisableTiming));
      for (auto& e : ctx->c.join) H2_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      H2_HIP(hipMalloc((void**)&ctx->c.overflow, sizeof(int)));
      (void)h2::scratch_address(device);  // once per device, with the device current
    } catch (...) {
      delete ctx;
      throw;
    }
    *out = ctx;
  });
}

void h2_context_destroy(h2_context ctx) {
  // the device resources go when the last matrix of this context is released
  delete ctx;
}

h2_status h2_build_cluster_tree(h2_context ctx, const double* points, int64_t n, int dim, int leaf_size,
                                h2_tree* out) {
  if (out) *out = nullptr;
  return guard([&] {
    require(ctx && out && points, "null argument");
    require(n >= 1 && dim >= 1 && dim <= 3 && leaf_size >= 1, "invalid sizes");
    for (int64_t i = 0; i < n * dim; ++i) require(std::isfinite(points[i]), "non-finite coordinate");
    auto* t = new h2_tree_s;
    t->t = h2::build_tree(points, n, dim, leaf_size);
    t->ctx = ctx;
    *out = t;
  });
}

h2_status h2_tree_permutation(h2_tree tree, int64_t* perm) {
  return guard([&] {
    require(tree && perm, "null argument");
    std::memcpy(perm, tree->t->perm.data(), tree->t->n * sizeof(int64_t));
  });
}

h2_status h2_tree_info(h2_tree tree, int64_t* n, int* ncl, int* depth, int* nleaves) {
  return guard([&] {
    require(tree != nullptr, "null tree");
    const auto& T = *tree->t;
    if (n) *n = T.n;
    if (ncl) *ncl = T.ncl;
    if (depth) *depth = T.depth;
    if (nleaves) {
      int c = 0;
      for (int i = 0; i < T.ncl; ++i) c += T.leaf(i);
      *nleaves = c;
    }
  });
}

h2_status h2_tree_clusters(h2_tree tree, int64_t* begin, int64_t* end, int* parent, int* level) {
  return guard([&] {
    require(tree != nullptr, "null tree");
    const auto& T = *tree->t;
    for (int i = 0; i < T.ncl; ++i) {
      if (begin) begin[i] = T.begin[i];
      if (end) end[i] = T.end[i];
      if (parent) parent[i] = T.parent[i];
      if (level) level[i] = T.level[i];
    }
  });
}

void h2_tree_destroy(h2_tree tree) { delete tree; }

h2_status h2_build_interpolated(h2_context ctx, h2_tree rows, h2_tree cols, int kernel, const double* normals,
                                int order, double eta, int diag, h2_matrix* out) {
  if (out) *out = nullptr;
  return guard([&] {
    require(ctx && rows && cols && out, "null argument");
    require(rows->t->dim == cols->t->dim, "row and column dimensions differ");
    require(kernel >= 0 && kernel <= 2, "unknown kernel");
    require(diag == H2_DIAG_ZERO || diag == H2_DIAG_ROW_NEARFIELD_MEAN, "unknown diagonal rule");
    require(order >= 1 && eta > 0 && std::isfinite(eta), "invalid order or eta");
    int k = 1;
    for (int a = 0; a < rows->t->dim; ++a) k *= order;
    require(k <= 64, "order^dim above 64");
    if (kernel == H2_KERNEL_LAPLACE_DLP) {
      require(normals != nullptr && cols->t->dim == 3, "double layer needs normals in 3D");
      for (int64_t i = 0; i < cols->t->n * 3; ++i) require(std::isfinite(normals[i]), "non-finite normal");
    }
    set_device(ctx);
    auto* m = new h2_matrix_s;
    try {
      m->m = h2::build_interpolated(&ctx->c, rows->t, cols->t, kernel, normals, order, eta, diag);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

void h2_mul_default_options(h2_mul_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = H2_PREC_FP64;
}

const char* h2_kernel_name(int i) { return h2k::kernel_name(i); }

h2_status h2_mul(h2_context ctx, h2_matrix X, h2_matrix Y, double eps, const h2_mul_options* opt, h2_matrix* C,
                 h2_mul_stats* stats) {
  if (C) *C = nullptr;
  return guard([&] {
    require(ctx && X && Y && C, "null argument");
    require(X->m->ctx == &ctx->c && Y->m->ctx == &ctx->c, "matrices belong to another context");
    h2_mul_options o;
    h2_mul_default_options(&o);
    if (opt) o = *opt;
    require(o.precision == H2_PREC_FP64 || o.precision == H2_PREC_FP32_BULK, "unknown precision");
    set_device(ctx);
    auto* m = new h2_matrix_s;
    try {
      m->m = h2::multiply(&ctx->c, X->m.get(), Y->m.get(), eps, o, stats);
    } catch (...) {
      delete m;
      throw;
    }
    *C = m;
  });
}

h2_status h2_context_set_lanes(h2_context ctx, int nlanes) {
  return guard([&] {
    require(ctx != nullptr, "null argument");
    require(nlanes >= 1 && nlanes <= 8, "nlanes must be in [1, 8]");
    set_device(ctx);
    for (auto& l : ctx->c.lanes) require(l->inflight == 0, "jobs still in flight");
    ctx->c.set_lanes(nlanes);
  });
}

h2_status h2_context_set_memory_limit(h2_context ctx, uint64_t bytes) {
  return guard([&] {
    require(ctx != nullptr, "null argument");
    ctx->c.mem_limit = bytes;
  });
}

h2_status h2_mul_submit(h2_context ctx, h2_matrix X, h2_matrix Y, double eps, const h2_mul_options* opt,
                        h2_job* job) {
  if (job) *job = nullptr;
  return guard([&] {
    require(ctx && X && Y && job, "null argument");
    require(X->m->ctx == &ctx->c && Y->m->ctx == &ctx->c, "matrices belong to another context");
    h2_mul_options o;
    h2_mul_default_options(&o);
    if (opt) o = *opt;
    require(o.precision == H2_PREC_FP64 || o.precision == H2_PREC_FP32_BULK, "unknown precision");
    set_device(ctx);
    h2::Job* j = h2::submit(&ctx->c, X->m.get(), Y->m.get(), eps, o);
    auto* h = new h2_job_s;
    h->j = j;
    h->ctx = ctx;
    *job = h;
  });
}

h2_status h2_job_poll(h2_job job, int* done) {
  return guard([&] {
    require(job && job->j && done, "null argument");
    set_device(job->ctx);
    *done = h2::poll(*job->j) ? 1 : 0;
  });
}

h2_status h2_job_wait(h2_job job, h2_matrix* C, h2_mul_stats* stats) {
  if (C) *C = nullptr;
  return guard([&] {
    require(job && job->j && C, "null argument");
    set_device(job->ctx);
    auto* m = new h2_matrix_s;
    try {
      m->m = h2::wait(*job->j, stats);
    } catch (...) {
      delete m;
      throw;
    }
    *C = m;
  });
}

void h2_job_destroy(h2_job job) {
  if (!job) return;
  (void)hipSetDevice(job->ctx->c.device);
  h2::destroy_job(job->j);
  delete job;
}

h2_status h2_to_dense(h2_matrix M, double* out, int64_t ld) {
  return guard([&] {
    require(M && out, "null argument");
    const auto& m = *M->m;
    require(ld >= m.cols->n, "ld below the number of columns");
    if ((double)m.rows->n * (double)m.cols->n > (double)(1LL << 26))
      throw h2::Error(H2_ERR_TOO_LARGE, "dense output above 2^26 entries");
    H2_HIP(hipSetDevice(m.ctx->device));
    h2::to_dense(m, out, ld);
  });
}

h2_status h2_block_tree_leaves(h2_tree rows, h2_tree cols, double eta, int64_t* n_adm, int64_t* n_inadm,
                               int* pairs) {
  return guard([&] {
    require(rows && cols && n_adm && n_inadm, "null argument");
    require(eta > 0.0 && std::isfinite(eta), "eta must be positive");
    require(rows->t->dim == cols->t->dim, "trees of different dimension");
    h2::BlockTree bt;
    h2::build_block_tree(bt, *rows->t, *cols->t, eta);
    *n_adm = (int64_t)bt.adm.size();
    *n_inadm = (int64_t)bt.inadm.size();
    if (pairs) {
      int64_t q = 0;
      for (int i : bt.adm) {
        pairs[q++] = bt.nodes[i].t;
        pairs[q++] = bt.nodes[i].s;
      }
      for (int i : bt.inadm) {
        pairs[q++] = bt.nodes[i].t;
        pairs[q++] = bt.nodes[i].s;
      }
    }
  });
}

h2_status h2_recompress(h2_context ctx, h2_tree rows, h2_tree cols, double eta, const int* ranks, const double* U,
                        const double* Z, const double* near, double eps, const h2_mul_options* opt, h2_matrix* C,
                        h2_mul_stats* stats) {
  if (C) *C = nullptr;
  return guard([&] {
    require(ctx && rows && cols && C, "null argument");
    require(rows->ctx == ctx && cols->ctx == ctx, "trees belong to another context");
    h2_mul_options o;
    h2_mul_default_options(&o);
    if (opt) o = *opt;
    set_device(ctx);
    h2::BlockTree bt;
    require(eta > 0.0 && std::isfinite(eta), "eta must be positive");
    h2::build_block_tree(bt, *rows->t, *cols->t, eta);
    int64_t nu = 0, nz = 0, nn = 0;
    if (!bt.adm.empty()) require(ranks && U && Z, "null factor arrays");
    for (size_t i = 0; i < bt.adm.size(); ++i) {
      require(ranks[i] >= 1 && ranks[i] <= 128, "block rank outside [1, 128]");
      nu += rows->t->size(bt.nodes[bt.adm[i]].t) * ranks[i];
      nz += cols->t->size(bt.nodes[bt.adm[i]].s) * ranks[i];
    }
    for (int i : bt.inadm) nn += rows->t->size(bt.nodes[i].t) * cols->t->size(bt.nodes[i].s);
    if (nn) require(near != nullptr, "null nearfield array");
    for (int64_t i = 0; i < nu; ++i) require(std::isfinite(U[i]), "non-finite factor entry");
    for (int64_t i = 0; i < nz; ++i) require(std::isfinite(Z[i]), "non-finite factor entry");
    for (int64_t i = 0; i < nn; ++i) require(std::isfinite(near[i]), "non-finite nearfield entry");
    auto* m = new h2_matrix_s;
    try {
      m->m = h2::recompress(&ctx->c, rows->t, cols->t, eta, ranks, U, Z, near, eps, o, stats);
    } catch (...) {
      delete m;
      throw;
    }
    *C = m;
  });
}

h2_status h2_matvec(h2_matrix M, int trans, int64_t nrhs, const double* x, double* y) {
  return guard([&] {
    require(M && x && y, "null argument");
    require(nrhs >= 1, "nrhs below 1");
    require(trans == 0 || trans == 1, "trans must be 0 or 1");
    auto& m = *M->m;
    H2_HIP(hipSetDevice(m.ctx->device));
    h2::matvec(&m, trans, nrhs, x, y);
  });
}

h2_status h2_matvec_noalloc(h2_matrix M, int trans, int64_t nrhs, const double* x, double* y) {
  return guard([&] {
    require(M && x && y, "null argument");
    require(nrhs >= 1, "nrhs below 1");
    require(trans == 0 || trans == 1, "trans must be 0 or 1");
    auto& m = *M->m;
    H2_HIP(hipSetDevice(m.ctx->device));
    h2::matvec_scratch(&m, trans, nrhs, x, y, h2::scratch_address(m.ctx->device), h2::scratch_bytes());
  });
}

h2_status h2_product_error(h2_matrix X, h2_matrix Y, h2_matrix C, int iters, const double* z0, double* err_norm,
                           double* xy_norm) {
  return guard([&] {
    require(X && Y && z0 && err_norm && xy_norm, "null argument");
    require(iters >= 1, "iters below 1");
    require(X->m->ctx == Y->m->ctx && (!C || C->m->ctx == X->m->ctx), "matrices belong to different contexts");
    for (int64_t i = 0; i < Y->m->cols->n; ++i) require(std::isfinite(z0[i]), "non-finite start vector");
    H2_HIP(hipSetDevice(X->m->ctx->device));
    h2::product_error(X->m.get(), Y->m.get(), C ? C->m.get() : nullptr, iters, z0, err_norm, xy_norm);
  });
}

h2_status h2_block_dense(h2_matrix M, int64_t b, double* out) {
  return guard([&] {
    require(M && out, "null argument");
    const auto& m = *M->m;
    require(b >= 0 && b < (int64_t)(m.bt.adm.size() + m.bt.inadm.size()), "block index out of range");
    H2_HIP(hipSetDevice(m.ctx->device));
    h2::block_dense(m, b, out);
  });
}

h2_status h2_matrix_info(h2_matrix M, int64_t* n_adm, int64_t* n_inadm, int* kcap, int* rmax_row, int* rmax_col) {
  return guard([&] {
    require(M != nullptr, "null matrix");
    const auto& m = *M->m;
    if (n_adm) *n_adm = m.bt.adm.size();
    if (n_inadm) *n_inadm = m.bt.inadm.size();
    if (kcap) *kcap = m.kc;
    int a = 0, b = 0;
    for (int r : m.rank_row) a = std::max(a, r);
    for (int r : m.rank_col) b = std::max(b, r);
    if (rmax_row) *rmax_row = a;
    if (rmax_col) *rmax_col = b;
  });
}

h2_status h2_matrix_blocks(h2_matrix M, int* pairs) {
  return guard([&] {
    require(M && pairs, "null argument");
    const auto& bt = M->m->bt;
    size_t j = 0;
    for (int i : bt.adm) {
      pairs[j++] = bt.nodes[i].t;
      pairs[j++] = bt.nodes[i].s;
    }
    for (int i : bt.inadm) {
      pairs[j++] = bt.nodes[i].t;
      pairs[j++] = bt.nodes[i].s;
    }
  });
}

h2_status h2_matrix_ranks(h2_matrix M, int* row_ranks, int* col_ranks) {
  return guard([&] {
    require(M != nullptr, "null matrix");
    const auto& m = *M->m;
    if (row_ranks) std::memcpy(row_ranks, m.rank_row.data(), m.rank_row.size() * sizeof(int));
    if (col_ranks) std::memcpy(col_ranks, m.rank_col.data(), m.rank_col.size() * sizeof(int));
  });
}

h2_status h2_export_host(h2_matrix M, h2_host_view* view) {
  return guard([&] {
    require(M && view, "null argument");
    const auto& m = *M->m;
    const auto& R = *m.rows;
    const auto& C = *m.cols;
    const int kc = m.kc;
    view->n_rows = R.n;
    view->n_cols = C.n;
    view->ncl_rows = R.ncl;
    view->ncl_cols = C.ncl;
    view->kc = kc;
    view->n_adm = (int64_t)m.bt.adm.size();
    view->n_inadm = (int64_t)m.bt.inadm.size();
    view->near_size = m.nsize;
    H2_HIP(hipSetDevice(m.ctx->device));
    H2_HIP(hipStreamSynchronize(m.ctx->stream));
    auto get = [](double* dst, const double* src, int64_t count) {
      if (dst && count > 0) H2_HIP(hipMemcpy(dst, src, count * sizeof(double), hipMemcpyDeviceToHost));
    };
    const int64_t kk = (int64_t)kc * kc;
    get(view->v_leaf, m.V.leaf, R.n * kc);
    get(view->w_leaf, m.W.leaf, C.n * kc);
    get(view->v_transfer, m.V.transfer, R.ncl * kk);
    get(view->w_transfer, m.W.transfer, C.ncl * kk);
    get(view->couplings, m.S, view->n_adm * kk);
    get(view->near, m.N, m.nsize);
    // the root has no parent: its transfer slot is never written
    for (int t = 0; t < R.ncl; ++t)
      if (view->v_transfer && R.parent[t] < 0) std::memset(view->v_transfer + t * kk, 0, kk * sizeof(double));
    for (int t = 0; t < C.ncl; ++t)
      if (view->w_transfer && C.parent[t] < 0) std::memset(view->w_transfer + t * kk, 0, kk * sizeof(double));
    if (view->near_offset) {
      for (int64_t i = 0; i < view->n_inadm; ++i) view->near_offset[i] = m.noff[i];
      view->near_offset[view->n_inadm] = m.nsize;
    }
    // interpolated operands have the full rank kc on every cluster
    for (int t = 0; t < R.ncl && view->rank_row; ++t) view->rank_row[t] = m.rank_row.empty() ? kc : m.rank_row[t];
    for (int t = 0; t < C.ncl && view->rank_col; ++t) view->rank_col[t] = m.rank_col.empty() ? kc : m.rank_col[t];
  });
}

h2_status h2_matrix_storage(h2_matrix M, int64_t* bytes) {
  return guard([&] {
    require(M && bytes, "null argument");
    const auto& m = *M->m;
    // rank-exact storage: leaf bases |t| k_t, transfers k_t k_parent, couplings k_t k_s, nearfield
    int64_t w = 0;
    const auto& R = *m.rows;
    const auto& C = *m.cols;
    for (int t = 0; t < R.ncl; ++t) {
      if (R.leaf(t)) w += R.size(t) * m.rank_row[t];
      if (R.parent[t] >= 0) w += (int64_t)m.rank_row[t] * m.rank_row[R.parent[t]];
    }
    for (int t = 0; t < C.ncl; ++t) {
      if (C.leaf(t)) w += C.size(t) * m.rank_col[t];
      if (C.parent[t] >= 0) w += (int64_t)m.rank_col[t] * m.rank_col[C.parent[t]];
    }
    for (int i : m.bt.adm) w += (int64_t)m.rank_row[m.bt.nodes[i].t] * m.rank_col[m.bt.nodes[i].s];
    w += m.nsize;
    *bytes = w * 8;
  });
}

h2_status h2_selftest(h2_context ctx, double* errors, int nerrors, int* ntests) {
  return guard([&] {
    require(ctx && errors && ntests, "null argument");
    set_device(ctx);
    *ntests = h2::selftest(ctx->c.stream, ctx->c.overflow, errors, nerrors);
  });
}

void h2_matrix_destroy(h2_matrix M) { delete M; }

}  // extern "C"

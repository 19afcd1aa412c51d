// Cluster trees, block trees, interpolated operands (setup, host FP64) and
// dense export of H2-matrices.
//
// Cluster tree: Definition 1 of the paper, built by geometric bisection of the
// points' bounding boxes.  Block tree: Definition 2 with the children rule
// (eq. block_children) and the recursive admissible/inadmissible split of
// Section 2.  Operands: tensor Chebyshev interpolation of the kernel
// (eq. interpolation, vsw) with exact transfer matrices (eq. transfer).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>

#include "h2_core.h"

namespace h2 {

// ------------------------------------------------------------------ trees
// Squared diameter and distance: plain products and sums in axis order (no
// fused multiply-add), the arithmetic of the oracle, so that exact ties of
// the admissibility condition are decided alike on both sides.
double Tree::diam2(int t) const {
#pragma clang fp contract(off)
  double s = 0;
  for (int a = 0; a < dim; ++a) {
    const double d = hi[t * dim + a] - lo[t * dim + a];
    s += d * d;
  }
  return s;
}
double Tree::diam(int t) const { return std::sqrt(diam2(t)); }

static double dist2_between(const Tree& R, int t, const Tree& C, int s) {
#pragma clang fp contract(off)
  double acc = 0;
  for (int a = 0; a < R.dim; ++a) {
    const double g =
        std::max(0.0, std::max(R.lo[t * R.dim + a] - C.hi[s * C.dim + a], C.lo[s * C.dim + a] - R.hi[t * R.dim + a]));
    acc += g * g;
  }
  return acc;
}
double Tree::dist(int t, int s) const { return std::sqrt(dist2_between(*this, t, *this, s)); }

std::shared_ptr<Tree> build_tree(const double* pts, int64_t n, int dim, int leaf_size) {
  auto T = std::make_shared<Tree>();
  T->n = n;
  T->dim = dim;
  T->leaf_size = leaf_size;
  T->pts.assign(pts, pts + n * dim);
  T->perm.resize(n);
  std::iota(T->perm.begin(), T->perm.end(), 0);
  std::vector<int64_t> tmp(n);
  std::function<int(int64_t, int64_t, int, int)> rec = [&](int64_t b, int64_t e, int par, int lev) -> int {
    int c = T->ncl++;
    T->begin.push_back(b);
    T->end.push_back(e);
    T->parent.push_back(par);
    T->level.push_back(lev);
    T->children.emplace_back();
    for (int a = 0; a < dim; ++a) {
      double lo = INFINITY, hi = -INFINITY;
      for (int64_t i = b; i < e; ++i) {
        double x = T->pts[T->perm[i] * dim + a];
        lo = std::min(lo, x);
        hi = std::max(hi, x);
      }
      T->lo.push_back(lo);
      T->hi.push_back(hi);
    }
    T->depth = std::max(T->depth, lev + 1);
    if (e - b <= leaf_size) return c;
    int ax = 0;
    double best = -1;
    for (int a = 0; a < dim; ++a) {
      double ext = T->hi[c * dim + a] - T->lo[c * dim + a];
      if (ext > best) { best = ext; ax = a; }
    }
    double mid = 0.5 * (T->lo[c * dim + ax] + T->hi[c * dim + ax]);
    int64_t nl = 0;
    for (int64_t i = b; i < e; ++i) nl += T->pts[T->perm[i] * dim + ax] < mid;
    if (nl == 0 || nl == e - b) {
      std::stable_sort(T->perm.begin() + b, T->perm.begin() + e, [&](int64_t x, int64_t y) {
        return T->pts[x * dim + ax] < T->pts[y * dim + ax];
      });
      nl = (e - b) / 2;
    } else {
      int64_t pl = b, pr = 0;
      for (int64_t i = b; i < e; ++i) {
        int64_t id = T->perm[i];
        if (T->pts[id * dim + ax] < mid) T->perm[pl++] = id;
        else tmp[pr++] = id;
      }
      for (int64_t i = 0; i < pr; ++i) T->perm[pl + i] = tmp[i];
    }
    int c0 = rec(b, b + nl, c, lev + 1);
    int c1 = rec(b + nl, e, c, lev + 1);
    T->children[c] = {c0, c1};
    return c;
  };
  rec(0, n, -1, 0);
  return T;
}

void build_block_tree(BlockTree& bt, const Tree& R, const Tree& C, double eta) {
  bt.rows = &R;
  bt.cols = &C;
  bt.eta = eta;
  bt.nodes.clear();
  bt.adm.clear();
  bt.inadm.clear();
  bt.index.clear();
  // breadth-first so that children are contiguous
  bt.nodes.push_back({0, 0, BK_SPLIT, -1, 0, -1, 0});
  for (size_t q = 0; q < bt.nodes.size(); ++q) {
    int t = bt.nodes[q].t, s = bt.nodes[q].s;
    bt.index[{t, s}] = (int)q;
    // max(diam) <= 2 eta dist, squared: max(diam^2) <= (2 eta)^2 dist^2
    const double e2 = (2.0 * eta) * (2.0 * eta);
    const bool adm = std::max(R.diam2(t), C.diam2(s)) <= e2 * dist2_between(R, t, C, s);
    if (adm) {
      bt.nodes[q].kind = BK_ADM;
      bt.nodes[q].leaf_index = (int)bt.adm.size();
      bt.adm.push_back((int)q);
      continue;
    }
    if (R.leaf(t) && C.leaf(s)) {
      bt.nodes[q].kind = BK_INADM;
      bt.nodes[q].leaf_index = (int)bt.inadm.size();
      bt.inadm.push_back((int)q);
      continue;
    }
    bt.nodes[q].kind = BK_SPLIT;
    bt.nodes[q].child0 = (int)bt.nodes.size();
    int dep = bt.nodes[q].depth + 1;
    if (R.leaf(t)) {
      for (int s2 : C.children[s]) bt.nodes.push_back({t, s2, BK_SPLIT, -1, 0, -1, dep});
    } else if (C.leaf(s)) {
      for (int t2 : R.children[t]) bt.nodes.push_back({t2, s, BK_SPLIT, -1, 0, -1, dep});
    } else {
      for (int t2 : R.children[t])
        for (int s2 : C.children[s]) bt.nodes.push_back({t2, s2, BK_SPLIT, -1, 0, -1, dep});
    }
    bt.nodes[q].nchild = (int)bt.nodes.size() - bt.nodes[q].child0;
  }
}

// ------------------------------------------------------------------ device memory
void DevBuf::alloc(size_t b) {
  release();
  if (b == 0) b = 256;
  const hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    // the failure is reported by the exception; a caller may recover (free
    // memory and try again), so it must not stay behind as the runtime's
    // last error, which the launch checks read
    (void)hipGetLastError();
    p = nullptr;
  }
  if (e == hipErrorOutOfMemory) {
    size_t freeb = 0, total = 0;
    (void)hipMemGetInfo(&freeb, &total);
    char msg[160];
    std::snprintf(msg, sizeof msg, "out of memory: a device allocation of %.3f GB failed (%.3f GB of %.3f GB free)",
                  b * 1e-9, freeb * 1e-9, total * 1e-9);
    throw Error(H2_ERR_OUT_OF_MEMORY, msg);
  }
  H2_HIP(e);
  bytes = b;
}
void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

Matrix::~Matrix() {
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->evict(id);
  }
  bufs.clear();
}

void Context::set_lanes(int n) {
  H2_HIP(hipSetDevice(device));
  for (auto& l : lanes)  // no job may still run on a lane that goes away
    for (hipStream_t s : {l->l.stream, l->l.aux[0], l->l.aux[1]})
      if (s) H2_HIP(hipStreamSynchronize(s));
  while ((int)lanes.size() > n) {
    auto& r = lanes.back();
    if (lanes.size() > 1) {
      for (auto& a : r->l.aux) (void)hipStreamDestroy(a);
      (void)hipStreamDestroy(r->l.stream);
      (void)hipEventDestroy(r->l.fork);
      for (auto& e : r->l.join) (void)hipEventDestroy(e);
    }
    (void)hipFree(r->flags);
    lanes.pop_back();
  }
  while ((int)lanes.size() < n) {
    auto r = std::make_unique<LaneRes>();
    if (lanes.empty()) {
      r->l = lane0();  // the context's own streams and events
    } else {
      H2_HIP(hipStreamCreateWithFlags(&r->l.stream, hipStreamNonBlocking));
      for (auto& a : r->l.aux) H2_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
      H2_HIP(hipEventCreateWithFlags(&r->l.fork, hipEventDisableTiming));
      for (auto& e : r->l.join) H2_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    H2_HIP(hipMalloc((void**)&r->flags, kFlagSlots * sizeof(int)));
    for (int i = kFlagSlots - 1; i >= 0; --i) r->free_slots.push_back(i);
    lanes.push_back(std::move(r));
  }
}

Context::~Context() {
  (void)hipSetDevice(device);
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto& l : lanes)
    if (l->l.stream) (void)hipStreamSynchronize(l->l.stream);
  plans.clear();
  mvplans.clear();
  mvhost.clear();
  try {
    set_lanes(0);
  } catch (...) {
  }
  if (overflow) (void)hipFree(overflow);
  for (auto& a : aux)
    if (a) {
      (void)hipStreamSynchronize(a);
      (void)hipStreamDestroy(a);
    }
  if (fork) (void)hipEventDestroy(fork);
  for (auto& e : join)
    if (e) (void)hipEventDestroy(e);
  if (stream) (void)hipStreamDestroy(stream);
}

void Context::evict(uint64_t matrix_id) {
  for (auto it = plans.begin(); it != plans.end();) {
    if (it->first.first == matrix_id || (it->first.second >> 2) == matrix_id) it = plans.erase(it);
    else ++it;
  }
  for (auto it = mvplans.begin(); it != mvplans.end();) {
    if (std::get<0>(it->first) == matrix_id) it = mvplans.erase(it);
    else ++it;
  }
  for (auto it = mvhost.begin(); it != mvhost.end();) {
    if (std::get<0>(it->first) == matrix_id) it = mvhost.erase(it);
    else ++it;
  }
  for (auto it = kc_raised.begin(); it != kc_raised.end();) {
    if (it->first.first == matrix_id || it->first.second == matrix_id) it = kc_raised.erase(it);
    else ++it;
  }
  for (auto it = fp32_fail_eps.begin(); it != fp32_fail_eps.end();) {
    if (it->first.first == matrix_id || it->first.second == matrix_id) it = fp32_fail_eps.erase(it);
    else ++it;
  }
}

double* Matrix::alloc64(size_t count) {
  bufs.emplace_back(new DevBuf);
  bufs.back()->alloc(count * sizeof(double));
  H2_HIP(hipMemsetAsync(bufs.back()->p, 0, bufs.back()->bytes, ctx->stream));
  return bufs.back()->as<double>();
}
float* Matrix::alloc32(size_t count) {
  bufs.emplace_back(new DevBuf);
  bufs.back()->alloc(count * sizeof(float));
  return bufs.back()->as<float>();
}

void Matrix::ensure_fp32(hipStream_t s) {
  if (has32) return;
  auto cvt = [&](const double* src, int64_t cnt) -> float* {
    float* d = alloc32(std::max<int64_t>(cnt, 1));
    h2k::launch_convert_f64_to_f32(src, d, cnt, s);
    return d;
  };
  int64_t kk = (int64_t)kc * kc;
  V.leaf32 = cvt(V.leaf, rows->n * kc);
  V.transfer32 = cvt(V.transfer, rows->ncl * kk);
  if (w_is_v) {
    W.leaf32 = V.leaf32;
    W.transfer32 = V.transfer32;
  } else {
    W.leaf32 = cvt(W.leaf, cols->n * kc);
    W.transfer32 = cvt(W.transfer, cols->ncl * kk);
  }
  S32 = cvt(S, (int64_t)bt.adm.size() * kk);
  N32 = cvt(N, nsize);
  H2_HIP(hipStreamSynchronize(s));
  has32 = true;
}

// ------------------------------------------------------------------ interpolation
namespace {

struct Cheb {
  int p, dim, k;
  std::vector<double> a, b;  // per cluster widened box
};

double kernel_value(int kernel, const double* x, const double* y, const double* ny, int dim) {
  double d[3] = {0, 0, 0}, r2 = 0;
  for (int i = 0; i < dim; ++i) {
    d[i] = x[i] - y[i];
    r2 += d[i] * d[i];
  }
  if (r2 == 0.0) return 0.0;
  double r = std::sqrt(r2);
  switch (kernel) {
    case H2_KERNEL_NEG_LOG: return -std::log(r);
    case H2_KERNEL_LAPLACE_SLP: return 1.0 / (4.0 * M_PI * r);
    default: {
      double dot = 0;
      for (int i = 0; i < dim; ++i) dot += d[i] * ny[i];
      return dot / (4.0 * M_PI * r * r2);
    }
  }
}

// 1D Chebyshev nodes (first kind) of order p on [a, b]
void nodes1d(double a, double b, int p, double* out) {
  for (int j = 0; j < p; ++j) out[j] = 0.5 * (a + b) + 0.5 * (b - a) * std::cos((2 * j + 1) * M_PI / (2.0 * p));
}

// values l_j(x) and derivatives l_j'(x)
void lag1d(const double* nd, int p, double x, double* L, double* D) {
  for (int j = 0; j < p; ++j) {
    double v = 1.0;
    for (int m = 0; m < p; ++m)
      if (m != j) v *= (x - nd[m]) / (nd[j] - nd[m]);
    L[j] = v;
    if (D) {
      double dv = 0.0;
      for (int q = 0; q < p; ++q) {
        if (q == j) continue;
        double term = 1.0 / (nd[j] - nd[q]);
        for (int m = 0; m < p; ++m)
          if (m != j && m != q) term *= (x - nd[m]) / (nd[j] - nd[m]);
        dv += term;
      }
      D[j] = dv;
    }
  }
}

}  // namespace

std::unique_ptr<Matrix> build_interpolated(Context* ctx, std::shared_ptr<Tree> rows, std::shared_ptr<Tree> cols,
                                           int kernel, const double* normals, int order, double eta, int diag) {
  const Tree& R = *rows;
  const Tree& C = *cols;
  const int dim = R.dim;
  int k = 1;
  for (int a = 0; a < dim; ++a) k *= order;
  auto M = std::make_unique<Matrix>();
  M->ctx = ctx;
  M->hold = ctx->self.lock();
  M->id = ctx->next_id++;
  M->rows = rows;
  M->cols = cols;
  M->kc = k;
  M->w_is_v = (kernel != H2_KERNEL_LAPLACE_DLP) && rows.get() == cols.get();
  build_block_tree(M->bt, R, C, eta);
  const int p = order;
  // widened boxes and nodes per cluster
  // an edge shorter than max(1e-12 root diameter, 1e-2 longest edge of the
  // box) is widened to that length: a flat cluster (inside one face of a
  // polyhedral surface) would otherwise give normal derivatives of the
  // Lagrange polynomials of size 1/width
  auto make_nodes = [&](const Tree& T, std::vector<double>& nodes_out) {
    const double root_w = 1e-12 * T.diam(0);
    nodes_out.assign((size_t)T.ncl * dim * p, 0.0);
    for (int t = 0; t < T.ncl; ++t)
      for (int a = 0; a < dim; ++a) {
        double longest = 0.0;
        for (int b = 0; b < dim; ++b) longest = std::max(longest, T.hi[t * dim + b] - T.lo[t * dim + b]);
        const double minw = std::max(root_w, 1e-2 * longest);
        double lo = T.lo[t * dim + a], hi = T.hi[t * dim + a];
        if (hi - lo < minw) {
          double c = 0.5 * (lo + hi);
          lo = c - 0.5 * minw;
          hi = c + 0.5 * minw;
        }
        nodes1d(lo, hi, p, &nodes_out[((size_t)t * dim + a) * p]);
      }
  };
  std::vector<double> ndR, ndC;
  make_nodes(R, ndR);
  make_nodes(C, ndC);
  auto tensor_node = [&](const std::vector<double>& nd, int t, int nu, double* x) {
    for (int a = 0; a < dim; ++a) {
      int j = nu % p;
      nu /= p;
      x[a] = nd[((size_t)t * dim + a) * p + j];
    }
  };
  // l_{t,nu}(x) for all nu (and optionally n . grad)
  auto lagrange = [&](const std::vector<double>& nd, int t, const double* x, const double* nrm, double* out) {
    double L[3][16], D[3][16];
    for (int a = 0; a < dim; ++a) lag1d(&nd[((size_t)t * dim + a) * p], p, x[a], L[a], nrm ? D[a] : nullptr);
    for (int nu = 0; nu < k; ++nu) {
      int idx[3], q = nu;
      for (int a = 0; a < dim; ++a) { idx[a] = q % p; q /= p; }
      if (!nrm) {
        double v = 1.0;
        for (int a = 0; a < dim; ++a) v *= L[a][idx[a]];
        out[nu] = v;
      } else {
        double v = 0.0;
        for (int g = 0; g < dim; ++g) {
          double term = nrm[g];
          for (int a = 0; a < dim; ++a) term *= (a == g) ? D[a][idx[a]] : L[a][idx[a]];
          v += term;
        }
        out[nu] = v;
      }
    }
  };
  auto basis = [&](const Tree& T, const std::vector<double>& nd, const double* nrm, std::vector<double>& leaf,
                   std::vector<double>& tr) {
    leaf.assign((size_t)T.n * k, 0.0);
    tr.assign((size_t)T.ncl * k * k, 0.0);
#pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < T.ncl; ++t) {
      if (T.leaf(t)) {
        for (int64_t i = T.begin[t]; i < T.end[t]; ++i) {
          int64_t id = T.perm[i];
          lagrange(nd, t, &T.pts[id * dim], nrm ? &nrm[id * 3] : nullptr, &leaf[(size_t)i * k]);
        }
      }
      int par = T.parent[t];
      if (par >= 0) {
        double x[3];
        for (int nu2 = 0; nu2 < k; ++nu2) {
          tensor_node(nd, t, nu2, x);
          lagrange(nd, par, x, nullptr, &tr[((size_t)t * k + nu2) * k]);
        }
      }
    }
  };
  std::vector<double> hVl, hVt, hWl, hWt;
  basis(R, ndR, nullptr, hVl, hVt);
  if (!M->w_is_v) basis(C, ndC, kernel == H2_KERNEL_LAPLACE_DLP ? normals : nullptr, hWl, hWt);
  // couplings
  const int gk = kernel == H2_KERNEL_LAPLACE_DLP ? H2_KERNEL_LAPLACE_SLP : kernel;
  const size_t nadm = M->bt.adm.size();
  std::vector<double> hS(nadm * k * k);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < (int64_t)nadm; ++i) {
    const auto& nd = M->bt.nodes[M->bt.adm[i]];
    double x[3], y[3];
    for (int nu = 0; nu < k; ++nu) {
      tensor_node(ndR, nd.t, nu, x);
      for (int mu = 0; mu < k; ++mu) {
        tensor_node(ndC, nd.s, mu, y);
        hS[(i * k + nu) * k + mu] = kernel_value(gk, x, y, nullptr, dim);
      }
    }
  }
  // nearfield
  const size_t ninad = M->bt.inadm.size();
  M->noff.resize(ninad + 1);
  int64_t off = 0;
  for (size_t i = 0; i < ninad; ++i) {
    const auto& nd = M->bt.nodes[M->bt.inadm[i]];
    M->noff[i] = off;
    off += R.size(nd.t) * C.size(nd.s);
  }
  M->noff[ninad] = off;
  M->nsize = off;
  std::vector<double> hN(off);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < (int64_t)ninad; ++i) {
    const auto& nd = M->bt.nodes[M->bt.inadm[i]];
    double* blk = &hN[M->noff[i]];
    int64_t cs = C.size(nd.s);
    for (int64_t a = R.begin[nd.t]; a < R.end[nd.t]; ++a)
      for (int64_t b = C.begin[nd.s]; b < C.end[nd.s]; ++b) {
        int64_t ia = R.perm[a], ib = C.perm[b];
        blk[(a - R.begin[nd.t]) * cs + (b - C.begin[nd.s])] =
            kernel_value(kernel, &R.pts[ia * dim], &C.pts[ib * dim], normals ? &normals[ib * 3] : nullptr, dim);
      }
  }
  if (diag == H2_DIAG_ROW_NEARFIELD_MEAN && rows.get() == cols.get()) {
    std::vector<double> sum(R.n, 0.0), cnt(R.n, 0.0);
    for (size_t i = 0; i < ninad; ++i) {
      const auto& nd = M->bt.nodes[M->bt.inadm[i]];
      const double* blk = &hN[M->noff[i]];
      int64_t cs = C.size(nd.s);
      for (int64_t a = R.begin[nd.t]; a < R.end[nd.t]; ++a)
        for (int64_t b = C.begin[nd.s]; b < C.end[nd.s]; ++b)
          if (a != b) {
            sum[a] += blk[(a - R.begin[nd.t]) * cs + (b - C.begin[nd.s])];
            cnt[a] += 1.0;
          }
    }
    for (size_t i = 0; i < ninad; ++i) {
      const auto& nd = M->bt.nodes[M->bt.inadm[i]];
      if (nd.t != nd.s) continue;
      double* blk = &hN[M->noff[i]];
      int64_t cs = C.size(nd.s);
      for (int64_t a = R.begin[nd.t]; a < R.end[nd.t]; ++a)
        blk[(a - R.begin[nd.t]) * cs + (a - C.begin[nd.s])] = cnt[a] > 0 ? sum[a] / cnt[a] : 0.0;
    }
  }
  // upload
  auto up = [&](const std::vector<double>& h) -> double* {
    double* d = M->alloc64(std::max<size_t>(h.size(), 1));
    if (!h.empty()) H2_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    return d;
  };
  M->V.leaf = up(hVl);
  M->V.transfer = up(hVt);
  if (M->w_is_v) {
    M->W = M->V;
  } else {
    M->W.leaf = up(hWl);
    M->W.transfer = up(hWt);
  }
  M->S = up(hS);
  M->N = up(hN);
  H2_HIP(hipStreamSynchronize(ctx->stream));
  M->rank_row.assign(R.ncl, k);
  M->rank_col.assign(C.ncl, k);
  return M;
}

// ------------------------------------------------------------------ dense export
namespace {

struct HostBasis {
  const Tree* T;
  int kc;
  std::vector<double> leaf, tr;
  std::vector<int> rank;
  // full basis of t restricted to its rows: |t| x kc (row-major)
  std::vector<double> full(int t) const {
    int64_t m = T->size(t);
    std::vector<double> out((size_t)m * kc, 0.0);
    if (T->leaf(t)) {
      std::copy(leaf.begin() + T->begin[t] * kc, leaf.begin() + T->end[t] * kc, out.begin());
      return out;
    }
    for (int c : T->children[t]) {
      std::vector<double> fc = full(c);
      const double* E = &tr[(size_t)c * kc * kc];
      int64_t off = T->begin[c] - T->begin[t];
      for (int64_t i = 0; i < T->size(c); ++i)
        for (int a = 0; a < kc; ++a) {
          double v = fc[i * kc + a];
          if (v == 0.0) continue;
          for (int b = 0; b < kc; ++b) out[(off + i) * kc + b] += v * E[a * kc + b];
        }
    }
    return out;
  }
};

void fetch(std::vector<double>& h, const double* d, size_t count) {
  h.resize(count);
  if (count) H2_HIP(hipMemcpy(h.data(), d, count * sizeof(double), hipMemcpyDeviceToHost));
}

}  // namespace

void to_dense(const Matrix& M, double* out, int64_t ld) {
  const Tree& R = *M.rows;
  const Tree& C = *M.cols;
  H2_HIP(hipStreamSynchronize(M.ctx->stream));
  HostBasis V{&R, M.kc}, W{&C, M.kc};
  fetch(V.leaf, M.V.leaf, R.n * M.kc);
  fetch(V.tr, M.V.transfer, (size_t)R.ncl * M.kc * M.kc);
  fetch(W.leaf, M.W.leaf, C.n * M.kc);
  fetch(W.tr, M.W.transfer, (size_t)C.ncl * M.kc * M.kc);
  std::vector<double> S, N;
  fetch(S, M.S, M.bt.adm.size() * M.kc * M.kc);
  fetch(N, M.N, M.nsize);
  std::vector<std::vector<double>> Vf(R.ncl), Wf(C.ncl);
  const int kc = M.kc;
  for (size_t i = 0; i < M.bt.adm.size(); ++i) {
    const auto& nd = M.bt.nodes[M.bt.adm[i]];
    if (Vf[nd.t].empty()) Vf[nd.t] = V.full(nd.t);
    if (Wf[nd.s].empty()) Wf[nd.s] = W.full(nd.s);
    const double* Sb = &S[i * kc * kc];
    int64_t m = R.size(nd.t), n = C.size(nd.s);
    std::vector<double> VS((size_t)m * kc, 0.0);
    for (int64_t a = 0; a < m; ++a)
      for (int q = 0; q < kc; ++q) {
        double v = Vf[nd.t][a * kc + q];
        if (v == 0.0) continue;
        for (int r = 0; r < kc; ++r) VS[a * kc + r] += v * Sb[q * kc + r];
      }
    for (int64_t a = 0; a < m; ++a)
      for (int64_t b = 0; b < n; ++b) {
        double s = 0;
        for (int r = 0; r < kc; ++r) s += VS[a * kc + r] * Wf[nd.s][b * kc + r];
        out[R.perm[R.begin[nd.t] + a] * ld + C.perm[C.begin[nd.s] + b]] = s;
      }
  }
  for (size_t i = 0; i < M.bt.inadm.size(); ++i) {
    const auto& nd = M.bt.nodes[M.bt.inadm[i]];
    int64_t m = R.size(nd.t), n = C.size(nd.s);
    for (int64_t a = 0; a < m; ++a)
      for (int64_t b = 0; b < n; ++b)
        out[R.perm[R.begin[nd.t] + a] * ld + C.perm[C.begin[nd.s] + b]] = N[M.noff[i] + a * n + b];
  }
}

void block_dense(const Matrix& M, int64_t b, double* out) {
  const Tree& R = *M.rows;
  const Tree& C = *M.cols;
  H2_HIP(hipStreamSynchronize(M.ctx->stream));
  const int64_t nadm = M.bt.adm.size();
  const int kc = M.kc;
  if (b >= nadm) {
    int64_t i = b - nadm;
    const auto& nd = M.bt.nodes[M.bt.inadm[i]];
    int64_t cnt = R.size(nd.t) * C.size(nd.s);
    H2_HIP(hipMemcpy(out, M.N + M.noff[i], cnt * sizeof(double), hipMemcpyDeviceToHost));
    return;
  }
  const auto& nd = M.bt.nodes[M.bt.adm[b]];
  // subtree of a cluster = contiguous pre-order id range [t, t + count)
  auto subtree_end = [](const Tree& T, int t) {
    int e = t + 1;
    while (e < T.ncl && T.level[e] > T.level[t]) ++e;
    return e;
  };
  auto load = [&](const Tree& T, const BasisDev& B, int t, HostBasis& hb) {
    hb.T = &T;
    hb.kc = kc;
    hb.leaf.assign(T.n * kc, 0.0);
    hb.tr.assign((size_t)T.ncl * kc * kc, 0.0);
    int64_t rb = T.begin[t], re = T.end[t];
    H2_HIP(hipMemcpy(&hb.leaf[rb * kc], B.leaf + rb * kc, (re - rb) * kc * sizeof(double), hipMemcpyDeviceToHost));
    int te = subtree_end(T, t);
    H2_HIP(hipMemcpy(&hb.tr[(size_t)t * kc * kc], B.transfer + (size_t)t * kc * kc,
                     (size_t)(te - t) * kc * kc * sizeof(double), hipMemcpyDeviceToHost));
  };
  HostBasis hv, hw;
  load(R, M.V, nd.t, hv);
  load(C, M.W, nd.s, hw);
  std::vector<double> Vt = hv.full(nd.t), Ws = hw.full(nd.s), Sb((size_t)kc * kc);
  H2_HIP(hipMemcpy(Sb.data(), M.S + (size_t)b * kc * kc, Sb.size() * sizeof(double), hipMemcpyDeviceToHost));
  int64_t m = R.size(nd.t), n = C.size(nd.s);
  std::vector<double> VS((size_t)m * kc, 0.0);
  for (int64_t a = 0; a < m; ++a)
    for (int q = 0; q < kc; ++q) {
      double v = Vt[a * kc + q];
      if (v == 0.0) continue;
      for (int r = 0; r < kc; ++r) VS[a * kc + r] += v * Sb[q * kc + r];
    }
  for (int64_t a = 0; a < m; ++a)
    for (int64_t c = 0; c < n; ++c) {
      double s = 0;
      for (int r = 0; r < kc; ++r) s += VS[a * kc + r] * Ws[c * kc + r];
      out[a * n + c] = s;
    }
}

}  // namespace h2

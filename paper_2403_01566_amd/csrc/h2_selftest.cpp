// Kernel self-test behind h2_selftest(): runs each gfx950 kernel on seeded
// random data and reports its error against a plain host evaluation of the
// same definition (matrix product, R^T R = A^T A, singular values and
// A A^T U = U S^2, Cholesky identities).  Diagnostic only; the product path
// never calls it.
#include <cmath>
#include <cstring>
#include <vector>

#include "h2_core.h"

namespace {

struct Lcg {
  uint64_t s;
  explicit Lcg(uint64_t seed) : s(seed * 6364136223846793005ULL + 1442695040888963407ULL) {}
  double next() {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return ((s >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
  }
};

template <typename T>
T* up(const std::vector<T>& h, std::vector<void*>& keep) {
  void* p = nullptr;
  H2_HIP(hipMalloc(&p, std::max<size_t>(h.size(), 1) * sizeof(T)));
  H2_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  keep.push_back(p);
  return (T*)p;
}
template <typename T>
std::vector<T> down(const T* d, size_t n) {
  std::vector<T> h(n);
  H2_HIP(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
  return h;
}

// kdev > 0: item 0 takes its inner dimension min(k, kdev) from a device int
// (its operands hold nonzero values beyond it, which must not contribute),
// and the task's size report (m, n, sum of device-side k) is checked too.
template <typename T>
double gemm_test(hipStream_t s, int flags, int m, int n, int k, int nitem, int kdev = 0) {
  std::vector<void*> keep;
  Lcg g(17 + flags + m);
  const bool ta = flags & h2k::IT_TRANS_A, tb = flags & h2k::IT_TRANS_B;
  std::vector<std::vector<T>> A(nitem), B(nitem);
  std::vector<h2k::GemmItem<T>> items(nitem);
  for (int i = 0; i < nitem; ++i) {
    A[i].resize((size_t)m * k);
    B[i].resize((size_t)k * n);
    for (auto& x : A[i]) x = (T)g.next();
    for (auto& x : B[i]) x = (T)g.next();
    items[i].a = up(A[i], keep);
    items[i].b = up(B[i], keep);
    items[i].scale = nullptr;
    items[i].lda = ta ? m : k;
    items[i].ldb = tb ? k : n;
    items[i].k = k;
    items[i].flags = flags;
    items[i].alpha = 1.0 + 0.5 * i;
  }
  std::vector<T> c0((size_t)m * n);
  for (auto& x : c0) x = (T)g.next();
  T* dc = up(c0, keep);
  int* dstat = up(std::vector<int>{-1, -1, -1}, keep);
  if (kdev > 0) {
    items[0].k_dev = up(std::vector<int>{kdev - 3}, keep);
    items[0].k_dev2 = up(std::vector<int>{3}, keep);
  }
  h2k::GemmTask<T> task{dc, nullptr, nullptr, nullptr, nullptr, dstat, n, m, n, 0, nitem, 1, 0, 0};
  const int k0eff = kdev > 0 ? std::min(k, kdev) : k;
  std::vector<h2k::GemmTile> tiles;
  for (int i = 0; i < m; i += 64)
    for (int j = 0; j < n; j += 64) tiles.push_back({0, i, j, 0});
  auto* di = up(items, keep);
  auto* dt = up(std::vector<h2k::GemmTask<T>>{task}, keep);
  auto* dl = up(tiles, keep);
  if (std::is_same<T, double>::value)
    h2k::launch_gemm_f64((const h2k::GemmItem<double>*)di, (const h2k::GemmTask<double>*)dt, dl, (int)tiles.size(), s);
  else
    h2k::launch_gemm_f32((const h2k::GemmItem<float>*)di, (const h2k::GemmTask<float>*)dt, dl, (int)tiles.size(), s);
  H2_HIP(hipStreamSynchronize(s));
  auto c = down(dc, c0.size());
  double err = 0, ref = 0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double v = c0[(size_t)i * n + j];
      for (int it = 0; it < nitem; ++it)
        for (int q = 0; q < (it == 0 ? k0eff : k); ++q) {
          double a = ta ? A[it][(size_t)q * m + i] : A[it][(size_t)i * k + q];
          double b = tb ? B[it][(size_t)j * k + q] : B[it][(size_t)q * n + j];
          v += (1.0 + 0.5 * it) * a * b;
        }
      err = std::max(err, std::fabs(v - (double)c[(size_t)i * n + j]));
      ref = std::max(ref, std::fabs(v));
    }
  const auto st = down(dstat, 3);
  const bool stat_ok = st[0] == m && st[1] == n && st[2] == k0eff + (nitem - 1) * k;
  for (void* p : keep) (void)hipFree(p);
  return stat_ok ? err / std::max(ref, 1e-300) : 1.0;
}

double qr_test(hipStream_t s, int m, int w) {
  std::vector<void*> keep;
  Lcg g(99 + m + w);
  std::vector<double> A((size_t)m * w);
  for (auto& x : A) x = g.next();
  // make it rank-deficient in the last columns
  for (int i = 0; i < m; ++i) A[(size_t)i * w + w - 1] = A[(size_t)i * w];
  double* da = up(A, keep);
  std::vector<double> R0((size_t)w * w, 0.0);
  double* dr = up(R0, keep);
  h2k::QrTask t{da, dr, nullptr, nullptr, nullptr, nullptr, w, w, m, w, 0, 0, -1, 0};
  auto* dt = up(std::vector<h2k::QrTask>{t}, keep);
  h2k::launch_qr(dt, 1, w, s);
  H2_HIP(hipStreamSynchronize(s));
  auto R = down(dr, R0.size());
  double err = 0, ref = 0;
  for (int i = 0; i < w; ++i)
    for (int j = 0; j < w; ++j) {
      double g1 = 0, g2 = 0;
      for (int r = 0; r < m; ++r) g1 += A[(size_t)r * w + i] * A[(size_t)r * w + j];
      for (int r = 0; r < w; ++r) g2 += R[(size_t)r * w + i] * R[(size_t)r * w + j];
      err = std::max(err, std::fabs(g1 - g2));
      ref = std::max(ref, std::fabs(g1));
      if (i > j && R[(size_t)i * w + j] != 0.0) err = 1.0;  // not upper triangular
    }
  for (void* p : keep) (void)hipFree(p);
  return err / ref;
}

// qrcp == 0: relative spectral threshold 1e-6; singular values, rank and the
// leading singular vectors are checked.  qrcp == 1: pivoted-QR rank reveal
// with an absolute Frobenius threshold tau; checked are the orthonormality of
// the kept basis, the projection error ||A - U U^T A||_F <= tau and that the
// rank is no more than the one of the exact SVD at tau / 2.
// Two-stage form: the R factors of the two row halves of A, restricted to the
// first we < w columns (device-side width), stacked compactly (part), then the
// R factor of the stack (mul_we).  Checked: R^T R = A_we^T A_we and zeros
// beyond we.
double qr_split_test(hipStream_t s, int m, int w, int we) {
  std::vector<void*> keep;
  Lcg g(7 + m + w + we);
  std::vector<double> A((size_t)m * w);
  for (auto& x : A) x = g.next();
  double* da = up(A, keep);
  std::vector<double> S0((size_t)2 * w * w, 7.0), R0((size_t)w * w, 7.0);
  double* dst = up(S0, keep);
  double* dr = up(R0, keep);
  int* dwe = up(std::vector<int>{we}, keep);
  const int h = m / 2;
  h2k::QrTask t1{da, dst, dwe, nullptr, nullptr, nullptr, w, w, h, w, 0, 0, 0, 0};
  h2k::QrTask t2{da + (size_t)h * w, dst, dwe, nullptr, nullptr, nullptr, w, w, m - h, w, 0, 0, 1, 0};
  h2k::QrTask t3{dst, dr, dwe, nullptr, nullptr, nullptr, w, w, 2 * w, w, 0, 2, -1, 0};
  auto* d1 = up(std::vector<h2k::QrTask>{t1, t2}, keep);
  auto* d3 = up(std::vector<h2k::QrTask>{t3}, keep);
  h2k::launch_qr(d1, 2, w, s);
  h2k::launch_qr(d3, 1, w, s);
  H2_HIP(hipStreamSynchronize(s));
  auto R = down(dr, R0.size());
  double err = 0, ref = 0;
  for (int i = 0; i < w; ++i)
    for (int j = 0; j < w; ++j) {
      if (i >= we || j >= we) {
        if (R[(size_t)i * w + j] != 0.0) err = 1.0;
        continue;
      }
      double g1 = 0, g2 = 0;
      for (int r = 0; r < m; ++r) g1 += A[(size_t)r * w + i] * A[(size_t)r * w + j];
      for (int r = 0; r < w; ++r) g2 += R[(size_t)r * w + i] * R[(size_t)r * w + j];
      err = std::max(err, std::fabs(g1 - g2));
      ref = std::max(ref, std::fabs(g1));
      if (i > j && R[(size_t)i * w + j] != 0.0) err = 1.0;
    }
  for (void* p : keep) (void)hipFree(p);
  return err / ref;
}

// A split task whose two children both have rank 0 (effective width 0): rank
// 0, zero singular values and zero vectors in both outputs, whatever the
// output buffers held before.  Returns 0 when so, 1 otherwise.
double svd_empty_test(hipStream_t s, int* overflow) {
  std::vector<void*> keep;
  const int w = 16, kc = 8;
  std::vector<double> A((size_t)w * w, 1.0), U0((size_t)kc * kc, 7.0), S0(w, 7.0);
  std::vector<int> ints = {0, 0, 12345};  // child ranks, then the output rank
  double* da = up(A, keep);
  double* du = up(U0, keep);
  double* du2 = up(U0, keep);
  double* ds = up(S0, keep);
  int* di = up(ints, keep);
  h2k::SvdTask t{da, du, du2, ds, di + 2, nullptr, di, di + 1, di, nullptr, 0.0, 1e-6, 0.0,
                 w, kc, w, w, kc, 0, 1, 1, kc, 0};
  auto* dt = up(std::vector<h2k::SvdTask>{t}, keep);
  h2k::launch_svd(dt, 1, w, overflow, s);
  H2_HIP(hipStreamSynchronize(s));
  double err = down(di, 3)[2] == 0 ? 0.0 : 1.0;
  for (double v : down(du, U0.size())) err = std::max(err, v == 0.0 ? 0.0 : 1.0);
  for (double v : down(du2, U0.size())) err = std::max(err, v == 0.0 ? 0.0 : 1.0);
  for (double v : down(ds, S0.size())) err = std::max(err, v == 0.0 ? 0.0 : 1.0);
  for (void* p : keep) (void)hipFree(p);
  return err;
}

// copies > 1: the same matrix as `copies` tasks of one launch, each with its
// own outputs (a launch that large takes the narrow first pass of the widest
// class); the first copy is checked as above and every other copy must
// reproduce its outputs exactly.
double svd_test(hipStream_t s, int w, int* overflow, int qrcp = 0, double decades = 10.0, int copies = 1) {
  std::vector<void*> keep;
  Lcg g(7 + w);
  // A = U diag(sig) V^T with decaying singular values, formed densely
  std::vector<double> A((size_t)w * w, 0.0);
  std::vector<double> sig(w);
  for (int i = 0; i < w; ++i) sig[i] = std::pow(10.0, -decades * i / std::max(1, w - 1));
  std::vector<double> X((size_t)w * w), Y((size_t)w * w);
  for (auto& x : X) x = g.next();
  for (auto& x : Y) x = g.next();
  auto gs = [&](std::vector<double>& Q) {  // Gram-Schmidt on columns, twice
    for (int pass = 0; pass < 2; ++pass)
      for (int c = 0; c < w; ++c) {
        for (int d = 0; d < c; ++d) {
          double dot = 0;
          for (int r = 0; r < w; ++r) dot += Q[(size_t)r * w + c] * Q[(size_t)r * w + d];
          for (int r = 0; r < w; ++r) Q[(size_t)r * w + c] -= dot * Q[(size_t)r * w + d];
        }
        double nn = 0;
        for (int r = 0; r < w; ++r) nn += Q[(size_t)r * w + c] * Q[(size_t)r * w + c];
        nn = std::sqrt(nn);
        for (int r = 0; r < w; ++r) Q[(size_t)r * w + c] /= nn;
      }
  };
  gs(X);
  gs(Y);
  for (int i = 0; i < w; ++i)
    for (int j = 0; j < w; ++j)
      for (int q = 0; q < w; ++q) A[(size_t)i * w + j] += X[(size_t)i * w + q] * sig[q] * Y[(size_t)j * w + q];
  double* da = up(A, keep);
  const size_t nu = (size_t)w * w;
  std::vector<double> U0(nu * copies, 0.0), S0((size_t)w * copies, 0.0);
  double* du = up(U0, keep);
  double* ds = up(S0, keep);
  std::vector<int> rk0(copies, 0);
  int* dk = up(rk0, keep);
  const double tau = 1e-5;
  std::vector<h2k::SvdTask> tv;
  for (int c = 0; c < copies; ++c)
    tv.push_back(h2k::SvdTask{da, du + nu * c, nullptr, ds + (size_t)w * c, dk + c, nullptr, nullptr, nullptr,
                              nullptr, nullptr, qrcp ? tau : 0.0, qrcp ? 0.0 : 1e-6, 0.0,
                              w, w, w, w, w, 0, qrcp, 1, 0, qrcp});
  auto* dt = up(tv, keep);
  h2k::launch_svd(dt, copies, w, overflow, s);
  H2_HIP(hipStreamSynchronize(s));
  auto Uall = down(du, U0.size());
  auto Sall = down(ds, S0.size());
  auto rkall = down(dk, copies);
  std::vector<double> U(Uall.begin(), Uall.begin() + nu), S(Sall.begin(), Sall.begin() + w);
  std::vector<int> rk(rkall.begin(), rkall.begin() + 1);
  double err = 0;
  for (int c = 1; c < copies; ++c) {
    if (rkall[c] != rk[0]) err = 1.0;
    for (size_t e = 0; e < nu; ++e)
      if (Uall[nu * c + e] != U[e]) err = 1.0;
    for (int i = 0; i < w; ++i)
      if (Sall[(size_t)w * c + i] != S[i]) err = 1.0;
  }
  if (qrcp) {
    const int k = rk[0];
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        double d = 0;
        for (int r = 0; r < w; ++r) d += U[(size_t)r * w + a] * U[(size_t)r * w + b];
        err = std::max(err, std::fabs(d - (a == b)));
      }
    // P = U^T A (k x w), residual A - U P
    double res = 0;
    for (int j = 0; j < w; ++j) {
      std::vector<double> pj(k, 0.0);
      for (int a = 0; a < k; ++a)
        for (int r = 0; r < w; ++r) pj[a] += U[(size_t)r * w + a] * A[(size_t)r * w + j];
      for (int r = 0; r < w; ++r) {
        double v = A[(size_t)r * w + j];
        for (int a = 0; a < k; ++a) v -= U[(size_t)r * w + a] * pj[a];
        res += v * v;
      }
    }
    if (std::sqrt(res) > tau) err = 1.0;
    double tail = 0;
    int kmax = w;
    for (int i = w - 1; i >= 0; --i) {
      if (tail + sig[i] * sig[i] > 0.25 * tau * tau) break;
      tail += sig[i] * sig[i];
      kmax = i;
    }
    if (k > kmax || k < 1) err = 1.0;
    for (void* p : keep) (void)hipFree(p);
    return err;
  }
  for (int i = 0; i < w; ++i) err = std::max(err, std::fabs(S[i] - sig[i]) / sig[0]);
  int expect = 0;
  for (int i = 0; i < w; ++i) expect += sig[i] > 1e-6 * sig[0];
  if (rk[0] != expect) err = 1.0;
  // kept columns orthonormal and spanning the leading left singular space
  for (int a = 0; a < rk[0]; ++a)
    for (int b = 0; b < rk[0]; ++b) {
      double d = 0;
      for (int r = 0; r < w; ++r) d += U[(size_t)r * w + a] * U[(size_t)r * w + b];
      err = std::max(err, std::fabs(d - (a == b)));
    }
  for (int a = 0; a < rk[0]; ++a) {
    double d = 0;
    for (int r = 0; r < w; ++r) d += U[(size_t)r * w + a] * X[(size_t)r * w + a];
    err = std::max(err, std::fabs(std::fabs(d) - 1.0));
  }
  for (void* p : keep) (void)hipFree(p);
  return err;
}

double chol_test(hipStream_t s, int w, int m) {
  std::vector<void*> keep;
  Lcg g(3 + w);
  std::vector<double> Yh((size_t)m * w);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < w; ++j) Yh[(size_t)i * w + j] = g.next() * std::pow(10.0, -j * 0.5);
  std::vector<double> G((size_t)w * w, 0.0);
  for (int i = 0; i < w; ++i)
    for (int j = 0; j < w; ++j)
      for (int r = 0; r < m; ++r) G[(size_t)i * w + j] += Yh[(size_t)r * w + i] * Yh[(size_t)r * w + j];
  double* dg = up(G, keep);
  std::vector<double> z((size_t)w * w, 0.0);
  double* dtt = up(z, keep);
  double* drr = up(z, keep);
  h2k::CholTask t{dg, dtt, drr, nullptr, w, w, w, w};
  auto* dt = up(std::vector<h2k::CholTask>{t}, keep);
  h2k::launch_chol(dt, 1, w, s);
  H2_HIP(hipStreamSynchronize(s));
  auto T = down(dtt, z.size());
  auto R = down(drr, z.size());
  // Q = Y T orthonormal, and Q R = Y
  std::vector<double> Q((size_t)m * w, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < w; ++j)
      for (int q = 0; q < w; ++q) Q[(size_t)i * w + j] += Yh[(size_t)i * w + q] * T[(size_t)q * w + j];
  double err = 0;
  for (int a = 0; a < w; ++a)
    for (int b = 0; b < w; ++b) {
      double d = 0;
      for (int r = 0; r < m; ++r) d += Q[(size_t)r * w + a] * Q[(size_t)r * w + b];
      err = std::max(err, std::fabs(d - (a == b)));
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < w; ++j) {
      double v = 0;
      for (int q = 0; q < w; ++q) v += Q[(size_t)i * w + q] * R[(size_t)q * w + j];
      err = std::max(err, std::fabs(v - Yh[(size_t)i * w + j]));
    }
  for (void* p : keep) (void)hipFree(p);
  return err;
}

}  // namespace

namespace h2 {
int selftest(hipStream_t s, int* overflow, double* errors, int nerrors) {
  std::vector<double> e;
  const int flags[4] = {0, h2k::IT_TRANS_A, h2k::IT_TRANS_B, h2k::IT_TRANS_A | h2k::IT_TRANS_B};
  for (int f : flags) e.push_back(gemm_test<double>(s, f, 77, 45, 70, 3));
  for (int f : flags) e.push_back(gemm_test<float>(s, f, 130, 64, 33, 2));
  e.push_back(qr_test(s, 301, 20));
  e.push_back(qr_test(s, 97, 64));
  e.push_back(qr_test(s, 150, 128));
  e.push_back(qr_split_test(s, 333, 100, 77));
  e.push_back(qr_split_test(s, 130, 48, 40));
  e.push_back(svd_test(s, 24, overflow));
  e.push_back(svd_test(s, 64, overflow));
  e.push_back(svd_test(s, 128, overflow));
  e.push_back(svd_test(s, 40, overflow, 1));
  e.push_back(svd_test(s, 128, overflow, 1));
  e.push_back(svd_test(s, 100, overflow, 1, 30.0));  // short rank (about 20) of a wide matrix
  e.push_back(chol_test(s, 12, 200));
  e.push_back(chol_test(s, 32, 300));
  e.push_back(chol_test(s, 50, 400));
  e.push_back(svd_empty_test(s, overflow));
  // launches of 1024 matrices: the narrow first pass of the 128-wide class
  // finishes the short rank, defers the full one at 64 columns and the
  // relative-threshold form at once
  e.push_back(svd_test(s, 100, overflow, 1, 30.0, 1024));
  e.push_back(svd_test(s, 128, overflow, 1, 10.0, 1024));
  e.push_back(svd_test(s, 128, overflow, 0, 10.0, 1024));
  // device-side inner dimension (the operands are nonzero beyond it)
  e.push_back(gemm_test<double>(s, h2k::IT_TRANS_B, 70, 90, 77, 2, 21));
  e.push_back(gemm_test<float>(s, h2k::IT_TRANS_A, 65, 40, 50, 3, 9));
  // the narrow QR classes over several 128-row chunks, the last one ragged
  e.push_back(qr_test(s, 300, 50));
  e.push_back(qr_test(s, 129, 32));
  for (int i = 0; i < nerrors && i < (int)e.size(); ++i) errors[i] = e[i];
  return (int)e.size();
}
}  // namespace h2

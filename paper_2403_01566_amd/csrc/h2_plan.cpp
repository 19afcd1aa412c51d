// Product planner and executor.
//
// Once per operand pair the host builds the integer structure of the product
// (Sections 3-5 of the paper) and emits level-batched launches of the gfx950
// kernels; every floating-point operation of the product runs in those
// kernels.
//
// Exact product (Sections 3 and 4).  The host walks the union of the induced
// block tree (Definition 8) and the prescribed result block tree.  Every node
// (t,r) routes its pending sub-products X|_{t x s} Y|_{s x r} by the four
// accumulator cases of Section 3.2 and carries, as its accumulator
// (Definition 5):
//   C_tr (kX x kY)  uniform part V_{X,t} C_tr W_{Y,r}^*: the products with both
//                   factors admissible, S_{X,ts} P_s S_{Y,sr} (Section 4.1);
//   A_tr (|t| x kY) right semi-uniform part A_tr W_{Y,r}^* (case 1);
//   B_tr (|r| x kX) left semi-uniform part V_{X,t} B_tr^* (case 2);
//   N_tr            dense part (case 3; only where t or r is a leaf cluster).
// Splitting (Sections 3.3, 4.3): C_{t'r'} = E_{X,t'} C_tr F_{Y,r'}^*,
// A_{t'r'} = A_tr|_{t'} F_{Y,r'}^*, B_{t'r'} = B_tr|_{r'} E_{X,t'}^*, N
// restricted; the product-tree children refine the pending triples.
// The semi-uniform terms X|_{t x s} V_{Y,s} and Y|_{s x r}^* W_{X,s} (the
// yields of the basis trees of Section 4.2) are formed bottom-up, level by
// level, over the operand block trees (Phi, Psi).
//
// Coarsening (Section 5.1): below each admissible result leaf the exact
// blocks are agglomerated pairwise along the induced tree; every merge is a
// truncated SVD (QR of the factors, pivoted-QR rank reveal and one-sided
// Jacobi on the small core) whose dropped tail has Frobenius norm at most
// tau_b = delta_c nu_b / sum_h sqrt(n_h) (n_h merges at height h, nu_b a lower
// bound of ||G_b||).  Merges of one height act on disjoint sub-blocks, so the
// accumulated error stays below delta_c ||G_b|| (the bound of Remark 13).
//
// Adaptive bases (Sections 5.2, 5.3): row basis bottom-up with weights
// omega = theta^{(level s - level t)/2} ||G_b||, leaf SVD of the weighted
// condensed blocks, non-leaf SVD of the stacked projections, truncation at
// eps_r = delta_r sqrt(1 - sigma theta); the column basis the same way on the
// adjoint; couplings S_b = V_t^* G~_b W_r.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <set>
#include <climits>
#include <tuple>
#include <type_traits>
#include <unordered_map>
#include <deque>
#include <cstdio>
#include <cstdlib>

#include "h2_core.h"

namespace h2 {

using h2k::GemmItem;
using h2k::GemmTask;
using h2k::GemmTile;

// ------------------------------------------------------------------ device references
enum : int { WS_NONE = -1, WS_D = 0, WS_F = 1, WS_I = 2 };

template <typename T>
struct DRef {
  int ws = WS_NONE;
  T* ext = nullptr;
  int64_t off = 0;
  static DRef external(T* p) {
    DRef r;
    r.ext = p;
    return r;
  }
  DRef operator+(int64_t d) const {
    DRef r = *this;
    r.off += d;
    return r;
  }
};

template <typename T>
struct PItem {
  DRef<T> a, b;
  DRef<double> scale;
  DRef<int> kd1, kd2;  // device-side inner dimension (sum of both), if set
  int lda, ldb, k, flags;
  double alpha;
};
template <typename T>
struct PTask {
  DRef<T> c;
  int ldc, m, n, item0, nitem, beta;
  DRef<int> m_dev, n_dev, coff_dev, roff_dev;
};
struct PQr {
  DRef<double> a, r;
  int lda, ldr, m, w, trans_r;
  DRef<int> w_dev, w_dev2;
  DRef<int> m_dev;
  int mul_we = 0, part = -1, m_off = 0;
};
struct PSvd {
  DRef<double> a, u, sigma;
  DRef<int> rank;
  DRef<double> u2;
  DRef<int> w_dev, w_dev2, split_dev;
  int urows = 0;
  DRef<double> tolref;  // coarsening: per-block absolute reference (times delta_c)
  int tolkind;          // 0: coarsening (Frobenius tail), 1: row, 2: column (largest dropped value)
  double tolfactor;
  int lda, ldu, rows, cols, kcap;
  int trans_a = 0;
};
struct PRef {
  int first, count;
  double factor;
  DRef<double> out;
};
struct PRefMat {
  DRef<double> a;
  int lda, rows, cols;
  // a largest singular value of a truncated sub-block: counted as
  // sigma_1 / (1 + delta_c), a lower bound of the exact block's norm
  bool approx = false;
};
struct PScan {
  int first, count;
  DRef<int> offs, total;
};
struct PChol {
  DRef<double> g, t, r;
  DRef<int> weff;
  int ldg, ldt, ldr, w;
};
struct PFill {
  DRef<double> p;
  int ld, m, n, diag;
  double value;
};

enum StepKind { SK_GEMM_D, SK_GEMM_F, SK_QR, SK_SVD, SK_CHOL, SK_FILL, SK_CVT_F2D, SK_REF, SK_SCAN };

enum Phase { PH_PREP = 0, PH_EXACT = 1, PH_LEAF = 2, PH_COARSE = 3, PH_ROW = 4, PH_COL = 5, PH_COUPLE = 6 };

struct Step {
  StepKind kind;
  int phase = 0;
  std::vector<PItem<double>> itd;
  std::vector<PTask<double>> tkd;
  std::vector<PItem<float>> itf;
  std::vector<PTask<float>> tkf;
  std::vector<PQr> qr;
  std::vector<PSvd> svd;
  std::vector<PChol> chol;
  std::vector<PFill> fill;
  std::vector<PRef> ref;
  std::vector<PRefMat> refmat;
  std::vector<PScan> scan;
  std::vector<DRef<int>> scansrc;
  DRef<float> cvt_in;
  DRef<double> cvt_out;
  int64_t cvt_n = 0;
  int wmax = 0;
  size_t desc_off = 0, desc2_off = 0, tiles_off = 0;
  int ndesc = 0, ntiles = 0;
  int64_t nitems = 0;  // GEMM: items at desc_off (ndesc tasks at desc2_off)
  double flops = 0, bytes = 0;
  double flops_tile = 0;  // GEMM: MFMA work incl. padding to 32 x 32 quarters and 16-wide slices
  int64_t stat_off = -1;  // QR / SVD: per-task size reports (int workspace)
};

struct Plan {
  std::deque<Step> steps;  // deque: references to earlier steps stay valid
  // asynchronous use: jobs submitted and not yet waited for, and their lane
  // (a plan's workspace admits one product at a time, so they share a lane)
  int inflight = 0;
  int lane = -1;
  int64_t wsd = 0, wsf = 0, wsi = 0;
  std::vector<int64_t> base_d, base_f;  // allocation starts in the planned (unshared) layout
  int64_t wsd_planned = 0, wsf_planned = 0;
  DevBuf bufd, buff, bufi, desc;
  // workspace base pointers that descriptors are resolved against: the
  // plan's own buffers, or the arena of the lane it is bound to (product
  // plans: the plans of one lane run one at a time and share its arena)
  double* wd = nullptr;
  float* wf = nullptr;
  int* wi = nullptr;
  size_t ws_bytes = 0;  // FP64, FP32 and int workspaces, each 256-byte aligned
  bool keep_protos = false;
  bool own_protos = false;  // descriptors rebuilt from the protos on every use (matrix-vector plans)
  // the uploaded descriptors: their size and the workspace base they were
  // resolved against (a moved workspace is handled by rebasing them)
  size_t desc_size = 0;
  char* desc_base = nullptr;
  int bound_lane = -1;
  uint64_t bound_epoch = 0;
  uint64_t last_use = 0;  // submission counter of the context at the plan's last use (cache eviction)
  // HIP graph of the product's launches (captured from the plan's streams).
  // Most kernels read their descriptors from device memory, so eps patches
  // keep it valid; emit() (new workspace pointers) drops it, because the
  // conversion kernels take workspace pointers as arguments. Graph runs
  // report overflows in gflag (a kernel argument fixed in the graph),
  // copied to the job's flag afterwards.
  hipGraphExec_t gexec = nullptr;
  const void* g_desc = nullptr;
  DevBuf gflag;
  ~Plan() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
  }
  int kc = 0, kappa_cap = 0;
  DRef<double> res_vleaf, res_vtr, res_wleaf, res_wtr, res_S, res_N;
  DRef<int> res_rank_row, res_rank_col;
  DRef<double> coarse_sigma_roots;   // not used directly
  BlockTree cbt;
  std::vector<int64_t> cnoff;
  int64_t cnsize = 0;
  // workspace regions filled from the host before the first step (inputs of a
  // recompression): live from the first step on
  std::vector<DRef<double>> inputs;
  double bytes_alg = 0, flops_alg = 0;
  int64_t n_adm = 0, n_inadm = 0;
  bool f32 = false;
  double eps_set = -1;
  double theta = 0.25, sigma_br = 2.0;
  int qrcp = 1;  // pivoted-QR rank reveal before the Jacobi (square SVDs)
  double budget[3] = {0.25, 0.25, 0.25};
  int sweeps = 40;  // Jacobi sweep cap of the SVD descriptors
  int nchunk = 1;   // chunks of the exact product and coarsening (memory)
  int64_t launches = 0;
  int max_coarse_K = 0;
  // per kernel (h2k::KernelId): device ms, launches; algorithmic units, flops, bytes
  double t_k[h2k::K_COUNT] = {0}, units_k[h2k::K_COUNT] = {0}, flops_k[h2k::K_COUNT] = {0},
         bytes_k[h2k::K_COUNT] = {0};
  int64_t launches_k[h2k::K_COUNT] = {0};
};

// ------------------------------------------------------------------ plan builder
struct Builder {
  Plan& P;
  int phase = 0;
  explicit Builder(Plan& p) : P(p) {}
  DRef<double> wd(int64_t n) {
    DRef<double> r;
    r.ws = WS_D;
    r.off = P.wsd;
    P.base_d.push_back(P.wsd);
    P.wsd += (std::max<int64_t>(n, 1) + 31) & ~int64_t(31);
    return r;
  }
  DRef<float> wf(int64_t n) {
    DRef<float> r;
    r.ws = WS_F;
    r.off = P.wsf;
    P.base_f.push_back(P.wsf);
    P.wsf += (std::max<int64_t>(n, 1) + 63) & ~int64_t(63);
    return r;
  }
  DRef<int> wi(int64_t n) {
    DRef<int> r;
    r.ws = WS_I;
    r.off = P.wsi;
    P.wsi += (std::max<int64_t>(n, 1) + 63) & ~int64_t(63);
    return r;
  }
  Step& step(StepKind k) {
    P.steps.emplace_back();
    P.steps.back().kind = k;
    P.steps.back().phase = phase;
    return P.steps.back();
  }
};

#ifndef H2_QR_SPLIT_ROWS
#define H2_QR_SPLIT_ROWS 2048
#endif

// Streaming QR of a tall matrix (R only).  Matrices with many rows are cut
// into row blocks factored in parallel (stage 1); their R factors are stacked
// and factored again (stage 2), which gives the R factor of the whole matrix.
struct QrSplit {
  Builder& B;
  Step* s1;
  Step* s2 = nullptr;
  // Row blocks of at most kRows rows.  A step with few matrices would leave
  // most of the GPU idle while single workgroups walk long matrices, so it
  // splits at a quarter of that height (more, shorter, parallel pieces).
  int kRows = H2_QR_SPLIT_ROWS;
  QrSplit(Builder& b, int wmax, size_t ntasks) : B(b) {
    s1 = &B.step(SK_QR);
    s1->wmax = wmax;
    if (ntasks < 2048) kRows = std::max(128, H2_QR_SPLIT_ROWS / 4);
  }
  // m_dev: optional device-side row count (at most m)
  void add(DRef<double> a, int lda, int m, int w, DRef<double> r, int ldr, int trans_r,
           DRef<int> w1 = DRef<int>(), DRef<int> w2 = DRef<int>(), DRef<int> m_dev = DRef<int>()) {
    if (m <= kRows) {
      PQr q{a, r, lda, ldr, m, w, trans_r, w1, w2};
      q.m_dev = m_dev;
      s1->qr.push_back(q);
      return;
    }
    if (!s2) {
      s2 = &B.step(SK_QR);
      s2->wmax = s1->wmax;
    }
    // stage 1: the R factor of every row block, stacked compactly (w_eff rows
    // each); stage 2: the R factor of the stack (parts * w_eff rows)
    const int parts = (m + kRows - 1) / kRows;
    DRef<double> stack = B.wd((int64_t)parts * w * w);
    for (int p = 0; p < parts; ++p) {
      const int r0 = p * kRows, rows = std::min(kRows, m - r0);
      PQr q{a + (int64_t)r0 * lda, stack, lda, w, rows, w, 0, w1, w2};
      q.part = p;
      q.m_dev = m_dev;
      q.m_off = r0;
      s1->qr.push_back(q);
    }
    PQr q{stack, r, w, ldr, parts * w, w, trans_r, w1, w2};
    q.mul_we = parts;
    s2->qr.push_back(q);
  }
};

template <typename T>
struct WS;
template <>
struct WS<double> {
  static DRef<double> get(Builder& b, int64_t n) { return b.wd(n); }
  static constexpr StepKind kind = SK_GEMM_D;
  static std::vector<PItem<double>>& items(Step& s) { return s.itd; }
  static std::vector<PTask<double>>& tasks(Step& s) { return s.tkd; }
};
template <>
struct WS<float> {
  static DRef<float> get(Builder& b, int64_t n) { return b.wf(n); }
  static constexpr StepKind kind = SK_GEMM_F;
  static std::vector<PItem<float>>& items(Step& s) { return s.itf; }
  static std::vector<PTask<float>>& tasks(Step& s) { return s.tkf; }
};

// GEMM step writer.  Items follow their task.
template <typename T>
struct GW {
  Step* s;
  explicit GW(Step& st) : s(&st) {}
  void task(DRef<T> c, int ldc, int m, int n, int beta = 0) {
    s->bytes += (double)sizeof(T) * m * n * (beta ? 2 : 1);
    PTask<T> t;
    t.c = c;
    t.ldc = ldc;
    t.m = m;
    t.n = n;
    t.item0 = (int)WS<T>::items(*s).size();
    t.nitem = 0;
    t.beta = beta;
    WS<T>::tasks(*s).push_back(t);
  }
  // sizes / column offset of the last task known only on the device
  void dev(DRef<int> n_dev, DRef<int> coff_dev = DRef<int>(), DRef<int> m_dev = DRef<int>(),
           DRef<int> roff_dev = DRef<int>()) {
    auto& t = WS<T>::tasks(*s).back();
    t.n_dev = n_dev;
    t.coff_dev = coff_dev;
    t.m_dev = m_dev;
    t.roff_dev = roff_dev;
  }
  void mm(DRef<T> a, int lda, DRef<T> b, int ldb, int k, int flags = 0, double alpha = 1.0,
          DRef<double> scale = DRef<double>()) {
    if (k <= 0) return;
    PItem<T> x;
    x.a = a;
    x.b = b;
    x.scale = scale;
    x.lda = lda;
    x.ldb = ldb;
    x.k = k;
    x.flags = flags;
    x.alpha = alpha;
    WS<T>::items(*s).push_back(x);
    auto& tk = WS<T>::tasks(*s).back();
    tk.nitem++;
    s->flops += 2.0 * tk.m * tk.n * k;
    s->flops_tile += 2.0 * ((tk.m + 31) & ~31) * ((tk.n + 31) & ~31) * ((k + 15) & ~15);
    s->bytes += (double)sizeof(T) * ((double)tk.m * k + (double)k * tk.n);
  }
  // inner dimension of the last item known only on the device: *k1 + *k2
  // (at most its planned k; the operands are zero beyond it)
  void kdev(DRef<int> k1, DRef<int> k2 = DRef<int>()) {
    auto& x = WS<T>::items(*s).back();
    x.kd1 = k1;
    x.kd2 = k2;
  }
  void copy(DRef<T> a, int lda, int flags = 0, double alpha = 1.0) {
    PItem<T> x;
    x.a = a;
    x.b = DRef<T>();
    x.lda = lda;
    x.ldb = 0;
    x.k = 0;
    x.flags = flags | h2k::IT_COPY;
    x.alpha = alpha;
    WS<T>::items(*s).push_back(x);
    auto& tk = WS<T>::tasks(*s).back();
    tk.nitem++;
    s->bytes += (double)sizeof(T) * tk.m * tk.n;
  }
};

// ------------------------------------------------------------------ union tree node
struct UNode {
  int t = 0, r = 0, parent = -1, depth = 0;
  int tc = -1;      // node of the result block tree, -1 below an admissible result leaf
  int below = -1;   // admissible result leaf (result tree node) owning this node, or -1
  bool split = false, fin = false;
  int child0 = -1, nchild = 0;
  std::vector<std::pair<int, int>> aa, sa, sb, nn, ns, sn;  // (X block node, Y block node)
  bool hasC = false, hasA = false, hasB = false, hasN = false;
  int64_t offC = -1, offTmp = -1, offA = -1, offB = -1, offN = -1, offVC = -1;
  int ldA = 0, ldB = 0;
  int form = 0;        // 0 internal, 1 semi-uniform leaf, 2 dense U=G, 3 dense Z=G^T, 4 nearfield output
  int64_t offG = -1;   // phase-A precision: U (semi-uniform) or G / G^T (dense)
  int64_t offZa = -1;  // phase-A precision: Z (semi-uniform)
  // coarsening (FP64 workspace offsets)
  int height = -1, K = 0, m = 0, n = 0;
  int64_t U = -1, Z = -1, RZ = -1, Gh = -1, RGt = -1, Vk = -1, Yk = -1, Gy = -1, T1 = -1, R1 = -1, Uh = -1,
          Tm = -1, Zh = -1, Gz = -1, T2 = -1, R2 = -1, Vh = -1, Sb = -1, Sig = -1, Kap = -1;
  int nmerge = 1;
};

static inline DRef<double> Dw(int64_t off) {
  DRef<double> d;
  d.ws = WS_D;
  d.off = off;
  return d;
}
static inline DRef<int> Iw(int64_t off) {
  DRef<int> d;
  d.ws = WS_I;
  d.off = off;
  return d;
}
template <typename T>
static inline DRef<T> Tw(int64_t off) {
  DRef<T> d;
  d.ws = std::is_same<T, float>::value ? WS_F : WS_D;
  d.off = off;
  return d;
}

// full cluster basis references in phase-A precision
template <typename T>
struct FB {
  const Tree* T_ = nullptr;
  int k = 0;
  DRef<T> leaf, tr;
  std::vector<DRef<T>> lvl;
  DRef<T> full(int t) const {
    if (T_->leaf(t)) return leaf + T_->begin[t] * k;
    return lvl[T_->level[t]] + T_->begin[t] * k;
  }
  DRef<T> E(int t) const { return tr + (int64_t)t * k * k; }
};

// ------------------------------------------------------------------ planner
// A node of the merge tree below an admissible result leaf (coarsening):
// a final node of the induced tree (exact factors U, Z) or a merge of two
// children.
struct MNode {
  int t = 0, r = 0, m = 0, n = 0, K = 0, height = 0, below = -1, unode = -1;
  int c0 = -1, c1 = -1;  // merged children (MNode indices), -1 for leaves
  // dense leaf forms: U = I (uI) or Z = I (zI); the identity factor is never
  // formed and the steps that would multiply by it are skipped
  bool uI = false, zI = false;
  // dense leaf block of at most 128 x 128: the left singular vectors U^ of
  // G come straight from the SVD of G (no QR, no Y = G^ V_k orthonormalisation)
  bool direct = false;
  // merges: the two children share the merged block's rows (hz: Z is block
  // diagonal) or its columns (vt: U is block diagonal)
  bool hz = false, vt = false;
  int64_t U = -1, Z = -1, RZ = -1, Gh = -1, RGt = -1, Vk = -1, Yk = -1, Gy = -1, T1 = -1, R1 = -1, Uh = -1,
          Tm = -1, Zh = -1, Gz = -1, T2 = -1, R2 = -1, Vh = -1, Sb = -1, Sig = -1, Kap = -1, Wc = -1;
  int64_t Wsum = -1;  // merge: packed width kappa_a + kappa_b (device int)
  // hz / vt merges: C (kcap x kcap), P (rows x kcap) and R_P (kcap x kcap)
  // of the Gram-Schmidt step against piece a
  int64_t Cb = -1, Pb = -1, Rp = -1;
};

class Planner {
 public:
  Context* ctx;
  Matrix* X;
  Matrix* Y;
  const Tree& TI;
  const Tree& TJ;
  const Tree& TK;
  int kX, kY;
  Plan& P;
  Builder B;
  BlockTree& C;
  std::vector<UNode> un;
  std::vector<int> phi_need, psi_need, dy_need, dx_need;
  int kc, kcap;  // result rank cap, coarsened rank cap
  std::vector<std::map<int, int64_t>> row_proj, col_proj;
  std::vector<int> bnode;  // admissible result leaf -> union node rooting its coarsening
  // chunks of the exact product and coarsening (memory): union node -> chunk
  // (-1: above chunk_depth), admissible result leaf -> chunk (-1: rooted above)
  int nchunk = 1, chunk_depth = 0;
  std::vector<int> uchunk, bchunk;
  void assign_chunks(int nch);
  // merge trees of the coarsening
  std::vector<MNode> mn;
  std::vector<int> of_un;
  std::vector<std::pair<int, int>> dense_asm;  // (MNode, union node of the result leaf)
  int maxh = 0;
  std::map<int, int> hmax;
  std::map<int, double> barea;
  std::map<int, int64_t> tau;
  double share(const MNode& x) { return std::sqrt((double)x.m * x.n / barea[x.below]) / (hmax[x.below] + 1); }
  int group_of(const MNode& x) const { return x.below < 0 ? 0 : bchunk[C.nodes[x.below].leaf_index] + 1; }
  void coarsen_prepare();
  void coarsen_group(int g);
  void coarsen_finish();

  Planner(Context* c, Matrix* x, Matrix* y, Plan& p, int kc_, int kcap_)
      : ctx(c), X(x), Y(y), TI(*x->rows), TJ(*x->cols), TK(*y->cols), kX(x->kc), kY(y->kc), P(p), B(p),
        C(p.cbt), kc(kc_), kcap(kcap_) {}
  // recompression of given blocks: no operands, only the result's trees (the
  // coarsening, basis and coupling stages read nothing else)
  Planner(Context* c, const Tree& rows, const Tree& cols, Plan& p, int kc_, int kcap_)
      : ctx(c), X(nullptr), Y(nullptr), TI(rows), TJ(rows), TK(cols), kX(0), kY(0), P(p), B(p), C(p.cbt), kc(kc_),
        kcap(kcap_) {}

  void build_union();
  template <typename T>
  void phaseA();  // exact product, leaf forms and (per chunk) the coarsening
  void coarsen();  // the coarsening alone (recompression)
  void bases();
  void couplings();
};

void Planner::build_union() {
  const BlockTree& bx = X->bt;
  const BlockTree& by = Y->bt;
  phi_need.assign(bx.nodes.size(), 0);
  dx_need.assign(bx.nodes.size(), 0);
  psi_need.assign(by.nodes.size(), 0);
  dy_need.assign(by.nodes.size(), 0);
  un.clear();
  UNode root;
  root.tc = 0;
  if (C.nodes[0].kind == BK_ADM) root.below = 0;
  un.push_back(root);
  std::vector<std::vector<int>> pend(1, std::vector<int>{0});
  for (size_t q = 0; q < un.size(); ++q) {
    std::vector<int> cur = std::move(pend[q]);
    const int t = un[q].t, r = un[q].r;
    std::vector<int> rest;
    for (;;) {
      rest.clear();
      for (int s : cur) {
        int ix = bx.find(t, s), iy = by.find(s, r);
        if (ix < 0 || iy < 0) throw Error(H2_ERR_DEVICE, "planner: inconsistent product tree");
        int kx = bx.nodes[ix].kind, ky = by.nodes[iy].kind;
        if (ky == BK_ADM) {  // case 1 (first match wins when both factors are admissible)
          if (kx == BK_ADM) un[q].aa.push_back({ix, iy});
          else {
            un[q].sa.push_back({ix, iy});
            phi_need[ix] = 1;
          }
        } else if (kx == BK_ADM) {  // case 2
          un[q].sb.push_back({ix, iy});
          psi_need[iy] = 1;
        } else if (kx == BK_INADM || ky == BK_INADM) {  // case 3
          if (kx == BK_INADM && ky == BK_INADM) un[q].nn.push_back({ix, iy});
          else if (kx == BK_INADM) {
            un[q].ns.push_back({ix, iy});
            dy_need[iy] = 1;
          } else {
            un[q].sn.push_back({ix, iy});
            dx_need[ix] = 1;
          }
        } else {  // case 4
          rest.push_back(s);
        }
      }
      if (!rest.empty() && TI.leaf(t) && TK.leaf(r)) {
        std::vector<int> nx;  // both clusters are leaves: refine the triples in place
        for (int s : rest) {
          const auto& nd = bx.nodes[bx.find(t, s)];
          for (int c = 0; c < nd.nchild; ++c) nx.push_back(bx.nodes[nd.child0 + c].s);
        }
        cur = std::move(nx);
        continue;
      }
      break;
    }
    {
      UNode& u = un[q];
      const int par = u.parent;
      u.hasC = !u.aa.empty() || (par >= 0 && un[par].hasC);
      u.hasA = !u.sa.empty() || (par >= 0 && un[par].hasA);
      u.hasB = !u.sb.empty() || (par >= 0 && un[par].hasB);
      u.hasN = !u.nn.empty() || !u.ns.empty() || !u.sn.empty() || (par >= 0 && un[par].hasN);
    }
    const bool tc_split = un[q].tc >= 0 && C.nodes[un[q].tc].kind == BK_SPLIT;
    if (rest.empty() && !tc_split) {
      un[q].fin = true;
      continue;
    }
    un[q].split = true;
    std::vector<int> ct = TI.leaf(t) ? std::vector<int>{t} : TI.children[t];
    std::vector<int> cr = TK.leaf(r) ? std::vector<int>{r} : TK.children[r];
    const int belowq = un[q].below, depq = un[q].depth;
    un[q].child0 = (int)un.size();
    un[q].nchild = (int)(ct.size() * cr.size());
    for (int t2 : ct)
      for (int r2 : cr) {
        std::vector<int> p2;  // product-tree children (Definition 7)
        for (int s : rest) {
          const auto& nx = bx.nodes[bx.find(t, s)];
          const auto& ny = by.nodes[by.find(s, r)];
          for (int c = 0; c < nx.nchild; ++c) {
            const auto& cx = bx.nodes[nx.child0 + c];
            if (cx.t != t2) continue;
            int iy2 = by.find(cx.s, r2);
            if (iy2 >= ny.child0 && iy2 < ny.child0 + ny.nchild) p2.push_back(cx.s);
          }
        }
        UNode cn;
        cn.t = t2;
        cn.r = r2;
        cn.parent = (int)q;
        cn.depth = depq + 1;
        if (tc_split) {
          cn.tc = C.find(t2, r2);
          if (cn.tc < 0) throw Error(H2_ERR_DEVICE, "planner: result tree mismatch");
          cn.below = C.nodes[cn.tc].kind == BK_ADM ? cn.tc : -1;
        } else {
          cn.tc = -1;
          cn.below = belowq;
        }
        un.push_back(cn);
        pend.push_back(std::move(p2));
      }
  }
  // Phi / Psi of split blocks need their split children
  for (size_t i = 0; i < bx.nodes.size(); ++i)
    if (phi_need[i] && bx.nodes[i].kind == BK_SPLIT)
      for (int c = 0; c < bx.nodes[i].nchild; ++c) {
        int ci = bx.nodes[i].child0 + c;
        if (bx.nodes[ci].kind == BK_SPLIT) phi_need[ci] = 1;
      }
  for (size_t i = 0; i < by.nodes.size(); ++i)
    if (psi_need[i] && by.nodes[i].kind == BK_SPLIT)
      for (int c = 0; c < by.nodes[i].nchild; ++c) {
        int ci = by.nodes[i].child0 + c;
        if (by.nodes[ci].kind == BK_SPLIT) psi_need[ci] = 1;
      }
  bnode.assign(C.adm.size(), -1);
  for (size_t i = 0; i < un.size(); ++i)
    if (un[i].tc >= 0 && C.nodes[un[i].tc].kind == BK_ADM) bnode[C.nodes[un[i].tc].leaf_index] = (int)i;
}

template <typename T>
void Planner::phaseA() {
  const BlockTree& bx = X->bt;
  const BlockTree& by = Y->bt;
  constexpr bool isf = std::is_same<T, float>::value;
  auto W = [&](int64_t n) { return WS<T>::get(B, n); };
  auto ext = [&](double* d, float* f) {
    if constexpr (isf) return DRef<float>::external(f);
    else return DRef<double>::external(d);
  };
  auto newstep = [&]() { return GW<T>(B.step(WS<T>::kind)); };
  auto R = [&](int64_t off) { return Tw<T>(off); };
  const int kk = kX * kY;
  B.phase = PH_PREP;
  // ---------------- full cluster bases (eq. transfer), shared when identical ----------------
  FB<T> VX, WX, VY, WY;
  VX.T_ = &TI; VX.k = kX; VX.leaf = ext(X->V.leaf, X->V.leaf32); VX.tr = ext(X->V.transfer, X->V.transfer32);
  WX.T_ = &TJ; WX.k = kX; WX.leaf = ext(X->W.leaf, X->W.leaf32); WX.tr = ext(X->W.transfer, X->W.transfer32);
  VY.T_ = &TJ; VY.k = kY; VY.leaf = ext(Y->V.leaf, Y->V.leaf32); VY.tr = ext(Y->V.transfer, Y->V.transfer32);
  WY.T_ = &TK; WY.k = kY; WY.leaf = ext(Y->W.leaf, Y->W.leaf32); WY.tr = ext(Y->W.transfer, Y->W.transfer32);
  FB<T>* all[4] = {&VX, &WX, &VY, &WY};
  std::vector<FB<T>*> uniq;
  int alias[4];
  for (int i = 0; i < 4; ++i) {
    alias[i] = -1;
    for (int j = 0; j < (int)uniq.size(); ++j)
      if (uniq[j]->leaf.ext == all[i]->leaf.ext && uniq[j]->T_ == all[i]->T_) alias[i] = j;
    if (alias[i] < 0) {
      alias[i] = (int)uniq.size();
      uniq.push_back(all[i]);
    }
  }
  int depth = 0;
  for (auto* b : uniq) {
    depth = std::max(depth, b->T_->depth);
    b->lvl.assign(b->T_->depth, DRef<T>());
    for (int l = 0; l + 1 < b->T_->depth; ++l) b->lvl[l] = W(b->T_->n * b->k);
  }
  for (int l = depth - 2; l >= 0; --l) {
    GW<T> g = newstep();
    for (auto* b : uniq) {
      const Tree& Tr = *b->T_;
      if (l + 1 >= Tr.depth) continue;
      for (int t = 0; t < Tr.ncl; ++t) {
        if (Tr.level[t] != l || Tr.leaf(t)) continue;
        for (int c : Tr.children[t]) {
          g.task(b->lvl[l] + Tr.begin[c] * b->k, b->k, (int)Tr.size(c), b->k);
          g.mm(b->full(c), b->k, b->E(c), b->k, b->k);
        }
      }
    }
  }
  for (int i = 0; i < 4; ++i)
    if (uniq[alias[i]] != all[i]) all[i]->lvl = uniq[alias[i]]->lvl;
  // ---------------- basis products P_s = W_{X,s}^* V_{Y,s} (Section 4.1) ----------------
  // Only clusters that carry an admissible block of X (column) or Y (row)
  // need P_s.  A sum over |s| > KS rows is split into row chunks of KS whose
  // partial products are added by a second step, so no single tile walks a
  // long K range.
  DRef<T> Pm = W((int64_t)TJ.ncl * kk);
  {
    constexpr int KS = 256;
    std::vector<char> need(TJ.ncl, 0);
    for (int node : bx.adm) need[bx.nodes[node].s] = 1;
    for (int node : by.adm) need[by.nodes[node].t] = 1;
    int64_t nparts = 0;
    for (int s = 0; s < TJ.ncl; ++s)
      if (need[s] && TJ.size(s) > KS) nparts += (TJ.size(s) + KS - 1) / KS;
    DRef<T> Pp = nparts ? W(nparts * kk) : DRef<T>();
    GW<T> g = newstep();
    int64_t part = 0;
    for (int s = 0; s < TJ.ncl; ++s) {
      if (!need[s]) continue;
      const int ns = (int)TJ.size(s);
      if (ns <= KS) {
        g.task(Pm + (int64_t)s * kk, kY, kX, kY);
        g.mm(WX.full(s), kX, VY.full(s), kY, ns, h2k::IT_TRANS_A);
        continue;
      }
      for (int r0 = 0; r0 < ns; r0 += KS, ++part) {
        g.task(Pp + part * kk, kY, kX, kY);
        g.mm(WX.full(s) + (int64_t)r0 * kX, kX, VY.full(s) + (int64_t)r0 * kY, kY, std::min(KS, ns - r0),
             h2k::IT_TRANS_A);
      }
    }
    if (nparts) {
      GW<T> g2 = newstep();
      part = 0;
      for (int s = 0; s < TJ.ncl; ++s) {
        if (!need[s] || TJ.size(s) <= KS) continue;
        g2.task(Pm + (int64_t)s * kk, kY, kX, kY);
        for (int64_t r0 = 0; r0 < TJ.size(s); r0 += KS, ++part) g2.copy(Pp + part * kk, kY);
      }
    }
  }
  auto Pref = [&](int s) { return Pm + (int64_t)s * kk; };
  auto SX = [&](int node) { return ext(X->S, X->S32) + (int64_t)bx.nodes[node].leaf_index * kX * kX; };
  auto SY = [&](int node) { return ext(Y->S, Y->S32) + (int64_t)by.nodes[node].leaf_index * kY * kY; };
  auto NX = [&](int node) { return ext(X->N, X->N32) + X->noff[bx.nodes[node].leaf_index]; };
  auto NY = [&](int node) { return ext(Y->N, Y->N32) + Y->noff[by.nodes[node].leaf_index]; };
  // Q_{ts} = S_{X,ts} P_s for X's admissible leaves, Q'_{sr} = P_s S_{Y,sr} for Y's
  DRef<T> Qx = W((int64_t)bx.adm.size() * kk), Qy = W((int64_t)by.adm.size() * kk);
  auto QX = [&](int node) { return Qx + (int64_t)bx.nodes[node].leaf_index * kk; };
  auto QY = [&](int node) { return Qy + (int64_t)by.nodes[node].leaf_index * kk; };
  {
    GW<T> g = newstep();
    for (int node : bx.adm) {
      g.task(QX(node), kY, kX, kY);
      g.mm(SX(node), kX, Pref(bx.nodes[node].s), kY, kX);
    }
    for (int node : by.adm) {
      g.task(QY(node), kY, kX, kY);
      g.mm(Pref(by.nodes[node].t), kY, SY(node), kY, kY);
    }
  }
  // ---------------- coefficients of admissible children for Phi / Psi ----------------
  // Phi_{ts}|_{t'} gets V_{X,t'} * sum_{s' : (t',s') adm} Q_{t's'} E_{Y,s'}
  // Psi_{sr}|_{r'} gets W_{Y,r'} * sum_{s' : (s',r') adm} Q'_{s'r'}^* F_{X,s'}
  std::map<std::pair<int, int>, int64_t> cphi, cpsi;
  {
    GW<T> g = newstep();
    for (size_t i = 0; i < bx.nodes.size(); ++i) {
      if (!phi_need[i] || bx.nodes[i].kind != BK_SPLIT) continue;
      const auto& nd = bx.nodes[i];
      std::vector<int> rowsc;
      for (int c = 0; c < nd.nchild; ++c) {
        const auto& ch = bx.nodes[nd.child0 + c];
        if (ch.kind == BK_ADM && std::find(rowsc.begin(), rowsc.end(), ch.t) == rowsc.end()) rowsc.push_back(ch.t);
      }
      for (int t2 : rowsc) {
        DRef<T> d = W(kk);
        cphi[{(int)i, t2}] = d.off;
        g.task(d, kY, kX, kY);
        for (int c = 0; c < nd.nchild; ++c) {
          const auto& ch = bx.nodes[nd.child0 + c];
          if (ch.kind != BK_ADM || ch.t != t2) continue;
          if (ch.s == nd.s) g.copy(QX(nd.child0 + c), kY);
          else g.mm(QX(nd.child0 + c), kY, VY.E(ch.s), kY, kY);
        }
      }
    }
    for (size_t i = 0; i < by.nodes.size(); ++i) {
      if (!psi_need[i] || by.nodes[i].kind != BK_SPLIT) continue;
      const auto& nd = by.nodes[i];
      std::vector<int> colsc;
      for (int c = 0; c < nd.nchild; ++c) {
        const auto& ch = by.nodes[nd.child0 + c];
        if (ch.kind == BK_ADM && std::find(colsc.begin(), colsc.end(), ch.s) == colsc.end()) colsc.push_back(ch.s);
      }
      for (int r2 : colsc) {
        DRef<T> d = W(kk);
        cpsi[{(int)i, r2}] = d.off;
        g.task(d, kX, kY, kX);
        for (int c = 0; c < nd.nchild; ++c) {
          const auto& ch = by.nodes[nd.child0 + c];
          if (ch.kind != BK_ADM || ch.s != r2) continue;
          if (ch.t == nd.t) g.copy(QY(nd.child0 + c), kY, h2k::IT_TRANS_A);
          else g.mm(QY(nd.child0 + c), kY, WX.E(ch.t), kX, kX, h2k::IT_TRANS_A);
        }
      }
    }
  }
  // ---------------- Phi_{ts} = X|_{t x s} V_{Y,s},  Psi_{sr} = Y|_{s x r}^* W_{X,s} ----------------
  std::vector<int64_t> phi(bx.nodes.size(), -1), psi(by.nodes.size(), -1);
  int maxd = 0;
  for (size_t i = 0; i < bx.nodes.size(); ++i)
    if (phi_need[i]) {
      phi[i] = W(TI.size(bx.nodes[i].t) * kY).off;
      maxd = std::max(maxd, bx.nodes[i].depth);
    }
  for (size_t i = 0; i < by.nodes.size(); ++i)
    if (psi_need[i]) {
      psi[i] = W(TK.size(by.nodes[i].s) * kX).off;
      maxd = std::max(maxd, by.nodes[i].depth);
    }
  for (int d = maxd; d >= 0; --d) {
    GW<T> g = newstep();
    for (size_t i = 0; i < bx.nodes.size(); ++i) {
      if (!phi_need[i] || bx.nodes[i].depth != d) continue;
      const auto& nd = bx.nodes[i];
      const int t = nd.t, s = nd.s;
      if (nd.kind == BK_INADM) {
        g.task(R(phi[i]), kY, (int)TI.size(t), kY);
        g.mm(NX((int)i), (int)TJ.size(s), VY.full(s), kY, (int)TJ.size(s));
        continue;
      }
      std::vector<int> rowsc = TI.leaf(t) ? std::vector<int>{t} : TI.children[t];
      for (int t2 : rowsc) {
        g.task(R(phi[i]) + (TI.begin[t2] - TI.begin[t]) * kY, kY, (int)TI.size(t2), kY);
        auto it = cphi.find({(int)i, t2});
        if (it != cphi.end()) g.mm(VX.full(t2), kX, R(it->second), kY, kX);
        for (int c = 0; c < nd.nchild; ++c) {
          const int ci = nd.child0 + c;
          const auto& ch = bx.nodes[ci];
          if (ch.t != t2) continue;
          if (ch.kind == BK_INADM) {
            g.mm(NX(ci), (int)TJ.size(ch.s), VY.full(s) + (TJ.begin[ch.s] - TJ.begin[s]) * kY, kY,
                 (int)TJ.size(ch.s));
          } else if (ch.kind == BK_SPLIT) {
            if (ch.s == s) g.copy(R(phi[ci]), kY);
            else g.mm(R(phi[ci]), kY, VY.E(ch.s), kY, kY);
          }
        }
      }
    }
    for (size_t i = 0; i < by.nodes.size(); ++i) {
      if (!psi_need[i] || by.nodes[i].depth != d) continue;
      const auto& nd = by.nodes[i];
      const int s = nd.t, r = nd.s;
      if (nd.kind == BK_INADM) {
        g.task(R(psi[i]), kX, (int)TK.size(r), kX);
        g.mm(NY((int)i), (int)TK.size(r), WX.full(s), kX, (int)TJ.size(s), h2k::IT_TRANS_A);
        continue;
      }
      std::vector<int> colsc = TK.leaf(r) ? std::vector<int>{r} : TK.children[r];
      for (int r2 : colsc) {
        g.task(R(psi[i]) + (TK.begin[r2] - TK.begin[r]) * kX, kX, (int)TK.size(r2), kX);
        auto it = cpsi.find({(int)i, r2});
        if (it != cpsi.end()) g.mm(WY.full(r2), kY, R(it->second), kX, kY);
        for (int c = 0; c < nd.nchild; ++c) {
          const int ci = nd.child0 + c;
          const auto& ch = by.nodes[ci];
          if (ch.s != r2) continue;
          if (ch.kind == BK_INADM) {
            g.mm(NY(ci), (int)TK.size(r2), WX.full(s) + (TJ.begin[ch.t] - TJ.begin[s]) * kX, kX,
                 (int)TJ.size(ch.t), h2k::IT_TRANS_A);
          } else if (ch.kind == BK_SPLIT) {
            if (ch.t == s) g.copy(R(psi[ci]), kX);
            else g.mm(R(psi[ci]), kX, WX.E(ch.t), kX, kX);
          }
        }
      }
    }
  }
  // ---------------- dense strips for one-sided nearfield products (case 3) ----------------
  // D^Y_{sr} = Y|_{s x r} for s a leaf, D^X_{ts} = X|_{t x s} for s a leaf
  std::vector<int64_t> dy(by.nodes.size(), -1), dx(bx.nodes.size(), -1);
  {
    std::function<void(const BlockTree&, int, std::vector<int>&)> leaves = [&](const BlockTree& bt, int i,
                                                                                std::vector<int>& out) {
      const auto& nd = bt.nodes[i];
      if (nd.kind != BK_SPLIT) {
        out.push_back(i);
        return;
      }
      for (int c = 0; c < nd.nchild; ++c) leaves(bt, nd.child0 + c, out);
    };
    std::map<int, int64_t> vs, sw;
    GW<T> g1 = newstep();
    for (size_t i = 0; i < by.nodes.size(); ++i) {
      if (!dy_need[i]) continue;
      const auto& nd = by.nodes[i];
      dy[i] = W(TJ.size(nd.t) * TK.size(nd.s)).off;
      std::vector<int> lv;
      leaves(by, (int)i, lv);
      for (int l : lv)
        if (by.nodes[l].kind == BK_ADM && !vs.count(l)) {
          vs[l] = W(TJ.size(nd.t) * kY).off;
          g1.task(R(vs[l]), kY, (int)TJ.size(nd.t), kY);
          g1.mm(VY.full(nd.t), kY, SY(l), kY, kY);
        }
    }
    for (size_t i = 0; i < bx.nodes.size(); ++i) {
      if (!dx_need[i]) continue;
      const auto& nd = bx.nodes[i];
      dx[i] = W(TI.size(nd.t) * TJ.size(nd.s)).off;
      std::vector<int> lv;
      leaves(bx, (int)i, lv);
      for (int l : lv)
        if (bx.nodes[l].kind == BK_ADM && !sw.count(l)) {
          sw[l] = W((int64_t)kX * TJ.size(nd.s)).off;
          g1.task(R(sw[l]), (int)TJ.size(nd.s), kX, (int)TJ.size(nd.s));
          g1.mm(SX(l), kX, WX.full(nd.s), kX, kX, h2k::IT_TRANS_B);
        }
    }
    GW<T> g2 = newstep();
    for (size_t i = 0; i < by.nodes.size(); ++i) {
      if (!dy_need[i]) continue;
      const auto& nd = by.nodes[i];
      const int s = nd.t, r = nd.s;
      const int ld = (int)TK.size(r);
      std::vector<int> lv;
      leaves(by, (int)i, lv);
      for (int l : lv) {
        const auto& lf = by.nodes[l];
        g2.task(R(dy[i]) + (TK.begin[lf.s] - TK.begin[r]), ld, (int)TJ.size(s), (int)TK.size(lf.s));
        if (lf.kind == BK_ADM) g2.mm(R(vs[l]), kY, WY.full(lf.s), kY, kY, h2k::IT_TRANS_B);
        else g2.copy(NY(l), (int)TK.size(lf.s));
      }
    }
    for (size_t i = 0; i < bx.nodes.size(); ++i) {
      if (!dx_need[i]) continue;
      const auto& nd = bx.nodes[i];
      const int t = nd.t, s = nd.s;
      const int ld = (int)TJ.size(s);
      std::vector<int> lv;
      leaves(bx, (int)i, lv);
      for (int l : lv) {
        const auto& lf = bx.nodes[l];
        g2.task(R(dx[i]) + (TI.begin[lf.t] - TI.begin[t]) * ld, ld, (int)TI.size(lf.t), ld);
        if (lf.kind == BK_ADM) g2.mm(VX.full(lf.t), kX, R(sw[l]), ld, kX);
        else g2.copy(NX(l), ld);
      }
    }
  }
  // ---------------- union tree: accumulators, top-down per depth ----------------
  // Chunks (memory): the union nodes at depth >= chunk_depth form nchunk
  // groups of whole subtrees.  Each chunk runs its exact product, the leaf
  // forms of its final nodes and the coarsening of the result blocks that
  // lie inside it before the next chunk starts, so the workspace of a chunk
  // is reused by the next (buffers share memory by lifetime).  Result blocks
  // rooted above chunk_depth ("top" blocks) collect their final forms from
  // every chunk and are coarsened last.  One chunk reproduces the unchunked
  // order.  The arithmetic of every task is the same either way.
  B.phase = PH_EXACT;
  const int kU = kY + kX;
  const int ngroup = nchunk + 1;  // group g = chunk g - 1, group 0 = top
  auto group_of_block = [&](int below) { return below < 0 ? 0 : bchunk[C.nodes[below].leaf_index] + 1; };
  // final forms of each group's blocks: one allocation per group (one
  // conversion per group in FP32 bulk), offsets inside it (pass 1: sizes)
  std::vector<int64_t> fin_used(ngroup, 0), fin_first(ngroup, -1), fin64(ngroup, -1);
  std::vector<int> fgroup(un.size(), -1);
  auto fin_alloc = [&](int g, int64_t n) {
    const int64_t o = fin_used[g];
    fin_used[g] += (std::max<int64_t>(n, 1) + (isf ? 63 : 31)) & ~int64_t(isf ? 63 : 31);
    return o;
  };
  for (size_t i = 0; i < un.size(); ++i) {
    UNode& u = un[i];
    if (!u.fin) continue;
    const int64_t m = TI.size(u.t), n = TK.size(u.r);
    if (u.tc >= 0 && C.nodes[u.tc].kind == BK_INADM) {
      u.form = 4;
      continue;
    }
    const int g = fgroup[i] = group_of_block(u.below);
    if (u.hasN || std::min(m, n) < kU) {
      u.form = (m >= n) ? 2 : 3;
      u.offG = fin_alloc(g, m * n);
    } else {
      u.form = 1;
      u.offG = fin_alloc(g, m * kU);
      u.offZa = fin_alloc(g, n * kU);
    }
  }
  for (int g = 0; g < ngroup; ++g) {
    if (fin_used[g] == 0) continue;
    fin_first[g] = W(fin_used[g]).off;
    fin64[g] = isf ? B.wd(fin_used[g]).off : fin_first[g];  // FP64 copy of the region (FP32 bulk)
  }
  for (size_t i = 0; i < un.size(); ++i) {
    UNode& u = un[i];
    if (!u.fin || u.form == 4) continue;
    const int g = fgroup[i];
    const int64_t shift = fin64[g];
    u.m = (int)TI.size(u.t);
    u.n = (int)TK.size(u.r);
    if (u.form == 1) {
      u.K = kU;
      u.U = u.offG + shift;
      u.Z = u.offZa + shift;
      u.offZa += fin_first[g];
    } else if (u.form == 2) {  // U = G, Z = I
      u.K = u.n;
      u.U = u.offG + shift;
      u.Z = -2;
    } else {  // U = I, Z = G^T
      u.K = u.m;
      u.U = -2;
      u.Z = u.offG + shift;
    }
    u.offG += fin_first[g];
  }
  int maxdep = 0;
  for (auto& u : un) {
    maxdep = std::max(maxdep, u.depth);
    const int64_t m = TI.size(u.t), n = TK.size(u.r);
    if (u.hasC) u.offC = W(kk).off;
    if (u.hasA) {
      if (u.form == 1) { u.offA = u.offG; u.ldA = kU; }
      else { u.offA = W(m * kY).off; u.ldA = kY; }
    }
    if (u.hasB) {
      if (u.form == 1) { u.offB = u.offZa + kY; u.ldB = kU; }
      else { u.offB = W(n * kX).off; u.ldB = kX; }
    }
    if (u.hasN) u.offN = W(m * n).off;
    if (u.parent >= 0 && un[u.parent].hasC && u.hasC && u.t != un[u.parent].t) u.offTmp = W(kk).off;
    if (u.fin && u.hasC && u.form != 1) u.offVC = W(m * kY).off;
  }
  // result nearfield (inadmissible leaves of the result tree)
  P.cnoff.assign(C.inadm.size() + 1, 0);
  int64_t noff = 0;
  for (size_t i = 0; i < C.inadm.size(); ++i) {
    P.cnoff[i] = noff;
    const auto& nd = C.nodes[C.inadm[i]];
    noff += TI.size(nd.t) * TK.size(nd.s);
  }
  P.cnoff[C.inadm.size()] = noff;
  P.cnsize = noff;
  P.res_N = B.wd(noff);
  DRef<T> nearT;
  if constexpr (isf) nearT = W(noff);
  else nearT = P.res_N;
  // the merge trees of the coarsening (their buffers are placed as the
  // groups' steps are emitted)
  coarsen_prepare();

  // steps of the exact product at depth d for the union nodes of chunk c (-1: above the chunks)
  auto exact_depth = [&](int d, int c) {
    GW<T> g1 = newstep();
    for (size_t i = 0; i < un.size(); ++i) {
      const UNode& u = un[i];
      if (u.depth != d || uchunk[i] != c || u.offTmp < 0) continue;
      g1.task(R(u.offTmp), kY, kX, kY);
      g1.mm(VX.E(u.t), kX, R(un[u.parent].offC), kY, kX);
    }
    GW<T> g2 = newstep();
    for (size_t i = 0; i < un.size(); ++i) {
      const UNode& u = un[i];
      if (u.depth != d || uchunk[i] != c) continue;
      const int t = u.t, r = u.r;
      const int64_t m = TI.size(t), n = TK.size(r);
      const UNode* p = u.parent >= 0 ? &un[u.parent] : nullptr;
      if (u.hasC) {
        g2.task(R(u.offC), kY, kX, kY);
        if (p && p->hasC) {
          DRef<T> src = u.offTmp >= 0 ? R(u.offTmp) : R(p->offC);
          if (r == p->r) g2.copy(src, kY);
          else g2.mm(src, kY, WY.E(r), kY, kY, h2k::IT_TRANS_B);
        }
        for (auto& pr : u.aa) g2.mm(QX(pr.first), kY, SY(pr.second), kY, kY);
      }
      if (u.hasA) {
        g2.task(R(u.offA), u.ldA, (int)m, kY);
        if (p && p->hasA) {
          DRef<T> src = R(p->offA) + (TI.begin[t] - TI.begin[p->t]) * p->ldA;
          if (r == p->r) g2.copy(src, p->ldA);
          else g2.mm(src, p->ldA, WY.E(r), kY, kY, h2k::IT_TRANS_B);
        }
        for (auto& pr : u.sa) g2.mm(R(phi[pr.first]), kY, SY(pr.second), kY, kY);
      }
      if (u.hasB) {
        g2.task(R(u.offB), u.ldB, (int)n, kX);
        if (p && p->hasB) {
          DRef<T> src = R(p->offB) + (TK.begin[r] - TK.begin[p->r]) * p->ldB;
          if (t == p->t) g2.copy(src, p->ldB);
          else g2.mm(src, p->ldB, VX.E(t), kX, kX, h2k::IT_TRANS_B);
        }
        for (auto& pr : u.sb) g2.mm(R(psi[pr.second]), kX, SX(pr.first), kX, kX, h2k::IT_TRANS_B);
      }
      if (u.hasN) {
        g2.task(R(u.offN), (int)n, (int)m, (int)n);
        if (p && p->hasN) {
          const int64_t pn = TK.size(p->r);
          g2.copy(R(p->offN) + (TI.begin[t] - TI.begin[p->t]) * pn + (TK.begin[r] - TK.begin[p->r]), (int)pn);
        }
        for (auto& pr : u.nn) {
          const int s = bx.nodes[pr.first].s;
          g2.mm(NX(pr.first), (int)TJ.size(s), NY(pr.second), (int)n, (int)TJ.size(s));
        }
        for (auto& pr : u.ns) {
          const int s = bx.nodes[pr.first].s;
          g2.mm(NX(pr.first), (int)TJ.size(s), R(dy[pr.second]), (int)n, (int)TJ.size(s));
        }
        for (auto& pr : u.sn) {
          const int s = bx.nodes[pr.first].s;
          g2.mm(R(dx[pr.first]), (int)TJ.size(s), NY(pr.second), (int)n, (int)TJ.size(s));
        }
      }
    }
  };
  // leaf forms of the final nodes of chunk c (-1: above the chunks)
  auto leaf_forms = [&](int c) {
    B.phase = PH_LEAF;
    GW<T> g1 = newstep();
    for (size_t i = 0; i < un.size(); ++i) {
      const UNode& u = un[i];
      if (u.offVC < 0 || uchunk[i] != c) continue;
      g1.task(R(u.offVC), kY, (int)TI.size(u.t), kY);
      g1.mm(VX.full(u.t), kX, R(u.offC), kY, kX);
    }
    GW<T> g2 = newstep();
    for (size_t i = 0; i < un.size(); ++i) {
      const UNode& u = un[i];
      if (!u.fin || uchunk[i] != c) continue;
      const int t = u.t, r = u.r;
      const int64_t m = TI.size(t), n = TK.size(r);
      if (u.form == 1) {
        // U = [A + V_X C | V_X],  Z = [W_Y | B]
        g2.task(R(u.offG), kU, (int)m, kY, u.hasA ? 1 : 0);
        if (u.hasC) g2.mm(VX.full(t), kX, R(u.offC), kY, kX);
        g2.task(R(u.offG) + kY, kU, (int)m, kX);
        g2.copy(VX.full(t), kX);
        g2.task(R(u.offZa), kU, (int)n, kY);
        g2.copy(WY.full(r), kY);
        if (!u.hasB) g2.task(R(u.offZa) + kY, kU, (int)n, kX);
        continue;
      }
      // G = A W^* + (V C) W^* + V B^* + N, or its transpose for form 3
      DRef<T> out = (u.form == 4) ? nearT + P.cnoff[C.nodes[u.tc].leaf_index] : R(u.offG);
      if (u.form != 3) {
        g2.task(out, (int)n, (int)m, (int)n);
        if (u.hasA) g2.mm(R(u.offA), u.ldA, WY.full(r), kY, kY, h2k::IT_TRANS_B);
        if (u.hasC) g2.mm(R(u.offVC), kY, WY.full(r), kY, kY, h2k::IT_TRANS_B);
        if (u.hasB) g2.mm(VX.full(t), kX, R(u.offB), u.ldB, kX, h2k::IT_TRANS_B);
        if (u.hasN) g2.copy(R(u.offN), (int)n);
      } else {
        g2.task(out, (int)m, (int)n, (int)m);
        if (u.hasA) g2.mm(WY.full(r), kY, R(u.offA), u.ldA, kY, h2k::IT_TRANS_B);
        if (u.hasC) g2.mm(WY.full(r), kY, R(u.offVC), kY, kY, h2k::IT_TRANS_B);
        if (u.hasB) g2.mm(R(u.offB), u.ldB, VX.full(t), kX, kX, h2k::IT_TRANS_B);
        if (u.hasN) g2.copy(R(u.offN), (int)n, h2k::IT_TRANS_A);
      }
    }
  };
  // FP32 bulk: the group's final forms handed over to the FP64 recompression
  auto hand_over = [&](int g) {
    if constexpr (isf) {
      if (fin_used[g] > 0) {
        Step& st = B.step(SK_CVT_F2D);
        st.cvt_in = Tw<float>(fin_first[g]);
        st.cvt_out = Dw(fin64[g]);
        st.cvt_n = fin_used[g];
      }
    }
  };
  for (int d = 0; d < chunk_depth; ++d) exact_depth(d, -1);
  for (int c = 0; c < nchunk; ++c) {
    B.phase = PH_EXACT;
    for (int d = chunk_depth; d <= maxdep; ++d) exact_depth(d, c);
    leaf_forms(c);
    hand_over(c + 1);
    coarsen_group(c + 1);
  }
  leaf_forms(-1);
  hand_over(0);
  if constexpr (isf) {
    if (noff > 0) {
      Step& st = B.step(SK_CVT_F2D);
      st.cvt_in = nearT;
      st.cvt_out = P.res_N;
      st.cvt_n = noff;
    }
  }
  coarsen_group(0);
  coarsen_finish();
}

// ------------------------------------------------------------------ coarsening
// Merge trees of all admissible result leaves (host only; the steps are
// emitted per group by coarsen_group).
void Planner::coarsen_prepare() {
  // Merge tree below every admissible result leaf: the leaves are the final
  // nodes of the induced tree (exact factors U, Z); every split node of the
  // induced tree merges its children pairwise (first the column pairs of
  // each row child, then the rows), so a merge never joins more than two
  // truncated pieces (width <= 2 * kcap).
  mn.clear();
  dense_asm.clear();
  of_un.assign(un.size(), -1);
  std::function<int(int)> make = [&](int ui) -> int {
    UNode& u = un[ui];
    MNode x;
    x.t = u.t;
    x.r = u.r;
    x.m = (int)TI.size(u.t);
    x.n = (int)TK.size(u.r);
    x.below = u.below;
    x.unode = ui;
    if (u.fin) {
      x.K = u.K;
      x.U = u.U;
      x.Z = u.Z;
      mn.push_back(x);
      return of_un[ui] = (int)mn.size() - 1;
    }
    std::vector<int> kids;
    for (int c = 0; c < u.nchild; ++c) kids.push_back(make(u.child0 + c));
    auto merge = [&](int a, int b, int t, int r) {
      MNode y;
      y.t = t;
      y.r = r;
      y.m = (int)TI.size(t);
      y.n = (int)TK.size(r);
      y.below = u.below;
      y.c0 = a;
      y.c1 = b;
      y.height = 1 + std::max(mn[a].height, mn[b].height);
      mn.push_back(y);
      return (int)mn.size() - 1;
    };
    int root;
    if (kids.size() == 4) {  // children (t1,r1), (t1,r2), (t2,r1), (t2,r2)
      int v1 = merge(kids[0], kids[1], mn[kids[0]].t, u.r);
      int v2 = merge(kids[2], kids[3], mn[kids[2]].t, u.r);
      root = merge(v1, v2, u.t, u.r);
    } else if (kids.size() == 2) {
      root = merge(kids[0], kids[1], u.t, u.r);
    } else {
      throw Error(H2_ERR_DEVICE, "planner: unexpected number of induced children");
    }
    mn[root].unode = ui;
    return of_un[ui] = root;
  };
  // Result blocks of at most 128 x 128 whose induced sub-blocks are finer are
  // assembled densely from their exact pieces and truncated once (a direct
  // SVD of the block instead of a merge tree of small truncations).
  for (size_t li = 0; li < C.adm.size(); ++li) {
    UNode& u = un[bnode[li]];
    const int m = (int)TI.size(u.t), n = (int)TK.size(u.r);
    if (u.fin || m > 128 || n > 128) {
      make(bnode[li]);
      continue;
    }
    MNode x;
    x.t = u.t;
    x.r = u.r;
    x.m = m;
    x.n = n;
    x.K = n;
    x.U = B.wd((int64_t)m * n).off;
    x.Z = -2;  // identity
    x.below = u.below;
    x.unode = bnode[li];
    mn.push_back(x);
    of_un[bnode[li]] = (int)mn.size() - 1;
    dense_asm.push_back({(int)mn.size() - 1, bnode[li]});
  }
  maxh = 0;
  for (auto& x : mn) maxh = std::max(maxh, x.height);
  if (std::getenv("H2_TRACE")) {  // shape summary of the merge tree
    std::map<std::tuple<int, int, int, int>, int> hist;  // (height, m bucket, n bucket, K)
    auto bk = [](int v) { int b = 16; while (b < v) b *= 2; return b; };
    for (auto& x : mn) hist[std::make_tuple(x.height, bk(x.m), bk(x.n), x.c0 >= 0 ? -1 : x.K)]++;
    for (auto& kv : hist)
      std::fprintf(stderr, "[h2 merge] height %d m<=%d n<=%d K %d count %d\n", std::get<0>(kv.first),
                   std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first), kv.second);
  }
  // Truncation errors of all merges of a block add up exactly.  Merges of
  // equal height act on disjoint sub-blocks, so their errors add in squares
  // (Frobenius norm).  A merge of an m x n sub-block of the M x N block b
  // keeps a Frobenius tail <= delta_c nu_b sqrt(m n / (M N)) / (H_b + 1)
  // (H_b: highest merge of b); the errors of one height then total at most
  // delta_c nu_b / (H_b + 1), and those of all heights delta_c nu_b.  nu_b is
  // a lower bound of ||G_b|| held on the device: first the largest row or
  // column norm of the leaves' condensed factors, raised after every height
  // by the largest singular values of that height's merged sub-blocks.
  hmax.clear();
  barea.clear();
  tau.clear();
  for (auto& x : mn) {
    hmax[x.below] = std::max(hmax[x.below], x.height);
    barea[x.below] = std::max(barea[x.below], (double)x.m * x.n);
  }
  for (auto& kv : hmax) tau[kv.first] = B.wd(1).off;
  P.max_coarse_K = 0;
}

// Steps of the coarsening of the result blocks of group g (0: blocks rooted
// above the chunks, c + 1: chunk c), after the group's final forms exist.
void Planner::coarsen_group(int grp) {
  B.phase = PH_COARSE;
  {  // dense assembly of the group's small blocks
    bool any = false;
    for (auto& d : dense_asm) any |= group_of(mn[d.first]) == grp;
    if (any) {
      GW<double> g(B.step(SK_GEMM_D));
      std::function<void(const MNode&, int)> add = [&](const MNode& x, int ui) {
        const UNode& f = un[ui];
        if (!f.fin) {
          for (int c = 0; c < f.nchild; ++c) add(x, f.child0 + c);
          return;
        }
        const int64_t ro = TI.begin[f.t] - TI.begin[x.t], co = TK.begin[f.r] - TK.begin[x.r];
        g.task(Dw(x.U) + ro * x.n + co, x.n, f.m, f.n);
        if (f.form == 1) g.mm(Dw(f.U), f.K, Dw(f.Z), f.K, f.K, h2k::IT_TRANS_B);
        else if (f.form == 2) g.copy(Dw(f.U), f.K);
        else g.copy(Dw(f.Z), f.K, h2k::IT_TRANS_A);
      };
      for (auto& d : dense_asm)
        if (group_of(mn[d.first]) == grp) add(mn[d.first], d.second);
    }
  }
  for (int h = 0; h <= maxh; ++h) {
    std::vector<int> lv;
    for (size_t i = 0; i < mn.size(); ++i)
      if (mn[i].height == h && group_of(mn[i]) == grp) lv.push_back((int)i);
    if (lv.empty()) continue;
    if (h > 0) {  // U = [ext(U^_a S_a), ext(U^_b S_b)],  Z = [ext(V^_a), ext(V^_b)]
      for (int i : lv) {
        MNode& x = mn[i];
        x.K = 2 * kcap;
        x.U = B.wd((int64_t)x.m * x.K).off;
        x.Z = B.wd((int64_t)x.n * x.K).off;
        x.hz = mn[x.c0].t == x.t && mn[x.c1].t == x.t;
        x.vt = mn[x.c0].r == x.r && mn[x.c1].r == x.r;
      }
      {  // packed width of every merge: kappa_a + kappa_b
        Step& sc = B.step(SK_SCAN);
        for (int i : lv) {
          MNode& x = mn[i];
          x.Wsum = B.wi(1).off;
          PScan c;
          c.first = (int)sc.scansrc.size();
          c.count = 2;
          c.offs = Iw(B.wi(2).off);
          c.total = Iw(x.Wsum);
          sc.scansrc.push_back(Iw(mn[x.c0].Kap));
          sc.scansrc.push_back(Iw(mn[x.c1].Kap));
          sc.scan.push_back(c);
        }
      }
      // Children's columns packed: [0, kappa_a) from a, [kappa_a, kappa_a +
      // kappa_b) from b, each zero-extended to the rows of the merged block
      // (tasks without items write the zeros).  Columns from kappa_a + kappa_b
      // on are never written: every reader of U and Z takes that width from
      // the device (QR widths, GEMM inner dimensions, the rows of U^* U^).
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        int kid[2] = {x.c0, x.c1};
        for (int c = 0; c < 2; ++c) {
          const MNode& ch = mn[kid[c]];
          const int64_t ro = TI.begin[ch.t] - TI.begin[x.t], co = TK.begin[ch.r] - TK.begin[x.r];
          const DRef<int> off = c == 0 ? DRef<int>() : Iw(mn[x.c0].Kap);
          const DRef<int> kap = Iw(ch.Kap);
          auto zero = [&](int64_t base, int64_t r0, int64_t r1) {
            if (r1 <= r0) return;
            g.task(Dw(base) + r0 * x.K, x.K, (int)(r1 - r0), kcap);
            g.dev(kap, off);
          };
          g.task(Dw(x.U) + ro * x.K, x.K, ch.m, kcap);
          g.dev(kap, off);
          g.copy(Dw(ch.Wc), kcap);
          zero(x.U, 0, ro);
          zero(x.U, ro + ch.m, x.m);
          g.task(Dw(x.Z) + co * x.K, x.K, ch.n, kcap);
          g.dev(kap, off);
          g.copy(Dw(ch.Vh), kcap);
          zero(x.Z, 0, co);
          zero(x.Z, co + ch.n, x.n);
        }
        if (x.hz || x.vt) {  // C of the Gram-Schmidt step below, in the same launch
          const MNode &a = mn[x.c0], &b = mn[x.c1];
          x.Cb = B.wd((int64_t)kcap * kcap).off;
          g.task(Dw(x.Cb), kcap, kcap, kcap);
          g.dev(Iw(b.Kap), DRef<int>(), Iw(a.Kap));
          if (x.hz) g.mm(Dw(a.Uh), kcap, Dw(b.Wc), kcap, x.m, h2k::IT_TRANS_A);
          else g.mm(Dw(a.Vh), kcap, Dw(b.Vh), kcap, x.n, h2k::IT_TRANS_A);
        }
      }
    } else {
      for (int i : lv) {
        MNode& x = mn[i];
        x.uI = x.U == -2;
        x.zI = x.Z == -2;
        x.direct = (x.uI || x.zI) && std::max(x.m, x.n) <= 128;
      }
    }
    int wmax = 0;
    for (int i : lv) {
      MNode& x = mn[i];
      wmax = std::max(wmax, x.K);
      P.max_coarse_K = std::max(P.max_coarse_K, x.K);
      if (x.K > 128) throw Error(H2_ERR_TOO_LARGE, "coarsening width above 128");
      if (!x.direct) {
        if (!x.zI && !x.hz && !x.vt) x.RZ = B.wd((int64_t)x.K * x.K).off;
        if (!x.zI && !x.uI && !x.hz) x.Gh = B.wd((int64_t)x.m * x.K).off;
        if (x.hz || x.vt) {
          x.Pb = B.wd((int64_t)(x.hz ? x.m : x.n) * kcap).off;
          x.Rp = B.wd((int64_t)kcap * kcap).off;
        }
        if (!x.uI) x.RGt = B.wd((int64_t)x.K * x.K).off;
        x.Vk = B.wd((int64_t)x.K * kcap).off;
        x.Yk = B.wd((int64_t)x.m * kcap).off;
        x.Gy = B.wd((int64_t)kcap * kcap).off;
        x.T1 = B.wd((int64_t)kcap * kcap).off;
        x.R1 = B.wd((int64_t)kcap * kcap).off;
      }
      x.Sig = B.wd(std::max(x.K, x.n)).off;
      x.Kap = B.wi(1).off;
      x.Uh = B.wd((int64_t)x.m * kcap).off;
      if (!x.uI) x.Tm = B.wd((int64_t)x.K * kcap).off;
      if (!x.zI) x.Zh = B.wd((int64_t)x.n * kcap).off;
      x.Gz = B.wd((int64_t)kcap * kcap).off;
      x.T2 = B.wd((int64_t)kcap * kcap).off;
      x.R2 = B.wd((int64_t)kcap * kcap).off;
      x.Vh = B.wd((int64_t)x.n * kcap).off;
      x.Sb = B.wd((int64_t)kcap * kcap).off;
      x.Wc = B.wd((int64_t)x.m * kcap).off;
    }
    // effective width of a merge: kappa of the two children (device side)
    auto wd1 = [&](const MNode& x) { return x.c0 >= 0 ? Iw(mn[x.c0].Kap) : DRef<int>(); };
    auto wd2 = [&](const MNode& x) { return x.c1 >= 0 ? Iw(mn[x.c1].Kap) : DRef<int>(); };
    // A merge joins two truncated pieces W_a V^_a^* and W_b V^_b^* (W = U^ S,
    // U^ and V^ with orthonormal columns; columns [0, kappa_a) of U and Z
    // come from a, [kappa_a, kappa_a + kappa_b) from b).  The SVD needs a
    // matrix whose Gram matrix is the one of G^ = U R_Z^*.  One Gram-Schmidt
    // step against piece a's orthonormal factor gives it, with a QR of
    // kappa_b columns only:
    //  - the children share the merged block's rows (hz): Z is block diagonal
    //    with orthonormal columns, R_Z = I and G^ = U = [W_a, W_b].  With
    //    C = U^_a^* W_b and P = W_b - U^_a C = Q_P R_P,
    //    U = [U^_a, Q_P] [[S_a, C], [0, R_P]], which is R_G.
    //  - they share its columns (vt): Z = [V^_a, V^_b].  With C = V^_a^* V^_b
    //    and P = V^_b - V^_a C = Q_P R_P, R_Z = [[I, C], [0, R_P]], so G^ has
    //    the rows [W_a, 0] (of a) and [W_b C^*, W_b R_P^*] (of b), and
    //    G^ = diag(U^_a, U^_b) M with M = [[S_a, 0], [S_b C^*, S_b R_P^*]]:
    //    M^* M = G^^* G^, and M^* takes the place of R_G^*.
    bool anygs = false;
    for (int i : lv) anygs |= (mn[i].hz || mn[i].vt) && !mn[i].direct;
    if (anygs) {
      auto gs = [&](const MNode& x) { return (x.hz || x.vt) && !x.direct; };
      {  // P = (W_b or V^_b) - (U^_a or V^_a) C  (C formed with the packing of U and Z)
        GW<double> g(B.step(SK_GEMM_D));
        for (int i : lv) {
          MNode& x = mn[i];
          if (!gs(x)) continue;
          const MNode &a = mn[x.c0], &b = mn[x.c1];
          g.task(Dw(x.Pb), kcap, x.hz ? x.m : x.n, kcap);
          g.dev(Iw(b.Kap));
          g.copy(Dw(x.hz ? b.Wc : b.Vh), kcap);
          g.mm(Dw(x.hz ? a.Uh : a.Vh), kcap, Dw(x.Cb), kcap, kcap, 0, -1.0);
          g.kdev(Iw(a.Kap));
        }
      }
      {  // R_P (kappa_b columns)
        size_t n = 0;
        for (int i : lv) n += gs(mn[i]);
        QrSplit q(B, kcap, n);
        for (int i : lv) {
          MNode& x = mn[i];
          if (gs(x)) q.add(Dw(x.Pb), kcap, x.hz ? x.m : x.n, kcap, Dw(x.Rp), kcap, 0, Iw(mn[x.c1].Kap));
        }
      }
      {  // R_G^* (hz) or M^* (vt), and G^ of the vt merges
        GW<double> g(B.step(SK_GEMM_D));
        for (int i : lv) {
          MNode& x = mn[i];
          if (!gs(x)) continue;
          const MNode &a = mn[x.c0], &b = mn[x.c1];
          const DRef<int> ka = Iw(a.Kap), kb = Iw(b.Kap);
          const DRef<double> rg = Dw(x.RGt);
          const int K = x.K;
          g.task(rg, K, kcap, kcap);  // [0, ka) x [0, ka): S_a^*
          g.dev(ka, DRef<int>(), ka);
          g.copy(Dw(a.Sb), kcap, h2k::IT_TRANS_A);
          if (x.hz) {
            g.task(rg, K, kcap, kcap);  // [0, ka) x [ka, ka + kb): 0
            g.dev(kb, ka, ka);
            g.task(rg, K, kcap, kcap);  // [ka, ka + kb) x [0, ka): C^*
            g.dev(ka, DRef<int>(), kb, ka);
            g.copy(Dw(x.Cb), kcap, h2k::IT_TRANS_A);
            g.task(rg, K, kcap, kcap);  // [ka, ka + kb) x [ka, ka + kb): R_P^*
            g.dev(kb, ka, kb, ka);
            g.copy(Dw(x.Rp), kcap, h2k::IT_TRANS_A);
            continue;
          }
          g.task(rg, K, kcap, kcap);  // [0, ka) x [ka, ka + kb): C S_b^*
          g.dev(kb, ka, ka);
          g.mm(Dw(x.Cb), kcap, Dw(b.Sb), kcap, kcap, h2k::IT_TRANS_B);
          g.kdev(kb);
          g.task(rg, K, kcap, kcap);  // [ka, ka + kb) x [0, ka): 0
          g.dev(ka, DRef<int>(), kb, ka);
          g.task(rg, K, kcap, kcap);  // [ka, ka + kb) x [ka, ka + kb): R_P S_b^*
          g.dev(kb, ka, kb, ka);
          g.mm(Dw(x.Rp), kcap, Dw(b.Sb), kcap, kcap, h2k::IT_TRANS_B);
          g.kdev(kb);
          // G^: rows of a [W_a, 0], rows of b [W_b C^*, W_b R_P^*]
          const int64_t ra = TI.begin[a.t] - TI.begin[x.t], rb = TI.begin[b.t] - TI.begin[x.t];
          g.task(Dw(x.Gh) + ra * K, K, a.m, kcap);
          g.dev(ka);
          g.copy(Dw(a.Wc), kcap);
          g.task(Dw(x.Gh) + ra * K, K, a.m, kcap);
          g.dev(kb, ka);
          g.task(Dw(x.Gh) + rb * K, K, b.m, kcap);
          g.dev(ka);
          g.mm(Dw(b.Wc), kcap, Dw(x.Cb), kcap, kcap, h2k::IT_TRANS_B);
          g.kdev(kb);
          g.task(Dw(x.Gh) + rb * K, K, b.m, kcap);
          g.dev(kb, ka);
          g.mm(Dw(b.Wc), kcap, Dw(x.Rp), kcap, kcap, h2k::IT_TRANS_B);
          g.kdev(kb);
        }
      }
    }
    bool anyrz = false, anygh = false, anyrg = false;
    for (int i : lv) {
      const MNode& x = mn[i];
      if (x.direct || x.hz || x.vt) continue;
      anyrz |= !x.zI;
      anygh |= !x.uI && !x.zI;
      anyrg |= !x.uI;
    }
    if (anyrz) {  // R_Z: R factor of Z (Z = I: R_Z = I, skipped)
      QrSplit q(B, wmax, lv.size());
      for (int i : lv) {
        MNode& x = mn[i];
        if (!x.zI && !x.hz && !x.vt && !x.direct) q.add(Dw(x.Z), x.K, x.n, x.K, Dw(x.RZ), x.K, 0, wd1(x), wd2(x));
      }
    }
    for (int i : lv)
      if (mn[i].hz && !mn[i].direct) mn[i].Gh = mn[i].U;
    if (anygh) {  // condensed block G^ = U R_Z^* (same singular values as U Z^*);
                  // Z = I: G^ = U;  U = I: G^ = R_Z^*, used through a transposed operand
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.direct || x.uI || x.hz || x.vt) continue;
        if (x.zI) {
          x.Gh = x.U;
          continue;
        }
        g.task(Dw(x.Gh), x.K, x.m, x.K);
        g.mm(Dw(x.U), x.K, Dw(x.RZ), x.K, x.K, h2k::IT_TRANS_B);
        if (x.c0 >= 0) g.kdev(wd1(x), wd2(x));
      }
    } else {
      for (int i : lv)
        if (mn[i].zI && !mn[i].direct && !mn[i].uI) mn[i].Gh = mn[i].U;
    }
    if (anyrg) {  // R factor of G^, stored transposed.  U = I: R_Z has the right singular
                  // vectors of G^ = R_Z^* as its left ones and replaces R_G^*
      QrSplit q(B, wmax, lv.size());
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.direct || x.hz || x.vt) continue;
        if (x.uI) {
          x.RGt = x.RZ;
          continue;
        }
        q.add(Dw(x.Gh), x.K, x.m, x.K, Dw(x.RGt), x.K, 1, wd1(x), wd2(x));
      }
    } else {
      for (int i : lv)
        if (mn[i].uI && !mn[i].direct) mn[i].RGt = mn[i].RZ;
    }
    if (h == 0) {  // lower bounds of the block norms: largest column norm of the leaves' condensed factors
      Step& st = B.step(SK_REF);
      std::map<int, std::vector<int>> byb;
      for (int i : lv) byb[mn[i].below].push_back(i);
      for (auto& kv : byb) {
        PRef r;
        r.first = (int)st.refmat.size();
        r.count = (int)kv.second.size();
        r.factor = 1.0;
        r.out = Dw(tau[kv.first]);
        for (int i : kv.second) {
          const MNode& x = mn[i];
          // any row norm of G (or of a factor with the same Gram matrix) is a lower bound of its norm
          if (!x.direct) st.refmat.push_back({Dw(x.RGt), x.K, x.K, x.K});
          else if (x.zI) st.refmat.push_back({Dw(x.U), x.K, x.m, x.n});
          else st.refmat.push_back({Dw(x.Z), x.K, x.n, x.m});
        }
        st.ref.push_back(r);
      }
    }
    {  // right singular vectors of G^ (left ones of R^*), Frobenius tail <= tau_b
      Step& st = B.step(SK_SVD);
      st.wmax = wmax;
      for (int i : lv) {
        MNode& x = mn[i];
        PSvd s;
        s.a = Dw(x.RGt);
        s.u = Dw(x.Vk);
        s.sigma = Dw(x.Sig);
        s.rank = Iw(x.Kap);
        s.tolref = Dw(tau[x.below]);
        s.tolkind = 0;
        s.tolfactor = share(x);
        s.w_dev = wd1(x);
        s.w_dev2 = wd2(x);
        s.lda = x.K;
        s.ldu = kcap;
        s.rows = x.K;
        s.cols = x.K;
        s.kcap = kcap;
        if (x.direct) {  // left singular vectors of G (m x n) itself
          s.a = x.zI ? Dw(x.U) : Dw(x.Z);
          s.trans_a = x.zI ? 0 : 1;
          s.u = Dw(x.Uh);
          s.rows = x.m;
          s.cols = x.n;
          st.wmax = std::max(st.wmax, std::max(x.m, x.n));
        }
        st.svd.push_back(s);
      }
    }
    std::map<int, std::vector<int>> byb;  // blocks with merges above this height
    for (int i : lv)
      if (hmax[mn[i].below] > h) byb[mn[i].below].push_back(i);
    if (!byb.empty()) {  // raise nu_b: sigma_1 of this height's merged sub-blocks of b
      Step& st = B.step(SK_REF);
      for (auto& kv : byb) {
        PRef r;
        r.first = (int)st.refmat.size();
        r.count = 1 + (int)kv.second.size();
        r.factor = 1.0;
        r.out = Dw(tau[kv.first]);
        st.refmat.push_back({Dw(tau[kv.first]), 1, 1, 1});
        for (int i : kv.second) st.refmat.push_back({Dw(mn[i].Sig), 1, 1, 1, true});
        st.ref.push_back(r);
      }
    }
    {  // Y = G^ V_k  (= U^ Sigma)
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.direct) continue;
        g.task(Dw(x.Yk), kcap, x.m, kcap);
        if (x.uI) g.mm(Dw(x.RZ), x.K, Dw(x.Vk), kcap, x.K, h2k::IT_TRANS_A);
        else g.mm(Dw(x.Gh), x.K, Dw(x.Vk), kcap, x.K);
        if (x.c0 >= 0) g.kdev(wd1(x), wd2(x));
      }
    }
    {
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.direct) continue;
        g.task(Dw(x.Gy), kcap, kcap, kcap);
        g.mm(Dw(x.Yk), kcap, Dw(x.Yk), kcap, x.m, h2k::IT_TRANS_A);
      }
    }
    {
      Step& st = B.step(SK_CHOL);
      st.wmax = kcap;
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.direct) continue;
        st.chol.push_back({Dw(x.Gy), Dw(x.T1), Dw(x.R1), Iw(x.Kap), kcap, kcap, kcap, kcap});
      }
    }
    {  // U^ = Y T1 (orthonormal columns)
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.direct) continue;
        g.task(Dw(x.Uh), kcap, x.m, kcap);
        g.mm(Dw(x.Yk), kcap, Dw(x.T1), kcap, kcap);
        g.kdev(Iw(x.Kap));
      }
    }
    {  // T = U^* U^  (U = I: T = U^)
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.uI) {
          x.Tm = x.Uh;
          continue;
        }
        g.task(Dw(x.Tm), kcap, x.K, kcap);
        if (x.c0 >= 0) g.dev(DRef<int>(), DRef<int>(), Iw(x.Wsum));  // rows beyond the packed width unused
        g.mm(Dw(x.U), x.K, Dw(x.Uh), kcap, x.m, h2k::IT_TRANS_A);
      }
    }
    {  // Z^ = Z (U^* U^) = G^* U^:  G~ = U^ U^^* G = U^ Z^^*  (Z = I: Z^ = T)
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        if (x.zI) {
          x.Zh = x.Tm;
          continue;
        }
        g.task(Dw(x.Zh), kcap, x.n, kcap);
        g.mm(Dw(x.Z), x.K, Dw(x.Tm), kcap, x.K);
        if (x.c0 >= 0) g.kdev(wd1(x), wd2(x));
      }
    }
    {
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        g.task(Dw(x.Gz), kcap, kcap, kcap);
        g.mm(Dw(x.Zh), kcap, Dw(x.Zh), kcap, x.n, h2k::IT_TRANS_A);
      }
    }
    {
      Step& st = B.step(SK_CHOL);
      st.wmax = kcap;
      for (int i : lv) {
        MNode& x = mn[i];
        st.chol.push_back({Dw(x.Gz), Dw(x.T2), Dw(x.R2), Iw(x.Kap), kcap, kcap, kcap, kcap});
      }
    }
    {  // V^ = Z^ T2, S = R2^*:  G~ = U^ S V^^*
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        g.task(Dw(x.Vh), kcap, x.n, kcap);
        g.mm(Dw(x.Zh), kcap, Dw(x.T2), kcap, kcap);
        g.kdev(Iw(x.Kap));
        g.task(Dw(x.Sb), kcap, kcap, kcap);
        g.copy(Dw(x.R2), kcap, h2k::IT_TRANS_A);
      }
    }
    {  // W = U^ S, the row factor handed to the parent merge
      GW<double> g(B.step(SK_GEMM_D));
      for (int i : lv) {
        MNode& x = mn[i];
        g.task(Dw(x.Wc), kcap, x.m, kcap);
        g.mm(Dw(x.Uh), kcap, Dw(x.Sb), kcap, kcap);
        g.kdev(Iw(x.Kap));
      }
    }
  }
}

// Outputs of each block's root merge, used by the basis construction.
void Planner::coarsen_finish() {
  for (size_t li = 0; li < C.adm.size(); ++li) {
    UNode& u = un[bnode[li]];
    const MNode& x = mn[of_un[bnode[li]]];
    u.Uh = x.Uh;
    u.Vh = x.Vh;
    u.Sb = x.Sb;
    u.Sig = x.Sig;
    u.Kap = x.Kap;
  }
}

// The whole coarsening in one group (no exact product before it).
void Planner::coarsen() {
  assign_chunks(1);
  coarsen_prepare();
  for (int g = nchunk; g >= 0; --g) coarsen_group(g);
  coarsen_finish();
}

// Chunks of nch groups of union subtrees below the shallowest depth with at
// least 4 nch union nodes (one chunk: every node, from the root).
void Planner::assign_chunks(int nch) {
  nchunk = std::max(1, nch);
  uchunk.assign(un.size(), 0);
  bchunk.assign(C.adm.size(), 0);
  chunk_depth = 0;
  if (nchunk > 1) {
    std::map<int, int> per_depth;
    for (auto& u : un) per_depth[u.depth]++;
    chunk_depth = -1;
    for (auto& kv : per_depth)
      if (kv.second >= 4 * nchunk) {
        chunk_depth = kv.first;
        break;
      }
    if (chunk_depth < 0) {  // too few nodes for chunks
      nchunk = 1;
      chunk_depth = 0;
    }
  }
  if (nchunk > 1) {
    int count = 0;
    for (auto& u : un) count += u.depth == chunk_depth;
    int seen = 0;
    for (size_t i = 0; i < un.size(); ++i) {  // parents come before their children
      const UNode& u = un[i];
      if (u.depth < chunk_depth) uchunk[i] = -1;
      else if (u.depth == chunk_depth) uchunk[i] = (int)((int64_t)(seen++) * nchunk / count);
      else uchunk[i] = uchunk[u.parent];
    }
  }
  for (size_t li = 0; li < C.adm.size(); ++li) bchunk[li] = bnode[li] >= 0 ? uchunk[bnode[li]] : -1;
}

// ------------------------------------------------------------------ adaptive bases
void Planner::bases() {
  // Row and column bases are independent: both are built bottom-up in the
  // same launches, level by level (more tasks per launch on the small levels).
  B.phase = PH_ROW;
  struct Side {
    bool rows;
    const Tree* T;
    std::vector<std::vector<int>> own, star;  // star: row*(s) / col*(s)
    std::vector<std::map<int, int64_t>> proj;
    DRef<double> leafout, trout;
    DRef<int> rankout;
    int sflag;
    std::vector<int> cl, wcol;
    std::vector<int64_t> gst, rt, poff, ptot;
  };
  Side side[2];
  const int kk = kc * kc;
  const double th = P.theta;
  int maxdepth = 0;
  for (int sd = 0; sd < 2; ++sd) {
    Side& X = side[sd];
    X.rows = sd == 0;
    X.T = X.rows ? &TI : &TK;
    const Tree& T = *X.T;
    X.own.assign(T.ncl, {});
    for (size_t li = 0; li < C.adm.size(); ++li) {
      const auto& nd = C.nodes[C.adm[li]];
      X.own[X.rows ? nd.t : nd.s].push_back((int)li);
    }
    X.leafout = X.rows ? P.res_vleaf : P.res_wleaf;
    X.trout = X.rows ? P.res_vtr : P.res_wtr;
    X.rankout = X.rows ? P.res_rank_row : P.res_rank_col;
    X.sflag = X.rows ? h2k::IT_TRANS_A : 0;
    X.proj.assign(T.ncl, {});
    X.star.assign(T.ncl, {});
    for (int s = 0; s < T.ncl; ++s) {
      for (int a = s; a >= 0; a = T.parent[a])
        for (int li : X.own[a]) X.star[s].push_back(li);
      for (int li : X.star[s]) X.proj[s][li] = B.wd((int64_t)kc * kcap).off;
    }
    X.gst.assign(T.ncl, -1);
    X.rt.assign(T.ncl, -1);
    X.poff.assign(T.ncl, -1);
    X.ptot.assign(T.ncl, -1);
    X.wcol.assign(T.ncl, 0);
    maxdepth = std::max(maxdepth, T.depth);
  }
  for (int lev = maxdepth - 1; lev >= 0; --lev) {
    size_t ncl = 0;
    for (Side& X : side) {
      X.cl.clear();
      for (int s = 0; s < X.T->ncl; ++s)
        if (X.T->level[s] == lev) X.cl.push_back(s);
      ncl += X.cl.size();
    }
    if (ncl == 0) continue;
    {  // row offsets of the pieces: the kappa_b rows of block b follow each other
      Step& sc = B.step(SK_SCAN);
      for (Side& X : side)
        for (int s : X.cl) {
          PScan c;
          c.first = (int)sc.scansrc.size();
          c.count = (int)X.star[s].size();
          X.poff[s] = B.wi(std::max<int64_t>(c.count, 1)).off;
          X.ptot[s] = B.wi(1).off;
          c.offs = Iw(X.poff[s]);
          c.total = Iw(X.ptot[s]);
          for (int li : X.star[s]) sc.scansrc.push_back(Iw(un[bnode[li]].Kap));
          sc.scan.push_back(c);
        }
    }
    {  // weighted condensed blocks (transposed, kappa_b rows per block, stacked compactly)
      GW<double> g(B.step(SK_GEMM_D));
      for (Side& X : side) {
        const Tree& T = *X.T;
        for (int s : X.cl) {
          const bool lf = T.leaf(s);
          const int w = lf ? (int)T.size(s) : 2 * kc;
          X.wcol[s] = w;
          const int nrow = (int)X.star[s].size() * kcap;
          X.gst[s] = B.wd((int64_t)std::max(nrow, 1) * w).off;
          for (size_t j = 0; j < X.star[s].size(); ++j) {
            const int li = X.star[s][j];
            const UNode& u = un[bnode[li]];
            const auto& nd = C.nodes[C.adm[li]];
            const int owner = X.rows ? nd.t : nd.s;
            // 1/omega = theta^{-(level s - level owner)/2} / ||G~_b||
            const double alpha = std::pow(th, -0.5 * (T.level[s] - T.level[owner]));
            const DRef<double> out = Dw(X.gst[s]);
            const DRef<int> kap = Iw(u.Kap), ro = Iw(X.poff[s]) + (int64_t)j;
            const int fl = X.sflag | h2k::IT_TRANS_B | h2k::IT_SCALE_INV;
            if (lf) {
              const int64_t roff = T.begin[s] - T.begin[owner];
              g.task(out, w, kcap, w);
              g.dev(DRef<int>(), DRef<int>(), kap, ro);
              g.mm(Dw(u.Sb), kcap, Dw(X.rows ? u.Uh : u.Vh) + roff * kcap, kcap, kcap, fl, alpha, Dw(u.Sig));
              g.kdev(kap);
            } else {
              // children's coefficients packed: [0, k_c0) and [k_c0, k_c0 + k_c1)
              const int c0 = T.children[s][0], c1 = T.children[s][1];
              g.task(out, w, kcap, kc);
              g.dev(X.rankout + c0, DRef<int>(), kap, ro);
              g.mm(Dw(u.Sb), kcap, Dw(X.proj[c0][li]), kcap, kcap, fl, alpha, Dw(u.Sig));
              g.kdev(kap);
              g.task(out, w, kcap, kc);
              g.dev(X.rankout + c1, X.rankout + c0, kap, ro);
              g.mm(Dw(u.Sb), kcap, Dw(X.proj[c1][li]), kcap, kcap, fl, alpha, Dw(u.Sig));
              g.kdev(kap);
            }
          }
        }
      }
    }
    {  // R^* of the weighted matrix (the launcher picks the width class per task)
      int wmax = 0;
      for (Side& X : side)
        for (int s : X.cl) wmax = std::max(wmax, X.wcol[s]);
      if (wmax > 128) throw Error(H2_ERR_TOO_LARGE, "leaf size above 128");
      QrSplit q(B, wmax, ncl);
      for (Side& X : side) {
        const Tree& T = *X.T;
        for (int s : X.cl) {
          const int w = X.wcol[s];
          X.rt[s] = B.wd((int64_t)w * w).off;
          DRef<int> w1, w2;
          if (!T.leaf(s)) {
            w1 = X.rankout + T.children[s][0];
            w2 = X.rankout + T.children[s][1];
          }
          q.add(Dw(X.gst[s]), w, (int)X.star[s].size() * kcap, w, Dw(X.rt[s]), w, 1, w1, w2, Iw(X.ptot[s]));
        }
      }
    }
    {  // left singular vectors of the weighted matrix
      Step& st = B.step(SK_SVD);
      for (Side& X : side) {
        const Tree& T = *X.T;
        for (int s : X.cl) {
          const int w = X.wcol[s];
          st.wmax = std::max(st.wmax, w);
          PSvd v;
          v.a = Dw(X.rt[s]);
          if (T.leaf(s)) v.u = X.leafout + T.begin[s] * kc;
          else {
            // stacked transfers: rows [0, k_c0) give E_c0, the rest E_c1
            const int c0 = T.children[s][0], c1 = T.children[s][1];
            v.u = X.trout + (int64_t)c0 * kk;
            v.u2 = X.trout + (int64_t)c1 * kk;
            v.split_dev = X.rankout + c0;
            v.w_dev = X.rankout + c0;
            v.w_dev2 = X.rankout + c1;
            v.urows = kc;
          }
          v.sigma = Dw(B.wd(w).off);
          v.rank = X.rankout + s;
          v.tolkind = X.rows ? 1 : 2;
          v.tolfactor = 1.0;
          v.lda = w;
          v.ldu = kc;
          v.rows = w;
          v.cols = w;
          v.kcap = kc;
          st.svd.push_back(v);
        }
      }
    }
    {  // transfers and projections G^_{s,b} = V_s^* G^c_b|_s (coefficient part)
      GW<double> g(B.step(SK_GEMM_D));
      for (Side& X : side) {
        const Tree& T = *X.T;
        for (int s : X.cl) {
          if (T.leaf(s)) {
            for (int li : X.star[s]) {
              const UNode& u = un[bnode[li]];
              const auto& nd = C.nodes[C.adm[li]];
              const int owner = X.rows ? nd.t : nd.s;
              const int64_t roff = T.begin[s] - T.begin[owner];
              g.task(Dw(X.proj[s][li]), kcap, kc, kcap);
              g.mm(X.leafout + T.begin[s] * kc, kc, Dw(X.rows ? u.Uh : u.Vh) + roff * kcap, kcap, (int)T.size(s),
                   h2k::IT_TRANS_A);
            }
          } else {
            const int c0 = T.children[s][0], c1 = T.children[s][1];
            for (int li : X.star[s]) {
              g.task(Dw(X.proj[s][li]), kcap, kc, kcap);
              g.mm(X.trout + (int64_t)c0 * kk, kc, Dw(X.proj[c0][li]), kcap, kc, h2k::IT_TRANS_A);
              g.kdev(X.rankout + c0);
              g.mm(X.trout + (int64_t)c1 * kk, kc, Dw(X.proj[c1][li]), kcap, kc, h2k::IT_TRANS_A);
              g.kdev(X.rankout + c1);
            }
          }
        }
      }
    }
  }
  row_proj = std::move(side[0].proj);
  col_proj = std::move(side[1].proj);
}

// ------------------------------------------------------------------ couplings
void Planner::couplings() {
  B.phase = PH_COUPLE;
  const int kk = kc * kc;
  std::vector<int64_t> tmp(C.adm.size());
  {
    GW<double> g(B.step(SK_GEMM_D));
    for (size_t li = 0; li < C.adm.size(); ++li) {
      const auto& nd = C.nodes[C.adm[li]];
      const UNode& u = un[bnode[li]];
      tmp[li] = B.wd((int64_t)kc * kcap).off;
      g.task(Dw(tmp[li]), kcap, kc, kcap);
      g.mm(Dw(row_proj[nd.t][(int)li]), kcap, Dw(u.Sb), kcap, kcap);
      g.kdev(Iw(u.Kap));
    }
  }
  {  // S_b = (V_t^* U^) S (W_r^* V^)^*
    GW<double> g(B.step(SK_GEMM_D));
    for (size_t li = 0; li < C.adm.size(); ++li) {
      const auto& nd = C.nodes[C.adm[li]];
      g.task(P.res_S + (int64_t)li * kk, kc, kc, kc);
      g.mm(Dw(tmp[li]), kcap, Dw(col_proj[nd.s][(int)li]), kcap, kcap, h2k::IT_TRANS_B);
      g.kdev(Iw(un[bnode[li]].Kap));
    }
  }
}

// ------------------------------------------------------------------ finalisation
template <typename T>
static T* res(const DRef<T>& r, const Plan& P) {
  if (r.ws == WS_NONE) return r.ext ? r.ext + r.off : nullptr;
  if (r.ws == WS_D) return reinterpret_cast<T*>(P.wd + r.off);
  if (r.ws == WS_F) return reinterpret_cast<T*>(P.wf + r.off);
  return reinterpret_cast<T*>(P.wi + r.off);
}

template <typename T>
static void emit_gemm(Plan& P, Step& st, std::vector<char>& blob, const std::vector<PItem<T>>& it,
                      const std::vector<PTask<T>>& tk) {
  auto align = [&](size_t a) {
    while (blob.size() % a) blob.push_back(0);
  };
  align(64);
  st.desc_off = blob.size();
  std::vector<GemmItem<T>> items(it.size());
  for (size_t i = 0; i < it.size(); ++i) {
    items[i].a = res(it[i].a, P);
    items[i].b = res(it[i].b, P);
    items[i].scale = res(it[i].scale, P);
    items[i].k_dev = res(it[i].kd1, P);
    items[i].k_dev2 = res(it[i].kd2, P);
    items[i].lda = it[i].lda;
    items[i].ldb = it[i].ldb;
    items[i].k = it[i].k;
    items[i].flags = it[i].flags;
    items[i].alpha = it[i].alpha;
  }
  blob.insert(blob.end(), (char*)items.data(), (char*)(items.data() + items.size()));
  st.nitems = (int64_t)items.size();
  align(64);
  st.desc2_off = blob.size();
  std::vector<GemmTask<T>> tasks(tk.size());
  std::vector<GemmTile> tiles;
  for (size_t i = 0; i < tk.size(); ++i) {
    tasks[i].c = res(tk[i].c, P);
    tasks[i].m_dev = res(tk[i].m_dev, P);
    tasks[i].n_dev = res(tk[i].n_dev, P);
    tasks[i].coff_dev = res(tk[i].coff_dev, P);
    tasks[i].roff_dev = res(tk[i].roff_dev, P);
    tasks[i].ldc = tk[i].ldc;
    tasks[i].m = tk[i].m;
    tasks[i].n = tk[i].n;
    tasks[i].item0 = tk[i].item0;
    tasks[i].nitem = tk[i].nitem;
    tasks[i].beta = tk[i].beta;
    tasks[i].stat = st.stat_off >= 0 ? P.wi + st.stat_off + 3 * (int64_t)i : nullptr;
    tasks[i].ncopy = 0;
    tasks[i].pad = 0;
    for (int q = 0; q < tk[i].nitem; ++q)
      if (it[tk[i].item0 + q].flags & h2k::IT_COPY) ++tasks[i].ncopy;
    for (int m0 = 0; m0 < tk[i].m; m0 += 64)
      for (int n0 = 0; n0 < tk[i].n; n0 += 64) tiles.push_back({(int)i, m0, n0, 0});
  }
  blob.insert(blob.end(), (char*)tasks.data(), (char*)(tasks.data() + tasks.size()));
  align(64);
  st.tiles_off = blob.size();
  blob.insert(blob.end(), (char*)tiles.data(), (char*)(tiles.data() + tiles.size()));
  st.ntiles = (int)tiles.size();
  st.ndesc = (int)tasks.size();
}

static std::vector<h2k::SvdTask> svd_tasks(Plan& P, Step& st, double eps) {
  std::vector<h2k::SvdTask> v(st.svd.size());
  const double dc = eps * P.budget[0], dr = eps * P.budget[1], dw = eps * P.budget[2];
  const double scale = std::sqrt(1.0 - P.sigma_br * P.theta);
  for (size_t i = 0; i < st.svd.size(); ++i) {
    const PSvd& s = st.svd[i];
    v[i].a = res(s.a, P);
    v[i].u = res(s.u, P);
    v[i].u2 = res(s.u2, P);
    v[i].w_dev = res(s.w_dev, P);
    v[i].w_dev2 = res(s.w_dev2, P);
    v[i].split_dev = res(s.split_dev, P);
    v[i].stat = P.wi + st.stat_off + 4 * i;
    v[i].urows = s.urows;
    v[i].qrcp = P.qrcp;
    v[i].maxsw = P.sweeps;
    v[i].sigma = res(s.sigma, P);
    v[i].rank = res(s.rank, P);
    v[i].tol_abs = 0.0;
    v[i].tol_rel = 0.0;
    v[i].tol_ptr = res(s.tolref, P);
    v[i].tol_scale = 0.0;
    v[i].frob = 0;
    if (s.tolkind == 0) {
      v[i].tol_scale = dc * s.tolfactor;
      v[i].frob = 1;
      v[i].ovf_bit = 1;
    } else {
      v[i].tol_abs = (s.tolkind == 1 ? dr : dw) * scale;
      v[i].ovf_bit = 2;
    }
    v[i].lda = s.lda;
    v[i].ldu = s.ldu;
    v[i].rows = s.rows;
    v[i].cols = s.cols;
    v[i].kcap = s.kcap;
    v[i].trans_a = s.trans_a;
  }
  return v;
}

// The step's SVD descriptors appended to the blob.
static void resolve_svd(Plan& P, Step& st, std::vector<char>& blob, double eps) {
  const std::vector<h2k::SvdTask> v = svd_tasks(P, st, eps);
  while (blob.size() % 64) blob.push_back(0);
  st.desc_off = blob.size();
  blob.insert(blob.end(), (const char*)v.data(), (const char*)(v.data() + v.size()));
  st.ndesc = (int)v.size();
}

// ------------------------------------------------------------------ workspace sharing
// A workspace buffer lives from the first to the last step that refers to it
// (steps run in order on one stream); buffers with disjoint lifetimes share
// memory.  Buffers of equal lifetime form a group; groups are placed in order
// of their first use, best fit into the gaps left by groups that died before
// (a group that fits no gap buffer by buffer), else at the top.  The result
// arrays stay live to the end (they are copied out after the product).
// Calls f on every workspace reference of a step; refs of one vector are
// visited in parallel when there are many (f must be safe for that).
template <typename V, typename F>
static void each_par(V& v, F&& f) {
  const int64_t n = (int64_t)v.size();
  if (n < 8192) {
    for (auto& x : v) f(x);
    return;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) f(v[i]);
}
template <typename F>
static void visit_refs_par(Step& st, F&& f) {
  each_par(st.itd, [&](auto& x) {
    f(x.a);
    f(x.b);
    f(x.scale);
  });
  each_par(st.tkd, [&](auto& x) { f(x.c); });
  each_par(st.itf, [&](auto& x) {
    f(x.a);
    f(x.b);
    f(x.scale);
  });
  each_par(st.tkf, [&](auto& x) { f(x.c); });
  each_par(st.qr, [&](auto& x) {
    f(x.a);
    f(x.r);
  });
  each_par(st.svd, [&](auto& x) {
    f(x.a);
    f(x.u);
    f(x.sigma);
    f(x.u2);
    f(x.tolref);
  });
  each_par(st.chol, [&](auto& x) {
    f(x.g);
    f(x.t);
    f(x.r);
  });
  each_par(st.fill, [&](auto& x) { f(x.p); });
  each_par(st.ref, [&](auto& x) { f(x.out); });
  each_par(st.refmat, [&](auto& x) { f(x.a); });
  f(st.cvt_in);
  f(st.cvt_out);
}

template <typename F>
static void visit_refs(Step& st, F&& f) {
  for (auto& x : st.itd) {
    f(x.a);
    f(x.b);
    f(x.scale);
  }
  for (auto& x : st.tkd) f(x.c);
  for (auto& x : st.itf) {
    f(x.a);
    f(x.b);
    f(x.scale);
  }
  for (auto& x : st.tkf) f(x.c);
  for (auto& x : st.qr) {
    f(x.a);
    f(x.r);
  }
  for (auto& x : st.svd) {
    f(x.a);
    f(x.u);
    f(x.sigma);
    f(x.u2);
    f(x.tolref);
  }
  for (auto& x : st.chol) {
    f(x.g);
    f(x.t);
    f(x.r);
  }
  for (auto& x : st.fill) f(x.p);
  for (auto& x : st.ref) f(x.out);
  for (auto& x : st.refmat) f(x.a);
  f(st.cvt_in);
  f(st.cvt_out);
}

struct ArenaPlan {
  const std::vector<int64_t>& base;
  int64_t total;
  std::vector<int> first, last;
  std::vector<int64_t> placed;
  static constexpr int kPage = 12;  // lookup pages of 4096 elements
  std::vector<int> page;            // first allocation overlapping each page
  ArenaPlan(const std::vector<int64_t>& b, int64_t t)
      : base(b), total(t), first(b.size(), INT32_MAX), last(b.size(), -1), placed(b.size(), 0) {
    page.assign((size_t)(t >> kPage) + 2, 0);
    size_t i = 0;
    for (size_t p = 0; p < page.size(); ++p) {
      const int64_t o = (int64_t)p << kPage;
      while (i + 1 < base.size() && base[i + 1] <= o) ++i;
      page[p] = (int)i;
    }
  }
  size_t find(int64_t off) const {  // allocation containing element `off`
    const size_t p = std::min((size_t)(off >> kPage), page.size() - 2);
    const auto lo = base.begin() + page[p], hi = base.begin() + std::min<size_t>(page[p + 1] + 1, base.size());
    auto it = std::upper_bound(lo, hi, off);
    return (size_t)(it - base.begin()) - 1;
  }
  int64_t size(size_t i) const { return (i + 1 < base.size() ? base[i + 1] : total) - base[i]; }
  // Steps are recorded in increasing order; the references of one step may
  // be recorded from several threads, which all store the same step number.
  void use(int64_t off, int step) {
    if (base.empty()) return;
    const size_t i = find(off);
    if (__atomic_load_n(&first[i], __ATOMIC_RELAXED) > step) __atomic_store_n(&first[i], step, __ATOMIC_RELAXED);
    if (__atomic_load_n(&last[i], __ATOMIC_RELAXED) < step) __atomic_store_n(&last[i], step, __ATOMIC_RELAXED);
  }
  // Buffers with the same lifetime (first and last step) form one group.
  // Groups are placed in order of their first step: best fit of the whole
  // group (its buffers contiguous, in index order) into the gaps left by
  // groups that died before; a group that fits no gap places its buffers
  // one by one, best fit each, else at the top.
  int64_t place() {
    std::unordered_map<int64_t, int> gid;
    std::vector<int> grp(base.size(), -1);
    std::vector<int64_t> gsize;
    std::vector<int> gfirst, glast;
    const int64_t span = (int64_t)INT32_MAX + 1;
    for (size_t i = 0; i < base.size(); ++i) {
      if (last[i] < 0) continue;
      const int64_t key = (int64_t)first[i] * span + last[i];
      auto ins = gid.emplace(key, (int)gsize.size());
      if (ins.second) {
        gsize.push_back(0);
        gfirst.push_back(first[i]);
        glast.push_back(last[i]);
      }
      const int g = ins.first->second;
      grp[i] = g;
      placed[i] = gsize[g];  // offset inside the group while the group is whole
      gsize[g] += size(i);
    }
    const size_t ng = gsize.size();
    // members of each group, in index order
    std::vector<int64_t> mbeg(ng + 1, 0);
    for (size_t i = 0; i < base.size(); ++i)
      if (grp[i] >= 0) ++mbeg[grp[i] + 1];
    for (size_t g = 0; g < ng; ++g) mbeg[g + 1] += mbeg[g];
    std::vector<size_t> mem(mbeg[ng]);
    {
      std::vector<int64_t> fill(mbeg.begin(), mbeg.end() - 1);
      for (size_t i = 0; i < base.size(); ++i)
        if (grp[i] >= 0) mem[fill[grp[i]]++] = i;
    }
    std::vector<size_t> order(ng);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return gfirst[a] < gfirst[b]; });
    std::vector<int64_t> gplaced(ng, -1);  // -1: placed buffer by buffer
    std::map<int64_t, int64_t> byoff;                  // free gaps: offset -> size
    std::set<std::pair<int64_t, int64_t>> bysize;      // (size, offset)
    auto erase_gap = [&](std::map<int64_t, int64_t>::iterator g) {
      bysize.erase({g->second, g->first});
      byoff.erase(g);
    };
    auto add_gap = [&](int64_t off, int64_t sz) {
      auto nx = byoff.lower_bound(off);
      if (nx != byoff.end() && nx->first == off + sz) {
        sz += nx->second;
        erase_gap(nx);
      }
      auto pv = byoff.lower_bound(off);
      if (pv != byoff.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
          off = pv->first;
          sz += pv->second;
          erase_gap(pv);
        }
      }
      byoff[off] = sz;
      bysize.emplace(sz, off);
    };
    int64_t top = 0;
    auto take = [&](int64_t need) -> int64_t {  // best fit, else the top
      auto f = bysize.lower_bound({need, INT64_MIN});
      if (f == bysize.end()) {
        top += need;
        return top - need;
      }
      const int64_t off = f->second, sz = f->first;
      erase_gap(byoff.find(off));
      if (sz > need) add_gap(off + need, sz - need);
      return off;
    };
    typedef std::pair<int, size_t> Live;  // (last step, group)
    std::priority_queue<Live, std::vector<Live>, std::greater<Live>> live;
    for (size_t g : order) {
      while (!live.empty() && live.top().first < gfirst[g]) {
        const size_t j = live.top().second;
        live.pop();
        if (gplaced[j] >= 0) add_gap(gplaced[j], gsize[j]);
        else
          for (int64_t q = mbeg[j]; q < mbeg[j + 1]; ++q) add_gap(placed[mem[q]], size(mem[q]));
      }
      const int64_t need = gsize[g];
      if (bysize.empty() || bysize.rbegin()->first >= need) {
        gplaced[g] = take(need);
        for (int64_t q = mbeg[g]; q < mbeg[g + 1]; ++q) placed[mem[q]] += gplaced[g];
      } else {
        for (int64_t q = mbeg[g]; q < mbeg[g + 1]; ++q) placed[mem[q]] = take(size(mem[q]));
      }
      live.emplace(glast[g], g);
    }
    return top;
  }
  int64_t remap(int64_t off) const {
    if (base.empty()) return off;
    const size_t i = find(off);
    return placed[i] + (off - base[i]);
  }
};

static void share_workspace(Plan& P) {
  const bool trace = std::getenv("H2_TRACE") != nullptr;
  auto t0 = std::chrono::steady_clock::now();
  ArenaPlan ad(P.base_d, P.wsd), af(P.base_f, P.wsf);
  const int nst = (int)P.steps.size();
  int si = 0;
  auto use = [&](auto& r) {
    if (r.ws == WS_D) ad.use(r.off, si);
    else if (r.ws == WS_F) af.use(r.off, si);
  };
  for (auto& r : P.inputs) use(r);  // filled before the first step
  for (auto& st : P.steps) {
    visit_refs_par(st, use);
    ++si;
  }
  const auto t_use = std::chrono::steady_clock::now();
  si = nst;  // result arrays: live to the end
  for (DRef<double>* r : {&P.res_vleaf, &P.res_vtr, &P.res_wleaf, &P.res_wtr, &P.res_S, &P.res_N}) use(*r);
  P.wsd_planned = P.wsd;
  P.wsf_planned = P.wsf;
  if (std::getenv("H2_TRACE")) {  // live FP64 workspace per step; at the peak, split by the phase of first use
    std::vector<int64_t> diff(nst + 2, 0);
    for (size_t i = 0; i < ad.base.size(); ++i)
      if (ad.last[i] >= 0) {
        diff[ad.first[i]] += ad.size(i);
        diff[ad.last[i] + 1] -= ad.size(i);
      }
    int64_t cur = 0, peak = 0;
    int pk = 0;
    for (int k = 0; k <= nst; ++k) {
      cur += diff[k];
      if (cur > peak) peak = cur, pk = k;
    }
    double by[8] = {0};
    for (size_t i = 0; i < ad.base.size(); ++i)
      if (ad.last[i] >= 0 && ad.first[i] <= pk && ad.last[i] >= pk)
        by[ad.first[i] < nst ? P.steps[ad.first[i]].phase : 7] += ad.size(i) * 8e-9;
    std::vector<std::pair<int64_t, size_t>> big;
    for (size_t i = 0; i < ad.base.size(); ++i)
      if (ad.last[i] >= 0 && ad.first[i] <= pk && ad.last[i] >= pk) big.push_back({ad.size(i), i});
    std::sort(big.rbegin(), big.rend());
    for (size_t j = 0; j < std::min<size_t>(big.size(), 6); ++j)
      std::fprintf(stderr, "[h2 plan]   live at peak: %.3f GB, steps %d..%d\n", big[j].first * 8e-9,
                   ad.first[big[j].second], ad.last[big[j].second]);
    std::fprintf(stderr, "[h2 plan]   %zu buffers live at peak\n", big.size());
    std::map<std::pair<int, int>, std::pair<int64_t, int>> grp;
    for (auto& b : big) {
      auto& g = grp[{ad.first[b.second], ad.last[b.second]}];
      g.first += b.first;
      g.second += 1;
    }
    std::vector<std::pair<int64_t, std::pair<int, int>>> gs;
    for (auto& g : grp) gs.push_back({g.second.first, g.first});
    std::sort(gs.rbegin(), gs.rend());
    for (size_t j = 0; j < std::min<size_t>(gs.size(), 12); ++j)
      std::fprintf(stderr, "[h2 plan]   group steps %d..%d (kinds %d..%d): %.3f GB in %d buffers\n",
                   gs[j].second.first, gs[j].second.second, (int)P.steps[gs[j].second.first].kind,
                   gs[j].second.second < nst ? (int)P.steps[gs[j].second.second].kind : -1, gs[j].first * 8e-9,
                   grp[gs[j].second].second);
    std::fprintf(stderr,
                 "[h2 plan] peak live fp64 %.3f GB at step %d (phase %d): by phase of first use prep %.3f exact "
                 "%.3f leaf %.3f coarse %.3f row %.3f col %.3f couple %.3f result %.3f GB\n",
                 peak * 8e-9, pk, pk < nst ? P.steps[pk].phase : -1, by[0], by[1], by[2], by[3], by[4], by[5], by[6],
                 by[7]);
  }
  auto t1 = std::chrono::steady_clock::now();
  P.wsd = ad.place();
  P.wsf = af.place();
  auto t2 = std::chrono::steady_clock::now();
  auto remap = [&](auto& r) {
    if (r.ws == WS_D) r.off = ad.remap(r.off);
    else if (r.ws == WS_F) r.off = af.remap(r.off);
  };
  for (auto& st : P.steps) visit_refs_par(st, remap);
  if (trace) {
    auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
    std::fprintf(stderr, "[h2 plan] sharing: %zu + %zu buffers, lifetimes %.0f ms, placement %.0f ms, remap %.0f ms\n",
                 ad.base.size(), af.base.size(), ms(t0, t_use), ms(t1, t2), ms(t2, std::chrono::steady_clock::now()));
  }
  for (DRef<double>* r : {&P.res_vleaf, &P.res_vtr, &P.res_wleaf, &P.res_wtr, &P.res_S, &P.res_N}) remap(*r);
  for (auto& r : P.inputs) remap(r);
}

// Scale of a matrix in a block-norm bound: an approximate sub-block's
// sigma_1 exceeds the exact sub-block's norm by at most the truncation error
// made so far, which is <= delta_c times the block's norm.
static double ref_scale(const Plan& P, const PRefMat& m, double eps) {
  return m.approx ? 1.0 / (1.0 + eps * P.budget[0]) : 1.0;
}

// Sizes of the workspaces (the QR / SVD size reports go after the int
// buffers) and their total in bytes.
static size_t ws_part(int64_t count, size_t elem) { return ((size_t)std::max<int64_t>(count, 1) * elem + 255) & ~size_t(255); }

static void layout(Plan& P) {
  for (auto& st : P.steps) {
    const bool gemm = st.kind == SK_GEMM_D || st.kind == SK_GEMM_F;
    const int per = st.kind == SK_QR ? 2 : (st.kind == SK_SVD ? 4 : (gemm ? 3 : 0));
    const size_t n = st.kind == SK_QR ? st.qr.size()
                                      : (st.kind == SK_SVD ? st.svd.size() : (st.kind == SK_GEMM_D ? st.tkd.size() : st.tkf.size()));
    if (!per || !n) continue;
    st.stat_off = P.wsi;
    P.wsi += ((int64_t)(per * n) + 63) & ~int64_t(63);
  }
  P.ws_bytes = ws_part(P.wsd, sizeof(double)) + ws_part(P.wsf, sizeof(float)) + ws_part(P.wsi, sizeof(int));
  if (std::getenv("H2_TRACE"))
    std::fprintf(stderr, "[h2 plan] workspace %.3f GB fp64, %.3f GB fp32, %.3f GB int, %zu steps\n",
                 P.wsd * 8e-9, P.wsf * 4e-9, P.wsi * 4e-9, P.steps.size());
}

// Points the workspaces at `base` (ws_bytes long).
static void set_base(Plan& P, char* base) {
  P.wd = reinterpret_cast<double*>(base);
  P.wf = reinterpret_cast<float*>(base + ws_part(P.wsd, sizeof(double)));
  P.wi = reinterpret_cast<int*>(base + ws_part(P.wsd, sizeof(double)) + ws_part(P.wsf, sizeof(float)));
}

// Descriptors of every step resolved against the current workspace pointers
// (host bytes; st.desc_off etc. are offsets into them).
static std::vector<char> build_blob(Plan& P, double eps) {
  std::vector<char> blob;
  auto align = [&](size_t a) {
    while (blob.size() % a) blob.push_back(0);
  };
  for (auto& st : P.steps) {
    switch (st.kind) {
      case SK_GEMM_D: emit_gemm(P, st, blob, st.itd, st.tkd); break;
      case SK_GEMM_F: emit_gemm(P, st, blob, st.itf, st.tkf); break;
      case SK_QR: {
        align(64);
        st.desc_off = blob.size();
        for (size_t i = 0; i < st.qr.size(); ++i) {
          const PQr& q = st.qr[i];
          int* stat = P.wi + st.stat_off + 2 * i;
          h2k::QrTask t;
          std::memset(&t, 0, sizeof t);  // deterministic bytes, padding included
          t = h2k::QrTask{res(q.a, P), res(q.r, P), res(q.w_dev, P), res(q.w_dev2, P), res(q.m_dev, P), stat,
                          q.lda,       q.ldr,       q.m,               q.w,                q.trans_r,         q.mul_we,
                          q.part,      q.m_off};
          blob.insert(blob.end(), (char*)&t, (char*)&t + sizeof(t));
        }
        st.ndesc = (int)st.qr.size();
        break;
      }
      case SK_SVD: resolve_svd(P, st, blob, eps); break;
      case SK_CHOL: {
        align(64);
        st.desc_off = blob.size();
        for (auto& c : st.chol) {
          h2k::CholTask t;
          std::memset(&t, 0, sizeof t);
          t = h2k::CholTask{res(c.g, P), res(c.t, P), res(c.r, P), res(c.weff, P), c.ldg, c.ldt, c.ldr, c.w};
          blob.insert(blob.end(), (char*)&t, (char*)&t + sizeof(t));
        }
        st.ndesc = (int)st.chol.size();
        break;
      }
      case SK_FILL: {
        align(64);
        st.desc_off = blob.size();
        for (auto& f : st.fill) {
          h2k::FillTask t;
          std::memset(&t, 0, sizeof t);
          t = h2k::FillTask{res(f.p, P), f.ld, f.m, f.n, 0, f.value, f.diag, 8};
          blob.insert(blob.end(), (char*)&t, (char*)&t + sizeof(t));
        }
        st.ndesc = (int)st.fill.size();
        break;
      }
      case SK_REF: {
        align(64);
        st.desc_off = blob.size();
        for (auto& r : st.ref) {
          h2k::RefTask t;
          std::memset(&t, 0, sizeof t);
          t = h2k::RefTask{r.first, r.count, r.factor, res(r.out, P)};
          blob.insert(blob.end(), (char*)&t, (char*)&t + sizeof(t));
        }
        align(64);
        st.desc2_off = blob.size();
        for (auto& m : st.refmat) {
          h2k::RefMat t;
          std::memset(&t, 0, sizeof t);  // 4 bytes of padding before scale
          t.a = res(m.a, P);
          t.lda = m.lda;
          t.rows = m.rows;
          t.cols = m.cols;
          t.scale = ref_scale(P, m, eps);
          blob.insert(blob.end(), (char*)&t, (char*)&t + sizeof(t));
        }
        st.ndesc = (int)st.ref.size();
        break;
      }
      case SK_SCAN: {
        align(64);
        st.desc_off = blob.size();
        for (auto& c : st.scan) {
          h2k::ScanTask t;
          std::memset(&t, 0, sizeof t);
          t = h2k::ScanTask{c.first, c.count, res(c.offs, P), res(c.total, P)};
          blob.insert(blob.end(), (char*)&t, (char*)&t + sizeof(t));
        }
        align(64);
        st.desc2_off = blob.size();
        for (auto& r : st.scansrc) {
          const int* ptr = res(r, P);
          blob.insert(blob.end(), (char*)&ptr, (char*)&ptr + sizeof(ptr));
        }
        st.ndesc = (int)st.scan.size();
        break;
      }
      case SK_CVT_F2D: break;
    }
  }
  return blob;
}

// Workspace base of a plan's descriptors (its FP64 part starts the arena).
static char* ws_base(const Plan& P) { return reinterpret_cast<char*>(P.wd); }

// Shifts every workspace pointer of a descriptor blob (host copy) that lies
// in [from, from + len) by `to - from`.  Pointers outside that range (the
// operands, null) stay: they were allocated before the descriptors, while
// the old workspace was live, so they cannot lie in it.
static void rebase_blob(const Plan& P, std::vector<char>& blob, const char* from, const char* to, size_t len) {
  auto fix = [&](auto& ptr) {
    const char* q = reinterpret_cast<const char*>(ptr);
    if (q >= from && q < from + len)
      ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(const_cast<char*>(to + (q - from)));
  };
  auto arr = [&](size_t off, size_t n, auto* tag, auto&& f) {
    using D = std::remove_pointer_t<decltype(tag)>;
    D* a = reinterpret_cast<D*>(blob.data() + off);
    for (size_t i = 0; i < n; ++i) f(a[i]);
  };
  for (const auto& st : P.steps) {
    switch (st.kind) {
      case SK_GEMM_D:
      case SK_GEMM_F: {
        auto items = [&](auto& it) {
          fix(it.a);
          fix(it.b);
          fix(it.scale);
          fix(it.k_dev);
          fix(it.k_dev2);
        };
        auto tasks = [&](auto& t) {
          fix(t.c);
          fix(t.m_dev);
          fix(t.n_dev);
          fix(t.coff_dev);
          fix(t.roff_dev);
          fix(t.stat);
        };
        if (st.kind == SK_GEMM_D) {
          arr(st.desc_off, st.nitems, (h2k::GemmItem<double>*)nullptr, items);
          arr(st.desc2_off, st.ndesc, (h2k::GemmTask<double>*)nullptr, tasks);
        } else {
          arr(st.desc_off, st.nitems, (h2k::GemmItem<float>*)nullptr, items);
          arr(st.desc2_off, st.ndesc, (h2k::GemmTask<float>*)nullptr, tasks);
        }
        break;
      }
      case SK_QR:
        arr(st.desc_off, st.ndesc, (h2k::QrTask*)nullptr, [&](h2k::QrTask& t) {
          fix(t.a);
          fix(t.r);
          fix(t.w_dev);
          fix(t.w_dev2);
          fix(t.m_dev);
          fix(t.stat);
        });
        break;
      case SK_SVD:
        arr(st.desc_off, st.ndesc, (h2k::SvdTask*)nullptr, [&](h2k::SvdTask& t) {
          fix(t.a);
          fix(t.u);
          fix(t.u2);
          fix(t.sigma);
          fix(t.rank);
          fix(t.tol_ptr);
          fix(t.w_dev);
          fix(t.w_dev2);
          fix(t.split_dev);
          fix(t.stat);
        });
        break;
      case SK_CHOL:
        arr(st.desc_off, st.ndesc, (h2k::CholTask*)nullptr, [&](h2k::CholTask& t) {
          fix(t.g);
          fix(t.t);
          fix(t.r);
          fix(t.weff);
        });
        break;
      case SK_FILL:
        arr(st.desc_off, st.ndesc, (h2k::FillTask*)nullptr, [&](h2k::FillTask& t) { fix(t.p); });
        break;
      case SK_REF:
        arr(st.desc_off, st.ndesc, (h2k::RefTask*)nullptr, [&](h2k::RefTask& t) { fix(t.out); });
        arr(st.desc2_off, st.refmat.size(), (h2k::RefMat*)nullptr, [&](h2k::RefMat& t) { fix(t.a); });
        break;
      case SK_SCAN:
        arr(st.desc_off, st.ndesc, (h2k::ScanTask*)nullptr, [&](h2k::ScanTask& t) {
          fix(t.offs);
          fix(t.total);
        });
        arr(st.desc2_off, st.scansrc.size(), (const int**)nullptr, [&](const int*& q) { fix(q); });
        break;
      case SK_CVT_F2D:
        break;
    }
  }
}

static void drop_protos(Plan& P);

// Descriptors uploaded to the plan's own descriptor buffer.  Built from the
// step protos the first time; afterwards (the workspace moved: a new arena)
// the uploaded descriptors are rebased, which keeps the tolerances they were
// patched to (P.eps_set).
static void emit(Plan& P, double eps) {
  // a captured graph holds workspace pointers as kernel arguments (the
  // FP32 -> FP64 conversions): new pointers need a new capture
  if (P.gexec) {
    H2_HIP(hipGraphExecDestroy(P.gexec));
    P.gexec = nullptr;
  }
  static const bool check = std::getenv("H2_CHECK_REBASE") != nullptr;
  if (P.desc.p && P.desc_base && !P.keep_protos) {
    if (P.desc_base == ws_base(P)) return;  // the new arena is where the old one was
    std::vector<char> blob(P.desc_size);
    H2_HIP(hipMemcpy(blob.data(), P.desc.p, blob.size(), hipMemcpyDeviceToHost));
    rebase_blob(P, blob, P.desc_base, ws_base(P), P.ws_bytes);
    H2_HIP(hipMemcpy(P.desc.p, blob.data(), blob.size(), hipMemcpyHostToDevice));
    P.desc_base = ws_base(P);
    return;
  }
  if (check && P.desc.p && P.desc_base && P.keep_protos && !P.own_protos) {
    // diagnostic: a rebase of the uploaded descriptors equals a fresh build
    std::vector<char> blob(P.desc_size);
    H2_HIP(hipMemcpy(blob.data(), P.desc.p, blob.size(), hipMemcpyDeviceToHost));
    rebase_blob(P, blob, P.desc_base, ws_base(P), P.ws_bytes);
    const std::vector<char> fresh = build_blob(P, P.eps_set);
    if (fresh.size() != blob.size() || std::memcmp(fresh.data(), blob.data(), blob.size()) != 0) {
      size_t at = 0;
      while (at < std::min(fresh.size(), blob.size()) && fresh[at] == blob[at]) ++at;
      int sk = -1, kind = -1;
      size_t rel = 0;
      for (size_t i = 0; i < P.steps.size(); ++i)
        if (P.steps[i].desc_off <= at && (sk < 0 || P.steps[i].desc_off >= P.steps[sk].desc_off)) sk = (int)i;
      if (sk >= 0) {
        kind = (int)P.steps[sk].kind;
        rel = at - P.steps[sk].desc_off;
      }
      char msg[200];
      std::snprintf(msg, sizeof msg,
                    "descriptor rebase differs from a fresh build: byte %zu of %zu/%zu, step %d (kind %d) +%zu", at,
                    blob.size(), fresh.size(), sk, kind, rel);
      throw Error(H2_ERR_DEVICE, msg);
    }
    std::fprintf(stderr, "[h2 plan] rebase of %.3f GB of descriptors checked\n", blob.size() * 1e-9);
  }
  std::vector<char> blob = build_blob(P, eps);
  if (std::getenv("H2_TRACE")) {
    size_t proto = 0;
    for (const auto& st : P.steps)
      proto += st.itd.capacity() * sizeof(st.itd[0]) + st.tkd.capacity() * sizeof(st.tkd[0]) +
               st.itf.capacity() * sizeof(st.itf[0]) + st.tkf.capacity() * sizeof(st.tkf[0]) +
               st.qr.capacity() * sizeof(st.qr[0]) + st.svd.capacity() * sizeof(st.svd[0]) +
               st.chol.capacity() * sizeof(st.chol[0]) + st.refmat.capacity() * sizeof(st.refmat[0]);
    std::fprintf(stderr, "[h2 plan] descriptors %.3f GB on the device, step protos %.3f GB on the host\n",
                 blob.size() * 1e-9, proto * 1e-9);
  }
  if (P.desc.bytes < blob.size() || !P.desc.p) P.desc.alloc(std::max<size_t>(blob.size(), 64));
  H2_HIP(hipMemcpy(P.desc.p, blob.data(), blob.size(), hipMemcpyHostToDevice));
  P.desc_size = blob.size();
  P.desc_base = ws_base(P);
  P.eps_set = eps;
  drop_protos(P);
}

static void drop_protos(Plan& P) {
  // Plans that rebuild their descriptors on every use keep the protos;
  // product plans rebase theirs when the workspace moves and keep only the
  // protos that tolerance changes and the counting call read (SVD, REF,
  // QR).  H2_CHECK_REBASE keeps them all, to check every rebase.
  static const bool check = std::getenv("H2_CHECK_REBASE") != nullptr;
  if (P.own_protos || check) return;
  P.keep_protos = false;
  for (auto& st : P.steps) {
    std::vector<PItem<double>>().swap(st.itd);
    std::vector<PTask<double>>().swap(st.tkd);
    std::vector<PItem<float>>().swap(st.itf);
    std::vector<PTask<float>>().swap(st.tkf);
    std::vector<PChol>().swap(st.chol);
    std::vector<PFill>().swap(st.fill);
  }
}

// A plan with workspaces of its own (matrix-vector products, recompression).
static void finalize(Plan& P, double eps) {
  layout(P);
  P.bufd.alloc(P.ws_bytes);
  set_base(P, P.bufd.as<char>());
  emit(P, eps);
}

// Frees the arenas of the lanes other than `keep` that have no jobs in
// flight (their plans are re-emitted at their next use).
static void release_idle_arenas(Context* ctx, const LaneRes* keep) {
  for (auto& o : ctx->lanes)
    if (o.get() != keep && o->inflight == 0 && o->arena.p) {
      for (hipStream_t s : {o->l.stream, o->l.aux[0], o->l.aux[1]}) H2_HIP(hipStreamSynchronize(s));
      o->arena.release();
      o->epoch = 0;
    }
}

// A product plan bound to a lane: its workspaces are the lane's arena, grown
// to the plan's size if needed (after the lane's work has finished; the
// plans bound to it before are re-emitted at their next use). Only a plan
// without jobs in flight changes lanes.
static void bind(Context* ctx, Plan& P, int lane, double eps) {
  LaneRes& LR = *ctx->lanes[lane];
  if (LR.arena.bytes < P.ws_bytes) {
    for (hipStream_t s : {LR.l.stream, LR.l.aux[0], LR.l.aux[1]}) H2_HIP(hipStreamSynchronize(s));
    LR.arena.release();
    LR.epoch = 0;
    try {
      LR.arena.alloc(P.ws_bytes);
    } catch (const Error& e) {
      if (e.code != H2_ERR_OUT_OF_MEMORY) throw;
      release_idle_arenas(ctx, &LR);
      LR.arena.alloc(P.ws_bytes);
    }
    LR.epoch = ++ctx->arena_epoch;
  }
  {
    // the plan's descriptors and the result are allocated outside the arena:
    // with less than a tenth of the device free, idle arenas make room
    size_t freeb = 0, total = 0;
    H2_HIP(hipMemGetInfo(&freeb, &total));
    if (freeb < total / 10) release_idle_arenas(ctx, &LR);
  }
  if (P.bound_lane != lane || P.bound_epoch != LR.epoch || LR.epoch == 0 || !P.desc.p) {
    if (P.bound_lane != lane) {
      if (P.bound_lane >= 0 && P.bound_lane < (int)ctx->lanes.size()) --ctx->lanes[P.bound_lane]->nplans;
      ++LR.nplans;
    }
    set_base(P, LR.arena.as<char>());
    P.bound_lane = lane;
    P.bound_epoch = LR.epoch;
    emit(P, eps);
  }
}

// Resolved tolerance settings of a product: error budgets (fractions of eps
// for coarsening, rows, columns) and the Jacobi sweep cap.
struct Tol {
  double budget[3];
  int sweeps;
};

static Tol resolve_tol(const h2_mul_options& opt) {
  Tol t;
  const double b[3] = {opt.budget_coarse, opt.budget_row, opt.budget_col};
  double sum = 0.0;
  for (int i = 0; i < 3; ++i) {
    if (!std::isfinite(b[i]) || b[i] < 0.0) throw Error(H2_ERR_INVALID_ARG, "error budgets must be finite and >= 0");
    t.budget[i] = b[i] > 0.0 ? b[i] : 0.25;
    sum += t.budget[i];
  }
  if (sum > 1.0 + 1e-12) throw Error(H2_ERR_INVALID_ARG, "error budgets sum above 1");
  if (opt.jacobi_sweeps < 0) throw Error(H2_ERR_INVALID_ARG, "jacobi_sweeps below 0");
  if (!std::isfinite(opt.theta) || opt.theta < 0.0) throw Error(H2_ERR_INVALID_ARG, "theta must be finite and >= 0");
  t.sweeps = opt.jacobi_sweeps > 0 ? opt.jacobi_sweeps : 40;
  return t;
}

static bool tol_differs(const Plan& P, double eps, const Tol& t) {
  return P.eps_set != eps || P.sweeps != t.sweeps || P.budget[0] != t.budget[0] || P.budget[1] != t.budget[1] ||
         P.budget[2] != t.budget[2];
}

// Patches the descriptors that depend on eps, the budgets or the sweep cap
// (SVD thresholds, block-norm scales) in place on the device.
static void set_tolerances(Plan& P, double eps, const Tol& t) {
  if (!tol_differs(P, eps, t)) return;
  for (int i = 0; i < 3; ++i) P.budget[i] = t.budget[i];
  P.sweeps = t.sweeps;
  // (no host copy of the descriptors is kept: the SVD tasks are rebuilt from
  // the step's protos, the block-norm matrices read back from the device)
  for (auto& st : P.steps)
    if (st.kind == SK_SVD) {
      const std::vector<h2k::SvdTask> v = svd_tasks(P, st, eps);
      H2_HIP(hipMemcpy((char*)P.desc.p + st.desc_off, v.data(), v.size() * sizeof(h2k::SvdTask),
                       hipMemcpyHostToDevice));
    } else if (st.kind == SK_REF) {
      bool any = false;
      for (const auto& rm : st.refmat) any |= rm.approx;
      if (!any) continue;
      std::vector<h2k::RefMat> mats(st.refmat.size());
      H2_HIP(hipMemcpy(mats.data(), (char*)P.desc.p + st.desc2_off, mats.size() * sizeof(h2k::RefMat),
                       hipMemcpyDeviceToHost));
      for (size_t i = 0; i < st.refmat.size(); ++i)
        if (st.refmat[i].approx) mats[i].scale = ref_scale(P, st.refmat[i], eps);
      H2_HIP(hipMemcpy((char*)P.desc.p + st.desc2_off, mats.data(), mats.size() * sizeof(h2k::RefMat),
                       hipMemcpyHostToDevice));
    }
  P.eps_set = eps;
}

// Overflow word of a finished product -> error.
static void check_overflow_bits(int ovf) {
  if (ovf & h2k::kOvfNotConverged)
    throw Error(H2_ERR_NOT_CONVERGED, "a Jacobi SVD still rotated after its sweep cap (raise jacobi_sweeps)");
}

// Algorithmic flops of a Householder QR (R only) of an m x w matrix.
static double qr_flops(double m, double w) {
  return m >= w ? 2.0 * m * w * w - 2.0 / 3.0 * w * w * w : 2.0 * w * m * m - 2.0 / 3.0 * m * m * m;
}

// timing: 0 none, 1 per-phase events, 2 also events around every kernel launch,
// 3 also the algorithmic work from the sizes the QR / SVD kernels report.
static void execute(Context* ctx, const Lane& L, Plan& P, int timing, double* t_phase, char* desc_base = nullptr) {
  (void)ctx;
  // the launch check below must see only this execution's launches
  (void)hipGetLastError();
  hipStream_t s = L.stream;
  char* base = desc_base ? desc_base : (char*)P.desc.p;
  std::vector<hipEvent_t> ev;
  int cur_phase = -1;
  std::vector<int> phase_mark;  // event index -> phase
  int nev = 0;
  auto mark = [&](int ph) {
    if (!timing) return;
    if (nev == (int)ev.size()) {  // chunked plans change phase more often
      ev.emplace_back();
      H2_HIP(hipEventCreate(&ev.back()));
    }
    H2_HIP(hipEventRecord(ev[nev], s));
    phase_mark.push_back(ph);
    ++nev;
  };
  P.launches = 0;
  for (int i = 0; i < h2k::K_COUNT; ++i) {
    P.t_k[i] = P.units_k[i] = P.flops_k[i] = P.bytes_k[i] = 0;
    P.launches_k[i] = 0;
  }
  const bool per_kernel = timing >= 2;
  struct KEv {
    int kid;
    size_t step;
    hipEvent_t a, b;
  };
  std::vector<KEv> kev;
  auto timed_on = [&](hipStream_t on, int kid, size_t step, auto&& launch) {
    ++P.launches;
    ++P.launches_k[kid];
    if (!per_kernel) {
      launch();
      return;
    }
    KEv e{kid, step, nullptr, nullptr};
    H2_HIP(hipEventCreate(&e.a));
    H2_HIP(hipEventCreate(&e.b));
    H2_HIP(hipEventRecord(e.a, on));
    launch();
    H2_HIP(hipEventRecord(e.b, on));
    kev.push_back(e);
  };
  auto timed = [&](int kid, size_t step, auto&& launch) { timed_on(s, kid, step, launch); };
  // The size classes of a QR or SVD step are independent launches over the
  // same tasks (each workgroup exits unless its task's device-side width is
  // in the class): class c > 0 runs on aux stream c - 1, forked from and
  // joined back into the main stream.
  auto classes = [&](int ncls, auto&& launch_class) {
    if (ncls > 1) {
      H2_HIP(hipEventRecord(L.fork, s));
      for (int c = 1; c < ncls; ++c) H2_HIP(hipStreamWaitEvent(L.aux[c - 1], L.fork, 0));
    }
    for (int c = 0; c < ncls; ++c) launch_class(c, c == 0 ? s : L.aux[c - 1]);
    for (int c = 1; c < ncls; ++c) {
      H2_HIP(hipEventRecord(L.join[c - 1], L.aux[c - 1]));
      H2_HIP(hipStreamWaitEvent(s, L.join[c - 1], 0));
    }
  };
  size_t si = 0;
  for (auto& st : P.steps) {
    if (st.phase != cur_phase) {
      mark(st.phase);
      cur_phase = st.phase;
    }
    switch (st.kind) {
      case SK_GEMM_D:
        if (st.ntiles > 0)
          timed(h2k::K_GEMM_F64, si, [&] {
            h2k::launch_gemm_f64((const GemmItem<double>*)(base + st.desc_off),
                                 (const GemmTask<double>*)(base + st.desc2_off), (const GemmTile*)(base + st.tiles_off),
                                 st.ntiles, s);
          });
        break;
      case SK_GEMM_F:
        if (st.ntiles > 0)
          timed(h2k::K_GEMM_F32, si, [&] {
            h2k::launch_gemm_f32((const GemmItem<float>*)(base + st.desc_off),
                                 (const GemmTask<float>*)(base + st.desc2_off), (const GemmTile*)(base + st.tiles_off),
                                 st.ntiles, s);
          });
        break;
      case SK_QR:
        if (st.ndesc > 0)
          classes(h2k::size_classes(st.wmax), [&](int c, hipStream_t on) {
            timed_on(on, h2k::K_QR32 + c, si,
                     [&] { h2k::launch_qr_class((const h2k::QrTask*)(base + st.desc_off), st.ndesc, c, on); });
          });
        break;
      case SK_SVD:
        if (st.ndesc > 0)
          classes(h2k::size_classes(st.wmax), [&](int c, hipStream_t on) {
            timed_on(on, h2k::K_SVD32 + c, si, [&] {
              h2k::launch_svd_class((const h2k::SvdTask*)(base + st.desc_off), st.ndesc, c, L.overflow, on);
            });
          });
        break;
      case SK_CHOL:
        if (st.ndesc > 0)
          timed(h2k::K_CHOL, si,
                [&] { h2k::launch_chol((const h2k::CholTask*)(base + st.desc_off), st.ndesc, st.wmax, s); });
        break;
      case SK_FILL:
        if (st.ndesc > 0)
          timed(h2k::K_FILL, si, [&] { h2k::launch_fill((const h2k::FillTask*)(base + st.desc_off), st.ndesc, s); });
        break;
      case SK_CVT_F2D:
        if (st.cvt_n > 0)
          timed(h2k::K_CVT, si,
                [&] { h2k::launch_convert_f32_to_f64(res(st.cvt_in, P), res(st.cvt_out, P), st.cvt_n, s); });
        break;
      case SK_SCAN:
        if (st.ndesc > 0)
          timed(h2k::K_SCAN, si, [&] {
            h2k::launch_scan((const h2k::ScanTask*)(base + st.desc_off), (const int* const*)(base + st.desc2_off),
                             st.ndesc, s);
          });
        break;
      case SK_REF:
        if (st.ndesc > 0)
          timed(h2k::K_REF, si, [&] {
            h2k::launch_ref((const h2k::RefTask*)(base + st.desc_off), (const h2k::RefMat*)(base + st.desc2_off),
                            st.ndesc, s);
          });
        break;
    }
    H2_HIP(hipGetLastError());
    ++si;
  }
  mark(99);
  if (per_kernel) {
    if (!kev.empty()) H2_HIP(hipEventSynchronize(kev.back().b));
    std::vector<double> step_ms(P.steps.size(), 0.0);
    static const char* trace = std::getenv("H2_TRACE");
    for (auto& e : kev) {
      float ms = 0;
      H2_HIP(hipEventElapsedTime(&ms, e.a, e.b));
      P.t_k[e.kid] += ms;
      step_ms[e.step] += ms;
      if (trace && ms > 0.5)
        std::fprintf(stderr, "[h2 launch] step %3zu phase %d %-24s %8.3f ms\n", e.step, P.steps[e.step].phase,
                     h2k::kernel_name(e.kid), ms);
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    if (trace) {
      static const char* kname[] = {"gemm64", "gemm32", "qr", "svd", "chol", "fill", "cvt", "ref", "scan"};
      for (size_t i = 0; i < P.steps.size(); ++i) {
        const Step& st = P.steps[i];
        std::fprintf(stderr,
                     "[h2 step %3zu] phase %d %-6s tasks %7d tiles %8d wmax %4d  %9.3f ms  %.3g GF %.3g GB  tile GF %.3g\n",
                     i, st.phase, kname[(int)st.kind], st.ndesc, st.ntiles, st.wmax, step_ms[i], st.flops * 1e-9,
                     st.bytes * 1e-9, st.flops_tile * 1e-9);
      }
    }
  }
  if (timing >= 3) {
    // algorithmic work: QR / SVD from the sizes the kernels reported, the
    // other kernels from the planned sizes
    H2_HIP(hipStreamSynchronize(s));
    std::vector<int> stat;
    double svs[3][5] = {{0}};
    double qrs[3][4] = {{0}};  // per QR class: tasks, sum m, sum w, max m
    size_t stepno = 0;
    for (auto& st : P.steps) {
      ++stepno;
      const int kind = (int)st.kind;
      if (kind == SK_QR || kind == SK_SVD) {
        const int per = kind == SK_QR ? 2 : 4;
        const size_t n = kind == SK_QR ? st.qr.size() : st.svd.size();
        stat.resize(per * n);
        if (n)
          H2_HIP(hipMemcpy(stat.data(), P.wi + st.stat_off, per * n * sizeof(int),
                           hipMemcpyDeviceToHost));
        if (kind == SK_SVD && n && std::getenv("H2_TRACE")) {  // per-step shape summary
          double sm[4] = {0, 0, 0, 0};
          int mx[4] = {0, 0, 0, 0};
          for (size_t i = 0; i < n; ++i) {
            for (int c = 0; c < 4; ++c) {
              sm[c] += stat[4 * i + c];
              mx[c] = std::max(mx[c], stat[4 * i + c]);
            }
          }
          std::fprintf(stderr,
                       "[h2 svd step %3zu] tasks %zu  mean/max rows %.1f/%d cols %.1f/%d jacobi cols %.1f/%d "
                       "sweeps %.2f/%d\n",
                       stepno - 1, n, sm[0] / n, mx[0], sm[1] / n, mx[1], sm[2] / n, mx[2], sm[3] / n, mx[3]);
        }
        for (size_t i = 0; i < n; ++i) {
          if (kind == SK_QR) {
            const double m = stat[2 * i], w = stat[2 * i + 1];
            if (w <= 0) continue;
            const int kid = h2k::K_QR32 + (w > 64 ? 2 : (w > 32 ? 1 : 0));
            double* q = qrs[kid - h2k::K_QR32];
            q[0] += 1;
            q[1] += m;
            q[2] += w;
            q[3] = std::max(q[3], m);
            P.units_k[kid] += 1;
            P.flops_k[kid] += qr_flops(m, w);
            P.bytes_k[kid] += 8.0 * (m * w + (double)st.qr[i].w * st.qr[i].w);
          } else {
            const double rows = stat[4 * i], cols = stat[4 * i + 1], r = stat[4 * i + 2], sw = stat[4 * i + 3];
            const double wc = std::max(rows, cols);
            if (wc <= 0) continue;
            const int kid = h2k::K_SVD32 + (wc > 64 ? 2 : (wc > 32 ? 1 : 0));
            double fl = 0;
            if (P.qrcp)  // pivoted QR of the cols x rows transpose, stopped after r steps
              for (int j = 0; j < (int)r; ++j) fl += 4.0 * (rows - j) * (cols - j);
            fl += sw * r * (r - 1) / 2.0 * 12.0 * rows;  // Jacobi: 3 dots and a rotation per pair
            if (std::getenv("H2_TRACE")) {
              svs[kid - h2k::K_SVD32][0] += 1;
              svs[kid - h2k::K_SVD32][1] += rows;
              svs[kid - h2k::K_SVD32][2] += cols;
              svs[kid - h2k::K_SVD32][3] += r;
              svs[kid - h2k::K_SVD32][4] += sw;
            }
            P.units_k[kid] += 1;
            P.flops_k[kid] += fl;
            P.bytes_k[kid] += 8.0 * (rows * cols + rows * st.svd[i].kcap + cols);
          }
        }
      } else if ((kind == SK_GEMM_D || kind == SK_GEMM_F) && st.stat_off >= 0 && st.ndesc > 0) {
        // GEMM: the device-side sizes each task reported (m, n and the sum
        // of its product items' inner dimensions), each operand read once and
        // the output written once (read too with beta); beta and the copy
        // count from the task descriptors on the device
        const int kid = kind == SK_GEMM_D ? h2k::K_GEMM_F64 : h2k::K_GEMM_F32;
        const double w = kind == SK_GEMM_D ? 8.0 : 4.0;
        const size_t n = st.ndesc;
        stat.resize(3 * n);
        H2_HIP(hipMemcpy(stat.data(), P.wi + st.stat_off, 3 * n * sizeof(int), hipMemcpyDeviceToHost));
        std::vector<int> beta_copy(2 * n);
        {
          const size_t tsz = kind == SK_GEMM_D ? sizeof(h2k::GemmTask<double>) : sizeof(h2k::GemmTask<float>);
          std::vector<char> tb(n * tsz);
          H2_HIP(hipMemcpy(tb.data(), base + st.desc2_off, tb.size(), hipMemcpyDeviceToHost));
          for (size_t i = 0; i < n; ++i) {
            if (kind == SK_GEMM_D) {
              const auto& t = reinterpret_cast<const h2k::GemmTask<double>*>(tb.data())[i];
              beta_copy[2 * i] = t.beta;
              beta_copy[2 * i + 1] = t.ncopy;
            } else {
              const auto& t = reinterpret_cast<const h2k::GemmTask<float>*>(tb.data())[i];
              beta_copy[2 * i] = t.beta;
              beta_copy[2 * i + 1] = t.ncopy;
            }
          }
        }
        for (size_t i = 0; i < n; ++i) {
          const int beta = beta_copy[2 * i], ncopy = beta_copy[2 * i + 1];
          const double m = std::max(stat[3 * i], 0), nn = std::max(stat[3 * i + 1], 0), ks = stat[3 * i + 2];
          P.units_k[kid] += 1;
          P.flops_k[kid] += 2.0 * m * nn * ks;
          P.bytes_k[kid] += w * (m * ks + ks * nn + m * nn * (1 + (beta ? 1 : 0) + ncopy));
        }
      } else {
        static const int kmap[] = {h2k::K_GEMM_F64, h2k::K_GEMM_F32, -1, -1, h2k::K_CHOL, h2k::K_FILL, h2k::K_CVT,
                                   h2k::K_REF, h2k::K_SCAN};
        const int kid = kmap[kind];
        P.units_k[kid] += kind == SK_CVT_F2D ? (st.cvt_n > 0) : st.ndesc;
        P.flops_k[kid] += st.flops;
        P.bytes_k[kid] += st.bytes;
      }
    }
    if (std::getenv("H2_TRACE"))
      for (int c = 0; c < 3; ++c)
        if (qrs[c][0] > 0)
          std::fprintf(stderr, "[h2 qr class %d] tasks %.0f  mean rows %.1f (max %.0f) cols %.1f\n", c, qrs[c][0],
                       qrs[c][1] / qrs[c][0], qrs[c][3], qrs[c][2] / qrs[c][0]);
    if (std::getenv("H2_TRACE"))
      for (int c = 0; c < 3; ++c)
        if (svs[c][0] > 0)
          std::fprintf(stderr, "[h2 svd class %d] tasks %.0f  mean rows %.1f cols %.1f revealed %.1f sweeps %.2f\n",
                       c, svs[c][0], svs[c][1] / svs[c][0], svs[c][2] / svs[c][0], svs[c][3] / svs[c][0],
                       svs[c][4] / svs[c][0]);
  }
  if (timing) {
    H2_HIP(hipEventSynchronize(ev[nev - 1]));
    for (int i = 0; i < 8; ++i) t_phase[i] = 0.0;
    for (int i = 0; i + 1 < nev; ++i) {
      float ms = 0;
      H2_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      int ph = phase_mark[i];
      if (ph >= 0 && ph < 7) t_phase[ph] += ms;
    }
    float tot = 0;
    H2_HIP(hipEventElapsedTime(&tot, ev[0], ev[nev - 1]));
    t_phase[7] = tot;
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
}

// ------------------------------------------------------------------ multiply
// Algorithmic flops and bytes of the QR, SVD, Cholesky, fill and conversion
// steps from their planned sizes (GEMM steps count theirs when emitted).
static void count_work(Plan& P) {
  // A QR task walks its matrix in chunks of rows with one barrier per column,
  // so its time grows with m * w, and a step's launch lasts until its longest
  // task ends.  Workgroups start in task order: the longest tasks of a step
  // go first, so that the last workgroups to start are short ones.
  for (auto& st : P.steps)
    if (st.kind == SK_QR)
      std::stable_sort(st.qr.begin(), st.qr.end(), [](const PQr& a, const PQr& b) {
        return (int64_t)a.m * a.w > (int64_t)b.m * b.w;
      });
  double fl = 0;
  for (auto& st : P.steps) {
    if (st.kind == SK_QR)
      for (auto& q : st.qr) {
        st.flops += 2.0 * q.m * q.w * q.w;
        st.bytes += 8.0 * ((double)q.m * q.w + (double)q.w * q.w);
      }
    if (st.kind == SK_SVD)
      for (auto& v : st.svd) {
        st.flops += 8.0 * 4.0 * v.rows * (double)v.cols * v.cols;  // about 8 sweeps of w^2/2 rotations
        st.bytes += 8.0 * ((double)v.rows * v.cols + (double)v.rows * v.kcap + v.cols);
      }
    if (st.kind == SK_CHOL)
      for (auto& c : st.chol) {
        st.flops += 2.0 * c.w * c.w * c.w;
        st.bytes += 8.0 * 3.0 * c.w * c.w;
      }
    if (st.kind == SK_FILL)
      for (auto& f : st.fill) st.bytes += 8.0 * f.m * f.n;
    if (st.kind == SK_CVT_F2D) st.bytes += 12.0 * st.cvt_n;
    fl += st.flops;
  }
  P.flops_alg = fl;
}

// Waits for the device work of asynchronous jobs still running on a plan, so
// that the plan's descriptors and workspace may be changed or reused.
static void quiesce(Context* ctx, Plan& P) {
  if (P.inflight <= 0 || P.lane < 0) return;
  const hipStream_t s = P.lane == 0 ? ctx->stream : ctx->lanes[P.lane]->l.stream;
  H2_HIP(hipStreamSynchronize(s));
}

static std::shared_ptr<Plan> make_plan_chunks(Context* ctx, Matrix* X, Matrix* Y, bool f32, int kc, int kcap,
                                              const h2_mul_options& opt, double eps, int nchunk) {
  auto P = std::make_shared<Plan>();
  P->f32 = f32;
  P->kc = kc;
  P->kappa_cap = kcap;
  int sigma_br = 2;
  for (auto& ch : X->rows->children) sigma_br = std::max<int>(sigma_br, (int)ch.size());
  for (auto& ch : Y->cols->children) sigma_br = std::max<int>(sigma_br, (int)ch.size());
  P->sigma_br = sigma_br;
  P->theta = opt.theta > 0 ? opt.theta : 1.0 / (2.0 * sigma_br);
  if (!(P->theta * sigma_br < 1.0)) throw Error(H2_ERR_INVALID_ARG, "theta must be below 1/sigma");
  {
    const Tol tol = resolve_tol(opt);
    for (int i = 0; i < 3; ++i) P->budget[i] = tol.budget[i];
    P->sweeps = tol.sweeps;
  }
  build_block_tree(P->cbt, *X->rows, *Y->cols, X->bt.eta);
  Planner pl(ctx, X, Y, *P, kc, kcap);
  Builder& B = pl.B;
  pl.build_union();
  pl.assign_chunks(nchunk);
  P->nchunk = pl.nchunk;
  // result arrays
  P->res_vleaf = B.wd(X->rows->n * kc);
  P->res_vtr = B.wd((int64_t)X->rows->ncl * kc * kc);
  P->res_wleaf = B.wd(Y->cols->n * kc);
  P->res_wtr = B.wd((int64_t)Y->cols->ncl * kc * kc);
  P->res_S = B.wd((int64_t)P->cbt.adm.size() * kc * kc);
  P->res_rank_row = B.wi(X->rows->ncl);
  P->res_rank_col = B.wi(Y->cols->ncl);
  const bool tr = std::getenv("H2_TRACE") != nullptr;
  const auto tp0 = std::chrono::steady_clock::now();
  auto ws = [&](const char* what) {
    if (tr)
      std::fprintf(stderr, "[h2 plan] after %-8s fp64 workspace %.3f GB, host %.0f ms\n", what, P->wsd * 8e-9,
                   std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count());
  };
  ws("union");
  if (f32) pl.phaseA<float>();  // exact product, leaf forms and coarsening, chunk by chunk
  else pl.phaseA<double>();
  ws("coarsen");
  pl.bases();
  ws("bases");
  pl.couplings();
  P->n_adm = P->cbt.adm.size();
  P->n_inadm = P->cbt.inadm.size();
  count_work(*P);
  // algorithmic bytes: operand storage read once, result written once, and every
  // intermediate array written once and read once
  const double w8 = 8.0;
  double opbytes = 0;
  for (Matrix* M : {X, Y}) {
    opbytes += (double)(M->rows->n + M->cols->n) * M->kc * (f32 ? 4 : 8);
    opbytes += (double)(M->rows->ncl + M->cols->ncl) * M->kc * M->kc * (f32 ? 4 : 8);
    opbytes += (double)M->bt.adm.size() * M->kc * M->kc * (f32 ? 4 : 8) + (double)M->nsize * (f32 ? 4 : 8);
  }
  P->bytes_alg = opbytes + 2.0 * ((double)P->wsd * w8 + (double)P->wsf * 4.0);
  ws("counts");
  share_workspace(*P);
  ws("sharing");
  if (std::getenv("H2_TRACE"))
    std::fprintf(stderr, "[h2 plan] shared workspace: fp64 %.3f GB of %.3f GB, fp32 %.3f GB of %.3f GB\n",
                 P->wsd * 8e-9, P->wsd_planned * 8e-9, P->wsf * 4e-9, P->wsf_planned * 4e-9);
  layout(*P);
  P->keep_protos = true;  // descriptors are emitted when the plan is bound to a lane
  ws("final");
  return P;
}

// A plan whose workspace fits the device: one chunk first; while the
// shared workspace exceeds what the device can hold (free memory plus the
// lane arenas, which a plan's binding may replace, less a margin), the plan
// is rebuilt with four times as many chunks (opt.chunks > 0 fixes the count).
static std::shared_ptr<Plan> make_plan(Context* ctx, Matrix* X, Matrix* Y, bool f32, int kc, int kcap,
                                       const h2_mul_options& opt, double eps) {
  int nch = opt.chunks > 0 ? opt.chunks : 1;
  auto P = make_plan_chunks(ctx, X, Y, f32, kc, kcap, opt, eps, nch);
  if (opt.chunks > 0) return P;
  const size_t freeb = ctx->admissible_free();
  size_t held = 0;
  for (auto& l : ctx->lanes) held += l->arena.bytes;
  // room for the result, operands and allocator granularity: 15 % of the memory
  const size_t budget = (freeb + held) / 20 * 17;
  while (P->ws_bytes > budget && nch < 256 && P->nchunk == nch) {
    nch *= 4;
    if (std::getenv("H2_TRACE"))
      std::fprintf(stderr, "[h2 plan] workspace %.1f GB above the budget %.1f GB: %d chunks\n", P->ws_bytes * 1e-9,
                   budget * 1e-9, nch);
    P = make_plan_chunks(ctx, X, Y, f32, kc, kcap, opt, eps, nch);
  }
  return P;
}

// multiply() (the synchronous product) is submit + wait, defined with the
// asynchronous products below.

// ------------------------------------------------------------------ matrix-vector products
// y = M x for an H2-matrix (Section 2: O(nk) with the nested bases), as
// level-batched GEMM steps on nrhs vectors at once:
//   forward   x^_s = W_s^* x|_s      (leaves), x^_s = sum_c E_c^* x^_c (upwards)
//   couplings y^_t = sum_{(t,s) admissible} S_ts x^_s
//   backward  y^_c += E_c y^_parent (downwards), y|_t = V_t y^_t (leaves)
//   nearfield y|_t += N_ts x|_s      (inadmissible leaves)
// The adjoint swaps the roles of the two bases and transposes S and N.
// Vectors are held in tree order inside the plan's workspace.
struct MvPlan {
  std::shared_ptr<Plan> P;
  int64_t in_off = 0, out_off = 0;  // input / output vectors in the plan's FP64 workspace
  const Tree* tin = nullptr;
  const Tree* tout = nullptr;
  int64_t nrhs = 1;
  double* in() const { return P->wd + in_off; }
  double* out() const { return P->wd + out_off; }
};

// The plan's steps and workspace layout (host only: no device memory).
static std::shared_ptr<MvPlan> build_mv_host(Matrix* M, int trans, int64_t nrhs) {
  auto mv = std::make_shared<MvPlan>();
  mv->P = std::make_shared<Plan>();
  Plan& P = *mv->P;
  Builder B(P);
  const Tree& Ti = trans ? *M->rows : *M->cols;
  const Tree& To = trans ? *M->cols : *M->rows;
  const BasisDev& Bi = trans ? M->V : M->W;
  const BasisDev& Bo = trans ? M->W : M->V;
  const int kc = M->kc, nr = (int)nrhs;
  mv->tin = &Ti;
  mv->tout = &To;
  mv->nrhs = nrhs;
  const DRef<double> X = B.wd(Ti.n * nrhs), Y = B.wd(To.n * nrhs);
  const DRef<double> xh = B.wd((int64_t)Ti.ncl * kc * nrhs), yh = B.wd((int64_t)To.ncl * kc * nrhs);
  mv->in_off = X.off;
  mv->out_off = Y.off;
  auto ext = [](const double* p) { return DRef<double>::external(const_cast<double*>(p)); };
  auto XH = [&](int s) { return xh + (int64_t)s * kc * nrhs; };
  auto YH = [&](int t) { return yh + (int64_t)t * kc * nrhs; };
  const auto& bt = M->bt;
  // forward transform
  {
    GW<double> g(B.step(SK_GEMM_D));
    for (int s = 0; s < Ti.ncl; ++s) {
      if (!Ti.leaf(s)) continue;
      g.task(XH(s), nr, kc, nr);
      g.mm(ext(Bi.leaf) + Ti.begin[s] * kc, kc, X + Ti.begin[s] * nrhs, nr, (int)Ti.size(s), h2k::IT_TRANS_A);
    }
  }
  for (int l = Ti.depth - 2; l >= 0; --l) {
    GW<double> g(B.step(SK_GEMM_D));
    for (int s = 0; s < Ti.ncl; ++s) {
      if (Ti.level[s] != l || Ti.leaf(s)) continue;
      g.task(XH(s), nr, kc, nr);
      for (int c : Ti.children[s]) g.mm(ext(Bi.transfer) + (int64_t)c * kc * kc, kc, XH(c), nr, kc, h2k::IT_TRANS_A);
    }
  }
  // couplings (every output cluster gets y^, zero without admissible blocks)
  {
    std::vector<std::vector<int>> of(To.ncl);
    for (size_t i = 0; i < bt.adm.size(); ++i) {
      const auto& nd = bt.nodes[bt.adm[i]];
      of[trans ? nd.s : nd.t].push_back((int)i);
    }
    GW<double> g(B.step(SK_GEMM_D));
    for (int t = 0; t < To.ncl; ++t) {
      g.task(YH(t), nr, kc, nr);
      for (int i : of[t]) {
        const auto& nd = bt.nodes[bt.adm[i]];
        g.mm(ext(M->S) + (int64_t)i * kc * kc, kc, XH(trans ? nd.t : nd.s), nr, kc, trans ? h2k::IT_TRANS_A : 0);
      }
    }
  }
  // backward transform
  for (int l = 1; l < To.depth; ++l) {
    GW<double> g(B.step(SK_GEMM_D));
    for (int c = 0; c < To.ncl; ++c) {
      if (To.level[c] != l) continue;
      g.task(YH(c), nr, kc, nr, 1);
      g.mm(ext(Bo.transfer) + (int64_t)c * kc * kc, kc, YH(To.parent[c]), nr, kc);
    }
  }
  // leaves and nearfield; nearfield blocks of a non-leaf output cluster
  // follow in one step per level (their rows overlap the leaves')
  std::vector<std::vector<int>> near(To.ncl);
  for (size_t i = 0; i < bt.inadm.size(); ++i) {
    const auto& nd = bt.nodes[bt.inadm[i]];
    near[trans ? nd.s : nd.t].push_back((int)i);
  }
  auto near_items = [&](GW<double>& g, int t) {
    for (int i : near[t]) {
      const auto& nd = bt.nodes[bt.inadm[i]];
      const int64_t m = M->rows->size(nd.t), n = M->cols->size(nd.s);
      if (!trans) g.mm(ext(M->N) + M->noff[i], (int)n, X + M->cols->begin[nd.s] * nrhs, nr, (int)n);
      else g.mm(ext(M->N) + M->noff[i], (int)n, X + M->rows->begin[nd.t] * nrhs, nr, (int)m, h2k::IT_TRANS_A);
    }
  };
  {
    GW<double> g(B.step(SK_GEMM_D));
    for (int t = 0; t < To.ncl; ++t) {
      if (!To.leaf(t)) continue;
      g.task(Y + To.begin[t] * nrhs, nr, (int)To.size(t), nr);
      g.mm(ext(Bo.leaf) + To.begin[t] * kc, kc, YH(t), nr, kc);
      near_items(g, t);
    }
  }
  for (int l = 0; l < To.depth; ++l) {
    bool any = false;
    for (int t = 0; t < To.ncl; ++t) any |= To.level[t] == l && !To.leaf(t) && !near[t].empty();
    if (!any) continue;
    GW<double> g(B.step(SK_GEMM_D));
    for (int t = 0; t < To.ncl; ++t) {
      if (To.level[t] != l || To.leaf(t) || near[t].empty()) continue;
      g.task(Y + To.begin[t] * nrhs, nr, (int)To.size(t), nr, 1);
      near_items(g, t);
    }
  }
  layout(P);
  return mv;
}

static std::shared_ptr<MvPlan> build_mv(Matrix* M, int trans, int64_t nrhs) {
  auto mv = build_mv_host(M, trans, nrhs);
  Plan& P = *mv->P;
  P.bufd.alloc(P.ws_bytes);
  set_base(P, P.bufd.as<char>());
  emit(P, 0.0);
  return mv;
}

static std::shared_ptr<MvPlan> get_mv(Matrix* M, int trans, int64_t nrhs) {
  Context* ctx = M->ctx;
  const auto key = std::make_tuple(M->id, trans, nrhs);
  auto it = ctx->mvplans.find(key);
  if (it != ctx->mvplans.end()) return it->second;
  auto mv = build_mv(M, trans, nrhs);
  ctx->mvplans[key] = mv;
  return mv;
}

void matvec(Matrix* M, int trans, int64_t nrhs, const double* x, double* y) {
  Context* ctx = M->ctx;
  hipStream_t s = ctx->stream;
  auto mv = get_mv(M, trans, nrhs);
  const Tree& Ti = *mv->tin;
  const Tree& To = *mv->tout;
  std::vector<double> xt((size_t)Ti.n * nrhs), yt((size_t)To.n * nrhs);
  for (int64_t i = 0; i < Ti.n; ++i) std::memcpy(&xt[i * nrhs], x + Ti.perm[i] * nrhs, nrhs * sizeof(double));
  H2_HIP(hipMemcpyAsync(mv->in(), xt.data(), xt.size() * sizeof(double), hipMemcpyHostToDevice, s));
  execute(ctx, ctx->lane0(), *mv->P, 0, nullptr);
  H2_HIP(hipMemcpyAsync(yt.data(), mv->out(), yt.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  H2_HIP(hipStreamSynchronize(s));
  for (int64_t i = 0; i < To.n; ++i) std::memcpy(y + To.perm[i] * nrhs, &yt[i * nrhs], nrhs * sizeof(double));
}

// y = M x with every device buffer of the call (vectors, coefficient
// vectors, launch descriptors) inside `scratch` (bytes long, 256-byte
// aligned): no device allocation.  The plan's host part is cached per
// (matrix, trans, nrhs); its descriptors are rebuilt against `scratch` and
// copied there on every call, since other calls may have overwritten it.
void matvec_scratch(Matrix* M, int trans, int64_t nrhs, const double* x, double* y, char* scratch, size_t bytes) {
  Context* ctx = M->ctx;
  hipStream_t s = ctx->stream;
  const auto key = std::make_tuple(M->id, trans, nrhs);
  std::shared_ptr<MvPlan> mv;
  auto it = ctx->mvhost.find(key);
  if (it != ctx->mvhost.end()) {
    mv = it->second;
  } else {
    mv = build_mv_host(M, trans, nrhs);
    mv->P->keep_protos = true;  // descriptors are rebuilt on every call
    mv->P->own_protos = true;
    ctx->mvhost[key] = mv;
  }
  Plan& P = *mv->P;
  const size_t desc_at = (P.ws_bytes + 255) & ~size_t(255);
  if (desc_at > bytes)
    throw Error(H2_ERR_TOO_LARGE, "matrix-vector product needs " + std::to_string(desc_at) +
                                      " bytes of scratch workspace, above the scratch size " + std::to_string(bytes));
  set_base(P, scratch);
  const std::vector<char> blob = build_blob(P, 0.0);
  if (desc_at + blob.size() > bytes)
    throw Error(H2_ERR_TOO_LARGE, "matrix-vector product needs " + std::to_string(desc_at + blob.size()) +
                                      " bytes of scratch (workspace and descriptors), above the scratch size " +
                                      std::to_string(bytes));
  const Tree& Ti = *mv->tin;
  const Tree& To = *mv->tout;
  std::vector<double> xt((size_t)Ti.n * nrhs), yt((size_t)To.n * nrhs);
  for (int64_t i = 0; i < Ti.n; ++i) std::memcpy(&xt[i * nrhs], x + Ti.perm[i] * nrhs, nrhs * sizeof(double));
  // blob and xt stay alive until the stream is synchronised below
  H2_HIP(hipMemcpyAsync(scratch + desc_at, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
  H2_HIP(hipMemcpyAsync(mv->in(), xt.data(), xt.size() * sizeof(double), hipMemcpyHostToDevice, s));
  execute(ctx, ctx->lane0(), P, 0, nullptr, scratch + desc_at);
  H2_HIP(hipMemcpyAsync(yt.data(), mv->out(), yt.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  H2_HIP(hipStreamSynchronize(s));
  for (int64_t i = 0; i < To.n; ++i) std::memcpy(y + To.perm[i] * nrhs, &yt[i * nrhs], nrhs * sizeof(double));
}

// Power iteration on E^* E (E = XY - C, or XY): z = z0 / ||z0||; each step
// w = E z, sigma = ||w|| (the Rayleigh estimate of the largest singular value
// for the unit vector z), z = E^* w / ||E^* w||.  The estimate after `iters`
// steps is the sigma of the last step.
void product_error(Matrix* X, Matrix* Y, Matrix* C, int iters, const double* z0, double* err, double* nxy) {
  Context* ctx = X->ctx;
  hipStream_t s = ctx->stream;
  auto same = [](const Tree& a, const Tree& b) { return &a == &b || (a.n == b.n && a.perm == b.perm); };
  if (!same(*X->cols, *Y->rows)) throw Error(H2_ERR_INCOMPATIBLE, "X columns and Y rows use different cluster trees");
  if (C && (!same(*C->rows, *X->rows) || !same(*C->cols, *Y->cols)))
    throw Error(H2_ERR_INCOMPATIBLE, "C does not have the row tree of X and the column tree of Y");
  auto pY = get_mv(Y, 0, 1), pX = get_mv(X, 0, 1), pXt = get_mv(X, 1, 1), pYt = get_mv(Y, 1, 1);
  std::shared_ptr<MvPlan> pC, pCt;
  if (C) {
    pC = get_mv(C, 0, 1);
    pCt = get_mv(C, 1, 1);
  }
  const Tree& Tc = *Y->cols;
  const int64_t nc = Tc.n, nr = X->rows->n, nm = Y->rows->n;
  DevBuf z, zs, part;
  z.alloc(nc * sizeof(double));
  zs.alloc(nc * sizeof(double));
  part.alloc(h2k::kDotBlocks * sizeof(double));
  {
    std::vector<double> zt(nc);
    for (int64_t i = 0; i < nc; ++i) zt[i] = z0[Tc.perm[i]];
    H2_HIP(hipMemcpy(zs.p, zt.data(), nc * sizeof(double), hipMemcpyHostToDevice));
  }
  auto dot = [&](const double* a, const double* b, int64_t n) {
    std::vector<double> ph(h2k::kDotBlocks);
    h2k::launch_dot(a, b, n, part.as<double>(), s);
    H2_HIP(hipMemcpyAsync(ph.data(), part.p, ph.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    H2_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : ph) t += v;
    return t;
  };
  auto copy = [&](double* dst, const double* src, int64_t n) {
    H2_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  };
  auto power = [&](bool withC) {
    copy(z.as<double>(), zs.as<double>(), nc);
    const double n0 = std::sqrt(dot(z.as<double>(), z.as<double>(), nc));
    if (n0 == 0.0) throw Error(H2_ERR_INVALID_ARG, "zero start vector");
    h2k::launch_axpby(z.as<double>(), z.as<double>(), nc, 0.0, 1.0 / n0, s);
    double sig = 0.0;
    for (int it = 0; it < iters; ++it) {
      // w = E z
      copy(pY->in(), z.as<double>(), nc);
      execute(ctx, ctx->lane0(), *pY->P, 0, nullptr);
      copy(pX->in(), pY->out(), nm);
      execute(ctx, ctx->lane0(), *pX->P, 0, nullptr);
      double* w = pX->out();
      if (withC) {
        copy(pC->in(), z.as<double>(), nc);
        execute(ctx, ctx->lane0(), *pC->P, 0, nullptr);
        h2k::launch_axpby(pC->out(), w, nr, -1.0, 1.0, s);
      }
      sig = std::sqrt(dot(w, w, nr));
      // z = E^* w / ||E^* w||
      copy(pXt->in(), w, nr);
      execute(ctx, ctx->lane0(), *pXt->P, 0, nullptr);
      copy(pYt->in(), pXt->out(), nm);
      execute(ctx, ctx->lane0(), *pYt->P, 0, nullptr);
      double* zt = pYt->out();
      if (withC) {
        copy(pCt->in(), w, nr);
        execute(ctx, ctx->lane0(), *pCt->P, 0, nullptr);
        h2k::launch_axpby(pCt->out(), zt, nc, -1.0, 1.0, s);
      }
      const double nz = std::sqrt(dot(zt, zt, nc));
      if (nz == 0.0) break;
      h2k::launch_axpby(zt, z.as<double>(), nc, 1.0 / nz, 0.0, s);
    }
    return sig;
  };
  *err = C ? power(true) : 0.0;
  *nxy = power(false);
  H2_HIP(hipStreamSynchronize(s));
}

}  // namespace h2

// ------------------------------------------------------------------ H -> H2 recompression
// An H-matrix given on the block tree of (R, Cc, eta) by factors G_b = U_b Z_b^*
// of its admissible leaves and dense nearfield blocks is turned into an
// H2-matrix with adaptive row and column bases (Section 5: the truncation of
// each block to its Frobenius tail, then the weighted bases and the couplings
// of Sections 5.2 and 5.3). The plan is built per call: the factors are
// uploaded into workspace regions that stay live from the first step on.
namespace h2 {
std::unique_ptr<Matrix> recompress(Context* ctx, std::shared_ptr<Tree> R, std::shared_ptr<Tree> Cc, double eta,
                                   const int* ranks, const double* U, const double* Z, const double* near,
                                   double eps, const h2_mul_options& opt, h2_mul_stats* stats) {
  if (!(eps > 0.0 && eps < 1.0) || !std::isfinite(eps)) throw Error(H2_ERR_INVALID_ARG, "eps must be in (0,1)");
  if (!(eta > 0.0) || !std::isfinite(eta)) throw Error(H2_ERR_INVALID_ARG, "eta must be positive");
  if (R->dim != Cc->dim) throw Error(H2_ERR_INCOMPATIBLE, "row and column trees of different dimension");
  const int kc = opt.max_rank > 0 ? opt.max_rank : 64;
  const int kcap = opt.coarse_rank > 0 ? opt.coarse_rank : 64;
  if (kc > 64 || kcap > 64 || kc < 1 || kcap < 1) throw Error(H2_ERR_INVALID_ARG, "rank caps out of range");
  auto t0 = std::chrono::steady_clock::now();
  auto P = std::make_shared<Plan>();
  P->kc = kc;
  P->kappa_cap = kcap;
  int sigma_br = 2;
  for (auto& ch : R->children) sigma_br = std::max<int>(sigma_br, (int)ch.size());
  for (auto& ch : Cc->children) sigma_br = std::max<int>(sigma_br, (int)ch.size());
  P->sigma_br = sigma_br;
  P->theta = opt.theta > 0 ? opt.theta : 1.0 / (2.0 * sigma_br);
  if (!(P->theta * sigma_br < 1.0)) throw Error(H2_ERR_INVALID_ARG, "theta must be below 1/sigma");
  {
    const Tol tol = resolve_tol(opt);
    for (int i = 0; i < 3; ++i) P->budget[i] = tol.budget[i];
    P->sweeps = tol.sweeps;
  }
  build_block_tree(P->cbt, *R, *Cc, eta);
  const BlockTree& bt = P->cbt;
  Planner pl(ctx, *R, *Cc, *P, kc, kcap);
  Builder& B = pl.B;
  P->res_vleaf = B.wd(R->n * kc);
  P->res_vtr = B.wd((int64_t)R->ncl * kc * kc);
  P->res_wleaf = B.wd(Cc->n * kc);
  P->res_wtr = B.wd((int64_t)Cc->ncl * kc * kc);
  P->res_S = B.wd((int64_t)bt.adm.size() * kc * kc);
  P->res_rank_row = B.wi(R->ncl);
  P->res_rank_col = B.wi(Cc->ncl);
  // factors of the admissible leaves, packed in leaf order
  int64_t nu = 0, nz = 0;
  for (size_t li = 0; li < bt.adm.size(); ++li) {
    const int k = ranks[li];
    if (k < 1 || k > 128) throw Error(H2_ERR_INVALID_ARG, "block rank outside [1, 128]");
    nu += R->size(bt.nodes[bt.adm[li]].t) * k;
    nz += Cc->size(bt.nodes[bt.adm[li]].s) * k;
  }
  const DRef<double> inU = B.wd(nu), inZ = B.wd(nz);
  pl.un.assign(bt.adm.size(), UNode());
  pl.bnode.resize(bt.adm.size());
  int64_t uo = 0, zo = 0;
  for (size_t li = 0; li < bt.adm.size(); ++li) {
    const auto& nd = bt.nodes[bt.adm[li]];
    UNode& u = pl.un[li];
    u.t = nd.t;
    u.r = nd.s;
    u.fin = true;
    u.form = 1;
    u.below = bt.adm[li];
    u.K = ranks[li];
    u.m = (int)R->size(nd.t);
    u.n = (int)Cc->size(nd.s);
    u.U = inU.off + uo;
    u.Z = inZ.off + zo;
    uo += (int64_t)u.m * u.K;
    zo += (int64_t)u.n * u.K;
    pl.bnode[li] = (int)li;
  }
  // nearfield: copied into the result as given
  P->cnoff.assign(bt.inadm.size() + 1, 0);
  int64_t noff = 0;
  for (size_t i = 0; i < bt.inadm.size(); ++i) {
    P->cnoff[i] = noff;
    noff += R->size(bt.nodes[bt.inadm[i]].t) * Cc->size(bt.nodes[bt.inadm[i]].s);
  }
  P->cnoff[bt.inadm.size()] = noff;
  P->cnsize = noff;
  P->res_N = B.wd(noff);
  P->inputs = {inU, inZ, P->res_N};
  pl.coarsen();
  pl.bases();
  pl.couplings();
  P->n_adm = bt.adm.size();
  P->n_inadm = bt.inadm.size();
  count_work(*P);
  P->bytes_alg = 8.0 * (double)(nu + nz + noff) + 2.0 * (double)P->wsd * 8.0;
  share_workspace(*P);
  finalize(*P, eps);
  set_tolerances(*P, eps, resolve_tol(opt));
  const double tplan = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  const std::pair<const double*, int64_t> host_in[3] = {{U, nu}, {Z, nz}, {near, noff}};
  for (int i = 0; i < 3; ++i)
    if (host_in[i].second)
      H2_HIP(hipMemcpyAsync(res(P->inputs[i], *P), host_in[i].first, host_in[i].second * sizeof(double),
                            hipMemcpyHostToDevice, ctx->stream));
  H2_HIP(hipMemsetAsync(ctx->overflow, 0, sizeof(int), ctx->stream));
  double tph[8] = {0};
  execute(ctx, ctx->lane0(), *P, opt.timing, tph);
  int ovf = 0;
  H2_HIP(hipMemcpyAsync(&ovf, ctx->overflow, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  H2_HIP(hipStreamSynchronize(ctx->stream));
  check_overflow_bits(ovf);
  if (ovf)
    throw Error(H2_ERR_TOO_LARGE, (ovf & 1) ? "truncated block rank above coarse_rank cap"
                                             : "basis rank above max_rank cap");
  auto Cm = std::make_unique<Matrix>();
  Cm->ctx = ctx;
  Cm->hold = ctx->self.lock();
  Cm->id = ctx->next_id++;
  Cm->rows = R;
  Cm->cols = Cc;
  build_block_tree(Cm->bt, *R, *Cc, eta);
  Cm->kc = kc;
  Cm->w_is_v = false;
  const int64_t n_vleaf = R->n * kc, n_vtr = (int64_t)R->ncl * kc * kc, n_wleaf = Cc->n * kc,
                n_wtr = (int64_t)Cc->ncl * kc * kc, n_s = (int64_t)bt.adm.size() * kc * kc;
  auto take = [&](int64_t c) { return Cm->alloc64((size_t)std::max<int64_t>(c, 1)); };
  Cm->V.leaf = take(n_vleaf);
  Cm->V.transfer = take(n_vtr);
  Cm->W.leaf = take(n_wleaf);
  Cm->W.transfer = take(n_wtr);
  Cm->S = take(n_s);
  Cm->N = take(noff);
  auto cp = [&](double* d, const DRef<double>& src, int64_t count) {
    if (count) H2_HIP(hipMemcpyAsync(d, res(src, *P), count * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  };
  cp(Cm->V.leaf, P->res_vleaf, n_vleaf);
  cp(Cm->V.transfer, P->res_vtr, n_vtr);
  cp(Cm->W.leaf, P->res_wleaf, n_wleaf);
  cp(Cm->W.transfer, P->res_wtr, n_wtr);
  cp(Cm->S, P->res_S, n_s);
  cp(Cm->N, P->res_N, noff);
  Cm->noff = P->cnoff;
  Cm->nsize = noff;
  Cm->rank_row.resize(R->ncl);
  Cm->rank_col.resize(Cc->ncl);
  H2_HIP(hipMemcpyAsync(Cm->rank_row.data(), res(P->res_rank_row, *P), R->ncl * sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  H2_HIP(hipMemcpyAsync(Cm->rank_col.data(), res(P->res_rank_col, *P), Cc->ncl * sizeof(int),
                        hipMemcpyDeviceToHost, ctx->stream));
  H2_HIP(hipStreamSynchronize(ctx->stream));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    for (int i = 0; i < 8; ++i) stats->t_phase[i] = tph[i];
    stats->t_plan_ms = tplan;
    stats->bytes_alg = P->bytes_alg;
    stats->flops_alg = P->flops_alg;
    stats->prec_used = H2_PREC_FP64;
    stats->rank_max_row = Cm->rank_row.empty() ? 0 : *std::max_element(Cm->rank_row.begin(), Cm->rank_row.end());
    stats->rank_max_col = Cm->rank_col.empty() ? 0 : *std::max_element(Cm->rank_col.begin(), Cm->rank_col.end());
    stats->coarse_rank_max = P->max_coarse_K;
    stats->n_adm = P->n_adm;
    stats->n_inadm = P->n_inadm;
    stats->launches = P->launches;
    for (int i = 0; i < h2k::K_COUNT; ++i) {
      stats->t_kernel[i] = P->t_k[i];
      stats->launches_kernel[i] = P->launches_k[i];
      stats->units_kernel[i] = P->units_k[i];
      stats->flops_kernel[i] = P->flops_k[i];
      stats->bytes_kernel[i] = P->bytes_k[i];
    }
  }
  return Cm;
}
}  // namespace h2

// ------------------------------------------------------------------ asynchronous products
// submit() plans (or reuses the cached plan), enqueues the product and the
// copies of its result arrays on a lane and returns; wait() completes it.
// Products on different lanes overlap on the device; jobs of one plan share
// its lane and run in order.
namespace h2 {
struct Job {
  Context* ctx = nullptr;
  Matrix* X = nullptr;
  Matrix* Y = nullptr;
  double eps = 0;
  h2_mul_options opt{};
  std::shared_ptr<Plan> P;
  std::pair<uint64_t, uint64_t> key;
  bool f32 = false, built = false;
  int kc = 0, lane = 0;
  int slot = -1;        // this job's overflow flag: a slot of the lane's flags
  int* flag = nullptr;
  double tplan = 0;
  double tph[8] = {0};
  hipEvent_t done = nullptr;
  std::unique_ptr<Matrix> C;
  int* dev_ranks = nullptr;  // row then column ranks, copied out of the plan
  bool finished = false;
  // gives the flag slot back and drops the in-flight counts (once)
  void release() {
    if (finished) return;
    finished = true;
    if (ctx && slot >= 0) {
      if (P) --P->inflight;
      LaneRes& LR = *ctx->lanes[lane];
      --LR.inflight;
      LR.free_slots.push_back(slot);
    }
  }
  ~Job() {
    release();
    if (done) (void)hipEventDestroy(done);
  }
};

// Device bytes of a product's result arrays (bases padded to kc columns,
// couplings, nearfield, ranks; allocated when the product is submitted).
static size_t result_bytes(const Matrix* X, const Matrix* Y, const Plan& P, int kc) {
  const int64_t n = X->rows->n * kc + (int64_t)X->rows->ncl * kc * kc + Y->cols->n * kc +
                    (int64_t)Y->cols->ncl * kc * kc + (int64_t)P.cbt.adm.size() * kc * kc + P.cnsize +
                    X->rows->ncl + Y->cols->ncl;
  return (size_t)(n + 7 * 32) * sizeof(double);
}

// Upper estimate of a plan's device descriptor bytes before they are built.
static size_t desc_estimate(const Plan& P) {
  size_t b = 0;
  for (const auto& st : P.steps) {
    b += st.itd.size() * sizeof(h2k::GemmItem<double>) + st.itf.size() * sizeof(h2k::GemmItem<float>);
    b += (st.tkd.size() + st.tkf.size()) * (sizeof(h2k::GemmTask<double>) + 16 * sizeof(h2k::GemmTile));
    b += (st.qr.size() * 2 + st.svd.size() + st.chol.size()) * 256 + st.refmat.size() * 64 + st.ref.size() * 64;
    b += 4096;
  }
  return b;
}

// Admission by predicted footprint: the memory a product still needs (a
// larger arena for its lane, its descriptors if not uploaded yet, its
// result) against what the device can give (free memory, the lane's own
// arena if it must be replaced, the arenas of idle lanes).  A product that
// cannot fit is refused before anything is allocated.
size_t Context::admissible_free() const {
  size_t freeb = 0, total = 0;
  H2_HIP(hipMemGetInfo(&freeb, &total));
  if (mem_limit == 0) return freeb;
  const size_t used = total - freeb;
  return used >= mem_limit ? 0 : std::min<size_t>(freeb, mem_limit - used);
}

static void admit(Context* ctx, const LaneRes& LR, const Plan& P, size_t res_bytes) {
  size_t need = res_bytes, give = 0;
  if (LR.arena.bytes < P.ws_bytes) {
    need += P.ws_bytes;
    give += LR.arena.bytes;
  }
  if (!P.desc.p) need += desc_estimate(P);
  give += ctx->admissible_free();
  for (auto& o : ctx->lanes)
    if (o.get() != &LR && o->inflight == 0) give += o->arena.bytes;
  // not enough: the least recently used cached plans without jobs go (their
  // descriptors are freed; such a plan is built again when its operands
  // are multiplied again), if dropping them all would make room
  auto idle = [&](const std::shared_ptr<Plan>& q) {
    return q.get() != &P && q->inflight == 0 && q.use_count() == 1;
  };
  if (need > give) {
    size_t evictable = 0;
    for (auto& kv : ctx->plans)
      if (idle(kv.second)) evictable += kv.second->desc.bytes;
    while (need > give && need <= give + evictable) {
      auto victim = ctx->plans.end();
      for (auto it = ctx->plans.begin(); it != ctx->plans.end(); ++it)
        if (idle(it->second) && (victim == ctx->plans.end() || it->second->last_use < victim->second->last_use))
          victim = it;
      if (victim == ctx->plans.end()) break;
      const size_t freed = victim->second->desc.bytes;
      Plan& V = *victim->second;
      if (V.bound_lane >= 0 && V.bound_lane < (int)ctx->lanes.size()) --ctx->lanes[V.bound_lane]->nplans;
      ctx->plans.erase(victim);
      give += freed;
      evictable -= freed;
    }
  }
  if (need > give) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "out of memory: the product needs about %.3f GB more device memory, %.3f GB can be freed now",
                  need * 1e-9, give * 1e-9);
    throw Error(H2_ERR_OUT_OF_MEMORY, msg);
  }
}

Job* submit(Context* ctx, Matrix* X, Matrix* Y, double eps, const h2_mul_options& opt) {
  if (X->cols.get() != Y->rows.get()) throw Error(H2_ERR_INCOMPATIBLE, "X's column tree is not Y's row tree");
  if (!(eps > 0.0 && eps < 1.0) || !std::isfinite(eps)) throw Error(H2_ERR_INVALID_ARG, "eps must be in (0,1)");
  if (X->kc > 64 || Y->kc > 64) throw Error(H2_ERR_TOO_LARGE, "operand rank above 64");
  const Tol tol = resolve_tol(opt);  // validates budgets, theta and the sweep cap
  if (ctx->lanes.empty()) ctx->set_lanes(4);
  auto J = std::make_unique<Job>();
  J->ctx = ctx;
  J->X = X;
  J->Y = Y;
  J->eps = eps;
  J->opt = opt;
  // FP32 bulk only where its rounding (about 1e-7 of a block's norm) stays well
  // below the truncation tolerances; tighter eps runs the bulk in FP64.
  bool f32 = opt.precision == H2_PREC_FP32_BULK && eps >= 1e-5;
  if (f32) {
    auto f = ctx->fp32_fail_eps.find({X->id, Y->id});
    if (f != ctx->fp32_fail_eps.end() && eps <= f->second) f32 = false;
  }
  const int kmax = std::max(X->kc, Y->kc);
  int kc = opt.max_rank > 0 ? opt.max_rank : std::min(64, std::max(32, (2 * kmax + 15) / 16 * 16));
  if (opt.max_rank == 0) {
    auto f = ctx->kc_raised.find({X->id, Y->id});
    if (f != ctx->kc_raised.end()) kc = std::max(kc, f->second);
  }
  const int kcap = opt.coarse_rank > 0 ? opt.coarse_rank : 64;
  if (kc > 64 || kcap > 64 || kc < 1 || kcap < 1) throw Error(H2_ERR_INVALID_ARG, "rank caps out of range");
  auto t0 = std::chrono::steady_clock::now();
  J->key = std::make_pair(X->id, Y->id * 4 + (f32 ? 1 : 0));
  auto it = ctx->plans.find(J->key);
  if (it != ctx->plans.end() && it->second->kc == kc && it->second->kappa_cap == kcap &&
      it->second->theta == (opt.theta > 0 ? opt.theta : it->second->theta) &&
      (opt.chunks <= 0 || it->second->nchunk == opt.chunks)) {
    J->P = it->second;
  } else {
    if (it != ctx->plans.end()) quiesce(ctx, *it->second);
    if (f32) {
      X->ensure_fp32(ctx->stream);
      Y->ensure_fp32(ctx->stream);
      H2_HIP(hipStreamSynchronize(ctx->stream));
    }
    J->P = make_plan(ctx, X, Y, f32, kc, kcap, opt, eps);
    ctx->plans[J->key] = J->P;
    J->built = true;
  }
  Plan& P = *J->P;
  // lane: the one the plan is bound to (moving re-emits all its
  // descriptors); a plan not bound yet goes to the lane with the fewest
  // plans bound to it, then the fewest jobs in flight
  int lane;
  if (P.inflight > 0 && P.lane >= 0) {
    lane = P.lane;
  } else if (P.bound_lane >= 0 && P.bound_lane < (int)ctx->lanes.size()) {
    lane = P.bound_lane;
  } else {
    lane = 0;
    for (int i = 1; i < (int)ctx->lanes.size(); ++i) {
      const LaneRes &a = *ctx->lanes[i], &b = *ctx->lanes[lane];
      if (a.nplans < b.nplans || (a.nplans == b.nplans && a.inflight < b.inflight)) lane = i;
    }
  }
  LaneRes& LR = *ctx->lanes[lane];
  if (LR.free_slots.empty()) throw Error(H2_ERR_TOO_LARGE, "more than 64 jobs in flight on one lane");
  if (tol_differs(P, eps, tol)) quiesce(ctx, P);  // descriptors change: the plan's earlier jobs must be done
  admit(ctx, LR, P, result_bytes(X, Y, P, kc));
  P.last_use = ++ctx->submissions;
  bind(ctx, P, lane, eps);
  set_tolerances(P, eps, tol);
  J->f32 = f32;
  J->kc = kc;
  J->lane = lane;
  J->slot = LR.free_slots.back();
  LR.free_slots.pop_back();
  J->flag = LR.flags + J->slot;
  ++P.inflight;  // from here on release() undoes these
  P.lane = lane;
  ++LR.inflight;
  J->tplan = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  Lane L = LR.l;
  L.overflow = J->flag;
  const hipStream_t s = L.stream;
  H2_HIP(hipMemsetAsync(J->flag, 0, sizeof(int), s));
  if (opt.graph && opt.timing == 0) {
    if (!P.gflag.p) P.gflag.alloc(sizeof(int));
    if (!P.gexec || P.g_desc != P.desc.p) {
      if (P.gexec) {
        H2_HIP(hipGraphExecDestroy(P.gexec));
        P.gexec = nullptr;
      }
      Lane G = L;
      G.overflow = P.gflag.as<int>();
      hipGraph_t graph = nullptr;
      H2_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      try {
        execute(ctx, G, P, 0, J->tph);
      } catch (...) {
        (void)hipStreamEndCapture(s, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      H2_HIP(hipStreamEndCapture(s, &graph));
      const hipError_t e = hipGraphInstantiate(&P.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      H2_HIP(e);
      P.g_desc = P.desc.p;
    }
    H2_HIP(hipMemsetAsync(P.gflag.p, 0, sizeof(int), s));
    H2_HIP(hipGraphLaunch(P.gexec, s));
    H2_HIP(hipMemcpyAsync(J->flag, P.gflag.p, sizeof(int), hipMemcpyDeviceToDevice, s));
  } else {
    execute(ctx, L, P, opt.timing, J->tph);
  }
  // result arrays: one allocation while the device works, filled by copies
  // queued behind the product (if it fails, the queued work is waited for
  // before the job is released)
  auto Cm = std::make_unique<Matrix>();
  Cm->ctx = ctx;
  Cm->hold = ctx->self.lock();
  Cm->id = ctx->next_id++;
  Cm->rows = X->rows;
  Cm->cols = Y->cols;
  build_block_tree(Cm->bt, *X->rows, *Y->cols, X->bt.eta);
  Cm->kc = kc;
  const int64_t n_vleaf = X->rows->n * kc, n_vtr = (int64_t)X->rows->ncl * kc * kc, n_wleaf = Y->cols->n * kc,
                n_wtr = (int64_t)Y->cols->ncl * kc * kc, n_s = (int64_t)P.cbt.adm.size() * kc * kc,
                n_n = P.cnsize, n_r = X->rows->ncl + Y->cols->ncl;
  auto pad = [](int64_t c) { return (std::max<int64_t>(c, 1) + 31) & ~int64_t(31); };
  Cm->bufs.emplace_back(new DevBuf);
  try {
    Cm->bufs.back()->alloc((size_t)(pad(n_vleaf) + pad(n_vtr) + pad(n_wleaf) + pad(n_wtr) + pad(n_s) + pad(n_n) +
                                    pad(n_r)) *
                           sizeof(double));
  } catch (...) {
    for (hipStream_t q : {LR.l.stream, LR.l.aux[0], LR.l.aux[1]}) (void)hipStreamSynchronize(q);
    throw;
  }
  double* carve = Cm->bufs.back()->as<double>();
  auto take = [&](int64_t c) {
    double* d = carve;
    carve += pad(c);
    return d;
  };
  Cm->V.leaf = take(n_vleaf);
  Cm->V.transfer = take(n_vtr);
  Cm->W.leaf = take(n_wleaf);
  Cm->W.transfer = take(n_wtr);
  Cm->S = take(n_s);
  Cm->N = take(n_n);
  J->dev_ranks = (int*)take(n_r);
  auto cp = [&](void* d, const void* src, int64_t bytes) {
    if (bytes) H2_HIP(hipMemcpyAsync(d, src, bytes, hipMemcpyDeviceToDevice, s));
  };
  cp(Cm->V.leaf, res(P.res_vleaf, P), n_vleaf * 8);
  cp(Cm->V.transfer, res(P.res_vtr, P), n_vtr * 8);
  cp(Cm->W.leaf, res(P.res_wleaf, P), n_wleaf * 8);
  cp(Cm->W.transfer, res(P.res_wtr, P), n_wtr * 8);
  cp(Cm->S, res(P.res_S, P), n_s * 8);
  cp(Cm->N, res(P.res_N, P), n_n * 8);
  cp(J->dev_ranks, res(P.res_rank_row, P), X->rows->ncl * sizeof(int));
  cp(J->dev_ranks + X->rows->ncl, res(P.res_rank_col, P), Y->cols->ncl * sizeof(int));
  Cm->noff = P.cnoff;
  Cm->nsize = P.cnsize;
  J->C = std::move(Cm);
  H2_HIP(hipEventCreateWithFlags(&J->done, hipEventDisableTiming));
  H2_HIP(hipEventRecord(J->done, s));
  return J.release();
}

bool poll(Job& J) {
  if (J.finished) return true;
  const hipError_t e = hipEventQuery(J.done);
  if (e == hipSuccess) return true;
  if (e == hipErrorNotReady) return false;
  H2_HIP(e);
  return false;
}

std::unique_ptr<Matrix> wait(Job& J, h2_mul_stats* stats) {
  if (J.finished) throw Error(H2_ERR_INVALID_ARG, "job already waited for");
  Context* ctx = J.ctx;
  H2_HIP(hipEventSynchronize(J.done));
  int ovf = 0;
  H2_HIP(hipMemcpy(&ovf, J.flag, sizeof(int), hipMemcpyDeviceToHost));
  J.release();
  if (ovf & h2k::kOvfNotConverged) J.C.reset();
  check_overflow_bits(ovf);
  if (ovf) {
    J.C.reset();
    if (J.f32) {
      // FP32 rounding of the exact blocks reached the truncation tolerance
      // (cancellation in the product): rounding noise would be kept as rank.
      // Run this product, and tighter ones on the same pair, in FP64.
      double& fe = ctx->fp32_fail_eps[{J.X->id, J.Y->id}];
      fe = std::max(fe, J.eps);
      ctx->plans.erase(J.key);
      J.P.reset();
      h2_mul_options o2 = J.opt;
      o2.precision = H2_PREC_FP64;
      return multiply(ctx, J.X, J.Y, J.eps, o2, stats);
    }
    if ((ovf & 2) && J.opt.max_rank == 0 && J.kc < 64) {
      // the default cap was too small for this product: retry once with the
      // largest cap, and start there for later products of the pair
      ctx->kc_raised[{J.X->id, J.Y->id}] = 64;
      ctx->plans.erase(J.key);
      J.P.reset();
      return multiply(ctx, J.X, J.Y, J.eps, J.opt, stats);
    }
    throw Error(H2_ERR_TOO_LARGE, (ovf & 1) ? "coarsened rank above coarse_rank cap"
                                             : "basis rank above max_rank cap");
  }
  Matrix& C = *J.C;
  const int nr = J.X->rows->ncl, nc = J.Y->cols->ncl;
  std::vector<int> rk(nr + nc);
  H2_HIP(hipMemcpy(rk.data(), J.dev_ranks, rk.size() * sizeof(int), hipMemcpyDeviceToHost));
  C.rank_row.assign(rk.begin(), rk.begin() + nr);
  C.rank_col.assign(rk.begin() + nr, rk.end());
  if (stats) {
    const Plan& P = *J.P;
    std::memset(stats, 0, sizeof(*stats));
    for (int i = 0; i < 8; ++i) stats->t_phase[i] = J.tph[i];
    stats->t_plan_ms = J.built ? J.tplan : 0.0;
    stats->bytes_alg = P.bytes_alg;
    stats->flops_alg = P.flops_alg;
    stats->prec_used = J.f32 ? H2_PREC_FP32_BULK : H2_PREC_FP64;
    stats->rank_max_row = C.rank_row.empty() ? 0 : *std::max_element(C.rank_row.begin(), C.rank_row.end());
    stats->rank_max_col = C.rank_col.empty() ? 0 : *std::max_element(C.rank_col.begin(), C.rank_col.end());
    stats->coarse_rank_max = P.max_coarse_K;
    stats->n_adm = P.n_adm;
    stats->n_inadm = P.n_inadm;
    stats->launches = P.launches;
    static_assert(h2k::K_COUNT == H2_NKERNEL, "kernel count");
    for (int i = 0; i < h2k::K_COUNT; ++i) {
        stats->t_kernel[i] = P.t_k[i];
        stats->launches_kernel[i] = P.launches_k[i];
        stats->units_kernel[i] = P.units_k[i];
        stats->flops_kernel[i] = P.flops_k[i];
        stats->bytes_kernel[i] = P.bytes_k[i];
    }
  }
  return std::move(J.C);
}

std::unique_ptr<Matrix> multiply(Context* ctx, Matrix* X, Matrix* Y, double eps, const h2_mul_options& opt,
                                 h2_mul_stats* stats) {
  std::unique_ptr<Job> J(submit(ctx, X, Y, eps, opt));
  return wait(*J, stats);
}

void destroy_job(Job* J) {
  if (!J) return;
  if (!J->finished && J->done) (void)hipEventSynchronize(J->done);  // buffers in use until then
  J->release();
  delete J;
}
}  // namespace h2

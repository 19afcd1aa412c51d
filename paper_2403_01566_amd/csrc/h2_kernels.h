// Internal interface between the host planner and the gfx950 kernels.
// Every floating-point step of the product runs in these kernels; the host
// only builds integer work lists (plans) and launches them.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace h2k {

// Item flags.
enum : int {
  IT_TRANS_A = 1,     // use A^T
  IT_TRANS_B = 2,     // use B^T
  IT_COPY = 4,        // C += alpha * op(A) (A is m x n, B unused)
  IT_SCALE_INV = 8,   // multiply alpha by 1/(*scale) (0 if *scale == 0)
};

// One contribution alpha * op(A) * op(B) (or alpha * op(A)) to a task's output.
// Matrices are row-major with the given leading dimensions.  Optional device
// ints k_dev, k_dev2 lower the inner dimension to min(k, *k_dev + *k_dev2)
// (a width known only on the device, e.g. the packed columns of a merge; the
// part beyond it is zero padding, so leaving it out changes no sum).
template <typename T>
struct GemmItem {
  const T* a;
  const T* b;
  const double* scale;  // optional device scalar (see IT_SCALE_INV)
  const int* k_dev;
  const int* k_dev2;
  int lda, ldb, k, flags;
  double alpha;
};

// Width of the K slices of the batched GEMM.
constexpr int kGemmSliceK = 8;

// One output matrix C (m x n, row-major, ldc): C = (beta ? C : 0) + sum of items.
// Optional device ints: m_dev / n_dev lower m / n to min(m, *m_dev) etc.,
// coff_dev shifts the output by *coff_dev columns and roff_dev by *roff_dev
// rows (sizes known only on the device, e.g. truncation ranks).
// Optional stat (3 ints, written by the task's first tile): the device-side
// m and n and the sum of the product items' device-side k.
template <typename T>
struct GemmTask {
  T* c;
  const int* m_dev;
  const int* n_dev;
  const int* coff_dev;
  const int* roff_dev;
  int* stat;
  int ldc, m, n, item0, nitem, beta;
  int ncopy;   // copy items
  int pad;
};

struct GemmTile {
  int task, m0, n0, pad;
};

// Streaming Householder QR, R factor only: A (m x w, row-major, lda) -> R (w x w).
// R is upper triangular (rows >= min(m,w) are zero); with trans_r the kernel
// stores R^T instead.  Only the first w_eff = (w_dev ? *w_dev : w) +
// (w_dev2 ? *w_dev2 : 0) columns (at most w) are factored, R is written as
// w x w with zeros beyond w_eff.  Rows: the first m, lowered to *m_dev when
// m_dev is set and to mul_we * w_eff when mul_we > 0.  part >= 0 writes the
// w_eff x w upper part only, at row offset part * w_eff (row-major, ldr; for
// stacking the R factors of row blocks compactly).  With m_dev the row count
// is min(m, *m_dev - m_off) (a row block of a matrix whose height is known
// on the device).  Optional stat (2 ints): the number of rows factored and
// w_eff.
struct QrTask {
  const double* a;
  double* r;
  const int* w_dev;
  const int* w_dev2;
  const int* m_dev;
  int* stat;
  int lda, ldr, m, w, trans_r, mul_we, part, m_off;
};

// One-sided Jacobi on a small matrix A (rows x cols, row-major, lda), rotating
// columns: A J = B with orthogonal columns.  Singular values are the column
// norms of B; the left singular vectors are the normalised columns.  Outputs:
// sigma (descending, cols entries), the number kept, and an orthonormal basis
// of the kept left singular vectors (rows x kcap, zero beyond kept, ldu).
// Threshold tau = tol_abs + tol_rel * sigma_1 + tol_scale * (tol_ptr ? *tol_ptr : 0).
// frob == 0: keep sigma_i > tau (largest dropped value below tau);
// frob == 1: keep the fewest values such that the Frobenius norm of the
// dropped tail is at most tau.  Overflow sets bits `ovf_bit` in *overflow.
// Square case with w_dev/w_dev2 as in QrTask: rows = cols = w_eff.  With u2,
// the output rows are split at *split_dev: rows below go to u, the rest to u2
// (each written as kcap_rows x kcap, zero elsewhere).
struct SvdTask {
  const double* a;
  double* u;
  double* u2;
  double* sigma;    // cols entries
  int* rank;        // 1 entry
  const double* tol_ptr;
  const int* w_dev;
  const int* w_dev2;
  const int* split_dev;
  int* stat;  // optional, 4 ints: rows, cols, columns after the rank reveal, Jacobi sweeps
  double tol_abs, tol_rel, tol_scale;
  int lda, ldu, rows, cols, kcap, trans_a, frob, ovf_bit, urows;
  // qrcp != 0 (absolute threshold only): first a column-pivoted Householder
  // QR of A^T that stops once the remaining Frobenius norm is at most tau/8;
  // the Jacobi then runs on the rows x r factor only, with the threshold
  // 3 tau / 4.  The projection error of the result stays <= tau; sigma holds
  // the singular values of the factor (within tau/8 of those of A).
  int qrcp;
  // Jacobi sweep cap (0 => 40).  A Jacobi that still rotates after the cap
  // sets bit kOvfNotConverged in *overflow.
  int maxsw;
};
// Overflow-word bit of a Jacobi that did not converge within its sweep cap
// (bits 1 and 2 are the rank-cap overflows of the coarsening and the bases).
constexpr int kOvfNotConverged = 4;

// Lower bound of a block norm from factors of its pieces: for every group,
// out = factor * max over its matrices of the largest row or column norm
// (every row and column norm of a matrix is at most its spectral norm; the
// matrices are pieces of the block or factors with the same Gram matrix).
struct RefMat {
  const double* a;
  int lda, rows, cols;
  double scale;  // the matrix's largest row or column norm counts times scale
};
struct RefTask {
  int first, count;
  double factor;
  double* out;
};

// Scaled Cholesky step for orthonormalising a tall m x w matrix Y from its
// Gram matrix G = Y^T Y (w x w): D = diag(G)^(1/2), D^-1 G D^-1 = R'^T R',
// outputs T = D^-1 R'^-1 (so Y T has orthonormal columns) and R = R' D
// (so Y = (Y T) R).  Only the first *weff columns are used (rest zero).
struct CholTask {
  const double* g;
  double* t;
  double* r;
  const int* weff;  // optional; null = w
  int ldg, ldt, ldr, w;
};

// Exclusive prefix sums of device ints: offs[i] = sum_{j<i} *src[first + j],
// *total = the full sum.
struct ScanTask {
  int first, count;
  int* offs;
  int* total;
};

struct FillTask {
  void* p;
  int ld, m, n, pad;
  double value;       // diagonal value when diag != 0, fill value otherwise
  int diag, elem;     // elem: 8 double / 4 float
};

void launch_gemm_f64(const GemmItem<double>* items, const GemmTask<double>* tasks, const GemmTile* tiles,
                     int ntiles, hipStream_t s);
void launch_gemm_f32(const GemmItem<float>* items, const GemmTask<float>* tasks, const GemmTile* tiles,
                     int ntiles, hipStream_t s);
void launch_qr(const QrTask* tasks, int ntasks, int wmax, hipStream_t s);
void launch_svd(const SvdTask* tasks, int ntasks, int wmax, int* overflow, hipStream_t s);
// The QR and SVD launchers run one kernel per size class (widths <= 32, <= 64,
// <= 128); the class-wise forms serve per-kernel timing.
int size_classes(int wmax);
void launch_qr_class(const QrTask* tasks, int ntasks, int cls, hipStream_t s);
void launch_svd_class(const SvdTask* tasks, int ntasks, int cls, int* overflow, hipStream_t s);

// Kernel identities for per-kernel statistics (the names are the template
// instantiations a profiler shows).
enum KernelId {
  K_GEMM_F64, K_GEMM_F32, K_QR32, K_QR64, K_QR128, K_SVD32, K_SVD64, K_SVD128,
  K_CHOL, K_FILL, K_CVT, K_REF, K_SCAN, K_COUNT
};
const char* kernel_name(int id);
void launch_chol(const CholTask* tasks, int ntasks, int wmax, hipStream_t s);
void launch_ref(const RefTask* tasks, const RefMat* mats, int ntasks, hipStream_t s);
void launch_fill(const FillTask* tasks, int ntasks, hipStream_t s);
void launch_scan(const ScanTask* tasks, const int* const* src, int ntasks, hipStream_t s);
// Vector kernels of the power iteration: y = a x + b y (x may alias y), and
// partial sums of x . y, one per workgroup of kDotBlocks (the host adds them
// in index order).
constexpr int kDotBlocks = 256;
void launch_axpby(const double* x, double* y, int64_t n, double a, double b, hipStream_t s);
void launch_dot(const double* x, const double* y, int64_t n, double* partial, hipStream_t s);
void launch_convert_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
void launch_convert_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s);

}  // namespace h2k

// gfx950 kernels for the adaptive H2-matrix product.
//
//  * gemm: plan-driven batched GEMM on MFMA (v_mfma_f64_16x16x4f64 /
//    v_mfma_f32_16x16x4f32).  One 64x64 output tile per workgroup; each tile
//    accumulates all items of its task in a fixed order (deterministic
//    segmented sums, no atomics).
//  * qr: streaming Householder QR that keeps only R.  Rows stream through LDS
//    in chunks; each chunk is eliminated against the current triangle with
//    reflectors of length 1 + chunk rows (R-factor of [R; C]).
//  * svd: one-sided (Hestenes) Jacobi on a matrix held in LDS, round-robin
//    pair ordering, followed by sorting, rank selection by threshold and
//    output of the kept normalised left singular vectors.
//  * chol: scaled Cholesky factorisation of a small Gram matrix, giving the
//    triangular transform that orthonormalises a tall near-orthogonal matrix.
#include "h2_kernels.h"

#include <cmath>

namespace h2k {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4v acc;
  __device__ static inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row of accumulator register v held by `lane` (rows interleaved by 4)
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef f4v acc;
  __device__ static inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output row of accumulator register v held by `lane` (4 consecutive rows)
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int GBM = 64, GBN = 64, GBK = 16;

// MFMA 16x16x4 register layout used below (gfx950, checked on the device):
//   A operand: lane l supplies A[l % 16][k0 + l / 16]
//   B operand: lane l supplies B[k0 + l / 16][l % 16]
//   D: lane l, register v holds D[row][l % 16] with row = 4 (l / 16) + v for
//      f32 and row = l / 16 + 4 v for f64 (Mfma<T>::row).
template <typename T>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmItem<T>* __restrict__ items,
                                                   const GemmTask<T>* __restrict__ tasks,
                                                   const GemmTile* __restrict__ tiles) {
  __shared__ T As[GBK][GBM + 4];
  __shared__ T Bs[GBK][GBN + 4];
  typedef typename Mfma<T>::acc acc_t;
  const GemmTile tl = tiles[blockIdx.x];
  const GemmTask<T> tk = tasks[tl.task];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = tl.m0, n0 = tl.n0;
  acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) acc[a][b][v] = T(0);

  for (int it = 0; it < tk.nitem; ++it) {
    const GemmItem<T> item = items[tk.item0 + it];
    double alpha = item.alpha;
    if (item.scale) {
      double s = *item.scale;
      if (item.flags & IT_SCALE_INV) alpha = (s != 0.0) ? alpha / s : 0.0;
      else alpha *= s;
    }
    const T al = T(alpha);
    const bool ta = item.flags & IT_TRANS_A, tb = item.flags & IT_TRANS_B;
    if (item.flags & IT_COPY) {
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int v = 0; v < 4; ++v) {
            int row = m0 + wm * 32 + a * 16 + Mfma<T>::row(lane, v);
            int col = n0 + wn * 32 + b * 16 + (lane & 15);
            if (row < tk.m && col < tk.n) {
              T x = ta ? item.a[(int64_t)col * item.lda + row] : item.a[(int64_t)row * item.lda + col];
              acc[a][b][v] += al * x;
            }
          }
      continue;
    }
    const int K = item.k;
    for (int k0 = 0; k0 < K; k0 += GBK) {
      __syncthreads();
      // A tile: op(A)[m0+i][k0+kk], i < 64, kk < 16
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int e = tid + 256 * q;
        int i, kk;
        if (!ta) { i = e >> 4; kk = e & 15; } else { kk = e >> 6; i = e & 63; }
        int gi = m0 + i, gk = k0 + kk;
        T x = T(0);
        if (gi < tk.m && gk < K)
          x = ta ? item.a[(int64_t)gk * item.lda + gi] : item.a[(int64_t)gi * item.lda + gk];
        As[kk][i] = al * x;
      }
      // B tile: op(B)[k0+kk][n0+j]
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int e = tid + 256 * q;
        int j, kk;
        if (!tb) { kk = e >> 6; j = e & 63; } else { j = e >> 4; kk = e & 15; }
        int gj = n0 + j, gk = k0 + kk;
        T x = T(0);
        if (gj < tk.n && gk < K)
          x = tb ? item.b[(int64_t)gj * item.ldb + gk] : item.b[(int64_t)gk * item.ldb + gj];
        Bs[kk][j] = x;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < GBK; kk += 4) {
        T av[2], bv[2];
        for (int a = 0; a < 2; ++a) av[a] = As[kk + (lane >> 4)][wm * 32 + a * 16 + (lane & 15)];
        for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][wn * 32 + b * 16 + (lane & 15)];
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::op(av[a], bv[b], acc[a][b]);
      }
    }
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) {
        int row = m0 + wm * 32 + a * 16 + Mfma<T>::row(lane, v);
        int col = n0 + wn * 32 + b * 16 + (lane & 15);
        if (row < tk.m && col < tk.n) {
          T* p = tk.c + (int64_t)row * tk.ldc + col;
          *p = tk.beta ? (*p + acc[a][b][v]) : acc[a][b][v];
        }
      }
}

void launch_gemm_f64(const GemmItem<double>* items, const GemmTask<double>* tasks, const GemmTile* tiles,
                     int ntiles, hipStream_t s) {
  if (ntiles > 0) hipLaunchKernelGGL(gemm_kernel<double>, dim3(ntiles), dim3(256), 0, s, items, tasks, tiles);
}
void launch_gemm_f32(const GemmItem<float>* items, const GemmTask<float>* tasks, const GemmTile* tiles,
                     int ntiles, hipStream_t s) {
  if (ntiles > 0) hipLaunchKernelGGL(gemm_kernel<float>, dim3(ntiles), dim3(256), 0, s, items, tasks, tiles);
}

// ---------------------------------------------------------------------------
// Streaming Householder QR (R only).
// ---------------------------------------------------------------------------
template <int WMAX, int CH>
__global__ __launch_bounds__(256) void qr_kernel(const QrTask* __restrict__ tasks) {
  __shared__ double R[WMAX * WMAX];
  __shared__ double C[CH * WMAX];
  __shared__ double sh_tau, sh_scal;
  const QrTask tk = tasks[blockIdx.x];
  const int w = tk.w, m = tk.m, tid = threadIdx.x;
  for (int e = tid; e < w * w; e += blockDim.x) R[e] = 0.0;
  for (int row0 = 0; row0 < m; row0 += CH) {
    const int cr = min(CH, m - row0);
    __syncthreads();
    for (int e = tid; e < cr * w; e += blockDim.x) {
      int i = e / w, l = e - i * w;
      C[i * w + l] = tk.a[(int64_t)(row0 + i) * tk.lda + l];
    }
    __syncthreads();
    for (int j = 0; j < w; ++j) {
      if (tid < 64) {
        double x2 = 0.0;
        for (int i = tid; i < cr; i += 64) {
          double x = C[i * w + j];
          x2 += x * x;
        }
        for (int off = 32; off > 0; off >>= 1) x2 += __shfl_xor(x2, off, 64);
        if (tid == 0) {
          double alpha = R[j * w + j];
          if (x2 == 0.0) {
            sh_tau = 0.0;
            sh_scal = 0.0;
          } else {
            double nrm = sqrt(alpha * alpha + x2);
            double beta = alpha >= 0.0 ? -nrm : nrm;
            sh_tau = (beta - alpha) / beta;
            sh_scal = 1.0 / (alpha - beta);
            R[j * w + j] = beta;
          }
        }
      }
      __syncthreads();
      const double tau = sh_tau, scal = sh_scal;
      if (tau != 0.0) {
        for (int l = j + 1 + tid; l < w; l += blockDim.x) {
          double dot = 0.0;
          for (int i = 0; i < cr; ++i) dot += C[i * w + j] * C[i * w + l];
          dot = R[j * w + l] + scal * dot;
          R[j * w + l] -= tau * dot;
          const double f = tau * scal * dot;
          for (int i = 0; i < cr; ++i) C[i * w + l] -= f * C[i * w + j];
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += blockDim.x) {
    int i = e / w, l = e - i * w;
    double v = (l >= i) ? R[i * w + l] : 0.0;
    if (tk.trans_r) tk.r[(int64_t)l * tk.ldr + i] = v;
    else tk.r[(int64_t)i * tk.ldr + l] = v;
  }
}

void launch_qr(const QrTask* tasks, int ntasks, int wmax, hipStream_t s) {
  if (ntasks <= 0) return;
  if (wmax <= 32) hipLaunchKernelGGL((qr_kernel<32, 64>), dim3(ntasks), dim3(64), 0, s, tasks);
  else if (wmax <= 64) hipLaunchKernelGGL((qr_kernel<64, 64>), dim3(ntasks), dim3(64), 0, s, tasks);
  else hipLaunchKernelGGL((qr_kernel<128, 16>), dim3(ntasks), dim3(128), 0, s, tasks);
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD (left vectors).
// ---------------------------------------------------------------------------
template <int WMAX>
__global__ __launch_bounds__(256) void svd_kernel(const SvdTask* __restrict__ tasks, int* overflow) {
  // M[c * WMAX + r] holds column c (contiguous rows)
  __shared__ double M[WMAX * WMAX];
  __shared__ double nrm[WMAX];
  __shared__ int order[WMAX];
  __shared__ int sh_rot;
  const SvdTask tk = tasks[blockIdx.x];
  const int rows = tk.rows, cols = tk.cols, tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < cols * WMAX; e += nt) {
    int c = e / WMAX, r = e - c * WMAX;
    double v = 0.0;
    if (r < rows) v = tk.trans_a ? tk.a[(int64_t)c * tk.lda + r] : tk.a[(int64_t)r * tk.lda + c];
    M[e] = v;
  }
  const int np = (cols + 1) & ~1;   // players incl. a dummy when cols is odd
  const int npairs = np / 2;
  // threads per pair: groups of G lanes inside one wave
  const int G = (npairs * 4 <= nt) ? 4 : ((npairs * 2 <= nt) ? 2 : 1);
  const int grp = tid / G, gl = tid % G;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) sh_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      for (int g = grp; g < npairs; g += nt / G) {
        int p, q;
        if (g == 0) { p = np - 1; q = rnd; }
        else { p = (rnd + g) % (np - 1); q = (rnd - g + (np - 1)) % (np - 1); }
        bool valid = p < cols && q < cols;
        double a = 0.0, b = 0.0, c = 0.0;
        double* cp = M + (valid ? p : 0) * WMAX;
        double* cq = M + (valid ? q : 0) * WMAX;
        if (valid)
          for (int r = gl; r < rows; r += G) {
            double x = cp[r], y = cq[r];
            a += x * x; b += y * y; c += x * y;
          }
        for (int off = 1; off < G; off <<= 1) {
          a += __shfl_xor(a, off, 64);
          b += __shfl_xor(b, off, 64);
          c += __shfl_xor(c, off, 64);
        }
        if (valid && c != 0.0 && fabs(c) > 1e-15 * sqrt(a * b)) {
          double zeta = (b - a) / (2.0 * c);
          double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int r = gl; r < rows; r += G) {
            double x = cp[r], y = cq[r];
            cp[r] = cs * x - sn * y;
            cq[r] = sn * x + cs * y;
          }
          if (gl == 0) sh_rot = 1;
        }
      }
      __syncthreads();
    }
    if (!sh_rot) break;
    __syncthreads();
  }
  // singular values and descending order
  for (int c = tid; c < cols; c += nt) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += M[c * WMAX + r] * M[c * WMAX + r];
    nrm[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < cols; c += nt) {
    int rk = 0;
    double v = nrm[c];
    for (int d = 0; d < cols; ++d) rk += (nrm[d] > v) || (nrm[d] == v && d < c);
    order[rk] = c;
  }
  __syncthreads();
  const double smax = cols > 0 ? nrm[order[0]] : 0.0;
  const double thr = tk.tol_abs + tk.tol_rel * smax + (tk.tol_ptr ? tk.tol_scale * *tk.tol_ptr : 0.0);
  int keep = 0;
  if (!tk.frob) {
    for (int i = 0; i < cols; ++i) keep += nrm[i] > thr;
  } else {
    // fewest kept values whose dropped tail has Frobenius norm <= thr
    double tail = 0.0;
    keep = cols;
    const double thr2 = thr * thr;
    for (int i = cols - 1; i >= 0; --i) {
      double v = nrm[order[i]];
      if (tail + v * v > thr2) break;
      tail += v * v;
      keep = i;
    }
  }
  if (keep > tk.kcap) {
    if (tid == 0 && overflow) atomicOr(overflow, tk.ovf_bit);
    keep = tk.kcap;
  }
  for (int i = tid; i < cols; i += nt) tk.sigma[i] = nrm[order[i]];
  if (tid == 0) *tk.rank = keep;
  for (int e = tid; e < rows * tk.kcap; e += nt) {
    int r = e / tk.kcap, i = e - r * tk.kcap;
    double v = 0.0;
    if (i < keep) {
      int c = order[i];
      v = M[c * WMAX + r] / nrm[c];
    }
    tk.u[(int64_t)r * tk.ldu + i] = v;
  }
}

void launch_svd(const SvdTask* tasks, int ntasks, int wmax, int* overflow, hipStream_t s) {
  if (ntasks <= 0) return;
  if (wmax <= 32) hipLaunchKernelGGL((svd_kernel<32>), dim3(ntasks), dim3(64), 0, s, tasks, overflow);
  else if (wmax <= 64) hipLaunchKernelGGL((svd_kernel<64>), dim3(ntasks), dim3(128), 0, s, tasks, overflow);
  else hipLaunchKernelGGL((svd_kernel<128>), dim3(ntasks), dim3(256), 0, s, tasks, overflow);
}

// ---------------------------------------------------------------------------
// Scaled Cholesky orthonormalisation step.
// ---------------------------------------------------------------------------
template <int WMAX>
__global__ __launch_bounds__(64) void chol_kernel(const CholTask* __restrict__ tasks) {
  __shared__ double H[WMAX][WMAX + 1];
  __shared__ double Ri[WMAX][WMAX + 1];
  __shared__ double d[WMAX];
  const CholTask tk = tasks[blockIdx.x];
  const int w = tk.w, tid = threadIdx.x;
  const int we = tk.weff ? min(*tk.weff, w) : w;
  for (int i = tid; i < w; i += 64) {
    double g = (i < we) ? tk.g[(int64_t)i * tk.ldg + i] : 0.0;
    d[i] = g > 0.0 ? sqrt(g) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += 64) {
    int i = e / w, l = e - i * w;
    double v = 0.0;
    if (i < we && l < we) {
      if (d[i] > 0.0 && d[l] > 0.0) v = tk.g[(int64_t)i * tk.ldg + l] / (d[i] * d[l]);
      else v = (i == l) ? 1.0 : 0.0;
    } else if (i == l) {
      v = 1.0;
    }
    H[i][l] = v;
    Ri[i][l] = 0.0;
  }
  __syncthreads();
  // right-looking Cholesky, upper factor stored in the upper triangle of H
  for (int j = 0; j < w; ++j) {
    if (tid == 0) H[j][j] = sqrt(fmax(H[j][j], 1e-300));
    __syncthreads();
    for (int l = j + 1 + tid; l < w; l += 64) H[j][l] /= H[j][j];
    __syncthreads();
    for (int e = tid; e < (w - j - 1) * (w - j - 1); e += 64) {
      int i = j + 1 + e / (w - j - 1), l = j + 1 + e % (w - j - 1);
      if (l >= i) H[i][l] -= H[j][i] * H[j][l];
    }
    __syncthreads();
  }
  // inverse of the upper factor, one column per thread (back substitution)
  for (int l = tid; l < w; l += 64) {
    for (int i = l; i >= 0; --i) {
      double s = (i == l) ? 1.0 : 0.0;
      for (int k2 = i + 1; k2 <= l; ++k2) s -= H[i][k2] * Ri[k2][l];
      Ri[i][l] = s / H[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += 64) {
    int i = e / w, l = e - i * w;
    bool in = i < we && l < we;
    double tv = 0.0, rv = 0.0;
    if (in && l >= i) {
      tv = d[i] > 0.0 ? Ri[i][l] / d[i] : 0.0;
      rv = H[i][l] * d[l];
    }
    tk.t[(int64_t)i * tk.ldt + l] = tv;
    tk.r[(int64_t)i * tk.ldr + l] = rv;
  }
}

void launch_chol(const CholTask* tasks, int ntasks, int wmax, hipStream_t s) {
  if (ntasks <= 0) return;
  if (wmax <= 32) hipLaunchKernelGGL((chol_kernel<32>), dim3(ntasks), dim3(64), 0, s, tasks);
  else hipLaunchKernelGGL((chol_kernel<64>), dim3(ntasks), dim3(64), 0, s, tasks);
}

// ---------------------------------------------------------------------------
// Block-norm lower bounds for the coarsening tolerance.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ref_kernel(const RefTask* __restrict__ tasks, const RefMat* __restrict__ mats) {
  __shared__ double red[256];
  const RefTask tk = tasks[blockIdx.x];
  double best = 0.0;
  for (int q = 0; q < tk.count; ++q) {
    const RefMat m = mats[tk.first + q];
    for (int r = threadIdx.x; r < m.rows; r += blockDim.x) {
      double s = 0.0;
      for (int c = 0; c < m.cols; ++c) {
        double x = m.a[(int64_t)r * m.lda + c];
        s += x * x;
      }
      best = fmax(best, s);
    }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *tk.out = tk.factor * sqrt(red[0]);
}

void launch_ref(const RefTask* tasks, const RefMat* mats, int ntasks, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(ref_kernel, dim3(ntasks), dim3(256), 0, s, tasks, mats);
}

// ---------------------------------------------------------------------------
// Fills and conversions.
// ---------------------------------------------------------------------------
__global__ void fill_kernel(const FillTask* __restrict__ tasks) {
  const FillTask tk = tasks[blockIdx.y];
  const int64_t total = (int64_t)tk.m * tk.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e / tk.n), j = (int)(e - (int64_t)i * tk.n);
    double v = tk.diag ? (i == j ? tk.value : 0.0) : tk.value;
    if (tk.elem == 8) ((double*)tk.p)[(int64_t)i * tk.ld + j] = v;
    else ((float*)tk.p)[(int64_t)i * tk.ld + j] = (float)v;
  }
}

void launch_fill(const FillTask* tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  // grid.y indexes tasks; keep it within the hardware limit by chunking
  for (int t0 = 0; t0 < ntasks; t0 += 65535) {
    int nt = ntasks - t0 < 65535 ? ntasks - t0 : 65535;
    hipLaunchKernelGGL(fill_kernel, dim3(8, nt), dim3(256), 0, s, tasks + t0);
  }
}

__global__ void cvt_d2f(const double* in, float* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void cvt_f2d(const float* in, double* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}
void launch_convert_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(cvt_d2f, dim3(1024), dim3(256), 0, s, in, out, n);
}
void launch_convert_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(cvt_f2d, dim3(1024), dim3(256), 0, s, in, out, n);
}

}  // namespace h2k

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

#include <algorithm>
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

constexpr int GBM = 64, GBN = 64, GBK = kGemmSliceK;
constexpr int GQA = GBM * GBK / 256, GQB = GBN * GBK / 256;  // loads per thread and slice
static_assert(GQA >= 1 && GQB >= 1 && GBM * GBK % 256 == 0 && GBK % 4 == 0, "GEMM tile shape");

// MFMA 16x16x4 register layout used below (gfx950, checked on the device):
//   A operand: lane l supplies A[l % 16][k0 + l / 16]
//   B operand: lane l supplies B[k0 + l / 16][l % 16]
//   D: lane l, register v holds D[row][l % 16] with row = 4 (l / 16) + v for
//      f32 and row = l / 16 + 4 v for f64 (Mfma<T>::row).
//
// One workgroup (4 waves, each a 32 x 32 quarter) per 64 x 64 output tile.
// The K dimension of all items of the task is walked as one sequence of
// GBK-wide slices: while the MFMAs consume slice s from one LDS buffer, the
// global loads of slice s + 1 are in flight into registers and then land in
// the other buffer, so each slice costs one barrier.  A wave whose quarter
// lies outside the task's (device-side) size skips its MFMAs.
// Loads and stores through global-address-space pointers: the operands are
// plain device memory, and global (not flat) instructions are counted only by
// the vector-memory counter, so waiting on LDS never waits on them.
template <typename T>
__device__ inline T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ inline void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

template <typename T>
struct GemmSlice {
  T a[GQA], b[GQB];
};

// The occupancy hint (at least 5 waves per SIMD) keeps the accumulators in
// VGPRs: 69 registers and no AGPRs give 7 waves per SIMD, where the default
// choice (accumulators in AGPRs, 100 registers) gives 4.
template <typename T>
__global__ __launch_bounds__(256, 5) void gemm_kernel(const GemmItem<T>* __restrict__ items,
                                                   const GemmTask<T>* __restrict__ tasks,
                                                   const GemmTile* __restrict__ tiles) {
  __shared__ T As[2][GBK][GBM + 1];  // odd row stride: the lanes that store one column of a slice hit distinct banks
  __shared__ T Bs[2][GBK][GBN + 1];
  typedef typename Mfma<T>::acc acc_t;
  const GemmTile tl = tiles[blockIdx.x];
  GemmTask<T> tk = tasks[tl.task];
  if (tk.m_dev) tk.m = min(tk.m, *tk.m_dev);
  if (tk.n_dev) tk.n = min(tk.n, *tk.n_dev);
  if (tk.coff_dev) tk.c += *tk.coff_dev;
  if (tk.roff_dev) tk.c += (int64_t)*tk.roff_dev * tk.ldc;
  if (tl.m0 >= tk.m || tl.n0 >= tk.n) {  // whole tile outside the device-side size
    if (tk.stat && tl.m0 == 0 && tl.n0 == 0 && threadIdx.x == 0) {  // an empty task
      tk.stat[0] = max(tk.m, 0);
      tk.stat[1] = max(tk.n, 0);
      tk.stat[2] = 0;
    }
    return;
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = tl.m0, n0 = tl.n0;
  const bool active = m0 + wm * 32 < tk.m && n0 + wn * 32 < tk.n;
  acc_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) acc[a][b][v] = T(0);

  // copies (IT_COPY items) go straight into the accumulators; a task
  // without copies never walks its item list here
  for (int it = 0; it < (tk.ncopy > 0 ? tk.nitem : 0); ++it) {
    const GemmItem<T> item = items[tk.item0 + it];
    if (!(item.flags & IT_COPY)) continue;
    double alpha = item.alpha;
    if (item.scale) {
      double s = *item.scale;
      if (item.flags & IT_SCALE_INV) alpha = (s != 0.0) ? alpha / s : 0.0;
      else alpha *= s;
    }
    const T al = T(alpha);
    const bool ta = item.flags & IT_TRANS_A;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int v = 0; v < 4; ++v) {
          int row = m0 + wm * 32 + a * 16 + Mfma<T>::row(lane, v);
          int col = n0 + wn * 32 + b * 16 + (lane & 15);
          if (row < tk.m && col < tk.n) {
            T x = ta ? gload(item.a + (int64_t)col * item.lda + row) : gload(item.a + (int64_t)row * item.lda + col);
            acc[a][b][v] += al * x;
          }
        }
  }

  // number of K slices: the product items' device-side widths in slices of
  // GBK (the part beyond a device-side width is zero padding)
  int nsl = 0, ksum = 0;
  for (int i = 0; i < tk.nitem; ++i) {
    const GemmItem<T>* ip = items + tk.item0 + i;
    if (ip->flags & IT_COPY) continue;
    int ke = ip->k;
    if (ip->k_dev) ke = min(ke, __builtin_amdgcn_readfirstlane(*ip->k_dev + (ip->k_dev2 ? *ip->k_dev2 : 0)));
    ke = max(ke, 0);
    ksum += ke;
    nsl += (ke + GBK - 1) / GBK;
  }
  if (tk.stat && m0 == 0 && n0 == 0 && tid == 0) {
    tk.stat[0] = tk.m;
    tk.stat[1] = tk.n;
    tk.stat[2] = ksum;
  }
  if (nsl > 0) {
    // slice cursor over the product items (each item's K range lowered to its
    // device-side width)
    int it = -1, k0 = 0, kend = 0;
    GemmItem<T> item{};
    T al = T(0);
    auto advance = [&]() -> bool {  // move to the next slice; false at the end
      k0 += GBK;
      while (k0 >= kend) {
        ++it;
        while (it < tk.nitem && (items[tk.item0 + it].flags & IT_COPY)) ++it;
        if (it >= tk.nitem) return false;
        item = items[tk.item0 + it];
        double alpha = item.alpha;
        if (item.scale) {
          double s = *item.scale;
          if (item.flags & IT_SCALE_INV) alpha = (s != 0.0) ? alpha / s : 0.0;
          else alpha *= s;
        }
        al = T(alpha);
        k0 = 0;
        kend = item.k;
        if (item.k_dev) kend = min(kend, __builtin_amdgcn_readfirstlane(*item.k_dev + (item.k_dev2 ? *item.k_dev2 : 0)));
      }
      return true;
    };
    // Loads are unconditional (an out-of-range element reads element 0 of the
    // same operand, replaced by zero when stored), so the eight loads of a
    // slice issue back to back and stay in flight during the MFMAs.
    auto load = [&](GemmSlice<T>& g) {
      const bool ta = item.flags & IT_TRANS_A, tb = item.flags & IT_TRANS_B;
      const int64_t sa = ta ? 1 : item.lda, ska = ta ? item.lda : 1;
      const int64_t sb = tb ? item.ldb : 1, skb = tb ? 1 : item.ldb;
#pragma unroll
      for (int q = 0; q < GQA; ++q) {
        int e = tid + 256 * q;
        int i, kk;
        if (!ta) { i = e / GBK; kk = e % GBK; } else { kk = e / GBM; i = e % GBM; }
        const int gi = m0 + i, gk = k0 + kk;
        const bool in = gi < tk.m && gk < kend;
        g.a[q] = gload(item.a + (in ? gi * sa + gk * ska : 0));
      }
#pragma unroll
      for (int q = 0; q < GQB; ++q) {
        int e = tid + 256 * q;
        int j, kk;
        if (!tb) { kk = e / GBN; j = e % GBN; } else { j = e / GBK; kk = e % GBK; }
        const int gj = n0 + j, gk = k0 + kk;
        const bool in = gj < tk.n && gk < kend;
        g.b[q] = gload(item.b + (in ? gj * sb + gk * skb : 0));
      }
    };
    auto store = [&](const GemmSlice<T>& g, int buf) {  // same item and k0 as the load
      const bool ta = item.flags & IT_TRANS_A, tb = item.flags & IT_TRANS_B;
#pragma unroll
      for (int q = 0; q < GQA; ++q) {
        int e = tid + 256 * q;
        int i, kk;
        if (!ta) { i = e / GBK; kk = e % GBK; } else { kk = e / GBM; i = e % GBM; }
        const bool in = m0 + i < tk.m && k0 + kk < kend;
        As[buf][kk][i] = in ? al * g.a[q] : T(0);
      }
#pragma unroll
      for (int q = 0; q < GQB; ++q) {
        int e = tid + 256 * q;
        int j, kk;
        if (!tb) { kk = e / GBN; j = e % GBN; } else { j = e / GBK; kk = e % GBK; }
        const bool in = n0 + j < tk.n && k0 + kk < kend;
        Bs[buf][kk][j] = in ? g.b[q] : T(0);
      }
    };
    k0 = -GBK;
    kend = 0;
    advance();
    GemmSlice<T> g;
    load(g);
    store(g, 0);
    __syncthreads();
    int buf = 0;
    // the loop exits at its bottom only, so every path back to its head
    // passes the store of the loaded slice
    for (int sl = 1; sl <= nsl; ++sl) {
      const bool more = sl < nsl;
      if (more) {
        advance();
        load(g);  // next slice in flight during the MFMAs below
      }
      if (active) {
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 4) {
          T av[2], bv[2];
          for (int a = 0; a < 2; ++a) av[a] = As[buf][kk + (lane >> 4)][wm * 32 + a * 16 + (lane & 15)];
          for (int b = 0; b < 2; ++b) bv[b] = Bs[buf][kk + (lane >> 4)][wn * 32 + b * 16 + (lane & 15)];
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::op(av[a], bv[b], acc[a][b]);
        }
      }
      if (more) {
        store(g, buf ^ 1);
        __syncthreads();
        buf ^= 1;
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
          gstore(p, tk.beta ? T(gload(p) + acc[a][b][v]) : T(acc[a][b][v]));
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

// Lane exchange within a row of 16 lanes through DPP (a VALU operand
// modifier, no LDS round trip): CTRL is a quad permutation or a row mirror.
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of g consecutive lanes (g in 1, 2, 4, 8, 16), the
// result in every lane of the group: lane pairs, quads, half rows, rows.
__device__ inline double dpp_group_sum(double v, int g) {
  if (g >= 2) v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  if (g >= 4) v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  if (g >= 8) v += dpp_mov<0x141>(v);  // row_half_mirror
  if (g >= 16) v += dpp_mov<0x140>(v); // row_mirror
  return v;
}
// Ordering of LDS accesses between the lanes of one wave (no workgroup barrier).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ inline int dpp_mov_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

// Reciprocal and reciprocal square root from the hardware approximations
// (v_rcp_f64, v_rsq_f64), each refined by two Newton steps (the error
// squares per step): a short dependent chain in place of the compiler's
// correctly rounded division and square root, for the Jacobi rotations.
// Arguments are normal and positive (rsq) or nonzero (rcp) where used.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ inline double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x * y;
  y = fma(y, fma(-h, y, 0.5), y);  // y (3 - x y^2) / 2
  h = 0.5 * x * y;
  y = fma(y, fma(-h, y, 0.5), y);
  return y;
}

// ---------------------------------------------------------------------------
// Streaming Householder QR (R only), one workgroup per matrix.
// ---------------------------------------------------------------------------
__device__ inline int eff_width(int w, const int* a, const int* b) {
  if (!a && !b) return w;
  int v = (a ? *a : 0) + (b ? *b : 0);
  return v < w ? v : w;
}

// packed upper triangle of a w x w matrix, row by row
__device__ inline int pk(int j, int l, int w) { return j * w - (j * (j - 1)) / 2 + (l - j); }

// The rows arrive in chunks of CH = RPT * TPC.  Column l of a chunk lives in
// the registers of the TPC consecutive lanes of group l (lane `sub` holds rows
// sub, sub + TPC, ...); R (packed upper triangle) stays in LDS across chunks.
// Column step j applies the reflector of column j to every column l > j (a
// dot product over the group's registers, one shuffle reduction, an update of
// the registers and of R's row j).  The group of column j + 1 then builds the
// next reflector at once from its updated registers and publishes it (the
// vector's chunk part and tau) in a double-buffered LDS slot, so every column
// step costs one barrier.
template <int WMAX, int NT, int CH>
__global__ __launch_bounds__(NT) void qr_kernel(const QrTask* __restrict__ tasks, int wlo) {
  constexpr int TPC = NT / WMAX;  // lanes per column
  constexpr int RPT = CH / TPC;   // chunk rows per lane
  static_assert(TPC >= 1 && (TPC & (TPC - 1)) == 0 && TPC <= 16 && RPT * TPC == CH, "lanes per column");
  __shared__ double R[WMAX * (WMAX + 1) / 2];
  constexpr int VS = RPT + 2;  // padded run per lane: the TPC runs start on different LDS banks
  __shared__ double vb[2][TPC * VS];
  __shared__ double tb[2][2];
  const QrTask tk = tasks[blockIdx.x];
  const int we = eff_width(tk.w, tk.w_dev, tk.w_dev2);
  if (we <= wlo || we > WMAX) return;  // another launch handles this width class
  int m = tk.m;
  if (tk.m_dev) m = min(m, *tk.m_dev - tk.m_off);
  if (tk.mul_we > 0) m = min(m, tk.mul_we * we);
  m = max(m, 0);
  const int tid = threadIdx.x, sub = tid % TPC, l = tid / TPC;
  for (int e = tid; e < we * (we + 1) / 2; e += NT) R[e] = 0.0;

  // reflector of column c from (alpha = R[c][c], the group's chunk registers);
  // the vector goes to LDS lane-major (vb[slot][sub * VS + q] is chunk row
  // sub + TPC q), so each lane moves contiguous runs
  auto reflect = [&](const double* c, int col, int slot) {
    const int pd = pk(col, col, we);
    const double alpha = R[pd];
    double s4[4] = {0.0, 0.0, 0.0, 0.0};  // four partial sums: a shorter dependent chain
#pragma unroll
    for (int q = 0; q < RPT; ++q) s4[q & 3] += c[q] * c[q];
    double x2 = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    x2 = dpp_group_sum(x2, TPC);
    double tau = 0.0, scal = 0.0;
    if (x2 != 0.0) {
      const double nrm = sqrt(alpha * alpha + x2);
      const double beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
      if (sub == 0) R[pd] = beta;
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) vb[slot][sub * VS + q] = c[q];
    if (sub == 0) {
      tb[slot][0] = tau;
      tb[slot][1] = scal;
    }
  };

  double c[RPT];
  for (int r0 = 0; r0 < m; r0 += CH) {
    const int cr = min(CH, m - r0);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = sub + TPC * q;
      c[q] = (i < cr && l < we) ? gload(tk.a + (int64_t)(r0 + i) * tk.lda + l) : 0.0;
    }
    __syncthreads();  // R of the previous chunk complete, both slots free
    if (l == 0) reflect(c, 0, 0);
    __syncthreads();
    for (int j = 0; j < we; ++j) {
      const int b = j & 1;
      if (l > j && l < we) {
        const int p = pk(j, l, we);
        const double rjl = R[p];
        const double tau = tb[b][0], scal = tb[b][1];
        if (tau != 0.0) {
          double w[RPT];
          double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            w[q] = vb[b][sub * VS + q];
            d4[q & 3] += w[q] * c[q];
          }
          double dot = (d4[0] + d4[1]) + (d4[2] + d4[3]);
          dot = dpp_group_sum(dot, TPC);
          const double full = rjl + scal * dot;
          const double f = tau * scal * full;
#pragma unroll
          for (int q = 0; q < RPT; ++q) c[q] -= f * w[q];
          if (sub == 0) R[p] = rjl - tau * full;
        }
        if (l == j + 1) reflect(c, j + 1, b ^ 1);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  const int w = tk.w;
  if (tk.part >= 0) {  // compact output: rows [0, we) at row offset part * we
    double* out = tk.r + (int64_t)tk.part * we * tk.ldr;
    for (int e = tid; e < we * w; e += NT) {
      int i = e / w, ll = e - i * w;
      out[(int64_t)i * tk.ldr + ll] = (ll < we && ll >= i) ? R[pk(i, ll, we)] : 0.0;
    }
  } else {
    for (int e = tid; e < w * w; e += NT) {
      int i = e / w, ll = e - i * w;
      double v = (i < we && ll < we && ll >= i) ? R[pk(i, ll, we)] : 0.0;
      if (tk.trans_r) tk.r[(int64_t)ll * tk.ldr + i] = v;
      else tk.r[(int64_t)i * tk.ldr + ll] = v;
    }
  }
  if (tk.stat && tid == 0) {
    tk.stat[0] = m;
    tk.stat[1] = we;
  }
}

int size_classes(int wmax) { return wmax > 64 ? 3 : (wmax > 32 ? 2 : 1); }

// Workgroup shapes per width class.  The two narrow classes walk 128-row
// chunks with 8 lanes per column (half the column steps of 64-row chunks, as
// many registers per lane).  The 128-wide class keeps 64-row chunks on 4
// lanes per column: its packed R takes 66 KB of LDS, two workgroups per CU,
// and 128-row chunks would need 1024 lanes per workgroup and leave one.
#ifndef H2_QR32_NT
#define H2_QR32_NT 256
#endif
#ifndef H2_QR64_NT
#define H2_QR64_NT 512
#endif
#ifndef H2_QR32_CH
#define H2_QR32_CH 128
#endif
#ifndef H2_QR64_CH
#define H2_QR64_CH 128
#endif
#ifndef H2_QR128_CH
#define H2_QR128_CH 64
#endif
#ifndef H2_QR128_NT
#define H2_QR128_NT 512
#endif
void launch_qr_class(const QrTask* tasks, int ntasks, int cls, hipStream_t s) {
  if (ntasks <= 0) return;
  // each workgroup exits unless its task's effective width falls into the class
  if (cls == 0)
    hipLaunchKernelGGL((qr_kernel<32, H2_QR32_NT, H2_QR32_CH>), dim3(ntasks), dim3(H2_QR32_NT), 0, s, tasks, 0);
  if (cls == 1)
    hipLaunchKernelGGL((qr_kernel<64, H2_QR64_NT, H2_QR64_CH>), dim3(ntasks), dim3(H2_QR64_NT), 0, s, tasks, 32);
  if (cls == 2)
    hipLaunchKernelGGL((qr_kernel<128, H2_QR128_NT, H2_QR128_CH>), dim3(ntasks), dim3(H2_QR128_NT), 0, s, tasks, 64);
}

void launch_qr(const QrTask* tasks, int ntasks, int wmax, hipStream_t s) {
  for (int c = 0; c < size_classes(wmax); ++c) launch_qr_class(tasks, ntasks, c, s);
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD (left vectors).
// ---------------------------------------------------------------------------
// Sum over the workgroup (result in every thread): wave shuffles, then one
// exchange of the per-wave sums through LDS.
// (red holds NT / 16 entries)
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  v = dpp_group_sum(v, 16);
  __syncthreads();
  if ((threadIdx.x & 15) == 0) red[threadIdx.x >> 4] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NT / 16; ++w) t += red[w];
  return t;
}

// Sum over the G consecutive lanes of a group (G a power of two <= 16).
template <int G>
__device__ inline double group_sum(double v) {
  static_assert(G <= 16, "groups within a DPP row");
  return dpp_group_sum(v, G);
}

// Sweeps of one-sided Jacobi on the columns of M (M[c * LD + r], rows x
// cols) with round-robin pair ordering.  The G consecutive lanes of a group
// share a pair: each lane keeps its K rows of both columns in registers
// between the three dot products and the rotation.  One barrier per round.
// Returns the number of sweeps (at most maxsw; the last one without rotations
// unless the cap was reached: then *sh_rot is still set on return).
template <int WMAX, int NT, int G>
__device__ inline int jacobi_sweeps(double* M, int rows, int cols, int* sh_rot, int maxsw) {
  constexpr int LD = WMAX + 1;
  constexpr int K = (WMAX + G - 1) / G;
  const int tid = threadIdx.x;
  const int np = (cols + 1) & ~1;  // players incl. a dummy when cols is odd
  const int npairs = np / 2, m1 = np - 1;
  const int grp = tid / G, gl = tid % G;
  int sweeps = 0;
  for (int sweep = 0; sweep < maxsw && np > 1; ++sweep) {
    if (tid == 0) *sh_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < m1; ++rnd) {
      for (int g = grp; g < npairs; g += NT / G) {
        int p, q;
        if (g == 0) {
          p = m1;
          q = rnd;
        } else {
          p = rnd + g;
          if (p >= m1) p -= m1;
          q = rnd - g;
          if (q < 0) q += m1;
        }
        if (p >= cols || q >= cols) continue;  // the dummy player (whole group)
        double* cp = M + p * LD;
        double* cq = M + q * LD;
        double x[K], y[K];
        double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int r = gl + k * G;
          x[k] = r < rows ? cp[r] : 0.0;
          y[k] = r < rows ? cq[r] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          a += x[k] * x[k];
          b += y[k] * y[k];
          c += x[k] * y[k];
        }
        a = dpp_group_sum(a, G);
        b = dpp_group_sum(b, G);
        c = dpp_group_sum(c, G);
        if (c != 0.0 && c * c > 1e-30 * (a * b)) {
          // tan of the rotation angle: sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
          // zeta = (b - a) / 2c; c^2 > 0 keeps 2c normal.  Above 1e150,
          // sqrt(1 + zeta^2) is |zeta| in FP64 (and zeta^2 may overflow).
          const double zeta = (b - a) * rcp_nr(2.0 * c);
          const double az = fabs(zeta), u = 1.0 + zeta * zeta;
          const double root = az > 1e150 ? az : u * rsq_nr(u);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(az + root);
          const double cs = rsq_nr(1.0 + t * t), sn = cs * t;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int r = gl + k * G;
            if (r < rows) {
              cp[r] = cs * x[k] - sn * y[k];
              cq[r] = sn * x[k] + cs * y[k];
            }
          }
          if (gl == 0) *sh_rot = 1;
        }
      }
      __syncthreads();
    }
    ++sweeps;
    if (!*sh_rot) break;
    __syncthreads();
  }
  return sweeps;
}

// Truncated SVD (left singular vectors) of a small matrix A (rows x cols).
//
// With an absolute threshold tau (coarsening and basis truncations) the rank
// is revealed first by a column-pivoted Householder QR of X = A^T, stopped
// once the remaining columns have Frobenius norm <= tau/8.  Column l of X
// (row l of A) lives in the registers of the TPC consecutive lanes of group l
// (lane `sub` holds rows sub, sub + TPC, ...), so pivoting moves no data: a
// pivoted column is only marked done.  Each step costs two barriers (the
// pivot reduction and the publication of the reflector).  The r x cols factor
// R, transposed to rows x r, then goes to one-sided Jacobi at threshold
// 3 tau / 4; the projection error stays below tau (tau/8 + 3 tau/4).
// Without such a threshold A itself goes to the Jacobi.
//
// Jacobi: M[c * LD + r] holds column c (contiguous rows); the odd stride keeps
// lanes that read different columns on different LDS banks.
//
// RMAX < WMAX gives the narrow first pass of a size class: LDS for RMAX
// revealed columns only (two workgroups per CU instead of one) and the
// reflector re-read from LDS instead of held in registers.  A matrix whose
// rank reveal would go past RMAX columns is left to the full kernel: the
// narrow pass writes rank -1, and the full kernel, launched after it with
// `deferred` set, takes exactly those matrices.
template <int WMAX, int NT, int RMAX>
__device__ __forceinline__ void svd_task(const SvdTask& tk, int* overflow, int wlo, int deferred) {
  constexpr bool NARROW = RMAX < WMAX;
  constexpr int LD = WMAX + 1;
  constexpr int TPC = NT / WMAX;  // lanes per column of A^T in the rank reveal
  constexpr int RPL = WMAX / TPC; // rows per lane
  constexpr int NR = NT / 16;     // DPP rows of the workgroup
  constexpr int NW = NT / 64;     // waves of the workgroup
  static_assert(TPC >= 1 && (TPC & (TPC - 1)) == 0 && NT % 64 == 0, "launch shape");
  __shared__ double M[RMAX * LD];
  __shared__ double nrm[WMAX], snrm[WMAX], inv[WMAX];
  __shared__ int order[WMAX];
  constexpr int VS = RPL + 2;  // padded run per lane: the TPC runs start on different LDS banks
  __shared__ double vb[TPC * VS];  // reflector, lane-major: vb[sub * VS + q] is row sub + TPC q
  __shared__ double red[NR], wmx[NR];
  __shared__ int widx[NR];
  __shared__ int sh_rot, sh_keep;
  __shared__ double sh_tau, sh_scal;
  const bool sq = tk.w_dev || tk.w_dev2;
  const int we = eff_width(tk.cols, tk.w_dev, tk.w_dev2);
  const int rows = sq ? we : tk.rows;
  int cols = sq ? we : tk.cols;
  const int wcls = rows > cols ? rows : cols;
  // another launch handles this size class; the smallest class also takes
  // empty tasks (both children of rank 0), which report rank 0 and zero vectors
  if ((wlo > 0 && wcls <= wlo) || wcls > WMAX) return;
  if (deferred && *tk.rank != -1) return;  // finished by the narrow pass
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double ref = tk.tol_ptr ? tk.tol_scale * *tk.tol_ptr : 0.0;
  const bool qr = tk.qrcp && tk.tol_rel == 0.0;
  if (NARROW && !qr) {  // the whole matrix would go to the Jacobi
    if (tid == 0) *tk.rank = -1;
    return;
  }
  bool defer = false;
  const int cols_in = cols;
  int sweeps = 0;
  double jthr_scale = 1.0;
  bool empty;
  if (!qr) {
    double ss = 0.0;
    for (int e = tid; e < cols * WMAX; e += NT) {
      int c = e / WMAX, r = e - c * WMAX;
      double v = 0.0;
      if (r < rows) v = tk.trans_a ? tk.a[(int64_t)c * tk.lda + r] : tk.a[(int64_t)r * tk.lda + c];
      M[c * LD + r] = v;
      ss += v * v;
    }
    const double fro = sqrt(block_sum<NT>(ss, red));
    // every singular value is below the Frobenius norm: nothing survives an
    // absolute threshold above it
    empty = cols == 0 || ((tk.tol_rel == 0.0) && (fro <= tk.tol_abs + ref));
  } else {
    const int nl = rows, ni = cols;
    const int l = tid / TPC, sub = tid % TPC;
    double x[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int i = sub + TPC * q;
      double v = 0.0;
      if (l < nl && i < ni) v = tk.trans_a ? tk.a[(int64_t)i * tk.lda + l] : tk.a[(int64_t)l * tk.lda + i];
      x[q] = v;
    }
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) ss += x[q] * x[q];
    const double cn0 = group_sum<TPC>(ss);  // squared norm of this column
    const double fro = sqrt(block_sum<NT>(ss, red));
    empty = cols == 0 || fro <= tk.tol_abs + ref;
    if (!empty) {
      const double tq = 0.125 * (tk.tol_abs + ref);
      double cn = cn0;   // squared norm of the rows below the current step
      int done = -1;     // step at which this column was the pivot
      int r = 0;
      const int jmax = nl < ni ? nl : ni;
      // The registers hold a window of rows: lane sub keeps rows
      // j0 + sub + TPC q (j0 = j rounded down to a multiple of TPC), so row j
      // sits in x[0] of lane j % TPC.  A finished row leaves the registers
      // (its R entry goes straight to M, the register is zeroed), and every
      // TPC steps the window moves on; sums and updates then run over all
      // registers without per-row predicates.
      for (int j = 0; j < jmax; ++j) {
        const int sj = j % TPC;
        if (j > 0 && sj == 0) {
#pragma unroll
          for (int q = 0; q + 1 < RPL; ++q) x[q] = x[q + 1];
          x[RPL - 1] = 0.0;
        }
        // remaining Frobenius norm and pivot (largest column, lowest index on
        // ties): DPP within rows of 16 lanes, lane shuffles across the four
        // rows of a wave, then the NW wave results through LDS
        const bool act = l < nl && done < 0;
        double v = act ? cn : -1.0, sv = (act && sub == 0) ? cn : 0.0;
        int id = act ? l : WMAX;
        sv = dpp_group_sum(sv, 16);
        {
          double ov = dpp_mov<0xB1>(v);
          int oi = dpp_mov_int<0xB1>(id);
          if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }
          ov = dpp_mov<0x4E>(v);
          oi = dpp_mov_int<0x4E>(id);
          if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }
          ov = dpp_mov<0x141>(v);
          oi = dpp_mov_int<0x141>(id);
          if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }
          ov = dpp_mov<0x140>(v);
          oi = dpp_mov_int<0x140>(id);
          if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }
#pragma unroll
          for (int off = 16; off < 64; off <<= 1) {
            sv += __shfl_xor(sv, off);
            ov = __shfl_xor(v, off);
            oi = __shfl_xor(id, off);
            if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }
          }
        }
        if (lane == 0) {
          red[wv] = sv;
          wmx[wv] = v;
          widx[wv] = id;
        }
        __syncthreads();
        double tot = 0.0, bv = -1.0;
        int p = WMAX;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          tot += red[w];
          if (wmx[w] > bv || (wmx[w] == bv && widx[w] < p)) {
            bv = wmx[w];
            p = widx[w];
          }
        }
        if (tot <= tq * tq) break;
        if (NARROW && j >= RMAX) {
          defer = true;
          break;
        }
        r = j + 1;
        if (l == p) {  // reflector of the pivot column on rows >= j
          const double xj = group_sum<TPC>(sub == sj ? x[0] : 0.0);
          if (sub == sj) x[0] = 0.0;
          double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < RPL; ++q) s4[q & 3] += x[q] * x[q];
          const double x2 = group_sum<TPC>((s4[0] + s4[1]) + (s4[2] + s4[3]));
          double tau = 0.0, scal = 0.0, beta = xj;
          if (x2 != 0.0) {
            const double nn = sqrt(xj * xj + x2);
            beta = xj >= 0.0 ? -nn : nn;
            tau = (beta - xj) / beta;
            scal = 1.0 / (xj - beta);
          }
#pragma unroll
          for (int q = 0; q < RPL; ++q) vb[sub * VS + q] = x[q];
          if (sub == 0) {
            sh_tau = tau;
            sh_scal = scal;
            M[j * LD + l] = beta;
          }
          done = j;
        }
        __syncthreads();
        if (l < nl && done < 0) {  // apply to the remaining columns
          const double tau = sh_tau, scal = sh_scal;
          const double xj = group_sum<TPC>(sub == sj ? x[0] : 0.0);
          double rjl = xj;  // R entry of row j
          if (tau != 0.0) {
            double d4[4] = {0.0, 0.0, 0.0, 0.0};
            if constexpr (NARROW) {
#pragma unroll
              for (int q = 0; q < RPL; ++q) d4[q & 3] += vb[sub * VS + q] * x[q];
              const double dot = group_sum<TPC>((d4[0] + d4[1]) + (d4[2] + d4[3]));
              const double full = xj + scal * dot;
              const double f = tau * scal * full;
              __asm__ volatile("" ::: "memory");  // read the reflector again: no registers held across the sum
#pragma unroll
              for (int q = 0; q < RPL; ++q) x[q] -= f * vb[sub * VS + q];
              rjl = xj - tau * full;
            } else {
              double w[RPL];
#pragma unroll
              for (int q = 0; q < RPL; ++q) {
                w[q] = vb[sub * VS + q];
                d4[q & 3] += w[q] * x[q];
              }
              const double dot = group_sum<TPC>((d4[0] + d4[1]) + (d4[2] + d4[3]));
              const double full = xj + scal * dot;
              const double f = tau * scal * full;
#pragma unroll
              for (int q = 0; q < RPL; ++q) x[q] -= f * w[q];
              rjl = xj - tau * full;
            }
          }
          if (sub == 0) M[j * LD + l] = rjl;
          if (sub == sj) x[0] = 0.0;
          double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < RPL; ++q) s4[q & 3] += x[q] * x[q];
          cn = group_sum<TPC>((s4[0] + s4[1]) + (s4[2] + s4[3]));
        }
      }
      // Jacobi matrix (nl x r): column i, row l = R[i][l], written step by
      // step above; a pivoted column has no entries below its step
      if (l < nl && done >= 0)
        for (int i = done + 1 + sub; i < r; i += TPC) M[i * LD + l] = 0.0;
      cols = r;
      jthr_scale = 0.75;
    }
    __syncthreads();
    if (defer) {  // uniform: every thread took the same break
      if (tid == 0) *tk.rank = -1;
      return;
    }
  }
  if (!empty) {
    // G lanes per pair, at most a DPP row of 16, all pairs of a round at once
    // (2 TPC lanes per pair always fit: at most WMAX / 2 pairs)
    const int npairs = ((cols + 1) & ~1) / 2;
    const int maxsw = tk.maxsw > 0 ? tk.maxsw : 40;
    if constexpr (NARROW) {
      static_assert(RMAX / 2 * 16 <= NT, "narrow pass: 16 lanes for every pair");
      sweeps = jacobi_sweeps<WMAX, NT, 16>(M, rows, cols, &sh_rot, maxsw);
    } else {
      if (npairs * 16 <= NT) sweeps = jacobi_sweeps<WMAX, NT, 16>(M, rows, cols, &sh_rot, maxsw);
      else if (npairs * 8 <= NT) sweeps = jacobi_sweeps<WMAX, NT, 8>(M, rows, cols, &sh_rot, maxsw);
      else sweeps = jacobi_sweeps<WMAX, NT, (2 * TPC < 8 ? 2 * TPC : 8)>(M, rows, cols, &sh_rot, maxsw);
    }
    // still rotating after the cap: the columns are not yet orthogonal, so
    // they are not singular vectors (read after the last round's barrier)
    if (sweeps >= maxsw && cols > 1 && sh_rot && tid == 0 && overflow) atomicOr(overflow, kOvfNotConverged);
  }
  if (tk.stat && tid == 0) {
    tk.stat[0] = rows;
    tk.stat[1] = cols_in;
    tk.stat[2] = empty ? 0 : cols;
    tk.stat[3] = sweeps;
  }
  const int c_all = sq ? we : tk.cols;  // number of singular values reported
  // column norms, 16 lanes per column
  for (int c = tid / 16; c < c_all; c += NT / 16) {
    double v = 0.0;
    if (!empty && c < cols)
      for (int r = tid % 16; r < rows; r += 16) v += M[c * LD + r] * M[c * LD + r];
    v = dpp_group_sum(v, 16);
    if (tid % 16 == 0) nrm[c] = sqrt(v);
  }
  if (tid == 0) sh_keep = c_all;
  __syncthreads();
  // descending order (ties by index); snrm holds the sorted values
  for (int c = tid; c < c_all; c += NT) {
    int rk = 0;
    const double v = nrm[c];
#pragma unroll 8
    for (int d = 0; d < c_all; ++d) {
      const double w = nrm[d];
      rk += (w > v) || (w == v && d < c);
    }
    order[rk] = c;
    snrm[rk] = v;
  }
  __syncthreads();
  const double smax = c_all > 0 ? snrm[0] : 0.0;
  const double thr = jthr_scale * (tk.tol_abs + tk.tol_rel * smax + ref);
  int keep = 0;
  if (!tk.frob) {
#pragma unroll 8
    for (int i = 0; i < c_all; ++i) keep += snrm[i] > thr;
  } else {
    // fewest kept values whose dropped tail has Frobenius norm <= thr: the
    // tail sums s_i (accumulated from the smallest value up) grow as i
    // falls, and keep is the smallest i with s_i <= thr^2
    const double thr2 = thr * thr;
    for (int i = tid; i < c_all; i += NT) {
      double tail = 0.0;
#pragma unroll 8
      for (int d = c_all - 1; d >= i; --d) tail += snrm[d] * snrm[d];
      if (tail <= thr2) atomicMin(&sh_keep, i);
    }
    __syncthreads();
    keep = sh_keep;
  }
  if (keep > tk.kcap) {
    if (tid == 0 && overflow) atomicOr(overflow, tk.ovf_bit);
    keep = tk.kcap;
  }
  const int sc = sq ? tk.cols : c_all;
  for (int i = tid; i < sc; i += NT) tk.sigma[i] = i < c_all ? snrm[i] : 0.0;
  if (tid == 0) *tk.rank = keep;
  for (int i = tid; i < keep; i += NT) inv[i] = 1.0 / snrm[i];
  __syncthreads();
  // kept normalised columns; lanes run along the columns of U (coalesced rows)
  const int kc = tk.kcap;
  for (int i0 = 0; i0 < kc; i0 += 64) {
    const int i = i0 + lane;
    const bool kept = i < keep;
    const int off = kept ? order[i] * LD : 0;
    const double s = kept ? inv[i] : 0.0;
    if (i < kc) {
      if (!tk.u2) {
        const int ur = sq ? tk.rows : rows;
        for (int r = wv; r < ur; r += NW) tk.u[(int64_t)r * tk.ldu + i] = (kept && r < rows) ? M[off + r] * s : 0.0;
      } else {
        const int split = tk.split_dev ? *tk.split_dev : 0;
        for (int r = wv; r < tk.urows; r += NW) {
          tk.u[(int64_t)r * tk.ldu + i] = (kept && r < split && r < rows) ? M[off + r] * s : 0.0;
          tk.u2[(int64_t)r * tk.ldu + i] = (kept && split + r < rows) ? M[off + split + r] * s : 0.0;
        }
      }
    }
  }
}

template <int WMAX, int NT>
__global__ __launch_bounds__(NT) void svd_kernel(const SvdTask* __restrict__ tasks, int* overflow, int wlo,
                                                 int deferred) {
  svd_task<WMAX, NT, WMAX>(tasks[blockIdx.x], overflow, wlo, deferred);
}

// two workgroups per CU: 4 waves per SIMD at NT = 512, at most 128 VGPRs
template <int WMAX, int NT, int RMAX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void svd_narrow_kernel(const SvdTask* __restrict__ tasks, int* overflow, int wlo) {
  svd_task<WMAX, NT, RMAX>(tasks[blockIdx.x], overflow, wlo, 0);
}

void launch_svd_class(const SvdTask* tasks, int ntasks, int cls, int* overflow, hipStream_t s) {
  if (ntasks <= 0) return;
  if (cls == 0) hipLaunchKernelGGL((svd_kernel<32, 64>), dim3(ntasks), dim3(64), 0, s, tasks, overflow, 0, 0);
  if (cls == 1) hipLaunchKernelGGL((svd_kernel<64, 256>), dim3(ntasks), dim3(256), 0, s, tasks, overflow, 32, 0);
  if (cls == 2) {
    // Narrow pass, then the full kernel for the matrices it left (rank -1).
    // A launch of fewer matrices leaves CUs idle anyway; there the narrow
    // pass would only repeat the rank reveal of the matrices it defers.
    const bool narrow = ntasks >= 1024;
    if (narrow)
      hipLaunchKernelGGL((svd_narrow_kernel<128, 512, 64>), dim3(ntasks), dim3(512), 0, s, tasks, overflow, 64);
    hipLaunchKernelGGL((svd_kernel<128, 512>), dim3(ntasks), dim3(512), 0, s, tasks, overflow, 64, narrow ? 1 : 0);
  }
}

void launch_svd(const SvdTask* tasks, int ntasks, int wmax, int* overflow, hipStream_t s) {
  for (int c = 0; c < size_classes(wmax); ++c) launch_svd_class(tasks, ntasks, c, overflow, s);
}

// ---------------------------------------------------------------------------
// Scaled Cholesky orthonormalisation step.
// ---------------------------------------------------------------------------
// One wave per task; lane l owns column l.  H holds the scaled Gram matrix,
// then the upper Cholesky factor U in its upper triangle; the inverse
// X = U^-1 is built in the strict lower triangle (X[i][l] at H[l][i]) with
// its diagonal in xd.  Every loop runs over a row or column index shared by
// all lanes (a lane outside the range is idle), so the LDS reads of U are
// broadcasts and consecutive iterations are independent.
template <int WMAX>
__global__ __launch_bounds__(64) void chol_kernel(const CholTask* __restrict__ tasks) {
  __shared__ double H[WMAX][WMAX + 1];
  __shared__ double d[WMAX], xd[WMAX];
  const CholTask tk = tasks[blockIdx.x];
  const int w = tk.w, l = threadIdx.x;
  const int we = tk.weff ? min(*tk.weff, w) : w;
  if (l < w) {
    const double g = (l < we) ? gload(tk.g + (int64_t)l * tk.ldg + l) : 0.0;
    d[l] = g > 0.0 ? sqrt(g) : 0.0;
  }
  wave_sync();
  if (l < w) {
    const double dl = d[l];
    for (int i = 0; i < w; ++i) {
      double v = 0.0;
      if (i < we && l < we) {
        if (d[i] > 0.0 && dl > 0.0) v = gload(tk.g + (int64_t)i * tk.ldg + l) / (d[i] * dl);
        else v = (i == l) ? 1.0 : 0.0;
      } else if (i == l) {
        v = 1.0;
      }
      H[i][l] = v;
    }
  }
  wave_sync();
  // right-looking Cholesky of the leading we x we block (identity beyond)
  for (int j = 0; j < we; ++j) {
    const double piv = sqrt(fmax(H[j][j], 1e-300));
    if (l >= j && l < we) H[j][l] = (l == j) ? piv : H[j][l] / piv;
    wave_sync();
    if (l > j && l < we) {
      const double ujl = H[j][l];
      for (int i = j + 1; i <= l; ++i) H[i][l] -= H[j][i] * ujl;
    }
    wave_sync();
  }
  // X = U^-1, row by row from the bottom: X[i][l] = (delta_il - sum_{k=i+1..l} U[i][k] X[k][l]) / U[i][i]
  for (int i = we - 1; i >= 0; --i) {
    if (l >= i && l < we) {
      double s = (i == l) ? 1.0 : 0.0;
      for (int k = i + 1; k <= l; ++k) s -= H[i][k] * (k == l ? xd[l] : H[l][k]);
      const double x = s / H[i][i];
      if (i == l) xd[l] = x;
      else H[l][i] = x;
    }
  }
  wave_sync();
  if (l < w) {
    const double dl = d[l];
    for (int i = 0; i < w; ++i) {
      const bool in = i < we && l < we && l >= i;
      double tv = 0.0, rv = 0.0;
      if (in) {
        tv = d[i] > 0.0 ? (i == l ? xd[l] : H[l][i]) / d[i] : 0.0;
        rv = H[i][l] * dl;
      }
      tk.t[(int64_t)i * tk.ldt + l] = tv;
      tk.r[(int64_t)i * tk.ldr + l] = rv;
    }
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
// Largest row or column norm over the task's matrices, each times its scale
// (a 1 x 1 matrix gives its value: a norm bound or a largest singular value
// computed earlier).  A matrix of at most
// 128 columns is read once, row by row: the lanes of a wave cover a row (two
// coalesced loads), a wave reduction gives its norm, and each lane keeps the
// sums of its two columns (combined over the four waves in LDS).  Wider
// matrices take the plain per-thread loops.
__global__ __launch_bounds__(256) void ref_kernel(const RefTask* __restrict__ tasks, const RefMat* __restrict__ mats) {
  __shared__ double red[256];
  __shared__ double cols4[4][128];
  const RefTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double best = 0.0;
  for (int q = 0; q < tk.count; ++q) {
    const RefMat m = mats[tk.first + q];
    double bm = 0.0;  // largest squared row or column norm of this matrix
    if (m.cols <= 128) {
      const bool in0 = lane < m.cols, in1 = lane + 64 < m.cols;
      double c0 = 0.0, c1 = 0.0;
      for (int r = wv; r < m.rows; r += 4) {
        const double* row = m.a + (int64_t)r * m.lda;
        const double x0 = in0 ? gload(row + lane) : 0.0;
        const double x1 = in1 ? gload(row + lane + 64) : 0.0;
        c0 += x0 * x0;
        c1 += x1 * x1;
        double s = x0 * x0 + x1 * x1;
        s = dpp_group_sum(s, 16);
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        bm = fmax(bm, s);
      }
      cols4[wv][lane] = c0;
      cols4[wv][lane + 64] = c1;
      __syncthreads();
      if (tid < 128) bm = fmax(bm, (cols4[0][tid] + cols4[1][tid]) + (cols4[2][tid] + cols4[3][tid]));
      __syncthreads();
    } else {
      for (int r = tid; r < m.rows; r += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < m.cols; ++c) {
          const double x = m.a[(int64_t)r * m.lda + c];
          s += x * x;
        }
        bm = fmax(bm, s);
      }
      for (int c = tid; c < m.cols; c += blockDim.x) {
        double s = 0.0;
        for (int r = 0; r < m.rows; ++r) {
          const double x = m.a[(int64_t)r * m.lda + c];
          s += x * x;
        }
        bm = fmax(bm, s);
      }
    }
    best = fmax(best, bm * (m.scale * m.scale));
  }
  red[tid] = best;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
    __syncthreads();
  }
  if (tid == 0) *tk.out = tk.factor * sqrt(red[0]);
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

__global__ void axpby_kernel(const double* x, double* y, int64_t n, double a, double b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}
void launch_axpby(const double* x, double* y, int64_t n, double a, double b, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks), dim3(256), 0, s, x, y, n, a, b);
}

// Grid-stride partial sums; each workgroup reduces its lanes (DPP rows, lane
// shuffles, then LDS over the four waves) into partial[blockIdx.x].
__global__ __launch_bounds__(256) void dot_kernel(const double* x, const double* y, int64_t n, double* partial) {
  __shared__ double red[4];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) v += x[i] * y[i];
  v = dpp_group_sum(v, 16);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
void launch_dot(const double* x, const double* y, int64_t n, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(kDotBlocks), dim3(256), 0, s, x, y, n, partial);
}

__global__ void scan_kernel(const ScanTask* __restrict__ tasks, const int* const* __restrict__ src, int ntasks) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  const ScanTask tk = tasks[t];
  int acc = 0;
  for (int i = 0; i < tk.count; ++i) {
    tk.offs[i] = acc;
    acc += *src[tk.first + i];
  }
  *tk.total = acc;
}
void launch_scan(const ScanTask* tasks, const int* const* src, int ntasks, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(scan_kernel, dim3((ntasks + 63) / 64), dim3(64), 0, s, tasks, src, ntasks);
}

const char* kernel_name(int id) {
  static const char* names[K_COUNT] = {
      "gemm_kernel<double>",       "gemm_kernel<float>",         "qr_kernel<32, 256, 128>",
      "qr_kernel<64, 512, 128>",   "qr_kernel<128, 512, 64>",    "svd_kernel<32, 64>",
      "svd_kernel<64, 256>",       "svd_narrow_kernel<128, 512, 64> + svd_kernel<128, 512>",       "chol_kernel",
      "fill_kernel",               "convert kernels",            "ref_kernel",
      "scan_kernel"};
  return (id >= 0 && id < K_COUNT) ? names[id] : "";
}

}  // namespace h2k

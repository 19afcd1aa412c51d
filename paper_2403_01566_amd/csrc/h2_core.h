// Host-side structures of the H2 product library: cluster/block trees,
// resident H2-matrices, the product plan (integer work lists) and its
// executor.  All floating-point work of the product runs in h2_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <tuple>
#include <memory>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/h2.h"
#include "h2_kernels.h"

namespace h2 {

struct Error : std::runtime_error {
  h2_status code;
  Error(h2_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define H2_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      if (e_ == hipErrorOutOfMemory)                                                          \
        throw ::h2::Error(H2_ERR_OUT_OF_MEMORY, std::string(#call) + ": " + hipGetErrorString(e_)); \
      throw ::h2::Error(H2_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));    \
    }                                                                                         \
  } while (0)

// ---------------------------------------------------------------- trees
struct Tree {
  int64_t n = 0;
  int dim = 0, leaf_size = 0, ncl = 0, depth = 0;
  std::vector<double> pts;        // original points, n x dim
  std::vector<int64_t> perm;      // tree position -> original index
  std::vector<int64_t> begin, end;
  std::vector<int> parent, level;
  std::vector<std::vector<int>> children;
  std::vector<double> lo, hi;     // ncl x dim bounding boxes
  int64_t size(int t) const { return end[t] - begin[t]; }
  bool leaf(int t) const { return children[t].empty(); }
  double diam(int t) const;
  double dist(int t, int s) const;
  double diam2(int t) const;  // squared, without fused multiply-add (see the admissibility test)
};

std::shared_ptr<Tree> build_tree(const double* pts, int64_t n, int dim, int leaf_size);

enum BlockKind : int { BK_ADM = 0, BK_INADM = 1, BK_SPLIT = 2 };

struct BlockTree {
  const Tree* rows = nullptr;
  const Tree* cols = nullptr;
  double eta = 0;
  struct Node {
    int t, s, kind;
    int child0, nchild;  // children in `nodes`
    int leaf_index;      // index among adm (kind ADM) or inadm (kind INADM) leaves
    int depth;
  };
  std::vector<Node> nodes;
  std::vector<int> adm, inadm;           // node indices of leaves
  std::map<std::pair<int, int>, int> index;
  int find(int t, int s) const {
    auto it = index.find({t, s});
    return it == index.end() ? -1 : it->second;
  }
};

void build_block_tree(BlockTree& bt, const Tree& rows, const Tree& cols, double eta);

// ---------------------------------------------------------------- device memory
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t b);
  void release();
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

struct Context;

// A cluster basis in padded layout: leaf rows of all leaves in one n x kc
// array (tree order), transfers ncl x kc x kc (E[t]: k_t x k_parent, i.e.
// V_parent restricted to t equals V_t E_t), ranks per cluster.
struct BasisDev {
  double* leaf = nullptr;
  double* transfer = nullptr;
  float* leaf32 = nullptr;
  float* transfer32 = nullptr;
};

struct Matrix {
  Context* ctx = nullptr;
  std::shared_ptr<Context> hold;  // keeps the context (stream, plan cache) alive
  ~Matrix();
  std::shared_ptr<Tree> rows, cols;
  BlockTree bt;
  int kc = 0;             // rank cap (= operand rank for interpolated matrices)
  bool w_is_v = false;    // column basis identical to row basis
  BasisDev V, W;
  double* S = nullptr;    // n_adm x kc x kc couplings
  double* N = nullptr;    // packed nearfield
  float* S32 = nullptr;
  float* N32 = nullptr;
  std::vector<int64_t> noff;  // per inadm leaf offset into N
  int64_t nsize = 0;
  std::vector<int> rank_row, rank_col;  // host copies
  std::vector<std::unique_ptr<DevBuf>> bufs;
  bool has32 = false;
  uint64_t id = 0;
  double* alloc64(size_t count);
  float* alloc32(size_t count);
  void ensure_fp32(hipStream_t s);
};

struct Plan;
struct MvPlan;

// Where a plan executes: a stream, two more streams (default priority) for
// the size classes of one QR or SVD step, fork and join events and the
// device flag the rank-capped kernels set on an overflow.
struct Lane {
  hipStream_t stream = nullptr;
  hipStream_t aux[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
  int* overflow = nullptr;
};
// An extra lane of the context (lane 0 is the context's own stream): its
// streams and events, and overflow flags used round-robin by its jobs.
struct LaneRes {
  Lane l;
  int* flags = nullptr;         // kFlagSlots device ints
  std::vector<int> free_slots;  // flags not held by a job that is still to be waited for
  int inflight = 0;
  DevBuf arena;        // workspaces of the product plans bound to this lane
  int nplans = 0;      // plans bound to this lane
  uint64_t epoch = 0;  // changes whenever the arena is (re)allocated
};
constexpr int kFlagSlots = 64;

// Device, stream and plan cache.  Shared by the context handle and every
// matrix created in it, so handles may be released in any order.
struct Context {
  int device = 0;
  hipStream_t stream = nullptr;
  // two more streams (default priority) for the size classes of one QR or SVD
  // step, which are independent launches; fork and join events
  hipStream_t aux[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
  int* overflow = nullptr;  // device flag set by rank-cap overflows
  std::map<std::pair<uint64_t, uint64_t>, std::shared_ptr<Plan>> plans;
  // operand pairs whose FP32 bulk exceeded a rank cap: largest such eps (those
  // products, and tighter ones, run the bulk in FP64)
  std::map<std::pair<uint64_t, uint64_t>, double> fp32_fail_eps;
  // operand pairs whose products needed the largest result rank cap: later
  // products of the pair start there (one plan, not a plan per cap)
  std::map<std::pair<uint64_t, uint64_t>, int> kc_raised;
  // matrix-vector plans: (matrix id, transposed, number of vectors)
  std::map<std::tuple<uint64_t, int, int64_t>, std::shared_ptr<MvPlan>> mvplans;
  // host parts of the matrix-vector plans of the allocation-free entry point
  std::map<std::tuple<uint64_t, int, int64_t>, std::shared_ptr<MvPlan>> mvhost;
  // lanes for asynchronous products: lanes[0] shares the context's stream
  // (its flags are separate from `overflow`); created by set_lanes
  std::vector<std::unique_ptr<LaneRes>> lanes;
  uint64_t arena_epoch = 0;  // source of LaneRes::epoch values (unique per allocation)
  uint64_t submissions = 0;  // products submitted (the plans' last-use stamps)
  uint64_t mem_limit = 0;    // admission limit on device memory in use (0: the whole device)
  // free device memory as the admission sees it: min(free, limit - in use)
  size_t admissible_free() const;
  Lane lane0() const {
    Lane l;
    l.stream = stream;
    l.aux[0] = aux[0];
    l.aux[1] = aux[1];
    l.fork = fork;
    l.join[0] = join[0];
    l.join[1] = join[1];
    l.overflow = overflow;
    return l;
  }
  void set_lanes(int n);
  uint64_t next_id = 1;
  std::weak_ptr<Context> self;
  ~Context();
  void evict(uint64_t matrix_id);
};

std::unique_ptr<Matrix> build_interpolated(Context* ctx, std::shared_ptr<Tree> rows, std::shared_ptr<Tree> cols,
                                           int kernel, const double* normals, int order, double eta, int diag);

std::unique_ptr<Matrix> multiply(Context* ctx, Matrix* X, Matrix* Y, double eps, const h2_mul_options& opt,
                                 h2_mul_stats* stats);

// Asynchronous products: submit enqueues on a lane and returns; wait
// completes (a rank overflow falls back to multiply); destroy_job waits for
// the device work of a job that is dropped without wait.
struct Job;
Job* submit(Context* ctx, Matrix* X, Matrix* Y, double eps, const h2_mul_options& opt);  // owned by the caller
bool poll(Job& J);
std::unique_ptr<Matrix> wait(Job& J, h2_mul_stats* stats);
void destroy_job(Job* J);

// H -> H2 recompression of an H-matrix on the block tree of (R, C, eta):
// factors U_b (|t| x k_b) and Z_b (|s| x k_b) of the admissible leaves packed
// in leaf order, dense nearfield blocks packed in inadmissible-leaf order
// (host arrays, tree order, row-major).
std::unique_ptr<Matrix> recompress(Context* ctx, std::shared_ptr<Tree> R, std::shared_ptr<Tree> C, double eta,
                                   const int* ranks, const double* U, const double* Z, const double* near,
                                   double eps, const h2_mul_options& opt, h2_mul_stats* stats);

// y = M x (trans = 0) or M^T x (trans = 1) for nrhs vectors, host arrays in
// the original point order, row-major (one vector per column).
void matvec(Matrix* M, int trans, int64_t nrhs, const double* x, double* y);
// The same product with every device buffer of the call inside `scratch`
// (`bytes` long): TOO_LARGE if it does not fit; allocates no device memory.
void matvec_scratch(Matrix* M, int trans, int64_t nrhs, const double* x, double* y, char* scratch, size_t bytes);
// The library's static scratch array of this device (h2_scratch.hip): its
// device address, resolved once per device with that device current, and size.
char* scratch_address(int device);
size_t scratch_bytes();
// Power-iteration estimates of ||XY - C||_2 (C may be null: 0) and ||XY||_2,
// started from z0 (cols(Y) entries, original order).
void product_error(Matrix* X, Matrix* Y, Matrix* C, int iters, const double* z0, double* err, double* nxy);

void to_dense(const Matrix& M, double* out, int64_t ld);
void block_dense(const Matrix& M, int64_t b, double* out);
int selftest(hipStream_t s, int* overflow, double* errors, int nerrors);

}  // namespace h2

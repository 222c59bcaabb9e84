// Internal runtime shared by the berryhip translation units: the context,
// workspace carving, error plumbing and small device helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/berryhip.h"

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Workspace slots: each pipeline stage carves its scratch from its own slot,
// so a stage may call another stage without their scratch overlapping.
enum { WS_EIGH = 0, WS_WILSON = 1, WS_OUTER = 2, WS_MISC = 3, WS_UNIT = 4, WS_SLOTS = 5 };

// Per-name launch timer: hipEvent pairs recorded around launches while
// profiling is on; resolved (synchronously) when queried.
struct ProfEntry {
  double total_ms = 0.0;
  int64_t launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

struct be_ctx {
  int device = 0;
  bool prof_on = false;
  std::map<std::string, ProfEntry> prof;
  std::vector<hipEvent_t> event_pool;
  void *ws[WS_SLOTS] = {};  // device workspaces (grow on demand)
  size_t ws_bytes[WS_SLOTS] = {};
  void *pinned = nullptr;  // small pinned host buffer for scalar read-backs
  std::string err;
  int n_cu = 256;
  // tuning knobs (be_tune_set, be_tune_set_orders)
  int tune_panel_threads = 512;   // threads per matrix of the Householder panel kernel
  int tune_panel_loads = 0;       // loads in flight per lane of the 512-thread FP32 panel (0: by order)
  int dbg_bisect_max_iter = 128;  // bisection steps per eigenvalue after the multisection (a debug cap)
  struct TuneRange {
    int n_lo, n_hi;  // orders N in [n_lo, n_hi]
    int elem;        // bytes per element of the reduction (8: mixed paths, 16: FP64), 0: both
    int value;
  };
  std::vector<TuneRange> tune_panel_ranges;  // per-order panel thread counts (last match wins)
  std::vector<TuneRange> tune_loads_ranges;  // per-order loads in flight (last match wins)
  std::string prof_scope;         // prefix of launch-timer names (nested calls)
};

namespace be {

// Threads per matrix of the Householder panel kernel for order N and element
// size elem (bytes): the last matching per-order setting, else the default.
inline int tune_value(const std::vector<be_ctx::TuneRange> &ranges, int v, int N, size_t elem) {
  for (const auto &r : ranges)
    if (N >= r.n_lo && N <= r.n_hi && (r.elem == 0 || size_t(r.elem) == elem)) v = r.value;
  return v;
}
inline int panel_threads(const be_ctx *ctx, int N, size_t elem) {
  return tune_value(ctx->tune_panel_ranges, ctx->tune_panel_threads, N, elem);
}

// Loads in flight per lane of the panel kernel's matrix-vector product (the
// columns of one transposed column sum): 4 for the FP64 reduction and the
// 256-thread FP32 one, 8 for the 1024-thread FP32 one. The 512-thread FP32
// kernel comes in both forms (4 loads at six waves per SIMD, 8 loads at four,
// the register budget of each): the knob's value for the order, else 8 from
// order kPanelLoads8From on (measured on MI355X: 4 loads faster up to order
// 800, 8 loads from 1024 on, where the larger matrices leave fewer resident
// workgroups to hide the load latency).
constexpr int kPanelLoads8From = 960;
inline int panel_loads(const be_ctx *ctx, int N, size_t elem, int nt) {
  if (elem != 8 || nt == 256) return 4;
  if (nt == 1024) return 8;
  const int v = tune_value(ctx->tune_loads_ranges, ctx->tune_panel_loads, N, elem);
  return v ? v : (N >= kPanelLoads8From ? 8 : 4);
}

// ---------------------------------------------------------------- errors
int set_err(be_ctx *ctx, int code, const std::string &msg);

// A failed HIP call is reported as BE_EHIP; HIP's last-error state is cleared
// so that the caller's next unrelated HIP call does not see it again.
#define BE_HIP_TRY(ctx, expr)                                                         \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) {                                                           \
      (void)hipGetLastError();                                                        \
      return ::be::set_err((ctx), BE_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    }                                                                                 \
  } while (0)

#define BE_CHECK_ARG(ctx, cond, msg)                                    \
  do {                                                                  \
    if (!(cond)) return ::be::set_err((ctx), BE_EINVAL, (msg));         \
  } while (0)

#define BE_RET_IF(rc) \
  do {                \
    int _r = (rc);    \
    if (_r) return _r; \
  } while (0)

// ---------------------------------------------------------------- workspace
// Carves one contiguous device workspace into 256-byte aligned pieces.
// Usage: declare every piece with add(), then call commit() once, then read
// the resolved pointers.
class Carve {
 public:
  template <typename T>
  void add(T **slot, size_t count) {
    slots_.push_back(reinterpret_cast<void **>(slot));
    offs_.push_back(total_);
    total_ += (count * sizeof(T) + 255) & ~size_t(255);
  }
  size_t total() const { return total_; }
  int commit(be_ctx *ctx, hipStream_t stream, int slot);
  // resolve the pointers into caller-provided memory of at least total() bytes
  void place(void *base) {
    char *b = static_cast<char *>(base);
    for (size_t k = 0; k < slots_.size(); ++k) *slots_[k] = b + offs_[k];
  }

 private:
  std::vector<void **> slots_;
  std::vector<size_t> offs_;
  size_t total_ = 0;
};

// ---------------------------------------------------------------- profiling
// RAII scope recording a start/stop event pair on `stream` under `name`
// when profiling is enabled on the context.
class ProfScope {
 public:
  ProfScope(be_ctx *ctx, const char *name, hipStream_t stream);
  ~ProfScope();

 private:
  be_ctx *ctx_;
  std::string name_;
  hipStream_t stream_;
  hipEvent_t start_ = nullptr;
};

void prof_resolve_all(be_ctx *ctx);

// ---------------------------------------------------------------- launches
// Kernel launch error check (after hipLaunchKernelGGL).
int check_launch(be_ctx *ctx, const char *what);

// True while `stream` is being captured into a HIP graph: calls then take no
// host read-back (fixed iteration schedules with per-item predicates) and
// may not grow the workspace.
inline bool stream_capturing(hipStream_t stream) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st == hipStreamCaptureStatusActive;
}

// Number of workgroups for an XCD-aware 1D grid over `work` items: rounded
// up to a multiple of 8 so that item w maps to XCD w / per_xcd.
inline uint32_t xcd_grid(int64_t work) {
  int64_t per = (work + 7) / 8;
  return static_cast<uint32_t>(per * 8);
}

// Linear workgroup id -> work item, so that consecutive work items land on
// the same XCD (workgroups are dealt round-robin over the 8 XCDs).
__device__ __forceinline__ int64_t xcd_work_id(int64_t total) {
  int64_t L = blockIdx.x;
  int64_t per = (total + 7) / 8;
  return (L & 7) * per + (L >> 3);
}

// ---------------------------------------------------------------- complex
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// ---------------------------------------------------------------- batched complex GEMM (internal)
// Element offset of batch item q:
//   (q / (n0*n1)) * s2 + ((q / n0) % n1) * s1 + ((q % n0 + shift) % n0) * s0
// i.e. a three-level index (outer, middle, inner) with a cyclic shift of the
// inner index (used for the closing link of a Wilson loop).
struct ZBatch {
  int64_t s0 = 0, s1 = 0, s2 = 0;
  int32_t n0 = 1, n1 = 1;
  int32_t shift = 0;
  static ZBatch strided(int64_t s) {
    ZBatch b;
    b.s2 = s;
    return b;
  }
  // inner index cyclic over n0 (stride s0, shifted), outer stride s2
  static ZBatch cyclic(int64_t s0, int32_t n0, int32_t shift, int64_t s_outer) {
    ZBatch b;
    b.s0 = s0;
    b.n0 = n0;
    b.shift = shift;
    b.s2 = s_outer;
    return b;
  }
};

__host__ __device__ inline int64_t zbatch_off(const ZBatch &b, int64_t q) {
  int64_t inner = q % b.n0, rest = q / b.n0;
  int64_t mid = rest % b.n1, outer = rest / b.n1;
  inner += b.shift;
  if (inner >= b.n0) inner -= b.n0;
  return outer * b.s2 + mid * b.s1 + inner * b.s0;
}

struct ZGemm {
  int M = 0, N = 0, K = 0;
  int opA = 0, opB = 0;  // 0: none, 1: conjugate transpose
  const double2 *A = nullptr;
  int lda = 0;
  ZBatch bA;
  const double2 *B = nullptr;
  int ldb = 0;
  ZBatch bB;
  double2 *C = nullptr;
  int ldc = 0;
  ZBatch bC;
  double2 alpha = {1.0, 0.0};
  double2 beta = {0.0, 0.0};
  int64_t batch = 0;
  const char *tag = "zgemm";  // profiling label of the call site
  // C (square) is Hermitian and the update keeps it so: only tiles on or
  // below the diagonal are computed, and each strictly lower tile's conjugate
  // transpose is written to the upper triangle (the old upper values are not
  // read), unless herm_mirror is false (callers that read the lower triangle only)
  bool herm = false;
  bool herm_mirror = true;
  // complex products in the four-product form instead of three real products
  // (Gauss): for Hermitian outputs that feed an eigensolver, whose diagonal
  // tiles it keeps bitwise Hermitian with exactly real diagonals
  bool four_mult = false;
  // optional per-item predicate: items with act[q] == 0 are skipped (C left as it is)
  const int *act = nullptr;
  // optional real row scaling of B (opB = 'N' only): op(B_q) = diag(s_q) B_q
  // with s_q = scaleB + (q / scaleB_div) * scaleB_ld, applied as B is loaded
  const double *scaleB = nullptr;
  int64_t scaleB_div = 1, scaleB_ld = 0;
};

// C = alpha op(A) op(B) + beta C, FP64 MFMA. C must not alias A or B.
int zgemm(be_ctx *ctx, const ZGemm &g, hipStream_t stream);

// Single-precision complex variant (FP32 MFMA, FP32 accumulation).
struct CGemm {
  int M = 0, N = 0, K = 0;
  int opA = 0, opB = 0;
  const float2 *A = nullptr;
  int lda = 0;
  ZBatch bA;
  const float2 *B = nullptr;
  int ldb = 0;
  ZBatch bB;
  float2 *C = nullptr;
  int ldc = 0;
  ZBatch bC;
  float2 alpha = {1.0f, 0.0f};
  float2 beta = {0.0f, 0.0f};
  int64_t batch = 0;
  const char *tag = "cgemm";
  bool herm = false;  // as in ZGemm
  bool herm_mirror = true;
  bool four_mult = false;  // as in ZGemm
  const int *act = nullptr;  // as in ZGemm
  // products on the bf16 matrix cores with each FP32 operand split into two
  // bf16 parts (three products per real product, ~2^-16 relative error)
  bool bf16x3 = false;
};
int cgemm(be_ctx *ctx, const CGemm &g, hipStream_t stream);

// Real FP64 batched GEMM, op in {0: none, 1: transpose}.
struct DGemm {
  int M = 0, N = 0, K = 0;
  int opA = 0, opB = 0;
  const double *A = nullptr;
  int lda = 0;
  ZBatch bA;
  const double *B = nullptr;
  int ldb = 0;
  ZBatch bB;
  double *C = nullptr;
  int ldc = 0;
  ZBatch bC;
  double alpha = 1.0;
  double beta = 0.0;
  int64_t batch = 0;
  const char *tag = "dgemm";
  bool sym = false;  // C (square) is symmetric: as ZGemm::herm, without conjugation
  const int *act = nullptr;  // as in ZGemm
};
int dgemm(be_ctx *ctx, const DGemm &g, hipStream_t stream);

// Device address of the fixed scratch of the no-allocation entry point for
// `device` (current), looked up once; called by be_create.
int noalloc_scratch_init(be_ctx *ctx, int device);

// Batched eigensolver for bands [band_lo, band_hi) (uses slot WS_EIGH): FP64,
// or mixed (c64 input, FP32 reduction and back-transformation, FP64
// tridiagonal solve and orthonormalization, c128 eigenvectors out).
int eigh_fp64(be_ctx *ctx, double2 *H, int N, int ld, int64_t mat_stride, int64_t n_mat, int band_lo, int band_hi,
              double *evals, double2 *U, int ldu, int64_t u_stride, uint32_t *status, hipStream_t stream,
              double clu_rel = 1e-12);
int eigh_mixed(be_ctx *ctx, float2 *H, int N, int ld, int64_t mat_stride, int64_t n_mat, int band_lo, int band_hi,
               double *evals, double2 *U, int ldu, int64_t u_stride, uint32_t *status, hipStream_t stream,
               bool bf16x3 = false);

}  // namespace be

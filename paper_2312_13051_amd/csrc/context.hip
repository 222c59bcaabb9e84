// Context, error text and workspace management.
#include <algorithm>

#include "common.hpp"

namespace be {

int set_err(be_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int Carve::commit(be_ctx *ctx, hipStream_t stream, int slot) {
  size_t need = std::max<size_t>(total_, 256);
  if (need > ctx->ws_bytes[slot]) {
    if (stream_capturing(stream))
      return set_err(ctx, BE_ENOMEM, "workspace of " + std::to_string(ctx->ws_bytes[slot]) + " bytes too small for a "
                                     "call under graph capture (" + std::to_string(need) + " needed): run the same "
                                     "call once outside capture first (it sizes the workspace)");
    // Growing: wait for work that may still use the old buffer.
    BE_HIP_TRY(ctx, hipStreamSynchronize(stream));
    BE_HIP_TRY(ctx, hipDeviceSynchronize());
    if (ctx->ws[slot]) {
      BE_HIP_TRY(ctx, hipFree(ctx->ws[slot]));
      ctx->ws[slot] = nullptr;
      ctx->ws_bytes[slot] = 0;
    }
    size_t grow = need + need / 8;
    if (hipMalloc(&ctx->ws[slot], grow) != hipSuccess) {
      (void)hipGetLastError();
      ctx->ws[slot] = nullptr;
      return set_err(ctx, BE_ENOMEM, "device workspace allocation of " + std::to_string(grow) + " bytes failed");
    }
    ctx->ws_bytes[slot] = grow;
  }
  char *base = static_cast<char *>(ctx->ws[slot]);
  for (size_t k = 0; k < slots_.size(); ++k) *slots_[k] = base + offs_[k];
  return BE_OK;
}

static hipEvent_t take_event(be_ctx *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(be_ctx *ctx, const char *name, hipStream_t stream) : ctx_(ctx), stream_(stream) {
  if (!ctx_ || !ctx_->prof_on) return;
  name_ = ctx_->prof_scope + name;
  start_ = take_event(ctx_);
  if (start_) (void)hipEventRecord(start_, stream_);
}

ProfScope::~ProfScope() {
  if (!start_) return;
  hipEvent_t stop = take_event(ctx_);
  if (!stop) return;
  (void)hipEventRecord(stop, stream_);
  ctx_->prof[name_].pending.emplace_back(start_, stop);
}

static void prof_resolve(be_ctx *ctx) {
  for (auto &kv : ctx->prof) {
    for (auto &pr : kv.second.pending) {
      float ms = 0.f;
      if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        kv.second.total_ms += ms;
        kv.second.launches += 1;
      }
      ctx->event_pool.push_back(pr.first);
      ctx->event_pool.push_back(pr.second);
    }
    kv.second.pending.clear();
  }
}

int check_launch(be_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, BE_EHIP, std::string("launch of ") + what + ": " + hipGetErrorString(e));
  return BE_OK;
}

void prof_resolve_all(be_ctx *ctx) { prof_resolve(ctx); }

}  // namespace be

extern "C" {

int be_create(be_ctx **ctx, int device) {
  if (!ctx) return BE_EINVAL;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return BE_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return BE_EHIP;
  be_ctx *c = new be_ctx();
  c->device = device;
  if (hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return BE_ENOMEM;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  const int rc = be::noalloc_scratch_init(c, device);
  if (rc != BE_OK) {
    (void)hipHostFree(c->pinned);
    delete c;
    return rc;
  }
  *ctx = c;
  return BE_OK;
}

int be_destroy(be_ctx *ctx) {
  if (!ctx) return BE_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  be::prof_resolve_all(ctx);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  for (int k = 0; k < WS_SLOTS; ++k)
    if (ctx->ws[k]) (void)hipFree(ctx->ws[k]);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return BE_OK;
}

const char *be_last_error(const be_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t be_workspace_bytes(const be_ctx *ctx) {
  if (!ctx) return 0;
  size_t t = 0;
  for (int k = 0; k < WS_SLOTS; ++k) t += ctx->ws_bytes[k];
  return t;
}

int be_profile_enable(be_ctx *ctx, int on) {
  if (!ctx) return BE_EINVAL;
  be::prof_resolve(ctx);
  ctx->prof.clear();
  ctx->prof_on = on != 0;
  return BE_OK;
}

int be_profile_query(be_ctx *ctx, const char *name, double *total_ms, int64_t *launches) {
  if (!ctx || !name || !total_ms || !launches) return BE_EINVAL;
  be::prof_resolve(ctx);
  auto it = ctx->prof.find(name);
  *total_ms = it == ctx->prof.end() ? 0.0 : it->second.total_ms;
  *launches = it == ctx->prof.end() ? 0 : it->second.launches;
  return BE_OK;
}

namespace {
// The tunable knobs: default value, per-order settings, accepted values.
struct Knob {
  int *value;
  std::vector<be_ctx::TuneRange> *ranges;
  int reset;
  bool (*ok)(int);
  const char *allowed;
};
bool find_knob(be_ctx *ctx, const std::string &k, Knob *kn) {
  if (k == "hetrd_panel_threads") {
    *kn = {&ctx->tune_panel_threads, &ctx->tune_panel_ranges, 512,
           [](int v) { return v == 256 || v == 512 || v == 1024; }, "hetrd_panel_threads takes 256, 512 or 1024"};
    return true;
  }
  if (k == "hetrd_panel_loads") {
    *kn = {&ctx->tune_panel_loads, &ctx->tune_loads_ranges, 0, [](int v) { return v == 0 || v == 4 || v == 8; },
           "hetrd_panel_loads takes 0 (by order), 4 or 8"};
    return true;
  }
  if (k == "tri_bisect_max_iter") {  // a debug cap (forces BE_ST_NONCONVERGED), no per-order settings
    *kn = {&ctx->dbg_bisect_max_iter, nullptr, 128, [](int v) { return v >= 1 && v <= 128; },
           "tri_bisect_max_iter takes 1 .. 128"};
    return true;
  }
  return false;
}
}  // namespace

int be_tune_set(be_ctx *ctx, const char *knob, int32_t value) {
  if (!ctx || !knob) return BE_EINVAL;
  Knob kn;
  if (!find_knob(ctx, knob, &kn)) return be::set_err(ctx, BE_EINVAL, std::string("unknown tuning knob: ") + knob);
  BE_CHECK_ARG(ctx, kn.ok(value), kn.allowed);
  *kn.value = value;
  return BE_OK;
}

int be_tune_set_orders(be_ctx *ctx, const char *knob, int32_t n_lo, int32_t n_hi, int32_t precision, int32_t value) {
  if (!ctx || !knob) return BE_EINVAL;
  Knob kn;
  if (!find_knob(ctx, knob, &kn)) return be::set_err(ctx, BE_EINVAL, std::string("unknown tuning knob: ") + knob);
  BE_CHECK_ARG(ctx, kn.ranges != nullptr, std::string("be_tune_set_orders: ") + knob + " has no per-order settings");
  BE_CHECK_ARG(ctx, kn.ok(value), kn.allowed);
  BE_CHECK_ARG(ctx, 1 <= n_lo && n_lo <= n_hi, "be_tune_set_orders: need 1 <= n_lo <= n_hi");
  BE_CHECK_ARG(ctx, precision == -1 || precision == BE_FP64 || precision == BE_MIXED_FP32 ||
                        precision == BE_MIXED_FP32_REFINED,
               "be_tune_set_orders: precision must be -1, BE_FP64, BE_MIXED_FP32 or BE_MIXED_FP32_REFINED");
  const int elem = precision == -1 ? 0 : precision == BE_FP64 ? 16 : 8;
  kn.ranges->push_back({n_lo, n_hi, elem, value});
  return BE_OK;
}

int be_tune_clear(be_ctx *ctx, const char *knob) {
  if (!ctx || !knob) return BE_EINVAL;
  Knob kn;
  if (!find_knob(ctx, knob, &kn)) return be::set_err(ctx, BE_EINVAL, std::string("unknown tuning knob: ") + knob);
  if (kn.ranges) kn.ranges->clear();
  *kn.value = kn.reset;
  return BE_OK;
}

int be_tune_get(be_ctx *ctx, const char *knob, int32_t *value) {
  if (!ctx || !knob || !value) return BE_EINVAL;
  Knob kn;
  if (!find_knob(ctx, knob, &kn)) return be::set_err(ctx, BE_EINVAL, std::string("unknown tuning knob: ") + knob);
  *value = *kn.value;
  return BE_OK;
}

int be_profile_names(be_ctx *ctx, char *buf, size_t len) {
  if (!ctx || !buf || len == 0) return BE_EINVAL;
  be::prof_resolve(ctx);
  std::string s;
  for (auto &kv : ctx->prof) {
    if (!s.empty()) s += ",";
    s += kv.first;
  }
  size_t n = std::min(len - 1, s.size());
  std::copy(s.begin(), s.begin() + n, buf);
  buf[n] = 0;
  return BE_OK;
}

}  // extern "C"

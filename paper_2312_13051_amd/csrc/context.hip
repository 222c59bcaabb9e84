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

int check_launch(be_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(ctx, BE_EHIP, std::string("launch of ") + what + ": " + hipGetErrorString(e));
  return BE_OK;
}

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
  *ctx = c;
  return BE_OK;
}

int be_destroy(be_ctx *ctx) {
  if (!ctx) return BE_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
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

}  // extern "C"

// Rows (a1) and (a2): hopping list -> device plan -> Bloch Hamiltonians.
//
// The host packer merges duplicate keys, checks Hermiticity and keeps the
// upper triangle grouped into (row, col) pairs, sorted by column then row,
// so that consecutive threads of the scatter kernel write consecutive rows of
// one column. The device side is two kernels per call: a zero fill of every
// matrix and a phase-weighted scatter with one thread per (pair, matrix):
//   H[r, c] = sum_e t_e exp(2 pi i kappa . R_e),  H[c, r] = conj(H[r, c]).
// The diagonal is written with an exactly zero imaginary part, so H is
// bitwise Hermitian, and each element is summed by one thread in a fixed
// order, so the result is deterministic.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "hk_pack.hpp"

static_assert(sizeof(be::hkpack::PairRC) == sizeof(int2) && sizeof(be::hkpack::EntR) == sizeof(int4) &&
                  sizeof(be::hkpack::EntT) == sizeof(double2),
              "packed host arrays are uploaded as int2 / int4 / double2");

struct be_hk_plan {
  int device = 0;
  int n_sys = 0;
  std::vector<int32_t> N;        // per system
  std::vector<int32_t> dim;      // per system
  std::vector<int64_t> pair_off; // per system, into pair arrays
  std::vector<int32_t> n_pairs;  // per system
  int64_t total_pairs = 0;
  int64_t total_ents = 0;
  int2 *d_pair_rc = nullptr;      // (row, col), row <= col
  int32_t *d_pair_start = nullptr;// entry start per pair (+1 sentinel per system, global index)
  int4 *d_ent_R = nullptr;        // R (x, y, z, 0)
  double2 *d_ent_t = nullptr;     // amplitude
  // per-system descriptors on the device
  int32_t *d_sys_dim = nullptr;
  int64_t *d_sys_pair_off = nullptr;
  int32_t *d_sys_npairs = nullptr;
};

namespace {

__global__ void hk_zero_c128(double2 *H, int64_t stride, int32_t ld, int32_t N, int64_t n_k) {
  int64_t per = int64_t(N) * N;
  int64_t q = blockIdx.y;
  for (; q < n_k; q += gridDim.y) {
    double2 *Hq = H + q * stride;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < per; e += int64_t(gridDim.x) * blockDim.x) {
      int64_t c = e / N, r = e - c * N;
      Hq[r + c * ld] = make_double2(0.0, 0.0);
    }
  }
}

__global__ void hk_zero_c64(float2 *H, int64_t stride, int32_t ld, int32_t N, int64_t n_k) {
  int64_t per = int64_t(N) * N;
  int64_t q = blockIdx.y;
  for (; q < n_k; q += gridDim.y) {
    float2 *Hq = H + q * stride;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < per; e += int64_t(gridDim.x) * blockDim.x) {
      int64_t c = e / N, r = e - c * N;
      Hq[r + c * ld] = make_float2(0.f, 0.f);
    }
  }
}

// Sum of t exp(2 pi i kappa.R) over the entries of one pair; the phase
// argument is reduced to [-1/2, 1/2] before sincospi.
__device__ __forceinline__ double2 pair_sum(const int32_t *start, int64_t p, const int4 *R, const double2 *t,
                                            double k0, double k1, double k2, int dim) {
  double2 acc = make_double2(0.0, 0.0);
  int32_t e0 = start[p], e1 = start[p + 1];
  for (int32_t e = e0; e < e1; ++e) {
    int4 r = R[e];
    double x = k0 * r.x;
    if (dim > 1) x = fma(k1, double(r.y), x);
    if (dim > 2) x = fma(k2, double(r.z), x);
    x -= rint(x);
    double s, c;
    sincospi(2.0 * x, &s, &c);
    double2 te = t[e];
    acc.x = fma(te.x, c, fma(-te.y, s, acc.x));
    acc.y = fma(te.x, s, fma(te.y, c, acc.y));
  }
  return acc;
}

template <typename OUT>
__device__ __forceinline__ void put(OUT *Hq, int64_t idx, double2 v);
template <>
__device__ __forceinline__ void put<double2>(double2 *Hq, int64_t idx, double2 v) { Hq[idx] = v; }
template <>
__device__ __forceinline__ void put<float2>(float2 *Hq, int64_t idx, double2 v) {
  Hq[idx] = make_float2(float(v.x), float(v.y));
}

template <typename OUT>
__global__ void hk_scatter(OUT *H, int64_t stride, int32_t ld, int32_t sys_first, const double *kappa, int32_t n_kap,
                           int64_t n_mat, const int2 *pair_rc, const int32_t *pair_start, const int4 *ent_R,
                           const double2 *ent_t, const int32_t *sys_dim, const int64_t *sys_pair_off,
                           const int32_t *sys_npairs) {
  for (int64_t q = blockIdx.y; q < n_mat; q += gridDim.y) {
    int s = sys_first + static_cast<int>(q / n_kap);
    int k = static_cast<int>(q % n_kap);
    int np = sys_npairs[s];
    int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= np) continue;
    p += sys_pair_off[s];
    int2 rc = pair_rc[p];
    double2 v = pair_sum(pair_start, p, ent_R, ent_t, kappa[3 * k], kappa[3 * k + 1], kappa[3 * k + 2], sys_dim[s]);
    OUT *Hq = H + q * stride;
    if (rc.x == rc.y) {
      v.y = 0.0;
      put<OUT>(Hq, rc.x + int64_t(rc.y) * ld, v);
    } else {
      put<OUT>(Hq, rc.x + int64_t(rc.y) * ld, v);
      put<OUT>(Hq, rc.y + int64_t(rc.x) * ld, be::cconj(v));
    }
  }
}

}  // namespace

extern "C" {

int be_hk_plan_create(be_ctx *ctx, const be_hoplist *sys_h, int32_t n_sys, be_hk_plan **plan) {
  using namespace be;
  BE_CHECK_ARG(ctx, ctx && sys_h && plan && n_sys > 0, "be_hk_plan_create: null argument or n_sys <= 0");
  *plan = nullptr;
  auto *P = new be_hk_plan();
  P->device = ctx->device;
  P->n_sys = n_sys;
  be::hkpack::Packed pk;
  for (int s = 0; s < n_sys; ++s) {
    const be_hoplist &h = sys_h[s];
    int32_t np = 0;
    const std::string why = be::hkpack::pack_system(h.N, h.dim, h.nnz, h.i, h.j, h.R, h.t, pk, &np);
    if (!why.empty()) {
      delete P;
      return set_err(ctx, BE_EINVAL, "be_hk_plan_create: system " + std::to_string(s) + ": " + why);
    }
    P->N.push_back(h.N);
    P->dim.push_back(h.dim);
    P->pair_off.push_back(static_cast<int64_t>(pk.rc.size()) - np);
    P->n_pairs.push_back(np);
  }
  pk.start.push_back(static_cast<int32_t>(pk.R.size()));
  P->total_pairs = static_cast<int64_t>(pk.rc.size());
  P->total_ents = static_cast<int64_t>(pk.R.size());
  auto up = [&](void **dst, const void *src, size_t bytes) -> int {
    size_t b = std::max<size_t>(bytes, 16);
    if (hipMalloc(dst, b) != hipSuccess) return BE_ENOMEM;
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return BE_EHIP;
    return BE_OK;
  };
  int rc = 0;
  rc |= up(reinterpret_cast<void **>(&P->d_pair_rc), pk.rc.data(), pk.rc.size() * sizeof(int2));
  rc |= up(reinterpret_cast<void **>(&P->d_pair_start), pk.start.data(), pk.start.size() * sizeof(int32_t));
  rc |= up(reinterpret_cast<void **>(&P->d_ent_R), pk.R.data(), pk.R.size() * sizeof(int4));
  rc |= up(reinterpret_cast<void **>(&P->d_ent_t), pk.t.data(), pk.t.size() * sizeof(double2));
  rc |= up(reinterpret_cast<void **>(&P->d_sys_dim), P->dim.data(), P->dim.size() * sizeof(int32_t));
  rc |= up(reinterpret_cast<void **>(&P->d_sys_pair_off), P->pair_off.data(), P->pair_off.size() * sizeof(int64_t));
  rc |= up(reinterpret_cast<void **>(&P->d_sys_npairs), P->n_pairs.data(), P->n_pairs.size() * sizeof(int32_t));
  if (rc) {
    be_hk_plan_destroy(P);
    return set_err(ctx, BE_ENOMEM, "be_hk_plan_create: device upload failed");
  }
  *plan = P;
  return BE_OK;
}

int be_hk_plan_destroy(be_hk_plan *P) {
  if (!P) return BE_EINVAL;
  (void)hipSetDevice(P->device);
  void *ptrs[] = {P->d_pair_rc, P->d_pair_start, P->d_ent_R, P->d_ent_t, P->d_sys_dim, P->d_sys_pair_off, P->d_sys_npairs};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete P;
  return BE_OK;
}

int32_t be_hk_plan_N(const be_hk_plan *P, int32_t s) {
  if (!P || s < 0 || s >= P->n_sys) return -1;
  return P->N[s];
}

int be_build_hk(be_ctx *ctx, const be_hk_plan *P, int32_t sys_first, int32_t n_sys_call, const double *kappa,
                int32_t n_kap, void *H, int64_t mat_stride, int32_t ld, int32_t dtype, hipStream_t stream) {
  using namespace be;
  BE_CHECK_ARG(ctx, ctx && P && kappa && H, "be_build_hk: null argument");
  BE_CHECK_ARG(ctx, n_kap >= 0 && n_sys_call >= 0, "be_build_hk: negative count");
  BE_CHECK_ARG(ctx, sys_first >= 0 && sys_first + n_sys_call <= P->n_sys, "be_build_hk: system range out of the plan");
  BE_CHECK_ARG(ctx, dtype == BE_C128 || dtype == BE_C64, "be_build_hk: dtype must be BE_C128 or BE_C64");
  if (n_kap == 0 || n_sys_call == 0) return BE_OK;
  int32_t N = P->N[sys_first], maxp = 0;
  for (int32_t s = sys_first; s < sys_first + n_sys_call; ++s) {
    BE_CHECK_ARG(ctx, P->N[s] == N, "be_build_hk: all systems of one call must have the same N");
    maxp = std::max(maxp, P->n_pairs[s]);
  }
  BE_CHECK_ARG(ctx, ld >= N, "be_build_hk: ld < N");
  BE_CHECK_ARG(ctx, mat_stride >= int64_t(ld) * N, "be_build_hk: mat_stride < ld*N");
  int64_t n_mat = int64_t(n_sys_call) * n_kap;
  int64_t per = int64_t(N) * N;
  dim3 zb(256), zg(static_cast<uint32_t>(std::min<int64_t>((per + 255) / 256, 4096)),
                   static_cast<uint32_t>(std::min<int64_t>(n_mat, 65535)));
  dim3 sb(256), sg(static_cast<uint32_t>(std::max(1, (maxp + 255) / 256)), static_cast<uint32_t>(std::min<int64_t>(n_mat, 65535)));
  ProfScope prof(ctx, "hk_build", stream);
  if (dtype == BE_C128) {
    hipLaunchKernelGGL(hk_zero_c128, zg, zb, 0, stream, static_cast<double2 *>(H), mat_stride, ld, N, n_mat);
    BE_RET_IF(check_launch(ctx, "hk_zero"));
    hipLaunchKernelGGL(hk_scatter<double2>, sg, sb, 0, stream, static_cast<double2 *>(H), mat_stride, ld, sys_first, kappa,
                       n_kap, n_mat, P->d_pair_rc, P->d_pair_start, P->d_ent_R, P->d_ent_t, P->d_sys_dim,
                       P->d_sys_pair_off, P->d_sys_npairs);
  } else {
    hipLaunchKernelGGL(hk_zero_c64, zg, zb, 0, stream, static_cast<float2 *>(H), mat_stride, ld, N, n_mat);
    BE_RET_IF(check_launch(ctx, "hk_zero"));
    hipLaunchKernelGGL(hk_scatter<float2>, sg, sb, 0, stream, static_cast<float2 *>(H), mat_stride, ld, sys_first, kappa,
                       n_kap, n_mat, P->d_pair_rc, P->d_pair_start, P->d_ent_R, P->d_ent_t, P->d_sys_dim,
                       P->d_sys_pair_off, P->d_sys_npairs);
  }
  return check_launch(ctx, "hk_scatter");
}

}  // extern "C"

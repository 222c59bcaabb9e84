// Rows (a6)-(a10): overlaps, polar factors, ordered products, eigenphases,
// Chern winding, nested Wilson loop and spin-resolved Wilson loop.
//
// Every stage works on "grids": matrix (line, j) of a grid lives at
// base + (line * n_loop + j) * stride, with j running along the closed loop.
//   overlaps      F_{line,j} = U_{line,j+1}^H U_{line,j}      (batched MFMA GEMM,
//                 the closing link via a cyclic batch index)
//   polar         X <- X (3 I - X^H X) / 2  (Newton-Schulz, FP64 MFMA GEMMs),
//                 iterated to convergence of max |X^H X - I|; the limit is the
//                 unitary polar factor of F for every nonsingular F with
//                 singular values in (0, sqrt 3), which holds since ||F|| <= 1
//   chain         W_line = F_{n-1} ... F_0 as a binary tree of batched GEMMs
//                 that keeps the left-to-right order
//   eigenphases   one wave per W: Householder reduction to Hessenberg form,
//                 then single-shift complex QR with Wilkinson shifts; a
//                 subdiagonal entry is negligible below 32 eps times its two
//                 diagonal neighbours (the level to which a product of polar
//                 factors is unitary: phases that close are not separated
//                 further, and deflating changes W's eigenvalues, W being
//                 normal, by no more than that)
//   winding       Phi_i = sum theta mod 2pi, C = (1/2pi) sum wrap(dPhi)
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "common.hpp"

namespace {

constexpr double TWO_PI = 6.283185307179586476925286766559;

struct Grid {
  const double2 *base;
  int ld;
  int64_t stride;
};

__device__ __forceinline__ double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

__device__ __forceinline__ double2 csqrt_d(double2 z) {
  double r = hypot(z.x, z.y);
  if (r == 0.0) return make_double2(0.0, 0.0);
  double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
  return make_double2(fabs(z.y) / (2.0 * t), z.y >= 0.0 ? t : -t);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

__device__ __forceinline__ double wrap_pi(double x) {
  // into (-pi, pi]
  x = x - TWO_PI * floor(x / TWO_PI + 0.5);
  if (x <= -M_PI) x += TWO_PI;
  if (x > M_PI) x -= TWO_PI;
  return x;
}

__device__ __forceinline__ double arg_pi(double2 z) {
  double t = atan2(z.y, z.x);
  return t <= -M_PI ? M_PI : t;
}

// ---------------------------------------------------------------- small kernels
__global__ void k_zero_u32(uint32_t *p, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Newton-Schulz polar iteration with a state per matrix (act): 1 iterating,
// 2 taking its last step, 0 done. One step is G = X^H X, then k_ns_prep
// (G <- 1.5 I - 0.5 G, err = max |G - I| before it, and the next state: done
// without a step once err < 1e-30; a last step once err < 1e-7, which leaves
// about (3/4) err^2 < 1e-14), then X_new = X G and k_ns_post. Matrices in
// state 0 are skipped by both GEMMs, so each matrix stops at its own
// convergence. loc[q] records which of the two buffers holds matrix q's
// latest iterate. tpm threads per matrix (64 for m*m <= 64: four matrices per
// block of 256; else 256: one matrix per block).
__global__ void k_ns_prep(double2 *G, int m, int64_t n_mat, int tpm, double *err, int *act) {
  const int per_blk = blockDim.x / tpm;
  const int sub = threadIdx.x / tpm, t = threadIdx.x % tpm;
  const int64_t q = int64_t(blockIdx.x) * per_blk + sub;
  const bool live = q < n_mat && act[q] != 0;  // uniform over the matrix's threads
  double e = 0.0;
  if (live) {
    double2 *Gq = G + q * int64_t(m) * m;
    for (int k = t; k < m * m; k += tpm) {
      int r = k % m, c = k / m;
      double2 g = Gq[k];
      double dr = g.x - (r == c ? 1.0 : 0.0);
      e = fmax(e, fmax(fabs(dr), fabs(g.y)));
      Gq[k] = make_double2((r == c ? 1.5 : 0.0) - 0.5 * g.x, -0.5 * g.y);
    }
  }
  for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o, 64));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  double v = e;
  if (tpm != 64) {
    v = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
  }
  if (live && t == 0) {
    if (!(v == v)) v = INFINITY;
    err[q] = v;
    act[q] = v < 1e-30 ? 0 : v < 1e-7 ? 2 : 1;
  }
}

// After the step into buffer `parity`: the matrices that took it have their
// iterate there; those in their last step are done. *n_left (zeroed before)
// counts the matrices still iterating.
__global__ void k_ns_post(int *act, unsigned char *loc, int64_t n, unsigned char parity, int *n_left) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int left = 0;
  if (q < n && act[q] != 0) {
    loc[q] = parity;
    if (act[q] == 2) act[q] = 0;
    else left = 1;
  }
  for (int o = 32; o > 0; o >>= 1) left += __shfl_xor(left, o, 64);
  if ((threadIdx.x & 63) == 0 && left) atomicAdd(n_left, left);
}

__global__ void k_ns_init(int *act, unsigned char *loc, int64_t n) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < n) {
    act[q] = 1;
    loc[q] = 0;
  }
}

__global__ void k_zero_i32(int *p) { *p = 0; }

// dst[q] = src[q] for the matrices whose latest iterate is in src (loc[q] == 1)
__global__ void k_copy_mats_loc(const double2 *src, double2 *dst, int64_t mm, int64_t n, const unsigned char *loc) {
  int64_t q = blockIdx.y;
  for (; q < n; q += gridDim.y) {
    if (!loc[q]) continue;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < mm; k += int64_t(gridDim.x) * blockDim.x)
      dst[q * mm + k] = src[q * mm + k];
  }
}

// status[line] |= bit where err of any of the line's n_loop matrices > tol
__global__ void k_flag_err(const double *err, int64_t n_lines, int n_loop, double tol, uint32_t bit, uint32_t *st) {
  int64_t line = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (line >= n_lines) return;
  for (int j = 0; j < n_loop; ++j)
    if (!(err[line * n_loop + j] <= tol)) {
      st[line] |= bit;
      break;
    }
}

__global__ void k_copy_mats(const double2 *src, int64_t s_src, double2 *dst, int64_t s_dst, int64_t count, int64_t n) {
  int64_t q = blockIdx.y;
  for (; q < n; q += gridDim.y)
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < count; k += int64_t(gridDim.x) * blockDim.x)
      dst[q * s_dst + k] = src[q * s_src + k];
}

// Chain-tree carry: dst[line*n_dst + n_dst - 1] = src[line*n_src + n_src - 1]
__global__ void k_carry_last(const double2 *src, int n_src, double2 *dst, int n_dst, int64_t mm, int64_t n_lines) {
  int64_t line = blockIdx.y;
  for (; line < n_lines; line += gridDim.y) {
    const double2 *s = src + (line * n_src + n_src - 1) * mm;
    double2 *d = dst + (line * n_dst + n_dst - 1) * mm;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < mm; k += int64_t(gridDim.x) * blockDim.x) d[k] = s[k];
  }
}

// ---------------------------------------------------------------- unitary eigenproblem
// One 64-lane workgroup per matrix. W: m x m (ld m). H: scratch m x m. Z: optional
// Schur vectors (m x m). Outputs: theta_sorted[q*ldt + 0..m-1] ascending in
// (-pi, pi]; theta_raw[q*m + n] (optional) = phase of the eigenvalue belonging
// to column n of Z.
// INLDS: the whole m x m matrix is held in LDS (orders up to 100, no
// eigenvectors): every access of the reduction and of the QR sweeps is an LDS
// access instead of a dependent global round trip.
template <bool INLDS>
__global__ __launch_bounds__(64) void k_unitary_eig(const double2 *W, int m, int64_t n_mat, double2 *Hs,
                                                    double2 *Zs, double *theta_sorted, int ldt, double *theta_raw,
                                                    uint32_t *flags, int flag_div, const int *act) {
  extern __shared__ double2 sv[];  // Householder vector (m), eigenvalues (m), [INLDS: the matrix (m x m)]
  double2 *slam = sv + m;
  const int64_t q = blockIdx.x;
  if (q >= n_mat || (act && act[q] == 0)) return;
  const int lane = threadIdx.x;
  const double2 *Wq = W + q * int64_t(m) * m;
  double2 *H = INLDS ? slam + m : Hs + q * int64_t(m) * m;
  if (INLDS) Zs = nullptr;
  double2 *Z = Zs ? Zs + q * int64_t(m) * m : nullptr;
  for (int k = lane; k < m * m; k += 64) {
    H[k] = Wq[k];
    if (Z) Z[k] = make_double2((k % m) == (k / m) ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const double eps = DBL_EPSILON;
  // ---- Hessenberg reduction: H <- P^H H P, P = I - tau v v^H
  for (int k = 0; k + 2 < m; ++k) {
    double xn = 0.0;
    for (int r = k + 2 + lane; r < m; r += 64) {
      double2 a = H[r + int64_t(k) * m];
      xn = fma(a.x, a.x, fma(a.y, a.y, xn));
    }
    for (int o = 32; o > 0; o >>= 1) xn += __shfl_xor(xn, o, 64);
    double2 alpha = H[(k + 1) + int64_t(k) * m];
    double2 tau, scal;
    double beta;
    if (xn == 0.0 && alpha.y == 0.0) {
      tau = make_double2(0.0, 0.0);
      scal = make_double2(0.0, 0.0);
      beta = alpha.x;
    } else {
      double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn);
      beta = alpha.x >= 0.0 ? -nrm : nrm;
      tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
      scal = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
    }
    __syncthreads();
    for (int r = lane; r < m; r += 64) {
      double2 v;
      if (r <= k) v = make_double2(0.0, 0.0);
      else if (r == k + 1) v = make_double2(1.0, 0.0);
      else v = be::cmul(H[r + int64_t(k) * m], scal);
      sv[r] = v;
    }
    __syncthreads();
    for (int r = k + 1 + lane; r < m; r += 64) H[r + int64_t(k) * m] = r == k + 1 ? make_double2(beta, 0.0) : make_double2(0.0, 0.0);
    if (tau.x != 0.0 || tau.y != 0.0) {
      const double2 ctau = be::cconj(tau);
      // left: columns k+1..m-1, rows k+1..m-1
      for (int c = k + 1 + lane; c < m; c += 64) {
        double2 s = make_double2(0.0, 0.0);
        for (int r = k + 1; r < m; ++r) s = be::cadd(s, be::cmulc(sv[r], H[r + int64_t(c) * m]));
        double2 f = be::cmul(ctau, s);
        for (int r = k + 1; r < m; ++r) H[r + int64_t(c) * m] = be::csub(H[r + int64_t(c) * m], be::cmul(sv[r], f));
      }
      __syncthreads();
      // right: rows 0..m-1, columns k+1..m-1
      for (int i = lane; i < m; i += 64) {
        double2 s = make_double2(0.0, 0.0);
        for (int c = k + 1; c < m; ++c) s = be::cadd(s, be::cmul(H[i + int64_t(c) * m], sv[c]));
        double2 f = be::cmul(tau, s);
        for (int c = k + 1; c < m; ++c) H[i + int64_t(c) * m] = be::csub(H[i + int64_t(c) * m], be::cmul(f, be::cconj(sv[c])));
        if (Z) {
          double2 sz = make_double2(0.0, 0.0);
          for (int c = k + 1; c < m; ++c) sz = be::cadd(sz, be::cmul(Z[i + int64_t(c) * m], sv[c]));
          double2 fz = be::cmul(tau, sz);
          for (int c = k + 1; c < m; ++c) Z[i + int64_t(c) * m] = be::csub(Z[i + int64_t(c) * m], be::cmul(fz, be::cconj(sv[c])));
        }
      }
    }
    __syncthreads();
  }
  // ---- single-shift QR on the Hessenberg matrix
  const double tol = 32.0 * eps;  // relative to the two diagonal neighbours
  int ihi = m - 1, its = 0, total = 0;
  bool failed = false;
  while (ihi >= 0) {
    int l = 0;
    for (int k = ihi; k >= 1; --k) {
      if (cabs1(H[k + int64_t(k - 1) * m]) <=
          fmax(tol * (cabs1(H[(k - 1) + int64_t(k - 1) * m]) + cabs1(H[k + int64_t(k) * m])), DBL_MIN)) {
        l = k;
        break;
      }
    }
    __syncthreads();
    if (l == ihi) {
      if (lane == 0) {
        slam[ihi] = H[ihi + int64_t(ihi) * m];
        if (ihi > 0) H[ihi + int64_t(ihi - 1) * m] = make_double2(0.0, 0.0);
      }
      --ihi;
      its = 0;
      __syncthreads();
      continue;
    }
    if (l > 0 && lane == 0) H[l + int64_t(l - 1) * m] = make_double2(0.0, 0.0);
    double2 mu;
    const double2 dd = H[ihi + int64_t(ihi) * m];
    // exceptional shifts every 10 steps without a deflation, alternately from
    // the bottom and from the top of the active block (a Wilkinson shift can
    // cycle without converging, e.g. for eigenvalues placed symmetrically
    // about it, which a unitary W can have)
    if (its > 0 && its % 20 == 10) {
      mu = make_double2(dd.x + 0.75 * cabs1(H[ihi + int64_t(ihi - 1) * m]), dd.y);
    } else if (its > 0 && its % 20 == 0) {
      const double2 dl = H[l + int64_t(l) * m];
      mu = make_double2(dl.x + 0.75 * cabs1(H[(l + 1) + int64_t(l) * m]), dl.y);
    } else {
      const double2 a = H[(ihi - 1) + int64_t(ihi - 1) * m], b = H[(ihi - 1) + int64_t(ihi) * m],
                    c = H[ihi + int64_t(ihi - 1) * m];
      const double2 t = make_double2(0.5 * (a.x - dd.x), 0.5 * (a.y - dd.y));
      const double2 disc = csqrt_d(be::cadd(be::cmul(t, t), be::cmul(b, c)));
      const double sgn = (t.x * disc.x + t.y * disc.y) >= 0.0 ? -1.0 : 1.0;
      mu = make_double2(dd.x + t.x + sgn * disc.x, dd.y + t.y + sgn * disc.y);
    }
    __syncthreads();
    for (int k = l; k < ihi; ++k) {
      double2 f, g;
      if (k == l) {
        f = be::csub(H[l + int64_t(l) * m], mu);
        g = H[(l + 1) + int64_t(l) * m];
      } else {
        f = H[k + int64_t(k - 1) * m];
        g = H[(k + 1) + int64_t(k - 1) * m];
      }
      // rotation [c s; -conj(s) c] [f; g] = [r; 0]
      double cr;
      double2 sn, rr;
      const double af = hypot(f.x, f.y), ag = hypot(g.x, g.y);
      if (ag == 0.0) {
        cr = 1.0;
        sn = make_double2(0.0, 0.0);
        rr = f;
      } else if (af == 0.0) {
        cr = 0.0;
        sn = make_double2(g.x / ag, -g.y / ag);
        rr = make_double2(ag, 0.0);
      } else {
        const double nrm = hypot(af, ag);
        const double2 fu = make_double2(f.x / af, f.y / af);
        cr = af / nrm;
        sn = be::cscale(be::cmul(fu, be::cconj(g)), 1.0 / nrm);
        rr = be::cscale(fu, nrm);
      }
      __syncthreads();
      if (k > l && lane == 0) {
        H[k + int64_t(k - 1) * m] = rr;
        H[(k + 1) + int64_t(k - 1) * m] = make_double2(0.0, 0.0);
      }
      // rows k, k+1 over columns k..ihi
      for (int c = k + lane; c <= ihi; c += 64) {
        double2 x = H[k + int64_t(c) * m], y = H[(k + 1) + int64_t(c) * m];
        H[k + int64_t(c) * m] = be::cadd(be::cscale(x, cr), be::cmul(sn, y));
        H[(k + 1) + int64_t(c) * m] = be::csub(be::cscale(y, cr), be::cmul(be::cconj(sn), x));
      }
      __syncthreads();
      // columns k, k+1 over rows l..min(k+2, ihi)
      const int rmax = min(k + 2, ihi);
      for (int r = l + lane; r <= rmax; r += 64) {
        double2 x = H[r + int64_t(k) * m], y = H[r + int64_t(k + 1) * m];
        H[r + int64_t(k) * m] = be::cadd(be::cscale(x, cr), be::cmul(be::cconj(sn), y));
        H[r + int64_t(k + 1) * m] = be::csub(be::cscale(y, cr), be::cmul(sn, x));
      }
      if (Z) {
        for (int r = lane; r < m; r += 64) {
          double2 x = Z[r + int64_t(k) * m], y = Z[r + int64_t(k + 1) * m];
          Z[r + int64_t(k) * m] = be::cadd(be::cscale(x, cr), be::cmul(be::cconj(sn), y));
          Z[r + int64_t(k + 1) * m] = be::csub(be::cscale(y, cr), be::cmul(sn, x));
        }
      }
      __syncthreads();
    }
    ++its;
    ++total;
    if (total > 60 * m + 60) {
      failed = true;
      // take the remaining diagonal as it stands
      for (int r = lane; r <= ihi; r += 64) slam[r] = H[r + int64_t(r) * m];
      __syncthreads();
      break;
    }
  }
  __syncthreads();
  // ---- phases, ascending rank sort
  for (int n = lane; n < m; n += 64) {
    double2 z = slam[n];
    double th = arg_pi(z);
    if (theta_raw) theta_raw[q * m + n] = th;
    int rank = 0;
    for (int k = 0; k < m; ++k) {
      double tk = arg_pi(slam[k]);
      rank += (tk < th) || (tk == th && k < n);
    }
    theta_sorted[q * int64_t(ldt) + rank] = th;
  }
  if (failed && lane == 0) atomicOr(&flags[q / flag_div], BE_ST_NONCONVERGED);
}

// LDS ordering between the lanes of one wave (the wave's LDS operations
// complete in program order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Window of the QR sweep held in LDS: rows and columns rb .. rb + QW - 1.
constexpr int QW = 64, QLD = QW + 1;
constexpr int kUnitaryWgLds = QW * QLD;  // double2 entries of the window

// The same eigenphases for large orders (no Schur vectors): one workgroup of
// NT threads per matrix, H held row-major in global scratch so that the
// reduction's accesses are coalesced: the Householder step's left update
// runs with threads over columns, its right update with a wave per row
// (lanes over columns, wave sums). A QR sweep chases its bulge through
// windows of QW rows and columns copied to LDS: one wave applies the
// window's rotations there (no workgroup barrier per rotation), and the
// parts of those rotations outside the window (the rows' entries to the
// right of it, the columns' entries above it) are applied afterwards by the
// whole workgroup, each thread streaming one column (or row) through the
// window's rotations in order. Shifts and deflation tests are computed
// redundantly by every thread from the same entries, between barriers.
template <int NT>
__global__ __launch_bounds__(NT) void k_unitary_eig_wg(const double2 *W, int m, int64_t n_mat, double2 *Hs,
                                                       double *theta_sorted, int ldt, double *theta_raw,
                                                       uint32_t *flags, int flag_div, const int *act) {
  // Householder vector (m) during the reduction, the QR window (QW x QLD)
  // afterwards; then the eigenvalues (m)
  extern __shared__ double2 sv[];
  double2 *const Bw = sv;
  double2 *slam = sv + max(m, kUnitaryWgLds);
  __shared__ double rot_c[QW];
  __shared__ double2 rot_s[QW];
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  const int64_t q = blockIdx.x;
  if (q >= n_mat || (act && act[q] == 0)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = NT / 64;
  const double2 *Wq = W + q * int64_t(m) * m;
  double2 *H = Hs + q * int64_t(m) * m;  // row-major: H[r * m + c]
  for (int64_t k = tid; k < int64_t(m) * m; k += NT) {
    const int r = int(k % m), c = int(k / m);
    H[int64_t(r) * m + c] = Wq[k];
  }
  __syncthreads();
  auto at = [&](int r, int c) -> double2 & { return H[int64_t(r) * m + c]; };
  auto bsum = [&](double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
  };
  // ---- Hessenberg reduction: H <- P^H H P, P = I - tau v v^H
  for (int k = 0; k + 2 < m; ++k) {
    double xn = 0.0;
    for (int r = k + 2 + tid; r < m; r += NT) {
      const double2 a = at(r, k);
      xn = fma(a.x, a.x, fma(a.y, a.y, xn));
    }
    xn = bsum(xn);
    const double2 alpha = at(k + 1, k);
    double2 tau, scal;
    double beta;
    if (xn == 0.0 && alpha.y == 0.0) {
      tau = make_double2(0.0, 0.0);
      scal = make_double2(0.0, 0.0);
      beta = alpha.x;
    } else {
      const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn);
      beta = alpha.x >= 0.0 ? -nrm : nrm;
      tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
      scal = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
    }
    for (int r = tid; r < m; r += NT) {
      double2 v;
      if (r <= k) v = make_double2(0.0, 0.0);
      else if (r == k + 1) v = make_double2(1.0, 0.0);
      else v = be::cmul(at(r, k), scal);
      sv[r] = v;
    }
    __syncthreads();
    for (int r = k + 1 + tid; r < m; r += NT) at(r, k) = r == k + 1 ? make_double2(beta, 0.0) : make_double2(0.0, 0.0);
    if (tau.x != 0.0 || tau.y != 0.0) {
      const double2 ctau = be::cconj(tau);
      // left: rows k+1..m-1, threads over columns k+1..m-1. Loads are issued
      // HB at a time ahead of their use (the stores of a column's update would
      // otherwise keep each next load waiting: the compiler cannot tell the
      // rows apart)
      constexpr int HB = 8;
      for (int c = k + 1 + tid; c < m; c += NT) {
        double2 sacc = make_double2(0.0, 0.0);
        for (int r0 = k + 1; r0 < m; r0 += HB) {
          double2 a[HB];
#pragma unroll
          for (int u = 0; u < HB; ++u) a[u] = r0 + u < m ? at(r0 + u, c) : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < HB; ++u)
            if (r0 + u < m) sacc = be::cadd(sacc, be::cmulc(sv[r0 + u], a[u]));
        }
        const double2 f = be::cmul(ctau, sacc);
        for (int r0 = k + 1; r0 < m; r0 += HB) {
          double2 a[HB];
#pragma unroll
          for (int u = 0; u < HB; ++u) a[u] = r0 + u < m ? at(r0 + u, c) : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < HB; ++u)
            if (r0 + u < m) at(r0 + u, c) = be::csub(a[u], be::cmul(sv[r0 + u], f));
        }
      }
      __syncthreads();
      // right: every row, columns k+1..m-1: a wave per row, lanes over columns
      for (int i = wave; i < m; i += nw) {
        double sr = 0.0, si = 0.0;
        for (int c = k + 1 + lane; c < m; c += 64) {
          const double2 h = at(i, c), v = sv[c];
          sr += h.x * v.x - h.y * v.y;
          si += h.x * v.y + h.y * v.x;
        }
        for (int o = 32; o > 0; o >>= 1) {
          sr += __shfl_xor(sr, o, 64);
          si += __shfl_xor(si, o, 64);
        }
        const double2 f = be::cmul(tau, make_double2(sr, si));
        for (int c0 = k + 1 + lane; c0 < m; c0 += 64 * 4) {
          double2 a[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) a[u] = c0 + 64 * u < m ? at(i, c0 + 64 * u) : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (c0 + 64 * u < m) at(i, c0 + 64 * u) = be::csub(a[u], be::cmul(f, be::cconj(sv[c0 + 64 * u])));
        }
      }
    }
    __syncthreads();
  }
  // ---- single-shift QR on the Hessenberg matrix
  const double tol = 32.0 * DBL_EPSILON;  // relative to the two diagonal neighbours (as in k_unitary_eig)
  int ihi = m - 1, its = 0, total = 0;
  bool failed = false;
  while (ihi >= 0) {
    // deflation: the largest k <= ihi with a negligible subdiagonal (block max)
    int lk = 0;
    for (int k = 1 + tid; k <= ihi; k += NT)
      if (cabs1(at(k, k - 1)) <= fmax(tol * (cabs1(at(k - 1, k - 1)) + cabs1(at(k, k))), DBL_MIN)) lk = max(lk, k);
    for (int o = 32; o > 0; o >>= 1) lk = max(lk, __shfl_xor(lk, o, 64));
    if (lane == 0) redi[wave] = lk;
    __syncthreads();
    int l = 0;
    for (int w = 0; w < nw; ++w) l = max(l, redi[w]);
    __syncthreads();
    if (l == ihi) {
      if (tid == 0) {
        slam[ihi] = at(ihi, ihi);
        if (ihi > 0) at(ihi, ihi - 1) = make_double2(0.0, 0.0);
      }
      --ihi;
      its = 0;
      __syncthreads();
      continue;
    }
    __syncthreads();
    if (l > 0 && tid == 0) at(l, l - 1) = make_double2(0.0, 0.0);
    double2 mu;
    const double2 dd = at(ihi, ihi);
    // exceptional shifts every 10 steps without a deflation (as in k_unitary_eig)
    if (its > 0 && its % 20 == 10) {
      mu = make_double2(dd.x + 0.75 * cabs1(at(ihi, ihi - 1)), dd.y);
    } else if (its > 0 && its % 20 == 0) {
      const double2 dl = at(l, l);
      mu = make_double2(dl.x + 0.75 * cabs1(at(l + 1, l)), dl.y);
    } else {
      const double2 a = at(ihi - 1, ihi - 1), b = at(ihi - 1, ihi), c = at(ihi, ihi - 1);
      const double2 t = make_double2(0.5 * (a.x - dd.x), 0.5 * (a.y - dd.y));
      const double2 disc = csqrt_d(be::cadd(be::cmul(t, t), be::cmul(b, c)));
      const double sgn = (t.x * disc.x + t.y * disc.y) >= 0.0 ? -1.0 : 1.0;
      mu = make_double2(dd.x + t.x + sgn * disc.x, dd.y + t.y + sgn * disc.y);
    }
    __syncthreads();
    // the sweep's rotations k = l .. ihi-1, window by window: a window holds
    // rows and columns rb .. k1 and takes the rotations k0 <= k < ke whose
    // rows (k, k+1) and column updates (down to row k+2) stay inside it
    for (int k0 = l; k0 < ihi;) {
      const int rb = k0 == l ? l : k0 - 1;
      const int k1 = min(ihi, rb + QW - 1);
      const int ke = k1 == ihi ? ihi : k1 - 1;
      const int nb = k1 - rb + 1;
      auto B = [&](int r, int c) -> double2 & { return Bw[(r - rb) * QLD + (c - rb)]; };
      for (int e = tid; e < nb * nb; e += NT) {
        const int r = rb + e / nb, c = rb + e % nb;
        B(r, c) = at(r, c);
      }
      __syncthreads();
      if (wave == 0) {
        for (int k = k0; k < ke; ++k) {
          double2 f, g;
          if (k == l) {
            f = be::csub(B(l, l), mu);
            g = B(l + 1, l);
          } else {
            f = B(k, k - 1);
            g = B(k + 1, k - 1);
          }
          double cr;
          double2 sn, rr;
          const double af = hypot(f.x, f.y), ag = hypot(g.x, g.y);
          if (ag == 0.0) {
            cr = 1.0;
            sn = make_double2(0.0, 0.0);
            rr = f;
          } else if (af == 0.0) {
            cr = 0.0;
            sn = make_double2(g.x / ag, -g.y / ag);
            rr = make_double2(ag, 0.0);
          } else {
            const double nrm = hypot(af, ag);
            const double2 fu = make_double2(f.x / af, f.y / af);
            cr = af / nrm;
            sn = be::cscale(be::cmul(fu, be::cconj(g)), 1.0 / nrm);
            rr = be::cscale(fu, nrm);
          }
          wave_lds_sync();
          if (lane == 0) {
            rot_c[k - k0] = cr;
            rot_s[k - k0] = sn;
            if (k > l) {
              B(k, k - 1) = rr;
              B(k + 1, k - 1) = make_double2(0.0, 0.0);
            }
          }
          // rows k, k+1 over the window's columns k..k1
          for (int c = k + lane; c <= k1; c += 64) {
            const double2 x = B(k, c), y = B(k + 1, c);
            B(k, c) = be::cadd(be::cscale(x, cr), be::cmul(sn, y));
            B(k + 1, c) = be::csub(be::cscale(y, cr), be::cmul(be::cconj(sn), x));
          }
          wave_lds_sync();
          // columns k, k+1 over the window's rows rb..min(k+2, ihi)
          const int rmax = min(k + 2, ihi);
          for (int r = rb + lane; r <= rmax; r += 64) {
            const double2 x = B(r, k), y = B(r, k + 1);
            B(r, k) = be::cadd(be::cscale(x, cr), be::cmul(be::cconj(sn), y));
            B(r, k + 1) = be::csub(be::cscale(y, cr), be::cmul(sn, x));
          }
          wave_lds_sync();
        }
      }
      __syncthreads();
      for (int e = tid; e < nb * nb; e += NT) {
        const int r = rb + e / nb, c = rb + e % nb;
        at(r, c) = B(r, c);
      }
      // rows k0..ke right of the window: each thread a column, the rotations
      // in order, the column's entries loaded RB at a time ahead of their use
      constexpr int RB = 8;
      for (int c = k1 + 1 + tid; c <= ihi; c += NT) {
        double2 x = at(k0, c);
        for (int kb = k0; kb < ke; kb += RB) {
          double2 y[RB];
#pragma unroll
          for (int u = 0; u < RB; ++u) y[u] = kb + u < ke ? at(kb + u + 1, c) : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            if (kb + u < ke) {
              const double cr = rot_c[kb + u - k0];
              const double2 sn = rot_s[kb + u - k0];
              at(kb + u, c) = be::cadd(be::cscale(x, cr), be::cmul(sn, y[u]));
              x = be::csub(be::cscale(y[u], cr), be::cmul(be::cconj(sn), x));
            }
          }
        }
        at(ke, c) = x;
      }
      // columns k0..ke above the window: each thread a row
      for (int r = l + tid; r < rb; r += NT) {
        double2 x = at(r, k0);
        for (int kb = k0; kb < ke; kb += RB) {
          double2 y[RB];
#pragma unroll
          for (int u = 0; u < RB; ++u) y[u] = kb + u < ke ? at(r, kb + u + 1) : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            if (kb + u < ke) {
              const double cr = rot_c[kb + u - k0];
              const double2 sn = rot_s[kb + u - k0];
              at(r, kb + u) = be::cadd(be::cscale(x, cr), be::cmul(be::cconj(sn), y[u]));
              x = be::csub(be::cscale(y[u], cr), be::cmul(sn, x));
            }
          }
        }
        at(r, ke) = x;
      }
      __syncthreads();
      k0 = ke;
    }
    ++its;
    ++total;
    if (total > 60 * m + 60) {
      failed = true;
      for (int r = tid; r <= ihi; r += NT) slam[r] = at(r, r);
      __syncthreads();
      break;
    }
  }
  __syncthreads();
  // ---- phases, ascending rank sort
  for (int n = tid; n < m; n += NT) {
    const double th = arg_pi(slam[n]);
    if (theta_raw) theta_raw[q * m + n] = th;
    int rank = 0;
    for (int k = 0; k < m; ++k) {
      const double tk = arg_pi(slam[k]);
      rank += (tk < th) || (tk == th && k < n);
    }
    theta_sorted[q * int64_t(ldt) + rank] = th;
  }
  if (failed && tid == 0) atomicOr(&flags[q / flag_div], BE_ST_NONCONVERGED);
}

// ---- eigenphases of large unitary matrices through a Hermitian eigenproblem.
// A = (e^{-i phi} W + e^{i phi} W^H) / 2 is Hermitian, has W's eigenvectors and
// the eigenvalues cos(theta - phi); for an eigenvector v, sin(theta - phi) =
// Im(e^{-i phi} v^H W v). The shift phi keeps pairs theta, -theta (frequent in
// Wilson loops of symmetric models) apart in A's spectrum. Eigenvalues of W
// that still share a cosine (theta_a + theta_b = 2 phi) leave eigenvectors of
// A that are not W's; they show in the residual |W v - e^{i theta} v|, and
// such matrices are handed to the QR kernels.
constexpr double kHermShift = 0.6180339887498949;

// Lower triangle and diagonal of A from W (both column-major m x m), by
// 32 x 32 tile pairs: tile (bj, bi) of W is staged in LDS so that W(c, r) is
// read coalesced for the lower tile (bi, bj).
__global__ __launch_bounds__(256) void k_herm_of_unitary(const double2 *W, int m, int64_t n_mat, double2 *A) {
  __shared__ double2 t[32][33];  // t[col - 32 bi][row - 32 bj] = W(row, col) of tile (bj, bi)
  const int nt = (m + 31) / 32;
  int p = blockIdx.x, bj = 0;
  while (p >= nt - bj) {
    p -= nt - bj;
    ++bj;
  }
  const int bi = bj + p;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double cs = cos(kHermShift), sn = sin(kHermShift);
  const int64_t mm = int64_t(m) * m;
  for (int64_t q = blockIdx.y; q < n_mat; q += gridDim.y) {
    const double2 *Wq = W + q * mm;
    double2 *Aq = A + q * mm;
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
      const int row = bj * 32 + tx, col = bi * 32 + c;
      t[c][tx] = (row < m && col < m) ? Wq[row + int64_t(col) * m] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
      const int r = bi * 32 + tx, cc = bj * 32 + c;
      if (r >= m || cc >= m || r < cc) continue;
      const double2 a = Wq[r + int64_t(cc) * m], b = t[tx][c];  // W(r, cc), W(cc, r)
      // (e^{-i phi} a + e^{i phi} conj(b)) / 2
      double2 v = make_double2(0.5 * (cs * a.x + sn * a.y + cs * b.x + sn * b.y),
                               0.5 * (cs * a.y - sn * a.x - cs * b.y + sn * b.x));
      if (r == cc) v.y = 0.0;
      Aq[r + int64_t(cc) * m] = v;
    }
  }
}

// Phases from the eigenpairs of A. c_n (the eigenvalue, from bisection:
// complete and accurate whatever the vectors) fixes |theta_n - phi| =
// acos(c_n); s_n = Im(e^{-i phi} v_n^H (W v_n)) gives the sign. A vector
// inside a cluster of nearly equal phases may be any mix of the cluster's
// eigenvectors (W matrices of disordered supercells hold hundreds of phases
// within 1e-9 of 0): its s_n keeps the common sign and |s_n| stays at
// sqrt(1 - c_n^2), which is checked (a mix of a pair theta, 2 phi - theta
// would break it). Within 0.05 of the branch points (sin ~ 0), and whenever
// eigenvectors are returned, theta_n = phi + atan2(s_n, c_n) from a vector
// whose residual |W v - e^{i theta} v| must be below 1e-10 (and the
// eigensolver's status clear). Ascending sort; optional raw phases and
// eigenvectors. One workgroup per matrix, a wave per column. fb[q] = 1 where
// the QR kernel must take over.
__global__ __launch_bounds__(256) void k_herm_phases(const double *ev, const uint32_t *est, const double2 *V,
                                                     const double2 *WV, int m, int64_t n_mat, double *theta_sorted,
                                                     int ldt, double *theta_raw, double2 *Zout, int *fb) {
  extern __shared__ double sth[];  // m phases
  __shared__ int s_bad;
  const int64_t q = blockIdx.x;
  if (q >= n_mat) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t mm = int64_t(m) * m;
  const double2 *Vq = V + q * mm, *Gq = WV + q * mm;
  const double cs = cos(kHermShift), sn = sin(kHermShift);
  const bool vectors = Zout != nullptr;
  if (tid == 0) s_bad = (est[q] & (vectors ? ~0u : uint32_t(BE_ST_NAN_INF))) ? 1 : 0;
  __syncthreads();
  for (int n = wave; n < m; n += 4) {
    const double2 *v = Vq + int64_t(n) * m, *g = Gq + int64_t(n) * m;
    double pr = 0.0, pi = 0.0, vv = 0.0;
    for (int r = lane; r < m; r += 64) {
      const double2 a = v[r], b = g[r];
      pr += a.x * b.x + a.y * b.y;
      pi += a.x * b.y - a.y * b.x;
      vv += a.x * a.x + a.y * a.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
      pr += __shfl_xor(pr, o, 64);
      pi += __shfl_xor(pi, o, 64);
      vv += __shfl_xor(vv, o, 64);
    }
    // Im(e^{-i phi} v^H W v) / v^H v (the vectors of a crowd of nearly equal
    // phases need not come out normalized)
    const double s = (cs * pi - sn * pr) / vv;
    const double c = fmin(1.0, fmax(-1.0, ev[q * (m + 2) + 1 + n]));
    const double sabs = sqrt(fmax(0.0, 1.0 - c * c));
    const bool by_cos = !vectors && sabs >= 0.05;
    double th = kHermShift + (by_cos ? copysign(acos(c), s) : atan2(s, c));
    if (th > M_PI) th -= 2.0 * M_PI;
    bool bad = !(th == th);
    if (by_cos) {
      bad = bad || !(fabs(fabs(s) - sabs) <= 1e-3);
    } else {
      const double er = cos(th), ei = sin(th);
      double res = 0.0;
      for (int r = lane; r < m; r += 64) {
        const double2 a = v[r], b = g[r];
        const double dx = b.x - (er * a.x - ei * a.y), dy = b.y - (er * a.y + ei * a.x);
        res += dx * dx + dy * dy;
      }
      for (int o = 32; o > 0; o >>= 1) res += __shfl_xor(res, o, 64);
      bad = bad || !(res <= 1e-20);  // |W v - e^{i theta} v| > 1e-10, or NaN
    }
    if (lane == 0) {
      sth[n] = th;
      if (bad) s_bad = 1;
    }
  }
  __syncthreads();
  for (int n = tid; n < m; n += 256) {
    const double th = sth[n];
    if (theta_raw) theta_raw[q * m + n] = th;
    int rank = 0;
    for (int k = 0; k < m; ++k) {
      const double tk = sth[k];
      rank += (tk < th) || (tk == th && k < n);
    }
    theta_sorted[q * int64_t(ldt) + rank] = th;
  }
  if (Zout)
    for (int64_t k = tid; k < mm; k += 256) Zout[q * mm + k] = Vq[k];
  if (tid == 0) fb[q] = s_bad;
}

// Chern winding of each system from theta [line][ldt] (first m valid).
__global__ void k_winding(const double *theta, int ldt, int m, int n_sys, int n_perp, double *phi, int32_t *winding,
                          uint32_t *status) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  double total = 0.0, dmax = 0.0;
  double prev = 0.0, first = 0.0;
  for (int i = 0; i <= n_perp; ++i) {
    double ph;
    if (i < n_perp) {
      double acc = 0.0;
      const double *th = theta + (int64_t(s) * n_perp + i) * ldt;
      for (int n = 0; n < m; ++n) acc += th[n];
      ph = acc - TWO_PI * floor(acc / TWO_PI);
      if (ph >= TWO_PI) ph -= TWO_PI;
      if (phi) phi[int64_t(s) * n_perp + i] = ph;
      if (i == 0) first = ph;
    } else {
      ph = first;
    }
    if (i > 0) {
      double d = ph - prev;
      d -= TWO_PI * rint(d / TWO_PI);
      total += d;
      dmax = fmax(dmax, fabs(d));
    }
    prev = ph;
  }
  double c = total / TWO_PI;
  int ci = int(rint(c));
  winding[s] = ci;
  if (dmax > 0.8 * M_PI || fabs(c - ci) > 1e-6) atomicOr(&status[s], BE_ST_WINDING_UNRESOLVED);
}

// OR line flags into system flags
__global__ void k_or_lines(const uint32_t *line_st, int64_t n_lines, int per_sys, uint32_t *sys_st) {
  int64_t line = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (line >= n_lines) return;
  uint32_t v = line_st[line];
  if (v) atomicOr(&sys_st[line / per_sys], v);
}

}  // namespace

namespace be {

static int unitary_phases(be_ctx *ctx, const double2 *cur, int m, int64_t n_lines, double2 *Hs, double2 *Zout,
                          double *theta_sorted, int ldt, double *theta_raw, uint32_t *line_status, hipStream_t stream, bool unitary = true);

// Wilson loops of n_lines closed lines of a grid of N x m matrices.
// theta_sorted: [line][ldt]; Zout/theta_raw: optional eigenvectors of each W
// (m x m per line) and the phase of each column. Fkeep: if non-null receives
// the (polar) overlaps, [line][n_loop] m x m, which stay valid until the next
// call that uses slot WS_WILSON. line_status: [n_lines], OR-ed.
static int wilson_core(be_ctx *ctx, Grid U, int N, int m, int64_t n_lines, int n_loop, int mode, double *theta_sorted,
                       int ldt, double2 *Zout, double *theta_raw, uint32_t *line_status, const double2 **Fkeep,
                       hipStream_t stream, double2 *Wout = nullptr) {
  if (n_lines == 0) return BE_OK;
  if (m == 0) return BE_OK;
  const int64_t mm = int64_t(m) * m;
  const int64_t nm = n_lines * n_loop;
  double2 *F = nullptr, *B1 = nullptr, *B2 = nullptr, *Hs = nullptr;
  double *err = nullptr;
  int *act = nullptr, *n_left = nullptr;
  unsigned char *loc = nullptr;
  Carve cv;
  cv.add(&F, size_t(nm * mm));
  cv.add(&B1, size_t(nm * mm));
  cv.add(&B2, size_t(nm * mm));
  cv.add(&Hs, size_t(n_lines * mm));
  cv.add(&err, size_t(nm));
  cv.add(&act, size_t(nm));
  cv.add(&loc, size_t(nm));
  cv.add(&n_left, 1);
  BE_RET_IF(cv.commit(ctx, stream, WS_WILSON));
  // ---- overlaps
  {
    ZGemm g;
    g.M = m;
    g.N = m;
    g.K = N;
    g.opA = 1;
    g.opB = 0;
    g.A = U.base;
    g.lda = U.ld;
    g.bA = ZBatch::cyclic(U.stride, n_loop, 1, int64_t(n_loop) * U.stride);
    g.B = U.base;
    g.ldb = U.ld;
    g.bB = ZBatch::cyclic(U.stride, n_loop, 0, int64_t(n_loop) * U.stride);
    g.C = F;
    g.ldc = m;
    g.bC = ZBatch::strided(mm);
    g.batch = nm;
    g.tag = "overlap";
    BE_RET_IF(zgemm(ctx, g, stream));
  }
  // ---- polar factors (Newton-Schulz, per-matrix convergence). Up to 51
  // steps (sigma_min = 1e-8 converges at the 51st check); outside graph
  // capture the host stops the schedule once no matrix is left (read back
  // every other step from the fourth on), under capture every step is
  // launched and finished matrices skip it.
  if (mode == BE_OVL_POLAR) {
    const bool capturing = stream_capturing(stream);
    int *hleft = static_cast<int *>(ctx->pinned);
    double2 *X = F, *Xn = B2;
    unsigned char parity = 0;  // buffer of X: 0 = F, 1 = B2
    hipLaunchKernelGGL(k_ns_init, dim3(static_cast<uint32_t>((nm + 255) / 256)), dim3(256), 0, stream, act, loc, nm);
    BE_RET_IF(check_launch(ctx, "ns_init"));
    const int tpm = m * m <= 64 ? 64 : 256;
    for (int it = 0; it < 51; ++it) {
      ZGemm g;  // G = X^H X
      g.M = m;
      g.N = m;
      g.K = m;
      g.opA = 1;
      g.A = X;
      g.lda = m;
      g.bA = ZBatch::strided(mm);
      g.B = X;
      g.ldb = m;
      g.bB = ZBatch::strided(mm);
      g.C = B1;
      g.ldc = m;
      g.bC = ZBatch::strided(mm);
      g.batch = nm;
      g.tag = "polar";
      g.herm = true;  // X^H X: lower tiles, mirrored
      g.act = act;
      BE_RET_IF(zgemm(ctx, g, stream));
      hipLaunchKernelGGL(k_ns_prep, dim3(static_cast<uint32_t>((nm + 256 / tpm - 1) / (256 / tpm))), dim3(256), 0,
                         stream, B1, m, nm, tpm, err, act);
      BE_RET_IF(check_launch(ctx, "ns_prep"));
      ZGemm h;  // Xn = X (1.5 I - 0.5 G)
      h.M = m;
      h.N = m;
      h.K = m;
      h.A = X;
      h.lda = m;
      h.bA = ZBatch::strided(mm);
      h.B = B1;
      h.ldb = m;
      h.bB = ZBatch::strided(mm);
      h.C = Xn;
      h.ldc = m;
      h.bC = ZBatch::strided(mm);
      h.batch = nm;
      h.tag = "polar";
      h.act = act;
      BE_RET_IF(zgemm(ctx, h, stream));
      hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, stream, n_left);
      hipLaunchKernelGGL(k_ns_post, dim3(static_cast<uint32_t>((nm + 255) / 256)), dim3(256), 0, stream, act, loc, nm,
                         static_cast<unsigned char>(parity ^ 1), n_left);
      BE_RET_IF(check_launch(ctx, "ns_post"));
      std::swap(X, Xn);
      parity ^= 1;
      if (!capturing && it >= 3 && (it & 1)) {
        BE_HIP_TRY(ctx, hipMemcpyAsync(hleft, n_left, sizeof(int), hipMemcpyDeviceToHost, stream));
        BE_HIP_TRY(ctx, hipStreamSynchronize(stream));
        if (*hleft == 0) break;
      }
    }
    // every matrix's latest iterate into F
    hipLaunchKernelGGL(k_copy_mats_loc, dim3(64, static_cast<uint32_t>(std::min<int64_t>(nm, 65535))), dim3(256), 0,
                       stream, B2, F, mm, nm, loc);
    BE_RET_IF(check_launch(ctx, "copy_mats_loc"));
    // matrices whose last Gram error stayed at or above 1e-7 did not
    // converge: (near) singular overlaps
    hipLaunchKernelGGL(k_flag_err, dim3(static_cast<uint32_t>((n_lines + 255) / 256)), dim3(256), 0, stream, err,
                       n_lines, n_loop, 1e-7 * (1.0 - 1e-12), BE_ST_OVERLAP_SINGULAR, line_status);
    BE_RET_IF(check_launch(ctx, "flag_err"));
  }
  if (Fkeep) *Fkeep = F;
  // ---- ordered product W = F_{n-1} ... F_0 (tree)
  const double2 *cur = F;
  int n = n_loop;
  double2 *bufs[2] = {B1, B2};
  int which = 0;
  while (n > 1) {
    const int half = n / 2, n2 = (n + 1) / 2;
    double2 *dst = bufs[which];
    ZGemm g;  // dst[k] = cur[2k+1] cur[2k]
    g.M = m;
    g.N = m;
    g.K = m;
    g.A = cur + mm;
    g.lda = m;
    g.bA = ZBatch::cyclic(2 * mm, half, 0, int64_t(n) * mm);
    g.B = cur;
    g.ldb = m;
    g.bB = ZBatch::cyclic(2 * mm, half, 0, int64_t(n) * mm);
    g.C = dst;
    g.ldc = m;
    g.bC = ZBatch::cyclic(mm, half, 0, int64_t(n2) * mm);
    g.batch = n_lines * half;
    g.tag = "chain";
    BE_RET_IF(zgemm(ctx, g, stream));
    if (n & 1) {
      hipLaunchKernelGGL(k_carry_last, dim3(16, static_cast<uint32_t>(std::min<int64_t>(n_lines, 65535))), dim3(256), 0,
                         stream, cur, n, dst, n2, mm, n_lines);
      BE_RET_IF(check_launch(ctx, "carry_last"));
    }
    cur = dst;
    which ^= 1;
    n = n2;
  }
  // cur now holds W per line (n_loop == 1 means W = F_0)
  if (Wout) {  // the caller takes the eigenphases of all lines at once
    hipLaunchKernelGGL(k_copy_mats, dim3(64, static_cast<uint32_t>(std::min<int64_t>(n_lines, 65535))), dim3(256), 0,
                       stream, cur, mm, Wout, mm, mm, n_lines);
    return check_launch(ctx, "copy_w");
  }
  return unitary_phases(ctx, cur, m, n_lines, Hs, Zout, theta_sorted, ldt, theta_raw, line_status, stream,
                        mode == BE_OVL_POLAR);
}

// Eigenphases of n_lines unitary m x m matrices W (ascending into
// theta_sorted [line][ldt]); Zout/theta_raw as for wilson_core; Hs: scratch of
// n_lines m x m matrices (unused when the matrices fit LDS).
static int unitary_phases(be_ctx *ctx, const double2 *cur, int m, int64_t n_lines, double2 *Hs, double2 *Zout,
                          double *theta_sorted, int ldt, double *theta_raw, uint32_t *line_status, hipStream_t stream, bool unitary) {
  ProfScope prof(ctx, "unitary_eig", stream);
  const size_t esm_lds = (size_t(m) * m + 2 * size_t(m)) * sizeof(double2);
  const bool inlds = Zout == nullptr && esm_lds <= 160 * 1024;
  if (inlds || m <= 32) {  // orders up to 100 (up to 32 with eigenvectors): one wave per matrix, QR
    const size_t esm = inlds ? esm_lds : 2 * size_t(m) * sizeof(double2);
    auto kern = inlds ? &k_unitary_eig<true> : &k_unitary_eig<false>;
    if (esm > 65536)
      BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(esm)));
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(n_lines)), dim3(64), esm, stream, cur, m, n_lines, Hs, Zout,
                       theta_sorted, ldt, theta_raw, line_status, 1, nullptr);
    return check_launch(ctx, "unitary_eig");
  }
  if (!unitary) {  // raw overlaps: W is not unitary, the QR kernels take every matrix
    const size_t esm = Zout ? 2 * size_t(m) * sizeof(double2)
                            : (size_t(std::max(m, kUnitaryWgLds)) + size_t(m)) * sizeof(double2);
    BE_CHECK_ARG(ctx, esm <= 150 * 1024, "Wilson loop: order of the Wilson matrices too large for the eigenphase kernel");
    const void *kp = Zout ? reinterpret_cast<const void *>(&k_unitary_eig<false>)
                          : reinterpret_cast<const void *>(&k_unitary_eig_wg<256>);
    if (esm > 65536) BE_HIP_TRY(ctx, hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, int(esm)));
    if (Zout)
      hipLaunchKernelGGL(k_unitary_eig<false>, dim3(static_cast<uint32_t>(n_lines)), dim3(64), esm, stream, cur, m,
                         n_lines, Hs, Zout, theta_sorted, ldt, theta_raw, line_status, 1, nullptr);
    else
      hipLaunchKernelGGL(k_unitary_eig_wg<256>, dim3(static_cast<uint32_t>(n_lines)), dim3(256), esm, stream, cur, m,
                         n_lines, Hs, theta_sorted, ldt, theta_raw, line_status, 1, nullptr);
    return check_launch(ctx, "unitary_eig");
  }
  // larger orders: the Hermitian eigenproblem of (e^{-i phi} W + e^{i phi} W^H) / 2
  // (batched FP64 eigensolver, all bands), in chunks of lines within ~4 GiB;
  // matrices it cannot resolve go to the QR kernels (a workgroup per matrix,
  // or one wave with Schur vectors when eigenvectors are wanted)
  const int64_t mm = int64_t(m) * m;
  const int64_t per = 3 * mm * int64_t(sizeof(double2)) + (m + 2) * 8 + 4096;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(n_lines, (int64_t(4) << 30) / per));
  double2 *A = nullptr, *V = nullptr, *WV = nullptr;
  double *ev = nullptr;
  uint32_t *est = nullptr;
  int *fb = nullptr;
  Carve cv;
  cv.add(&A, size_t(cap * mm));
  cv.add(&V, size_t(cap * mm));
  cv.add(&WV, size_t(cap * mm));
  cv.add(&ev, size_t(cap * (m + 2)));
  cv.add(&est, size_t(cap));
  cv.add(&fb, size_t(cap));
  BE_RET_IF(cv.commit(ctx, stream, WS_UNIT));
  const size_t esm_wg = (size_t(std::max(m, kUnitaryWgLds)) + size_t(m)) * sizeof(double2);
  BE_CHECK_ARG(ctx, esm_wg <= 150 * 1024, "Wilson loop: order of the Wilson matrices too large for the eigenphase kernel");
  if (esm_wg > 65536)
    BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&k_unitary_eig_wg<256>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(esm_wg)));
  const size_t esm_1w = 2 * size_t(m) * sizeof(double2);
  if (esm_1w > 65536)
    BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&k_unitary_eig<false>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(esm_1w)));
  const int nt = (m + 31) / 32;
  for (int64_t l0 = 0; l0 < n_lines; l0 += cap) {
    const int64_t nl = std::min<int64_t>(cap, n_lines - l0);
    const double2 *Wc = cur + l0 * mm;
    hipLaunchKernelGGL(k_herm_of_unitary, dim3(static_cast<uint32_t>(nt * (nt + 1) / 2),
                                               static_cast<uint32_t>(std::min<int64_t>(nl, 65535))),
                       dim3(256), 0, stream, Wc, m, nl, A);
    BE_RET_IF(check_launch(ctx, "herm_of_unitary"));
    const std::string scope = ctx->prof_scope;
    ctx->prof_scope = scope + "unitary_";  // launch-timer names of the inner eigensolver
    // clusters only at 64 eps: W's nearly equal phases (often hundreds within
    // 1e-9 of each other) are then resolved one by one, each vector checked below
    const int erc = eigh_fp64(ctx, A, m, m, mm, nl, 0, m, ev, V, m, mm, est, stream, 64.0 * DBL_EPSILON);
    ctx->prof_scope = scope;
    BE_RET_IF(erc);
    ZGemm g;  // W V
    g.M = m;
    g.N = m;
    g.K = m;
    g.A = Wc;
    g.lda = m;
    g.bA = ZBatch::strided(mm);
    g.B = V;
    g.ldb = m;
    g.bB = ZBatch::strided(mm);
    g.C = WV;
    g.ldc = m;
    g.bC = ZBatch::strided(mm);
    g.batch = nl;
    g.tag = "unitary_wv";
    BE_RET_IF(zgemm(ctx, g, stream));
    double *ths = theta_sorted + l0 * ldt, *thr = theta_raw ? theta_raw + l0 * m : nullptr;
    double2 *Zc = Zout ? Zout + l0 * mm : nullptr;
    hipLaunchKernelGGL(k_herm_phases, dim3(static_cast<uint32_t>(nl)), dim3(256), size_t(m) * sizeof(double), stream, ev,
                       est, V, WV, m, nl, ths, ldt, thr, Zc, fb);
    BE_RET_IF(check_launch(ctx, "herm_phases"));
    if (Zout)
      hipLaunchKernelGGL(k_unitary_eig<false>, dim3(static_cast<uint32_t>(nl)), dim3(64), esm_1w, stream, Wc, m, nl,
                         Hs + l0 * mm, Zc, ths, ldt, thr, line_status + l0, 1, fb);
    else
      hipLaunchKernelGGL(k_unitary_eig_wg<256>, dim3(static_cast<uint32_t>(nl)), dim3(256), esm_wg, stream, Wc, m, nl,
                         Hs + l0 * mm, ths, ldt, thr, line_status + l0, 1, fb);
    BE_RET_IF(check_launch(ctx, "unitary_eig"));
  }
  return BE_OK;
}

}  // namespace be

// ============================================================================ C ABI

namespace {

int check_grid_args(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride, int32_t n_sys,
                    int32_t n_par, int32_t n_perp, int32_t mode) {
  using namespace be;
  BE_CHECK_ARG(ctx, ctx && U, "null U");
  BE_CHECK_ARG(ctx, N >= 1 && m >= 0 && m <= N, "need 0 <= m <= N");
  BE_CHECK_ARG(ctx, ldu >= N && u_stride >= int64_t(ldu) * std::max(m, 1), "ldu < N or u_stride < ldu*m");
  BE_CHECK_ARG(ctx, n_sys >= 0 && n_par >= 1 && n_perp >= 1, "need n_sys >= 0, n_par >= 1, n_perp >= 1");
  BE_CHECK_ARG(ctx, mode == BE_OVL_POLAR || mode == BE_OVL_RAW, "mode must be BE_OVL_POLAR or BE_OVL_RAW");
  return BE_OK;
}

}  // namespace

extern "C" int be_wilson_loop(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                              int32_t n_sys, int32_t n_par, int32_t n_perp, int32_t mode, double *theta, double *phi,
                              int32_t *winding, uint32_t *status, hipStream_t stream) {
  using namespace be;
  BE_RET_IF(check_grid_args(ctx, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, mode));
  BE_CHECK_ARG(ctx, theta && phi && winding && status, "be_wilson_loop: null output");
  if (n_sys == 0) return BE_OK;
  const int64_t n_lines = int64_t(n_sys) * n_perp;
  uint32_t *line_st = nullptr;
  Carve cv;
  cv.add(&line_st, size_t(n_lines));
  BE_RET_IF(cv.commit(ctx, stream, WS_OUTER));
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((n_lines + 255) / 256)), dim3(256), 0, stream, line_st, n_lines);
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((n_sys + 255) / 256)), dim3(256), 0, stream, status,
                     int64_t(n_sys));
  BE_RET_IF(check_launch(ctx, "zero"));
  // lines in passes whose overlaps, polar and product buffers (three m x m
  // matrices per link) stay within about 4 GiB of workspace; with more than
  // one pass, each pass leaves its Wilson matrices and the eigenphases of all
  // lines are taken in one launch (the eigenphase kernel runs a workgroup per
  // line: one launch keeps as many compute units busy as there are lines)
  const int64_t mm = int64_t(std::max(m, 1)) * std::max(m, 1);
  const int64_t per_line = int64_t(n_par) * 3 * mm * 16 + 4096;
  const int64_t lp = std::max<int64_t>(1, std::min<int64_t>(n_lines, (int64_t(4) << 30) / per_line));
  if (lp >= n_lines || m == 0) {
    Grid g{static_cast<const double2 *>(U), ldu, u_stride};
    BE_RET_IF(wilson_core(ctx, g, N, m, n_lines, n_par, mode, theta, m, nullptr, nullptr, line_st, nullptr, stream));
  } else {
    double2 *Wall = nullptr, *Hs = nullptr;
    Carve cw;
    cw.add(&Wall, size_t(n_lines * mm));
    cw.add(&Hs, size_t(n_lines * mm));
    BE_RET_IF(cw.commit(ctx, stream, WS_MISC));
    for (int64_t l0 = 0; l0 < n_lines; l0 += lp) {
      const int64_t nl = std::min<int64_t>(lp, n_lines - l0);
      Grid g{static_cast<const double2 *>(U) + l0 * n_par * u_stride, ldu, u_stride};
      BE_RET_IF(wilson_core(ctx, g, N, m, nl, n_par, mode, theta + l0 * m, m, nullptr, nullptr, line_st + l0, nullptr,
                            stream, Wall + l0 * mm));
    }
    BE_RET_IF(unitary_phases(ctx, Wall, m, n_lines, Hs, nullptr, theta, m, nullptr, line_st, stream,
                             mode == BE_OVL_POLAR));
  }
  hipLaunchKernelGGL(k_or_lines, dim3(static_cast<uint32_t>((n_lines + 255) / 256)), dim3(256), 0, stream, line_st,
                     n_lines, n_perp, status);
  hipLaunchKernelGGL(k_winding, dim3((n_sys + 63) / 64), dim3(64), 0, stream, theta, m, m, n_sys, n_perp, phi, winding,
                     status);
  return check_launch(ctx, "winding");
}

// ---------------------------------------------------------------- nested Wilson loop
namespace {

// Per line: sector = columns n of Z with x = theta_raw/2pi in (lo, hi).
// Writes s_line[line]; flags WANNIER_GAP if a phase is within 1e-6 of a window edge.
__global__ void k_sector_count(const double *theta_raw, int m, int64_t n_lines, double lo, double hi, int32_t *s_line,
                               uint32_t *line_st) {
  int64_t line = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (line >= n_lines) return;
  int s = 0;
  bool edge = false;
  for (int n = 0; n < m; ++n) {
    double x = theta_raw[line * m + n] / TWO_PI;
    if (x > lo && x < hi) ++s;
    if (fabs(x - lo) < 1e-6 || fabs(x - hi) < 1e-6) edge = true;
  }
  s_line[line] = s;
  if (edge) line_st[line] |= BE_ST_WANNIER_GAP;
}

// Per system: sector size of line 0; WANNIER_GAP if any line differs.
__global__ void k_sector_sys(const int32_t *s_line, int n_sys, int n_perp, int32_t *s_sys, uint32_t *status) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  int s0 = s_line[int64_t(s) * n_perp];
  for (int i = 1; i < n_perp; ++i)
    if (s_line[int64_t(s) * n_perp + i] != s0) atomicOr(&status[s], BE_ST_WANNIER_GAP);
  s_sys[s] = s0;
}

// nu[line][0] = Z_line[:, sector] (m x sc, ld m), in the order of the columns.
__global__ void k_gather_sector(const double2 *Z, const double *theta_raw, int m, int64_t n_lines, double lo, double hi,
                                int sc, int n_loop, double2 *nu) {
  int64_t line = blockIdx.x;
  if (line >= n_lines) return;
  int col = 0;
  for (int n = 0; n < m; ++n) {
    double x = theta_raw[line * m + n] / TWO_PI;
    if (x > lo && x < hi) {
      if (col < sc)
        for (int r = threadIdx.x; r < m; r += blockDim.x)
          nu[(line * n_loop) * int64_t(m) * sc + r + int64_t(col) * m] = Z[line * int64_t(m) * m + r + int64_t(n) * m];
      ++col;
    }
  }
}

// p[s][j] and p_mean[s] from nested theta [s][j][ldt] (first sc valid).
__global__ void k_nested_p(const double *th, int ldt, int sc, int n_sys, int n_par, double *p, double *p_mean) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  double prev = 0.0, acc_u = 0.0, sum = 0.0;
  for (int j = 0; j < n_par; ++j) {
    double a = 0.0;
    const double *t = th + (int64_t(s) * n_par + j) * ldt;
    for (int n = 0; n < sc; ++n) a += t[n];
    double pj = a / TWO_PI;
    pj -= rint(pj);
    if (pj <= -0.5) pj += 1.0;
    if (pj > 0.5) pj -= 1.0;
    if (fabs(fabs(pj) - 0.5) < 1e-15) pj = 0.5;
    p[int64_t(s) * n_par + j] = pj;
    if (j == 0) {
      acc_u = pj;
    } else {
      double d = pj - prev;
      d -= rint(d);
      acc_u += d;
    }
    sum += acc_u;
    prev = pj;
  }
  double mean = sum / n_par;
  mean -= floor(mean);
  if (mean >= 1.0) mean -= 1.0;
  p_mean[s] = mean;
}

__global__ void k_fill_nan(double *p, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = NAN;
}

}  // namespace

extern "C" int be_nested_wilson(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                                int32_t n_sys, int32_t n_par, int32_t n_perp, int32_t mode, double win_lo,
                                double win_hi, double *nested_theta, double *p, double *p_mean, int32_t *s_out_h,
                                uint32_t *status, hipStream_t stream) {
  using namespace be;
  BE_RET_IF(check_grid_args(ctx, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, mode));
  BE_CHECK_ARG(ctx, nested_theta && p && p_mean && s_out_h && status, "be_nested_wilson: null output");
  BE_CHECK_ARG(ctx, win_lo < win_hi, "be_nested_wilson: need win_lo < win_hi");
  if (n_sys == 0) return BE_OK;
  const int64_t n_lines = int64_t(n_sys) * n_perp;
  const int64_t mm = int64_t(m) * m;
  uint32_t *line_st = nullptr, *line_st2 = nullptr;
  double *th0 = nullptr, *thraw = nullptr;
  double2 *Z = nullptr, *nu = nullptr, *w = nullptr;
  int32_t *s_line = nullptr, *s_sys = nullptr;
  Carve cv;
  cv.add(&line_st, size_t(n_lines));
  cv.add(&line_st2, size_t(int64_t(n_sys) * n_par));
  cv.add(&th0, size_t(n_lines * std::max(m, 1)));
  cv.add(&thraw, size_t(n_lines * std::max(m, 1)));
  cv.add(&Z, size_t(n_lines * std::max<int64_t>(mm, 1)));
  cv.add(&nu, size_t(n_lines * n_par * std::max<int64_t>(mm, 1)));
  cv.add(&w, size_t(n_lines * n_par * int64_t(N) * std::max(m, 1)));
  cv.add(&s_line, size_t(n_lines));
  cv.add(&s_sys, size_t(n_sys));
  BE_RET_IF(cv.commit(ctx, stream, WS_OUTER));
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((n_lines + 255) / 256)), dim3(256), 0, stream, line_st, n_lines);
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((n_sys * int64_t(n_par) + 255) / 256)), dim3(256), 0, stream,
                     line_st2, int64_t(n_sys) * n_par);
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((n_sys + 255) / 256)), dim3(256), 0, stream, status,
                     int64_t(n_sys));
  hipLaunchKernelGGL(k_fill_nan, dim3(static_cast<uint32_t>((int64_t(n_sys) * n_par * std::max(m, 1) + 255) / 256)), dim3(256),
                     0, stream, nested_theta, int64_t(n_sys) * n_par * std::max(m, 1));
  BE_RET_IF(check_launch(ctx, "zero"));
  for (int s = 0; s < n_sys; ++s) s_out_h[s] = 0;
  if (m == 0) return BE_OK;
  // ---- first Wilson loop at base point 0 with eigenvectors; keep the overlaps
  Grid g{static_cast<const double2 *>(U), ldu, u_stride};
  const double2 *F = nullptr;
  BE_RET_IF(wilson_core(ctx, g, N, m, n_lines, n_par, mode, th0, m, Z, thraw, line_st, &F, stream));
  // ---- sector sizes
  hipLaunchKernelGGL(k_sector_count, dim3(static_cast<uint32_t>((n_lines + 255) / 256)), dim3(256), 0, stream, thraw, m,
                     n_lines, win_lo, win_hi, s_line, line_st);
  hipLaunchKernelGGL(k_or_lines, dim3(static_cast<uint32_t>((n_lines + 255) / 256)), dim3(256), 0, stream, line_st,
                     n_lines, n_perp, status);
  hipLaunchKernelGGL(k_sector_sys, dim3((n_sys + 63) / 64), dim3(64), 0, stream, s_line, n_sys, n_perp, s_sys, status);
  BE_RET_IF(check_launch(ctx, "sector"));
  int32_t *hs = static_cast<int32_t *>(ctx->pinned);
  BE_CHECK_ARG(ctx, n_sys <= 1024, "be_nested_wilson: at most 1024 systems per call");
  BE_HIP_TRY(ctx, hipMemcpyAsync(hs, s_sys, sizeof(int32_t) * n_sys, hipMemcpyDeviceToHost, stream));
  BE_HIP_TRY(ctx, hipStreamSynchronize(stream));
  for (int s = 0; s < n_sys; ++s) s_out_h[s] = hs[s];
  // ---- pass 1, per run of systems with equal sector size: carry the sector
  // to every base point and form w (needs the overlaps F of the first loop)
  std::vector<int64_t> w_off(n_sys + 1, 0);
  for (int s = 0; s < n_sys; ++s) w_off[s + 1] = w_off[s] + int64_t(n_perp) * n_par * N * s_out_h[s];
  for (int s0 = 0; s0 < n_sys;) {
    const int sc = s_out_h[s0];
    int s1 = s0 + 1;
    while (s1 < n_sys && s_out_h[s1] == sc) ++s1;
    if (sc == 0) {
      s0 = s1;
      continue;
    }
    const int64_t l0 = int64_t(s0) * n_perp, nl = int64_t(s1 - s0) * n_perp;
    const int64_t nus = int64_t(m) * sc;  // one nu block
    hipLaunchKernelGGL(k_gather_sector, dim3(static_cast<uint32_t>(nl)), dim3(64), 0, stream, Z + l0 * mm, thraw + l0 * m, m,
                       nl, win_lo, win_hi, sc, n_par, nu);
    BE_RET_IF(check_launch(ctx, "gather_sector"));
    // transport nu[line][j+1] = F[line][j] nu[line][j]
    for (int j = 0; j + 1 < n_par; ++j) {
      ZGemm t;
      t.M = m;
      t.N = sc;
      t.K = m;
      t.A = F + (l0 * n_par + j) * mm;
      t.lda = m;
      t.bA = ZBatch::strided(int64_t(n_par) * mm);
      t.B = nu + int64_t(j) * nus;
      t.ldb = m;
      t.bB = ZBatch::strided(int64_t(n_par) * nus);
      t.C = nu + int64_t(j + 1) * nus;
      t.ldc = m;
      t.bC = ZBatch::strided(int64_t(n_par) * nus);
      t.batch = nl;
      t.tag = "transport";
      BE_RET_IF(zgemm(ctx, t, stream));
    }
    // w[s][j][i] = U[s][i][j] nu[(s,i)][j]   (N x sc, ld N)
    const int64_t ws = int64_t(N) * sc;
    ZGemm t;
    t.M = N;
    t.N = sc;
    t.K = m;
    t.A = static_cast<const double2 *>(U) + l0 * n_par * u_stride;
    t.lda = ldu;
    t.bA = ZBatch::strided(u_stride);
    t.B = nu;
    t.ldb = m;
    t.bB = ZBatch::strided(nus);
    t.C = w + w_off[s0];
    t.ldc = N;
    ZBatch bc;
    bc.s0 = int64_t(n_perp) * ws;  // j
    bc.n0 = n_par;
    bc.s1 = ws;  // i
    bc.n1 = n_perp;
    bc.s2 = int64_t(n_par) * n_perp * ws;
    t.bC = bc;
    t.batch = nl * n_par;
    t.tag = "wannier_states";
    BE_RET_IF(zgemm(ctx, t, stream));
    s0 = s1;
  }
  // ---- pass 2: nested loops along the transverse direction, one per (system, j)
  for (int s0 = 0; s0 < n_sys;) {
    const int sc = s_out_h[s0];
    int s1 = s0 + 1;
    while (s1 < n_sys && s_out_h[s1] == sc) ++s1;
    if (sc == 0) {
      s0 = s1;
      continue;
    }
    const int64_t ws = int64_t(N) * sc;
    Grid gw{w + w_off[s0], N, ws};
    const int64_t nl2 = int64_t(s1 - s0) * n_par;
    BE_RET_IF(wilson_core(ctx, gw, N, sc, nl2, n_perp, mode, nested_theta + int64_t(s0) * n_par * m, m, nullptr, nullptr,
                          line_st2 + int64_t(s0) * n_par, nullptr, stream));
    hipLaunchKernelGGL(k_or_lines, dim3(static_cast<uint32_t>((nl2 + 255) / 256)), dim3(256), 0, stream,
                       line_st2 + int64_t(s0) * n_par, nl2, n_par, status + s0);
    hipLaunchKernelGGL(k_nested_p, dim3((s1 - s0 + 63) / 64), dim3(64), 0, stream, nested_theta + int64_t(s0) * n_par * m, m,
                       sc, s1 - s0, n_par, p + int64_t(s0) * n_par, p_mean + s0);
    BE_RET_IF(check_launch(ctx, "nested_p"));
    s0 = s1;
  }
  return BE_OK;
}

// ---------------------------------------------------------------- spin-resolved Wilson loop
namespace {

// c128 -> c64 (rounded), n elements
__global__ void k_narrow(const double2 *a, int64_t n, float2 *b) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = make_float2(float(a[i].x), float(a[i].y));
}

// Projected-spin eigenvalues: copy into the output, count negatives, flag gaps.
__global__ void k_pso_post(const double *ev, const uint32_t *eig_st, int m, int64_t n_k, int64_t k_per_sys, double *pso,
                           int32_t *cnt, uint32_t *status) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_k) return;
  int c = 0;
  double mn = INFINITY;
  for (int n = 0; n < m; ++n) {
    double v = ev[k * (m + 2) + 1 + n];
    pso[k * m + n] = v;
    c += v < 0.0;
    mn = fmin(mn, fabs(v));
  }
  cnt[k] = c;
  if (!(mn >= 1e-6)) atomicOr(&status[k / k_per_sys], BE_ST_PSO_GAP);
  // the projected-spin eigensolver's own conditions (its gap bits do not apply)
  const uint32_t es = eig_st[k] & (BE_ST_NONCONVERGED | BE_ST_NAN_INF);
  if (es) atomicOr(&status[k / k_per_sys], es);
}

__global__ void k_pso_sys(const int32_t *cnt, int n_sys, int64_t k_per_sys, int32_t *m_dn, uint32_t *status) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  int c0 = cnt[int64_t(s) * k_per_sys];
  for (int64_t k = 1; k < k_per_sys; ++k)
    if (cnt[int64_t(s) * k_per_sys + k] != c0) {
      atomicOr(&status[s], BE_ST_PSO_GAP);
      break;
    }
  m_dn[s] = c0;
}

// Sector sizes given by the caller for a captured call (at most 256 systems).
struct SectorSizes {
  int32_t v[256];
};

// Under graph capture the spin-down sector sizes are the caller's (the
// graph's shapes depend on them): a system whose actual count differs is
// flagged PSO_GAP (its sector results are then invalid).
__global__ void k_pso_expect(const int32_t *mdn, int n_sys, SectorSizes want, uint32_t *status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n_sys && mdn[s] != want.v[s]) atomicOr(&status[s], BE_ST_PSO_GAP);
}

__global__ void k_spin_chern(const int32_t *cd, const int32_t *cu, int n, double *cs) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) cs[s] = 0.5 * double(cu[s] - cd[s]);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

namespace {

// The projected spin operator A = U^H S U of every k-point and its
// eigendecomposition (mu ascending, eigenvectors Q, m x m per k-point), the
// per-k PSO_GAP test and the per-system spin-down sector size m_dn_h (read
// back, so the stream is synchronized once; under graph capture m_dn_h is
// the caller's input instead, checked on the device).
int spin_operator_eig(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride, int32_t n_sys,
                      int64_t kps, int32_t precision, const double *spin_diag, double *pso_evals, double2 *A32buf,
                      double2 *A, double2 *Q, double *ev, uint32_t *kst, int32_t *cnt, int32_t *mdn, int32_t *m_dn_h,
                      uint32_t *status, hipStream_t stream) {
  using namespace be;
  const int64_t n_k = int64_t(n_sys) * kps;
  const int64_t mm = int64_t(m) * std::max(m, 1);
  // ---- A = U^H S U, S applied to the rows of U as the GEMM loads them
  {
    ZGemm g;
    g.M = m;
    g.N = m;
    g.K = N;
    g.opA = 1;
    g.A = static_cast<const double2 *>(U);
    g.lda = ldu;
    g.bA = ZBatch::strided(u_stride);
    g.B = static_cast<const double2 *>(U);
    g.ldb = ldu;
    g.bB = ZBatch::strided(u_stride);
    g.scaleB = spin_diag;
    g.scaleB_div = kps;
    g.scaleB_ld = N;
    g.C = A;
    g.ldc = m;
    g.bC = ZBatch::strided(mm);
    g.batch = n_k;
    g.tag = "pso";
    g.herm = true;  // U^H S U is Hermitian: lower tiles computed, mirrored (bitwise Hermitian for the eigensolver)
    g.four_mult = true;  // diagonal tiles bitwise Hermitian too
    BE_RET_IF(zgemm(ctx, g, stream));
  }
  // ---- eigh of the m x m projected spin operator (all bands)
  ctx->prof_scope = "pso_";  // launch-timer names of the inner eigensolver
  int erc;
  // BE_MIXED_FP32_REFINED takes the FP64 solver here (order m: the sectors'
  // subspaces are then FP64-accurate, as the refined eigenvectors U are)
  if (precision == BE_MIXED_FP32 || precision == BE_MIXED_BF16X) {
    // c64 copy of the projected operator
    float2 *A32 = reinterpret_cast<float2 *>(A32buf);
    hipLaunchKernelGGL(k_narrow, dim3(static_cast<uint32_t>(std::min<int64_t>((n_k * mm + 255) / 256, 65535))),
                       dim3(256), 0, stream, A, n_k * mm, A32);
    erc = check_launch(ctx, "k_narrow");
    if (erc == BE_OK)
      erc = eigh_mixed(ctx, A32, m, m, mm, n_k, 0, m, ev, Q, m, mm, kst, stream, precision == BE_MIXED_BF16X);
  } else {
    erc = eigh_fp64(ctx, A, m, m, mm, n_k, 0, m, ev, Q, m, mm, kst, stream);
  }
  ctx->prof_scope.clear();
  BE_RET_IF(erc);
  hipLaunchKernelGGL(k_pso_post, dim3(static_cast<uint32_t>((n_k + 255) / 256)), dim3(256), 0, stream, ev, kst, m, n_k,
                     kps, pso_evals, cnt, status);
  hipLaunchKernelGGL(k_pso_sys, dim3((n_sys + 63) / 64), dim3(64), 0, stream, cnt, n_sys, kps, mdn, status);
  BE_RET_IF(check_launch(ctx, "pso"));
  if (stream_capturing(stream)) {
    BE_CHECK_ARG(ctx, n_sys <= 256, "spin sectors under graph capture: at most 256 systems per call");
    SectorSizes want{};
    for (int s = 0; s < n_sys; ++s) {
      BE_CHECK_ARG(ctx, m_dn_h[s] >= 0 && m_dn_h[s] <= m, "spin sectors under graph capture: m_dn_h[s] must hold "
                                                           "the sector sizes (0..m) of an earlier uncaptured call");
      want.v[s] = m_dn_h[s];
    }
    hipLaunchKernelGGL(k_pso_expect, dim3((n_sys + 63) / 64), dim3(64), 0, stream, mdn, n_sys, want, status);
    return check_launch(ctx, "pso_expect");
  }
  int32_t *hm = static_cast<int32_t *>(ctx->pinned);
  BE_HIP_TRY(ctx, hipMemcpyAsync(hm, mdn, sizeof(int32_t) * n_sys, hipMemcpyDeviceToHost, stream));
  BE_HIP_TRY(ctx, hipStreamSynchronize(stream));
  for (int s = 0; s < n_sys; ++s) m_dn_h[s] = hm[s];
  return BE_OK;
}

}  // namespace

extern "C" int be_spin_resolved_wilson(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                                       int32_t n_sys, int32_t n_par, int32_t n_perp, int32_t mode, int32_t precision,
                                       const double *spin_diag, double *pso_evals, double *theta_dn, double *theta_up,
                                       int32_t *C_dn, int32_t *C_up, double *C_s, int32_t *m_dn_h, uint32_t *status,
                                       hipStream_t stream) {
  using namespace be;
  BE_RET_IF(check_grid_args(ctx, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, mode));
  BE_CHECK_ARG(ctx, spin_diag && pso_evals && theta_dn && theta_up && C_dn && C_up && C_s && m_dn_h && status,
               "be_spin_resolved_wilson: null argument");
  BE_CHECK_ARG(ctx, n_sys <= 1024, "be_spin_resolved_wilson: at most 1024 systems per call");
  BE_CHECK_ARG(ctx, precision == BE_FP64 || precision == BE_MIXED_FP32 || precision == BE_MIXED_FP32_REFINED ||
                        precision == BE_MIXED_BF16X,
               "be_spin_resolved_wilson: bad precision");
  if (n_sys == 0) return BE_OK;
  const int64_t kps = int64_t(n_par) * n_perp;
  const int64_t n_k = int64_t(n_sys) * kps;
  const int64_t n_lines = int64_t(n_sys) * n_perp;
  const int64_t mm = int64_t(m) * std::max(m, 1);
  const int64_t Nm = int64_t(N) * std::max(m, 1);
  double2 *A32buf = nullptr, *A = nullptr, *Q = nullptr, *V = nullptr;
  double *ev = nullptr;
  uint32_t *kst = nullptr, *lst = nullptr;
  int32_t *cnt = nullptr, *mdn = nullptr;
  Carve cv;
  cv.add(&A32buf, size_t((n_k * mm + 1) / 2));  // c64 m x m per k (mixed path)
  cv.add(&A, size_t(n_k * mm));
  cv.add(&Q, size_t(n_k * mm));
  cv.add(&V, size_t(n_k * Nm));
  cv.add(&ev, size_t(n_k * (m + 2)));
  cv.add(&kst, size_t(n_k));
  cv.add(&lst, size_t(2 * n_lines));
  cv.add(&cnt, size_t(n_k));
  cv.add(&mdn, size_t(n_sys));
  BE_RET_IF(cv.commit(ctx, stream, WS_OUTER));
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((n_sys + 255) / 256)), dim3(256), 0, stream, status,
                     int64_t(n_sys));
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((2 * n_lines + 255) / 256)), dim3(256), 0, stream, lst,
                     2 * n_lines);
  BE_RET_IF(check_launch(ctx, "zero"));
  if (!stream_capturing(stream))  // under capture m_dn_h holds the caller's sector sizes
    for (int s = 0; s < n_sys; ++s) m_dn_h[s] = 0;
  if (m == 0) return BE_OK;
  BE_RET_IF(spin_operator_eig(ctx, U, N, m, ldu, u_stride, n_sys, kps, precision, spin_diag, pso_evals, A32buf, A, Q, ev,
                              kst, cnt, mdn, m_dn_h, status, stream));
  hipLaunchKernelGGL(k_fill_nan, dim3(static_cast<uint32_t>((n_lines * m + 255) / 256)), dim3(256), 0, stream, theta_dn,
                     n_lines * m);
  hipLaunchKernelGGL(k_fill_nan, dim3(static_cast<uint32_t>((n_lines * m + 255) / 256)), dim3(256), 0, stream, theta_up,
                     n_lines * m);
  hipLaunchKernelGGL(k_fill_i32, dim3((n_sys + 255) / 256), dim3(256), 0, stream, C_dn, int64_t(n_sys), 0);
  hipLaunchKernelGGL(k_fill_i32, dim3((n_sys + 255) / 256), dim3(256), 0, stream, C_up, int64_t(n_sys), 0);
  BE_RET_IF(check_launch(ctx, "fill"));
  // ---- V = U Q for all systems at once (columns in ascending mu: the first
  // m_dn_h[s] span the spin-down sector), then per run of systems with equal
  // sector sizes, the Wilson loop of each sector on its column slice of V
  {
    ZGemm g;
    g.M = N;
    g.N = m;
    g.K = m;
    g.A = static_cast<const double2 *>(U);
    g.lda = ldu;
    g.bA = ZBatch::strided(u_stride);
    g.B = Q;
    g.ldb = m;
    g.bB = ZBatch::strided(mm);
    g.C = V;
    g.ldc = N;
    g.bC = ZBatch::strided(Nm);
    g.batch = n_k;
    g.tag = "spin_sector";
    BE_RET_IF(zgemm(ctx, g, stream));
  }
  for (int s0 = 0; s0 < n_sys;) {
    const int md = m_dn_h[s0];
    int s1 = s0 + 1;
    while (s1 < n_sys && m_dn_h[s1] == md) ++s1;
    const int64_t k0 = int64_t(s0) * kps;
    const int64_t l0 = int64_t(s0) * n_perp, nl = int64_t(s1 - s0) * n_perp;
    for (int sector = 0; sector < 2; ++sector) {
      const int ms = sector == 0 ? md : m - md;
      const int c0 = sector == 0 ? 0 : md;
      if (ms == 0) continue;
      Grid gv{V + k0 * Nm + int64_t(c0) * N, N, Nm};
      double *th = (sector == 0 ? theta_dn : theta_up) + l0 * m;
      uint32_t *ls = lst + sector * n_lines + l0;
      BE_RET_IF(wilson_core(ctx, gv, N, ms, nl, n_par, mode, th, m, nullptr, nullptr, ls, nullptr, stream));
      hipLaunchKernelGGL(k_or_lines, dim3(static_cast<uint32_t>((nl + 255) / 256)), dim3(256), 0, stream, ls, nl, n_perp,
                         status + s0);
      hipLaunchKernelGGL(k_winding, dim3((s1 - s0 + 63) / 64), dim3(64), 0, stream, th, m, ms, s1 - s0, n_perp, nullptr,
                         (sector == 0 ? C_dn : C_up) + s0, status + s0);
      BE_RET_IF(check_launch(ctx, "spin winding"));
    }
    s0 = s1;
  }
  hipLaunchKernelGGL(k_spin_chern, dim3((n_sys + 255) / 256), dim3(256), 0, stream, C_dn, C_up, n_sys, C_s);
  return check_launch(ctx, "spin_chern");
}

extern "C" int be_spin_sectors(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                               int32_t n_sys, int32_t n_k_sys, int32_t precision, const double *spin_diag,
                               double *pso_evals, void *V, int32_t ldv, int64_t v_stride, int32_t *m_dn_h,
                               uint32_t *status, hipStream_t stream) {
  using namespace be;
  BE_RET_IF(check_grid_args(ctx, U, N, m, ldu, u_stride, n_sys, n_k_sys, 1, BE_OVL_POLAR));
  BE_CHECK_ARG(ctx, spin_diag && pso_evals && V && m_dn_h && status, "be_spin_sectors: null argument");
  BE_CHECK_ARG(ctx, ldv >= N && v_stride >= int64_t(ldv) * std::max(m, 1), "be_spin_sectors: ldv < N or v_stride < ldv*m");
  BE_CHECK_ARG(ctx, n_sys <= 1024, "be_spin_sectors: at most 1024 systems per call");
  BE_CHECK_ARG(ctx, precision == BE_FP64 || precision == BE_MIXED_FP32 || precision == BE_MIXED_FP32_REFINED ||
                        precision == BE_MIXED_BF16X,
               "be_spin_sectors: bad precision");
  if (n_sys == 0) return BE_OK;
  const int64_t kps = n_k_sys;
  const int64_t n_k = int64_t(n_sys) * kps;
  const int64_t mm = int64_t(m) * std::max(m, 1);
  const int64_t Nm = int64_t(N) * std::max(m, 1);
  double2 *A32buf = nullptr, *A = nullptr, *Q = nullptr;
  double *ev = nullptr;
  uint32_t *kst = nullptr;
  int32_t *cnt = nullptr, *mdn = nullptr;
  Carve cv;
  cv.add(&A32buf, size_t((n_k * mm + 1) / 2));  // c64 m x m per k (mixed path)
  cv.add(&A, size_t(n_k * mm));
  cv.add(&Q, size_t(n_k * mm));
  cv.add(&ev, size_t(n_k * (m + 2)));
  cv.add(&kst, size_t(n_k));
  cv.add(&cnt, size_t(n_k));
  cv.add(&mdn, size_t(n_sys));
  BE_RET_IF(cv.commit(ctx, stream, WS_OUTER));
  hipLaunchKernelGGL(k_zero_u32, dim3(static_cast<uint32_t>((n_sys + 255) / 256)), dim3(256), 0, stream, status,
                     int64_t(n_sys));
  BE_RET_IF(check_launch(ctx, "zero"));
  if (!stream_capturing(stream))  // under capture m_dn_h holds the caller's sector sizes
    for (int s = 0; s < n_sys; ++s) m_dn_h[s] = 0;
  if (m == 0) return BE_OK;
  BE_RET_IF(spin_operator_eig(ctx, U, N, m, ldu, u_stride, n_sys, kps, precision, spin_diag, pso_evals, A32buf, A, Q, ev,
                              kst, cnt, mdn, m_dn_h, status, stream));
  ZGemm g;  // V = U Q: spin-down columns first (mu ascending)
  g.M = N;
  g.N = m;
  g.K = m;
  g.A = static_cast<const double2 *>(U);
  g.lda = ldu;
  g.bA = ZBatch::strided(u_stride);
  g.B = Q;
  g.ldb = m;
  g.bB = ZBatch::strided(mm);
  g.C = static_cast<double2 *>(V);
  g.ldc = ldv;
  g.bC = ZBatch::strided(v_stride);
  g.batch = n_k;
  g.tag = "spin_sector";
  return zgemm(ctx, g, stream);
}

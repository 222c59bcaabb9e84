// Berry flux through the plaquettes of a k-grid (the coupling-matrix method
// of the disordered quadrupolar-insulator example, Sec. IV: the zone is cut
// into plaquettes and the Berry flux through each is integrated along its
// closed boundary; applied to the occupied bands or to one spin sector).
//
// Link variables between neighbouring grid points, along the loop direction
// and across it (both periodic), det(U(k')^H U(k)):
//   links    batched MFMA GEMMs U(k')^H U(k) (the across-direction batch runs
//            with the transverse index innermost and cyclic),
//   phases   k_det_phase: blocked LU with partial pivoting, one workgroup per link,
//            arg det = sum of the pivots' arguments (+ pi per row swap),
//            log |det| = sum of log |pivot|. A link is singular, its
//            variable det/|det| undetermined, when its smallest singular
//            value is below 1e-8 (the test the Wilson loop applies to its
//            overlaps). No singular value of an overlap of orthonormal bases
//            exceeds 1, so |det| <= sigma_min: |det| >= 1e-8 proves the link
//            regular. Otherwise (a near-singular link, or only a high order:
//            0.97^640 < 1e-8) sigma_min is estimated from the LU factors by
//            inverse iteration on (M^H M)^{-1}, whose Rayleigh quotient
//            bounds 1/sigma_min^2 from below,
//   flux     k_plaquette: F(i, j) = wrap(phi_par(i+1, j) - phi_par(i, j)
//            + phi_perp(i, j) - phi_perp(i, j+1)) in (-pi, pi], oriented so
//            that the sum over the zone is 2 pi times the winding of eq. 6;
//            each link enters two plaquettes with opposite signs, so the sum
//            is an exact multiple of 2 pi (the Chern number).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <mutex>
#include <string>

#include "common.hpp"

namespace {

constexpr int DT = 256;  // threads per determinant
constexpr double kPi = 3.14159265358979323846;
constexpr double kLogSingular = -18.420680743952367;  // log(1e-8)

__device__ __forceinline__ double wrap_pi(double x) {
  x -= 2.0 * kPi * rint(x / (2.0 * kPi));
  return x <= -kPi ? kPi : x;
}

// Sum over the NT threads of the block (NT a multiple of 64); red: NT/64
// doubles of LDS (unused for one wave). Every thread gets the sum.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if constexpr (NT > 64) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    v = 0.0;
    for (int w = 0; w < NT / 64; ++w) v += red[w];
  }
  return v;
}

// Smallest singular value of an m x m matrix from its LU factors P M = L U,
// stored in place (row-major rows of length m; unit lower L strictly below
// the diagonal, U on and above it): logical row i of the factors is row
// rowmap[i] of A, or row i when rowmap is null. Row interchanges do not
// change singular values, so sigma_min(M) = sigma_min(L U). Two steps of
// inverse iteration on (LU)^{-1} (LU)^{-H} from a fixed start vector whose
// entries have modulus one, then the Rayleigh quotient rq = |(LU)^{-H} x|^2
// of the normalized iterate: rq <= 1/sigma_min^2, so the returned 1/sqrt(rq)
// is an upper bound of sigma_min, equal to it once the iterate has converged
// (each step scales the other singular directions down by
// (sigma_min/sigma_k)^2 against the smallest one). Returns 0 when a solve
// overflows (singular to working precision).
// Triangular solves are column-oriented with a fixed owner per row (thread
// r mod NT), one barrier per column: the pivot column's value is published
// through a double-buffered LDS slot. Solves with U^H and L^H read rows of
// the factors (coalesced); solves with L and U read columns.
// x: m double2 of LDS, slot: 2 double2 of LDS, red: as for block_sum.
template <int NT>
__device__ double lu_smin(const double2 *A, int m, const int *rowmap, double2 *x, double2 *slot, double *red) {
  const int tid = threadIdx.x;
  auto rowp = [&](int i) { return A + int64_t(rowmap ? rowmap[i] : i) * m; };
  auto first_above = [&](int c) {  // smallest r > c owned by this thread
    int r = tid;
    if (r <= c) r += ((c - r) / NT + 1) * NT;
    return r;
  };
  for (int i = tid; i < m; i += NT) {
    const uint32_t h = uint32_t(i + 1) * 2654435761u;
    double sn, cs;
    sincospi(double(h) * (2.0 / 4294967296.0), &sn, &cs);
    x[i] = make_double2(cs, sn);
  }
  for (int it = 0;; ++it) {
    // normalize
    double ss = 0.0;
    for (int i = tid; i < m; i += NT) ss += x[i].x * x[i].x + x[i].y * x[i].y;
    ss = block_sum<NT>(ss, red);
    if (!(ss > 0.0) || !isfinite(ss)) return 0.0;
    const double inv = 1.0 / sqrt(ss);
    for (int i = tid; i < m; i += NT) x[i] = make_double2(x[i].x * inv, x[i].y * inv);
    __syncthreads();
    // U^H t = x, forward: t_c = x_c / conj(u_cc), x_r -= conj(U(c, r)) t_c (r > c)
    for (int c = 0; c < m; ++c) {
      const double2 *Ac = rowp(c);
      if (tid == c % NT) {
        const double2 u = Ac[c], xc = x[c];
        const double den = u.x * u.x + u.y * u.y;
        const double2 t = make_double2((xc.x * u.x - xc.y * u.y) / den, (xc.x * u.y + xc.y * u.x) / den);
        x[c] = t;
        slot[c & 1] = t;
      }
      __syncthreads();
      const double2 t = slot[c & 1];
      for (int r = first_above(c); r < m; r += NT) {
        const double2 a = Ac[r];
        x[r] = make_double2(x[r].x - (a.x * t.x + a.y * t.y), x[r].y - (a.x * t.y - a.y * t.x));
      }
    }
    __syncthreads();
    // L^H y = t, backward (unit diagonal): t_r -= conj(L(c, r)) y_c (r < c)
    for (int c = m - 1; c >= 0; --c) {
      const double2 *Ac = rowp(c);
      if (tid == c % NT) slot[c & 1] = x[c];
      __syncthreads();
      const double2 y = slot[c & 1];
      for (int r = tid; r < c; r += NT) {
        const double2 a = Ac[r];
        x[r] = make_double2(x[r].x - (a.x * y.x + a.y * y.y), x[r].y - (a.x * y.y - a.y * y.x));
      }
    }
    __syncthreads();
    double rq = 0.0;
    for (int i = tid; i < m; i += NT) rq += x[i].x * x[i].x + x[i].y * x[i].y;
    rq = block_sum<NT>(rq, red);
    if (!(rq > 0.0) || !isfinite(rq)) return 0.0;
    if (it == 2) return 1.0 / sqrt(rq);
    // L v = y, forward (unit diagonal): y_r -= L(r, c) v_c (r > c)
    for (int c = 0; c < m; ++c) {
      if (tid == c % NT) slot[c & 1] = x[c];
      __syncthreads();
      const double2 v = slot[c & 1];
      for (int r = first_above(c); r < m; r += NT) {
        const double2 a = rowp(r)[c];
        x[r] = make_double2(x[r].x - (a.x * v.x - a.y * v.y), x[r].y - (a.x * v.y + a.y * v.x));
      }
    }
    __syncthreads();
    // U z = v, backward: z_c = v_c / u_cc, v_r -= U(r, c) z_c (r < c)
    for (int c = m - 1; c >= 0; --c) {
      if (tid == c % NT) {
        const double2 u = rowp(c)[c], vc = x[c];
        const double den = u.x * u.x + u.y * u.y;
        const double2 z = make_double2((vc.x * u.x + vc.y * u.y) / den, (vc.y * u.x - vc.x * u.y) / den);
        x[c] = z;
        slot[c & 1] = z;
      }
      __syncthreads();
      const double2 z = slot[c & 1];
      for (int r = tid; r < c; r += NT) {
        const double2 a = rowp(r)[c];
        x[r] = make_double2(x[r].x - (a.x * z.x - a.y * z.y), x[r].y - (a.x * z.y + a.y * z.x));
      }
    }
    __syncthreads();
  }
}

// Singular-value certificate of a link from its LU: log |det| when that is at
// least log(1e-8) (then sigma_min >= |det| >= 1e-8), else log of the inverse
// iteration's upper bound of sigma_min (-inf for a zero pivot). The link is
// flagged singular when the certificate is below log(1e-8).
//
// arg det and log |det| of A_q (m x m, ld m) by blocked LU with partial
// pivoting, in place. The factorization runs on M = A_q^T (det M = det A_q),
// whose rows are contiguous in memory, so that row interchanges, the block
// row of U and the trailing update are all coalesced. Per panel of NB columns:
//   1. load rows k0.. of the panel into LDS (column by column), find the
//      first pivot while loading;
//   2. factor the panel in LDS, column by column (pivot, interchange within
//      the panel, multipliers, rank-1 update of the panel's later columns,
//      search for the next pivot fused with the update: two barriers per
//      column);
//   3. one thread per trailing column: apply the panel's interchanges and
//      solve with the unit lower triangle L11 (the panel's block row of U);
//   4. trailing update M22 -= L21 U12: a wave per row stream, lanes over
//      consecutive columns, U12 in registers, L21 broadcast from LDS.
// The factored panel is written back and its interchanges are applied to the
// columns left of it, so M ends holding the LU factors of its row-permuted
// self (read by lu_smin when |det| < 1e-8).
// phase[q] = sum of the pivots' arguments (+ pi per interchange), wrapped to
// (-pi, pi]; lsig[q] = the singular-value certificate above. A zero pivot
// leaves a zero column below it: nothing is eliminated.
template <int NB>
__global__ __launch_bounds__(DT) void k_det_phase(double2 *A, int m, int64_t sA, double *phase, double *lsig) {
  extern __shared__ double2 sP[];  // panel, column-major: sP[c * rows + r]
  __shared__ double s_v[DT / 64];
  __shared__ int s_i[DT / 64];
  __shared__ int s_piv[NB];
  __shared__ double s_la;
  double2 *M = A + int64_t(blockIdx.x) * sA;  // M[r][c] = M[r * m + c]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double ph = 0.0, la = 0.0;

  auto wave_best = [&](double best, int bi) {
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_v[wave] = best;
      s_i[wave] = bi;
    }
  };

  for (int k0 = 0; k0 < m; k0 += NB) {
    const int nbp = min(NB, m - k0), rows = m - k0;
    // ---- 1. panel load, pivot search of its first column
    {
      double best = -1.0;
      int bi = 0;
      for (int e = tid; e < rows * nbp; e += DT) {
        const int r = e / nbp, c = e - r * nbp;
        const double2 v = M[int64_t(k0 + r) * m + k0 + c];
        sP[c * rows + r] = v;
        if (c == 0) {
          const double a2 = v.x * v.x + v.y * v.y;
          if (a2 > best || (a2 == best && r < bi)) {
            best = a2;
            bi = r;
          }
        }
      }
      wave_best(best, bi);
    }
    __syncthreads();
    // ---- 2. panel factorization
    for (int c = 0; c < nbp; ++c) {
      double b = s_v[0];
      int p = s_i[0];
      for (int w = 1; w < DT / 64; ++w)
        if (s_v[w] > b || (s_v[w] == b && s_i[w] < p)) {
          b = s_v[w];
          p = s_i[w];
        }
      if (b < 0.0) p = c;  // no rows (cannot happen for c < rows)
      if (p != c)
        for (int cc = tid; cc < nbp; cc += DT) {
          const double2 t = sP[cc * rows + c];
          sP[cc * rows + c] = sP[cc * rows + p];
          sP[cc * rows + p] = t;
        }
      if (tid == 0) s_piv[c] = p;
      __syncthreads();
      const double2 piv = sP[c * rows + c];
      const double den = piv.x * piv.x + piv.y * piv.y;
      if (tid == 0) {
        ph += atan2(piv.y, piv.x) + (p != c ? kPi : 0.0);
        la += 0.5 * log(den);
      }
      const double2 ipv = den > 0.0 ? make_double2(piv.x / den, -piv.y / den) : make_double2(0.0, 0.0);
      double best = -1.0;
      int bi = c + 1;
      for (int r = c + 1 + tid; r < rows; r += DT) {
        const double2 a = sP[c * rows + r];
        const double2 l = make_double2(a.x * ipv.x - a.y * ipv.y, a.x * ipv.y + a.y * ipv.x);
        sP[c * rows + r] = l;
        for (int cc = c + 1; cc < nbp; ++cc) {
          const double2 u = sP[cc * rows + c];
          double2 x = sP[cc * rows + r];
          x.x -= l.x * u.x - l.y * u.y;
          x.y -= l.x * u.y + l.y * u.x;
          sP[cc * rows + r] = x;
          if (cc == c + 1) {
            const double a2 = x.x * x.x + x.y * x.y;
            if (a2 > best) {
              best = a2;
              bi = r;
            }
          }
        }
      }
      wave_best(best, bi);
      __syncthreads();
    }
    // the factored panel (L21 below, U11 on and above the diagonal) back to
    // M, and its interchanges applied to the columns left of it, so that M
    // ends as the LU factors of the row-permuted matrix (for sigma_min)
    for (int e = tid; e < rows * nbp; e += DT) {
      const int r = e / nbp, c = e - r * nbp;
      M[int64_t(k0 + r) * m + k0 + c] = sP[c * rows + r];
    }
#pragma unroll 1
    for (int jj = tid; jj < k0; jj += DT) {
#pragma unroll 1
      for (int c = 0; c < nbp; ++c) {
        const int p = s_piv[c];
        if (p != c) {
          const double2 t = M[int64_t(k0 + c) * m + jj];
          M[int64_t(k0 + c) * m + jj] = M[int64_t(k0 + p) * m + jj];
          M[int64_t(k0 + p) * m + jj] = t;
        }
      }
    }
    if (k0 + nbp >= m) break;
    // ---- 3. interchanges and U12 = L11^{-1} (P A12), one thread per trailing column
    const int j0 = k0 + nbp, C = m - j0;
#pragma unroll 1
    for (int jj = tid; jj < C; jj += DT) {
      const int j = j0 + jj;
#pragma unroll 1
      for (int c = 0; c < nbp; ++c) {
        const int p = s_piv[c];
        if (p != c) {
          const double2 t = M[int64_t(k0 + c) * m + j];
          M[int64_t(k0 + c) * m + j] = M[int64_t(k0 + p) * m + j];
          M[int64_t(k0 + p) * m + j] = t;
        }
      }
      double2 u[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < nbp) {
          double2 x = M[int64_t(k0 + c) * m + j];
#pragma unroll
          for (int cc = 0; cc < c; ++cc) {
            const double2 l = sP[cc * rows + c];
            x.x -= l.x * u[cc].x - l.y * u[cc].y;
            x.y -= l.x * u[cc].y + l.y * u[cc].x;
          }
          u[c] = x;
          M[int64_t(k0 + c) * m + j] = x;
        }
      }
    }
    __syncthreads();
    // ---- 4. trailing update M22 -= L21 U12
    for (int jb = 0; jb < C; jb += 64) {
      const int j = j0 + jb + lane;
      const bool ok = jb + lane < C;
      double2 u[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) u[c] = (ok && c < nbp) ? M[int64_t(k0 + c) * m + j] : make_double2(0.0, 0.0);
#pragma unroll 1
      for (int r = nbp + wave; r < rows; r += DT / 64) {
        if (!ok) continue;
        double2 x = M[int64_t(k0 + r) * m + j];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const double2 l = sP[c * rows + r];  // same address across the wave
          x.x -= l.x * u[c].x - l.y * u[c].y;
          x.y -= l.x * u[c].y + l.y * u[c].x;
        }
        M[int64_t(k0 + r) * m + j] = x;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    phase[blockIdx.x] = m > 0 ? wrap_pi(ph) : 0.0;
    s_la = la;
  }
  __syncthreads();
  la = s_la;
  if (la < kLogSingular && la > -INFINITY) {
    const double sg = lu_smin<DT>(M, m, nullptr, sP, sP + m, s_v);
    la = sg > 0.0 ? log(sg) : -INFINITY;
  }
  if (tid == 0) lsig[blockIdx.x] = la;
}

// The same factorization by one wave per link (orders up to 128), with the
// row interchanges kept as a permutation in LDS instead of moving rows in
// memory: the panel's rows are read through the permutation, the block row
// of U is solved in registers by the lane that owns its column and applied
// to the trailing rows at once, and no barrier waits for another wave. The
// pivots, their arguments and moduli are those of the workgroup kernel.
template <int NB>
__global__ __launch_bounds__(64) void k_det_phase_w(double2 *A, int m, int64_t sA, double *phase, double *lsig) {
  extern __shared__ double2 sP[];            // panel, column-major: sP[c * rows + r]
  int *perm = reinterpret_cast<int *>(sP + int64_t(m) * NB);  // logical row -> physical row
  double2 *M = A + int64_t(blockIdx.x) * sA;  // M[r][c] = M[r * m + c]
  const int lane = threadIdx.x;
  double ph = 0.0, la = 0.0;
  for (int r = lane; r < m; r += 64) perm[r] = r;
  __syncthreads();
  auto wave_best = [&](double best, int bi, double &ob, int &oi) {
    for (int o = 32; o > 0; o >>= 1) {
      const double v = __shfl_xor(best, o, 64);
      const int i = __shfl_xor(bi, o, 64);
      if (v > best || (v == best && i < bi)) {
        best = v;
        bi = i;
      }
    }
    ob = best;
    oi = bi;
  };
  for (int k0 = 0; k0 < m; k0 += NB) {
    const int nbp = min(NB, m - k0), rows = m - k0;
    double best = -1.0;
    int bi = 0;
    // panel load through the permutation, pivot search of its first column
    for (int e = lane; e < rows * nbp; e += 64) {
      const int r = e / nbp, c = e - r * nbp;
      const double2 v = M[int64_t(perm[k0 + r]) * m + k0 + c];
      sP[c * rows + r] = v;
      if (c == 0) {
        const double a2 = v.x * v.x + v.y * v.y;
        if (a2 > best || (a2 == best && r < bi)) {
          best = a2;
          bi = r;
        }
      }
    }
    double bv;
    int p;
    wave_best(best, bi, bv, p);
    __syncthreads();
    for (int c = 0; c < nbp; ++c) {
      if (bv < 0.0) p = c;
      if (p != c) {
        for (int cc = lane; cc < nbp; cc += 64) {
          const double2 t = sP[cc * rows + c];
          sP[cc * rows + c] = sP[cc * rows + p];
          sP[cc * rows + p] = t;
        }
        if (lane == 0) {
          const int t = perm[k0 + c];
          perm[k0 + c] = perm[k0 + p];
          perm[k0 + p] = t;
        }
      }
      __syncthreads();
      const double2 piv = sP[c * rows + c];
      const double den = piv.x * piv.x + piv.y * piv.y;
      ph += atan2(piv.y, piv.x) + (p != c ? kPi : 0.0);
      la += 0.5 * log(den);
      const double2 ipv = den > 0.0 ? make_double2(piv.x / den, -piv.y / den) : make_double2(0.0, 0.0);
      best = -1.0;
      bi = c + 1;
      for (int r = c + 1 + lane; r < rows; r += 64) {
        const double2 a = sP[c * rows + r];
        const double2 l = make_double2(a.x * ipv.x - a.y * ipv.y, a.x * ipv.y + a.y * ipv.x);
        sP[c * rows + r] = l;
        for (int cc = c + 1; cc < nbp; ++cc) {
          const double2 u = sP[cc * rows + c];
          double2 x = sP[cc * rows + r];
          x.x -= l.x * u.x - l.y * u.y;
          x.y -= l.x * u.y + l.y * u.x;
          sP[cc * rows + r] = x;
          if (cc == c + 1) {
            const double a2 = x.x * x.x + x.y * x.y;
            if (a2 > best) {
              best = a2;
              bi = r;
            }
          }
        }
      }
      wave_best(best, bi, bv, p);
      __syncthreads();
    }
    // the factored panel back to M (rows through the permutation), for sigma_min
    for (int e = lane; e < rows * nbp; e += 64) {
      const int r = e / nbp, c = e - r * nbp;
      M[int64_t(perm[k0 + r]) * m + k0 + c] = sP[c * rows + r];
    }
    if (k0 + nbp >= m) break;
    // block row of U (in registers, and stored) and trailing update, one lane per column
    const int j0 = k0 + nbp, C = m - j0;
    for (int jb = 0; jb < C; jb += 64) {
      const int j = j0 + jb + lane;
      if (jb + lane < C) {
        double2 u[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          if (c < nbp) {
            double2 x = M[int64_t(perm[k0 + c]) * m + j];
#pragma unroll
            for (int cc = 0; cc < c; ++cc) {
              const double2 l = sP[cc * rows + c];
              x.x -= l.x * u[cc].x - l.y * u[cc].y;
              x.y -= l.x * u[cc].y + l.y * u[cc].x;
            }
            u[c] = x;
            M[int64_t(perm[k0 + c]) * m + j] = x;
          } else {
            u[c] = make_double2(0.0, 0.0);
          }
        }
#pragma unroll 1
        for (int r = nbp; r < rows; ++r) {
          double2 *pr = M + int64_t(perm[k0 + r]) * m + j;
          double2 x = *pr;
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            const double2 l = sP[c * rows + r];
            x.x -= l.x * u[c].x - l.y * u[c].y;
            x.y -= l.x * u[c].y + l.y * u[c].x;
          }
          *pr = x;
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (la < kLogSingular && la > -INFINITY) {
    const double sg = lu_smin<64>(M, m, perm, sP, sP + m, nullptr);
    la = sg > 0.0 ? log(sg) : -INFINITY;
  }
  if (lane == 0) {
    phase[blockIdx.x] = m > 0 ? wrap_pi(ph) : 0.0;
    lsig[blockIdx.x] = la;
  }
}

// Panel width for order m: the widest whose panel (m x NB c128) fits in
// 160 KiB of LDS, preferring at most 64 KiB (several workgroups per CU).
int det_panel_width(int m) {
  if (m <= 256) return 16;
  if (m <= 512) return 8;
  if (m <= 2544) return 4;
  return 0;
}

// One workgroup per system: flux of every plaquette, its sum, Chern number
// and status. phi_par[(s n_perp + i) n_par + j]; phi_perp[(s n_par + j) n_perp + i].
__global__ __launch_bounds__(256) void k_plaquette(const double *phi_par, const double *phi_perp, const double *ls_par,
                                                   const double *ls_perp, int n_par, int n_perp, double *flux,
                                                   int32_t *chern, double *total, uint32_t *status) {
  const int64_t s = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t kps = int64_t(n_par) * n_perp;
  double sum = 0.0, fmx = 0.0, mpmin = INFINITY;
  for (int64_t e = tid; e < kps; e += 256) {
    const int i = int(e / n_par), j = int(e % n_par);
    const int i1 = i + 1 == n_perp ? 0 : i + 1, j1 = j + 1 == n_par ? 0 : j + 1;
    const double *pp = phi_par + s * kps;
    const double *pq = phi_perp + s * kps;
    const double F = wrap_pi(pp[int64_t(i1) * n_par + j] - pp[int64_t(i) * n_par + j] + pq[int64_t(j) * n_perp + i] -
                             pq[int64_t(j1) * n_perp + i]);
    flux[s * kps + e] = F;
    sum += F;
    fmx = fmax(fmx, fabs(F));
    mpmin = fmin(mpmin, fmin(ls_par[s * kps + e], ls_perp[s * kps + int64_t(j) * n_perp + i]));
  }
  for (int o = 32; o > 0; o >>= 1) {
    sum += __shfl_xor(sum, o, 64);
    fmx = fmax(fmx, __shfl_xor(fmx, o, 64));
    mpmin = fmin(mpmin, __shfl_xor(mpmin, o, 64));
  }
  __shared__ double r[3][4];
  if (lane == 0) {
    r[0][wave] = sum;
    r[1][wave] = fmx;
    r[2][wave] = mpmin;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0, c = INFINITY;
    for (int w = 0; w < 4; ++w) {
      a += r[0][w];
      b = fmax(b, r[1][w]);
      c = fmin(c, r[2][w]);
    }
    const double t = a / (2.0 * kPi);
    const double rt = rint(t);
    uint32_t st = 0;
    if (c < kLogSingular) st |= BE_ST_OVERLAP_SINGULAR;
    if (b > 0.8 * kPi || fabs(t - rt) > 1e-6) st |= BE_ST_WINDING_UNRESOLVED;
    const bool fin = isfinite(t) && fabs(t) < 1e9;
    if (!fin) st |= BE_ST_NAN_INF;
    total[s] = t;
    chern[s] = fin ? int32_t(rt) : 0;
    status[s] |= st;
  }
}

__global__ void k_zero_st(uint32_t *p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

// ---------------------------------------------------------------- scratch without allocation
// Fixed device scratch of be_plaquette_flux_noalloc (one copy per device,
// held for the life of the process). Host code never uses the array's name
// as an address: its device address comes from hipGetSymbolAddress, taken
// once per device at context creation.
static __device__ __align__(256) unsigned char scratch[BE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

namespace be {
// Called by be_create with `device` current.
int noalloc_scratch_init(be_ctx *ctx, int device) {
  if (device < 0 || device >= kMaxDevices) return set_err(ctx, BE_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return BE_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return set_err(ctx, BE_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_ptr[device] = ptr;
  return BE_OK;
}
}  // namespace be

namespace {

// Scratch of one flux call: the links of one direction for spp systems and
// four per-link arrays (phases and singular-value certificates, both directions).
struct FluxScratch {
  double2 *L = nullptr;
  double *ph_par = nullptr, *ph_perp = nullptr, *ls_par = nullptr, *ls_perp = nullptr;
  void declare(be::Carve &cv, int64_t spp, int64_t kps, int64_t mm) {
    cv.add(&L, size_t(spp * kps * mm));
    cv.add(&ph_par, size_t(spp * kps));
    cv.add(&ph_perp, size_t(spp * kps));
    cv.add(&ls_par, size_t(spp * kps));
    cv.add(&ls_perp, size_t(spp * kps));
  }
};

int check_flux_args(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride, int32_t n_sys,
                    int32_t n_par, int32_t n_perp, double *flux, int32_t *chern, double *total, uint32_t *status) {
  using namespace be;
  BE_CHECK_ARG(ctx, ctx && U && flux && chern && total && status, "be_plaquette_flux: null argument");
  BE_CHECK_ARG(ctx, N >= 1 && m >= 0 && m <= N, "be_plaquette_flux: need 0 <= m <= N");
  BE_CHECK_ARG(ctx, ldu >= N && u_stride >= int64_t(ldu) * std::max(m, 1), "be_plaquette_flux: ldu < N or u_stride < ldu*m");
  BE_CHECK_ARG(ctx, n_sys >= 0 && n_par >= 1 && n_perp >= 1, "be_plaquette_flux: need n_sys >= 0, n_par, n_perp >= 1");
  BE_CHECK_ARG(ctx, det_panel_width(m) > 0, "be_plaquette_flux: m > 2544 not supported");
  return BE_OK;
}

// The flux computation on scratch `fs` holding the links of spp systems.
int flux_run(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride, int32_t n_sys,
             int32_t n_par, int32_t n_perp, double *flux, int32_t *chern, double *total, uint32_t *status,
             const FluxScratch &fs, int64_t spp, hipStream_t stream) {
  using namespace be;
  const int nbw = det_panel_width(m);
  // dynamic LDS up to the panel size of the width in use (set on every call:
  // a cheap host call, valid for whichever device is current)
  if (nbw == 4)
    BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&k_det_phase<4>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 2544 * 4 * 16));
  else if (nbw == 8)
    BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&k_det_phase<8>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 512 * 8 * 16));
  else
    BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&k_det_phase<16>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 256 * 16 * 16));
  const int64_t kps = int64_t(n_par) * n_perp;
  const int64_t mm = int64_t(std::max(m, 1)) * std::max(m, 1);
  hipLaunchKernelGGL(k_zero_st, dim3((n_sys + 255) / 256), dim3(256), 0, stream, status, int64_t(n_sys));
  BE_RET_IF(check_launch(ctx, "zero"));
  double2 *L = fs.L;
  const double2 *Ud = static_cast<const double2 *>(U);
  for (int64_t s0 = 0; s0 < n_sys; s0 += spp) {
    const int64_t ns = std::min<int64_t>(spp, n_sys - s0);
    const int64_t nk = ns * kps;
    const double2 *Us = Ud + s0 * kps * u_stride;
    for (int dir = 0; dir < 2; ++dir) {
      if (m > 0) {
        ZGemm g;  // links U(k')^H U(k)
        g.M = m;
        g.N = m;
        g.K = N;
        g.opA = 1;
        g.A = Us;
        g.lda = ldu;
        g.B = Us;
        g.ldb = ldu;
        if (dir == 0) {  // k' = k(i, j+1): batch (s, i, j), j innermost and cyclic
          g.bA = ZBatch::cyclic(u_stride, n_par, 1, int64_t(n_par) * u_stride);
          g.bB = ZBatch::strided(u_stride);
        } else {  // k' = k(i+1, j): batch (s, j, i), i innermost and cyclic
          ZBatch a = ZBatch::cyclic(int64_t(n_par) * u_stride, n_perp, 1, kps * u_stride);
          a.s1 = u_stride;
          a.n1 = n_par;
          ZBatch b = a;
          b.shift = 0;
          g.bA = a;
          g.bB = b;
        }
        g.C = L;
        g.ldc = m;
        g.bC = ZBatch::strided(mm);
        g.batch = nk;
        g.tag = "flux_links";
        BE_RET_IF(zgemm(ctx, g, stream));
      }
      {
        ProfScope prof(ctx, "det_phase", stream);
        const size_t lds = size_t(std::max(m, 1)) * nbw * sizeof(double2);
        double *ph = dir == 0 ? fs.ph_par : fs.ph_perp, *ls = dir == 0 ? fs.ls_par : fs.ls_perp;
        const dim3 grid(static_cast<uint32_t>(nk));
        if (m <= 128)
          hipLaunchKernelGGL(k_det_phase_w<8>, grid, dim3(64), size_t(m) * 8 * sizeof(double2) + size_t(m) * 4,
                             stream, L, m, mm, ph, ls);
        else if (nbw == 16)
          hipLaunchKernelGGL(k_det_phase<16>, grid, dim3(DT), lds, stream, L, m, mm, ph, ls);
        else if (nbw == 8)
          hipLaunchKernelGGL(k_det_phase<8>, grid, dim3(DT), lds, stream, L, m, mm, ph, ls);
        else
          hipLaunchKernelGGL(k_det_phase<4>, grid, dim3(DT), lds, stream, L, m, mm, ph, ls);
      }
      BE_RET_IF(check_launch(ctx, "det_phase"));
    }
    hipLaunchKernelGGL(k_plaquette, dim3(static_cast<uint32_t>(ns)), dim3(256), 0, stream, fs.ph_par, fs.ph_perp,
                       fs.ls_par, fs.ls_perp, n_par, n_perp, flux + s0 * kps, chern + s0, total + s0, status + s0);
    BE_RET_IF(check_launch(ctx, "plaquette"));
  }
  return BE_OK;
}

}  // namespace

extern "C" int be_plaquette_flux(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                                 int32_t n_sys, int32_t n_par, int32_t n_perp, double *flux, int32_t *chern,
                                 double *total, uint32_t *status, hipStream_t stream) {
  using namespace be;
  BE_RET_IF(check_flux_args(ctx, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status));
  if (n_sys == 0) return BE_OK;
  const int64_t kps = int64_t(n_par) * n_perp;
  const int64_t mm = int64_t(std::max(m, 1)) * std::max(m, 1);
  // systems per pass: the links of one direction within about 1 GiB
  const int64_t per = std::max<int64_t>(1, (int64_t(1) << 30) / (kps * mm * int64_t(sizeof(double2))));
  const int64_t spp = std::min<int64_t>(per, n_sys);
  FluxScratch fs;
  Carve cv;
  fs.declare(cv, spp, kps, mm);
  BE_RET_IF(cv.commit(ctx, stream, WS_WILSON));
  return flux_run(ctx, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status, fs, spp, stream);
}

extern "C" int be_plaquette_flux_noalloc(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu,
                                         int64_t u_stride, int32_t n_sys, int32_t n_par, int32_t n_perp, double *flux,
                                         int32_t *chern, double *total, uint32_t *status, hipStream_t stream) {
  using namespace be;
  BE_RET_IF(check_flux_args(ctx, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status));
  if (n_sys == 0) return BE_OK;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch_ptr[ctx->device] : nullptr;
  }
  if (!base) return set_err(ctx, BE_EHIP, "be_plaquette_flux_noalloc: no scratch address for this device");
  const int64_t kps = int64_t(n_par) * n_perp;
  const int64_t mm = int64_t(std::max(m, 1)) * std::max(m, 1);
  // as many systems per pass as the fixed scratch holds (at least one)
  auto bytes = [&](int64_t spp) {
    FluxScratch f;
    Carve c;
    f.declare(c, spp, kps, mm);
    return c.total();
  };
  const size_t cap = size_t(BE_NOALLOC_SCRATCH_BYTES);
  if (bytes(1) > cap)
    return set_err(ctx, BE_EINVAL, "be_plaquette_flux_noalloc: one system needs " + std::to_string(bytes(1)) +
                                       " bytes of scratch, more than the fixed " + std::to_string(cap));
  int64_t spp = std::min<int64_t>(n_sys, std::max<int64_t>(1, int64_t(cap / bytes(1))));
  while (spp > 1 && bytes(spp) > cap) --spp;
  FluxScratch fs;
  Carve cv;
  fs.declare(cv, spp, kps, mm);
  cv.place(base);
  return flux_run(ctx, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status, fs, spp, stream);
}

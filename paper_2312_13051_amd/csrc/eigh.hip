// Rows (a3)-(a5): batched Hermitian eigensolver for the selected bands.
//
// 1. Blocked Householder reduction to real symmetric tridiagonal form,
//    Q^H H Q = T with Q = H_0 H_1 ... H_{N-2}, H_j = I - tau_j v_j v_j^H.
//    One workgroup per matrix runs a panel of nb columns (hetrd_panel): for
//    each column it applies the panel's earlier reflectors to that column,
//    builds the reflector, forms the matrix-vector product with the trailing
//    matrix from its lower triangle only (each 64 x 64 tile read once and
//    applied as A v and A^H v) and the symmetric rank-2 correction vector w.
//    The trailing matrix is then updated once per panel by a rank-2nb MFMA
//    GEMM, C -= [V W] [W V]^H, on its lower tiles only (the upper triangle is
//    never read again). The
//    panel's compact-WY factor T (Q_panel = I - V T V^H) is accumulated on the
//    fly from the same dot products.
// 2. FP64 tridiagonal eigensolver (tri_bisect, tri_invit, tri_gs): bisection with Sturm counts,
//    one lane per eigenvalue, for the selected indices and their neighbours;
//    T is split where an off-diagonal is negligible (an eigenvalue of
//    multiplicity k forces k-1 such splits), and the k lanes of a k-fold
//    eigenvalue run inverse iteration (partial pivoting, pseudo-random start)
//    on k distinct blocks that hold it, so their vectors have disjoint
//    supports; lanes that must share a block fall back to Gram-Schmidt. The
//    vectors are then orthonormalized in FP64 by Newton-Schulz steps on the
//    Gram matrix (symmetric orthonormalization, MFMA DGEMMs) until
//    max |Z^T Z - I| < 1e-14 (5e-8 on the mixed path).
// 3. Back-transformation U = Q Z by pairs of panels in reverse order, each
//    pair one compact-WY block of 64 columns, V = [V1 V2],
//    T = [[T1, -T1 (V1^H V2) T2], [0, T2]], applied with three MFMA GEMMs:
//    X = V^H U, Y = T X, U -= V Y.
// 4. Mixed precision: the reduction and back-transformation run in FP32 on
//    FP32 MFMA; the tridiagonal solve and the orthonormalization stay FP64.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "common.hpp"

namespace {

constexpr int NB = 32;   // panel width
constexpr int PT = 256;   // threads of the tridiagonal and small kernels

template <typename T>
struct CT;
template <>
struct CT<double> {
  typedef double2 c;
};
template <>
struct CT<float> {
  typedef float2 c;
};

template <typename C>
__host__ __device__ __forceinline__ C mk(double x, double y) {
  C r;
  r.x = x;
  r.y = y;
  return r;
}

// Byte offset of the panel kernel's partial vectors in its dynamic LDS: after
// v, y (N each), four NB vectors, the NB x NB T factor and the reduction
// scratch (2 values per wave), 64-byte aligned.
__host__ __device__ inline size_t panel_part_offset(int N, size_t csize, int nt) {
  return ((2 * size_t(N) + 4 * NB + NB * NB) * csize + 2 * size_t(nt / 64) * (csize / 2) + 63) & ~size_t(63);
}

// Column groups per tile of the panel's matrix-vector product for a trailing
// matrix of nrb 64-row blocks: small trailing matrices have few tiles, so each
// tile is split into S groups of 64/S columns to give every wave work.
__host__ __device__ inline int panel_split(int nrb) { return nrb >= 5 ? 1 : nrb >= 3 ? 2 : 4; }

// ---------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of two values (all threads get the result).
template <typename T>
__device__ __forceinline__ void block_sum2(T &a, T &b, T *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane == 0) {
    red[2 * wave] = a;
    red[2 * wave + 1] = b;
  }
  __syncthreads();
  T sa = 0, sb = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    sa += red[2 * w];
    sb += red[2 * w + 1];
  }
  a = sa;
  b = sb;
  __syncthreads();
}

// Column sums over the 64 lanes of a wave for CW columns at once (CW = 4, 8
// or 16): lane L holds the products of its row with the CW columns in
// (pr[c], pi[c]). Butterfly transpose: at offset o (32, 16, ...) each lane
// keeps the half of its columns selected by bit o of L, adds the partner's
// copy of that half and passes on the other half, so every exchange halves
// the columns a lane holds; after log2(CW) exchanges lane L holds one column,
// c = L >> log2(64/CW), summed over the lanes that differ in the upper bits,
// and the remaining offsets (lanes holding the same column) are summed
// plainly. Every lane returns the complete sum of its column c; the order of
// the additions is fixed.
template <int CW, typename C>
__device__ __forceinline__ C xpose_colsum(C (&p)[CW], int lane) {
  constexpr int LOG = CW == 16 ? 4 : CW == 8 ? 3 : CW == 4 ? 2 : 1;
#pragma unroll
  for (int st = 0; st < LOG; ++st) {
    const int h = CW >> (st + 1), o = 32 >> st;
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int t = 0; t < h; ++t) {
      const C lo = p[t], hi = p[t + h];
      const C send = up ? lo : hi;
      const C keep = up ? hi : lo;
      p[t].x = keep.x + __shfl_xor(send.x, o, 64);
      p[t].y = keep.y + __shfl_xor(send.y, o, 64);
    }
  }
  C a = p[0];
#pragma unroll
  for (int o = 32 / CW; o >= 1; o >>= 1) {
    a.x += __shfl_xor(a.x, o, 64);
    a.y += __shfl_xor(a.y, o, 64);
  }
  return a;
}

// ---------------------------------------------------------------- panel kernel
// A: matrices (lower triangle and diagonal read; the upper triangle is
// ignored), VW: [V | W | V] panel buffers (N x 3NB, leading dimension N), Tm:
// per-matrix NB x NB compact-WY factor of each panel, d/e: FP64 tridiagonal
// output. Partial vectors of the matrix-vector product: in LDS after the
// panel's other arrays (PL), else at Pg + q*sPg (global scratch of
// (nrb+1)*nrb*64 elements, nrb = ceil((N-1)/64)). CW: loads in flight per
// lane in the matrix-vector product (columns per transposed column sum, 4 or
// 8); the FP32 kernels of up to 512 threads with 4 loads keep six waves per
// SIMD resident, with 8 loads four (the registers the loads take).
template <typename T, int NT, bool PL, int CW>
__global__ __launch_bounds__(NT, sizeof(T) == 4 ? (NT == 1024 ? 1 : CW == 4 ? 6 : 4) : 1) void hetrd_panel(typename CT<T>::c *A, int64_t sA, int lda, int N, int p0, int nbp,
                                                  typename CT<T>::c *VW, int64_t sVW, typename CT<T>::c *Tm,
                                                  int64_t sTm, double *d, double *e, int64_t sDE,
                                                  typename CT<T>::c *Pg, int64_t sPg, uint32_t *status) {
  typedef typename CT<T>::c C;
  static_assert(CW == 4 || CW == 8, "4 or 8 loads in flight");
  constexpr int CSH = CW == 8 ? 3 : 4;  // lane -> column shift of xpose_colsum<CW>
  extern __shared__ unsigned char smem_raw[];
  C *sv = reinterpret_cast<C *>(smem_raw);  // v, length N
  C *sy = sv + N;                           // y / w, length N
  C *sVr = sy + N;                          // row j of V (NB)
  C *sWr = sVr + NB;                        // row j of W (NB)
  C *st1 = sWr + NB;                        // W^H v (NB)
  C *st2 = st1 + NB;                        // V^H v (NB)
  C *sT = st2 + NB;                         // NB x NB, column-major
  T *red = reinterpret_cast<T *>(sT + NB * NB);  // 2 * waves
  __shared__ C s_tau, s_scal;
  __shared__ T s_beta;

  const int64_t q = blockIdx.x;
  C *Aq = A + q * sA;
  C *part = PL ? reinterpret_cast<C *>(smem_raw + panel_part_offset(N, sizeof(C), NT)) : Pg + q * sPg;
  C *V = VW + q * sVW;
  C *W = V + int64_t(NB) * N;
  C *V2 = W + int64_t(NB) * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = NT / 64;

  for (int e2 = tid; e2 < NB * NB; e2 += NT) sT[e2] = mk<C>(0, 0);
  __syncthreads();

  for (int jj = 0; jj < nbp; ++jj) {
    const int j = p0 + jj;
    // ---- (1) apply the panel's earlier reflectors to column j,
    //   a -= V(r,c) conj(W(j,c)) + W(r,c) conj(V(j,c)),  c < jj.
    // The terms c < jj-1 were applied during the previous column's pass over
    // V and W (step 6); the term c = jj-1 uses that column's v and w, which
    // are still in LDS.
    for (int r = j + tid; r < N; r += NT) {
      C a = Aq[r + int64_t(j) * lda];
      T ar = a.x, ai = a.y;
      if (jj > 0) {
        const C vr = sv[r], wr = sy[r], wj = sy[j], vj = sv[j];
        ar -= vr.x * wj.x + vr.y * wj.y + wr.x * vj.x + wr.y * vj.y;
        ai -= vr.y * wj.x - vr.x * wj.y + wr.y * vj.x - wr.x * vj.y;
      }
      if (r == j) {
        ai = 0;
        d[q * sDE + j] = double(ar);
      }
      Aq[r + int64_t(j) * lda] = mk<C>(ar, ai);
    }
    // row j+1 of V and W (columns < jj), for step 6's share of column j+1
    for (int c = tid; c < jj; c += NT) {
      if (j + 1 < N) {
        sVr[c] = V[j + 1 + int64_t(c) * N];
        sWr[c] = W[j + 1 + int64_t(c) * N];
      }
    }
    __syncthreads();
    if (j == N - 1) {
      // last column: no reflector. Column j of V and W is zero.
      for (int r = tid; r < N; r += NT) {
        Aq[r + int64_t(j) * lda] = mk<C>(0, 0);
        V[r + int64_t(jj) * N] = mk<C>(0, 0);
        W[r + int64_t(jj) * N] = mk<C>(0, 0);
        V2[r + int64_t(jj) * N] = mk<C>(0, 0);
      }
      __syncthreads();
      break;
    }
    // ---- (2) reflector from A(j+1:N, j)
    T xn = 0, dummy = 0;
    for (int r = j + 2 + tid; r < N; r += NT) {
      C a = Aq[r + int64_t(j) * lda];
      xn += a.x * a.x + a.y * a.y;
    }
    block_sum2(xn, dummy, red);
    if (tid == 0) {
      C alpha = Aq[(j + 1) + int64_t(j) * lda];
      C tau, scal;
      T beta;
      if (xn == T(0) && alpha.y == T(0)) {
        tau = mk<C>(0, 0);
        scal = mk<C>(0, 0);
        beta = alpha.x;
      } else {
        T nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn);
        beta = alpha.x >= T(0) ? -nrm : nrm;
        tau = mk<C>((beta - alpha.x) / beta, -alpha.y / beta);
        // scal = 1 / (alpha - beta)
        T dr = alpha.x - beta, di = alpha.y;
        T den = dr * dr + di * di;
        scal = mk<C>(dr / den, -di / den);
      }
      s_tau = tau;
      s_scal = scal;
      s_beta = beta;
      e[q * sDE + j] = double(beta);
    }
    __syncthreads();
    const C tau = s_tau, scal = s_scal;
    // v: zero above j+1, one at j+1, scaled x below; into LDS, A's column j, V and V2
    for (int r = tid; r < N; r += NT) {
      C v;
      if (r <= j) {
        v = mk<C>(0, 0);
      } else if (r == j + 1) {
        v = mk<C>(1, 0);
      } else {
        C a = Aq[r + int64_t(j) * lda];
        v = mk<C>(a.x * scal.x - a.y * scal.y, a.x * scal.y + a.y * scal.x);
      }
      sv[r] = v;
      sy[r] = mk<C>(0, 0);
      Aq[r + int64_t(j) * lda] = v;
      V[r + int64_t(jj) * N] = v;
      V2[r + int64_t(jj) * N] = v;
    }
    __syncthreads();
    // ---- (3) y = A(j+1:N, j+1:N) v from the lower triangle only. The
    // trailing matrix is cut into 64 x 64 tiles (bi, bj), bi >= bj, counted
    // from row j+1, each split into S groups of columns (S = 1 unless the
    // trailing matrix is small); a work item (tile, group) is read once, by one
    // wave (lane = row, coalesced 64-row column segments), and applied twice:
    // A_t v (row sums in the lane) to block bi and A_t^H v (column sums over
    // lanes, xpose_colsum) to block bj. A diagonal tile reads only its entries
    // on and below the diagonal. The partial vectors go to slots of 64
    // elements, per block b: first a row slot for each (bj <= b, group), then
    // a column slot for each bi >= b (bi = b: the diagonal tile's column
    // part); the slots of a row are summed in this order, so the result does
    // not depend on scheduling.
    const int r0 = j + 1;
    const int nrb = (N - r0 + 63) >> 6;
    const int S = panel_split(nrb), gw = 64 / S;  // groups per tile, columns per group
    const int nslot = nrb * S + 1;                // slots per block (at most)
    {
      // items it = t S + g over tiles t = bi (bi + 1) / 2 + bj in row-major
      // order of the lower triangle, dealt round-robin to the waves; all
      // indices stay wave-uniform (scalar)
      const int wv = __builtin_amdgcn_readfirstlane(wave);
      const int nitem = nrb * (nrb + 1) / 2 * S;
      int it = wv, t = it / S, bi = 0, bj = t;
      while (bj > bi) {
        bj -= bi + 1;
        ++bi;
      }
      while (it < nitem) {
        const int g = it - t * S;
        const bool diag = bi == bj;
        const int r = r0 + 64 * bi + lane, cb0 = r0 + 64 * bj + g * gw;
        const bool rok = r < N;
        const C vr = rok ? sv[r] : mk<C>(0, 0);
        const uint32_t roff = uint32_t(rok ? r : r0) * uint32_t(sizeof(C));
        C *pcol = part + (bj * nslot + (bj + 1) * S + (bi - bj)) * 64 + g * gw;
        T yr = 0, yi = 0;
        // one chunk of CW columns: loads (all in flight), row part, column part
        auto chunk = [&](const int k, auto full_tag) {
          constexpr bool full = decltype(full_tag)::value;  // interior tile: nothing masked
          const int c0 = cb0 + k;
          const C *cp = Aq + int64_t(c0) * lda;  // uniform: column c0, row 0
          C a[CW];
#pragma unroll
          for (int u = 0; u < CW; ++u) {
            const int c = c0 + u;
            // uniform column base plus one 32-bit per-lane row offset
            const C *ap = reinterpret_cast<const C *>(reinterpret_cast<const char *>(cp + int64_t(u) * lda) + roff);
            if (full)
              a[u] = *ap;
            else
              a[u] = (c < N && rok && (!diag || r >= c)) ? *ap : mk<C>(0, 0);
          }
#pragma unroll
          for (int u = 0; u < CW; ++u) {
            const int c = c0 + u;
            const C vc = (full || c < N) ? sv[c] : mk<C>(0, 0);
            const bool dg = !full && diag && r == c;
            const T ax = a[u].x, ay = dg ? T(0) : a[u].y;  // the diagonal is real
            yr += ax * vc.x - ay * vc.y;
            yi += ax * vc.y + ay * vc.x;
            // column part: conj(a) v_r (the diagonal entry is in the row part)
            a[u] = dg ? mk<C>(0, 0) : mk<C>(ax * vr.x + ay * vr.y, ax * vr.y - ay * vr.x);
          }
          const C sc = xpose_colsum<CW>(a, lane);
          if ((lane & ((1 << CSH) - 1)) == 0) pcol[k + (lane >> CSH)] = sc;
        };
        if (!diag && 64 * (bi + 1) <= N - r0) {
#pragma unroll 1
          for (int k = 0; k < gw; k += CW) chunk(k, std::true_type{});
        } else {
#pragma unroll 1
          for (int k = 0; k < gw; k += CW) chunk(k, std::false_type{});
        }
        part[(bi * nslot + bj * S + g) * 64 + lane] = mk<C>(yr, yi);
        it += nw;
        const int t2 = it / S;
        bj += t2 - t;
        t = t2;
        while (bj > bi) {
          bj -= bi + 1;
          ++bi;
        }
      }
    }
    __syncthreads();
    for (int r = r0 + tid; r < N; r += NT) {
      const int b = (r - r0) >> 6, l = (r - r0) & 63;
      const C *pb = part + b * nslot * 64 + l;
      T sr = 0, si = 0;
      for (int s2 = 0; s2 < (b + 1) * S + nrb - b; ++s2) {  // row slots, then column slots
        const C x = pb[s2 * 64];
        sr += x.x;
        si += x.y;
      }
      sy[r] = mk<C>(sr, si);
    }
    // ---- (4) t1 = W^H v, t2 = V^H v over rows j+1..N-1 (one wave per column c)
    for (int c = wave; c < jj; c += nw) {
      T a_r = 0, a_i = 0, b_r = 0, b_i = 0;
      for (int r = r0 + lane; r < N; r += 64) {
        C v = sv[r], w = W[r + int64_t(c) * N], vv = V[r + int64_t(c) * N];
        a_r += w.x * v.x + w.y * v.y;
        a_i += w.x * v.y - w.y * v.x;
        b_r += vv.x * v.x + vv.y * v.y;
        b_i += vv.x * v.y - vv.y * v.x;
      }
      a_r = wave_sum(a_r);
      a_i = wave_sum(a_i);
      b_r = wave_sum(b_r);
      b_i = wave_sum(b_i);
      if (lane == 0) {
        st1[c] = mk<C>(a_r, a_i);
        st2[c] = mk<C>(b_r, b_i);
      }
    }
    __syncthreads();
    // y -= V t1 + W t2; with the same loads of V(r, c) and W(r, c), the
    // terms c < jj of step 1 for column j+1 when it belongs to this panel
    const bool fuse = jj > 0 && jj + 1 < nbp && j + 1 < N;
    for (int r = r0 + tid; r < N; r += NT) {
      C y = sy[r];
      T yr = y.x, yi = y.y, pr = 0, pi = 0;
      for (int c = 0; c < jj; ++c) {
        C vv = V[r + int64_t(c) * N], w = W[r + int64_t(c) * N], a = st1[c], b = st2[c];
        yr -= vv.x * a.x - vv.y * a.y + w.x * b.x - w.y * b.y;
        yi -= vv.x * a.y + vv.y * a.x + w.x * b.y + w.y * b.x;
        const C wj = sWr[c], vj = sVr[c];
        pr += vv.x * wj.x + vv.y * wj.y + w.x * vj.x + w.y * vj.y;
        pi += vv.y * wj.x - vv.x * wj.y + w.y * vj.x - w.x * vj.y;
      }
      // w = tau * y
      sy[r] = mk<C>(tau.x * yr - tau.y * yi, tau.x * yi + tau.y * yr);
      if (fuse) {
        const C a0 = Aq[r + int64_t(j + 1) * lda];
        Aq[r + int64_t(j + 1) * lda] = mk<C>(a0.x - pr, a0.y - pi);
      }
    }
    // compact-WY column: T(0:jj, jj) = -tau T(0:jj, 0:jj) t2, T(jj, jj) = tau
    if (tid < jj) {
      const int rr = tid;
      T xr = 0, xi = 0;
      for (int c = rr; c < jj; ++c) {
        C tt = sT[rr + c * NB], b = st2[c];
        xr += tt.x * b.x - tt.y * b.y;
        xi += tt.x * b.y + tt.y * b.x;
      }
      sT[rr + jj * NB] = mk<C>(-(tau.x * xr - tau.y * xi), -(tau.x * xi + tau.y * xr));
    }
    if (tid == 0) sT[jj + jj * NB] = tau;
    __syncthreads();
    // ---- (5) w += alpha v with alpha = -1/2 tau (w^H v)
    T dr = 0, di = 0;
    for (int r = r0 + tid; r < N; r += NT) {
      C w = sy[r], v = sv[r];
      dr += w.x * v.x + w.y * v.y;
      di += w.x * v.y - w.y * v.x;
    }
    block_sum2(dr, di, red);
    const T alr = T(-0.5) * (tau.x * dr - tau.y * di), ali = T(-0.5) * (tau.x * di + tau.y * dr);
    for (int r = tid; r < N; r += NT) {
      C w;
      if (r < r0) {
        w = mk<C>(0, 0);
      } else {
        C y = sy[r], v = sv[r];
        w = mk<C>(y.x + alr * v.x - ali * v.y, y.y + alr * v.y + ali * v.x);
      }
      W[r + int64_t(jj) * N] = w;
      sy[r] = w;  // kept for step 1 of the next column
    }
    __syncthreads();
  }
  // ---- write the panel's T factor
  C *Tq = Tm + q * sTm;
  for (int e2 = tid; e2 < NB * NB; e2 += NT) Tq[e2] = sT[e2];
  (void)status;
}

// ---------------------------------------------------------------- tridiagonal solver
// a / b as a times the hardware reciprocal of b refined by one Newton-Raphson
// step: within a few ulps of the rounded quotient, for normal b (the Sturm
// recurrence keeps |b| >= pivmin >= DBL_MIN, so 1/b and a/b stay finite).
__device__ __forceinline__ double div_nr(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  return a * r;
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T
// factorization of T - x I). The quotient uses div_nr: the count is that of a
// matrix within a few ulps of T, the same kind of backward error the
// correctly rounded division gives.
__device__ __forceinline__ int sturm_count(const double *sd, const double *se2, int N, double x, double pivmin) {
  int cnt = 0;
  double qv = sd[0] - x;
  if (fabs(qv) < pivmin) qv = -pivmin;
  cnt += qv < 0.0;
  for (int i = 1; i < N; ++i) {
    qv = (sd[i] - x) - div_nr(se2[i - 1], qv);
    if (fabs(qv) < pivmin) qv = -pivmin;
    cnt += qv < 0.0;
  }
  return cnt;
}

// The same count from the interleaved pairs sde[i] = (d_i, e_{i-1}^2): one
// LDS read per step, four steps' reads issued together.
__device__ __forceinline__ int sturm_count_i(const double2 *sde, int N, double x, double pivmin) {
  int cnt = 0;
  double qv = sde[0].x - x;
  if (fabs(qv) < pivmin) qv = -pivmin;
  cnt += qv < 0.0;
#pragma unroll 4
  for (int i = 1; i < N; ++i) {
    const double2 de = sde[i];
    qv = (de.x - x) - div_nr(de.y, qv);
    if (fabs(qv) < pivmin) qv = -pivmin;
    cnt += qv < 0.0;
  }
  return cnt;
}

__device__ __forceinline__ double hash_unit(uint64_t a, uint64_t b) {
  // splitmix64 of (a, b) -> uniform in (-1, 1)
  uint64_t z = a * 0x9E3779B97F4A7C15ull + b + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Per-matrix scratch of the tridiagonal solver: lam [m + 1] = (||T||, selected
// eigenvalues), Zs: 4 arrays [N][mp] (the diagonals met by the elimination of
// inverse iteration, two arrays of orthonormalization scratch, x) with the
// eigenvector index fastest, marks [m] (1 at the first index of a cluster whose vectors
// share a block of T).

// Loads d, e of matrix q into LDS; returns false (and flags the matrix, with
// NaN outputs) if an entry is not finite.
__device__ bool load_tridiag(const double *d, const double *e, int64_t q, int64_t sDE, int N, double *sd, double *se,
                             double *se2, int *s_bad) {
  const int tid = threadIdx.x;
  if (tid == 0) *s_bad = 0;
  __syncthreads();
  for (int i = tid; i < N; i += blockDim.x) {
    const double di = d[q * sDE + i];
    const double ei = i < N - 1 ? e[q * sDE + i] : 0.0;
    if (!isfinite(di) || !isfinite(ei)) *s_bad = 1;
    sd[i] = di;
    if (se) se[i] = ei;
    se2[i] = ei * ei;
  }
  __syncthreads();
  return *s_bad == 0;
}

// (a4) eigenvalues by bisection with Sturm counts, one lane per wanted index:
// the selected [lo, hi), their neighbours lo-1 and hi (for the gap test) and
// the extremes 0 and N-1 (for the scale). At most max_it bisection steps per
// eigenvalue after the multisection (128 does not bind: see tol_abs); an
// eigenvalue left wider than its tolerance flags the matrix
// BE_ST_NONCONVERGED.
__global__ __launch_bounds__(PT) void tri_bisect(const double *d, const double *e, int64_t sDE, int N, int lo, int hi,
                                                 double bis_rel, int max_it, double *evals, double *lamg, double2 *U,
                                                 int ldu, int64_t sU, uint32_t *status) {
  extern __shared__ double2 tsm2[];
  double2 *sde = tsm2;                                // N: (d_i, e_{i-1}^2)
  double *sd = reinterpret_cast<double *>(sde + N);  // N
  double *se2 = sd + N;                               // N
  double *slam = se2 + N;  // m + 4: [lambda_0, lambda_{N-1}, lambda_{lo-1}, lambda_{hi}, lambda_lo..]
  const int m = hi - lo;
  __shared__ int s_bad;
  __shared__ double mm[3 * (PT / 64)];
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = PT / 64;
  if (!load_tridiag(d, e, q, sDE, N, sd, nullptr, se2, &s_bad)) {
    if (tid == 0) status[q] |= BE_ST_NAN_INF;
    for (int c = tid; c < m + 2; c += PT) evals[q * (m + 2) + c] = NAN;
    for (int c = tid; c <= m; c += PT) lamg[q * (m + 1) + c] = NAN;
    for (int64_t k = tid; k < int64_t(N) * m; k += PT) {
      const int c = int(k / N), r = int(k % N);
      U[q * sU + r + int64_t(c) * ldu] = make_double2(NAN, NAN);
    }
    return;
  }
  for (int i = tid; i < N; i += PT) sde[i] = make_double2(sd[i], i > 0 ? se2[i - 1] : 0.0);
  // Gershgorin interval and pivot threshold
  double gl = INFINITY, gu = -INFINITY, emax2 = 0.0;
  for (int i = tid; i < N; i += PT) {
    const double rad = sqrt(se2[i]) + (i > 0 ? sqrt(se2[i - 1]) : 0.0);
    gl = fmin(gl, sd[i] - rad);
    gu = fmax(gu, sd[i] + rad);
    emax2 = fmax(emax2, se2[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, o, 64));
    gu = fmax(gu, __shfl_xor(gu, o, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
  }
  if (lane == 0) {
    mm[3 * wave] = gl;
    mm[3 * wave + 1] = gu;
    mm[3 * wave + 2] = emax2;
  }
  __syncthreads();
  gl = mm[0];
  gu = mm[1];
  emax2 = mm[2];
  for (int w = 1; w < nw; ++w) {
    gl = fmin(gl, mm[3 * w]);
    gu = fmax(gu, mm[3 * w + 1]);
    emax2 = fmax(emax2, mm[3 * w + 2]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double eps = DBL_EPSILON;
  gl -= 2.0 * eps * tnorm + 2.0 * pivmin;
  gu += 2.0 * eps * tnorm + 2.0 * pivmin;
  // absolute floor eps^2 ||T||: far below any attainable accuracy, it only
  // ends the halving at an eigenvalue (near) zero, where eps |lambda| alone
  // would ask for ~1000 steps; from an interval of 1/257 of the Gershgorin
  // width it takes at most ~97 steps
  const double tol_abs = fmax(bis_rel, DBL_EPSILON * DBL_EPSILON) * tnorm;
  // multisection: Sturm counts at PT points spread over the Gershgorin
  // interval (one per thread) bracket every eigenvalue to one of PT + 1
  // subintervals, which replaces the first ~8 bisection steps of every lane
  __shared__ int s_cnt[PT];
  const double hstep = (gu - gl) / double(PT + 1);
  s_cnt[tid] = sturm_count_i(sde, N, gl + double(tid + 1) * hstep, pivmin);
  __syncthreads();
  const int nidx = m + 4;
  for (int t = tid; t < nidx; t += PT) {
    int k;
    if (t == 0) k = 0;
    else if (t == 1) k = N - 1;
    else if (t == 2) k = lo > 0 ? lo - 1 : -1;
    else if (t == 3) k = hi < N ? hi : -1;
    else k = lo + (t - 4);
    double val = NAN;
    if (k >= 0) {
      // subinterval u: count(x_u) <= k < count(x_{u+1}), x_0 = gl, x_{PT+1} = gu
      int u = 0;
      while (u < PT && s_cnt[u] <= k) ++u;
      double a = u == 0 ? gl : gl + double(u) * hstep, b = u == PT ? gu : gl + double(u + 1) * hstep;
      bool conv = false;
      for (int it = 0; it <= max_it; ++it) {
        const double mid = 0.5 * (a + b);
        conv = b - a <= fmax(2.0 * eps * fmax(fabs(a), fabs(b)) + pivmin, tol_abs) || mid <= a || mid >= b;
        if (conv || it == max_it) break;
        if (sturm_count_i(sde, N, mid, pivmin) > k) b = mid;
        else a = mid;
      }
      if (!conv) atomicOr(&status[q], BE_ST_NONCONVERGED);
      val = 0.5 * (a + b);
    }
    slam[t] = val;
  }
  __syncthreads();
  const double *lam = slam + 4;
  for (int c = tid; c < m + 2; c += PT) evals[q * (m + 2) + c] = c == 0 ? slam[2] : (c == m + 1 ? slam[3] : lam[c - 1]);
  for (int c = tid; c <= m; c += PT) lamg[q * (m + 1) + c] = c == 0 ? tnorm : lam[c - 1];
  if (tid == 0) {
    const double scale = fmax(1.0, fmax(fabs(slam[0]), fabs(slam[1])));
    double g = INFINITY;
    if (lo > 0 && m > 0) g = fmin(g, lam[0] - slam[2]);
    if (hi < N && m > 0) g = fmin(g, slam[3] - lam[m - 1]);
    if (g < 1e-9 * scale) atomicOr(&status[q], BE_ST_GAP_CLOSED);
  }
}

// Tolerances relative to ||T||: split < block window < cluster gap, so a
// cluster's window never reaches the next cluster. Eigenvalues closer than
// the cluster tolerance (clu_rel, by default kCluRel = 1e-12) form a cluster, whose vectors are
// computed as one invariant subspace (any orthonormal basis of it): inverse
// iteration separates two eigenvalues only to about eps ||T|| / gap, so
// below that gap their vectors can come out nearly parallel (a cluster of
// eigenvalues spread over 1e-12 ||T|| - e.g. the projected spin operator's
// +-1 clusters computed from refined eigenvectors, whose T splits into many
// blocks - would otherwise have lanes pick blocks by windows narrower than
// the cluster, and leave an orthonormalization that cannot converge). A
// caller that needs the vectors of nearly equal eigenvalues resolved one by
// one (and validates them) may pass a smaller tolerance.
constexpr double kCluRel = 1e-12;
__device__ __forceinline__ double tol_split(double tnorm) { return 16.0 * DBL_EPSILON * tnorm; }
__device__ __forceinline__ double tol_window(double tnorm, double clu_rel) { return 0.5 * clu_rel * tnorm; }
__device__ __forceinline__ double tol_cluster(double tnorm, double clu_rel) { return clu_rel * tnorm; }

// (a4) eigenvectors by inverse iteration, one lane per eigenvector. T is
// split where an off-diagonal is negligible; the k lanes of a k-fold
// eigenvalue (equal within the cluster tolerance) take k distinct blocks that
// hold it, so their vectors have disjoint supports; clusters whose lanes must
// share a block are marked for Gram-Schmidt (tri_gs).
__global__ __launch_bounds__(PT) void tri_invit(const double *d, const double *e, int64_t sDE, int N, int m,
                                                const double *lamg, double *Zs, int64_t sZ, int mp, int *marks,
                                                double clu_rel, uint32_t *status) {
  extern __shared__ double tsm[];
  double *sd = tsm;        // N
  double *se = sd + N;     // N
  double *se2 = se + N;    // N
  double *lam = se2 + N;   // m
  int *sblk = reinterpret_cast<int *>(lam + m);  // block starts (N + 1)
  int *smark = sblk + N + 1;                     // m: group id per lane
  int *sbad = smark + m;                         // m: cluster start -> a lane found no block
  __shared__ int s_bad, s_nblk;
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x;
  if (status[q] & BE_ST_NAN_INF) return;
  if (!load_tridiag(d, e, q, sDE, N, sd, se, se2, &s_bad)) return;
  for (int c = tid; c < m; c += PT) {
    lam[c] = lamg[q * (m + 1) + 1 + c];
    smark[c] = 0;
    sbad[c] = 0;
  }
  const double tnorm = lamg[q * (m + 1)];
  const double eps = DBL_EPSILON;
  double emax2 = 0.0;
  for (int i = 0; i < N; ++i) emax2 = fmax(emax2, se2[i]);
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  if (tid == 0) {
    const double splittol = tol_split(tnorm);
    int nb = 0;
    sblk[nb++] = 0;
    for (int i = 1; i < N; ++i)
      if (fabs(se[i - 1]) <= splittol) sblk[nb++] = i;
    sblk[nb] = N;
    s_nblk = nb;
  }
  __syncthreads();
  const int nblk = s_nblk;
  double *Z0 = Zs + q * sZ;
  double *X = Z0 + int64_t(3) * N * mp;  // the fourth array (arrays 1 and 2 unused here)
  const double tiny = eps * fmax(tnorm, DBL_MIN);
  const double dblk = tol_window(tnorm, clu_rel), dclu = tol_cluster(tnorm, clu_rel);
  bool lane_bad = false;
  for (int c = tid; c < m; c += PT) {
    int c0 = c, c1 = c + 1;
    while (c0 > 0 && lam[c0] - lam[c0 - 1] <= dclu) --c0;
    while (c1 < m && lam[c1] - lam[c1 - 1] <= dclu) ++c1;
    const double wlo = lam[c0] - dblk, whi = lam[c1 - 1] + dblk;
    const int jr = c - c0;
    int bs = 0, bt = N, cnt = 0;
    bool found = false, shared = false;
    for (int b = 0; b < nblk && !found; ++b) {
      const int s0 = sblk[b], t0 = sblk[b + 1];
      const int nb = sturm_count(sd + s0, se2 + s0, t0 - s0, whi, pivmin) -
                     sturm_count(sd + s0, se2 + s0, t0 - s0, wlo, pivmin);
      if (nb > 0 && cnt + nb > jr) {
        bs = s0;
        bt = t0;
        found = true;
        shared = nb > 1;
      }
      cnt += nb;
    }
    // group id of the lane for the orthonormalization: lanes sharing a block
    // (block start + 2); a lane that found no block makes its whole cluster
    // one group (id 1, set below)
    if (shared) smark[c] = bs + 2;
    if (!found) sbad[c0] = 1;
    // Lanes that share a block with other members of their cluster take
    // shifts a few eps ||T|| apart: far larger than the splitting of a
    // degenerate pair (so neither member dominates a lane's solve and each
    // lane returns an independent combination of the cluster's vectors),
    // far smaller than the distance to the next cluster.
    const double lm = (!found || shared) ? lam[c] + (jr - 0.5 * (c1 - c0 - 1)) * 2.0 * eps * tnorm : lam[c];
    for (int i = 0; i < N; ++i)
      if (i < bs || i >= bt) X[int64_t(i) * mp + c] = 0.0;
    // two solves: from a pseudo-random start the first already amplifies the
    // wanted direction by ~1/(eps ||T||) against ~1/gap for the others. The
    // second solve recomputes the same factorization (same operations, same
    // factors) instead of storing it again, and takes the first solution's
    // normalization as it reads it. Of the factorization only the diagonal
    // a_i met at each elimination step is stored: the pivot choice of row i
    // (|a_i| < |e_i|) and every factor entry follow from a_i, a_{i-1} and T,
    // recomputed by the same operations in the back substitution.
    // The loads of each sweep are issued PF rows ahead of the recurrence that
    // consumes them, so the serial chain waits on memory once per PF rows.
    // The start vector depends on the column only, not on the matrix's place
    // in the batch: a matrix gets the same eigenvectors, bit for bit, in any
    // batch (inside a degenerate cluster the start decides the basis).
    constexpr int PF = 4;
    double scale = 1.0;
    for (int it = 0; it < 2; ++it) {
      // forward elimination with partial pivoting on [T_block - lm I | rhs]
      double a = sd[bs] - lm, b = bt - bs > 1 ? se[bs] : 0.0;
      double r = it == 0 ? hash_unit(uint64_t(c) + 1, bs) : X[int64_t(bs) * mp + c] * scale;
      // one elimination step at row i (i + 1 < bt) with right-hand side entry rn of row i + 1
      auto step = [&](int i, double rn) {
        const double ei = se[i], Dn = sd[i + 1] - lm, en = (i + 2 < bt) ? se[i + 1] : 0.0;
        const int64_t o = int64_t(i) * mp + c;
        if (it == 0) Z0[o] = a;
        // without interchange: l = e_i / a (a = 0 only with e_i = 0, then
        // taken as tiny), row i keeps (a, b); with interchange: l = a / e_i
        const bool keep = fabs(a) >= fabs(ei);
        const double ad = (keep && a == 0.0) ? tiny : a;
        const double l = (keep ? ei : ad) / (keep ? ad : ei);
        X[o] = keep ? r : rn;
        const double p1 = keep ? Dn : b, p2 = keep ? b : Dn;
        const double q1 = keep ? rn : r, q2 = keep ? r : rn;
        a = p1 - l * p2;
        b = keep ? en : -l * en;
        r = q1 - l * q2;
      };
      if (it == 0) {
        for (int i = bs; i + 1 < bt; ++i) step(i, hash_unit(uint64_t(c) + 1, i + 1));
      } else {
        for (int i0 = bs; i0 + 1 < bt; i0 += PF) {
          double rv[PF];
#pragma unroll
          for (int u = 0; u < PF; ++u) rv[u] = i0 + u + 1 < bt ? X[int64_t(i0 + u + 1) * mp + c] : 0.0;
#pragma unroll
          for (int u = 0; u < PF; ++u)
            if (i0 + u + 1 < bt) step(i0 + u, rv[u] * scale);
        }
      }
      {
        const int64_t o = int64_t(bt - 1) * mp + c;
        if (it == 0) Z0[o] = a;
        X[o] = r;
      }
      // back substitution: row i of the triangular factor is (e_i, D_{i+1},
      // e_{i+1}) where row i was interchanged, else (a_i, b_i, 0) with b_i =
      // e_i, or -(a_{i-1} / e_{i-1}) e_i after an interchange at row i-1
      double x1 = 0.0, x2 = 0.0, nrm = 0.0;
      double ai = Z0[int64_t(bt - 1) * mp + c];
      for (int i0 = bt - 1; i0 >= bs; i0 -= PF) {
        double xv[PF], av[PF];
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int i = i0 - u;
          xv[u] = i >= bs ? X[int64_t(i) * mp + c] : 0.0;
          av[u] = i > bs ? Z0[int64_t(i - 1) * mp + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int i = i0 - u;
          if (i >= bs) {
            const double ap = av[u];
            double z0, z1 = 0.0, z2 = 0.0;
            if (i == bt - 1) {
              z0 = ai == 0.0 ? tiny : ai;
            } else if (fabs(ai) >= fabs(se[i])) {
              z0 = ai == 0.0 ? tiny : ai;
              z1 = se[i];
              if (i > bs && !(fabs(ap) >= fabs(se[i - 1]))) {
                const double l = ap / se[i - 1];
                z1 = -l * se[i];
              }
            } else {
              z0 = se[i];
              z1 = sd[i + 1] - lm;
              z2 = (i + 2 < bt) ? se[i + 1] : 0.0;
            }
            const double xi = (xv[u] - z1 * x1 - z2 * x2) / z0;
            X[int64_t(i) * mp + c] = xi;
            x2 = x1;
            x1 = xi;
            nrm = fma(xi, xi, nrm);
            ai = ap;
          }
        }
      }
      const double inv = 1.0 / sqrt(nrm);
      if (!isfinite(inv) || inv == 0.0) lane_bad = true;
      if (it == 0) {
        scale = inv;
      } else {
        for (int i0 = bs; i0 < bt; i0 += PF) {
          double xv[PF];
#pragma unroll
          for (int u = 0; u < PF; ++u) xv[u] = i0 + u < bt ? X[int64_t(i0 + u) * mp + c] : 0.0;
#pragma unroll
          for (int u = 0; u < PF; ++u)
            if (i0 + u < bt) X[int64_t(i0 + u) * mp + c] = xv[u] * inv;
        }
      }
    }
  }
  __syncthreads();
  for (int c = tid; c < m; c += PT) {
    int c0 = c;
    while (c0 > 0 && lam[c0] - lam[c0 - 1] <= dclu) --c0;
    marks[q * m + c] = sbad[c0] ? 1 : smark[c];
  }
  if (lane_bad) atomicOr(&status[q], uint32_t(BE_ST_NONCONVERGED));
}

// End of the orthonormalization group starting at c0: the following lanes of
// the same cluster with the same group id (0: no group, a group of one).
__device__ __forceinline__ int group_end(const double *lam, const int *mk, int m, int c0, double dclu) {
  int c1 = c0 + 1;
  if (mk[c0] == 0) return c1;
  while (c1 < m && mk[c1] == mk[c0] && lam[c1] - lam[c1 - 1] <= dclu) ++c1;
  return c1;
}

// Groups of vectors that share a block of T (inside a cluster of equal
// eigenvalues; vectors in different blocks have disjoint supports and are
// orthogonal already) are orthonormalized by Cholesky QR (two passes; one
// for groups larger than GK)
// (G = V^T V = R^T R, V <- V R^-1), done in lanes: the groups are packed into
// 64-lane bins (no group straddles a bin), a bin is one wave, vector c sits
// on one lane, and the rows of X are swept with coalesced loads (the
// eigenvector index is the fastest dimension of X). A Gram sweep reads the
// other members of a lane's group by cross-lane permutes; the first member of
// each group factors G in LDS; an apply sweep solves y R = x row by row, the
// members finalizing y in order and passing it on by permutes. Groups larger
// than GK run one such pass with the whole workgroup; a breakdown of the
// Cholesky factorization falls back to modified Gram-Schmidt with one wave
// per group.
constexpr int GK = 32;

__host__ __device__ inline int gs_bins_max(int m) { return m / (64 - GK + 1) + 2; }

size_t gs_smem(int m) {
  return size_t(PT) * GK * sizeof(double) + size_t(std::max(m, 1)) * sizeof(double) +
         (3 * size_t(gs_bins_max(m)) * 64 + 2 * size_t(std::max(m, 1))) * sizeof(int);
}

__global__ __launch_bounds__(PT) void tri_gs(int N, int m, const double *lamg, double *Zs, int64_t sZ, int mp,
                                             const int *marks, double *Gm, double clu_rel, const uint32_t *status) {
  extern __shared__ double gsm[];
  const int nbmax = gs_bins_max(m);
  int *sv = reinterpret_cast<int *>(gsm + PT * GK + m);  // bin lane -> vector (-1: idle)
  int *sb = sv + nbmax * 64;                         // bin lane -> lane of its group's first member
  int *sk = sb + nbmax * 64;                         // bin lane -> group size
  int *sfl = sk + nbmax * 64;                        // group start -> Cholesky breakdown
  int *mk_q = sfl + m;                               // group id per vector
  double *lam = gsm + PT * GK;                       // selected eigenvalues (m)
  __shared__ int s_nbins;
  const int64_t q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = PT / 64;
  if (status[q] & BE_ST_NAN_INF) return;
  const double dclu = tol_cluster(lamg[q * (m + 1)], clu_rel);
  double *X = Zs + q * sZ + int64_t(3) * N * mp;
  for (int c = tid; c < m; c += PT) {
    sfl[c] = 0;
    mk_q[c] = marks[q * m + c];
    lam[c] = lamg[q * (m + 1) + 1 + c];
  }
  __syncthreads();
  if (tid == 0) {
    int nb = 0, fill = 0;
    for (int c0 = 0; c0 < m;) {
      const int c1 = group_end(lam, mk_q, m, c0, dclu);
      const int k = c1 - c0;
      if (mk_q[c0] && k > 1 && k <= GK) {
        if (fill + k > 64) {
          for (int l = fill; l < 64; ++l) sv[nb * 64 + l] = -1;
          ++nb;
          fill = 0;
        }
        for (int t = 0; t < k; ++t) {
          sv[nb * 64 + fill + t] = c0 + t;
          sb[nb * 64 + fill + t] = fill;
          sk[nb * 64 + fill + t] = k;
        }
        fill += k;
      }
      c0 = c1;
    }
    if (fill > 0) {
      for (int l = fill; l < 64; ++l) sv[nb * 64 + l] = -1;
      ++nb;
    }
    s_nbins = nb;
  }
  __syncthreads();
  const int nbins = s_nbins;
  double *G = gsm + wave * 64 * GK;  // this wave's Gram rows, G[lane][t]
  for (int j0 = 0; j0 < nbins; j0 += nw) {
    const int j = j0 + wave;
    const int c = j < nbins ? sv[j * 64 + lane] : -1;
    const bool act = c >= 0;
    const int b = act ? sb[j * 64 + lane] : lane;
    const int k = act ? sk[j * 64 + lane] : 1;
    const int rel = lane - b;
    int kmax = k;
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
    for (int pass = 0; pass < 2; ++pass) {
      // Gram sweep: g[t] = <x_c, x_{b+t}>
      double g[GK];
#pragma unroll
      for (int t = 0; t < GK; ++t) g[t] = 0.0;
      for (int i = 0; i < N; ++i) {
        const double x = act ? X[int64_t(i) * mp + c] : 0.0;
#pragma unroll
        for (int t = 0; t < GK; ++t)
          if (t < kmax) g[t] = fma(x, __shfl(x, min(63, b + t), 64), g[t]);
      }
#pragma unroll
      for (int t = 0; t < GK; ++t) G[lane * GK + t] = g[t];
      __syncthreads();
      // Cholesky G = R^T R in place (upper triangle), by the group's first lane
      if (act && rel == 0 && !sfl[c]) {
        for (int jj = 0; jj < k; ++jj) {
          double dg = G[(b + jj) * GK + jj];
          const double g0 = dg;
          for (int p = 0; p < jj; ++p) dg -= G[(b + p) * GK + jj] * G[(b + p) * GK + jj];
          if (!(dg > 1e-12 * g0)) {
            sfl[c] = 1;
            break;
          }
          const double rjj = sqrt(dg);
          G[(b + jj) * GK + jj] = rjj;
          for (int t = jj + 1; t < k; ++t) {
            double v = G[(b + jj) * GK + t];
            for (int p = 0; p < jj; ++p) v -= G[(b + p) * GK + jj] * G[(b + p) * GK + t];
            G[(b + jj) * GK + t] = v / rjj;
          }
        }
      }
      __syncthreads();
      const bool ok = act && !sfl[c - rel];
      // column rel of R: rcol[s] = R[s][rel] for s < rel; inverse of R[rel][rel]
      double rcol[GK];
#pragma unroll
      for (int t = 0; t < GK; ++t) rcol[t] = (ok && t < rel) ? G[(b + t) * GK + rel] : 0.0;
      const double rinv = ok ? 1.0 / G[lane * GK + rel] : 0.0;
      // apply sweep: y R = x, row by row
      for (int i = 0; i < N; ++i) {
        const int64_t o = int64_t(i) * mp + (act ? c : 0);
        const double x = act ? X[o] : 0.0;
        double y = 0.0, acc = 0.0;
#pragma unroll
        for (int t = 0; t < GK; ++t) {
          if (t < kmax) {
            if (rel == t) y = (x - acc) * rinv;
            const double yt = __shfl(y, min(63, b + t), 64);
            if (rel > t) acc = fma(yt, rcol[t], acc);
          }
        }
        if (ok) X[o] = y;
      }
      __syncthreads();
    }
  }
  // groups larger than GK: one Cholesky-QR pass by the whole workgroup (its
  // O(cond^2 eps) loss of orthogonality is removed by the symmetric
  // Newton-Schulz orthonormalization of all vectors that follows). The Gram
  // matrix and its factor are kept packed (upper
  // triangle, row by row) in LDS next to a tile of the cluster's rows when
  // they fit (k(k+1)/2 + k <= PT*GK), else in the matrix's m x m scratch Gq.
  // The Gram matrix is accumulated tile by tile, the factorization runs one
  // column per step, R is inverted in place, and X_c R^-1 is formed from
  // rows staged in the LDS tile, one (row, column) dot product per thread.
  double *Gq = Gm + q * int64_t(m) * m;
  for (int c0 = 0; c0 < m;) {
    const int c1 = group_end(lam, mk_q, m, c0, dclu);
    const int k = c1 - c0;
    if (mk_q[c0] && k > GK) {
      const int npk = k * (k + 1) / 2;
      const bool in_lds = npk + k <= PT * GK;
      double *Rp = in_lds ? gsm : Gq;              // packed upper triangle
      double *tile = in_lds ? gsm + npk : gsm;     // rows of the group
      const int RB = in_lds ? (PT * GK - npk) / k : (PT * GK) / k;
      // packed index of (s, t), s <= t
      auto pk = [k](int s2, int t) { return s2 * k - (s2 * (s2 - 1)) / 2 + (t - s2); };
      for (int pass = 0; pass < 1 && !sfl[c0]; ++pass) {
        __syncthreads();
        for (int e = tid; e < npk; e += PT) Rp[e] = 0.0;
        // Gram matrix, upper triangle, tile by tile (16 threads per row s2)
        for (int i0 = 0; i0 < N; i0 += RB) {
          const int nr = min(RB, N - i0);
          __syncthreads();
          for (int e = tid; e < nr * k; e += PT) {
            const int r = e / k, col = e - r * k;
            tile[e] = X[int64_t(i0 + r) * mp + c0 + col];
          }
          __syncthreads();
          for (int s2 = tid >> 4; s2 < k; s2 += PT >> 4)
            for (int t = s2 + (tid & 15); t < k; t += 16) {
              double acc = 0.0;
              for (int r = 0; r < nr; ++r) acc = fma(tile[r * k + s2], tile[r * k + t], acc);
              Rp[pk(s2, t)] += acc;
            }
        }
        __syncthreads();
        // right-looking Cholesky, one column per step
        for (int j = 0; j < k; ++j) {
          if (tid == 0) {
            const double dg = Rp[pk(j, j)];
            if (!(dg > 1e-12) || !isfinite(dg)) sfl[c0] = 1;  // columns enter with unit norm
            Rp[pk(j, j)] = sqrt(fmax(dg, DBL_MIN));
          }
          __syncthreads();
          if (sfl[c0]) break;
          const double rjj = Rp[pk(j, j)];
          for (int t = j + 1 + tid; t < k; t += PT) Rp[pk(j, t)] /= rjj;
          __syncthreads();
          for (int s2 = j + 1 + (tid >> 4); s2 < k; s2 += PT >> 4) {
            const double rs = Rp[pk(j, s2)];
            for (int t = s2 + (tid & 15); t < k; t += 16) Rp[pk(s2, t)] -= rs * Rp[pk(j, t)];
          }
          __syncthreads();
        }
        if (sfl[c0]) break;
        // R^-1 in place, rows from the bottom: row i needs rows > i of R^-1
        for (int i = k - 1; i >= 0; --i) {
          const double rii = Rp[pk(i, i)];
          for (int j = i + tid; j < k; j += PT) {
            double v = j == i ? 1.0 : 0.0;
            for (int p = i + 1; p <= j; ++p) v -= Rp[pk(i, p)] * Rp[pk(p, j)];
            tile[j] = v / rii;
          }
          __syncthreads();
          for (int j = i + tid; j < k; j += PT) Rp[pk(i, j)] = tile[j];
          __syncthreads();
        }
        // X_c <- X_c R^-1: rows staged in LDS, independent (row, column) dot products
        for (int i0 = 0; i0 < N; i0 += RB) {
          const int nr = min(RB, N - i0);
          __syncthreads();
          for (int e = tid; e < nr * k; e += PT) {
            const int r = e / k, col = e - r * k;
            tile[e] = X[int64_t(i0 + r) * mp + c0 + col];
          }
          __syncthreads();
          for (int e = tid; e < nr * k; e += PT) {
            const int r = e / k, j = e - r * k;
            const double *xr = tile + r * k;
            double v = 0.0;
            for (int p = 0, ix = j; p <= j; ix += k - p - 1, ++p) v = fma(xr[p], Rp[ix], v);
            X[int64_t(i0 + r) * mp + c0 + j] = v;
          }
        }
        __syncthreads();
      }
    }
    c0 = c1;
  }
  __syncthreads();
  // clusters left to the fallback: a Cholesky breakdown
  for (int c0 = 0, w = 0; c0 < m;) {
    const int c1 = group_end(lam, mk_q, m, c0, dclu);
    const int k = c1 - c0;
    if (mk_q[c0] && k > 1 && sfl[c0]) {
      if (w++ % nw == wave) {
        for (int pass = 0; pass < 2; ++pass) {
          for (int t = c0; t < c1; ++t) {
            for (int s2 = c0; s2 < t; ++s2) {
              double dt = 0.0;
              for (int i = lane; i < N; i += 64) dt = fma(X[int64_t(i) * mp + s2], X[int64_t(i) * mp + t], dt);
              dt = wave_sum(dt);
              for (int i = lane; i < N; i += 64) X[int64_t(i) * mp + t] -= dt * X[int64_t(i) * mp + s2];
            }
            double nr = 0.0;
            for (int i = lane; i < N; i += 64) {
              const double v = X[int64_t(i) * mp + t];
              nr = fma(v, v, nr);
            }
            nr = wave_sum(nr);
            // a vector in the span of the earlier ones is left at zero (the
            // orthonormalization that follows then flags the matrix) rather
            // than divided by zero
            const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
            for (int i = lane; i < N; i += 64) X[int64_t(i) * mp + t] *= inv;
          }
        }
      }
    }
    c0 = c1;
  }
}

// One Newton-Schulz step of the symmetric orthonormalization of X (m x N),
// with a state per matrix (act): 1 iterating, 2 taking its last step, 0 done.
// G = X X^T is replaced by (3 I - G) / 2 and err[q] = max |G - I| (before the
// update); the next state is 0 (done, no step) once err <= tol, 2 once err <
// 1e-8 (the step leaves about (3/4) err^2 < 1e-16), else 1. Matrices in state
// 0 are skipped here and by the two GEMMs of the step.
__global__ __launch_bounds__(PT) void ns_prep_real(double *G, int m, double *err, int *act, double tol) {
  const int64_t q = blockIdx.x;
  if (act[q] == 0) return;
  double *Gq = G + q * int64_t(m) * m;
  double e = 0.0;
  for (int k = threadIdx.x; k < m * m; k += PT) {
    const int r = k % m, c = k / m;
    const double g = Gq[k];
    e = fmax(e, fabs(g - (r == c ? 1.0 : 0.0)));
    Gq[k] = (r == c ? 1.5 : 0.0) - 0.5 * g;
  }
  for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o, 64));
  __shared__ double red[PT / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < PT / 64; ++w) t = fmax(t, red[w]);
    if (!(t == t)) t = INFINITY;
    err[q] = t;
    // beyond 1 (columns of unit norm cannot differ from orthonormal by more
    // elementwise) the iteration is outside its basin and would grow without
    // bound: stop, the error stays and flags the matrix
    act[q] = t <= tol ? 0 : t < 1e-8 ? 2 : t > 1.0 ? 0 : 1;
  }
}

// After the step into buffer `parity`: matrices that took it have their
// iterate there; those in their last step are done (error taken as zero).
// *n_left (zeroed before) counts the matrices still iterating.
__global__ void ns_post_real(int *act, unsigned char *loc, double *err, int64_t n, unsigned char parity, int *n_left) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int left = 0;
  if (q < n && act[q] != 0) {
    loc[q] = parity;
    if (act[q] == 2) {
      act[q] = 0;
      err[q] = 0.0;
    } else {
      left = 1;
    }
  }
  for (int o = 32; o > 0; o >>= 1) left += __shfl_xor(left, o, 64);
  if ((threadIdx.x & 63) == 0 && left) atomicAdd(n_left, left);
}

__global__ void ns_init_real(int *act, unsigned char *loc, int64_t n) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < n) {
    act[q] = 1;
    loc[q] = 0;
  }
}

__global__ void zero_i32(int *p) { *p = 0; }

// status[q] |= NONCONVERGED where the last orthonormality error stayed above tol
__global__ void flag_nonorth(const double *err, int64_t n, double tol, uint32_t *status) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < n && !(err[q] <= tol)) status[q] |= BE_ST_NONCONVERGED;
}

// U[q](r, c) = X[q](c, r) as complex (X: m x N column-major, leading dimension
// mp), by 64 x 64 tiles staged in LDS: rows of X are read along c and columns
// of U written along r, both coalesced. Grid: (tiles of N x m, matrices).
template <typename C>
__global__ __launch_bounds__(256) void z_to_u(const double *X0, const double *X1, const unsigned char *loc, int64_t sX,
                                              int mp, int N, int m, C *U, int ldu, int64_t sU) {
  __shared__ double s[64 * 65];
  const int64_t q = blockIdx.y;
  const int ntr = (N + 63) / 64;
  const int r0 = int(blockIdx.x % ntr) * 64, c0 = int(blockIdx.x / ntr) * 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double *Xq = (loc[q] ? X1 : X0) + q * sX;  // the buffer holding matrix q's latest iterate
  for (int rr = w; rr < 64; rr += 4) {
    const int r = r0 + rr, c = c0 + lane;
    s[rr * 65 + lane] = (r < N && c < m) ? Xq[int64_t(r) * mp + c] : 0.0;
  }
  __syncthreads();
  C *Uq = U + q * sU;
  for (int cc = w; cc < 64; cc += 4) {
    const int r = r0 + lane, c = c0 + cc;
    if (r < N && c < m) Uq[r + int64_t(c) * ldu] = mk<C>(s[lane * 65 + cc], 0.0);
  }
}

// c64 (N x m, leading dim N) -> c128 output
__global__ void widen_u(const float2 *Uw, int64_t sW, int N, int m, double2 *U, int ldu, int64_t sU) {
  const int64_t q = blockIdx.y;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < int64_t(N) * m; k += int64_t(gridDim.x) * blockDim.x) {
    int c = int(k / N), r = int(k % N);
    float2 v = Uw[q * sW + k];
    U[q * sU + r + int64_t(c) * ldu] = make_double2(double(v.x), double(v.y));
  }
}

__global__ void zero_u32(uint32_t *p, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename C>
__global__ void zero_c(C *p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = mk<C>(0, 0);
}

// T of a pair of panels (ld 2 NB): the diagonal blocks T1 (nb1 x nb1) and T2
// (nb2 x nb2) and the zero lower-left block; the upper-right block is written
// by a GEMM.
template <typename C>
__global__ void assemble_tpair(const C *T1, const C *T2, int64_t sT, C *Tb, int nb1, int nb2) {
  const int64_t q = blockIdx.x;
  const int nbc = nb1 + nb2;
  C *Tq = Tb + q * int64_t(4) * NB * NB;
  for (int e = threadIdx.x; e < nbc * nbc; e += blockDim.x) {
    const int i = e % nbc, j = e / nbc;
    C v;
    if (i < nb1 && j < nb1) v = T1[q * sT + i + j * NB];
    else if (i >= nb1 && j >= nb1) v = T2[q * sT + (i - nb1) + (j - nb1) * NB];
    else if (i >= nb1) v = mk<C>(0, 0);
    else continue;  // upper-right block: -T1 S12 T2
    Tq[i + j * (2 * NB)] = v;
  }
}

size_t panel_smem(int N, size_t csize, int nt) { return panel_part_offset(N, csize, nt) + 64; }

// Bytes of the matrix-vector product's partial vectors for trailing matrices
// of order up to n: nrb S + 1 slots of 64 elements per 64-row block, the
// largest over nrb <= ceil(n / 64).
size_t panel_part_bytes(int n, size_t csize) {
  const int nrb_max = (std::max(n, 0) + 63) / 64;
  size_t slots = 0;
  for (int nrb = 1; nrb <= nrb_max; ++nrb) slots = std::max(slots, size_t(nrb) * (size_t(nrb) * panel_split(nrb) + 1));
  return slots * 64 * csize;
}

// The partial vectors stay in LDS while the panel's LDS remains within
// 53 KiB (three workgroups per compute unit); larger orders keep them in a
// global scratch slot per matrix (written and read back through L2).
constexpr size_t kPanelLdsMax = 53 * 1024;
bool panel_part_lds(int N, size_t csize, int nt) {
  return panel_smem(N, csize, nt) + panel_part_bytes(N - 1, csize) <= kPanelLdsMax;
}
size_t panel_lds(int N, size_t csize, int nt) {
  return panel_smem(N, csize, nt) + (panel_part_lds(N, csize, nt) ? panel_part_bytes(N - 1, csize) : 0);
}

template <typename T>
using PanelFn = void (*)(typename CT<T>::c *, int64_t, int, int, int, int, typename CT<T>::c *, int64_t,
                         typename CT<T>::c *, int64_t, double *, double *, int64_t, typename CT<T>::c *, int64_t,
                         uint32_t *);

// The panel kernel for nt threads, partial vectors in LDS (pl) or not, and
// cw loads in flight (as panel_loads gives it: only the 512-thread FP32
// kernel has both forms; FP64 has 4 everywhere).
template <typename T, bool PL>
PanelFn<T> panel_kernel_pl(int nt, int cw) {
  constexpr bool f32 = sizeof(T) == 4;
  if (nt == 256) return &hetrd_panel<T, 256, PL, 4>;
  if (nt == 512) return (f32 && cw == 8) ? &hetrd_panel<T, 512, PL, f32 ? 8 : 4> : &hetrd_panel<T, 512, PL, 4>;
  return &hetrd_panel<T, 1024, PL, f32 ? 8 : 4>;
}
template <typename T>
PanelFn<T> panel_kernel(int nt, int cw, bool pl) {
  return pl ? panel_kernel_pl<T, true>(nt, cw) : panel_kernel_pl<T, false>(nt, cw);
}


// ---------------------------------------------------------------- FP64 refinement of the mixed path
// Full Hermitian FP64 copy of H (upper triangle mirrored from the lower one,
// diagonal taken real) and its FP32 rounding (the FP32 reduction's input),
// by 32 x 32 tile pairs staged in LDS: tile (bi, bj), bi >= bj, is read once
// with coalesced columns and written to (bi, bj) and, conjugate-transposed,
// to (bj, bi). Matrices q = blockIdx.y, blockIdx.y + gridDim.y, ...
__global__ __launch_bounds__(256) void split_h(const double2 *H, int64_t ms, int ld, int N, int64_t n_mat, double2 *Hf,
                                               float2 *Hc) {
  __shared__ double2 t[32][33];  // t[column][row] of the lower tile
  const int nt = (N + 31) / 32;
  int p = blockIdx.x, bj = 0;
  while (p >= nt - bj) {
    p -= nt - bj;
    ++bj;
  }
  const int bi = bj + p;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t NN = int64_t(N) * N;
  for (int64_t q = blockIdx.y; q < n_mat; q += gridDim.y) {
    const double2 *Hq = H + q * ms;
    double2 *F = Hf + q * NN;
    float2 *Cq = Hc + q * NN;
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
      const int r = bi * 32 + tx, col = bj * 32 + c;
      t[c][tx] = (r < N && col < N) ? Hq[r + int64_t(col) * ld] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
      const int r = bi * 32 + tx, col = bj * 32 + c;
      if (r >= N || col >= N) continue;
      double2 v = (bi != bj || tx >= c) ? t[c][tx] : be::cconj(t[tx][c]);
      if (r == col) v.y = 0.0;
      F[r + int64_t(col) * N] = v;
      Cq[r + int64_t(col) * N] = make_float2(float(v.x), float(v.y));
    }
    if (bi != bj) {
      for (int c = ty; c < 32; c += 8) {
        const int r = bj * 32 + tx, col = bi * 32 + c;
        if (r >= N || col >= N) continue;
        const double2 v = be::cconj(t[tx][c]);
        F[r + int64_t(col) * N] = v;
        Cq[r + int64_t(col) * N] = make_float2(float(v.x), float(v.y));
      }
    }
  }
}

// Window columns lo .. lo+m-1 of the all-band eigenvectors (N x N, ld N)
// into the right half of GU (N x 2m, ld N) and into the output U.
__global__ void refine_copy_u(const double2 *Uall, int N, int lo, int m, int64_t n_mat, double2 *GU, double2 *U,
                              int ldu, int64_t us) {
  for (int64_t q = blockIdx.y; q < n_mat; q += gridDim.y) {
    const double2 *Uq = Uall + q * int64_t(N) * N + int64_t(lo) * N;
    double2 *G = GU + q * int64_t(N) * 2 * m + int64_t(m) * N;
    double2 *O = U + q * us;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < int64_t(N) * m;
         k += int64_t(gridDim.x) * blockDim.x) {
      const int r = int(k % N), c = int(k / N);
      const double2 v = Uq[k];
      G[k] = v;
      O[r + int64_t(c) * ldu] = v;
    }
  }
}

// First-order correction of the window's invariant subspace from the
// complement (bands outside [lo, hi)), for approximate eigenvectors that
// are not exactly orthonormal: with s_ij = v_i^H H u_j and p_ij = v_i^H u_j
// (both in FP64 from the stored vectors), the error of u_j along v_i is
// e_ij = (s_ij - lambda_j p_ij) / (lambda_i - lambda_j); the correction
// coefficient f_ij = -e_ij replaces s_ij in S2. S2: nc x 2m (ld nc), left
// half S, right half P; complement row i is band i (i < lo) or i + m.
__global__ void refine_coef(double2 *S2, int nc, int m, int lo, int N, const double *lam_all, int64_t n_mat) {
  const int64_t per = int64_t(nc) * m;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n_mat * per;
       k += int64_t(gridDim.x) * blockDim.x) {
    const int64_t q = k / per;
    const int64_t e = k % per;
    const int i = int(e % nc), j = int(e / nc);
    const double *lam = lam_all + q * (N + 2) + 1;
    const double li = lam[i < lo ? i : i + m], lj = lam[lo + j];
    double2 *Sq = S2 + q * int64_t(nc) * 2 * m;
    const double2 s = Sq[i + int64_t(j) * nc], pp = Sq[i + int64_t(m + j) * nc];
    const double d = lj - li;
    double2 f = make_double2(0.0, 0.0);
    if (d != 0.0 && d == d) f = make_double2((s.x - lj * pp.x) / d, (s.y - lj * pp.y) / d);
    Sq[i + int64_t(j) * nc] = f;
  }
}

// Refined eigenvalues of the window (Rayleigh quotients u_j^H H u_j / u_j^H u_j
// of the uncorrected vectors: errors of second order in the vectors' error),
// the neighbours lo-1 and hi from the FP32 reduction's spectrum, and the gap
// flag of the window. One workgroup per matrix, a wave per column.
__global__ __launch_bounds__(PT) void refine_evals(const double2 *GU, int N, int m, int lo, const double *lam_all,
                                                   double *evals, uint32_t *status) {
  const int64_t q = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double2 *G = GU + q * int64_t(N) * 2 * m, *Uo = G + int64_t(m) * N;
  const double *lam = lam_all + q * (N + 2) + 1;
  double *ev = evals + q * (m + 2);
  for (int j = wave; j < m; j += PT / 64) {
    double num = 0.0, den = 0.0;
    for (int r = lane; r < N; r += 64) {
      const double2 u = Uo[r + int64_t(j) * N], g = G[r + int64_t(j) * N];
      num += u.x * g.x + u.y * g.y;
      den += u.x * u.x + u.y * u.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
      num += __shfl_xor(num, o, 64);
      den += __shfl_xor(den, o, 64);
    }
    if (lane == 0) ev[1 + j] = num / den;
  }
  if (threadIdx.x == 0) {
    const int hi = lo + m;
    ev[0] = lo > 0 ? lam[lo - 1] : NAN;
    ev[m + 1] = hi < N ? lam[hi] : NAN;
    const double scale = fmax(1.0, fmax(fabs(lam[0]), fabs(lam[N - 1])));
    double g = INFINITY;
    if (lo > 0 && m > 0) g = fmin(g, lam[lo] - lam[lo - 1]);
    if (hi < N && m > 0) g = fmin(g, lam[hi] - lam[hi - 1]);
    if (g < 1e-9 * scale) atomicOr(&status[q], BE_ST_GAP_CLOSED);
  }
}

// Newton-Schulz step preparation for complex N x m matrices (as ns_prep_real):
// err = max |G - I|, G <- (3 I - G) / 2, state 0 (done, err <= tol), 2 (last
// step, err < last: the step leaves about 3/4 err^2), 1 (iterating).
__global__ __launch_bounds__(PT) void ns_prep_cplx(double2 *G, int m, double *err, int *act, double tol, double last) {
  const int64_t q = blockIdx.x;
  if (act[q] == 0) return;
  double2 *Gq = G + q * int64_t(m) * m;
  double e = 0.0;
  for (int k = threadIdx.x; k < m * m; k += PT) {
    const int r = k % m, c = k / m;
    const double2 g = Gq[k];
    const double dr = g.x - (r == c ? 1.0 : 0.0);
    e = fmax(e, sqrt(dr * dr + g.y * g.y));
    Gq[k] = make_double2((r == c ? 1.5 : 0.0) - 0.5 * g.x, -0.5 * g.y);
  }
  for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o, 64));
  __shared__ double red[PT / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < PT / 64; ++w) t = fmax(t, red[w]);
    if (!(t == t)) t = INFINITY;
    err[q] = t;
    act[q] = t <= tol ? 0 : t < last ? 2 : t > 1.0 ? 0 : 1;  // beyond 1: outside the basin (as in ns_prep_real)
  }
}

// Matrices whose latest Newton-Schulz iterate is in the scratch buffer
// (loc = 1) copy it back to the output.
__global__ void refine_copy_back(const double2 *Ub, int64_t sUb, int N, int m, const unsigned char *loc, int64_t n_mat,
                                 double2 *U, int ldu, int64_t us) {
  for (int64_t q = blockIdx.y; q < n_mat; q += gridDim.y) {
    if (loc[q] != 1) continue;
    const double2 *B = Ub + q * sUb;
    double2 *O = U + q * us;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < int64_t(N) * m;
         k += int64_t(gridDim.x) * blockDim.x) {
      const int r = int(k % N), c = int(k / N);
      O[r + int64_t(c) * ldu] = B[k];
    }
  }
}

}  // namespace

namespace be {

template <typename T>
struct GemmOf;
template <>
struct GemmOf<double> {
  typedef ZGemm type;
  static int run(be_ctx *ctx, const ZGemm &g, hipStream_t s) { return zgemm(ctx, g, s); }
};
template <>
struct GemmOf<float> {
  typedef CGemm type;
  static int run(be_ctx *ctx, const CGemm &g, hipStream_t s) { return cgemm(ctx, g, s); }
};

// One sub-batch of nb_mat matrices. T is the working precision of the
// Householder reduction and back-transformation (double: FP64 path, float:
// mixed path); the tridiagonal solve and the re-orthonormalization are FP64.
// Hin: nb_mat matrices of CT<T>::c; U: c128 output.
// bf16x3 (T = float only): the trailing update and the back-transformation
// take the split-bf16 products of the complex GEMM.
template <typename T>
static int eigh_chunk(be_ctx *ctx, typename CT<T>::c *H, int N, int ld, int64_t ms, int64_t nb_mat, int lo, int hi,
                      double *evals, double2 *U, int ldu, int64_t us, uint32_t *status, hipStream_t stream,
                      double clu_rel = kCluRel, bool bf16x3 = false) {
  typedef typename CT<T>::c C;
  typedef typename GemmOf<T>::type G;
  const int m = hi - lo;
  const int P = (N + NB - 1) / NB;
  const int mp = std::max(64, (m + 63) / 64 * 64);
  const bool mixed = sizeof(T) == sizeof(float);
  C *VW = nullptr, *Tm = nullptr, *Xb = nullptr, *Yb = nullptr, *Uw = nullptr;
  double *dd = nullptr, *ee = nullptr, *Zs = nullptr;
  Carve cv;
  cv.add(&VW, size_t(nb_mat) * N * 3 * NB);
  cv.add(&Tm, size_t(nb_mat) * P * NB * NB);
  cv.add(&dd, size_t(nb_mat) * N);
  cv.add(&ee, size_t(nb_mat) * N);
  cv.add(&Zs, size_t(nb_mat) * 4 * N * mp);
  double *lamg = nullptr;
  int *marks = nullptr;
  cv.add(&lamg, size_t(nb_mat) * (m + 1));
  cv.add(&marks, size_t(nb_mat) * std::max(m, 1));
  double *Gm = nullptr, *oerr = nullptr;
  int *nact = nullptr, *n_left = nullptr;
  unsigned char *nloc = nullptr;
  cv.add(&Gm, size_t(nb_mat) * std::max(m, 1) * std::max(m, 1));
  cv.add(&oerr, size_t(nb_mat));
  cv.add(&nact, size_t(nb_mat));
  cv.add(&nloc, size_t(nb_mat));
  cv.add(&n_left, 1);
  cv.add(&Xb, size_t(nb_mat) * 2 * NB * std::max(m, 1));
  cv.add(&Yb, size_t(nb_mat) * 2 * NB * std::max(m, 1));
  C *Tb = nullptr, *Sw = nullptr, *Ww = nullptr;  // paired back-transformation: T of a pair, V1^H V2, T1 V1^H V2
  cv.add(&Tb, size_t(nb_mat) * 4 * NB * NB);
  cv.add(&Sw, size_t(nb_mat) * NB * NB);
  cv.add(&Ww, size_t(nb_mat) * NB * NB);
  if (mixed) cv.add(&Uw, size_t(nb_mat) * N * std::max(m, 1));
  // panel kernel: 256, 512 or 1024 threads per matrix; partial vectors of its
  // matrix-vector product in LDS or in global scratch
  const int pnt = panel_threads(ctx, N, sizeof(C));
  const bool pl = panel_part_lds(N, sizeof(C), pnt);
  const size_t psm = panel_lds(N, sizeof(C), pnt);
  const int64_t sPg = pl ? 0 : int64_t(panel_part_bytes(N - 1, 1));
  C *Pg = nullptr;
  if (!pl) cv.add(&Pg, size_t(nb_mat) * sPg);
  BE_RET_IF(cv.commit(ctx, stream, WS_EIGH));
  hipLaunchKernelGGL(zero_u32, dim3((nb_mat + 255) / 256), dim3(256), 0, stream, status, nb_mat);
  BE_RET_IF(check_launch(ctx, "zero_u32"));
  const int64_t sVW = int64_t(N) * 3 * NB;
  const int64_t sT = int64_t(P) * NB * NB;
  PanelFn<T> panel = panel_kernel<T>(pnt, panel_loads(ctx, N, sizeof(C), pnt), pl);
  if (psm > 65536)
    BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(panel),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(psm)));
  // ---- Householder reduction
  for (int p = 0; p < P; ++p) {
    const int p0 = p * NB, nbp = std::min(NB, N - p0);
    {
      ProfScope prof(ctx, "hetrd_panel", stream);
      hipLaunchKernelGGL(panel, dim3(nb_mat), dim3(pnt), psm, stream, H, ms, ld, N, p0, nbp, VW, sVW,
                         Tm + int64_t(p) * NB * NB, sT, dd, ee, int64_t(N), Pg, sPg, status);
    }
    BE_RET_IF(check_launch(ctx, "hetrd_panel"));
    const int n2 = N - p0 - NB;
    if (n2 > 0) {
      G g;
      g.M = n2;
      g.N = n2;
      g.K = 2 * NB;
      g.opA = 0;
      g.opB = 1;
      g.A = VW + (p0 + NB);
      g.lda = N;
      g.bA = ZBatch::strided(sVW);
      g.B = VW + int64_t(NB) * N + (p0 + NB);
      g.ldb = N;
      g.bB = ZBatch::strided(sVW);
      g.C = H + (p0 + NB) + int64_t(p0 + NB) * ld;
      g.ldc = ld;
      g.bC = ZBatch::strided(ms);
      g.alpha = mk<C>(-1.0, 0.0);
      g.beta = mk<C>(1.0, 0.0);
      g.batch = nb_mat;
      g.tag = "her2k";
      g.herm = true;
      g.herm_mirror = false;  // the panel reads the lower triangle only
      if constexpr (std::is_same<G, CGemm>::value) g.bf16x3 = bf16x3;
      BE_RET_IF(GemmOf<T>::run(ctx, g, stream));
    }
  }
  // ---- tridiagonal eigenpairs: bisection, inverse iteration, Gram-Schmidt of shared-block clusters
  {
    const size_t smb = (4 * size_t(N) + m + 4) * sizeof(double);
    if (smb > 65536)
      BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&tri_bisect),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(smb)));
    ProfScope prof(ctx, "tri_bisect", stream);
    // eigenvalues to eps |lambda|: inverse iteration must separate the
    // closely spaced ones (bis_rel > 0 would stop at bis_rel ||T||)
    const double bis_rel = 0.0;
    hipLaunchKernelGGL(tri_bisect, dim3(nb_mat), dim3(PT), smb, stream, dd, ee, int64_t(N), N, lo, hi, bis_rel,
                       ctx->dbg_bisect_max_iter, evals, lamg, U, ldu, us, status);
  }
  BE_RET_IF(check_launch(ctx, "tri_bisect"));
  if (m == 0) return BE_OK;
  {
    const size_t smi = (3 * size_t(N) + m) * sizeof(double) + (size_t(N) + 1 + 2 * size_t(m)) * sizeof(int);
    if (smi > 65536)
      BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&tri_invit),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(smi)));
    ProfScope prof(ctx, "tri_invit", stream);
    hipLaunchKernelGGL(tri_invit, dim3(nb_mat), dim3(PT), smi, stream, dd, ee, int64_t(N), N, m, lamg, Zs,
                       int64_t(4) * N * mp, mp, marks, clu_rel, status);
  }
  BE_RET_IF(check_launch(ctx, "tri_invit"));
  {
    const size_t smg = gs_smem(m);
    if (smg > 65536)
      BE_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(&tri_gs),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(smg)));
    ProfScope prof(ctx, "tri_gs", stream);
    hipLaunchKernelGGL(tri_gs, dim3(nb_mat), dim3(PT), smg, stream, N, m, lamg, Zs, int64_t(4) * N * mp, mp, marks, Gm,
                       clu_rel, status);
  }
  BE_RET_IF(check_launch(ctx, "tri_gs"));
  // back-transformation target: the output itself (FP64) or an FP32 copy (mixed)
  C *Ut = mixed ? Uw : reinterpret_cast<C *>(U);
  const int ldt = mixed ? N : ldu;
  const int64_t ust = mixed ? int64_t(N) * m : us;
  // ---- symmetric orthonormalization of Z (Newton-Schulz on the Gram matrix),
  // Z held as X = Z^T (m x N, leading dim mp), each matrix until max |X X^T - I|
  // is below 1e-14 (FP64 path), or 2e-7 on the mixed path, whose FP32
  // back-transformation leaves errors of that order in U = QZ anyway (inverse
  // iteration alone typically gives 1e-8 there: no Newton-Schulz step is
  // then taken). At most 8 steps; outside graph capture the host stops once no
  // matrix is left (read back after every step), under capture every step is
  // launched and finished matrices skip it.
  {
    const double tol_orth = mixed ? 2e-7 : 1e-14;
    const bool capturing = stream_capturing(stream);
    const int64_t sZ = int64_t(4) * N * mp;
    double *const X0 = Zs + int64_t(3) * N * mp, *const X1 = Zs;
    double *Xa = X0, *Xt = X1;
    unsigned char parity = 0;
    int *hleft = static_cast<int *>(ctx->pinned);
    hipLaunchKernelGGL(ns_init_real, dim3((nb_mat + 255) / 256), dim3(256), 0, stream, nact, nloc, nb_mat);
    BE_RET_IF(check_launch(ctx, "ns_init_real"));
    for (int it = 0; it < 8; ++it) {
      DGemm g;  // G = X X^T
      g.M = m;
      g.N = m;
      g.K = N;
      g.opA = 0;
      g.opB = 1;
      g.A = Xa;
      g.lda = mp;
      g.bA = ZBatch::strided(sZ);
      g.B = Xa;
      g.ldb = mp;
      g.bB = ZBatch::strided(sZ);
      g.C = Gm;
      g.ldc = m;
      g.bC = ZBatch::strided(int64_t(m) * m);
      g.batch = nb_mat;
      g.tag = "reorth";
      g.sym = true;
      g.act = nact;
      BE_RET_IF(dgemm(ctx, g, stream));
      hipLaunchKernelGGL(ns_prep_real, dim3(nb_mat), dim3(PT), 0, stream, Gm, m, oerr, nact, tol_orth);
      BE_RET_IF(check_launch(ctx, "ns_prep_real"));
      DGemm h;  // X <- (3 I - G) X / 2
      h.M = m;
      h.N = N;
      h.K = m;
      h.A = Gm;
      h.lda = m;
      h.bA = ZBatch::strided(int64_t(m) * m);
      h.B = Xa;
      h.ldb = mp;
      h.bB = ZBatch::strided(sZ);
      h.C = Xt;
      h.ldc = mp;
      h.bC = ZBatch::strided(sZ);
      h.batch = nb_mat;
      h.tag = "reorth";
      h.act = nact;
      BE_RET_IF(dgemm(ctx, h, stream));
      hipLaunchKernelGGL(zero_i32, dim3(1), dim3(1), 0, stream, n_left);
      hipLaunchKernelGGL(ns_post_real, dim3((nb_mat + 255) / 256), dim3(256), 0, stream, nact, nloc, oerr, nb_mat,
                         static_cast<unsigned char>(parity ^ 1), n_left);
      BE_RET_IF(check_launch(ctx, "ns_post_real"));
      std::swap(Xa, Xt);
      parity ^= 1;
      if (!capturing) {
        BE_HIP_TRY(ctx, hipMemcpyAsync(hleft, n_left, sizeof(int), hipMemcpyDeviceToHost, stream));
        BE_HIP_TRY(ctx, hipStreamSynchronize(stream));
        if (*hleft == 0) break;
      }
    }
    hipLaunchKernelGGL(flag_nonorth, dim3((nb_mat + 255) / 256), dim3(256), 0, stream, oerr, nb_mat,
                       std::max(tol_orth, 1e-10), status);
    const int zt = ((N + 63) / 64) * ((m + 63) / 64);
    hipLaunchKernelGGL(z_to_u<C>, dim3(static_cast<uint32_t>(zt), static_cast<uint32_t>(nb_mat)), dim3(256), 0, stream,
                       X0, X1, nloc, sZ, mp, N, m, Ut, ldt, ust);
    BE_RET_IF(check_launch(ctx, "z_to_u"));
  }
  // ---- back-transformation by pairs of panels (pa, pb = pa + 1), last pair
  // first; with an odd panel count the first panel runs alone at the end.
  // Columns p0 .. p0 + nbc of H hold V = [V1 V2] explicitly (zeros above the
  // unit entries), so one compact-WY block of nbc <= 2 NB columns needs only
  // T = [[T1, -T1 (V1^H V2) T2], [0, T2]].
  constexpr int NB2 = 2 * NB;
  auto gemm = [&](int M_, int N_, int K_, int opA, const C *A_, int lda_, int64_t sA_, const C *B_, int ldb_,
                  int64_t sB_, C *C_, int ldc_, int64_t sC_, double alpha, double beta) {
    G g;
    g.M = M_;
    g.N = N_;
    g.K = K_;
    g.opA = opA;
    g.opB = 0;
    g.A = A_;
    g.lda = lda_;
    g.bA = ZBatch::strided(sA_);
    g.B = B_;
    g.ldb = ldb_;
    g.bB = ZBatch::strided(sB_);
    g.C = C_;
    g.ldc = ldc_;
    g.bC = ZBatch::strided(sC_);
    g.alpha = mk<C>(alpha, 0.0);
    g.beta = mk<C>(beta, 0.0);
    g.batch = nb_mat;
    g.tag = "unmtr";
    if constexpr (std::is_same<G, CGemm>::value) g.bf16x3 = bf16x3;
    return GemmOf<T>::run(ctx, g, stream);
  };
  const int64_t sXY = int64_t(NB2) * std::max(m, 1);
  for (int pb = P - 1; pb >= 0; pb -= 2) {
    const int pa = pb - 1;
    const bool pair = pa >= 0;
    const int p0 = (pair ? pa : pb) * NB;
    const int nb1 = pair ? NB : 0, nb2 = std::min(NB, N - pb * NB), nbc = nb1 + nb2;
    const int K = N - p0 - 1;
    if (K <= 0) continue;
    const C *Tblk = Tm + int64_t(pb) * NB * NB;
    int ldT = NB;
    int64_t sTb = sT;
    if (pair) {
      const int p0b = pb * NB, K12 = N - p0b - 1;
      // S12 = V1^H V2 (V2 is zero above row p0b + 1)
      if (K12 > 0) {
        BE_RET_IF(gemm(nb1, nb2, K12, 1, H + (p0b + 1) + int64_t(p0) * ld, ld, ms, H + (p0b + 1) + int64_t(p0b) * ld,
                       ld, ms, Sw, NB, int64_t(NB) * NB, 1.0, 0.0));
      } else {
        hipLaunchKernelGGL(zero_c<C>, dim3((nb_mat * NB * NB + 255) / 256), dim3(256), 0, stream, Sw,
                           nb_mat * NB * NB);
        BE_RET_IF(check_launch(ctx, "zero_c"));
      }
      // W = T1 S12; upper-right block of T = -W T2
      BE_RET_IF(gemm(nb1, nb2, nb1, 0, Tm + int64_t(pa) * NB * NB, NB, sT, Sw, NB, int64_t(NB) * NB, Ww, NB,
                     int64_t(NB) * NB, 1.0, 0.0));
      BE_RET_IF(gemm(nb1, nb2, nb2, 0, Ww, NB, int64_t(NB) * NB, Tm + int64_t(pb) * NB * NB, NB, sT,
                     Tb + int64_t(nb1) * NB2, NB2, int64_t(NB2) * NB2, -1.0, 0.0));
      hipLaunchKernelGGL(assemble_tpair<C>, dim3(static_cast<uint32_t>(nb_mat)), dim3(256), 0, stream,
                         Tm + int64_t(pa) * NB * NB, Tm + int64_t(pb) * NB * NB, sT, Tb, nb1, nb2);
      BE_RET_IF(check_launch(ctx, "assemble_tpair"));
      Tblk = Tb;
      ldT = NB2;
      sTb = int64_t(NB2) * NB2;
    }
    // X = V^H U(p0+1:, :), Y = T X, U(p0+1:, :) -= V Y
    BE_RET_IF(gemm(nbc, m, K, 1, H + (p0 + 1) + int64_t(p0) * ld, ld, ms, Ut + (p0 + 1), ldt, ust, Xb, NB2, sXY,
                   1.0, 0.0));
    BE_RET_IF(gemm(nbc, m, nbc, 0, Tblk, ldT, sTb, Xb, NB2, sXY, Yb, NB2, sXY, 1.0, 0.0));
    BE_RET_IF(gemm(K, m, nbc, 0, H + (p0 + 1) + int64_t(p0) * ld, ld, ms, Yb, NB2, sXY, Ut + (p0 + 1), ldt, ust,
                   -1.0, 1.0));
  }
  if (mixed) {
    hipLaunchKernelGGL(widen_u, dim3(64, static_cast<uint32_t>(nb_mat)), dim3(256), 0, stream,
                       reinterpret_cast<const float2 *>(Uw), int64_t(N) * m, N, m, U, ldu, us);
    BE_RET_IF(check_launch(ctx, "widen_u"));
  }
  return BE_OK;
}

// Matrices the panel kernel holds resident on the whole device at once (one
// workgroup per matrix): CUs times resident workgroups per CU.
template <typename T>
static int64_t panel_slots(be_ctx *ctx, int N) {
  typedef typename CT<T>::c C;
  const int pnt = panel_threads(ctx, N, sizeof(C));
  const size_t psm = panel_lds(N, sizeof(C), pnt);
  PanelFn<T> panel = panel_kernel<T>(pnt, panel_loads(ctx, N, sizeof(C), pnt), panel_part_lds(N, sizeof(C), pnt));
  int per_cu = 0;
  if (psm > 65536 && hipFuncSetAttribute(reinterpret_cast<const void *>(panel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(psm)) != hipSuccess)
    (void)hipGetLastError();
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(panel), pnt, psm) !=
      hipSuccess) {
    (void)hipGetLastError();
    per_cu = 0;
  }
  return int64_t(std::max(per_cu, 1)) * ctx->n_cu;
}

// The panel vectors and the tridiagonal solver's arrays live in LDS.
static int check_eigh_lds(be_ctx *ctx, int N, int m, size_t cs) {
  const size_t lds_need = std::max({panel_lds(N, cs, panel_threads(ctx, N, cs)), (4 * size_t(N) + m + 4) * sizeof(double),
                                    (3 * size_t(N) + m) * sizeof(double) + (size_t(N) + 1 + 2 * size_t(m)) * sizeof(int),
                                    gs_smem(m)});
  BE_CHECK_ARG(ctx, lds_need <= 160 * 1024, "be_eigh_batched: order too large for the LDS-resident kernels");
  return BE_OK;
}

// Workspace bytes per matrix of eigh_chunk for order N and m bands.
template <typename T>
static size_t eigh_chunk_bytes(be_ctx *ctx, int N, int m) {
  const int P = (N + NB - 1) / NB;
  const int mp = std::max(64, (m + 63) / 64 * 64);
  const size_t cs = sizeof(typename CT<T>::c);
  return cs * (size_t(N) * 3 * NB + size_t(P) * NB * NB + 4 * size_t(NB) * std::max(m, 1) + 6 * size_t(NB) * NB +
               size_t(N) * std::max(m, 1)) +
         (panel_part_lds(N, cs, panel_threads(ctx, N, cs)) ? 0 : panel_part_bytes(N - 1, cs)) +
         sizeof(double) * (3 * size_t(N) + 4 * size_t(N) * mp + size_t(std::max(m, 1)) * std::max(m, 1) + size_t(m) +
                           1) +
         sizeof(int) * size_t(std::max(m, 1)) + 16 * 256;
}

// Matrices per sub-batch for `per` workspace bytes per matrix: at most ~4 GiB
// of workspace; where that holds fewer than one device-wide round of resident
// panel workgroups (large N), up to one round within 48 GiB (or half the free
// device memory plus the `reusable` bytes the context already holds). The
// panel kernel streams at full bandwidth only while the device is full: a
// sub-batch is a whole number of device-wide rounds of resident workgroups
// where the cap allows one, and the sub-batches are made equal, so that no
// short remainder costs a full round per panel (4,608 matrices of order 400
// with 768 resident: six sub-batches of 768; 9,216: twelve).
template <typename T>
static int64_t eigh_sub_batch(be_ctx *ctx, int N, size_t per, size_t reusable, int64_t n_mat) {
  const int64_t slots = panel_slots<T>(ctx, N);
  int64_t cap = std::max<int64_t>(1, int64_t((size_t(4) << 30) / per));
  if (cap < slots) {
    size_t free_b = 0, total_b = 0;
    size_t budget = size_t(48) << 30;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
      budget = std::min(budget, free_b / 2 + reusable);
    else
      (void)hipGetLastError();
    cap = std::max<int64_t>(cap, std::min<int64_t>(slots, int64_t(budget / per)));
  }
  if (cap >= slots) cap = cap / slots * slots;
  const int64_t n_sub = (n_mat + cap - 1) / cap;
  return (n_mat + n_sub - 1) / n_sub;
}

template <typename T>
static int eigh_run(be_ctx *ctx, typename CT<T>::c *H, int N, int ld, int64_t mat_stride, int64_t n_mat, int band_lo,
                    int band_hi, double *evals, double2 *U, int ldu, int64_t u_stride, uint32_t *status,
                    hipStream_t stream, double clu_rel = kCluRel, bool bf16x3 = false) {
  const int m = band_hi - band_lo;
  BE_RET_IF(check_eigh_lds(ctx, N, m, sizeof(typename CT<T>::c)));
  if (n_mat == 0) return BE_OK;
  const size_t per = eigh_chunk_bytes<T>(ctx, N, m);
  const int64_t cap = eigh_sub_batch<T>(ctx, N, per, ctx->ws_bytes[WS_EIGH], n_mat);
  for (int64_t b0 = 0; b0 < n_mat; b0 += cap) {
    const int64_t nb_mat = std::min<int64_t>(cap, n_mat - b0);
    BE_RET_IF(eigh_chunk<T>(ctx, H + b0 * mat_stride, N, ld, mat_stride, nb_mat, band_lo, band_hi, evals + b0 * (m + 2),
                            U + b0 * u_stride, ldu, u_stride, status + b0, stream, clu_rel, bf16x3));
  }
  return BE_OK;
}

// Refined mixed precision (BE_MIXED_FP32_REFINED), one sub-batch: the mixed
// path for all N bands of an FP32 copy of H, then, in FP64 with the FP64 H,
// one first-order correction of the window's invariant subspace from the
// complement's vectors V (G = H U_w, [S | P] = V^H [G | U_w], F from S, P and
// the eigenvalues, U_w += V F), Rayleigh-quotient eigenvalues and a
// Newton-Schulz orthonormalization of U_w. The error of the FP32 subspace
// (~1e-6 relative) enters the result squared.
static int eigh_refined_chunk(be_ctx *ctx, const double2 *H, int N, int ld, int64_t ms, int64_t nb, int lo, int hi,
                              double *evals, double2 *U, int ldu, int64_t us, uint32_t *status, hipStream_t stream) {
  const int m = hi - lo, nc = N - m;
  const int mm = std::max(m, 1);
  const int64_t NN = int64_t(N) * N, sGU = int64_t(N) * 2 * mm, sS2 = int64_t(std::max(nc, 1)) * 2 * mm;
  double2 *Hf = nullptr, *Uall = nullptr, *GU = nullptr, *S2 = nullptr, *Gm = nullptr;
  float2 *Hc = nullptr;
  double *lam = nullptr, *err = nullptr;
  int *act = nullptr, *n_left = nullptr;
  unsigned char *loc = nullptr;
  Carve cv;
  cv.add(&Hf, size_t(nb * NN));
  cv.add(&Hc, size_t(nb * NN));
  cv.add(&Uall, size_t(nb * NN));
  cv.add(&lam, size_t(nb * (N + 2)));
  cv.add(&GU, size_t(nb * sGU));
  cv.add(&S2, size_t(nb * sS2));
  cv.add(&Gm, size_t(nb) * mm * mm);
  cv.add(&err, size_t(nb));
  cv.add(&act, size_t(nb));
  cv.add(&loc, size_t(nb));
  cv.add(&n_left, 1);
  BE_RET_IF(cv.commit(ctx, stream, WS_MISC));
  const uint32_t gy = static_cast<uint32_t>(std::min<int64_t>(nb, 65535));
  {
    const int nt = (N + 31) / 32;
    hipLaunchKernelGGL(split_h, dim3(static_cast<uint32_t>(nt * (nt + 1) / 2), gy), dim3(256), 0, stream, H, ms, ld,
                       N, nb, Hf, Hc);
    BE_RET_IF(check_launch(ctx, "split_h"));
  }
  // all bands on the mixed path (zeroes status)
  BE_RET_IF(eigh_chunk<float>(ctx, Hc, N, N, NN, nb, 0, N, lam, Uall, N, NN, status, stream));
  auto zg = [&](int M_, int N_, int K_, int opA, const double2 *A_, int lda_, int64_t sA_, const double2 *B_, int ldb_,
                int64_t sB_, double2 *C_, int ldc_, int64_t sC_, double beta, const char *tag) {
    ZGemm g;
    g.M = M_;
    g.N = N_;
    g.K = K_;
    g.opA = opA;
    g.opB = 0;
    g.A = A_;
    g.lda = lda_;
    g.bA = ZBatch::strided(sA_);
    g.B = B_;
    g.ldb = ldb_;
    g.bB = ZBatch::strided(sB_);
    g.C = C_;
    g.ldc = ldc_;
    g.bC = ZBatch::strided(sC_);
    g.alpha = make_double2(1.0, 0.0);
    g.beta = make_double2(beta, 0.0);
    g.batch = nb;
    g.tag = tag;
    return zgemm(ctx, g, stream);
  };
  if (m > 0) {
    hipLaunchKernelGGL(refine_copy_u, dim3(64, gy), dim3(256), 0, stream, Uall, N, lo, m, nb, GU, U, ldu, us);
    BE_RET_IF(check_launch(ctx, "refine_copy_u"));
    // G = H U_w into the left half of GU
    BE_RET_IF(zg(N, m, N, 0, Hf, N, NN, Uall + int64_t(lo) * N, N, NN, GU, N, sGU, 0.0, "refine_hu"));
  }
  hipLaunchKernelGGL(refine_evals, dim3(static_cast<uint32_t>(nb)), dim3(PT), 0, stream, GU, N, m, lo, lam, evals,
                     status);
  BE_RET_IF(check_launch(ctx, "refine_evals"));
  if (m == 0) return BE_OK;
  if (nc > 0) {
    // [S | P] = V^H [G | U_w]: the complement's rows, bands below lo then above hi
    if (lo > 0) BE_RET_IF(zg(lo, 2 * m, N, 1, Uall, N, NN, GU, N, sGU, S2, nc, sS2, 0.0, "refine_proj"));
    if (hi < N)
      BE_RET_IF(zg(N - hi, 2 * m, N, 1, Uall + int64_t(hi) * N, N, NN, GU, N, sGU, S2 + lo, nc, sS2, 0.0,
                   "refine_proj"));
    const int64_t work = nb * int64_t(nc) * m;
    hipLaunchKernelGGL(refine_coef, dim3(static_cast<uint32_t>(std::min<int64_t>((work + 255) / 256, 65536))),
                       dim3(256), 0, stream, S2, nc, m, lo, N, lam, nb);
    BE_RET_IF(check_launch(ctx, "refine_coef"));
    // U_w += V F
    if (lo > 0) BE_RET_IF(zg(N, m, lo, 0, Uall, N, NN, S2, nc, sS2, U, ldu, us, 1.0, "refine_corr"));
    if (hi < N)
      BE_RET_IF(zg(N, m, N - hi, 0, Uall + int64_t(hi) * N, N, NN, S2 + lo, nc, sS2, U, ldu, us, 1.0, "refine_corr"));
  }
  // Newton-Schulz orthonormalization in FP64, ping-pong between U (buffer 0)
  // and the left half of GU (buffer 1); a matrix whose error is below 1e-8
  // takes its last step, which leaves rounding (a last step from 1e-6 left
  // about 1e-12, enough to spread the +-1 eigenvalues of a projected spin
  // operator formed from these vectors over 1e-12, where the eigensolver's
  // cluster tolerance splits them into nearly parallel inverse-iteration
  // vectors)
  struct Buf {
    double2 *p;
    int ld;
    int64_t s;
  } buf[2] = {{U, ldu, us}, {GU, N, sGU}};
  const bool capturing = stream_capturing(stream);
  int *hleft = static_cast<int *>(ctx->pinned);
  hipLaunchKernelGGL(ns_init_real, dim3(static_cast<uint32_t>((nb + 255) / 256)), dim3(256), 0, stream, act, loc, nb);
  BE_RET_IF(check_launch(ctx, "ns_init_real"));
  int cur = 0;
  for (int it = 0; it < 4; ++it) {
    const Buf &X = buf[cur], &Y = buf[cur ^ 1];
    ZGemm g;  // Gm = X^H X
    g.M = m;
    g.N = m;
    g.K = N;
    g.opA = 1;
    g.opB = 0;
    g.A = X.p;
    g.lda = X.ld;
    g.bA = ZBatch::strided(X.s);
    g.B = X.p;
    g.ldb = X.ld;
    g.bB = ZBatch::strided(X.s);
    g.C = Gm;
    g.ldc = m;
    g.bC = ZBatch::strided(int64_t(m) * m);
    g.batch = nb;
    g.tag = "refine_orth";
    g.herm = true;
    g.four_mult = true;  // the Gram matrix's small off-diagonal entries to full relative accuracy
    g.act = act;
    BE_RET_IF(zgemm(ctx, g, stream));
    hipLaunchKernelGGL(ns_prep_cplx, dim3(static_cast<uint32_t>(nb)), dim3(PT), 0, stream, Gm, m, err, act, 1e-14,
                       1e-8);
    BE_RET_IF(check_launch(ctx, "ns_prep_cplx"));
    ZGemm h;  // Y = X (3 I - Gm) / 2
    h.M = N;
    h.N = m;
    h.K = m;
    h.A = X.p;
    h.lda = X.ld;
    h.bA = ZBatch::strided(X.s);
    h.B = Gm;
    h.ldb = m;
    h.bB = ZBatch::strided(int64_t(m) * m);
    h.C = Y.p;
    h.ldc = Y.ld;
    h.bC = ZBatch::strided(Y.s);
    h.batch = nb;
    h.tag = "refine_orth";
    h.act = act;
    BE_RET_IF(zgemm(ctx, h, stream));
    hipLaunchKernelGGL(zero_i32, dim3(1), dim3(1), 0, stream, n_left);
    hipLaunchKernelGGL(ns_post_real, dim3(static_cast<uint32_t>((nb + 255) / 256)), dim3(256), 0, stream, act, loc, err,
                       nb, static_cast<unsigned char>(cur ^ 1), n_left);
    BE_RET_IF(check_launch(ctx, "ns_post_real"));
    cur ^= 1;
    if (!capturing) {
      BE_HIP_TRY(ctx, hipMemcpyAsync(hleft, n_left, sizeof(int), hipMemcpyDeviceToHost, stream));
      BE_HIP_TRY(ctx, hipStreamSynchronize(stream));
      if (*hleft == 0) break;
    }
  }
  hipLaunchKernelGGL(flag_nonorth, dim3(static_cast<uint32_t>((nb + 255) / 256)), dim3(256), 0, stream, err, nb, 1e-10,
                     status);
  hipLaunchKernelGGL(refine_copy_back, dim3(64, gy), dim3(256), 0, stream, GU, sGU, N, m, loc, nb, U, ldu, us);
  return check_launch(ctx, "refine_copy_back");
}

static int eigh_refined(be_ctx *ctx, const double2 *H, int N, int ld, int64_t ms, int64_t n_mat, int lo, int hi,
                        double *evals, double2 *U, int ldu, int64_t us, uint32_t *status, hipStream_t stream) {
  const int m = hi - lo, nc = N - m;
  BE_RET_IF(check_eigh_lds(ctx, N, N, sizeof(float2)));
  if (n_mat == 0) return BE_OK;
  const int mm = std::max(m, 1);
  const size_t own = 16 * (3 * size_t(N) * N + size_t(N) * 2 * mm + size_t(std::max(nc, 1)) * 2 * mm +
                           size_t(mm) * mm) -
                     8 * size_t(N) * N + 8 * (size_t(N) + 2) + 16 + 6 * 256;
  const size_t per = eigh_chunk_bytes<float>(ctx, N, N) + own;
  const int64_t cap =
      eigh_sub_batch<float>(ctx, N, per, ctx->ws_bytes[WS_EIGH] + ctx->ws_bytes[WS_MISC], n_mat);
  for (int64_t b0 = 0; b0 < n_mat; b0 += cap) {
    const int64_t nb = std::min<int64_t>(cap, n_mat - b0);
    BE_RET_IF(eigh_refined_chunk(ctx, H + b0 * ms, N, ld, ms, nb, lo, hi, evals + b0 * (m + 2), U + b0 * us, ldu, us,
                                 status + b0, stream));
  }
  return BE_OK;
}

int eigh_fp64(be_ctx *ctx, double2 *H, int N, int ld, int64_t mat_stride, int64_t n_mat, int band_lo, int band_hi,
              double *evals, double2 *U, int ldu, int64_t u_stride, uint32_t *status, hipStream_t stream,
              double clu_rel) {
  return eigh_run<double>(ctx, H, N, ld, mat_stride, n_mat, band_lo, band_hi, evals, U, ldu, u_stride, status, stream, clu_rel);
}

int eigh_mixed(be_ctx *ctx, float2 *H, int N, int ld, int64_t mat_stride, int64_t n_mat, int band_lo, int band_hi,
               double *evals, double2 *U, int ldu, int64_t u_stride, uint32_t *status, hipStream_t stream,
               bool bf16x3) {
  return eigh_run<float>(ctx, H, N, ld, mat_stride, n_mat, band_lo, band_hi, evals, U, ldu, u_stride, status, stream,
                         kCluRel, bf16x3);
}

}  // namespace be

extern "C" int be_eigh_batched(be_ctx *ctx, void *H, int32_t dtype, int32_t N, int32_t ld, int64_t mat_stride,
                               int32_t n_mat, int32_t band_lo, int32_t band_hi, int32_t precision, double *evals,
                               void *U, int32_t ldu, int64_t u_stride, uint32_t *status, hipStream_t stream) {
  using namespace be;
  BE_CHECK_ARG(ctx, ctx && H && evals && U && status, "be_eigh_batched: null argument");
  BE_CHECK_ARG(ctx, N >= 1 && n_mat >= 0, "be_eigh_batched: N < 1 or n_mat < 0");
  BE_CHECK_ARG(ctx, 0 <= band_lo && band_lo <= band_hi && band_hi <= N, "be_eigh_batched: need 0 <= lo <= hi <= N");
  BE_CHECK_ARG(ctx, ld >= N && mat_stride >= int64_t(ld) * N, "be_eigh_batched: ld < N or mat_stride < ld*N");
  const int m = band_hi - band_lo;
  BE_CHECK_ARG(ctx, ldu >= N && u_stride >= int64_t(ldu) * std::max(m, 1), "be_eigh_batched: ldu < N or u_stride too small");
  if (precision == BE_FP64) {
    BE_CHECK_ARG(ctx, dtype == BE_C128, "be_eigh_batched: BE_FP64 needs BE_C128 matrices");
    return eigh_run<double>(ctx, static_cast<double2 *>(H), N, ld, mat_stride, n_mat, band_lo, band_hi, evals,
                            static_cast<double2 *>(U), ldu, u_stride, status, stream);
  }
  if (precision == BE_MIXED_FP32_REFINED) {
    BE_CHECK_ARG(ctx, dtype == BE_C128, "be_eigh_batched: BE_MIXED_FP32_REFINED needs BE_C128 matrices");
    return eigh_refined(ctx, static_cast<const double2 *>(H), N, ld, mat_stride, n_mat, band_lo, band_hi, evals,
                        static_cast<double2 *>(U), ldu, u_stride, status, stream);
  }
  if (precision == BE_MIXED_FP32 || precision == BE_MIXED_BF16X) {
    BE_CHECK_ARG(ctx, dtype == BE_C64, "be_eigh_batched: BE_MIXED_FP32 and BE_MIXED_BF16X need BE_C64 matrices");
    return eigh_run<float>(ctx, static_cast<float2 *>(H), N, ld, mat_stride, n_mat, band_lo, band_hi, evals,
                           static_cast<double2 *>(U), ldu, u_stride, status, stream, kCluRel,
                           precision == BE_MIXED_BF16X);
  }
  return set_err(ctx, BE_EINVAL, "be_eigh_batched: unknown precision");
}

extern "C" int be_eigh_round(be_ctx *ctx, int32_t N, int32_t precision, int64_t *round) {
  using namespace be;
  BE_CHECK_ARG(ctx, ctx && round, "be_eigh_round: null argument");
  BE_CHECK_ARG(ctx, N >= 1, "be_eigh_round: N < 1");
  if (precision == BE_FP64) {
    *round = panel_slots<double>(ctx, N);
  } else if (precision == BE_MIXED_FP32 || precision == BE_MIXED_FP32_REFINED || precision == BE_MIXED_BF16X) {
    *round = panel_slots<float>(ctx, N);
  } else {
    return set_err(ctx, BE_EINVAL, "be_eigh_round: unknown precision");
  }
  return BE_OK;
}

// Batched complex GEMM on CDNA4 matrix cores.
//
//   C_q = alpha op(A_q) op(B_q) + beta C_q,  op in {none, conjugate transpose}
//
// Complex products use three real MFMAs per 16x16 tile and k-step (Gauss:
// Ar Br, Ai Bi and (Ar + Ai)(Br + Bi) accumulated apart; at the end
// Cr = Ar Br - Ai Bi and Ci = (Ar + Ai)(Br + Bi) - Ar Br - Ai Bi), a quarter
// less matrix-core work than the four products of the textbook form, which
// callers can ask for (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br) where a
// Hermitian product must come out bitwise Hermitian. Tiles of A and B are staged
// through LDS as separate real and imaginary planes laid out [k][row], so
// every MFMA operand fetch is one conflict-free 8-byte (4-byte) LDS read per
// lane. The MFMA's "A" operand is taken from the B tile and its "B" operand
// from the A tile, so that the accumulator registers of a lane hold one row
// index i = lane % 16 and four column indices (the register-to-row map of
// the accumulator differs between the FP64 and FP32 instructions): the
// epilogue then writes 16 consecutive rows of a column-major C per
// quarter-wave.
//
// Workgroups are mapped XCD-aware: the tiles of one batch item are given
// consecutive work ids, which land on the same XCD (shared L2).
#include "common.hpp"

namespace {

constexpr int KB = 16;  // complex k per LDS stage (4 MFMA k-steps of 4)

template <typename T>
struct MF;

template <>
struct MF<double> {
  typedef v4d acc_t;
  typedef double2 cplx;
  static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register r of lane (lk = lane / 16) holds output row lk + 4 r
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};

template <>
struct MF<float> {
  typedef v4f acc_t;
  typedef float2 cplx;
  static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register r of lane (lk = lane / 16) holds output row 4 lk + r
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

template <typename T>
struct GP {
  typedef typename MF<T>::cplx cplx;
  int M, N, K;
  const cplx *A;
  int lda;
  be::ZBatch bA;
  const cplx *B;
  int ldb;
  be::ZBatch bB;
  cplx *C;
  int ldc;
  be::ZBatch bC;
  cplx alpha, beta;
  int64_t batch;
  int tiles_m, tiles_n;
  int herm;  // Hermitian C: lower tiles only, strictly lower tiles mirrored into the upper triangle (if mirror)
  int mirror;
  int four_mult;  // complex products in the four-product form
  const int *act;  // per batch item: 0 skips the item (its C is left untouched), or null
  const double *sB;  // row scales of B (OPB == 0), or null: s_q = sB + (q / sB_div) * sB_ld
  int64_t sB_div, sB_ld;
};

// BM x BN block tile, WM x WN waves, each wave (BM/WM) x (BN/WN).
template <typename T, int BM, int BN, int WM, int WN, int OPA, int OPB, bool M3>
__global__ __launch_bounds__(64 * WM * WN) void zgemm_kernel(GP<T> p) {
  typedef typename MF<T>::cplx cplx;
  typedef typename MF<T>::acc_t acc_t;
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int PA = BM + 2;  // LDS pitch (elements)
  constexpr int PB = BN + 2;
  __shared__ T sAr[KB * PA], sAi[KB * PA], sBr[KB * PB], sBi[KB * PB];

  const int64_t tiles = int64_t(p.tiles_m) * p.tiles_n;
  const int64_t total = tiles * p.batch;
  const int64_t w = be::xcd_work_id(total);
  if (w >= total) return;
  const int64_t q = w / tiles;
  const int t2 = static_cast<int>(w - q * tiles);
  const int tm = t2 % p.tiles_m, tn = t2 / p.tiles_m;
  const int i0 = tm * BM, j0 = tn * BN;
  static_assert(BM == BN, "square tiles (Hermitian mode pairs tile (tm, tn) with (tn, tm))");
  if (p.herm && tm < tn) return;
  if (p.act && p.act[q] == 0) return;
  const cplx *A = p.A + be::zbatch_off(p.bA, q);
  const cplx *B = p.B + be::zbatch_off(p.bB, q);
  cplx *C = p.C + be::zbatch_off(p.bC, q);
  const double *sBq = (OPB == 0 && p.sB) ? p.sB + (q / p.sB_div) * p.sB_ld : nullptr;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lk = lane >> 4;

  // M3: complex products by three real MFMAs (Gauss); else the four-product
  // form, which callers ask for where it matters that the Gauss form takes Ci
  // as a difference of large terms: the (i, j) and (j, i) entries of a
  // Hermitian product are then not exact conjugates, nor its diagonal real
  acc_t accr[TM][TN], acci[TM][TN], acc2[M3 ? TM : 1][M3 ? TN : 1];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      accr[a][b] = acc_t{0, 0, 0, 0};
      acci[a][b] = acc_t{0, 0, 0, 0};
      if constexpr (M3) acc2[a][b] = acc_t{0, 0, 0, 0};
    }

  // Software pipeline: the global loads of k-tile t+1 are issued into
  // registers before the MFMAs of tile t, and stored to LDS after them.
  constexpr int EA = (BM * KB + NT - 1) / NT;
  constexpr int EB = (BN * KB + NT - 1) / NT;
  cplx ga[EA], gb[EB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + u * NT;
      int i, k;
      if (OPA == 0) {
        i = e % BM;
        k = e / BM;
      } else {
        k = e % KB;
        i = e / KB;
      }
      const int gi = i0 + i, gk = k0 + k;
      cplx v;
      v.x = 0;
      v.y = 0;
      if (e < BM * KB && gi < p.M && gk < p.K) v = OPA == 0 ? A[gi + int64_t(gk) * p.lda] : A[gk + int64_t(gi) * p.lda];
      ga[u] = v;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + u * NT;
      int j, k;
      if (OPB == 0) {
        k = e % KB;
        j = e / KB;
      } else {
        j = e % BN;
        k = e / BN;
      }
      const int gj = j0 + j, gk = k0 + k;
      cplx v;
      v.x = 0;
      v.y = 0;
      if (e < BN * KB && gj < p.N && gk < p.K) {
        v = OPB == 0 ? B[gk + int64_t(gj) * p.ldb] : B[gj + int64_t(gk) * p.ldb];
        if (sBq) {
          const T sc = T(sBq[gk]);
          v.x *= sc;
          v.y *= sc;
        }
      }
      gb[u] = v;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + u * NT;
      if (e >= BM * KB) break;
      const int i = OPA == 0 ? e % BM : e / KB, k = OPA == 0 ? e / BM : e % KB;
      sAr[k * PA + i] = ga[u].x;
      sAi[k * PA + i] = OPA == 0 ? ga[u].y : -ga[u].y;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + u * NT;
      if (e >= BN * KB) break;
      const int j = OPB == 0 ? e / KB : e % BN, k = OPB == 0 ? e % KB : e / BN;
      sBr[k * PB + j] = gb[u].x;
      sBi[k * PB + j] = OPB == 0 ? gb[u].y : -gb[u].y;
    }
  };

  gload(0);
  for (int k0 = 0; k0 < p.K; k0 += KB) {
    sstore();
    __syncthreads();
    if (k0 + KB < p.K) gload(k0 + KB);
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
      T ar[TM], ai[TM], br[TN], bi[TN], nbi[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        int ii = wm * (BM / WM) + a * 16 + li;
        ar[a] = sAr[(kk + lk) * PA + ii];
        ai[a] = sAi[(kk + lk) * PA + ii];
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        int jj = wn * (BN / WN) + b * 16 + li;
        br[b] = sBr[(kk + lk) * PB + jj];
        bi[b] = sBi[(kk + lk) * PB + jj];
        nbi[b] = -bi[b];
      }
      if constexpr (M3) {
        // three real products per complex one: Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          const T as = ar[a] + ai[a];
#pragma unroll
          for (int b = 0; b < TN; ++b) {
            accr[a][b] = MF<T>::mfma(br[b], ar[a], accr[a][b]);
            acc2[a][b] = MF<T>::mfma(bi[b], ai[a], acc2[a][b]);
            acci[a][b] = MF<T>::mfma(br[b] + bi[b], as, acci[a][b]);
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) {
            accr[a][b] = MF<T>::mfma(br[b], ar[a], accr[a][b]);
            accr[a][b] = MF<T>::mfma(nbi[b], ai[a], accr[a][b]);
            acci[a][b] = MF<T>::mfma(bi[b], ar[a], acci[a][b]);
            acci[a][b] = MF<T>::mfma(br[b], ai[a], acci[a][b]);
          }
      }
    }
    __syncthreads();
  }
  if constexpr (M3) {  // Cr = Ar Br - Ai Bi, Ci = (Ar + Ai)(Br + Bi) - Ar Br - Ai Bi
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        acci[a][b] = acci[a][b] - accr[a][b] - acc2[a][b];
        accr[a][b] = accr[a][b] - acc2[a][b];
      }
  }

  // ---- epilogue: lane holds C(i = i_base + li, j = j_base + row(lk, r))
  const bool use_beta = (p.beta.x != T(0)) || (p.beta.y != T(0));
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      int gi = i0 + wm * (BM / WM) + a * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gj = j0 + wn * (BN / WN) + b * 16 + MF<T>::row(lk, r);
        if (gi < p.M && gj < p.N) {
          T xr = accr[a][b][r], xi = acci[a][b][r];
          cplx out;
          out.x = p.alpha.x * xr - p.alpha.y * xi;
          out.y = p.alpha.x * xi + p.alpha.y * xr;
          int64_t idx = gi + int64_t(gj) * p.ldc;
          if (use_beta) {
            cplx c = C[idx];
            out.x += p.beta.x * c.x - p.beta.y * c.y;
            out.y += p.beta.x * c.y + p.beta.y * c.x;
          }
          C[idx] = out;
          if (p.herm && p.mirror && tm > tn) {
            cplx o2 = out;
            o2.y = -out.y;
            C[gj + int64_t(gi) * p.ldc] = o2;
          }
        }
      }
    }
}

template <typename T, int BM, int BN, int WM, int WN>
int launch_cfg(be_ctx *ctx, GP<T> p, int opA, int opB, hipStream_t s) {
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + BN - 1) / BN;
  int64_t total = int64_t(p.tiles_m) * p.tiles_n * p.batch;
  dim3 grid(be::xcd_grid(total)), block(64 * WM * WN);
  if (p.four_mult) {
    if (opA == 0 && opB == 0) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 0, 0, false>), grid, block, 0, s, p);
    if (opA == 0 && opB == 1) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 0, 1, false>), grid, block, 0, s, p);
    if (opA == 1 && opB == 0) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 1, 0, false>), grid, block, 0, s, p);
    if (opA == 1 && opB == 1) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 1, 1, false>), grid, block, 0, s, p);
  } else {
    if (opA == 0 && opB == 0) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 0, 0, true>), grid, block, 0, s, p);
    if (opA == 0 && opB == 1) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 0, 1, true>), grid, block, 0, s, p);
    if (opA == 1 && opB == 0) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 1, 0, true>), grid, block, 0, s, p);
    if (opA == 1 && opB == 1) hipLaunchKernelGGL((zgemm_kernel<T, BM, BN, WM, WN, 1, 1, true>), grid, block, 0, s, p);
  }
  return be::check_launch(ctx, "zgemm");
}

// Fraction of the computed tile area that lies inside an M x N output for
// square tiles of side b.
inline double tile_fill(int M, int N, int b) {
  return (double(M) * N) / (double((M + b - 1) / b * b) * double((N + b - 1) / b * b));
}

// 64 x 64 tiles, unless 32 x 32 tiles waste clearly less of the output edge
// (e.g. 200 x 200: 61 % of the 64-tile area is output, 80 % of the 32-tile
// area); measured faster on the order-200 and order-400 products.
inline bool use_big_tiles(int M, int N) {
  return M >= 48 && N >= 48 && tile_fill(M, N, 64) * 1.15 >= tile_fill(M, N, 32);
}

template <typename T>
int dispatch(be_ctx *ctx, GP<T> p, int opA, int opB, hipStream_t s) {
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return BE_OK;
  // Tile choice by output size; small outputs use one-wave tiles.
  // 64 x 64 tiles with 8 waves (each 16 x 32): fewer registers per wave than
  // with 4 waves, twice the resident waves per SIMD (measured faster)
  if (use_big_tiles(p.M, p.N)) return launch_cfg<T, 64, 64, 4, 2>(ctx, p, opA, opB, s);
  if (p.M >= 24 && p.N >= 24) return launch_cfg<T, 32, 32, 2, 2>(ctx, p, opA, opB, s);
  return launch_cfg<T, 16, 16, 1, 1>(ctx, p, opA, opB, s);
}

// ---------------------------------------------------------------- split-bf16 complex GEMM
// The FP32 complex GEMM on the bf16 matrix cores: every FP32 operand x is
// split into x_hi = bf16(x) and x_lo = bf16(x - x_hi) (round to nearest even),
// and each real product x y is taken as x_hi y_hi + x_hi y_lo + x_lo y_hi
// (three v_mfma_f32_16x16x16_bf16, FP32 accumulation): about 16 significant
// bits per operand instead of FP32's 24, relative error ~2^-16 per product.
// Same tiles, work mapping, Hermitian mode and epilogue as zgemm_kernel;
// tiles of A and B are staged in LDS as bf16 planes (hi and lo of the real and
// imaginary parts) laid out [row][k], so that each lane's operand of four
// consecutive k is one 8-byte read. Operand lanes (checked on the device):
// lane l supplies row l % 16 of its operand at k = 4 (l / 16) + 0..3, and its
// accumulator register r holds output (4 (l / 16) + r, l % 16).
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite x)
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(uint32_t(h) << 16); }

template <int BM, int BN, int WM, int WN, int OPA, int OPB>
__global__ __launch_bounds__(64 * WM * WN) void zgemm_bf16x3_kernel(GP<float> p) {
  typedef float2 cplx;
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int KS = 16;        // k per stage: one bf16 MFMA step
  constexpr int KP = KS + 4;    // LDS row pitch (bf16 elements, a multiple of 4: 8-byte reads)
  // planes: 0 re hi, 1 re lo, 2 im hi, 3 im lo
  __shared__ __align__(16) unsigned short sA[4][BM * KP], sB[4][BN * KP];

  const int64_t tiles = int64_t(p.tiles_m) * p.tiles_n;
  const int64_t total = tiles * p.batch;
  const int64_t w = be::xcd_work_id(total);
  if (w >= total) return;
  const int64_t q = w / tiles;
  const int t2 = static_cast<int>(w - q * tiles);
  const int tm = t2 % p.tiles_m, tn = t2 / p.tiles_m;
  const int i0 = tm * BM, j0 = tn * BN;
  static_assert(BM == BN, "square tiles (Hermitian mode pairs tile (tm, tn) with (tn, tm))");
  if (p.herm && tm < tn) return;
  if (p.act && p.act[q] == 0) return;
  const cplx *A = p.A + be::zbatch_off(p.bA, q);
  const cplx *B = p.B + be::zbatch_off(p.bB, q);
  cplx *C = p.C + be::zbatch_off(p.bC, q);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lk = lane >> 4;

  v4f accr[TM][TN], acci[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      accr[a][b] = v4f{0, 0, 0, 0};
      acci[a][b] = v4f{0, 0, 0, 0};
    }

  constexpr int EA = (BM * KS + NT - 1) / NT;
  constexpr int EB = (BN * KS + NT - 1) / NT;
  cplx ga[EA], gb[EB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + u * NT;
      const int i = OPA == 0 ? e % BM : e / KS, k = OPA == 0 ? e / BM : e % KS;
      const int gi = i0 + i, gk = k0 + k;
      cplx v = {0.f, 0.f};
      if (e < BM * KS && gi < p.M && gk < p.K) v = OPA == 0 ? A[gi + int64_t(gk) * p.lda] : A[gk + int64_t(gi) * p.lda];
      ga[u] = v;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + u * NT;
      const int j = OPB == 0 ? e / KS : e % BN, k = OPB == 0 ? e % KS : e / BN;
      const int gj = j0 + j, gk = k0 + k;
      cplx v = {0.f, 0.f};
      if (e < BN * KS && gj < p.N && gk < p.K) v = OPB == 0 ? B[gk + int64_t(gj) * p.ldb] : B[gj + int64_t(gk) * p.ldb];
      gb[u] = v;
    }
  };
  auto split_store = [&](unsigned short (*pl)[(BM > BN ? BM : BN) * KP], int off, float re, float im) {
    const unsigned short rh = bf16_rne(re), ih = bf16_rne(im);
    pl[0][off] = rh;
    pl[1][off] = bf16_rne(re - bf16_to_f(rh));
    pl[2][off] = ih;
    pl[3][off] = bf16_rne(im - bf16_to_f(ih));
  };
  auto sstore = [&]() {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + u * NT;
      if (e >= BM * KS) break;
      const int i = OPA == 0 ? e % BM : e / KS, k = OPA == 0 ? e / BM : e % KS;
      split_store(sA, i * KP + k, ga[u].x, OPA == 0 ? ga[u].y : -ga[u].y);
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + u * NT;
      if (e >= BN * KS) break;
      const int j = OPB == 0 ? e / KS : e % BN, k = OPB == 0 ? e % KS : e / BN;
      split_store(sB, j * KP + k, gb[u].x, OPB == 0 ? gb[u].y : -gb[u].y);
    }
  };
  auto rd = [&](const unsigned short *plane, int row) {
    return *reinterpret_cast<const v4s *>(plane + row * KP + 4 * lk);
  };
  auto mf = [](v4s x, v4s y, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, c, 0, 0, 0); };
  const v4s sgn = {short(0x8000), short(0x8000), short(0x8000), short(0x8000)};

  gload(0);
  for (int k0 = 0; k0 < p.K; k0 += KS) {
    sstore();
    __syncthreads();
    if (k0 + KS < p.K) gload(k0 + KS);
    v4s arh[TM], arl[TM], aih[TM], ail[TM];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int ii = wm * (BM / WM) + a * 16 + li;
      arh[a] = rd(sA[0], ii);
      arl[a] = rd(sA[1], ii);
      aih[a] = rd(sA[2], ii);
      ail[a] = rd(sA[3], ii);
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int jj = wn * (BN / WN) + b * 16 + li;
      const v4s brh = rd(sB[0], jj), brl = rd(sB[1], jj), bih = rd(sB[2], jj), bil = rd(sB[3], jj);
      const v4s nbih = bih ^ sgn, nbil = bil ^ sgn;
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        // the MFMA's first operand from the B tile, its second from the A
        // tile: each lane's accumulators hold one output row
        v4f cr = accr[a][b], ci = acci[a][b];
        cr = mf(brl, arh[a], cr);   // Ar Br (small terms first)
        cr = mf(brh, arl[a], cr);
        cr = mf(brh, arh[a], cr);
        cr = mf(nbil, aih[a], cr);  // - Ai Bi
        cr = mf(nbih, ail[a], cr);
        cr = mf(nbih, aih[a], cr);
        ci = mf(bil, arh[a], ci);   // Ar Bi
        ci = mf(bih, arl[a], ci);
        ci = mf(bih, arh[a], ci);
        ci = mf(brl, aih[a], ci);   // Ai Br
        ci = mf(brh, ail[a], ci);
        ci = mf(brh, aih[a], ci);
        accr[a][b] = cr;
        acci[a][b] = ci;
      }
    }
    __syncthreads();
  }

  // ---- epilogue (as zgemm_kernel<float>): lane holds C(i_base + li, j_base + 4 lk + r)
  const bool use_beta = (p.beta.x != 0.f) || (p.beta.y != 0.f);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int gi = i0 + wm * (BM / WM) + a * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gj = j0 + wn * (BN / WN) + b * 16 + 4 * lk + r;
        if (gi < p.M && gj < p.N) {
          const float xr = accr[a][b][r], xi = acci[a][b][r];
          cplx out;
          out.x = p.alpha.x * xr - p.alpha.y * xi;
          out.y = p.alpha.x * xi + p.alpha.y * xr;
          const int64_t idx = gi + int64_t(gj) * p.ldc;
          if (use_beta) {
            const cplx c = C[idx];
            out.x += p.beta.x * c.x - p.beta.y * c.y;
            out.y += p.beta.x * c.y + p.beta.y * c.x;
          }
          C[idx] = out;
          if (p.herm && p.mirror && tm > tn) C[gj + int64_t(gi) * p.ldc] = make_float2(out.x, -out.y);
        }
      }
    }
}

template <int BM, int BN, int WM, int WN>
int launch_bf16x3(be_ctx *ctx, GP<float> p, int opA, int opB, hipStream_t s) {
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + BN - 1) / BN;
  int64_t total = int64_t(p.tiles_m) * p.tiles_n * p.batch;
  dim3 grid(be::xcd_grid(total)), block(64 * WM * WN);
  if (opA == 0 && opB == 0) hipLaunchKernelGGL((zgemm_bf16x3_kernel<BM, BN, WM, WN, 0, 0>), grid, block, 0, s, p);
  if (opA == 0 && opB == 1) hipLaunchKernelGGL((zgemm_bf16x3_kernel<BM, BN, WM, WN, 0, 1>), grid, block, 0, s, p);
  if (opA == 1 && opB == 0) hipLaunchKernelGGL((zgemm_bf16x3_kernel<BM, BN, WM, WN, 1, 0>), grid, block, 0, s, p);
  if (opA == 1 && opB == 1) hipLaunchKernelGGL((zgemm_bf16x3_kernel<BM, BN, WM, WN, 1, 1>), grid, block, 0, s, p);
  return be::check_launch(ctx, "zgemm_bf16x3");
}

int dispatch_bf16x3(be_ctx *ctx, GP<float> p, int opA, int opB, hipStream_t s) {
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return BE_OK;
  if (use_big_tiles(p.M, p.N)) return launch_bf16x3<64, 64, 4, 2>(ctx, p, opA, opB, s);
  if (p.M >= 24 && p.N >= 24) return launch_bf16x3<32, 32, 2, 2>(ctx, p, opA, opB, s);
  return launch_bf16x3<16, 16, 1, 1>(ctx, p, opA, opB, s);
}

// ---------------------------------------------------------------- real FP64 GEMM
// C = alpha op(A) op(B) + beta C with op in {none, transpose}; one MFMA per
// 16x16 tile and k-step, same staging and epilogue as the complex kernel.
struct DP {
  int M, N, K;
  const double *A;
  int lda;
  be::ZBatch bA;
  const double *B;
  int ldb;
  be::ZBatch bB;
  double *C;
  int ldc;
  be::ZBatch bC;
  double alpha, beta;
  int64_t batch;
  int tiles_m, tiles_n;
  int sym;  // symmetric C: lower tiles only, strictly lower tiles mirrored into the upper triangle
  const int *act;  // per batch item: 0 skips the item, or null
};

template <int BM, int BN, int WM, int WN, int OPA, int OPB>
__global__ __launch_bounds__(64 * WM * WN) void dgemm_kernel(DP p) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int DKB = 32;
  constexpr int PA = BM + 2;
  constexpr int PB = BN + 2;
  __shared__ double sA[DKB * PA], sB[DKB * PB];
  const int64_t tiles = int64_t(p.tiles_m) * p.tiles_n;
  const int64_t total = tiles * p.batch;
  const int64_t w = be::xcd_work_id(total);
  if (w >= total) return;
  const int64_t q = w / tiles;
  const int t2 = static_cast<int>(w - q * tiles);
  const int tm = t2 % p.tiles_m, tn = t2 / p.tiles_m;
  const int i0 = tm * BM, j0 = tn * BN;
  static_assert(BM == BN, "square tiles (symmetric mode pairs tile (tm, tn) with (tn, tm))");
  if (p.sym && tm < tn) return;
  if (p.act && p.act[q] == 0) return;
  const double *A = p.A + be::zbatch_off(p.bA, q);
  const double *B = p.B + be::zbatch_off(p.bB, q);
  double *C = p.C + be::zbatch_off(p.bC, q);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lk = lane >> 4;
  v4d acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  for (int k0 = 0; k0 < p.K; k0 += DKB) {
    for (int e = tid; e < BM * DKB; e += NT) {
      int i, k;
      if (OPA == 0) {
        i = e % BM;
        k = e / BM;
      } else {
        k = e % DKB;
        i = e / DKB;
      }
      int gi = i0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < p.M && gk < p.K) v = OPA == 0 ? A[gi + int64_t(gk) * p.lda] : A[gk + int64_t(gi) * p.lda];
      sA[k * PA + i] = v;
    }
    for (int e = tid; e < BN * DKB; e += NT) {
      int j, k;
      if (OPB == 0) {
        k = e % DKB;
        j = e / DKB;
      } else {
        j = e % BN;
        k = e / BN;
      }
      int gj = j0 + j, gk = k0 + k;
      double v = 0.0;
      if (gj < p.N && gk < p.K) v = OPB == 0 ? B[gk + int64_t(gj) * p.ldb] : B[gj + int64_t(gk) * p.ldb];
      sB[k * PB + j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < DKB; kk += 4) {
      double av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = sA[(kk + lk) * PA + wm * (BM / WM) + a * 16 + li];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = sB[(kk + lk) * PB + wn * (BN / WN) + b * 16 + li];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = MF<double>::mfma(bv[b], av[a], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      int gi = i0 + wm * (BM / WM) + a * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gj = j0 + wn * (BN / WN) + b * 16 + MF<double>::row(lk, r);
        if (gi < p.M && gj < p.N) {
          int64_t idx = gi + int64_t(gj) * p.ldc;
          double out = p.alpha * acc[a][b][r];
          if (p.beta != 0.0) out += p.beta * C[idx];
          C[idx] = out;
          if (p.sym && tm > tn) C[gj + int64_t(gi) * p.ldc] = out;
        }
      }
    }
}

template <int BM, int BN, int WM, int WN>
int dlaunch(be_ctx *ctx, DP p, int opA, int opB, hipStream_t s) {
  p.tiles_m = (p.M + BM - 1) / BM;
  p.tiles_n = (p.N + BN - 1) / BN;
  int64_t total = int64_t(p.tiles_m) * p.tiles_n * p.batch;
  dim3 grid(be::xcd_grid(total)), block(64 * WM * WN);
  if (opA == 0 && opB == 0) hipLaunchKernelGGL((dgemm_kernel<BM, BN, WM, WN, 0, 0>), grid, block, 0, s, p);
  if (opA == 0 && opB == 1) hipLaunchKernelGGL((dgemm_kernel<BM, BN, WM, WN, 0, 1>), grid, block, 0, s, p);
  if (opA == 1 && opB == 0) hipLaunchKernelGGL((dgemm_kernel<BM, BN, WM, WN, 1, 0>), grid, block, 0, s, p);
  if (opA == 1 && opB == 1) hipLaunchKernelGGL((dgemm_kernel<BM, BN, WM, WN, 1, 1>), grid, block, 0, s, p);
  return be::check_launch(ctx, "dgemm");
}

}  // namespace

namespace be {

int dgemm(be_ctx *ctx, const DGemm &g, hipStream_t stream) {
  ProfScope prof(ctx, g.tag, stream);
  DP p;
  p.M = g.M;
  p.N = g.N;
  p.K = g.K;
  p.A = g.A;
  p.lda = g.lda;
  p.bA = g.bA;
  p.B = g.B;
  p.ldb = g.ldb;
  p.bB = g.bB;
  p.C = g.C;
  p.ldc = g.ldc;
  p.bC = g.bC;
  p.alpha = g.alpha;
  p.beta = g.beta;
  p.batch = g.batch;
  p.sym = g.sym ? 1 : 0;
  p.act = g.act;
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return BE_OK;
  if (use_big_tiles(p.M, p.N)) return dlaunch<64, 64, 4, 2>(ctx, p, g.opA, g.opB, stream);
  if (p.M >= 24 && p.N >= 24) return dlaunch<32, 32, 2, 2>(ctx, p, g.opA, g.opB, stream);
  return dlaunch<16, 16, 1, 1>(ctx, p, g.opA, g.opB, stream);
}

int zgemm(be_ctx *ctx, const ZGemm &g, hipStream_t stream) {
  ProfScope prof(ctx, g.tag, stream);
  GP<double> p;
  p.M = g.M;
  p.N = g.N;
  p.K = g.K;
  p.A = g.A;
  p.lda = g.lda;
  p.bA = g.bA;
  p.B = g.B;
  p.ldb = g.ldb;
  p.bB = g.bB;
  p.C = g.C;
  p.ldc = g.ldc;
  p.bC = g.bC;
  p.alpha = g.alpha;
  p.beta = g.beta;
  p.batch = g.batch;
  p.herm = g.herm ? 1 : 0;
  p.mirror = g.herm_mirror ? 1 : 0;
  p.four_mult = g.four_mult ? 1 : 0;
  p.act = g.act;
  BE_CHECK_ARG(ctx, !g.scaleB || (g.opB == 0 && g.scaleB_div >= 1), "zgemm: row scaling of B needs opB = 'N'");
  p.sB = g.scaleB;
  p.sB_div = g.scaleB_div;
  p.sB_ld = g.scaleB_ld;
  return dispatch<double>(ctx, p, g.opA, g.opB, stream);
}

int cgemm(be_ctx *ctx, const CGemm &g, hipStream_t stream) {
  ProfScope prof(ctx, g.tag, stream);
  GP<float> p;
  p.M = g.M;
  p.N = g.N;
  p.K = g.K;
  p.A = g.A;
  p.lda = g.lda;
  p.bA = g.bA;
  p.B = g.B;
  p.ldb = g.ldb;
  p.bB = g.bB;
  p.C = g.C;
  p.ldc = g.ldc;
  p.bC = g.bC;
  p.alpha = g.alpha;
  p.beta = g.beta;
  p.batch = g.batch;
  p.herm = g.herm ? 1 : 0;
  p.mirror = g.herm_mirror ? 1 : 0;
  p.four_mult = g.four_mult ? 1 : 0;
  p.act = g.act;
  p.sB = nullptr;
  p.sB_div = 1;
  p.sB_ld = 0;
  if (g.bf16x3) return dispatch_bf16x3(ctx, p, g.opA, g.opB, stream);
  return dispatch<float>(ctx, p, g.opA, g.opB, stream);
}

}  // namespace be

extern "C" int be_zgemm_strided(be_ctx *ctx, char opA, char opB, int32_t M, int32_t Ncol, int32_t K,
                                const double *alpha2_h, const void *A, int32_t lda, int64_t strideA, const void *B,
                                int32_t ldb, int64_t strideB, const double *beta2_h, void *C, int32_t ldc,
                                int64_t strideC, int32_t batch, hipStream_t stream) {
  using namespace be;
  BE_CHECK_ARG(ctx, ctx && alpha2_h && beta2_h && A && B && C, "be_zgemm_strided: null argument");
  BE_CHECK_ARG(ctx, (opA == 'N' || opA == 'C') && (opB == 'N' || opB == 'C'), "be_zgemm_strided: op must be 'N' or 'C'");
  BE_CHECK_ARG(ctx, M >= 0 && Ncol >= 0 && K >= 0 && batch >= 0, "be_zgemm_strided: negative size");
  int ra = opA == 'N' ? M : K, rb = opB == 'N' ? K : Ncol;
  BE_CHECK_ARG(ctx, lda >= std::max(1, ra) && ldb >= std::max(1, rb) && ldc >= std::max(1, M),
               "be_zgemm_strided: leading dimension too small");
  ZGemm g;
  g.M = M;
  g.N = Ncol;
  g.K = K;
  g.opA = opA == 'C';
  g.opB = opB == 'C';
  g.A = static_cast<const double2 *>(A);
  g.lda = lda;
  g.bA = ZBatch::strided(strideA);
  g.B = static_cast<const double2 *>(B);
  g.ldb = ldb;
  g.bB = ZBatch::strided(strideB);
  g.C = static_cast<double2 *>(C);
  g.ldc = ldc;
  g.bC = ZBatch::strided(strideC);
  g.alpha = make_double2(alpha2_h[0], alpha2_h[1]);
  g.beta = make_double2(beta2_h[0], beta2_h[1]);
  g.batch = batch;
  return zgemm(ctx, g, stream);
}

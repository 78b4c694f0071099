// Products of Algorithm 1 on the matrix cores: the sketch A^T Omega, the
// power-iteration products A Qbar and A^T Q, the projection A^T Q, the Gram
// matrices X^T X of the Cholesky QR panels and the small X * M products.
//
// One kernel template, C = op(A) * B with op(A) = A or A^T and B column-major
// (K-contiguous).  Tiles of BM x BN outputs per workgroup, 4 waves; each wave
// owns WM x WN blocks of 16 x 16 and issues 16x16x4 MFMAs (fp64 or fp32).
// A and B tiles of depth BK are staged through LDS (double-buffered, with a
// register prefetch of the next tile).  The sketch products have a skinny
// output (N = d), so one workgroup covers all d columns and A is streamed
// from HBM once per product; split-K adds parallelism along the long
// contraction.  Partial sums are reduced in a fixed order (bitwise
// reproducible).  Gram products compute only upper tiles and mirror them.
#include <algorithm>
#include <vector>

#include "rqlp_internal.h"

namespace rqlp {
namespace {

template <typename TC>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double4_t acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef float4_t acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <typename TI, typename TC, typename TO, bool TA, int WAVES_M, int WAVES_N, int WM,
          int WN, int BK>
__device__ __forceinline__ void gemm_body(const TI* __restrict__ A, int64_t lda,
                                          const TI* __restrict__ B, int64_t ldb,
                                          TO* __restrict__ C, int64_t ldc, int64_t strideS,
                                          int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                          int gram, const int tile_m, const int tile_n,
                                          const int split) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M;
  constexpr int BN = 16 * WN * WAVES_N;
  constexpr int LA = BM + 1;
  constexpr int LB = BN + 1;
  constexpr int NA = (BM * BK + NT - 1) / NT;
  constexpr int NB = (BK * BN + NT - 1) / NT;
  typedef typename Mfma<TC>::acc_t acc_t;

  __shared__ TI As[2][BK][LA];
  __shared__ TI Bs[2][BK][LB];

  if (gram && tile_m > tile_n) return;  // whole workgroup leaves together
  const int64_t i0 = (int64_t)tile_m * BM, j0 = (int64_t)tile_n * BN;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wave_m = wave % WAVES_M, wave_n = wave / WAVES_M;

  acc_t acc[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  TI ra[NA], rb[NB];

  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + e * NT;
      int ii, kk;
      if (TA) {
        kk = idx % BK;
        ii = idx / BK;
      } else {
        ii = idx % BM;
        kk = idx / BM;
      }
      const int64_t gi = i0 + ii, gk = k0 + kk;
      TI v = (TI)0;
      if ((NA * NT == BM * BK || idx < BM * BK) && gi < M && gk < kend)
        v = TA ? A[gk + gi * lda] : A[gi + gk * lda];
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + e * NT;
      const int kk = idx % BK, jj = idx / BK;
      const int64_t gj = j0 + jj, gk = k0 + kk;
      TI v = (TI)0;
      if ((NB * NT == BK * BN || idx < BK * BN) && gj < N && gk < kend) v = B[gk + gj * ldb];
      rb[e] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int idx = tid + e * NT;
      if (NA * NT != BM * BK && idx >= BM * BK) continue;
      int ii, kk;
      if (TA) {
        kk = idx % BK;
        ii = idx / BK;
      } else {
        ii = idx % BM;
        kk = idx / BM;
      }
      As[buf][kk][ii] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + e * NT;
      if (NB * NT != BK * BN && idx >= BK * BN) continue;
      const int kk = idx % BK, jj = idx / BK;
      Bs[buf][kk][jj] = rb[e];
    }
  };

  const int64_t nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
    __syncthreads();
    for (int64_t it = 0; it < nk; ++it) {
      const int buf = (int)(it & 1);
      if (it + 1 < nk) gload(kbeg + (it + 1) * BK);
#pragma unroll
      for (int kq = 0; kq < BK / 4; ++kq) {
        const int kr = kq * 4 + (lane >> 4);
        TC af[WM], bf[WN];
#pragma unroll
        for (int a = 0; a < WM; ++a)
          af[a] = (TC)As[buf][kr][(wave_m * WM + a) * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < WN; ++b)
          bf[b] = (TC)Bs[buf][kr][(wave_n * WN + b) * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
          for (int b = 0; b < WN; ++b) acc[a][b] = Mfma<TC>::mma(af[a], bf[b], acc[a][b]);
      }
      if (it + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  }

  TO* Cs = C + (int64_t)split * strideS;
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      const int64_t col = j0 + (wave_n * WN + b) * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + (wave_m * WM + a) * 16 + acc_row<TC>(lane, r);
        if (row < M && col < N) Cs[row + col * ldc] = (TO)acc[a][b][r];
      }
    }
}

template <typename TI, typename TC, typename TO, bool TA, int WAVES_M, int WAVES_N, int WM,
          int WN, int BK>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void gemm_kernel(
    const TI* __restrict__ A, int64_t lda, const TI* __restrict__ B, int64_t ldb,
    TO* __restrict__ C, int64_t ldc, int64_t strideS, int64_t M, int64_t N, int64_t K,
    int64_t kchunk, int gram) {
  gemm_body<TI, TC, TO, TA, WAVES_M, WAVES_N, WM, WN, BK>(A, lda, B, ldb, C, ldc, strideS, M, N,
                                                          K, kchunk, gram, blockIdx.x,
                                                          blockIdx.y, blockIdx.z);
}

// Grouped form: workgroup b computes tile (bmap[b].y, bmap[b].z) of product
// descs[bmap[b].x] over its whole contraction (no split).
template <typename TI, typename TC, typename TO, bool TA, int WAVES_M, int WAVES_N, int WM,
          int WN, int BK>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void gemm_grouped_kernel(
    const GroupGemm* __restrict__ descs, const int4* __restrict__ bmap) {
  const int4 b = bmap[blockIdx.x];
  const GroupGemm g = descs[b.x];
  gemm_body<TI, TC, TO, TA, WAVES_M, WAVES_N, WM, WN, BK>(
      (const TI*)g.A, g.lda, (const TI*)g.B, g.ldb, (TO*)g.C, g.ldc, 0, g.M, g.N, g.K, g.K, 0,
      b.y, b.z, 0);
}

// C = sum_s P[s] in split order.  gram_bm > 0: element (i, j) in a lower
// tile (i / gram_bm > j / gram_bm) is read from its mirror (j, i).
template <typename TP, typename TO>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const TP* __restrict__ P, int64_t M,
                                                            int64_t N, int S,
                                                            TO* __restrict__ C, int64_t ldc,
                                                            int gram_bm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx % M, j = idx / M;
  int64_t si = i, sj = j;
  if (gram_bm > 0 && (i / gram_bm) > (j / gram_bm)) {
    si = j;
    sj = i;
  }
  const int64_t off = si + sj * M, stride = M * N;
  TP s = (TP)0;
#pragma unroll 8
  for (int t = 0; t < S; ++t) s += P[off + t * stride];
  C[i + j * ldc] = (TO)s;
}

// Precision form: C (fp32) = sum_k A16[k + i lda] B16[k + j ldb] with both
// operands 16-bit (bf16 or fp16) and contiguous along the contraction, fp32
// accumulation on the 16x16x32 MFMA.  A16 is the one-time rounded copy of A
// (or of A^T), B16 the rounded panel (convert_panel16_kernel).  Both are
// zero-padded along the contraction to a multiple of 64 (k16BK), so every
// tile is whole and the main loop carries no bounds checks; rows >= M and
// columns >= N read a clamped (valid) row or column and are never stored.
//
// Workgroup tile (32 WAVES) x (16 WN): the waves are stacked along M, each
// owning 32 rows (two 16-row blocks) and all 16 WN columns.  A rows belong to
// a single wave, so A fragments go from HBM straight into registers (one
// 32-byte load per lane and block covers two MFMA k-steps, prefetched one
// tile ahead); the panel tile, shared by the waves, is staged through LDS
// (double-buffered, 16-byte row padding so the 16 columns of a fragment read
// fall in distinct banks).  Within a 64-deep tile, MFMA k-step s takes, for
// lane group g = lane / 16, the tile rows 16 g + 8 s + [0, 8): the same
// permutation of k for both operands, so the sum is unchanged.
//
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2); the linear workgroup id is remapped so that each XCD works through a
// contiguous range of (row tile, column tile, split) items with the row tile
// fastest: the panel chunk of one (column tile, split) then stays in one L2.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

template <typename T16>
struct Mfma16;
template <>
struct Mfma16<__bf16> {
  typedef bf16x8_t v8;
  static __device__ __forceinline__ float4_t mma(v8 a, v8 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma16<_Float16> {
  typedef f16x8_t v8;
  static __device__ __forceinline__ float4_t mma(v8 a, v8 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ __bf16 to16(float x, __bf16*) {
  // round to nearest even on the upper 16 bits (NaN kept quiet)
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return __builtin_bit_cast(__bf16, (unsigned short)((u >> 16) | 0x40));
  u += 0x7fffu + ((u >> 16) & 1u);
  return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}
__device__ __forceinline__ _Float16 to16(float x, _Float16*) { return (_Float16)x; }

constexpr int k16BK = 64;     // contraction depth of one tile (and the zero padding unit)
constexpr int k16Waves = 4;   // waves per workgroup (32 rows each)
constexpr int k16BM = 32 * k16Waves;
constexpr int k16MaxWN = 17;  // up to 272 columns per workgroup
constexpr int kXcds = 8;

// Linear workgroup id -> work item such that the ids one XCD receives
// (those congruent to x mod 8) form one contiguous range of work items.
__device__ __forceinline__ int64_t xcd_remap(int64_t L, int64_t T) {
  const int64_t x = L % kXcds, j = L / kXcds;
  const int64_t per = T / kXcds, rem = T % kXcds;
  return (x < rem) ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

template <typename T16, int WN>
__global__ __launch_bounds__(64 * k16Waves, 2) void gemm16_kernel(
    const T16* __restrict__ A, int64_t lda, const T16* __restrict__ B, int64_t ldb,
    float* __restrict__ C, int64_t ldc, int64_t strideS, int64_t M, int64_t N, int64_t Kp,
    int64_t kchunk, int tiles_m, int tiles_n) {
  constexpr int NT = 64 * k16Waves;
  constexpr int WM = 2, BK = k16BK, LK = BK + 8, CH = BK / 8;
  constexpr int BN = 16 * WN;
  constexpr int CB = BN * CH, NB = (CB + NT - 1) / NT;
  typedef typename Mfma16<T16>::v8 v8;
  __shared__ __attribute__((aligned(16))) T16 Bs[2][BN][LK];

  const int64_t T = (int64_t)gridDim.x;
  const int64_t w = xcd_remap(blockIdx.x, T);
  const int tile_m = (int)(w % tiles_m);
  const int tile_n = (int)((w / tiles_m) % tiles_n);
  const int split = (int)(w / ((int64_t)tiles_m * tiles_n));
  const int64_t i0 = (int64_t)tile_m * k16BM, j0 = (int64_t)tile_n * BN;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = (kbeg + kchunk < Kp) ? kbeg + kchunk : Kp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane >> 4, r16 = lane & 15;

  // this lane's A rows (clamped); its 16 k of a tile start at 16 * grp
  const T16* arow[WM];
#pragma unroll
  for (int a = 0; a < WM; ++a) {
    int64_t row = i0 + wave * 32 + a * 16 + r16;
    row = row < M ? row : M - 1;
    arow[a] = A + row * lda + 16 * grp;
  }
  // this thread's panel chunks (clamped columns)
  const T16* bsrc[NB];
  int bdst[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int ch = tid + e * NT;
    const int col = (ch < CB ? ch : CB - 1) / CH, kc = (ch % CH) * 8;
    int64_t gj = j0 + col;
    gj = gj < N ? gj : N - 1;
    bsrc[e] = B + gj * ldb + kc;
    bdst[e] = col * LK + kc;
  }

  float4_t acc[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) acc[a][b] = float4_t{0, 0, 0, 0};

  v8 acur[WM][2], anext[WM][2], rb[NB];
  auto loadA = [&](v8 (&dst)[WM][2], int64_t k0) {
#pragma unroll
    for (int a = 0; a < WM; ++a) {
      dst[a][0] = *(const v8*)(arow[a] + k0);
      dst[a][1] = *(const v8*)(arow[a] + k0 + 8);
    }
  };
  auto loadB = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < NB; ++e)
      if (NB * NT == CB || tid + e * NT < CB) rb[e] = *(const v8*)(bsrc[e] + k0);
  };
  auto storeB = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NB; ++e)
      if (NB * NT == CB || tid + e * NT < CB) *(v8*)(&Bs[buf][0][0] + bdst[e]) = rb[e];
  };

  const int64_t nk = (kend - kbeg) / BK;  // whole tiles (kbeg, kend multiples of BK)
  if (nk > 0) {
    loadA(acur, kbeg);
    loadB(kbeg);
    storeB(0);
    __syncthreads();
    for (int64_t it = 0; it < nk; ++it) {
      const int buf = (int)(it & 1);
      const bool more = it + 1 < nk;
      if (more) {
        const int64_t k1 = kbeg + (it + 1) * BK;
        loadB(k1);
        loadA(anext, k1);
      }
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int b = 0; b < WN; ++b) {
          const v8 bf = *(const v8*)&Bs[buf][b * 16 + r16][16 * grp + 8 * s];
#pragma unroll
          for (int a = 0; a < WM; ++a) acc[a][b] = Mfma16<T16>::mma(acur[a][s], bf, acc[a][b]);
        }
      if (more) {
        storeB(buf ^ 1);
#pragma unroll
        for (int a = 0; a < WM; ++a) {
          acur[a][0] = anext[a][0];
          acur[a][1] = anext[a][1];
        }
      }
      __syncthreads();
    }
  }
  float* Cs = C + (int64_t)split * strideS;
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      const int64_t col = j0 + b * 16 + r16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + wave * 32 + a * 16 + acc_row_f32(lane, r);
        if (row < M && col < N) Cs[row + col * ldc] = acc[a][b][r];
      }
    }
}

// X (rows x d fp32, ldx) -> X16 (rows x d, ldy), rounded to nearest even;
// rows [rows, ldy) of X16 are set to zero (contraction padding).
template <typename T16>
__global__ __launch_bounds__(256) void convert_panel16_kernel(const float* __restrict__ X,
                                                              int64_t rows, int64_t d,
                                                              int64_t ldx, T16* __restrict__ Y,
                                                              int64_t ldy) {
  const int64_t total = ldy * d;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % ldy, j = idx / ldy;
    Y[idx] = i < rows ? to16(X[i + j * ldx], (T16*)nullptr) : (T16)0.0f;
  }
}

// A (m x n fp32, lda) -> A16 (m x n, ld16) and At16 = A^T (n x m, ldt16), both
// rounded to 16 bits (nearest even).  ld16 and ldt16 are m and n rounded up
// to multiples of 64; the padding rows of both copies are written as zeros
// (the contraction padding of gemm16_kernel).  64 x 64 tiles through LDS keep
// the transposed writes coalesced; the grid covers exactly the padded sizes.
// If rerr is given, each workgroup also writes the sum of squared rounding
// errors (a - a16)^2 of its tile (fp64) to rerr[its linear index].
template <typename T16>
__global__ __launch_bounds__(256) void convert16_kernel(const float* __restrict__ A, int64_t m,
                                                        int64_t n, int64_t lda,
                                                        T16* __restrict__ A16, int64_t ld16,
                                                        T16* __restrict__ At16, int64_t ldt16,
                                                        double* __restrict__ rerr) {
  __shared__ T16 tile[64][66];
  __shared__ double red[256];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  double err = 0.0;
  for (int jj = ty; jj < 64; jj += 4) {
    const int64_t i = i0 + tx, j = j0 + jj;
    T16 v = (T16)0.0f;
    if (i < m && j < n) {
      const float a = A[i + j * lda];
      v = to16(a, (T16*)nullptr);
      const double e = (double)a - (double)(float)v;
      err += e * e;
    }
    if (j < n) A16[i + j * ld16] = v;  // i < ld16 always
    tile[jj][tx] = v;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t j = j0 + tx, i = i0 + ii;
    if (i < m) At16[j + i * ldt16] = tile[tx][ii];  // j < ldt16 always
  }
  if (rerr) {
    red[threadIdx.x] = err;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) rerr[blockIdx.x + (int64_t)blockIdx.y * gridDim.x] = red[0];
  }
}

constexpr int kWavesM = 2, kWavesN = 2, kWM = 2, kBK = 16;
constexpr int kBM = 16 * kWM * kWavesM;  // 64
constexpr int kGramWM = 1;               // Gram products: 32 x 32 tiles
constexpr int kGramBM = 16 * kGramWM * kWavesM;
constexpr int kTargetWG = 1024;

// Compute units of the current device (cached per device).
int cu_count() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Workgroups of one kernel instantiation that fit on a CU at once (from its
// register and LDS use; 1 when the query fails, e.g. without a device).
template <typename F>
int occupancy_of(F kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

template <typename TI, typename TC, typename TO, bool TA, int WM, int WN>
int gemm_occupancy() {
  static const int nb = occupancy_of(gemm_kernel<TI, TC, TO, TA, kWavesM, kWavesN, WM, WN, kBK>,
                                     64 * kWavesM * kWavesN);
  return nb;
}

template <typename TI, typename TC, typename TO, bool TA>
int gemm_occupancy_wn(int wn) {
  switch (wn) {
    case 1: return gemm_occupancy<TI, TC, TO, TA, kWM, 1>();
    case 2: return gemm_occupancy<TI, TC, TO, TA, kWM, 2>();
    case 3: return gemm_occupancy<TI, TC, TO, TA, kWM, 3>();
    case 4: return gemm_occupancy<TI, TC, TO, TA, kWM, 4>();
    case 5: return gemm_occupancy<TI, TC, TO, TA, kWM, 5>();
    case 6: return gemm_occupancy<TI, TC, TO, TA, kWM, 6>();
    case 7: return gemm_occupancy<TI, TC, TO, TA, kWM, 7>();
    default: return gemm_occupancy<TI, TC, TO, TA, kWM, 8>();
  }
}

// Resident workgroups on the whole device for the product kernel chosen.
int gemm_slots(Dtype in_t, Dtype out_t, int trans_a, bool gram, int wn) {
  int nb = 1;
  if (gram) {
    if (in_t == DT_F64)
      nb = gemm_occupancy<double, double, double, true, kGramWM, 1>();
    else if (out_t == DT_F64)
      nb = gemm_occupancy<float, double, double, true, kGramWM, 1>();
    else
      nb = gemm_occupancy<float, float, float, true, kGramWM, 1>();
  } else if (in_t == DT_F64) {
    nb = trans_a ? gemm_occupancy_wn<double, double, double, true>(wn)
                 : gemm_occupancy_wn<double, double, double, false>(wn);
  } else {
    nb = trans_a ? gemm_occupancy_wn<float, float, float, true>(wn)
                 : gemm_occupancy_wn<float, float, float, false>(wn);
  }
  return nb * cu_count();
}

// Split-K choice by a small cost model: the grid runs in rounds of `slots`
// resident workgroups, each round taking one chunk's worth of tile work at
// `rate` flop/s over the device; each split beyond the first writes and the
// reduction reads one partial output (out_bytes) at ~4 TB/s.  Returns the
// chunk length (a multiple of bk) and the resulting split count.
void choose_splits(int64_t tiles, int64_t K, int bk, int64_t max_s, int64_t slots,
                   double tile_flops_per_k, double rate, double out_bytes, int64_t* chunk_out,
                   int* splits_out) {
  double best = 1e300;
  int64_t best_chunk = (K + bk - 1) / bk * bk;
  int best_s = 1;
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(max_s, 64));
  for (int64_t s0 = 1; s0 <= cap; ++s0) {
    int64_t chunk = (K + s0 - 1) / s0;
    chunk = (chunk + bk - 1) / bk * bk;
    if (chunk < bk) chunk = bk;
    const int64_t s = (K + chunk - 1) / chunk;
    const int64_t T = tiles * s;
    const int64_t rounds = (T + slots - 1) / slots;
    const double t = (double)rounds * (double)chunk * tile_flops_per_k / (rate / (double)slots) +
                     (s > 1 ? (double)s * out_bytes * 2.0 / 4e12 : 0.0);
    if (t < best * (1.0 - 1e-3)) {
      best = t;
      best_chunk = chunk;
      best_s = (int)s;
    }
  }
  *chunk_out = best_chunk;
  *splits_out = best_s;
}

struct Plan {
  int wn;          // 16-column blocks per wave along N (BN = 32 * wn)
  int64_t tiles_m, tiles_n;
  int splits;
  int64_t kchunk;
};

// Tile and split choice.  The A-streaming products (K = m or n, long) get
// one N tile covering d when d <= 256 (A is then read once), except that
// the A-row-major product (trans_a = 0) keeps at most 4 blocks per wave so
// it stays at two waves per SIMD; split-K is chosen by choose_splits with the
// kernel's real occupancy.  Short contractions cannot split, so they narrow
// the N tiles instead.  Gram products use 32 x 32 tiles (upper ones only).
Plan make_plan(int trans_a, int64_t M, int64_t N, int64_t K, bool gram, Dtype in_t,
               Dtype out_t) {
  Plan p;
  if (gram) {
    p.wn = 1;  // 32 x 32 tiles (kGramWM = 1)
  } else {
    const int cap = trans_a ? 8 : 4;
    const int64_t ntn = (N + 32 * cap - 1) / (32 * cap);
    const int64_t per = (N + ntn - 1) / ntn;
    p.wn = (int)std::max<int64_t>(1, std::min<int64_t>(cap, (per + 31) / 32));
  }
  p.tiles_m = gram ? (M + kGramBM - 1) / kGramBM : (M + kBM - 1) / kBM;
  const int64_t max_s = std::max<int64_t>(1, K / (kBK * 8));
  if (!gram && max_s == 1) {
    while (p.wn > 1 && p.tiles_m * ((N + 32 * p.wn - 1) / (32 * p.wn)) < kTargetWG / 2)
      p.wn = (p.wn + 1) / 2;
  }
  const int64_t BN = 32 * p.wn;
  p.tiles_n = (N + BN - 1) / BN;
  const int64_t tiles = gram ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  const int64_t BMx = gram ? kGramBM : kBM;
  const double rate = in_t == DT_F64 ? 45e12 : 110e12;
  const double es = out_t == DT_F64 ? 8.0 : 4.0;
  choose_splits(tiles, K, kBK, gram ? std::min<int64_t>(max_s, 48) : max_s,
                gemm_slots(in_t, out_t, trans_a, gram, p.wn), 2.0 * BMx * BN, rate,
                es * (double)M * (double)N, &p.kchunk, &p.splits);
  return p;
}

template <typename TI, typename TC, typename TO, bool TA, int WN>
void run_gemm(const GemmArgs& g, const Plan& p, TO* dst, int64_t lddst, int64_t strideS,
              hipStream_t st) {
  dim3 grid((unsigned)p.tiles_m, (unsigned)p.tiles_n, (unsigned)p.splits);
  hipLaunchKernelGGL((gemm_kernel<TI, TC, TO, TA, kWavesM, kWavesN, kWM, WN, kBK>), grid,
                     dim3(64 * kWavesM * kWavesN), 0, st, (const TI*)g.A, g.lda,
                     (const TI*)g.B, g.ldb, dst, lddst, strideS, g.M, g.N, g.K, p.kchunk,
                     g.gram ? 1 : 0);
}

template <typename TI, typename TC, typename TO, bool TA>
void dispatch_wn(const GemmArgs& g, const Plan& p, TO* dst, int64_t lddst, int64_t strideS,
                 hipStream_t st) {
  switch (p.wn) {
    case 1: run_gemm<TI, TC, TO, TA, 1>(g, p, dst, lddst, strideS, st); break;
    case 2: run_gemm<TI, TC, TO, TA, 2>(g, p, dst, lddst, strideS, st); break;
    case 3: run_gemm<TI, TC, TO, TA, 3>(g, p, dst, lddst, strideS, st); break;
    case 4: run_gemm<TI, TC, TO, TA, 4>(g, p, dst, lddst, strideS, st); break;
    case 5: run_gemm<TI, TC, TO, TA, 5>(g, p, dst, lddst, strideS, st); break;
    case 6: run_gemm<TI, TC, TO, TA, 6>(g, p, dst, lddst, strideS, st); break;
    case 7: run_gemm<TI, TC, TO, TA, 7>(g, p, dst, lddst, strideS, st); break;
    default: run_gemm<TI, TC, TO, TA, 8>(g, p, dst, lddst, strideS, st); break;
  }
}

template <typename TI, typename TC, typename TO>
hipError_t gemm_typed(const GemmArgs& g, hipStream_t st) {
  const Plan p = make_plan(g.trans_a, g.M, g.N, g.K, g.gram, g.in_t, g.out_t);
  const bool direct = (p.splits == 1) && !g.gram;
  TO* dst = direct ? (TO*)g.C : (TO*)g.partial;
  const int64_t lddst = direct ? g.ldc : g.M;
  const int64_t strideS = g.M * g.N;
  if (!direct && (g.partial == nullptr ||
                  g.partial_bytes < (size_t)p.splits * (size_t)strideS * sizeof(TO)))
    return hipErrorInvalidValue;
  if (g.ev_begin) (void)hipEventRecord((hipEvent_t)g.ev_begin, st);
  if (g.gram) {
    dim3 grid((unsigned)p.tiles_m, (unsigned)p.tiles_n, (unsigned)p.splits);
    hipLaunchKernelGGL((gemm_kernel<TI, TC, TO, true, kWavesM, kWavesN, kGramWM, 1, kBK>), grid,
                       dim3(64 * kWavesM * kWavesN), 0, st, (const TI*)g.A, g.lda,
                       (const TI*)g.B, g.ldb, dst, lddst, strideS, g.M, g.N, g.K, p.kchunk, 1);
  } else if (g.trans_a) {
    dispatch_wn<TI, TC, TO, true>(g, p, dst, lddst, strideS, st);
  } else {
    dispatch_wn<TI, TC, TO, false>(g, p, dst, lddst, strideS, st);
  }
  if (g.ev_end) (void)hipEventRecord((hipEvent_t)g.ev_end, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || direct) return e;
  const int64_t total = g.M * g.N;
  hipLaunchKernelGGL((splitk_reduce_kernel<TO, TO>), dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, st, (const TO*)g.partial, g.M, g.N, p.splits, (TO*)g.C,
                     g.ldc, g.gram ? kGramBM : 0);
  return hipGetLastError();
}

}  // namespace

size_t gemm_partial_bytes(int trans_a, int64_t M, int64_t N, int64_t K, Dtype in_t,
                          Dtype out_t, bool gram) {
  const Plan p = make_plan(trans_a, M, N, K, gram, in_t, out_t);
  if (p.splits == 1 && !gram) return 0;
  return (size_t)p.splits * (size_t)M * (size_t)N * (out_t == DT_F64 ? 8 : 4);
}

// Precision-form plan: k16BM-row tiles, N covered by as few tiles of at most
// 16 k16MaxWN columns as possible (A is read once per N tile), split-K up to
// ~1024 workgroups with at least four whole tiles per split.  Kp is the
// padded contraction length (a multiple of k16BK).
struct Plan16 {
  int wn;
  int64_t tiles_m, tiles_n;
  int splits;
  int64_t kchunk;
};

int64_t pad16(int64_t K) { return (K + k16BK - 1) / k16BK * k16BK; }

template <typename T16, int WN>
int gemm16_occupancy() {
  static const int nb = occupancy_of(gemm16_kernel<T16, WN>, 64 * k16Waves);
  return nb;
}

template <typename T16, int WN>
int gemm16_occupancy_wn(int wn) {
  if constexpr (WN > 1) {
    if (wn < WN) return gemm16_occupancy_wn<T16, WN - 1>(wn);
  }
  return gemm16_occupancy<T16, WN>();
}

Plan16 make_plan16(int64_t M, int64_t N, int64_t K, bool f16) {
  Plan16 p;
  const int64_t Kp = pad16(K);
  const int64_t nblk = (N + 15) / 16;
  p.tiles_n = (nblk + k16MaxWN - 1) / k16MaxWN;
  p.wn = (int)((nblk + p.tiles_n - 1) / p.tiles_n);
  p.tiles_m = (M + k16BM - 1) / k16BM;
  const int64_t tiles = p.tiles_m * p.tiles_n;
  const int64_t max_s = std::max<int64_t>(1, Kp / (4 * k16BK));
  const int occ = f16 ? gemm16_occupancy_wn<_Float16, k16MaxWN>(p.wn)
                      : gemm16_occupancy_wn<__bf16, k16MaxWN>(p.wn);
  choose_splits(tiles, Kp, k16BK, max_s, (int64_t)occ * cu_count(), 2.0 * k16BM * 16 * p.wn,
                900e12, 4.0 * (double)M * (double)N, &p.kchunk, &p.splits);
  return p;
}

template <typename T16, int WN>
static void run_gemm16(const Gemm16Args& g, const Plan16& p, float* dst, int64_t lddst,
                       int64_t strideS, hipStream_t st) {
  const unsigned T = (unsigned)(p.tiles_m * p.tiles_n * p.splits);
  hipLaunchKernelGGL((gemm16_kernel<T16, WN>), dim3(T), dim3(64 * k16Waves), 0, st,
                     (const T16*)g.A, g.lda, (const T16*)g.B, g.ldb, dst, lddst, strideS, g.M,
                     g.N, pad16(g.K), p.kchunk, (int)p.tiles_m, (int)p.tiles_n);
}

template <typename T16, int WN>
static void dispatch16(const Gemm16Args& g, const Plan16& p, float* dst, int64_t lddst,
                       int64_t strideS, hipStream_t st) {
  if constexpr (WN > 1) {
    if (p.wn < WN) return dispatch16<T16, WN - 1>(g, p, dst, lddst, strideS, st);
  }
  run_gemm16<T16, WN>(g, p, dst, lddst, strideS, st);
}

template <typename T16>
static hipError_t gemm16_typed(const Gemm16Args& g, hipStream_t st) {
  const Plan16 p = make_plan16(g.M, g.N, g.K, g.f16);
  const bool direct = (p.splits == 1);
  float* dst = direct ? g.C : (float*)g.partial;
  const int64_t lddst = direct ? g.ldc : g.M;
  const int64_t strideS = g.M * g.N;
  if (!direct && (g.partial == nullptr ||
                  g.partial_bytes < (size_t)p.splits * (size_t)strideS * sizeof(float)))
    return hipErrorInvalidValue;
  // whole 16-byte fragment loads over the zero-padded contraction
  if (g.lda < pad16(g.K) || g.ldb < pad16(g.K) || (g.lda % 8) != 0 || (g.ldb % 8) != 0 ||
      (((uintptr_t)g.A | (uintptr_t)g.B) & 15) != 0)
    return hipErrorInvalidValue;
  if (g.ev_begin) (void)hipEventRecord((hipEvent_t)g.ev_begin, st);
  dispatch16<T16, k16MaxWN>(g, p, dst, lddst, strideS, st);
  if (g.ev_end) (void)hipEventRecord((hipEvent_t)g.ev_end, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || direct) return e;
  const int64_t total = g.M * g.N;
  hipLaunchKernelGGL((splitk_reduce_kernel<float, float>), dim3((unsigned)((total + 255) / 256)),
                     dim3(256), 0, st, (const float*)g.partial, g.M, g.N, p.splits, g.C, g.ldc,
                     0);
  return hipGetLastError();
}

hipError_t launch_gemm16(const Gemm16Args& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  return g.f16 ? gemm16_typed<_Float16>(g, st) : gemm16_typed<__bf16>(g, st);
}

size_t gemm16_partial_bytes(int64_t M, int64_t N, int64_t K, bool f16) {
  const Plan16 p = make_plan16(M, N, K, f16);
  return p.splits == 1 ? 0 : (size_t)p.splits * (size_t)M * (size_t)N * 4;
}

int64_t gemm16_ld(int64_t K) { return pad16(K); }

hipError_t launch_convert_panel16(const float* X, int64_t rows, int64_t d, int64_t ldx, void* Y,
                                  int64_t ldy, bool f16, hipStream_t st) {
  if (rows <= 0 || d <= 0) return hipSuccess;
  if (ldy < pad16(rows) || ldy % k16BK != 0) return hipErrorInvalidValue;
  const int64_t total = ldy * d;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  if (f16)
    hipLaunchKernelGGL(convert_panel16_kernel<_Float16>, dim3(blocks), dim3(256), 0, st, X, rows,
                       d, ldx, (_Float16*)Y, ldy);
  else
    hipLaunchKernelGGL(convert_panel16_kernel<__bf16>, dim3(blocks), dim3(256), 0, st, X, rows, d,
                       ldx, (__bf16*)Y, ldy);
  return hipGetLastError();
}

int64_t convert16_blocks(int64_t m, int64_t n) { return ((m + 63) / 64) * ((n + 63) / 64); }

hipError_t launch_convert16(const float* A, int64_t m, int64_t n, int64_t lda, void* A16,
                            int64_t ld16, void* At16, int64_t ldt16, bool f16, hipStream_t st,
                            double* rerr) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (ld16 < pad16(m) || ldt16 < pad16(n)) return hipErrorInvalidValue;
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  if (f16)
    hipLaunchKernelGGL(convert16_kernel<_Float16>, grid, dim3(256), 0, st, A, m, n, lda,
                       (_Float16*)A16, ld16, (_Float16*)At16, ldt16, rerr);
  else
    hipLaunchKernelGGL(convert16_kernel<__bf16>, grid, dim3(256), 0, st, A, m, n, lda,
                       (__bf16*)A16, ld16, (__bf16*)At16, ldt16, rerr);
  return hipGetLastError();
}

namespace {

template <typename TI, typename TC, typename TO, bool TA, int WM, int WN>
void run_grouped(const GroupGemm* descs, const int4* bmap, int64_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL((gemm_grouped_kernel<TI, TC, TO, TA, kWavesM, kWavesN, WM, WN, kBK>),
                     dim3((unsigned)nblocks), dim3(64 * kWavesM * kWavesN), 0, st, descs, bmap);
}

template <typename T, bool TA>
void grouped_wn(int wn, const GroupGemm* descs, const int4* bmap, int64_t nblocks,
                hipStream_t st) {
  if (wn <= 1) run_grouped<T, T, T, TA, kWM, 1>(descs, bmap, nblocks, st);
  else if (wn <= 2) run_grouped<T, T, T, TA, kWM, 2>(descs, bmap, nblocks, st);
  else if (wn <= 4) run_grouped<T, T, T, TA, kWM, 4>(descs, bmap, nblocks, st);
  else run_grouped<T, T, T, TA, kWM, 8>(descs, bmap, nblocks, st);
}

}  // namespace

int grouped_wn_round(int wn) { return wn <= 1 ? 1 : wn <= 2 ? 2 : wn <= 4 ? 4 : 8; }

void gemm_grouped_blocks(const GroupGemm& g, int idx, bool gram, int wn,
                         std::vector<int4>& out) {
  const int64_t BM = gram ? kGramBM : kBM;
  const int64_t BN = gram ? 32 : 32 * grouped_wn_round(wn);
  const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  for (int64_t j = 0; j < tn; ++j)
    for (int64_t i = 0; i < tm; ++i)
      if (!gram || i >= j) out.push_back(int4{idx, (int)i, (int)j, 0});
}

hipError_t launch_gemm_grouped(Dtype in_t, Dtype out_t, int trans_a, bool gram, int wn,
                               const GroupGemm* descs, const int4* bmap, int64_t nblocks,
                               hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (gram) {
    if (in_t == DT_F64)
      run_grouped<double, double, double, true, kGramWM, 1>(descs, bmap, nblocks, st);
    else if (out_t == DT_F64)
      run_grouped<float, double, double, true, kGramWM, 1>(descs, bmap, nblocks, st);
    else
      return hipErrorInvalidValue;
  } else if (in_t != out_t) {
    return hipErrorInvalidValue;
  } else if (in_t == DT_F64) {
    if (trans_a) grouped_wn<double, true>(wn, descs, bmap, nblocks, st);
    else grouped_wn<double, false>(wn, descs, bmap, nblocks, st);
  } else {
    if (trans_a) grouped_wn<float, true>(wn, descs, bmap, nblocks, st);
    else grouped_wn<float, false>(wn, descs, bmap, nblocks, st);
  }
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.in_t == DT_F64 && g.out_t == DT_F64) return gemm_typed<double, double, double>(g, st);
  if (g.in_t == DT_F32 && g.out_t == DT_F32) return gemm_typed<float, float, float>(g, st);
  if (g.in_t == DT_F32 && g.out_t == DT_F64 && g.gram)
    return gemm_typed<float, double, double>(g, st);
  return hipErrorInvalidValue;
}

}  // namespace rqlp

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
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void gemm_kernel(
    const TI* __restrict__ A, int64_t lda, const TI* __restrict__ B, int64_t ldb,
    TO* __restrict__ C, int64_t ldc, int64_t strideS, int64_t M, int64_t N, int64_t K,
    int64_t kchunk, int gram) {
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

  const int tile_m = blockIdx.x, tile_n = blockIdx.y, split = blockIdx.z;
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

// Precision form: C (fp32) = A16^T X with A16 a 16-bit copy of A whose
// contraction index is contiguous (A16[k + i lda16]) and X an fp32 panel
// (X[k + j ldx]) rounded to 16 bits (nearest even) as it is staged.  Both
// operands sit in LDS with k contiguous, so one 16-byte read gives a lane
// the 8 consecutive k of its 16x16x32 MFMA fragment; fp32 accumulation.
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

template <typename T16, int WM, int WN, int BK>
__global__ __launch_bounds__(256) void gemm16_kernel(const T16* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ B, int64_t ldb,
                                                     float* __restrict__ C, int64_t ldc,
                                                     int64_t strideS, int64_t M, int64_t N,
                                                     int64_t K, int64_t kchunk) {
  constexpr int NT = 256;
  constexpr int BM = 32 * WM, BN = 32 * WN;
  constexpr int LK = BK + 8;  // padded row (elements)
  constexpr int CA = BM * BK / 8, CB = BN * BK / 8;  // 8-element chunks per tile
  constexpr int NA = (CA + NT - 1) / NT, NB = (CB + NT - 1) / NT;
  typedef typename Mfma16<T16>::v8 v8;
  __shared__ __attribute__((aligned(16))) T16 As[2][BM][LK];
  __shared__ __attribute__((aligned(16))) T16 Bs[2][BN][LK];

  const int tile_m = blockIdx.x, tile_n = blockIdx.y, split = blockIdx.z;
  const int64_t i0 = (int64_t)tile_m * BM, j0 = (int64_t)tile_n * BN;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wave_m = wave & 1, wave_n = wave >> 1;

  float4_t acc[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) acc[a][b] = float4_t{0, 0, 0, 0};

  v8 ra[NA], rb[NB];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int ch = tid + e * NT;
      const int ii = ch / (BK / 8), kk = (ch % (BK / 8)) * 8;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      v8 v;
      if ((NA * NT == CA || ch < CA) && gi < M && gk + 8 <= kend) {
        v = *(const v8*)(A + gk + gi * lda);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          v[t] = ((NA * NT == CA || ch < CA) && gi < M && gk + t < kend) ? A[gk + t + gi * lda]
                                                                          : (T16)0.0f;
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int ch = tid + e * NT;
      const int jj = ch / (BK / 8), kk = (ch % (BK / 8)) * 8;
      const int64_t gj = j0 + jj, gk = k0 + kk;
      v8 v;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float x = ((NB * NT == CB || ch < CB) && gj < N && gk + t < kend)
                            ? B[gk + t + gj * ldb] : 0.0f;
        v[t] = to16(x, (T16*)nullptr);
      }
      rb[e] = v;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int ch = tid + e * NT;
      if (NA * NT != CA && ch >= CA) continue;
      *(v8*)&As[buf][ch / (BK / 8)][(ch % (BK / 8)) * 8] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int ch = tid + e * NT;
      if (NB * NT != CB && ch >= CB) continue;
      *(v8*)&Bs[buf][ch / (BK / 8)][(ch % (BK / 8)) * 8] = rb[e];
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
      for (int kq = 0; kq < BK / 32; ++kq) {
        const int kc = kq * 32 + 8 * (lane >> 4);
        v8 af[WM], bf[WN];
#pragma unroll
        for (int a = 0; a < WM; ++a) af[a] = *(const v8*)&As[buf][(wave_m * WM + a) * 16 + (lane & 15)][kc];
#pragma unroll
        for (int b = 0; b < WN; ++b) bf[b] = *(const v8*)&Bs[buf][(wave_n * WN + b) * 16 + (lane & 15)][kc];
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
          for (int b = 0; b < WN; ++b) acc[a][b] = Mfma16<T16>::mma(af[a], bf[b], acc[a][b]);
      }
      if (it + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  }
  float* Cs = C + (int64_t)split * strideS;
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      const int64_t col = j0 + (wave_n * WN + b) * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + (wave_m * WM + a) * 16 + acc_row_f32(lane, r);
        if (row < M && col < N) Cs[row + col * ldc] = acc[a][b][r];
      }
    }
}

// A (m x n fp32, lda) -> A16 (m x n, ld16) and At16 = A^T (n x m, ldt16), both
// rounded to 16 bits (nearest even).  64 x 64 tiles through LDS keep the
// transposed writes coalesced.
template <typename T16>
__global__ __launch_bounds__(256) void convert16_kernel(const float* __restrict__ A, int64_t m,
                                                        int64_t n, int64_t lda,
                                                        T16* __restrict__ A16, int64_t ld16,
                                                        T16* __restrict__ At16, int64_t ldt16) {
  __shared__ T16 tile[64][66];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int jj = ty; jj < 64; jj += 4) {
    const int64_t i = i0 + tx, j = j0 + jj;
    T16 v = (T16)0.0f;
    if (i < m && j < n) {
      v = to16(A[i + j * lda], (T16*)nullptr);
      A16[i + j * ld16] = v;
    }
    tile[jj][tx] = v;
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t j = j0 + tx, i = i0 + ii;
    if (i < m && j < n) At16[j + i * ldt16] = tile[tx][ii];
  }
}

constexpr int kWavesM = 2, kWavesN = 2, kWM = 2, kBK = 16;
constexpr int kBM = 16 * kWM * kWavesM;  // 64
constexpr int kGramWM = 1;               // Gram products: 32 x 32 tiles
constexpr int kGramBM = 16 * kGramWM * kWavesM;
constexpr int kTargetWG = 1024;

struct Plan {
  int wn;          // 16-column blocks per wave along N (BN = 32 * wn)
  int64_t tiles_m, tiles_n;
  int splits;
  int64_t kchunk;
};

// Tile and split choice.  The A-streaming products (K = m or n, long) get
// one N tile covering d when d <= 256 (A is then read once), except that
// the A-row-major product (trans_a = 0) keeps at most 4 blocks per wave so
// it stays at two waves per SIMD; split-K brings the grid to ~1024
// workgroups.  Short contractions cannot split, so they narrow the N tiles
// instead.  Gram products use 32 x 32 tiles (upper ones only).
Plan make_plan(int trans_a, int64_t M, int64_t N, int64_t K, bool gram) {
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
  int64_t s = (kTargetWG + tiles - 1) / tiles;
  s = std::max<int64_t>(1, std::min(s, max_s));
  if (gram) s = std::min<int64_t>(s, 48);
  int64_t chunk = (K + s - 1) / s;
  chunk = (chunk + kBK - 1) / kBK * kBK;
  s = (K + chunk - 1) / chunk;
  if (s < 1) s = 1;
  p.splits = (int)s;
  p.kchunk = chunk > 0 ? chunk : kBK;
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
  const Plan p = make_plan(g.trans_a, g.M, g.N, g.K, g.gram);
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

int64_t gemm_tile_count(int trans_a, int64_t M, int64_t N, int64_t K, bool gram) {
  const Plan p = make_plan(trans_a, M, N, K, gram);
  return p.tiles_m * p.tiles_n;
}

size_t gemm_partial_bytes(int trans_a, int64_t M, int64_t N, int64_t K, Dtype in_t,
                          Dtype out_t, bool gram) {
  (void)in_t;
  const Plan p = make_plan(trans_a, M, N, K, gram);
  if (p.splits == 1 && !gram) return 0;
  return (size_t)p.splits * (size_t)M * (size_t)N * (out_t == DT_F64 ? 8 : 4);
}

template <typename T16, int WN>
static void run_gemm16(const Gemm16Args& g, const Plan& p, float* dst, int64_t lddst,
                       int64_t strideS, hipStream_t st) {
  dim3 grid((unsigned)p.tiles_m, (unsigned)p.tiles_n, (unsigned)p.splits);
  hipLaunchKernelGGL((gemm16_kernel<T16, 2, WN, 32>), grid, dim3(256), 0, st, (const T16*)g.A,
                     g.lda, g.B, g.ldb, dst, lddst, strideS, g.M, g.N, g.K, p.kchunk);
}

template <typename T16>
static hipError_t gemm16_typed(const Gemm16Args& g, hipStream_t st) {
  const Plan p = make_plan(1, g.M, g.N, g.K, false);
  const bool direct = (p.splits == 1);
  float* dst = direct ? g.C : (float*)g.partial;
  const int64_t lddst = direct ? g.ldc : g.M;
  const int64_t strideS = g.M * g.N;
  if (!direct && (g.partial == nullptr ||
                  g.partial_bytes < (size_t)p.splits * (size_t)strideS * sizeof(float)))
    return hipErrorInvalidValue;
  if (g.ev_begin) (void)hipEventRecord((hipEvent_t)g.ev_begin, st);
  switch (p.wn) {
    case 1: run_gemm16<T16, 1>(g, p, dst, lddst, strideS, st); break;
    case 2: run_gemm16<T16, 2>(g, p, dst, lddst, strideS, st); break;
    case 3: run_gemm16<T16, 3>(g, p, dst, lddst, strideS, st); break;
    case 4: run_gemm16<T16, 4>(g, p, dst, lddst, strideS, st); break;
    case 5: run_gemm16<T16, 5>(g, p, dst, lddst, strideS, st); break;
    case 6: run_gemm16<T16, 6>(g, p, dst, lddst, strideS, st); break;
    case 7: run_gemm16<T16, 7>(g, p, dst, lddst, strideS, st); break;
    default: run_gemm16<T16, 8>(g, p, dst, lddst, strideS, st); break;
  }
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

size_t gemm16_partial_bytes(int64_t M, int64_t N, int64_t K) {
  const Plan p = make_plan(1, M, N, K, false);
  return p.splits == 1 ? 0 : (size_t)p.splits * (size_t)M * (size_t)N * 4;
}

hipError_t launch_convert16(const float* A, int64_t m, int64_t n, int64_t lda, void* A16,
                            int64_t ld16, void* At16, int64_t ldt16, bool f16, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  if (f16)
    hipLaunchKernelGGL(convert16_kernel<_Float16>, grid, dim3(256), 0, st, A, m, n, lda,
                       (_Float16*)A16, ld16, (_Float16*)At16, ldt16);
  else
    hipLaunchKernelGGL(convert16_kernel<__bf16>, grid, dim3(256), 0, st, A, m, n, lda,
                       (__bf16*)A16, ld16, (__bf16*)At16, ldt16);
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

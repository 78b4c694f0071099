// Products of Algorithm 1 on the matrix cores: the sketch A^T Omega, the
// power-iteration products A Qbar and A^T Q, the projection A^T Q, the Gram
// matrices X^T X of the Cholesky QR panels and the small X * M products
// (the precision form's 16-bit products live in gemm16.hip).
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
// The fp64 products with A use gemm_stream_f64_kernel (gemm_f64.hip).
#include <algorithm>
#include <type_traits>
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

// REMV > 0 (with WAVES_N = 1): the tile is 16 WN + REMV columns wide; the
// last REMV columns (the ragged end of a skinny product, e.g. d = 210 =
// 13 x 16 + 2) are computed on the vector ALUs from the same A fragments
// the MFMAs use, instead of padding them to a whole 16-column MFMA block.
// Each lane sums its quarter of the k values; the four quarters are added
// across lanes (fixed order) at the end.
template <typename TI, typename TC, typename TO, bool TA, int WAVES_M, int WAVES_N, int WM,
          int WN, int BK, int REMV = 0>
__device__ __forceinline__ void gemm_body(const TI* __restrict__ A, int64_t lda,
                                          const TI* __restrict__ B, int64_t ldb,
                                          TO* __restrict__ C, int64_t ldc, int64_t strideS,
                                          int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                          int gram, const int tile_m, const int tile_n,
                                          const int split) {
  static_assert(REMV == 0 || WAVES_N == 1, "vector-ALU columns need one wave column");
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int BM = 16 * WM * WAVES_M;
  constexpr int BN = 16 * WN * WAVES_N + REMV;
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
  TC vacc[WM][REMV > 0 ? REMV : 1];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int c = 0; c < (REMV > 0 ? REMV : 1); ++c) vacc[a][c] = (TC)0;

  TI ra[NA], rb[NB];
  // global-address-space views (the grouped kernels pass pointers read from
  // descriptors, which the compiler would otherwise access with FLAT
  // instructions)
  const global_ptr<const TI> Ag = (global_ptr<const TI>)A;
  const global_ptr<const TI> Bg = (global_ptr<const TI>)B;

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
        v = TA ? Ag[gk + gi * lda] : Ag[gi + gk * lda];
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int idx = tid + e * NT;
      const int kk = idx % BK, jj = idx / BK;
      const int64_t gj = j0 + jj, gk = k0 + kk;
      TI v = (TI)0;
      if ((NB * NT == BK * BN || idx < BK * BN) && gj < N && gk < kend) v = Bg[gk + gj * ldb];
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
        if constexpr (REMV > 0) {
#pragma unroll
          for (int c = 0; c < REMV; ++c) {
            const TC bv = (TC)Bs[buf][kr][16 * WN + c];
#pragma unroll
            for (int a = 0; a < WM; ++a) vacc[a][c] = af[a] * bv + vacc[a][c];
          }
        }
      }
      if (it + 1 < nk) sstore(buf ^ 1);
      __syncthreads();
    }
  }

  const global_ptr<TO> Cs = (global_ptr<TO>)C + (int64_t)split * strideS;
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
  if constexpr (REMV > 0) {
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
      for (int c = 0; c < REMV; ++c) {
        TC v = vacc[a][c];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        const int64_t row = i0 + (wave_m * WM + a) * 16 + (lane & 15);
        const int64_t col = j0 + 16 * WN + c;
        if (lane < 16 && row < M && col < N) Cs[row + col * ldc] = (TO)v;
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

// Skinny products with a ragged width: 8 waves stacked along M (16 rows
// each in fp64, 32 in fp32, whose half-size registers leave room for a
// second row block that reuses every panel fragment read from LDS), WN MFMA
// blocks of 16 columns plus 4 vector-ALU columns per tile.  Every workgroup
// reads the panel tile of each k-step from L2, so taller workgroups read the
// panel fewer times: 8 waves (one workgroup per CU) measured 51.8 TFLOP/s in
// fp64 at 8000 x 8000, d = 210, against 47.9 with 4 waves (two per CU).
constexpr int kRemWavesM = 8, kRemV = 4;
// The grouped form keeps 4 waves: many small matrices have few row tiles,
// and 8-wave tiles measured a slower batch (51.1 against 49.7 ms).
constexpr int kRemGroupedWavesM = 4;
template <typename TI>
constexpr int rem_wm() { return sizeof(TI) == 4 ? 2 : 1; }
template <typename TI, typename TC, typename TO, bool TA, int WN>
__global__ __launch_bounds__(64 * kRemWavesM) void gemm_rem_kernel(
    const TI* __restrict__ A, int64_t lda, const TI* __restrict__ B, int64_t ldb,
    TO* __restrict__ C, int64_t ldc, int64_t strideS, int64_t M, int64_t N, int64_t K,
    int64_t kchunk) {
  // 8-deep tiles for A X (row tiles of A strided in memory: keeps the
  // register count within two waves per SIMD) and for the widest tiles
  // (keeps the LDS of one workgroup under the per-workgroup limit); 32-deep
  // tiles for narrow A^T X (up to 4 blocks, such as the predictor's 64-column
  // sketch), whose streaming of A is bound by the bytes one workgroup keeps
  // in flight
  gemm_body<TI, TC, TO, TA, kRemWavesM, 1, rem_wm<TI>(), WN,
            (TA && WN <= 4) ? 32 : ((TA && WN <= 13) ? 16 : 8), kRemV>(
      A, lda, B, ldb, C, ldc, strideS, M, N, K, kchunk, 0, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Grouped form of gemm_rem_kernel (whole contraction, no split).
template <typename TI, typename TC, typename TO, bool TA, int WN>
__global__ __launch_bounds__(64 * kRemGroupedWavesM) void gemm_rem_grouped_kernel(
    const GroupGemm* __restrict__ descs, const int4* __restrict__ bmap) {
  const int4 b = bmap[blockIdx.x];
  const GroupGemm g = descs[b.x];
  gemm_body<TI, TC, TO, TA, kRemGroupedWavesM, 1, rem_wm<TI>(), WN, (TA && WN <= 13) ? 16 : 8, kRemV>(
      (const TI*)g.A, g.lda, (const TI*)g.B, g.ldb, (TO*)g.C, g.ldc, 0, g.M, g.N, g.K, g.K, 0,
      b.y, b.z, 0);
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
// tile (i / gram_bm > j / gram_bm) is read from its mirror (j, i).  Grid:
// (ceil(M / (2 * 256)), N); each thread sums rows i, i + 1 of column j, with
// pair loads when `pairs` (M even, P aligned to a pair, no mirroring).
template <typename TP, typename TO>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const TP* __restrict__ P, int64_t M,
                                                            int64_t N, int S,
                                                            TO* __restrict__ C, int64_t ldc,
                                                            int gram_bm, int pairs) {
  typedef TP pair_t __attribute__((ext_vector_type(2)));
  const int64_t j = blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
  if (i0 >= M) return;
  const int64_t stride = M * N;
  if (pairs) {
    const TP* p = P + i0 + j * M;
    pair_t s = {(TP)0, (TP)0};
#pragma unroll 8
    for (int t = 0; t < S; ++t) s += *(const pair_t*)(p + t * stride);
    C[i0 + j * ldc] = (TO)s[0];
    C[i0 + 1 + j * ldc] = (TO)s[1];
    return;
  }
  for (int64_t i = i0; i < i0 + 2 && i < M; ++i) {
    int64_t si = i, sj = j;
    if (gram_bm > 0 && (i / gram_bm) > (j / gram_bm)) {
      si = j;
      sj = i;
    }
    const int64_t off = si + sj * M;
    TP s = (TP)0;
#pragma unroll 8
    for (int t = 0; t < S; ++t) s += P[off + t * stride];
    C[i + j * ldc] = (TO)s;
  }
}

// Small outputs with many splits (the d x d Gram matrices): four threads per
// output element, thread q summing the splits q, q + 4, ... in order, then
// the four quarters added in a fixed order -- deterministic, and four times
// the loads in flight of one thread per element; each thread issues all its
// loads (up to 16) before adding.  Element e = i + j M of the tight M x N
// partials.  gram_bm > 0 (a Gram matrix whose partials hold the upper tiles
// of gram_bm x gram_bm): only elements i <= j are read, from their own
// column (coalesced), and each is written to (i, j) and (j, i).
template <typename TP, typename TO>
__global__ __launch_bounds__(256) void splitk_reduce4_kernel(const TP* __restrict__ P, int64_t M,
                                                             int64_t N, int S,
                                                             TO* __restrict__ C, int64_t ldc,
                                                             int gram_bm) {
  __shared__ TP part[4][64];
  const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t total = M * N;
  const int64_t e = (int64_t)blockIdx.x * 64 + l;
  const int64_t i = e % M, j = e / M;
  const bool active = e < total && (gram_bm == 0 || i <= j);
  TP s = (TP)0;
  if (active) {
    const TP* p = P + e;
    constexpr int U = 16;
    TP v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = q + 4 * u;
      v[u] = t < S ? p[(int64_t)t * total] : (TP)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];  // adding +0 past S leaves s unchanged
    for (int t = q + 4 * U; t < S; t += 4) s += p[(int64_t)t * total];
  }
  part[q][l] = s;
  __syncthreads();
  if (q == 0 && active) {
    const TO r = (TO)((part[0][l] + part[1][l]) + (part[2][l] + part[3][l]));
    C[i + j * ldc] = r;
    if (gram_bm > 0 && i < j) C[j + i * ldc] = r;
  }
}

// The one-thread-per-element reduction is bound by the latency of its S
// dependent loads when the output is small; above this many elements it has
// enough threads.
constexpr int64_t kReduce4MaxElems = (int64_t)1 << 20;

dim3 splitk_reduce_grid(int64_t M, int64_t N) {
  return dim3((unsigned)((M + 511) / 512), (unsigned)N);
}

template <typename TP>
int splitk_pairs(const TP* P, int64_t M, int gram_bm) {
  return gram_bm == 0 && (M & 1) == 0 && ((uintptr_t)P % (2 * sizeof(TP))) == 0;
}

constexpr int kWavesM = 2, kWavesN = 2, kWM = 2, kBK = 16;
constexpr int kBM = 16 * kWM * kWavesM;  // 64
constexpr int kGramWM = 1;               // Gram products: 32 x 32 tiles
constexpr int kGramBM = 16 * kGramWM * kWavesM;

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

struct Plan {
  int wn;          // 16-column blocks per wave along N (BN = 32 * wn; rem: 16 * wn + 4)
  int64_t tiles_m, tiles_n;
  int splits;
  int64_t kchunk;
  bool rem = false;  // gemm_rem_kernel layout
  bool stream = false;  // gemm_stream_f64_kernel (fp64, wn <= kStrMaxWN)
  int rv = kRemV;        // its vector-ALU columns (2 or 4)
};

template <typename TI, typename TC, typename TO, bool TA, int WN>
int rem_occupancy() {
  static const int nb = occupancy_of(gemm_rem_kernel<TI, TC, TO, TA, WN>, 64 * kRemWavesM);
  return nb;
}

template <typename T, bool TA, int WN = 16>
int rem_occupancy_wn(int wn) {
  if constexpr (WN > 1) {
    if (wn < WN) return rem_occupancy_wn<T, TA, WN - 1>(wn);
  }
  return rem_occupancy<T, T, T, TA, WN>();
}

constexpr int kRemMaxWN = 16;

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
  // (an fp32 product with fewer rows than one remainder tile, such as the
  // d x d product Q^T Z, keeps the 64-row tiles below)
  const bool small_f32 = in_t == DT_F32 && M < 16 * kRemWavesM * rem_wm<float>();
  if (!gram && max_s > 1 && in_t == out_t && !small_f32) {
    // A-streaming product: MFMA blocks plus vector-ALU columns, as few N
    // tiles (of at most 16 x 16 + 4 columns) as possible.
    const int64_t wmax = 16 * kRemMaxWN + kRemV;
    const int64_t ntn = (N + wmax - 1) / wmax;
    const int64_t per = (N + ntn - 1) / ntn;
    int64_t wn = per / 16;
    if (per % 16 > kRemV) ++wn;
    p.wn = (int)std::max<int64_t>(1, std::min<int64_t>(wn, kRemMaxWN));
    p.rem = true;
    const int64_t BMr = 16 * kRemWavesM * (in_t == DT_F64 ? rem_wm<double>() : rem_wm<float>());
    p.tiles_m = (M + BMr - 1) / BMr;
    p.stream = in_t == DT_F64 && p.wn <= kStrMaxWN;
    if (p.stream && per - 16 * p.wn <= 2) p.rv = 2;
    const int64_t BN = 16 * p.wn + p.rv;
    p.tiles_n = (N + BN - 1) / BN;
    const int occ = p.stream ? gemm_stream_f64_occupancy(trans_a, p.wn)
                    : in_t == DT_F64
                        ? (trans_a ? rem_occupancy_wn<double, true>(p.wn)
                                   : rem_occupancy_wn<double, false>(p.wn))
                        : (trans_a ? rem_occupancy_wn<float, true>(p.wn)
                                   : rem_occupancy_wn<float, false>(p.wn));
    choose_splits(p.tiles_m * p.tiles_n, K, p.stream ? kStrBK : kBK, max_s,
                  (int64_t)occ * cu_count(),
                  2.0 * BMr * BN, in_t == DT_F64 ? 45e12 : 110e12,
                  (out_t == DT_F64 ? 8.0 : 4.0) * (double)M * (double)N, &p.kchunk, &p.splits);
    return p;
  }
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

template <typename TI, typename TC, typename TO, bool TA, int WN>
void dispatch_rem(const GemmArgs& g, const Plan& p, TO* dst, int64_t lddst, int64_t strideS,
                  hipStream_t st) {
  if constexpr (WN > 1) {
    if (p.wn < WN) return dispatch_rem<TI, TC, TO, TA, WN - 1>(g, p, dst, lddst, strideS, st);
  }
  dim3 grid((unsigned)p.tiles_m, (unsigned)p.tiles_n, (unsigned)p.splits);
  hipLaunchKernelGGL((gemm_rem_kernel<TI, TC, TO, TA, WN>), grid, dim3(64 * kRemWavesM), 0, st,
                     (const TI*)g.A, g.lda, (const TI*)g.B, g.ldb, dst, lddst, strideS, g.M, g.N,
                     g.K, p.kchunk);
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
  } else if (p.stream && (g.ldb % 2) == 0 && g.ldb < (1 << 20) && ((uintptr_t)g.B % 16) == 0) {
    if constexpr (std::is_same<TI, double>::value && std::is_same<TO, double>::value)
      launch_gemm_stream_f64(g.trans_a, p.wn, p.rv, p.tiles_m, p.tiles_n, p.splits,
                             (const double*)g.A, g.lda, (const double*)g.B, g.ldb, dst, lddst,
                             strideS, g.M, g.N, g.K, p.kchunk, st);
  } else if (p.rem) {
    // (also the fp64 products whose panel cannot take 16-byte direct loads:
    // same tiles, splits and k chunks)
    if constexpr (std::is_same<TI, TO>::value) {
      if (g.trans_a) dispatch_rem<TI, TC, TO, true, kRemMaxWN>(g, p, dst, lddst, strideS, st);
      else dispatch_rem<TI, TC, TO, false, kRemMaxWN>(g, p, dst, lddst, strideS, st);
    }
  } else if (g.trans_a) {
    dispatch_wn<TI, TC, TO, true>(g, p, dst, lddst, strideS, st);
  } else {
    dispatch_wn<TI, TC, TO, false>(g, p, dst, lddst, strideS, st);
  }
  if (g.ev_end) (void)hipEventRecord((hipEvent_t)g.ev_end, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || direct) return e;
  const int gbm = g.gram ? kGramBM : 0;
  if (g.M * g.N <= kReduce4MaxElems && p.splits >= 4)
    hipLaunchKernelGGL((splitk_reduce4_kernel<TO, TO>),
                       dim3((unsigned)((g.M * g.N + 63) / 64)), dim3(256), 0, st,
                       (const TO*)g.partial, g.M, g.N, p.splits, (TO*)g.C, g.ldc, gbm);
  else
    hipLaunchKernelGGL((splitk_reduce_kernel<TO, TO>), splitk_reduce_grid(g.M, g.N),
                       dim3(256), 0, st, (const TO*)g.partial, g.M, g.N, p.splits, (TO*)g.C,
                       g.ldc, gbm, splitk_pairs((const TO*)g.partial, g.M, gbm));
  return hipGetLastError();
}

}  // namespace

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

hipError_t launch_splitk_reduce_f32(const float* P, int64_t M, int64_t N, int S, float* C,
                                    int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL((splitk_reduce_kernel<float, float>), splitk_reduce_grid(M, N), dim3(256), 0,
                     st, P, M, N, S, C, ldc, 0, splitk_pairs(P, M, 0));
  return hipGetLastError();
}

size_t gemm_partial_bytes(int trans_a, int64_t M, int64_t N, int64_t K, Dtype in_t,
                          Dtype out_t, bool gram) {
  const Plan p = make_plan(trans_a, M, N, K, gram, in_t, out_t);
  if (p.splits == 1 && !gram) return 0;
  return (size_t)p.splits * (size_t)M * (size_t)N * (out_t == DT_F64 ? 8 : 4);
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

// Remainder-layout classes of the grouped products: 16 wn + 4 columns.
int grouped_rem_class(int64_t d) {
  for (int c : kRemClasses)
    if (d <= 16 * c + 4) return c;
  return kRemClasses[sizeof(kRemClasses) / sizeof(kRemClasses[0]) - 1];
}

void gemm_rem_grouped_blocks(const GroupGemm& g, int idx, int wn, Dtype dt,
                             std::vector<int4>& out) {
  const int64_t BN = 16 * wn + kRemV;
  const int64_t BMr = 16 * kRemGroupedWavesM * (dt == DT_F64 ? rem_wm<double>() : rem_wm<float>());
  const int64_t tm = (g.M + BMr - 1) / BMr, tn = (g.N + BN - 1) / BN;
  for (int64_t j = 0; j < tn; ++j)
    for (int64_t i = 0; i < tm; ++i) out.push_back(int4{idx, (int)i, (int)j, 0});
}

namespace {
template <typename T, bool TA, int WN>
void run_rem_grouped(const GroupGemm* descs, const int4* bmap, int64_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL((gemm_rem_grouped_kernel<T, T, T, TA, WN>), dim3((unsigned)nblocks),
                     dim3(64 * kRemGroupedWavesM), 0, st, descs, bmap);
}
template <typename T, bool TA>
void rem_grouped_wn(int wn, const GroupGemm* descs, const int4* bmap, int64_t nblocks,
                    hipStream_t st) {
  switch (wn) {
    case 2: run_rem_grouped<T, TA, 2>(descs, bmap, nblocks, st); break;
    case 3: run_rem_grouped<T, TA, 3>(descs, bmap, nblocks, st); break;
    case 4: run_rem_grouped<T, TA, 4>(descs, bmap, nblocks, st); break;
    case 5: run_rem_grouped<T, TA, 5>(descs, bmap, nblocks, st); break;
    case 6: run_rem_grouped<T, TA, 6>(descs, bmap, nblocks, st); break;
    case 7: run_rem_grouped<T, TA, 7>(descs, bmap, nblocks, st); break;
    case 8: run_rem_grouped<T, TA, 8>(descs, bmap, nblocks, st); break;
    case 9: run_rem_grouped<T, TA, 9>(descs, bmap, nblocks, st); break;
    default: run_rem_grouped<T, TA, 13>(descs, bmap, nblocks, st); break;
  }
}
}  // namespace

hipError_t launch_gemm_rem_grouped(Dtype dt, int trans_a, int wn, const GroupGemm* descs,
                                   const int4* bmap, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (dt == DT_F64) {
    if (trans_a) rem_grouped_wn<double, true>(wn, descs, bmap, nblocks, st);
    else rem_grouped_wn<double, false>(wn, descs, bmap, nblocks, st);
  } else {
    if (trans_a) rem_grouped_wn<float, true>(wn, descs, bmap, nblocks, st);
    else rem_grouped_wn<float, false>(wn, descs, bmap, nblocks, st);
  }
  return hipGetLastError();
}

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

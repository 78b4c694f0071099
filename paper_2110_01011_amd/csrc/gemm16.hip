// Precision form of the products with A: C (fp32) = op(A) X with A and X
// rounded to 16 bits (bf16 or fp16) and fp32 accumulation on the 16x16x32
// MFMA, plus the conversions that produce the 16-bit operands.
#include <algorithm>
#include <utility>

#include "rqlp_internal.h"

namespace rqlp {
namespace {

// Precision form: C (fp32) = sum_k A16(i, k) B16(k, j) with both operands
// 16-bit (bf16 or fp16), fp32 accumulation on the 16x16x32 MFMA.
// A16 is the one-time rounded copy of A (or of A^T) in a packed layout
// (convert16_kernel): for each 16-row block and 64-deep k-tile one 2 KB
// chunk, k-tiles of a block consecutive, and within a chunk element
// (r, k) at 512 ((k % 16) / 8) + 8 (16 (k / 16) + r) + k % 8 -- exactly the
// two 16-byte fragments lane 16 (k / 16) + r loads, so each fragment load
// of a wave is 1 KB contiguous and a block's k-chunk streams through DRAM
// pages in order.  B16 is the rounded panel (convert_panel16_kernel), also
// packed: each 64-deep k-tile as 1 KB blocks in the order the direct loads
// below move them to LDS.  Both are zero-padded along the contraction to a
// multiple of 64 (k16BK), so every tile is whole and the main loop carries
// no bounds checks; rows >= M and columns >= N read a clamped (valid) block
// or a zero slack block of the panel and are never stored.
//
// Workgroup tile (32 WAVES) x (16 WN): the waves are stacked along M, each
// owning 32 rows (two 16-row blocks) and all 16 WN columns.  A rows belong to
// a single wave, so A fragments go from HBM straight into registers (one
// 16-byte load per lane, block and MFMA k-step, two tiles ahead); the panel
// tile, shared by the waves, goes to a ring of three LDS slots by direct
// loads.  Results leave as 16-byte stores.  Within a 64-deep tile,
// MFMA k-step s takes, for lane group g = lane / 16, the tile rows 16 g +
// 8 s + [0, 8): the same permutation of k for both operands, so the sum is
// unchanged.
//
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2); the linear workgroup id is remapped so that each XCD works through a
// contiguous range of (column tile, row tile, split) items with the column
// tile fastest: the workgroups of one row tile then read its rows of A
// together from one L2, and the panel chunk of one split stays in that L2.
//
// Split bf16 product (A2, B2 given): with A = A16 + A2 and X = B16 + B2 split
// into a rounded part and its rounding residual (both bf16), the splits
// come in three segments of seg_splits each, A16 B16, A16 B2 and A2 B16,
// whose partial sums the fixed-order reduction adds: the three-term bf16
// product that approximates the fp32 one (the A2 B2 term is below the
// rounding of the other three).
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
// Waves per workgroup (32 rows each): 8, so that each panel tile read from
// L2 serves 256 rows (one workgroup per CU, two waves per SIMD).
constexpr int waves16(int) { return 8; }
constexpr int bm16(int wn) { return 32 * waves16(wn); }
constexpr int k16MaxWN = 17;  // up to 272 columns per workgroup
constexpr int kXcds = 8;

// Linear workgroup id -> work item such that the ids one XCD receives
// (those congruent to x mod 8) form one contiguous range of work items.
__device__ __forceinline__ int64_t xcd_remap(int64_t L, int64_t T) {
  const int64_t x = L % kXcds, j = L / kXcds;
  const int64_t per = T / kXcds, rem = T % kXcds;
  return (x < rem) ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

// f(std::integral_constant<int, I>{}) for I in the sequence, in order.
template <int... I, typename F>
__device__ __forceinline__ void for_each_index(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}

template <typename T16, int WN>
__global__ __launch_bounds__(64 * waves16(WN), 1) void gemm16_kernel(
    const T16* __restrict__ A, const T16* __restrict__ B, int64_t ldb,
    float* __restrict__ C, int64_t ldc, int64_t strideS, int64_t M, int64_t N, int64_t Kp,
    int64_t kchunk, int tiles_m, int tiles_n, const T16* __restrict__ A2,
    const T16* __restrict__ B2, int seg_splits) {
  constexpr int WM = 2, BK = k16BK;
  constexpr int BN = 16 * WN;
  typedef typename Mfma16<T16>::v8 v8;

  const int64_t T = (int64_t)gridDim.x;
  const int64_t w = xcd_remap(blockIdx.x, T);
  // column tile fastest: the tiles_n workgroups that read the same rows of A
  // run side by side on one XCD, so A comes from HBM about once and the
  // other column tiles find it in that XCD's L2
  const int tile_n = (int)(w % tiles_n);
  const int tile_m = (int)((w / tiles_n) % tiles_m);
  const int split = (int)(w / ((int64_t)tiles_m * tiles_n));
  const int seg = split / seg_splits;  // 0: A B, 1: A B2, 2: A2 B
  if (seg == 2) A = A2;
  if (seg == 1) B = B2;
  const int64_t i0 = (int64_t)tile_m * bm16(WN), j0 = (int64_t)tile_n * BN;
  const int64_t kbeg = (int64_t)(split - seg * seg_splits) * kchunk;
  const int64_t kend = (kbeg + kchunk < Kp) ? kbeg + kchunk : Kp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = lane >> 4, r16 = lane & 15;

  // this lane's fragments of the wave's two A blocks (clamped to the last
  // block holding rows < M); tile t's are 1024 t elements further
  const T16* arow[WM];
#pragma unroll
  for (int a = 0; a < WM; ++a) {
    int64_t rb = (i0 + wave * 32 + a * 16) / 16;
    rb = rb < (M - 1) / 16 ? rb : (M - 1) / 16;
    arow[a] = A + rb * 16 * Kp + 8 * lane;
  }
  // The panel tile goes into LDS by 16-byte direct loads: block q = 2 b + s
  // (column block b, MFMA step s) is 1 KB, where lane (g, r) of a wave finds
  // at position 8 lane the fragment it multiplies -- tile rows 16 g + 8 s
  // .. + 7 of column 16 b + r, 16 contiguous bytes of the column-major
  // panel, fetched by the same lane of the loading wave.  Fragment reads
  // are 1 KB contiguous per wave (no bank conflicts) and no staging
  // registers or LDS stores are needed.  Every wave issues the same number
  // of direct loads (NQW); the blocks past 2 WN land in a pad.
  constexpr int NW = waves16(WN), NQ = 2 * WN, NQW = (NQ + NW - 1) / NW;
  constexpr int BLK = 512;  // 16-bit elements per 1 KB block
  __shared__ __attribute__((aligned(16))) T16 Bs0[NQW * NW * BLK];
  __shared__ __attribute__((aligned(16))) T16 Bs1[NQW * NW * BLK];
  __shared__ __attribute__((aligned(16))) T16 Bs2[NQW * NW * BLK];
  // Wave w loads blocks q = w + NW u: column block q / 2 = NW u / 2 + w / 2,
  // step q % 2 = w % 2 (NW is even).  Each block has a buffer resource whose
  // base is that wave-uniform part of the address; the lane adds its column
  // 16 bytes at position 16 lane (voffset), the tile its k-tile (soffset):
  // the panel is packed (convert_panel16_kernel), so each direct load moves
  // one contiguous 1 KB block.  The buffer form of the direct load is
  // counted on vmcnt alone, so the fragment reads below wait for their own
  // LDS reads only (the global form, being FLAT-encoded, is also counted on
  // lgkmcnt and makes the compiler wait for every outstanding LDS read
  // before each fragment is used).  Offsets are 32-bit: the launcher
  // bounds the panel's size.  Blocks past N (the ragged last tile and the
  // pad blocks) are read from the panel's slack blocks (kGemm16PanelSlack
  // columns, zeros) and never stored: the last one read is at most
  // N / 16 + NQW NW / 2 - 1.
  static_assert(NW % 2 == 0, "waves per workgroup must be even");
  static_assert(16 * (NQW * NW / 2) <= kGemm16PanelSlack, "panel slack too small");
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int64_t nb = (N + 15) / 16 + kGemm16PanelSlack / 16;  // column blocks of the panel
  const int64_t pbytes = ldb / BK * nb * 2048;                // the whole panel
  const T16* qbase[NQW];
  int qbytes[NQW];
#pragma unroll
  for (int u = 0; u < NQW; ++u) {
    const int64_t blk = (j0 / 16 + NW / 2 * u + (wv >> 1)) * 2 + (wv & 1);
    qbase[u] = B + blk * 512;
    qbytes[u] = (int)std::min<int64_t>(pbytes - blk * 1024, 0x7fffffff);
  }
  const int voff = 16 * lane;

  float4_t acc[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) acc[a][b] = float4_t{0, 0, 0, 0};

  // Three tiles in flight: A fragments in a ring of registers, panel tiles
  // in a ring of LDS buffers; tile t + 2 loads while tile t is multiplied.
  v8 ra0[WM][2], ra1[WM][2], ra2[WM][2];
  auto load = [&](int64_t t, v8 (&dst)[WM][2], T16* bs) {
    const int64_t k0 = kbeg + t * BK;
#pragma unroll
    for (int u = 0; u < NQW; ++u)
      buffer_load_lds16(qbase[u], qbytes[u], voff, (int)(k0 / BK * nb * 2048),
                        bs + (u * NW + wave) * BLK);
#pragma unroll
    for (int a = 0; a < WM; ++a) {
      dst[a][0] = *(const v8*)(arow[a] + 16 * k0);
      dst[a][1] = *(const v8*)(arow[a] + 16 * k0 + 512);
    }
  };
  // 2 WN fragment reads per tile, each feeding WM MFMAs, in groups of G:
  // the reads of group g + 1 are issued before the MFMAs of group g (two
  // register sets, a scheduling fence between groups), so LDS latency
  // overlaps the MFMAs; read one at a time before its MFMAs, each fragment
  // was waited on and the matrix cores idled.
  constexpr int G = 4, NF = 2 * WN, NG = (NF + G - 1) / G;
  auto frag = [&](const T16* bs, int i) {
    const int b = i % WN, sb = i / WN;
    return *(const v8*)(bs + (2 * b + sb) * BLK + 8 * lane);
  };
  // One of the NL = NQW + 2 WM loads of a tile (direct loads first).  In the
  // loop they are issued among the MFMAs of the tile two steps earlier, a
  // few per fragment group: a wave issues in order, and the loads issued
  // as one burst ahead of the tile held back its MFMAs while the memory
  // pipeline took them (7% of the time at 20000 x 16000, d = 520).
  auto load_part = [&](int64_t t, v8 (&dst)[WM][2], T16* bs, int i) {
    const int64_t k0 = kbeg + t * BK;
    if (i < NQW) {
      buffer_load_lds16(qbase[i], qbytes[i], voff, (int)(k0 / BK * nb * 2048),
                        bs + (i * NW + wave) * BLK);
    } else {
      const int a = (i - NQW) >> 1, hf = (i - NQW) & 1;
      dst[a][hf] = *(const v8*)(arow[a] + 16 * k0 + 512 * hf);
    }
  };
  constexpr int NL = NQW + 2 * WM;
  auto compute = [&](const v8 (&ra)[WM][2], const T16* bs, auto&& ld) {
    v8 bf[2][G];
#pragma unroll
    for (int u = 0; u < G; ++u)
      if (u < NF) bf[0][u] = frag(bs, u);
    auto group = [&](auto gic) {
      constexpr int gi = decltype(gic)::value;
      constexpr int nr = std::min(G, std::max(0, NF - (gi + 1) * G));  // reads of group gi + 1
      constexpr int nm = WM * std::min(G, NF - gi * G);                // MFMAs of group gi
      constexpr int l0 = gi * NL / NG, l1 = (gi + 1) * NL / NG;        // loads of tile t + 2
      constexpr int nl = l1 - l0, per = nm / (nl + 1);
#pragma unroll
      for (int u = 0; u < nr; ++u) bf[(gi + 1) & 1][u] = frag(bs, (gi + 1) * G + u);
#pragma unroll
      for (int u = l0; u < l1; ++u) ld(u);
#pragma unroll
      for (int u = 0; u < nm / WM; ++u) {
        const int i = gi * G + u;
        const int b = i % WN, sb = i / WN;
#pragma unroll
        for (int a = 0; a < WM; ++a)
          acc[a][b] = Mfma16<T16>::mma(ra[a][sb], bf[gi & 1][u], acc[a][b]);
      }
      // this group's fragments stay live to the end of the group, so the
      // next group's reads cannot take their registers (and wait for them)
#pragma unroll
      for (int u = 0; u < nm / WM; ++u) asm volatile("" ::"v"(bf[gi & 1][u]));
      if constexpr (nr > 0) __builtin_amdgcn_sched_group_barrier(0x100, nr, 0);
#pragma unroll
      for (int u = 0; u < nl; ++u) {
        if constexpr (per > 0) __builtin_amdgcn_sched_group_barrier(0x008, per > 0 ? per : 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
      }
      if constexpr (nm - nl * per > 0)
        __builtin_amdgcn_sched_group_barrier(0x008, nm - nl * per > 0 ? nm - nl * per : 1, 0);
      __builtin_amdgcn_sched_barrier(0);
    };
    __builtin_amdgcn_sched_barrier(0);
    for_each_index(std::make_integer_sequence<int, NG>{}, group);
  };
  // The loads of one tile per wave: NQW direct loads + 2 WM fragment loads.
  // Waiting until at most that many are outstanding completes the tile
  // before them (loads return in order), and the barrier then hands it to
  // all waves.  __syncthreads() would wait for every load (its fence
  // implies vmcnt(0)), tile t + 2's included.  The wait is the builtin, so
  // the compiler knows which loads it covers (no conservative wait before
  // the next tile's LDS reads); the empty asm statements with a memory
  // clobber keep memory accesses from moving across the barrier.  The
  // buffer a tile's direct loads overwrite was read for tile t - 1, before
  // the previous barrier.
  constexpr int L = NQW + 2 * WM;
  static_assert(L < 64, "vmcnt range");
  constexpr int wait_imm = (L & 15) | ((L >> 4) << 14) | (7 << 4) | (15 << 8);
  auto sync_tile = [&]() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(wait_imm);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  };

  const int64_t nk = (kend - kbeg) / BK;  // whole tiles (kbeg, kend multiples of BK)
  if (nk > 0) {
    // loads past the last tile re-read it (unused), so every step issues
    // the same loads
    auto tc = [&](int64_t t) { return t < nk ? t : nk - 1; };
    load(0, ra0, Bs0);
    load(tc(1), ra1, Bs1);
    sync_tile();
    int64_t t = 0;
    for (; t + 2 < nk; t += 3) {
      compute(ra0, Bs0, [&](int i) { load_part(tc(t + 2), ra2, Bs2, i); });
      sync_tile();
      compute(ra1, Bs1, [&](int i) { load_part(tc(t + 3), ra0, Bs0, i); });
      sync_tile();
      compute(ra2, Bs2, [&](int i) { load_part(tc(t + 4), ra1, Bs1, i); });
      sync_tile();
    }
    // 1 or 2 tiles left: the last one's loads may still be in flight (the
    // waits above leave one tile outstanding), so wait for all of them and
    // hand both tiles to every wave
    if (t < nk) {
      __syncthreads();
      compute(ra0, Bs0, [](int) {});
      if (t + 1 < nk) compute(ra1, Bs1, [](int) {});
    }
  }
  // Lane (g, r) holds rows 4 g .. 4 g + 3 of column r of each block: one
  // 16-byte store where C's address and ldc allow it and the four rows
  // exist; the two blocks of a column are stored back to back (one 128-byte
  // line when aligned).
  float* Cs = C + (int64_t)split * strideS;
  const bool vec = ((((uintptr_t)Cs) & 15) == 0) && ((ldc & 3) == 0);
#pragma unroll
  for (int b = 0; b < WN; ++b) {
    const int64_t col = j0 + b * 16 + r16;
#pragma unroll
    for (int a = 0; a < WM; ++a) {
      const int64_t row0 = i0 + wave * 32 + a * 16 + acc_row_f32(lane, 0);
      if (col >= N) continue;
      if (vec && row0 + 3 < M) {
        *(float4_t*)(Cs + row0 + col * ldc) = acc[a][b];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row0 + r < M) Cs[row0 + r + col * ldc] = acc[a][b][r];
      }
    }
  }
}

// X (rows x d fp32, ldx) -> X16, rounded to nearest even, in the packed
// panel layout gemm16_kernel loads: for each 64-deep k-tile kt, column
// block b (of nb = panel16_blocks(d)) and MFMA step s, 512 consecutive
// elements with lane L = 16 g + r's fragment (k = 64 kt + 16 g + 8 s ..
// + 7 of column 16 b + r) at 8 L -- the 1 KB a wave's direct load moves to
// LDS in one piece.  k past rows (up to kp, a multiple of 64) and columns
// past d (the slack blocks) are zeros.  If Ylo is given it receives the
// rounded residual x - x16 (exact in fp32) the same way.  One thread per
// lane position of both steps: 16 consecutive k of one column read (64
// contiguous bytes, as four 16-byte loads where X's alignment allows),
// two 16-byte pieces written.
template <typename T16>
__global__ __launch_bounds__(256) void convert_panel16_kernel(const float* __restrict__ X,
                                                              int64_t rows, int64_t d,
                                                              int64_t ldx, T16* __restrict__ Y,
                                                              int64_t kp, int64_t nb,
                                                              T16* __restrict__ Ylo) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  typedef T16 t16x8 __attribute__((ext_vector_type(8)));
  const bool vec = ((((uintptr_t)X) & 15) == 0) && ((ldx & 3) == 0);
  const int64_t units = kp / k16BK * nb * 64;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int L = (int)(u & 63);
    const int64_t rest = u >> 6, b = rest % nb, kt = rest / nb;
    const int64_t k0 = kt * k16BK + 16 * (L >> 4), col = 16 * b + (L & 15);
    float x[16];
    if (col < d && vec && k0 + 15 < rows) {
      const float4* src = (const float4*)(X + k0 + col * ldx);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = src[q];
        x[4 * q] = v.x;
        x[4 * q + 1] = v.y;
        x[4 * q + 2] = v.z;
        x[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) x[e] = (col < d && k0 + e < rows) ? X[k0 + e + col * ldx] : 0.0f;
    }
    const int64_t o = (kt * nb + b) * 1024 + 8 * L;  // step 0; step 1 at + 512
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      t16x8 hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        hi[e] = to16(x[8 * st + e], (T16*)nullptr);
        lo[e] = to16(x[8 * st + e] - (float)hi[e], (T16*)nullptr);
      }
      *(u32x4*)(Y + o + 512 * st) = __builtin_bit_cast(u32x4, hi);
      if (Ylo) *(u32x4*)(Ylo + o + 512 * st) = __builtin_bit_cast(u32x4, lo);
    }
  }
}

// A (m x n fp32, lda) -> A16 and At16, A and A^T rounded to 16 bits (nearest
// even) in the packed operand layout of gemm16_kernel: A16's rows are A's n
// columns with contraction k = A's row (length k16 = m rounded up to 64),
// At16's rows are A's m rows with k = A's column (kt16 = n rounded up).
// Each copy covers its rows rounded up to 64; padding rows and padding k
// are zeros.  One workgroup takes a 64 x 64 tile of A: read once (8-byte
// pairs when A's address and lda allow, each thread a 2 x 2 block), rounded
// into LDS in both orientations, then stored as four whole 2 KB chunks of
// each copy.
// If rerr is given, each workgroup also writes the sum of squared rounding
// errors (a - a16)^2 of its tile (fp64) to rerr[its linear index] and the
// tile's sum of squares a^2 to rerr[nblocks + its linear index].  A16lo /
// At16lo, if given, receive the rounded residual a - a16 (exact in fp32) in
// the layout of A16 / At16.
// Power-of-two exponent s with max|a| 2^s in [2^13, 2^14): the fp16 copy's
// scale (finite values up to 65504, normal ones from 2^-14), so that the
// largest entry sits well inside the range whatever ||A|| is.  0 for a zero
// or non-finite maximum.
__device__ __forceinline__ int f16_scale_exponent(unsigned amax_bits) {
  const float mx = __uint_as_float(amax_bits);
  if (!(mx > 0.0f) || !(mx <= 3.0e38f)) return 0;
  int e = 0;
  (void)frexpf(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  return min(max(14 - e, -100), 100);
}

// amax_bits = bit pattern of max |a| over A (m x n, lda); non-negative floats
// order like their bit patterns, so an unsigned atomic max does.  *amax_bits
// must start at zero.
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ A, int64_t m,
                                                     int64_t n, int64_t lda,
                                                     unsigned* __restrict__ amax_bits) {
  __shared__ unsigned red[256];
  unsigned mx = 0u;
  const int64_t total = m * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % m, j = idx / m;
    mx = max(mx, __float_as_uint(A[i + j * lda]) & 0x7fffffffu);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(amax_bits, red[0]);
}

// C (rows x d, ldc) *= 2^-s with s = *scale_exp (undoes the fp16 copy's scale).
__global__ __launch_bounds__(256) void unscale_kernel(float* __restrict__ C, int64_t rows,
                                                      int64_t d, int64_t ldc,
                                                      const int* __restrict__ scale_exp) {
  const float f = ldexpf(1.0f, -*scale_exp);
  const int64_t total = rows * d;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % rows, j = idx / rows;
    C[i + j * ldc] *= f;
  }
}

template <typename T16>
__global__ __launch_bounds__(256) void convert16_kernel(const float* __restrict__ A, int64_t m,
                                                        int64_t n, int64_t lda,
                                                        T16* __restrict__ A16, int64_t k16,
                                                        T16* __restrict__ At16, int64_t kt16,
                                                        double* __restrict__ rerr,
                                                        T16* __restrict__ A16lo,
                                                        T16* __restrict__ At16lo,
                                                        const unsigned* __restrict__ amax_bits,
                                                        int* __restrict__ scale_out) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  typedef T16 pair_t __attribute__((ext_vector_type(2)));
  // The rounded tile twice, [j][i] for A16 and [i][j] for At16, in 4-byte
  // pairs; the residuals go through the same arrays in a second round (the
  // LDS footprint allows eight workgroups per CU).  Rows are 35 words
  // apart: thread tx's pair writes to rows 2 tx (+1) of the [i][j] copy
  // then fall in distinct banks (35 is odd).
  constexpr int LD = 70;
  __shared__ __attribute__((aligned(16))) T16 tj[64][LD];
  __shared__ __attribute__((aligned(16))) T16 ti[64][LD];
  __shared__ double red[256];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const bool pairs = ((((uintptr_t)A) & 7) == 0) && ((lda & 1) == 0);
  // the copy holds 2^s a (exact: a power of two); errors are taken unscaled
  const int sexp = amax_bits ? f16_scale_exponent(*amax_bits) : 0;
  const float sc = ldexpf(1.0f, sexp), inv = ldexpf(1.0f, -sexp);
  if (scale_out && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *scale_out = sexp;
  double err = 0.0, nrm = 0.0;
  // thread (tx, ty): rows 2 tx, 2 tx + 1 and column pairs ty + 8 r of the
  // tile, r = 0..3; v / vl [r][column][row]
  T16 v[4][2][2], vl[4][2][2];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int jp = ty + 8 * r;
    const int64_t i = i0 + 2 * tx;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int64_t j = j0 + 2 * jp + c;
      float a[2] = {0.0f, 0.0f};
      if (j < n) {
        const float* src = A + i + j * lda;
        if (pairs && i + 1 < m) {
          const float2 t = *(const float2*)src;
          a[0] = t.x;
          a[1] = t.y;
        } else {
          if (i < m) a[0] = src[0];
          if (i + 1 < m) a[1] = src[1];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float as = a[u] * sc;
        v[r][c][u] = to16(as, (T16*)nullptr);
        vl[r][c][u] = to16(as - (float)v[r][c][u], (T16*)nullptr);
        const double e = (double)a[u] - (double)((float)v[r][c][u] * inv);
        err += e * e;
        nrm += (double)a[u] * (double)a[u];
      }
    }
  }
  auto stage = [&](const T16 (&x)[4][2][2]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jp = ty + 8 * r;
#pragma unroll
      for (int c = 0; c < 2; ++c) *(pair_t*)&tj[2 * jp + c][2 * tx] = pair_t{x[r][c][0], x[r][c][1]};
#pragma unroll
      for (int u = 0; u < 2; ++u) *(pair_t*)&ti[2 * tx + u][2 * jp] = pair_t{x[r][0][u], x[r][1][u]};
    }
  };
  // Packed stores: the 64 x 64 tile is, in both copies, one 64-deep k-tile
  // of four 16-row blocks, i.e. four whole 2 KB chunks; unit u = (block,
  // half, lane) is 16 bytes, 8 consecutive k of one row (four LDS words).
  // A16's rows are A's columns (k = i), At16's are A's rows (k = j).
  // Elements outside A are zeros in the tiles.
  const int64_t nk = k16 / k16BK, nkt = kt16 / k16BK;
  auto row8 = [](const T16* p) {
    const unsigned* w = (const unsigned*)p;
    return u32x4{w[0], w[1], w[2], w[3]};
  };
  auto store = [&](T16* Y, T16* Yt) {
    for (int u = threadIdx.x; u < 512; u += 256) {
      const int blk = u >> 7, h = (u >> 6) & 1, ln = u & 63;
      const int rr = 16 * blk + (ln & 15), kk = 16 * (ln >> 4) + 8 * h;
      const int64_t oa = (((j0 / 16 + blk) * nk + i0 / k16BK) * 2 + h) * 512 + 8 * ln;
      const int64_t ot = (((i0 / 16 + blk) * nkt + j0 / k16BK) * 2 + h) * 512 + 8 * ln;
      if (Y) *(u32x4*)(Y + oa) = row8(&tj[rr][kk]);
      if (Yt) *(u32x4*)(Yt + ot) = row8(&ti[rr][kk]);
    }
  };
  stage(v);
  __syncthreads();
  store(A16, At16);
  if (A16lo || At16lo) {
    __syncthreads();
    stage(vl);
    __syncthreads();
    store(A16lo, At16lo);
  }
  if (rerr) {
    const int64_t nb = (int64_t)gridDim.x * gridDim.y;
    const int64_t bid = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    for (int pass = 0; pass < 2; ++pass) {
      red[threadIdx.x] = pass == 0 ? err : nrm;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) rerr[bid + pass * nb] = red[0];
      __syncthreads();
    }
  }
}

}  // namespace

// Precision-form plan: bm16(wn)-row tiles, N covered by as few tiles of at most
// 16 k16MaxWN columns as possible (A is read once per N tile), split-K up to
// ~1024 workgroups with at least four whole tiles per split.  Kp is the
// padded contraction length (a multiple of k16BK).  nseg = 3 plans the split
// bf16 product: splits is then per segment.
struct Plan16 {
  int wn;
  int64_t tiles_m, tiles_n;
  int splits;
  int64_t kchunk;
};

int64_t pad16(int64_t K) { return (K + k16BK - 1) / k16BK * k16BK; }

template <typename T16, int WN>
int gemm16_occupancy() {
  static const int nb = occupancy_of(gemm16_kernel<T16, WN>, 64 * waves16(WN));
  return nb;
}

template <typename T16, int WN>
int gemm16_occupancy_wn(int wn) {
  if constexpr (WN > 1) {
    if (wn < WN) return gemm16_occupancy_wn<T16, WN - 1>(wn);
  }
  return gemm16_occupancy<T16, WN>();
}

Plan16 make_plan16(int64_t M, int64_t N, int64_t K, bool f16, int nseg) {
  Plan16 p;
  const int64_t Kp = pad16(K);
  const int64_t nblk = (N + 15) / 16;
  p.tiles_n = (nblk + k16MaxWN - 1) / k16MaxWN;
  p.wn = (int)((nblk + p.tiles_n - 1) / p.tiles_n);
  p.tiles_m = (M + bm16(p.wn) - 1) / bm16(p.wn);
  const int64_t tiles = p.tiles_m * p.tiles_n;
  const int64_t max_s = std::max<int64_t>(1, Kp / (4 * k16BK));
  const int occ = f16 ? gemm16_occupancy_wn<_Float16, k16MaxWN>(p.wn)
                      : gemm16_occupancy_wn<__bf16, k16MaxWN>(p.wn);
  choose_splits(tiles * nseg, Kp, k16BK, max_s, (int64_t)occ * cu_count(), 2.0 * bm16(p.wn) * 16 * p.wn,
                900e12, 4.0 * (double)M * (double)N, &p.kchunk, &p.splits);
  return p;
}

template <typename T16, int WN>
static void run_gemm16(const Gemm16Args& g, const Plan16& p, int nseg, float* dst,
                       int64_t lddst, int64_t strideS, hipStream_t st) {
  const unsigned T = (unsigned)(p.tiles_m * p.tiles_n * p.splits * nseg);
  hipLaunchKernelGGL((gemm16_kernel<T16, WN>), dim3(T), dim3(64 * waves16(WN)), 0, st,
                     (const T16*)g.A, (const T16*)g.B, g.ldb, dst, lddst, strideS, g.M,
                     g.N, pad16(g.K), p.kchunk, (int)p.tiles_m, (int)p.tiles_n,
                     (const T16*)g.A2, (const T16*)g.B2, p.splits);
}

template <typename T16, int WN>
static void dispatch16(const Gemm16Args& g, const Plan16& p, int nseg, float* dst,
                       int64_t lddst, int64_t strideS, hipStream_t st) {
  if constexpr (WN > 1) {
    if (p.wn < WN) return dispatch16<T16, WN - 1>(g, p, nseg, dst, lddst, strideS, st);
  }
  run_gemm16<T16, WN>(g, p, nseg, dst, lddst, strideS, st);
}

template <typename T16>
static hipError_t gemm16_typed(const Gemm16Args& g, hipStream_t st) {
  const int nseg = g.A2 ? 3 : 1;
  const Plan16 p = make_plan16(g.M, g.N, g.K, g.f16, nseg);
  const int slabs = p.splits * nseg;
  const bool direct = (slabs == 1);
  float* dst = direct ? g.C : (float*)g.partial;
  const int64_t lddst = direct ? g.ldc : g.M;
  const int64_t strideS = g.M * g.N;
  if (!direct && (g.partial == nullptr ||
                  g.partial_bytes < (size_t)slabs * (size_t)strideS * sizeof(float)))
    return hipErrorInvalidValue;
  // whole 16-byte fragment loads over the zero-padded contraction (A and
  // the panel packed, contractions padded to the tile depth); the residual
  // copies share the layouts of A and B; the panel's buffer offsets fit in
  // 31 bits
  if (g.lda != pad16(g.K) || g.ldb < pad16(g.K) || (g.ldb % k16BK) != 0 ||
      (int64_t)gemm16_panel_bytes(g.ldb, g.N) >= ((int64_t)1 << 31) ||
      (((uintptr_t)g.A | (uintptr_t)g.B | (uintptr_t)g.A2 | (uintptr_t)g.B2) & 15) != 0 ||
      ((g.A2 == nullptr) != (g.B2 == nullptr)) || (g.A2 && g.f16))
    return hipErrorInvalidValue;
  if (g.ev_begin) (void)hipEventRecord((hipEvent_t)g.ev_begin, st);
  dispatch16<T16, k16MaxWN>(g, p, nseg, dst, lddst, strideS, st);
  if (g.ev_end) (void)hipEventRecord((hipEvent_t)g.ev_end, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || direct) return e;
  return launch_splitk_reduce_f32((const float*)g.partial, g.M, g.N, slabs, g.C, g.ldc, st);
}

hipError_t launch_gemm16(const Gemm16Args& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  return g.f16 ? gemm16_typed<_Float16>(g, st) : gemm16_typed<__bf16>(g, st);
}

size_t gemm16_partial_bytes(int64_t M, int64_t N, int64_t K, bool f16, int nseg) {
  const Plan16 p = make_plan16(M, N, K, f16, nseg);
  const int slabs = p.splits * nseg;
  return slabs == 1 ? 0 : (size_t)slabs * (size_t)M * (size_t)N * 4;
}

int64_t gemm16_ld(int64_t K) { return pad16(K); }

size_t gemm16_packed_bytes(int64_t rows, int64_t K) {
  return (size_t)((rows + k16BK - 1) / k16BK * k16BK) * (size_t)pad16(K) * 2;
}

int64_t panel16_blocks(int64_t d) { return (d + 15) / 16 + kGemm16PanelSlack / 16; }

size_t gemm16_panel_bytes(int64_t K, int64_t d) {
  return (size_t)(pad16(K) / k16BK) * (size_t)panel16_blocks(d) * 1024 * 2;
}

hipError_t launch_convert_panel16(const float* X, int64_t rows, int64_t d, int64_t ldx, void* Y,
                                  int64_t ldy, bool f16, hipStream_t st, void* Ylo) {
  if (rows <= 0 || d <= 0) return hipSuccess;
  if (ldy < pad16(rows) || ldy % k16BK != 0 ||
      ((((uintptr_t)Y) | ((uintptr_t)Ylo)) & 15) != 0)
    return hipErrorInvalidValue;
  const int64_t nb = panel16_blocks(d);
  const int64_t units = ldy / k16BK * nb * 64;
  const unsigned blocks = (unsigned)std::min<int64_t>((units + 255) / 256, 8192);
  if (f16)
    hipLaunchKernelGGL(convert_panel16_kernel<_Float16>, dim3(blocks), dim3(256), 0, st, X, rows,
                       d, ldx, (_Float16*)Y, ldy, nb, (_Float16*)Ylo);
  else
    hipLaunchKernelGGL(convert_panel16_kernel<__bf16>, dim3(blocks), dim3(256), 0, st, X, rows, d,
                       ldx, (__bf16*)Y, ldy, nb, (__bf16*)Ylo);
  return hipGetLastError();
}

int64_t convert16_blocks(int64_t m, int64_t n) { return ((m + 63) / 64) * ((n + 63) / 64); }

hipError_t launch_convert16(const float* A, int64_t m, int64_t n, int64_t lda, void* A16,
                            int64_t ld16, void* At16, int64_t ldt16, bool f16, hipStream_t st,
                            double* rerr, void* A16lo, void* At16lo, unsigned* amax,
                            int* scale_out) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (f16 && amax) {  // the fp16 copy is scaled by a power of two from max |a|
    hipError_t e = launch_zero_ints((int*)amax, 1, st);
    if (e != hipSuccess) return e;
    const int64_t tot = m * n;
    const unsigned nb = (unsigned)std::min<int64_t>(2048, std::max<int64_t>(1, (tot + 255) / 256));
    hipLaunchKernelGGL(absmax_kernel, dim3(nb), dim3(256), 0, st, A, m, n, lda, amax);
  } else {
    amax = nullptr;
    scale_out = nullptr;
  }
  // packed copies: contraction lengths padded to the tile depth, 16-byte
  // aligned chunks
  if (ld16 != pad16(m) || ldt16 != pad16(n) ||
      (((uintptr_t)A16 | (uintptr_t)At16 | (uintptr_t)A16lo | (uintptr_t)At16lo) & 15))
    return hipErrorInvalidValue;
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  if (f16)
    hipLaunchKernelGGL(convert16_kernel<_Float16>, grid, dim3(256), 0, st, A, m, n, lda,
                       (_Float16*)A16, ld16, (_Float16*)At16, ldt16, rerr, (_Float16*)A16lo,
                       (_Float16*)At16lo, (const unsigned*)amax, scale_out);
  else
    hipLaunchKernelGGL(convert16_kernel<__bf16>, grid, dim3(256), 0, st, A, m, n, lda,
                       (__bf16*)A16, ld16, (__bf16*)At16, ldt16, rerr, (__bf16*)A16lo,
                       (__bf16*)At16lo, (const unsigned*)nullptr, (int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_unscale(float* C, int64_t rows, int64_t d, int64_t ldc, const int* scale_exp,
                          hipStream_t st) {
  if (rows <= 0 || d <= 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<int64_t>(2048, (rows * d + 255) / 256);
  hipLaunchKernelGGL(unscale_kernel, dim3(nb), dim3(256), 0, st, C, rows, d, ldc, scale_exp);
  return hipGetLastError();
}

}  // namespace rqlp

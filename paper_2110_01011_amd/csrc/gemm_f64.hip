// fp64 products with A of Algorithm 1 (the sketch A^T Omega, the power
// products A Qbar and A^T Q, the projection A^T Q) for the skinny case: a
// d-column panel, d up to 16 kStrMaxWN + 4, and a long contraction split
// into kchunk slabs whose partial outputs the caller reduces in a fixed
// order.  The launcher in gemm.hip plans tiles and splits and falls back to
// its LDS-staged kernel when the panel cannot take 16-byte direct loads.
#include "rqlp_internal.h"

namespace rqlp {
namespace {

__device__ __forceinline__ double buffer_load_f64(const void* base, int nbytes, int voff, int soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nbytes, 0x00020000),
      voff, soff, 0);
  return __builtin_bit_cast(double, v);
}

// The tile of the LDS-staged kernel (8 waves x 16 rows, WN MFMA column
// blocks + vector-ALU columns) with its operands moved differently.  Each
// wave loads its A fragments from memory straight into registers, and the
// panel B is copied into LDS by the direct global-to-LDS loads (no staging
// registers, no LDS stores).  The freed registers and LDS buy 32-deep
// k-tiles, one barrier per 32 k, and loads of tile t + 1 (A and B) issued
// while tile t is multiplied: the LDS-staged form, with one 8- or 16-deep
// tile in flight, left the matrix cores idle a third of the time waiting
// on its loads.  In the steady state the loads go out one after each MFMA
// of the tile's first two steps (the A fragments by buffer loads, the panel
// blocks by direct loads at fixed offsets): a wave issues in order, and its
// 15 loads issued as one burst ahead of the tile held back its MFMAs while
// the memory pipeline took them (the kernel ran 12% longer that way).
//
// Lane (r, g) holds row r of the wave's 16 rows and k = 8 h + 2 g + e at
// MFMA step 2 h + e (h = 0..3 in a tile).  LDS layout of a B tile: for
// column block b and k-octet h, 128 consecutive doubles hold k = 8 h + 2 p
// + e of column 16 b + r at position 2 (16 p + r) + e -- exactly what one
// 16-byte direct load per lane writes (lane 16 p + r fetches the pair k,
// k + 1 of its column) -- and one 16-byte LDS read per lane returns the
// fragments of both steps 2 h and 2 h + 1, a wave reading 1 KB contiguous
// (no bank conflicts).  The vector-ALU columns take one more 128-double
// block (pair p of column c at 8 p + 2 c + e); RV of its 4 columns are
// computed (2 when the tile is at most 16 WN + 2 wide, e.g. d = 210).
// Direct loads need B 16-byte aligned with an even ldb below 2^20 (the
// launcher checks; buffer offsets are 32-bit); a k-tile that ends past the
// split (the last one when K is not a multiple of 32) is staged through
// registers instead, with zeros past the end.  Rows past M and columns past N read clamped in-bounds data whose
// results are never stored.
constexpr int kStrWaves = 8;

// Linear workgroup id L of T -> work item (split-major, S splits of T / S
// items), such that the ids one of the 8 XCDs receives (those congruent mod
// 8) map to one contiguous range.  When S divides 8, XCD x takes items of
// split x % S only (the XCDs x = s, s + S, ... share split s in turn; their
// counts add up to T / S exactly), so each XCD's L2 holds one panel slab.
__device__ __forceinline__ uint32_t xcd_item(uint32_t L, uint32_t T, uint32_t S) {
  const uint32_t x = L % 8, j = L / 8, per = T / 8, rem = T % 8;
  if (8 % S == 0) {
    const uint32_t s = x % S;
    uint32_t off = 0;
    for (uint32_t y = s; y < x; y += S) off += per + (y < rem ? 1u : 0u);
    return s * (T / S) + off + j;
  }
  return (x < rem) ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}
template <int WN>
constexpr int str_tile_doubles() { return (4 * WN + 1) * 128; }

template <bool TA, int WN, int RV>
__global__ __launch_bounds__(64 * kStrWaves) void gemm_stream_f64_kernel(
    const double* __restrict__ A, int64_t lda, const double* __restrict__ B, int64_t ldb,
    double* __restrict__ C, int64_t ldc, int64_t strideS, int64_t M, int64_t N, int64_t K,
    int64_t kchunk) {
  constexpr int BK = kStrBK, NW = kStrWaves, BM = 16 * NW, BN = 16 * WN + RV;
  constexpr int NQ = 4 * WN + 1;  // 128-double blocks per B tile
  // two buffers as separate objects, so the compiler can tell the direct
  // loads into one from the reads of the other
  __shared__ __align__(16) double Bs0[str_tile_doubles<WN>()];
  __shared__ __align__(16) double Bs1[str_tile_doubles<WN>()];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  // The dispatcher hands workgroups to the 8 XCDs in turn by linear id, and
  // each XCD has its own L2.  The work item of linear id L is renumbered so
  // that the ids one XCD receives form one contiguous run of (column tile,
  // row tile, split) items, column tile fastest: the workgroups of one XCD
  // then need one split's slab of the panel (one or two when the split
  // count does not divide 8), not all of it, and read each row block of A
  // side by side.
  // (uniform values: kept in scalar registers for the buffer offsets)
  const uint32_t nx = gridDim.x, ny = gridDim.y, T = nx * ny * gridDim.z;
  const uint32_t w = xcd_item(blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z), T, gridDim.z);
  const int64_t tile_n = __builtin_amdgcn_readfirstlane(w % ny);
  const int64_t tile_m = __builtin_amdgcn_readfirstlane((w / ny) % nx);
  const int64_t split = __builtin_amdgcn_readfirstlane(w / (nx * ny));
  const int64_t i0 = tile_m * BM, j0 = tile_n * BN;
  const int64_t kbeg = split * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  const int64_t nt = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;

  double4_t acc[WN];
#pragma unroll
  for (int b = 0; b < WN; ++b) acc[b] = double4_t{0, 0, 0, 0};
  double vacc[RV];
#pragma unroll
  for (int c = 0; c < RV; ++c) vacc[c] = 0.0;
  double ra0[BK / 4], ra1[BK / 4];

  // Per-lane address terms: the lane's row of op(A) and its panel column in
  // each of the wave's blocks are fixed for the whole loop, so a full tile
  // costs one address add per load (the uniform tile offset) and no
  // multiplications.  `fresh` passes a lane id through an empty asm
  // statement where a term should be recomputed per tile instead of held.
  auto fresh = [](int v) {
    asm volatile("" : "+v"(v));
    return v;
  };
  // the same for a uniform offset, so that `base + offset` is not split
  // into a loop-invariant per-lane pointer per load
  auto opaque = [](int64_t v) {
    asm volatile("" : "+s"(v));
    return v;
  };
  const int64_t arow = (i0 + wave * 16 + r16 < M) ? i0 + wave * 16 + r16 : M - 1;
  // Direct loads of the panel use buffer addressing from the tile's first
  // column: a uniform base and extent, a per-lane 32-bit byte offset fixed
  // for the loop, and the tile's uniform k offset (the launcher bounds ldb
  // so that the offsets fit).  Block q = wave + 8 i of the wave: column
  // 16 (wave / 4) + 32 i + r of the tile, k offset 8 (wave % 4) + 2 g.
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const double* const bt = B + j0 * ldb;
  const int bt_bytes = (int)min(((N - 1 - j0) * ldb + K) * 8, (int64_t)0x7fffffff);
  const int vb = (int)(((16 * (wv >> 2) + r16) * ldb + 8 * (wv & 3) + 2 * g) * 8);
  // the vector-ALU block (q = 4 WN, one wave): column 16 WN + l % 4 (clamped
  // to N - 1), k offset 2 (l / 4)
  const int64_t rcol = (j0 + 16 * WN + (lane & 3) < N) ? j0 + 16 * WN + (lane & 3) : N - 1;
  const int vr = (int)(((rcol - j0) * ldb + 2 * (lane >> 2)) * 8);
  // A fragments of tile t (k = 8 h + 2 g + e for step 2 h + e); in a tile
  // that ends past the split, k is clamped to its last k (B is zero there)
  auto load_a = [&](int64_t t, double (&ra)[BK / 4]) {
    const int64_t kb = kbeg + t * BK;
    if (kb + BK <= kend) {
      // the lane's row pointer is recomputed here, not held through the
      // interleaved loop (whose buffer loads use a 32-bit offset instead)
      const int l = fresh(lane);
      const int64_t r = i0 + wave * 16 + (l & 15);
      const int64_t row = r < M ? r : M - 1;
      const double* const pa = TA ? A + row * lda + 2 * (l >> 4) : A + row + 2 * (l >> 4) * lda;
#pragma unroll
      for (int j = 0; j < BK / 4; ++j) {
        const int off = 8 * (j >> 1) + (j & 1);
        ra[j] = TA ? pa[opaque(kb) + off] : pa[opaque((kb + off) * lda)];
      }
    } else {
      const int l = fresh(lane);
      const int64_t r = i0 + wave * 16 + (l & 15);
      const int64_t row = r < M ? r : M - 1;
#pragma unroll
      for (int j = 0; j < BK / 4; ++j) {
        const int64_t kj = kb + 8 * (j >> 1) + 2 * (l >> 4) + (j & 1);
        const int64_t k = kj < kend ? kj : kend - 1;
        ra[j] = TA ? A[row * lda + k] : A[row + k * lda];
      }
    }
  };
  // Source of block q, lane l of a B tile: column and k offset in the tile.
  auto b_src = [&](int q, int l, int& col, int& kk) {
    if (q < 4 * WN) {
      col = 16 * (q >> 2) + (l & 15);
      kk = 8 * (q & 3) + 2 * (l >> 4);
    } else {
      col = 16 * WN + (l & 3);
      kk = 2 * (l >> 2);
    }
  };
  // Full tile: direct loads, wave w issuing blocks w, w + 8, ...; a block
  // whose 16 columns all lie before N needs no clamping (uniform test)
  auto dma_b = [&](int64_t t, double* bs) {
    const int kb8 = (int)((kbeg + t * BK) * 8);
#pragma unroll
    for (int q0 = 0; q0 < NQ; q0 += NW) {
      const int q = q0 + wv;
      if (q < 4 * WN && j0 + 16 * (q >> 2) + 15 < N) {
        buffer_load_lds16(bt, bt_bytes, vb, kb8 + (int)(4 * q0 * ldb * 8), bs + 128 * q);
      } else if (q == 4 * WN) {
        buffer_load_lds16(bt, bt_bytes, vr, kb8, bs + 128 * q);
      } else if (q < NQ) {
        int col, kk;
        b_src(q, fresh(lane), col, kk);
        const int64_t gc = (j0 + col < N) ? j0 + col : N - 1;
        buffer_load_lds16(bt, bt_bytes, (int)(((gc - j0) * ldb + kk) * 8), kb8, bs + 128 * q);
      }
    }
  };
  // Interleaved form, for full tiles when every MFMA block lies before N and
  // every A offset of the chunk fits in 31 bits: A by buffer loads from the
  // workgroup's origin (a fixed per-lane byte offset, the tile and fragment
  // offsets uniform), the panel's MFMA blocks by direct loads at fixed
  // offsets, both issued one after each MFMA.
  const double* const aorg = TA ? A + i0 * lda + kbeg : A + i0 + kbeg * lda;
  const int64_t aext =
      TA ? ((M - 1 - i0) * lda + K - kbeg) * 8 : ((M - i0) + (K - 1 - kbeg) * lda) * 8;
  const int a_bytes = (int)min(aext, (int64_t)0x7fffffff);
  const bool il_ok = j0 + 16 * WN <= N &&
                     (TA ? (BM * lda + kchunk + BK) * 8 < 0x7fffffff
                         : (BM + (kchunk + BK) * lda) * 8 < 0x7fffffff);
  const int va = il_ok ? (TA ? (int)(((arow - i0) * lda + 2 * g) * 8)
                             : (int)(((arow - i0) + 2 * g * lda) * 8))
                       : 0;
  auto load_a1 = [&](int64_t t, double (&ra)[BK / 4], int j) {
    const int off = 8 * (j >> 1) + (j & 1);
    const int so = TA ? (int)((t * BK + off) * 8) : (int)((t * BK + off) * lda * 8);
    ra[j] = buffer_load_f64(aorg, a_bytes, va, so);
  };
  constexpr int NI = (4 * WN) / NW;  // groups i whose blocks 8 i + w are all MFMA blocks
  auto dma_full = [&](int64_t t, double* bs, int i) {
    const int kb8 = (int)((kbeg + t * BK) * 8);
    buffer_load_lds16(bt, bt_bytes, vb, kb8 + (int)(4 * NW * i * ldb * 8),
                      bs + 128 * (NW * i + wv));
  };
  auto dma_tail = [&](int64_t t, double* bs) {
    const int kb8 = (int)((kbeg + t * BK) * 8);
#pragma unroll
    for (int q0 = NW * NI; q0 < NQ; q0 += NW) {
      const int q = q0 + wv;
      if (q < 4 * WN) {
        buffer_load_lds16(bt, bt_bytes, vb, kb8 + (int)(4 * q0 * ldb * 8), bs + 128 * q);
      } else if (q == 4 * WN) {
        buffer_load_lds16(bt, bt_bytes, vr, kb8, bs + 128 * q);
      }
    }
  };
  // Ragged tile: the same layout through registers, zero past kend.
  auto stage_b = [&](int64_t t, double* bs) {
    const int64_t kb = kbeg + t * BK;
    const int l = fresh(lane);
#pragma unroll
    for (int q0 = 0; q0 < NQ; q0 += NW) {
      const int q = q0 + wave;
      if (q < NQ) {
        int col, kk;
        b_src(q, l, col, kk);
        const int64_t gc = (j0 + col < N) ? j0 + col : N - 1;
        const double* src = B + gc * ldb;
        const double v0 = (kb + kk < kend) ? src[kb + kk] : 0.0;
        const double v1 = (kb + kk + 1 < kend) ? src[kb + kk + 1] : 0.0;
        bs[128 * q + 2 * l] = v0;
        bs[128 * q + 2 * l + 1] = v1;
      }
    }
  };
  // Steps 2 h and 2 h + 1 of lane (g, r) use the pair k = 8 h + 2 g + e
  // (e = 0, 1) of its column, which one 16-byte LDS read returns: block b at
  // 128 (4 b + h) + 2 (16 g + r), the position this lane's own direct load
  // wrote (a wave reads 1 KB contiguous: no bank conflicts); vector-ALU
  // column c at 128 (4 WN) + 32 h + 8 g + 2 c.
  typedef double double2_t __attribute__((ext_vector_type(2)));
  const int fo = 2 * (16 * g + r16), ro = 8 * g;
  auto frag = [&](const double* bs, int h, int b) {
    return *(const double2_t*)(bs + 128 * (4 * b + h) + fo);
  };
  // Double step h: 2 WN MFMAs and the vector-ALU columns; the fragments of
  // h + 1 are read into each block's registers as soon as its second MFMA
  // has been issued.
  auto compute = [&](auto ilc, const double (&ra)[BK / 4], const double* bs, int64_t tn,
                     double (&ran)[BK / 4], double* bsn) {
    constexpr bool IL = decltype(ilc)::value;
    double2_t bf[WN];
#pragma unroll
    for (int b = 0; b < WN; ++b) bf[b] = frag(bs, 0, b);
#pragma unroll
    for (int h = 0; h < BK / 8; ++h) {
      double2_t br[RV];
#pragma unroll
      for (int c = 0; c < RV; ++c)
        br[c] = *(const double2_t*)(bs + 128 * (4 * WN) + 32 * h + ro + 2 * c);
#pragma unroll
      for (int b = 0; b < WN; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[2 * h], bf[b].x, acc[b], 0, 0, 0);
      // issue order: the first MFMA of step 2 h, the panel reads of the
      // vector-ALU columns, the other MFMAs (so that no more than 15 LDS
      // reads are ever outstanding past the one an MFMA waits for: the
      // counter the waits use saturates at 15); in the interleaved form the
      // next tile's A loads (step 0) or panel loads (step 2) one after each
      // of these MFMAs
      if constexpr (IL) {
        if (h == 0) {
#pragma unroll
          for (int j = 0; j < BK / 4; ++j) load_a1(tn, ran, j);
        } else if (h == 1) {
#pragma unroll
          for (int i = 0; i < NI; ++i) dma_full(tn, bsn, i);
        }
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, RV, 0);
      if (IL && h == 0) {
#pragma unroll
        for (int u = 0; u < BK / 4; ++u) {
          if (u < WN - 1) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
        }
        if constexpr (WN - 1 > BK / 4)
          __builtin_amdgcn_sched_group_barrier(0x008, WN - 1 - BK / 4, 0);
      } else if (IL && h == 1) {
#pragma unroll
        for (int u = 0; u < NI; ++u) {
          if (u < WN - 1) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
        }
        if constexpr (WN - 1 > NI) __builtin_amdgcn_sched_group_barrier(0x008, WN - 1 - NI, 0);
      } else {
        __builtin_amdgcn_sched_group_barrier(0x008, WN - 1, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (IL) {
        if (h == 1) dma_tail(tn, bsn);
      }
#pragma unroll
      for (int b = 0; b < WN; ++b) {
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[2 * h + 1], bf[b].y, acc[b], 0, 0,
                                                      0);
        if (h + 1 < BK / 8) bf[b] = frag(bs, h + 1, b);
      }
#pragma unroll
      for (int c = 0; c < RV; ++c) {
        vacc[c] = ra[2 * h] * br[c].x + vacc[c];
        vacc[c] = ra[2 * h + 1] * br[c].y + vacc[c];
        asm volatile("" : "+v"(vacc[c]));  // keep the update in this step
      }
      // issue order: the FMAs (their panel values arrived during step 2 h),
      // then each MFMA of step 2 h + 1 followed by the read that refills its
      // block's fragment registers
      __builtin_amdgcn_sched_group_barrier(0x002, 2 * RV, 1);
#pragma unroll
      for (int b = 0; b < WN; ++b) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);
        if (h + 1 < BK / 8) __builtin_amdgcn_sched_group_barrier(0x100, 1, 1);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto full = [&](int64_t t) { return kbeg + (t + 1) * BK <= kend; };
  // vmcnt(0): every load of this wave done (direct loads included) before
  // the barrier that hands the tile to the other waves
  auto wait_loads = [&]() { __builtin_amdgcn_s_waitcnt(0x0F70); };
  // multiply the tile in (ra, bs) while tile tn loads into (ran, bsn)
  auto half = [&](const double (&ra)[BK / 4], const double* bs, int64_t tn,
                  double (&ran)[BK / 4], double* bsn) {
    const bool fn = full(tn);
    if (fn) dma_b(tn, bsn);
    load_a(tn, ran);
    compute(std::false_type{}, ra, bs, tn, ran, bsn);
    if (!fn) stage_b(tn, bsn);
    wait_loads();
    __syncthreads();
  };
  // the same for a full tile tn in the interleaved form
  auto half_il = [&](const double (&ra)[BK / 4], const double* bs, int64_t tn,
                     double (&ran)[BK / 4], double* bsn) {
    compute(std::true_type{}, ra, bs, tn, ran, bsn);
    wait_loads();
    __syncthreads();
  };

  if (nt > 0) {
    if (full(0)) dma_b(0, Bs0);
    else stage_b(0, Bs0);
    load_a(0, ra0);
    wait_loads();
    __syncthreads();
    // pairs of tiles; the loads past the last tile re-read it (unused)
    int64_t t = 0;
    // pairs of tiles whose successors are both full, interleaved; then the
    // rest (at most three tiles, or all when the interleaved form does not
    // apply) with the loads issued ahead of each tile
    const int64_t nf = (kend - kbeg) / BK;
    if (il_ok) {
      for (; t + 2 < nf; t += 2) {
        half_il(ra0, Bs0, t + 1, ra1, Bs1);
        half_il(ra1, Bs1, t + 2, ra0, Bs0);
      }
    }
    for (; t + 1 < nt; t += 2) {
      half(ra0, Bs0, t + 1, ra1, Bs1);
      half(ra1, Bs1, t + 2 < nt ? t + 2 : nt - 1, ra0, Bs0);
    }
    if (t < nt) compute(std::false_type{}, ra0, Bs0, t, ra1, Bs1);
  }

  double* Cs = C + split * strideS;
#pragma unroll
  for (int b = 0; b < WN; ++b) {
    const int64_t col = j0 + b * 16 + r16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = i0 + wave * 16 + acc_row<double>(lane, r);
      if (row < M && col < N) Cs[row + col * ldc] = acc[b][r];
    }
  }
#pragma unroll
  for (int c = 0; c < RV; ++c) {
    double v = vacc[c];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    const int64_t row = i0 + wave * 16 + r16;
    const int64_t col = j0 + 16 * WN + c;
    if (lane < 16 && row < M && col < N) Cs[row + col * ldc] = v;
  }
}

template <bool TA, int WN>
int stream_occupancy() {
  static const int nb = occupancy_of(gemm_stream_f64_kernel<TA, WN, 4>, 64 * kStrWaves);
  return nb;
}

template <bool TA, int WN = kStrMaxWN>
int stream_occupancy_wn(int wn) {
  if constexpr (WN > 1) {
    if (wn < WN) return stream_occupancy_wn<TA, WN - 1>(wn);
  }
  return stream_occupancy<TA, WN>();
}

template <bool TA, int WN>
void dispatch_stream(int wn, int rv, dim3 grid, const double* A, int64_t lda, const double* B,
                     int64_t ldb, double* C, int64_t ldc, int64_t strideS, int64_t M, int64_t N,
                     int64_t K, int64_t kchunk, hipStream_t st) {
  if constexpr (WN > 1) {
    if (wn < WN)
      return dispatch_stream<TA, WN - 1>(wn, rv, grid, A, lda, B, ldb, C, ldc, strideS, M, N, K,
                                         kchunk, st);
  }
  if (rv == 2)
    hipLaunchKernelGGL((gemm_stream_f64_kernel<TA, WN, 2>), grid, dim3(64 * kStrWaves), 0, st,
                       A, lda, B, ldb, C, ldc, strideS, M, N, K, kchunk);
  else
    hipLaunchKernelGGL((gemm_stream_f64_kernel<TA, WN, 4>), grid, dim3(64 * kStrWaves), 0, st,
                       A, lda, B, ldb, C, ldc, strideS, M, N, K, kchunk);
}

}  // namespace

int gemm_stream_f64_occupancy(int trans_a, int wn) {
  return trans_a ? stream_occupancy_wn<true>(wn) : stream_occupancy_wn<false>(wn);
}

void launch_gemm_stream_f64(int trans_a, int wn, int rv, int64_t tiles_m, int64_t tiles_n,
                            int splits, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double* C, int64_t ldc, int64_t strideS, int64_t M,
                            int64_t N, int64_t K, int64_t kchunk, hipStream_t st) {
  const dim3 grid((unsigned)tiles_m, (unsigned)tiles_n, (unsigned)splits);
  if (trans_a)
    dispatch_stream<true, kStrMaxWN>(wn, rv, grid, A, lda, B, ldb, C, ldc, strideS, M, N, K,
                                     kchunk, st);
  else
    dispatch_stream<false, kStrMaxWN>(wn, rv, grid, A, lda, B, ldb, C, ldc, strideS, M, N, K,
                                      kchunk, st);
}

}  // namespace rqlp

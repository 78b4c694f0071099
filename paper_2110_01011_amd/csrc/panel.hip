// orth() of Algorithm 1 for tall-skinny panels: Cholesky QR building blocks.
//
// For a rows x d panel X with Gram matrix G = X^T X (formed by the GEMM
// kernels in fp64):
//   cholesky_kernel  G (+ shift I) = R^T R, R upper with R_jj >= 0, plus the
//                    inverses of R's 16 x 16 diagonal blocks.  One workgroup
//                    of 8 waves holds the lower 16 x 16 tiles of G in MFMA
//                    accumulator registers (d <= 224), factors each diagonal
//                    tile on one wave, solves the block column with MFMA and
//                    applies the rank-16 trailing update with MFMA.  A pivot at
//                    or below tol_dep * (original diagonal) marks its column as
//                    numerically dependent: that row of R is set to zero.
//   trsm_kernel      Qx = X R^+ by block forward substitution: each wave owns
//                    16 rows of X, keeps its finished columns in LDS and uses
//                    the staged column block of R and the diagonal inverse.
// plus small kernels: R2 * R1, L = R^T, trace, casts, flag counts, NaN scan.
#include "rqlp_internal.h"

namespace rqlp {
namespace {

__device__ __forceinline__ double4_t mma64(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// two doubles at an 8-byte aligned address (one 16-byte vector store)
typedef double double2_a8 __attribute__((ext_vector_type(2), aligned(8)));

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Cholesky workgroup: wave 0 factors the diagonal tiles; wave 4 (which
// shares wave 0's SIMD) holds nothing, so no MFMA work competes with the
// pivot chain; the six other waves hold the lower tiles.
constexpr int kCholWaves = 8;
constexpr int kTileWaves = 6;
constexpr int kCholSlots = 18;  // ceil(105 lower tiles (d <= 224) / 6 waves)

__device__ __forceinline__ int tile_wave_id(int idx) { return idx < 3 ? idx + 1 : idx + 2; }
__device__ __forceinline__ int tile_wave_idx(int wave) { return wave < 4 ? wave - 1 : wave - 2; }

// Factor the 16 x 16 diagonal tile held in dg (row-major, full symmetric) in
// place into its lower Cholesky factor L_JJ and write X = L_JJ^{-1} into dgi.
// Run by one wave.  Lanes 0..15 own one row of the tile each; lanes 16..31
// own one column of X, which they build in the same pivot steps by forward
// substitution (X row s = Y row s / l_ss, then Y row j -= l_js X row s), so
// both use the same broadcast column of L.  Every lane evaluates the pivot
// test and 1/sqrt on its own diagonal entry (without a branch: 1/sqrt of 1
// where the test fails).  The pivot chain runs through registers and lane
// reads only: lane s + 1 forms its next pivot from its own l (the value the
// broadcast would give it), and 1/sqrt of it is issued before the rest of
// step s; every lane takes 1/l_ss (from lane s), l_{s+1,s} and l_{s+2,s}
// (from lanes s + 1, s + 2) by lane reads, which is all steps s + 1 and
// s + 2 need of step s.  The rest of the column of L, for the updates of
// entries s + 3 .. 15, goes through a per-step row of LDS (bc): read back
// as broadcasts at the start of step s + 1 and applied after that step's
// pivot work (scheduling fences keep the two apart), so the LDS latency is
// off the chain.  The wave's own LDS accesses complete in order, so no wait
// separates the write and the reads.  The updates of an entry thus arrive
// in a fixed order that differs from k order (rounding level only).  A
// dependent pivot (<= tol_dep of the column's original diagonal, or
// non-finite) gives a zero column of L and a zero row of X.  The pivot
// tests are evaluated after the chain: flags go to *sflag, the per-column
// dependence marks to colf (LDS).  The tile comes in registers (a, from
// load_diag_rows), read by the caller ahead of the barrier it waits at.
__device__ __forceinline__ void load_diag_rows(const double (*dg)[17], double (&a)[16]) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15;
  const bool rowlane = lane < 16;
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = rowlane ? dg[i][c] : ((c == i) ? 1.0 : 0.0);
}

__device__ __forceinline__ void factor_diag_tile(double (&a)[16], double (*dg)[17],
                                                 double (*dgi)[17], double (*bc)[16],
                                                 const double* odiag, int J, int d,
                                                 double tol_dep, double tol_warn, int* colf,
                                                 int* sflag) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15;
  const bool rowlane = lane < 16;
  const double orig = odiag[16 * J + i];
  const double thr = tol_dep * orig;
  double mypiv = 0.0;
  // 1 / sqrt(p) where p passes the pivot test, else 0 (NaN and dependent
  // pivots included)
  auto rinv = [&](double p) {
    const bool ok = p > thr;
    const double r = rsqrt(ok ? p : 1.0);
    return ok ? r : 0.0;
  };
  double p = a[0];  // the next pivot, on lane s
  double y = readlane_d(rinv(p), 0);  // 1 / l_ss
  double vp = 0.0;                    // v of the previous step
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    // the previous step's column, entries s + 2 .. 15
    double bj[16];
#pragma unroll
    for (int j = s + 2; j < 16; ++j) bj[j] = (s >= 1) ? bc[s - 1][j] : 0.0;
    __builtin_amdgcn_sched_barrier(0);
    mypiv = (i == s) ? p : mypiv;
    // rows: l_is (l_ss itself on lane s, 0 above the diagonal); columns of
    // X: the finished entry X[s][c]
    const double w = a[s] * y;
    const double v = (!rowlane || i >= s) ? w : 0.0;
    a[s] = v;
    if (s + 1 < 16) {
      // lane s + 1's next pivot from its own l, and its 1/sqrt, first
      p = fma(-w, w, a[s + 1]);
      const double yn = rinv(p);
      a[s + 1] = fma(-v, readlane_d(v, s + 1), a[s + 1]);
      if (s + 2 < 16) a[s + 2] = fma(-v, readlane_d(v, s + 2), a[s + 2]);
      y = readlane_d(yn, s + 1);
      if (s + 3 < 16 && rowlane) bc[s][i] = v;
    }
    __builtin_amdgcn_sched_barrier(0);
    if (s >= 1) {
#pragma unroll
      for (int j = s + 2; j < 16; ++j) a[j] = fma(-vp, bj[j], a[j]);
    }
    vp = v;
  }
  if (lane < 32) {
    // rows of L to dg (zeros above the diagonal), columns of X to dgi: one
    // store per entry for both halves
    double* base = rowlane ? &dg[i][0] : &dgi[0][i];
    const int step = rowlane ? 1 : 17;
#pragma unroll
    for (int c = 0; c < 16; ++c) base[c * step] = (rowlane && c > i) ? 0.0 : a[c];
  }
  const int gj = 16 * J + i;
  if (rowlane && gj < d) {
    const bool nonfinite = !__builtin_isfinite(mypiv);
    const bool dep = nonfinite || !(mypiv > thr);
    int bits = 0;
    if (nonfinite) bits |= FLAG_NONFINITE;
    if (dep) bits |= FLAG_NONPOS_PIVOT;
    if (!dep && mypiv < tol_warn * orig) bits |= FLAG_SECOND_PASS;
    colf[gj] = dep ? 1 : 0;
    if (bits) atomicOr(sflag, bits);
  }
}

// Tile-wave part of the Cholesky kernel.  Each lower tile (I, J), I >= J, is
// held transposed, T = G_IJ^T, in MFMA accumulator layout: register r of
// lane l holds T[(l >> 4) + 4 r][l & 15] = G[16 I + (l & 15)][16 J + (l >> 4)
// + 4 r], so the loads from the column-major G are contiguous along lanes,
// and register r is also the B operand of k-step r of a product X T.  With
// this layout the panel solve is L_IJ^T = L_JJ^{-1} T (four MFMAs from
// registers), and the trailing update is T_IK -= L_KJ L_IJ^T.  Each updated
// diagonal tile goes to the factor wave.  R = L^T is written as the tiles
// become final (the idle wave writes the zero tiles below its diagonal), so
// no store is left for the end of the kernel.
__device__ __forceinline__ void chol_tile_wave(
    const double* __restrict__ G, int d, int64_t ldg, double sh, double (*dg2)[16][17],
    double (*dgi_all)[16][17], double (*pan)[17], double (*tpan2)[16][17],
    double (*tdia2)[16][17], int* ready, int* pan_done, int wave, double* __restrict__ R,
    int64_t ldr) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (d + 15) / 16;
  const int T = nt * (nt + 1) / 2;
  const int twi = tile_wave_idx(wave);
  double4_t acc[kCholSlots];
  int tI[kCholSlots], tJ[kCholSlots];
  // Byte offsets stay 32-bit (d <= 224 and the leading dimensions are small)
  // so that the loads and stores use a scalar base and one vector offset.
  const global_ptr<const char> Gb = (global_ptr<const char>)reinterpret_cast<const char*>(G);
  const unsigned ldg8 = 8u * (unsigned)ldg;
  const global_ptr<char> Rb = (global_ptr<char>)reinterpret_cast<char*>(R);
  const unsigned ldr8 = 8u * (unsigned)ldr;
  const int q0 = 4 * lk;  // R stores: each lane writes rows q0 .. q0 + 3 of one column
  // Four consecutive rows (row0 ..) of column col of R; rows past d dropped.
  auto store4 = [&](int row0, int col, double v0, double v1, double v2, double v3) {
    if (col >= d) return;
    const global_ptr<double> dst =
        (global_ptr<double>)(Rb + (8u * (unsigned)row0 + __umul24((unsigned)col, ldr8)));
    if (row0 + 3 < d) {
      *(global_ptr<double2_a8>)dst = double2_a8{v0, v1};
      *(global_ptr<double2_a8>)(dst + 2) = double2_a8{v2, v3};
    } else {
      if (row0 < d) dst[0] = v0;
      if (row0 + 1 < d) dst[1] = v1;
      if (row0 + 2 < d) dst[2] = v2;
    }
  };
  // All loads first (addresses clamped into G), so that every slot's loads
  // are in flight together.  Slot s holds tile t = twi + 6 s; its row index
  // I only grows with s.
  int I = 0;
#pragma unroll
  for (int s = 0; s < kCholSlots; ++s) {
    const int t = twi + kTileWaves * s;
    tI[s] = -1;
    tJ[s] = -1;
    acc[s] = double4_t{0, 0, 0, 0};
    if (t < T) {
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      const int Jt = t - I * (I + 1) / 2;
      tI[s] = I;
      tJ[s] = Jt;
      const unsigned grow8 = 8u * (unsigned)min(16 * I + li, d - 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const unsigned gcol = (unsigned)min(16 * Jt + acc_row_f64(lane, r), d - 1);
        acc[s][r] = *(global_ptr<const double>)(Gb + (grow8 + __umul24(gcol, ldg8)));
      }
    }
  }
  // Padding and the shift, slot by slot (slot 0 first: it may hold tile 0,
  // which goes to the factor wave as soon as it is in).
  auto owner = [&](int J) { return tile_wave_id((J * (J + 3) / 2) % kTileWaves); };
  auto slot = [&](int J) { return (J * (J + 3) / 2) / kTileWaves; };
  auto publish0 = [&](double4_t c) {  // tile 0 to the factor wave: dg = T^T (row-major)
#pragma unroll
    for (int r = 0; r < 4; ++r) dg2[0][li][acc_row_f64(lane, r)] = c[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) __hip_atomic_store(ready, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  // Tiles (Jn + 1, Jn) and (Jn + 1, Jn + 1), up to date through step Jn - 1,
  // to LDS (accumulator layout) for the factor wave's lookahead in step Jn.
  auto stash = [&](int Jn) {
    if (Jn + 1 >= nt) return;
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s) {
      if (tI[s] != Jn + 1 || tJ[s] < Jn) continue;
      double (*dst)[17] = (tJ[s] == Jn) ? tpan2[Jn & 1] : tdia2[Jn & 1];
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[acc_row_f64(lane, r)][li] = acc[s][r];
    }
  };
#pragma unroll
  for (int s = 0; s < kCholSlots; ++s) {
    if (tI[s] < 0) continue;
    const int grow = 16 * tI[s] + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gcol = 16 * tJ[s] + acc_row_f64(lane, r);
      if (grow >= d || gcol >= d)
        acc[s][r] = (grow == gcol) ? 1.0 : 0.0;
      else if (grow == gcol)
        acc[s][r] += sh;
    }
    if (s == slot(0) && wave == owner(0)) publish0(acc[s]);
  }
  stash(0);
  // Every load has landed; an explicit wait on all counters tells the
  // compiler so, and keeps it from waiting on pending stores of R before
  // later uses of these registers.
  __builtin_amdgcn_s_waitcnt(0);
  for (int J = 0; J < nt; ++J) {
    __syncthreads();  // L_JJ and its inverse are ready
    double (*dgi)[17] = dgi_all[J];
    double (*dg)[17] = dg2[J & 1];
    // Panel: L_IJ^T = L_JJ^{-1} G_IJ^T for the tiles below the diagonal; pan
    // receives L_IJ (row-major rows 16 I ..), and the final tiles go to R.
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s) {
      if (tJ[s] != J) continue;
      const int I = tI[s];
      if (I == J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[s][r] = dg[li][acc_row_f64(lane, r)];  // L_JJ^T
        // R tile (J, J) = L_JJ^T: R[16 J + q][16 J + li] = L_JJ[li][q]
        store4(16 * J + q0, 16 * J + li, dg[li][q0], dg[li][q0 + 1], dg[li][q0 + 2],
               dg[li][q0 + 3]);
      } else {
        double4_t res = {0, 0, 0, 0};
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) res = mma64(dgi[li][kq * 4 + lk], acc[s][kq], res);
        acc[s] = res;
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[16 * I + li][acc_row_f64(lane, r)] = res[r];
        wave_sync_lds();
        // R tile (J, I) = L_IJ^T: R[16 J + q][16 I + li] = L_IJ[li][q]
        const double* pr = pan[16 * I + li];
        store4(16 * J + q0, 16 * I + li, pr[q0], pr[q0 + 1], pr[q0 + 2], pr[q0 + 3]);
      }
    }
    // Panel J is ready once the six tile waves have written their tiles: an
    // LDS count (each wave adds 1 after its writes; every tile wave adds
    // before it waits, so the wait ends).  The factor wave takes no part: it
    // goes on to the next diagonal tile while the panel and the trailing
    // update run.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0)
      __hip_atomic_fetch_add(pan_done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (__hip_atomic_load(pan_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) <
           kTileWaves * (J + 1))
      __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // Trailing update (the factor wave has already brought tile (J+1, J+1)
    // up to date for itself; the copy here only feeds the next stash).
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s) {
      const int I = tI[s], K = tJ[s];
      if (K <= J) continue;
      double4_t c = acc[s];
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) {
        const double a = pan[16 * K + li][kq * 4 + lk];
        const double b = pan[16 * I + li][kq * 4 + lk];
        c = mma64(-a, b, c);
      }
      acc[s] = c;
    }
    stash(J + 1);
  }
}

// Cholesky of G + shift I (d <= 224) on one workgroup of 8 waves.  Wave 0
// factors each 16 x 16 diagonal tile as soon as its owner publishes it
// (an LDS flag; the owner never waits on wave 0, so the wait always ends);
// wave 4 shares wave 0's SIMD and issues no MFMA, so nothing competes with
// the pivot chain; it writes each diagonal-block inverse out as soon as it
// is ready.  The six other waves hold the tiles.  One workgroup barrier per
// step (L_JJ and its inverse ready, next tiles stashed); the tile waves wait
// for each other's panel writes on an LDS count instead of a second
// barrier, so the factor wave starts on tile J + 1 while they solve panel J
// (a second barrier held it back about 300 cycles a step: 62.6 -> 60.8 us
// at d = 210).
__device__ __forceinline__ void cholesky_body(
    const double* __restrict__ G, int d, int64_t ldg, double shift,
    const double* __restrict__ shift_dev, double tol_dep, double tol_warn,
    double* __restrict__ R, int64_t ldr, double* __restrict__ dinv,
    int* __restrict__ col_flags, int* __restrict__ flags,
    const double* __restrict__ odiag_src, int64_t odiag_stride) {
  __shared__ double dg2[2][16][17];  // diagonal tile J in dg2[J & 1]
  __shared__ double bc[16][16];      // the factor wave's column broadcasts
  __shared__ double dgi_all[CHOL_MAX_D / 16][16][17];  // inverse of L_JJ for every J
  // stashed tiles (J+1, J), (J+1, J+1) for step J, by the parity of J (the
  // tile waves stash step J + 1's while the factor wave may still read step
  // J's)
  __shared__ double tpan2[2][16][17], tdia2[2][16][17];
  __shared__ double wl[16][17];                       // the factor wave's L_{J+1,J}
  __shared__ double pan[CHOL_MAX_D][17];
  __shared__ double odiag[CHOL_MAX_D];
  __shared__ int colf[CHOL_MAX_D];
  __shared__ int sflag;
  __shared__ int ready;     // index of the last diagonal tile published in dg
  __shared__ int pan_done;  // tile waves done with their panel writes, over all steps

  const int nt = (d + 15) / 16;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double sh = (shift_dev != nullptr) ? *shift_dev : shift;
  if (tid == 0) {
    sflag = 0;
    ready = -1;
    pan_done = 0;
  }
  __syncthreads();  // the flags are initialised
  if (wave == 0) {
    // Pivots are judged against the original diagonal (of the whole matrix
    // when this call factors a trailing Schur complement); the factor wave
    // reads it while the tile waves load their tiles.
    double ov[CHOL_MAX_D / 64 + 1];
#pragma unroll
    for (int u = 0; u * 64 < CHOL_MAX_D; ++u) {  // all loads in flight together
      const int j = min(lane + 64 * u, d - 1);
      ov[u] = odiag_src ? odiag_src[(int64_t)j * odiag_stride] : G[j + (int64_t)j * ldg];
    }
#pragma unroll
    for (int u = 0; u * 64 < CHOL_MAX_D; ++u) {
      const int j = lane + 64 * u;
      if (j < CHOL_MAX_D) odiag[j] = (j >= d) ? 1.0 : ov[u] + sh;
    }
    const int li = lane & 15, lk = lane >> 4;
    while (__hip_atomic_load(&ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < 0)
      __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double a[16];  // the next diagonal tile's rows
    load_diag_rows(dg2[0], a);
    for (int J = 0; J < nt; ++J) {
      factor_diag_tile(a, dg2[J & 1], dgi_all[J], bc, odiag, J, d, tol_dep, tol_warn, colf,
                       &sflag);
      __syncthreads();  // L_JJ and its inverse are ready; tiles (J+1, J), (J+1, J+1) stashed
      if (J + 1 < nt) {
        // Lookahead: L_{J+1,J}^T = L_JJ^{-1} T_{J+1,J}, then tile (J+1, J+1)
        // less L_{J+1,J} L_{J+1,J}^T, straight into the next diagonal buffer.
        const double (*x)[17] = dgi_all[J];
        double4_t t, c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          t[r] = tpan2[J & 1][acc_row_f64(lane, r)][li];
          c[r] = tdia2[J & 1][acc_row_f64(lane, r)][li];
        }
        double4_t res = {0, 0, 0, 0};
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) res = mma64(x[li][kq * 4 + lk], t[kq], res);
#pragma unroll
        for (int r = 0; r < 4; ++r) wl[li][acc_row_f64(lane, r)] = res[r];
        wave_sync_lds();
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
          const double a = wl[li][kq * 4 + lk];
          c = mma64(-a, a, c);
        }
        double (*dn)[17] = dg2[(J + 1) & 1];
#pragma unroll
        for (int r = 0; r < 4; ++r) dn[li][acc_row_f64(lane, r)] = c[r];
        wave_sync_lds();
        load_diag_rows(dn, a);  // only this wave wrote dn
      }
    }
  } else if (wave == 4) {
    const int li = lane & 15, q0 = 4 * (lane >> 4);
    for (int J = 0; J < nt; ++J) {
      __syncthreads();
      // R below the diagonal tiles is zero: in step J the tiles (J + 1, K),
      // K <= J (rows and columns past d dropped), four rows of one column
      // per lane.
      if (J + 1 < nt) {
        const int row0 = 16 * (J + 1) + q0;
        for (int K = 0; K <= J; ++K) {
          const int col = 16 * K + li;
          double* dst = R + row0 + (int64_t)col * ldr;
          if (row0 + 3 < d) {
            *reinterpret_cast<double2_a8*>(dst) = double2_a8{0.0, 0.0};
            *reinterpret_cast<double2_a8*>(dst + 2) = double2_a8{0.0, 0.0};
          } else {
            for (int q = 0; q < 3; ++q)
              if (row0 + q < d) dst[q] = 0.0;
          }
        }
      }
      // the inverse of block J ((L_JJ^{-1})^T, column-major) and its marks
      const double (*x)[17] = dgi_all[J];
#pragma unroll
      for (int e = lane; e < 256; e += 64) dinv[J * 256 + e] = x[(e >> 4) & 15][e & 15];
      if (col_flags != nullptr && lane < 16 && 16 * J + lane < d)
        col_flags[16 * J + lane] = colf[16 * J + lane];
    }
  } else {
    chol_tile_wave(G, d, ldg, sh, dg2, dgi_all, pan, tpan2, tdia2, &ready, &pan_done, wave, R,
                   ldr);
  }
  __syncthreads();
  if (tid == 0 && sflag) atomicOr(flags, sflag);
}

__global__ __launch_bounds__(512) void cholesky_kernel(
    const double* __restrict__ G, int d, int64_t ldg, double shift,
    const double* __restrict__ shift_dev, double tol_dep, double tol_warn,
    double* __restrict__ R, int64_t ldr, double* __restrict__ dinv,
    int* __restrict__ col_flags, int* __restrict__ flags,
    const double* __restrict__ odiag_src, int64_t odiag_stride) {
  cholesky_body(G, d, ldg, shift, shift_dev, tol_dep, tol_warn, R, ldr, dinv, col_flags, flags,
                odiag_src, odiag_stride);
}

// Grouped form: workgroup i factors problem i.
__global__ __launch_bounds__(512) void cholesky_grouped_kernel(const GroupChol* __restrict__ descs) {
  const GroupChol c = descs[blockIdx.x];
  cholesky_body(c.G, c.d, c.ldg, 0.0, nullptr, c.tol_dep, c.tol_warn, c.R, c.ldr, c.dinv,
                nullptr, c.flags, nullptr, 0);
}

// Qx = X R^+ by block forward substitution.  One wave (one workgroup) owns 16
// rows.  Their whole block of X goes to the wave's LDS panel first (all
// loads in flight together); then for each 16-column block J the wave forms
// V_J = X_J - sum_{K<J} Q_K R_KJ with MFMA (A fragments from its finished
// columns in LDS, B fragments of R from L2) and Q_J = V_J R_JJ^{-1} in
// place.  The B fragments come in batches of 16 k-steps, each loaded while
// the previous batch's MFMAs run, the prefetch running on into the first
// batch of the next block; the next diagonal-block inverse is loaded at the
// start of each block.  Q leaves LDS at the end, so no global access waits
// inside the block loop.  X and Qx may be the same array (a wave reads all
// of its rows before it writes any).
// B: k-steps per batch of B fragments; TL: the type the row block is kept
// in (LDS), double by default.
template <typename TX, typename TO, int B = 16, typename TL = double>
__device__ __forceinline__ void trsm_body(const TX* X, int64_t rows, int d, int64_t ldx,
                                          const double* __restrict__ R, int64_t ldr,
                                          const double* __restrict__ dinv, TO* Qx, int64_t ldq,
                                          const int64_t r0) {
  extern __shared__ double lds_raw[];
  TL* const Qw = reinterpret_cast<TL*>(lds_raw);
  constexpr int XC = 16;  // X values per lane per load round
  const int nt = (d + 15) / 16, dp = nt * 16, lq = dp + 1;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  // X block -> LDS: lane (li, lk) takes row r0 + li of columns lk, lk + 4, ...
  {
    const bool rowok = r0 + li < rows;
    const global_ptr<const TX> xr = (global_ptr<const TX>)X + (rowok ? r0 + li : r0);
    for (int c0 = 0; c0 < dp; c0 += 4 * XC) {
      double xv[XC];
#pragma unroll
      for (int u = 0; u < XC; ++u) {
        const int c = c0 + lk + 4 * u;
        xv[u] = (rowok && c < d) ? (double)xr[(int64_t)c * ldx] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < XC; ++u) {
        const int c = c0 + lk + 4 * u;
        if (c < dp) Qw[li * lq + c] = (TL)xv[u];
      }
    }
  }
  // B fragment of k-step q of block Jb (Jb >= 1): R[4 q + lk][16 Jb + li].
  // Every load is issued and its value used as loaded, so that the batch
  // stays in flight until its MFMAs (a load behind a branch, or a select
  // on its value, makes the compiler wait for it at once): the k-step is
  // clamped to the block's last (its A operand is zero there) and a column
  // past d to column 0 (its results land in padding columns of the panel,
  // which no later block reads and which are not stored).  The pointers are
  // global ones, so the loads are counted on vmcnt only.
  typedef __attribute__((address_space(1))) const double gdouble;
  const gdouble* const Rg = (const gdouble*)R;
  const gdouble* const Dg = (const gdouble*)dinv;
  auto load_batch = [&](int Jb, int base, double* dst) {
    const int colR = 16 * Jb + li;
    const gdouble* Rc = Rg + (int64_t)(colR < d ? colR : 0) * ldr + lk;
    const int nk = 4 * Jb;
#pragma unroll
    for (int q = 0; q < B; ++q) dst[q] = Rc[min(base + q, nk - 1) * 4];
  };
  auto load_inv = [&](int Jb, double* dst) {
    const gdouble* T = Dg + (int64_t)Jb * 256;
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) dst[q4] = T[q4 * 4 + lk + li * 16];
  };
  double bc[B], bn[B], tb[4], tn[4];
  load_inv(0, tb);
  if (nt > 1) load_batch(1, 0, bc);
  wave_sync_lds();
  for (int J = 0; J < nt; ++J) {
    const int kk = 16 * J, nk = 4 * J;
    if (J + 1 < nt) load_inv(J + 1, tn);
    double4_t acc0, acc1 = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0}, acc3 = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc0[r] = (double)Qw[acc_row_f64(lane, r) * lq + kk + li];
    for (int base = 0; base < nk; base += B) {
      if (base + B < nk)
        load_batch(J, base + B, bn);
      else if (J + 1 < nt)
        load_batch(J + 1, 0, bn);
      double ac[B];
#pragma unroll
      for (int q = 0; q < B; ++q)
        ac[q] = (base + q < nk) ? (double)Qw[li * lq + (base + q) * 4 + lk] : 0.0;
#pragma unroll
      for (int q = 0; q < B; q += 4) {
        acc0 = mma64(-ac[q], bc[q], acc0);
        acc1 = mma64(-ac[q + 1], bc[q + 1], acc1);
        acc2 = mma64(-ac[q + 2], bc[q + 2], acc2);
        acc3 = mma64(-ac[q + 3], bc[q + 3], acc3);
      }
#pragma unroll
      for (int q = 0; q < B; ++q) bc[q] = bn[q];
    }
    acc0 += acc1;
    acc2 += acc3;
    acc0 += acc2;
#pragma unroll
    for (int r = 0; r < 4; ++r) Qw[acc_row_f64(lane, r) * lq + kk + li] = (TL)acc0[r];
    wave_sync_lds();
    double4_t res = {0, 0, 0, 0};
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4)
      res = mma64((double)Qw[li * lq + kk + q4 * 4 + lk], tb[q4], res);
    wave_sync_lds();
#pragma unroll
    for (int r = 0; r < 4; ++r) Qw[acc_row_f64(lane, r) * lq + kk + li] = (TL)res[r];
    wave_sync_lds();
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) tb[q4] = tn[q4];
  }
  // Q block -> Qx
  if (r0 + li < rows) {
    const global_ptr<TO> qr = (global_ptr<TO>)Qx + r0 + li;
    for (int c = lk; c < d; c += 4) qr[(int64_t)c * ldq] = (TO)Qw[li * lq + c];
  }
}

// Qx = X R^+ for d <= CHOL_MAX_D, right-looking, kTrsmWaves waves per 16-row
// block.  Column block K belongs to wave K % kTrsmWaves, which keeps V_K (X_K less the
// contributions of the finished blocks) in MFMA accumulators.  Step J: once
// Q_J is in LDS, each wave subtracts Q_J R_JK from its blocks K > J; the
// owner of block J + 1 does that block first and turns it into Q_{J+1} =
// V_{J+1} R_{J+1,J+1}^{-1} at once, so the chain between steps is one
// barrier and eight MFMAs while the rest of the update runs beside it.  The
// R fragments of the next step are loaded during the current one.  X (the
// whole row block, less P when P is given) passes through LDS on the way in
// and Q on the way out.
// Four waves: each applies Q_J to at most 4 of its blocks per step (two
// waves: 7), which measured 1-2% faster factorisations than two waves; seven
// waves gained nothing more.
constexpr int kTrsmWaves = 4;
constexpr int kTrsmOwn = (CHOL_MAX_D / 16 + kTrsmWaves - 1) / kTrsmWaves;  // blocks per wave

template <typename TX, typename TO>
__device__ __forceinline__ void trsm_rl_body(const TX* X, int64_t rows, int d, int64_t ldx,
                                             const TX* P, int64_t ldp,
                                             const double* __restrict__ R, int64_t ldr,
                                             const double* __restrict__ dinv, TO* Qx, int64_t ldq,
                                             const int64_t r0) {
  extern __shared__ double Qw[];
  const int nt = (d + 15) / 16, dp = nt * 16, lq = dp + 1;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  // X (- P) block -> LDS: thread t takes row r0 + (t & 15) of columns
  // t >> 4, + CS, ... (CS = threads / 16)
  constexpr int CS = 4 * kTrsmWaves;
  {
    const int xr_i = tid & 15, xc0 = tid >> 4;
    const bool rowok = r0 + xr_i < rows;
    const TX* xr = X + (rowok ? r0 + xr_i : r0);
    if (P == nullptr) {
      for (int c0 = 0; c0 < dp; c0 += CS * 16) {
        double xv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int c = c0 + xc0 + CS * u;
          xv[u] = (rowok && c < d) ? (double)xr[(int64_t)c * ldx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int c = c0 + xc0 + CS * u;
          if (c < dp) Qw[xr_i * lq + c] = xv[u];
        }
      }
    } else {
      const TX* pr = P + (rowok ? r0 + xr_i : r0);
      for (int c0 = 0; c0 < dp; c0 += CS * 8) {
        double xv[8], pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + xc0 + CS * u;
          const bool ok = rowok && c < d;
          xv[u] = ok ? (double)xr[(int64_t)c * ldx] : 0.0;
          pv[u] = ok ? (double)pr[(int64_t)c * ldp] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + xc0 + CS * u;
          if (c < dp) Qw[xr_i * lq + c] = xv[u] - pv[u];
        }
      }
    }
  }
  // B fragment (k-step q) of R_JK: R[16 J + 4 q + lk][16 K + li]; only the
  // blocks K > J are used (their rows 16 J .. 16 J + 15 are all below d)
  auto load_rf = [&](int J, int K, double* dst) {
    const int col = 16 * K + li;
    const bool ok = K > J && K < nt && col < d;
    const double* Rc = R + (int64_t)(ok ? col : 0) * ldr + 16 * J + lk;
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = ok ? Rc[4 * q] : 0.0;
  };
  auto load_inv = [&](int K, double* dst) {
    const double* T = dinv + (int64_t)(K < nt ? K : 0) * 256;
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = T[q * 4 + lk + li * 16];
  };
  // Q_K = V_K R_KK^{-1}, through this wave's columns of the LDS panel.
  auto solve = [&](int K, double4_t v, const double* tb) {
    const int kk = 16 * K;
#pragma unroll
    for (int r = 0; r < 4; ++r) Qw[acc_row_f64(lane, r) * lq + kk + li] = v[r];
    wave_sync_lds();
    double4_t r0v = {0, 0, 0, 0}, r1v = {0, 0, 0, 0};  // two short chains
    r0v = mma64(Qw[li * lq + kk + lk], tb[0], r0v);
    r1v = mma64(Qw[li * lq + kk + 4 + lk], tb[1], r1v);
    r0v = mma64(Qw[li * lq + kk + 8 + lk], tb[2], r0v);
    r1v = mma64(Qw[li * lq + kk + 12 + lk], tb[3], r1v);
    const double4_t res = r0v + r1v;
    wave_sync_lds();
#pragma unroll
    for (int r = 0; r < 4; ++r) Qw[acc_row_f64(lane, r) * lq + kk + li] = res[r];
  };
  double rf[kTrsmOwn][4], rn[kTrsmOwn][4], tb[4];
#pragma unroll
  for (int j = 0; j < kTrsmOwn; ++j) load_rf(0, w + kTrsmWaves * j, rf[j]);  // step 0
  load_inv(w, tb);  // the first block this wave solves: w (step -1 or 0)
  __syncthreads();  // X is in LDS
  double4_t V[kTrsmOwn];
#pragma unroll
  for (int j = 0; j < kTrsmOwn; ++j) {
    const int K = w + kTrsmWaves * j;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      V[j][r] = (K < nt) ? Qw[acc_row_f64(lane, r) * lq + 16 * K + li] : 0.0;
  }
  if (w == 0) solve(0, V[0], tb);           // Q_0
  if (w == 0) load_inv(kTrsmWaves, tb);     // wave w solves w, w + kTrsmWaves, ...
  for (int J = 0; J + 1 < nt; ++J) {
    __syncthreads();  // Q_J is in LDS
#pragma unroll
    for (int j = 0; j < kTrsmOwn; ++j) load_rf(J + 1, w + kTrsmWaves * j, rn[j]);
    double aq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) aq[q] = Qw[li * lq + 16 * J + 4 * q + lk];
    // the owner of block J + 1: that block first (two short MFMA chains),
    // then its solve
    const int jn = (J + 1 - w) / kTrsmWaves;  // V index of block J + 1 if this wave owns it
    if ((J + 1) % kTrsmWaves == w) {
#pragma unroll
      for (int j = 0; j < kTrsmOwn; ++j) {
        if (j != jn) continue;
        double4_t c0 = V[j], c1 = {0, 0, 0, 0};
        c0 = mma64(-aq[0], rf[j][0], c0);
        c1 = mma64(-aq[1], rf[j][1], c1);
        c0 = mma64(-aq[2], rf[j][2], c0);
        c1 = mma64(-aq[3], rf[j][3], c1);
        V[j] = c0 + c1;
        solve(J + 1, V[j], tb);
      }
      load_inv(J + 1 + kTrsmWaves, tb);
    }
    // the remaining blocks K > J + 1, k-step outermost so that consecutive
    // MFMAs are independent
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int j = 0; j < kTrsmOwn; ++j) {
        const int K = w + kTrsmWaves * j;
        if (K <= J + 1 || K >= nt) continue;
        V[j] = mma64(-aq[q], rf[j][q], V[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < kTrsmOwn; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) rf[j][q] = rn[j][q];
  }
  __syncthreads();  // every Q_K is in LDS
  {
    const int xr_i = tid & 15, xc0 = tid >> 4;
    if (r0 + xr_i < rows) {
      TO* qr = Qx + r0 + xr_i;
      for (int c = xc0; c < d; c += CS) qr[(int64_t)c * ldq] = (TO)Qw[xr_i * lq + c];
    }
  }
}

template <typename TX, typename TO>
__global__ __launch_bounds__(64 * kTrsmWaves) void trsm_rl_kernel(const TX* X, int64_t rows, int d,
                                                      int64_t ldx, const TX* P, int64_t ldp,
                                                      const double* __restrict__ R,
                                                      int64_t ldr, const double* __restrict__ dinv,
                                                      TO* Qx, int64_t ldq) {
  trsm_rl_body<TX, TO>(X, rows, d, ldx, P, ldp, R, ldr, dinv, Qx, ldq,
                       (int64_t)blockIdx.x * 16);
}

template <typename TX, typename TO>
__global__ __launch_bounds__(64) void trsm_kernel(const TX* X, int64_t rows, int d, int64_t ldx,
                                                  const double* __restrict__ R, int64_t ldr,
                                                  const double* __restrict__ dinv, TO* Qx,
                                                  int64_t ldq) {
  trsm_body<TX, TO>(X, rows, d, ldx, R, ldr, dinv, Qx, ldq, (int64_t)blockIdx.x * 16);
}

// Grouped form: workgroup b solves rows 16 bmap[b].y.. of problem bmap[b].x.
// The fp32 form keeps its row block in LDS in fp32 (its output precision)
// and loads R in batches of 8 k-steps: half the LDS and fewer registers, so
// three waves fit per SIMD instead of two.
template <typename T>
__global__ __launch_bounds__(64) void trsm_grouped_kernel(const GroupTrsm* __restrict__ descs,
                                                          const int2* __restrict__ bmap) {
  const int2 b = bmap[blockIdx.x];
  const GroupTrsm t = descs[b.x];
  constexpr bool f32 = sizeof(T) == 4;
  trsm_body<T, T, f32 ? 8 : 16, T>((const T*)t.X, t.rows, t.d, t.ldx, t.R, t.ldr, t.dinv,
                                   (T*)t.Qx, t.ldq, (int64_t)b.y * 16);
}

// Second Cholesky QR pass to first order.  For a nearly orthonormal Q1 the
// Gram matrix is G2 = I + E with small E, and chol(I + E) = I + F + O(|E|^2)
// with F = (strict upper part of E) + diag(E) / 2.  Writes B = I - F (so
// Q = Q1 B = Q1 R2^{-1} + O(|E|^2)), R2 = I + F, and raises FLAG_SECOND_PASS
// when max |E| exceeds tol (then the expansion is not accurate enough).
__global__ __launch_bounds__(256) void first_order_pass_kernel(const double* __restrict__ G2,
                                                               int d, double tol,
                                                               double* __restrict__ B,
                                                               double* __restrict__ R2,
                                                               int* __restrict__ flags) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)d * d) return;
  const int i = (int)(idx % d), j = (int)(idx / d);
  // E is symmetric: read it from the lower triangle
  const double e = (i < j ? G2[j + (int64_t)i * d] : G2[idx]) - (i == j ? 1.0 : 0.0);
  double f = 0.0;
  if (i < j) f = e;
  else if (i == j) f = 0.5 * e;
  B[idx] = (i == j ? 1.0 : 0.0) - f;
  R2[idx] = (i == j ? 1.0 : 0.0) + f;
  if (!(fabs(e) <= tol)) atomicOr(flags, FLAG_SECOND_PASS);
}

// T (cols x rows, ldt) = S^T for S (rows x cols, lds).
__global__ __launch_bounds__(256) void transpose_kernel(const double* __restrict__ S, int64_t rows,
                                                        int64_t cols, int64_t lds,
                                                        double* __restrict__ T, int64_t ldt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  T[j + i * ldt] = S[i + j * lds];
}

// S (n x n, tight) = G22 (+ shift on the diagonal) - C, and the zero block
// Z (n rows x m cols, ldz) below a factored leading block.
__global__ __launch_bounds__(256) void schur_kernel(const double* __restrict__ G22, int64_t ldg,
                                                    const double* __restrict__ C, int64_t n,
                                                    double shift, const double* shift_dev,
                                                    double* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx % n, j = idx / n;
  const double sh = shift_dev ? *shift_dev : shift;
  S[idx] = G22[i + j * ldg] + (i == j ? sh : 0.0) - C[idx];
}

__global__ __launch_bounds__(256) void zero_block_kernel(double* __restrict__ Z, int64_t rows,
                                                         int64_t cols, int64_t ldz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  Z[idx % rows + (idx / rows) * ldz] = 0.0;
}

__global__ __launch_bounds__(256) void trmm_upper_kernel(const double* __restrict__ R2,
                                                         const double* __restrict__ R1,
                                                         double* __restrict__ Ro, int d) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)d * d) return;
  const int i = (int)(idx % d), j = (int)(idx / d);
  double s = 0.0;
  for (int t = i; t <= j; ++t) s += R2[i + (int64_t)t * d] * R1[t + (int64_t)j * d];
  Ro[i + (int64_t)j * d] = s;
}

__global__ __launch_bounds__(256) void lower_from_upper_kernel(const double* __restrict__ R,
                                                               int d, double* __restrict__ L,
                                                               int64_t ldl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)d * d) return;
  const int i = (int)(idx % d), j = (int)(idx / d);
  L[i + j * ldl] = (i >= j) ? R[j + (int64_t)i * d] : 0.0;
}

__global__ __launch_bounds__(256) void trace_kernel(const double* __restrict__ G, int d,
                                                    int64_t ldg, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int j = threadIdx.x; j < d; j += 256) s += G[j + (int64_t)j * ldg];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void scale_scalar_kernel(const double* in, double c, double* out) {
  // shift = c * trace, or 1 for an all-zero panel (then every column is dependent)
  const double v = c * in[0];
  out[0] = (v > 0.0) ? v : 1.0;
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void copy_panel_kernel(const TS* __restrict__ s, int64_t lds,
                                                         TD* __restrict__ t, int64_t ldt,
                                                         int64_t rows, int64_t d) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * d) return;
  const int64_t i = idx % rows, j = idx / rows;
  t[i + j * ldt] = (TD)s[i + j * lds];
}

__global__ __launch_bounds__(256) void count_flags_kernel(const int* __restrict__ f, int d,
                                                          int* __restrict__ count) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  int mine = 0;
  for (int j = threadIdx.x; j < d; j += 256) mine += f[j] ? 1 : 0;
  if (mine) atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) count[0] += c;
}

template <typename T>
__global__ __launch_bounds__(256) void check_finite_kernel(const T* __restrict__ A, int64_t m,
                                                           int64_t n, int64_t lda,
                                                           int* __restrict__ flags) {
  const int64_t total = m * n;
  bool bad = false;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % m, j = idx / m;
    if (!__builtin_isfinite((double)A[i + j * lda])) bad = true;
  }
  if (bad) atomicOr(flags, FLAG_NONFINITE);
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Grouped first-order pass: one workgroup per problem (see the single form).
template <typename TB>
__global__ __launch_bounds__(256) void first_order_grouped_kernel(
    const GroupFirstOrder* __restrict__ descs) {
  const GroupFirstOrder g = descs[blockIdx.x];
  const int d = g.d;
  int bad = 0;
  for (int64_t idx = threadIdx.x; idx < (int64_t)d * d; idx += 256) {
    const int i = (int)(idx % d), j = (int)(idx / d);
    const double e = (i < j ? g.G2[j + (int64_t)i * d] : g.G2[idx]) - (i == j ? 1.0 : 0.0);
    double f = 0.0;
    if (i < j) f = e;
    else if (i == j) f = 0.5 * e;
    ((TB*)g.B)[idx] = (TB)((i == j ? 1.0 : 0.0) - f);
    g.R2[idx] = (i == j ? 1.0 : 0.0) + f;
    if (!(fabs(e) <= g.tol)) bad = 1;
  }
  if (bad) atomicOr(g.flags, FLAG_SECOND_PASS);
}

__global__ __launch_bounds__(256) void lower_grouped_kernel(const GroupLower* __restrict__ descs) {
  const GroupLower g = descs[blockIdx.x];
  for (int64_t idx = threadIdx.x; idx < (int64_t)g.d * g.d; idx += 256) {
    const int i = (int)(idx % g.d), j = (int)(idx / g.d);
    g.L[i + j * g.ldl] = (i >= j) ? g.R[j + (int64_t)i * g.d] : 0.0;
  }
}

__global__ __launch_bounds__(256) void zero_ints_kernel(int* __restrict__ p, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) p[idx] = 0;
}

__global__ __launch_bounds__(64) void copy_ints_kernel(const int* __restrict__ src,
                                                       int* __restrict__ dst, int n) {
  if ((int)threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

}  // namespace

hipError_t launch_cholesky_tile(const double* G, int64_t d, int64_t ldg, double shift,
                                const double* shift_dev, double tol_dep, double tol_warn,
                                double* R, int64_t ldr, double* dinv, int* col_flags,
                                int* flags, const double* odiag_src, int64_t odiag_stride,
                                hipStream_t st) {
  // the kernel addresses G and R with 32-bit byte offsets
  if (d > CHOL_MAX_D || ldg > (1 << 20) || ldr > (1 << 20)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(512), 0, st, G, (int)d, ldg, shift,
                     shift_dev, tol_dep, tol_warn, R, ldr, dinv, col_flags, flags, odiag_src,
                     odiag_stride);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* S, int64_t rows, int64_t cols, int64_t lds, double* T,
                            int64_t ldt, hipStream_t st) {
  if (rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, st, S, rows,
                     cols, lds, T, ldt);
  return hipGetLastError();
}

hipError_t launch_schur(const double* G22, int64_t ldg, const double* C, int64_t n, double shift,
                        const double* shift_dev, double* S, hipStream_t st) {
  hipLaunchKernelGGL(schur_kernel, dim3(grid_for(n * n)), dim3(256), 0, st, G22, ldg, C, n,
                     shift, shift_dev, S);
  return hipGetLastError();
}

hipError_t launch_zero_block(double* Z, int64_t rows, int64_t cols, int64_t ldz, hipStream_t st) {
  if (rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_block_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, st, Z, rows,
                     cols, ldz);
  return hipGetLastError();
}

template <typename TX, typename TO>
static hipError_t trsm_typed(const void* X, int64_t rows, int64_t d, int64_t ldx,
                             const double* R, int64_t ldr, const double* dinv, void* Qx,
                             int64_t ldq, hipStream_t st, const void* P, int64_t ldp) {
  const int nt = (int)((d + 15) / 16), dp = nt * 16;
  const size_t lds = sizeof(double) * (size_t)16 * (dp + 1);
  const int64_t blocks = (rows + 15) / 16;
  if (d <= CHOL_MAX_D) {
    hipLaunchKernelGGL((trsm_rl_kernel<TX, TO>), dim3((unsigned)blocks), dim3(64 * kTrsmWaves), lds,
                       st,
                       (const TX*)X, rows, (int)d, ldx, (const TX*)P, ldp, R, ldr, dinv,
                       (TO*)Qx, ldq);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((trsm_kernel<TX, TO>), dim3((unsigned)blocks), dim3(64), lds, st,
                     (const TX*)X, rows, (int)d, ldx, R, ldr, dinv, (TO*)Qx, ldq);
  return hipGetLastError();
}

hipError_t launch_trsm(const void* X, int64_t rows, int64_t d, int64_t ldx, const double* R,
                       int64_t ldr, const double* dinv, void* Qx, int64_t ldq, Dtype dt,
                       hipStream_t st, const void* P, int64_t ldp) {
  if (d > TRSM_MAX_D) return hipErrorInvalidValue;
  if (P != nullptr && (d > CHOL_MAX_D || ldp < rows)) return hipErrorInvalidValue;
  if (rows <= 0 || d <= 0) return hipSuccess;
  if (dt == DT_F64)
    return trsm_typed<double, double>(X, rows, d, ldx, R, ldr, dinv, Qx, ldq, st, P, ldp);
  return trsm_typed<float, float>(X, rows, d, ldx, R, ldr, dinv, Qx, ldq, st, P, ldp);
}

hipError_t launch_first_order_pass(const double* G2, int64_t d, double tol, double* B,
                                   double* R2, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(first_order_pass_kernel, dim3(grid_for(d * d)), dim3(256), 0, st, G2,
                     (int)d, tol, B, R2, flags);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(const double* R2, const double* R1, double* Rout, int64_t d,
                             hipStream_t st) {
  hipLaunchKernelGGL(trmm_upper_kernel, dim3(grid_for(d * d)), dim3(256), 0, st, R2, R1, Rout,
                     (int)d);
  return hipGetLastError();
}

hipError_t launch_lower_from_upper(const double* R, int64_t d, double* L, int64_t ldl,
                                   hipStream_t st) {
  hipLaunchKernelGGL(lower_from_upper_kernel, dim3(grid_for(d * d)), dim3(256), 0, st, R,
                     (int)d, L, ldl);
  return hipGetLastError();
}

hipError_t launch_trace(const double* G, int64_t d, int64_t ldg, double* out, hipStream_t st) {
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, st, G, (int)d, ldg, out);
  return hipGetLastError();
}

hipError_t launch_scale_scalar(const double* in, double c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(scale_scalar_kernel, dim3(1), dim3(1), 0, st, in, c, out);
  return hipGetLastError();
}

hipError_t launch_copy_panel(const void* src, Dtype s_t, int64_t ld_src, void* dst, Dtype d_t,
                             int64_t ld_dst, int64_t rows, int64_t d, hipStream_t st) {
  const unsigned g = grid_for(rows * d);
  if (rows * d <= 0) return hipSuccess;
  if (s_t == DT_F32 && d_t == DT_F64)
    hipLaunchKernelGGL((copy_panel_kernel<float, double>), dim3(g), dim3(256), 0, st,
                       (const float*)src, ld_src, (double*)dst, ld_dst, rows, d);
  else if (s_t == DT_F64 && d_t == DT_F32)
    hipLaunchKernelGGL((copy_panel_kernel<double, float>), dim3(g), dim3(256), 0, st,
                       (const double*)src, ld_src, (float*)dst, ld_dst, rows, d);
  else if (s_t == DT_F64)
    hipLaunchKernelGGL((copy_panel_kernel<double, double>), dim3(g), dim3(256), 0, st,
                       (const double*)src, ld_src, (double*)dst, ld_dst, rows, d);
  else
    hipLaunchKernelGGL((copy_panel_kernel<float, float>), dim3(g), dim3(256), 0, st,
                       (const float*)src, ld_src, (float*)dst, ld_dst, rows, d);
  return hipGetLastError();
}

hipError_t launch_count_flags(const int* col_flags, int64_t d, int* count, hipStream_t st) {
  hipLaunchKernelGGL(count_flags_kernel, dim3(1), dim3(256), 0, st, col_flags, (int)d, count);
  return hipGetLastError();
}

hipError_t launch_check_finite(const void* A, int64_t m, int64_t n, int64_t lda, Dtype dt,
                               int* flags, hipStream_t st) {
  const int64_t total = m * n;
  if (total <= 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>(4096, (total + 255) / 256);
  if (dt == DT_F64)
    hipLaunchKernelGGL(check_finite_kernel<double>, dim3(g), dim3(256), 0, st,
                       (const double*)A, m, n, lda, flags);
  else
    hipLaunchKernelGGL(check_finite_kernel<float>, dim3(g), dim3(256), 0, st, (const float*)A,
                       m, n, lda, flags);
  return hipGetLastError();
}

hipError_t launch_cholesky_grouped(const GroupChol* descs, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(cholesky_grouped_kernel, dim3(count), dim3(512), 0, st, descs);
  return hipGetLastError();
}

void trsm_grouped_blocks(const GroupTrsm& t, int idx, std::vector<int2>& out) {
  for (int64_t r = 0; r < (t.rows + 15) / 16; ++r) out.push_back(int2{idx, (int)r});
}

hipError_t launch_trsm_grouped(Dtype dt, const GroupTrsm* descs, const int2* bmap,
                               int64_t nblocks, int dmax, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const int dp = (dmax + 15) / 16 * 16;
  const size_t lds = (size_t)16 * (dp + 1) * (dt == DT_F64 ? sizeof(double) : sizeof(float));
  if (dt == DT_F64)
    hipLaunchKernelGGL(trsm_grouped_kernel<double>, dim3((unsigned)nblocks), dim3(64), lds, st,
                       descs, bmap);
  else
    hipLaunchKernelGGL(trsm_grouped_kernel<float>, dim3((unsigned)nblocks), dim3(64), lds, st,
                       descs, bmap);
  return hipGetLastError();
}

hipError_t launch_first_order_grouped(Dtype dt, const GroupFirstOrder* descs, int count,
                                      hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (dt == DT_F64)
    hipLaunchKernelGGL(first_order_grouped_kernel<double>, dim3(count), dim3(256), 0, st, descs);
  else
    hipLaunchKernelGGL(first_order_grouped_kernel<float>, dim3(count), dim3(256), 0, st, descs);
  return hipGetLastError();
}

hipError_t launch_lower_grouped(const GroupLower* descs, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(lower_grouped_kernel, dim3(count), dim3(256), 0, st, descs);
  return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_ints_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_copy_ints(const int* src, int* dst, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_ints_kernel, dim3(1), dim3(64), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace rqlp

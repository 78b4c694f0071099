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
// place into its lower Cholesky factor L_JJ, and write the inverse of that
// factor into dgi (and R_JJ^{-1} = L_JJ^{-T} into dinv).  Run by one wave:
// lanes 0..15 own one row each; pivots travel by readlane, so the chain of
// 16 pivots needs no LDS round trips.  1/l_ss comes from rsqrt (no divide on
// the chain).  A dependent pivot (<= tol_dep of the column's original
// diagonal, or non-finite) gives a zero column of L and a zero row of the
// inverse.
__device__ __forceinline__ void factor_diag_tile(double (*dg)[17], double (*dgi)[17], double* invd,
                                 const double* odiag, int J, int d, double tol_dep,
                                 double tol_warn, int* __restrict__ col_flags,
                                 double* __restrict__ dinv, int* sflag) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15;
  int bits = 0;
  {
    double a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = dg[i][c];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const double piv = readlane_d(a[s], s);
      const int gj = 16 * J + s;
      const double orig = odiag[gj];
      const bool nonfinite = !__builtin_isfinite(piv);
      const bool dep = nonfinite || !(piv > tol_dep * orig);
      if (gj < d) {
        if (nonfinite) bits |= FLAG_NONFINITE;
        if (dep) bits |= FLAG_NONPOS_PIVOT;
        if (!dep && piv < tol_warn * orig) bits |= FLAG_SECOND_PASS;
        if (col_flags != nullptr && lane == 0) col_flags[gj] = dep ? 1 : 0;
      }
      const double y = dep ? 0.0 : rsqrt(piv);  // 1 / l_ss
      const double lss = piv * y;
      if (lane == 0) invd[s] = y;
      const double lis = (i > s) ? a[s] * y : ((i == s) ? lss : 0.0);
      a[s] = lis;
#pragma unroll
      for (int j = s + 1; j < 16; ++j) {
        const double ljs = readlane_d(lis, j);
        a[j] = fma(-lis, ljs, a[j]);
      }
    }
    if (lane < 16) {
#pragma unroll
      for (int c = 0; c < 16; ++c) dg[i][c] = (c > i) ? 0.0 : a[c];
    }
    wave_sync_lds();
  }
  // Inverse by forward substitution, one column per lane:
  // X[r][c] = (delta_rc - sum_{t<r} L[r][t] X[t][c]) / L[r][r]  (0 if dependent).
  const int c = lane & 15;
  double x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double v0 = (r == c) ? 1.0 : 0.0, v1 = 0.0;
#pragma unroll
    for (int t = 0; t < r; t += 2) {
      v0 = fma(-dg[r][t], x[t], v0);
      if (t + 1 < r) v1 = fma(-dg[r][t + 1], x[t + 1], v1);
    }
    x[r] = (v0 + v1) * invd[r];
  }
  if (lane < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      dgi[r][c] = x[r];
      dinv[(int64_t)J * 256 + c + r * 16] = x[r];  // (L^{-1})^T, column-major block
    }
  }
  if (lane == 0 && bits) *sflag |= bits;
}

// Tile-wave part of the Cholesky kernel: holds its lower tiles of G in MFMA
// layout, applies panel solves and trailing updates, hands each updated
// diagonal tile to the factor wave, and finally writes its part of R.
__device__ __forceinline__ void chol_tile_wave(
    const double* __restrict__ G, int d, int64_t ldg, double sh, double (*dg)[17],
    double (*dgi)[17], double (*pan)[17], int* ready, int wave, double* __restrict__ R,
    int64_t ldr) {
  const int lane = threadIdx.x & 63;
  const int nt = (d + 15) / 16;
  const int T = nt * (nt + 1) / 2;
  const int twi = tile_wave_idx(wave);
  double4_t acc[kCholSlots];
  int tI[kCholSlots], tJ[kCholSlots];
#pragma unroll
  for (int s = 0; s < kCholSlots; ++s) {
    const int t = twi + kTileWaves * s;
    tI[s] = -1;
    tJ[s] = -1;
    acc[s] = double4_t{0, 0, 0, 0};
    if (t < T) {
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      const int Jt = t - I * (I + 1) / 2;
      tI[s] = I;
      tJ[s] = Jt;
      const int col = 16 * Jt + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * I + acc_row_f64(lane, r);
        double v;
        if (row < d && col < d) {
          v = G[row + (int64_t)col * ldg];
          if (row == col) v += sh;
        } else {
          v = (row == col) ? 1.0 : 0.0;
        }
        acc[s][r] = v;
      }
    }
  }
  // Diagonal tile J lives at t = J (J + 3) / 2.
  auto owner = [&](int J) { return tile_wave_id((J * (J + 3) / 2) % kTileWaves); };
  auto slot = [&](int J) { return (J * (J + 3) / 2) / kTileWaves; };
  auto publish = [&](int J, double4_t c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) dg[acc_row_f64(lane, r)][lane & 15] = c[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) __hip_atomic_store(ready, J, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  __syncthreads();  // odiag and the flags are initialised
  if (wave == owner(0)) {
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s)
      if (s == slot(0)) publish(0, acc[s]);
  }
  for (int J = 0; J < nt; ++J) {
    __syncthreads();  // L_JJ and its inverse are ready
    // Panel: L_IJ = G_IJ L_JJ^{-T} for the tiles below the diagonal.
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s) {
      if (tJ[s] != J) continue;
      const int I = tI[s];
      if (I == J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[s][r] = dg[acc_row_f64(lane, r)][lane & 15];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[16 * I + acc_row_f64(lane, r)][lane & 15] = acc[s][r];
        wave_sync_lds();
        double4_t res = {0, 0, 0, 0};
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
          const double a = pan[16 * I + (lane & 15)][kq * 4 + (lane >> 4)];
          const double b = dgi[lane & 15][kq * 4 + (lane >> 4)];
          res = mma64(a, b, res);
        }
        acc[s] = res;
        wave_sync_lds();
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[16 * I + acc_row_f64(lane, r)][lane & 15] = res[r];
      }
    }
    __syncthreads();  // panel J is ready
    // Lookahead: bring tile (J+1, J+1) up to date and hand it to wave 0,
    // then apply the rest of the trailing update.
    const bool ahead = (J + 1 < nt) && (wave == owner(J + 1));
    if (ahead) {
#pragma unroll
      for (int s = 0; s < kCholSlots; ++s) {
        if (s != slot(J + 1)) continue;
        double4_t c = acc[s];
        const int I = J + 1;
#pragma unroll
        for (int kq = 0; kq < 4; ++kq) {
          const double a = pan[16 * I + (lane & 15)][kq * 4 + (lane >> 4)];
          c = mma64(-a, a, c);
        }
        acc[s] = c;
        publish(J + 1, c);
      }
    }
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s) {
      const int I = tI[s], K = tJ[s];
      if (K <= J) continue;
      if (ahead && I == J + 1 && K == J + 1) continue;
      double4_t c = acc[s];
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) {
        const double a = pan[16 * I + (lane & 15)][kq * 4 + (lane >> 4)];
        const double b = pan[16 * K + (lane & 15)][kq * 4 + (lane >> 4)];
        c = mma64(-a, b, c);
      }
      acc[s] = c;
    }
  }
  // R = L^T (upper), with explicit zeros in the lower triangle.
#pragma unroll
  for (int s = 0; s < kCholSlots; ++s) {
    if (tI[s] < 0) continue;
    const int I = tI[s], Jt = tJ[s];
    const int col = 16 * Jt + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * I + acc_row_f64(lane, r);
      if (row < d && col < d) {
        R[col + (int64_t)row * ldr] = acc[s][r];
        if (I > Jt) R[row + (int64_t)col * ldr] = 0.0;
      }
    }
  }
}

// Cholesky of G + shift I (d <= 224) on one workgroup of 8 waves.  Wave 0
// factors each 16 x 16 diagonal tile as soon as its owner publishes it
// (an LDS flag; the owner never waits on wave 0, so the wait always ends);
// wave 4 shares wave 0's SIMD and stays idle so no MFMA issue competes with
// the pivot chain; the six other waves hold the tiles.
__device__ __forceinline__ void cholesky_body(
    const double* __restrict__ G, int d, int64_t ldg, double shift,
    const double* __restrict__ shift_dev, double tol_dep, double tol_warn,
    double* __restrict__ R, int64_t ldr, double* __restrict__ dinv,
    int* __restrict__ col_flags, int* __restrict__ flags,
    const double* __restrict__ odiag_src, int64_t odiag_stride) {
  __shared__ double dg[16][17];
  __shared__ double dgi[16][17];
  __shared__ double invd[16];
  __shared__ double pan[CHOL_MAX_D][17];
  __shared__ double odiag[CHOL_MAX_D];
  __shared__ int sflag;
  __shared__ int ready;  // index of the last diagonal tile published in dg

  const int nt = (d + 15) / 16;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double sh = (shift_dev != nullptr) ? *shift_dev : shift;
  // Pivots are judged against the original diagonal (of the whole matrix
  // when this call factors a trailing Schur complement).
  for (int j = tid; j < CHOL_MAX_D; j += blockDim.x)
    odiag[j] = (j >= d) ? 1.0
               : (odiag_src ? odiag_src[(int64_t)j * odiag_stride] + sh
                            : G[j + (int64_t)j * ldg] + sh);
  if (tid == 0) {
    sflag = 0;
    ready = -1;
  }
  if (wave == 0) {
    __syncthreads();
    for (int J = 0; J < nt; ++J) {
      while (__hip_atomic_load(&ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < J)
        __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      factor_diag_tile(dg, dgi, invd, odiag, J, d, tol_dep, tol_warn, col_flags, dinv, &sflag);
      __syncthreads();  // L_JJ and its inverse are ready
      __syncthreads();  // panel J is ready
    }
  } else if (wave == 4) {
    __syncthreads();
    for (int J = 0; J < nt; ++J) {
      __syncthreads();
      __syncthreads();
    }
  } else {
    chol_tile_wave(G, d, ldg, sh, dg, dgi, pan, &ready, wave, R, ldr);
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
// rows: for each 16-column block J it forms V_J = X_J - sum_{K<J} Q_K R_KJ
// with MFMA (A fragments from its finished columns kept in LDS, B fragments
// of R read from L2), then Q_J = V_J R_JJ^{-1}.  The k-steps run in batches
// of 16 whose next batch of fragments is loaded while the current batch's
// MFMAs execute (two accumulator chains).  No workgroup barriers; X and Q
// move through the wave's LDS panel so global accesses stay coalesced.  X
// and Qx may be the same array (each wave reads a block of its rows before
// overwriting it).
template <typename TX, typename TO>
__device__ __forceinline__ void trsm_body(const TX* X, int64_t rows, int d, int64_t ldx,
                                          const double* __restrict__ R, int64_t ldr,
                                          const double* __restrict__ dinv, TO* Qx, int64_t ldq,
                                          const int64_t r0) {
  extern __shared__ double Qw[];
  constexpr int B = 16;
  const int nt = (d + 15) / 16, dp = nt * 16, lq = dp + 1;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  for (int J = 0; J < nt; ++J) {
    const int kk = 16 * J;
    const int colR = kk + li;
    const bool colok = colR < d;
    const double* Rc = R + (int64_t)(colok ? colR : 0) * ldr + lk;
    const int nk = 4 * J;
    double bc[B], bn[B];
#pragma unroll
    for (int q = 0; q < B; ++q) bc[q] = (q < nk && colok) ? Rc[q * 4] : 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = lane + 64 * e;
      const int rr = idx & 15, cc = idx >> 4;
      const int64_t row = r0 + rr;
      const int col = kk + cc;
      Qw[rr * lq + col] = (row < rows && col < d) ? (double)X[row + (int64_t)col * ldx] : 0.0;
    }
    wave_sync_lds();
    double4_t acc0, acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc0[r] = Qw[acc_row_f64(lane, r) * lq + kk + li];
    for (int base = 0; base < nk; base += B) {
      const int nb = base + B;
#pragma unroll
      for (int q = 0; q < B; ++q) bn[q] = (nb + q < nk && colok) ? Rc[(nb + q) * 4] : 0.0;
      double ac[B];
#pragma unroll
      for (int q = 0; q < B; ++q) ac[q] = (base + q < nk) ? Qw[li * lq + (base + q) * 4 + lk] : 0.0;
#pragma unroll
      for (int q = 0; q < B; q += 2) {
        acc0 = mma64(-ac[q], bc[q], acc0);
        acc1 = mma64(-ac[q + 1], bc[q + 1], acc1);
      }
#pragma unroll
      for (int q = 0; q < B; ++q) bc[q] = bn[q];
    }
    acc0 += acc1;
    double tb[4];
    const double* T = dinv + (int64_t)J * 256;
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) tb[q4] = T[q4 * 4 + lk + li * 16];
#pragma unroll
    for (int r = 0; r < 4; ++r) Qw[acc_row_f64(lane, r) * lq + kk + li] = acc0[r];
    wave_sync_lds();
    double4_t res = {0, 0, 0, 0};
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) res = mma64(Qw[li * lq + kk + q4 * 4 + lk], tb[q4], res);
    wave_sync_lds();
#pragma unroll
    for (int r = 0; r < 4; ++r) Qw[acc_row_f64(lane, r) * lq + kk + li] = res[r];
    wave_sync_lds();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = lane + 64 * e;
      const int rr = idx & 15, cc = idx >> 4;
      const int64_t row = r0 + rr;
      const int col = kk + cc;
      if (row < rows && col < d) Qx[row + (int64_t)col * ldq] = (TO)Qw[rr * lq + col];
    }
  }
}

template <typename TX, typename TO>
__global__ __launch_bounds__(64) void trsm_kernel(const TX* X, int64_t rows, int d, int64_t ldx,
                                                  const double* __restrict__ R, int64_t ldr,
                                                  const double* __restrict__ dinv, TO* Qx,
                                                  int64_t ldq) {
  trsm_body<TX, TO>(X, rows, d, ldx, R, ldr, dinv, Qx, ldq, (int64_t)blockIdx.x * 16);
}

// Grouped form: workgroup b solves rows 16 bmap[b].y.. of problem bmap[b].x.
template <typename T>
__global__ __launch_bounds__(64) void trsm_grouped_kernel(const GroupTrsm* __restrict__ descs,
                                                          const int2* __restrict__ bmap) {
  const int2 b = bmap[blockIdx.x];
  const GroupTrsm t = descs[b.x];
  trsm_body<T, T>((const T*)t.X, t.rows, t.d, t.ldx, t.R, t.ldr, t.dinv, (T*)t.Qx, t.ldq,
                  (int64_t)b.y * 16);
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

}  // namespace

hipError_t launch_cholesky_tile(const double* G, int64_t d, int64_t ldg, double shift,
                                const double* shift_dev, double tol_dep, double tol_warn,
                                double* R, int64_t ldr, double* dinv, int* col_flags,
                                int* flags, const double* odiag_src, int64_t odiag_stride,
                                hipStream_t st) {
  if (d > CHOL_MAX_D) return hipErrorInvalidValue;
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
                             int64_t ldq, hipStream_t st) {
  const int nt = (int)((d + 15) / 16), dp = nt * 16;
  const size_t lds = sizeof(double) * (size_t)16 * (dp + 1);
  const int64_t blocks = (rows + 15) / 16;
  hipLaunchKernelGGL((trsm_kernel<TX, TO>), dim3((unsigned)blocks), dim3(64), lds, st,
                     (const TX*)X, rows, (int)d, ldx, R, ldr, dinv, (TO*)Qx, ldq);
  return hipGetLastError();
}

hipError_t launch_trsm(const void* X, int64_t rows, int64_t d, int64_t ldx, const double* R,
                       int64_t ldr, const double* dinv, void* Qx, int64_t ldq, Dtype dt,
                       hipStream_t st) {
  if (d > TRSM_MAX_D) return hipErrorInvalidValue;
  if (rows <= 0 || d <= 0) return hipSuccess;
  if (dt == DT_F64)
    return trsm_typed<double, double>(X, rows, d, ldx, R, ldr, dinv, Qx, ldq, st);
  return trsm_typed<float, float>(X, rows, d, ldx, R, ldr, dinv, Qx, ldq, st);
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
  const size_t lds = (size_t)16 * (dp + 1) * sizeof(double);
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

}  // namespace rqlp

// The learned power-iteration predictor and the a-posteriori error judge.
//
// Features: the singular values of the 64-column sketch Y = A^T Omega[:, :64]
// (the leading Philox columns of the method's own sketch) from the
// eigenvalues of its fp64 Gram matrix (tridiagonal reduction and bisection
// in one workgroup),
// turned into 65 numbers: log10(sigma_i / sigma_1) clamped to [-6, 0] and
// divided by 6 (i = 1..64), then k / 256.
//
// MLP (fp32): 65 -> 128 (ReLU) -> 128 (ReLU) -> 6 logits (q = 0..4 and
// "more than 4").  Parameters are one flat vector [W1 b1 W2 b2 W3 b3], each
// W (fan_in x fan_out) stored column by column.  Activations are row-major
// (one sample's values contiguous).  Training is softmax cross-entropy with
// Adam; every reduction runs in a fixed order, so training is reproducible
// bit for bit.
//
// Error judge: sums of squares in fp64 with a fixed two-level reduction.
#include <algorithm>
#include <cmath>

#include "randqlp.h"
#include "rqlp_internal.h"

namespace rqlp {
namespace {

constexpr int kNs = 64;            // sketch columns read by the predictor
constexpr int kFeatThreads = 256;

// LDS writes of this wave are visible to its own later reads
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// a double from another lane through DPP (two 32-bit moves); lanes whose
// source is out of range or masked off get 0
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROW_MASK, BANK_MASK, true);
  const int hi =
      __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROW_MASK, BANK_MASK, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave, on every lane: a prefix sum within each
// row of 16 lanes (row_shr 1, 2, 4, 8), then the row totals carried across
// rows (row_bcast 15 and 31) into lane 63, which is read back.
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0x111, 0xf, 0xf>(v);  // row_shr:1
  v += dpp_d<0x112, 0xf, 0xf>(v);  // row_shr:2
  v += dpp_d<0x114, 0xf, 0xf>(v);  // row_shr:4
  v += dpp_d<0x118, 0xf, 0xf>(v);  // row_shr:8
  v += dpp_d<0x142, 0xa, 0xf>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc, 0xf>(v);  // row_bcast:31 into rows 2 and 3
  return readlane_d(v, 63);
}

// ---------------------------------------------------------------- features
// Eigenvalues of the symmetric 64 x 64 G (column-major, ldg) in one
// workgroup: Householder reduction to tridiagonal form (62 reflections,
// each a reduction for the vector, a symmetric matrix-vector product and a
// rank-2 update, the 64 columns shared by the four waves), then
// bisection with Sturm
// counts, four threads per eigenvalue (the quad for eigenvalue i finds the
// i-th smallest, so the order comes for free; each round cuts its interval
// to a fifth).  Both steps are backward stable: the
// eigenvalues carry an absolute error of a few units of roundoff times
// ||G||, which resolves sigma_i / sigma_1 = sqrt(lambda_i / lambda_1) well
// below the features' clamp at 1e-6.  Then the features as described above.
__device__ __forceinline__ int sturm_count(const double* dg, const double* eo2, int n,
                                           double x, double pivmin) {
  // number of eigenvalues of the tridiagonal (dg, off-diagonal^2 eo2) below x:
  // the negative pivots of T - x I = L D L^T.  1 / q is the hardware
  // reciprocal refined by one Newton step (a relative error of a few units
  // of roundoff, which the count tolerates as it does the rounding of the
  // other operations).
  int cnt = 0;
  double q = dg[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int j = 1; j < n; ++j) {
    const double r0 = __builtin_amdgcn_rcp(q);
    const double r = fma(r0, fma(-q, r0, 1.0), r0);
    q = (dg[j] - x) - eo2[j - 1] * r;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__global__ __launch_bounds__(kFeatThreads) void features_kernel(const double* __restrict__ G,
                                                                 int64_t ldg, int k,
                                                                 float* __restrict__ feat) {
  __shared__ double a[kNs][kNs + 1];
  __shared__ double dg[kNs], eo2[kNs];
  __shared__ double lam[kNs];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kNs * kNs; e += kFeatThreads) {
    const int i = e % kNs, j = e / kNs;
    a[i][j] = G[i + (int64_t)j * ldg];
  }
  __syncthreads();
  // Householder reduction to tridiagonal form by the four waves together:
  // lane i of wave w keeps A[i][16 w .. 16 w + 15] in registers.  Step kk
  // reflects rows r0 = kk + 1 .. 63 of column kk: v = x - alpha e_r0 with
  // alpha = -sign(x_r0) ||x||, beta = 2 / v^T v, p = beta A v,
  // w = p - (beta / 2) (p^T v) v, A -= v w^T + w v^T.  v and w vanish
  // outside rows r0 .., so the full-width update leaves the finished part
  // alone.  The wave holding column kk puts it in LDS (barrier); every wave
  // then forms v (the reductions over the 64 lanes give every wave the same
  // values), its share of A v over its 16 columns goes to LDS (barrier),
  // and each wave adds the four shares in the same order and updates its
  // columns.  The diagonal entry a[kk][kk] is final after step kk; the new
  // off-diagonal entry is alpha.  (With one wave doing all of it the kernel
  // took 182 us, with the four 148 us: the reductions, the two barriers and
  // the LDS round trips of each step remain on its critical path.)
  __shared__ double xcol[2][kNs];         // column kk, by step parity
  __shared__ double part[2][4][kNs];      // the waves' shares of A v
  __shared__ double wcol[4][kNs];         // w, one copy per wave
  static_assert(kFeatThreads == 4 * kNs, "four waves of 64 lanes");
  {
    constexpr int CW = kNs / 4;  // columns per wave
    double ar[CW];
#pragma unroll
    for (int jj = 0; jj < CW; ++jj) ar[jj] = a[lane][CW * wave + jj];
    for (int kk = 0; kk < kNs - 2; ++kk) {
      const int r0 = kk + 1, par = kk & 1;
      if (wave == kk / CW) {
        const int oc = kk % CW;
        double c = 0.0;
#pragma unroll
        for (int jj = 0; jj < CW; ++jj) c = (jj == oc) ? ar[jj] : c;
        xcol[par][lane] = c;
      }
      __syncthreads();
      const double* xb = xcol[par];
      const bool mine = lane >= r0;
      const double x = mine ? xb[lane] : 0.0;
      const double ss = wave_sum_d(x * x);
      const double x0 = xb[r0];
      const double nrm = sqrt(ss);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double vv = lane == r0 ? x0 - alpha : x;
      const double v2 = wave_sum_d(vv * vv);
      const double beta = v2 > 0.0 ? 2.0 / v2 : 0.0;
      if (tid == 0) {
        dg[kk] = xb[kk];
        const double o = v2 > 0.0 ? alpha : x0;
        eo2[kk] = o * o;
      }
      double vc[CW];
#pragma unroll
      for (int jj = 0; jj < CW; ++jj) {
        const int j = CW * wave + jj;
        vc[jj] = j < r0 ? 0.0 : (j == r0 ? x0 - alpha : xb[j]);
      }
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int jj = 0; jj < CW; jj += 4) {
        s0 = fma(ar[jj], vc[jj], s0);
        s1 = fma(ar[jj + 1], vc[jj + 1], s1);
        s2 = fma(ar[jj + 2], vc[jj + 2], s2);
        s3 = fma(ar[jj + 3], vc[jj + 3], s3);
      }
      part[par][wave][lane] = (s0 + s1) + (s2 + s3);
      __syncthreads();
      const double pf = (part[par][0][lane] + part[par][1][lane]) +
                        (part[par][2][lane] + part[par][3][lane]);
      const double pp = mine ? beta * pf : 0.0;
      const double pv = wave_sum_d(pp * vv);
      const double wv = pp - 0.5 * beta * pv * vv;
      wcol[wave][lane] = wv;
      wave_sync_lds();
#pragma unroll
      for (int jj = 0; jj < CW; ++jj) ar[jj] -= vv * wcol[wave][CW * wave + jj] + wv * vc[jj];
      wave_sync_lds();
    }
    if (wave == 3) {
      if (lane == kNs - 2) dg[kNs - 2] = ar[CW - 2];
      if (lane == kNs - 1) {
        dg[kNs - 1] = ar[CW - 1];
        eo2[kNs - 2] = ar[CW - 2] * ar[CW - 2];
        eo2[kNs - 1] = 0.0;
      }
    }
  }
  __syncthreads();
  {
    // Gershgorin interval and a pivot floor relative to ||T||
    double lo = 1e300, hi = -1e300, tn = 0.0, dmax = 0.0;
    for (int j = 0; j < kNs; ++j) {
      const double r = (j > 0 ? sqrt(eo2[j - 1]) : 0.0) + (j + 1 < kNs ? sqrt(eo2[j]) : 0.0);
      lo = fmin(lo, dg[j] - r);
      hi = fmax(hi, dg[j] + r);
      tn = fmax(tn, fabs(dg[j]) + r);
      dmax = fmax(dmax, dg[j]);
    }
    const double pivmin = fmax(tn, 1e-300) * 1e-300 + 1e-300;
    const double tol = 4.0 * 2.220446049250313e-16 * fmax(tn, 1e-300);
    // Below 1e-13 lambda_max (lambda_max >= every diagonal entry) sigma_i /
    // sigma_1 < 1e-6 and the feature is clamped; above it a relative width
    // of 2^-24 is finer than the float features resolve.
    const double floor_clamp = 1e-13 * dmax;
    // Four threads per eigenvalue (a quad of lanes): each iteration they
    // count at the four interior points of five equal parts of [l, h], and
    // all four keep the part that holds eigenvalue e (the e-th smallest:
    // count(l) <= e < count(h)).
    const int e = tid >> 2, sub = tid & 3;
    double l = lo, h = hi;
    for (int it = 0; it < 64; ++it) {
      const double wdt = h - l;
      const bool done = wdt <= fmax(tol, 0x1p-24 * fmax(fabs(l), fabs(h))) || h <= floor_clamp;
      if (__all(done)) break;
      const double x = l + wdt * (double)(sub + 1) * 0.2;
      const int c = sturm_count(dg, eo2, kNs, x, pivmin);
      const int c0 = __shfl(c, (lane & ~3) + 0), c1 = __shfl(c, (lane & ~3) + 1);
      const int c2 = __shfl(c, (lane & ~3) + 2), c3 = __shfl(c, (lane & ~3) + 3);
      const double x0 = __shfl(x, (lane & ~3) + 0), x1 = __shfl(x, (lane & ~3) + 1);
      const double x2 = __shfl(x, (lane & ~3) + 2), x3 = __shfl(x, (lane & ~3) + 3);
      if (!done) {
        double nl = l, nh = h;
        if (c0 > e) nh = x0;
        else if (c1 > e) { nl = x0; nh = x1; }
        else if (c2 > e) { nl = x1; nh = x2; }
        else if (c3 > e) { nl = x2; nh = x3; }
        else nl = x3;
        l = nl;
        h = nh;
      }
    }
    if (sub == 0) lam[e] = sqrt(fmax(0.5 * (l + h), 0.0));
  }
  __syncthreads();
  if (tid < kNs) {
    const double s1 = lam[kNs - 1];   // the largest (ascending order)
    const double v0 = lam[tid];
    float f = -1.0f;
    if (s1 > 0.0 && v0 > 0.0) {
      const double lg = log10(v0 / s1);
      f = (float)(fmin(fmax(lg, -6.0), 0.0) / 6.0);
    }
    feat[kNs - 1 - tid] = f;            // descending order
  }
  if (tid == 0) feat[kNs] = (float)k / 256.0f;
}

// -------------------------------------------------------------------- MLP
// Y (B x nout, row-major) = act(X (B x nin, row-major, ldx) W + bias).
__global__ __launch_bounds__(256) void linear_forward_kernel(const float* __restrict__ X,
                                                             int ldx, const float* __restrict__ W,
                                                             const float* __restrict__ bias,
                                                             float* __restrict__ Y, int B, int nin,
                                                             int nout, int relu) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * nout) return;
  const int b = (int)(idx / nout), j = (int)(idx % nout);
  const float* x = X + (int64_t)b * ldx;
  const float* w = W + (int64_t)j * nin;
  float s = bias[j];
  for (int i = 0; i < nin; ++i) s = fmaf(x[i], w[i], s);
  Y[idx] = relu ? fmaxf(s, 0.0f) : s;
}

// Softmax cross-entropy: loss[b] = -log softmax(Z_b)[y_b] and
// dZ = (softmax(Z) - onehot(y)) * inv_batch.
__global__ __launch_bounds__(256) void softmax_xent_kernel(const float* __restrict__ Z,
                                                           const int* __restrict__ y, int B,
                                                           int C, float inv_batch,
                                                           float* __restrict__ dZ,
                                                           float* __restrict__ loss) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float* z = Z + (int64_t)b * C;
  float mx = z[0];
  for (int c = 1; c < C; ++c) mx = fmaxf(mx, z[c]);
  float sum = 0.0f;
  for (int c = 0; c < C; ++c) sum += expf(z[c] - mx);
  const int t = y[b];
  loss[b] = logf(sum) - (z[t] - mx);
  if (dZ) {
    for (int c = 0; c < C; ++c) {
      const float pc = expf(z[c] - mx) / sum;
      dZ[(int64_t)b * C + c] = (pc - (c == t ? 1.0f : 0.0f)) * inv_batch;
    }
  }
}

// dX (B x nin) = (dY (B x nout) W^T) masked by H > 0 (H: the layer input,
// itself a ReLU output).
__global__ __launch_bounds__(256) void linear_backward_input_kernel(
    const float* __restrict__ dY, const float* __restrict__ W, const float* __restrict__ H,
    float* __restrict__ dX, int B, int nin, int nout) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * nin) return;
  const int b = (int)(idx / nin), i = (int)(idx % nin);
  const float* g = dY + (int64_t)b * nout;
  float s = 0.0f;
  for (int j = 0; j < nout; ++j) s = fmaf(g[j], W[i + (int64_t)j * nin], s);
  dX[idx] = H[idx] > 0.0f ? s : 0.0f;
}

// dW (nin x nout, column-major) = X^T dY and db = column sums of dY, summed
// over the batch in order.
__global__ __launch_bounds__(256) void linear_backward_weight_kernel(
    const float* __restrict__ X, int ldx, const float* __restrict__ dY, float* __restrict__ dW,
    float* __restrict__ db, int B, int nin, int nout) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nw = (int64_t)nin * nout;
  if (idx < nw) {
    const int i = (int)(idx % nin), j = (int)(idx / nin);
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s = fmaf(X[(int64_t)b * ldx + i], dY[(int64_t)b * nout + j], s);
    dW[idx] = s;
  } else if (idx < nw + nout) {
    const int j = (int)(idx - nw);
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dY[(int64_t)b * nout + j];
    db[j] = s;
  }
}

// Adam (Kingma & Ba), step t >= 1, bias-corrected.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ theta,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t count, float lr, float beta1,
                                                   float beta2, float eps, float corr1,
                                                   float corr2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / corr1, vh = vi / corr2;
  theta[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Minibatch gather: rows idx(b) = (a * (start + b) + c) mod N of X and y.
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ X,
                                                     const int* __restrict__ y, int64_t N,
                                                     int64_t a, int64_t c, int64_t start, int B,
                                                     int nin, float* __restrict__ Xb,
                                                     int* __restrict__ yb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * nin) return;
  const int b = (int)(idx / nin), i = (int)(idx % nin);
  // a, c < N and N < 2^31, so the products stay within 64 bits
  const int64_t r = (a * ((start + b) % N) + c) % N;
  Xb[idx] = X[r * nin + i];
  if (i == 0) yb[b] = y[r];
}

// Deterministic sum of n floats (one workgroup, fixed order).
__global__ __launch_bounds__(256) void sum_kernel(const float* __restrict__ x, int64_t n,
                                                  float scale, float* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)(red[0] * scale);
}

// Predicted class of one feature vector x (RQLP_MLP_INPUTS floats): the
// three layers of the MLP with the parameters th = [W1 b1 W2 b2 W3 b3] (each
// W row-major per output unit), in the summation order of
// linear_forward_kernel, then the argmax of the logits (ties to the lower
// class); one workgroup of RQLP_MLP_HIDDEN threads.  out (optional) gets the
// activations h1, h2 and the logits.
constexpr int kNI = RQLP_MLP_INPUTS, kNH = RQLP_MLP_HIDDEN, kNC = RQLP_MLP_CLASSES;
static_assert(kNI <= kNH && kNC <= kNH, "one thread per hidden unit covers the inputs and logits");
// The three layers on xs (shared, kNI floats) into z (shared, kNC logits);
// the whole workgroup of kNH threads takes part.  h1, h2: shared scratch.
__device__ void mlp_logits(const float* __restrict__ th, const float* xs, float* h1, float* h2,
                           float* z) {
  constexpr int oW1 = 0, oB1 = oW1 + kNI * kNH, oW2 = oB1 + kNH, oB2 = oW2 + kNH * kNH,
                oW3 = oB2 + kNH, oB3 = oW3 + kNH * kNC;
  const int t = threadIdx.x;
  {
    const float* w = th + oW1 + t * kNI;
    float s = th[oB1 + t];
    for (int i = 0; i < kNI; ++i) s = fmaf(xs[i], w[i], s);
    h1[t] = fmaxf(s, 0.0f);
  }
  __syncthreads();
  {
    const float* w = th + oW2 + t * kNH;
    float s = th[oB2 + t];
    for (int i = 0; i < kNH; ++i) s = fmaf(h1[i], w[i], s);
    h2[t] = fmaxf(s, 0.0f);
  }
  __syncthreads();
  if (t < kNC) {
    const float* w = th + oW3 + t * kNH;
    float s = th[oB3 + t];
    for (int i = 0; i < kNH; ++i) s = fmaf(h2[i], w[i], s);
    z[t] = s;
  }
  __syncthreads();
}

// argmax over the kNC logits (ties to the lower class).
__device__ int argmax_logits(const float* z) {
  int best = 0;
  for (int c = 1; c < kNC; ++c)
    if (z[c] > z[best]) best = c;
  return best;
}

__global__ __launch_bounds__(kNH) void predict_class_kernel(const float* __restrict__ th,
                                                            const float* __restrict__ x,
                                                            float* __restrict__ out,
                                                            int* __restrict__ cls) {
  __shared__ float xs[kNI], h1[kNH], h2[kNH], z[kNC];
  const int t = threadIdx.x;
  if (t < kNI) xs[t] = x[t];
  __syncthreads();
  mlp_logits(th, xs, h1, h2, z);
  if (out) {
    out[t] = h1[t];
    out[kNH + t] = h2[t];
    if (t < kNC) out[2 * kNH + t] = z[t];
  }
  if (t == 0) *cls = argmax_logits(z);
}

// Rank, then power rounds: the rank network (th_k) reads the 64 spectrum
// features with rank_feat in the last input and picks class ck, the rank
// k_hat = min(8 * 2^ck, k_max); the power-round network (th_q) then reads
// the same spectrum with k_hat / 256 in the last input.  out[0] = q class,
// out[1] = rank class, out[2] = k_hat.
__global__ __launch_bounds__(kNH) void predict_rank_q_kernel(const float* __restrict__ th_q,
                                                             const float* __restrict__ th_k,
                                                             const float* __restrict__ x,
                                                             float rank_feat, int k_max,
                                                             int* __restrict__ out) {
  __shared__ float xs[kNI], h1[kNH], h2[kNH], z[kNC];
  __shared__ int khat;
  const int t = threadIdx.x;
  if (t < kNI) xs[t] = t < kNI - 1 ? x[t] : rank_feat;
  __syncthreads();
  mlp_logits(th_k, xs, h1, h2, z);
  if (t == 0) {
    const int ck = argmax_logits(z);
    khat = min(8 << ck, k_max);
    out[1] = ck;
    out[2] = khat;
    xs[kNI - 1] = (float)khat / 256.0f;
  }
  __syncthreads();
  mlp_logits(th_q, xs, h1, h2, z);
  if (t == 0) out[0] = argmax_logits(z);
}

// Rank-k errors of QLP factors from L alone: with nrm2 = ||A||_F^2 and the
// squared column norms c_j of L (d x d lower-triangular, ldl),
// e_k^2 = (nrm2 - c_1 - ... - c_k) / nrm2 (the residual of the rank-k
// truncation is orthogonal to Q L[:, :k] P[:, :k]^T).  Writes res[0] = the
// smallest k with e_k <= tol (d if none) and res[1] = that e_k.  One
// workgroup; the sum runs in column order (deterministic).
__global__ __launch_bounds__(256) void rank_scan_kernel(const double* __restrict__ L,
                                                        int64_t ldl, int d,
                                                        const double* __restrict__ nrm2,
                                                        double tol, double* __restrict__ res) {
  extern __shared__ double colsq[];
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double s = 0.0;
    for (int i = j; i < d; ++i) {
      const double v = L[i + (int64_t)j * ldl];
      s = fma(v, v, s);
    }
    colsq[j] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double a2 = *nrm2;
  double acc = 0.0, e = a2 > 0.0 ? 1.0 : 0.0;
  int k = d;
  for (int j = 0; j < d; ++j) {
    acc += colsq[j];
    const double r = a2 > 0.0 ? fmax(0.0, (a2 - acc) / a2) : 0.0;
    e = sqrt(r);
    if (e <= tol) {
      k = j + 1;
      break;
    }
  }
  res[0] = (double)k;
  res[1] = e;
}

// argmax of the 6 logits -> predicted class (ties to the lower class).
__global__ void argmax_kernel(const float* __restrict__ Z, int C, int* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int best = 0;
  for (int c = 1; c < C; ++c)
    if (Z[c] > Z[best]) best = c;
  *out = best;
}

// ------------------------------------------------------------ error judge
// Partial sums of squares of X (rows x cols, ld) or of X - Y, per
// workgroup, in fp64; finished by sumsq_finish_kernel in a fixed order.
constexpr int kSumsqBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial_kernel(const T* __restrict__ X, int64_t ldx,
                                                            const T* __restrict__ Y, int64_t ldy,
                                                            int64_t rows, int64_t cols,
                                                            double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t total = rows * cols;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e % rows, j = e / rows;
    double v = (double)X[i + j * ldx];
    if (Y) v -= (double)Y[i + j * ldy];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sumsq_finish_kernel(const double* __restrict__ part,
                                                           int64_t nparts, double* __restrict__ out) {
  __shared__ double red[256];
  // eight loads in flight per thread, summed in a fixed order
  double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i0 = threadIdx.x; i0 < nparts; i0 += 8 * 256) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + 256 * u;
      s8[u] += i < nparts ? part[i] : 0.0;
    }
  }
  const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_features(const double* G, int64_t ldg, int k, float* feat, hipStream_t st) {
  hipLaunchKernelGGL(features_kernel, dim3(1), dim3(kFeatThreads), 0, st, G, ldg, k, feat);
  return hipGetLastError();
}

hipError_t launch_linear_forward(const float* X, int ldx, const float* W, const float* bias,
                                 float* Y, int B, int nin, int nout, bool relu, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(linear_forward_kernel, dim3(blocks_for((int64_t)B * nout)), dim3(256), 0,
                     st, X, ldx, W, bias, Y, B, nin, nout, relu ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_softmax_xent(const float* Z, const int* y, int B, int C, float* dZ,
                               float* loss, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(softmax_xent_kernel, dim3(blocks_for(B)), dim3(256), 0, st, Z, y, B, C,
                     1.0f / (float)B, dZ, loss);
  return hipGetLastError();
}

hipError_t launch_linear_backward_input(const float* dY, const float* W, const float* H,
                                        float* dX, int B, int nin, int nout, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(linear_backward_input_kernel, dim3(blocks_for((int64_t)B * nin)), dim3(256),
                     0, st, dY, W, H, dX, B, nin, nout);
  return hipGetLastError();
}

hipError_t launch_linear_backward_weight(const float* X, int ldx, const float* dY, float* dW,
                                         float* db, int B, int nin, int nout, hipStream_t st) {
  hipLaunchKernelGGL(linear_backward_weight_kernel,
                     dim3(blocks_for((int64_t)nin * nout + nout)), dim3(256), 0, st, X, ldx, dY,
                     dW, db, B, nin, nout);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* g, float* m, float* v, int64_t count, float lr,
                       float beta1, float beta2, float eps, int64_t t, hipStream_t st) {
  const float corr1 = 1.0f - powf(beta1, (float)t), corr2 = 1.0f - powf(beta2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count)), dim3(256), 0, st, theta, g, m, v,
                     count, lr, beta1, beta2, eps, corr1, corr2);
  return hipGetLastError();
}

hipError_t launch_gather(const float* X, const int* y, int64_t N, int64_t a, int64_t c,
                         int64_t start, int B, int nin, float* Xb, int* yb, hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel, dim3(blocks_for((int64_t)B * nin)), dim3(256), 0, st, X, y,
                     N, a, c, start, B, nin, Xb, yb);
  return hipGetLastError();
}

hipError_t launch_sum(const float* x, int64_t n, float scale, float* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, x, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_predict_class(const float* th, const float* feat, float* out, int* cls,
                                hipStream_t st) {
  hipLaunchKernelGGL(predict_class_kernel, dim3(1), dim3(kNH), 0, st, th, feat, out, cls);
  return hipGetLastError();
}

hipError_t launch_predict_rank_q(const float* th_q, const float* th_k, const float* feat,
                                 float rank_feat, int k_max, int* out, hipStream_t st) {
  hipLaunchKernelGGL(predict_rank_q_kernel, dim3(1), dim3(kNH), 0, st, th_q, th_k, feat,
                     rank_feat, k_max, out);
  return hipGetLastError();
}

hipError_t launch_rank_scan(const double* L, int64_t ldl, int64_t d, const double* nrm2,
                            double tol, double* res, hipStream_t st) {
  hipLaunchKernelGGL(rank_scan_kernel, dim3(1), dim3(256), (size_t)d * sizeof(double), st, L,
                     ldl, (int)d, nrm2, tol, res);
  return hipGetLastError();
}

hipError_t launch_argmax(const float* Z, int C, int* out, hipStream_t st) {
  hipLaunchKernelGGL(argmax_kernel, dim3(1), dim3(64), 0, st, Z, C, out);
  return hipGetLastError();
}

size_t sumsq_scratch_bytes() { return (size_t)kSumsqBlocks * sizeof(double); }

hipError_t launch_sum_f64(const double* x, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sumsq_finish_kernel, dim3(1), dim3(256), 0, st, x, (int)n, out);
  return hipGetLastError();
}

hipError_t launch_sumsq(const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t rows,
                        int64_t cols, Dtype dt, double* scratch, double* out, hipStream_t st) {
  if (rows <= 0 || cols <= 0) {
    hipLaunchKernelGGL(sumsq_finish_kernel, dim3(1), dim3(256), 0, st, scratch, 0, out);
    return hipGetLastError();
  }
  const int64_t total = rows * cols;
  const int nb = (int)std::min<int64_t>(kSumsqBlocks, (total + 255) / 256);
  if (dt == DT_F64)
    hipLaunchKernelGGL(sumsq_partial_kernel<double>, dim3(nb), dim3(256), 0, st,
                       (const double*)X, ldx, (const double*)Y, ldy, rows, cols, scratch);
  else
    hipLaunchKernelGGL(sumsq_partial_kernel<float>, dim3(nb), dim3(256), 0, st, (const float*)X,
                       ldx, (const float*)Y, ldy, rows, cols, scratch);
  hipLaunchKernelGGL(sumsq_finish_kernel, dim3(1), dim3(256), 0, st, scratch, nb, out);
  return hipGetLastError();
}

}  // namespace rqlp

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

#include "rqlp_internal.h"

namespace rqlp {
namespace {

constexpr int kNs = 64;            // sketch columns read by the predictor
constexpr int kJacobiThreads = 256;

// ---------------------------------------------------------------- features
// Eigenvalues of the symmetric 64 x 64 G (column-major, ldg) in one
// workgroup: Householder reduction to tridiagonal form (62 reflections,
// each a reduction for the vector, a symmetric matrix-vector product and a
// rank-2 update on the trailing block in LDS), then bisection with Sturm
// counts, one thread per eigenvalue (thread i finds the i-th smallest, so
// the order comes for free).  Both steps are backward stable: the
// eigenvalues carry an absolute error of a few units of roundoff times
// ||G||, which resolves sigma_i / sigma_1 = sqrt(lambda_i / lambda_1) well
// below the features' clamp at 1e-6.  Then the features as described above.
__device__ __forceinline__ int sturm_count(const double* dg, const double* eo2, int n,
                                           double x, double pivmin) {
  // number of eigenvalues of the tridiagonal (dg, off-diagonal^2 eo2) below x
  int cnt = 0;
  double q = dg[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int j = 1; j < n; ++j) {
    q = (dg[j] - x) - eo2[j - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__global__ __launch_bounds__(kJacobiThreads) void features_kernel(const double* __restrict__ G,
                                                                 int64_t ldg, int k,
                                                                 float* __restrict__ feat) {
  __shared__ double a[kNs][kNs + 1];
  __shared__ double v[kNs], pw[kNs];
  __shared__ double dg[kNs], eo2[kNs];
  __shared__ double lam[kNs];
  __shared__ double scal[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kNs * kNs; e += kJacobiThreads) {
    const int i = e % kNs, j = e / kNs;
    a[i][j] = G[i + (int64_t)j * ldg];
  }
  __syncthreads();
  for (int kk = 0; kk < kNs - 2; ++kk) {
    const int r0 = kk + 1, len = kNs - r0;  // reflect rows r0..63 of column kk
    if (wave == 0) {
      const double x = lane < len ? a[r0 + lane][kk] : 0.0;
      double ss = x * x;
      for (int w = 32; w > 0; w >>= 1) ss += __shfl_xor(ss, w);
      const double x0 = __shfl(x, 0);
      const double nrm = sqrt(ss);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double vv = lane == 0 ? x0 - alpha : x;
      double v2 = vv * vv;
      for (int w = 32; w > 0; w >>= 1) v2 += __shfl_xor(v2, w);
      if (lane < len) v[lane] = vv;
      if (lane == 0) {
        scal[0] = v2 > 0.0 ? 2.0 / v2 : 0.0;   // beta
        scal[1] = v2 > 0.0 ? alpha : x0;         // the new off-diagonal entry
      }
    }
    __syncthreads();
    const double beta = scal[0];
    // p = beta A22 v: four threads per row, 16 columns each, summed across lanes
    if (tid < 4 * kNs) {
      const int row = tid >> 2, part = tid & 3;
      double sacc = 0.0;
      if (row < len) {
        for (int j = part; j < len; j += 4) sacc += a[r0 + row][r0 + j] * v[j];
      }
      sacc += __shfl_xor(sacc, 1);
      sacc += __shfl_xor(sacc, 2);
      if (part == 0 && row < len) pw[row] = beta * sacc;
    }
    __syncthreads();
    // w = p - (beta / 2) (p^T v) v
    if (wave == 0) {
      double pv = lane < len ? pw[lane] * v[lane] : 0.0;
      for (int w = 32; w > 0; w >>= 1) pv += __shfl_xor(pv, w);
      const double K = 0.5 * beta * pv;
      if (lane < len) pw[lane] -= K * v[lane];
    }
    __syncthreads();
    // A22 -= v w^T + w v^T; column kk becomes (alpha, 0, ..., 0) below the diagonal
    for (int e = tid; e < len * len; e += kJacobiThreads) {
      const int i = e % len, j = e / len;
      a[r0 + i][r0 + j] -= v[i] * pw[j] + pw[i] * v[j];
    }
    if (tid < len) {
      const double val = tid == 0 ? scal[1] : 0.0;
      a[r0 + tid][kk] = val;
      a[kk][r0 + tid] = val;
    }
    __syncthreads();
  }
  if (tid < kNs) {
    dg[tid] = a[tid][tid];
    const double o = tid + 1 < kNs ? a[tid + 1][tid] : 0.0;
    eo2[tid] = o * o;
  }
  __syncthreads();
  if (tid < kNs) {
    // Gershgorin interval and a pivot floor relative to ||T||
    double lo = 1e300, hi = -1e300, tn = 0.0;
    for (int j = 0; j < kNs; ++j) {
      const double r = (j > 0 ? sqrt(eo2[j - 1]) : 0.0) + (j + 1 < kNs ? sqrt(eo2[j]) : 0.0);
      lo = fmin(lo, dg[j] - r);
      hi = fmax(hi, dg[j] + r);
      tn = fmax(tn, fabs(dg[j]) + r);
    }
    const double pivmin = fmax(tn, 1e-300) * 1e-300 + 1e-300;
    const double tol = 4.0 * 2.220446049250313e-16 * fmax(tn, 1e-300);
    // the (tid)-th smallest eigenvalue: count(x) <= tid < count(hi)
    double l = lo, h = hi;
    for (int it = 0; it < 200 && h - l > tol; ++it) {
      const double mid = 0.5 * (l + h);
      if (sturm_count(dg, eo2, kNs, mid, pivmin) <= tid) l = mid;
      else h = mid;
    }
    lam[tid] = sqrt(fmax(0.5 * (l + h), 0.0));
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
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) s += part[i];
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
  hipLaunchKernelGGL(features_kernel, dim3(1), dim3(kJacobiThreads), 0, st, G, ldg, k, feat);
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

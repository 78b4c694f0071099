// The learned power-iteration predictor and the a-posteriori error judge.
//
// Features: the singular values of the 64-column sketch Y = A^T Omega[:, :64]
// (the leading Philox columns of the method's own sketch) from the
// eigenvalues of its fp64 Gram matrix, by cyclic Jacobi in one workgroup,
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
// Cyclic Jacobi eigenvalues of the symmetric 64 x 64 G (column-major, ldg),
// round-robin ordering: in each of the 63 steps of a sweep the 32 disjoint
// pairs are rotated at once (rotations first, then rows, then columns).
// Sweeps stop when the off-diagonal mass falls below (1e-14)^2 of the
// diagonal's or after 30 sweeps.  Then the features as described above.
__global__ __launch_bounds__(kJacobiThreads) void features_kernel(const double* __restrict__ G,
                                                                 int64_t ldg, int k,
                                                                 float* __restrict__ feat) {
  __shared__ double a[kNs][kNs + 1];
  __shared__ double cs[kNs / 2], sn[kNs / 2];
  __shared__ int pp[kNs / 2], qq[kNs / 2];
  __shared__ double red[kJacobiThreads];
  __shared__ double lam[kNs];
  __shared__ int stop;
  const int tid = threadIdx.x;
  for (int e = tid; e < kNs * kNs; e += kJacobiThreads) {
    const int i = e % kNs, j = e / kNs;
    a[i][j] = G[i + (int64_t)j * ldg];
  }
  if (tid == 0) stop = 0;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    // convergence test on the current matrix
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < kNs * kNs; e += kJacobiThreads) {
      const int i = e % kNs, j = e / kNs;
      const double v = a[i][j] * a[i][j];
      if (i == j) dia += v; else off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int s = kJacobiThreads / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double off_all = red[0];
    __syncthreads();
    red[tid] = dia;
    __syncthreads();
    for (int s = kJacobiThreads / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) stop = (off_all <= 1e-28 * red[0]) ? 1 : 0;
    __syncthreads();
    if (stop) break;
    for (int step = 0; step < kNs - 1; ++step) {
      if (tid < kNs / 2) {
        // tournament pairing: slot 0 fixed, slots 1..63 rotate by `step`
        const int s1 = tid, s2 = kNs - 1 - tid;
        const int p = (s1 == 0) ? 0 : ((s1 - 1 + step) % (kNs - 1)) + 1;
        const int q = ((s2 - 1 + step) % (kNs - 1)) + 1;
        const double apq = a[p][q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double tau = (a[q][q] - a[p][p]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      // rows: (A_p, A_q) <- (c A_p - s A_q, s A_p + c A_q)
      for (int e = tid; e < (kNs / 2) * kNs; e += kJacobiThreads) {
        const int r = e / kNs, j = e % kNs;
        const int p = pp[r], q = qq[r];
        const double c = cs[r], s = sn[r];
        const double x = a[p][j], y = a[q][j];
        a[p][j] = c * x - s * y;
        a[q][j] = s * x + c * y;
      }
      __syncthreads();
      // columns: (A_:p, A_:q) <- (c A_:p - s A_:q, s A_:p + c A_:q)
      for (int e = tid; e < (kNs / 2) * kNs; e += kJacobiThreads) {
        const int r = e / kNs, i = e % kNs;
        const int p = pp[r], q = qq[r];
        const double c = cs[r], s = sn[r];
        const double x = a[i][p], y = a[i][q];
        a[i][p] = c * x - s * y;
        a[i][q] = s * x + c * y;
      }
      __syncthreads();
    }
  }
  // sigma_i = sqrt(max(lambda_i, 0)), sorted descending by rank counting
  if (tid < kNs) lam[tid] = sqrt(fmax(a[tid][tid], 0.0));
  __syncthreads();
  if (tid < kNs) {
    const double v = lam[tid];
    int rank = 0;
    for (int j = 0; j < kNs; ++j) {
      const double w = lam[j];
      rank += (w > v || (w == v && j < tid)) ? 1 : 0;
    }
    double s1 = 0.0;
    for (int j = 0; j < kNs; ++j) s1 = fmax(s1, lam[j]);
    float f = -1.0f;
    if (s1 > 0.0 && v > 0.0) {
      const double lg = log10(v / s1);
      f = (float)(fmin(fmax(lg, -6.0), 0.0) / 6.0);
    }
    feat[rank] = f;
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

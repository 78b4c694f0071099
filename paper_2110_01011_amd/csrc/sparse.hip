// Sparse input (Section 5.1 factors sparse SuiteSparse matrices): the
// products of the method with a CSR matrix A, and the device-side transpose
// that gives A^T in the same format.
//
// The dense panels of the method are column-major.  A sparse product reads
// whole rows of the panel for each nonzero, so the panel is first turned
// d-contiguous (row-major), the product runs one wavefront per output row
// with the lanes across the d columns (every nonzero then gathers one
// contiguous panel row), and the result is turned back column-major.  Each
// output element sums its row's nonzeros in CSR order: deterministic.
//
// A^T: column counts (atomic increments), an exclusive scan, a scatter
// (atomic cursors), then each column's entries sorted by row index, so the
// result does not depend on the scatter's order.
#include <hip/hip_runtime.h>

#include "rqlp_internal.h"

namespace rqlp {
namespace {

constexpr int kSpWaves = 4;      // wavefronts (output rows) per workgroup
constexpr int kSpCols = 4;       // panel columns per lane per pass (64 * 4 = 256)
constexpr int kTile = 32;        // transpose tile

// C (rows x d, d-contiguous) = A_csr X (K x d, d-contiguous).
template <typename T>
__global__ __launch_bounds__(64 * kSpWaves) void spmm_rows_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const T* __restrict__ vals, int64_t rows, const T* __restrict__ X, int64_t d,
    T* __restrict__ C) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kSpWaves + (threadIdx.x >> 6);
  if (i >= rows) return;
  const int64_t t0 = rowptr[i], t1 = rowptr[i + 1];
  for (int64_t c0 = 0; c0 < d; c0 += 64 * kSpCols) {
    T acc[kSpCols];
#pragma unroll
    for (int u = 0; u < kSpCols; ++u) acc[u] = T(0);
    for (int64_t t = t0; t < t1; ++t) {
      const T a = vals[t];
      const T* xr = X + (int64_t)colind[t] * d + c0 + lane;
#pragma unroll
      for (int u = 0; u < kSpCols; ++u)
        if (c0 + lane + 64 * u < d) acc[u] += a * xr[64 * u];
    }
    T* cr = C + i * d + c0 + lane;
#pragma unroll
    for (int u = 0; u < kSpCols; ++u)
      if (c0 + lane + 64 * u < d) cr[64 * u] = acc[u];
  }
}

// Y (cols x rows, ldy) = X^T for X (rows x cols, ldx), through an LDS tile.
template <typename T>
__global__ __launch_bounds__(256) void transpose_tile_kernel(const T* __restrict__ X,
                                                             int64_t ldx, int64_t rows,
                                                             int64_t cols, T* __restrict__ Y,
                                                             int64_t ldy) {
  __shared__ T tile[kTile][kTile + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kTile, c0 = (int64_t)blockIdx.y * kTile;
  const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;  // 32 x 8
  for (int j = ty; j < kTile; j += 256 / kTile) {
    const int64_t r = r0 + tx, c = c0 + j;
    if (r < rows && c < cols) tile[j][tx] = X[r + c * ldx];
  }
  __syncthreads();
  for (int j = ty; j < kTile; j += 256 / kTile) {
    const int64_t c = c0 + tx, r = r0 + j;
    if (r < rows && c < cols) Y[c + r * ldy] = tile[tx][j];
  }
}

// Structure check of a CSR matrix: rowptr[0] = 0, non-decreasing,
// rowptr[rows] = nnz, every column index in [0, cols).  Raises *bad.
__global__ __launch_bounds__(256) void csr_check_kernel(const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ colind,
                                                        int64_t rows, int64_t cols, int64_t nnz,
                                                        int* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = g; i <= rows; i += stride) {
    const int64_t r = rowptr[i];
    const bool ok = (i == 0) ? (r == 0)
                             : (r >= rowptr[i - 1] && (i < rows || r == nnz) && r <= nnz);
    if (!ok) atomicOr(bad, 1);
  }
  for (int64_t t = g; t < nnz; t += stride) {
    const int32_t j = colind[t];
    if (j < 0 || (int64_t)j >= cols) atomicOr(bad, 2);
  }
}

__global__ __launch_bounds__(256) void count_cols_kernel(const int32_t* __restrict__ colind,
                                                         int64_t nnz, int* __restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz; t += stride)
    atomicAdd(&cnt[colind[t]], 1);
}

// colptr[0..n] = exclusive scan of cnt[0..n); cursor = colptr[0..n).  One
// workgroup, chunks of 1024 with a running carry.
__global__ __launch_bounds__(1024) void scan_kernel(const int* __restrict__ cnt, int64_t n,
                                                    int64_t* __restrict__ colptr,
                                                    int64_t* __restrict__ cursor) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < n ? cnt[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
      const int64_t add = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < n) {
      const int64_t ex = carry + buf[threadIdx.x] - v;
      colptr[i] = ex;
      cursor[i] = ex;
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) colptr[n] = carry;
}

// One thread per row: its entries go to their columns at atomic cursors.
template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind,
                                                      const T* __restrict__ vals, int64_t rows,
                                                      unsigned long long* __restrict__ cursor,
                                                      int32_t* __restrict__ rowind_t,
                                                      T* __restrict__ vals_t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
    const unsigned long long pos = atomicAdd(&cursor[colind[t]], 1ull);
    rowind_t[pos] = (int32_t)i;
    vals_t[pos] = vals[t];
  }
}

// One thread per column: insertion sort of its segment by row index (the
// scatter left them in arrival order).
template <typename T>
__global__ __launch_bounds__(256) void sort_segments_kernel(const int64_t* __restrict__ colptr,
                                                            int64_t n,
                                                            int32_t* __restrict__ rowind_t,
                                                            T* __restrict__ vals_t) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t a = colptr[j], b = colptr[j + 1];
  for (int64_t t = a + 1; t < b; ++t) {
    const int32_t r = rowind_t[t];
    const T v = vals_t[t];
    int64_t u = t - 1;
    while (u >= a && rowind_t[u] > r) {
      rowind_t[u + 1] = rowind_t[u];
      vals_t[u + 1] = vals_t[u];
      --u;
    }
    rowind_t[u + 1] = r;
    vals_t[u + 1] = v;
  }
}

__global__ void zero_i64_kernel(int64_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

unsigned blocks_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }
unsigned grid_stride_blocks(int64_t n) {
  return (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
}

}  // namespace

size_t csr_transpose_bytes(int64_t n, int64_t nnz, Dtype dt) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return al((size_t)(n + 1) * 8) + al((size_t)n * 8) + al((size_t)n * 4) +
         al((size_t)nnz * 4) + al((size_t)nnz * (dt == DT_F64 ? 8 : 4));
}

hipError_t launch_csr_check(const int64_t* rowptr, const int32_t* colind, int64_t rows,
                            int64_t cols, int64_t nnz, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(csr_check_kernel, dim3(grid_stride_blocks(std::max(rows + 1, nnz))),
                     dim3(256), 0, st, rowptr, colind, rows, cols, nnz, bad);
  return hipGetLastError();
}

hipError_t launch_csr_transpose(const int64_t* rowptr, const int32_t* colind, const void* vals,
                                int64_t m, int64_t n, int64_t nnz, Dtype dt, void* ws,
                                CsrView* out, hipStream_t st) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* p = (char*)ws;
  int64_t* colptr = (int64_t*)p;
  p += al((size_t)(n + 1) * 8);
  int64_t* cursor = (int64_t*)p;
  p += al((size_t)n * 8);
  int* cnt = (int*)p;
  p += al((size_t)n * 4);
  int32_t* rowind_t = (int32_t*)p;
  p += al((size_t)nnz * 4);
  void* vals_t = p;
  out->rowptr = colptr;
  out->colind = rowind_t;
  out->vals = vals_t;
  out->rows = n;
  out->cols = m;
  out->nnz = nnz;
  if (n > 0) {
    hipError_t e = launch_zero_ints(cnt, n, st);
    if (e != hipSuccess) return e;
    if (nnz > 0)
      hipLaunchKernelGGL(count_cols_kernel, dim3(grid_stride_blocks(nnz)), dim3(256), 0, st,
                         colind, nnz, cnt);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, cnt, n, colptr, cursor);
  } else {
    hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(64), 0, st, colptr, (int64_t)1);
  }
  if (nnz > 0 && m > 0) {
    if (dt == DT_F64) {
      hipLaunchKernelGGL(scatter_kernel<double>, dim3(blocks_of(m, 256)), dim3(256), 0, st,
                         rowptr, colind, (const double*)vals, m, (unsigned long long*)cursor,
                         rowind_t, (double*)vals_t);
      hipLaunchKernelGGL(sort_segments_kernel<double>, dim3(blocks_of(n, 256)), dim3(256), 0,
                         st, colptr, n, rowind_t, (double*)vals_t);
    } else {
      hipLaunchKernelGGL(scatter_kernel<float>, dim3(blocks_of(m, 256)), dim3(256), 0, st,
                         rowptr, colind, (const float*)vals, m, (unsigned long long*)cursor,
                         rowind_t, (float*)vals_t);
      hipLaunchKernelGGL(sort_segments_kernel<float>, dim3(blocks_of(n, 256)), dim3(256), 0, st,
                         colptr, n, rowind_t, (float*)vals_t);
    }
  }
  return hipGetLastError();
}

hipError_t launch_spmm(const CsrView& A, const void* X, int64_t ldx, int64_t d, void* C,
                       int64_t ldc, Dtype dt, void* xr, void* cr, hipStream_t st) {
  const int64_t K = A.cols, rows = A.rows;
  if (rows == 0 || d == 0) return hipSuccess;
  const dim3 tb(256);
  if (dt == DT_F64) {
    if (K > 0)
      hipLaunchKernelGGL(transpose_tile_kernel<double>,
                         dim3(blocks_of(K, kTile), blocks_of(d, kTile)), tb, 0, st,
                         (const double*)X, ldx, K, d, (double*)xr, d);
    hipLaunchKernelGGL(spmm_rows_kernel<double>, dim3(blocks_of(rows, kSpWaves)),
                       dim3(64 * kSpWaves), 0, st, A.rowptr, A.colind, (const double*)A.vals,
                       rows, (const double*)xr, d, (double*)cr);
    hipLaunchKernelGGL(transpose_tile_kernel<double>,
                       dim3(blocks_of(d, kTile), blocks_of(rows, kTile)), tb, 0, st,
                       (const double*)cr, d, d, rows, (double*)C, ldc);
  } else {
    if (K > 0)
      hipLaunchKernelGGL(transpose_tile_kernel<float>,
                         dim3(blocks_of(K, kTile), blocks_of(d, kTile)), tb, 0, st,
                         (const float*)X, ldx, K, d, (float*)xr, d);
    hipLaunchKernelGGL(spmm_rows_kernel<float>, dim3(blocks_of(rows, kSpWaves)),
                       dim3(64 * kSpWaves), 0, st, A.rowptr, A.colind, (const float*)A.vals,
                       rows, (const float*)xr, d, (float*)cr);
    hipLaunchKernelGGL(transpose_tile_kernel<float>,
                       dim3(blocks_of(d, kTile), blocks_of(rows, kTile)), tb, 0, st,
                       (const float*)cr, d, d, rows, (float*)C, ldc);
  }
  return hipGetLastError();
}

}  // namespace rqlp

// Gaussian test matrix of Algorithm 1 (the randn step), on the GPU.
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 4 x 64-bit counter,
// 2 x 64-bit key, ten rounds.  A round multiplies counter words 0 and 2 by
// fixed odd 64-bit constants and forms (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1,
// lo0); the key advances by two Weyl constants between rounds.
// Element (i, j) of an m-row matrix has column-major index l = i + j*m and
// takes lane l % 4 of block counter (l / 4, 0, 0, 0) under key (seed,
// stream).  Words become uniforms u = ((w >> 12) + 0.5) * 2^-52 and pairs of
// uniforms become normals by Box-Muller, evaluated in double precision.
// One thread produces one Philox block (four consecutive elements).
#include "rqlp_internal.h"

namespace rqlp {
namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
constexpr double kTwoPi = 6.283185307179586;  // 2 * (double)pi, exact doubling

__device__ __forceinline__ void philox_block(uint64_t ctr0, uint64_t k0, uint64_t k1,
                                             uint64_t w[4]) {
  uint64_t c0 = ctr0, c1 = 0, c2 = 0, c3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  w[0] = c0;
  w[1] = c1;
  w[2] = c2;
  w[3] = c3;
}

__device__ __forceinline__ double unif(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

__device__ __forceinline__ void block_normals(uint64_t blk, uint64_t seed, uint64_t sid,
                                              double z[4]) {
  uint64_t w[4];
  philox_block(blk, seed, sid, w);
#pragma unroll
  for (int pr = 0; pr < 2; ++pr) {
    const double ua = unif(w[2 * pr]), ub = unif(w[2 * pr + 1]);
    const double r = sqrt(-2.0 * log(ua));
    const double t = kTwoPi * ub;
    z[2 * pr] = r * cos(t);
    z[2 * pr + 1] = r * sin(t);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gaussian_kernel(T* __restrict__ out, int64_t m,
                                                       int64_t total, int64_t ld,
                                                       uint64_t seed, uint64_t sid) {
  const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t l0 = blk * 4;
  if (l0 >= total) return;
  double z[4];
  block_normals((uint64_t)blk, seed, sid, z);
  int64_t j = l0 / m, i = l0 - j * m;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (l0 + t < total) out[i + j * ld] = (T)z[t];
    if (++i == m) {
      i = 0;
      ++j;
    }
  }
}

// Columns j with flags[j] != 0 of a rows x d panel get fresh normals
// (index l = i + j*rows under key (seed, sid)); other columns untouched.
template <typename T>
__global__ __launch_bounds__(256) void gaussian_columns_kernel(T* __restrict__ X, int64_t rows,
                                                               int64_t ldx,
                                                               const int* __restrict__ flags,
                                                               int64_t d, uint64_t seed,
                                                               uint64_t sid) {
  const int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = rows * d;
  const int64_t l0 = blk * 4;
  if (l0 >= total) return;
  double z[4];
  bool any = false;
  {
    int64_t j = l0 / rows, i = l0 - j * rows;
    for (int t = 0; t < 4; ++t) {
      if (l0 + t < total && flags[j]) any = true;
      if (++i == rows) {
        i = 0;
        ++j;
      }
    }
  }
  if (!any) return;
  block_normals((uint64_t)blk, seed, sid, z);
  int64_t j = l0 / rows, i = l0 - j * rows;
  for (int t = 0; t < 4; ++t) {
    if (l0 + t < total && flags[j]) X[i + j * ldx] = (T)z[t];
    if (++i == rows) {
      i = 0;
      ++j;
    }
  }
}

// Grouped form: workgroup b fills the 1024 values starting at
// 1024 bmap[b].y of sketch bmap[b].x (same values as the single form).
template <typename T>
__global__ __launch_bounds__(256) void gaussian_grouped_kernel(const GroupGauss* __restrict__ descs,
                                                               const int2* __restrict__ bmap) {
  const int2 b = bmap[blockIdx.x];
  const GroupGauss g = descs[b.x];
  const int64_t total = g.m * g.d;
  const int64_t blk = (int64_t)b.y * 256 + threadIdx.x;
  const int64_t l0 = blk * 4;
  if (l0 >= total) return;
  double z[4];
  block_normals((uint64_t)blk, g.seed, 0, z);
  int64_t j = l0 / g.m, i = l0 - j * g.m;
  T* out = (T*)g.out;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (l0 + t < total) out[i + j * g.ld] = (T)z[t];
    if (++i == g.m) {
      i = 0;
      ++j;
    }
  }
}

}  // namespace

hipError_t launch_gaussian(void* out, int64_t m, int64_t d, int64_t ld, uint64_t seed,
                           uint64_t sid, Dtype dt, hipStream_t st) {
  const int64_t total = m * d;
  if (total <= 0) return hipSuccess;
  const int64_t nblk = (total + 3) / 4;
  const unsigned grid = (unsigned)((nblk + 255) / 256);
  if (dt == DT_F64)
    hipLaunchKernelGGL(gaussian_kernel<double>, dim3(grid), dim3(256), 0, st, (double*)out, m,
                       total, ld, seed, sid);
  else
    hipLaunchKernelGGL(gaussian_kernel<float>, dim3(grid), dim3(256), 0, st, (float*)out, m,
                       total, ld, seed, sid);
  return hipGetLastError();
}

hipError_t launch_gaussian_columns(void* X, int64_t rows, int64_t ldx, const int* col_flags,
                                   int64_t d, uint64_t seed, uint64_t sid, Dtype dt,
                                   hipStream_t st) {
  const int64_t total = rows * d;
  if (total <= 0) return hipSuccess;
  const int64_t nblk = (total + 3) / 4;
  const unsigned grid = (unsigned)((nblk + 255) / 256);
  if (dt == DT_F64)
    hipLaunchKernelGGL(gaussian_columns_kernel<double>, dim3(grid), dim3(256), 0, st,
                       (double*)X, rows, ldx, col_flags, d, seed, sid);
  else
    hipLaunchKernelGGL(gaussian_columns_kernel<float>, dim3(grid), dim3(256), 0, st,
                       (float*)X, rows, ldx, col_flags, d, seed, sid);
  return hipGetLastError();
}

void gauss_grouped_blocks(const GroupGauss& g, int idx, std::vector<int2>& out) {
  const int64_t nb = (g.m * g.d + 1023) / 1024;
  for (int64_t b = 0; b < nb; ++b) out.push_back(int2{idx, (int)b});
}

hipError_t launch_gaussian_grouped(Dtype dt, const GroupGauss* descs, const int2* bmap,
                                   int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (dt == DT_F64)
    hipLaunchKernelGGL(gaussian_grouped_kernel<double>, dim3((unsigned)nblocks), dim3(256), 0, st,
                       descs, bmap);
  else
    hipLaunchKernelGGL(gaussian_grouped_kernel<float>, dim3((unsigned)nblocks), dim3(256), 0, st,
                       descs, bmap);
  return hipGetLastError();
}

}  // namespace rqlp

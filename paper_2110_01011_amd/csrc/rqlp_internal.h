// Internal declarations shared by the HIP translation units of librandqlp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

namespace rqlp {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Row (within a 16 x 16 block) of accumulator element r held by `lane` for
// the 16x16x4 MFMAs; the column is lane % 16.  The fp64 instruction spreads
// a lane's four values over rows lane/16 + 4r; the fp32 one keeps them in
// four consecutive rows 4 (lane/16) + r.
__device__ __forceinline__ int acc_row_f64(int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ __forceinline__ int acc_row_f32(int lane, int r) { return 4 * (lane >> 4) + r; }

// A pointer read from memory (a grouped launch's descriptor) is generic, so
// the compiler accesses it with FLAT instructions, which count on lgkmcnt as
// well as vmcnt: every wait for an LDS read then also waits for all
// outstanding global loads.  Accesses through a global-address-space
// pointer (the memory is device memory) are global instructions.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;

// 16 bytes per lane from base + voffset + soffset (bytes) into LDS at lds +
// 16 lane, by the buffer form of the direct load: base and nbytes (the
// readable extent from base; reads past it return zeros) are wave-uniform,
// soffset is uniform.  The buffer form is counted on vmcnt only; the
// FLAT-encoded global form is also counted on lgkmcnt, and the compiler then
// waits for every outstanding LDS read before using any of them.
__device__ __forceinline__ void buffer_load_lds16(const void* base, int nbytes, int voffset,
                                                  int soffset, void* lds) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nbytes, 0x00020000),
      (__attribute__((address_space(3))) void*)lds, 16, voffset, soffset, 0, 0);
}
template <typename T>
__device__ __forceinline__ int acc_row(int lane, int r);
template <>
__device__ __forceinline__ int acc_row<double>(int lane, int r) { return acc_row_f64(lane, r); }
template <>
__device__ __forceinline__ int acc_row<float>(int lane, int r) { return acc_row_f32(lane, r); }

// Flag bits written by device kernels into the per-call status word.
enum : int {
  FLAG_NONPOS_PIVOT = 1,   // Cholesky pivot <= tolerance (panel numerically dependent)
  FLAG_NONFINITE = 2,      // NaN/Inf met in a Gram matrix or pivot
  FLAG_SECOND_PASS = 4,    // second Cholesky pass far from identity (unsafe)
};

// Element type tags for the launchers.
enum Dtype : int { DT_F64 = 0, DT_F32 = 1 };

constexpr int CHOL_MAX_D = 224;   // single-workgroup Cholesky tile limit (14 x 14 tiles of 16)
constexpr int TRSM_MAX_D = 1024;  // TRSM keeps a 16 x d panel per wave in LDS
constexpr int RQLP_MAX_D = 8192;  // largest sketch width (blocked Cholesky above CHOL_MAX_D)

// ---- philox.hip ----
hipError_t launch_gaussian(void* out, int64_t m, int64_t d, int64_t ld, uint64_t seed,
                           uint64_t stream_id, Dtype dt, hipStream_t st);
// Fill columns listed in cols[0..ncols) of X (rows x ?, ldx) with Gaussian
// values from (seed, stream_id); used to complete dependent panel columns.
hipError_t launch_gaussian_columns(void* X, int64_t rows, int64_t ldx, const int* col_flags,
                                   int64_t d, uint64_t seed, uint64_t stream_id, Dtype dt,
                                   hipStream_t st);

// ---- gemm.hip ----
// C[s] (M x N) = sum over k in split s of op(A)(i,k) * B(k,j);
// op(A)(i,k) = trans_a ? A[k + i*lda] : A[i + k*lda]; B(k,j) = B[k + j*ldb].
// If splits == 1 the result goes straight to C (ldc); otherwise partial sums
// go to `partial` and a fixed-order reduction writes C.
struct GemmArgs {
  int trans_a;
  const void* A; int64_t lda;
  const void* B; int64_t ldb;
  void* C; int64_t ldc;
  int64_t M, N, K;
  Dtype in_t;     // type of A and B
  Dtype out_t;    // type of C
  bool gram;      // C = A^T A (B == A, trans_a): compute only upper tiles, mirror
  void* partial;  // workspace for split-K partials (may be null if splits == 1)
  size_t partial_bytes;
  void* ev_begin = nullptr;  // optional hipEvent_t recorded around the main kernel
  void* ev_end = nullptr;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);
size_t gemm_partial_bytes(int trans_a, int64_t M, int64_t N, int64_t K, Dtype in_t,
                          Dtype out_t, bool gram);

// Precision form: C (M x N fp32) = A16 B16, A16 (M x K) a 16-bit copy in the
// packed layout launch_convert16 writes (lda = gemm16_ld(K)), B16 (K x N) a
// 16-bit panel in the packed layout launch_convert_panel16 writes (ldb = its
// contraction extent, a multiple of 64 >= gemm16_ld(K));
// split-K partials in `partial` (fixed-order reduction).  With A2 and B2
// (bf16 only): the rounding residuals of A and B in the layouts of A and B,
// and C = A16 B16 + A16 B2 + A2 B16 (split bf16 product).
struct Gemm16Args {
  bool f16;  // false: bf16, true: fp16
  const void* A; int64_t lda;  // 16-bit, packed, lda == gemm16_ld(K), 16-byte aligned
  const void* B; int64_t ldb;  // 16-bit packed panel (launch_convert_panel16 with d = N),
                               // ldb its contraction extent
  float* C; int64_t ldc;
  const void* A2 = nullptr;  // residual of A (lda), or null
  const void* B2 = nullptr;  // residual of the panel (ldb), or null
  int64_t M, N, K;
  void* partial;
  size_t partial_bytes;
  void* ev_begin = nullptr;
  void* ev_end = nullptr;
};
hipError_t launch_gemm16(const Gemm16Args& g, hipStream_t st);
// Columns past N of the packed panel (and of its residual), zeros, that the
// 16-bit product kernel reads without bounds checks; their values never
// reach C.
constexpr int64_t kGemm16PanelSlack = 320;
// Bytes of a packed 16-bit panel with contraction K and d columns (slack
// included).
size_t gemm16_panel_bytes(int64_t K, int64_t d);
size_t gemm16_partial_bytes(int64_t M, int64_t N, int64_t K, bool f16, int nseg = 1);
// Leading dimension of a 16-bit operand with contraction length K: K rounded
// up to the kernel's tile depth; the padding must hold zeros.
int64_t gemm16_ld(int64_t K);
// Bytes of a packed 16-bit operand with `rows` rows and contraction K (rows
// rounded up to 64, K to gemm16_ld(K)).
size_t gemm16_packed_bytes(int64_t rows, int64_t K);
// X (rows x d fp32, ldx) -> Y, 16-bit, nearest even, in the packed panel
// layout of the 16-bit product kernel: contraction extent ldy (a multiple of
// the tile depth >= gemm16_ld(rows)), d columns plus kGemm16PanelSlack,
// gemm16_panel_bytes(ldy, d) bytes, 16-byte aligned; k past rows and the
// slack columns are zeros.  Ylo (optional, same layout): the rounded
// residual x - y.
hipError_t launch_convert_panel16(const float* X, int64_t rows, int64_t d, int64_t ldx, void* Y,
                                  int64_t ldy, bool f16, hipStream_t st, void* Ylo = nullptr);
// A (m x n fp32) -> packed 16-bit copies A16 (rows: A's n columns,
// contraction m, ld16 = gemm16_ld(m), gemm16_packed_bytes(n, m) bytes) and
// At16 (rows: A's m rows, contraction n, ldt16 = gemm16_ld(n),
// gemm16_packed_bytes(m, n) bytes), 16-byte aligned, zero padding.
// rerr (optional): per-workgroup sums of the squared rounding errors, one
// double for each of the nb = convert16_blocks(m, n) workgroups, followed by
// the nb per-workgroup sums of squares of A (2 nb doubles in all).  A16lo /
// At16lo (optional): the rounded residuals a - a16 in the layouts of A16 / At16.
// f16 (amax, scale_out given): the copies hold 2^s a with s chosen from
// max |a| (amax: one device unsigned of scratch) so that the largest entry
// lies in [2^13, 2^14); *scale_out (device int) receives s.  rerr stays in
// A's own units.  Products with the copies then carry the factor 2^s, which
// orth() removes (exactly: a power of two) and launch_unscale undoes.
hipError_t launch_convert16(const float* A, int64_t m, int64_t n, int64_t lda, void* A16,
                            int64_t ld16, void* At16, int64_t ldt16, bool f16, hipStream_t st,
                            double* rerr = nullptr, void* A16lo = nullptr,
                            void* At16lo = nullptr, unsigned* amax = nullptr,
                            int* scale_out = nullptr);
// C (rows x d fp32, ldc) *= 2^-(*scale_exp).
hipError_t launch_unscale(float* C, int64_t rows, int64_t d, int64_t ldc, const int* scale_exp,
                          hipStream_t st);
int64_t convert16_blocks(int64_t m, int64_t n);

// ---- panel.hip ----
// One-workgroup Cholesky of G + shift*I (d x d, double, ldg; d <= CHOL_MAX_D)
// into R (upper, ldr) and the inverses of its 16 x 16 diagonal blocks (dinv,
// ceil(d/16)*256 doubles, each block column-major).  The shift is *shift_dev
// when shift_dev is non-null, else `shift`.  A pivot <= tol_dep * (original
// diagonal) marks its column dependent: that row of R is zeroed,
// col_flags[j] = 1 (col_flags may be null) and FLAG_NONPOS_PIVOT is raised;
// a kept pivot below tol_warn * (original diagonal) raises FLAG_SECOND_PASS.
// The original diagonal is odiag_src[j * odiag_stride] + shift when
// odiag_src is given (trailing Schur complements), else G's own diagonal.
hipError_t launch_cholesky_tile(const double* G, int64_t d, int64_t ldg, double shift,
                                const double* shift_dev, double tol_dep, double tol_warn,
                                double* R, int64_t ldr, double* dinv, int* col_flags,
                                int* flags, const double* odiag_src, int64_t odiag_stride,
                                hipStream_t st);
// T (cols x rows, ldt) = S^T.
hipError_t launch_transpose(const double* S, int64_t rows, int64_t cols, int64_t lds, double* T,
                            int64_t ldt, hipStream_t st);
// S (n x n, tight) = G22 (+ shift I) - C (n x n, tight).
hipError_t launch_schur(const double* G22, int64_t ldg, const double* C, int64_t n, double shift,
                        const double* shift_dev, double* S, hipStream_t st);
hipError_t launch_zero_block(double* Z, int64_t rows, int64_t cols, int64_t ldz, hipStream_t st);
// Qx (rows x d) = (X - P) R^+ with R upper (d x d, ldr) and its
// diagonal-block inverses; Qx may be X itself (same ld).  P (rows x d, ldp,
// the type of X) is optional and needs d <= CHOL_MAX_D.
hipError_t launch_trsm(const void* X, int64_t rows, int64_t d, int64_t ldx, const double* R,
                       int64_t ldr, const double* dinv, void* Qx, int64_t ldq, Dtype dt,
                       hipStream_t st, const void* P = nullptr, int64_t ldp = 0);
// Second Cholesky QR pass to first order from G2 = Q1^T Q1 = I + E:
// B = I - F, R2 = I + F with F = triu(E, 1) + diag(E) / 2 (d x d, tight);
// raises FLAG_SECOND_PASS if max |E| > tol.
hipError_t launch_first_order_pass(const double* G2, int64_t d, double tol, double* B,
                                   double* R2, int* flags, hipStream_t st);
// Rout = R2 * R1 (upper-triangular d x d, double, tight).
hipError_t launch_trmm_upper(const double* R2, const double* R1, double* Rout, int64_t d,
                             hipStream_t st);
// L (d x d, ldl) = R^T with exact zeros above the diagonal.
hipError_t launch_lower_from_upper(const double* R, int64_t d, double* L, int64_t ldl,
                                   hipStream_t st);
// trace of G (d x d) into *out (device double) -- used for the shift.
hipError_t launch_trace(const double* G, int64_t d, int64_t ldg, double* out, hipStream_t st);
// *shift_out = c * (*trace) with c chosen from the panel size (shifted Cholesky QR).
hipError_t launch_scale_scalar(const double* in, double c, double* out, hipStream_t st);
// Convert a float panel to double or back (rows x d, strided).
hipError_t launch_copy_panel(const void* src, Dtype st_t, int64_t ld_src, void* dst,
                             Dtype dt_t, int64_t ld_dst, int64_t rows, int64_t d,
                             hipStream_t st);
// Flags: any nonzero in col_flags[0..d) -> count into *count (device int).
hipError_t launch_count_flags(const int* col_flags, int64_t d, int* count, hipStream_t st);
// Scan A (m x n, lda) for NaN / Inf; raise FLAG_NONFINITE in *flags.
hipError_t launch_check_finite(const void* A, int64_t m, int64_t n, int64_t lda, Dtype dt,
                               int* flags, hipStream_t st);

// ---- sparse.hip ----
// A CSR matrix on the device: rows x cols, row i's entries at
// [rowptr[i], rowptr[i + 1]) of colind / vals (vals of the panel type).
struct CsrView {
  const int64_t* rowptr;
  const int32_t* colind;
  const void* vals;
  int64_t rows, cols, nnz;
};
// Raise *bad (a device int) unless rowptr[0] = 0, rowptr is non-decreasing,
// rowptr[rows] = nnz and every column index lies in [0, cols).
hipError_t launch_csr_check(const int64_t* rowptr, const int32_t* colind, int64_t rows,
                            int64_t cols, int64_t nnz, int* bad, hipStream_t st);
// Device bytes of the transpose of an m x n CSR matrix with nnz entries.
size_t csr_transpose_bytes(int64_t n, int64_t nnz, Dtype dt);
// A^T of a (checked) m x n CSR matrix in CSR form, built in ws
// (csr_transpose_bytes); entries of each row of A^T in ascending column order.
hipError_t launch_csr_transpose(const int64_t* rowptr, const int32_t* colind, const void* vals,
                                int64_t m, int64_t n, int64_t nnz, Dtype dt, void* ws,
                                CsrView* out, hipStream_t st);
// C (A.rows x d, ldc) = A X (X: A.cols x d, ldx), both column-major; xr and
// cr hold A.cols x d and A.rows x d elements of scratch.  rows < 2^21.
hipError_t launch_spmm(const CsrView& A, const void* X, int64_t ldx, int64_t d, void* C,
                       int64_t ldc, Dtype dt, void* xr, void* cr, hipStream_t st);

// ---- launch planning shared by the product kernels (gemm.hip) ----
int cu_count();
void choose_splits(int64_t tiles, int64_t K, int bk, int64_t max_s, int64_t slots,
                   double tile_flops_per_k, double rate, double out_bytes, int64_t* chunk_out,
                   int* splits_out);
constexpr int kTargetWG = 1024;

// fp64 skinny products with A (gemm_f64.hip): 32-deep k-tiles, up to 13
// MFMA column blocks (+ 2 or 4 vector-ALU columns) in one 128-row tile.
// The panel B must be 16-byte aligned with an even ldb.
constexpr int kStrBK = 32, kStrMaxWN = 13;
int gemm_stream_f64_occupancy(int trans_a, int wn);
void launch_gemm_stream_f64(int trans_a, int wn, int rv, int64_t tiles_m, int64_t tiles_n,
                            int splits, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double* C, int64_t ldc, int64_t strideS, int64_t M,
                            int64_t N, int64_t K, int64_t kchunk, hipStream_t st);
// Workgroups of one kernel instantiation that fit on a CU at once (from its
// register and LDS use; 1 when the query fails, e.g. without a device).
template <typename F>
inline int occupancy_of(F kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

// C (M x N, ldc) = sum over s < S of P[s] (each M x N, tight), fixed order.
hipError_t launch_splitk_reduce_f32(const float* P, int64_t M, int64_t N, int S, float* C,
                                    int64_t ldc, hipStream_t st);

// ---- grouped launches (many independent problems in one launch) ----
// One product C = op(A) B of a grouped launch (whole contraction, no split).
struct GroupGemm {
  const void* A; int64_t lda;
  const void* B; int64_t ldb;
  void* C; int64_t ldc;
  int64_t M, N, K;
};
// Appends the workgroups (descriptor idx, tile_m, tile_n) of product g for
// a grouped launch with tile width wn (16-column blocks per wave; rounded up
// to 1, 2, 4 or 8).  gram: the 32 x 32 Gram tiling, lower tiles only (the
// part the panel kernels read).
void gemm_grouped_blocks(const GroupGemm& g, int idx, bool gram, int wn, std::vector<int4>& out);
int grouped_wn_round(int wn);
// The remainder layout (16 wn MFMA columns + 4 vector-ALU columns per tile):
// class width for a product of width d, block list, and launch.  A product
// takes the narrowest class that covers d (classes one block apart up to 9,
// so little of the tile is padding).
constexpr int kRemClasses[] = {2, 3, 4, 5, 6, 7, 8, 9, 13};
int grouped_rem_class(int64_t d);
void gemm_rem_grouped_blocks(const GroupGemm& g, int idx, int wn, Dtype dt,
                             std::vector<int4>& out);
hipError_t launch_gemm_rem_grouped(Dtype dt, int trans_a, int wn, const GroupGemm* descs,
                                   const int4* bmap, int64_t nblocks, hipStream_t st);
hipError_t launch_gemm_grouped(Dtype in_t, Dtype out_t, int trans_a, bool gram, int wn,
                               const GroupGemm* descs, const int4* bmap, int64_t nblocks,
                               hipStream_t st);

// One Cholesky factorisation (d <= CHOL_MAX_D) of a grouped launch.
struct GroupChol {
  const double* G; int64_t ldg;
  double* R; int64_t ldr;
  double* dinv;
  int* flags;
  int d;
  double tol_dep, tol_warn;
};
hipError_t launch_cholesky_grouped(const GroupChol* descs, int count, hipStream_t st);

// One triangular solve Qx = X R^+ of a grouped launch; blocks (idx, 16-row block).
struct GroupTrsm {
  const void* X; int64_t rows, ldx;
  const double* R; int64_t ldr;
  const double* dinv;
  void* Qx; int64_t ldq;
  int d;
};
void trsm_grouped_blocks(const GroupTrsm& t, int idx, std::vector<int2>& out);
hipError_t launch_trsm_grouped(Dtype dt, const GroupTrsm* descs, const int2* bmap,
                               int64_t nblocks, int dmax, hipStream_t st);

// First-order second pass of a grouped launch (one workgroup per problem):
// from G2 = Q1^T Q1 (d x d, read from its lower triangle) writes B (d x d,
// in the panel type) and R2 (double), raising FLAG_SECOND_PASS in flags.
struct GroupFirstOrder {
  const double* G2;
  void* B;
  double* R2;
  int* flags;
  int d;
  double tol;
};
hipError_t launch_first_order_grouped(Dtype dt, const GroupFirstOrder* descs, int count,
                                      hipStream_t st);
// L (d x d, ldl) = R^T of each upper-triangular R (d x d, tight); one workgroup each.
struct GroupLower {
  const double* R;
  double* L; int64_t ldl;
  int d;
};
hipError_t launch_lower_grouped(const GroupLower* descs, int count, hipStream_t st);
// Zero n ints (a kernel, so that graph capture records no memset node).
hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t st);
// dst[0..n) = src[0..n) for n <= 64 ints (a kernel: no memcpy node in a graph).
hipError_t launch_copy_ints(const int* src, int* dst, int n, hipStream_t st);

// Gaussian sketches of a grouped launch: blocks (idx, local block).
struct GroupGauss {
  void* out; int64_t m, d, ld;
  uint64_t seed;
};
void gauss_grouped_blocks(const GroupGauss& g, int idx, std::vector<int2>& out);
hipError_t launch_gaussian_grouped(Dtype dt, const GroupGauss* descs, const int2* bmap,
                                   int64_t nblocks, hipStream_t st);

// ---- learned.hip ----
// Predictor features (65 floats) from the fp64 Gram G (64 x 64, ldg) of the
// 64-column sketch; one workgroup.
hipError_t launch_features(const double* G, int64_t ldg, int k, float* feat, hipStream_t st);
// MLP layers (fp32, activations row-major, W column-major fan_in x fan_out).
hipError_t launch_linear_forward(const float* X, int ldx, const float* W, const float* bias,
                                 float* Y, int B, int nin, int nout, bool relu, hipStream_t st);
hipError_t launch_softmax_xent(const float* Z, const int* y, int B, int C, float* dZ,
                               float* loss, hipStream_t st);
hipError_t launch_linear_backward_input(const float* dY, const float* W, const float* H,
                                        float* dX, int B, int nin, int nout, hipStream_t st);
hipError_t launch_linear_backward_weight(const float* X, int ldx, const float* dY, float* dW,
                                         float* db, int B, int nin, int nout, hipStream_t st);
hipError_t launch_adam(float* theta, const float* g, float* m, float* v, int64_t count, float lr,
                       float beta1, float beta2, float eps, int64_t t, hipStream_t st);
hipError_t launch_gather(const float* X, const int* y, int64_t N, int64_t a, int64_t c,
                         int64_t start, int B, int nin, float* Xb, int* yb, hipStream_t st);
hipError_t launch_sum(const float* x, int64_t n, float scale, float* out, hipStream_t st);
hipError_t launch_argmax(const float* Z, int C, int* out, hipStream_t st);
// One feature vector -> MLP (parameters th, the layout of randqlp_mlp_forward)
// -> predicted class in *cls; out (optional, 2 * hidden + classes floats)
// receives the activations and logits.  One launch.
hipError_t launch_predict_class(const float* th, const float* feat, float* out, int* cls,
                                hipStream_t st);
// Rank network (th_k, last input rank_feat) -> rank class ck and
// k_hat = min(8 * 2^ck, k_max); then the power-round network (th_q, last
// input k_hat / 256).  out[0] = q class, out[1] = ck, out[2] = k_hat.
hipError_t launch_predict_rank_q(const float* th_q, const float* th_k, const float* feat,
                                 float rank_feat, int k_max, int* out, hipStream_t st);
// res[0] = smallest k with sqrt((nrm2 - sum_{j<k} ||L[:, j]||^2) / nrm2) <= tol
// (d if none), res[1] = that error; nrm2 is a device double.  d <= 8192.
hipError_t launch_rank_scan(const double* L, int64_t ldl, int64_t d, const double* nrm2,
                            double tol, double* res, hipStream_t st);
// ||X||_F^2 or ||X - Y||_F^2 (Y may be null) in fp64, deterministic order;
// scratch holds sumsq_scratch_bytes().
size_t sumsq_scratch_bytes();
// out = sum of the n doubles in x, fixed order.
hipError_t launch_sum_f64(const double* x, int64_t n, double* out, hipStream_t st);
hipError_t launch_sumsq(const void* X, int64_t ldx, const void* Y, int64_t ldy, int64_t rows,
                        int64_t cols, Dtype dt, double* scratch, double* out, hipStream_t st);

}  // namespace rqlp

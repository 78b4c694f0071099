// Host orchestration and C ABI of librandqlp (declared in include/randqlp.h).
//
// randqlp_factor runs the generalised Algorithm 1 (Section 3.1) as a
// stream-ordered sequence of the kernels in philox.hip, gemm.hip and
// panel.hip:
//   Omega -> Y = A^T Omega -> Qbar = orth(Y)
//   q x [ Z = A Qbar -> Q = orth(Z) -> Y = A^T Q -> Qbar = orth(Y) ]
//   Z = A Qbar -> Q = orth(Z) -> W = A^T Q -> (P, R) = orth(W) -> L = R^T
// orth() is Cholesky QR run twice (fast path) or the robust sequence
// (shifted pass, completion of dependent columns, two more passes).  Device
// kernels raise bits in a status word; the call reads it back once at the
// end and, in AUTO mode, recomputes everything with the robust orth() if a
// pass reported an unsafe pivot.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/randqlp.h"
#include "rqlp_internal.h"

using namespace rqlp;

namespace {

thread_local std::string g_last_error;

rqlp_status fail(rqlp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

}  // namespace

// The same, for the library's other translation units.
rqlp_status rqlp_fail(rqlp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

namespace {

#define HIP_TRY(expr)                   \
  do {                                  \
    hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

constexpr double kUnit = 1.1102230246251565e-16;  // 2^-53
// Fast path: a first-pass pivot below this fraction of its column's squared
// norm is at rounding level -> treat as breakdown.
constexpr double kTolDepFast = 64.0 * kUnit;
// Second pass: Q1^T Q1 should be near I; a pivot below this fraction means
// the first pass lost too much orthogonality for two passes to be enough.
constexpr double kTolWarnSecond = 0.05;
// Robust path: after the shifted pass, a pivot below this fraction of the
// column norm is numerically dependent and the column is completed.
constexpr double kTolDepRobust = 1e-12;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kPredCols = 64;  // sketch columns the predictor reads
constexpr int kRankMaxD = 4096;  // widest sketch of the rank-predicting form (rank scan in LDS)
constexpr int64_t kSparseMaxRows = (int64_t)1 << 21;  // sparse products: rows per grid dimension
// Offsets of the MLP parameters [W1 b1 W2 b2 W3 b3] (floats).
constexpr int kNI = RQLP_MLP_INPUTS, kNH = RQLP_MLP_HIDDEN, kNC = RQLP_MLP_CLASSES;
constexpr int64_t kOW1 = 0, kOB1 = kOW1 + kNI * kNH, kOW2 = kOB1 + kNH, kOB2 = kOW2 + kNH * kNH,
                  kOW3 = kOB2 + kNH, kOB3 = kOW3 + kNH * kNC, kNParams = kOB3 + kNC;
static_assert(kNParams == RQLP_MLP_PARAMS, "MLP parameter count");
// The error judge accepts q_predicted when one more power round would lower
// the squared residual by at most this fraction: (1 + 0.02)^2 - 1.
constexpr double kJudgeSlack = 0.0404;

struct Layout {
  size_t m1, m2, n1, n2, part, part_bytes, G, R[4], Racc[2], Rfin, dinv, colf, scal, flags,
      chs, tsub, tsr, a16, at16, p16, a16lo, p16lo, amax, total;
  int64_t ld16, ldt16;  // leading dimensions of the 16-bit copies of A and A^T
  int64_t ldp16;        // contraction extent of the packed 16-bit copy of a panel
  // predictor and error judge (randqlp_factor_auto only)
  size_t y64, g64, feat, mlp, cls, jd, sums, sres, rerr;
  size_t part2, part2_bytes;  // split-K scratch of the predictor's products
  size_t flags_bytes;  // status words cleared at the start of a call
  int64_t omega_cols;  // columns of Omega drawn into m1: d, or at least the
                       // predictor's kPredCols when the predictor reads them
};

size_t elem_size(Dtype dt) { return dt == DT_F64 ? 8 : 4; }

// mixed: 16-bit copies of A for the sketch and power products; split: also
// the bf16 residual of A and of the panel for the split final projection.
Layout make_layout(int64_t m, int64_t n, int64_t d, Dtype dt, bool mixed = false,
                   bool autoq = false, bool split = false) {
  Layout L;
  const size_t es = elem_size(dt);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  // Omega lives in m1 at the start of a call; the predictor reads its leading
  // kPredCols columns, so m1 holds at least that many (the Gaussian is
  // indexed by i + j m, so the method's own d columns are unchanged).
  L.omega_cols = autoq ? std::max<int64_t>(d, kPredCols) : d;
  L.m1 = take((size_t)m * L.omega_cols * es);
  L.m2 = take((size_t)m * d * es);
  L.n1 = take((size_t)n * d * es);
  L.n2 = take((size_t)n * d * es);
  size_t part = 0;
  part = std::max(part, gemm_partial_bytes(1, n, d, m, dt, dt, false));
  part = std::max(part, gemm_partial_bytes(0, m, d, n, dt, dt, false));
  part = std::max(part, gemm_partial_bytes(1, d, d, m, dt, DT_F64, true));
  part = std::max(part, gemm_partial_bytes(1, d, d, n, dt, DT_F64, true));
  for (int64_t dd = d; dd > CHOL_MAX_D; dd -= CHOL_MAX_D)  // Schur-complement Grams
    part = std::max(part, gemm_partial_bytes(1, dd - CHOL_MAX_D, dd - CHOL_MAX_D, CHOL_MAX_D,
                                             DT_F64, DT_F64, true));
  for (int64_t j0 = CHOL_MAX_D; j0 < d; j0 += CHOL_MAX_D)  // blocked TRSM products
    for (int64_t rows : {m, n})
      part = std::max(part, gemm_partial_bytes(0, rows, std::min<int64_t>(CHOL_MAX_D, d - j0),
                                               j0, dt, dt, false));
  if (mixed) {
    for (bool f16 : {false, true}) {
      part = std::max(part, gemm16_partial_bytes(n, d, m, f16));
      part = std::max(part, gemm16_partial_bytes(m, d, n, f16));
    }
    if (split) part = std::max(part, gemm16_partial_bytes(n, d, m, false, 3));
  }
  size_t part2 = 0;
  if (autoq) {
    // the predictor runs on a second stream beside the first sketch: its
    // products get their own split-K scratch
    part2 = std::max(part2, gemm_partial_bytes(1, n, kPredCols, m, dt, dt, false));
    part2 = std::max(part2, gemm_partial_bytes(1, kPredCols, kPredCols, n, dt, DT_F64, true));
    part = std::max(part, gemm_partial_bytes(1, d, d, m, dt, dt, false));
    part = std::max(part, gemm_partial_bytes(0, m, d, d, dt, dt, false));
  }
  L.part = take(part);
  L.part_bytes = part;
  L.part2 = autoq ? take(std::max<size_t>(part2, 256)) : 0;
  L.part2_bytes = autoq ? std::max<size_t>(part2, 256) : 0;
  L.G = take((size_t)d * d * 8);
  for (int i = 0; i < 4; ++i) L.R[i] = take((size_t)d * d * 8);
  for (int i = 0; i < 2; ++i) L.Racc[i] = take((size_t)d * d * 8);
  L.Rfin = take((size_t)d * d * 8);
  L.chs = take((size_t)4 * d * d * 8);  // blocked Cholesky: off-diagonal solve + Schur blocks
  if (d > CHOL_MAX_D) {  // blocked TRSM: P of one column block, fp32 copy of R's block column
    L.tsub = take((size_t)std::max(m, n) * CHOL_MAX_D * es);
    L.tsr = take((size_t)d * CHOL_MAX_D * 4);
  } else {
    L.tsub = L.tsr = 0;
  }
  L.dinv = take((size_t)((d + 15) / 16) * 256 * 8);
  L.colf = take((size_t)d * 4);
  if (mixed) {
    L.ld16 = gemm16_ld(m);
    L.ldt16 = gemm16_ld(n);
    L.a16 = take(gemm16_packed_bytes(n, m));
    L.at16 = take(gemm16_packed_bytes(m, n));
    L.ldp16 = gemm16_ld(std::max(m, n));
    L.p16 = take(gemm16_panel_bytes(L.ldp16, d));
    L.amax = take(16);  // max |a| of the fp16 form's scale
  } else {
    L.ld16 = L.ldt16 = L.ldp16 = 0;
    L.a16 = L.at16 = L.p16 = L.amax = 0;
  }
  if (mixed && split) {
    L.a16lo = take(gemm16_packed_bytes(n, m));
    L.p16lo = take(gemm16_panel_bytes(L.ldp16, d));
  } else {
    L.a16lo = L.p16lo = 0;
  }
  if (autoq) {
    L.y64 = take((size_t)n * kPredCols * es);
    L.g64 = take((size_t)kPredCols * kPredCols * 8);
    L.feat = take(RQLP_MLP_INPUTS * 4);
    L.mlp = take((2 * RQLP_MLP_HIDDEN + RQLP_MLP_CLASSES) * 4);
    L.cls = take(16);
    L.jd = take((size_t)d * d * es);
    L.sums = take(sumsq_scratch_bytes());
    L.sres = take(8 * 8);
    L.rerr = mixed ? take((size_t)convert16_blocks(m, n) * 2 * 8) : 0;
  } else {
    L.y64 = L.g64 = L.feat = L.mlp = L.cls = L.jd = L.sums = L.sres = L.rerr = 0;
  }
  L.scal = take(64);
  L.flags = take(64);
  L.flags_bytes = 64;
  L.total = off;
  return L;
}

// Library-managed workspace: one growing buffer per (device, stream).  A call
// holds its entry's lock until it returns (every such call completes its work
// before returning), so calls on one stream are serialised and calls on
// different streams run independently.
struct WsEntry {
  int dev = 0;
  hipStream_t st = nullptr;
  std::mutex mu;
  void* ptr = nullptr;
  size_t size = 0;
};
struct WsCache {
  std::mutex mu;  // guards the list, not the buffers
  std::vector<std::unique_ptr<WsEntry>> entries;
};
WsCache g_ws;

struct Ctx {
  hipStream_t st;
  Dtype dt;
  int mixed = 0;  // 0: no; 1: bf16 products; 2: fp16 products; 3: bf16 + split projection
  bool noalloc = false;  // no allocation of any kind (static scratch, pageable read-backs)
  // sparse input: A and A^T in CSR form, and the panel scratch of the sparse
  // products (offsets into ws); null for a dense A
  const CsrView* sp = nullptr;
  const CsrView* spt = nullptr;
  size_t sp_xr = 0, sp_cr = 0;
  size_t extra_off = 0;  // start of the caller-specific region after the layout
  char* ws;
  Layout lay;
  int64_t d;
  uint64_t seed;
  int orth_calls;
  template <typename T>
  T* at(size_t off) const {
    return (T*)(ws + off);
  }
  int* flags() const { return at<int>(lay.flags); }
};

// Optional kernel timing of the products with A (the dominant kernel): HIP
// events recorded on the call's stream around each launch, read after the
// call has synchronised.  Diagnostics only; not thread-safe.
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<double> work_flops, work_bytes;
  size_t used = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
  long long launches = 0;
};
Prof g_prof;

void prof_collect() {
  for (size_t i = 0; i < g_prof.used; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) == hipSuccess) {
      g_prof.ms += t;
      g_prof.flops += g_prof.work_flops[i];
      g_prof.bytes += g_prof.work_bytes[i];
      g_prof.launches += 1;
    }
  }
  g_prof.used = 0;
}

hipError_t gemm(Ctx& c, int trans_a, const void* A, int64_t lda, const void* B, int64_t ldb,
                void* C, int64_t ldc, int64_t M, int64_t N, int64_t K, Dtype in_t, Dtype out_t,
                bool gram, bool timed = false) {
  GemmArgs g;
  g.trans_a = trans_a;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.in_t = in_t;
  g.out_t = out_t;
  g.gram = gram;
  g.partial = c.ws + c.lay.part;
  g.partial_bytes = c.lay.part_bytes;
  if (timed && g_prof.on && !c.noalloc) {
    const size_t i = g_prof.used++;
    while (g_prof.ev.size() < 2 * g_prof.used) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
      g_prof.ev.push_back(e);
    }
    g_prof.work_flops.resize(g_prof.used);
    g_prof.work_bytes.resize(g_prof.used);
    const double es = (in_t == DT_F64) ? 8.0 : 4.0;
    g_prof.work_flops[i] = 2.0 * (double)M * (double)N * (double)K;
    g_prof.work_bytes[i] = es * ((double)M * K + (double)K * N + (double)M * N);
    g.ev_begin = g_prof.ev[2 * i];
    g.ev_end = g_prof.ev[2 * i + 1];
  }
  return launch_gemm(g, c.st);
}

// Precision-form product C (rows x d, fp32) = op(A) X on the 16-bit copies:
// trans_a = 1 uses A16 (C = A^T X, rows = n, K = m), trans_a = 0 uses the
// copy of A^T (C = A X, rows = m, K = n).  X is rounded to 16 bits first.
// split (trans_a = 1, bf16): the three-term product with the residuals of A
// and X, which approximates the fp32 product.
hipError_t gemm16(Ctx& c, int trans_a, int64_t m, int64_t n, const float* X, int64_t ldx,
                  float* C, int64_t ldc, int64_t d, bool split = false) {
  Gemm16Args g;
  g.f16 = (c.mixed == 2);
  g.A = trans_a ? (const void*)(c.ws + c.lay.a16) : (const void*)(c.ws + c.lay.at16);
  g.lda = trans_a ? c.lay.ld16 : c.lay.ldt16;
  g.B = c.ws + c.lay.p16;
  g.ldb = c.lay.ldp16;
  g.C = C;
  g.ldc = ldc;
  g.M = trans_a ? n : m;
  g.N = d;
  g.K = trans_a ? m : n;
  g.partial = c.ws + c.lay.part;
  g.partial_bytes = c.lay.part_bytes;
  if (split) {
    if (!trans_a || g.f16 || !c.lay.a16lo) return hipErrorInvalidValue;
    g.A2 = c.ws + c.lay.a16lo;
    g.B2 = c.ws + c.lay.p16lo;
  }
  hipError_t e = launch_convert_panel16(X, g.K, d, ldx, c.ws + c.lay.p16, c.lay.ldp16, g.f16, c.st,
                                        split ? c.ws + c.lay.p16lo : nullptr);
  if (e != hipSuccess) return e;
  if (g_prof.on && !c.noalloc) {
    const size_t i = g_prof.used++;
    while (g_prof.ev.size() < 2 * g_prof.used) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) return hipErrorOutOfMemory;
      g_prof.ev.push_back(ev);
    }
    g_prof.work_flops.resize(g_prof.used);
    g_prof.work_bytes.resize(g_prof.used);
    g_prof.work_flops[i] = 2.0 * (double)g.M * (double)g.N * (double)g.K;
    g_prof.work_bytes[i] = 2.0 * ((double)g.M * g.K + (double)g.K * g.N) + 4.0 * (double)g.M * g.N;
    g.ev_begin = g_prof.ev[2 * i];
    g.ev_end = g_prof.ev[2 * i + 1];
  }
  return launch_gemm16(g, c.st);
}

// Cholesky of G + shift I for any d <= RQLP_MAX_D into R (ldr) and the
// diagonal-block inverses.  Right-looking, in blocks of CHOL_MAX_D columns:
// the diagonal block on the one-workgroup kernel; R12 = R11^{-T} G12,
// computed as the TRSM of G21 = G12^T; the Schur complement
// G22 - R12^T R12 through the Gram product; then the same on the complement.
// The complements alternate between two tight buffers, so the scratch stays
// at 3 d^2 + CHOL_MAX_D d doubles for any d.  Pivot tolerances stay relative
// to the original diagonal (odiag_src when given, else G's own).  The shift
// applies to the original diagonal only.
hipError_t chol_any(Ctx& c, const double* G, int64_t d, int64_t ldg, double shift,
                    const double* shift_dev, double tol_dep, double tol_warn, double* R,
                    int64_t ldr, double* dinv, int* col_flags, const double* odiag_src,
                    int64_t odiag_stride, double* scratch) {
  if (d <= CHOL_MAX_D)
    return launch_cholesky_tile(G, d, ldg, shift, shift_dev, tol_dep, tol_warn, R, ldr, dinv,
                                col_flags, c.flags(), odiag_src, odiag_stride, c.st);
  double* Wbuf[2] = {scratch, scratch + d * d};  // trailing complements, tight
  double* C = scratch + 2 * d * d;                // R12^T R12
  double* Xs = C + d * d;                         // G21 R11^{-1} = R12^T
  const double* src = G;                          // current trailing block
  int64_t lds = ldg;
  for (int64_t j0 = 0, lvl = 0; j0 < d; j0 += CHOL_MAX_D, ++lvl) {
    const int64_t b = std::min<int64_t>(CHOL_MAX_D, d - j0), d2 = d - j0 - b;
    const bool top = (j0 == 0);
    // original diagonal of this block (for the pivot tolerances)
    const double* od = top ? odiag_src
                           : (odiag_src ? odiag_src + j0 * odiag_stride : G + j0 + j0 * ldg);
    const int64_t ods = top ? odiag_stride : (odiag_src ? odiag_stride : ldg + 1);
    double* Rjj = R + j0 + j0 * ldr;
    HIP_TRY(launch_cholesky_tile(src, b, lds, top ? shift : 0.0, top ? shift_dev : nullptr,
                                 tol_dep, tol_warn, Rjj, ldr, dinv + (j0 / 16) * 256,
                                 col_flags ? col_flags + j0 : nullptr, c.flags(), od, ods,
                                 c.st));
    if (d2 == 0) break;
    HIP_TRY(launch_trsm(src + b, d2, b, lds, Rjj, ldr, dinv + (j0 / 16) * 256, Xs, d2, DT_F64,
                        c.st));
    double* R12 = R + j0 + (j0 + b) * ldr;
    HIP_TRY(launch_transpose(Xs, d2, b, d2, R12, ldr, c.st));
    HIP_TRY(launch_zero_block(R + (j0 + b) + j0 * ldr, d2, b, ldr, c.st));
    HIP_TRY(gemm(c, 1, R12, ldr, R12, ldr, C, d2, d2, d2, b, DT_F64, DT_F64, true));
    double* S = Wbuf[lvl & 1];
    HIP_TRY(launch_schur(src + b + b * lds, lds, C, d2, top ? shift : 0.0,
                         top ? shift_dev : nullptr, S, c.st));
    src = S;
    lds = d2;
  }
  return hipSuccess;
}

// Qx = X R^+ (rows x d; Qx may be X with the same ld).  Up to CHOL_MAX_D
// columns this is one TRSM launch.  Wider panels go in column blocks of
// CHOL_MAX_D: for block j, one product over all finished columns gives
// P_j = Q_{<j} R_{<j,j}, and the TRSM solves (X_j - P_j) R_jj^{-1}.  The
// product runs in the panel's precision (fp32 panels use an fp32 copy of
// R's block column).
hipError_t trsm_any(Ctx& c, const void* X, int64_t rows, int64_t ldx, const double* R,
                    int64_t ldr, const double* dinv, void* Qx, int64_t ldq) {
  const int64_t d = c.d;
  if (d <= CHOL_MAX_D) return launch_trsm(X, rows, d, ldx, R, ldr, dinv, Qx, ldq, c.dt, c.st);
  const size_t es = elem_size(c.dt);
  void* P = c.ws + c.lay.tsub;
  for (int64_t j0 = 0; j0 < d; j0 += CHOL_MAX_D) {
    const int64_t bj = std::min<int64_t>(CHOL_MAX_D, d - j0);
    const void* Xj = (const char*)X + (size_t)j0 * ldx * es;
    void* Qj = (char*)Qx + (size_t)j0 * ldq * es;
    const double* Rjj = R + j0 + j0 * ldr;
    const double* dj = dinv + (j0 / 16) * 256;
    if (j0 == 0) {
      HIP_TRY(launch_trsm(Xj, rows, bj, ldx, Rjj, ldr, dj, Qj, ldq, c.dt, c.st));
      continue;
    }
    const void* Rb = R + j0 * ldr;
    int64_t ldrb = ldr;
    if (c.dt == DT_F32) {
      HIP_TRY(launch_copy_panel(R + j0 * ldr, DT_F64, ldr, c.ws + c.lay.tsr, DT_F32, j0, j0, bj,
                                c.st));
      Rb = c.ws + c.lay.tsr;
      ldrb = j0;
    }
    HIP_TRY(gemm(c, 0, Qx, ldq, Rb, ldrb, P, rows, rows, bj, j0, c.dt, c.dt, false));
    HIP_TRY(launch_trsm(Xj, rows, bj, ldx, Rjj, ldr, dj, Qj, ldq, c.dt, c.st, P, rows));
  }
  return hipSuccess;
}

// One Cholesky QR pass: X (rows x d) -> Qx = X R^+, R into Rbuf.
hipError_t chol_pass(Ctx& c, const void* X, int64_t rows, int64_t ldx, void* Qx, int64_t ldq,
                     double* Rbuf, const double* shift_dev, double tol_dep, double tol_warn,
                     int* col_flags) {
  const int64_t d = c.d;
  double* G = c.at<double>(c.lay.G);
  double* dinv = c.at<double>(c.lay.dinv);
  HIP_TRY(gemm(c, 1, X, ldx, X, ldx, G, d, d, d, rows, c.dt, DT_F64, true));
  HIP_TRY(chol_any(c, G, d, d, 0.0, shift_dev, tol_dep, tol_warn, Rbuf, d, dinv, col_flags,
                   nullptr, 0, c.at<double>(c.lay.chs)));
  return trsm_any(c, X, rows, ldx, Rbuf, d, dinv, Qx, ldq);
}

// Panel QR strategies, cheapest first.
//  FAST     intermediate panels (whose range is all the next product uses):
//           one Cholesky QR pass, in place.  Final panels (Q and P): one
//           pass, then the second pass to first order in E = Q1^T Q1 - I.
//  CHOLQR2  two full Cholesky QR passes on every panel.
//  ROBUST   shifted pass, completion of dependent columns, two more passes.
enum PanelMode { PM_FAST = 0, PM_CHOLQR2 = 1, PM_ROBUST = 2 };

// max |E| for which the first-order second pass is used; the neglected terms
// are O(|E|^2), so the final Q and P keep an orthogonality error of about
// |E|^2: at most 1e-16 for fp64 panels (the rounding level), and at most
// 1e-6 (about 17 fp32 units) for fp32 panels, whose factors are held to the
// error bar of the reduced-precision forms (1.05x the fp64 error) rather than
// to fp32 rounding; a larger |E| raises FLAG_SECOND_PASS and the call reruns
// with two full passes.
double first_order_tol(Dtype dt) { return dt == DT_F64 ? 1e-8 : 1e-3; }

// orth(): X (rows x d, ldx) -> out (rows x d, ldo), using tmp (rows x d,
// ld = rows).  out may alias X (same ld); tmp may alias neither.  If Rout is
// given it receives R with X = out * R.  final_panel selects the two-pass
// treatment in FAST mode.
hipError_t orth(Ctx& c, const void* X, int64_t rows, int64_t ldx, void* out, int64_t ldo,
                void* tmp, double* Rout, PanelMode mode, bool final_panel) {
  const int64_t d = c.d;
  double* R[4] = {c.at<double>(c.lay.R[0]), c.at<double>(c.lay.R[1]),
                  c.at<double>(c.lay.R[2]), c.at<double>(c.lay.R[3])};
  const int call = c.orth_calls++;
  double* G = c.at<double>(c.lay.G);
  if (mode == PM_FAST) {
    if (!final_panel) {
      // out = X R^{-1}; the TRSM may run in place (each wave reads a block
      // of its own rows before overwriting it).
      return chol_pass(c, X, rows, ldx, out, ldo, R[0], nullptr, kTolDepFast, 0.0, nullptr);
    }
    HIP_TRY(chol_pass(c, X, rows, ldx, tmp, rows, R[0], nullptr, kTolDepFast, 0.0, nullptr));
    HIP_TRY(gemm(c, 1, tmp, rows, tmp, rows, G, d, d, d, rows, c.dt, DT_F64, true));
    HIP_TRY(launch_first_order_pass(G, d, first_order_tol(c.dt), R[2], R[1], c.flags(), c.st));
    const void* B = R[2];
    if (c.dt == DT_F32) {
      HIP_TRY(launch_copy_panel(R[2], DT_F64, d, R[3], DT_F32, d, d, d, c.st));
      B = R[3];
    }
    HIP_TRY(gemm(c, 0, tmp, rows, B, d, out, ldo, rows, d, d, c.dt, c.dt, false));
    if (Rout) HIP_TRY(gemm(c, 0, R[1], d, R[0], d, Rout, d, d, d, d, DT_F64, DT_F64, false));
    return hipSuccess;
  }
  if (mode == PM_CHOLQR2) {
    HIP_TRY(chol_pass(c, X, rows, ldx, tmp, rows, R[0], nullptr, kTolDepFast, 0.0, nullptr));
    HIP_TRY(chol_pass(c, tmp, rows, rows, out, ldo, R[1], nullptr, kTolDepFast, kTolWarnSecond,
                      nullptr));
    if (Rout) HIP_TRY(gemm(c, 0, R[1], d, R[0], d, Rout, d, d, d, d, DT_F64, DT_F64, false));
    return hipSuccess;
  }
  double* scal = c.at<double>(c.lay.scal);
  int* colf = c.at<int>(c.lay.colf);
  // pass 1: shifted Cholesky QR, shift = 11 (rows d + d (d + 1)) u ||X||_F^2
  HIP_TRY(gemm(c, 1, X, ldx, X, ldx, G, d, d, d, rows, c.dt, DT_F64, true));
  HIP_TRY(launch_trace(G, d, d, scal, c.st));
  const double cshift = 11.0 * ((double)rows * d + (double)d * (d + 1)) * kUnit;
  HIP_TRY(launch_scale_scalar(scal, cshift, scal + 1, c.st));
  double* dinv = c.at<double>(c.lay.dinv);
  HIP_TRY(chol_any(c, G, d, d, 0.0, scal + 1, 0.0, 0.0, R[0], d, dinv, nullptr, nullptr, 0,
                   c.at<double>(c.lay.chs)));
  HIP_TRY(trsm_any(c, X, rows, ldx, R[0], d, dinv, tmp, rows));
  // pass 2: detect dependent columns (zeroed), then complete them
  HIP_TRY(chol_pass(c, tmp, rows, rows, out, ldo, R[1], nullptr, kTolDepRobust, 0.0, colf));
  HIP_TRY(launch_count_flags(colf, d, c.flags() + 2, c.st));
  HIP_TRY(launch_gaussian_columns(out, rows, ldo, colf, d, c.seed, 0x1000ull + (uint64_t)call,
                                  c.dt, c.st));
  // passes 3 and 4: Cholesky QR twice on the completed panel
  HIP_TRY(chol_pass(c, out, rows, ldo, tmp, rows, R[2], nullptr, 0.0, 0.0, nullptr));
  HIP_TRY(chol_pass(c, tmp, rows, rows, out, ldo, R[3], nullptr, 0.0, 0.0, nullptr));
  if (Rout) {
    double* A0 = c.at<double>(c.lay.Racc[0]);
    double* A1 = c.at<double>(c.lay.Racc[1]);
    HIP_TRY(gemm(c, 0, R[1], d, R[0], d, A0, d, d, d, d, DT_F64, DT_F64, false));
    HIP_TRY(gemm(c, 0, R[2], d, A0, d, A1, d, d, d, d, DT_F64, DT_F64, false));
    HIP_TRY(gemm(c, 0, R[3], d, A1, d, Rout, d, d, d, d, DT_F64, DT_F64, false));
  }
  return hipSuccess;
}

struct FactorArgs {
  const void* A;
  int64_t m, n, lda;
  int q;
  void* Q;
  int64_t ldq;
  double* L;
  int64_t ldl;
  void* P;
  int64_t ldp;
};

// A product of the power iteration with A: C (rows x d) = op(A) X.  The
// precision form runs it on the 16-bit copies; `full` (the final projection)
// asks for fp32 accuracy: the fp32 product, or the split bf16 product.
hipError_t prod(Ctx& c, const FactorArgs& f, int trans_a, const void* X, int64_t ldx, void* C,
                int64_t ldc, bool full = false) {
  if (c.sp)  // sparse A: A^T X uses the CSR form of A^T
    return launch_spmm(trans_a ? *c.spt : *c.sp, X, ldx, c.d, C, ldc, c.dt, c.ws + c.sp_xr,
                       c.ws + c.sp_cr, c.st);
  const int64_t rows = trans_a ? f.n : f.m, K = trans_a ? f.m : f.n;
  if (c.mixed && !full)
    return gemm16(c, trans_a, f.m, f.n, (const float*)X, ldx, (float*)C, ldc, c.d);
  if (c.mixed == 3 && trans_a)
    return gemm16(c, 1, f.m, f.n, (const float*)X, ldx, (float*)C, ldc, c.d, true);
  return gemm(c, trans_a, f.A, f.lda, X, ldx, C, ldc, rows, c.d, K, c.dt, c.dt, false, true);
}

// Stages of the generalised Algorithm 1.  Panels: Zm / Tm (m x d) and
// Yn / Tn (n x d) in the workspace; Qbar lives in Yn between stages.
// start: Omega (in Zm), then the 16-bit copies of A, Y = A^T Omega and
// Qbar = orth(Y).
hipError_t stage_omega(Ctx& c, const FactorArgs& f) {
  return launch_gaussian(c.ws + c.lay.m1, f.m, c.lay.omega_cols, f.m, c.seed, 0, c.dt,
                         c.st);                                                // randn
}

hipError_t stage_sketch(Ctx& c, const FactorArgs& f, PanelMode mode) {
  const int64_t m = f.m, n = f.n;
  void* Zm = c.ws + c.lay.m1;
  void* Yn = c.ws + c.lay.n1;
  void* Tn = c.ws + c.lay.n2;
  if (c.mixed)  // (fp16: the copies carry a power-of-two scale, exponent in flags[3])
    HIP_TRY(launch_convert16((const float*)f.A, m, n, f.lda, c.ws + c.lay.a16, c.lay.ld16,
                             c.ws + c.lay.at16, c.lay.ldt16, c.mixed == 2, c.st,
                             c.lay.rerr ? c.at<double>(c.lay.rerr) : nullptr,
                             c.lay.a16lo ? c.ws + c.lay.a16lo : nullptr, nullptr,
                             c.at<unsigned>(c.lay.amax), c.flags() + 3));
  HIP_TRY(prod(c, f, 1, Zm, m, Yn, n));                                        // A^T Omega
  return orth(c, Yn, n, n, Yn, n, Tn, nullptr, mode, false);                   // Qbar
}

hipError_t stage_start(Ctx& c, const FactorArgs& f, PanelMode mode) {
  HIP_TRY(stage_omega(c, f));
  return stage_sketch(c, f, mode);
}

// `count` power rounds: Q = orth(A Qbar), Qbar = orth(A^T Q).
hipError_t stage_rounds(Ctx& c, const FactorArgs& f, PanelMode mode, int count) {
  const int64_t m = f.m, n = f.n;
  void* Zm = c.ws + c.lay.m1;
  void* Tm = c.ws + c.lay.m2;
  void* Yn = c.ws + c.lay.n1;
  void* Tn = c.ws + c.lay.n2;
  for (int it = 0; it < count; ++it) {
    HIP_TRY(prod(c, f, 0, Yn, n, Zm, m));                                      // A Qbar
    HIP_TRY(orth(c, Zm, m, m, Zm, m, Tm, nullptr, mode, false));
    HIP_TRY(prod(c, f, 1, Zm, m, Yn, n));                                      // A^T Q
    HIP_TRY(orth(c, Yn, n, n, Yn, n, Tn, nullptr, mode, false));
  }
  return hipSuccess;
}

// From Z = A Qbar (in Zm): Q = orth(Z), W = A^T Q, (P, R) = orth(W), L = R^T.
hipError_t stage_finish_from_z(Ctx& c, const FactorArgs& f, PanelMode mode) {
  const int64_t m = f.m, n = f.n, d = c.d;
  void* Zm = c.ws + c.lay.m1;
  void* Tm = c.ws + c.lay.m2;
  void* Yn = c.ws + c.lay.n1;
  void* Tn = c.ws + c.lay.n2;
  double* Rfin = c.at<double>(c.lay.Rfin);
  HIP_TRY(orth(c, Zm, m, m, f.Q, f.ldq, Tm, nullptr, mode, true));             // Q
  HIP_TRY(prod(c, f, 1, f.Q, f.ldq, Yn, n, true));                             // A^T Q
  HIP_TRY(orth(c, Yn, n, n, f.P, f.ldp, Tn, Rfin, mode, true));                // P, R
  return launch_lower_from_upper(Rfin, d, f.L, f.ldl, c.st);                  // L = R^T
}

// Z = A Qbar, then stage_finish_from_z.
hipError_t stage_finish(Ctx& c, const FactorArgs& f, PanelMode mode) {
  HIP_TRY(prod(c, f, 0, c.ws + c.lay.n1, f.n, c.ws + c.lay.m1, f.m));          // A Qbar
  return stage_finish_from_z(c, f, mode);
}

// Zero the status words with a fill kernel (no memset node if captured).
hipError_t clear_flags(Ctx& c) {
  return launch_zero_ints(c.flags(), (int64_t)(c.lay.flags_bytes / sizeof(int)), c.st);
}

hipError_t run_pipeline(Ctx& c, const FactorArgs& f, PanelMode mode) {
  c.orth_calls = 0;
  HIP_TRY(clear_flags(c));
  HIP_TRY(stage_start(c, f, mode));
  HIP_TRY(stage_rounds(c, f, mode, f.q));
  return stage_finish(c, f, mode);
}

}  // namespace

extern "C" {

void rqlp_opts_default(rqlp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->precision = RQLP_F64;
  o->panel_qr = RQLP_PANEL_AUTO;
}

int64_t randqlp_sketch_width(int64_t m, int64_t n, int k, int p) {
  if (m < 1 || n < 1 || k < 1 || p < 0) return -1;
  int64_t d = (int64_t)k + p;
  if (d > m) d = m;
  if (d > n) d = n;
  return d;
}

const char* randqlp_status_string(rqlp_status s) {
  switch (s) {
    case RQLP_OK: return "RQLP_OK";
    case RQLP_E_INVALID_ARG: return "RQLP_E_INVALID_ARG";
    case RQLP_E_NONFINITE: return "RQLP_E_NONFINITE";
    case RQLP_E_NOMEM: return "RQLP_E_NOMEM";
    case RQLP_E_WORKSPACE: return "RQLP_E_WORKSPACE";
    case RQLP_E_HIP: return "RQLP_E_HIP";
    case RQLP_E_UNSUPPORTED: return "RQLP_E_UNSUPPORTED";
  }
  return "RQLP_E_UNKNOWN";
}

const char* randqlp_last_error(void) { return g_last_error.c_str(); }

#ifndef RQLP_BUILD_ID
#define RQLP_BUILD_ID "unknown"
#endif
const char* randqlp_build_id(void) { return RQLP_BUILD_ID; }

void randqlp_profile_enable(int on) {
  g_prof.on = (on != 0);
  g_prof.used = 0;
}

void randqlp_profile_read(double* ms, int64_t* launches, double* flops, double* bytes) {
  if (ms) *ms = g_prof.ms;
  if (launches) *launches = g_prof.launches;
  if (flops) *flops = g_prof.flops;
  if (bytes) *bytes = g_prof.bytes;
  g_prof.ms = g_prof.flops = g_prof.bytes = 0.0;
  g_prof.launches = 0;
}

size_t randqlp_workspace_size(int64_t m, int64_t n, int k, int p, int q, const rqlp_opts* o) {
  const int64_t d = randqlp_sketch_width(m, n, k, p);
  if (d < 1 || q < 0) return 0;
  const int prec = o ? o->precision : RQLP_F64;
  if (prec < RQLP_F64 || prec > RQLP_MIXED_BF16X3) return 0;
  return make_layout(m, n, d, prec == RQLP_F64 ? DT_F64 : DT_F32, prec >= RQLP_MIXED_BF16, false,
                     prec == RQLP_MIXED_BF16X3)
      .total;
}

}  // extern "C"

namespace {

// Acquire `bytes` of device scratch: the caller's buffer or the cache entry
// of (current device, o.stream), grown under that entry's lock, which stays
// held (in lk) until the call returns.
rqlp_status acquire_ws(const rqlp_opts& o, size_t bytes, char** out,
                       std::unique_lock<std::mutex>& lk) {
  if (o.workspace != nullptr) {
    if (o.workspace_bytes < bytes)
      return fail(RQLP_E_WORKSPACE, "workspace has %zu bytes, %zu needed", o.workspace_bytes,
                  bytes);
    *out = (char*)o.workspace;
    return RQLP_OK;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RQLP_E_HIP, "hipGetDevice failed");
  const hipStream_t st = (hipStream_t)o.stream;
  WsEntry* ent = nullptr;
  {
    std::lock_guard<std::mutex> g(g_ws.mu);
    for (auto& e : g_ws.entries)
      if (e->dev == dev && e->st == st) ent = e.get();
    if (!ent) {
      g_ws.entries.emplace_back(new WsEntry);
      ent = g_ws.entries.back().get();
      ent->dev = dev;
      ent->st = st;
    }
  }
  lk = std::unique_lock<std::mutex>(ent->mu);
  if (ent->size < bytes) {
    if (ent->ptr) {
      // earlier calls on this stream have completed (each synchronises)
      (void)hipStreamSynchronize(st);
      (void)hipFree(ent->ptr);
      ent->ptr = nullptr;
      ent->size = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(RQLP_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    ent->ptr = p;
    ent->size = bytes;
  }
  *out = (char*)ent->ptr;
  return RQLP_OK;
}

// Small read-backs (status words, sums, the predicted class): up to two
// device ranges copied into a pinned buffer of the calling thread (256 bytes,
// allocated on first use, usable from every device, kept until the process
// ends), one stream synchronisation, then copied out.  A copy straight to
// pageable memory measured about 10 us more.
hipError_t read_back(hipStream_t st, void* h0, const void* d0, size_t n0, void* h1 = nullptr,
                     const void* d1 = nullptr, size_t n1 = 0, bool pinned = true) {
  constexpr size_t kPin = 256;
  thread_local char* pin = nullptr;
  if (!pinned) {  // straight to the caller's (pageable) memory: nothing allocated
    HIP_TRY(hipMemcpyAsync(h0, d0, n0, hipMemcpyDeviceToHost, st));
    if (n1) HIP_TRY(hipMemcpyAsync(h1, d1, n1, hipMemcpyDeviceToHost, st));
    return hipStreamSynchronize(st);
  }
  if (!pin && hipHostMalloc((void**)&pin, kPin, hipHostMallocPortable) != hipSuccess) {
    (void)hipGetLastError();
    pin = nullptr;
  }
  if (!pin || n0 + n1 > kPin) {  // pageable copies
    HIP_TRY(hipMemcpyAsync(h0, d0, n0, hipMemcpyDeviceToHost, st));
    if (n1) HIP_TRY(hipMemcpyAsync(h1, d1, n1, hipMemcpyDeviceToHost, st));
    return hipStreamSynchronize(st);
  }
  HIP_TRY(hipMemcpyAsync(pin, d0, n0, hipMemcpyDeviceToHost, st));
  if (n1) HIP_TRY(hipMemcpyAsync(pin + n0, d1, n1, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::memcpy(h0, pin, n0);
  if (n1) std::memcpy(h1, pin + n0, n1);
  return hipSuccess;
}

rqlp_status read_flags(Ctx& c, int host[4]) {
  hipError_t e = read_back(c.st, host, c.flags(), 4 * sizeof(int), nullptr, nullptr, 0,
                           !c.noalloc);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "status read-back: %s", hipGetErrorString(e));
  if (g_prof.on) prof_collect();
  return RQLP_OK;
}


// ---- static scratch of randqlp_factor_noalloc
// Device memory that the library never allocates at run time: a file-scope
// array that each device holds from the time the library's code object is
// loaded on it until the process ends.  Host code must not pass `scratch`
// itself to a kernel (on the host it only names the symbol): the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and only that address is used.
constexpr size_t kStaticScratchBytes = (size_t)RQLP_NOALLOC_SCRATCH_BYTES;

}  // namespace

static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;            // guards g_scratch_ptr
void* g_scratch_ptr[64] = {};       // device address of `scratch` per device
std::mutex g_scratch_call_mu[64];   // one randqlp_factor_noalloc call per device at a time

// Device address of the static scratch on device `dev` (current).
rqlp_status static_scratch(int dev, char** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(RQLP_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = (char*)g_scratch_ptr[dev];
  return RQLP_OK;
}

// Rank classes of the rank network: class c means k = 8 * 2^c, capped at
// the caller's k_max.
constexpr int kRankClasses = RQLP_MLP_CLASSES;
int rank_of_class(int c, int k_max) { return std::min(8 << c, k_max); }

// Workspace of the rank-predicting form: the largest layout among the sketch
// widths the predicted rank can give (each class, and k_max).
size_t rank_layout_bytes(int64_t m, int64_t n, int p, int k_max, Dtype dt, bool mixed,
                         bool split) {
  size_t b = make_layout(m, n, randqlp_sketch_width(m, n, k_max, p), dt, mixed, true, split).total;
  for (int c = 0; c < kRankClasses; ++c)
    b = std::max(b, make_layout(m, n, randqlp_sketch_width(m, n, rank_of_class(c, k_max), p), dt,
                                mixed, true, split)
                        .total);
  return b;
}

// ---- shared set-up of randqlp_factor / randqlp_factor_auto
rqlp_status setup_factor(const void* A, int64_t m, int64_t n, int k, int p, int q,
                         uint64_t seed, void* Q, void* L, void* P, const rqlp_opts* opts,
                         bool autoq, Ctx& c, FactorArgs& f, rqlp_opts& o,
                         std::unique_lock<std::mutex>& lk, bool noalloc = false,
                         int rank_kmax = 0, size_t extra = 0) {
  if (opts)
    o = *opts;
  else
    rqlp_opts_default(&o);
  if (m < 1 || n < 1) return fail(RQLP_E_INVALID_ARG, "m = %lld, n = %lld must be >= 1", (long long)m, (long long)n);
  if (k < 1) return fail(RQLP_E_INVALID_ARG, "k = %d must be >= 1", k);
  if (p < 0) return fail(RQLP_E_INVALID_ARG, "p = %d must be >= 0", p);
  if (q < 0) return fail(RQLP_E_INVALID_ARG, "q = %d must be >= 0", q);
  if (!A || !Q || !L || !P) return fail(RQLP_E_INVALID_ARG, "null matrix pointer");
  if (o.precision < RQLP_F64 || o.precision > RQLP_MIXED_BF16X3)
    return fail(RQLP_E_INVALID_ARG, "unknown precision %d", o.precision);
  if (o.panel_qr < RQLP_PANEL_AUTO || o.panel_qr > RQLP_PANEL_ROBUST)
    return fail(RQLP_E_INVALID_ARG, "unknown panel_qr %d", o.panel_qr);
  const int64_t d = randqlp_sketch_width(m, n, k, p);
  const int64_t lda = o.lda ? o.lda : m, ldq = o.ldq ? o.ldq : m;
  const int64_t ldl = o.ldl ? o.ldl : d, ldp = o.ldp ? o.ldp : n;
  if (lda < m || ldq < m || ldl < d || ldp < n)
    return fail(RQLP_E_INVALID_ARG, "leading dimension smaller than the row count");
  if (d > RQLP_MAX_D)
    return fail(RQLP_E_UNSUPPORTED, "sketch width d = %lld exceeds %d", (long long)d, RQLP_MAX_D);
  const Dtype dt = (o.precision == RQLP_F64) ? DT_F64 : DT_F32;
  const int mixed = (o.precision == RQLP_MIXED_BF16)     ? 1
                    : (o.precision == RQLP_MIXED_F16)   ? 2
                    : (o.precision == RQLP_MIXED_BF16X3) ? 3
                                                        : 0;
  c.st = (hipStream_t)o.stream;
  c.dt = dt;
  c.mixed = mixed;
  c.lay = make_layout(m, n, d, dt, mixed != 0, autoq, mixed == 3);
  c.d = d;
  c.seed = seed;
  c.orth_calls = 0;
  rqlp_status s = RQLP_OK;
  if (noalloc) {
    if (o.workspace != nullptr)
      return fail(RQLP_E_INVALID_ARG, "opts->workspace must be NULL: this entry point uses the "
                  "library's static scratch");
    c.extra_off = align_up(c.lay.total);
    if (c.extra_off + extra > kStaticScratchBytes)
      return fail(RQLP_E_WORKSPACE, "these sizes need %zu bytes of scratch; the static scratch "
                  "holds %zu (use randqlp_factor with a workspace)", c.extra_off + extra,
                  kStaticScratchBytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
      return fail(RQLP_E_HIP, "hipGetDevice failed");
    lk = std::unique_lock<std::mutex>(g_scratch_call_mu[dev]);
    if ((s = static_scratch(dev, &c.ws)) != RQLP_OK) return s;
    c.noalloc = true;
  } else {
    // the rank-predicting form re-lays the workspace out for the predicted
    // width: take enough for every width it can pick
    const size_t bytes = rank_kmax > 0 ? rank_layout_bytes(m, n, p, rank_kmax, dt, mixed != 0,
                                                           mixed == 3)
                                       : c.lay.total;
    c.extra_off = align_up(bytes);
    s = acquire_ws(o, c.extra_off + extra, &c.ws, lk);
    if (s != RQLP_OK) return s;
  }
  f = FactorArgs{A, m, n, lda, q, Q, ldq, (double*)L, ldl, P, ldp};
  return RQLP_OK;
}

PanelMode start_mode(const rqlp_opts& o) {
  return (o.panel_qr == RQLP_PANEL_ROBUST)    ? PM_ROBUST
         : (o.panel_qr == RQLP_PANEL_CHOLQR2) ? PM_CHOLQR2
                                              : PM_FAST;
}

struct Outcome {
  int breakdowns = 0, reran = 0, completed = 0;
};

// The method with f.q rounds; in AUTO mode a panel that reports an unsafe
// pivot (or an inaccurate second pass) makes the whole call rerun with the
// stronger panel QR.
rqlp_status run_with_escalation(Ctx& c, const FactorArgs& f, const rqlp_opts& o,
                                PanelMode mode, Outcome& r) {
  int fl[4] = {0, 0, 0, 0};
  rqlp_status s;
  for (;;) {
    hipError_t e = run_pipeline(c, f, mode);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "launch failed: %s", hipGetErrorString(e));
    if ((s = read_flags(c, fl)) != RQLP_OK) return s;
    if (fl[0] & FLAG_NONFINITE) {
      int fin[4] = {0, 0, 0, 0};
      e = clear_flags(c);
      if (e == hipSuccess) {
        if (c.sp)  // the stored entries of a sparse A, as one row
          e = c.sp->nnz > 0 ? launch_check_finite(c.sp->vals, 1, c.sp->nnz, 1, c.dt, c.flags(),
                                                  c.st)
                            : hipSuccess;
        else
          e = launch_check_finite(f.A, f.m, f.n, f.lda, c.dt, c.flags(), c.st);
      }
      if (e != hipSuccess) return fail(RQLP_E_HIP, "finite check: %s", hipGetErrorString(e));
      if ((s = read_flags(c, fin)) != RQLP_OK) return s;
      if (fin[0] & FLAG_NONFINITE) return fail(RQLP_E_NONFINITE, "A holds NaN or Inf");
      if (mode == PM_ROBUST)
        return fail(RQLP_E_NONFINITE, "non-finite intermediate (overflow) in the factorisation");
    }
    const bool pivot_bad = (fl[0] & (FLAG_NONPOS_PIVOT | FLAG_NONFINITE)) != 0;
    const bool second_bad = (fl[0] & FLAG_SECOND_PASS) != 0;
    if (mode == PM_ROBUST || (!pivot_bad && !second_bad)) break;
    ++r.breakdowns;
    if (o.panel_qr != RQLP_PANEL_AUTO) break;  // explicit strategy: no retry
    // A second pass that was not accurate enough: two full passes suffice
    // unless a pivot itself was unsafe, which needs the robust panels.
    mode = (!pivot_bad && mode == PM_FAST) ? PM_CHOLQR2 : PM_ROBUST;
    r.reran = 1;
  }
  r.completed = fl[2];
  return RQLP_OK;
}

void fill_info(const rqlp_opts& o, int64_t d, int q_used, const Outcome& r) {
  if (!o.info) return;
  o.info->d = (int32_t)d;
  o.info->q_used = q_used;
  o.info->breakdowns = r.breakdowns;
  o.info->robust_rerun = r.reran;
  o.info->completed = r.completed;
  o.info->reserved = 0;
}

// ---- predictor
struct MlpScratch {
  float *Xb, *H1, *H2, *Z, *dZ, *dH1, *dH2, *lossv, *grad, *step_loss;
  int* yb;
};

size_t mlp_scratch_bytes(int64_t B, int64_t steps) {
  return align_up((size_t)B * kNI * 4) + align_up((size_t)B * 4) +
         4 * align_up((size_t)B * kNH * 4) + 2 * align_up((size_t)B * kNC * 4) +
         align_up((size_t)B * 4) + align_up((size_t)kNParams * 4) +
         align_up((size_t)std::max<int64_t>(steps, 1) * 4);
}

void mlp_scratch_map(char* ws, int64_t B, int64_t steps, MlpScratch& sc) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = ws + off;
    off += align_up(bytes);
    return p;
  };
  sc.Xb = (float*)take((size_t)B * kNI * 4);
  sc.yb = (int*)take((size_t)B * 4);
  sc.H1 = (float*)take((size_t)B * kNH * 4);
  sc.H2 = (float*)take((size_t)B * kNH * 4);
  sc.dH1 = (float*)take((size_t)B * kNH * 4);
  sc.dH2 = (float*)take((size_t)B * kNH * 4);
  sc.Z = (float*)take((size_t)B * kNC * 4);
  sc.dZ = (float*)take((size_t)B * kNC * 4);
  sc.lossv = (float*)take((size_t)B * 4);
  sc.grad = (float*)take((size_t)kNParams * 4);
  sc.step_loss = (float*)take((size_t)std::max<int64_t>(steps, 1) * 4);
}

hipError_t mlp_forward_dev(const float* th, const float* X, int B, float* H1, float* H2,
                           float* Z, hipStream_t st) {
  HIP_TRY(launch_linear_forward(X, kNI, th + kOW1, th + kOB1, H1, B, kNI, kNH, true, st));
  HIP_TRY(launch_linear_forward(H1, kNH, th + kOW2, th + kOB2, H2, B, kNH, kNH, true, st));
  return launch_linear_forward(H2, kNH, th + kOW3, th + kOB3, Z, B, kNH, kNC, false, st);
}

// Mean cross-entropy and its gradient by backpropagation through the three
// layers (the ReLU masks come from the stored activations).
hipError_t mlp_loss_grad_dev(const float* th, const float* X, const int* y, int B,
                             const MlpScratch& sc, float* grad, float* loss, hipStream_t st) {
  HIP_TRY(mlp_forward_dev(th, X, B, sc.H1, sc.H2, sc.Z, st));
  HIP_TRY(launch_softmax_xent(sc.Z, y, B, kNC, sc.dZ, sc.lossv, st));
  HIP_TRY(launch_sum(sc.lossv, B, 1.0f / (float)B, loss, st));
  HIP_TRY(launch_linear_backward_weight(sc.H2, kNH, sc.dZ, grad + kOW3, grad + kOB3, B, kNH,
                                        kNC, st));
  HIP_TRY(launch_linear_backward_input(sc.dZ, th + kOW3, sc.H2, sc.dH2, B, kNH, kNC, st));
  HIP_TRY(launch_linear_backward_weight(sc.H1, kNH, sc.dH2, grad + kOW2, grad + kOB2, B, kNH,
                                        kNH, st));
  HIP_TRY(launch_linear_backward_input(sc.dH2, th + kOW2, sc.H1, sc.dH1, B, kNH, kNH, st));
  return launch_linear_backward_weight(X, kNI, sc.dH1, grad + kOW1, grad + kOB1, B, kNI, kNH,
                                       st);
}

// The 64-column sketch of A (in A's precision) with the leading columns om
// (ld m) of the method's own Gaussian sketch, its fp64 Gram and the
// features.
hipError_t feature_sketch(Ctx& c, const void* A, int64_t m, int64_t n, int64_t lda, int k,
                          const void* om, void* y64, double* g64, float* feat) {
  HIP_TRY(gemm(c, 1, A, lda, om, m, y64, n, n, kPredCols, m, c.dt, c.dt, false));
  HIP_TRY(gemm(c, 1, y64, n, y64, n, g64, kPredCols, kPredCols, kPredCols, n, c.dt, DT_F64,
               true));
  return launch_features(g64, kPredCols, k, feat, c.st);
}

// A second stream per device (default priority) for work that can run
// beside the main sequence; created once, kept for the process.
hipError_t aux_stream(hipStream_t* out) {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!streams[dev]) HIP_TRY(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  *out = streams[dev];
  return hipSuccess;
}

// Features -> MLP -> predicted class (to the device word at c.lay.cls),
// enqueued on stream `st` with the predictor's own scratch so that it runs
// beside the main sequence; Omega (Zm) must be drawn and must stay in place
// until the class has been computed.
hipError_t predict_q(Ctx& c, const FactorArgs& f, int k, const float* params, hipStream_t st) {
  Ctx cp = c;
  cp.st = st;
  cp.lay.part = c.lay.part2;
  cp.lay.part_bytes = c.lay.part2_bytes;
  float* mlp = c.at<float>(c.lay.mlp);
  int* dcls = c.at<int>(c.lay.cls);
  HIP_TRY(feature_sketch(cp, f.A, f.m, f.n, f.lda, k, c.ws + c.lay.m1, c.ws + c.lay.y64,
                         c.at<double>(c.lay.g64), c.at<float>(c.lay.feat)));
  return launch_predict_class(params, c.at<float>(c.lay.feat), mlp, dcls, st);
}

// Error judge after a run with q_hat rounds: sums = {||A||^2, ||L||^2,
// ||(I - Q Q^T) Z||^2, floor}; Zm keeps Z = A P (the next round's product, in
// the precision the rounds use).  In the precision form Z is the 16-bit
// product, which carries the rounding error dA = A16 - A of A; more rounds
// cannot remove it, so `floor` = (d / n) ||dA||_F^2 -- the expected energy of
// dA P for an orthonormal P -- is what Delta holds beyond the round's gain.
hipError_t judge(Ctx& c, const FactorArgs& f, double sums[4], int flags_out[4]) {
  const int64_t m = f.m, d = c.d;
  void* Zm = c.ws + c.lay.m1;
  void* Tm = c.ws + c.lay.m2;
  void* C1 = c.ws + c.lay.jd;
  double* scr = c.at<double>(c.lay.sums);
  double* res = c.at<double>(c.lay.sres);
  const int64_t nb16 = convert16_blocks(f.m, f.n);
  if (c.mixed && c.lay.rerr)  // ||A||^2 came with the 16-bit conversion
    HIP_TRY(launch_sum_f64(c.at<double>(c.lay.rerr) + nb16, nb16, res, c.st));
  else
    HIP_TRY(launch_sumsq(f.A, f.lda, nullptr, 0, f.m, f.n, c.dt, scr, res, c.st));
  HIP_TRY(launch_sumsq(f.L, f.ldl, nullptr, 0, d, d, DT_F64, scr, res + 1, c.st));
  HIP_TRY(prod(c, f, 0, f.P, f.ldp, Zm, m));                                   // Z = A P
  HIP_TRY(gemm(c, 1, f.Q, f.ldq, Zm, m, C1, d, d, d, m, c.dt, c.dt, false));   // Q^T Z
  HIP_TRY(gemm(c, 0, f.Q, f.ldq, C1, d, Tm, m, m, d, d, c.dt, c.dt, false));   // Q Q^T Z
  HIP_TRY(launch_sumsq(Zm, m, Tm, m, m, d, c.dt, scr, res + 2, c.st));
  if (c.mixed && c.lay.rerr)
    HIP_TRY(launch_sum_f64(c.at<double>(c.lay.rerr), nb16, res + 3, c.st));
  else
    HIP_TRY(launch_zero_block(res + 3, 1, 1, 1, c.st));
  // the four sums and the status words in one read-back
  HIP_TRY(read_back(c.st, sums, res, 4 * sizeof(double), flags_out, c.flags(), 4 * sizeof(int),
                    !c.noalloc));
  if (g_prof.on) prof_collect();
  sums[3] *= (double)d / (double)f.n;
  if (c.mixed == 2) sums[2] = std::ldexp(sums[2], -2 * flags_out[3]);  // Z carries 2^s
  return hipSuccess;
}

// Rank check of the returned factors (rank-predicting form): ||A||_F^2 into
// sres[0] unless the judge left it there, then the smallest k whose rank-k
// truncation Q L[:, :k] P[:, :k]^T meets tol, and its error, from the column
// norms of L (rank_scan); out = {k, e_k}, plus the status words.
hipError_t rank_check(Ctx& c, const FactorArgs& f, double tol, bool have_nrm, double out[2],
                      int flags_out[4]) {
  double* scr = c.at<double>(c.lay.sums);
  double* res = c.at<double>(c.lay.sres);
  if (!have_nrm) {
    const int64_t nb16 = convert16_blocks(f.m, f.n);
    if (c.mixed && c.lay.rerr)
      HIP_TRY(launch_sum_f64(c.at<double>(c.lay.rerr) + nb16, nb16, res, c.st));
    else
      HIP_TRY(launch_sumsq(f.A, f.lda, nullptr, 0, f.m, f.n, c.dt, scr, res, c.st));
  }
  HIP_TRY(launch_rank_scan(f.L, f.ldl, c.d, res, tol, res + 4, c.st));
  HIP_TRY(read_back(c.st, out, res + 4, 2 * sizeof(double), flags_out, c.flags(),
                    4 * sizeof(int), !c.noalloc));
  if (g_prof.on) prof_collect();
  return hipSuccess;
}

// Continue from Z = A Qbar_{j} in Zm with `more` further full rounds, then
// finish (more = 0: Q = orth(Z) is the final range basis).
hipError_t resume(Ctx& c, const FactorArgs& f, PanelMode mode, int more) {
  const int64_t m = f.m, n = f.n;
  void* Zm = c.ws + c.lay.m1;
  void* Tm = c.ws + c.lay.m2;
  void* Yn = c.ws + c.lay.n1;
  void* Tn = c.ws + c.lay.n2;
  HIP_TRY(clear_flags(c));
  if (more == 0) return stage_finish_from_z(c, f, mode);
  HIP_TRY(orth(c, Zm, m, m, Zm, m, Tm, nullptr, mode, false));                 // Q
  HIP_TRY(prod(c, f, 1, Zm, m, Yn, n));                                        // A^T Q
  HIP_TRY(orth(c, Yn, n, n, Yn, n, Tn, nullptr, mode, false));                 // Qbar
  HIP_TRY(stage_rounds(c, f, mode, more - 1));
  return stage_finish(c, f, mode);
}

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

extern "C" {

rqlp_status randqlp_factor(const void* A, int64_t m, int64_t n, int k, int p, int q,
                           uint64_t seed, void* Q, void* L, void* P, const rqlp_opts* opts) {
  Ctx c;
  FactorArgs f;
  rqlp_opts o;
  std::unique_lock<std::mutex> lk;
  rqlp_status s = setup_factor(A, m, n, k, p, q, seed, Q, L, P, opts, false, c, f, o, lk);
  if (s != RQLP_OK) return s;
  Outcome r;
  if ((s = run_with_escalation(c, f, o, start_mode(o), r)) != RQLP_OK) return s;
  fill_info(o, c.d, q, r);
  g_last_error.clear();
  return RQLP_OK;
}

rqlp_status randqlp_factor_csr(const int64_t* rowptr, const int32_t* colind, const void* vals,
                               int64_t m, int64_t n, int64_t nnz, int k, int p, int q,
                               uint64_t seed, void* Q, void* L, void* P, const rqlp_opts* opts) {
  if (nnz < 0) return fail(RQLP_E_INVALID_ARG, "nnz = %lld must be >= 0", (long long)nnz);
  if (!rowptr || (nnz > 0 && (!colind || !vals)))
    return fail(RQLP_E_INVALID_ARG, "null CSR array");
  rqlp_opts o0;
  if (opts)
    o0 = *opts;
  else
    rqlp_opts_default(&o0);
  o0.lda = 0;  // no dense A
  o0.workspace = nullptr;  // the layout has sparse regions: the library's cache
  o0.workspace_bytes = 0;
  if (o0.precision != RQLP_F64 && o0.precision != RQLP_F32)
    return fail(RQLP_E_UNSUPPORTED, "sparse input takes precision RQLP_F64 or RQLP_F32");
  if (m >= kSparseMaxRows || n >= kSparseMaxRows)
    return fail(RQLP_E_UNSUPPORTED, "sparse input needs m, n < %lld", (long long)kSparseMaxRows);
  const Dtype dt = o0.precision == RQLP_F64 ? DT_F64 : DT_F32;
  const int64_t d = randqlp_sketch_width(m, n, k, p);
  const size_t es = elem_size(dt);
  const size_t panel = d > 0 ? align_up((size_t)std::max(m, n) * d * es) : 0;
  const size_t tb = align_up(csr_transpose_bytes(n, nnz, dt));
  Ctx c;
  FactorArgs f;
  rqlp_opts o;
  std::unique_lock<std::mutex> lk;
  rqlp_status s = setup_factor(rowptr, m, n, k, p, q, seed, Q, L, P, &o0, false, c, f, o, lk,
                               false, 0, tb + 2 * panel + 256);
  if (s != RQLP_OK) return s;
  char* tws = c.ws + c.extra_off;
  c.sp_xr = c.extra_off + tb;
  c.sp_cr = c.sp_xr + panel;
  int* bad = (int*)(c.ws + c.sp_cr + panel);
  // structure check before any kernel indexes with the arrays
  int hbad = 0;
  hipError_t e = launch_zero_ints(bad, 1, c.st);
  if (e == hipSuccess) e = launch_csr_check(rowptr, colind, m, n, nnz, bad, c.st);
  if (e == hipSuccess)
    e = read_back(c.st, &hbad, bad, sizeof(int), nullptr, nullptr, 0, !c.noalloc);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "CSR check: %s", hipGetErrorString(e));
  if (hbad)
    return fail(RQLP_E_INVALID_ARG, "CSR arrays invalid (%s)",
                (hbad & 1) ? "rowptr must rise from 0 to nnz" : "column index outside [0, n)");
  const CsrView A{rowptr, colind, vals, m, n, nnz};
  CsrView At;
  e = launch_csr_transpose(rowptr, colind, vals, m, n, nnz, dt, tws, &At, c.st);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "CSR transpose: %s", hipGetErrorString(e));
  c.sp = &A;
  c.spt = &At;
  Outcome r;
  if ((s = run_with_escalation(c, f, o, start_mode(o), r)) != RQLP_OK) return s;
  fill_info(o, c.d, q, r);
  g_last_error.clear();
  return RQLP_OK;
}

rqlp_status randqlp_factor_async(const void* A, int64_t m, int64_t n, int k, int p, int q,
                                 uint64_t seed, void* Q, void* L, void* P,
                                 const rqlp_opts* opts, int* status) {
  if (!status) return fail(RQLP_E_INVALID_ARG, "null status pointer");
  if (!opts || !opts->workspace)
    return fail(RQLP_E_INVALID_ARG, "the asynchronous form needs opts with a workspace");
  Ctx c;
  FactorArgs f;
  rqlp_opts o;
  std::unique_lock<std::mutex> lk;
  rqlp_status s = setup_factor(A, m, n, k, p, q, seed, Q, L, P, opts, false, c, f, o, lk);
  if (s != RQLP_OK) return s;
  c.noalloc = true;  // no pinned buffer, no profiling events: nothing but launches
  // AUTO has no host to rerun from: the fast path, judged by the caller
  hipError_t e = run_pipeline(c, f, start_mode(o));
  if (e == hipSuccess) e = launch_copy_ints(c.flags(), status, 4, c.st);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "launch failed: %s", hipGetErrorString(e));
  if (o.info) {
    std::memset(o.info, 0, sizeof *o.info);
    o.info->d = (int32_t)c.d;
    o.info->q_used = q;
  }
  g_last_error.clear();
  return RQLP_OK;
}

rqlp_status randqlp_factor_noalloc(const void* A, int64_t m, int64_t n, int k, int p, int q,
                                   uint64_t seed, void* Q, void* L, void* P,
                                   const rqlp_opts* opts) {
  Ctx c;
  FactorArgs f;
  rqlp_opts o;
  std::unique_lock<std::mutex> lk;
  rqlp_status s = setup_factor(A, m, n, k, p, q, seed, Q, L, P, opts, false, c, f, o, lk, true);
  if (s != RQLP_OK) return s;
  Outcome r;
  if ((s = run_with_escalation(c, f, o, start_mode(o), r)) != RQLP_OK) return s;
  fill_info(o, c.d, q, r);
  g_last_error.clear();
  return RQLP_OK;
}

rqlp_status randqlp_factor_auto(const void* A, int64_t m, int64_t n, int k, int p,
                                int q_fallback, uint64_t seed, const float* params, void* Q,
                                void* L, void* P, const rqlp_opts* opts,
                                rqlp_auto_info* ainfo) {
  if (!params) return fail(RQLP_E_INVALID_ARG, "null predictor parameters");
  const bool rank_mode = k <= 0;
  double tol = 0.0;
  int k_max = 0;
  if (rank_mode) {
    if (!opts)
      return fail(RQLP_E_INVALID_ARG, "k <= 0 (predict the rank) needs opts->tol and opts->k_max");
    tol = opts->tol;
    k_max = opts->k_max;
    if (!(tol > 0.0 && tol <= 1.0))
      return fail(RQLP_E_INVALID_ARG, "tol = %g must lie in (0, 1]", tol);
    if (k_max < 1) return fail(RQLP_E_INVALID_ARG, "k_max = %d must be >= 1", k_max);
    if (p >= 0 && (int64_t)k_max + p > kRankMaxD)
      return fail(RQLP_E_UNSUPPORTED, "k_max + p = %lld exceeds %d", (long long)k_max + p,
                  kRankMaxD);
  }
  Ctx c;
  FactorArgs f;
  rqlp_opts o;
  std::unique_lock<std::mutex> lk;
  rqlp_status s = setup_factor(A, m, n, rank_mode ? k_max : k, p, q_fallback, seed, Q, L, P, opts,
                               true, c, f, o, lk, false, rank_mode ? k_max : 0);
  if (s != RQLP_OK) return s;
  rqlp_auto_info ai;
  std::memset(&ai, 0, sizeof ai);
  int cls = 0;
  Outcome r;
  int q_used = q_fallback;
  bool done = false;
  const PanelMode mode0 = start_mode(o);
  const int64_t d_max = c.d;
  c.orth_calls = 0;
  hipError_t e = hipSuccess;
  if (rank_mode) {
    // Omega (at least 64 columns), the feature sketch and both networks on
    // the call's stream; the sketch width follows from the predicted rank.
    const float rank_feat =
        (float)(std::min(std::max(-std::log10(tol), 0.0), 6.0) / 6.0);
    int pc[4] = {0, 0, 0, 0};
    int* dcls = c.at<int>(c.lay.cls);
    e = clear_flags(c);
    if (e == hipSuccess) e = stage_omega(c, f);
    // the feature sketch has 64 columns (d may be fewer): the predictor's
    // own split-K scratch
    Ctx cp = c;
    cp.lay.part = c.lay.part2;
    cp.lay.part_bytes = c.lay.part2_bytes;
    if (e == hipSuccess)
      e = feature_sketch(cp, f.A, f.m, f.n, f.lda, 1, c.ws + c.lay.m1, c.ws + c.lay.y64,
                         c.at<double>(c.lay.g64), c.at<float>(c.lay.feat));
    if (e == hipSuccess)
      e = launch_predict_rank_q(params, params + RQLP_MLP_PARAMS, c.at<float>(c.lay.feat),
                                rank_feat, k_max, dcls, c.st);
    if (e == hipSuccess)
      e = read_back(c.st, pc, dcls, 3 * sizeof(int), nullptr, nullptr, 0, !c.noalloc);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "predictor: %s", hipGetErrorString(e));
    cls = pc[0];
    ai.k_predicted = pc[2];
    // Omega stays where it is: m1 is the first region of every layout (ld m)
    const int64_t d = randqlp_sketch_width(m, n, pc[2], p);
    c.lay = make_layout(m, n, d, c.dt, c.mixed != 0, true, c.mixed == 3);
    c.d = d;
    e = stage_sketch(c, f, mode0);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "launch failed: %s", hipGetErrorString(e));
  } else {
    // The first sketch and its orth() do not depend on q.  Omega comes
    // first; the predictor (whose sketch uses Omega's leading columns) is
    // enqueued on the second stream right after it, then the rest of the
    // first sketch on the main stream, and the class is read back when the
    // predictor is done.
    hipStream_t aux = nullptr;
    hipEvent_t ready = nullptr;
    e = aux_stream(&aux);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    if (e == hipSuccess) e = clear_flags(c);
    if (e == hipSuccess) e = stage_omega(c, f);
    if (e == hipSuccess) e = hipEventRecord(ready, c.st);           // Omega is in Zm
    if (e == hipSuccess) e = hipStreamWaitEvent(aux, ready, 0);
    if (e == hipSuccess) e = predict_q(c, f, k, params, aux);
    if (e == hipSuccess) e = stage_sketch(c, f, mode0);
    // (the read-back waits for the predictor: enqueue it last)
    if (e == hipSuccess) e = read_back(aux, &cls, c.at<int>(c.lay.cls), sizeof(int));
    if (ready) (void)hipEventDestroy(ready);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "predictor: %s", hipGetErrorString(e));
    ai.k_predicted = k;
  }
  ai.q_predicted = cls;
  if (cls < q_fallback) {
    // the method with q_hat, then the judge
    f.q = cls;
    e = stage_rounds(c, f, mode0, cls);
    if (e == hipSuccess) e = stage_finish(c, f, mode0);
    double sums[4] = {0, 0, 0, 0};
    int fl[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = judge(c, f, sums, fl);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "launch failed: %s", hipGetErrorString(e));
    const bool clean = (fl[0] & (FLAG_NONPOS_PIVOT | FLAG_NONFINITE | FLAG_SECOND_PASS)) == 0;
    if (clean) {
      const double e2 = sums[0] - sums[1], delta = std::max(0.0, sums[2] - sums[3]);
      ai.judged = 1;
      ai.judge_ratio = e2 > 0.0 ? delta / e2 : (delta > 0.0 ? 1e300 : 0.0);
      ai.est_rel_err = sums[0] > 0.0 ? std::sqrt(std::max(0.0, e2 / sums[0])) : 0.0;
      if (ai.judge_ratio <= kJudgeSlack) {
        q_used = cls;
        r.completed = fl[2];
        done = true;
      } else {
        // resume from Z = A P = A Qbar_{q_hat + 1} up to q_fallback
        ai.resumed = 1;
        f.q = q_fallback;
        e = resume(c, f, mode0, q_fallback - (cls + 1));
        if (e != hipSuccess) return fail(RQLP_E_HIP, "launch failed: %s", hipGetErrorString(e));
        if ((s = read_flags(c, fl)) != RQLP_OK) return s;
        if ((fl[0] & (FLAG_NONPOS_PIVOT | FLAG_NONFINITE | FLAG_SECOND_PASS)) == 0) {
          r.completed = fl[2];
          done = true;
        }
      }
    }
  } else {
    // q_hat >= q_fallback: continue the plain method with q_fallback
    f.q = q_fallback;
    e = stage_rounds(c, f, mode0, q_fallback);
    if (e == hipSuccess) e = stage_finish(c, f, mode0);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "launch failed: %s", hipGetErrorString(e));
    int fl[4] = {0, 0, 0, 0};
    if ((s = read_flags(c, fl)) != RQLP_OK) return s;
    if ((fl[0] & (FLAG_NONPOS_PIVOT | FLAG_NONFINITE | FLAG_SECOND_PASS)) == 0) {
      r.completed = fl[2];
      done = true;
    }
  }
  if (!done) {
    // a panel needed the stronger treatment: the plain method with
    // q_fallback from the start, escalating as randqlp_factor does
    f.q = q_fallback;
    q_used = q_fallback;
    if ((s = run_with_escalation(c, f, o, mode0, r)) != RQLP_OK) return s;
  }
  if (rank_mode) {
    // does some rank k <= d of the returned factors meet tol?  If not, the
    // predicted rank (or q) was too low: the plain method with k_max and
    // q_fallback, and the same check on its factors.
    double rk[2] = {0.0, 0.0};
    int fl[4] = {0, 0, 0, 0};
    e = rank_check(c, f, tol, ai.judged != 0 && done, rk, fl);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "rank check: %s", hipGetErrorString(e));
    if (rk[1] > tol && (c.d < d_max || q_used < q_fallback)) {
      ai.rank_fallback = 1;
      c.lay = make_layout(m, n, d_max, c.dt, c.mixed != 0, true, c.mixed == 3);
      c.d = d_max;
      f.q = q_fallback;
      q_used = q_fallback;
      r = Outcome();
      if ((s = run_with_escalation(c, f, o, mode0, r)) != RQLP_OK) return s;
      e = rank_check(c, f, tol, false, rk, fl);
      if (e != hipSuccess) return fail(RQLP_E_HIP, "rank check: %s", hipGetErrorString(e));
    }
    ai.k_used = (int32_t)rk[0];
    ai.rank_err = rk[1];
  } else {
    ai.k_used = k;
  }
  ai.d = (int32_t)c.d;
  ai.q_used = q_used;
  fill_info(o, c.d, q_used, r);
  if (ainfo) *ainfo = ai;
  g_last_error.clear();
  return RQLP_OK;
}

rqlp_status randqlp_features(const void* A, int64_t m, int64_t n, int64_t lda, int k,
                             uint64_t seed, int precision, float* feat, void* stream) {
  if (m < 1 || n < 1 || !A || !feat || lda < m || k < 1)
    return fail(RQLP_E_INVALID_ARG, "bad size, pointer, leading dimension or k");
  if (precision != RQLP_F64 && precision != RQLP_F32)
    return fail(RQLP_E_INVALID_ARG, "unknown precision %d", precision);
  const Dtype dt = precision == RQLP_F64 ? DT_F64 : DT_F32;
  const size_t es = elem_size(dt);
  const size_t part = std::max(gemm_partial_bytes(1, n, kPredCols, m, dt, dt, false),
                               gemm_partial_bytes(1, kPredCols, kPredCols, n, dt, DT_F64, true));
  const size_t o_om = 0, o_y = align_up((size_t)m * kPredCols * es);
  const size_t o_g = o_y + align_up((size_t)n * kPredCols * es);
  const size_t o_p = o_g + align_up((size_t)kPredCols * kPredCols * 8);
  rqlp_opts o;
  rqlp_opts_default(&o);
  o.stream = stream;  // the workspace cache entry of the stream the call runs on
  std::unique_lock<std::mutex> lk;
  char* ws = nullptr;
  rqlp_status s = acquire_ws(o, o_p + std::max<size_t>(part, 256), &ws, lk);
  if (s != RQLP_OK) return s;
  Ctx c;
  c.st = (hipStream_t)stream;
  c.dt = dt;
  c.ws = ws;
  c.lay.part = o_p;
  c.lay.part_bytes = part;
  hipError_t e = launch_gaussian(ws + o_om, m, kPredCols, m, seed, 0, dt, c.st);
  if (e == hipSuccess)
    e = feature_sketch(c, A, m, n, lda, k, ws + o_om, ws + o_y, (double*)(ws + o_g), feat);
  if (e == hipSuccess) e = hipStreamSynchronize(c.st);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "features: %s", hipGetErrorString(e));
  return RQLP_OK;
}

rqlp_status randqlp_mlp_forward(const float* params, const float* X, int B, float* logits,
                                void* stream) {
  if (!params || !X || !logits || B < 1)
    return fail(RQLP_E_INVALID_ARG, "bad pointer or batch size");
  rqlp_opts o;
  rqlp_opts_default(&o);
  o.stream = stream;  // the workspace cache entry of the stream the call runs on
  std::unique_lock<std::mutex> lk;
  char* ws = nullptr;
  rqlp_status s = acquire_ws(o, 2 * align_up((size_t)B * kNH * 4), &ws, lk);
  if (s != RQLP_OK) return s;
  float* H1 = (float*)ws;
  float* H2 = (float*)(ws + align_up((size_t)B * kNH * 4));
  const hipStream_t st = (hipStream_t)stream;
  hipError_t e = mlp_forward_dev(params, X, B, H1, H2, logits, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "mlp forward: %s", hipGetErrorString(e));
  return RQLP_OK;
}

rqlp_status randqlp_mlp_loss_grad(const float* params, const float* X, const int* y, int B,
                                  float* grad, float* loss, void* stream) {
  if (!params || !X || !y || !grad || !loss || B < 1)
    return fail(RQLP_E_INVALID_ARG, "bad pointer or batch size");
  rqlp_opts o;
  rqlp_opts_default(&o);
  o.stream = stream;  // the workspace cache entry of the stream the call runs on
  std::unique_lock<std::mutex> lk;
  char* ws = nullptr;
  MlpScratch sc;
  rqlp_status s = acquire_ws(o, mlp_scratch_bytes(B, 0), &ws, lk);
  if (s != RQLP_OK) return s;
  mlp_scratch_map(ws, B, 0, sc);
  const hipStream_t st = (hipStream_t)stream;
  hipError_t e = mlp_loss_grad_dev(params, X, y, B, sc, grad, loss, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "mlp gradient: %s", hipGetErrorString(e));
  return RQLP_OK;
}

rqlp_status randqlp_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t t,
                             float lr, void* stream) {
  if (!params || !grad || !m || !v || t < 1 || !(lr > 0.0f))
    return fail(RQLP_E_INVALID_ARG, "bad pointer, step or learning rate");
  hipError_t e = launch_adam(params, grad, m, v, kNParams, lr, 0.9f, 0.999f, 1e-8f, t,
                             (hipStream_t)stream);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "adam: %s", hipGetErrorString(e));
  return RQLP_OK;
}

rqlp_status randqlp_mlp_train(float* params, float* m, float* v, const float* X, const int* y,
                              int64_t N, int epochs, int batch, float lr, uint64_t seed,
                              int64_t* step, float* epoch_loss, void* stream) {
  if (!params || !m || !v || !X || !y || !step || !epoch_loss || N < 1 || N >= (1ll << 31) ||
      epochs < 0 || batch < 1 || !(lr > 0.0f) || *step < 0)
    return fail(RQLP_E_INVALID_ARG, "bad pointer, size, batch, step or learning rate");
  const int64_t steps = (N + batch - 1) / batch;
  rqlp_opts o;
  rqlp_opts_default(&o);
  o.stream = stream;  // the workspace cache entry of the stream the call runs on
  std::unique_lock<std::mutex> lk;
  char* ws = nullptr;
  rqlp_status s = acquire_ws(o, mlp_scratch_bytes(batch, steps), &ws, lk);
  if (s != RQLP_OK) return s;
  MlpScratch sc;
  mlp_scratch_map(ws, batch, steps, sc);
  const hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
    // visiting order i -> (a i + c) mod N, a coprime to N
    uint64_t h = splitmix64(seed ^ (0x9E3779B97F4A7C15ull * (uint64_t)(ep + 1)));
    int64_t a = (int64_t)(h % (uint64_t)N);
    if (a == 0) a = 1;
    while (gcd64(a, N) != 1) a = (a + 1) % N == 0 ? 1 : a + 1;
    const int64_t cc = (int64_t)(splitmix64(h) % (uint64_t)N);
    for (int64_t it = 0; it < steps && e == hipSuccess; ++it) {
      const int64_t start = it * batch;
      const int B = (int)std::min<int64_t>(batch, N - start);
      e = launch_gather(X, y, N, a, cc, start, B, kNI, sc.Xb, sc.yb, st);
      if (e == hipSuccess) e = mlp_loss_grad_dev(params, sc.Xb, sc.yb, B, sc, sc.grad,
                                                 sc.step_loss + it, st);
      if (e == hipSuccess)
        e = launch_adam(params, sc.grad, m, v, kNParams, lr, 0.9f, 0.999f, 1e-8f, ++*step, st);
    }
    if (e == hipSuccess) e = launch_sum(sc.step_loss, steps, 1.0f / (float)steps, epoch_loss + ep, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "mlp training: %s", hipGetErrorString(e));
  return RQLP_OK;
}

rqlp_status randqlp_gaussian(void* out, int64_t m, int64_t d, int64_t ld, uint64_t seed,
                             uint64_t stream_id, int precision, void* stream) {
  if (m < 0 || d < 0 || (m * d > 0 && (!out || ld < m)))
    return fail(RQLP_E_INVALID_ARG, "bad size, pointer or leading dimension");
  if (precision != RQLP_F64 && precision != RQLP_F32)
    return fail(RQLP_E_INVALID_ARG, "unknown precision %d", precision);
  hipError_t e = launch_gaussian(out, m, d, ld, seed, stream_id,
                                 precision == RQLP_F64 ? DT_F64 : DT_F32, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "gaussian launch: %s", hipGetErrorString(e));
  return RQLP_OK;
}

rqlp_status randqlp_gemm(int trans_a, const void* A, int64_t m, int64_t n, int64_t lda,
                         const void* X, int64_t d, int64_t ldx, void* C, int64_t ldc,
                         int precision, void* stream) {
  if (m < 1 || n < 1 || d < 1 || !A || !X || !C || lda < m)
    return fail(RQLP_E_INVALID_ARG, "bad size, pointer or leading dimension");
  const int64_t rows = trans_a ? n : m, K = trans_a ? m : n;
  if (ldx < K || ldc < rows) return fail(RQLP_E_INVALID_ARG, "bad leading dimension");
  if (precision < RQLP_F64 || precision > RQLP_MIXED_BF16X3)
    return fail(RQLP_E_INVALID_ARG, "unknown precision %d", precision);
  const hipStream_t st = (hipStream_t)stream;
  rqlp_opts o;
  rqlp_opts_default(&o);
  o.stream = stream;  // the workspace cache entry of the stream the call runs on
  std::unique_lock<std::mutex> lk;
  char* ws = nullptr;
  hipError_t e = hipSuccess;
  if (precision >= RQLP_MIXED_BF16) {
    // 16-bit copies of op(A) (packed) and of X (contraction-contiguous),
    // then the precision-form product kernel.
    // RQLP_MIXED_BF16X3: the split product, with the residual copies of
    // op(A) and X after the rounded ones.
    const bool f16 = precision == RQLP_MIXED_F16;
    const bool split = precision == RQLP_MIXED_BF16X3;
    const int64_t ld16 = gemm16_ld(m), ldt16 = gemm16_ld(n), ldx16 = gemm16_ld(K);
    const size_t part = gemm16_partial_bytes(rows, d, K, f16, split ? 3 : 1);
    const size_t bytes_op = trans_a ? gemm16_packed_bytes(n, m) : gemm16_packed_bytes(m, n);
    const size_t off_a = 0, off_at = align_up(gemm16_packed_bytes(n, m));
    const size_t off_x = off_at + align_up(gemm16_packed_bytes(m, n));
    const size_t xbytes = gemm16_panel_bytes(ldx16, d);
    const size_t off_alo = off_x + align_up(xbytes);
    const size_t off_xlo = off_alo + (split ? align_up(bytes_op) : 0);
    const size_t off_p = off_xlo + (split ? align_up(xbytes) : 0);
    const size_t off_s = off_p + align_up(std::max<size_t>(part, 256));  // fp16 scale words
    rqlp_status s = acquire_ws(o, off_s + 256, &ws, lk);
    if (s != RQLP_OK) return s;
    unsigned* amax = (unsigned*)(ws + off_s);
    int* sexp = (int*)(ws + off_s + 16);
    e = launch_convert16((const float*)A, m, n, lda, ws + off_a, ld16, ws + off_at, ldt16, f16, st,
                         nullptr, (split && trans_a) ? ws + off_alo : nullptr,
                         (split && !trans_a) ? ws + off_alo : nullptr, amax, sexp);
    if (e == hipSuccess)
      e = launch_convert_panel16((const float*)X, K, d, ldx, ws + off_x, ldx16, f16, st,
                                 split ? ws + off_xlo : nullptr);
    if (e == hipSuccess) {
      Gemm16Args g;
      g.f16 = f16;
      g.A = trans_a ? (const void*)(ws + off_a) : (const void*)(ws + off_at);
      g.lda = trans_a ? ld16 : ldt16;
      g.B = ws + off_x;
      g.ldb = ldx16;
      g.C = (float*)C;
      g.ldc = ldc;
      g.M = rows;
      g.N = d;
      g.K = K;
      g.partial = ws + off_p;
      g.partial_bytes = part;
      if (split) {
        g.A2 = ws + off_alo;
        g.B2 = ws + off_xlo;
      }
      e = launch_gemm16(g, st);
      if (e == hipSuccess && f16)  // the fp16 copy of A carried 2^s
        e = launch_unscale((float*)C, rows, d, ldc, sexp, st);
    }
  } else {
    const Dtype dt = precision == RQLP_F64 ? DT_F64 : DT_F32;
    const size_t part = gemm_partial_bytes(trans_a, rows, d, K, dt, dt, false);
    rqlp_status s = acquire_ws(o, part > 0 ? part : 256, &ws, lk);
    if (s != RQLP_OK) return s;
    GemmArgs g;
    g.trans_a = trans_a ? 1 : 0;
    g.A = A;
    g.lda = lda;
    g.B = X;
    g.ldb = ldx;
    g.C = C;
    g.ldc = ldc;
    g.M = rows;
    g.N = d;
    g.K = K;
    g.in_t = dt;
    g.out_t = dt;
    g.gram = false;
    g.partial = ws;
    g.partial_bytes = part;
    e = launch_gemm(g, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // cache may be reused
  if (e != hipSuccess) return fail(RQLP_E_HIP, "gemm: %s", hipGetErrorString(e));
  return RQLP_OK;
}

rqlp_status randqlp_orth(const void* X, int64_t rows, int64_t d, int64_t ldx, void* Qx,
                         int64_t ldq, double* R, int64_t ldr, int precision, int panel_qr,
                         void* stream) {
  if (rows < 1 || d < 1 || rows < d || !X || !Qx || ldx < rows || ldq < rows)
    return fail(RQLP_E_INVALID_ARG, "bad size, pointer or leading dimension");
  if (R && ldr < d) return fail(RQLP_E_INVALID_ARG, "ldr < d");
  if (precision != RQLP_F64 && precision != RQLP_F32)
    return fail(RQLP_E_INVALID_ARG, "unknown precision %d", precision);
  if (panel_qr < RQLP_PANEL_AUTO || panel_qr > RQLP_PANEL_ROBUST)
    return fail(RQLP_E_INVALID_ARG, "unknown panel_qr %d", panel_qr);
  if (d > RQLP_MAX_D)
    return fail(RQLP_E_UNSUPPORTED, "d = %lld exceeds %d", (long long)d, RQLP_MAX_D);
  const Dtype dt = precision == RQLP_F64 ? DT_F64 : DT_F32;
  Ctx c;
  c.st = (hipStream_t)stream;
  c.dt = dt;
  // a panel of `rows` rows uses the m-side buffers of a rows x d layout
  c.lay = make_layout(rows, d, d, dt);
  c.d = d;
  c.seed = 0x5eedull;
  c.orth_calls = 0;
  rqlp_opts o;
  rqlp_opts_default(&o);
  o.stream = stream;  // the workspace cache entry of the stream the call runs on
  std::unique_lock<std::mutex> lk;
  rqlp_status s = acquire_ws(o, c.lay.total, &c.ws, lk);
  if (s != RQLP_OK) return s;
  double* Rfin = c.at<double>(c.lay.Rfin);
  PanelMode mode = (panel_qr == RQLP_PANEL_ROBUST)    ? PM_ROBUST
                   : (panel_qr == RQLP_PANEL_CHOLQR2) ? PM_CHOLQR2
                                                      : PM_FAST;
  int fl[4] = {0, 0, 0, 0};
  for (;;) {
    c.orth_calls = 0;
    hipError_t e = clear_flags(c);
    if (e == hipSuccess)
      e = orth(c, X, rows, ldx, Qx, ldq, c.ws + c.lay.m2, Rfin, mode, true);
    if (e == hipSuccess && R)
      e = hipMemcpy2DAsync(R, ldr * sizeof(double), Rfin, d * sizeof(double),
                           d * sizeof(double), d, hipMemcpyDeviceToDevice, c.st);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "orth: %s", hipGetErrorString(e));
    if ((s = read_flags(c, fl)) != RQLP_OK) return s;
    const bool pivot_bad = (fl[0] & (FLAG_NONPOS_PIVOT | FLAG_NONFINITE)) != 0;
    const bool second_bad = (fl[0] & FLAG_SECOND_PASS) != 0;
    if (mode == PM_ROBUST && (fl[0] & FLAG_NONFINITE))
      return fail(RQLP_E_NONFINITE, "non-finite panel");
    if (mode == PM_ROBUST || (!pivot_bad && !second_bad) || panel_qr != RQLP_PANEL_AUTO) break;
    mode = (!pivot_bad && mode == PM_FAST) ? PM_CHOLQR2 : PM_ROBUST;
  }
  return RQLP_OK;
}

}  // extern "C"

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

struct Layout {
  size_t m1, m2, n1, n2, part, part_bytes, G, R[4], Racc[2], Rfin, dinv, colf, scal, flags,
      chs, a16, at16, p16, total;
  int64_t ld16, ldt16;  // leading dimensions of the 16-bit copies of A and A^T
  int64_t ldp16;        // leading dimension of the 16-bit copy of a panel
  size_t flags_bytes;  // status words cleared at the start of a call
};

size_t elem_size(Dtype dt) { return dt == DT_F64 ? 8 : 4; }

Layout make_layout(int64_t m, int64_t n, int64_t d, Dtype dt, bool mixed = false) {
  Layout L;
  const size_t es = elem_size(dt);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.m1 = take((size_t)m * d * es);
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
  if (mixed) {
    for (bool f16 : {false, true}) {
      part = std::max(part, gemm16_partial_bytes(n, d, m, f16));
      part = std::max(part, gemm16_partial_bytes(m, d, n, f16));
    }
  }
  L.part = take(part);
  L.part_bytes = part;
  L.G = take((size_t)d * d * 8);
  for (int i = 0; i < 4; ++i) L.R[i] = take((size_t)d * d * 8);
  for (int i = 0; i < 2; ++i) L.Racc[i] = take((size_t)d * d * 8);
  L.Rfin = take((size_t)d * d * 8);
  L.chs = take((size_t)4 * d * d * 8);  // blocked Cholesky: off-diagonal solve + Schur blocks
  L.dinv = take((size_t)((d + 15) / 16) * 256 * 8);
  L.colf = take((size_t)d * 4);
  if (mixed) {
    L.ld16 = gemm16_ld(m);
    L.ldt16 = gemm16_ld(n);
    L.a16 = take((size_t)L.ld16 * n * 2);
    L.at16 = take((size_t)L.ldt16 * m * 2);
    L.ldp16 = gemm16_ld(std::max(m, n));
    L.p16 = take((size_t)L.ldp16 * d * 2);
  } else {
    L.ld16 = L.ldt16 = L.ldp16 = 0;
    L.a16 = L.at16 = L.p16 = 0;
  }
  L.scal = take(64);
  L.flags = take(64);
  L.flags_bytes = 64;
  L.total = off;
  return L;
}

// Library-managed workspace: one growing buffer per device.
struct WsCache {
  std::mutex mu;
  void* ptr[64] = {};
  size_t size[64] = {};
};
WsCache g_ws;

struct Ctx {
  hipStream_t st;
  Dtype dt;
  int mixed = 0;  // 0: no; 1: bf16 products; 2: fp16 products
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
  if (timed && g_prof.on) {
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
hipError_t gemm16(Ctx& c, int trans_a, int64_t m, int64_t n, const float* X, int64_t ldx,
                  float* C, int64_t ldc, int64_t d) {
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
  hipError_t e = launch_convert_panel16(X, g.K, d, ldx, c.ws + c.lay.p16, c.lay.ldp16, g.f16, c.st);
  if (e != hipSuccess) return e;
  if (g_prof.on) {
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
// diagonal-block inverses.  Blocked right-looking: the leading CHOL_MAX_D
// columns on the one-workgroup kernel; R12 = R11^{-T} G12, computed as the
// TRSM of G21 = G12^T; the Schur complement G22 - R12^T R12 through the Gram
// product; then the same on the complement.  Pivot tolerances stay relative
// to the original diagonal.  scratch holds 4 d^2 doubles.
hipError_t chol_any(Ctx& c, const double* G, int64_t d, int64_t ldg, double shift,
                    const double* shift_dev, double tol_dep, double tol_warn, double* R,
                    int64_t ldr, double* dinv, int* col_flags, const double* odiag_src,
                    int64_t odiag_stride, double* scratch) {
  if (d <= CHOL_MAX_D)
    return launch_cholesky_tile(G, d, ldg, shift, shift_dev, tol_dep, tol_warn, R, ldr, dinv,
                                col_flags, c.flags(), odiag_src, odiag_stride, c.st);
  const int64_t d1 = CHOL_MAX_D, d2 = d - d1;
  HIP_TRY(launch_cholesky_tile(G, d1, ldg, shift, shift_dev, tol_dep, tol_warn, R, ldr, dinv,
                               col_flags, c.flags(), odiag_src, odiag_stride, c.st));
  double* Xs = scratch;          // G21 R11^{-1} = R12^T, d2 x d1
  double* C = Xs + d2 * d1;      // R12^T R12, d2 x d2
  double* S = C + d2 * d2;       // Schur complement, d2 x d2
  HIP_TRY(launch_trsm(G + d1, d2, d1, ldg, R, ldr, dinv, Xs, d2, DT_F64, c.st));
  double* R12 = R + d1 * ldr;
  HIP_TRY(launch_transpose(Xs, d2, d1, d2, R12, ldr, c.st));
  HIP_TRY(launch_zero_block(R + d1, d2, d1, ldr, c.st));
  HIP_TRY(gemm(c, 1, R12, ldr, R12, ldr, C, d2, d2, d2, d1, DT_F64, DT_F64, true));
  HIP_TRY(launch_schur(G + d1 + d1 * ldg, ldg, C, d2, shift, shift_dev, S, c.st));
  const double* od = odiag_src ? odiag_src + d1 * odiag_stride : G + d1 + d1 * ldg;
  const int64_t ods = odiag_src ? odiag_stride : ldg + 1;
  return chol_any(c, S, d2, d2, 0.0, nullptr, tol_dep, tol_warn, R + d1 + d1 * ldr, ldr,
                  dinv + (d1 / 16) * 256, col_flags ? col_flags + d1 : nullptr, od, ods,
                  S + d2 * d2);
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
  return launch_trsm(X, rows, d, ldx, Rbuf, d, dinv, Qx, ldq, c.dt, c.st);
}

// Panel QR strategies, cheapest first.
//  FAST     intermediate panels (whose range is all the next product uses):
//           one Cholesky QR pass, in place.  Final panels (Q and P): one
//           pass, then the second pass to first order in E = Q1^T Q1 - I.
//  CHOLQR2  two full Cholesky QR passes on every panel.
//  ROBUST   shifted pass, completion of dependent columns, two more passes.
enum PanelMode { PM_FAST = 0, PM_CHOLQR2 = 1, PM_ROBUST = 2 };

// max |E| for which the first-order second pass is accurate to the
// precision's rounding level (the neglected terms are O(|E|^2)).
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
  HIP_TRY(launch_trsm(X, rows, d, ldx, R[0], d, dinv, tmp, rows, c.dt, c.st));
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

// Precision form of the pipeline: products with A on the 16-bit copies,
// final projection in fp32.
hipError_t run_pipeline_mixed(Ctx& c, const FactorArgs& f, PanelMode mode) {
  const int64_t m = f.m, n = f.n, d = c.d;
  float* Zm = c.at<float>(c.lay.m1);
  void* Tm = c.ws + c.lay.m2;
  float* Yn = c.at<float>(c.lay.n1);
  void* Tn = c.ws + c.lay.n2;
  double* Rfin = c.at<double>(c.lay.Rfin);
  c.orth_calls = 0;
  HIP_TRY(hipMemsetAsync(c.flags(), 0, c.lay.flags_bytes, c.st));
  HIP_TRY(launch_convert16((const float*)f.A, m, n, f.lda, c.ws + c.lay.a16, c.lay.ld16,
                           c.ws + c.lay.at16, c.lay.ldt16, c.mixed == 2, c.st));
  HIP_TRY(launch_gaussian(Zm, m, d, m, c.seed, 0, DT_F32, c.st));             // randn
  HIP_TRY(gemm16(c, 1, m, n, Zm, m, Yn, n, d));                                // A^T Omega
  HIP_TRY(orth(c, Yn, n, n, Yn, n, Tn, nullptr, mode, false));
  for (int it = 0; it < f.q; ++it) {
    HIP_TRY(gemm16(c, 0, m, n, Yn, n, Zm, m, d));                              // A Qbar
    HIP_TRY(orth(c, Zm, m, m, Zm, m, Tm, nullptr, mode, false));
    HIP_TRY(gemm16(c, 1, m, n, Zm, m, Yn, n, d));                              // A^T Q
    HIP_TRY(orth(c, Yn, n, n, Yn, n, Tn, nullptr, mode, false));
  }
  HIP_TRY(gemm16(c, 0, m, n, Yn, n, Zm, m, d));                                // A Qbar
  HIP_TRY(orth(c, Zm, m, m, f.Q, f.ldq, Tm, nullptr, mode, true));             // Q
  HIP_TRY(gemm(c, 1, f.A, f.lda, f.Q, f.ldq, Yn, n, n, d, m, DT_F32, DT_F32, false, true));
  HIP_TRY(orth(c, Yn, n, n, f.P, f.ldp, Tn, Rfin, mode, true));                // P, R
  HIP_TRY(launch_lower_from_upper(Rfin, d, f.L, f.ldl, c.st));                // L = R^T
  return hipSuccess;
}

hipError_t run_pipeline(Ctx& c, const FactorArgs& f, PanelMode mode) {
  if (c.mixed) return run_pipeline_mixed(c, f, mode);
  const int64_t m = f.m, n = f.n, d = c.d;
  void* Zm = c.ws + c.lay.m1;
  void* Tm = c.ws + c.lay.m2;
  void* Yn = c.ws + c.lay.n1;
  void* Tn = c.ws + c.lay.n2;
  double* Rfin = c.at<double>(c.lay.Rfin);
  c.orth_calls = 0;
  HIP_TRY(hipMemsetAsync(c.flags(), 0, c.lay.flags_bytes, c.st));
  HIP_TRY(launch_gaussian(Zm, m, d, m, c.seed, 0, c.dt, c.st));                     // randn
  HIP_TRY(gemm(c, 1, f.A, f.lda, Zm, m, Yn, n, n, d, m, c.dt, c.dt, false, true));  // A^T Omega
  HIP_TRY(orth(c, Yn, n, n, Yn, n, Tn, nullptr, mode, false));                       // Qbar
  for (int it = 0; it < f.q; ++it) {
    HIP_TRY(gemm(c, 0, f.A, f.lda, Yn, n, Zm, m, m, d, n, c.dt, c.dt, false, true));  // A Qbar
    HIP_TRY(orth(c, Zm, m, m, Zm, m, Tm, nullptr, mode, false));
    HIP_TRY(gemm(c, 1, f.A, f.lda, Zm, m, Yn, n, n, d, m, c.dt, c.dt, false, true));  // A^T Q
    HIP_TRY(orth(c, Yn, n, n, Yn, n, Tn, nullptr, mode, false));
  }
  HIP_TRY(gemm(c, 0, f.A, f.lda, Yn, n, Zm, m, m, d, n, c.dt, c.dt, false, true));  // A Qbar
  HIP_TRY(orth(c, Zm, m, m, f.Q, f.ldq, Tm, nullptr, mode, true));                   // Q
  HIP_TRY(gemm(c, 1, f.A, f.lda, f.Q, f.ldq, Yn, n, n, d, m, c.dt, c.dt, false, true));  // A^T Q
  HIP_TRY(orth(c, Yn, n, n, f.P, f.ldp, Tn, Rfin, mode, true));                      // P, R
  HIP_TRY(launch_lower_from_upper(Rfin, d, f.L, f.ldl, c.st));                      // L = R^T
  return hipSuccess;
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
  if (prec < RQLP_F64 || prec > RQLP_MIXED_F16) return 0;
  return make_layout(m, n, d, prec == RQLP_F64 ? DT_F64 : DT_F32, prec >= RQLP_MIXED_BF16).total;
}

}  // extern "C"

namespace {

// Acquire `bytes` of device scratch: the caller's buffer or the per-device
// cache (grown under the lock; the lock is held for the whole call).
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
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return fail(RQLP_E_HIP, "hipGetDevice failed");
  lk = std::unique_lock<std::mutex>(g_ws.mu);
  if (g_ws.size[dev] < bytes) {
    if (g_ws.ptr[dev]) {
      (void)hipDeviceSynchronize();
      (void)hipFree(g_ws.ptr[dev]);
      g_ws.ptr[dev] = nullptr;
      g_ws.size[dev] = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(RQLP_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    g_ws.ptr[dev] = p;
    g_ws.size[dev] = bytes;
  }
  *out = (char*)g_ws.ptr[dev];
  return RQLP_OK;
}

rqlp_status read_flags(Ctx& c, int host[4]) {
  hipError_t e = hipMemcpyAsync(host, c.flags(), 4 * sizeof(int), hipMemcpyDeviceToHost, c.st);
  if (e == hipSuccess) e = hipStreamSynchronize(c.st);
  if (e != hipSuccess) return fail(RQLP_E_HIP, "status read-back: %s", hipGetErrorString(e));
  if (g_prof.on) prof_collect();
  return RQLP_OK;
}

}  // namespace

extern "C" {

rqlp_status randqlp_factor(const void* A, int64_t m, int64_t n, int k, int p, int q,
                           uint64_t seed, void* Q, void* L, void* P, const rqlp_opts* opts) {
  rqlp_opts o;
  if (opts)
    o = *opts;
  else
    rqlp_opts_default(&o);
  if (m < 1 || n < 1) return fail(RQLP_E_INVALID_ARG, "m = %lld, n = %lld must be >= 1", (long long)m, (long long)n);
  if (k < 1) return fail(RQLP_E_INVALID_ARG, "k = %d must be >= 1", k);
  if (p < 0) return fail(RQLP_E_INVALID_ARG, "p = %d must be >= 0", p);
  if (q < 0) return fail(RQLP_E_INVALID_ARG, "q = %d must be >= 0", q);
  if (!A || !Q || !L || !P) return fail(RQLP_E_INVALID_ARG, "null matrix pointer");
  if (o.precision < RQLP_F64 || o.precision > RQLP_MIXED_F16)
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
  const int mixed = (o.precision == RQLP_MIXED_BF16) ? 1 : (o.precision == RQLP_MIXED_F16) ? 2 : 0;

  Ctx c;
  c.st = (hipStream_t)o.stream;
  c.dt = dt;
  c.mixed = mixed;
  c.lay = make_layout(m, n, d, dt, mixed != 0);
  c.d = d;
  c.seed = seed;
  c.orth_calls = 0;
  std::unique_lock<std::mutex> lk;
  rqlp_status s = acquire_ws(o, c.lay.total, &c.ws, lk);
  if (s != RQLP_OK) return s;

  FactorArgs f{A, m, n, lda, q, Q, ldq, (double*)L, ldl, P, ldp};
  PanelMode mode = (o.panel_qr == RQLP_PANEL_ROBUST)    ? PM_ROBUST
                   : (o.panel_qr == RQLP_PANEL_CHOLQR2) ? PM_CHOLQR2
                                                        : PM_FAST;
  int fl[4] = {0, 0, 0, 0};
  int reran = 0, breakdowns = 0;
  for (;;) {
    hipError_t e = run_pipeline(c, f, mode);
    if (e != hipSuccess) return fail(RQLP_E_HIP, "launch failed: %s", hipGetErrorString(e));
    if ((s = read_flags(c, fl)) != RQLP_OK) return s;
    if (fl[0] & FLAG_NONFINITE) {
      int fin[4] = {0, 0, 0, 0};
      e = hipMemsetAsync(c.flags(), 0, 64, c.st);
      if (e == hipSuccess) e = launch_check_finite(A, m, n, lda, dt, c.flags(), c.st);
      if (e != hipSuccess) return fail(RQLP_E_HIP, "finite check: %s", hipGetErrorString(e));
      if ((s = read_flags(c, fin)) != RQLP_OK) return s;
      if (fin[0] & FLAG_NONFINITE) return fail(RQLP_E_NONFINITE, "A holds NaN or Inf");
      if (mode == PM_ROBUST)
        return fail(RQLP_E_NONFINITE, "non-finite intermediate (overflow) in the factorisation");
    }
    const bool pivot_bad = (fl[0] & (FLAG_NONPOS_PIVOT | FLAG_NONFINITE)) != 0;
    const bool second_bad = (fl[0] & FLAG_SECOND_PASS) != 0;
    if (mode == PM_ROBUST || (!pivot_bad && !second_bad)) break;
    ++breakdowns;
    if (o.panel_qr != RQLP_PANEL_AUTO) break;  // explicit strategy: no retry
    // A second pass that was not accurate enough: two full passes suffice
    // unless a pivot itself was unsafe, which needs the robust panels.
    mode = (!pivot_bad && mode == PM_FAST) ? PM_CHOLQR2 : PM_ROBUST;
    reran = 1;
  }
  if (o.info) {
    o.info->d = (int32_t)d;
    o.info->q_used = q;
    o.info->breakdowns = breakdowns;
    o.info->robust_rerun = reran;
    o.info->completed = fl[2];
    o.info->reserved = 0;
  }
  g_last_error.clear();
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
  if (precision < RQLP_F64 || precision > RQLP_MIXED_F16)
    return fail(RQLP_E_INVALID_ARG, "unknown precision %d", precision);
  const hipStream_t st = (hipStream_t)stream;
  rqlp_opts o;
  rqlp_opts_default(&o);
  std::unique_lock<std::mutex> lk;
  char* ws = nullptr;
  hipError_t e = hipSuccess;
  if (precision >= RQLP_MIXED_BF16) {
    // 16-bit copies of op(A) (contraction-contiguous) and of X, then the
    // precision-form product kernel.
    const bool f16 = precision == RQLP_MIXED_F16;
    const int64_t ld16 = gemm16_ld(m), ldt16 = gemm16_ld(n), ldx16 = gemm16_ld(K);
    const size_t part = gemm16_partial_bytes(rows, d, K, f16);
    const size_t off_a = 0, off_at = align_up((size_t)ld16 * n * 2);
    const size_t off_x = off_at + align_up((size_t)ldt16 * m * 2);
    const size_t off_p = off_x + align_up((size_t)ldx16 * d * 2);
    rqlp_status s = acquire_ws(o, off_p + std::max<size_t>(part, 256), &ws, lk);
    if (s != RQLP_OK) return s;
    e = launch_convert16((const float*)A, m, n, lda, ws + off_a, ld16, ws + off_at, ldt16, f16, st);
    if (e == hipSuccess)
      e = launch_convert_panel16((const float*)X, K, d, ldx, ws + off_x, ldx16, f16, st);
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
      e = launch_gemm16(g, st);
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
    hipError_t e = hipMemsetAsync(c.flags(), 0, c.lay.flags_bytes, c.st);
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

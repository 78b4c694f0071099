// Batched Rand-QLP: many independent matrices of different shapes factored
// together.  Every step of the generalised Algorithm 1 (Section 3.1) runs as
// one grouped launch over all matrices -- the Gaussian sketches, each
// product with A, each Gram matrix, each Cholesky factorisation, each
// triangular solve -- driven by device tables of per-matrix descriptors and
// per-workgroup block maps built once per plan.  The whole sequence is
// captured into a HIP graph and replayed.  Each launch is independent of the
// others' progress (no workgroup ever waits on another), so every wave
// always finishes.
//
// Panels use the fast Cholesky QR of the single-matrix path.  Matrices whose
// panels report an unsafe pivot, and matrices with d above the one-workgroup
// Cholesky limit, are factored afterwards one by one with randqlp_factor
// (which escalates to the robust panels).
//
// Tile widths of the products with A come from a table: tuned on the plan's
// own data when asked (each candidate timed with HIP events), kept per
// (precision, product orientation, bucket of the largest d), and saved to /
// loaded from a text file.  Candidates: one width for every matrix, or
// width 0 = per class (each matrix gets the width that covers its d in one
// tile, one launch per width present, so A is read once), or 16 = the
// remainder layout per class (MFMA blocks plus vector-ALU columns).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/randqlp.h"
#include "rqlp_internal.h"

using namespace rqlp;

// Status helpers shared with randqlp.hip.
rqlp_status rqlp_fail(rqlp_status s, const char* fmt, ...);

namespace {

constexpr double kUnitB = 1.1102230246251565e-16;
constexpr double kTolDepFastB = 64.0 * kUnitB;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }
size_t esize(Dtype dt) { return dt == DT_F64 ? 8 : 4; }

// ---- tile-width table
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune;  // (dtype, trans, dbucket) -> wn

int dbucket(int64_t dmax) { return dmax <= 32 ? 32 : dmax <= 64 ? 64 : dmax <= 128 ? 128 : 256; }

int lookup_wn(Dtype dt, int trans, int64_t dmax, int fallback) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find({(int)dt, trans, dbucket(dmax)});
  return it == g_tune.end() ? fallback : it->second;
}

struct Launch {
  size_t desc = 0, map = 0;  // byte offsets into the plan's table buffer
  int64_t count = 0, nblocks = 0;
};

// A product step: one launch per tile width used.  wn in 1..8: every matrix
// with that width; wn = 0 ("per class"): each matrix with the width that
// covers its d in one tile (1, 2, 4 or 8 blocks of 32 columns), one launch
// per width present; wn = kRemSet: the remainder layout (16 c MFMA columns
// plus 4 vector-ALU columns, c from grouped_rem_class), one launch per class.
constexpr int kRemSet = 16;
struct ProdSet {
  int wn = 2;
  bool rem = false;
  std::vector<std::pair<int, Launch>> parts;  // (width, launch)
};

int class_wn(int64_t d) { return grouped_wn_round((int)((d + 31) / 32)); }

}  // namespace

struct rqlp_batch {
  int count = 0, q = 0;
  Dtype dt = DT_F32;
  std::vector<int64_t> m, n, d, lda, ldq, ldl, ldp;
  std::vector<int> k;
  int p = 0;
  std::vector<uint64_t> seed;
  std::vector<const void*> A;
  std::vector<void*> Q, P;
  std::vector<double*> L;
  std::vector<int> grouped;      // indices factored by the grouped launches
  std::vector<int> individual;   // factored one by one (d too large)
  char* ws = nullptr;            // per-matrix panels and small factors
  char* tab = nullptr;           // descriptor tables and block maps
  int* flags = nullptr;          // 16 ints per grouped matrix
  int64_t dmax = 0;
  int wn_tn = 2, wn_nn = 2;
  double tune_ms = 0.0;
  int last_fallbacks = 0;
  // launches
  Launch gauss, gramY, gramZ, gramTm, gramTn, chol, trsmY, trsmZ, trsmZT, trsmYT, fo, qfin, pfin,
      rcomb, lower;
  ProdSet tn, nn, tn_final;
  // candidate product sets per width (0 = per class)
  std::map<int, ProdSet> tn_alt, nn_alt, tnf_alt;
  hipStream_t cap = nullptr;
  // side streams and events: the width classes of one product run side by
  // side (forked from the calling stream and joined back, also in the graph)
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kSide] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // host staging of the tables
  std::vector<char> host_tab;
};

namespace {

template <typename T>
size_t put(std::vector<char>& buf, const std::vector<T>& v) {
  size_t off = align_up(buf.size());
  buf.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

template <typename T>
const T* at(const rqlp_batch* b, size_t off) {
  return (const T*)(b->tab + off);
}

// Longest contraction first: the workgroups of the big matrices start in
// the first rounds and the short ones fill the tail.
void longest_first(const std::vector<GroupGemm>& descs, std::vector<int4>& map) {
  std::stable_sort(map.begin(), map.end(), [&](const int4& x, const int4& y) {
    return descs[x.x].K > descs[y.x].K;
  });
}

Launch gemm_launch(std::vector<char>& buf, const std::vector<GroupGemm>& descs, bool gram,
                   int wn) {
  std::vector<int4> map;
  for (size_t i = 0; i < descs.size(); ++i) gemm_grouped_blocks(descs[i], (int)i, gram, wn, map);
  longest_first(descs, map);
  Launch l;
  l.desc = put(buf, descs);
  l.map = put(buf, map);
  l.count = (int64_t)descs.size();
  l.nblocks = (int64_t)map.size();
  return l;
}

ProdSet prod_set(std::vector<char>& buf, const std::vector<GroupGemm>& descs, int wn, Dtype dt) {
  ProdSet ps;
  ps.wn = wn;
  if (wn == kRemSet) {
    ps.rem = true;
    for (int c : kRemClasses) {
      std::vector<int4> map;
      for (size_t i = 0; i < descs.size(); ++i)
        if (grouped_rem_class(descs[i].N) == c)
          gemm_rem_grouped_blocks(descs[i], (int)i, c, dt, map);
      if (map.empty()) continue;
      longest_first(descs, map);
      Launch l;
      l.desc = put(buf, descs);
      l.map = put(buf, map);
      l.count = (int64_t)descs.size();
      l.nblocks = (int64_t)map.size();
      ps.parts.push_back({c, l});
    }
    return ps;
  }
  if (wn > 0) {
    ps.parts.push_back({wn, gemm_launch(buf, descs, false, wn)});
    return ps;
  }
  for (int c : {1, 2, 4, 8}) {
    std::vector<int4> map;
    for (size_t i = 0; i < descs.size(); ++i)
      if (class_wn(descs[i].N) == c) gemm_grouped_blocks(descs[i], (int)i, false, c, map);
    if (map.empty()) continue;
    longest_first(descs, map);
    Launch l;
    l.desc = put(buf, descs);
    l.map = put(buf, map);
    l.count = (int64_t)descs.size();
    l.nblocks = (int64_t)map.size();
    ps.parts.push_back({c, l});
  }
  return ps;
}

Launch trsm_launch(std::vector<char>& buf, const std::vector<GroupTrsm>& descs) {
  std::vector<int2> map;
  for (size_t i = 0; i < descs.size(); ++i) trsm_grouped_blocks(descs[i], (int)i, map);
  Launch l;
  l.desc = put(buf, descs);
  l.map = put(buf, map);
  l.count = (int64_t)descs.size();
  l.nblocks = (int64_t)map.size();
  return l;
}

hipError_t run_gemm(const rqlp_batch* b, const Launch& l, Dtype in_t, Dtype out_t, int trans,
                    bool gram, int wn, hipStream_t st) {
  return launch_gemm_grouped(in_t, out_t, trans, gram, wn, at<GroupGemm>(b, l.desc),
                             at<int4>(b, l.map), l.nblocks, st);
}

hipError_t run_part(const rqlp_batch* b, const ProdSet& ps, size_t i, int trans,
                    hipStream_t st) {
  const auto& pl = ps.parts[i];
  return ps.rem ? launch_gemm_rem_grouped(b->dt, trans, pl.first,
                                          at<GroupGemm>(b, pl.second.desc),
                                          at<int4>(b, pl.second.map), pl.second.nblocks, st)
                : run_gemm(b, pl.second, b->dt, b->dt, trans, false, pl.first, st);
}

// One product over all matrices: one launch per width class.  Classes after
// the first go to the side streams (each waits for the calling stream's work
// so far and the calling stream waits for them at the end), so the classes
// overlap and one class's tail does not idle the device.
hipError_t run_prod(const rqlp_batch* b, const ProdSet& ps, int trans, hipStream_t st) {
  const size_t np = ps.parts.size();
  if (np == 0) return hipSuccess;
  const size_t nside = std::min<size_t>(np - 1, rqlp_batch::kSide);
  if (nside == 0 || !b->fork_ev) return run_part(b, ps, 0, trans, st);
  hipError_t e = hipEventRecord(b->fork_ev, st);
  for (size_t i = 1; e == hipSuccess && i < np; ++i) {
    const size_t sd = (i - 1) % nside;
    hipStream_t ss = b->side[sd];
    if (i <= nside) e = hipStreamWaitEvent(ss, b->fork_ev, 0);
    if (e == hipSuccess) e = run_part(b, ps, i, trans, ss);
  }
  if (e == hipSuccess) e = run_part(b, ps, 0, trans, st);
  for (size_t sd = 0; e == hipSuccess && sd < nside; ++sd) {
    e = hipEventRecord(b->join_ev[sd], b->side[sd]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->join_ev[sd], 0);
  }
  return e;
}

hipError_t run_trsm(const rqlp_batch* b, const Launch& l, hipStream_t st) {
  return launch_trsm_grouped(b->dt, at<GroupTrsm>(b, l.desc), at<int2>(b, l.map), l.nblocks,
                             (int)b->dmax, st);
}

hipError_t run_chol(const rqlp_batch* b, hipStream_t st) {
  return launch_cholesky_grouped(at<GroupChol>(b, b->chol.desc), (int)b->chol.count, st);
}

hipError_t run_fo(const rqlp_batch* b, hipStream_t st) {
  return launch_first_order_grouped(b->dt, at<GroupFirstOrder>(b, b->fo.desc),
                                    (int)b->fo.count, st);
}

#define B_TRY(expr)                  \
  do {                               \
    hipError_t e_ = (expr);          \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// The whole grouped sequence (the same steps, in the same order, as the
// single-matrix fast path).
hipError_t enqueue(const rqlp_batch* b, hipStream_t st) {
  const Dtype dt = b->dt;
  if (b->grouped.empty()) return hipSuccess;
  auto orth_inplace = [&](const Launch& gram, const Launch& trsm) -> hipError_t {
    B_TRY(run_gemm(b, gram, dt, DT_F64, 1, true, 1, st));
    B_TRY(run_chol(b, st));
    return run_trsm(b, trsm, st);
  };
  B_TRY(launch_zero_ints(b->flags, (int64_t)b->grouped.size() * 16, st));
  B_TRY(launch_gaussian_grouped(dt, at<GroupGauss>(b, b->gauss.desc), at<int2>(b, b->gauss.map),
                                b->gauss.nblocks, st));                       // randn
  B_TRY(run_prod(b, b->tn, 1, st));                                           // A^T Omega
  B_TRY(orth_inplace(b->gramY, b->trsmY));                                    // Qbar
  for (int it = 0; it < b->q; ++it) {
    B_TRY(run_prod(b, b->nn, 0, st));                                         // A Qbar
    B_TRY(orth_inplace(b->gramZ, b->trsmZ));
    B_TRY(run_prod(b, b->tn, 1, st));                                         // A^T Q
    B_TRY(orth_inplace(b->gramY, b->trsmY));
  }
  B_TRY(run_prod(b, b->nn, 0, st));                                           // A Qbar
  // Q: Cholesky QR, then the second pass to first order
  B_TRY(run_gemm(b, b->gramZ, dt, DT_F64, 1, true, 1, st));
  B_TRY(run_chol(b, st));
  B_TRY(run_trsm(b, b->trsmZT, st));
  B_TRY(run_gemm(b, b->gramTm, dt, DT_F64, 1, true, 1, st));
  B_TRY(run_fo(b, st));
  B_TRY(run_gemm(b, b->qfin, dt, dt, 0, false, 2, st));
  // W = A^T Q; P, R
  B_TRY(run_prod(b, b->tn_final, 1, st));
  B_TRY(run_gemm(b, b->gramY, dt, DT_F64, 1, true, 1, st));
  B_TRY(run_chol(b, st));
  B_TRY(run_trsm(b, b->trsmYT, st));
  B_TRY(run_gemm(b, b->gramTn, dt, DT_F64, 1, true, 1, st));
  B_TRY(run_fo(b, st));
  B_TRY(run_gemm(b, b->pfin, dt, dt, 0, false, 2, st));
  B_TRY(run_gemm(b, b->rcomb, DT_F64, DT_F64, 0, false, 2, st));             // R = R2 R1
  return launch_lower_grouped(at<GroupLower>(b, b->lower.desc), (int)b->lower.count, st);
}

// Times one grouped product with the given block map (ms per launch).
double time_product(const rqlp_batch* b, const ProdSet& ps, int trans, hipStream_t st) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 1e30;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return 1e30;
  }
  double best = 1e30;
  (void)run_prod(b, ps, trans, st);  // warm-up
  for (int r = 0; r < 3; ++r) {
    (void)hipEventRecord(e0, st);
    (void)run_prod(b, ps, trans, st);
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

void free_batch(rqlp_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (int i = 0; i < rqlp_batch::kSide; ++i) {
    if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
    if (b->join_ev[i]) (void)hipEventDestroy(b->join_ev[i]);
  }
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->ws) (void)hipFree(b->ws);
  if (b->tab) (void)hipFree(b->tab);
  if (b->flags) (void)hipFree(b->flags);
  delete b;
}

}  // namespace

extern "C" {

rqlp_status randqlp_batch_create(int count, const void* const* A, const int64_t* m,
                                 const int64_t* n, const int64_t* lda, const int* k, int p, int q,
                                 const uint64_t* seeds, void* const* Q, const int64_t* ldq,
                                 void* const* L, const int64_t* ldl, void* const* P,
                                 const int64_t* ldp, int precision, int tune,
                                 rqlp_batch** out) {
  if (!out) return rqlp_fail(RQLP_E_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (count < 1 || !A || !m || !n || !k || !seeds || !Q || !L || !P)
    return rqlp_fail(RQLP_E_INVALID_ARG, "bad count or null array");
  if (p < 0 || q < 0) return rqlp_fail(RQLP_E_INVALID_ARG, "p and q must be >= 0");
  if (precision != RQLP_F64 && precision != RQLP_F32)
    return rqlp_fail(RQLP_E_INVALID_ARG, "batched precision must be RQLP_F64 or RQLP_F32");
  rqlp_batch* b = new rqlp_batch();
  b->count = count;
  b->q = q;
  b->p = p;
  b->dt = precision == RQLP_F64 ? DT_F64 : DT_F32;
  const size_t es = esize(b->dt);
  for (int i = 0; i < count; ++i) {
    const int64_t di = randqlp_sketch_width(m[i], n[i], k[i], p);
    const int64_t la = lda ? lda[i] : m[i], lq = ldq ? ldq[i] : m[i];
    const int64_t ll = ldl ? ldl[i] : di, lp = ldp ? ldp[i] : n[i];
    if (di < 1 || !A[i] || !Q[i] || !L[i] || !P[i] || la < m[i] || lq < m[i] || ll < di ||
        lp < n[i] || m[i] >= (1ll << 31) || n[i] >= (1ll << 31)) {
      free_batch(b);
      return rqlp_fail(RQLP_E_INVALID_ARG, "matrix %d: bad size, pointer or leading dimension", i);
    }
    b->m.push_back(m[i]);
    b->n.push_back(n[i]);
    b->d.push_back(di);
    b->k.push_back(k[i]);
    b->lda.push_back(la);
    b->ldq.push_back(lq);
    b->ldl.push_back(ll);
    b->ldp.push_back(lp);
    b->seed.push_back(seeds[i]);
    b->A.push_back(A[i]);
    b->Q.push_back(Q[i]);
    b->L.push_back((double*)L[i]);
    b->P.push_back(P[i]);
    if (di <= CHOL_MAX_D) {
      b->grouped.push_back(i);
      b->dmax = std::max(b->dmax, di);
    } else {
      b->individual.push_back(i);
    }
  }
  // per-matrix workspaces
  struct Off { size_t Zm, Tm, Yn, Tn, G, R0, R1, B, Rf, dinv; };
  std::vector<Off> off(count);
  size_t tot = 0;
  auto take = [&](size_t bytes) {
    size_t o = tot;
    tot += align_up(bytes);
    return o;
  };
  for (int i : b->grouped) {
    const size_t mi = b->m[i], ni = b->n[i], di = b->d[i];
    off[i].Zm = take(mi * di * es);
    off[i].Tm = take(mi * di * es);
    off[i].Yn = take(ni * di * es);
    off[i].Tn = take(ni * di * es);
    off[i].G = take(di * di * 8);
    off[i].R0 = take(di * di * 8);
    off[i].R1 = take(di * di * 8);
    off[i].B = take(di * di * es);
    off[i].Rf = take(di * di * 8);
    off[i].dinv = take((di + 15) / 16 * 256 * 8);
  }
  hipError_t e = hipSuccess;
  if (!b->grouped.empty()) {
    e = hipMalloc((void**)&b->ws, std::max<size_t>(tot, 256));
    if (e == hipSuccess) e = hipMalloc((void**)&b->flags, b->grouped.size() * 16 * sizeof(int));
  }
  if (e != hipSuccess) {
    free_batch(b);
    return rqlp_fail(RQLP_E_NOMEM, "batch workspace of %zu bytes: %s", tot, hipGetErrorString(e));
  }
  // descriptors (indices into the grouped list)
  std::vector<GroupGauss> gg;
  std::vector<GroupGemm> tn, nn, tnf, grY, grZ, grTm, grTn, qf, pf, rc;
  std::vector<GroupChol> ch;
  std::vector<GroupTrsm> tY, tZ, tZT, tYT;
  std::vector<GroupFirstOrder> fo;
  std::vector<GroupLower> lo;
  const double fo_tol = b->dt == DT_F64 ? 1e-8 : 1e-3;
  for (size_t g = 0; g < b->grouped.size(); ++g) {
    const int i = b->grouped[g];
    const int64_t mi = b->m[i], ni = b->n[i], di = b->d[i];
    char* w = b->ws;
    void *Zm = w + off[i].Zm, *Tm = w + off[i].Tm, *Yn = w + off[i].Yn, *Tn = w + off[i].Tn;
    double *G = (double*)(w + off[i].G), *R0 = (double*)(w + off[i].R0);
    double *R1 = (double*)(w + off[i].R1), *Rf = (double*)(w + off[i].Rf);
    double* dinv = (double*)(w + off[i].dinv);
    void* Bm = w + off[i].B;
    int* fl = b->flags + 16 * g;
    gg.push_back(GroupGauss{Zm, mi, di, mi, b->seed[i]});
    tn.push_back(GroupGemm{b->A[i], b->lda[i], Zm, mi, Yn, ni, ni, di, mi});
    nn.push_back(GroupGemm{b->A[i], b->lda[i], Yn, ni, Zm, mi, mi, di, ni});
    tnf.push_back(GroupGemm{b->A[i], b->lda[i], b->Q[i], b->ldq[i], Yn, ni, ni, di, mi});
    grY.push_back(GroupGemm{Yn, ni, Yn, ni, G, di, di, di, ni});
    grZ.push_back(GroupGemm{Zm, mi, Zm, mi, G, di, di, di, mi});
    grTm.push_back(GroupGemm{Tm, mi, Tm, mi, G, di, di, di, mi});
    grTn.push_back(GroupGemm{Tn, ni, Tn, ni, G, di, di, di, ni});
    qf.push_back(GroupGemm{Tm, mi, Bm, di, b->Q[i], b->ldq[i], mi, di, di});
    pf.push_back(GroupGemm{Tn, ni, Bm, di, b->P[i], b->ldp[i], ni, di, di});
    rc.push_back(GroupGemm{R1, di, R0, di, Rf, di, di, di, di});
    ch.push_back(GroupChol{G, di, R0, di, dinv, fl, (int)di, kTolDepFastB, 0.0});
    tY.push_back(GroupTrsm{Yn, ni, ni, R0, di, dinv, Yn, ni, (int)di});
    tZ.push_back(GroupTrsm{Zm, mi, mi, R0, di, dinv, Zm, mi, (int)di});
    tZT.push_back(GroupTrsm{Zm, mi, mi, R0, di, dinv, Tm, mi, (int)di});
    tYT.push_back(GroupTrsm{Yn, ni, ni, R0, di, dinv, Tn, ni, (int)di});
    fo.push_back(GroupFirstOrder{G, Bm, R1, fl, (int)di, fo_tol});
    lo.push_back(GroupLower{Rf, b->L[i], b->ldl[i], (int)di});
  }
  // tile widths: table, else cover the typical d
  std::vector<int64_t> ds;
  for (int i : b->grouped) ds.push_back(b->d[i]);
  std::sort(ds.begin(), ds.end());
  const int64_t dmed = ds.empty() ? 1 : ds[ds.size() / 2];
  (void)dmed;
  b->wn_tn = lookup_wn(b->dt, 1, b->dmax, kRemSet);
  b->wn_nn = lookup_wn(b->dt, 0, b->dmax, kRemSet);
  std::vector<char>& buf = b->host_tab;
  {
    std::vector<int2> map;
    for (size_t g = 0; g < gg.size(); ++g) gauss_grouped_blocks(gg[g], (int)g, map);
    b->gauss.desc = put(buf, gg);
    b->gauss.map = put(buf, map);
    b->gauss.count = (int64_t)gg.size();
    b->gauss.nblocks = (int64_t)map.size();
  }
  for (int wn : {0, 1, 2, 4, 8, kRemSet}) {
    b->tn_alt[wn] = prod_set(buf, tn, wn, b->dt);
    b->tnf_alt[wn] = prod_set(buf, tnf, wn, b->dt);
  }
  for (int wn : {0, 1, 2, 4, kRemSet}) b->nn_alt[wn] = prod_set(buf, nn, wn, b->dt);
  if (!b->tn_alt.count(b->wn_tn)) b->wn_tn = 0;
  if (!b->nn_alt.count(b->wn_nn)) b->wn_nn = 0;
  b->tn = b->tn_alt[b->wn_tn];
  b->nn = b->nn_alt[b->wn_nn];
  b->tn_final = b->tnf_alt[b->wn_tn];
  b->gramY = gemm_launch(buf, grY, true, 1);
  b->gramZ = gemm_launch(buf, grZ, true, 1);
  b->gramTm = gemm_launch(buf, grTm, true, 1);
  b->gramTn = gemm_launch(buf, grTn, true, 1);
  b->qfin = gemm_launch(buf, qf, false, 2);
  b->pfin = gemm_launch(buf, pf, false, 2);
  b->rcomb = gemm_launch(buf, rc, false, 2);
  b->chol.desc = put(buf, ch);
  b->chol.count = (int64_t)ch.size();
  b->trsmY = trsm_launch(buf, tY);
  b->trsmZ = trsm_launch(buf, tZ);
  b->trsmZT = trsm_launch(buf, tZT);
  b->trsmYT = trsm_launch(buf, tYT);
  b->fo.desc = put(buf, fo);
  b->fo.count = (int64_t)fo.size();
  b->lower.desc = put(buf, lo);
  b->lower.count = (int64_t)lo.size();
  if (!buf.empty()) {
    e = hipMalloc((void**)&b->tab, buf.size());
    if (e == hipSuccess) e = hipMemcpy(b->tab, buf.data(), buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_batch(b);
      return rqlp_fail(RQLP_E_NOMEM, "batch tables: %s", hipGetErrorString(e));
    }
  }
  e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  for (int i = 0; e == hipSuccess && i < rqlp_batch::kSide; ++i) {
    e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);  // default priority
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join_ev[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    free_batch(b);
    return rqlp_fail(RQLP_E_HIP, "stream: %s", hipGetErrorString(e));
  }
  if (tune && !b->grouped.empty()) {
    // time each candidate width of both products on this batch's data
    hipEvent_t t0, t1;
    float tms = 0.f;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    (void)hipEventRecord(t0, b->cap);
    e = launch_gaussian_grouped(b->dt, at<GroupGauss>(b, b->gauss.desc),
                                at<int2>(b, b->gauss.map), b->gauss.nblocks, b->cap);
    double best = 1e30;
    for (auto& kv : b->tn_alt) {
      const double t = time_product(b, kv.second, 1, b->cap);
      if (t < best) {
        best = t;
        b->wn_tn = kv.first;
      }
    }
    best = 1e30;
    for (auto& kv : b->nn_alt) {
      const double t = time_product(b, kv.second, 0, b->cap);
      if (t < best) {
        best = t;
        b->wn_nn = kv.first;
      }
    }
    (void)hipEventRecord(t1, b->cap);
    if (hipEventSynchronize(t1) == hipSuccess) (void)hipEventElapsedTime(&tms, t0, t1);
    b->tune_ms = tms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      g_tune[{(int)b->dt, 1, dbucket(b->dmax)}] = b->wn_tn;
      g_tune[{(int)b->dt, 0, dbucket(b->dmax)}] = b->wn_nn;
    }
    b->tn = b->tn_alt[b->wn_tn];
    b->nn = b->nn_alt[b->wn_nn];
    b->tn_final = b->tnf_alt[b->wn_tn];
  }
  // capture the grouped sequence
  e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t ee = enqueue(b, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (ee != hipSuccess) e = ee;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    free_batch(b);
    return rqlp_fail(RQLP_E_HIP, "graph capture: %s", hipGetErrorString(e));
  }
  *out = b;
  return RQLP_OK;
}

rqlp_status randqlp_batch_run(rqlp_batch* b, int use_graph, void* stream) {
  if (!b) return rqlp_fail(RQLP_E_INVALID_ARG, "null batch");
  const hipStream_t st = (hipStream_t)stream;
  hipError_t e = use_graph ? hipGraphLaunch(b->exec, st) : enqueue(b, st);
  std::vector<int> fl(b->grouped.size() * 16, 0);
  if (e == hipSuccess && !fl.empty())
    e = hipMemcpyAsync(fl.data(), b->flags, fl.size() * sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return rqlp_fail(RQLP_E_HIP, "batched run: %s", hipGetErrorString(e));
  std::vector<int> redo = b->individual;
  for (size_t g = 0; g < b->grouped.size(); ++g)
    if (fl[16 * g] & (FLAG_NONPOS_PIVOT | FLAG_NONFINITE | FLAG_SECOND_PASS))
      redo.push_back(b->grouped[g]);
  b->last_fallbacks = (int)redo.size();
  for (int i : redo) {
    rqlp_opts o;
    rqlp_opts_default(&o);
    o.precision = b->dt == DT_F64 ? RQLP_F64 : RQLP_F32;
    o.lda = b->lda[i];
    o.ldq = b->ldq[i];
    o.ldl = b->ldl[i];
    o.ldp = b->ldp[i];
    o.stream = stream;
    rqlp_status s = randqlp_factor(b->A[i], b->m[i], b->n[i], b->k[i], b->p, b->q, b->seed[i],
                                   b->Q[i], b->L[i], b->P[i], &o);
    if (s != RQLP_OK) return s;
  }
  return RQLP_OK;
}

rqlp_status randqlp_batch_query(const rqlp_batch* b, rqlp_batch_info* info) {
  if (!b || !info) return rqlp_fail(RQLP_E_INVALID_ARG, "null argument");
  info->count = b->count;
  info->grouped = (int32_t)b->grouped.size();
  info->fallbacks = b->last_fallbacks;
  info->wn_tn = b->wn_tn;
  info->wn_nn = b->wn_nn;
  info->dmax = (int32_t)b->dmax;
  info->tune_ms = b->tune_ms;
  return RQLP_OK;
}

void randqlp_batch_destroy(rqlp_batch* b) { free_batch(b); }

rqlp_status randqlp_factor_batched(int count, const void* const* A, const int64_t* m,
                                   const int64_t* n, const int* k, int p, int q,
                                   const uint64_t* seeds, void* const* Q, void* const* L,
                                   void* const* P, int precision, void* stream) {
  rqlp_batch* b = nullptr;
  rqlp_status s = randqlp_batch_create(count, A, m, n, nullptr, k, p, q, seeds, Q, nullptr, L,
                                       nullptr, P, nullptr, precision, 0, &b);
  if (s != RQLP_OK) return s;
  s = randqlp_batch_run(b, 1, stream);
  free_batch(b);
  return s;
}

rqlp_status randqlp_tune_save(const char* path) {
  if (!path) return rqlp_fail(RQLP_E_INVALID_ARG, "null path");
  FILE* f = std::fopen(path, "w");
  if (!f) return rqlp_fail(RQLP_E_INVALID_ARG, "cannot write %s", path);
  std::lock_guard<std::mutex> g(g_tune_mu);
  std::fprintf(f, "# dtype(0=f64,1=f32) trans dbucket wn\n");
  for (auto& kv : g_tune)
    std::fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first),
                 std::get<2>(kv.first), kv.second);
  std::fclose(f);
  return RQLP_OK;
}

rqlp_status randqlp_tune_load(const char* path) {
  if (!path) return rqlp_fail(RQLP_E_INVALID_ARG, "null path");
  FILE* f = std::fopen(path, "r");
  if (!f) return rqlp_fail(RQLP_E_INVALID_ARG, "cannot read %s", path);
  char line[256];
  int nread = 0;
  std::lock_guard<std::mutex> g(g_tune_mu);
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int dt = 0, tr = 0, bk = 0, wn = 0;
    if (std::sscanf(line, "%d %d %d %d", &dt, &tr, &bk, &wn) == 4 && (dt == 0 || dt == 1) &&
        (tr == 0 || tr == 1) && wn >= 0 && (wn <= 8 || wn == kRemSet)) {
      g_tune[{dt, tr, bk}] = (wn == 0 || wn == kRemSet) ? wn : grouped_wn_round(wn);
      ++nread;
    }
  }
  std::fclose(f);
  return RQLP_OK;
}

}  // extern "C"

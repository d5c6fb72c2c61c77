// C entry points: setup of the hierarchy, the combined smoother, the V-cycle
// and multigrid-preconditioned CG (paper Sec. 2 Algorithm alg:mg, Sec. 4.2,
// Sec. 6.2).  Host code here only orchestrates: every numerical step of the
// solve phase is one of the HIP kernels of solve.hip.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "mg_internal.h"

namespace mg {

void fail(mg_status code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error{code, std::string(buf)};
}

Ctx::~Ctx() {
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  for (int k = 0; k < 5; ++k) {
    if (cg_exec[k]) (void)hipGraphExecDestroy(cg_exec[k]);
    if (cg_graph[k]) (void)hipGraphDestroy(cg_graph[k]);
  }
  for (auto &e : events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (h_scal) (void)hipHostFree(h_scal);
  lv.clear();
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

enum { W_B = 0, W_U = 1, W_ALT = 2, W_D = 3, W_R = 4, W_T = 5 };

template <class T>
struct LV;
template <>
struct LV<double> {
  static double *w(Level &L, int k) { return L.w64[k].p; }
  static double *res(Level &L) { return L.res64.p; }
  static double *py(Level &L) { return L.py64.p; }
  static double *pz(Level &L) { return L.pz64.p; }
  static const double *dinv(Level &L) { return L.dinv64.p; }
};
template <>
struct LV<float> {
  static float *w(Level &L, int k) { return L.w32[k].p; }
  static float *res(Level &L) { return L.res32.p; }
  static float *py(Level &L) { return L.py32.p; }
  static float *pz(Level &L) { return L.pz32.p; }
  static const float *dinv(Level &L) { return L.dinv32.p; }
};

void ensure_work(Ctx &c, Level &L) {
  bool mixed = c.opt.precision == MG_MIXED;
  for (int k = 0; k < 6; ++k) {
    if (mixed) L.w32[k].alloc(L.nfree); else L.w64[k].alloc(L.nfree);
  }
  if (L.patch.total > 0) {
    if (mixed) {
      L.res32.alloc(L.patch.total);
      L.py32.alloc(L.patch.inv.ysize);
      L.pz32.alloc(std::max<int64_t>(1, L.patch.inv.zsize));
    } else {
      L.res64.alloc(L.patch.total);
      L.py64.alloc(L.patch.inv.ysize);
      L.pz64.alloc(std::max<int64_t>(1, L.patch.inv.zsize));
    }
  }
  if (L.patch.total > 0 && c.opt.patch_refine) {
    L.pst.alloc(L.nfree);
    fill<double>(c.stream, L.pst.p, L.nfree, 0.0);
  }
  if (L.coarsest) {
    L.cpy.alloc(L.cpk.ysize);
    L.cpz.alloc(std::max<int64_t>(1, L.cpk.zsize));
  }
}

// ---------------------------------------------------------------------------
// smoother and V-cycle
// ---------------------------------------------------------------------------
template <class T>
static void local_correction(Ctx &c, Level &L, const T *b, T *u, bool descending);

// device time (ms) of f() on the context's stream: the average launch of the
// fastest of three batches of five (clock and boost changes only slow a batch)
template <class F>
static double time_on_stream(Ctx &c, F f) {
  hipEvent_t e0, e1;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  struct G {
    hipEvent_t a, b;
    ~G() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } g{e0, e1};
  f();
  float best = -1;
  for (int batch = 0; batch < 3; ++batch) {
    MG_HIP(hipEventRecord(e0, c.stream));
    for (int r = 0; r < 5; ++r) f();
    MG_HIP(hipEventRecord(e1, c.stream));
    MG_HIP(hipEventSynchronize(e1));
    float t = 0;
    MG_HIP(hipEventElapsedTime(&t, e0, e1));
    if (best < 0 || t < best) best = t;
  }
  return best / 5.0;
}

// Lanes per patch row (1, 2, 4 or 8) of a level's patch-row residual: the
// option's value, else the fastest of the four on the residual launches of
// all colours (the first of the order 1, 2, 4, 8 within 2 % of the fastest).
// One lane per row is kept where the patch solves are refined (their
// refinement values share the rows' layout), where every colour can run the
// fused one-launch correction (whose residual reads whole slices of one lane
// per row), and on levels with fewer than 2^20 stored patch-row entries.
// The lanes per row set the order in which a row's products are summed.
static void tune_patch_rows(Ctx &c, Level &L) {
  Patches &P = L.patch;
  const bool mixed = c.opt.precision == MG_MIXED;
  const int fixed = c.opt.patch_rows_rpl;
  if (fixed) {
    relayout_patch_rows(c, L, mixed, fixed);
    return;
  }
  bool all_fused = c.opt.patch_fused && P.maxn <= 12 * PATCH_TILE;
  for (int col = 0; col < P.ncolour; ++col) all_fused &= P.colour_fused[col] != 0;
  if (c.opt.patch_refine || all_fused || P.rows.stored < (1 << 20)) {
    relayout_patch_rows(c, L, mixed, 1);
    return;
  }
  auto run = [&] {
    for (int col = 0; col < P.ncolour; ++col) {
      if (mixed) patch_residual<float>(c.stream, P, col, L.w32[0], L.w32[1], LV<float>::res(L));
      else patch_residual<double>(c.stream, P, col, L.w64[0], L.w64[1], LV<double>::res(L));
    }
  };
  if (mixed) {
    fill<float>(c.stream, L.w32[0], L.nfree, 0.5f);
    fill<float>(c.stream, L.w32[1], L.nfree, 0.5f);
  } else {
    fill<double>(c.stream, L.w64[0], L.nfree, 0.5);
    fill<double>(c.stream, L.w64[1], L.nfree, 0.5);
  }
  double best = -1;
  int pick = 1;
  for (int rpl : {1, 2, 4, 8}) {
    relayout_patch_rows(c, L, mixed, rpl);
    const double t = time_on_stream(c, run);
    if (best < 0 || t < 0.98 * best) {
      if (best < 0 || t < best) best = t;
      pick = rpl;
    }
  }
  relayout_patch_rows(c, L, mixed, pick);
}

// Patch-path autotuner of a level (setup): the packed-row chunk of the patch
// inverses (8, 16 or 32 tiles per row item) and the one-workgroup size class
// of the local correction (patches of up to 128, 256 or 384 DOFs, or the
// three-launch path), each timed on the level's whole local correction; of
// the candidates within 2 % of the fastest the first of the order (chunk 16,
// then 8, 32; the smallest one-workgroup class, then the larger ones, then the
// three-launch path) is kept, so that timing noise rarely changes the choice.
// The chunk sets the order in which a tile row's products are summed; the
// size class changes no result.  Levels whose patch inverses hold fewer than
// 4096 tiles keep chunk 16 and the smallest class (launch latency decides
// there).  The coarsest inverse's chunk is timed the same way (n >= 2048).
static void tune_patches(Ctx &c, Level &L) {
  const bool mixed = c.opt.precision == MG_MIXED;
  if (L.coarsest) {
    if (L.cnd.on) return;
    const int64_t n = L.nfree;
    const int fixed = c.opt.patch_chunk;
    if (fixed == 0 && n < 2048) return;
    std::vector<int32_t> kptr = {0, (int32_t)n};
    std::vector<int> cf = {0, 1};
    std::vector<int> cand = fixed ? std::vector<int>{fixed} : std::vector<int>{16, 8, 32};
    if (cand.size() == 1 && cand[0] == L.cpk.chunk) return;
    DBuf<double> b, u;
    b.alloc(n);
    u.alloc(n);
    fill<double>(c.stream, b.p, n, 0.5);
    double best = -1;
    int pick = cand[0];
    for (int ch : cand) {
      build_packed_layout(c.stream, kptr, cf, L.cpk, ch);
      L.cpy.alloc(L.cpk.ysize);
      const double t = time_on_stream(c, [&] { coarse_apply<double>(c.stream, L, b.p, u.p); });
      if (best < 0 || t < 0.98 * best) {
        if (best < 0 || t < best) best = t;
        pick = ch;
      }
    }
    if (L.cpk.chunk != pick) {
      build_packed_layout(c.stream, kptr, cf, L.cpk, pick);
      L.cpy.alloc(L.cpk.ysize);
    }
    return;
  }
  Patches &P = L.patch;
  P.small_nb = 0;
  if (P.n == 0 || !c.opt.local_correction) return;
  tune_patch_rows(c, L);
  // size classes that take every patch of the level
  std::vector<int> nbs;
  if (c.opt.patch_fused && !c.opt.patch_refine) {
    if (c.opt.patch_small_bound > 0) {
      if (c.opt.patch_small_bound >= P.maxn) nbs.push_back(c.opt.patch_small_bound / PATCH_TILE);
    } else if (c.opt.patch_small_bound == 0) {
      for (int nb : {4, 8, 12})
        if (nb * PATCH_TILE >= P.maxn) nbs.push_back(nb);
    }
  }
  std::vector<int> chunks = c.opt.patch_chunk ? std::vector<int>{c.opt.patch_chunk} : std::vector<int>{16, 8, 32};
  const int64_t tiles = P.inv.packed / (PATCH_TILE * PATCH_TILE);
  const bool timed = tiles >= 4096;
  auto relayout = [&](int ch) {
    if (P.inv.chunk == ch) return;
    build_packed_layout(c.stream, P.h_kptr, P.colour_first, P.inv, ch);
    if (mixed) L.py32.alloc(P.inv.ysize); else L.py64.alloc(P.inv.ysize);
  };
  if (!timed) {
    relayout(chunks[0]);
    if (!nbs.empty()) P.small_nb = nbs[0];
    return;
  }
  auto run = [&] {
    if (mixed) local_correction<float>(c, L, L.w32[0], L.w32[1], false);
    else local_correction<double>(c, L, L.w64[0], L.w64[1], false);
  };
  if (mixed) {
    fill<float>(c.stream, L.w32[0], L.nfree, 0.5f);
    fill<float>(c.stream, L.w32[1], L.nfree, 0.5f);
  } else {
    fill<double>(c.stream, L.w64[0], L.nfree, 0.5);
    fill<double>(c.stream, L.w64[1], L.nfree, 0.5);
  }
  // the chunk, on the three-launch path
  double best = -1;
  int pick = chunks[0];
  for (int ch : chunks) {
    relayout(ch);
    const double t = time_on_stream(c, run);
    if (best < 0 || t < 0.98 * best) {
      if (best < 0 || t < best) best = t;
      pick = ch;
    }
  }
  relayout(pick);
  // the size class (or the three-launch path, timed above)
  double best_nb = -1;
  int pick_nb = 0;
  for (int nb : nbs) {
    P.small_nb = nb;
    const double t = time_on_stream(c, run);
    if (best_nb < 0 || t < 0.98 * best_nb) {
      if (best_nb < 0 || t < best_nb) best_nb = t;
      pick_nb = nb;
    }
  }
  P.small_nb = (best_nb >= 0 && best_nb <= 1.02 * best) ? pick_nb : 0;
}
// slot: the level of a full Chebyshev step, or the coarsest level's index
// for the coarsest solve
static void time_begin(Ctx &c, int slot) {
  if (!c.timing) return;
  if (c.events_used == c.events.size()) {
    // timing only: no system-scope fence when the event is recorded (the
    // default one writes back and invalidates the caches, which would slow
    // the kernel that follows); the times are read after a stream sync
    hipEvent_t a, b;
    MG_HIP(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
    MG_HIP(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
    c.events.push_back({a, b});
    c.event_slot.push_back(0);
  }
  c.event_slot[c.events_used] = slot;
  MG_HIP(hipEventRecord(c.events[c.events_used].first, c.stream));
}
static void time_end(Ctx &c) {
  if (!c.timing) return;
  MG_HIP(hipEventRecord(c.events[c.events_used].second, c.stream));
  ++c.events_used;
}

template <class T>
static void local_correction(Ctx &c, Level &L, const T *b, T *u, bool descending) {
  for (int k = 0; k < L.patch.ncolour; ++k) {
    int col = descending ? L.patch.ncolour - 1 - k : k;
    if (c.opt.patch_refine) {
      patch_residual<T>(c.stream, L.patch, col, b, u, LV<T>::res(L));
      patch_apply_refined<T>(c.stream, L.patch, col, LV<T>::res(L), LV<T>::py(L), LV<T>::pz(L), u, L.pst.p);
      continue;
    }
    if (L.patch.small_nb && L.patch.colour_fused[col] && L.patch.rows.rpl == 1) {
      patch_correct_small<T>(c.stream, L.patch, col, b, (const T *)nullptr, u);
      continue;
    }
    patch_residual<T>(c.stream, L.patch, col, b, u, LV<T>::res(L));
    if (L.patch.small_nb) {
      patch_correct_small<T>(c.stream, L.patch, col, b, LV<T>::res(L), u);
      continue;
    }
    patch_apply<T>(c.stream, L.patch, col, LV<T>::res(L), LV<T>::py(L), LV<T>::pz(L), u);
  }
}

// k Chebyshev-Jacobi steps (paper Sec. 3.2; see the recurrence in solve.hip).
// zero_start: u vanishes outside the patch DOFs of the level (the first
// sandwich of a V-cycle level, which starts from u = 0: after S_c only the
// patch DOFs are nonzero, and without S_c nothing is), so the first step needs
// the row products only on the rows coupled to the patch DOFs.
template <class T>
static void chebyshev(Ctx &c, int l, const T *b, T *&u, T *&alt, bool zero_start) {
  Level &L = c.lv[l];
  const double theta = 0.5 * (L.hi + L.lo), delta = 0.5 * (L.hi - L.lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  T *d = LV<T>::w(L, W_D);
  // step flags: 1 = first step (no previous direction), 2 = last step (the
  // direction is not stored)
  const int k = c.opt.cheb_degree;
  if (zero_start) {
    const bool on_patches = c.opt.local_correction && L.patch.n > 0;
    cheb_step_zero<T>(c.stream, L.nfree, on_patches ? &L.patch.nbr : nullptr, L.patch.nbr_pos, LV<T>::dinv(L), b, u,
                      alt, k == 1 ? nullptr : d, 1.0 / theta);
  } else {
    time_begin(c, l);
    cheb_step<T>(c.stream, L.S, LV<T>::dinv(L), b, u, alt, d, k == 1 ? 3 : 1, 0.0, 1.0 / theta);
    time_end(c);
  }
  std::swap(u, alt);
  for (int j = 1; j < k; ++j) {
    double rho_new = 1.0 / (2.0 * sigma - rho);
    time_begin(c, l);
    cheb_step<T>(c.stream, L.S, LV<T>::dinv(L), b, u, alt, d, j == k - 1 ? 2 : 0, rho_new * rho,
                 2.0 * rho_new / delta);
    time_end(c);
    std::swap(u, alt);
    rho = rho_new;
  }
}

// symmetric Gauss-Seidel as S_g: colours ascending, then descending, in place
template <class T>
static void sgs_sweeps(Ctx &c, int l, const T *b, T *u) {
  Level &L = c.lv[l];
  const int nc = (int)L.sgs.size();
  for (int k = 0; k < nc; ++k) sgs_colour_sweep<T>(c.stream, L.sgs[k], L.sgs_pos[k], LV<T>::dinv(L), b, u);
  for (int k = nc - 1; k >= 0; --k) sgs_colour_sweep<T>(c.stream, L.sgs[k], L.sgs_pos[k], LV<T>::dinv(L), b, u);
}

// u <- S^nu (b, u): nu applications of S_c -> S_g -> S_c (paper Sec. 4.2);
// zero_start: u = 0 on entry
template <class T>
static void smooth(Ctx &c, int l, const T *b, T *u, int nu, bool zero_start = false) {
  Level &L = c.lv[l];
  bool local = c.opt.local_correction && L.patch.n > 0;
  T *cur = u, *alt = LV<T>::w(L, W_ALT);
  if (u == alt) alt = LV<T>::w(L, W_T);
  for (int s = 0; s < nu; ++s) {
    if (local) local_correction<T>(c, L, b, cur, false);
    if (c.opt.global_smoother == MG_SMOOTHER_SGS) sgs_sweeps<T>(c, l, b, cur);
    else chebyshev<T>(c, l, b, cur, alt, zero_start && s == 0);
    if (local) local_correction<T>(c, L, b, cur, true);
  }
  if (cur != u) convert<T, T>(c.stream, cur, u, L.nfree);
}

// u = V_l(b) from a zero initial guess (Algorithm alg:mg, correction scheme)
template <class T>
static void vcycle_zero(Ctx &c, int l, const T *b, T *u) {
  Level &L = c.lv[l];
  if (L.coarsest) {
    time_begin(c, l);
    coarse_apply<T>(c.stream, L, b, u);
    time_end(c);
    return;
  }
  // u = 0; without local correction the first Chebyshev step from zero
  // reads no u and writes every entry, so the fill is needed only before a
  // local correction, a Gauss-Seidel sweep or when nothing smooths
  const bool local = c.opt.local_correction && L.patch.n > 0;
  if (local || c.opt.global_smoother != MG_SMOOTHER_CHEBYSHEV || c.opt.nu < 1) fill<T>(c.stream, u, L.nfree, T(0));
  smooth<T>(c, l, b, u, c.opt.nu, true);
  T *r = LV<T>::w(L, W_R);
  sell_spmv<T>(c.stream, L.S, u, r, SPMV_RESID, b);
  Level &C = c.lv[l + 1];
  sell_spmv<T>(c.stream, L.R, r, LV<T>::w(C, W_B), SPMV_SET, nullptr);
  vcycle_zero<T>(c, l + 1, LV<T>::w(C, W_B), LV<T>::w(C, W_U));
  sell_spmv<T>(c.stream, L.P, LV<T>::w(C, W_U), u, SPMV_ADD, nullptr);
  smooth<T>(c, l, b, u, c.opt.nu);
}

// z = B r (FP64 in and out); mixed precision runs the cycle in FP32
static void precondition_eager(Ctx &c, const double *r, double *z) {
  Level &L0 = c.lv[0];
  if (c.opt.precision == MG_MIXED) {
    convert<double, float>(c.stream, r, L0.w32[W_B], L0.nfree);
    vcycle_zero<float>(c, 0, L0.w32[W_B], L0.w32[W_U]);
    convert<float, double>(c.stream, L0.w32[W_U], z, L0.nfree);
  } else {
    vcycle_zero<double>(c, 0, r, z);
  }
}

// the graph replays the cycle on the context's fixed buffers c.r -> c.z
static void precondition(Ctx &c) {
  if (c.opt.use_graph && !c.timing) {
    if (!c.graph_exec) {
      MG_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
      try {
        precondition_eager(c, c.r, c.z);
      } catch (...) {
        hipGraph_t g;
        (void)hipStreamEndCapture(c.stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      MG_HIP(hipStreamEndCapture(c.stream, &c.graph));
      MG_HIP(hipGraphInstantiate(&c.graph_exec, c.graph, nullptr, nullptr, 0));
    }
    MG_HIP(hipGraphLaunch(c.graph_exec, c.stream));
  } else {
    precondition_eager(c, c.r, c.z);
  }
}

static double read_scalar(Ctx &c, const double *d) {
  double h = 0;
  MG_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  MG_HIP(hipStreamSynchronize(c.stream));
  return h;
}

static void dot_to(Ctx &c, const double *x, const double *y, int64_t n, double *out) {
  int nb = dot_blocks(n);
  dot_partials(c.stream, x, y, n, c.partial, nb);
  finish_sum(c.stream, c.partial, nb, out);
}

// ---------------------------------------------------------------------------
// block solve: K right-hand sides of the same operator advanced together
// (block vectors, unknown i of column q at i K + q).  The cycle is the
// single-vector cycle above, column by column; the operator streams
// (smoother, residual, transfers, patch rows) are shared by the K columns,
// the dense patch and coarsest products run once per column.
// ---------------------------------------------------------------------------
template <class T>
struct LB;
template <>
struct LB<double> {
  static double *w(Level &L, int k) { return L.bw64[k].p; }
  static double *res(Level &L) { return L.bres64.p; }
};
template <>
struct LB<float> {
  static float *w(Level &L, int k) { return L.bw32[k].p; }
  static float *res(Level &L) { return L.bres32.p; }
};

static void ensure_block_work(Ctx &c) {
  if (c.kr.p) return;
  const bool mixed = c.opt.precision == MG_MIXED;
  for (Level &L : c.lv) {
    const int64_t n = L.nfree * MG_BLOCK_MAX;
    for (int k = 0; k < 6; ++k) {
      if (mixed) L.bw32[k].alloc(n); else L.bw64[k].alloc(n);
    }
    if (L.patch.total > 0) {
      if (mixed) L.bres32.alloc(L.patch.total * MG_BLOCK_MAX);
      else L.bres64.alloc(L.patch.total * MG_BLOCK_MAX);
    }
  }
  const int64_t n0 = c.lv[0].nfree * MG_BLOCK_MAX;
  c.kz.alloc(n0);
  c.kp.alloc(n0);
  c.kq.alloc(n0);
  c.kx.alloc(n0);
  c.kb.alloc(n0);
  const int64_t pb = std::max<int64_t>(1024, spmv_dot_blocks(c.lv[0].S));
  c.kpartial.alloc(pb * MG_BLOCK_MAX);
  c.kr.alloc(n0);  // last: marks the block work as allocated
}

template <class T>
static void local_correction_block(Ctx &c, Level &L, int K, const T *b, T *u, bool descending) {
  T *res = LB<T>::res(L);
  for (int k = 0; k < L.patch.ncolour; ++k) {
    int col = descending ? L.patch.ncolour - 1 - k : k;
    patch_residual_block<T>(c.stream, L.patch, col, K, b, u, res);
    for (int q = 0; q < K; ++q) {
      if (c.opt.patch_refine)
        patch_apply_refined<T>(c.stream, L.patch, col, res + q, LV<T>::py(L), LV<T>::pz(L), u + q, L.pst.p, K);
      else
        patch_apply<T>(c.stream, L.patch, col, res + q, LV<T>::py(L), LV<T>::pz(L), u + q, K);
    }
  }
}

template <class T>
static void chebyshev_block(Ctx &c, int l, int K, const T *b, T *&u, T *&alt, bool zero_start) {
  Level &L = c.lv[l];
  const double theta = 0.5 * (L.hi + L.lo), delta = 0.5 * (L.hi - L.lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  T *d = LB<T>::w(L, W_D);
  const int k = c.opt.cheb_degree;
  if (zero_start) {
    const bool on_patches = c.opt.local_correction && L.patch.n > 0;
    cheb_step_zero_block<T>(c.stream, L.nfree, K, on_patches ? &L.patch.nbr : nullptr, L.patch.nbr_pos,
                            LV<T>::dinv(L), b, u, alt, k == 1 ? nullptr : d, 1.0 / theta);
  } else {
    cheb_step_block<T>(c.stream, L.S, K, LV<T>::dinv(L), b, u, alt, d, k == 1 ? 3 : 1, 0.0, 1.0 / theta);
  }
  std::swap(u, alt);
  for (int j = 1; j < k; ++j) {
    double rho_new = 1.0 / (2.0 * sigma - rho);
    cheb_step_block<T>(c.stream, L.S, K, LV<T>::dinv(L), b, u, alt, d, j == k - 1 ? 2 : 0, rho_new * rho,
                       2.0 * rho_new / delta);
    std::swap(u, alt);
    rho = rho_new;
  }
}

template <class T>
static void smooth_block(Ctx &c, int l, int K, const T *b, T *u, int nu, bool zero_start) {
  Level &L = c.lv[l];
  bool local = c.opt.local_correction && L.patch.n > 0;
  T *cur = u, *alt = LB<T>::w(L, W_ALT);
  if (u == alt) alt = LB<T>::w(L, W_T);
  for (int s = 0; s < nu; ++s) {
    if (local) local_correction_block<T>(c, L, K, b, cur, false);
    if (c.opt.global_smoother == MG_SMOOTHER_SGS) {
      const int nc = (int)L.sgs.size();
      for (int k = 0; k < nc; ++k)
        sgs_colour_sweep_block<T>(c.stream, L.sgs[k], K, L.sgs_pos[k], LV<T>::dinv(L), b, cur);
      for (int k = nc - 1; k >= 0; --k)
        sgs_colour_sweep_block<T>(c.stream, L.sgs[k], K, L.sgs_pos[k], LV<T>::dinv(L), b, cur);
    } else {
      chebyshev_block<T>(c, l, K, b, cur, alt, zero_start && s == 0);
    }
    if (local) local_correction_block<T>(c, L, K, b, cur, true);
  }
  if (cur != u) convert<T, T>(c.stream, cur, u, L.nfree * K);
}

template <class T>
static void vcycle_zero_block(Ctx &c, int l, int K, const T *b, T *u) {
  Level &L = c.lv[l];
  if (L.coarsest) {
    for (int q = 0; q < K; ++q) coarse_apply<T>(c.stream, L, b + q, u + q, K);
    return;
  }
  fill<T>(c.stream, u, L.nfree * K, T(0));
  smooth_block<T>(c, l, K, b, u, c.opt.nu, true);
  T *r = LB<T>::w(L, W_R);
  sell_spmv_block<T>(c.stream, L.S, K, u, r, SPMV_RESID, b);
  Level &C = c.lv[l + 1];
  sell_spmv_block<T>(c.stream, L.R, K, r, LB<T>::w(C, W_B), SPMV_SET, nullptr);
  vcycle_zero_block<T>(c, l + 1, K, LB<T>::w(C, W_B), LB<T>::w(C, W_U));
  sell_spmv_block<T>(c.stream, L.P, K, LB<T>::w(C, W_U), u, SPMV_ADD, nullptr);
  smooth_block<T>(c, l, K, b, u, c.opt.nu, false);
}

// c.kz = B c.kr for K columns (FP64 in and out; mixed runs the cycle in FP32)
static void precondition_block_eager(Ctx &c, int K) {
  Level &L0 = c.lv[0];
  const int64_t n = L0.nfree * K;
  if (c.opt.precision == MG_MIXED) {
    convert<double, float>(c.stream, c.kr, L0.bw32[W_B], n);
    vcycle_zero_block<float>(c, 0, K, L0.bw32[W_B], L0.bw32[W_U]);
    convert<float, double>(c.stream, L0.bw32[W_U], c.kz, n);
  } else {
    vcycle_zero_block<double>(c, 0, K, c.kr, c.kz);
  }
}

static void dot_block_to(Ctx &c, int K, const double *x, const double *y, int64_t n, double *out) {
  const int nb = dot_blocks(n);
  dot_partials_block(c.stream, K, x, y, n, c.kpartial, nb);
  finish_sum_block(c.stream, K, c.kpartial, nb, out);
}

// ---------------------------------------------------------------------------
// Preconditioned CG (Sec. 6.2) as a host state machine over device work.
// Every iteration is the same device sequence: z = B r (one V-cycle),
// rho' = r.z, beta = rho' / rho, p = z + beta p, q = A p with p.q,
// alpha = rho' / p.q, x += alpha p, r -= alpha q with r.r, and the scalars
// written to pinned host memory.  The first iteration is that sequence from
// p = 0 and rho = 1, which gives p = z.  The host reads r.r once the
// iteration has run and decides; with use_graph the sequence is captured
// once per block width and replayed, so that an iteration costs one graph
// launch and one wait.  A run is one vector (K = 1, the buffers of
// mg_pcg_solve) or a block of K = 2 or 4 interleaved columns (padding
// columns zero); a column of a block that has converged is frozen by its
// device-side active flag while the others go on.
// Device scalars (slot j K + q of column q): 0 rho = r.z, 1 p.q, 2 alpha,
// 3 r.r, 4 rho', 5 beta, 6 breakdown flag, 7 b.b (later the true residual's
// square), 8 active flag (blocks only).
// ---------------------------------------------------------------------------
struct CgBufs {
  double *x, *r, *z, *p, *q, *b;
};
static CgBufs cg_bufs(Ctx &c, int K) {
  if (K == 1) return {c.xpos, c.r, c.z, c.p, c.q, c.bpos};
  return {c.kx, c.kr, c.kz, c.kp, c.kq, c.kb};
}

static void cg_iteration_eager(Ctx &c, int K) {
  Level &L0 = c.lv[0];
  const int64_t n = L0.nfree;
  hipStream_t s = c.stream;
  double *scal = c.scal.p;
  const CgBufs v = cg_bufs(c, K);
  const int nb = dot_blocks(n), sb = spmv_dot_blocks(L0.S);
  if (K == 1) {
    precondition_eager(c, v.r, v.z);
    dot_to(c, v.r, v.z, n, scal + 4);
    cg_beta(s, scal);
    cg_update_p(s, v.p, v.z, scal, n);
    spmv_dot(s, L0.S, v.p, v.q, c.partial);
    finish_sum(s, c.partial, sb, scal + 1);
    cg_alpha(s, scal);
    cg_update_xr(s, v.x, v.r, v.p, v.q, scal, n, c.partial, nb);
    finish_sum(s, c.partial, nb, scal + 3);
    scal_to_host(s, scal, c.h_scal_dev, 8);
  } else {
    precondition_block_eager(c, K);
    dot_block_to(c, K, v.r, v.z, n, scal + 4 * K);
    cg_beta_block(s, K, scal);
    cg_update_p_block(s, K, v.p, v.z, scal, n);
    spmv_dot_block(s, L0.S, K, v.p, v.q, c.kpartial);
    finish_sum_block(s, K, c.kpartial, sb, scal + K);
    cg_alpha_block(s, K, scal);
    cg_update_xr_block(s, K, v.x, v.r, v.p, v.q, scal, n, c.kpartial, nb);
    finish_sum_block(s, K, c.kpartial, nb, scal + 3 * K);
    scal_to_host(s, scal, c.h_scal_dev, 9 * K);
  }
}

static void cg_iteration(Ctx &c, int K) {
  if (!c.opt.use_graph || c.timing) {
    cg_iteration_eager(c, K);
    return;
  }
  if (!c.cg_exec[K]) {
    MG_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    try {
      cg_iteration_eager(c, K);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    MG_HIP(hipStreamEndCapture(c.stream, &c.cg_graph[K]));
    MG_HIP(hipGraphInstantiate(&c.cg_exec[K], c.cg_graph[K], nullptr, nullptr, 0));
  }
  MG_HIP(hipGraphLaunch(c.cg_exec[K], c.stream));
}

struct CgRun {
  Ctx *c = nullptr;
  int K = 1, ncols = 1;  // block width and real columns (ncols <= K)
  const double *b[MG_BLOCK_MAX] = {};
  double *u[MG_BLOCK_MAX] = {};
  double rtol = 0;
  int maxit = 0;
  mg_solve_stats *st = nullptr;  // ncols records or NULL
  enum Phase { START, ITERATE, END, DONE } phase = START;
  bool warm = false;
  double bnorm[MG_BLOCK_MAX] = {}, rel[MG_BLOCK_MAX] = {};
  int iters[MG_BLOCK_MAX] = {};
  bool conv[MG_BLOCK_MAX] = {};
  std::vector<double> hist[MG_BLOCK_MAX];
  unsigned mask = 0;  // columns still iterating
  int it = 0, broken = -1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CgRun() = default;
  CgRun(const CgRun &) = delete;
  CgRun &operator=(const CgRun &) = delete;
  ~CgRun() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// enqueues the start: b (and x_0) in solve order, r_0, b.b (and r_0.r_0)
static void cg_begin(CgRun &R) {
  Ctx &c = *R.c;
  const int K = R.K;
  if (K > 1) ensure_block_work(c);
  Level &L0 = c.lv[0];
  const int64_t n = L0.nfree;
  hipStream_t s = c.stream;
  double *scal = c.scal.p;
  const CgBufs v = cg_bufs(c, K);
  R.warm = c.opt.use_initial_guess != 0;
  MG_HIP(hipEventCreate(&R.e0));
  MG_HIP(hipEventCreate(&R.e1));
  MG_HIP(hipEventRecord(R.e0, s));
  fill<double>(s, scal, 9 * K, 0.0);
  if (K == 1) {
    gather_perm<double, double>(s, R.b[0], L0.perm, v.b, n);
    if (R.warm) gather_perm<double, double>(s, R.u[0], L0.perm, v.x, n);
  } else {
    gather_block(s, K, R.b, L0.perm, v.b, n);
    if (R.warm) gather_block(s, K, R.u, L0.perm, v.x, n);
  }
  if (R.warm) {  // r_0 = b - A x_0
    if (K == 1) {
      sell_spmv<double>(s, L0.S, v.x, v.r, SPMV_RESID, v.b);
      dot_to(c, v.r, v.r, n, scal + 3);
    } else {
      sell_spmv_block<double>(s, L0.S, K, v.x, v.r, SPMV_RESID, v.b);
      dot_block_to(c, K, v.r, v.r, n, scal + 3 * K);
    }
  } else {
    fill<double>(s, v.x, n * K, 0.0);
    copy64(s, v.b, v.r, n * K);
  }
  if (K == 1) dot_to(c, v.b, v.b, n, scal + 7);
  else dot_block_to(c, K, v.b, v.b, n, scal + 7 * K);
  scal_to_host(s, scal, c.h_scal_dev, 8 * K);
  R.phase = CgRun::START;
}

// enqueues the end: x back to the caller's order, the end event, the true
// residual b - A x in FP64
static void cg_end(CgRun &R) {
  Ctx &c = *R.c;
  const int K = R.K;
  Level &L0 = c.lv[0];
  const int64_t n = L0.nfree;
  hipStream_t s = c.stream;
  double *scal = c.scal.p;
  const CgBufs v = cg_bufs(c, K);
  if (K == 1) {
    if (R.bnorm[0] == 0.0) fill<double>(s, v.x, n, 0.0);  // b = 0: u = 0 whatever the start
    scatter_perm<double, double>(s, v.x, L0.perm, R.u[0], n);
  } else {
    scatter_block(s, K, v.x, L0.perm, R.u, n);
    for (int q = 0; q < R.ncols; ++q)
      if (R.bnorm[q] == 0.0 && R.warm) fill<double>(s, R.u[q], n, 0.0);
  }
  MG_HIP(hipEventRecord(R.e1, s));
  if (K == 1) {
    sell_spmv<double>(s, L0.S, v.x, v.q, SPMV_RESID, v.b);
    dot_to(c, v.q, v.q, n, scal + 7);
  } else {
    sell_spmv_block<double>(s, L0.S, K, v.x, v.q, SPMV_RESID, v.b);
    dot_block_to(c, K, v.q, v.q, n, scal + 7 * K);
  }
  scal_to_host(s, scal, c.h_scal_dev, 8 * K);
  R.phase = CgRun::END;
}

// launches the next iteration, refreshing the device-side active flags of a
// block when the host's set of iterating columns has changed
static void cg_next(CgRun &R, bool mask_changed) {
  if (R.K > 1 && mask_changed) cg_active_block(R.c->stream, R.K, R.mask, R.c->scal.p);
  cg_iteration(*R.c, R.K);
  R.phase = CgRun::ITERATE;
}

// the host side of a run once its enqueued work has completed (the scalars
// are in pinned memory): reads them, decides, and enqueues what comes next.
// Returns false when the run is over (its statistics written).
static bool cg_advance(CgRun &R) {
  Ctx &c = *R.c;
  const int K = R.K;
  const double *h = c.h_scal;
  switch (R.phase) {
    case CgRun::START: {
      for (int q = 0; q < K; ++q) {
        // a non-finite b (or warm-start residual) is a breakdown before the
        // first iteration, not a zero right-hand side
        if (!std::isfinite(h[7 * K + q]) || (R.warm && !std::isfinite(h[3 * K + q]))) {
          R.broken = q;
          break;
        }
        R.bnorm[q] = std::sqrt(h[7 * K + q]);
        R.rel[q] = R.bnorm[q] > 0 ? (R.warm ? std::sqrt(h[3 * K + q]) / R.bnorm[q] : 1.0) : 0.0;
        R.hist[q].push_back(R.rel[q]);
        R.conv[q] = R.bnorm[q] == 0.0 || R.rel[q] <= R.rtol;
        if (!R.conv[q]) R.mask |= 1u << q;
      }
      if (R.broken >= 0 || !R.mask || R.maxit <= 0) {
        cg_end(R);
        return true;
      }
      // p = 0 and rho = 1: the first iteration's beta p vanishes, p = z
      const CgBufs v = cg_bufs(c, K);
      fill<double>(c.stream, v.p, c.lv[0].nfree * K, 0.0);
      fill<double>(c.stream, c.scal.p, K, 1.0);
      cg_next(R, true);
      return true;
    }
    case CgRun::ITERATE: {
      ++R.it;
      const unsigned before = R.mask;
      for (int q = 0; q < K; ++q) {
        if (!((R.mask >> q) & 1u)) continue;
        const double rr = h[3 * K + q];
        if (h[6 * K + q] != 0.0 || !std::isfinite(rr)) {
          R.broken = q;
          break;
        }
        R.rel[q] = std::sqrt(rr) / R.bnorm[q];
        R.hist[q].push_back(R.rel[q]);
        R.iters[q] = R.it;
        if (R.rel[q] <= R.rtol) {
          R.conv[q] = true;
          R.mask &= ~(1u << q);
        }
      }
      if (R.broken >= 0 || !R.mask || R.it >= R.maxit) cg_end(R);
      else cg_next(R, R.mask != before);
      return true;
    }
    case CgRun::END: {
      float tms = 0;
      MG_HIP(hipEventElapsedTime(&tms, R.e0, R.e1));
      if (R.st) {
        for (int q = 0; q < R.ncols; ++q) {
          mg_solve_stats &o = R.st[q];
          std::memset(&o, 0, sizeof(o));
          o.iterations = R.iters[q];
          o.converged = R.conv[q] ? 1 : 0;
          o.rel_residual = R.rel[q];
          o.true_rel_residual = R.bnorm[q] > 0 ? std::sqrt(h[7 * K + q]) / R.bnorm[q] : 0.0;
          o.solve_ms = tms;
          o.n_history = (int32_t)std::min<size_t>(R.hist[q].size(), MG_MAX_HISTORY);
          for (int k = 0; k < o.n_history; ++k) o.history[k] = R.hist[q][k];
        }
      }
      R.phase = CgRun::DONE;
      if (R.broken >= 0) {
        if (K == 1) fail(MG_ERR_BREAKDOWN, "CG breakdown at iteration %d (p.Ap <= 0 or a non-finite value)", R.it);
        fail(MG_ERR_BREAKDOWN, "CG breakdown in column %d at iteration %d (p.Ap <= 0 or a non-finite value)",
             R.broken, R.it);
      }
      return false;
    }
    default:
      return false;
  }
}

// The right-hand sides of one context cut into runs: groups of 4 columns; a
// remainder of 3 is padded with a zero column, 2 runs as a block of two and
// 1 as a single vector.
struct CgPlan {
  int first, K, ncols;
};
static std::vector<CgPlan> cg_plan(int nrhs) {
  std::vector<CgPlan> out;
  for (int i = 0; i < nrhs;) {
    const int left = nrhs - i;
    const int K = left == 1 ? 1 : left == 2 ? 2 : 4, ncols = std::min(left, K);
    out.push_back({i, K, ncols});
    i += ncols;
  }
  return out;
}


}  // namespace mg

using namespace mg;

static thread_local std::string g_error;

// Staging vectors of mg_vcycle_noalloc: one static device array per GPU,
// created with the code object and held until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: host code
// uses only the device address that hipGetSymbolAddress returns for the
// current device (resolve_noalloc, called by mg_setup), never the name.
static __device__ __align__(256) double scratch[MG_NOALLOC_SCRATCH_BYTES / sizeof(double)];

static std::mutex g_noalloc_mu;
static std::unordered_map<int, double *> g_noalloc_ptr;  // device -> address of its array

// address of `scratch` on `device`, which must be the current device; looked
// up once per device
static double *resolve_noalloc(int device) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(device);
  if (it != g_noalloc_ptr.end()) return it->second;
  double *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&ptr), HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    fail(MG_ERR_HIP, "hipGetSymbolAddress of the static staging array failed on device %d: %s", device,
         hipGetErrorString(e));
  }
  g_noalloc_ptr.emplace(device, ptr);
  return ptr;
}

#define MG_API_BEGIN try {
#define MG_API_END(ctxp)                                        \
  }                                                             \
  catch (const Error &e) {                                      \
    if (ctxp) (ctxp)->err = e.msg; else g_error = e.msg;        \
    return e.code;                                              \
  }                                                             \
  catch (const std::exception &e) {                             \
    if (ctxp) (ctxp)->err = e.what(); else g_error = e.what();  \
    return MG_ERR_HIP;                                          \
  }

struct mg_ctx {
  Ctx impl;
  // per level: slices of the operator's SELL layout in the eight/sixteen-window,
  // the 32-bit and the sixteen-window column forms (counted once at setup, for
  // mg_get_level_info)
  std::vector<std::array<int64_t, 3>> slice_forms;
};

template <class T>
static void copy_out(hipStream_t s, const T *d, size_t n, void *out) {
  if (n == 0) return;
  if (!d) fail(MG_ERR_ARG, "array not available on this level");
  MG_HIP(hipMemcpyAsync(out, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
}

// The vectors of one context's nrhs systems: none NULL, no solution aliasing
// another vector.
static void check_vectors(int nrhs, const double *const *b, double *const *u) {
  for (int i = 0; i < nrhs; ++i) {
    if (!b[i] || !u[i]) fail(MG_ERR_ARG, "NULL vector of right-hand side %d", i);
    for (int j = 0; j < nrhs; ++j)
      if (u[i] == b[j] || (j < i && u[i] == u[j])) fail(MG_ERR_ARG, "solution %d aliases another vector", i);
  }
}

// Solves the nrhs systems of each of n_inst distinct contexts (b, u and st
// indexed i * nrhs + r) from one host thread.  Each context works through
// its runs (cg_plan) one after another; a context whose enqueued work has
// completed is advanced at once (polled with hipStreamQuery when there are
// several), so that the contexts' iterations overlap on the GPU with no
// common barrier.  status[i]: MG_OK, MG_NOT_CONVERGED, or context i's first
// error (its message in the context).
static void cg_drive(mg_ctx *const *cs, int n_inst, int nrhs, const double *const *b, double *const *u,
                     double rtol, int maxit, mg_solve_stats *st, std::vector<mg_status> &status) {
  const std::vector<CgPlan> plan = cg_plan(nrhs);
  struct Inst {
    size_t next = 0;  // next run of the plan
    std::unique_ptr<CgRun> run;
    bool busy = false;
  };
  std::vector<Inst> in(n_inst);
  status.assign(n_inst, MG_OK);
  auto start_next = [&](int i) {
    Inst &I = in[i];
    I.run.reset();
    I.busy = false;
    if (I.next >= plan.size()) return;
    const CgPlan &g = plan[I.next++];
    I.run = std::make_unique<CgRun>();
    CgRun &R = *I.run;
    R.c = &cs[i]->impl;
    R.K = g.K;
    R.ncols = g.ncols;
    R.rtol = rtol;
    R.maxit = maxit;
    const int64_t k = (int64_t)i * nrhs + g.first;
    for (int q = 0; q < g.ncols; ++q) {
      R.b[q] = b[k + q];
      R.u[q] = u[k + q];
    }
    R.st = st ? st + k : nullptr;
    I.busy = true;
    cg_begin(R);
  };
  // runs f for context i; an error ends the context's work
  auto guarded = [&](int i, const auto &f) {
    try {
      f();
      return;
    } catch (const Error &e) {
      status[i] = e.code;
      cs[i]->impl.err = e.msg;
    } catch (const std::exception &e) {
      status[i] = MG_ERR_HIP;
      cs[i]->impl.err = e.what();
    }
    in[i].busy = false;
    in[i].run.reset();
  };
  for (int i = 0; i < n_inst; ++i)
    guarded(i, [&] {
      check_vectors(nrhs, b + (int64_t)i * nrhs, u + (int64_t)i * nrhs);
      start_next(i);
    });
  for (;;) {
    bool busy = false, progressed = false;
    for (int i = 0; i < n_inst; ++i) {
      Inst &I = in[i];
      if (!I.busy) continue;
      busy = true;
      hipStream_t s = I.run->c->stream;
      hipError_t q = hipSuccess;
      if (n_inst == 1) q = hipStreamSynchronize(s);
      else if ((q = hipStreamQuery(s)) == hipErrorNotReady) continue;
      progressed = true;
      guarded(i, [&] {
        if (q != hipSuccess) fail(MG_ERR_HIP, "waiting for the stream: %s", hipGetErrorString(q));
        CgRun &R = *I.run;
        if (cg_advance(R)) return;
        for (int c = 0; c < R.ncols; ++c)
          if (!R.conv[c]) status[i] = MG_NOT_CONVERGED;
        start_next(i);
      });
    }
    if (!busy) break;
    if (!progressed) std::this_thread::yield();
  }
  // a context that failed may still have work in flight
  for (int i = 0; i < n_inst; ++i)
    if (status[i] < 0) (void)hipStreamSynchronize(cs[i]->impl.stream);
}


extern "C" {

void mg_default_options(mg_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->degree = 1;
  o->precision = MG_FP64;
  o->nu = 2;
  o->cheb_degree = 2;
  o->cheb_lo_frac = 0.1;
  o->local_correction = 1;
  o->adjusted_eig = 1;
  o->patch_policy = MG_PATCH_MERGE;
  o->eig_tol = 1e-8;
  o->eig_maxit = 200;
  o->use_graph = 0;
  o->sell_sigma = 0;
  o->sell_unroll = 0;
  o->sell_mask = -1;
  o->sell_rpl = 0;
  o->patch_fused = 1;
  o->use_initial_guess = 0;
  o->sell_colform = 0;
  o->patch_factor_f32 = 1;
  o->patch_refine = 0;
  o->patch_inherit_levels = 0;
  o->patch_chunk = 0;
  o->patch_small_bound = 0;
  o->coarse_solver = 0;
  o->coarse_nd_leaf = 1024;
  o->sell_layout_levels = 0;
  o->sell_layout = nullptr;
  o->global_smoother = MG_SMOOTHER_CHEBYSHEV;
  o->problem = MG_PROBLEM_POISSON;
  o->young = 6.9e10;
  o->poisson_ratio = 0.33;
  o->stream = nullptr;
}

const char *mg_global_error(void) { return g_error.c_str(); }

const char *mg_last_error(const mg_ctx *c) { return c ? c->impl.err.c_str() : g_error.c_str(); }

void mg_destroy(mg_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->impl.stream);
  delete c;
}

static void validate_mesh(const mg_mesh &m, int dim, int l) {
  if (m.dim != dim) fail(MG_ERR_ARG, "level %d: dimension %d differs from level 0 (%d)", l, m.dim, dim);
  if (!m.coords || !m.cells || !m.dirichlet_vertex) fail(MG_ERR_ARG, "level %d: NULL mesh array", l);
  if (m.n_vertices < dim + 1 || m.n_cells < 1) fail(MG_ERR_ARG, "level %d: empty mesh", l);
  if (m.n_vertices > 2000000000LL || m.n_cells > 200000000LL) fail(MG_ERR_LIMIT, "level %d: mesh too large", l);
  int64_t nidx = m.n_cells * (dim + 1);
  for (int64_t i = 0; i < nidx; ++i)
    if (m.cells[i] < 0 || m.cells[i] >= m.n_vertices)
      fail(MG_ERR_MESH, "level %d: cell %lld has vertex index %d out of range", l, (long long)(i / (dim + 1)),
           m.cells[i]);
  for (int64_t i = 0; i < m.n_vertices * dim; ++i)
    if (!std::isfinite(m.coords[i])) fail(MG_ERR_MESH, "level %d: non-finite coordinate", l);
}

mg_status mg_setup(const mg_mesh *levels, int32_t n_levels, double quality_threshold, int32_t patch_layers,
                   const mg_options *opt, mg_ctx **out) {
  if (out) *out = nullptr;
  mg_ctx *h = nullptr;
  try {
    if (!levels || n_levels < 1 || !out) fail(MG_ERR_ARG, "levels, n_levels >= 1 and out are required");
    if (patch_layers < 0 || !(quality_threshold >= 0)) fail(MG_ERR_ARG, "bad quality threshold or patch layers");
    mg_options o;
    if (opt) o = *opt; else mg_default_options(&o);
    int dim = levels[0].dim;
    if (dim != 2 && dim != 3) fail(MG_ERR_ARG, "dim must be 2 or 3");
    if (o.degree < 1 || o.degree > 3 || (o.degree == 3 && dim != 2))
      fail(MG_ERR_ARG, "degree must be 1 or 2 (3 on triangles)");
    if (o.precision != MG_FP64 && o.precision != MG_MIXED) fail(MG_ERR_ARG, "bad precision");
    if (o.nu < 0 || o.cheb_degree < 1 || !(o.cheb_lo_frac >= 0 && o.cheb_lo_frac < 1) || o.eig_maxit < 1)
      fail(MG_ERR_ARG, "bad smoother options");
    if (o.problem != MG_PROBLEM_POISSON && o.problem != MG_PROBLEM_ELASTICITY)
      fail(MG_ERR_ARG, "problem must be MG_PROBLEM_POISSON or MG_PROBLEM_ELASTICITY");
    if (o.problem == MG_PROBLEM_ELASTICITY && !(o.young > 0 && o.poisson_ratio >= 0 && o.poisson_ratio < 0.5))
      fail(MG_ERR_ARG, "elasticity needs young > 0 and 0 <= poisson_ratio < 0.5");
    if (o.global_smoother != MG_SMOOTHER_CHEBYSHEV && o.global_smoother != MG_SMOOTHER_SGS)
      fail(MG_ERR_ARG, "global_smoother must be MG_SMOOTHER_CHEBYSHEV or MG_SMOOTHER_SGS");
    if (o.sell_sigma < 0 || (o.sell_sigma > 1 && o.sell_sigma % SELL_C))
      fail(MG_ERR_ARG, "sell_sigma must be 0, 1 or a multiple of 64");
    if (o.sell_unroll != 0 && o.sell_unroll != 4 && o.sell_unroll != 8)
      fail(MG_ERR_ARG, "sell_unroll must be 0, 4 or 8");
    if (o.sell_mask < -1 || o.sell_mask > 1) fail(MG_ERR_ARG, "sell_mask must be -1, 0 or 1");
    if (o.sell_rpl != 0 && o.sell_rpl != 1 && o.sell_rpl != 2 && o.sell_rpl != 4 && o.sell_rpl != 8 &&
        o.sell_rpl != 16 && o.sell_rpl != 32)
      fail(MG_ERR_ARG, "sell_rpl must be 0, 1, 2, 4, 8, 16 or 32");
    if (o.patch_fused != 0 && o.patch_fused != 1) fail(MG_ERR_ARG, "patch_fused must be 0 or 1");
    if (o.use_initial_guess != 0 && o.use_initial_guess != 1) fail(MG_ERR_ARG, "use_initial_guess must be 0 or 1");
    if (o.sell_colform < 0 || o.sell_colform > 3) fail(MG_ERR_ARG, "sell_colform must be 0, 1, 2 or 3");
    if (o.patch_factor_f32 != 0 && o.patch_factor_f32 != 1) fail(MG_ERR_ARG, "patch_factor_f32 must be 0 or 1");
    if (o.patch_refine != 0 && o.patch_refine != 1) fail(MG_ERR_ARG, "patch_refine must be 0 or 1");
    if (o.patch_inherit_levels < 0) fail(MG_ERR_ARG, "patch_inherit_levels must be >= 0");
    if (o.patch_chunk != 0 && o.patch_chunk != 8 && o.patch_chunk != 16 && o.patch_chunk != 32)
      fail(MG_ERR_ARG, "patch_chunk must be 0, 8, 16 or 32");
    if (o.coarse_solver < 0 || o.coarse_solver > 2) fail(MG_ERR_ARG, "coarse_solver must be 0, 1 or 2");
    if (o.coarse_nd_leaf < 32 || o.coarse_nd_leaf > 16384)
      fail(MG_ERR_ARG, "coarse_nd_leaf must lie in 32..16384");
    if (o.patch_small_bound != 0 && o.patch_small_bound != -1 && o.patch_small_bound != 128 &&
        o.patch_small_bound != 256 && o.patch_small_bound != 384)
      fail(MG_ERR_ARG, "patch_small_bound must be 0, -1, 128, 256 or 384");
    if (o.patch_rows_rpl != 0 && o.patch_rows_rpl != 1 && o.patch_rows_rpl != 2 && o.patch_rows_rpl != 4 &&
        o.patch_rows_rpl != 8)
      fail(MG_ERR_ARG, "patch_rows_rpl must be 0, 1, 2, 4 or 8");
    if (o.patch_refine && o.patch_rows_rpl > 1) fail(MG_ERR_ARG, "patch_refine needs patch_rows_rpl 0 or 1");
    if (o.sell_layout_levels < 0 || (o.sell_layout_levels > 0 && !o.sell_layout))
      fail(MG_ERR_ARG, "sell_layout must hold 4 values for each of sell_layout_levels levels");
    for (int l = 0; l < o.sell_layout_levels; ++l) {
      const int32_t *q = o.sell_layout + 4 * l;
      if (q[0] < 0 || (q[0] > 1 && q[0] % SELL_C) || (q[1] != 0 && q[1] != 4 && q[1] != 8) || q[2] < -1 ||
          q[2] > 1 || (q[3] != 0 && q[3] != 1 && q[3] != 2 && q[3] != 4 && q[3] != 8 && q[3] != 16 && q[3] != 32))
        fail(MG_ERR_ARG, "sell_layout of level %d: (sigma, unroll, mask, rpl) must each be a value the "
                         "options sell_sigma, sell_unroll, sell_mask, sell_rpl accept", l);
    }
    for (int l = 0; l < n_levels; ++l) validate_mesh(levels[l], dim, l);
    h = new mg_ctx();
    Ctx &c = h->impl;
    c.opt = o;
    if (o.sell_layout_levels > 0) c.layout.assign(o.sell_layout, o.sell_layout + 4 * o.sell_layout_levels);
    c.opt.sell_layout = nullptr;  // the caller's array is not kept
    c.opt.sell_layout_levels = 0;
    c.tau = quality_threshold;
    c.layers = patch_layers;
    if (o.stream) {
      c.stream = (hipStream_t)o.stream;
    } else {
      MG_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
      c.own_stream = true;
    }
    MG_HIP(hipGetDevice(&c.device));
    c.noalloc = resolve_noalloc(c.device);
    c.lv.resize(n_levels);
    const bool mixed = o.precision == MG_MIXED;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
    // MG_SETUP_LOG=1 reports every finished setup phase on stderr
    const char *env = std::getenv("MG_SETUP_LOG");
    const bool verbose = env && env[0] == '1';
    auto t_start = now();
    auto phase = [&](const char *what, int l) {
      if (verbose) {
        std::fprintf(stderr, "[mg setup] %8.1f ms  level %d: %s\n", ms(t_start, now()), l, what);
        std::fflush(stderr);
      }
    };
    for (int l = 0; l < n_levels; ++l) {
      auto t0 = now();
      Level &L = c.lv[l];
      L.degree = o.degree;
      L.coarsest = (l == n_levels - 1);
      build_dofmap(c, L, levels[l]);
      if (o.problem == MG_PROBLEM_ELASTICITY) {  // dim unknowns per DOF node
        L.ncomp = dim;
        L.nfree = L.nfree_s * dim;
      }
      compute_quality(c, L);
      if (!L.coarsest) build_patches(c, L, levels[l]);
      if (l == 0) assemble_fine(c, L);
      L.setup_ms += ms(t0, now());
      phase(l == 0 ? "DOF map, quality, patches, assembly" : "DOF map, quality, patches", l);
    }
    std::vector<std::vector<int32_t>> seeds;  // patches inherited through P
    if (o.local_correction && o.patch_inherit_levels > 0) patch_seeds(c, c.lv[0], seeds);
    for (int l = 0; l + 1 < n_levels; ++l) {
      auto t0 = now();
      build_prolongation(c, c.lv[l], c.lv[l + 1], levels[l + 1]);
      galerkin_product(c, c.lv[l], c.lv[l + 1]);
      if (l < o.patch_inherit_levels && l + 2 < n_levels && !seeds.empty())
        inherit_patches(c, c.lv[l], c.lv[l + 1], seeds);
      c.lv[l].setup_ms += ms(t0, now());
      phase("prolongation and Galerkin product", l);
    }
    for (int l = 0; l < n_levels; ++l) {
      auto t0 = now();
      Level &L = c.lv[l];
      {
        // a fixed per-level layout stands in for the global options while
        // this level's operator layout is chosen
        const mg_options keep = c.opt;
        int sigma = c.opt.sell_sigma;
        if (4 * l + 3 < (int)c.layout.size()) {
          const int32_t *q = &c.layout[4 * l];
          if (q[0]) sigma = q[0];
          if (q[1]) c.opt.sell_unroll = q[1];
          if (q[2] >= 0) c.opt.sell_mask = q[2];
          if (q[3]) c.opt.sell_rpl = q[3];
        }
        solve_order(c, L, L.coarsest ? 1 : sigma, mixed && !L.coarsest);
        c.opt = keep;
      }
      permute_patches(c, L);
      if (!L.coarsest) {
        build_patch_rows(c, L, mixed);
        if (o.patch_refine) build_patch_refine(c, L);
        build_patch_neighbours(c, L, mixed);
      }
      if (!L.coarsest && o.global_smoother == MG_SMOOTHER_SGS) build_sgs(c, L, mixed);
      L.setup_ms += ms(t0, now());
      phase("solve order", l);
    }
    for (int l = 0; l < n_levels; ++l) {
      auto t0 = now();
      Level &L = c.lv[l];
      if (!L.coarsest) {
        build_transfer_sell(c, L, c.lv[l + 1], mixed);
        L.Pc = Csr();
        L.Rc = Csr();
        factor_patches(c, L);
        phase("patch factorisation", l);
        if (o.global_smoother == MG_SMOOTHER_CHEBYSHEV) {  // Gauss-Seidel needs no spectral bound
          estimate_eigenvalues(c, L);
          phase("eigenvalue estimates", l);
        }
      } else {
        factor_coarsest(c, L);
        phase("coarsest factorisation", l);
      }
      ensure_work(c, L);
      tune_patches(c, L);
      L.setup_ms += ms(t0, now());
    }
    int64_t n0 = c.lv[0].nfree;
    c.r.alloc(n0);
    c.z.alloc(n0);
    c.p.alloc(n0);
    c.q.alloc(n0);
    c.ax.alloc(n0);
    c.bpos.alloc(n0);
    c.xpos.alloc(n0);
    int64_t pb = std::max<int64_t>(1024, spmv_dot_blocks(c.lv[0].S));
    c.partial.alloc(pb);
    c.scal.alloc(16 * MG_BLOCK_MAX);
    MG_HIP(hipHostMalloc((void **)&c.h_scal, 16 * MG_BLOCK_MAX * sizeof(double), hipHostMallocDefault));
    MG_HIP(hipHostGetDevicePointer((void **)&c.h_scal_dev, c.h_scal, 0));
    // column form of each slice: cbase[2 s] >= 0 two windows, -1 32-bit,
    // below -1 eight or sixteen windows
    for (const Level &L : c.lv) {
      std::array<int64_t, 3> f = {0, 0, 0};
      if (L.S.nslices > 0) {
        std::vector<int32_t> cb(2 * L.S.nslices);
        MG_HIP(hipMemcpyAsync(cb.data(), L.S.cbase.p, cb.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                              c.stream));
        MG_HIP(hipStreamSynchronize(c.stream));
        for (int64_t q = 0; q < L.S.nslices; ++q) {
          f[0] += cb[2 * q] < -1;
          f[1] += cb[2 * q] == -1;
          f[2] += cb[2 * q] == -3;
        }
      }
      h->slice_forms.push_back(f);
    }
    MG_HIP(hipStreamSynchronize(c.stream));
    *out = h;
    return MG_OK;
  } catch (const Error &e) {
    g_error = e.msg;
    delete h;
    return e.code;
  } catch (const std::exception &e) {
    g_error = e.what();
    delete h;
    return MG_ERR_HIP;
  }
}

mg_status mg_smooth(mg_ctx *h, int32_t level, const double *b, double *u, int32_t nu) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || !b || !u) fail(MG_ERR_ARG, "NULL argument");
  Ctx &c = h->impl;
  if (level < 0 || level >= (int)c.lv.size() || c.lv[level].coarsest)
    fail(MG_ERR_ARG, "level %d has no smoother", level);
  if (b == u) fail(MG_ERR_ARG, "b must not alias u");
  if (nu < 0) fail(MG_ERR_ARG, "nu must be >= 0");
  Level &L = c.lv[level];
  if (c.opt.precision == MG_MIXED) {
    gather_perm<double, float>(c.stream, b, L.perm, L.w32[W_B], L.nfree);
    gather_perm<double, float>(c.stream, u, L.perm, L.w32[W_U], L.nfree);
    smooth<float>(c, level, L.w32[W_B], L.w32[W_U], nu);
    scatter_perm<float, double>(c.stream, L.w32[W_U], L.perm, u, L.nfree);
  } else {
    gather_perm<double, double>(c.stream, b, L.perm, L.w64[W_B], L.nfree);
    gather_perm<double, double>(c.stream, u, L.perm, L.w64[W_U], L.nfree);
    smooth<double>(c, level, L.w64[W_B], L.w64[W_U], nu);
    scatter_perm<double, double>(c.stream, L.w64[W_U], L.perm, u, L.nfree);
  }
  MG_HIP(hipStreamSynchronize(c.stream));
  return MG_OK;
  MG_API_END(cp)
}

mg_status mg_vcycle(mg_ctx *h, const double *b, double *u) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || !b || !u) fail(MG_ERR_ARG, "NULL argument");
  Ctx &c = h->impl;
  if (b == u) fail(MG_ERR_ARG, "b must not alias u");
  Level &L0 = c.lv[0];
  // V(b, u) = u + B (b - A u): the cycle is affine in its initial guess
  gather_perm<double, double>(c.stream, b, L0.perm, c.bpos, L0.nfree);
  gather_perm<double, double>(c.stream, u, L0.perm, c.xpos, L0.nfree);
  sell_spmv<double>(c.stream, L0.S, c.xpos, c.r, SPMV_RESID, c.bpos);
  precondition(c);
  add64(c.stream, c.xpos, c.z, L0.nfree);
  scatter_perm<double, double>(c.stream, c.xpos, L0.perm, u, L0.nfree);
  MG_HIP(hipStreamSynchronize(c.stream));
  return MG_OK;
  MG_API_END(cp)
}

mg_status mg_vcycle_noalloc(mg_ctx *h, const double *b, double *u) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || !b || !u) fail(MG_ERR_ARG, "NULL argument");
  Ctx &c = h->impl;
  if (b == u) fail(MG_ERR_ARG, "b must not alias u");
  Level &L0 = c.lv[0];
  const int64_t n = L0.nfree;
  if (n > MG_NOALLOC_MAX_UNKNOWNS)
    fail(MG_ERR_LIMIT, "mg_vcycle_noalloc: level 0 has %lld unknowns, its static staging array holds %d",
         (long long)n, MG_NOALLOC_MAX_UNKNOWNS);
  if (!c.noalloc) fail(MG_ERR_HIP, "mg_vcycle_noalloc: no staging array on device %d", c.device);
  // four vectors, each starting on a 512-byte boundary: 4 * stride <= the
  // array's length whenever n <= MG_NOALLOC_MAX_UNKNOWNS
  const int64_t stride = (n + 63) / 64 * 64;
  double *bpos = c.noalloc, *xpos = bpos + stride, *r = xpos + stride, *z = r + stride;
  // no timing events (creating one may allocate) and no graph (it is bound
  // to the context's own buffers): the eager cycle, with the kernels and
  // arguments of mg_vcycle apart from these four addresses
  struct NoTiming {
    Ctx &c;
    bool was;
    ~NoTiming() { c.timing = was; }
  } keep{c, c.timing};
  c.timing = false;
  gather_perm<double, double>(c.stream, b, L0.perm, bpos, n);
  gather_perm<double, double>(c.stream, u, L0.perm, xpos, n);
  sell_spmv<double>(c.stream, L0.S, xpos, r, SPMV_RESID, bpos);
  precondition_eager(c, r, z);
  add64(c.stream, xpos, z, n);
  scatter_perm<double, double>(c.stream, xpos, L0.perm, u, n);
  return MG_OK;
  MG_API_END(cp)
}

mg_status mg_pcg_solve(mg_ctx *h, const double *b, double *u, double rtol, int32_t maxit, mg_solve_stats *st) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || !b || !u) fail(MG_ERR_ARG, "NULL argument");
  if (b == u) fail(MG_ERR_ARG, "b must not alias u");
  if (maxit < 0 || !(rtol >= 0)) fail(MG_ERR_ARG, "bad rtol or maxit");
  if (st) std::memset(st, 0, sizeof(*st));
  std::vector<mg_status> status;
  cg_drive(&h, 1, 1, &b, &u, rtol, maxit, st, status);
  return status[0];
  MG_API_END(cp)
}

mg_status mg_pcg_solve_multi(mg_ctx *h, int32_t nrhs, const double *const *b, double *const *u, double rtol,
                             int32_t maxit, mg_solve_stats *st) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || nrhs < 0 || (nrhs > 0 && (!b || !u))) fail(MG_ERR_ARG, "NULL argument or negative count");
  if (maxit < 0 || !(rtol >= 0)) fail(MG_ERR_ARG, "bad rtol or maxit");
  if (st && nrhs > 0) std::memset(st, 0, sizeof(*st) * nrhs);
  if (nrhs == 0) return MG_OK;
  std::vector<mg_status> status;
  cg_drive(&h, 1, nrhs, b, u, rtol, maxit, st, status);
  return status[0];
  MG_API_END(cp)
}

mg_status mg_vcycle_solve(mg_ctx *h, const double *b, double *u, double rtol, int32_t maxit, mg_solve_stats *st) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || !b || !u) fail(MG_ERR_ARG, "NULL argument");
  Ctx &c = h->impl;
  if (b == u) fail(MG_ERR_ARG, "b must not alias u");
  if (maxit < 0 || !(rtol >= 0)) fail(MG_ERR_ARG, "bad rtol or maxit");
  Level &L0 = c.lv[0];
  const int64_t n = L0.nfree;
  hipStream_t s = c.stream;
  if (st) std::memset(st, 0, sizeof(*st));
  hipEvent_t e0, e1;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } guard{e0, e1};
  MG_HIP(hipEventRecord(e0, s));
  double *scal = c.scal.p;
  double *x = c.xpos.p;
  const bool warm = c.opt.use_initial_guess != 0;
  gather_perm<double, double>(s, b, L0.perm, c.bpos, n);
  if (warm) {
    gather_perm<double, double>(s, u, L0.perm, x, n);
  } else {
    fill<double>(s, x, n, 0.0);
    copy64(s, c.bpos, c.r, n);
  }
  dot_to(c, c.bpos, c.bpos, n, scal + 7);
  const double bnorm = std::sqrt(read_scalar(c, scal + 7));
  if (!std::isfinite(bnorm)) fail(MG_ERR_BREAKDOWN, "the right-hand side holds a non-finite value");
  double rel = bnorm > 0 ? 1.0 : 0.0;
  if (bnorm == 0.0) {
    fill<double>(s, x, n, 0.0);  // b = 0: u = 0 whatever the start
  } else if (warm) {
    sell_spmv<double>(s, L0.S, x, c.r, SPMV_RESID, c.bpos);
    dot_to(c, c.r, c.r, n, scal + 7);
    rel = std::sqrt(read_scalar(c, scal + 7)) / bnorm;
  }
  std::vector<double> hist{rel};
  int it = 0;
  bool converged = bnorm == 0.0 || rel <= rtol, bad = false;
  // x <- x + B (b - A x): one V-cycle per iteration (the cycle is affine in
  // its initial guess), then the residual of the new iterate
  while (!converged && it < maxit) {
    precondition(c);
    add64(s, x, c.z, n);
    sell_spmv<double>(s, L0.S, x, c.r, SPMV_RESID, c.bpos);
    dot_to(c, c.r, c.r, n, scal + 7);
    const double rr = read_scalar(c, scal + 7);
    ++it;
    if (!std::isfinite(rr)) {
      bad = true;
      break;
    }
    rel = std::sqrt(rr) / bnorm;
    hist.push_back(rel);
    converged = rel <= rtol;
  }
  scatter_perm<double, double>(s, x, L0.perm, u, n);
  MG_HIP(hipEventRecord(e1, s));
  MG_HIP(hipEventSynchronize(e1));
  float tms = 0;
  MG_HIP(hipEventElapsedTime(&tms, e0, e1));
  if (st) {
    st->iterations = it;
    st->converged = converged ? 1 : 0;
    st->rel_residual = rel;
    st->true_rel_residual = rel;  // the recomputed residual is the true one
    st->solve_ms = tms;
    st->n_history = (int32_t)std::min<size_t>(hist.size(), MG_MAX_HISTORY);
    for (int k = 0; k < st->n_history; ++k) st->history[k] = hist[k];
  }
  if (bad) fail(MG_ERR_BREAKDOWN, "non-finite residual after cycle %d", it);
  return converged ? MG_OK : MG_NOT_CONVERGED;
  MG_API_END(cp)
}

mg_status mg_pcg_solve_batch(mg_ctx *const *cs, int32_t n_inst, int32_t nrhs, const double *const *b,
                             double *const *u, double rtol, int32_t maxit, mg_solve_stats *st, double *wall_ms) {
  if (!cs || n_inst < 0 || nrhs < 0 || (n_inst > 0 && nrhs > 0 && (!b || !u))) {
    g_error = "mg_pcg_solve_batch: NULL argument or negative count";
    return MG_ERR_ARG;
  }
  if (maxit < 0 || !(rtol >= 0)) {
    g_error = "mg_pcg_solve_batch: bad rtol or maxit";
    return MG_ERR_ARG;
  }
  for (int i = 0; i < n_inst; ++i) {
    if (!cs[i]) {
      g_error = "mg_pcg_solve_batch: NULL context";
      return MG_ERR_ARG;
    }
    for (int j = 0; j < i; ++j)
      if (cs[j] == cs[i]) {
        g_error = "mg_pcg_solve_batch: a context appears twice";
        return MG_ERR_ARG;
      }
  }
  if (st && n_inst > 0 && nrhs > 0) std::memset(st, 0, sizeof(*st) * (size_t)n_inst * nrhs);
  auto t0 = std::chrono::steady_clock::now();
  std::vector<mg_status> status(n_inst, MG_OK);
  if (n_inst > 0 && nrhs > 0) cg_drive(cs, n_inst, nrhs, b, u, rtol, maxit, st, status);
  if (wall_ms) *wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  mg_status worst = MG_OK;
  for (int i = 0; i < n_inst; ++i) {
    if (status[i] < 0) return status[i];
    if (status[i] == MG_NOT_CONVERGED) worst = MG_NOT_CONVERGED;
  }
  return worst;
}

mg_status mg_rhs_from_nodal(mg_ctx *h, const double *f, double *b) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || !f || !b) fail(MG_ERR_ARG, "NULL argument");
  Ctx &c = h->impl;
  if (c.opt.problem != MG_PROBLEM_POISSON) fail(MG_ERR_ARG, "b = M f_hat is provided for the Poisson problem only");
  if (c.M.nrows == 0) {
    assemble_mass(c, c.lv[0]);
    build_sell(c, c.M, c.Ms, 1, false);
  }
  sell_spmv<double>(c.stream, c.Ms, f, b, SPMV_SET, nullptr);
  MG_HIP(hipStreamSynchronize(c.stream));
  return MG_OK;
  MG_API_END(cp)
}

mg_status mg_get_level_info(const mg_ctx *h, int32_t level, mg_level_info *o) {
  if (!h || !o) return MG_ERR_ARG;
  const Ctx &c = h->impl;
  if (level < 0 || level >= (int)c.lv.size()) return MG_ERR_ARG;
  const Level &L = c.lv[level];
  std::memset(o, 0, sizeof(*o));
  o->n_vertices = L.nv;
  o->n_cells = L.nc;
  o->n_dofs = L.ndofs;
  o->n_free = L.nfree;
  o->nnz = L.A.nnz;
  o->n_flagged = L.nflagged;
  o->n_patches = L.patch.n;
  o->n_colours = L.patch.ncolour;
  o->max_patch = L.patch.maxn;
  o->sum_patch_dofs = L.patch.total;
  o->gamma_min = L.gamma_min;
  o->lambda_max = L.lam;
  o->lambda_adj = L.lam_adj;
  o->cheb_lo = L.lo;
  o->cheb_hi = L.hi;
  o->lanczos_steps = L.lanczos_steps;
  o->lanczos_steps_adj = L.lanczos_steps_adj;
  o->sell_sigma = L.S.sigma;
  o->sell_stored = L.S.stored;
  o->sell_nnz16 = L.S.nnz16;
  o->n_components = L.ncomp;
  o->sell_unroll = L.S.unroll;
  o->sell_mask = L.S.mask;
  o->sell_rpl = L.S.rpl;
  o->patch_fused_colours = 0;
  if (L.patch.small_nb)
    for (uint8_t f : L.patch.colour_fused) o->patch_fused_colours += f;
  o->sell_slices = L.S.nslices;
  if (level < (int)h->slice_forms.size()) {
    o->sell_slices_multiwindow = h->slice_forms[level][0];
    o->sell_slices_32bit = h->slice_forms[level][1];
    o->sell_slices_16window = h->slice_forms[level][2];
    o->patches_f32 = L.patch.n_factor32;
    o->patches_inherited = L.patch.n_inherited;
    o->patch_small_bound = L.patch.small_nb * PATCH_TILE;
    o->patch_chunk = L.coarsest ? L.cpk.chunk : L.patch.inv.chunk;
    o->patch_rows_rpl = L.patch.total > 0 ? L.patch.rows.rpl : 0;
    o->coarse_nd_supernodes = L.cnd.on ? L.cnd.nsup : 0;
    if (L.coarsest)
      o->coarse_solve_bytes = L.cnd.on ? (double)(L.cnd.dinv_bytes + L.cnd.b_bytes) * 2.0
                                       : (double)L.cpk.packed * 8.0;
  }
  o->is_coarsest = L.coarsest ? 1 : 0;
  o->setup_ms = L.setup_ms;
  return MG_OK;
}

mg_status mg_get_array(const mg_ctx *h, int32_t level, int32_t what, void *out) {
  const Ctx *cp = h ? &h->impl : nullptr;
  Ctx *mcp = const_cast<Ctx *>(cp);
  MG_API_BEGIN
  if (!h || !out) fail(MG_ERR_ARG, "NULL argument");
  const Ctx &c = h->impl;
  if (level < 0 || level >= (int)c.lv.size()) fail(MG_ERR_ARG, "bad level");
  const Level &L = c.lv[level];
  hipStream_t s = c.stream;
  switch (what) {
    case MG_ARR_QUALITY: copy_out(s, L.gamma.p, L.nc, out); break;
    case MG_ARR_FLAGS: copy_out(s, L.flags.p, L.nc, out); break;
    case MG_ARR_PATCH_PTR: std::memcpy(out, L.patch.h_ptr.data(), L.patch.h_ptr.size() * 4); break;
    case MG_ARR_PATCH_DOFS: std::memcpy(out, L.patch.h_dofs.data(), L.patch.h_dofs.size() * 4); break;
    case MG_ARR_PATCH_COLOUR: std::memcpy(out, L.patch.h_colour.data(), L.patch.h_colour.size() * 4); break;
    case MG_ARR_LOCATE: copy_out(s, L.locate.p, L.coarsest ? 0 : L.nfree_s, out); break;
    case MG_ARR_FREE_DOFS: copy_out(s, L.free_dofs.p, L.nfree_s, out); break;
    case MG_ARR_DOF_NODES: copy_out(s, L.nodes.p, L.ndofs * L.dim, out); break;
    case MG_ARR_A_ROWPTR: copy_out(s, L.A.rowptr.p, L.nfree + 1, out); break;
    case MG_ARR_A_COLS: copy_out(s, L.A.col.p, L.A.nnz, out); break;
    case MG_ARR_A_VALS: copy_out(s, L.A.val.p, L.A.nnz, out); break;
    case MG_ARR_P_COLS: copy_out(s, L.pcol.p, L.coarsest ? 0 : L.nfree * L.pw, out); break;
    case MG_ARR_P_VALS: copy_out(s, L.pval.p, L.coarsest ? 0 : L.nfree * L.pw, out); break;
    case MG_ARR_CELL_DOFS: copy_out(s, L.cell_dofs.p, L.nc * L.nloc, out); break;
    case MG_ARR_P_WIDTH: *(int32_t *)out = L.pw; break;
    case MG_ARR_SGS_COLOUR:
      if (!L.sgs_colour.p) fail(MG_ERR_ARG, "no Gauss-Seidel colouring on this level");
      copy_out(s, L.sgs_colour.p, L.nfree, out);
      break;
    default: fail(MG_ERR_ARG, "unknown array %d", what);
  }
  return MG_OK;
  MG_API_END(mcp)
}

mg_status mg_enable_kernel_timing(mg_ctx *h, int32_t enable) {
  if (!h) return MG_ERR_ARG;
  Ctx &c = h->impl;
  c.timing = enable != 0;
  c.events_used = 0;
  c.timed_launches.assign(c.lv.size(), 0);
  c.timed_ms.assign(c.lv.size(), 0.0);
  return MG_OK;
}

// folds the recorded event pairs into the per-slot sums
static void collect_times(Ctx &c) {
  MG_HIP(hipStreamSynchronize(c.stream));
  c.timed_launches.resize(c.lv.size(), 0);
  c.timed_ms.resize(c.lv.size(), 0.0);
  for (size_t k = 0; k < c.events_used; ++k) {
    float t = 0;
    MG_HIP(hipEventElapsedTime(&t, c.events[k].first, c.events[k].second));
    c.timed_ms[c.event_slot[k]] += t;
    ++c.timed_launches[c.event_slot[k]];
  }
  c.events_used = 0;
}

mg_status mg_kernel_time(mg_ctx *h, int64_t *launches, double *total_ms) {
  return mg_level_kernel_time(h, 0, launches, total_ms);
}

mg_status mg_level_kernel_time(mg_ctx *h, int32_t level, int64_t *launches, double *total_ms) {
  Ctx *cp = h ? &h->impl : nullptr;
  MG_API_BEGIN
  if (!h || !launches || !total_ms) fail(MG_ERR_ARG, "NULL argument");
  Ctx &c = h->impl;
  if (level < 0 || level >= (int)c.lv.size()) fail(MG_ERR_ARG, "no level %d", level);
  collect_times(c);
  *launches = c.timed_launches[level];
  *total_ms = c.timed_ms[level];
  return MG_OK;
  MG_API_END(cp)
}

mg_status mg_cheb_algorithmic_bytes(const mg_ctx *h, double *bytes) {
  if (!h || !bytes) return MG_ERR_ARG;
  const Level &L = h->impl.lv[0];
  if (L.coarsest) return MG_ERR_ARG;
  // average over the k steps of one Chebyshev polynomial: values and column
  // indices once (2-byte indices in 16-bit slices); x, b, D^-1 read and x'
  // written by every step, the direction d written by all but the last step
  // and read by all but the first
  const int k = h->impl.opt.cheb_degree;
  const double vecs = 4.0 + 2.0 * (k - 1) / k;
  const bool mixed = h->impl.opt.precision == MG_MIXED;
  const double vb = mixed ? 4.0 : 8.0;
  double n16 = (double)L.S.nnz16, n32 = (double)(L.S.nnz - L.S.nnz16), n = (double)L.nfree;
  *bytes = (vb + 2.0) * n16 + (vb + 4.0) * n32 + vb * vecs * n;
  return MG_OK;
}

}  // extern "C"

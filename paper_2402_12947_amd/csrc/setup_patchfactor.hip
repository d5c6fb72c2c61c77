// Batched factorisation of the local-correction patch systems (paper Sec. 4.1:
// the patch matrices A^[d] = I_d^T A I_d are factored once in setup and the
// local solves reuse the factors).
//
// One workgroup (four wavefronts) per patch runs the whole blocked sequence on
// 32 x 32 tiles held in a per-patch scratch matrix:
//   1. right-looking Cholesky A = L L^T: factor the diagonal tile in LDS (and
//      invert it), scale the panel below it by the tile's inverse transpose,
//      subtract the panel's outer product from the trailing lower triangle;
//   2. W = L^-1 by block forward substitution (right-looking);
//   3. A^-1 = W^T W (lower tiles, mirrored).
// Every tile product is a 32 x 32 x 32 product on the matrix cores, each
// wavefront owning one output tile (2 x 2 blocks of 16 x 16), its operands
// loaded straight from memory into the MFMA register layout (all 32 loads of
// a tile in flight at once); an update C - A B loads C into the accumulators
// with the operands and accumulates (-A) B onto it, one round trip to memory.  Tiles of one step are dealt to the four
// wavefronts, which run independently; steps are separated by workgroup
// barriers.  Only the diagonal tile and its inverse live in LDS.  Patches are
// launched largest first so the long ones start early (longest-processing-
// time order).
//
// Two precisions.  FP64 (v_mfma_f64_16x16x4) factors A^[d] as it is.  FP32
// (v_mfma_f32_16x16x4, FP32 accumulate; the mixed-precision cycle) first
// equilibrates symmetrically, S A^[d] S with S = diag(A^[d])^-1/2 (unit
// diagonal, computed in FP64 and rounded once), factors and inverts that in
// FP32 and returns S (S A^[d] S)^-1 S = (A^[d])^-1.  Every pivot of the scaled
// matrix lies in (0, 1]; a pivot below PIVOT_MIN_F32 means the FP32 inverse
// would lose more than about eps_32 / PIVOT_MIN_F32 of its accuracy, and the
// patch is marked for the FP64 path instead (the caller refactors it there).
#include <cmath>
#include <type_traits>

#include "devutil.h"
#include "mfma_tile.h"

namespace mg {

namespace {

constexpr int PT = 32;       // tile edge
constexpr int PLD = PT + 1;  // LDS row stride (bank spread)
// smallest accepted pivot of the equilibrated FP32 factorisation (2^-12)
constexpr float PIVOT_MIN_F32 = 1.0f / 4096.0f;

template <class T>
struct PatchSmem {
  T Ld[PT][PLD];             // diagonal tile (factor, in place)
  T Li[PT][PLD];             // its inverse
};

__device__ inline void tri_rc(int t, int &i, int &j) {
  // t -> (i, j), 0 <= j <= i, t = i (i + 1) / 2 + j
  int ii = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (ii * (ii + 1) / 2 > t) --ii;
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  i = ii;
  j = t - ii * (ii + 1) / 2;
}

}  // namespace

// list[blockIdx.x] = patch (kernel order); M and W: per-patch scratch at soff[k]
// (n_d^2 each, type T); the inverse goes to inv + ioff[patch] (n_d^2,
// row-major, FP64).  FP32 only: sc + ptr[patch] receives the equilibration
// scales (n_d), weak[patch] = 1 marks a patch whose scaled pivots fell below
// PIVOT_MIN_F32 (its inverse is not written).
// Element offsets inside a patch are int32 (n_d <= MAX_PATCH, n_d^2 < 2^31),
// which halves the address registers; the FP32 instantiation is held to 168
// registers, three wavefronts per SIMD (three patches per CU), the most that
// fit without spilling once the updated tile is loaded with the operands.
template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(std::is_same<T, float>::value ? 3 : 1)))
void k_patch_factor_mfma(const int64_t *rp, const int32_t *col, const double *val, const int32_t *list,
                         const int32_t *ptr, const int32_t *dofs, const int64_t *soff, T *scratch,
                         const int64_t *ioff, double *inv, int *bad, double *sc, int *weak) {
  using acc_t = typename MfmaAcc<T>::type;
  constexpr bool F32 = std::is_same<T, float>::value;
  __shared__ PatchSmem<T> sm;
  const int p = list[blockIdx.x];
  const int n = ptr[p + 1] - ptr[p];
  const int32_t *Bd = dofs + ptr[p];
  T *M = scratch + soff[blockIdx.x];
  T *W = M + (int64_t)n * n;
  double *X = inv + ioff[p];
  double *S = F32 ? sc + ptr[p] : nullptr;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nb = (n + PT - 1) / PT;

  // M = A[B_d, B_d] (FP32: S A[B_d, B_d] S), W = 0
  for (int64_t t = tid; t < (int64_t)n * n; t += 256) {
    M[t] = (T)0;
    W[t] = (T)0;
  }
  if (F32) {
    for (int i = tid; i < n; i += 256) {
      const int32_t r = Bd[i];
      double d = 0.0;
      for (int64_t k = rp[r]; k < rp[r + 1]; ++k)
        if (col[k] == r) d = val[k];
      S[i] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;  // d <= 0 fails at the first pivot
    }
  }
  __syncthreads();
  for (int i = wave; i < n; i += 4) {
    int32_t r = Bd[i];
    for (int64_t k = rp[r] + lane; k < rp[r + 1]; k += 64) {
      int32_t c = col[k];
      int lo = 0, hi = n;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (Bd[mid] < c) lo = mid + 1; else hi = mid;
      }
      if (lo < n && Bd[lo] == c) M[(int64_t)i * n + lo] = F32 ? (T)(S[i] * val[k] * S[lo]) : (T)val[k];
    }
  }
  __syncthreads();

  // 1. Cholesky
  for (int kb = 0; kb < nb; ++kb) {
    const int o = kb * PT, m = min(PT, n - o);
    for (int t = tid; t < PT * PT; t += 256) {
      int i = t / PT, j = t % PT;
      sm.Ld[i][j] = (i < m && j < m) ? M[(int64_t)(o + i) * n + o + j] : (T)(i == j ? 1 : 0);
    }
    for (int k = 0; k < m; ++k) {
      __syncthreads();
      T piv = sm.Ld[k][k];
      if (F32 ? !(piv >= (T)PIVOT_MIN_F32) : !(piv > (T)0)) {
        if (tid == 0) {
          if (F32) weak[p] = 1;  // refactored in FP64, which decides SPD
          else atomicMin(bad, p);
        }
        return;  // uniform: every thread read the same pivot
      }
      T d = sqrt(piv);
      __syncthreads();
      if (tid == 0) sm.Ld[k][k] = d;
      for (int i = k + 1 + tid; i < m; i += 256) sm.Ld[i][k] /= d;
      __syncthreads();
      for (int t = tid; t < PT * PT; t += 256) {
        int i = t / PT, j = t % PT;
        if (j > k && i >= j && i < m) sm.Ld[i][j] -= sm.Ld[i][k] * sm.Ld[j][k];
      }
    }
    __syncthreads();
    // Li = Ld^-1 (lower), one thread per column
    if (tid < PT) {
      int c = tid;
      for (int r = 0; r < PT; ++r) {
        if (r < c) {
          sm.Li[r][c] = (T)0;
          continue;
        }
        T acc = (T)(r == c ? 1 : 0);
        for (int k = c; k < r; ++k) acc -= sm.Ld[r][k] * sm.Li[k][c];
        sm.Li[r][c] = acc / sm.Ld[r][r];
      }
    }
    __syncthreads();
    for (int t = tid; t < m * m; t += 256) {
      int i = t / m, j = t % m;
      M[(int64_t)(o + i) * n + o + j] = j <= i ? sm.Ld[i][j] : (T)0;
      W[(int64_t)(o + i) * n + o + j] = j <= i ? sm.Li[i][j] : (T)0;
    }
    // panel: M[ib, kb] <- M[ib, kb] Li^T (tiles dealt to the wavefronts; the
    // operands come straight from memory, Li^T from LDS)
    const int rest = nb - kb - 1;
    for (int t = wave; t < rest; t += 4) {
      const int ib = kb + 1 + t;
      T a[16], b[16];
      fetch_ops<true, int32_t>(M, n, ib * PT, o, false, a, lane);
#pragma unroll
      for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) b[blk * 8 + s2] = sm.Li[16 * blk + (lane & 15)][4 * s2 + (lane >> 4)];
      acc_t acc[2][2];
      zero_acc(acc);
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int i, int j, T v) {
        if (ib * PT + i < n && o + j < n) M[(ib * PT + i) * n + o + j] = v;
      });
    }
    __syncthreads();
    // trailing lower triangle: M[ib, jb] -= M[ib, kb] M[jb, kb]^T, the tile
    // loaded into the accumulators with the operands and the product added
    // with -M[ib, kb]
    const int ntr = rest * (rest + 1) / 2;
    for (int t = wave; t < ntr; t += 4) {
      int i = 0, j = 0;
      tri_rc(t, i, j);
      const int ib = kb + 1 + i, jb = kb + 1 + j;
      T a[16], b[16];
      acc_t acc[2][2];
      fetch_ops<true, int32_t>(M, n, ib * PT, o, false, a, lane);
      fetch_ops<false, int32_t>(M, n, jb * PT, o, true, b, lane);
      load_acc<int32_t>(acc, M, n, ib * PT, jb * PT, lane);
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = -a[q];
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int r, int c, T v) {
        int gr = ib * PT + r, gc = jb * PT + c;
        if (gr < n && gc < n) M[gr * n + gc] = v;
      });
    }
    __syncthreads();
  }

  // 2. W = L^-1: block row kb is finished by W[kb, jb] <- Li_kk W[kb, jb]
  // (jb < kb), then pushed into the rows below: W[ib, jb] -= L[ib, kb] W[kb, jb]
  for (int kb = 0; kb < nb; ++kb) {
    for (int jb = wave; jb < kb; jb += 4) {
      T a[16], b[16];
      fetch_ops<true, int32_t>(W, n, kb * PT, kb * PT, false, a, lane);
      fetch_ops<false, int32_t>(W, n, kb * PT, jb * PT, false, b, lane);
      acc_t acc[2][2];
      zero_acc(acc);
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int r, int c, T v) {
        int gr = kb * PT + r, gc = jb * PT + c;
        if (gr < n && gc < n) W[gr * n + gc] = v;
      });
    }
    __syncthreads();
    const int below = nb - kb - 1, nt = below * (kb + 1);
    for (int t = wave; t < nt; t += 4) {
      const int ib = kb + 1 + t / (kb + 1), jb = t % (kb + 1);
      T a[16], b[16];
      acc_t acc[2][2];
      fetch_ops<true, int32_t>(M, n, ib * PT, kb * PT, false, a, lane);
      fetch_ops<false, int32_t>(W, n, kb * PT, jb * PT, false, b, lane);
      load_acc<int32_t>(acc, W, n, ib * PT, jb * PT, lane);
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = -a[q];
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int r, int c, T v) {
        int gr = ib * PT + r, gc = jb * PT + c;
        if (gr < n && gc < n) W[gr * n + gc] = v;
      });
    }
    __syncthreads();
  }

  // 3. X = W^T W: X[ib, jb] = sum_{k >= ib} W[k, ib]^T W[k, jb], jb <= ib, mirrored
  const int nx = nb * (nb + 1) / 2;
  for (int t = wave; t < nx; t += 4) {
    int ib = 0, jb = 0;
    tri_rc(t, ib, jb);
    acc_t acc[2][2];
    zero_acc(acc);
    for (int k = ib; k < nb; ++k) {
      T a[16], b[16];
      fetch_ops<true, int32_t>(W, n, k * PT, ib * PT, true, a, lane);
      fetch_ops<false, int32_t>(W, n, k * PT, jb * PT, false, b, lane);
      mma_ops(acc, a, b);
    }
    for_acc(acc, lane, [&](int r, int c, T v) {
      int gr = ib * PT + r, gc = jb * PT + c;
      if (gr < n && gc < n && (ib != jb || r >= c)) {  // diagonal tiles: lower half, mirrored
        const double x = F32 ? S[gr] * (double)v * S[gc] : (double)v;
        X[gr * n + gc] = x;
        X[gc * n + gr] = x;
      }
    });
  }
}

// Host side: the patches of `order` (each of at most BATCH_MAX DOFs) go
// through k_patch_factor_mfma in launches whose scratch stays under a quarter
// of the free device memory, largest first.  FP32 (f32 = true): sc receives
// the equilibration scales (kernel-order offsets), weak[k] = 1 marks the
// patches left for the FP64 path.
template <class T>
static void factor_list(Ctx &c, Level &L, std::vector<int32_t> order, int *bad, double *sc, int *weak) {
  Patches &P = L.patch;
  hipStream_t s = c.stream;
  size_t free_b = 0, total_b = 0;
  MG_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t SCRATCH_CAP = std::min<int64_t>(
      ((int64_t)48 << 30) / (int64_t)sizeof(T),
      std::max<int64_t>(((int64_t)1 << 30) / (int64_t)sizeof(T), (int64_t)(free_b / 4 / sizeof(T))));
  auto size = [&](int32_t k) { return (int64_t)(P.h_kptr[k + 1] - P.h_kptr[k]); };
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return size(a) > size(b); });
  size_t first = 0;
  while (first < order.size()) {
    std::vector<int32_t> list;
    std::vector<int64_t> soff;
    int64_t acc = 0;
    size_t k = first;
    for (; k < order.size(); ++k) {
      int64_t need = 2 * size(order[k]) * size(order[k]);
      if (!list.empty() && acc + need > SCRATCH_CAP) break;
      list.push_back(order[k]);
      soff.push_back(acc);
      acc += need;
    }
    first = k;
    DBuf<T> scratch;
    scratch.alloc(std::max<int64_t>(acc, 1));
    DBuf<int32_t> dlist;
    DBuf<int64_t> dsoff;
    upload(dlist, list.data(), list.size(), s);
    upload(dsoff, soff.data(), soff.size(), s);
    k_patch_factor_mfma<T><<<(unsigned)list.size(), 256, 0, s>>>(L.A.rowptr, L.A.col, L.A.val, dlist, P.ptr,
                                                                 P.dofs_canon, dsoff, scratch, P.inv_off,
                                                                 P.inv64, bad, sc, weak);
    MG_LAUNCH_CHECK();
    MG_HIP(hipStreamSynchronize(s));
  }
}

void factor_patches_batched(Ctx &c, Level &L, int batch_max, std::vector<int32_t> &rest, int *bad) {
  Patches &P = L.patch;
  hipStream_t s = c.stream;
  std::vector<int32_t> small;
  for (int k = 0; k < P.n; ++k) (P.h_kptr[k + 1] - P.h_kptr[k] <= batch_max ? small : rest).push_back(k);
  P.n_factor32 = 0;
  if (c.opt.precision == MG_MIXED && c.opt.patch_factor_f32 && !small.empty()) {
    // FP32 matrix cores first; the patches they cannot take go to FP64
    DBuf<double> sc;
    sc.alloc(std::max<int64_t>(1, P.total));
    DBuf<int> weak;
    weak.alloc(P.n);
    MG_HIP(hipMemsetAsync(weak.p, 0, P.n * sizeof(int), s));
    factor_list<float>(c, L, small, bad, sc.p, weak.p);
    std::vector<int> hw;
    download(hw, weak.p, (size_t)P.n, s);
    std::vector<int32_t> again;
    for (int32_t k : small)
      if (hw[k]) again.push_back(k);
    P.n_factor32 = (int)(small.size() - again.size());
    small.swap(again);
  }
  factor_list<double>(c, L, small, bad, nullptr, nullptr);
}

}  // namespace mg

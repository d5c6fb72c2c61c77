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
// Every tile product is a 32 x 32 x 32 FP64 product on the matrix cores
// (v_mfma_f64_16x16x4: each wavefront owns one output tile, 2 x 2 blocks of
// 16 x 16), its operands loaded straight from memory into the MFMA register
// layout (all 32 loads of a tile in flight at once).  Tiles of one step are
// dealt to the four wavefronts, which run independently; steps are separated
// by workgroup barriers.  Only the diagonal tile and its inverse live in LDS.  Patches are launched largest first so the
// long ones start early (longest-processing-time order).
#include <cmath>

#include "devutil.h"
#include "mfma_tile.h"

namespace mg {

namespace {

constexpr int PT = 32;       // tile edge
constexpr int PLD = PT + 1;  // LDS row stride (bank spread)

struct PatchSmem {
  double Ld[PT][PLD];        // diagonal tile (factor, in place)
  double Li[PT][PLD];        // its inverse
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
// (n_d^2 each); the inverse goes to inv + ioff[patch] (n_d^2, row-major).
__global__ __launch_bounds__(256) void k_patch_factor_mfma(const int64_t *rp, const int32_t *col,
                                                           const double *val, const int32_t *list,
                                                           const int32_t *ptr, const int32_t *dofs,
                                                           const int64_t *soff, double *scratch,
                                                           const int64_t *ioff, double *inv, int *bad) {
  __shared__ PatchSmem sm;
  const int p = list[blockIdx.x];
  const int n = ptr[p + 1] - ptr[p];
  const int32_t *Bd = dofs + ptr[p];
  double *M = scratch + soff[blockIdx.x];
  double *W = M + (int64_t)n * n;
  double *X = inv + ioff[p];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nb = (n + PT - 1) / PT;

  // M = A[B_d, B_d], W = 0
  for (int64_t t = tid; t < (int64_t)n * n; t += 256) {
    M[t] = 0.0;
    W[t] = 0.0;
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
      if (lo < n && Bd[lo] == c) M[(int64_t)i * n + lo] = val[k];
    }
  }
  __syncthreads();

  // 1. Cholesky
  for (int kb = 0; kb < nb; ++kb) {
    const int o = kb * PT, m = min(PT, n - o);
    for (int t = tid; t < PT * PT; t += 256) {
      int i = t / PT, j = t % PT;
      sm.Ld[i][j] = (i < m && j < m) ? M[(int64_t)(o + i) * n + o + j] : (i == j ? 1.0 : 0.0);
    }
    for (int k = 0; k < m; ++k) {
      __syncthreads();
      double piv = sm.Ld[k][k];
      if (!(piv > 0.0)) {
        if (tid == 0) atomicMin(bad, p);
        return;  // uniform: every thread read the same pivot
      }
      double d = sqrt(piv);
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
          sm.Li[r][c] = 0.0;
          continue;
        }
        double acc = (r == c) ? 1.0 : 0.0;
        for (int k = c; k < r; ++k) acc -= sm.Ld[r][k] * sm.Li[k][c];
        sm.Li[r][c] = acc / sm.Ld[r][r];
      }
    }
    __syncthreads();
    for (int t = tid; t < m * m; t += 256) {
      int i = t / m, j = t % m;
      M[(int64_t)(o + i) * n + o + j] = j <= i ? sm.Ld[i][j] : 0.0;
      W[(int64_t)(o + i) * n + o + j] = j <= i ? sm.Li[i][j] : 0.0;
    }
    // panel: M[ib, kb] <- M[ib, kb] Li^T (tiles dealt to the wavefronts; the
    // operands come straight from memory, Li^T from LDS)
    const int rest = nb - kb - 1;
    for (int t = wave; t < rest; t += 4) {
      const int ib = kb + 1 + t;
      double a[16], b[16];
      fetch_ops<true>(M, n, ib * PT, o, false, a, lane);
#pragma unroll
      for (int blk = 0; blk < 2; ++blk)
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) b[blk * 8 + s2] = sm.Li[16 * blk + (lane & 15)][4 * s2 + (lane >> 4)];
      v4d acc[2][2];
      zero_acc(acc);
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int i, int j, double v) {
        if (ib * PT + i < n && o + j < n) M[(int64_t)(ib * PT + i) * n + o + j] = v;
      });
    }
    __syncthreads();
    // trailing lower triangle: M[ib, jb] -= M[ib, kb] M[jb, kb]^T
    const int ntr = rest * (rest + 1) / 2;
    for (int t = wave; t < ntr; t += 4) {
      int i = 0, j = 0;
      tri_rc(t, i, j);
      const int ib = kb + 1 + i, jb = kb + 1 + j;
      double a[16], b[16];
      fetch_ops<true>(M, n, ib * PT, o, false, a, lane);
      fetch_ops<false>(M, n, jb * PT, o, true, b, lane);
      v4d acc[2][2];
      zero_acc(acc);
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int r, int c, double v) {
        int gr = ib * PT + r, gc = jb * PT + c;
        if (gr < n && gc < n) M[(int64_t)gr * n + gc] -= v;
      });
    }
    __syncthreads();
  }

  // 2. W = L^-1: block row kb is finished by W[kb, jb] <- Li_kk W[kb, jb]
  // (jb < kb), then pushed into the rows below: W[ib, jb] -= L[ib, kb] W[kb, jb]
  for (int kb = 0; kb < nb; ++kb) {
    for (int jb = wave; jb < kb; jb += 4) {
      double a[16], b[16];
      fetch_ops<true>(W, n, kb * PT, kb * PT, false, a, lane);
      fetch_ops<false>(W, n, kb * PT, jb * PT, false, b, lane);
      v4d acc[2][2];
      zero_acc(acc);
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int r, int c, double v) {
        int gr = kb * PT + r, gc = jb * PT + c;
        if (gr < n && gc < n) W[(int64_t)gr * n + gc] = v;
      });
    }
    __syncthreads();
    const int below = nb - kb - 1, nt = below * (kb + 1);
    for (int t = wave; t < nt; t += 4) {
      const int ib = kb + 1 + t / (kb + 1), jb = t % (kb + 1);
      double a[16], b[16];
      fetch_ops<true>(M, n, ib * PT, kb * PT, false, a, lane);
      fetch_ops<false>(W, n, kb * PT, jb * PT, false, b, lane);
      v4d acc[2][2];
      zero_acc(acc);
      mma_ops(acc, a, b);
      for_acc(acc, lane, [&](int r, int c, double v) {
        int gr = ib * PT + r, gc = jb * PT + c;
        if (gr < n && gc < n) W[(int64_t)gr * n + gc] -= v;
      });
    }
    __syncthreads();
  }

  // 3. X = W^T W: X[ib, jb] = sum_{k >= ib} W[k, ib]^T W[k, jb], jb <= ib, mirrored
  const int nx = nb * (nb + 1) / 2;
  for (int t = wave; t < nx; t += 4) {
    int ib = 0, jb = 0;
    tri_rc(t, ib, jb);
    v4d acc[2][2];
    zero_acc(acc);
    for (int k = ib; k < nb; ++k) {
      double a[16], b[16];
      fetch_ops<true>(W, n, k * PT, ib * PT, true, a, lane);
      fetch_ops<false>(W, n, k * PT, jb * PT, false, b, lane);
      mma_ops(acc, a, b);
    }
    for_acc(acc, lane, [&](int r, int c, double v) {
      int gr = ib * PT + r, gc = jb * PT + c;
      if (gr < n && gc < n && (ib != jb || r >= c)) {  // diagonal tiles: lower half, mirrored
        X[(int64_t)gr * n + gc] = v;
        X[(int64_t)gc * n + gr] = v;
      }
    });
  }
}

// Host side: patches of up to BATCH_MAX DOFs go through k_patch_factor_mfma in
// launches whose scratch stays under SCRATCH_CAP doubles; larger ones are
// factored one at a time by the multi-workgroup blocked path.
void factor_patches_batched(Ctx &c, Level &L, int batch_max, std::vector<int32_t> &rest, int *bad) {
  Patches &P = L.patch;
  hipStream_t s = c.stream;
  // scratch per launch: a quarter of the free device memory, 1-48 GiB
  size_t free_b = 0, total_b = 0;
  MG_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t SCRATCH_CAP =
      std::min<int64_t>((int64_t)6 << 30, std::max<int64_t>((int64_t)1 << 27, (int64_t)(free_b / 4 / 8)));
  std::vector<int32_t> order;
  for (int k = 0; k < P.n; ++k) (P.h_kptr[k + 1] - P.h_kptr[k] <= batch_max ? order : rest).push_back(k);
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
    DBuf<double> scratch;
    scratch.alloc(std::max<int64_t>(acc, 1));
    DBuf<int32_t> dlist;
    DBuf<int64_t> dsoff;
    upload(dlist, list.data(), list.size(), s);
    upload(dsoff, soff.data(), soff.size(), s);
    k_patch_factor_mfma<<<(unsigned)list.size(), 256, 0, s>>>(L.A.rowptr, L.A.col, L.A.val, dlist, P.ptr,
                                                              P.dofs_canon, dsoff, scratch, P.inv_off, P.inv64,
                                                              bad);
    MG_LAUNCH_CHECK();
    MG_HIP(hipStreamSynchronize(s));
  }
}

}  // namespace mg

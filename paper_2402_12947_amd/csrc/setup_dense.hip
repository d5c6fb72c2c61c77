// Dense direct solvers of the method: the patch systems A^[d] = I_d^T A I_d of
// the local correction (paper Sec. 4.1, eqs. local_system and local) and the
// coarsest-level system (Sec. 2, direct solver on the coarsest grid).
//
// Each system is factored A = L L^T (Cholesky) and the factor is turned into
// the explicit inverse A^-1 = L^-T L^-1, which the solve phase applies as a
// dense matrix-vector product over packed lower 32 x 32 tiles: that product is
// fully parallel, whereas a triangular substitution is a chain of n dependent
// steps.
//
// * Patches of up to BATCH_MAX DOFs: one workgroup per patch on the matrix
//   cores (setup_patchfactor.hip; FP64, or FP32 after equilibration in the
//   mixed cycle).  Larger patches go one at a time through the blocked path
//   below.  factor_patches packs every inverse in the cycle's precision.
// * Coarsest level (n above 512; smaller ones in one workgroup): blocked
//   right-looking Cholesky with 64 x 64 tiles (diagonal tile factored in LDS,
//   panel triangular solve, trailing symmetric update), then W = L^-1 by a
//   right-looking block solve of L W = I, and A^-1 = W^T W.  The 64 x 64 x 64
//   tile products (trailing update, block solve, W^T W) run on the FP64
//   matrix cores (v_mfma_f64_16x16x4, mfma_tile.h); the diagonal tiles are
//   factored and inverted in LDS on the vector units.
#include <cmath>

#include "devutil.h"
#include "mfma_tile.h"

namespace mg {

// ---------------------------------------------------------------------------
// patches: one workgroup per system
// ---------------------------------------------------------------------------
__device__ inline int find_sorted(const int32_t *a, int n, int32_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return (lo < n && a[lo] == key) ? lo : -1;
}

// Gathers A[B, B] into M (n x n, row-major).  B == nullptr means all rows.
__device__ void gather_block(const int64_t *rp, const int32_t *col, const double *val, const int32_t *B, int n,
                             double *M) {
  for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) M[t] = 0.0;
  __syncthreads();
  int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
  for (int i = wave; i < n; i += nw) {
    int32_t r = B ? B[i] : i;
    for (int64_t k = rp[r] + lane; k < rp[r + 1]; k += 64) {
      int j = B ? find_sorted(B, n, col[k]) : col[k];
      if (j >= 0) M[(int64_t)i * n + j] = val[k];
    }
  }
  __syncthreads();
}

// In-place lower Cholesky of M (n x n row-major).  Returns false (uniformly) on
// a non-positive pivot.
__device__ bool cholesky_inplace(double *M, int n) {
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    double piv = M[(int64_t)k * n + k];
    if (!(piv > 0.0)) return false;
    double d = sqrt(piv);
    __syncthreads();
    if (threadIdx.x == 0) M[(int64_t)k * n + k] = d;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) M[(int64_t)i * n + k] /= d;
    __syncthreads();
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
      double ljk = M[(int64_t)j * n + k];
      for (int i = j; i < n; ++i) M[(int64_t)i * n + j] -= M[(int64_t)i * n + k] * ljk;
    }
  }
  __syncthreads();
  return true;
}

// X = (L L^T)^-1 with one thread per column: forward L Y = I, backward L^T X = Y.
__device__ void inverse_from_factor(const double *Lf, int n, double *X) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    for (int i = 0; i < j; ++i) X[(int64_t)i * n + j] = 0.0;
    for (int i = j; i < n; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) acc -= Lf[(int64_t)i * n + k] * X[(int64_t)k * n + j];
      X[(int64_t)i * n + j] = acc / Lf[(int64_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double acc = X[(int64_t)i * n + j];
      for (int k = i + 1; k < n; ++k) acc -= Lf[(int64_t)k * n + i] * X[(int64_t)k * n + j];
      X[(int64_t)i * n + j] = acc / Lf[(int64_t)i * n + i];
    }
  }
  __syncthreads();
}

// patches above BATCH_MAX DOFs are factored one at a time by the blocked
// multi-workgroup path of the coarsest level; above MAX_PATCH they are refused
// (when the patches are set)
constexpr int BATCH_MAX = 2048;
// smallest coarsest level solved by nested dissection when coarse_solver = 0
constexpr int64_t COARSE_ND_MIN = 12288;

__global__ void k_gather_patch_dense(const int64_t *rp, const int32_t *col, const double *val, const int32_t *B,
                                     int n, double *M) {
  int i = blockIdx.x;
  for (int j = threadIdx.x; j < n; j += blockDim.x) M[(int64_t)i * n + j] = 0.0;
  __syncthreads();
  int32_t r = B[i];
  for (int64_t k = rp[r] + threadIdx.x; k < rp[r + 1]; k += blockDim.x) {
    int j = find_sorted(B, n, col[k]);
    if (j >= 0) M[(int64_t)i * n + j] = val[k];
  }
}

static void dense_spd_inverse(hipStream_t s, double *M, int64_t n, double *X, int *bad);

// one workgroup per patch: full row-major inverse -> packed lower tiles
template <class T>
__global__ __launch_bounds__(256) void k_pack_patch(const int32_t *ptr, const int64_t *ioff, const double *inv,
                                                    const int64_t *toff, T *pk) {
  constexpr int PT = PATCH_TILE;
  const int k = blockIdx.x;
  const int n = ptr[k + 1] - ptr[k];
  const int nb = (n + PT - 1) / PT;
  const double *X = inv + ioff[k];
  T *out = pk + toff[k];
  int64_t t = 0;
  for (int I = 0; I < nb; ++I)
    for (int J = 0; J <= I; ++J, ++t)
      for (int e = threadIdx.x; e < PT * PT; e += blockDim.x) {
        int r = I * PT + e / PT, cc = J * PT + e % PT;
        out[t * PT * PT + e] = (r < n && cc < n) ? (T)X[(int64_t)r * n + cc] : (T)0;
      }
}

void factor_patches(Ctx &c, Level &L) {
  Patches &P = L.patch;
  if (P.n == 0) return;
  hipStream_t s = c.stream;
  int64_t total = (int64_t)P.inv64.n;
  DBuf<int> bad;
  bad.alloc(1);
  int init = 2147483647;
  MG_HIP(hipMemcpyAsync(bad.p, &init, sizeof(int), hipMemcpyHostToDevice, s));
  std::vector<int32_t> large;
  factor_patches_batched(c, L, BATCH_MAX, large, bad);
  std::vector<int64_t> hoff;
  download(hoff, P.inv_off.p, (size_t)P.n, s);
  int hb = 0;
  for (int32_t k : large) {
    int n = P.h_kptr[k + 1] - P.h_kptr[k];
    DBuf<double> M;
    M.alloc((int64_t)n * n);
    DBuf<int> badl;
    badl.alloc(1);
    MG_HIP(hipMemcpyAsync(badl.p, &init, sizeof(int), hipMemcpyHostToDevice, s));
    k_gather_patch_dense<<<n, 256, 0, s>>>(L.A.rowptr, L.A.col, L.A.val, P.dofs_canon.p + P.h_kptr[k], n, M);
    MG_LAUNCH_CHECK();
    dense_spd_inverse(s, M, n, P.inv64.p + hoff[k], badl);
    MG_HIP(hipMemcpyAsync(&hb, badl.p, sizeof(int), hipMemcpyDeviceToHost, s));
    MG_HIP(hipStreamSynchronize(s));
    if (hb != 2147483647) fail(MG_ERR_NOT_SPD, "patch system %d has a non-positive Cholesky pivot", k);
  }
  MG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hb != 2147483647) fail(MG_ERR_NOT_SPD, "patch system %d has a non-positive Cholesky pivot", hb);
  // lower 32 x 32 tiles of every inverse, in the precision of the cycle
  (void)total;
  if (c.opt.precision == MG_MIXED) {
    P.inv.v32.alloc(P.inv.packed);
    k_pack_patch<float><<<P.n, 256, 0, s>>>(P.ptr, P.inv_off, P.inv64, P.inv.tile_off, P.inv.v32);
  } else {
    P.inv.v64.alloc(P.inv.packed);
    k_pack_patch<double><<<P.n, 256, 0, s>>>(P.ptr, P.inv_off, P.inv64, P.inv.tile_off, P.inv.v64);
  }
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(s));
  P.inv64.release();
}

// ---------------------------------------------------------------------------
// large dense SPD inverse: 64x64 tiles
// ---------------------------------------------------------------------------
constexpr int TB = 64;

__global__ void k_dense_from_csr(const int64_t *rp, const int32_t *col, const double *val, int64_t n, double *M) {
  int64_t r = blockIdx.x;
  if (r >= n) return;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) M[r * n + j] = 0.0;
  __syncthreads();
  for (int64_t k = rp[r] + threadIdx.x; k < rp[r + 1]; k += blockDim.x) M[r * n + col[k]] = val[k];
}

// factor the diagonal tile kb in LDS (one workgroup)
__global__ __launch_bounds__(256) void k_chol_diag(double *A, int64_t n, int kb, int *bad) {
  __shared__ double D[TB][TB + 1];
  int64_t o = (int64_t)kb * TB;
  int m = (int)min((int64_t)TB, n - o);
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) D[t / m][t % m] = A[(o + t / m) * n + o + t % m];
  for (int k = 0; k < m; ++k) {
    __syncthreads();
    double piv = D[k][k];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) atomicMin(bad, (int)(o + k));
      return;
    }
    double d = sqrt(piv);
    __syncthreads();
    if (threadIdx.x == 0) D[k][k] = d;
    for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) D[i][k] /= d;
    __syncthreads();
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      int i = t / m, j = t % m;
      if (j > k && i >= j) D[i][j] -= D[i][k] * D[j][k];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    int i = t / m, j = t % m;
    A[(o + i) * n + o + j] = j <= i ? D[i][j] : 0.0;
  }
}

// rows of block ib > kb: X = A[ib, kb] L[kb, kb]^-T (64 threads, one per row)
__global__ __launch_bounds__(64) void k_chol_panel(double *A, int64_t n, int kb) {
  __shared__ double Lk[TB][TB + 1];
  __shared__ double R[TB][TB + 1];
  int64_t o = (int64_t)kb * TB;
  int m = (int)min((int64_t)TB, n - o);
  int64_t ro = (int64_t)(kb + 1 + blockIdx.x) * TB;
  int mr = (int)min((int64_t)TB, n - ro);
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) Lk[t / m][t % m] = A[(o + t / m) * n + o + t % m];
  for (int t = threadIdx.x; t < mr * m; t += blockDim.x) R[t / m][t % m] = A[(ro + t / m) * n + o + t % m];
  __syncthreads();
  int r = threadIdx.x;
  if (r < mr) {
    for (int cc = 0; cc < m; ++cc) {
      double x = R[r][cc];
      for (int k = 0; k < cc; ++k) x -= R[r][k] * Lk[cc][k];
      R[r][cc] = x / Lk[cc][cc];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < mr * m; t += blockDim.x) A[(ro + t / m) * n + o + t % m] = R[t / m][t % m];
}

__device__ inline void tri_index(int64_t t, int &i, int &j) {
  // t -> (i, j) with 0 <= j <= i, t = i (i + 1) / 2 + j
  int64_t ii = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (ii * (ii + 1) / 2 > t) --ii;
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  i = (int)ii;
  j = (int)(t - ii * (ii + 1) / 2);
}

// The 64 x 64 tile products below run on the FP64 matrix cores: one workgroup
// per output tile, wavefront w owns the 32 x 32 quadrant (w >> 1, w & 1) and
// reads its operands straight into registers (mfma_tile.h).

// trailing update: A[ib, jb] -= L[ib, kb] L[jb, kb]^T for kb < jb <= ib
__global__ __launch_bounds__(256) void k_chol_update(double *A, int64_t n, int kb) {
  int i, j;
  tri_index(blockIdx.x, i, j);
  const int ib = kb + 1 + i, jb = kb + 1 + j;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, qr = wave >> 1, qc = wave & 1;
  v4d acc[2][2];
  zero_acc(acc);
  for (int kc = 0; kc < 2; ++kc) {
    double a[16], b[16];
    fetch_ops<true>(A, (int)n, ib * TB + 32 * qr, kb * TB + 32 * kc, false, a, lane);
    fetch_ops<false>(A, (int)n, jb * TB + 32 * qc, kb * TB + 32 * kc, true, b, lane);
    mma_ops(acc, a, b);
  }
  for_acc(acc, lane, [&](int r, int c, double v) {
    int64_t gr = (int64_t)ib * TB + 32 * qr + r, gc = (int64_t)jb * TB + 32 * qc + c;
    if (gr < n && gc < n) A[gr * n + gc] -= v;
  });
}

// W[jb, jb] = L[jb, jb]^-1 (one workgroup of 64 threads per diagonal tile)
__global__ __launch_bounds__(64) void k_trtri_diag(const double *Lm, double *W, int64_t n) {
  __shared__ double Lk[TB][TB + 1];
  __shared__ double X[TB][TB + 1];
  int64_t o = (int64_t)blockIdx.x * TB;
  int m = (int)min((int64_t)TB, n - o);
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) Lk[t / m][t % m] = Lm[(o + t / m) * n + o + t % m];
  __syncthreads();
  int cc = threadIdx.x;
  if (cc < m) {
    for (int r = 0; r < m; ++r) {
      if (r < cc) { X[r][cc] = 0.0; continue; }
      double acc = (r == cc) ? 1.0 : 0.0;
      for (int k = cc; k < r; ++k) acc -= Lk[r][k] * X[k][cc];
      X[r][cc] = acc / Lk[r][r];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) W[(o + t / m) * n + o + t % m] = X[t / m][t % m];
}

// Right-looking solve of L Y = I (Y = L^-1, lower triangular), one step per
// block row kb: Y[kb, jb] <- Linv[kb, kb] Y[kb, jb] for jb <= kb, then
// Y[ib, jb] -= L[ib, kb] Y[kb, jb] for ib > kb, jb <= kb.  Every tile of a step
// is independent, so each step is one wide launch.
__global__ __launch_bounds__(256) void k_trsm_rows(const double *Dinv, double *Y, int64_t n, int kb) {
  const int jb = blockIdx.x;  // 0..kb
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, qr = wave >> 1, qc = wave & 1;
  double a[2][16], b[2][16];
  for (int kc = 0; kc < 2; ++kc) {
    fetch_ops<true>(Dinv, (int)n, kb * TB + 32 * qr, kb * TB + 32 * kc, false, a[kc], lane);
    fetch_ops<false>(Y, (int)n, kb * TB + 32 * kc, jb * TB + 32 * qc, false, b[kc], lane);
  }
  __syncthreads();  // the tile is overwritten in place: all reads first
  v4d acc[2][2];
  zero_acc(acc);
  mma_ops(acc, a[0], b[0]);
  mma_ops(acc, a[1], b[1]);
  for_acc(acc, lane, [&](int r, int c, double v) {
    int64_t gr = (int64_t)kb * TB + 32 * qr + r, gc = (int64_t)jb * TB + 32 * qc + c;
    if (gr < n && gc < n) Y[gr * n + gc] = v;
  });
}

__global__ __launch_bounds__(256) void k_trsm_update(const double *Lm, double *Y, int64_t n, int kb) {
  const int ib = kb + 1 + blockIdx.x / (kb + 1), jb = blockIdx.x % (kb + 1);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, qr = wave >> 1, qc = wave & 1;
  v4d acc[2][2];
  zero_acc(acc);
  for (int kc = 0; kc < 2; ++kc) {
    double a[16], b[16];
    fetch_ops<true>(Lm, (int)n, ib * TB + 32 * qr, kb * TB + 32 * kc, false, a, lane);
    fetch_ops<false>(Y, (int)n, kb * TB + 32 * kc, jb * TB + 32 * qc, false, b, lane);
    mma_ops(acc, a, b);
  }
  for_acc(acc, lane, [&](int r, int c, double v) {
    int64_t gr = (int64_t)ib * TB + 32 * qr + r, gc = (int64_t)jb * TB + 32 * qc + c;
    if (gr < n && gc < n) Y[gr * n + gc] -= v;
  });
}

__global__ void k_identity(double *Y, int64_t n) {
  int64_t r = blockIdx.x;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) Y[r * n + j] = (j == r) ? 1.0 : 0.0;
}

// X[ib, jb] = sum_{k>=ib} W[k, ib]^T W[k, jb] for jb <= ib; mirrored to X[jb, ib]
__global__ __launch_bounds__(256) void k_lauum(const double *W, double *X, int64_t n, int nb) {
  int ib, jb;
  tri_index(blockIdx.x, ib, jb);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, qr = wave >> 1, qc = wave & 1;
  v4d acc[2][2];
  zero_acc(acc);
  for (int k = ib; k < nb; ++k)
    for (int kc = 0; kc < 2; ++kc) {
      double a[16], b[16];
      fetch_ops<true>(W, (int)n, k * TB + 32 * kc, ib * TB + 32 * qr, true, a, lane);
      fetch_ops<false>(W, (int)n, k * TB + 32 * kc, jb * TB + 32 * qc, false, b, lane);
      mma_ops(acc, a, b);
    }
  for_acc(acc, lane, [&](int r, int c, double v) {
    const int lr = 32 * qr + r, lc = 32 * qc + c;
    int64_t gr = (int64_t)ib * TB + lr, gc = (int64_t)jb * TB + lc;
    if (gr < n && gc < n && (ib != jb || lr >= lc)) {  // diagonal tiles: lower half, mirrored
      X[gr * n + gc] = v;
      X[gc * n + gr] = v;
    }
  });
}

__global__ __launch_bounds__(256) void k_single_inverse(const int64_t *rp, const int32_t *col, const double *val,
                                                        int n, double *scratch, double *inv, int *bad) {
  gather_block(rp, col, val, nullptr, n, scratch);
  if (!cholesky_inplace(scratch, n)) {
    if (threadIdx.x == 0) atomicMin(bad, 0);
    return;
  }
  inverse_from_factor(scratch, n, inv);
}

// In-place blocked Cholesky of the n x n SPD matrix M (row-major) and its
// explicit inverse in X; *bad receives the first non-positive pivot row.
// M = L L^T in place (lower triangle of M; the strict upper part keeps A's)
void dense_cholesky(hipStream_t s, double *M, int64_t n, int *bad) {
  int nb = (int)((n + TB - 1) / TB);
  for (int kb = 0; kb < nb; ++kb) {
    k_chol_diag<<<1, 256, 0, s>>>(M, n, kb, bad);
    MG_LAUNCH_CHECK();
    int rest = nb - kb - 1;
    if (rest > 0) {
      k_chol_panel<<<rest, 64, 0, s>>>(M, n, kb);
      MG_LAUNCH_CHECK();
      int64_t tiles = (int64_t)rest * (rest + 1) / 2;
      k_chol_update<<<(unsigned)tiles, 256, 0, s>>>(M, n, kb);
      MG_LAUNCH_CHECK();
    }
  }
}

// W = L^-1 (lower; L the lower triangle of M): inverses of the diagonal tiles,
// then a right-looking block solve of L W = I
void dense_lower_inverse(hipStream_t s, const double *M, int64_t n, double *W) {
  int nb = (int)((n + TB - 1) / TB);
  DBuf<double> Dinv;
  Dinv.alloc(n * n);
  k_trtri_diag<<<nb, 64, 0, s>>>(M, Dinv, n);
  MG_LAUNCH_CHECK();
  k_identity<<<(unsigned)n, 256, 0, s>>>(W, n);
  MG_LAUNCH_CHECK();
  for (int kb = 0; kb < nb; ++kb) {
    k_trsm_rows<<<kb + 1, 256, 0, s>>>(Dinv, W, n, kb);
    MG_LAUNCH_CHECK();
    int64_t tiles = (int64_t)(nb - kb - 1) * (kb + 1);
    if (tiles > 0) {
      k_trsm_update<<<(unsigned)tiles, 256, 0, s>>>(M, W, n, kb);
      MG_LAUNCH_CHECK();
    }
  }
  MG_HIP(hipStreamSynchronize(s));
}

// X = A^-1 = W^T W with W = L^-1 (M is overwritten by the factor)
static void dense_spd_inverse(hipStream_t s, double *M, int64_t n, double *X, int *bad) {
  const int nb = (int)((n + TB - 1) / TB);
  dense_cholesky(s, M, n, bad);
  DBuf<double> W;
  W.alloc(n * n);
  dense_lower_inverse(s, M, n, W);
  int64_t tiles = (int64_t)nb * (nb + 1) / 2;
  k_lauum<<<(unsigned)tiles, 256, 0, s>>>(W, X, n, nb);
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(s));
}

// one workgroup per packed tile of a single n x n system
__global__ __launch_bounds__(256) void k_pack_single(const double *X, int64_t n, double *pk) {
  constexpr int PT = PATCH_TILE;
  int I, J;
  tri_index(blockIdx.x, I, J);
  double *out = pk + (int64_t)blockIdx.x * PT * PT;
  for (int e = threadIdx.x; e < PT * PT; e += blockDim.x) {
    int64_t r = (int64_t)I * PT + e / PT, cc = (int64_t)J * PT + e % PT;
    out[e] = (r < n && cc < n) ? X[r * n + cc] : 0.0;
  }
}

void factor_coarsest(Ctx &c, Level &L) {
  hipStream_t s = c.stream;
  int64_t n = L.nfree;
  if (n > 60000) fail(MG_ERR_LIMIT, "coarsest level has %lld unknowns (limit 60000 for the dense solver)",
                      (long long)n);
  // nested dissection where the dense inverse's n^2 / 2 entries per solve
  // outweigh the dissection's launches
  const int mode = c.opt.coarse_solver;
  if (mode == 2 || (mode == 0 && n >= COARSE_ND_MIN)) {
    factor_coarsest_nd(c, L, c.opt.coarse_nd_leaf);
    return;
  }
  L.cinv.alloc(n * n);
  DBuf<int> bad;
  bad.alloc(1);
  int init = 2147483647;
  MG_HIP(hipMemcpyAsync(bad.p, &init, sizeof(int), hipMemcpyHostToDevice, s));
  DBuf<double> Lm;
  Lm.alloc(n * n);
  if (n <= 512) {
    k_single_inverse<<<1, 256, 0, s>>>(L.A.rowptr, L.A.col, L.A.val, (int)n, Lm, L.cinv, bad);
    MG_LAUNCH_CHECK();
  } else {
    k_dense_from_csr<<<(unsigned)n, 256, 0, s>>>(L.A.rowptr, L.A.col, L.A.val, n, Lm);
    MG_LAUNCH_CHECK();
    dense_spd_inverse(s, Lm, n, L.cinv, bad);
  }
  int hb = 0;
  MG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hb != 2147483647) fail(MG_ERR_NOT_SPD, "coarsest operator: non-positive pivot at row %d", hb);
  // packed lower tiles of the inverse (one system)
  std::vector<int32_t> kptr = {0, (int32_t)n};
  std::vector<int> cf = {0, 1};
  build_packed_layout(s, kptr, cf, L.cpk);
  upload(L.cptr, kptr.data(), kptr.size(), s);
  L.cpk.v64.alloc(L.cpk.packed);
  int64_t nbt = (n + PATCH_TILE - 1) / PATCH_TILE;
  int64_t tiles = nbt * (nbt + 1) / 2;
  k_pack_single<<<(unsigned)tiles, 256, 0, s>>>(L.cinv, n, L.cpk.v64);
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(s));
  L.cinv.release();
}

}  // namespace mg

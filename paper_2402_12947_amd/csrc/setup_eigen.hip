// Largest eigenvalue of the Jacobi-preconditioned operator for the Chebyshev
// smoother (paper Sec. 3.2, Sec. 6 intro) and the adjusted largest eigenvalue
// of Sec. 5: lambda_max(D_gg^-1 A_gg) on the DOFs outside every patch.
//
// The paper uses a Krylov-Schur solver with tolerance 1e-8; here Lanczos with
// full reorthogonalisation runs on H = m D^-1/2 A D^-1/2 m (m = 0/1 mask of the
// DOFs kept; H has the spectrum of D_gg^-1 A_gg plus zeros) and stops when the
// Ritz residual beta_(j+1) |s_j| <= tol * theta_max or after maxit steps.
// The start vector is a fixed pseudo-random vector: SplitMix64 (Steele, Lea,
// Flood, OOPSLA 2014) of the row index, top 53 bits mapped to [-1, 1).
// The iteration runs in the level's solve order (a symmetric permutation of
// the unknowns, which leaves the spectrum unchanged); the start vector is
// indexed by the canonical unknown so that it does not depend on that order.
// Matrix-vector products, inner products and the Gram-Schmidt sweep run on
// the GPU; the small tridiagonal eigenproblem runs on the host (bisection on
// the Sturm count for theta_max, inverse iteration for its eigenvector).
#include <cmath>

#include "devutil.h"

namespace mg {

__device__ inline double splitmix_unit(uint64_t i) {
  uint64_t z = i + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

// q[p] for solve-order unknown p = canonical unknown perm[p]
__global__ void k_lanczos_start(const uint8_t *mask, const int32_t *perm, int64_t n, double *q) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = (mask && !mask[i]) ? 0.0 : splitmix_unit((uint64_t)perm[i]);
}

// t = m s q   with s = sqrt(dinv)
__global__ void k_scale_in(const double *q, const double *dinv, const uint8_t *mask, int64_t n, double *t) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = (mask && !mask[i]) ? 0.0 : sqrt(dinv[i]) * q[i];
}
__global__ void k_scale_out(double *w, const double *dinv, const uint8_t *mask, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = (mask && !mask[i]) ? 0.0 : sqrt(dinv[i]) * w[i];
}
// w -= a q + b qprev
__global__ void k_lanczos_axpy(double *w, const double *q, const double *qp, double a, double b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = w[i] - a * q[i] - (qp ? b * qp[i] : 0.0);
}
__global__ void k_scale(double *y, const double *x, double a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// partial sums of Q[k] . w for k < m: part[k * nblk + block]; each block
// handles eight vectors at once (blockIdx.y) to amortise the reductions
__global__ __launch_bounds__(256) void k_multidot(const double *Q, int64_t n, int m, const double *w, double *part,
                                                  int nblk) {
  __shared__ double red[8][256];
  const int k0 = blockIdx.y * 8;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)nblk * 256) {
    double wi = w[i];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (k0 + q < m) s[q] += Q[(int64_t)(k0 + q) * n + i] * wi;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 8 && k0 + (int)threadIdx.x < m) part[(int64_t)(k0 + threadIdx.x) * nblk + blockIdx.x] =
      red[threadIdx.x][0];
}
__global__ void k_multidot_finish(const double *part, int m, int nblk, double *out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)k * nblk + b];
  out[k] = s;
}
// w -= sum_k c_k Q[k]
__global__ void k_multiaxpy(const double *Q, int64_t n, int m, const double *cvec, double *w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0;
  for (int k = 0; k < m; ++k) s += cvec[k] * Q[(int64_t)k * n + i];
  w[i] -= s;
}

// ---------------------------------------------------------------------------
// host: largest eigenpair of a symmetric tridiagonal matrix
// ---------------------------------------------------------------------------
static int sturm_count_below(const std::vector<double> &a, const std::vector<double> &b, double x) {
  // number of eigenvalues < x (LDL^T pivots of T - x I)
  int cnt = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++cnt;
  }
  return cnt;
}

static void tridiag_top(const std::vector<double> &a, const std::vector<double> &b, double &theta, double &slast) {
  size_t m = a.size();
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < m; ++i) {
    double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  // bisection for the largest eigenvalue: count(x) = m - 1 means x <= theta_max
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count_below(a, b, mid) >= (int)m) hi = mid; else lo = mid;
  }
  theta = 0.5 * (lo + hi);
  if (m == 1) {
    slast = 1.0;
    return;
  }
  // inverse iteration with mu just above theta_max: T - mu I is negative
  // definite, so its LDL^T factorisation (Thomas algorithm) needs no pivoting
  double mu = theta + 1e-12 * std::max(1.0, std::fabs(theta));
  std::vector<double> x(m, 1.0), dd(m), y(m);
  for (int sweep = 0; sweep < 3; ++sweep) {
    // forward: dd = pivots, y = L^-1 x
    dd[0] = a[0] - mu;
    y[0] = x[0];
    for (size_t i = 1; i < m; ++i) {
      double l = b[i - 1] / dd[i - 1];
      dd[i] = (a[i] - mu) - l * b[i - 1];
      y[i] = x[i] - l * y[i - 1];
    }
    // backward: solve (D L^T) z = y
    y[m - 1] /= dd[m - 1];
    for (int i = (int)m - 2; i >= 0; --i) y[i] = (y[i] - b[i] * y[i + 1]) / dd[i];
    double nrm = 0;
    for (double v : y) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (size_t i = 0; i < m; ++i) x[i] = y[i] / nrm;
  }
  slast = x[m - 1];
}

static double host_dot(hipStream_t s, const double *x, const double *y, int64_t n, DBuf<double> &part, double *dres) {
  int nb = dot_blocks(n);
  dot_partials(s, x, y, n, part, nb);
  finish_sum(s, part, nb, dres);
  double h = 0;
  MG_HIP(hipMemcpyAsync(&h, dres, sizeof(double), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  return h;
}

static double lanczos(Ctx &c, Level &L, const uint8_t *mask, int &steps) {
  hipStream_t s = c.stream;
  const int64_t n = L.nfree;
  const int maxit = std::max(1, c.opt.eig_maxit);
  const double tol = c.opt.eig_tol;
  DBuf<double> Q, w, t, part, dres, cvec, mpart;
  Q.alloc((size_t)(maxit + 1) * n);
  w.alloc(n);
  t.alloc(n);
  part.alloc(1024);
  dres.alloc(1);
  cvec.alloc(maxit + 1);
  const int nblk = (int)std::min<int64_t>(512, (n + 255) / 256);
  mpart.alloc((size_t)(maxit + 1) * nblk);
  const int g = grid_for(n, 256);
  k_lanczos_start<<<g, 256, 0, s>>>(mask, L.perm, n, Q);
  MG_LAUNCH_CHECK();
  double nrm = std::sqrt(host_dot(s, Q, Q, n, part, dres));
  if (nrm == 0.0) {
    steps = 0;
    return 0.0;
  }
  k_scale<<<g, 256, 0, s>>>(Q, Q, 1.0 / nrm, n);
  MG_LAUNCH_CHECK();
  std::vector<double> alpha, beta, hc;
  double theta = 0, slast = 1;
  for (int j = 0; j < maxit; ++j) {
    double *qj = Q.p + (size_t)j * n;
    k_scale_in<<<g, 256, 0, s>>>(qj, L.dinv64, mask, n, t);
    MG_LAUNCH_CHECK();
    sell_spmv<double>(s, L.S, t.p, w.p, SPMV_SET, nullptr);
    k_scale_out<<<g, 256, 0, s>>>(w, L.dinv64, mask, n);
    MG_LAUNCH_CHECK();
    double a = host_dot(s, qj, w, n, part, dres);
    k_lanczos_axpy<<<g, 256, 0, s>>>(w, qj, j ? Q.p + (size_t)(j - 1) * n : nullptr, a, j ? beta.back() : 0.0, n);
    MG_LAUNCH_CHECK();
    // full reorthogonalisation: w -= Q (Q^T w) over q_0..q_j
    int m = j + 1;
    k_multidot<<<dim3(nblk, (m + 7) / 8), 256, 0, s>>>(Q, n, m, w, mpart, nblk);
    MG_LAUNCH_CHECK();
    k_multidot_finish<<<(m + 255) / 256, 256, 0, s>>>(mpart, m, nblk, cvec);
    MG_LAUNCH_CHECK();
    k_multiaxpy<<<g, 256, 0, s>>>(Q, n, m, cvec, w);
    MG_LAUNCH_CHECK();
    double bnext = std::sqrt(std::max(0.0, host_dot(s, w, w, n, part, dres)));
    alpha.push_back(a);
    tridiag_top(alpha, beta, theta, slast);
    steps = j + 1;
    if (bnext * std::fabs(slast) <= tol * theta || bnext == 0.0) return theta;
    beta.push_back(bnext);
    k_scale<<<g, 256, 0, s>>>(Q.p + (size_t)(j + 1) * n, w, 1.0 / bnext, n);
    MG_LAUNCH_CHECK();
  }
  return theta;
}

__global__ void k_mask_from_patches(const int32_t *dofs, int64_t total, uint8_t *mask) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < total) mask[dofs[k]] = 0;
}

void estimate_eigenvalues(Ctx &c, Level &L) {
  hipStream_t s = c.stream;
  L.lam = lanczos(c, L, nullptr, L.lanczos_steps);
  bool use_local = c.opt.local_correction && L.patch.n > 0;
  if (use_local) {
    DBuf<uint8_t> mask;
    mask.alloc(L.nfree);
    MG_HIP(hipMemsetAsync(mask.p, 1, L.nfree, s));
    k_mask_from_patches<<<grid_for(L.patch.total, 256), 256, 0, s>>>(L.patch.dofs, L.patch.total, mask);
    MG_LAUNCH_CHECK();
    L.lam_adj = lanczos(c, L, mask.p, L.lanczos_steps_adj);
  } else {
    L.lam_adj = L.lam;
    L.lanczos_steps_adj = 0;
  }
  L.hi = (use_local && c.opt.adjusted_eig) ? L.lam_adj : L.lam;
  L.lo = c.opt.cheb_lo_frac * L.hi;
}

}  // namespace mg

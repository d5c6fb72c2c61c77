// Fine-level finite-element assembly (paper Sec. 2, eq. system_finest; Sec. 6.1)
// and the sparse formats used by the solve kernels.
//
// Element stiffness of a simplex T with barycentric gradients g_a:
//   K_T[i][j] = |T| sum_{a,b} (g_a . g_b) Kref[a][b][i][j],
//   Kref[a][b][i][j] = (1/|T_ref|) int dphi_i/dlam_a dphi_j/dlam_b,
// where the reference tensors are integrated on the host with a collapsed
// (Duffy) tensor Gauss-Legendre rule that is exact for the polynomial degrees
// involved.  Global assembly is atomic-free and deterministic: every element
// entry becomes a (row * n + col, value) pair, the pairs are radix-sorted
// (stable, so equal keys keep cell order) and each run of equal keys is summed
// sequentially.  Dirichlet rows and columns are dropped (u = 0 on Gamma_D).
#include <array>
#include <cmath>

#include "basis.h"
#include <algorithm>

#include "devutil.h"
#include "geom.h"

namespace mg {

// ---------------------------------------------------------------------------
// reference tensors (host)
// ---------------------------------------------------------------------------
static void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = 0.5 * (1 - z);
    w[i] = 1.0 / ((1 - z * z) * dp * dp);  // 2/((1-z^2)dp^2) scaled by 1/2 for [0,1]
  }
}

// barycentric quadrature points and weights on the reference simplex
static void simplex_rule(int dim, std::vector<std::array<double, 4>> &pts, std::vector<double> &wts) {
  const int n = 8;
  std::vector<double> x, w;
  gauss_legendre01(n, x, w);
  pts.clear();
  wts.clear();
  if (dim == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double u = x[i], v = x[j] * (1 - u);
        pts.push_back({1 - u - v, u, v, 0});
        wts.push_back(w[i] * w[j] * (1 - u));
      }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
          double u = x[i], v = x[j] * (1 - u), t = x[k] * (1 - x[i]) * (1 - x[j]);
          pts.push_back({1 - u - v - t, u, v, t});
          wts.push_back(w[i] * w[j] * w[k] * (1 - x[i]) * (1 - x[i]) * (1 - x[j]));
        }
  }
}

__constant__ double c_ref[1600];  // Kref[a][b][i][j] or Mref[i][j]

static void reference_tensor(int dim, int degree, bool mass, std::vector<double> &out) {
  int nl = n_local(dim, degree), nb = dim + 1;
  std::vector<std::array<double, 4>> pts;
  std::vector<double> wts;
  simplex_rule(dim, pts, wts);
  double vref = dim == 2 ? 0.5 : 1.0 / 6.0;
  if (mass) {
    out.assign(nl * nl, 0.0);
    for (size_t q = 0; q < pts.size(); ++q)
      for (int i = 0; i < nl; ++i)
        for (int j = 0; j < nl; ++j)
          out[i * nl + j] += wts[q] * basis_value(dim, degree, i, pts[q].data()) *
                             basis_value(dim, degree, j, pts[q].data()) / vref;
  } else {
    out.assign(nb * nb * nl * nl, 0.0);
    for (size_t q = 0; q < pts.size(); ++q)
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
          for (int i = 0; i < nl; ++i)
            for (int j = 0; j < nl; ++j)
              out[((a * nb + b) * nl + i) * nl + j] += wts[q] * basis_dlam(dim, degree, i, a, pts[q].data()) *
                                                      basis_dlam(dim, degree, j, b, pts[q].data()) / vref;
  }
}

// ---------------------------------------------------------------------------
// element matrices -> (key, value) pairs
// ---------------------------------------------------------------------------
// one thread per (cell, local row i): writes nloc pairs
__global__ void k_element_pairs(const double *X, const int32_t *cells, const int32_t *cell_dofs,
                                const int32_t *row_index, const int32_t *col_index, int64_t nc, int dim,
                                int nloc, int mass, uint64_t ncols, uint64_t sentinel, uint64_t *keys,
                                double *vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nloc) return;
  int64_t c = t / nloc;
  int i = (int)(t - c * nloc);
  int nb = dim + 1;
  double g[4][3];
  double vol = simplex_grads(X, cells + c * nb, dim, g);
  double G[4][4];
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      double s = 0;
      for (int x = 0; x < dim; ++x) s += g[a][x] * g[b][x];
      G[a][b] = s;
    }
  const int32_t *cd = cell_dofs + c * nloc;
  int32_t ri = row_index[cd[i]];
  for (int j = 0; j < nloc; ++j) {
    double v;
    if (mass) {
      v = vol * c_ref[i * nloc + j];
    } else {
      double s = 0;
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) s += G[a][b] * c_ref[((a * nb + b) * nloc + i) * nloc + j];
      v = vol * s;
    }
    int32_t cj = col_index ? col_index[cd[j]] : cd[j];
    int64_t o = t * nloc + j;
    keys[o] = (ri >= 0 && cj >= 0) ? (uint64_t)ri * ncols + (uint64_t)cj : sentinel;
    vals[o] = v;
  }
}

__global__ void k_segment_sum(const double *vals, const int32_t *len, const int64_t *off, int64_t n, double *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0;
  int64_t b = off[i];
  for (int32_t k = 0; k < len[i]; ++k) s += vals[b + k];
  out[i] = s;
}

__global__ void k_keys_to_csr(const uint64_t *keys, int64_t nnz, uint64_t ncols, int64_t nrows, int32_t *col,
                              int64_t *rowptr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  uint64_t k = keys[i];
  int64_t r = (int64_t)(k / ncols);
  col[i] = (int32_t)(k % ncols);
  int64_t rp = i == 0 ? -1 : (int64_t)(keys[i - 1] / ncols);
  for (int64_t q = rp + 1; q <= r; ++q) rowptr[q] = i;
  if (i == nnz - 1)
    for (int64_t q = r + 1; q <= nrows; ++q) rowptr[q] = nnz;
}

// Sorted unique keys (row * ncols + col) with values -> CSR.
static void csr_from_keys(hipStream_t s, const uint64_t *keys, const double *vals, int64_t nnz, int64_t nrows,
                          int64_t ncols, Csr &A) {
  A.nrows = nrows;
  A.ncols = ncols;
  A.nnz = nnz;
  A.rowptr.alloc(nrows + 1);
  A.col.alloc(nnz);
  A.val.alloc(nnz);
  if (nnz == 0) {
    MG_HIP(hipMemsetAsync(A.rowptr.p, 0, (nrows + 1) * sizeof(int64_t), s));
    return;
  }
  k_keys_to_csr<<<grid_for(nnz, 256), 256, 0, s>>>(keys, nnz, (uint64_t)ncols, nrows, A.col, A.rowptr);
  MG_LAUNCH_CHECK();
  MG_HIP(hipMemcpyAsync(A.val.p, vals, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
}

// Sort (key, value) pairs, sum duplicates, drop the sentinel, build CSR.
static void assemble_pairs(hipStream_t s, DBuf<uint64_t> &keys, DBuf<double> &vals, int64_t npairs,
                           uint64_t sentinel, int64_t nrows, int64_t ncols, Csr &A) {
  int endbit = bits_for(sentinel);
  DBuf<uint64_t> ks;
  DBuf<double> vs;
  ks.alloc(npairs);
  vs.alloc(npairs);
  sort_pairs(s, keys.p, ks.p, vals.p, vs.p, npairs, endbit);
  keys.release();
  vals.release();
  DBuf<uint64_t> uk;
  DBuf<int32_t> len;
  uk.alloc(npairs);
  len.alloc(npairs);
  int64_t nrun = run_length(s, ks.p, uk.p, len.p, npairs);
  uint64_t lastkey = 0;
  MG_HIP(hipMemcpyAsync(&lastkey, uk.p + nrun - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  int64_t nnz = (lastkey == sentinel) ? nrun - 1 : nrun;
  DBuf<int64_t> off;
  off.alloc(nrun);
  exclusive_scan(s, len.p, off.p, nrun);
  DBuf<double> sum;
  sum.alloc(nnz > 0 ? nnz : 1);
  if (nnz > 0) {
    k_segment_sum<<<grid_for(nnz, 256), 256, 0, s>>>(vs, len, off, nnz, sum);
    MG_LAUNCH_CHECK();
  }
  csr_from_keys(s, uk.p, sum.p, nnz, nrows, ncols, A);
  MG_HIP(hipStreamSynchronize(s));
}

static void element_assembly(Ctx &c, Level &L, bool mass, Csr &A) {
  hipStream_t s = c.stream;
  std::vector<double> ref;
  reference_tensor(L.dim, L.degree, mass, ref);
  MG_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_ref), ref.data(), ref.size() * sizeof(double), 0,
                                hipMemcpyHostToDevice, s));
  int64_t npairs = L.nc * L.nloc * L.nloc;
  uint64_t ncols = mass ? (uint64_t)L.ndofs : (uint64_t)L.nfree;
  uint64_t sentinel = (uint64_t)L.nfree * ncols;
  DBuf<uint64_t> keys;
  DBuf<double> vals;
  keys.alloc(npairs);
  vals.alloc(npairs);
  k_element_pairs<<<grid_for(L.nc * L.nloc, 256), 256, 0, s>>>(
      L.coords, L.cells, L.cell_dofs, L.free_index, mass ? nullptr : L.free_index.p, L.nc, L.dim, L.nloc,
      mass ? 1 : 0, ncols, sentinel, keys, vals);
  MG_LAUNCH_CHECK();
  assemble_pairs(s, keys, vals, npairs, sentinel, L.nfree, (int64_t)ncols, A);
}

// Linear elasticity (Sec. 6.2): vector unknown (DOF node s, component p) =
// s * dim + p; with int d_k phi_i d_l phi_j = |T| sum_ab g_a[k] g_b[l] Kref[a][b][i][j],
//   K[(i,p),(j,q)] = |T| sum_ab Kref[a][b][i][j] (mu delta_pq g_a.g_b
//                                               + mu g_a[q] g_b[p] + lambda g_a[p] g_b[q]).
// One thread per (cell, local DOF i, component p) writes nloc * dim pairs.
__global__ void k_element_pairs_elast(const double *X, const int32_t *cells, const int32_t *cell_dofs,
                                      const int32_t *free_index, int64_t nc, int dim, int nloc, double mu,
                                      double lam, uint64_t ncols, uint64_t sentinel, uint64_t *keys,
                                      double *vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nloc * dim) return;
  int64_t c = t / (nloc * dim);
  int ip = (int)(t - c * nloc * dim);
  int i = ip / dim, p = ip % dim;
  int nb = dim + 1;
  double g[4][3];
  double vol = simplex_grads(X, cells + c * nb, dim, g);
  // C[q][a][b] = mu delta_pq g_a.g_b + mu g_a[q] g_b[p] + lambda g_a[p] g_b[q]
  double C[3][4][4];
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      double gg = 0;
      for (int x = 0; x < dim; ++x) gg += g[a][x] * g[b][x];
      for (int q = 0; q < dim; ++q)
        C[q][a][b] = (q == p ? mu * gg : 0.0) + mu * g[a][q] * g[b][p] + lam * g[a][p] * g[b][q];
    }
  const int32_t *cd = cell_dofs + c * nloc;
  int32_t ri = free_index[cd[i]];
  for (int j = 0; j < nloc; ++j) {
    int32_t cj = free_index[cd[j]];
    for (int q = 0; q < dim; ++q) {
      double sum = 0;
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) sum += C[q][a][b] * c_ref[((a * nb + b) * nloc + i) * nloc + j];
      int64_t o = t * (int64_t)(nloc * dim) + j * dim + q;
      keys[o] = (ri >= 0 && cj >= 0) ? (uint64_t)(ri * dim + p) * ncols + (uint64_t)(cj * dim + q) : sentinel;
      vals[o] = vol * sum;
    }
  }
}

static void elasticity_assembly(Ctx &c, Level &L) {
  hipStream_t s = c.stream;
  std::vector<double> ref;
  reference_tensor(L.dim, L.degree, false, ref);
  MG_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_ref), ref.data(), ref.size() * sizeof(double), 0,
                                hipMemcpyHostToDevice, s));
  const double E = c.opt.young, nu = c.opt.poisson_ratio;
  const double mu = E / (2.0 * (1.0 + nu)), lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const int dim = L.dim;
  int64_t npairs = L.nc * (int64_t)(L.nloc * dim) * (L.nloc * dim);
  uint64_t ncols = (uint64_t)L.nfree;
  uint64_t sentinel = (uint64_t)L.nfree * ncols;
  DBuf<uint64_t> keys;
  DBuf<double> vals;
  keys.alloc(npairs);
  vals.alloc(npairs);
  k_element_pairs_elast<<<grid_for(L.nc * L.nloc * dim, 256), 256, 0, s>>>(
      L.coords, L.cells, L.cell_dofs, L.free_index, L.nc, dim, L.nloc, mu, lam, ncols, sentinel, keys, vals);
  MG_LAUNCH_CHECK();
  assemble_pairs(s, keys, vals, npairs, sentinel, L.nfree, (int64_t)ncols, L.A);
}

// ---------------------------------------------------------------------------
// Entries that vanish in exact arithmetic are not stored.  An off-diagonal
// a_ij with |a_ij| <= 1e-12 sqrt(|a_ii a_jj|) is what is left of contributions
// that cancel: for P2 on triangles the coupling of a vertex with the midpoint
// of the opposite edge is zero on every cell (about a quarter of the assembled
// pattern), for P3 some vertex-edge couplings likewise.  On the meshes here
// these residues are below 1e-16 in that measure and the smallest true entry
// is above 1e-8, so the cut changes A by rounding only.
// ---------------------------------------------------------------------------
constexpr double DROP_EPS = 1e-12;

__global__ void k_diag_sqrt(const int64_t *rowptr, const int32_t *col, const double *val, int64_t n, double *d) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double v = 0;
  for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
    if (col[k] == r) v = sqrt(fabs(val[k]));
  d[r] = v;
}

__device__ inline bool keep_entry(int64_t r, int32_t c, double v, const double *d) {
  return c == r || fabs(v) > DROP_EPS * d[r] * d[c];
}

__global__ void k_keep_count(const int64_t *rowptr, const int32_t *col, const double *val, const double *d,
                             int64_t n, int64_t *cnt) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t k = 0;
  for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) k += keep_entry(r, col[e], val[e], d) ? 1 : 0;
  cnt[r] = k;
}

__global__ void k_keep_copy(const int64_t *rowptr, const int32_t *col, const double *val, const double *d,
                            int64_t n, const int64_t *newptr, int32_t *col2, double *val2) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t o = newptr[r];
  for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
    if (keep_entry(r, col[e], val[e], d)) {
      col2[o] = col[e];
      val2[o] = val[e];
      ++o;
    }
}

void drop_cancelled(Ctx &c, Csr &A) {
  hipStream_t s = c.stream;
  const int64_t n = A.nrows;
  if (n == 0 || A.nnz == 0 || A.ncols != n) return;
  DBuf<double> d;
  DBuf<int64_t> cnt, ptr;
  d.alloc(n);
  cnt.alloc(n);
  ptr.alloc(n + 1);
  k_diag_sqrt<<<grid_for(n, 256), 256, 0, s>>>(A.rowptr, A.col, A.val, n, d);
  MG_LAUNCH_CHECK();
  k_keep_count<<<grid_for(n, 256), 256, 0, s>>>(A.rowptr, A.col, A.val, d, n, cnt);
  MG_LAUNCH_CHECK();
  const int64_t kept = exclusive_scan(s, cnt.p, ptr.p, n);
  if (kept == A.nnz) return;
  MG_HIP(hipMemcpyAsync(ptr.p + n, &kept, sizeof(int64_t), hipMemcpyHostToDevice, s));
  DBuf<int32_t> col2;
  DBuf<double> val2;
  col2.alloc(kept);
  val2.alloc(kept);
  k_keep_copy<<<grid_for(n, 256), 256, 0, s>>>(A.rowptr, A.col, A.val, d, n, ptr, col2, val2);
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(s));
  A.rowptr = std::move(ptr);
  A.col = std::move(col2);
  A.val = std::move(val2);
  A.nnz = kept;
}

void assemble_fine(Ctx &c, Level &L) {
  if (c.opt.problem == MG_PROBLEM_ELASTICITY) elasticity_assembly(c, L);
  else element_assembly(c, L, false, L.A);
  drop_cancelled(c, L.A);
}

void assemble_mass(Ctx &c, Level &L) { element_assembly(c, L, true, c.M); }

// ---------------------------------------------------------------------------
// diagonal
// ---------------------------------------------------------------------------
__global__ void k_dinv(const int64_t *rowptr, const int32_t *col, const double *val, int64_t n, double *d64,
                       float *d32, int *bad) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double d = 0;
  for (int64_t k = rowptr[r]; k < rowptr[r + 1]; ++k)
    if (col[k] == r) d = val[k];
  if (!(d > 0)) atomicMin(bad, (int)r);
  d64[r] = 1.0 / d;
  if (d32) d32[r] = (float)(1.0 / d);
}

static void dinv_of(Ctx &c, const Csr &A, DBuf<double> &d64, DBuf<float> *d32) {
  hipStream_t s = c.stream;
  d64.alloc(A.nrows);
  if (d32) d32->alloc(A.nrows);
  DBuf<int> bad;
  bad.alloc(1);
  int init = 2147483647;
  MG_HIP(hipMemcpyAsync(bad.p, &init, sizeof(int), hipMemcpyHostToDevice, s));
  k_dinv<<<grid_for(A.nrows, 256), 256, 0, s>>>(A.rowptr, A.col, A.val, A.nrows, d64, d32 ? d32->p : nullptr, bad);
  MG_LAUNCH_CHECK();
  int hb = 0;
  MG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hb != 2147483647)
    fail(MG_ERR_NOT_SPD, "operator row %d (solve order) has a non-positive diagonal (a coarse basis "
                         "function that no fine DOF node sees, or a singular system)", hb);
}

// ---------------------------------------------------------------------------
// SELL-C-sigma from CSR
// ---------------------------------------------------------------------------
__global__ void k_sort_keys_len(const int64_t *rowptr, int64_t n, int sigma, uint64_t *keys, int32_t *rows) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  uint64_t len = (uint64_t)(rowptr[r + 1] - rowptr[r]);
  uint64_t win = (uint64_t)(r / sigma);
  keys[r] = (win << 32) | (0xFFFFFFFFULL - len);
  rows[r] = (int32_t)r;
}

__global__ void k_identity_perm(int32_t *perm, int64_t npos, int64_t n) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < npos) perm[p] = p < n ? (int32_t)p : -1;
}

// Entries of a row of len entries that lane t of its rpl lanes holds
// (entries t, t + rpl, t + 2 rpl, ...).
__device__ inline int64_t lane_entries(int64_t len, int t, int rpl) {
  return len > t ? (len - t + rpl - 1) / rpl : 0;
}

// Row at each SELL position: rpl lanes per row, 64 / rpl rows per slice; -1
// past the last row.
__global__ void k_sell_rows(int32_t *perm, int64_t npos, int64_t n, int rpl) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npos) return;
  const int64_t r = (p / SELL_C) * (SELL_C / rpl) + (p % SELL_C) / rpl;
  perm[p] = r < n ? (int32_t)r : -1;
}

__global__ void k_slice_width(const int64_t *rowptr, const int32_t *perm, int64_t nslices, int rpl, int64_t *w64) {
  int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslices) return;
  int64_t w = 0;
  for (int l = 0; l < SELL_C; ++l) {
    int32_t r = perm[sl * SELL_C + l];
    if (r >= 0) {
      int64_t len = lane_entries(rowptr[r + 1] - rowptr[r], l % rpl, rpl);
      w = len > w ? len : w;
    }
  }
  w64[sl] = w * SELL_C;
}

// Position p = (slice, lane) holds entries t, t + rpl, ... (t = lane mod rpl)
// of its row, entry t + j rpl at column j of the slice.
__global__ void k_sell_fill(const int64_t *rowptr, const int32_t *ccol, const double *cval, const int32_t *perm,
                            const int64_t *sptr, int64_t npos, int rpl, int32_t *col, double *v64, float *v32,
                            uint16_t *rlen, unsigned long long *maxlen) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npos) return;
  int64_t sl = p / SELL_C;
  int lane = (int)(p - sl * SELL_C);
  const int t = lane % rpl;
  int64_t base = sptr[sl];
  int64_t w = (sptr[sl + 1] - base) / SELL_C;
  int32_t r = perm[p];
  int64_t b = r >= 0 ? rowptr[r] : 0, len = r >= 0 ? rowptr[r + 1] - rowptr[r] : 0;
  const int64_t mine = lane_entries(len, t, rpl);
  rlen[p] = (uint16_t)(mine < 0xFFFF ? mine : 0xFFFF);
  if (mine > 0xFFFF) atomicMax(maxlen, (unsigned long long)mine);
  int32_t pad = len > 0 ? ccol[b] : 0;
  for (int64_t j = 0; j < w; ++j) {
    int64_t o = base + j * SELL_C + lane;
    const int64_t e = t + j * rpl;
    int32_t cc = j < mine ? ccol[b + e] : pad;
    double vv = j < mine ? cval[b + e] : 0.0;
    col[o] = cc;
    v64[o] = vv;
    if (v32) v32[o] = (float)vv;
  }
}

__global__ void k_slice_min(const uint16_t *rlen, int64_t nslices, int32_t *smin) {
  int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslices) return;
  int m = 0xFFFF;
  for (int l = 0; l < SELL_C; ++l) m = min(m, (int)rlen[sl * SELL_C + l]);
  smin[sl] = m;
}

__device__ inline int wave_min_i(int v) {
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m));
  return v;
}

// Greedy cover of the slice's columns by at most W windows of 2^bits columns,
// each starting at the smallest column not yet covered (optimal for intervals).
// Returns the number of windows, or 0 if W are not enough.
template <int W>
__device__ int cover_windows(const int32_t *cp, int w, int bits, int *bases) {
  int cnt = 0;
  long long end = -1;  // columns below end are covered
  while (true) {
    int m = 2147483647;
    for (int j = 0; j < w; ++j) {
      int c = cp[(int64_t)j * SELL_C];
      if ((long long)c >= end) m = min(m, c);
    }
    m = wave_min_i(m);
    if (m == 2147483647) return cnt;
    if (cnt == W) return 0;
    bases[cnt++] = m;
    end = (long long)m + (1ll << bits);
  }
}

// One wavefront per slice: choose the narrowest 16-bit form that covers every
// column of the slice (two windows of 32768, else eight of 8192, else sixteen
// of 4096) and write it, or keep the slice at 32 bits.  narrowest = 1, 2, 3
// starts the search at the eight-window form, at the sixteen-window form, or
// keeps every slice at 32 bits (a form that covers a slice also covers it in
// every wider form, so this forces the form wherever the slice fits it).
__global__ __launch_bounds__(256) void k_compress_cols(int64_t nslices, const int64_t *sptr, const int32_t *col,
                                                       const uint16_t *rlen, int narrowest, uint16_t *col16,
                                                       int32_t *cbase, int32_t *ctab, unsigned long long *nnz16) {
  const int64_t sl = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (sl >= nslices) return;
  const int lane = threadIdx.x & 63;
  const int64_t base = sptr[sl];
  const int w = (int)((sptr[sl + 1] - base) / SELL_C);
  const int32_t *cp = col + base + lane;
  uint16_t *op = col16 + base + lane;
  int bases[16];
  int mode;
  int nb = narrowest == 0 ? cover_windows<2>(cp, w, 15, bases) : 0;
  if (nb > 0) {
    const int b0 = bases[0], b1 = nb > 1 ? bases[1] : bases[0];
    for (int j = 0; j < w; ++j) {
      int c = cp[(int64_t)j * SELL_C];
      op[(int64_t)j * SELL_C] = c - b0 < 32768 ? (uint16_t)(c - b0) : (uint16_t)(0x8000 | (c - b1));
    }
    if (lane == 0) {
      cbase[2 * sl] = b0;
      cbase[2 * sl + 1] = b1;
    }
    mode = 2;
  } else {
    int bits = 13;
    nb = narrowest <= 1 ? cover_windows<8>(cp, w, 13, bases) : 0;
    if (nb == 0) {
      bits = 12;
      nb = narrowest <= 2 ? cover_windows<16>(cp, w, 12, bases) : 0;
    }
    if (nb == 0) {
      if (lane == 0) {
        cbase[2 * sl] = -1;
        cbase[2 * sl + 1] = -1;
      }
      return;
    }
    for (int j = 0; j < w; ++j) {
      int c = cp[(int64_t)j * SELL_C];
      int k = 0;
      while (k + 1 < nb && c >= bases[k + 1]) ++k;
      op[(int64_t)j * SELL_C] = (uint16_t)((k << bits) | (c - bases[k]));
    }
    if (lane < 16) ctab[16 * sl + lane] = lane < nb ? bases[lane] : 0;
    if (lane == 0) {
      cbase[2 * sl] = bits == 13 ? -2 : -3;
      cbase[2 * sl + 1] = 0;
    }
    mode = bits;
  }
  (void)mode;
  unsigned long long len = rlen[sl * SELL_C + lane];
  for (int m = 32; m >= 1; m >>= 1) len += __shfl_xor(len, m);
  if (lane == 0) atomicAdd(nnz16, len);
}

// SELL-C layout of A with its rows in their given order (row = position); the
// solve order (solve_order) is applied to A beforehand.
void build_sell(Ctx &c, const Csr &A, Sell &S, int sigma, bool want32, int rpl) {
  hipStream_t s = c.stream;
  if (sigma != 1) fail(MG_ERR_ARG, "build_sell keeps the row order (sigma must be 1)");
  if (rpl != 1 && rpl != 2 && rpl != 4 && rpl != 8 && rpl != 16 && rpl != 32)
    fail(MG_ERR_ARG, "lanes per row must be 1, 2, 4, 8, 16 or 32");
  S.nrows = A.nrows;
  S.ncols = A.ncols;
  S.sigma = 1;
  S.rpl = rpl;
  const int64_t rows_per_slice = SELL_C / rpl;
  S.nslices = (A.nrows + rows_per_slice - 1) / rows_per_slice;
  int64_t npos = S.nslices * SELL_C;
  S.perm.alloc(npos);
  k_sell_rows<<<grid_for(npos, 256), 256, 0, s>>>(S.perm, npos, A.nrows, rpl);
  MG_LAUNCH_CHECK();
  DBuf<int64_t> w;
  w.alloc(S.nslices);
  k_slice_width<<<grid_for(S.nslices, 256), 256, 0, s>>>(A.rowptr, S.perm, S.nslices, rpl, w);
  MG_LAUNCH_CHECK();
  S.slice_ptr.alloc(S.nslices + 1);
  S.stored = exclusive_scan(s, w.p, S.slice_ptr.p, S.nslices);
  MG_HIP(hipMemcpyAsync(S.slice_ptr.p + S.nslices, &S.stored, sizeof(int64_t), hipMemcpyHostToDevice, s));
  S.col.alloc(S.stored);
  S.v64.alloc(S.stored);
  if (want32) S.v32.alloc(S.stored);
  S.rlen.alloc(npos);
  // cnt[0]: entries in 16-bit slices; cnt[1]: longest row above 65535 entries
  DBuf<unsigned long long> cnt;
  cnt.alloc(2);
  MG_HIP(hipMemsetAsync(cnt.p, 0, 2 * sizeof(unsigned long long), s));
  k_sell_fill<<<grid_for(npos, 256), 256, 0, s>>>(A.rowptr, A.col, A.val, S.perm, S.slice_ptr, npos, rpl, S.col,
                                                 S.v64, want32 ? S.v32.p : nullptr, S.rlen, cnt.p + 1);
  MG_LAUNCH_CHECK();
  S.smin.alloc(S.nslices);
  k_slice_min<<<grid_for(S.nslices, 256), 256, 0, s>>>(S.rlen, S.nslices, S.smin);
  MG_LAUNCH_CHECK();
  S.nnz = A.nnz;
  // variants before any timing: the options' fixed choices, else skip the
  // padding where it exceeds 2 % of the entries
  S.mask = c.opt.sell_mask >= 0 ? c.opt.sell_mask : (double)S.stored > 1.02 * (double)A.nnz;
  if (c.opt.sell_unroll) S.unroll = c.opt.sell_unroll;
  S.col16.alloc(S.stored);
  S.cbase.alloc(2 * S.nslices);
  S.ctab.alloc(16 * S.nslices);
  if (S.nslices > 0) {
    k_compress_cols<<<(unsigned)((S.nslices + 3) / 4), 256, 0, s>>>(S.nslices, S.slice_ptr, S.col, S.rlen,
                                                                    c.opt.sell_colform, S.col16, S.cbase, S.ctab,
                                                                    cnt);
    MG_LAUNCH_CHECK();
  }
  unsigned long long h[2] = {0, 0};
  MG_HIP(hipMemcpyAsync(h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (h[1] > 0) fail(MG_ERR_LIMIT, "a sparse row holds %llu entries (at most 65535 are supported)", h[1]);
  S.nnz16 = (int64_t)h[0];
}

// ---------------------------------------------------------------------------
// solve order: rows sorted by length (descending, stable) inside windows of
// sigma rows; the same permutation renumbers the unknowns, so every per-row
// vector access of the solve kernels is contiguous.
// ---------------------------------------------------------------------------
__global__ void k_perm_rowlen(const int64_t *rp, const int32_t *perm, int64_t n, int64_t *len) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) len[p] = rp[perm[p] + 1] - rp[perm[p]];
}
__global__ void k_perm_fill(const int64_t *rp, const int32_t *col, const double *val, const int32_t *perm,
                            const int32_t *iperm_cols, int64_t n, const int64_t *rp2, int32_t *col2, double *val2) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int64_t a = rp[perm[p]], b = rp[perm[p] + 1], o = rp2[p];
  for (int64_t k = a; k < b; ++k) {
    col2[o + k - a] = iperm_cols ? iperm_cols[col[k]] : col[k];
    val2[o + k - a] = val[k];
  }
}
__global__ void k_iperm(const int32_t *perm, int64_t n, int32_t *iperm) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) iperm[perm[p]] = (int32_t)p;
}

// B = A with rows taken in order perm and columns renumbered by iperm_cols
static void permute_csr(Ctx &c, const Csr &A, const int32_t *perm, int64_t nrows, const int32_t *iperm_cols,
                        int64_t ncols, Csr &B) {
  hipStream_t s = c.stream;
  DBuf<int64_t> len;
  len.alloc(nrows);
  k_perm_rowlen<<<grid_for(nrows, 256), 256, 0, s>>>(A.rowptr, perm, nrows, len);
  MG_LAUNCH_CHECK();
  B.nrows = nrows;
  B.ncols = ncols;
  B.rowptr.alloc(nrows + 1);
  B.nnz = exclusive_scan(s, len.p, B.rowptr.p, nrows);
  MG_HIP(hipMemcpyAsync(B.rowptr.p + nrows, &B.nnz, sizeof(int64_t), hipMemcpyHostToDevice, s));
  B.col.alloc(B.nnz);
  B.val.alloc(B.nnz);
  k_perm_fill<<<grid_for(nrows, 256), 256, 0, s>>>(A.rowptr, A.col, A.val, perm, iperm_cols, nrows, B.rowptr,
                                                  B.col, B.val);
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(s));
}

static void order_with(Ctx &c, Level &L, int sigma, bool want32, int rpl) {
  hipStream_t s = c.stream;
  const int64_t n = L.A.nrows;
  L.perm.alloc(n);
  L.iperm.alloc(n);
  if (sigma > 1) {
    DBuf<uint64_t> k, ks;
    DBuf<int32_t> r;
    k.alloc(n);
    ks.alloc(n);
    r.alloc(n);
    k_sort_keys_len<<<grid_for(n, 256), 256, 0, s>>>(L.A.rowptr, n, sigma, k, r);
    MG_LAUNCH_CHECK();
    int64_t nwin = (n + sigma - 1) / sigma;
    sort_pairs(s, k.p, ks.p, r.p, L.perm.p, n, 32 + bits_for((uint64_t)nwin));
  } else {
    k_identity_perm<<<grid_for(n, 256), 256, 0, s>>>(L.perm, n, n);
    MG_LAUNCH_CHECK();
  }
  k_iperm<<<grid_for(n, 256), 256, 0, s>>>(L.perm, n, L.iperm);
  MG_LAUNCH_CHECK();
  Csr B;
  permute_csr(c, L.A, L.perm, n, L.iperm, n, B);
  L.S = Sell();
  build_sell(c, B, L.S, 1, want32, rpl);
  L.S.sigma = sigma;
  dinv_of(c, B, L.dinv64, want32 ? &L.dinv32 : nullptr);
}

// Rows of A at the patch DOFs, one row per kernel-order patch entry, columns in
// the level's solve order: the patch residual streams them as a SELL matrix.
void build_patch_rows(Ctx &c, Level &L, bool want32) {
  Patches &P = L.patch;
  P.colour_fused.assign(P.ncolour, 0);
  if (P.total == 0) return;
  Csr B;
  permute_csr(c, L.A, P.dofs_canon, P.total, L.iperm, L.nfree, B);
  build_sell(c, B, P.rows, 1, want32);
  P.rows.perm.release();
  if (P.maxn > SMALL_PATCH || !c.opt.patch_fused) return;
  // which colours may run as one launch: no row of a patch reads a DOF of
  // another patch of its colour
  hipStream_t s = c.stream;
  std::vector<int64_t> rp(B.nrows + 1);
  std::vector<int32_t> col(B.nnz), pos(P.total);
  MG_HIP(hipMemcpyAsync(rp.data(), B.rowptr.p, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipMemcpyAsync(col.data(), B.col.p, col.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipMemcpyAsync(pos.data(), P.dofs.p, pos.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> owner(L.nfree, -1);
  for (int cl = 0; cl < P.ncolour; ++cl) {
    const int p0 = P.colour_first[cl], p1 = P.colour_first[cl + 1];
    for (int p = p0; p < p1; ++p)
      for (int32_t k = P.h_kptr[p]; k < P.h_kptr[p + 1]; ++k) owner[pos[k]] = p;
    bool ok = true;
    for (int p = p0; p < p1 && ok; ++p)
      for (int32_t k = P.h_kptr[p]; k < P.h_kptr[p + 1] && ok; ++k)
        for (int64_t e = rp[k]; e < rp[k + 1]; ++e) {
          const int32_t o = owner[col[e]];
          if (o >= 0 && o != p) {
            ok = false;
            break;
          }
        }
    P.colour_fused[cl] = ok;
    for (int p = p0; p < p1; ++p)
      for (int32_t k = P.h_kptr[p]; k < P.h_kptr[p + 1]; ++k) owner[pos[k]] = -1;
  }
}

// The patch rows' SELL with rpl lanes per row (a candidate of the patch-path
// autotuner): the same rows in the same kernel order, one slice per 64 / rpl
// rows.
void relayout_patch_rows(Ctx &c, Level &L, bool want32, int rpl) {
  Patches &P = L.patch;
  if (P.total == 0 || P.rows.rpl == rpl) return;
  Csr B;
  permute_csr(c, L.A, P.dofs_canon, P.total, L.iperm, L.nfree, B);
  build_sell(c, B, P.rows, 1, want32, rpl);
  P.rows.perm.release();
}

// The refinement values of the patch rows: loc = the values of P.rows with
// every column outside the row's own patch zeroed, so that the product with
// loc is A^[d] applied to a vector that holds a patch solve at its patch's
// DOFs.  A DOF lies in at most one patch of a colour, so the colours are
// marked one at a time: owner[DOF] = patch, then each row keeps the entries
// whose column its own patch owns.
__global__ void k_owner_mark(const int32_t *kpatch, const int32_t *dofs, int64_t k0, int64_t k1, int32_t *owner,
                             int clear) {
  int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < k1) owner[dofs[k]] = clear ? -1 : kpatch[k];
}
__global__ void k_patch_loc(int64_t k0, int64_t k1, const int64_t *sptr, const int32_t *col, const double *v64,
                            const int32_t *kpatch, const int32_t *owner, double *loc) {
  // one thread per (slice position, entry) of the slices covering [k0, k1)
  const int64_t s0 = k0 >> 6, s1 = (k1 + 63) >> 6;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t sl = s0 + (t >> 6);
  if (sl >= s1) return;
  const int lane = (int)(t & 63);
  const int64_t k = sl * 64 + lane;
  const int64_t base = sptr[sl], w = (sptr[sl + 1] - base) >> 6;
  const bool mine = k >= k0 && k < k1;
  for (int64_t j = 0; j < w; ++j) {
    const int64_t o = base + j * 64 + lane;
    if (mine) loc[o] = owner[col[o]] == kpatch[k] ? v64[o] : 0.0;
  }
}

void build_patch_refine(Ctx &c, Level &L) {
  Patches &P = L.patch;
  if (P.total == 0) return;
  if (P.rows.rpl != 1) fail(MG_ERR_ARG, "patch refinement needs one lane per patch row");
  hipStream_t s = c.stream;
  std::vector<int32_t> kp(P.total);
  for (int p = 0; p < P.n; ++p)
    for (int32_t k = P.h_kptr[p]; k < P.h_kptr[p + 1]; ++k) kp[k] = p;
  DBuf<int32_t> kpatch, owner;
  upload(kpatch, kp.data(), kp.size(), s);
  owner.alloc(L.nfree);
  fill<int32_t>(s, owner.p, L.nfree, -1);
  P.loc.alloc(P.rows.stored);
  fill<double>(s, P.loc.p, P.rows.stored, 0.0);
  for (int cl = 0; cl < P.ncolour; ++cl) {
    const int64_t k0 = P.h_kptr[P.colour_first[cl]], k1 = P.h_kptr[P.colour_first[cl + 1]];
    if (k1 <= k0) continue;
    k_owner_mark<<<grid_for(k1 - k0, 256), 256, 0, s>>>(kpatch, P.dofs, k0, k1, owner, 0);
    MG_LAUNCH_CHECK();
    const int64_t nthreads = (((k1 + 63) >> 6) - (k0 >> 6)) * 64;
    k_patch_loc<<<grid_for(nthreads, 256), 256, 0, s>>>(k0, k1, P.rows.slice_ptr, P.rows.col, P.rows.v64, kpatch,
                                                       owner, P.loc);
    MG_LAUNCH_CHECK();
    k_owner_mark<<<grid_for(k1 - k0, 256), 256, 0, s>>>(kpatch, P.dofs, k0, k1, owner, 1);
    MG_LAUNCH_CHECK();
  }
  MG_HIP(hipStreamSynchronize(s));
}

// Rows of A that couple to a patch DOF, as a SELL matrix in ascending solve
// order with their solve-order positions (nbr_pos).
__global__ void k_mark_dofs(const int32_t *dofs, int64_t m, uint8_t *flag) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) flag[dofs[k]] = 1;
}
__global__ void k_rows_touching(const int64_t *rowptr, const int32_t *col, const uint8_t *flag, const int32_t *perm,
                                int64_t n, int32_t *hit) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t r = perm[p];
  int32_t h = 0;
  for (int64_t k = rowptr[r]; k < rowptr[r + 1] && !h; ++k) h = flag[col[k]];
  hit[p] = h;
}
__global__ void k_compact_rows(const int32_t *hit, const int64_t *off, const int32_t *perm, int64_t n, int32_t *pos,
                               int32_t *rows) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || !hit[p]) return;
  pos[off[p]] = (int32_t)p;
  rows[off[p]] = perm[p];
}

void build_patch_neighbours(Ctx &c, Level &L, bool want32) {
  Patches &P = L.patch;
  if (P.total == 0) return;
  hipStream_t s = c.stream;
  const int64_t n = L.nfree;
  DBuf<uint8_t> flag;
  DBuf<int32_t> hit, rows;
  DBuf<int64_t> off;
  flag.alloc(n);
  hit.alloc(n);
  off.alloc(n);
  MG_HIP(hipMemsetAsync(flag.p, 0, n, s));
  k_mark_dofs<<<grid_for(P.total, 256), 256, 0, s>>>(P.dofs_canon, P.total, flag);
  MG_LAUNCH_CHECK();
  k_rows_touching<<<grid_for(n, 256), 256, 0, s>>>(L.A.rowptr, L.A.col, flag, L.perm, n, hit);
  MG_LAUNCH_CHECK();
  const int64_t m = exclusive_scan(s, hit.p, off.p, n);
  P.nbr_pos.alloc(m);
  rows.alloc(m);
  k_compact_rows<<<grid_for(n, 256), 256, 0, s>>>(hit, off, L.perm, n, P.nbr_pos, rows);
  MG_LAUNCH_CHECK();
  Csr B;
  permute_csr(c, L.A, rows, m, L.iperm, n, B);
  // the same lanes per row and gathers in flight as the level operator, so
  // that every coupled row sums its products in the same order as the full
  // step
  build_sell(c, B, P.nbr, 1, want32, L.S.rpl);
  P.nbr.perm.release();
  P.nbr.unroll = L.S.unroll;
}

// Multicolour symmetric Gauss-Seidel: greedy colouring of the matrix graph in
// canonical row order (row i takes the smallest colour not used by a coupled
// neighbour j < i), then the rows of every colour, in solve order, as a SELL
// matrix whose columns are solve-order positions.
void build_sgs(Ctx &c, Level &L, bool want32) {
  hipStream_t s = c.stream;
  const int64_t n = L.nfree;
  std::vector<int64_t> rp;
  std::vector<int32_t> col, ip;
  std::vector<double> val;
  download(rp, L.A.rowptr.p, (size_t)n + 1, s);
  download(col, L.A.col.p, (size_t)L.A.nnz, s);
  download(val, L.A.val.p, (size_t)L.A.nnz, s);
  download(ip, L.iperm.p, (size_t)n, s);
  // rows i and j are coupled if |a_ij| > 1e-12 sqrt(a_ii a_jj): Galerkin entries
  // that cancel to zero or to rounding noise are not couplings
  std::vector<double> dsq((size_t)n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
      if (col[k] == i) dsq[i] = std::sqrt(std::fabs(val[k]));
  std::vector<int32_t> colour((size_t)n, -1);
  std::vector<int64_t> mark;  // mark[k] == i: colour k is taken by a lower neighbour of row i
  int ncol = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      int32_t j = col[k];
      if (j < i && std::fabs(val[k]) > 1e-12 * dsq[i] * dsq[j]) {
        size_t cj = (size_t)colour[j];
        if (cj >= mark.size()) mark.resize(cj + 1, -1);
        mark[cj] = i;
      }
    }
    int k = 0;
    while ((size_t)k < mark.size() && mark[k] == i) ++k;
    colour[i] = k;
    ncol = std::max(ncol, k + 1);
  }
  upload(L.sgs_colour, colour.data(), colour.size(), s);
  std::vector<std::vector<int32_t>> rows(ncol);
  for (int64_t i = 0; i < n; ++i) rows[colour[i]].push_back((int32_t)i);
  L.sgs.clear();
  L.sgs_pos.clear();
  L.sgs.resize(ncol);
  L.sgs_pos.resize(ncol);
  for (int k = 0; k < ncol; ++k) {
    auto &r = rows[k];
    std::sort(r.begin(), r.end(), [&](int32_t a, int32_t b) { return ip[a] < ip[b]; });
    std::vector<int32_t> pos(r.size());
    for (size_t t = 0; t < r.size(); ++t) pos[t] = ip[r[t]];
    DBuf<int32_t> dr;
    upload(dr, r.data(), r.size(), s);
    Csr B;
    permute_csr(c, L.A, dr, (int64_t)r.size(), L.iperm, n, B);
    build_sell(c, B, L.sgs[k], 1, want32);
    L.sgs[k].perm.release();
    upload(L.sgs_pos[k], pos.data(), pos.size(), s);
  }
  MG_HIP(hipStreamSynchronize(s));
}

// The product variants (gathers in flight, padding skipped or not) the
// autotuner times for S: those the options leave open; skipping the padding
// only where the layout pads.
static std::vector<std::pair<int, int>> variants(const Ctx &c, const Sell &S) {
  std::vector<std::pair<int, int>> v;
  for (int m = 0; m < 2; ++m) {
    if (c.opt.sell_mask >= 0 ? m != c.opt.sell_mask : (m == 1 && S.stored <= S.nnz)) continue;
    for (int u : {8, 4})
      if (c.opt.sell_unroll == 0 || c.opt.sell_unroll == u) v.push_back({u, m});
  }
  return v;
}

// Lanes per row of a matrix whose layout is not timed: the fewest that give
// 4096 wavefronts (four per SIMD), as long as each lane keeps 8 entries on
// average.
static int rule_rpl(int64_t nrows, int64_t nnz) {
  const double avg = nrows ? (double)nnz / (double)nrows : 0.0;
  int r = 1;
  while (r < 8 && (nrows * r + 63) / 64 < 4096 && avg >= 8.0 * (2 * r)) r *= 2;
  return r;
}

// Keeps the fastest of 4 and 8 gathers in flight, with and (where the layout
// pads) without skipping the padding, for products y = S x (x of length nx,
// y of length ny) in the cycle's precision.
static float tune_unroll(Ctx &c, Sell &S, int64_t nx, int64_t ny, bool want32) {
  hipStream_t s = c.stream;
  hipEvent_t e0, e1;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  float best = -1;
  int best_u = 8, best_m = 0;
  const int reps = 5;
  auto timed = [&](auto *x, auto *y) {
    for (auto [u, m] : variants(c, S)) {
      S.unroll = u;
      S.mask = m;
      sell_spmv(s, S, x, y, SPMV_SET, decltype(x)(nullptr));
      // the fastest of three batches: clock and boost changes only slow a batch
      float t = -1;
      for (int batch = 0; batch < 3; ++batch) {
        MG_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) sell_spmv(s, S, x, y, SPMV_SET, decltype(x)(nullptr));
        MG_HIP(hipEventRecord(e1, s));
        MG_HIP(hipEventSynchronize(e1));
        float tb = 0;
        MG_HIP(hipEventElapsedTime(&tb, e0, e1));
        if (t < 0 || tb < t) t = tb;
      }
      if (best < 0 || t < best) {
        best = t;
        best_u = u;
        best_m = m;
      }
    }
  };
  if (want32) {
    DBuf<float> x, y;
    x.alloc(nx);
    y.alloc(ny);
    fill<float>(s, x.p, nx, 0.5f);
    timed(x.p, y.p);
  } else {
    DBuf<double> x, y;
    x.alloc(nx);
    y.alloc(ny);
    fill<double>(s, x.p, nx, 0.5);
    timed(x.p, y.p);
  }
  S.unroll = best_u;
  S.mask = best_m;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// time of the level's Chebyshev-step kernel in its current layout: the
// average launch of the fastest of three batches (clock and boost changes
// only slow a batch)
static double time_cheb(Ctx &c, Level &L, bool want32) {
  hipStream_t s = c.stream;
  const int64_t n = L.nfree;
  hipEvent_t e0, e1;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  float ms = -1;
  const int reps = 5;
  auto batch_ms = [&]() {
    float t = 0;
    MG_HIP(hipEventElapsedTime(&t, e0, e1));
    if (ms < 0 || t < ms) ms = t;
  };
  if (want32) {
    DBuf<float> v[4];
    for (auto &b : v) {
      b.alloc(n);
      fill<float>(s, b.p, n, 0.5f);
    }
    cheb_step<float>(s, L.S, L.dinv32, v[0], v[1], v[2], v[3], 0, 0.5, 0.5);
    for (int batch = 0; batch < 3; ++batch) {
      MG_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) cheb_step<float>(s, L.S, L.dinv32, v[0], v[1], v[2], v[3], 0, 0.5, 0.5);
      MG_HIP(hipEventRecord(e1, s));
      MG_HIP(hipEventSynchronize(e1));
      batch_ms();
    }
  } else {
    DBuf<double> v[4];
    for (auto &b : v) {
      b.alloc(n);
      fill<double>(s, b.p, n, 0.5);
    }
    cheb_step<double>(s, L.S, L.dinv64, v[0], v[1], v[2], v[3], 0, 0.5, 0.5);
    for (int batch = 0; batch < 3; ++batch) {
      MG_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) cheb_step<double>(s, L.S, L.dinv64, v[0], v[1], v[2], v[3], 0, 0.5, 0.5);
      MG_HIP(hipEventRecord(e1, s));
      MG_HIP(hipEventSynchronize(e1));
      batch_ms();
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

// Solve order of a level.  sigma >= 1 is used as given; sigma == 0 lets the
// autotuner choose: when the unsorted layout pads by more than 2 %, rows sorted
// inside windows of 128 and of 1024 rows are built as well and the layout whose
// Chebyshev-step kernel runs fastest on this GPU is kept (short windows cut most
// of the padding while neighbouring rows still gather neighbouring entries).
// Levels of at least 65536 unknowns time every layout with 4 and 8 gathers
// in flight per lane, with and without skipping the padding; the sorting
// window is chosen with one lane per row, and then, where rows hold at least
// 8 entries per lane on average, 2, 4 and 8 lanes per row are timed with it;
// of layouts within 2 % of the fastest the one storing the fewest entries is
// kept.  Smaller levels take no timing (their choice is the same on
// every run): the fewest lanes per row that give 4096 wavefronts (four per
// SIMD), as long as each lane keeps 8 entries on average; the long Galerkin
// rows of these levels otherwise leave most SIMDs with one wavefront or none.
void solve_order(Ctx &c, Level &L, int sigma, bool want32) {
  // the fastest of 4 and 8 gathers in flight, with and (where the layout
  // pads) without skipping the padding, for the current layout
  auto pick_unroll = [&]() {
    double best = -1;
    int best_u = 8, best_m = 0;
    for (auto [u, m] : variants(c, L.S)) {
      L.S.unroll = u;
      L.S.mask = m;
      const double t = time_cheb(c, L, want32);
      if (best < 0 || t < best) {
        best = t;
        best_u = u;
        best_m = m;
      }
    }
    L.S.unroll = best_u;
    L.S.mask = best_m;
    return best;
  };
  const bool tune = L.nfree >= 65536 && !L.coarsest;
  const double avg = L.A.nrows ? (double)L.A.nnz / (double)L.A.nrows : 0.0;
  std::vector<int> rpls;
  if (c.opt.sell_rpl) {
    rpls.push_back(c.opt.sell_rpl);
  } else if (tune) {
    rpls.push_back(1);
    for (int r : {2, 4, 8, 16, 32})
      if (avg >= 8.0 * r) rpls.push_back(r);
  } else {
    rpls.push_back(rule_rpl(L.A.nrows, L.A.nnz));
  }
  if (!tune) {
    order_with(c, L, sigma >= 1 ? sigma : 1, want32, rpls[0]);
    return;
  }
  // candidates within 2 % of the fastest count as equal (run-to-run noise of
  // these timings); among them the layout that stores the fewest entries is
  // kept, which moves the fewest bytes and makes the choice repeatable
  struct Cand {
    double t;
    int64_t stored;
    int sigma, rpl, unroll, mask;
  };
  std::vector<Cand> cands;
  int last_s = 0, last_r = 0;
  auto best_of = [&]() {
    double tmin = cands[0].t;
    for (const Cand &q : cands) tmin = std::min(tmin, q.t);
    const Cand *b = nullptr;
    for (const Cand &q : cands)
      if (q.t <= 1.02 * tmin && (!b || q.stored < b->stored)) b = &q;
    return *b;
  };
  auto consider = [&](int sg, int r) {
    order_with(c, L, sg, want32, r);
    last_s = sg;
    last_r = r;
    const double t = pick_unroll();
    cands.push_back({t, L.S.stored, sg, r, L.S.unroll, L.S.mask});
  };
  // the sorting window with the first lanes-per-row candidate, then the other
  // candidates with the best window found (each layout build streams the
  // whole operator, so not every pair is built)
  consider(sigma >= 1 ? sigma : 1, rpls[0]);
  if (sigma == 0 && (double)L.S.stored > 1.02 * (double)L.A.nnz)
    for (int cand : {128, 1024}) consider(cand, rpls[0]);
  const int sbest = best_of().sigma;
  for (size_t q = 1; q < rpls.size(); ++q) consider(sbest, rpls[q]);
  const Cand b = best_of();
  if (b.sigma != last_s || b.rpl != last_r) order_with(c, L, b.sigma, want32, b.rpl);
  L.S.unroll = b.unroll;
  L.S.mask = b.mask;
}

// ---------------------------------------------------------------------------
// ELL (row-major, -1 = empty) -> CSR, and its transpose
// ---------------------------------------------------------------------------
__global__ void k_ell_keys(const int32_t *col, const double *val, int64_t nrows, int width, uint64_t ncols,
                           int transpose, uint64_t nr_out, uint64_t sentinel, uint64_t *keys, double *vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * width) return;
  int64_t r = t / width;
  int32_t cc = col[t];
  if (cc < 0) {
    keys[t] = sentinel;
  } else {
    keys[t] = transpose ? (uint64_t)cc * (uint64_t)nrows + (uint64_t)r : (uint64_t)r * ncols + (uint64_t)cc;
  }
  vals[t] = val[t];
  (void)nr_out;
}

__global__ void k_ell_permute(const int32_t *col, const double *val, int64_t nrows, int width,
                              const int32_t *perm_rows, const int32_t *iperm_cols, int32_t *col2, double *val2) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * width) return;
  int64_t p = t / width;
  int j = (int)(t - p * width);
  int64_t src = (int64_t)perm_rows[p] * width + j;
  int32_t cc = col[src];
  col2[t] = cc >= 0 ? iperm_cols[cc] : -1;
  val2[t] = val[src];
}

void ell_to_csr(Ctx &c, int64_t nrows, int64_t ncols, int width, const int32_t *col, const double *val,
                bool transpose, Csr &A);

// P and R = P^T of the transfer between fine level F and coarse level C, in the
// two levels' solve orders
void build_transfer_sell(Ctx &c, Level &F, const Level &C, bool want32) {
  hipStream_t s = c.stream;
  int64_t n = F.nfree * F.pw;
  DBuf<int32_t> col;
  DBuf<double> val;
  col.alloc(n);
  val.alloc(n);
  k_ell_permute<<<grid_for(n, 256), 256, 0, s>>>(F.pcol, F.pval, F.nfree, F.pw, F.perm, C.iperm, col, val);
  MG_LAUNCH_CHECK();
  Csr Pp, Rp;
  ell_to_csr(c, F.nfree, C.nfree, F.pw, col, val, false, Pp);
  ell_to_csr(c, F.nfree, C.nfree, F.pw, col, val, true, Rp);
  // P: at most one entry per coarse basis function of a cell, one lane per
  // row; R = P^T: a coarse row gathers every fine node of its support, and
  // takes lanes per row like the level operators (timed where the fine level
  // has at least 65536 unknowns, else by rule_rpl)
  build_sell(c, Pp, F.P, 1, want32);
  const bool timing = F.nfree >= 65536;
  if (timing) tune_unroll(c, F.P, C.nfree, F.nfree, want32);
  if (!timing || c.opt.sell_rpl) {
    build_sell(c, Rp, F.R, 1, want32, c.opt.sell_rpl ? std::min(c.opt.sell_rpl, 8) : rule_rpl(Rp.nrows, Rp.nnz));
    if (timing) tune_unroll(c, F.R, F.nfree, C.nfree, want32);
    return;
  }
  const double avg = Rp.nrows ? (double)Rp.nnz / (double)Rp.nrows : 0.0;
  float best = -1;
  int best_r = 1;
  for (int r : {1, 2, 4, 8}) {
    if (r > 1 && avg < 8.0 * r) break;
    build_sell(c, Rp, F.R, 1, want32, r);
    const float t = tune_unroll(c, F.R, F.nfree, C.nfree, want32);
    if (best < 0 || t < best) {
      best = t;
      best_r = r;
    }
  }
  if (F.R.rpl != best_r) {
    build_sell(c, Rp, F.R, 1, want32, best_r);
    tune_unroll(c, F.R, F.nfree, C.nfree, want32);
  }
}

void ell_to_csr(Ctx &c, int64_t nrows, int64_t ncols, int width, const int32_t *col, const double *val,
                bool transpose, Csr &A) {
  hipStream_t s = c.stream;
  int64_t n = nrows * width;
  uint64_t sentinel = (uint64_t)nrows * (uint64_t)ncols;
  DBuf<uint64_t> keys;
  DBuf<double> vals;
  keys.alloc(n);
  vals.alloc(n);
  k_ell_keys<<<grid_for(n, 256), 256, 0, s>>>(col, val, nrows, width, (uint64_t)ncols, transpose ? 1 : 0,
                                             transpose ? ncols : nrows, sentinel, keys, vals);
  MG_LAUNCH_CHECK();
  if (transpose)
    assemble_pairs(s, keys, vals, n, sentinel, ncols, nrows, A);
  else
    assemble_pairs(s, keys, vals, n, sentinel, nrows, ncols, A);
}

}  // namespace mg

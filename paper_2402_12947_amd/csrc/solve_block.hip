// Block solve kernels: K right-hand sides of one operator advanced together.
//
// Every solve-phase step of the method is bound by the bandwidth of the
// operator's stream (SELL values and column indices, patch rows, transfer
// operators), so K systems that share the operator are solved with block
// vectors: unknown i of column q sits at index i K + q, one gather of a row
// fetches all K columns, and each matrix entry read from HBM is used K times.
// The arithmetic of each column is that of the single-vector kernels of
// solve.hip (the same recurrences, per column); only the summation order of a
// row product may differ when a gather is 32 bytes wide (FP64, K = 4).
// K is 2 or 4.
#include "mg_internal.h"
#include "sell_row.h"

namespace mg {

template <class T, int K>
using Row = BlockRow<T, K>;

template <class T, int K>
__device__ inline Row<T, K> ld(const T *p, int64_t i) {
  return reinterpret_cast<const Row<T, K> *>(p)[i];
}
template <class T, int K>
__device__ inline void st(T *p, int64_t i, const Row<T, K> &v) {
  reinterpret_cast<Row<T, K> *>(p)[i] = v;
}

// ---------------------------------------------------------------------------
// sparse products
// ---------------------------------------------------------------------------
template <class T, int K, int MODE>
__global__ __launch_bounds__(256) void k_spmv_k(int64_t nslices, int64_t nrows, SellCols cols,
                                                const T *__restrict__ val, const T *__restrict__ x,
                                                T *__restrict__ y, const T *__restrict__ b) {
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = pos >> 6;
  if (sl >= nslices) return;
  T acc[K];
  sell_row_k<T, K>(cols, val, x, sl, (int)(pos & 63), acc);
  const SellRow rw = sell_row_of(cols, pos);
  const int64_t i = rw.row;
  if (!rw.lead || i >= nrows) return;
  Row<T, K> o;
  if (MODE == SPMV_ADD) o = ld<T, K>(y, i);
  if (MODE == SPMV_RESID) o = ld<T, K>(b, i);
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (MODE == SPMV_SET) o.v[q] = acc[q];
    else if (MODE == SPMV_ADD) o.v[q] += acc[q];
    else o.v[q] -= acc[q];
  }
  st<T, K>(y, i, o);
}

template <class T, int K>
static void spmv_k(hipStream_t s, const Sell &S, const T *x, T *y, int mode, const T *b) {
  const unsigned g = sell_grid(S);
  const T *v = sell_vals<T>(S);
  if (mode == SPMV_SET) k_spmv_k<T, K, SPMV_SET><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, x, y, b);
  else if (mode == SPMV_ADD) k_spmv_k<T, K, SPMV_ADD><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, x, y, b);
  else k_spmv_k<T, K, SPMV_RESID><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, x, y, b);
  MG_LAUNCH_CHECK();
}

template <class T>
void sell_spmv_block(hipStream_t s, const Sell &S, int K, const T *x, T *y, int mode, const T *b) {
  if (S.nslices == 0) return;
  if (K == 2) spmv_k<T, 2>(s, S, x, y, mode, b);
  else if (K == 4) spmv_k<T, 4>(s, S, x, y, mode, b);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
}
template void sell_spmv_block<double>(hipStream_t, const Sell &, int, const double *, double *, int, const double *);
template void sell_spmv_block<float>(hipStream_t, const Sell &, int, const float *, float *, int, const float *);

// ---------------------------------------------------------------------------
// Chebyshev-Jacobi step per column: r = D^-1 (b - A x), d = c_d d + c_r r,
// x' = x + d (flags: 1 first step, 2 last step, as in cheb_step)
// ---------------------------------------------------------------------------
template <class T, int K, int FLAGS>
__global__ __launch_bounds__(256) void k_cheb_k(int64_t nslices, int64_t nrows, SellCols cols,
                                                const T *__restrict__ val, const T *__restrict__ dinv,
                                                const T *__restrict__ b, const T *__restrict__ x,
                                                T *__restrict__ xout, T *__restrict__ d, T c_d, T c_r) {
  // the update as written: no fused multiply-add across these statements, so
  // every variant of the step rounds identically
  #pragma clang fp contract(off)
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = pos >> 6;
  if (sl >= nslices) return;
  T acc[K];
  sell_row_k<T, K>(cols, val, x, sl, (int)(pos & 63), acc);
  const SellRow rw = sell_row_of(cols, pos);
  const int64_t i = rw.row;
  if (!rw.lead || i >= nrows) return;
  const T dv = dinv[i];
  const Row<T, K> bb = ld<T, K>(b, i), xx = ld<T, K>(x, i);
  Row<T, K> dd;
  if (!(FLAGS & 1)) dd = ld<T, K>(d, i);
  Row<T, K> dn, xo;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const T r = dv * (bb.v[q] - acc[q]);
    dn.v[q] = (FLAGS & 1) ? c_r * r : c_d * dd.v[q] + c_r * r;
    xo.v[q] = xx.v[q] + dn.v[q];
  }
  if (!(FLAGS & 2)) st<T, K>(d, i, dn);
  st<T, K>(xout, i, xo);
}

template <class T, int K>
static void cheb_k(hipStream_t s, const Sell &S, const T *dinv, const T *b, const T *x, T *xout, T *d, int flags,
                   T c_d, T c_r) {
  const unsigned g = sell_grid(S);
  const T *v = sell_vals<T>(S);
  switch (flags) {
    case 1: k_cheb_k<T, K, 1><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, dinv, b, x, xout, d, c_d, c_r); break;
    case 2: k_cheb_k<T, K, 2><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, dinv, b, x, xout, d, c_d, c_r); break;
    case 3: k_cheb_k<T, K, 3><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, dinv, b, x, xout, d, c_d, c_r); break;
    default: k_cheb_k<T, K, 0><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, dinv, b, x, xout, d, c_d, c_r);
  }
  MG_LAUNCH_CHECK();
}

template <class T>
void cheb_step_block(hipStream_t s, const Sell &S, int K, const T *dinv, const T *b, const T *x, T *xout, T *d,
                     int flags, double c_d, double c_r) {
  if (S.nslices == 0) return;
  if (K == 2) cheb_k<T, 2>(s, S, dinv, b, x, xout, d, flags, (T)c_d, (T)c_r);
  else if (K == 4) cheb_k<T, 4>(s, S, dinv, b, x, xout, d, flags, (T)c_d, (T)c_r);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
}
template void cheb_step_block<double>(hipStream_t, const Sell &, int, const double *, const double *, const double *,
                                      double *, double *, int, double, double);
template void cheb_step_block<float>(hipStream_t, const Sell &, int, const float *, const float *, const float *,
                                     float *, float *, int, double, double);

// The first step from an x that vanishes outside the rows coupled to the patch
// DOFs (cheb_step_zero, per column).
template <class T, int K>
__global__ __launch_bounds__(256) void k_cheb_zero_k(int64_t n, const T *__restrict__ dinv, const T *__restrict__ b,
                                                     const T *__restrict__ x, T *__restrict__ xout,
                                                     T *__restrict__ d, T c_r) {
  // the update as written: no fused multiply-add across these statements, so
  // every variant of the step rounds identically
  #pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const T dv = dinv[i];
  const Row<T, K> bb = ld<T, K>(b, i);
  Row<T, K> xx;
  if (x) xx = ld<T, K>(x, i);
  Row<T, K> dn, xo;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const T r = dv * bb.v[q];
    dn.v[q] = c_r * r;
    xo.v[q] = x ? xx.v[q] + dn.v[q] : dn.v[q];
  }
  if (d) st<T, K>(d, i, dn);
  st<T, K>(xout, i, xo);
}

template <class T, int K>
__global__ __launch_bounds__(256) void k_cheb_fix_k(int64_t nslices, int64_t nrows, SellCols cols,
                                                    const T *__restrict__ val, const int32_t *__restrict__ pos,
                                                    const T *__restrict__ dinv, const T *__restrict__ b,
                                                    const T *__restrict__ x, T *__restrict__ xout,
                                                    T *__restrict__ d, T c_r) {
  // the update as written: no fused multiply-add across these statements, so
  // every variant of the step rounds identically
  #pragma clang fp contract(off)
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = k >> 6;
  if (sl >= nslices) return;
  T acc[K];
  sell_row_k<T, K>(cols, val, x, sl, (int)(k & 63), acc);
  const SellRow rw = sell_row_of(cols, k);
  if (!rw.lead || rw.row >= nrows) return;
  const int32_t p = pos[rw.row];
  const T dv = dinv[p];
  const Row<T, K> bb = ld<T, K>(b, p), xx = ld<T, K>(x, p);
  Row<T, K> dn, xo;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const T r = dv * (bb.v[q] - acc[q]);
    dn.v[q] = c_r * r;
    xo.v[q] = xx.v[q] + dn.v[q];
  }
  if (d) st<T, K>(d, p, dn);
  st<T, K>(xout, p, xo);
}

template <class T, int K>
static void cheb_zero_k(hipStream_t s, int64_t n, const Sell *nbr, const int32_t *nbr_pos, const T *dinv, const T *b,
                        const T *x, T *xout, T *d, T c_r) {
  k_cheb_zero_k<T, K><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, dinv, b, nbr ? x : nullptr, xout, d, c_r);
  MG_LAUNCH_CHECK();
  if (!nbr || nbr->nslices == 0) return;
  k_cheb_fix_k<T, K><<<sell_grid(*nbr), 256, 0, s>>>(nbr->nslices, nbr->nrows, cols_of(*nbr), sell_vals<T>(*nbr),
                                                     nbr_pos, dinv, b, x, xout, d, c_r);
  MG_LAUNCH_CHECK();
}

template <class T>
void cheb_step_zero_block(hipStream_t s, int64_t n, int K, const Sell *nbr, const int32_t *nbr_pos, const T *dinv,
                          const T *b, const T *x, T *xout, T *d, double c_r) {
  if (n <= 0) return;
  if (K == 2) cheb_zero_k<T, 2>(s, n, nbr, nbr_pos, dinv, b, x, xout, d, (T)c_r);
  else if (K == 4) cheb_zero_k<T, 4>(s, n, nbr, nbr_pos, dinv, b, x, xout, d, (T)c_r);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
}
template void cheb_step_zero_block<double>(hipStream_t, int64_t, int, const Sell *, const int32_t *, const double *,
                                           const double *, const double *, double *, double *, double);
template void cheb_step_zero_block<float>(hipStream_t, int64_t, int, const Sell *, const int32_t *, const float *,
                                          const float *, const float *, float *, float *, double);

// ---------------------------------------------------------------------------
// one colour of multicolour Gauss-Seidel, per column (rows of a colour are
// not coupled, so the update in place is race-free)
// ---------------------------------------------------------------------------
template <class T, int K>
__global__ __launch_bounds__(256) void k_sgs_k(int64_t nslices, int64_t nrows, SellCols cols,
                                               const T *__restrict__ val, const int32_t *__restrict__ pos,
                                               const T *__restrict__ dinv, const T *__restrict__ b,
                                               T *__restrict__ u) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = k >> 6;
  if (sl >= nslices) return;
  T acc[K];
  sell_row_k<T, K>(cols, val, u, sl, (int)(k & 63), acc);
  const SellRow rw = sell_row_of(cols, k);
  if (!rw.lead || rw.row >= nrows) return;
  const int32_t r = pos[rw.row];
  const T dv = dinv[r];
  const Row<T, K> bb = ld<T, K>(b, r);
  Row<T, K> uu = ld<T, K>(u, r);
#pragma unroll
  for (int q = 0; q < K; ++q) uu.v[q] += dv * (bb.v[q] - acc[q]);
  st<T, K>(u, r, uu);
}

template <class T>
void sgs_colour_sweep_block(hipStream_t s, const Sell &S, int K, const int32_t *pos, const T *dinv, const T *b,
                            T *u) {
  if (S.nslices == 0) return;
  const unsigned g = sell_grid(S);
  if (K == 2) k_sgs_k<T, 2><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), sell_vals<T>(S), pos, dinv, b, u);
  else if (K == 4) k_sgs_k<T, 4><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), sell_vals<T>(S), pos, dinv, b, u);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
  MG_LAUNCH_CHECK();
}
template void sgs_colour_sweep_block<double>(hipStream_t, const Sell &, int, const int32_t *, const double *,
                                             const double *, double *);
template void sgs_colour_sweep_block<float>(hipStream_t, const Sell &, int, const int32_t *, const float *,
                                            const float *, float *);

// ---------------------------------------------------------------------------
// local correction: residuals of one colour's patch rows, all columns at once
// (res is a block vector over the patch DOFs in kernel order)
// ---------------------------------------------------------------------------
template <class T, int K>
__global__ __launch_bounds__(256) void k_patch_residual_k(int64_t k0, int64_t k1, SellCols cols,
                                                          const T *__restrict__ val,
                                                          const int32_t *__restrict__ dofs,
                                                          const T *__restrict__ b, const T *__restrict__ u,
                                                          T *__restrict__ res) {
  const int rps = 64 / cols.rpl;
  const int64_t pos = k0 / rps * 64 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if ((pos >> 6) > (k1 - 1) / rps) return;
  T acc[K];
  sell_row_k<T, K>(cols, val, u, pos >> 6, (int)(pos & 63), acc);
  const SellRow rw = sell_row_of(cols, pos);
  const int64_t k = rw.row;
  if (!rw.lead || k < k0 || k >= k1) return;
  Row<T, K> o = ld<T, K>(b, dofs[k]);
#pragma unroll
  for (int q = 0; q < K; ++q) o.v[q] -= acc[q];
  st<T, K>(res, k, o);
}

template <class T>
void patch_residual_block(hipStream_t s, const Patches &pt, int colour, int K, const T *b, const T *u, T *res) {
  const int p0 = pt.colour_first[colour], p1 = pt.colour_first[colour + 1];
  const int64_t k0 = pt.h_kptr[p0], k1 = pt.h_kptr[p1];
  if (k1 <= k0) return;
  const int64_t rps = 64 / pt.rows.rpl;
  const int64_t span = ((k1 - 1) / rps - k0 / rps + 1) * 64;
  const unsigned g = (unsigned)((span + 255) / 256);
  const T *v = sell_vals<T>(pt.rows);
  if (K == 2) k_patch_residual_k<T, 2><<<g, 256, 0, s>>>(k0, k1, cols_of(pt.rows), v, pt.dofs, b, u, res);
  else if (K == 4) k_patch_residual_k<T, 4><<<g, 256, 0, s>>>(k0, k1, cols_of(pt.rows), v, pt.dofs, b, u, res);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
  MG_LAUNCH_CHECK();
}
template void patch_residual_block<double>(hipStream_t, const Patches &, int, int, const double *, const double *,
                                           double *);
template void patch_residual_block<float>(hipStream_t, const Patches &, int, int, const float *, const float *,
                                          float *);

// ---------------------------------------------------------------------------
// block CG (FP64).  Device scalars are laid out scal[slot K + q] with the
// slots of the single-vector CG: 0 rho = r.z, 1 p.q, 2 alpha, 3 r.r,
// 4 rho_new, 5 beta, 6 breakdown flag, 7 b.b.  Partial sums: part[block K + q].
// Columns outside `mask` (converged, or a zero right-hand side) take
// alpha = beta = 0: their x and r no longer change.
// ---------------------------------------------------------------------------
template <int K>
__device__ inline void block_sums_out(const double (&v)[K], double *part) {
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double t = block_sum(v[q]);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * K + q] = t;
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_spmv_dot_k(int64_t nslices, int64_t nrows, SellCols cols,
                                                    const double *__restrict__ val, const double *__restrict__ p,
                                                    double *__restrict__ qv, double *__restrict__ part) {
  const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = pos >> 6;
  double contrib[K];
#pragma unroll
  for (int q = 0; q < K; ++q) contrib[q] = 0;
  if (sl < nslices) {
    double acc[K];
    sell_row_k<double, K>(cols, val, p, sl, (int)(pos & 63), acc);
    const SellRow rw = sell_row_of(cols, pos);
    if (rw.lead && rw.row < nrows) {
      const Row<double, K> pp = ld<double, K>(p, rw.row);
      Row<double, K> o;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        o.v[q] = acc[q];
        contrib[q] = acc[q] * pp.v[q];
      }
      st<double, K>(qv, rw.row, o);
    }
  }
  block_sums_out<K>(contrib, part);
}

void spmv_dot_block(hipStream_t s, const Sell &S, int K, const double *p, double *q, double *part) {
  const unsigned g = sell_grid(S);
  if (K == 2) k_spmv_dot_k<2><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), S.v64, p, q, part);
  else if (K == 4) k_spmv_dot_k<4><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), S.v64, p, q, part);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
  MG_LAUNCH_CHECK();
}

template <int K>
__global__ __launch_bounds__(256) void k_dot_k(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
                                               double *__restrict__ part) {
  double s[K];
#pragma unroll
  for (int q = 0; q < K; ++q) s[q] = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const Row<double, K> a = ld<double, K>(x, i), b = ld<double, K>(y, i);
#pragma unroll
    for (int q = 0; q < K; ++q) s[q] += a.v[q] * b.v[q];
  }
  block_sums_out<K>(s, part);
}

void dot_partials_block(hipStream_t s, int K, const double *x, const double *y, int64_t n, double *part,
                        int nblocks) {
  if (K == 2) k_dot_k<2><<<nblocks, 256, 0, s>>>(x, y, n, part);
  else if (K == 4) k_dot_k<4><<<nblocks, 256, 0, s>>>(x, y, n, part);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
  MG_LAUNCH_CHECK();
}

// one workgroup per column sums that column's partials in a fixed order
__global__ __launch_bounds__(256) void k_finish_k(const double *__restrict__ part, int nb, int K,
                                                  double *__restrict__ out) {
  const int q = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[(int64_t)i * K + q];
  s = block_sum(s);
  if (threadIdx.x == 0) out[q] = s;
}

void finish_sum_block(hipStream_t s, int K, const double *part, int nblocks, double *out) {
  k_finish_k<<<K, 256, 0, s>>>(part, nblocks, K, out);
  MG_LAUNCH_CHECK();
}

// scal[8 K + q] != 0: column q is still active; a frozen column gets
// alpha = beta = 0 (its x and r stay, p = z)
__global__ void k_cg_alpha_k(double *scal, int K) {
  const int q = threadIdx.x;
  if (q >= K) return;
  if (scal[8 * K + q] == 0.0) {
    scal[2 * K + q] = 0.0;
    return;
  }
  const double pq = scal[K + q];
  const bool bad = !(pq > 0.0) || !isfinite(pq) || !isfinite(scal[q]);
  scal[2 * K + q] = bad ? 0.0 : scal[q] / pq;
  if (bad) scal[6 * K + q] = 1.0;
}
void cg_alpha_block(hipStream_t s, int K, double *scal) {
  k_cg_alpha_k<<<1, 64, 0, s>>>(scal, K);
  MG_LAUNCH_CHECK();
}

template <int K>
__global__ __launch_bounds__(256) void k_cg_xr_k(double *__restrict__ x, double *__restrict__ r,
                                                 const double *__restrict__ p, const double *__restrict__ qv,
                                                 const double *__restrict__ scal, int64_t n,
                                                 double *__restrict__ part) {
  double a[K], s[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    a[q] = scal[2 * K + q];
    s[q] = 0;
  }
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    Row<double, K> xx = ld<double, K>(x, i), rr = ld<double, K>(r, i);
    const Row<double, K> pp = ld<double, K>(p, i), qq = ld<double, K>(qv, i);
#pragma unroll
    for (int q = 0; q < K; ++q) {
      xx.v[q] += a[q] * pp.v[q];
      rr.v[q] -= a[q] * qq.v[q];
      s[q] += rr.v[q] * rr.v[q];
    }
    st<double, K>(x, i, xx);
    st<double, K>(r, i, rr);
  }
  block_sums_out<K>(s, part);
}

void cg_update_xr_block(hipStream_t s, int K, double *x, double *r, const double *p, const double *q,
                        const double *scal, int64_t n, double *part, int nblocks) {
  if (K == 2) k_cg_xr_k<2><<<nblocks, 256, 0, s>>>(x, r, p, q, scal, n, part);
  else if (K == 4) k_cg_xr_k<4><<<nblocks, 256, 0, s>>>(x, r, p, q, scal, n, part);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
  MG_LAUNCH_CHECK();
}

__global__ void k_cg_beta_k(double *scal, int K) {
  const int q = threadIdx.x;
  if (q >= K) return;
  if (scal[8 * K + q] == 0.0) {
    scal[5 * K + q] = 0.0;
    return;
  }
  const double rn = scal[4 * K + q];
  const bool bad = !isfinite(rn) || scal[q] == 0.0;
  scal[5 * K + q] = bad ? 0.0 : rn / scal[q];
  scal[q] = rn;
  if (bad) scal[6 * K + q] = 1.0;
}
void cg_beta_block(hipStream_t s, int K, double *scal) {
  k_cg_beta_k<<<1, 64, 0, s>>>(scal, K);
  MG_LAUNCH_CHECK();
}

__global__ void k_cg_active_k(double *scal, int K, unsigned mask) {
  const int q = threadIdx.x;
  if (q < K) scal[8 * K + q] = ((mask >> q) & 1u) ? 1.0 : 0.0;
}
void cg_active_block(hipStream_t s, int K, unsigned mask, double *scal) {
  k_cg_active_k<<<1, 64, 0, s>>>(scal, K, mask);
  MG_LAUNCH_CHECK();
}

template <int K>
__global__ void k_cg_p_k(double *__restrict__ p, const double *__restrict__ z, const double *__restrict__ scal,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Row<double, K> pp = ld<double, K>(p, i);
  const Row<double, K> zz = ld<double, K>(z, i);
#pragma unroll
  for (int q = 0; q < K; ++q) pp.v[q] = zz.v[q] + scal[5 * K + q] * pp.v[q];
  st<double, K>(p, i, pp);
}
void cg_update_p_block(hipStream_t s, int K, double *p, const double *z, const double *scal, int64_t n) {
  if (n <= 0) return;
  const unsigned g = (unsigned)((n + 255) / 256);
  if (K == 2) k_cg_p_k<2><<<g, 256, 0, s>>>(p, z, scal, n);
  else if (K == 4) k_cg_p_k<4><<<g, 256, 0, s>>>(p, z, scal, n);
  else fail(MG_ERR_ARG, "block width %d is not 2 or 4", K);
  MG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// K separate canonical-order vectors <-> one solve-order block vector; a NULL
// column reads as zero and is not written back
// ---------------------------------------------------------------------------
struct ColIn {
  const double *p[MG_BLOCK_MAX];
};
struct ColOut {
  double *p[MG_BLOCK_MAX];
};

__global__ void k_gather_block(ColIn x, int K, const int32_t *__restrict__ perm, double *__restrict__ y,
                               int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t src = perm[i];
#pragma unroll
  for (int q = 0; q < MG_BLOCK_MAX; ++q)
    if (q < K) y[i * K + q] = x.p[q] ? x.p[q][src] : 0.0;
}

__global__ void k_scatter_block(const double *__restrict__ y, int K, const int32_t *__restrict__ perm, ColOut o,
                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t dst = perm[i];
#pragma unroll
  for (int q = 0; q < MG_BLOCK_MAX; ++q)
    if (q < K && o.p[q]) o.p[q][dst] = y[i * K + q];
}

void gather_block(hipStream_t s, int K, const double *const *cols, const int32_t *perm, double *y, int64_t n) {
  if (n <= 0) return;
  if (K < 1 || K > MG_BLOCK_MAX) fail(MG_ERR_ARG, "block width %d out of range", K);
  ColIn in{};
  for (int q = 0; q < K; ++q) in.p[q] = cols[q];
  k_gather_block<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, K, perm, y, n);
  MG_LAUNCH_CHECK();
}

void scatter_block(hipStream_t s, int K, const double *y, const int32_t *perm, double *const *cols, int64_t n) {
  if (n <= 0) return;
  if (K < 1 || K > MG_BLOCK_MAX) fail(MG_ERR_ARG, "block width %d out of range", K);
  ColOut out{};
  for (int q = 0; q < K; ++q) out.p[q] = cols[q];
  k_scatter_block<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y, K, perm, out, n);
  MG_LAUNCH_CHECK();
}

}  // namespace mg

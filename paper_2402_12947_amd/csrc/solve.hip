// Solve-phase kernels: the hot path of every V-cycle and CG iteration.
//
// * SELL-C sparse products (C = 64, one wavefront lane per row): the column
//   indices and values of the 64 rows of a slice are read as contiguous
//   256/512-byte lines (non-temporal: they are streamed once), the source
//   vector is gathered, 4 or 8 gathers in flight per lane (Sell::unroll,
//   chosen per level by timing; with 4 the kernel needs half the registers
//   and keeps 8 wavefronts per SIMD resident instead of 6), with or without
//   skipping each row's padding (Sell::mask, also chosen by timing).  Blocks
//   keep the hardware's round-robin spread over the 8 XCDs: renumbering them
//   into one contiguous slice range per XCD was measured 1.6x slower on this
//   kernel, into interleaved chunks of 1 to 1024 blocks per XCD no faster
//   (within the run-to-run spread, FP32 and FP64, levels 0 to 2 of the 3D P2
//   cube), and chunks that leave each XCD only a few runs slower again.
// * The Chebyshev-Jacobi step of the global smoother S_g (paper Sec. 3.2,
//   Sec. 5; classical Chebyshev acceleration on D^-1 A) is one fused pass:
//   r = D^-1 (b - A x), d = c_d d + c_r r, x' = x + d.
// * Local correction S_c (Sec. 4.1): patch-row residuals, then one workgroup
//   per patch applies the precomputed inverse of A^[d] (dense product) and
//   adds the correction to its own DOFs; patches of one colour share no DOF.
// * Coarsest level: dense product with the precomputed inverse (FP64).
// * CG vector updates and deterministic two-stage inner products.
#include "mg_internal.h"
#include "sell_row.h"

namespace mg {

// Unknowns are numbered in the operator's row order (solve order): the row of
// a SELL position is the position itself with one lane per row, position
// 64 s + l holds row s 64 / rpl + l / rpl with rpl lanes per row; rows past
// nrows are padding.
template <class T, int MODE, int U, bool M>
__global__ __launch_bounds__(256) void k_sell_spmv(
    int64_t nslices, int64_t nrows, SellCols cols, const T *__restrict__ val, const T *__restrict__ x,
    T *__restrict__ y, const T *__restrict__ b) {
  int64_t blk = blockIdx.x;
  int64_t pos = blk * 256 + threadIdx.x;
  int64_t sl = pos >> 6;
  if (sl >= nslices) return;
  T acc = sell_row<T, U, M>(cols, val, x, sl, (int)(pos & 63));
  const SellRow rw = sell_row_of(cols, pos);
  const int64_t i = rw.row;
  if (!rw.lead || i >= nrows) return;
  if (MODE == SPMV_SET) y[i] = acc;
  else if (MODE == SPMV_ADD) y[i] += acc;
  else y[i] = b[i] - acc;
}

template <class T, int U, bool M>
static void sell_spmv_u(hipStream_t s, const Sell &S, const T *x, T *y, int mode, const T *b) {
  const T *v = sell_vals<T>(S);
  unsigned g = sell_grid(S);
  if (mode == SPMV_SET)
    k_sell_spmv<T, SPMV_SET, U, M><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, x, y, b);
  else if (mode == SPMV_ADD)
    k_sell_spmv<T, SPMV_ADD, U, M><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, x, y, b);
  else
    k_sell_spmv<T, SPMV_RESID, U, M><<<g, 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), v, x, y, b);
  MG_LAUNCH_CHECK();
}

template <class T>
void sell_spmv(hipStream_t s, const Sell &S, const T *x, T *y, int mode, const T *b) {
  if (S.nslices == 0) return;
  if (S.unroll == 4) {
    if (S.mask) sell_spmv_u<T, 4, true>(s, S, x, y, mode, b);
    else sell_spmv_u<T, 4, false>(s, S, x, y, mode, b);
  } else {
    if (S.mask) sell_spmv_u<T, 8, true>(s, S, x, y, mode, b);
    else sell_spmv_u<T, 8, false>(s, S, x, y, mode, b);
  }
}
template void sell_spmv<double>(hipStream_t, const Sell &, const double *, double *, int, const double *);
template void sell_spmv<float>(hipStream_t, const Sell &, const float *, float *, int, const float *);

// ---------------------------------------------------------------------------
// Chebyshev-Jacobi step
// ---------------------------------------------------------------------------
template <class T, int FIRST, int U, bool M>
__global__ __launch_bounds__(256) void k_cheb(
    int64_t nslices, int64_t nrows, SellCols cols, const T *__restrict__ val, const T *__restrict__ dinv,
    const T *__restrict__ b, const T *__restrict__ x, T *__restrict__ xout, T *__restrict__ d, T c_d, T c_r) {
  // the update as written: no fused multiply-add across these statements, so
  // every variant of the step rounds identically
  #pragma clang fp contract(off)
  int64_t blk = blockIdx.x;
  int64_t pos = blk * 256 + threadIdx.x;
  int64_t sl = pos >> 6;
  if (sl >= nslices) return;
  T acc = sell_row<T, U, M>(cols, val, x, sl, (int)(pos & 63));
  const SellRow rw = sell_row_of(cols, pos);
  const int64_t i = rw.row;
  if (!rw.lead || i >= nrows) return;
  T r = dinv[i] * (b[i] - acc);
  T dn = (FIRST & 1) ? c_r * r : c_d * d[i] + c_r * r;
  if (!(FIRST & 2)) d[i] = dn;  // the last step of a polynomial needs no direction
  xout[i] = x[i] + dn;
}

template <class T, int U, bool M>
static void cheb_step_u(hipStream_t s, const Sell &S, const T *dinv, const T *b, const T *x, T *xout, T *d,
                        int first, T c_d, T c_r) {
  const T *v = sell_vals<T>(S);
  const unsigned g = sell_grid(S);
  const SellCols cs = cols_of(S);
  switch (first) {
    case 1: k_cheb<T, 1, U, M><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, v, dinv, b, x, xout, d, c_d, c_r); break;
    case 2: k_cheb<T, 2, U, M><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, v, dinv, b, x, xout, d, c_d, c_r); break;
    case 3: k_cheb<T, 3, U, M><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, v, dinv, b, x, xout, d, c_d, c_r); break;
    default: k_cheb<T, 0, U, M><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, v, dinv, b, x, xout, d, c_d, c_r);
  }
  MG_LAUNCH_CHECK();
}

template <class T>
void cheb_step(hipStream_t s, const Sell &S, const T *dinv, const T *b, const T *x, T *xout, T *d, int first,
               double c_d, double c_r) {
  if (S.unroll == 4) {
    if (S.mask) cheb_step_u<T, 4, true>(s, S, dinv, b, x, xout, d, first, (T)c_d, (T)c_r);
    else cheb_step_u<T, 4, false>(s, S, dinv, b, x, xout, d, first, (T)c_d, (T)c_r);
  } else {
    if (S.mask) cheb_step_u<T, 8, true>(s, S, dinv, b, x, xout, d, first, (T)c_d, (T)c_r);
    else cheb_step_u<T, 8, false>(s, S, dinv, b, x, xout, d, first, (T)c_d, (T)c_r);
  }
}
template void cheb_step<double>(hipStream_t, const Sell &, const double *, const double *, const double *, double *,
                                double *, int, double, double);
template void cheb_step<float>(hipStream_t, const Sell &, const float *, const float *, const float *, float *,
                               float *, int, double, double);

// First step from an x that vanishes outside the rows coupled to the patch
// DOFs: (A x)_i = 0 on every other row, where the step reduces to
// d = c_r D^-1 b, x' = x + d (the same operations as k_cheb with a zero row
// product); the coupled rows are then recomputed in full from their SELL.
template <class T>
__global__ __launch_bounds__(256) void k_cheb_zero(int64_t n, const T *__restrict__ dinv, const T *__restrict__ b,
                                                   const T *__restrict__ x, T *__restrict__ xout, T *__restrict__ d,
                                                   T c_r) {
  // the update as written: no fused multiply-add across these statements, so
  // every variant of the step rounds identically
  #pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const T r = dinv[i] * b[i];
  const T dn = c_r * r;
  if (d) d[i] = dn;
  xout[i] = x ? x[i] + dn : dn;
}

template <class T, int U>
__global__ __launch_bounds__(256) void k_cheb_fix(int64_t nslices, int64_t nrows, SellCols cols,
                                                  const T *__restrict__ val, const int32_t *__restrict__ pos,
                                                  const T *__restrict__ dinv, const T *__restrict__ b,
                                                  const T *__restrict__ x, T *__restrict__ xout, T *__restrict__ d,
                                                  T c_r) {
  // the update as written: no fused multiply-add across these statements, so
  // every variant of the step rounds identically
  #pragma clang fp contract(off)
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = k >> 6;
  if (sl >= nslices) return;
  const T acc = sell_row<T, U>(cols, val, x, sl, (int)(k & 63));
  const SellRow rw = sell_row_of(cols, k);
  if (!rw.lead || rw.row >= nrows) return;
  const int32_t p = pos[rw.row];
  const T r = dinv[p] * (b[p] - acc);
  const T dn = c_r * r;
  if (d) d[p] = dn;
  xout[p] = x[p] + dn;
}

template <class T>
void cheb_step_zero(hipStream_t s, int64_t n, const Sell *nbr, const int32_t *nbr_pos, const T *dinv,
                    const T *b, const T *x, T *xout, T *d, double c_r) {
  if (n <= 0) return;
  k_cheb_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, dinv, b, nbr ? x : nullptr, xout, d, (T)c_r);
  MG_LAUNCH_CHECK();
  if (!nbr || nbr->nslices == 0) return;
  const unsigned g = sell_grid(*nbr);
  if (nbr->unroll == 4)
    k_cheb_fix<T, 4><<<g, 256, 0, s>>>(nbr->nslices, nbr->nrows, cols_of(*nbr), sell_vals<T>(*nbr), nbr_pos, dinv, b,
                                      x, xout, d, (T)c_r);
  else
    k_cheb_fix<T, 8><<<g, 256, 0, s>>>(nbr->nslices, nbr->nrows, cols_of(*nbr), sell_vals<T>(*nbr), nbr_pos, dinv, b,
                                      x, xout, d, (T)c_r);
  MG_LAUNCH_CHECK();
}
template void cheb_step_zero<double>(hipStream_t, int64_t, const Sell *, const int32_t *, const double *,
                                     const double *, const double *, double *, double *, double);
template void cheb_step_zero<float>(hipStream_t, int64_t, const Sell *, const int32_t *, const float *,
                                    const float *, const float *, float *, float *, double);

// One colour of a multicolour Gauss-Seidel sweep: u_r += D^-1_r (b_r - (A u)_r)
// for the rows r of the colour (pos maps SELL rows to solve-order unknowns).
// Rows of one colour are not coupled, so the update in place is race-free.
template <class T>
__global__ __launch_bounds__(256) void k_sgs_colour(int64_t nslices, int64_t nrows, SellCols cols,
                                                    const T *__restrict__ val, const int32_t *__restrict__ pos,
                                                    const T *__restrict__ dinv, const T *__restrict__ b,
                                                    T *__restrict__ u) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t sl = k >> 6;
  if (sl >= nslices) return;
  T acc = sell_row(cols, val, u, sl, (int)(k & 63));
  const SellRow rw = sell_row_of(cols, k);
  if (!rw.lead || rw.row >= nrows) return;
  const int32_t r = pos[rw.row];
  u[r] += dinv[r] * (b[r] - acc);
}

template <class T>
void sgs_colour_sweep(hipStream_t s, const Sell &S, const int32_t *pos, const T *dinv, const T *b, T *u) {
  if (S.nslices == 0) return;
  k_sgs_colour<T><<<sell_grid(S), 256, 0, s>>>(S.nslices, S.nrows, cols_of(S), sell_vals<T>(S), pos, dinv, b, u);
  MG_LAUNCH_CHECK();
}
template void sgs_colour_sweep<double>(hipStream_t, const Sell &, const int32_t *, const double *, const double *,
                                       double *);
template void sgs_colour_sweep<float>(hipStream_t, const Sell &, const int32_t *, const float *, const float *,
                                      float *);

// ---------------------------------------------------------------------------
// local correction
// ---------------------------------------------------------------------------
// r = b - A u on the rows of one colour's patches: the patch rows of A are a
// SELL matrix of their own (kernel order, rpl lanes per row, chosen per level
// by timing), streamed like the level operator; a colour's rows [k0, k1) are
// the rows of the slices k0 / (64 / rpl) .. (k1 - 1) / (64 / rpl).
template <class T>
__global__ __launch_bounds__(256) void k_patch_residual(int64_t k0, int64_t k1, SellCols cols,
                                                        const T *__restrict__ val,
                                                        const int32_t *__restrict__ dofs, const T *__restrict__ b,
                                                        const T *__restrict__ u, T *__restrict__ res) {
  const int rps = 64 / cols.rpl;
  const int64_t pos = k0 / rps * 64 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t sl = pos >> 6;
  if (sl > (k1 - 1) / rps) return;
  const T acc = sell_row(cols, val, u, sl, (int)(pos & 63));
  const SellRow rw = sell_row_of(cols, pos);
  if (rw.lead && rw.row >= k0 && rw.row < k1) res[rw.row] = b[dofs[rw.row]] - acc;
}

template <class T>
void patch_residual(hipStream_t s, const Patches &pt, int colour, const T *b, const T *u, T *res) {
  int p0 = pt.colour_first[colour], p1 = pt.colour_first[colour + 1];
  int64_t k0 = pt.h_kptr[p0], k1 = pt.h_kptr[p1];
  if (k1 <= k0) return;
  const int64_t rps = 64 / pt.rows.rpl;
  const int64_t span = ((k1 - 1) / rps - k0 / rps + 1) * 64;
  k_patch_residual<T><<<(unsigned)((span + 255) / 256), 256, 0, s>>>(k0, k1, cols_of(pt.rows),
                                                                      sell_vals<T>(pt.rows), pt.dofs, b, u, res);
  MG_LAUNCH_CHECK();
}
template void patch_residual<double>(hipStream_t, const Patches &, int, const double *, const double *, double *);
template void patch_residual<float>(hipStream_t, const Patches &, int, const float *, const float *, float *);

// e = X r with X symmetric, stored as packed lower 32 x 32 tiles (PackedInv).
// Row items: one wavefront per (system k, tile row I, chunk of at most
// PACK_CHUNK tiles).  Lane (h, j) = (lane >> 5, lane & 31) reads rows 2 s + h,
// s = 0..15, column j of each tile, so every tile is read once, coalesced,
// the next tile already in flight.  Tile (I, J) gives
//   the column product X_IJ^T r_I  (J < I; lane-private, one 32-entry vector
//                                   per tile in pz, column-major over tiles),
//   the row product    X_IJ r_J     (the tile is transposed through the
//                                   wavefront's LDS area, lane (h, i) sums half
//                                   of row i),
// and the row products of the chunk are summed in registers into one py slot.
// TM is the storage and arithmetic type, TV the type of r.
template <class TM, class TV>
__global__ __launch_bounds__(256) void k_packed_rows(int i0, int i1, const int32_t *__restrict__ r_sys,
                                                     const int32_t *__restrict__ r_row,
                                                     const int32_t *__restrict__ r_chunk,
                                                     const int32_t *__restrict__ r_slot,
                                                     const int32_t *__restrict__ ptr,
                                                     const int64_t *__restrict__ toff,
                                                     const int64_t *__restrict__ zoff, const TM *__restrict__ pk,
                                                     const TV *__restrict__ res, int vs, TM *__restrict__ py,
                                                     TM *__restrict__ pz, int chunk) {
  constexpr int PT = PATCH_TILE;
  __shared__ TM tl[4][PT][PT + 1];
  __shared__ TM rl[4][PT];
  const int wave = threadIdx.x >> 6;
  const int item = i0 + (int)(blockIdx.x * 4 + wave);
  if (item >= i1) return;
  const int lane = threadIdx.x & 63, h = lane >> 5, j = lane & 31;
  TM(*Ts)[PT + 1] = tl[wave];
  TM *Rs = rl[wave];
  const int k = r_sys[item], I = r_row[item];
  const int J0 = r_chunk[item] * chunk, J1 = min(I + 1, J0 + chunk);
  const int k0 = ptr[k], n = ptr[k + 1] - k0, nb = (n + PT - 1) / PT;
  const TV *r = res + (int64_t)k0 * vs;  // entry i of the system at r[i vs]
  TM rI[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    int i = I * PT + 2 * s + h;
    rI[s] = i < n ? (TM)r[(int64_t)i * vs] : (TM)0;
  }
  const TM *tile = pk + toff[k] + ((int64_t)I * (I + 1) / 2 + J0) * PT * PT + h * PT + j;
  TM *zcol = pz + zoff[k] + (int64_t)(I - 1) * PT + j;  // + 32 (J nb - J (J + 1) / 2 - J)
  TM yrow = 0;
  TM v[16], nxt[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) nxt[s] = __builtin_nontemporal_load(tile + 2 * s * PT);
  for (int J = J0; J < J1; ++J) {
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = nxt[s];
    tile += PT * PT;
    if (J + 1 < J1) {
#pragma unroll
      for (int s = 0; s < 16; ++s) nxt[s] = __builtin_nontemporal_load(tile + 2 * s * PT);
    }
    if (J < I) {
      TM cs = 0;
#pragma unroll
      for (int s = 0; s < 16; ++s) cs += v[s] * rI[s];
      cs += __shfl_xor(cs, 32);
      if (h == 0) zcol[(int64_t)PT * ((int64_t)J * nb - (int64_t)J * (J + 1) / 2 - J)] = cs;
    }
    const int jj = J * PT + j;
    if (h == 0) Rs[j] = jj < n ? (TM)r[(int64_t)jj * vs] : (TM)0;
#pragma unroll
    for (int s = 0; s < 16; ++s) Ts[2 * s + h][j] = v[s];
    wave_sync();
    TM acc = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) acc += Ts[j][16 * h + t] * Rs[16 * h + t];
    yrow += acc + __shfl_xor(acc, 32);  // row j
    wave_sync();
  }
  if (h == 0) py[(int64_t)r_slot[item] * PT + j] = yrow;
}

// Gather items: e_J = (row products of the chunks of tile row J) + sum over
// I > J of the column products of tile (I, J), in a fixed order; then
//   GATHER_ADD:    u[map(i)] += e (patches of one colour share no DOF),
//   GATHER_SET:    u[i] = e (identity map),
//   GATHER_STAGE:  st[map(i)] = e (FP64 staging of a first patch solve),
//   GATHER_FINISH: u[map(i)] += e + st[map(i)], st[map(i)] = 0 (the refined
//                  solve: the staged first solve plus the correction e).
enum { GATHER_ADD = 0, GATHER_SET = 1, GATHER_STAGE = 2, GATHER_FINISH = 3 };
template <class TM, class TV, int MODE>
__global__ __launch_bounds__(256) void k_packed_gather(int i0, int i1, const int32_t *__restrict__ g_sys,
                                                       const int32_t *__restrict__ g_row,
                                                       const int32_t *__restrict__ g_slot,
                                                       const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ map,
                                                       const int64_t *__restrict__ zoff,
                                                       const TM *__restrict__ py, const TM *__restrict__ pz,
                                                       TV *__restrict__ u, int vs, double *__restrict__ st,
                                                       int chunk) {
  constexpr int PT = PATCH_TILE;
  const int item = i0 + (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (item >= i1) return;
  const int lane = threadIdx.x & 63, h = lane >> 5, j = lane & 31;
  const int k = g_sys[item], J = g_row[item];
  const int k0 = ptr[k], n = ptr[k + 1] - k0, nb = (n + PT - 1) / PT;
  const int nch = J / chunk + 1;
  TM e0 = 0, e1 = 0, e2 = 0, e3 = 0;
  const TM *y = py + (int64_t)g_slot[item] * PT + j;
  for (int c = h; c < nch; c += 2) e0 += y[(int64_t)c * PT];
  const int cnt = nb - J - 1;  // tiles below the diagonal in tile column J
  const TM *z = pz + zoff[k] + (int64_t)PT * ((int64_t)J * nb - (int64_t)J * (J + 1) / 2) + j;
  int t = h;
  for (; t + 6 < cnt; t += 8) {
    e0 += z[(int64_t)t * PT];
    e1 += z[(int64_t)(t + 2) * PT];
    e2 += z[(int64_t)(t + 4) * PT];
    e3 += z[(int64_t)(t + 6) * PT];
  }
  for (; t < cnt; t += 2) e0 += z[(int64_t)t * PT];
  TM e = (e0 + e1) + (e2 + e3);
  e += __shfl_xor(e, 32);
  const int i = J * PT + j;
  if (h == 0 && i < n) {
    if (MODE == GATHER_SET) {
      u[(int64_t)i * vs] = (TV)e;
    } else if (MODE == GATHER_ADD) {
      u[(int64_t)map[k0 + i] * vs] += (TV)e;
    } else if (MODE == GATHER_STAGE) {
      st[map[k0 + i]] = (double)e;
    } else {
      const int32_t q = map[k0 + i];
      u[(int64_t)q * vs] += (TV)((double)e + st[q]);
      st[q] = 0.0;
    }
  }
}

template <class TM, class TV, int MODE>
static void packed_apply(hipStream_t s, const PackedInv &P, const TM *pk, int colour, const int32_t *ptr,
                         const int32_t *map, const TV *res, TM *py, TM *pz, TV *u, int vs, double *st = nullptr) {
  int r0 = P.colour_r_first[colour], r1 = P.colour_r_first[colour + 1];
  int g0 = P.colour_g_first[colour], g1 = P.colour_g_first[colour + 1];
  if (r1 <= r0) return;
  k_packed_rows<TM, TV><<<(unsigned)((r1 - r0 + 3) / 4), 256, 0, s>>>(r0, r1, P.r_sys, P.r_row, P.r_chunk, P.r_slot,
                                                                      ptr, P.tile_off, P.zoff, pk, res, vs, py, pz,
                                                                      P.chunk);
  MG_LAUNCH_CHECK();
  k_packed_gather<TM, TV, MODE><<<(unsigned)((g1 - g0 + 3) / 4), 256, 0, s>>>(g0, g1, P.g_sys, P.g_row, P.g_slot,
                                                                              ptr, map, P.zoff, py, pz, u, vs, st,
                                                                              P.chunk);
  MG_LAUNCH_CHECK();
}

// res and u may be one column of a block vector: entry i at res[i vs], u[i vs]
template <class T>
void patch_apply(hipStream_t s, const Patches &pt, int colour, const T *res, T *py, T *pz, T *u, int vs) {
  const T *pk = std::is_same<T, double>::value ? (const T *)pt.inv.v64.p : (const T *)pt.inv.v32.p;
  packed_apply<T, T, GATHER_ADD>(s, pt.inv, pk, colour, pt.ptr, pt.dofs, res, py, pz, u, vs);
}

// One step of iterative refinement of the patch solves: r2 = r - A^[d] e with
// e the staged first solve (FP64, in the solve-order positions of the patch
// DOFs) and A^[d] the patch rows restricted to their own patch's columns
// (pt.loc: the rows' values with every other column zeroed), accumulated in
// FP64 and written over r.
template <class T>
__global__ __launch_bounds__(256) void k_patch_refine(int64_t k0, int64_t k1, SellCols cols,
                                                      const double *__restrict__ loc, const double *__restrict__ st,
                                                      T *__restrict__ res, int vs) {
  int64_t k = (k0 & ~(int64_t)63) + (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t sl = k >> 6;
  if (k >= ((k1 + 63) & ~(int64_t)63)) return;
  const double acc = sell_row<double>(cols, loc, st, sl, (int)(k & 63));
  if (k >= k0 && k < k1) res[k * vs] = (T)((double)res[k * vs] - acc);
}

// e = A^[d]^-1 r for the patches of one colour with one refinement step:
// e1 = X r (staged in FP64), r2 = r - A^[d] e1 (FP64), u += e1 + X r2.
// res is overwritten; st is all zero outside a call (and left so).
template <class T>
void patch_apply_refined(hipStream_t s, const Patches &pt, int colour, T *res, T *py, T *pz, T *u, double *st,
                         int vs) {
  const T *pk = std::is_same<T, double>::value ? (const T *)pt.inv.v64.p : (const T *)pt.inv.v32.p;
  packed_apply<T, T, GATHER_STAGE>(s, pt.inv, pk, colour, pt.ptr, pt.dofs, res, py, pz, (T *)nullptr, vs, st);
  const int p0 = pt.colour_first[colour], p1 = pt.colour_first[colour + 1];
  const int64_t k0 = pt.h_kptr[p0], k1 = pt.h_kptr[p1];
  if (k1 <= k0) return;
  const int64_t span = ((k1 + 63) & ~(int64_t)63) - (k0 & ~(int64_t)63);
  k_patch_refine<T><<<(unsigned)((span + 255) / 256), 256, 0, s>>>(k0, k1, cols_of(pt.rows), pt.loc, st, res, vs);
  MG_LAUNCH_CHECK();
  packed_apply<T, T, GATHER_FINISH>(s, pt.inv, pk, colour, pt.ptr, pt.dofs, res, py, pz, u, vs, st);
}
template void patch_apply_refined<double>(hipStream_t, const Patches &, int, double *, double *, double *, double *,
                                          double *, int);
template void patch_apply_refined<float>(hipStream_t, const Patches &, int, float *, float *, float *, float *,
                                         double *, int);
template void patch_apply<double>(hipStream_t, const Patches &, int, const double *, double *, double *, double *,
                                  int);
template void patch_apply<float>(hipStream_t, const Patches &, int, const float *, float *, float *, float *, int);

// The local correction of one colour whose patches all hold at most NB tile
// rows (NB = 4, 8 or 12: 128, 256 or 384 DOFs), one workgroup per patch, in
// one launch instead of three: the patch-row residual (whole SELL slices per
// wavefront, as in k_patch_residual), then one wavefront per tile row I of
// the packed inverse (the steps of k_packed_rows with the whole tile row as
// one chunk), then one wavefront per tile row J adding the row products and
// the column products of the tiles below in k_packed_gather's order.  The
// residual, the row products and the column products stay in LDS; every sum
// is formed as in the three-kernel path whenever a tile row fits one chunk of
// the packed layout, so the result is then bitwise the same (and the same for
// every NB).  With res given, the residual of the colour's patch rows comes
// from k_patch_residual (patches whose rows read DOFs of other patches of the
// colour need every residual before any update) and the launch replaces the
// two launches of the packed product.
template <class T, int NB>
__global__ __launch_bounds__(256) void k_patch_small(int p0, SellCols cols, const T *__restrict__ val,
                                                     const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ dofs,
                                                     const int64_t *__restrict__ toff, const T *__restrict__ pk,
                                                     const T *__restrict__ b, const T *__restrict__ res,
                                                     T *__restrict__ u) {
  constexpr int PT = PATCH_TILE;
  __shared__ T rs[NB * PT];
  __shared__ T ys[NB][PT];
  __shared__ T zs[NB * (NB - 1) / 2][PT];
  __shared__ T tl[4][PT][PT + 1];
  __shared__ T rl[4][PT];
  const int k = p0 + (int)blockIdx.x;
  const int k0 = ptr[k], n = ptr[k + 1] - k0, nb = (n + PT - 1) / PT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // 1. r = b - A u on the patch rows
  if (res) {
    for (int i = threadIdx.x; i < n; i += 256) rs[i] = res[k0 + i];
  } else if (n > 0) {
    const int64_t s0 = k0 >> 6, s1 = (int64_t)(k0 + n - 1) >> 6;
    for (int64_t sl = s0 + wave; sl <= s1; sl += 4) {
      const T acc = sell_row(cols, val, u, sl, lane);
      const int64_t kk = sl * 64 + lane;
      if (kk >= k0 && kk < k0 + n) rs[kk - k0] = b[dofs[kk]] - acc;
    }
  }
  __syncthreads();
  const int h = lane >> 5, j = lane & 31;
  // 2. tile rows: row products into ys, column products into zs; tile row I
  // holds I + 1 tiles, so rows I and nb - 1 - I form a pair of nb + 1 tiles
  // and wavefront w takes the pairs w, w + 4, ...
  for (int I = 0; I < nb; ++I) {
    if (min(I, nb - 1 - I) % 4 != wave) continue;
    T(*Ts)[PT + 1] = tl[wave];
    T *Rs = rl[wave];
    T rI[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = I * PT + 2 * q + h;
      rI[q] = i < n ? rs[i] : (T)0;
    }
    const T *tile = pk + toff[k] + (int64_t)I * (I + 1) / 2 * PT * PT + h * PT + j;
    T yrow = 0;
    T v[16], nxt[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) nxt[q] = __builtin_nontemporal_load(tile + 2 * q * PT);
    for (int J = 0; J <= I; ++J) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = nxt[q];
      tile += PT * PT;
      if (J + 1 <= I) {
#pragma unroll
        for (int q = 0; q < 16; ++q) nxt[q] = __builtin_nontemporal_load(tile + 2 * q * PT);
      }
      if (J < I) {
        T cs = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) cs += v[q] * rI[q];
        cs += __shfl_xor(cs, 32);
        if (h == 0) zs[J * nb - J * (J + 1) / 2 + (I - J - 1)][j] = cs;
      }
      const int jj = J * PT + j;
      if (h == 0) Rs[j] = jj < n ? rs[jj] : (T)0;
#pragma unroll
      for (int q = 0; q < 16; ++q) Ts[2 * q + h][j] = v[q];
      wave_sync();
      T acc = 0;
#pragma unroll
      for (int t = 0; t < 16; ++t) acc += Ts[j][16 * h + t] * Rs[16 * h + t];
      yrow += acc + __shfl_xor(acc, 32);
      wave_sync();
    }
    if (h == 0) ys[I][j] = yrow;
  }
  __syncthreads();
  // 3. e_J = row products of tile row J + column products of the tiles below
  for (int J = wave; J < nb; J += 4) {
    T e0 = 0, e1 = 0, e2 = 0, e3 = 0;
    if (h == 0) e0 += ys[J][j];
    const int cnt = nb - J - 1;
    const int zb = J * nb - J * (J + 1) / 2;
    int t = h;
    for (; t + 6 < cnt; t += 8) {
      e0 += zs[zb + t][j];
      e1 += zs[zb + t + 2][j];
      e2 += zs[zb + t + 4][j];
      e3 += zs[zb + t + 6][j];
    }
    for (; t < cnt; t += 2) e0 += zs[zb + t][j];
    T e = (e0 + e1) + (e2 + e3);
    e += __shfl_xor(e, 32);
    const int i = J * PT + j;
    if (h == 0 && i < n) u[dofs[k0 + i]] += e;
  }
}

template <class T>
void patch_correct_small(hipStream_t s, const Patches &pt, int colour, const T *b, const T *res, T *u) {
  const int p0 = pt.colour_first[colour], p1 = pt.colour_first[colour + 1];
  if (p1 <= p0) return;
  if (pt.small_nb * PATCH_TILE < pt.maxn) fail(MG_ERR_ARG, "patch_correct_small: patches too large");
  if (!res && pt.rows.rpl != 1) fail(MG_ERR_ARG, "patch_correct_small: the fused residual needs one lane per row");
  const T *pk = std::is_same<T, double>::value ? (const T *)pt.inv.v64.p : (const T *)pt.inv.v32.p;
  const unsigned g = (unsigned)(p1 - p0);
  if (pt.small_nb == 4)
    k_patch_small<T, 4><<<g, 256, 0, s>>>(p0, cols_of(pt.rows), sell_vals<T>(pt.rows), pt.ptr, pt.dofs,
                                         pt.inv.tile_off, pk, b, res, u);
  else if (pt.small_nb == 8)
    k_patch_small<T, 8><<<g, 256, 0, s>>>(p0, cols_of(pt.rows), sell_vals<T>(pt.rows), pt.ptr, pt.dofs,
                                         pt.inv.tile_off, pk, b, res, u);
  else if (pt.small_nb == 12)
    k_patch_small<T, 12><<<g, 256, 0, s>>>(p0, cols_of(pt.rows), sell_vals<T>(pt.rows), pt.ptr, pt.dofs,
                                          pt.inv.tile_off, pk, b, res, u);
  else
    fail(MG_ERR_ARG, "patch_correct_small: no one-workgroup size class");
  MG_LAUNCH_CHECK();
}
template void patch_correct_small<double>(hipStream_t, const Patches &, int, const double *, const double *,
                                          double *);
template void patch_correct_small<float>(hipStream_t, const Patches &, int, const float *, const float *, float *);

// coarsest level: u = A^-1 b with the packed FP64 inverse (FP64 arithmetic)
template <class T>
void coarse_apply(hipStream_t s, const Level &L, const T *b, T *u, int vs) {
  if (L.cnd.on) {
    coarse_apply_nd<T>(s, L, b, u, vs);
    return;
  }
  packed_apply<double, T, GATHER_SET>(s, L.cpk, L.cpk.v64.p, 0, L.cptr, nullptr, b, L.cpy.p, L.cpz.p, u, vs);
}
template void coarse_apply<double>(hipStream_t, const Level &, const double *, double *, int);
template void coarse_apply<float>(hipStream_t, const Level &, const float *, float *, int);



// ---------------------------------------------------------------------------
// vector kernels
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T *x, int64_t n, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
template <class T>
void fill(hipStream_t s, T *x, int64_t n, T v) {
  if (n <= 0) return;
  k_fill<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, v);
  MG_LAUNCH_CHECK();
}
template void fill<double>(hipStream_t, double *, int64_t, double);
template void fill<float>(hipStream_t, float *, int64_t, float);
template void fill<int32_t>(hipStream_t, int32_t *, int64_t, int32_t);

template <class A, class B>
__global__ void k_convert(const A *x, B *y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (B)x[i];
}
template <class A, class B>
void convert(hipStream_t s, const A *x, B *y, int64_t n) {
  if (n <= 0) return;
  k_convert<A, B><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
  MG_LAUNCH_CHECK();
}
template void convert<double, float>(hipStream_t, const double *, float *, int64_t);
template void convert<float, double>(hipStream_t, const float *, double *, int64_t);
template void convert<double, double>(hipStream_t, const double *, double *, int64_t);
template void convert<float, float>(hipStream_t, const float *, float *, int64_t);

void copy64(hipStream_t s, const double *x, double *y, int64_t n) { convert<double, double>(s, x, y, n); }

template <class A, class B>
__global__ void k_gather_perm(const A *x, const int32_t *perm, B *y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (B)x[perm[i]];
}
template <class A, class B>
__global__ void k_scatter_perm(const A *x, const int32_t *perm, B *y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[perm[i]] = (B)x[i];
}
template <class A, class B>
void gather_perm(hipStream_t s, const A *x, const int32_t *perm, B *y, int64_t n) {
  if (n <= 0) return;
  k_gather_perm<A, B><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, perm, y, n);
  MG_LAUNCH_CHECK();
}
template <class A, class B>
void scatter_perm(hipStream_t s, const A *x, const int32_t *perm, B *y, int64_t n) {
  if (n <= 0) return;
  k_scatter_perm<A, B><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, perm, y, n);
  MG_LAUNCH_CHECK();
}
template void gather_perm<double, double>(hipStream_t, const double *, const int32_t *, double *, int64_t);
template void gather_perm<double, float>(hipStream_t, const double *, const int32_t *, float *, int64_t);
template void scatter_perm<double, double>(hipStream_t, const double *, const int32_t *, double *, int64_t);
template void scatter_perm<float, double>(hipStream_t, const float *, const int32_t *, double *, int64_t);

template <class T>
__global__ void k_add(T *y, const T *x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}
void add64(hipStream_t s, double *y, const double *x, int64_t n) {
  k_add<double><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y, x, n);
  MG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// inner products: per-block partial sums, then one block sums them in order
// ---------------------------------------------------------------------------
int dot_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ x, const double *__restrict__ y, int64_t n,
                                             double *__restrict__ part) {
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += x[i] * y[i];
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
void dot_partials(hipStream_t s, const double *x, const double *y, int64_t n, double *part, int nblocks) {
  k_dot<<<nblocks, 256, 0, s>>>(x, y, n, part);
  MG_LAUNCH_CHECK();
}
__global__ __launch_bounds__(256) void k_finish(const double *part, int nb, double *out) {
  double s = 0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = s;
}
void finish_sum(hipStream_t s, const double *part, int nblocks, double *out) {
  k_finish<<<1, 256, 0, s>>>(part, nblocks, out);
  MG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// CG: scalars live on the device.  scal[]: 0 rho=r.z  1 p.q  2 alpha  3 r.r
// 4 rho_new  5 beta  6 breakdown flag
// ---------------------------------------------------------------------------
__global__ void k_cg_alpha(double *scal) {
  double pq = scal[1];
  bool bad = !(pq > 0.0) || !isfinite(pq) || !isfinite(scal[0]);
  scal[2] = bad ? 0.0 : scal[0] / pq;
  if (bad) scal[6] = 1.0;
}
void cg_alpha(hipStream_t s, double *scal) {
  k_cg_alpha<<<1, 1, 0, s>>>(scal);
  MG_LAUNCH_CHECK();
}

__global__ __launch_bounds__(256) void k_cg_xr(double *__restrict__ x, double *__restrict__ r,
                                               const double *__restrict__ p, const double *__restrict__ q,
                                               const double *__restrict__ scal, int64_t n, double *__restrict__ part) {
  double a = scal[2];
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] += a * p[i];
    double ri = r[i] - a * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
void cg_update_xr(hipStream_t s, double *x, double *r, const double *p, const double *q, const double *scal,
                  int64_t n, double *part, int nblocks) {
  k_cg_xr<<<nblocks, 256, 0, s>>>(x, r, p, q, scal, n, part);
  MG_LAUNCH_CHECK();
}

__global__ void k_cg_beta(double *scal) {
  double rn = scal[4];
  bool bad = !isfinite(rn) || scal[0] == 0.0;
  scal[5] = bad ? 0.0 : rn / scal[0];
  scal[0] = rn;
  if (bad) scal[6] = 1.0;
}
void cg_beta(hipStream_t s, double *scal) {
  k_cg_beta<<<1, 1, 0, s>>>(scal);
  MG_LAUNCH_CHECK();
}

__global__ void k_cg_p(double *__restrict__ p, const double *__restrict__ z, const double *__restrict__ scal,
                       int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + scal[5] * p[i];
}
void cg_update_p(hipStream_t s, double *p, const double *z, const double *scal, int64_t n) {
  k_cg_p<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, z, scal, n);
  MG_LAUNCH_CHECK();
}

// the CG scalars into pinned host memory (host_dev: its device address), made
// visible to the host before the kernel ends, so that a wait on the stream
// is enough to read them; a kernel rather than a copy so that it can sit in
// a captured graph
__global__ void k_scal_to_host(const double *__restrict__ scal, double *host_dev, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) host_dev[i] = scal[i];
  __threadfence_system();
}
void scal_to_host(hipStream_t s, const double *scal, double *host_dev, int count) {
  k_scal_to_host<<<1, 64, 0, s>>>(scal, host_dev, count);
  MG_LAUNCH_CHECK();
}

// q = A p (FP64 SELL) with partial sums of p.q
template <int U, bool M>
__global__ __launch_bounds__(256) void k_spmv_dot(
    int64_t nslices, int64_t nrows, SellCols cols, const double *__restrict__ val, const double *__restrict__ p,
    double *__restrict__ q, double *__restrict__ part) {
  int64_t blk = blockIdx.x;
  int64_t pos = blk * 256 + threadIdx.x;
  int64_t sl = pos >> 6;
  double contrib = 0;
  if (sl < nslices) {
    double acc = sell_row<double, U, M>(cols, val, p, sl, (int)(pos & 63));
    const SellRow rw = sell_row_of(cols, pos);
    if (rw.lead && rw.row < nrows) {
      q[rw.row] = acc;
      contrib = acc * p[rw.row];
    }
  }
  contrib = block_sum(contrib);
  if (threadIdx.x == 0) part[blk] = contrib;
}
int spmv_dot_blocks(const Sell &S) { return (int)sell_grid(S); }
void spmv_dot(hipStream_t s, const Sell &S, const double *p, double *q, double *part) {
  const unsigned g = sell_grid(S);
  const SellCols cs = cols_of(S);
  if (S.unroll == 4) {
    if (S.mask) k_spmv_dot<4, true><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, S.v64, p, q, part);
    else k_spmv_dot<4, false><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, S.v64, p, q, part);
  } else {
    if (S.mask) k_spmv_dot<8, true><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, S.v64, p, q, part);
    else k_spmv_dot<8, false><<<g, 256, 0, s>>>(S.nslices, S.nrows, cs, S.v64, p, q, part);
  }
  MG_LAUNCH_CHECK();
}

}  // namespace mg
